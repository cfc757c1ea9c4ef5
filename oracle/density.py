"""Oracle: density filter, smoothed Heaviside projection and their chain rule.

Test infrastructure only (see the package docstring).

Sources in the paper:
* Sec. 4.3: design variables are first density-filtered (neighbourhood filter
  with linearly decaying "hat" weights of radius r_min), then projected by the
  smoothed Heaviside of the projection equation with threshold eta and
  sharpness beta; sensitivities are carried back by the chain rule.
* Sec. 4.4: three realisations at eta = 0.3 (dilated), 0.5 (intermediate)
  and 0.7 (eroded).

Boundary treatment (not stated in the paper): the neighbourhood is truncated at
the domain boundary and the weights are renormalised over what remains.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp


def filter_matrix(p, rmin):
    """Row-normalised filter W with W[e, i] = w_ei / sum_k w_ek,
    w_ei = max(0, rmin - |x_e - x_i|) over element centroids."""
    dims = (p.nelx, p.nely) if p.dim == 2 else (p.nelx, p.nely, p.nelz)
    n_el = int(np.prod(dims))
    if rmin <= 1.0:
        return sp.identity(n_el, format="csr")
    R = int(np.ceil(rmin)) - 1
    grids = np.meshgrid(*[np.arange(n) for n in dims[::-1]], indexing="ij")
    coords = [g.ravel() for g in grids[::-1]]          # ex, ey(, ez) in element order
    strides = [1, dims[0]] + ([dims[0] * dims[1]] if p.dim == 3 else [])
    rows, cols, vals = [], [], []
    idx = np.arange(n_el)
    for off in itertools.product(range(-R, R + 1), repeat=p.dim):
        dist = np.sqrt(sum(o * o for o in off))
        w = rmin - dist
        if w <= 0:
            continue
        ok = np.ones(n_el, dtype=bool)
        nb = idx.copy()
        for a in range(p.dim):
            c = coords[a] + off[a]
            ok &= (c >= 0) & (c < dims[a])
            nb = nb + off[a] * strides[a]
        rows.append(idx[ok])
        cols.append(nb[ok])
        vals.append(np.full(ok.sum(), w))
    H = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n_el, n_el)).tocsr()
    Hs = np.asarray(H.sum(axis=1)).ravel()
    return sp.diags(1.0 / Hs) @ H


def filter_density(p, rho, rmin):
    """rho_tilde = W rho."""
    return filter_matrix(p, rmin) @ np.asarray(rho, dtype=np.float64)


def heaviside(rho_tilde, beta, eta):
    """Smoothed Heaviside projection (Sec. 4.3, projection equation)."""
    den = np.tanh(beta * eta) + np.tanh(beta * (1.0 - eta))
    return (np.tanh(beta * eta) + np.tanh(beta * (np.asarray(rho_tilde) - eta))) / den


def heaviside_derivative(rho_tilde, beta, eta):
    """d rho_bar / d rho_tilde."""
    den = np.tanh(beta * eta) + np.tanh(beta * (1.0 - eta))
    t = np.tanh(beta * (np.asarray(rho_tilde) - eta))
    return beta * (1.0 - t * t) / den


def filter_project(p, rho, rmin, beta, etas):
    """rho -> (rho_tilde, [rho_bar_eta for eta in etas])."""
    rt = filter_density(p, rho, rmin)
    return rt, np.stack([heaviside(rt, beta, e) for e in etas])


def filter_project_adjoint(p, rho_tilde, rmin, beta, etas, dc_drho_phys):
    """Chain rule: dc/drho_i = sum_e dc/drho_bar_e * H'(rho_tilde_e) * W[e, i]."""
    W = filter_matrix(p, rmin)
    out = []
    for s, e in enumerate(etas):
        g = np.asarray(dc_drho_phys[s]) * heaviside_derivative(rho_tilde, beta, e)
        out.append(W.T @ g)
    return np.stack(out)


def non_discreteness(rho_bar):
    """M_nd = sum 4 rho (1 - rho) / n  (Sec. 5.2)."""
    r = np.asarray(rho_bar)
    return float(np.sum(4.0 * r * (1.0 - r)) / r.size)


def robust_objective(c, dc, kappa=1.0, weights=None):
    """Robust objective of Sec. 4.4, f = E[c] + kappa sqrt(Var[c]) over the
    realisations (weights w_s, equal by default; population variance), and its
    gradient df = sum_s w_s (1 + kappa (c_s - E[c]) / sqrt(Var[c])) dc_s (the
    variance term's gradient taken as zero when Var[c] = 0).
    c: [nsys]; dc: [nsys][n] gradients of the realisations' compliances.
    Returns (f, mean, std, df)."""
    c = np.asarray(c, dtype=np.float64)
    dc = np.asarray(dc, dtype=np.float64)
    w = np.full(c.size, 1.0 / c.size) if weights is None else np.asarray(weights, dtype=np.float64)
    mean = float(np.sum(w * c))
    var = float(np.sum(w * (c - mean) ** 2))
    std = float(np.sqrt(var))
    a = w * (1.0 + (kappa * (c - mean) / std if std > 0.0 else 0.0))
    return mean + kappa * std, mean, std, np.tensordot(a, dc, axes=1)


def tile_design(p, x_cell, cell):
    """Element densities of a periodic design (Sec. 4.1): element e takes the
    design variable of its position in the unit cell of cell = (cx, cy[, cz])
    elements."""
    dims = (p.nelx, p.nely) if p.dim == 2 else (p.nelx, p.nely, p.nelz)
    grids = np.meshgrid(*[np.arange(n) for n in dims[::-1]], indexing="ij")
    coords = [g.ravel() for g in grids[::-1]]
    idx = coords[0] % cell[0] + cell[0] * (coords[1] % cell[1])
    if p.dim == 3:
        idx = idx + cell[0] * cell[1] * (coords[2] % cell[2])
    return np.asarray(x_cell)[idx], idx


def periodic_sum(p, g, cell):
    """Sensitivity of a periodic design variable (Sec. 4.1): the sum of the
    element sensitivities g over every element it controls."""
    n = int(np.prod(cell[:p.dim]))
    _, idx = tile_design(p, np.zeros(n), cell)
    return np.bincount(idx, weights=np.asarray(g, dtype=np.float64), minlength=n)
