"""Seeded synthetic workloads: meshes, supports, loads and raw design fields.

This module holds problem definitions only. It computes no part of the method
(no stiffness, no filtering, no projection, no solve), so that the CPU oracle
and the GPU path can both draw their inputs from it without sharing any
arithmetic of the method.

Index conventions (shared by every consumer):

* node  n = ix + (nelx+1) * (iy + (nely+1) * iz)
* dof     = dim * n + c            (c = 0:x, 1:y, 2:z)
* element e = ex + nelx * (ey + nely * ez)

The paper's beams are its own definitions (Sec. 3.1, Sec. 6); there is no
public dataset behind them. The problems below are synthetic stand-ins with the
shapes of the paper's workloads: periodic 0/1 microstructures with a 1e9
stiffness contrast (Sec. 6 uses E_max = 1, E_min = 1e-9), a filter radius of a
few elements, and a smoothed Heaviside projection at three thresholds
(Sec. 4.3, Sec. 4.4).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Problem:
    """A structured-mesh elasticity problem definition.

    dim: 2 (bilinear quads) or 3 (trilinear hexahedra); nel = (nelx, nely, nelz)
    with nelz = 1 in 2D; sub = subdomain (unit-cell) edge in elements; k = coarse
    vectors per subdomain; nsys = number of right-hand-side systems solved
    together (the robust realisations).
    """

    name: str
    dim: int
    nel: tuple
    sub: int
    k: int
    nsys: int = 1
    E0: float = 1.0
    Emin: float = 1e-9
    penal: float = 3.0
    nu: float = 0.3
    rmin: float = 0.0          # density filter radius in elements (0: no filter)
    beta: float = 8.0          # Heaviside sharpness
    etas: tuple = (0.5,)       # projection thresholds, one per system
    support: str = "cantilever"
    seed: int = 1000
    density: str = "pattern"
    extra: dict = field(default_factory=dict, hash=False, compare=False)

    @property
    def nelx(self):
        return self.nel[0]

    @property
    def nely(self):
        return self.nel[1]

    @property
    def nelz(self):
        return self.nel[2] if self.dim == 3 else 1

    @property
    def n_el(self):
        return self.nelx * self.nely * self.nelz

    @property
    def nnodes(self):
        nn = (self.nelx + 1) * (self.nely + 1)
        return nn * (self.nelz + 1) if self.dim == 3 else nn

    @property
    def n_dof(self):
        return self.dim * self.nnodes

    @property
    def n_sub(self):
        ns = (self.nelx // self.sub) * (self.nely // self.sub)
        return ns * (self.nelz // self.sub) if self.dim == 3 else ns


# ----------------------------------------------------------------------------
# Named workloads (sizes of the benchmark configurations)
# ----------------------------------------------------------------------------

def mbb_64x32() -> Problem:
    """2D MBB half-beam, 64x32 Q4 elements, 8x8 periodic 0/1 cells, s=8, k=4."""
    return Problem("mbb_64x32", 2, (64, 32, 1), sub=8, k=4, nsys=1,
                   support="mbb", seed=1000, density="tiled01", etas=(None,),
                   extra={"cell": 8})


def cantilever2d(nelx=1024, nely=512, sub=32, k=6, name=None) -> Problem:
    """2D cantilever: 16x16 periodic 0/1 cells times a smooth seeded field,
    filtered (r=2) and projected (beta=8) at eta = 0.3/0.5/0.7: 3 systems."""
    return Problem(name or f"cantilever2d_{nelx}x{nely}", 2, (nelx, nely, 1),
                   sub=sub, k=k, nsys=3, support="cantilever", seed=1001,
                   density="modulated", rmin=2.0, beta=8.0,
                   etas=(0.3, 0.5, 0.7), extra={"cell": 16})


def cantilever3d(nelx=192, nely=96, nelz=96, sub=16, k=8, name=None) -> Problem:
    """3D cantilever of H8 elements with a layered microstructure."""
    return Problem(name or f"cantilever3d_{nelx}x{nely}x{nelz}", 3,
                   (nelx, nely, nelz), sub=sub, k=k, nsys=1,
                   support="cantilever3d", seed=1003, density="layered",
                   etas=(None,), extra={"cell": 12})


# ----------------------------------------------------------------------------
# Supports and loads
# ----------------------------------------------------------------------------

def _node(p: Problem, ix, iy, iz=0):
    return ix + (p.nelx + 1) * (iy + (p.nely + 1) * iz)


def _anchor(p: Problem) -> int:
    """Offset (in elements) of the load and roller nodes from the bottom or top
    edge: the centre line of the first row of unit cells, where the cells'
    horizontal bar (or, in 3D, the first solid layer) carries them, so that no
    load or support acts on void material alone."""
    c = p.extra.get("cell", 0)
    if p.density == "layered":
        return 2
    return c // 2


def fixed_mask(p: Problem) -> np.ndarray:
    """uint8 [n_dof]: 1 where the displacement component is prescribed zero."""
    m = np.zeros(p.n_dof, dtype=np.uint8)
    d = p.dim
    a = _anchor(p)
    if p.support == "mbb":
        # symmetry line x = 0: u_x = 0; roller near the bottom-right corner: u_y = 0
        for iy in range(p.nely + 1):
            m[d * _node(p, 0, iy) + 0] = 1
        m[d * _node(p, p.nelx, a) + 1] = 1
    elif p.support == "cantilever":
        for iy in range(p.nely + 1):
            m[d * _node(p, 0, iy) + 0] = 1
            m[d * _node(p, 0, iy) + 1] = 1
    elif p.support == "cantilever3d":
        for iz in range(p.nelz + 1):
            for iy in range(p.nely + 1):
                n = _node(p, 0, iy, iz)
                m[d * n:d * n + 3] = 1
    else:
        raise ValueError(p.support)
    return m


def load_vector(p: Problem) -> np.ndarray:
    """float64 [n_dof] nodal forces."""
    f = np.zeros(p.n_dof, dtype=np.float64)
    d = p.dim
    a = _anchor(p)
    if p.support == "mbb":
        f[d * _node(p, 0, p.nely - a) + 1] = -1.0      # unit downward load near the top-left corner
    elif p.support == "cantilever":
        f[d * _node(p, p.nelx, a) + 1] = -1.0          # unit downward load near the bottom-right corner
    elif p.support == "cantilever3d":
        share = -1.0 / (p.nely + 1)                    # unit total -z load on the edge x = L, z = a
        for iy in range(p.nely + 1):
            f[d * _node(p, p.nelx, iy, a) + 2] = share
    else:
        raise ValueError(p.support)
    return f


# ----------------------------------------------------------------------------
# Raw design fields (before any filtering or projection)
# ----------------------------------------------------------------------------

def connected_cell(rng, c, ones, bar):
    """Seeded 0/1 unit cell of c x c elements with exactly `ones` solid elements,
    connected within the cell and to its periodic neighbours.

    Starts from a cross of bars of width `bar` through the cell centre (the
    cross microstructure of the paper's Sec. 3.1 test problem; tiled crosses
    join at the cell edges) and grows solid at random frontier elements (edge
    neighbours inside the cell) until `ones` elements are solid. The paper's
    microstructures are connected by construction (Sec. 1, Sec. 4.5); a
    pixel-random pattern would fall apart into islands held only by void.
    """
    cell = np.zeros((c, c), dtype=np.float64)
    lo = (c - bar) // 2
    cell[lo:lo + bar, :] = 1.0
    cell[:, lo:lo + bar] = 1.0
    if cell.sum() > ones:
        raise ValueError("cross alone exceeds the requested solid count")
    while cell.sum() < ones:
        solid = np.pad(cell > 0, 1)
        nb = (solid[:-2, 1:-1] | solid[2:, 1:-1] | solid[1:-1, :-2] |
              solid[1:-1, 2:]) & ~(cell > 0)
        cand = np.flatnonzero(nb.ravel())
        cell.ravel()[cand[rng.integers(cand.size)]] = 1.0
    return cell


def design_field(p: Problem) -> np.ndarray:
    """float64 [n_el] design densities in [0, 1] for problem p (seeded)."""
    rng = np.random.default_rng(p.seed)
    if p.density == "tiled01":
        c = p.extra["cell"]
        cell = connected_cell(rng, c, c * c // 2, bar=2)
        ey, ex = np.meshgrid(np.arange(p.nely), np.arange(p.nelx), indexing="ij")
        return cell[ey % c, ex % c].ravel().astype(np.float64)
    if p.density == "modulated":
        c = p.extra["cell"]
        cell = connected_cell(rng, c, c * c // 2, bar=4)
        ks = [(a, b) for b in range(3) for a in range(3) if (a, b) != (0, 0)]
        pick = rng.choice(len(ks), 4, replace=False)
        amp = rng.uniform(0.5, 1.0, 4)
        phase = rng.uniform(0.0, 2 * np.pi, 4)
        ey, ex = np.meshgrid(np.arange(p.nely), np.arange(p.nelx), indexing="ij")
        xs = (ex + 0.5) / p.nelx
        ys = (ey + 0.5) / p.nely
        s = np.zeros_like(xs)
        for q in range(4):
            kx, ky = ks[pick[q]]
            s += amp[q] * np.cos(2 * np.pi * (kx * xs + ky * ys) + phase[q])
        m = 0.85 + 0.15 * s / amp.sum()                # smooth field in [0.7, 1]
        return (cell[ey % c, ex % c] * m).ravel().astype(np.float64)
    if p.density == "layered":
        c = p.extra["cell"]
        holes = [rng.integers(0, c - 3 + 1, 3) for _ in range(3)]
        void = np.zeros((c, c, c), dtype=bool)          # [z][y][x] within a cell
        for (hx, hy, hz) in holes:
            void[hz:hz + 3, hy:hy + 3, hx:hx + 3] = True
        ez, ey, ex = np.meshgrid(np.arange(p.nelz), np.arange(p.nely),
                                 np.arange(p.nelx), indexing="ij")
        rho = ((ez // 4) % 2 == 0).astype(np.float64)
        rho[void[ez % c, ey % c, ex % c]] = 0.0
        return rho.ravel()
    if p.density == "uniform_random":
        return rng.uniform(0.2, 0.9, p.n_el)
    raise ValueError(p.density)


def with_density(p: Problem, density: str, seed: int | None = None) -> Problem:
    """Copy of p with another density recipe (used by small test meshes)."""
    from dataclasses import replace
    return replace(p, density=density, seed=p.seed if seed is None else seed)


# ----------------------------------------------------------------------------
# Serving stream: arrivals and design updates (synthetic stand-ins for the
# optimiser's requests; no part of the method)
# ----------------------------------------------------------------------------

SERVING_MESHES_2D = [(256, 128), (512, 256), (1024, 512), (2048, 1024), (4096, 3072)]
SERVING_MESHES_3D = [(48, 48, 48), (96, 48, 48)]


def serving_requests(n: int, rate_per_s: float, seed: int = 1005, with_3d: bool = True):
    """n requests with Poisson arrivals (exponential gaps at rate_per_s): list
    of (arrival time in s, Problem). Meshes uniformly from the 2D set (32 x 32
    cells, k = 6, filtered and projected designs, 3 realisations) and, with
    with_3d, the 3D set (16^3 cells, layered design, one realisation)."""
    rng = np.random.default_rng(seed)
    choices = [("2d", m) for m in SERVING_MESHES_2D]
    if with_3d:
        choices += [("3d", m) for m in SERVING_MESHES_3D]
    t = 0.0
    out = []
    for i in range(n):
        t += rng.exponential(1.0 / rate_per_s)
        kind, m = choices[rng.integers(len(choices))]
        if kind == "2d":
            p = cantilever2d(m[0], m[1], 32, 6, name=f"req{i}_cantilever2d_{m[0]}x{m[1]}")
        else:
            p = cantilever3d(m[0], m[1], m[2], 16, 16, name=f"req{i}_cantilever3d_{m[0]}x{m[1]}x{m[2]}")
        out.append((t, p))
    return out


def design_noise(p: Problem, step: int, seed: int) -> np.ndarray:
    """A smooth seeded field in [-1, 1] per element: the direction of a
    synthetic design update (rho <- clip(rho + 0.02 noise, 0, 1))."""
    rng = np.random.default_rng((seed, step))
    dims = (p.nelx, p.nely) if p.dim == 2 else (p.nelx, p.nely, p.nelz)
    grids = np.meshgrid(*[(np.arange(n) + 0.5) / n for n in dims[::-1]], indexing="ij")
    xs = [g.ravel() for g in grids[::-1]]
    s = np.zeros(p.n_el)
    amp = rng.uniform(0.5, 1.0, 4)
    for q in range(4):
        k = rng.integers(0, 3, p.dim)
        ph = rng.uniform(0.0, 2 * np.pi)
        s += amp[q] * np.cos(2 * np.pi * sum(k[a] * xs[a] for a in range(p.dim)) + ph)
    return s / amp.sum()
