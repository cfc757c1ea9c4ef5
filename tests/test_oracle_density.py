"""Pins for the oracle's density filter and Heaviside projection (paper
Sec. 4.3 neighbourhood filter and projection equation; Sec. 4.4 thresholds)."""
import math

import numpy as np
import pytest

from oracle import density
from paper_1411_3923_amd import workloads as W


def prob(nelx=9, nely=7, nelz=1, dim=2):
    return W.Problem("t", dim, (nelx, nely, nelz), sub=1, k=1, density="uniform_random", seed=5)


def brute_filter(p, rho, rmin):
    # explicit double loop over element pairs: the textbook definition
    dims = (p.nelx, p.nely, p.nelz)
    cen = [(x, y, z) for z in range(dims[2]) for y in range(dims[1]) for x in range(dims[0])]
    out = np.zeros(len(cen))
    for e, ce in enumerate(cen):
        num = den = 0.0
        for i, ci in enumerate(cen):
            w = rmin - math.dist(ce, ci)
            if w > 0:
                num += w * rho[i]
                den += w
        out[e] = num / den
    return out


@pytest.mark.parametrize("dim,rmin", [(2, 2.0), (2, 2.7), (3, 1.8)])
def test_filter_matches_brute_force(dim, rmin):
    p = prob(6, 5, 4, dim) if dim == 3 else prob()
    rho = W.design_field(p)
    np.testing.assert_allclose(density.filter_density(p, rho, rmin), brute_filter(p, rho, rmin),
                               rtol=1e-14, atol=1e-15)


def test_filter_special_cases():
    p = prob()
    rho = W.design_field(p)
    np.testing.assert_array_equal(density.filter_density(p, rho, 1.0), rho)   # rmin <= 1: identity
    np.testing.assert_allclose(density.filter_density(p, np.full(p.n_el, 0.37), 2.0), 0.37, rtol=1e-15)
    # interior hat weights at rmin = 2: 2 + 4 * 1 + 4 * (2 - sqrt 2)
    H = density.filter_matrix(p, 2.0)
    e = 3 + p.nelx * 3
    assert H[e, e] == pytest.approx(2.0 / (6.0 + 4.0 * (2.0 - math.sqrt(2.0))), rel=1e-15)
    assert 6.0 + 4.0 * (2.0 - math.sqrt(2.0)) == pytest.approx(8.343146, abs=1e-6)


def test_projection_closed_forms():
    H = density.heaviside
    assert H(0.0, 8.0, 0.3) == pytest.approx(0.0, abs=1e-15)
    assert H(1.0, 8.0, 0.7) == pytest.approx(1.0, abs=1e-15)
    assert H(0.5, 8.0, 0.5) == pytest.approx(0.5, abs=1e-15)
    t = math.tanh
    assert H(0.3, 8.0, 0.3) == pytest.approx(t(2.4) / (t(2.4) + t(5.6)), rel=1e-14)
    assert H(0.3, 8.0, 0.3) == pytest.approx(0.495892, abs=1e-6)
    assert H(0.5, 8.0, 0.3) == pytest.approx(0.960525, abs=1e-6)
    assert H(0.5, 8.0, 0.7) == pytest.approx(0.039475, abs=1e-6)
    x = np.linspace(0, 1, 11)
    np.testing.assert_allclose(H(x, 1e-7, 0.4), x, atol=1e-12)               # beta -> 0: identity
    h = 1e-6
    for eta in (0.3, 0.5, 0.7):
        fd = (H(x + h, 8.0, eta) - H(x - h, 8.0, eta)) / (2 * h)
        np.testing.assert_allclose(density.heaviside_derivative(x, 8.0, eta), fd, rtol=1e-7, atol=1e-9)


def test_adjoint_transpose_and_finite_differences():
    p = prob()
    rho = W.design_field(p)
    etas = (0.3, 0.5, 0.7)
    rt, rb = density.filter_project(p, rho, 2.0, 8.0, etas)
    rng = np.random.default_rng(1)
    g = rng.standard_normal((3, p.n_el))
    adj = density.filter_project_adjoint(p, rt, 2.0, 8.0, etas, g)
    # directional derivative of sum_s g_s . rho_bar_s equals adj . v
    v = rng.standard_normal(p.n_el)
    h = 1e-6
    _, bp = density.filter_project(p, rho + h * v, 2.0, 8.0, etas)
    _, bm = density.filter_project(p, rho - h * v, 2.0, 8.0, etas)
    for s in range(3):
        fd = g[s] @ (bp[s] - bm[s]) / (2 * h)
        assert adj[s] @ v == pytest.approx(fd, rel=1e-7)


def test_non_discreteness():
    assert density.non_discreteness(np.array([0.0, 1.0])) == 0.0
    assert density.non_discreteness(np.array([0.5, 0.5])) == 1.0
