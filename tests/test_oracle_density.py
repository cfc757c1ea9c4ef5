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


def test_robust_objective_closed_forms():
    # equal compliances: f = c, variance 0; two-point spread: mean and std by hand
    f, m, s, df = density.robust_objective([2.0, 2.0, 2.0], np.ones((3, 4)))
    assert (f, m, s) == (2.0, 2.0, 0.0)
    np.testing.assert_allclose(df, np.ones(4))
    f, m, s, _ = density.robust_objective([1.0, 3.0], np.zeros((2, 1)), kappa=1.0)
    assert m == 2.0 and s == 1.0 and f == 3.0
    f, m, s, _ = density.robust_objective([1.0, 2.0, 6.0], np.zeros((3, 1)), kappa=0.5)
    assert m == 3.0 and abs(s - math.sqrt(14.0 / 3.0)) < 1e-15
    assert abs(f - (3.0 + 0.5 * math.sqrt(14.0 / 3.0))) < 1e-15


def test_robust_objective_gradient_matches_finite_differences():
    # f(c(x)) with smooth c_s(x): the gradient through the aggregation
    rng = np.random.default_rng(4)
    A = rng.standard_normal((3, 5))
    B = rng.standard_normal((3, 5))
    x = rng.standard_normal(5)
    cfun = lambda v: np.exp(0.3 * A @ v) + (B @ v) ** 2
    dcfun = lambda v: 0.3 * np.exp(0.3 * A @ v)[:, None] * A + 2 * (B @ v)[:, None] * B
    _, _, _, g = density.robust_objective(cfun(x), dcfun(x), kappa=1.0)
    h = 1e-6
    for i in range(5):
        e = np.zeros(5)
        e[i] = h
        fp = density.robust_objective(cfun(x + e), np.zeros((3, 1)))[0]
        fm = density.robust_objective(cfun(x - e), np.zeros((3, 1)))[0]
        assert abs((fp - fm) / (2 * h) - g[i]) < 1e-7 * max(1.0, abs(g[i]))


@pytest.mark.parametrize("dim", [2, 3])
def test_periodic_sum_is_the_adjoint_of_tiling(dim):
    p = prob(12, 8, 6, dim) if dim == 3 else prob(12, 8)
    cell = (4, 2, 3)
    n = int(np.prod(cell[:dim]))
    rng = np.random.default_rng(9)
    x = rng.standard_normal(n)
    g = rng.standard_normal(p.n_el)
    tiled, _ = density.tile_design(p, x, cell)
    # <g, T x> = <T^T g, x>, and the copies of one variable are summed
    assert abs(g @ tiled - density.periodic_sum(p, g, cell) @ x) < 1e-12 * np.abs(g).sum()
    ones = density.periodic_sum(p, np.ones(p.n_el), cell)
    np.testing.assert_array_equal(ones, np.full(n, p.n_el / n))


def test_robust_periodic_chain_matches_finite_differences():
    # the whole robust step on a tiny cantilever: periodic design variables ->
    # tiled element densities -> filter and three projections -> three solves
    # -> E[c] + sqrt(Var[c]); its gradient from the self-adjoint sensitivities,
    # the projection and filter chain rule, the robust aggregation and the
    # periodic sum, against central differences
    from oracle import fem
    p = W.Problem("t", 2, (6, 4, 1), sub=2, k=1, support="cantilever", density="uniform_random",
                  seed=3, rmin=1.6, beta=8.0, etas=(0.3, 0.5, 0.7), Emin=1e-3)
    cell = (3, 2)
    f = W.load_vector(p)
    x0 = np.random.default_rng(2).uniform(0.3, 0.8, 6)

    def objective(x):
        rho, _ = density.tile_design(p, x, cell)
        rt, rb = density.filter_project(p, rho, p.rmin, p.beta, p.etas)
        us = [fem.solve(p, rb[s]) for s in range(3)]
        c = np.array([fem.compliance(f, u) for u in us])
        dcb = np.stack([fem.sensitivity(p, rb[s], us[s]) for s in range(3)])
        dc = density.filter_project_adjoint(p, rt, p.rmin, p.beta, p.etas, dcb)
        val, _, _, g = density.robust_objective(c, dc)
        return val, density.periodic_sum(p, g, cell)

    _, grad = objective(x0)
    h = 1e-6
    for i in range(6):
        e = np.zeros(6)
        e[i] = h
        fd = (objective(x0 + e)[0] - objective(x0 - e)[0]) / (2 * h)
        assert abs(fd - grad[i]) < 1e-6 * max(1.0, abs(grad[i])), (i, fd, grad[i])
