"""GPU robust objective (Sec. 4.4) and periodic sensitivity sum (Sec. 4.1)
against the oracle: on seeded inputs (element by element; both sides sum
the realisations in the same order, the copies in a different one:
bounds 1e-14 and 1e-12 relative), and through the whole robust step on a
cantilever (filter, three projections, three PCG solves to 1e-12, compliance,
sensitivities, chain rule, aggregation, periodic sum) against the oracle's
direct solves (bounds 1e-8 on the objective, 1e-6 on the gradient)."""
import numpy as np
import pytest

from oracle import density, fem
from paper_1411_3923_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from tests.gpu_common import dev, handle, host  # noqa: E402


@pytest.mark.parametrize("kappa,weights", [(1.0, None), (0.5, (0.2, 0.5, 0.3))])
def test_robust_objective_matches_oracle(kappa, weights):
    p = W.cantilever2d(128, 64, 16, 6)
    h = handle(p)
    rng = np.random.default_rng(21)
    c = rng.uniform(100.0, 200.0, 3)
    dc = rng.standard_normal((3, p.n_el))
    out = dev(np.zeros(3))
    df = dev(np.zeros(p.n_el))
    h.robust_objective(dev(c), out, dev(dc), df, kappa=kappa, weights=weights)
    f_o, m_o, s_o, df_o = density.robust_objective(c, dc, kappa, weights)
    o = host(out)
    np.testing.assert_allclose(o, [f_o, m_o, s_o], rtol=1e-15)
    np.testing.assert_allclose(host(df), df_o, rtol=1e-14, atol=1e-14 * np.abs(df_o).max())
    # equal realisations: no variance term
    h.robust_objective(dev(np.full(3, 5.0)), out, dev(dc), df)
    np.testing.assert_allclose(host(out), [5.0, 5.0, 0.0])
    np.testing.assert_allclose(host(df), dc.mean(axis=0), rtol=1e-14, atol=1e-15)
    h.close()


@pytest.mark.parametrize("dim,cell", [(2, (16, 16)), (2, (5, 3)), (3, (4, 3, 2))])
def test_periodic_sum_matches_oracle(dim, cell):
    p = W.cantilever2d(128, 64, 16, 6) if dim == 2 else W.cantilever3d(12, 6, 6, sub=3, k=6)
    h = handle(p)
    g = np.random.default_rng(22).standard_normal((2, p.n_el))
    n = int(np.prod(cell[:dim]))
    out = dev(np.zeros((2, n)))
    h.periodic_sum(dev(g), cell, out)
    for s in range(2):
        want = density.periodic_sum(p, g[s], cell)
        np.testing.assert_allclose(host(out)[s], want, rtol=1e-12, atol=1e-12 * np.abs(want).max())
    h.close()


def test_robust_step_matches_oracle():
    p = W.cantilever2d(128, 64, 16, 6)
    rho = W.design_field(p)
    f = W.load_vector(p)
    cell = (16, 16)
    # oracle: direct solves
    rt, rb = density.filter_project(p, rho, p.rmin, p.beta, p.etas)
    us = [fem.solve(p, rb[s]) for s in range(3)]
    c_o = np.array([fem.compliance(f, u) for u in us])
    dcb = np.stack([fem.sensitivity(p, rb[s], us[s]) for s in range(3)])
    dc_o = density.filter_project_adjoint(p, rt, p.rmin, p.beta, p.etas, dcb)
    f_o, _, _, df_o = density.robust_objective(c_o, dc_o)
    g_o = density.periodic_sum(p, df_o, cell)
    # GPU
    h = handle(p)
    R = dev(rho)
    RT, RB = dev(np.zeros(p.n_el)), dev(np.zeros((3, p.n_el)))
    h.filter_project(R, p.rmin, p.beta, p.etas, RT, RB)
    h.build_coarse_basis(RB, rep=0)
    F = dev(np.stack([f] * 3))
    u = dev(np.zeros((3, p.n_dof)))
    info = h.pcg_solve(RB, F, u, rtol=1e-12, maxit=3000)
    assert all(i["status"] == 0 for i in info)
    c = dev(np.zeros(3))
    dcb_g = dev(np.zeros((3, p.n_el)))
    h.compliance_and_sensitivity(RB, u, F, c, dcb_g)
    dc_g = dev(np.zeros((3, p.n_el)))
    h.filter_project_adjoint(RT, p.rmin, p.beta, p.etas, dcb_g, dc_g)
    out, df = dev(np.zeros(3)), dev(np.zeros(p.n_el))
    h.robust_objective(c, out, dc_g, df)
    gc = dev(np.zeros(256))
    h.periodic_sum(df, cell, gc)
    fo = host(out)
    e_f = abs(fo[0] - f_o) / abs(f_o)
    e_g = float(np.linalg.norm(host(gc) - g_o) / np.linalg.norm(g_o))
    print(f"robust step: objective {e_f:.3e} periodic gradient {e_g:.3e} "
          f"(std/mean {fo[2] / fo[1]:.3f})", flush=True)
    assert e_f < 1e-8 and e_g < 1e-6
    h.close()
