"""The coarse level as the HBM-resident block-tridiagonal factorisation
(coarse spaces too large for a dense inverse whose blocks do not fit the
on-chip factor kernels; Sec. 2.4 coarse projection equation): its coarse
solve against the dense inverse, against the oracle's preconditioner on the
GPU's own basis, and PCG against the direct solve, in 2-d and 3-d."""
import dataclasses

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fem, schwarz
from paper_1411_3923_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1411_3923_amd as T  # noqa: E402
from tests.gpu_common import dev, gpu_basis, handle, host, rel  # noqa: E402


def residual(p, seed):
    rng = np.random.default_rng(seed)
    r = rng.standard_normal(p.n_dof)
    r[W.fixed_mask(p) == 1] = 0.0
    return r


def oracle_precond(h, p, rho, r):
    """The oracle's local solves plus Phi (Phi^T K Phi)^-1 Phi^T r on the GPU's basis."""
    fixed = W.fixed_mask(p)
    K = fem.assemble(p, fem.simp_modulus(rho, p.E0, p.Emin, p.penal))
    z = schwarz.TwoLevelSchwarz(p, K, fixed, None).apply(r)
    Phi = gpu_basis(h, p)
    P = sp.diags((fixed == 0).astype(np.float64))
    Kc = (Phi.T @ (P @ K @ P) @ Phi).toarray()
    return z + P @ (Phi @ np.linalg.solve(Kc, Phi.T @ (P @ r)))


CASES = {
    # forced on the MBB beam (coarse blocks of 16, 8 block rows)
    "mbb_forced": (lambda: W.mbb_64x32(), dict(coarse_band=1)),
    # odd coarse blocks (5 vectors x 5 cells = 25) beyond a small dense limit:
    # the path the layout takes by itself
    "odd_blocks": (lambda: dataclasses.replace(W.mbb_64x32(), nel=(96, 40, 1), k=5,
                                               name="mbb_96x40"), dict(coarse_dense_max=64)),
    # 3-d, forced (blocks of 4 cells x 6 vectors)
    "h8_forced": (lambda: W.cantilever3d(12, 6, 6, sub=3, k=6), dict(coarse_band=1)),
}


@pytest.mark.parametrize("name", list(CASES))
def test_band_coarse_level_matches_oracle(name):
    mk, kw = CASES[name]
    p = mk()
    print(f"band {name}", flush=True)
    rho = W.design_field(p)
    h = handle(p, nsys=1, **kw)
    h.build_coarse_basis(dev(rho[None, :]), rep=0)
    r = residual(p, 13)
    z = dev(np.zeros(p.n_dof))
    h.apply_precond(dev(r), z)
    want = oracle_precond(h, p, rho, r)
    got = host(z)
    assert np.max(np.abs(got - want)) <= 1e-10 * np.max(np.abs(want))
    u = dev(np.zeros(p.n_dof))
    info = h.pcg_solve(dev(rho[None, :]), dev(W.load_vector(p)[None, :]), u, rtol=1e-12,
                       maxit=3000)[0]
    assert info["status"] == 0
    assert rel(host(u), fem.solve(p, rho)) < 1e-8


def test_band_equals_dense_inverse_three_systems():
    # the same basis and local factors: the two exact coarse solves agree to rounding
    p = W.cantilever2d(128, 64, 16, 6)
    from oracle import density
    _, rb = density.filter_project(p, W.design_field(p), p.rmin, p.beta, p.etas)
    out = []
    for kw in ({}, dict(coarse_band=1)):
        h = handle(p, **kw)
        h.build_coarse_basis(dev(rb), rep=0)
        r = np.stack([residual(p, 20 + s) for s in range(3)])
        z = dev(np.zeros_like(r))
        h.apply_precond(dev(r), z)
        out.append(host(z))
        F = dev(np.stack([W.load_vector(p)] * 3))
        u = dev(np.zeros((3, p.n_dof)))
        info = h.pcg_solve(dev(rb), F, u, rtol=1e-8)
        out.append([i["iters"] for i in info])
    assert np.max(np.abs(out[0] - out[2])) <= 1e-11 * np.max(np.abs(out[0]))
    assert all(abs(a - b) <= 1 for a, b in zip(out[1], out[3])), (out[1], out[3])
