"""The largest 2-d mesh of the serving stream: the 4096 x 3072 cantilever
(25.2M DOFs per system, three realisations, 12,288 cells of 32 x 32 and a
coarse space of 73,728 vectors on the HBM-resident block-tridiagonal coarse
factor). The counts equal those of the 1024 x 512 cantilever within the
mesh-sweep band, and the solution satisfies the oracle's element operator
on sections of the mesh (clamped edge, load, interior)."""
import numpy as np
import pytest

from oracle import fem
from paper_1411_3923_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from tests.gpu_common import dev, handle, host  # noqa: E402

C2_COUNTS = (91, 94, 138)   # the 1024 x 512 cantilever's counts (same cells, same k)


def section_residual(p, E, u, f, fixed, x0, y0, n=128):
    """||P (f - K u)|| over the nodes whose elements all lie in the window of
    n x n elements at (x0, y0): there K u is the window's own assembly."""
    ex, ey = np.meshgrid(np.arange(x0, x0 + n), np.arange(y0, y0 + n), indexing="xy")
    elems = (ex + p.nelx * ey).ravel()
    K = fem.assemble(p, E, elements=elems)
    ix = np.arange(x0 + (x0 > 0), x0 + n + 1 - (x0 + n < p.nelx))
    iy = np.arange(y0 + (y0 > 0), y0 + n + 1 - (y0 + n < p.nely))
    X, Y = np.meshgrid(ix, iy, indexing="xy")
    nodes = (X + (p.nelx + 1) * Y).ravel()
    dofs = (2 * nodes[:, None] + np.arange(2)[None, :]).ravel()
    dofs = dofs[fixed[dofs] == 0]
    return np.linalg.norm(f[dofs] - (K @ u)[dofs])


def test_cantilever_4096x3072():
    p = W.cantilever2d(4096, 3072)
    print("4096x3072: build", flush=True)
    h = handle(p)
    rt = dev(np.zeros(p.n_el))
    rb = dev(np.zeros((3, p.n_el)))
    h.filter_project(dev(W.design_field(p)), p.rmin, p.beta, p.etas, rt, rb)
    h.build_coarse_basis(rb, rep=0)
    f = W.load_vector(p)
    F = dev(np.stack([f] * 3))
    u = dev(np.zeros((3, p.n_dof)))
    print("4096x3072: solve", flush=True)
    info = h.pcg_solve(rb, F, u, rtol=1e-8, maxit=3000)
    assert all(i["status"] == 0 for i in info), info
    for i, c in zip(info, C2_COUNTS):
        assert abs(i["iters"] - c) <= 0.15 * c, (info, C2_COUNTS)
        assert i["true_relres"] <= 1.05e-8
    fixed = W.fixed_mask(p)
    fp = np.where(fixed == 0, f, 0.0)
    rbh, uh = host(rb), host(u)
    h.close()
    print("4096x3072: sections", flush=True)
    for s in range(3):
        E = fem.simp_modulus(rbh[s], p.E0, p.Emin, p.penal)
        for x0, y0 in ((0, 1472), (3968, 0), (2048, 1536)):
            res = section_residual(p, E, uh[s], f, fixed, x0, y0)
            assert res <= 1.05e-8 * np.linalg.norm(fp), (s, x0, y0, res)
