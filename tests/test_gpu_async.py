"""The asynchronous PCG solve (the serving path's form of the boundary's
solve): enqueued with no host wait, its per-system results in device
memory, bit for bit those of the synchronous solve."""
import ctypes

import numpy as np
import pytest

from paper_1411_3923_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1411_3923_amd as T  # noqa: E402
from tests.gpu_common import dev, handle, host  # noqa: E402


@pytest.mark.parametrize("precision", [T.FP64, T.MIXED], ids=["fp64", "mixed"])
def test_async_solve_equals_sync(precision):
    p = W.cantilever2d(128, 64, 16, 6)
    from oracle import density
    _, rb = density.filter_project(p, W.design_field(p), p.rmin, p.beta, p.etas)
    h = handle(p, precision=precision)
    h.build_coarse_basis(dev(rb), rep=0)
    F = dev(np.stack([W.load_vector(p)] * 3))
    u0 = dev(np.zeros((3, p.n_dof)))
    ref = h.pcg_solve(dev(rb), F, u0, rtol=1e-8, maxit=400)
    u1 = dev(np.zeros((3, p.n_dof)))
    info = torch.zeros(3 * ctypes.sizeof(T.Info), dtype=torch.uint8, device="cuda")
    h.pcg_solve_async(dev(rb), F, u1, info, rtol=1e-8, maxit=400)
    got = T.Handle.read_info(info, 3)
    assert np.array_equal(host(u1), host(u0))
    for a, b in zip(got, ref):
        assert (a["iters"], a["status"]) == (b["iters"], b["status"])
        assert a["relres"] == b["relres"] and a["true_relres"] == b["true_relres"]
    # maxit reached: ENOCONV in the record, the iterate of the steps taken
    u2 = dev(np.zeros((3, p.n_dof)))
    h.pcg_solve_async(dev(rb), F, u2, info, rtol=1e-8, maxit=10)
    got = T.Handle.read_info(info, 3)
    assert all(i["iters"] == 10 and i["status"] == 1 for i in got), got
