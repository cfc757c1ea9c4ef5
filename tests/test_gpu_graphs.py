"""PCG chunks replayed from HIP graphs against eager launches: the same
kernels with the same arguments (the iteration index read from the device
counter instead of the launch), so results must agree bit for bit. Each
solve replays its graphs many times with eager work (polls, copies, host
synchronisation) between the replays; the graphs are kept across solves with
the same arguments and captured again when the arguments change."""
import numpy as np
import pytest

from oracle import density, fem
from paper_1411_3923_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1411_3923_amd as T  # noqa: E402
from tests.gpu_common import dev, handle, host, rel  # noqa: E402


def problems():
    c = W.cantilever2d(128, 64, 16, 6)
    _, rb = density.filter_project(c, W.design_field(c), c.rmin, c.beta, c.etas)
    m = W.mbb_64x32()
    t = W.cantilever3d(12, 6, 6, sub=3, k=6)
    return [("cantilever", c, rb), ("mbb", m, W.design_field(m)[None, :]),
            ("3d", t, W.design_field(t)[None, :])]


@pytest.mark.parametrize("precision", [T.FP64, T.MIXED], ids=["fp64", "mixed"])
@pytest.mark.parametrize("case", range(3), ids=["cantilever", "mbb", "3d"])
def test_graph_replay_matches_eager(case, precision):
    name, p, rb = problems()[case]
    n = rb.shape[0]
    f = np.stack([W.load_vector(p)] * n)
    h = handle(p, precision=precision, nsys=n)
    h.build_coarse_basis(dev(rb), rep=0)
    R, F = dev(rb), dev(f)

    def solve(graphs, prof=False):
        h.set_graphs(graphs)
        h.set_profiling(prof)
        u = dev(np.zeros((n, p.n_dof)))
        info = h.pcg_solve(R, F, u, rtol=1e-10, maxit=3000)
        return host(u), info, h.last_graph_chunks(), h.profile_block_solves()

    ue, ie, ce, _ = solve(False)
    assert ce == 0
    for rep in range(3):
        ug, ig, cg, prof = solve(True)
        print(f"{name} {'fp64' if precision == T.FP64 else 'mixed'} replay {rep}: "
              f"iters {[i['iters'] for i in ig]} graph chunks {cg}", flush=True)
        assert cg > 0
        assert [i["iters"] for i in ig] == [i["iters"] for i in ie]
        np.testing.assert_array_equal(ug, ue)
        ue2, _, _, _ = solve(False)        # eager work between the replays
        np.testing.assert_array_equal(ue2, ue)
    # timing the local solves with events keeps the solve eager
    _, _, cp, prof = solve(True, prof=True)
    assert cp == 0 and prof["launches"] > 0 and prof["ms"] > 0.0
    h.set_profiling(False)
    tol = 1e-8 if precision == T.FP64 else 1e-6
    for s in range(n):
        assert rel(ug[s], fem.solve(p, rb[s])) < 100 * tol
    h.close()
