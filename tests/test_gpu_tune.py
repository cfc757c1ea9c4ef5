"""The autotuner changes launches only: every candidate it tries gives the
same bits as the fixed configuration, its choice is stored in the on-disk
cache, and a new handle of the same problem takes the stored choice."""
import numpy as np
import pytest

from paper_1411_3923_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1411_3923_amd as T  # noqa: E402
from tests.gpu_common import dev, handle, host  # noqa: E402


def built(p, rb, tune):
    h = handle(p)
    if tune:
        h.set_autotune(True)
    h.build_coarse_basis(dev(rb), rep=0)
    return h


def setup():
    p = W.cantilever2d(128, 64, 16, 6)
    from oracle import density
    _, rb = density.filter_project(p, W.design_field(p), p.rmin, p.beta, p.etas)
    F = dev(np.stack([W.load_vector(p)] * 3))
    return p, rb, F


def test_pcg_tuning_bitwise_neutral_and_cached(tmp_path, monkeypatch):
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("TPCG_TUNE_CACHE", str(cache))
    p, rb, F = setup()
    h0 = built(p, rb, False)
    u0 = dev(np.zeros((3, p.n_dof)))
    ref = h0.pcg_solve(dev(rb), F, u0, rtol=1e-8)
    want = host(u0)
    h1 = built(p, rb, True)
    for _ in range(10):
        u = dev(np.zeros((3, p.n_dof)))
        info = h1.pcg_solve(dev(rb), F, u, rtol=1e-8)
        assert [i["iters"] for i in info] == [i["iters"] for i in ref]
        assert np.array_equal(host(u), want)
    st = h1.query_tune()
    assert st["pcg_decided"] == 1 and st["from_cache"] == 0 and st["solves_measured"] == 9, st
    assert st["poll"] in (4, 8)
    assert "|pcg\t" in cache.read_text()
    h2 = built(p, rb, True)
    u = dev(np.zeros((3, p.n_dof)))
    h2.pcg_solve(dev(rb), F, u, rtol=1e-8)
    assert np.array_equal(host(u), want)
    st2 = h2.query_tune()
    assert st2["pcg_decided"] == 1 and st2["from_cache"] == 1, st2
    assert (st2["graphs"], st2["poll"]) == (st["graphs"], st["poll"])


def test_gmres_tuning_bitwise_neutral_and_cached(tmp_path, monkeypatch):
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("TPCG_TUNE_CACHE", str(cache))
    p, rb, F = setup()
    h0 = built(p, rb, False)
    u0 = dev(np.zeros((3, p.n_dof)))
    h0.gmres_solve(dev(rb), F, u0, rtol=1e-8, restart=30)
    h1 = built(p, rb, True)
    u1 = dev(np.zeros((3, p.n_dof)))
    h1.gmres_solve(dev(rb), F, u1, rtol=1e-8, restart=30)
    assert np.array_equal(host(u1), host(u0))
    st = h1.query_tune()
    assert st["gmres_decided"] == 1 and st["gmres_chunk"] in (4, 8, 16), st
    assert "|gmres\t" in cache.read_text()
