"""The entry point without device allocation
(tpcg_compliance_and_sensitivity_noalloc) against the handle-based
tpcg_compliance_and_sensitivity it mirrors: both run the same kernels on the
same inputs, so c and dc must agree bit for bit. Two calls in a row on one
device share the library's scratch array; the second uses a smaller input
(fewer systems, a smaller mesh) and must not see the first's contents.
"""
import numpy as np
import pytest

from paper_1411_3923_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_1411_3923_amd as T  # noqa: E402
from tests.gpu_common import dev, handle, host, problem_struct  # noqa: E402


def inputs(p, nsys, seed):
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.05, 1.0, (nsys, p.n_el))
    u = rng.standard_normal((nsys, p.n_dof))
    f = rng.standard_normal((nsys, p.n_dof))
    return rho, u, f


def reference(p, nsys, rho, u, f):
    h = handle(p, nsys=nsys)
    c = dev(np.zeros(nsys))
    dc = dev(np.zeros((nsys, p.n_el)))
    h.compliance_and_sensitivity(dev(rho), dev(u), dev(f), c, dc)
    out = host(c), host(dc)
    h.close()
    return out


def noalloc(p, nsys, rho, u, f, with_dc=True):
    pr = problem_struct(p, nsys=nsys)
    fixed = torch.as_tensor(W.fixed_mask(p).astype(np.uint8), device="cuda")
    c = dev(np.full(nsys, np.nan))
    dc = dev(np.full((nsys, p.n_el), np.nan)) if with_dc else None
    status = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    rc = T.compliance_and_sensitivity_noalloc(pr, fixed, dev(rho), dev(u), dev(f), c, dc, status)
    assert rc == 0
    return host(c), (host(dc) if with_dc else None), int(host(status)[0])


CASES = [
    # (first call, second call): the second input is smaller
    ((W.cantilever2d(128, 64, 32, 6), 3), (W.mbb_64x32(), 1)),
    ((W.cantilever3d(24, 12, 12, 4, 4), 2), (W.cantilever3d(12, 6, 6, 3, 4), 1)),
]


@pytest.mark.parametrize("case", range(len(CASES)), ids=["2d", "3d"])
def test_noalloc_matches_handle_entry_point(case):
    for i, (p, nsys) in enumerate(CASES[case]):
        rho, u, f = inputs(p, nsys, 40 + 7 * case + i)
        c_ref, dc_ref = reference(p, nsys, rho, u, f)
        c, dc, st = noalloc(p, nsys, rho, u, f)
        print(f"case {case} call {i}: mesh {p.nel[:p.dim]} nsys {nsys}", flush=True)
        assert st == 0
        np.testing.assert_array_equal(c, c_ref)
        np.testing.assert_array_equal(dc, dc_ref)
        c2, _, _ = noalloc(p, nsys, rho, u, f, with_dc=False)
        np.testing.assert_array_equal(c2, c_ref)


def test_noalloc_flags_invalid_density_and_rejects_sizes():
    p = W.mbb_64x32()
    rho, u, f = inputs(p, 1, 3)
    rho[0, 17] = 1.5
    _, _, st = noalloc(p, 1, rho, u, f)
    assert st == 1
    rho[0, 17] = 0.5
    _, _, st = noalloc(p, 1, rho, u, f)
    assert st == 0
    pr = problem_struct(p, nsys=1)
    fixed = torch.as_tensor(W.fixed_mask(p).astype(np.uint8), device="cuda")
    c = dev(np.zeros(5))
    rc = T.compliance_and_sensitivity_noalloc(pr, fixed, dev(np.tile(rho, (5, 1))),
                                              dev(np.tile(u, (5, 1))), dev(np.tile(f, (5, 1))), c)
    assert rc == -1
