"""Host-only checks of the C-ABI library: it loads and exports every entry
point declared in include/tpcg.h, and its sizing/validation logic works
without a GPU (no compute call is made)."""
import ctypes
import os
import re

import pytest

import paper_1411_3923_amd as T

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "tpcg.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tpcg_[A-Za-z_]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = declared()
    for want in ["tpcg_build_partition", "tpcg_build_coarse_basis", "tpcg_apply_K",
                 "tpcg_apply_precond", "tpcg_pcg_solve", "tpcg_compliance_and_sensitivity"]:
        assert want in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(os.path.join(ROOT, "paper_1411_3923_amd", "libtpcg.so")):
        pytest.skip("libtpcg.so not built")
    lib = T.load_library()
    for name in declared():
        assert hasattr(lib, name), name
    assert sorted(declared()) == sorted(T.EXPORTS)


def test_workspace_sizing_and_validation_on_host():
    if not os.path.exists(os.path.join(ROOT, "paper_1411_3923_amd", "libtpcg.so")):
        pytest.skip("libtpcg.so not built")
    lib = T.load_library()
    ok = T.make_problem(2, (1024, 512), 32, 6, 3)
    n = lib.tpcg_workspace_bytes(ctypes.byref(ok), 3)
    # at least the tiled FP64 local factors (3 systems x 512 subdomains x 33
    # blocks x 153 lower 4x4 tiles of D_b) and the packed Neumann factors of
    # the eigensolver (512 x 33 records of 66 x (66 + 4) doubles)
    assert n > 3 * 512 * 33 * 153 * 16 * 8 + 512 * 33 * 66 * 70 * 8
    bad = T.make_problem(2, (100, 50), 32, 6, 3)      # not a multiple of the subdomain size
    assert lib.tpcg_workspace_bytes(ctypes.byref(bad), 3) == 0
    mixed = T.make_problem(2, (1024, 512), 32, 6, 3, precision=T.MIXED)
    # FP32 factors are kept; the FP64 factorisation runs one system at a time
    assert lib.tpcg_workspace_bytes(ctypes.byref(mixed), 3) < n


def test_build_partition_rejects_bad_problems_before_any_device_call():
    # the validation runs on the host before the handle touches the device,
    # so these calls are safe without a GPU
    if not os.path.exists(os.path.join(ROOT, "paper_1411_3923_amd", "libtpcg.so")):
        pytest.skip("libtpcg.so not built")
    import numpy as np
    lib = T.load_library()
    good = dict(dim=2, nel=(64, 32), sub=8, ncoarse=4, nsys_max=1)
    cases = [
        dict(good, nel=(60, 32)),                       # nel % sub != 0
        dict(good, dim=4),                              # dim not in {2, 3}
        dict(good, sub=(8, 4)),                         # non-square cells
        dict(good, ncoarse=0),                          # k < 1
        dict(good, ncoarse=17),                         # k above 16
        dict(good, nsys_max=5),                         # nsys_max above 4
        dict(good, nsys_max=0),
        dict(good, overlap=2),                          # overlap != 1
        dict(good, Emin=0.0),                           # Emin <= 0
        dict(good, nu=0.5),                             # nu outside (-1, 0.5)
        dict(good, penal=0.5),                          # penal < 1
        dict(good, lambda_thresh=float("nan")),
        dict(good, coarse_dense_max=-1),
        dict(good, dim=2, nel=(2, 2), sub=1, ncoarse=9),  # k above the subdomain's 8 DOFs
    ]
    for c in cases:
        kw = dict(c)
        dim, nel, sub, k, ns = kw.pop("dim"), kw.pop("nel"), kw.pop("sub"), kw.pop("ncoarse"), \
            kw.pop("nsys_max")
        pr = T.make_problem(dim, nel, sub, k, ns, **kw)
        nel3 = tuple(nel) + (1,)
        ndof = (dim if dim in (2, 3) else 2) * (nel3[0] + 1) * (nel3[1] + 1)
        mask = np.zeros(max(ndof, 1), dtype=np.uint8)
        h = ctypes.c_void_p()
        rc = lib.tpcg_build_partition(ctypes.byref(pr), mask.ctypes.data_as(ctypes.c_void_p), None,
                                      ctypes.byref(h))
        assert rc == -1, c
        assert not h.value
        assert lib.tpcg_workspace_bytes(ctypes.byref(pr), 1) == 0 or c.get("nsys_max") in (0, 5)
    # null arguments
    pr = T.make_problem(2, (64, 32), 8, 4, 1)
    h = ctypes.c_void_p()
    assert lib.tpcg_build_partition(None, None, None, ctypes.byref(h)) == -1
    assert lib.tpcg_build_partition(ctypes.byref(pr), None, None, ctypes.byref(h)) == -1
