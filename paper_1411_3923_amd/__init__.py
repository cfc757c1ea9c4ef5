"""tpcg: spectral two-level PCG for SIMP elasticity on AMD MI355X.

Thin ctypes binding of libtpcg.so (C-ABI declared in include/tpcg.h). The
binding only marshals arguments: every step of the computation runs in the
library's HIP kernels. PyTorch provides device memory and the stream.
"""
from __future__ import annotations

import ctypes
import os

__all__ = ["Problem", "Handle", "Server", "TpcgError", "load_library", "FP64", "MIXED"]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libtpcg.so")
_lib = None

FP64 = 0
MIXED = 1
PC_ADDITIVE = 0   # tpcg_precond_kind
PC_MSFEM_SGS = 1

STATUS = {0: "OK", 1: "ENOCONV", 2: "EAGAIN", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ENOTSPD",
          -5: "EBREAKDOWN", -6: "ESTATE"}


class TpcgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"tpcg error {STATUS.get(code, code)}: {msg}")
        self.code = code


class Problem(ctypes.Structure):
    """Mirror of tpcg_problem."""
    _fields_ = [("dim", ctypes.c_int32), ("nel", ctypes.c_int32 * 3),
                ("E0", ctypes.c_double), ("Emin", ctypes.c_double),
                ("penal", ctypes.c_double), ("nu", ctypes.c_double),
                ("sub", ctypes.c_int32 * 3), ("overlap", ctypes.c_int32),
                ("ncoarse", ctypes.c_int32), ("nsys_max", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("eig_iters", ctypes.c_int32),
                ("eig_extra", ctypes.c_int32), ("eig_shift", ctypes.c_double),
                ("lambda_thresh", ctypes.c_double), ("coarse_dense_max", ctypes.c_int32),
                ("big_min_nb", ctypes.c_int32), ("coarse_band", ctypes.c_int32),
                ("dedup", ctypes.c_int32)]


class Info(ctypes.Structure):
    """Mirror of tpcg_info."""
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32),
                ("relres", ctypes.c_double), ("true_relres", ctypes.c_double),
                ("seconds", ctypes.c_double)]


class JobOpts(ctypes.Structure):
    """Mirror of tpcg_job_opts."""
    _fields_ = [("rtol", ctypes.c_double), ("maxit", ctypes.c_int32), ("rebuild", ctypes.c_int32),
                ("growth", ctypes.c_double), ("rmin", ctypes.c_double), ("beta", ctypes.c_double),
                ("eta", ctypes.c_double * 4), ("rep", ctypes.c_int32), ("refactor", ctypes.c_int32)]


class JobResult(ctypes.Structure):
    """Mirror of tpcg_job_result."""
    _fields_ = [("status_all", ctypes.c_int32), ("iters", ctypes.c_int32 * 4),
                ("status", ctypes.c_int32 * 4), ("relres", ctypes.c_double * 4),
                ("true_relres", ctypes.c_double * 4), ("rebuilt", ctypes.c_int32),
                ("refactored", ctypes.c_int32), ("rebuilds", ctypes.c_int32), ("queue_ms", ctypes.c_double),
                ("build_ms", ctypes.c_double), ("solve_ms", ctypes.c_double),
                ("total_ms", ctypes.c_double), ("m_nd", ctypes.c_double)]


EXPORTS = ["tpcg_build_partition", "tpcg_workspace_bytes", "tpcg_build_coarse_basis",
           "tpcg_apply_K", "tpcg_apply_precond", "tpcg_pcg_solve",
           "tpcg_compliance_and_sensitivity", "tpcg_filter_project",
           "tpcg_filter_project_adjoint", "tpcg_export_coarse_basis", "tpcg_query",
           "tpcg_set_profiling", "tpcg_profile_block_solves", "tpcg_export_eigenvalues",
           "tpcg_query_subspace", "tpcg_test_fail_alloc", "tpcg_last_error", "tpcg_destroy",
           "tpcg_compliance_and_sensitivity_noalloc", "tpcg_set_graphs",
           "tpcg_last_solve_graph_chunks", "tpcg_robust_objective", "tpcg_periodic_sum",
           "tpcg_nondiscreteness", "tpcg_refactor", "tpcg_export_local_record", "tpcg_server_create", "tpcg_server_session_bytes",
           "tpcg_server_open", "tpcg_server_submit", "tpcg_server_wait", "tpcg_server_test",
           "tpcg_server_close", "tpcg_server_free_bytes", "tpcg_server_destroy",
           "tpcg_apply_msfem", "tpcg_gmres_solve", "tpcg_set_autotune", "tpcg_query_tune",
           "tpcg_query_unique_cells", "tpcg_pcg_solve_async"]


def load_library(path: str | None = None):
    """Load libtpcg.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or _LIB_PATH
    if not os.path.exists(p):
        raise ImportError(f"{p} is missing: build it with `python -m paper_1411_3923_amd.build`")
    lib = ctypes.CDLL(p)
    P, I32, D, V = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_void_p
    lib.tpcg_build_partition.argtypes = [ctypes.POINTER(Problem), P, V, ctypes.POINTER(P)]
    lib.tpcg_workspace_bytes.argtypes = [ctypes.POINTER(Problem), I32]
    lib.tpcg_workspace_bytes.restype = ctypes.c_size_t
    lib.tpcg_build_coarse_basis.argtypes = [P, P, I32, I32]
    lib.tpcg_apply_K.argtypes = [P, P, P, P, I32]
    lib.tpcg_apply_precond.argtypes = [P, P, P, I32]
    lib.tpcg_pcg_solve.argtypes = [P, P, P, P, I32, D, I32, ctypes.POINTER(Info)]
    lib.tpcg_apply_msfem.argtypes = [P, P, P, P, I32]
    lib.tpcg_pcg_solve_async.argtypes = [P, P, P, P, I32, D, I32, P]
    lib.tpcg_set_autotune.argtypes = [P, I32]
    lib.tpcg_query_unique_cells.argtypes = [P]
    lib.tpcg_query_tune.argtypes = [P, ctypes.POINTER(I32)]
    lib.tpcg_gmres_solve.argtypes = [P, P, P, P, I32, D, I32, I32, I32, ctypes.POINTER(Info)]
    lib.tpcg_compliance_and_sensitivity.argtypes = [P, P, P, P, I32, P, P]
    lib.tpcg_filter_project.argtypes = [P, P, D, D, ctypes.POINTER(D), I32, P, P]
    lib.tpcg_filter_project_adjoint.argtypes = [P, P, D, D, ctypes.POINTER(D), I32, P, P]
    lib.tpcg_export_coarse_basis.argtypes = [P, P, P, P]
    lib.tpcg_query.argtypes = [P, ctypes.POINTER(ctypes.c_int64)]
    lib.tpcg_set_profiling.argtypes = [P, I32]
    lib.tpcg_profile_block_solves.argtypes = [P, ctypes.POINTER(D)]
    lib.tpcg_export_eigenvalues.argtypes = [P, P, I32, P]
    lib.tpcg_query_subspace.argtypes = [P]
    lib.tpcg_test_fail_alloc.argtypes = [I32]
    lib.tpcg_test_fail_alloc.restype = None
    lib.tpcg_last_error.argtypes = [P]
    lib.tpcg_last_error.restype = ctypes.c_char_p
    lib.tpcg_destroy.argtypes = [P]
    lib.tpcg_destroy.restype = None
    lib.tpcg_set_graphs.argtypes = [P, I32]
    lib.tpcg_nondiscreteness.argtypes = [P, P, P]
    lib.tpcg_refactor.argtypes = [P, P, I32]
    lib.tpcg_export_local_record.argtypes = [P, I32, I32, I32, P]
    I64 = ctypes.c_int64
    lib.tpcg_server_create.argtypes = [ctypes.c_size_t, I32, ctypes.POINTER(P)]
    lib.tpcg_server_session_bytes.argtypes = [ctypes.POINTER(Problem), I32]
    lib.tpcg_server_session_bytes.restype = ctypes.c_size_t
    lib.tpcg_server_open.argtypes = [P, ctypes.POINTER(Problem), P, I32, ctypes.POINTER(I64)]
    lib.tpcg_server_submit.argtypes = [P, I64, P, P, P, P, P, ctypes.POINTER(JobOpts),
                                       ctypes.POINTER(I64)]
    lib.tpcg_server_wait.argtypes = [P, I64, ctypes.POINTER(JobResult)]
    lib.tpcg_server_test.argtypes = [P, I64, ctypes.POINTER(JobResult)]
    lib.tpcg_server_close.argtypes = [P, I64]
    lib.tpcg_server_free_bytes.argtypes = [P]
    lib.tpcg_server_free_bytes.restype = ctypes.c_size_t
    lib.tpcg_server_destroy.argtypes = [P]
    lib.tpcg_server_destroy.restype = None
    lib.tpcg_robust_objective.argtypes = [P, P, P, I32, D, ctypes.POINTER(D), P, P]
    lib.tpcg_periodic_sum.argtypes = [P, P, I32, ctypes.POINTER(I32), P]
    lib.tpcg_last_solve_graph_chunks.argtypes = [P]
    lib.tpcg_compliance_and_sensitivity_noalloc.argtypes = [ctypes.POINTER(Problem), P, P, P, P,
                                                            I32, P, P, P, V]
    for name in EXPORTS:
        getattr(lib, name)
    if path is None:
        _lib = lib
    return lib


def make_problem(dim, nel, sub, ncoarse, nsys_max=1, E0=1.0, Emin=1e-9, penal=3.0, nu=0.3,
                 precision=FP64, eig_iters=0, eig_extra=0, eig_shift=0.0, lambda_thresh=0.0,
                 coarse_dense_max=0, overlap=1, big_min_nb=0, dedup=0, coarse_band=0) -> Problem:
    """tpcg_problem; `sub` is the subdomain edge (an int) or a per-axis tuple."""
    pr = Problem()
    pr.dim = dim
    nel = tuple(nel) + (1,) * (3 - len(nel))
    pr.nel[0], pr.nel[1], pr.nel[2] = nel[0], nel[1], nel[2] if dim == 3 else 1
    pr.E0, pr.Emin, pr.penal, pr.nu = E0, Emin, penal, nu
    subs = tuple(sub) if isinstance(sub, (tuple, list)) else (sub,) * dim
    subs = subs + (subs[-1],) * (3 - len(subs))
    pr.sub[0], pr.sub[1], pr.sub[2] = subs[0], subs[1], subs[2]
    pr.overlap, pr.ncoarse, pr.nsys_max = overlap, ncoarse, nsys_max
    pr.precision, pr.eig_iters, pr.eig_extra, pr.eig_shift = precision, eig_iters, eig_extra, eig_shift
    pr.lambda_thresh, pr.coarse_dense_max = lambda_thresh, coarse_dense_max
    pr.big_min_nb = big_min_nb
    pr.dedup = dedup
    pr.coarse_band = coarse_band
    return pr


def _ptr(t, dtype=None, n=None):
    """Device pointer of a contiguous CUDA tensor (argument checks only)."""
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected dtype {dtype}, got {t.dtype}")
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


class Handle:
    """Owns a tpcg_handle: partition, preconditioner and workspace on one GPU."""

    def __init__(self, problem: Problem, fixed_mask, stream=None):
        import numpy as np
        import torch
        self.lib = load_library()
        self.problem = problem
        fm = np.ascontiguousarray(np.asarray(fixed_mask, dtype=np.uint8))
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        h = ctypes.c_void_p()
        rc = self.lib.tpcg_build_partition(ctypes.byref(problem), fm.ctypes.data_as(ctypes.c_void_p),
                                           ctypes.c_void_p(self._stream.cuda_stream), ctypes.byref(h))
        if rc != 0:
            raise TpcgError(rc, "tpcg_build_partition failed (see stderr)")
        self.h = h
        q = (ctypes.c_int64 * 9)()
        self.lib.tpcg_query(self.h, q)
        (self.n_dof, self.n_el, self.n_sub, self.n_loc, self.k, self.nb, self.nblk,
         self.nbc, self.nblkc) = list(q)

    def _check(self, rc, allow_warn=False):
        if rc < 0 or (rc > 0 and not allow_warn):
            raise TpcgError(rc, self.lib.tpcg_last_error(self.h).decode())
        return rc

    def close(self):
        if getattr(self, "h", None):
            self.lib.tpcg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def build_coarse_basis(self, rho_phys, rep=0):
        import torch
        nsys = rho_phys.numel() // self.n_el
        return self._check(self.lib.tpcg_build_coarse_basis(
            self.h, _ptr(rho_phys, torch.float64, nsys * self.n_el), nsys, rep))

    def export_local_record(self, sys, sub, blk):
        """Dense C_b of the HBM-resident local factors (testing)."""
        import numpy as np
        out = np.zeros((self.nb, self.nb))
        self._check(self.lib.tpcg_export_local_record(self.h, sys, sub, blk,
                                                      out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def refactor(self, rho_phys):
        import torch
        nsys = rho_phys.numel() // self.n_el
        return self._check(self.lib.tpcg_refactor(self.h, _ptr(rho_phys, torch.float64, nsys * self.n_el), nsys))

    def apply_K(self, rho_phys, x, y):
        import torch
        nsys = x.numel() // self.n_dof
        self._check(self.lib.tpcg_apply_K(self.h, _ptr(rho_phys, torch.float64, nsys * self.n_el),
                                          _ptr(x, torch.float64, nsys * self.n_dof),
                                          _ptr(y, torch.float64, nsys * self.n_dof), nsys))
        return y

    def apply_precond(self, r, z):
        import torch
        nsys = r.numel() // self.n_dof
        self._check(self.lib.tpcg_apply_precond(self.h, _ptr(r, torch.float64, nsys * self.n_dof),
                                                _ptr(z, torch.float64, nsys * self.n_dof), nsys))
        return z

    def pcg_solve(self, rho_phys, f, u, rtol=1e-8, maxit=1000):
        import torch
        nsys = f.numel() // self.n_dof
        info = (Info * nsys)()
        rc = self.lib.tpcg_pcg_solve(self.h, _ptr(rho_phys, torch.float64, nsys * self.n_el),
                                     _ptr(f, torch.float64, nsys * self.n_dof),
                                     _ptr(u, torch.float64, nsys * self.n_dof), nsys, rtol, maxit,
                                     info)
        self._check(rc, allow_warn=True)
        return [dict(iters=i.iters, status=i.status, relres=i.relres,
                     true_relres=i.true_relres, seconds=i.seconds) for i in info]

    def unique_cells(self):
        """Local eigenproblems solved by the last basis build."""
        return self.lib.tpcg_query_unique_cells(self.h)

    def set_autotune(self, on=True):
        self._check(self.lib.tpcg_set_autotune(self.h, 1 if on else 0))

    def query_tune(self):
        out = (ctypes.c_int32 * 8)()
        self._check(self.lib.tpcg_query_tune(self.h, out))
        keys = ("on", "pcg_decided", "from_cache", "graphs", "poll", "gmres_decided",
                "gmres_chunk", "solves_measured")
        return dict(zip(keys, list(out)))

    def apply_msfem(self, rho_phys, r, z):
        """z = B r with the MsFEM cycle between symmetric Gauss-Seidel steps."""
        import torch
        nsys = r.numel() // self.n_dof
        self._check(self.lib.tpcg_apply_msfem(self.h, _ptr(rho_phys, torch.float64, nsys * self.n_el),
                                              _ptr(r, torch.float64, nsys * self.n_dof),
                                              _ptr(z, torch.float64, nsys * self.n_dof), nsys))
        return z

    def gmres_solve(self, rho_phys, f, u, rtol=1e-8, maxit=1000, restart=50, precond=PC_MSFEM_SGS):
        import torch
        nsys = f.numel() // self.n_dof
        info = (Info * nsys)()
        rc = self.lib.tpcg_gmres_solve(self.h, _ptr(rho_phys, torch.float64, nsys * self.n_el),
                                       _ptr(f, torch.float64, nsys * self.n_dof),
                                       _ptr(u, torch.float64, nsys * self.n_dof), nsys, rtol, maxit,
                                       restart, precond, info)
        self._check(rc, allow_warn=True)
        return [dict(iters=i.iters, status=i.status, relres=i.relres,
                     true_relres=i.true_relres, seconds=i.seconds) for i in info]

    def pcg_solve_async(self, rho_phys, f, u, info_dev, rtol=1e-8, maxit=1000):
        """Enqueue the solve; per-system results go to info_dev (a device
        uint8 tensor of nsys * sizeof(Info) bytes, read with read_info)."""
        import torch
        nsys = f.numel() // self.n_dof
        if info_dev.numel() < nsys * ctypes.sizeof(Info) or info_dev.device.type != "cuda":
            raise ValueError("info_dev: device tensor of nsys * sizeof(Info) bytes")
        rc = self.lib.tpcg_pcg_solve_async(self.h, _ptr(rho_phys, torch.float64, nsys * self.n_el),
                                           _ptr(f, torch.float64, nsys * self.n_dof),
                                           _ptr(u, torch.float64, nsys * self.n_dof), nsys, rtol,
                                           maxit, ctypes.c_void_p(info_dev.data_ptr()))
        self._check(rc)

    @staticmethod
    def read_info(info_dev, nsys):
        """Per-system results written by pcg_solve_async (synchronises)."""
        raw = bytes(info_dev.cpu().numpy().tobytes())[: nsys * ctypes.sizeof(Info)]
        info = (Info * nsys).from_buffer_copy(raw)
        return [dict(iters=i.iters, status=i.status, relres=i.relres,
                     true_relres=i.true_relres, seconds=i.seconds) for i in info]

    def compliance_and_sensitivity(self, rho_phys, u, f, c, dc=None):
        import torch
        nsys = u.numel() // self.n_dof
        self._check(self.lib.tpcg_compliance_and_sensitivity(
            self.h, _ptr(rho_phys, torch.float64, nsys * self.n_el),
            _ptr(u, torch.float64, nsys * self.n_dof), _ptr(f, torch.float64, nsys * self.n_dof),
            nsys, _ptr(c, torch.float64, nsys),
            _ptr(dc, torch.float64, nsys * self.n_el) if dc is not None else None))
        return c, dc

    def filter_project(self, rho, rmin, beta, etas, rho_tilde, rho_phys):
        import torch
        nsys = len(etas)
        eta = (ctypes.c_double * nsys)(*etas)
        self._check(self.lib.tpcg_filter_project(
            self.h, _ptr(rho, torch.float64, self.n_el), rmin, beta, eta, nsys,
            _ptr(rho_tilde, torch.float64, self.n_el), _ptr(rho_phys, torch.float64, nsys * self.n_el)))
        return rho_tilde, rho_phys

    def filter_project_adjoint(self, rho_tilde, rmin, beta, etas, dc_drho_phys, dc_drho):
        import torch
        nsys = len(etas)
        eta = (ctypes.c_double * nsys)(*etas)
        self._check(self.lib.tpcg_filter_project_adjoint(
            self.h, _ptr(rho_tilde, torch.float64, self.n_el), rmin, beta, eta, nsys,
            _ptr(dc_drho_phys, torch.float64, nsys * self.n_el),
            _ptr(dc_drho, torch.float64, nsys * self.n_el)))
        return dc_drho

    def robust_objective(self, c, out3, dc=None, df=None, kappa=1.0, weights=None):
        import torch
        nsys = c.numel()
        w = (ctypes.c_double * nsys)(*weights) if weights is not None else None
        self._check(self.lib.tpcg_robust_objective(
            self.h, _ptr(c, torch.float64, nsys),
            _ptr(dc, torch.float64, nsys * self.n_el) if dc is not None else None, nsys, kappa, w,
            _ptr(out3, torch.float64, 3), _ptr(df, torch.float64, self.n_el) if df is not None else None))
        return out3, df

    def periodic_sum(self, g, cell, gcell):
        import torch
        nsys = g.numel() // self.n_el
        cl = tuple(cell) + (1,) * (3 - len(cell))
        cv = (ctypes.c_int32 * 3)(*cl)
        self._check(self.lib.tpcg_periodic_sum(self.h, _ptr(g, torch.float64, nsys * self.n_el), nsys,
                                               cv, _ptr(gcell, torch.float64)))
        return gcell

    def set_graphs(self, on=True):
        self._check(self.lib.tpcg_set_graphs(self.h, 1 if on else 0))

    def last_graph_chunks(self):
        return int(self.lib.tpcg_last_solve_graph_chunks(self.h))

    def set_profiling(self, on=True):
        self._check(self.lib.tpcg_set_profiling(self.h, 1 if on else 0))

    def profile_block_solves(self):
        out = (ctypes.c_double * 3)()
        self._check(self.lib.tpcg_profile_block_solves(self.h, out))
        return dict(launches=int(out[0]), ms=out[1], bytes=out[2])

    def export_eigenvalues(self, m=None):
        """Ritz values [n_sub][m] (m defaults to the subspace width) and the
        coarse vectors in use per subdomain."""
        import numpy as np
        msub = self.lib.tpcg_query_subspace(self.h)
        m = msub if m is None else m
        lam = np.zeros((self.n_sub, m))
        kj = np.zeros(self.n_sub, dtype=np.int32)
        self._check(self.lib.tpcg_export_eigenvalues(self.h, lam.ctypes.data_as(ctypes.c_void_p), m,
                                                     kj.ctypes.data_as(ctypes.c_void_p)))
        return lam, kj

    def export_coarse_basis(self):
        import numpy as np
        import torch
        phi = torch.empty(self.n_sub * self.n_loc * self.k, dtype=torch.float64, device="cuda")
        lam = np.zeros((self.n_sub, self.k))
        res = np.zeros((self.n_sub, self.k))
        self._check(self.lib.tpcg_export_coarse_basis(
            self.h, _ptr(phi), lam.ctypes.data_as(ctypes.c_void_p), res.ctypes.data_as(ctypes.c_void_p)))
        return phi.view(self.n_sub, self.n_loc, self.k), lam, res


def compliance_and_sensitivity_noalloc(problem: Problem, fixed, rho_phys, u, f, c, dc=None,
                                       status=None, stream=None):
    """tpcg_compliance_and_sensitivity_noalloc: no handle, no device allocation.
    `fixed` is the support mask as a uint8 device tensor [n_dof]; `status`
    (an int32 device tensor of one element, optional) receives 1 for an
    invalid density. Returns the status code of the call."""
    import torch
    lib = load_library()
    nsys = c.numel()
    n_dof = fixed.numel()
    n_el = rho_phys.numel() // max(nsys, 1)
    st = stream if stream is not None else torch.cuda.current_stream()
    rc = lib.tpcg_compliance_and_sensitivity_noalloc(
        ctypes.byref(problem), _ptr(fixed, torch.uint8), _ptr(rho_phys, torch.float64, nsys * n_el),
        _ptr(u, torch.float64, nsys * n_dof), _ptr(f, torch.float64, nsys * n_dof), nsys,
        _ptr(c, torch.float64, nsys), _ptr(dc, torch.float64, nsys * n_el) if dc is not None else None,
        _ptr(status, torch.int32, 1) if status is not None else None, ctypes.c_void_p(st.cuda_stream))
    return rc


def _result(r: JobResult, nsys: int) -> dict:
    return dict(status_all=r.status_all, iters=list(r.iters)[:nsys], status=list(r.status)[:nsys],
                relres=list(r.relres)[:nsys], true_relres=list(r.true_relres)[:nsys],
                rebuilt=bool(r.rebuilt), refactored=bool(r.refactored), rebuilds=r.rebuilds, queue_ms=r.queue_ms,
                build_ms=r.build_ms, solve_ms=r.solve_ms, total_ms=r.total_ms, m_nd=r.m_nd)


class Server:
    """Owns a tpcg_server: sessions admitted by device-memory budget, one
    worker thread and stream per session, jobs = warm-started design updates."""

    def __init__(self, budget_bytes: int, max_active: int = 8):
        self.lib = load_library()
        s = ctypes.c_void_p()
        rc = self.lib.tpcg_server_create(int(budget_bytes), int(max_active), ctypes.byref(s))
        if rc != 0:
            raise TpcgError(rc, "tpcg_server_create failed")
        self.s = s
        self._nsys = {}
        self._jobs = {}

    def session_bytes(self, problem: Problem, nsys: int) -> int:
        return int(self.lib.tpcg_server_session_bytes(ctypes.byref(problem), nsys))

    def free_bytes(self) -> int:
        return int(self.lib.tpcg_server_free_bytes(self.s))

    def open(self, problem: Problem, fixed_mask, nsys: int):
        """Session id, or None when the budget or the session cap is full."""
        import numpy as np
        fm = np.ascontiguousarray(np.asarray(fixed_mask, dtype=np.uint8))
        sid = ctypes.c_int64()
        rc = self.lib.tpcg_server_open(self.s, ctypes.byref(problem), fm.ctypes.data_as(ctypes.c_void_p),
                                       nsys, ctypes.byref(sid))
        if rc == 2:
            return None
        if rc != 0:
            raise TpcgError(rc, "tpcg_server_open failed (see stderr)")
        self._nsys[sid.value] = (nsys, problem)
        return sid.value

    def submit(self, session, rho, f, u, c, dc=None, rtol=1e-8, maxit=2000, rebuild=0,
               growth=1.5, rmin=0.0, beta=8.0, etas=(0.5,), rep=0, refactor=True) -> int:
        import torch
        nsys, pr = self._nsys[session]
        o = JobOpts()
        o.rtol, o.maxit, o.rebuild, o.growth = rtol, maxit, rebuild, growth
        o.rmin, o.beta, o.rep, o.refactor = rmin, beta, rep, 1 if refactor else 0
        for i, e in enumerate(tuple(etas)[:4]):
            o.eta[i] = e
        job = ctypes.c_int64()
        rc = self.lib.tpcg_server_submit(self.s, session, _ptr(rho, torch.float64), _ptr(f, torch.float64),
                                         _ptr(u, torch.float64), _ptr(c, torch.float64, nsys),
                                         _ptr(dc, torch.float64) if dc is not None else None,
                                         ctypes.byref(o), ctypes.byref(job))
        if rc != 0:
            raise TpcgError(rc, "tpcg_server_submit failed")
        self._jobs[job.value] = nsys
        return job.value

    def wait(self, job) -> dict:
        r = JobResult()
        rc = self.lib.tpcg_server_wait(self.s, job, ctypes.byref(r))
        if rc != 0:
            raise TpcgError(rc, "tpcg_server_wait failed")
        return _result(r, self._jobs.pop(job))

    def test(self, job):
        r = JobResult()
        rc = self.lib.tpcg_server_test(self.s, job, ctypes.byref(r))
        if rc == 2:
            return None
        if rc != 0:
            raise TpcgError(rc, "tpcg_server_test failed")
        return _result(r, self._jobs.pop(job))

    def close(self, session):
        rc = self.lib.tpcg_server_close(self.s, session)
        self._nsys.pop(session, None)
        if rc != 0:
            raise TpcgError(rc, "tpcg_server_close failed")

    def destroy(self):
        if getattr(self, "s", None):
            self.lib.tpcg_server_destroy(self.s)
            self.s = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass
