"""Shared helpers of the GPU parity tests: problem set-up through the C-ABI
binding and the matching oracle objects. Inputs come from the seeded
generators only; nothing here computes a part of the method."""
import numpy as np
import torch

import paper_1411_3923_amd as T
from paper_1411_3923_amd import workloads as W


def problem_struct(p, precision=T.FP64, nsys=None, **kw):
    return T.make_problem(p.dim, p.nel[:p.dim], p.sub, p.k, nsys or p.nsys, p.E0, p.Emin,
                          p.penal, p.nu, precision, **kw)


def handle(p, precision=T.FP64, nsys=None, **kw):
    return T.Handle(problem_struct(p, precision, nsys, **kw), W.fixed_mask(p))


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))
