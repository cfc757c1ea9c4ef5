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


def gpu_basis(h, p):
    """The handle's exported coarse basis as a sparse [n_dof][n_sub k] matrix
    (subdomain j's column block j, its box DOFs in the handle's local order)."""
    import scipy.sparse as sp
    from oracle import schwarz
    phi = host(h.export_coarse_basis()[0])
    k = phi.shape[2]
    rows, cols, vals = [], [], []
    for j in range(p.n_sub):
        nodes = schwarz.subdomain_nodes(p, j)
        dofs = (p.dim * nodes[:, None] + np.arange(p.dim)[None, :]).ravel()
        for m in range(k):
            rows.append(dofs)
            cols.append(np.full(dofs.size, j * k + m))
            vals.append(phi[j][:, m])
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(p.n_dof, p.n_sub * k)).tocsc()
