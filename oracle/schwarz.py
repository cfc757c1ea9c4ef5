"""Oracle: spectral coarse space and two-level additive Schwarz PCG.

Test infrastructure only (see the package docstring).

Sources in the paper:
* Sec. 2.4: the fine mesh refines a coarse mesh of unit cells; each coarse
  region carries local generalised eigenproblems K_w psi = lambda M_w psi
  (discrete eigenproblem equation) whose local matrices keep the physical
  boundary conditions; the eigenvectors of the smallest eigenvalues, times a
  partition of unity, are the coarse basis functions phi; R_c^T stacks them;
  K_c = R_c K R_c^T (coarse projection equation).
* Sec. 3.2: the weighting matrix M_w is diag(K_w).
* Sec. 2.4.2: the coarse space is used inside a preconditioner for a Krylov
  method; the system and the preconditioner are symmetric positive definite,
  so PCG applies; the cited two-level additive Schwarz form is used here.

Readings taken where the paper is silent (each also listed in the design notes):
* Subdomains are the s^d-element unit cells. The unknowns of subdomain j are
  the free DOFs of the nodes of its closed cell (one element layer of overlap:
  the local Dirichlet problem lives on the cell grown by one element, with
  zero displacement on the grown boundary).
* Local solve matrix A_j: the principal submatrix of the global constrained K
  on those DOFs (it includes stiffness from the elements of the overlap ring).
* Eigenproblem matrix K_j^N: assembled from the cell's own elements only
  (natural boundary conditions on the artificial boundary, physical supports
  kept); weighting D_j = diag(K_j^N).
* A fixed number k of eigenvectors per subdomain (smallest eigenvalues).
* Partition of unity chi_j(n) = 1 / (number of subdomains containing node n).
* M^-1 = sum_j R_j^T A_j^-1 R_j + R_c^T K_c^-1 R_c.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import fem


# ---------------------------------------------------------------------------
# Partition (Sec. 2.4: coarse cells = unit cells of s^d elements)
# ---------------------------------------------------------------------------

def subdomain_grid(p):
    s = p.sub
    if p.nelx % s or p.nely % s or (p.dim == 3 and p.nelz % s):
        raise ValueError("mesh size must be a multiple of the subdomain size")
    return (p.nelx // s, p.nely // s) + ((p.nelz // s,) if p.dim == 3 else ())


def subdomain_nodes(p, j):
    """Global nodes of the closed cell of subdomain j (x fastest)."""
    g = subdomain_grid(p)
    s = p.sub
    nx, ny = p.nelx + 1, p.nely + 1
    jx = j % g[0]
    jy = (j // g[0]) % g[1]
    ix = np.arange(s * jx, s * jx + s + 1)
    iy = np.arange(s * jy, s * jy + s + 1)
    if p.dim == 2:
        Y, X = np.meshgrid(iy, ix, indexing="ij")
        return (X + nx * Y).ravel()
    jz = j // (g[0] * g[1])
    iz = np.arange(s * jz, s * jz + s + 1)
    Z, Y, X = np.meshgrid(iz, iy, ix, indexing="ij")
    return (X + nx * (Y + ny * Z)).ravel()


def subdomain_elements(p, j):
    """Elements inside the cell of subdomain j."""
    g = subdomain_grid(p)
    s = p.sub
    jx = j % g[0]
    jy = (j // g[0]) % g[1]
    ex = np.arange(s * jx, s * jx + s)
    ey = np.arange(s * jy, s * jy + s)
    if p.dim == 2:
        Y, X = np.meshgrid(ey, ex, indexing="ij")
        return (X + p.nelx * Y).ravel()
    jz = j // (g[0] * g[1])
    ez = np.arange(s * jz, s * jz + s)
    Z, Y, X = np.meshgrid(ez, ey, ex, indexing="ij")
    return (X + p.nelx * (Y + p.nely * Z)).ravel()


def subdomain_dofs(p, j, fixed):
    """Free global DOFs of subdomain j, in local order (node x fastest, then component)."""
    nodes = subdomain_nodes(p, j)
    dofs = (p.dim * nodes[:, None] + np.arange(p.dim)[None, :]).ravel()
    return dofs[np.asarray(fixed)[dofs] == 0]


def partition_of_unity(p):
    """chi(n) = 1 / multiplicity(n): the same weight for every subdomain containing n."""
    mult = np.zeros(p.nnodes)
    for j in range(p.n_sub):
        mult[subdomain_nodes(p, j)] += 1.0
    return 1.0 / mult


# ---------------------------------------------------------------------------
# Local eigenproblems (Sec. 2.4 discrete eigenproblem; Sec. 3.2 diag weighting)
# ---------------------------------------------------------------------------

def local_eigenpairs(p, E_rep, fixed, j, k, K0=None, method="dense"):
    """k smallest eigenpairs of K_j^N psi = lambda diag(K_j^N) psi (D-orthonormal psi).

    method "dense": LAPACK's generalised symmetric eigensolver on the dense
    matrices. method "sparse" (large cells): ARPACK in shift-invert mode on
    S = D^-1/2 K_j^N D^-1/2, whose eigenvalues are the same, shifted just
    below zero so that S - sigma I is definite for floating cells, with
    psi = D^-1/2 x; the same definition, for cells too large for a dense
    eigensolver.
    """
    dofs = subdomain_dofs(p, j, fixed)
    KN = fem.assemble(p, E_rep, K0, elements=subdomain_elements(p, j))
    KN = KN[dofs][:, dofs]
    if method == "sparse":
        import scipy.sparse.linalg as spla
        d = KN.diagonal()
        Dh = sp.diags(1.0 / np.sqrt(d))
        S = (Dh @ KN @ Dh).tocsc()
        lam, x = spla.eigsh(S, k=k, sigma=-1e-6, which="LM", tol=1e-13)
        order = np.argsort(lam)
        lam, x = lam[order], x[:, order]
        return lam, x / np.sqrt(d)[:, None], dofs
    KN = KN.toarray()
    D = np.diag(np.diag(KN))
    lam, psi = sla.eigh(KN, D, subset_by_index=[0, k - 1])
    return lam, psi, dofs


def unique_cells(p, E_rep, fixed):
    """Subdomains whose local eigenproblems are the same matrices (Sec. 2.4:
    periodic microstructures repeat the same agglomerate): equal moduli of the
    cell's elements in cell order and equal supports of the box DOFs in box
    order. Returns rep [J], the first subdomain with the same data, for each."""
    seen, rep = {}, []
    for j in range(p.n_sub):
        nodes = subdomain_nodes(p, j)
        dofs = (p.dim * nodes[:, None] + np.arange(p.dim)[None, :]).ravel()
        key = (np.asarray(E_rep)[subdomain_elements(p, j)].tobytes(),
               np.asarray(fixed)[dofs].tobytes())
        rep.append(seen.setdefault(key, j))
    return np.array(rep)


def coarse_basis(p, E_rep, fixed, k, K0=None, thresh=0.0, method="dense", dedup=False):
    """Global Phi = R_c^T (sparse) and the per-subdomain eigenvalues.

    thresh <= 0: the k smallest eigenvectors of every subdomain (n_dof x J*k).
    thresh > 0: Sec. 2.4's global threshold, the eigenvectors whose
    eigenvalue lies below thresh, at most k per subdomain; Phi then has
    sum_j k_j columns in subdomain order. Returns (Phi, lams [J][k], kj [J]).
    dedup: solve each distinct eigenproblem once (unique_cells) and give its
    eigenpairs to every subdomain with the same matrices; the partition of
    unity is still that of each subdomain.
    """
    chi = partition_of_unity(p)
    rows, cols, vals, lams, kj = [], [], [], [], []
    col = 0
    rep = unique_cells(p, E_rep, fixed) if dedup else np.arange(p.n_sub)
    solved = {}
    for j in range(p.n_sub):
        if rep[j] not in solved:
            solved[rep[j]] = local_eigenpairs(p, E_rep, fixed, rep[j], k, K0, method)[:2]
        lam, psi = solved[rep[j]]
        dofs = subdomain_dofs(p, j, fixed)
        use = k if thresh <= 0 else int(np.sum(lam < thresh))
        w = chi[dofs // p.dim]
        for m in range(use):
            rows.append(dofs)
            cols.append(np.full(dofs.size, col))
            vals.append(w * psi[:, m])
            col += 1
        lams.append(lam)
        kj.append(use)
    if col == 0:
        return sp.csc_matrix((p.n_dof, 0)), np.array(lams), np.array(kj)
    Phi = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                        shape=(p.n_dof, col)).tocsc()
    if thresh <= 0:
        return Phi, np.array(lams)
    return Phi, np.array(lams), np.array(kj)


# ---------------------------------------------------------------------------
# Two-level additive Schwarz preconditioner (Sec. 2.4.2)
# ---------------------------------------------------------------------------

class TwoLevelSchwarz:
    """M^-1 r = sum_j R_j^T A_j^-1 R_j r + Phi (Phi^T K Phi)^-1 Phi^T r.

    Built for one system (one stiffness K) with a coarse basis Phi that may come
    from another design (the robust formulation builds it from the dilated
    realisation, Sec. 5.3).
    """

    def __init__(self, p, K, fixed, Phi=None, local=True, banded=True):
        self.p = p
        self.fixed = np.asarray(fixed)
        self.local = []
        if local:
            Kc = fem.constrained(K, fixed)
            for j in range(p.n_sub):
                dofs = subdomain_dofs(p, j, fixed)
                A = Kc[dofs][:, dofs]
                if banded:
                    self.local.append((dofs, _BandedCholesky(A)))
                else:
                    self.local.append((dofs, _DenseCholesky(A.toarray())))
        self.Phi = Phi if (Phi is None or Phi.shape[1] > 0) else None
        if self.Phi is not None:
            Kc = (Phi.T @ (K @ Phi)).toarray()
            self.Kc = Kc
            self.Kc_chol = sla.cho_factor(Kc, lower=True)

    def apply(self, r):
        z = np.zeros_like(r)
        for dofs, fac in self.local:
            z[dofs] += fac.solve(r[dofs])
        if self.Phi is not None:
            yc = self.Phi.T @ r
            z += self.Phi @ sla.cho_solve(self.Kc_chol, yc)
        return z


class _DenseCholesky:
    def __init__(self, A):
        self.c = sla.cho_factor(A, lower=True)

    def solve(self, b):
        return sla.cho_solve(self.c, b)


class _BandedCholesky:
    """Cholesky of a sparse SPD matrix in LAPACK lower band storage."""

    def __init__(self, A):
        A = sp.csr_matrix(A)
        coo = A.tocoo()
        lower = coo.row >= coo.col
        bw = int(np.max(coo.row[lower] - coo.col[lower])) if lower.any() else 0
        n = A.shape[0]
        ab = np.zeros((bw + 1, n))
        r, c, v = coo.row[lower], coo.col[lower], coo.data[lower]
        np.add.at(ab, (r - c, c), v)
        self.cb = sla.cholesky_banded(ab, lower=True)

    def solve(self, b):
        return sla.cho_solve_banded((self.cb, True), b)


# ---------------------------------------------------------------------------
# Preconditioned conjugate gradients (Sec. 2.4.2: SPD system and preconditioner)
# ---------------------------------------------------------------------------

def pcg(matvec, precond, f, x0=None, rtol=1e-8, maxit=1000, callback=None):
    """Textbook PCG; stops when ||r||_2 <= rtol ||f||_2 on the recursive residual."""
    x = np.zeros_like(f) if x0 is None else np.array(x0, dtype=np.float64)
    r = f - matvec(x)
    fn = np.linalg.norm(f)
    if fn == 0.0:
        return x, 0, 0.0
    z = precond(r)
    pdir = z.copy()
    rz = float(r @ z)
    it = 0
    relres = np.linalg.norm(r) / fn
    while relres > rtol and it < maxit:
        q = matvec(pdir)
        alpha = rz / float(pdir @ q)
        x += alpha * pdir
        r -= alpha * q
        it += 1
        relres = np.linalg.norm(r) / fn
        if callback is not None:
            callback(it, x, relres)
        if relres <= rtol:
            break
        z = precond(r)
        rz_new = float(r @ z)
        pdir = z + (rz_new / rz) * pdir
        rz = rz_new
    return x, it, relres


def solve_pcg(p, rho_phys_sys, rho_rep, f, fixed, k=None, rtol=1e-8, maxit=1000,
              coarse=True, local=True, thresh=0.0, eig_method="dense"):
    """Oracle PCG for each system with the shared coarse basis from rho_rep
    (thresh > 0: the eigenvalue-threshold coarse space, at most k per cell)."""
    K0 = fem.element_K0(p.dim, p.nu)
    k = p.k if k is None else k
    Phi = None
    if coarse:
        E_rep = fem.simp_modulus(rho_rep, p.E0, p.Emin, p.penal)
        Phi = coarse_basis(p, E_rep, fixed, k, K0, thresh=thresh, method=eig_method)[0]
    out = []
    for rho in rho_phys_sys:
        E = fem.simp_modulus(rho, p.E0, p.Emin, p.penal)
        K = fem.assemble(p, E, K0)
        Kc = fem.constrained(K, fixed)
        M = TwoLevelSchwarz(p, K, fixed, Phi, local=local)
        free = (np.asarray(fixed) == 0)
        fp = np.where(free, f, 0.0)
        x, it, rr = pcg(lambda v: Kc @ v, M.apply, fp, rtol=rtol, maxit=maxit)
        out.append((x, it, rr))
    return out
