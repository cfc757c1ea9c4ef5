"""Oracle: the paper's own fine-scale solver (Sec. 2.4.2): the MsFEM coarse
solve, with one symmetric Gauss-Seidel smoothing step before and one after
it, used as the preconditioner of GMRES.

Test infrastructure only (see the package docstring): the product path never
imports this module.

What the paper fixes (Sec. 2.4.2): the fine-scale residual is restricted to
the coarse basis, the correction is computed by the MsFEM coarse solve
(K_c = Phi^T K Phi, Sec. 2.4 coarse projection equation) and prolonged back;
one pre- and one post-smoothing step of symmetric Gauss-Seidel surround it;
the whole is the preconditioner of GMRES. Convergence is measured by the
preconditioned residual relative to the preconditioned forcing vector
(Sec. 3.3, convergence study of the iteration counts).

Readings taken where the paper is silent (each also in the design notes):
* Gauss-Seidel acts on node blocks (the d x d block of a node's DOFs is
  solved exactly) in multicolour order: a node's colour is the parity of its
  grid coordinates, bit 0 for x, bit 1 for y, bit 2 for z (4 colours in 2-d,
  8 in 3-d). Two nodes of one colour never share an element, so the updates
  within a colour are independent. One symmetric step is a forward sweep
  over the colours in increasing order followed by a backward sweep in
  decreasing order.
* The cycle: x = S(r; 0); x += Phi K_c^-1 Phi^T (r - K x); x = S(r; x),
  S(r; x) one symmetric step on K x = r starting from x. The same
  symmetric smoother on both sides makes the preconditioner symmetric.
* GMRES is preconditioned from the left (so that its residual estimate is
  the preconditioned residual the paper's tolerance refers to), restarted
  every m steps; the Arnoldi vectors are orthogonalised by classical
  Gram-Schmidt applied twice; the small least-squares problem by Givens
  rotations. An iteration is one Arnoldi step.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import fem


def node_colours(p):
    """Colour of every node: parity of x, plus 2 x parity of y (plus 4 x parity of z)."""
    nx, ny = p.nelx + 1, p.nely + 1
    n = np.arange(p.nnodes)
    c = (n % nx) % 2 + 2 * ((n // nx) % ny % 2)
    if p.dim == 3:
        c = c + 4 * ((n // (nx * ny)) % 2)
    return c


class BlockSGS:
    """Node-block symmetric Gauss-Seidel in multicolour order on a constrained
    stiffness matrix K (fixed DOFs: identity rows and columns)."""

    def __init__(self, p, K):
        self.K = sp.csr_matrix(K)
        self.d = d = p.dim
        col = node_colours(p)
        self.groups = []
        for c in range(2 ** d):
            nodes = np.nonzero(col == c)[0]
            dofs = (d * nodes[:, None] + np.arange(d)[None, :]).ravel()
            # the d x d diagonal block of every node of the colour
            blk = np.empty((nodes.size, d, d))
            for a in range(d):
                for b in range(d):
                    blk[:, a, b] = np.asarray(self.K[d * nodes + a, d * nodes + b]).ravel()
            self.groups.append((dofs, self.K[dofs], np.linalg.inv(blk)))

    def _relax(self, group, r, x):
        dofs, Krows, Dinv = group
        t = (r[dofs] - Krows @ x).reshape(-1, self.d, 1)
        x[dofs] += (Dinv @ t).ravel()

    def step(self, r, x):
        """One symmetric step on K x = r from x (x is updated and returned)."""
        for g in self.groups:
            self._relax(g, r, x)
        for g in reversed(self.groups):
            self._relax(g, r, x)
        return x


class MsFEMCycle:
    """B r = S(r; Phi K_c^-1 Phi^T (r - K S(r; 0)) + S(r; 0)): the MsFEM coarse
    solve between one symmetric Gauss-Seidel step before and one after."""

    def __init__(self, p, K, fixed, Phi):
        self.K = fem.constrained(K, fixed)
        self.sgs = BlockSGS(p, self.K)
        self.Phi = sp.csc_matrix(Phi)
        Kc = (self.Phi.T @ (K @ self.Phi)).toarray()
        self.Kc_chol = sla.cho_factor(Kc, lower=True)

    def apply(self, r):
        x = self.sgs.step(r, np.zeros_like(r))
        t = r - self.K @ x
        x = x + self.Phi @ sla.cho_solve(self.Kc_chol, self.Phi.T @ t)
        return self.sgs.step(r, x)


def gmres(matvec, precond, f, x0=None, rtol=1e-8, restart=50, maxit=1000):
    """Left-preconditioned restarted GMRES.

    Stops when the preconditioned residual estimate falls to rtol times
    ||precond(f)||, or after maxit Arnoldi steps. Returns (x, iterations,
    estimated relative residual, history of the estimates)."""
    x = np.zeros_like(f) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.linalg.norm(precond(f))
    hist = []
    if bnorm == 0.0:
        return np.zeros_like(f), 0, 0.0, hist
    it = 0
    m = restart
    while True:
        r = precond(f - matvec(x))
        beta = np.linalg.norm(r)
        if beta <= rtol * bnorm or it >= maxit:
            return x, it, beta / bnorm, hist
        V = np.zeros((m + 1, f.size))
        V[0] = r / beta
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        done = False
        j = 0
        while j < m:
            w = precond(matvec(V[j]))
            Vj = V[: j + 1]
            h1 = Vj @ w
            w = w - Vj.T @ h1
            h2 = Vj @ w
            w = w - Vj.T @ h2
            H[: j + 1, j] = h1 + h2
            hn = np.linalg.norm(w)
            H[j + 1, j] = hn
            for i in range(j):   # earlier rotations
                a, b = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * b
                H[i + 1, j] = -sn[i] * a + cs[i] * b
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            j += 1
            rel = abs(g[j]) / bnorm
            hist.append(rel)
            if rel <= rtol or it >= maxit or hn == 0.0:
                done = True
                break
            V[j] = w / hn
        y = sla.solve_triangular(H[:j, :j], g[:j])
        x = x + V[:j].T @ y
        if done:
            return x, it, abs(g[j]) / bnorm, hist


def solve_gmres(p, rho_phys_sys, rho_rep, f, fixed, k=None, rtol=1e-8, restart=50,
                maxit=1000, precond="msfem", thresh=0.0, eig_method="dense", Phi=None):
    """GMRES for each system with the preconditioner `precond`: "msfem" (the
    cycle above) or "additive" (two-level additive Schwarz), on the shared
    coarse basis of rho_rep (or the given Phi)."""
    from . import schwarz
    K0 = fem.element_K0(p.dim, p.nu)
    k = p.k if k is None else k
    if Phi is None:
        E_rep = fem.simp_modulus(rho_rep, p.E0, p.Emin, p.penal)
        Phi = schwarz.coarse_basis(p, E_rep, fixed, k, K0, thresh=thresh, method=eig_method)[0]
    free = np.asarray(fixed) == 0
    fp = np.where(free, f, 0.0)
    out = []
    for rho in rho_phys_sys:
        E = fem.simp_modulus(rho, p.E0, p.Emin, p.penal)
        K = fem.assemble(p, E, K0)
        Kc = fem.constrained(K, fixed)
        if precond == "msfem":
            M = MsFEMCycle(p, K, fixed, Phi)
        else:
            M = schwarz.TwoLevelSchwarz(p, K, fixed, Phi)
        x, it, rr, _ = gmres(lambda v: Kc @ v, M.apply, fp, rtol=rtol, restart=restart,
                             maxit=maxit)
        out.append((x, it, rr))
    return out
