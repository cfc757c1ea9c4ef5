"""Pins for the oracle of the paper's own solver (Sec. 2.4.2: the MsFEM coarse
solve between one symmetric Gauss-Seidel step before and one after, as the
preconditioner of GMRES; convergence in the preconditioned norm as in
Sec. 3.3)."""
import dataclasses

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import fem, msfem, schwarz
from paper_1411_3923_amd import workloads as W


def mbb(nelx=16, nely=8, sub=4, k=3, Emin=1e-9):
    p = W.mbb_64x32()
    return dataclasses.replace(p, nel=(nelx, nely, 1), sub=sub, k=k, Emin=Emin)


def small3d(Emin=1e-9):
    p = W.cantilever3d(8, 4, 4, sub=4, k=4)
    return dataclasses.replace(p, Emin=Emin)


def system(p, seed=3):
    rng = np.random.default_rng(seed)
    rho = np.clip(W.design_field(p) + 0.2 * rng.random(p.n_el), 0.0, 1.0)
    fixed = W.fixed_mask(p)
    E = fem.simp_modulus(rho, p.E0, p.Emin, p.penal)
    K = fem.assemble(p, E)
    return rho, fixed, E, K


def node_of_dof(p):
    return np.arange(p.n_dof) // p.dim


@pytest.mark.parametrize("kind", ["2d", "3d"])
def test_sgs_step_is_two_block_triangular_solves(kind):
    # One symmetric step equals x1 = x0 + (D + L)^-1 (r - K x0),
    # x2 = x1 + (D + U)^-1 (r - K x1), where D + L keeps the entries whose row
    # node has a higher colour than the column node or is the same node, and
    # D + U the mirror image: solved here by a general sparse LU on the whole
    # matrix, not colour by colour.
    p = mbb() if kind == "2d" else small3d()
    _, fixed, _, K = system(p)
    Kc = sp.csr_matrix(fem.constrained(K, fixed))
    col = msfem.node_colours(p)
    nd = node_of_dof(p)
    coo = Kc.tocoo()
    ci, cj = col[nd[coo.row]], col[nd[coo.col]]
    same = nd[coo.row] == nd[coo.col]
    low = (ci > cj) | same
    up = (ci < cj) | same
    DL = sp.csc_matrix((coo.data[low], (coo.row[low], coo.col[low])), shape=Kc.shape)
    DU = sp.csc_matrix((coo.data[up], (coo.row[up], coo.col[up])), shape=Kc.shape)
    rng = np.random.default_rng(7)
    r = np.where(fixed == 0, rng.standard_normal(p.n_dof), 0.0)
    x0 = np.where(fixed == 0, rng.standard_normal(p.n_dof), 0.0)
    x1 = x0 + spla.spsolve(DL, r - Kc @ x0)
    x2 = x1 + spla.spsolve(DU, r - Kc @ x1)
    got = msfem.BlockSGS(p, Kc).step(r, x0.copy())
    np.testing.assert_allclose(got, x2, rtol=1e-10, atol=1e-12 * np.abs(x2).max())


def test_colours_never_share_an_element():
    for p in (mbb(), small3d()):
        col = msfem.node_colours(p)
        en = fem.element_nodes(p)
        assert len(np.unique(col)) == 2 ** p.dim
        # the corners of every element carry distinct colours
        assert all(len(set(col[row])) == 2 ** p.dim for row in en)


def test_sgs_step_converges_as_iteration():
    # Gauss-Seidel on an SPD matrix contracts the error in the energy norm
    p = mbb(Emin=1e-3)
    _, fixed, _, K = system(p)
    Kc = fem.constrained(K, fixed)
    S = msfem.BlockSGS(p, Kc)
    f = W.load_vector(p)
    u = fem.direct_solve(K, f, fixed)
    x = np.zeros(p.n_dof)
    prev = u @ (Kc @ u)
    for _ in range(5):
        x = S.step(f, x)
        e = u - x
        en = e @ (Kc @ e)
        assert en < prev
        prev = en


def _dense(apply, n):
    return np.column_stack([apply(np.eye(n)[:, i]) for i in range(n)])


def test_cycle_symmetric_positive_definite():
    p = mbb(8, 8, 4, 3)
    _, fixed, E, K = system(p)
    Phi, _ = schwarz.coarse_basis(p, E, fixed, p.k)
    B = _dense(msfem.MsFEMCycle(p, K, fixed, Phi).apply, p.n_dof)
    np.testing.assert_allclose(B, B.T, atol=1e-10 * np.abs(B).max())
    free = fixed == 0
    assert np.linalg.eigvalsh(B[np.ix_(free, free)]).min() > 0


def test_cycle_with_complete_coarse_space_is_exact():
    # coarse space = every free DOF: the coarse step solves exactly, and the
    # post-smoother leaves the exact solution unchanged
    p = mbb(8, 4, 4, 1, Emin=1e-3)
    _, fixed, _, K = system(p)
    free = np.nonzero(fixed == 0)[0]
    Phi = sp.csc_matrix((np.ones(free.size), (free, np.arange(free.size))),
                        shape=(p.n_dof, free.size))
    M = msfem.MsFEMCycle(p, K, fixed, Phi)
    rng = np.random.default_rng(11)
    r = np.where(fixed == 0, rng.standard_normal(p.n_dof), 0.0)
    np.testing.assert_allclose(M.apply(r), fem.direct_solve(K, r, fixed, refine=2),
                               rtol=1e-9, atol=1e-12)


def test_gmres_distinct_eigenvalues_finish_in_that_many_steps():
    # GMRES on a diagonalisable matrix with three distinct eigenvalues has the
    # exact solution after three steps (its minimal polynomial has degree 3)
    rng = np.random.default_rng(5)
    d = np.repeat([1.0, 3.0, 7.5], 20)
    A = sp.diags(d)
    b = rng.standard_normal(d.size)
    x, it, rr, hist = msfem.gmres(lambda v: A @ v, lambda v: v, b, rtol=1e-12, restart=10)
    assert it == 3
    np.testing.assert_allclose(x, b / d, rtol=1e-11)
    assert hist[0] > 1e-3 and hist[1] > 1e-6


def test_gmres_minimises_the_preconditioned_residual():
    # After j steps from x0 = 0 the iterate minimises ||M^-1 (b - A x)|| over
    # the Krylov space span{z, (M^-1 A) z, ...} with z = M^-1 b: checked by a
    # least-squares solve on an orthonormal basis of that space
    rng = np.random.default_rng(9)
    n = 40
    A = np.eye(n) + 0.4 * rng.standard_normal((n, n)) / np.sqrt(n)
    Mi = np.eye(n) + 0.2 * rng.standard_normal((n, n)) / np.sqrt(n)
    b = rng.standard_normal(n)
    z = Mi @ b
    for j in range(1, 7):
        x, it, rr, _ = msfem.gmres(lambda v: A @ v, lambda v: Mi @ v, b, rtol=1e-15,
                                   restart=50, maxit=j)
        assert it == j
        Kr = np.column_stack([np.linalg.matrix_power(Mi @ A, i) @ z for i in range(j)])
        Q, _ = np.linalg.qr(Kr)
        c = np.linalg.lstsq(Mi @ A @ Q, z, rcond=None)[0]
        best = np.linalg.norm(z - Mi @ A @ Q @ c)
        got = np.linalg.norm(Mi @ (b - A @ x))
        np.testing.assert_allclose(got, best, rtol=1e-9)
        np.testing.assert_allclose(rr, got / np.linalg.norm(z), rtol=1e-9)


def test_gmres_restart_still_converges_and_residual_history_is_monotone():
    rng = np.random.default_rng(4)
    n = 60
    A = np.diag(np.linspace(1.0, 20.0, n)) + 0.05 * rng.standard_normal((n, n))
    b = rng.standard_normal(n)
    for m in (5, 12, 60):
        x, it, rr, hist = msfem.gmres(lambda v: A @ v, lambda v: v, b, rtol=1e-10,
                                      restart=m, maxit=2000)
        assert rr <= 1e-10
        np.testing.assert_allclose(A @ x, b, atol=1e-8 * np.linalg.norm(b))
        assert np.all(np.diff(hist) <= 1e-14)   # the residual never grows, restarts included


@pytest.mark.parametrize("kind", ["2d", "3d"])
def test_msfem_gmres_matches_direct_solve(kind):
    p = mbb(32, 16, 8, 4) if kind == "2d" else small3d()
    rho = W.design_field(p)
    fixed, f = W.fixed_mask(p), W.load_vector(p)
    u = fem.solve(p, rho)
    (x, it, rr), = msfem.solve_gmres(p, [rho], rho, f, fixed, rtol=1e-10, restart=30)
    assert rr <= 1e-10
    assert np.linalg.norm(x - u) / np.linalg.norm(u) < 1e-7
    assert it < 60


def test_msfem_gmres_counts_do_not_grow_with_contrast():
    # the coarse space is contrast-aware: iteration counts stay flat as E_min falls
    its = []
    for Emin in (1e-3, 1e-6, 1e-9):
        p = dataclasses.replace(W.mbb_64x32(), Emin=Emin)
        rho = W.design_field(p)
        (x, it, rr), = msfem.solve_gmres(p, [rho], rho, W.load_vector(p), W.fixed_mask(p),
                                         rtol=1e-8, restart=50)
        its.append(it)
    assert max(its) - min(its) <= 0.15 * min(its) + 1, its
