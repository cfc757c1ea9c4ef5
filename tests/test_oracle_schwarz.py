"""Pins for the oracle's spectral coarse space and two-level Schwarz PCG
(paper Sec. 2.4 local eigenproblems, partition of unity and Galerkin coarse
matrix; Sec. 3.2 diag(K) weighting; Sec. 2.4.2 preconditioner inside a Krylov
solve of an SPD system)."""
import dataclasses

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import fem, schwarz
from paper_1411_3923_amd import workloads as W


def mbb(nelx=32, nely=16, sub=8, k=4, Emin=1e-9):
    p = W.mbb_64x32()
    return dataclasses.replace(p, nel=(nelx, nely, 1), sub=sub, k=k, Emin=Emin)


def test_partition_of_unity_sums_to_one():
    p = mbb()
    chi = schwarz.partition_of_unity(p)
    acc = np.zeros(p.nnodes)
    for j in range(p.n_sub):
        acc[schwarz.subdomain_nodes(p, j)] += chi[schwarz.subdomain_nodes(p, j)]
    np.testing.assert_allclose(acc, 1.0, rtol=1e-15)
    # interface nodes are shared by 2, cross points by 4
    assert set(np.unique(np.round(1 / chi))) == {1.0, 2.0, 4.0}


def test_eigenpairs_against_standard_form():
    # K psi = lambda D psi with D = diag(K) equals the standard problem of
    # D^-1/2 K D^-1/2; check with an independent routine (all eigenvalues)
    p = mbb()
    rho = W.design_field(p)
    E = fem.simp_modulus(rho, p.E0, p.Emin, p.penal)
    fixed = W.fixed_mask(p)
    for j in (0, 5, p.n_sub - 1):
        lam, psi, dofs = schwarz.local_eigenpairs(p, E, fixed, j, p.k)
        KN = fem.assemble(p, E, elements=schwarz.subdomain_elements(p, j))[dofs][:, dofs].toarray()
        d = np.diag(KN)
        S = KN / np.sqrt(np.outer(d, d))
        ev = np.linalg.eigvalsh(S)
        np.testing.assert_allclose(lam, ev[:p.k], rtol=1e-8, atol=1e-12)
        np.testing.assert_allclose(psi.T @ (d[:, None] * psi), np.eye(p.k), atol=1e-10)
        assert np.all(lam > -1e-12)


def test_floating_subdomain_has_three_zero_modes():
    p = mbb(Emin=1.0)                                    # uniform material
    E = np.ones(p.n_el)
    fixed = W.fixed_mask(p)
    j = 1 + 4 * 1                                        # an interior subdomain: no supports
    lam, psi, dofs = schwarz.local_eigenpairs(p, E, fixed, j, 5)
    assert np.all(np.abs(lam[:3]) < 1e-12)
    assert lam[3] > 1e-4
    # a subdomain on the symmetry line (u_x = 0) keeps one rigid motion (y translation)
    lam0, _, _ = schwarz.local_eigenpairs(p, E, fixed, 0, 3)
    assert np.sum(np.abs(lam0) < 1e-12) == 1


def _dense_precond(p, K, fixed, Phi):
    M = schwarz.TwoLevelSchwarz(p, K, fixed, Phi)
    n = p.n_dof
    return np.stack([M.apply(e) for e in np.eye(n)], axis=1)


def test_preconditioner_symmetric_positive_and_one_level_form():
    p = mbb(16, 8, 4, 3)
    rho = W.design_field(dataclasses.replace(p, nel=(16, 8, 1)))
    fixed = W.fixed_mask(p)
    E = fem.simp_modulus(rho, p.E0, p.Emin, p.penal)
    K = fem.assemble(p, E)
    Phi, _ = schwarz.coarse_basis(p, E, fixed, p.k)
    Minv = _dense_precond(p, K, fixed, Phi)
    np.testing.assert_allclose(Minv, Minv.T, atol=1e-9 * np.abs(Minv).max())
    free = fixed == 0
    ev = np.linalg.eigvalsh(Minv[np.ix_(free, free)])
    assert ev.min() > 0
    # one-level form equals the sum of explicitly inverted principal submatrices
    M1 = _dense_precond(p, K, fixed, None)
    Kd = fem.constrained(K, fixed).toarray()
    ref = np.zeros_like(M1)
    for j in range(p.n_sub):
        d = schwarz.subdomain_dofs(p, j, fixed)
        ref[np.ix_(d, d)] += np.linalg.inv(Kd[np.ix_(d, d)])
    np.testing.assert_allclose(M1, ref, atol=1e-8 * np.abs(ref).max())


def test_complete_coarse_basis_is_exact_inverse():
    # a single subdomain with every eigenvector kept: the coarse space is the
    # whole free space, so the coarse branch alone is K^-1 and PCG takes 1 step
    p = mbb(8, 8, 8, 1, Emin=1e-3)
    rho = W.design_field(p)
    fixed = W.fixed_mask(p)
    E = fem.simp_modulus(rho, p.E0, p.Emin, p.penal)
    K = fem.assemble(p, E)
    nj = len(schwarz.subdomain_dofs(p, 0, fixed))
    Phi, _ = schwarz.coarse_basis(p, E, fixed, nj)
    M = schwarz.TwoLevelSchwarz(p, K, fixed, Phi, local=False)
    f = W.load_vector(p)
    x, it, rr = schwarz.pcg(lambda v: fem.constrained(K, fixed) @ v, M.apply, f, rtol=1e-10)
    assert it == 1
    np.testing.assert_allclose(x, fem.direct_solve(K, f, fixed), rtol=1e-8, atol=1e-12)


def test_pcg_matches_direct_and_energy_grows():
    p = mbb()
    rho = W.design_field(p)
    fixed, f = W.fixed_mask(p), W.load_vector(p)
    u = fem.solve(p, rho)
    E = fem.simp_modulus(rho, p.E0, p.Emin, p.penal)
    K = fem.assemble(p, E)
    Kc = fem.constrained(K, fixed)
    Phi, _ = schwarz.coarse_basis(p, E, fixed, p.k)
    M = schwarz.TwoLevelSchwarz(p, K, fixed, Phi)
    energies = []
    x, it, rr = schwarz.pcg(lambda v: Kc @ v, M.apply, f, rtol=1e-12,
                            callback=lambda i, xx, r: energies.append(xx @ (Kc @ xx)))
    assert rr <= 1e-12
    assert np.linalg.norm(x - u) / np.linalg.norm(u) < 1e-8
    c = fem.compliance(f, u)
    # with x0 = 0: c* - x_k^T K x_k = ||e_k||_K^2 >= 0 and non-decreasing energy
    e = np.array(energies)
    assert np.all(e <= c * (1 + 1e-10))
    assert np.all(np.diff(e) >= -1e-10 * c)


def test_contrast_independent_iterations():
    # Sec. 3.1: iteration counts do not depend on E_min once it is small
    its = []
    for Emin in (1e-3, 1e-6, 1e-9):
        p = dataclasses.replace(W.mbb_64x32(), Emin=Emin)
        rho = W.design_field(p)
        r = schwarz.solve_pcg(p, [rho], rho, W.load_vector(p), W.fixed_mask(p), rtol=1e-8)
        its.append(r[0][1])
    assert max(its) - min(its) <= 0.15 * min(its), its
    p = W.mbb_64x32()
    rho = W.design_field(p)
    one = schwarz.solve_pcg(p, [rho], rho, W.load_vector(p), W.fixed_mask(p), rtol=1e-8, coarse=False)
    assert one[0][1] > 1.5 * its[-1]                     # the coarse space is doing work
