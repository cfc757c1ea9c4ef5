"""Pins for the oracle's assembly, direct solve, compliance and sensitivities
(paper Sec. 2.1 K u = f; Sec. 2.2 SIMP element stiffness and compliance
f^T u; Sec. 4.2 self-adjoint sensitivity)."""
import dataclasses
import os

import numpy as np
import pytest

from oracle import fem
from paper_1411_3923_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def small(dim, nel, density="uniform_random", seed=3, support=None):
    sup = support or ("cantilever" if dim == 2 else "cantilever3d")
    return W.Problem("t", dim, nel, sub=1, k=1, support=sup, density=density, seed=seed)


def test_paper_dof_count():
    # Sec. 6.1.1 prints 13,107,200 elements and 26,229,762 DOFs for M_x = 64
    vals = {}
    for line in open(os.path.join(GOLDEN, "paper_counts.txt")):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            vals[k] = int(v)
    p = W.Problem("paper", 2, (vals["nelx"], vals["nely"], 1), sub=40, k=1)
    assert p.n_el == vals["elements"]
    assert p.n_dof == vals["dofs"]


@pytest.mark.parametrize("dim,nel", [(2, (6, 4, 1)), (3, (3, 3, 2))])
def test_assembly_symmetric_rigid_kernel_spd(dim, nel):
    p = small(dim, nel)
    rho = W.design_field(p)
    E = fem.simp_modulus(rho)
    K = fem.assemble(p, E).toarray()
    np.testing.assert_allclose(K, K.T, atol=0)
    # global rigid motions of the unconstrained structure
    nn = p.nnodes
    nx, ny = p.nelx + 1, p.nely + 1
    n = np.arange(nn)
    X = np.stack([n % nx, (n // nx) % ny] + ([n // (nx * ny)] if dim == 3 else []), 1).astype(float)
    for t in np.eye(dim):
        assert np.abs(K @ np.tile(t, nn)).max() < 1e-12
    for a in range(dim):
        for b in range(a + 1, dim):
            u = np.zeros_like(X)
            u[:, a], u[:, b] = -X[:, b], X[:, a]
            assert np.abs(K @ u.ravel()).max() < 1e-12
    ev = np.linalg.eigvalsh(K)
    assert np.sum(np.abs(ev) < 1e-10) == (3 if dim == 2 else 6)
    free = W.fixed_mask(p) == 0
    np.linalg.cholesky(K[np.ix_(free, free)])        # positive definite once supported


@pytest.mark.parametrize("dim,nel", [(2, (5, 4, 1)), (3, (3, 3, 3))])
def test_patch_test(dim, nel):
    # uniform modulus, linear displacement field: zero force at interior nodes
    p = small(dim, nel, density="uniform_random")
    K = fem.assemble(p, np.full(p.n_el, 2.5)).toarray()
    nx, ny = p.nelx + 1, p.nely + 1
    n = np.arange(p.nnodes)
    X = np.stack([n % nx, (n // nx) % ny] + ([n // (nx * ny)] if dim == 3 else []), 1).astype(float)
    rng = np.random.default_rng(0)
    u = (X @ rng.standard_normal((dim, dim)).T).ravel()
    res = (K @ u).reshape(-1, dim)
    inner = np.all((X > 0) & (X < np.array([p.nelx, p.nely, p.nelz][:dim])), axis=1)
    assert np.abs(res[inner]).max() < 1e-12
    assert np.abs(res[~inner]).max() > 1e-3


def test_direct_solve_matches_dense_lapack_on_mbb():
    p = W.mbb_64x32()
    rho = W.design_field(p)
    fixed, f = W.fixed_mask(p), W.load_vector(p)
    u = fem.solve(p, rho)
    K = fem.assemble(p, fem.simp_modulus(rho, p.E0, p.Emin, p.penal)).toarray()
    free = fixed == 0
    ud = np.zeros(p.n_dof)
    ud[free] = np.linalg.solve(K[np.ix_(free, free)], f[free])
    assert np.linalg.norm(u - ud) / np.linalg.norm(ud) < 1e-8
    assert np.all(u[~free] == 0)


@pytest.mark.parametrize("dim,nel", [(2, (6, 4, 1)), (3, (3, 3, 3))])
def test_compliance_identities(dim, nel):
    p = small(dim, nel)
    rho = W.design_field(p)
    f = W.load_vector(p)
    u = fem.solve(p, rho)
    E = fem.simp_modulus(rho, p.E0, p.Emin, p.penal)
    K = fem.assemble(p, E)
    c = fem.compliance(f, u)
    assert c == pytest.approx(u @ (K @ u), rel=1e-10)
    assert c == pytest.approx(np.sum(E * fem.element_energies(p, u)), rel=1e-10)


@pytest.mark.parametrize("dim,nel", [(2, (6, 4, 1)), (3, (3, 3, 3))])
def test_sensitivity_central_differences(dim, nel):
    p = small(dim, nel)
    rho = W.design_field(p)                      # uniform in [0.2, 0.9]
    f = W.load_vector(p)
    u = fem.solve(p, rho)
    dc = fem.sensitivity(p, rho, u)
    h = 1e-6
    for e in range(p.n_el):
        rp, rm = rho.copy(), rho.copy()
        rp[e] += h
        rm[e] -= h
        fd = (fem.compliance(f, fem.solve(p, rp)) - fem.compliance(f, fem.solve(p, rm))) / (2 * h)
        assert dc[e] == pytest.approx(fd, rel=1e-6, abs=1e-9 * abs(fd) + 1e-12)
    # Euler identity for the homogeneous SIMP term:
    # sum_e rho_e dc/drho_e = -p (c - E_min sum_e q_e)
    q = fem.element_energies(p, u)
    c = fem.compliance(f, u)
    assert np.sum(rho * dc) == pytest.approx(-p.penal * (c - p.Emin * q.sum()), rel=1e-10)


def test_simp_endpoints():
    assert fem.simp_modulus(np.array([0.0]), 1.0, 1e-9, 3.0)[0] == 1e-9
    assert fem.simp_modulus(np.array([1.0]), 1.0, 1e-9, 3.0)[0] == 1.0
    assert fem.simp_modulus(np.array([0.5]), 1.0, 0.0, 3.0)[0] == 0.125
