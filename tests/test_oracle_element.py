"""Pins for the oracle's element stiffness (paper Sec. 2.1: isotropic linear
elasticity, unit reference modulus; Sec. 2.2: K0 is the unit-modulus element
matrix). The pins integrate the bilinear form in closed form with separable
1D integrals of the linear hat functions, so they share nothing with the
oracle's Gauss-quadrature code."""
import itertools

import numpy as np
import pytest

from oracle import fem

NU = 0.3


def _closed_form_K0(dim, lam, G):
    corners = ([(0, 0), (1, 0), (1, 1), (0, 1)] if dim == 2 else
               [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0),
                (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)])

    def m1(a, b):            # int phi_a phi_b on [0, 1], phi_0 = 1 - t, phi_1 = t
        return 1.0 / 3.0 if a == b else 1.0 / 6.0

    def s1(a, b):            # int phi_a' phi_b'
        return 1.0 if a == b else -1.0

    def c1(a, b):            # int phi_a' phi_b
        return (1.0 if a == 1 else -1.0) * 0.5

    def I(i, A, j, B):       # int d_i N_A d_j N_B over the unit cell
        v = 1.0
        for m in range(dim):
            a, b = A[m], B[m]
            if m == i and m == j:
                v *= s1(a, b)
            elif m == i:
                v *= c1(a, b)
            elif m == j:
                v *= c1(b, a)
            else:
                v *= m1(a, b)
        return v

    n = len(corners)
    K = np.zeros((dim * n, dim * n))
    for (ia, A), (ib, B) in itertools.product(enumerate(corners), repeat=2):
        for i in range(dim):
            for j in range(dim):
                v = lam * I(i, A, j, B) + G * I(j, A, i, B)
                if i == j:
                    v += G * sum(I(k, A, k, B) for k in range(dim))
                K[dim * ia + i, dim * ib + j] = v
    return K


def test_q4_matches_closed_form_integrals():
    lam_ps = NU / (1 - NU * NU)          # plane-stress Lame constant, E = 1
    G = 1.0 / (2 * (1 + NU))
    np.testing.assert_allclose(fem.q4_K0(NU), _closed_form_K0(2, lam_ps, G), rtol=0, atol=1e-14)


def test_h8_matches_closed_form_integrals():
    lam = NU / ((1 + NU) * (1 - 2 * NU))
    G = 1.0 / (2 * (1 + NU))
    np.testing.assert_allclose(fem.h8_K0(NU), _closed_form_K0(3, lam, G), rtol=0, atol=1e-14)


def test_q4_textbook_row_and_spectrum():
    # classical closed form of the unit-square plane-stress element (E = 1):
    # first row = 1/(1-nu^2) [1/2-nu/6, 1/8+nu/8, -1/4-nu/12, -1/8+3nu/8,
    #                          -1/4+nu/12, -1/8-nu/8, nu/6, 1/8-3nu/8]
    K = fem.q4_K0(NU)
    row = np.array([0.5 - NU / 6, 0.125 + NU / 8, -0.25 - NU / 12, -0.125 + 3 * NU / 8,
                    -0.25 + NU / 12, -0.125 - NU / 8, NU / 6, 0.125 - 3 * NU / 8]) / (1 - NU * NU)
    np.testing.assert_allclose(K[0], row, atol=1e-15)
    ev = np.sort(np.linalg.eigvalsh(K))
    # rigid modes (3), hourglass (2), deviatoric strain (2), volumetric strain (1)
    want = np.sort([0, 0, 0, (3 - NU) / (6 * (1 - NU ** 2)), (3 - NU) / (6 * (1 - NU ** 2)),
                    1 / (1 + NU), 1 / (1 + NU), 1 / (1 - NU)])
    np.testing.assert_allclose(ev, want, atol=1e-14)
    np.testing.assert_allclose(np.trace(K), 8 * row[0], atol=1e-14)   # all diagonal entries equal


def test_h8_diagonal_and_kernel():
    K = fem.h8_K0(NU)
    lam = NU / ((1 + NU) * (1 - 2 * NU))
    G = 1.0 / (2 * (1 + NU))
    # K[0,0] = (lam + 2G) int (dN/dx)^2 + G int (dN/dy)^2 + G int (dN/dz)^2 = (lam + 4G) / 9
    assert K[0, 0] == pytest.approx((lam + 4 * G) / 9, abs=1e-15)
    assert K[0, 1] == pytest.approx((lam + G) / 12, abs=1e-15)
    ev = np.sort(np.linalg.eigvalsh(K))
    assert np.all(np.abs(ev[:6]) < 1e-13)
    assert ev[6] > 1e-2
    np.testing.assert_allclose(K, K.T, atol=0)


@pytest.mark.parametrize("dim", [2, 3])
def test_rigid_modes_and_constant_strain_energy(dim):
    K = fem.element_K0(dim, NU)
    pts = (np.array([[0, 0], [1, 0], [1, 1], [0, 1]], float) if dim == 2 else
           np.array([[0, 0, 0], [1, 0, 0], [1, 1, 0], [0, 1, 0],
                     [0, 0, 1], [1, 0, 1], [1, 1, 1], [0, 1, 1]], float))
    # translations and infinitesimal rotations are in the kernel
    for t in np.eye(dim):
        assert np.abs(K @ np.tile(t, len(pts))).max() < 1e-14
    for a, b in itertools.combinations(range(dim), 2):
        u = np.zeros_like(pts)
        u[:, a] = -pts[:, b]
        u[:, b] = pts[:, a]
        assert np.abs(K @ u.ravel()).max() < 1e-14
    # a linear field u = G x has energy u^T K u = eps : C : eps * volume (exact)
    rng = np.random.default_rng(7)
    Gr = rng.standard_normal((dim, dim))
    u = (pts @ Gr.T).ravel()
    eps = 0.5 * (Gr + Gr.T)
    if dim == 2:
        lam = NU / (1 - NU * NU)
    else:
        lam = NU / ((1 + NU) * (1 - 2 * NU))
    mu = 1.0 / (2 * (1 + NU))
    energy = lam * np.trace(eps) ** 2 + 2 * mu * np.sum(eps * eps)
    assert u @ K @ u == pytest.approx(energy, rel=1e-13)


def test_quadrature_order_does_not_matter():
    # the integrand is at most quadratic per axis, so 2 Gauss points are exact
    np.testing.assert_allclose(fem.q4_K0(NU, npts=2), fem.q4_K0(NU, npts=5), atol=1e-14)
    np.testing.assert_allclose(fem.h8_K0(NU, npts=2), fem.h8_K0(NU, npts=4), atol=1e-14)


@pytest.mark.parametrize("nu", [0.17, 0.3, 0.45])
def test_q4_matrix_takes_eight_values_of_its_first_row(nu):
    """The square's reflections and quarter turn map every entry of the
    unit-square Q4 matrix onto an entry of its first row, whose eight entries
    are distinct: the GPU product keeps only those eight values (in scalar
    registers) and the library checks the index map on the host."""
    K = fem.q4_K0(nu)
    row = K[0]
    assert len(np.unique(np.round(row, 14))) == 8
    for v in K.ravel():
        assert np.min(np.abs(row - v)) < 1e-14


def _corner(a):
    """Position bits (x, y, z) of H8 corner a: counter-clockwise in x-y, bottom face first."""
    return (int((a & 3) in (1, 2)), int((a & 3) >= 2), int(a >= 4))


@pytest.mark.parametrize("nu", [0.17, 0.3, 0.45])
def test_h8_matrix_has_twelve_entry_classes(nu):
    """Reflecting the unit cube so that corner a becomes corner 0 maps corner
    b to the corner at |p_b - p_a| and flips the displacement components along
    the reflected axes: K0[(a,i),(b,c)] = tau_i(a) tau_c(a) R(e)[i][c], with
    R(e) the block of corner 0's rows. The axis permutations (which fix
    corner 0) and the symmetry of K0 leave twelve values in R up to sign. The
    GPU product keeps those twelve values in scalar registers; the library
    checks the structure on the host."""
    K = fem.h8_K0(nu)
    mx = np.abs(K).max()
    R = {}
    for e in range(8):
        R[_corner(e)] = K[0:3, 3 * e:3 * e + 3]
    for a in range(8):
        pa = _corner(a)
        for b in range(8):
            pb = _corner(b)
            e = tuple(x ^ y for x, y in zip(pa, pb))
            for i in range(3):
                for c in range(3):
                    s = (-1 if pa[i] else 1) * (-1 if pa[c] else 1)
                    assert abs(K[3 * a + i, 3 * b + c] - s * R[e][i][c]) < 1e-14 * mx
    # the permutations of the axes map R(e)[i][c] to R(pi e)[pi i][pi c]
    for perm in itertools.permutations(range(3)):
        for e in R:
            pe = tuple(e[perm.index(j)] for j in range(3))
            for i in range(3):
                for c in range(3):
                    assert abs(R[e][i][c] - R[pe][perm[i]][perm[c]]) < 1e-14 * mx
    # twelve magnitudes up to sign (with nu generic, no two classes coincide
    # except by the value identities of the element, so count the orbits)
    orbits = set()
    for e in R:
        for i in range(3):
            for c in range(3):
                key = min((tuple(e[perm.index(j)] for j in range(3)), perm[i], perm[c])
                          for perm in itertools.permutations(range(3)))
                # the transpose relation R(e)[i][c] = tau_i(e) tau_c(e) R(e)[c][i]
                s = (-1 if e[i] else 1) * (-1 if e[c] else 1)
                assert abs(R[e][i][c] - s * R[e][c][i]) < 1e-14 * mx
                key2 = min((tuple(e[perm.index(j)] for j in range(3)), perm[c], perm[i])
                           for perm in itertools.permutations(range(3)))
                orbits.add(min(key, key2))
    assert len(orbits) == 12
