"""Oracle: finite elements, SIMP, assembly, direct solve, compliance, sensitivities.

Test infrastructure only (see the package docstring).

Sources in the paper:
* Sec. 2.1: linear elasticity with C(x) = E(x) C0, unit reference modulus,
  Poisson ratio below 0.5, bilinear elements on a uniform mesh, K u = f.
* Sec. 2.2, element-stiffness equation: K_e = (E_min + (E_max - E_min) rho^p) K0.
* Sec. 2.2, compliance problem: objective f^T u.
* Sec. 4.1: the reference solution is a sparse direct solve.
* Sec. 4.2, sensitivity equations: df/drho_e = -u_e^T dK_e/drho_e u_e with
  dK_e/drho_e = p (E_max - E_min) rho_e^(p-1) K0.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

# ---------------------------------------------------------------------------
# Element stiffness K0 for unit modulus (Sec. 2.1, Sec. 2.2)
# ---------------------------------------------------------------------------


def _gauss(npts):
    """Gauss-Legendre points and weights on [-1, 1]."""
    return np.polynomial.legendre.leggauss(npts)

# reference coordinates of the element nodes: counter-clockwise from the
# lower-left corner; in 3D the bottom face, then the top face
Q4_NODES = np.array([[-1, -1], [1, -1], [1, 1], [-1, 1]], dtype=np.float64)
H8_NODES = np.array([[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1],
                     [-1, -1, 1], [1, -1, 1], [1, 1, 1], [-1, 1, 1]],
                    dtype=np.float64)


def plane_stress_D(E=1.0, nu=0.3):
    """Plane-stress constitutive matrix (Voigt: xx, yy, xy engineering shear)."""
    return E / (1.0 - nu * nu) * np.array([[1.0, nu, 0.0],
                                           [nu, 1.0, 0.0],
                                           [0.0, 0.0, (1.0 - nu) / 2.0]])


def isotropic_D(E=1.0, nu=0.3):
    """3D isotropic constitutive matrix (Voigt: xx, yy, zz, xy, yz, zx)."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    G = E / (2.0 * (1.0 + nu))
    D = np.zeros((6, 6))
    D[:3, :3] = lam
    D[0, 0] = D[1, 1] = D[2, 2] = lam + 2.0 * G
    D[3, 3] = D[4, 4] = D[5, 5] = G
    return D


def q4_K0(nu=0.3, npts=2):
    """8x8 stiffness of a unit-square bilinear element, E = 1, thickness 1.

    Integrates B^T D B over the element with a tensor Gauss rule (2 points per
    axis integrate it exactly). DOF order: (x, y) per node, nodes
    counter-clockwise from the lower-left corner.
    """
    D = plane_stress_D(1.0, nu)
    K = np.zeros((8, 8))
    pts, wts = _gauss(npts)
    for xi, wx in zip(pts, wts):
        for eta, wy in zip(pts, wts):
            dN = np.array([[0.25 * a * (1 + eta * b), 0.25 * b * (1 + xi * a)]
                           for a, b in Q4_NODES])       # d/dxi, d/deta
            dNdx = dN * 2.0                             # unit square: x = (xi+1)/2
            B = np.zeros((3, 8))
            B[0, 0::2] = dNdx[:, 0]
            B[1, 1::2] = dNdx[:, 1]
            B[2, 0::2] = dNdx[:, 1]
            B[2, 1::2] = dNdx[:, 0]
            K += B.T @ D @ B * (0.25 * wx * wy)         # det J = 1/4
    return K


def h8_K0(nu=0.3, npts=2):
    """24x24 stiffness of a unit-cube trilinear element, E = 1.

    DOF order (x, y, z) per node; nodes of the bottom face counter-clockwise,
    then the top face.
    """
    D = isotropic_D(1.0, nu)
    K = np.zeros((24, 24))
    pts, wts = _gauss(npts)
    for xi, wx in zip(pts, wts):
        for eta, wy in zip(pts, wts):
            for zeta, wz in zip(pts, wts):
                dN = np.array([[0.125 * a * (1 + eta * b) * (1 + zeta * c),
                                0.125 * b * (1 + xi * a) * (1 + zeta * c),
                                0.125 * c * (1 + xi * a) * (1 + eta * b)]
                               for a, b, c in H8_NODES])
                dNdx = dN * 2.0
                B = np.zeros((6, 24))
                B[0, 0::3] = dNdx[:, 0]
                B[1, 1::3] = dNdx[:, 1]
                B[2, 2::3] = dNdx[:, 2]
                B[3, 0::3] = dNdx[:, 1]
                B[3, 1::3] = dNdx[:, 0]
                B[4, 1::3] = dNdx[:, 2]
                B[4, 2::3] = dNdx[:, 1]
                B[5, 0::3] = dNdx[:, 2]
                B[5, 2::3] = dNdx[:, 0]
                K += B.T @ D @ B * (0.125 * wx * wy * wz)   # det J = 1/8
    return K


def element_K0(dim, nu=0.3):
    return q4_K0(nu) if dim == 2 else h8_K0(nu)


# ---------------------------------------------------------------------------
# Structured mesh indexing
# ---------------------------------------------------------------------------

def element_nodes(p):
    """int64 [n_el, 2^dim] global node numbers of each element (element order)."""
    nx, ny = p.nelx + 1, p.nely + 1
    if p.dim == 2:
        ey, ex = np.meshgrid(np.arange(p.nely), np.arange(p.nelx), indexing="ij")
        ex, ey = ex.ravel(), ey.ravel()
        n0 = ex + nx * ey
        return np.stack([n0, n0 + 1, n0 + 1 + nx, n0 + nx], axis=1)
    ez, ey, ex = np.meshgrid(np.arange(p.nelz), np.arange(p.nely),
                             np.arange(p.nelx), indexing="ij")
    ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()
    n0 = ex + nx * (ey + ny * ez)
    lay = nx * ny
    bot = [n0, n0 + 1, n0 + 1 + nx, n0 + nx]
    return np.stack(bot + [b + lay for b in bot], axis=1)


def element_dofs(p):
    """int64 [n_el, dim * 2^dim] global DOFs of each element."""
    en = element_nodes(p)
    d = p.dim
    return (d * en[:, :, None] + np.arange(d)[None, None, :]).reshape(en.shape[0], -1)


# ---------------------------------------------------------------------------
# SIMP and assembly (Sec. 2.2, element-stiffness equation)
# ---------------------------------------------------------------------------

def simp_modulus(rho_phys, E0=1.0, Emin=1e-9, penal=3.0):
    """E_e = E_min + (E0 - E_min) rho_e^p."""
    return Emin + (E0 - Emin) * np.power(rho_phys, penal)


def assemble(p, E, K0=None, elements=None):
    """Global stiffness sum_e E_e K0 scattered to the element DOFs (CSR)."""
    if K0 is None:
        K0 = element_K0(p.dim, p.nu)
    edof = element_dofs(p)
    if elements is not None:
        edof = edof[elements]
        E = np.asarray(E)[elements]
    nd = edof.shape[1]
    rows = np.repeat(edof, nd, axis=1).ravel()
    cols = np.tile(edof, (1, nd)).ravel()
    vals = (np.asarray(E)[:, None, None] * K0[None, :, :]).ravel()
    K = sp.coo_matrix((vals, (rows, cols)), shape=(p.n_dof, p.n_dof)).tocsr()
    K.sum_duplicates()
    return K


def constrained(K, fixed):
    """Projected operator P K P + (I - P): fixed rows and columns replaced by identity."""
    free = (np.asarray(fixed) == 0).astype(np.float64)
    P = sp.diags(free)
    return (P @ K @ P + sp.diags(1.0 - free)).tocsr()


# ---------------------------------------------------------------------------
# Direct solve (Sec. 4.1 reference solve) with FP64 iterative refinement
# ---------------------------------------------------------------------------

def direct_solve(K, f, fixed, refine=2):
    """u with u = 0 on fixed DOFs and K_ff u_f = f_f, by sparse LU plus refinement."""
    free = np.flatnonzero(np.asarray(fixed) == 0)
    Kff = K[free][:, free].tocsc()
    lu = spla.splu(Kff, permc_spec="MMD_AT_PLUS_A")
    ff = np.asarray(f)[free]
    uf = lu.solve(ff)
    for _ in range(refine):
        uf = uf + lu.solve(ff - Kff @ uf)
    u = np.zeros(K.shape[0])
    u[free] = uf
    return u


def solve(p, rho_phys, f=None, fixed=None):
    """Reference displacement for problem p at physical densities rho_phys."""
    from paper_1411_3923_amd import workloads as W
    fixed = W.fixed_mask(p) if fixed is None else fixed
    f = W.load_vector(p) if f is None else f
    E = simp_modulus(rho_phys, p.E0, p.Emin, p.penal)
    return direct_solve(assemble(p, E), f, fixed)


# ---------------------------------------------------------------------------
# Compliance and sensitivities (Sec. 2.2 objective; Sec. 4.2)
# ---------------------------------------------------------------------------

def compliance(f, u):
    """c = f^T u."""
    return float(np.dot(f, u))


def element_energies(p, u, K0=None):
    """q_e = u_e^T K0 u_e for every element."""
    if K0 is None:
        K0 = element_K0(p.dim, p.nu)
    ue = np.asarray(u)[element_dofs(p)]
    return np.einsum("ei,ij,ej->e", ue, K0, ue)


def sensitivity(p, rho_phys, u, K0=None):
    """dc/drho_e = -p (E0 - E_min) rho_e^(p-1) q_e (self-adjoint compliance)."""
    q = element_energies(p, u, K0)
    return -p.penal * (p.E0 - p.Emin) * np.power(rho_phys, p.penal - 1.0) * q
