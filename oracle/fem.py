"""Q1 finite elements on the slab (oracle; test infrastructure only).

Paper: Sec. 2 eq. (2) (conductivity tensors), Sec. 2.2 (Q1 space, lumped diagonal mass M,
stiffness a_pj = int D grad(phi_j) . grad(phi_p)).

Readings taken where the paper is silent:
  * axisymmetric tissue (sigma_n = sigma_t), so D = sigma_t I + (sigma_l - sigma_t) a_l a_l^T;
  * fibers in the xy-plane, a_l = (cos th, sin th, 0), th(z) = th0 + rot * z / Lz;
  * D evaluated at each of the 2x2x2 Gauss points of an element;
  * lumped mass m_p = sum over elements e containing p of |e| / 8 (= row sum of the
    consistent Q1 mass, i.e. the integral of phi_p);
  * the full 27-point pattern is kept, structural zeros included.

Node p = i + (nx+1)(j + (ny+1) k); element (ex, ey, ez) has local nodes l = a + 2b + 4c,
(a, b, c) in {0, 1}^3, at global (ex + a, ey + b, ez + c).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

# Two-point Gauss-Legendre rule on [0, 1]: nodes 1/2 -+ 1/(2 sqrt 3), weights 1/2.
GAUSS_1D = (0.5 - 0.5 / math.sqrt(3.0), 0.5 + 0.5 / math.sqrt(3.0))
GAUSS_W1D = (0.5, 0.5)


def fiber_direction(z: float, case) -> np.ndarray:
    th = case.fiber_theta0 + case.fiber_rotation * z / case.Lz
    return np.array([math.cos(th), math.sin(th), 0.0])


def conductivity(z: float, sig_l: float, sig_t: float, case) -> np.ndarray:
    """Eq. (2) with sigma_n = sigma_t: D = sigma_t I + (sigma_l - sigma_t) a_l a_l^T."""
    a = fiber_direction(z, case)
    return sig_t * np.eye(3) + (sig_l - sig_t) * np.outer(a, a)


def local_node_bits(l: int):
    return l & 1, (l >> 1) & 1, (l >> 2) & 1


def q1_basis_gradients(xi: float, eta: float, zeta: float, hx: float, hy: float, hz: float) -> np.ndarray:
    """Physical gradients (8 x 3) of the trilinear basis at reference point (xi, eta, zeta) in [0,1]^3."""
    N = lambda a, t: 1.0 - t if a == 0 else t
    dN = lambda a: -1.0 if a == 0 else 1.0
    G = np.zeros((8, 3))
    for l in range(8):
        a, b, c = local_node_bits(l)
        G[l, 0] = dN(a) * N(b, eta) * N(c, zeta) / hx
        G[l, 1] = N(a, xi) * dN(b) * N(c, zeta) / hy
        G[l, 2] = N(a, xi) * N(b, eta) * dN(c) / hz
    return G


def element_stiffness(case, ez: int, sig_l: float, sig_t: float) -> np.ndarray:
    """K_e[l, m] = int_e grad(phi_m)^T D grad(phi_l), 2x2x2 Gauss, D at each Gauss point.

    On the uniform slab every element of layer ez has the same matrix (D depends on z only).
    """
    hx, hy, hz = case.h
    K = np.zeros((8, 8))
    for gz, wz in zip(GAUSS_1D, GAUSS_W1D):
        D = conductivity((ez + gz) * hz, sig_l, sig_t, case)
        for gy, wy in zip(GAUSS_1D, GAUSS_W1D):
            for gx, wx in zip(GAUSS_1D, GAUSS_W1D):
                G = q1_basis_gradients(gx, gy, gz, hx, hy, hz)
                K += (wx * wy * wz * hx * hy * hz) * (G @ D @ G.T)
    return 0.5 * (K + K.T)  # exact symmetry (the two rounding orders of G D G^T agree to ~1 ulp)


def stencil_offset(di: int, dj: int, dk: int) -> int:
    return (di + 1) + 3 * (dj + 1) + 9 * (dk + 1)


def _stencil_to_csr(case, stencil: np.ndarray) -> sp.csr_matrix:
    """Turn per-node 27-point coefficients into CSR, keeping every in-range neighbour."""
    nxp, nyp, nzp = case.nx + 1, case.ny + 1, case.nz + 1
    n = nxp * nyp * nzp
    p = np.arange(n)
    i = p % nxp
    j = (p // nxp) % nyp
    k = p // (nxp * nyp)
    cols = np.empty((n, 27), dtype=np.int64)
    valid = np.empty((n, 27), dtype=bool)
    for dk in (-1, 0, 1):
        for dj in (-1, 0, 1):
            for di in (-1, 0, 1):
                t = stencil_offset(di, dj, dk)
                cols[:, t] = p + di + nxp * dj + nxp * nyp * dk
                valid[:, t] = ((i + di >= 0) & (i + di < nxp) & (j + dj >= 0) & (j + dj < nyp)
                               & (k + dk >= 0) & (k + dk < nzp))
    counts = valid.sum(axis=1)
    indptr = np.concatenate([[0], np.cumsum(counts)])
    # offsets are enumerated with dk slowest and di fastest, so columns come out sorted per row
    A = sp.csr_matrix((stencil[valid], cols[valid], indptr), shape=(n, n))
    A.has_sorted_indices = True
    return A


def assemble_stiffness(case, sig_l: float, sig_t: float) -> sp.csr_matrix:
    """Global Q1 stiffness A[p, q] = sum_e K_e[l(p), l(q)] over elements containing p and q."""
    nxp, nyp = case.nx + 1, case.ny + 1
    n = case.n
    Kz = np.stack([element_stiffness(case, ez, sig_l, sig_t) for ez in range(case.nz)])
    EZ, EY, EX = np.meshgrid(np.arange(case.nz), np.arange(case.ny), np.arange(case.nx), indexing="ij")
    EX, EY, EZ = EX.ravel(), EY.ravel(), EZ.ravel()
    stencil = np.zeros((n, 27))
    for l in range(8):
        a, b, c = local_node_bits(l)
        p_l = (EX + a) + nxp * ((EY + b) + nyp * (EZ + c))  # distinct for distinct elements
        for m in range(8):
            a2, b2, c2 = local_node_bits(m)
            t = stencil_offset(a2 - a, b2 - b, c2 - c)
            stencil[p_l, t] += Kz[EZ, l, m]
    return _stencil_to_csr(case, stencil)


def lumped_mass(case) -> np.ndarray:
    """m_p = sum_{e containing p} |e| / 8."""
    hx, hy, hz = case.h
    def per_axis(ne):
        c = np.full(ne + 1, 2.0)
        c[0] = c[-1] = 1.0
        return c
    cx, cy, cz = per_axis(case.nx), per_axis(case.ny), per_axis(case.nz)
    count = (cz[:, None, None] * cy[None, :, None] * cx[None, None, :]).ravel()
    return count * (hx * hy * hz / 8.0)


def assemble_operators(case):
    """The matrices of the decoupled step (eqs. (6), (7)): A_i, A_e, A_ell = A_i + A_e,
    A_par = (c_m / dt) M + A_i, and the lumped mass vector m."""
    Ai = assemble_stiffness(case, case.sig_il, case.sig_it)
    Ae = assemble_stiffness(case, case.sig_el, case.sig_et)
    m = lumped_mass(case)
    # all three operators share the 27-point pattern; add values entry by entry so that
    # the pattern (structural zeros included) is kept
    Aell = sp.csr_matrix((Ai.data + Ae.data, Ai.indices.copy(), Ai.indptr.copy()), shape=Ai.shape)
    diag_pos = diagonal_positions(Ai)
    par = Ai.data.copy()
    par[diag_pos] += case.cm / case.dt * m
    Apar = sp.csr_matrix((par, Ai.indices.copy(), Ai.indptr.copy()), shape=Ai.shape)
    return dict(Ai=Ai, Ae=Ae, Aell=Aell, Apar=Apar, m=m)


def diagonal_positions(A: sp.csr_matrix) -> np.ndarray:
    """Index into A.data of each row's diagonal entry."""
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    pos = np.flatnonzero(A.indices == rows)
    assert pos.size == A.shape[0], "every row must store its diagonal"
    return pos
