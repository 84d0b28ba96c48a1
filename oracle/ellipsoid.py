"""Q1 finite elements on the truncated ellipsoid (oracle; test infrastructure only).

Paper: Sec. 3, eq. (8) and Table 1 (the idealised left ventricle: a truncated ellipsoidal shell
x = a(r) cos(theta) cos(phi), y = b(r) sin(theta) cos(phi), z = c(r) sin(phi), with
a(r) = a1 + r (a2 - a1) and likewise b, c; theta in [-3 pi/2, pi/2], phi in [-3 pi/8, pi/8],
r in [0, 1]; a1 = b1 = 2.2, a2 = b2 = 3.3, c1 = 5.9, c2 = 6.4 cm); Sec. 2 eq. (2) (conductivity
tensors); Sec. 2.2 (Q1 space, lumped mass, stiffness a_pj = int D grad(phi_j) . grad(phi_p)).

Readings:
  * eq. (8) prints y = b(r) cos(theta) sin(phi), which would put every point of a theta-line in
    one plane; the ellipsoid is y = b(r) sin(theta) cos(phi);
  * theta spans one full period, so the mesh is periodic in theta: an n_theta x n_phi x n_r
    element mesh has n_theta (n_phi + 1)(n_r + 1) nodes, the count Sec. 6 Test 4 gives for the
    128 x 128 x 64 and 256 x 256 x 128 meshes (Tests 2 and 3 count instead two unknowns at each
    node of an (n_theta + 1)(n_phi + 1)(n_r + 1) grid, a seam of duplicated nodes; a duplicated
    seam without gluing would cut the tissue, so the periodic reading is taken);
  * node p = i + n_theta (j + (n_phi + 1) k) at parameters (theta_i, phi_j, r_k) on uniform grids
    (i periodic); element (i, j, k) has local node l = a + 2b + 4c at (i + a mod n_theta, j + b,
    k + c);
  * isoparametric trilinear elements: the geometry inside an element is the trilinear
    interpolation of its 8 nodal positions; 2x2x2 Gauss points; the lumped mass is the row sum of
    the consistent mass, int phi_p (exact with 2x2x2 Gauss points);
  * fibers: Sec. 2 describes fibers rotating counterclockwise from epi- (r = 1) to endocardium
    (r = 0), without angles; here a_l = cos(alpha) e_theta + sin(alpha) e_phi in the tangent frame of the
    parametrisation (e_theta = dX/dtheta normalised, e_phi the normalised part of dX/dphi
    orthogonal to it), alpha(r) = alpha_endo + r (alpha_epi - alpha_endo), alpha from +60 deg at
    the endocardium to -60 deg at the epicardium, evaluated at each Gauss point's parameters
    (the element-wise trilinear interpolation of the nodal (theta, phi, r));
  * axisymmetric tissue (sigma_n = sigma_t), as for the slab.

Every function takes a case with the attributes of bidomain_cases.EllipsoidCase (n_theta,
n_phi, n_r, the axes, the angle ranges, conductivities, fiber angles, cm, dt).
"""
from __future__ import annotations

import math
import numpy as np
import scipy.sparse as sp

from .fem import GAUSS_1D, GAUSS_W1D, local_node_bits


def nodes(e) -> int:
    return e.n_theta * (e.n_phi + 1) * (e.n_r + 1)


def parameters(e):
    """Nodal parameter grids (theta_i, phi_j, r_k)."""
    th = e.theta_min + (e.theta_max - e.theta_min) * np.arange(e.n_theta) / e.n_theta
    ph = e.phi_min + (e.phi_max - e.phi_min) * np.arange(e.n_phi + 1) / e.n_phi
    r = np.arange(e.n_r + 1) / e.n_r
    return th, ph, r


def position(e, th, ph, r):
    a = e.a1 + r * (e.a2 - e.a1)
    b = e.b1 + r * (e.b2 - e.b1)
    c = e.c1 + r * (e.c2 - e.c1)
    return np.stack([a * np.cos(th) * np.cos(ph), b * np.sin(th) * np.cos(ph), c * np.sin(ph)], axis=-1)


def node_positions(e) -> np.ndarray:
    th, ph, r = parameters(e)
    R, PH, TH = np.meshgrid(r, ph, th, indexing="ij")   # k slowest, i fastest
    return position(e, TH.ravel(), PH.ravel(), R.ravel())


def fiber_direction(e, th: float, ph: float, r: float) -> np.ndarray:
    a = e.a1 + r * (e.a2 - e.a1)
    b = e.b1 + r * (e.b2 - e.b1)
    c = e.c1 + r * (e.c2 - e.c1)
    d_th = np.array([-a * math.sin(th) * math.cos(ph), b * math.cos(th) * math.cos(ph), 0.0])
    d_ph = np.array([-a * math.cos(th) * math.sin(ph), -b * math.sin(th) * math.sin(ph), c * math.cos(ph)])
    e_th = d_th / np.linalg.norm(d_th)
    w = d_ph - (d_ph @ e_th) * e_th
    e_ph = w / np.linalg.norm(w)
    alpha = e.fiber_endo + r * (e.fiber_epi - e.fiber_endo)
    return math.cos(alpha) * e_th + math.sin(alpha) * e_ph


def conductivity(e, th, ph, r, sig_l, sig_t) -> np.ndarray:
    """Eq. (2) with sigma_n = sigma_t."""
    al = fiber_direction(e, th, ph, r)
    return sig_t * np.eye(3) + (sig_l - sig_t) * np.outer(al, al)


def element_nodes(e, i: int, j: int, k: int):
    """Global node of each local node l = a + 2b + 4c of element (i, j, k)."""
    out = []
    for l in range(8):
        a, b, c = local_node_bits(l)
        out.append((i + a) % e.n_theta + e.n_theta * ((j + b) + (e.n_phi + 1) * (k + c)))
    return out


def _ref_basis(xi, eta, zeta):
    """Trilinear basis values (8,) and reference gradients (8, 3) at a point of [0, 1]^3."""
    N = np.zeros(8)
    dN = np.zeros((8, 3))
    for l in range(8):
        a, b, c = local_node_bits(l)
        fx, fy, fz = (xi if a else 1 - xi), (eta if b else 1 - eta), (zeta if c else 1 - zeta)
        sx, sy, sz = (1.0 if a else -1.0), (1.0 if b else -1.0), (1.0 if c else -1.0)
        N[l] = fx * fy * fz
        dN[l] = (sx * fy * fz, fx * sy * fz, fx * fy * sz)
    return N, dN


def element_matrices(e, i: int, j: int, k: int, sig_l: float, sig_t: float):
    """(K_e, m_e): element stiffness int grad(N_m)^T D grad(N_l) and int N_l, 2x2x2 Gauss."""
    th, ph, r = parameters(e)
    dth = (e.theta_max - e.theta_min) / e.n_theta
    X = np.zeros((8, 3))
    for l in range(8):
        a, b, c = local_node_bits(l)
        X[l] = position(e, th[i] + a * dth, ph[j + b], r[k + c])
    K = np.zeros((8, 8))
    m = np.zeros(8)
    for gz, wz in zip(GAUSS_1D, GAUSS_W1D):
        for gy, wy in zip(GAUSS_1D, GAUSS_W1D):
            for gx, wx in zip(GAUSS_1D, GAUSS_W1D):
                N, dN = _ref_basis(gx, gy, gz)
                J = X.T @ dN                        # J[d, q] = d x_d / d xi_q
                detJ = np.linalg.det(J)
                G = dN @ np.linalg.inv(J)           # physical gradients, (8, 3)
                tg = th[i] + gx * dth
                pg = ph[j] + gy * (ph[j + 1] - ph[j])
                rg = r[k] + gz * (r[k + 1] - r[k])
                D = conductivity(e, tg, pg, rg, sig_l, sig_t)
                w = wx * wy * wz * detJ
                K += w * (G @ D @ G.T)
                m += w * N
    return 0.5 * (K + K.T), m


def assemble(e, sig_l: float, sig_t: float):
    """Global stiffness (27-point pattern, periodic in theta, structural zeros kept) and the
    lumped mass."""
    rows, cols, vals = [], [], []
    mass = np.zeros(nodes(e))
    for k in range(e.n_r):
        for j in range(e.n_phi):
            for i in range(e.n_theta):
                K, m = element_matrices(e, i, j, k, sig_l, sig_t)
                g = element_nodes(e, i, j, k)
                for l in range(8):
                    mass[g[l]] += m[l]
                    for q in range(8):
                        rows.append(g[l]); cols.append(g[q]); vals.append(K[l, q])
    A = sp.coo_matrix((vals, (rows, cols)), shape=(nodes(e), nodes(e))).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    return A, mass


def assemble_operators(e):
    """A_i, A_e, A_ell = A_i + A_e, A_par = (c_m / dt) M + A_i and the lumped mass m."""
    Ai, m = assemble(e, e.sig_il, e.sig_it)
    Ae, _ = assemble(e, e.sig_el, e.sig_et)
    Aell = (Ai + Ae).tocsr()
    Aell.sort_indices()
    Apar = (Ai + sp.diags(e.cm / e.dt * m)).tocsr()
    Apar.sort_indices()
    return dict(Ai=Ai, Ae=Ae, Aell=Aell, Apar=Apar, m=m)
