"""Pins for the oracle's Q1 assembly (CPU only).

Each test checks the oracle against something the paper or the mathematics fixes:
printed node counts, closed-form element matrices, the textbook isotropic stencil,
exact invariants, and O(h^2) convergence to manufactured solutions.
"""
import json
import math
import os
from dataclasses import replace

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import bidomain_cases as bc
from oracle import fem

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_dof_counts_match_paper_tables():
    g = json.load(open(os.path.join(GOLDEN, "paper_dofs.json")))
    for row in g["rows"]:
        nx, ny, nz = row["elements"]
        assert nx * ny * nz == 4096 * row["workers"]
        assert bc.SlabCase(nx, ny, nz).paper_dofs == row["dofs"]
    pw = g["per_worker"]
    assert bc.SlabCase(*pw["elements"]).paper_dofs == pw["dofs"]


def test_pattern_size_and_sorted_columns():
    c = bc.make_case(5, 4, 3, seed=0)
    A = fem.assemble_stiffness(c, 1e-3, 2e-4)
    assert A.shape == (c.n, c.n)
    assert A.nnz == c.nnz27
    for i in range(c.n):
        cols = A.indices[A.indptr[i]:A.indptr[i + 1]]
        assert np.all(np.diff(cols) > 0)


def _closed_form_element(D, hx, hy, hz):
    """K_e = sum_ab D_ab  kron(F_z, kron(F_y, F_x)) with 1-D factors: stiffness K1 on the axis
    differentiated twice, gradient-mass C1 (or its transpose) on an axis differentiated once,
    mass M1 otherwise; local index l = a + 2b + 4c (x fastest)."""
    def K1(h): return np.array([[1.0, -1.0], [-1.0, 1.0]]) / h
    def M1(h): return np.array([[2.0, 1.0], [1.0, 2.0]]) * h / 6.0
    def C1(h): return np.array([[-0.5, -0.5], [0.5, 0.5]])  # int N_i' N_j, derivative on row index
    hs = (hx, hy, hz)
    K = np.zeros((8, 8))
    for a in range(3):
        for b in range(3):
            F = []
            for d in range(3):
                if d == a and d == b:
                    F.append(K1(hs[d]))
                elif d == a:
                    F.append(C1(hs[d]))
                elif d == b:
                    F.append(C1(hs[d]).T)
                else:
                    F.append(M1(hs[d]))
            K += D[a, b] * np.kron(F[2], np.kron(F[1], F[0]))
    return K


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_element_stiffness_closed_form_constant_D(seed):
    rng = np.random.default_rng(seed)
    hx, hy, hz = rng.uniform(0.01, 0.2, 3)
    c = bc.SlabCase(4, 4, 4, Lx=4 * hx, Ly=4 * hy, Lz=4 * hz,
                    fiber_theta0=float(rng.uniform(-3, 3)), fiber_rotation=0.0)
    sl, st = rng.uniform(1e-4, 5e-3, 2)
    K = fem.element_stiffness(c, 2, sl, st)
    D = fem.conductivity(0.0, sl, st, c)
    K_ref = _closed_form_element(D, hx, hy, hz)
    assert np.max(np.abs(K - K_ref)) <= 1e-14 * np.max(np.abs(K_ref))


def test_isotropic_unit_stencil():
    g = json.load(open(os.path.join(GOLDEN, "q1_isotropic_stencil.json")))
    h = 0.25
    c = bc.SlabCase(4, 4, 4, Lx=1.0, Ly=1.0, Lz=1.0)
    A = fem.assemble_stiffness(c, 1.0, 1.0)
    p = 2 + 5 * (2 + 5 * 2)  # interior node (2, 2, 2)
    row = A.getrow(p).toarray().ravel()
    for dk in (-1, 0, 1):
        for dj in (-1, 0, 1):
            for di in (-1, 0, 1):
                q = p + di + 5 * dj + 25 * dk
                nonzero_axes = abs(di) + abs(dj) + abs(dk)
                key = ["center", "face", "edge", "corner"][nonzero_axes]
                assert row[q] == pytest.approx(g[key] * h / g["h"], abs=1e-15)


def test_symmetry_and_constant_kernel():
    c = bc.config_case("C1")
    ops = fem.assemble_operators(c)
    for key in ("Ai", "Ae", "Aell"):
        A = ops[key]
        assert (A - A.T).count_nonzero() == 0
        assert np.max(np.abs(A @ np.ones(c.n))) <= 1e-14 * np.max(np.abs(A.data))
    # parabolic operator: A_par 1 = (c_m / dt) m
    assert np.allclose(ops["Apar"] @ np.ones(c.n), c.cm / c.dt * ops["m"], rtol=0, atol=1e-14 * ops["Apar"].max())


def test_lumped_mass_closed_form():
    c = bc.make_case(6, 5, 4, seed=0)
    m = fem.lumped_mass(c)
    hx, hy, hz = c.h
    vol = hx * hy * hz
    nxp, nyp = c.nx + 1, c.ny + 1
    for (i, j, k), factor in [((3, 2, 2), 1.0), ((0, 2, 2), 0.5), ((0, 0, 2), 0.25), ((0, 0, 0), 0.125),
                              ((6, 5, 4), 0.125), ((6, 2, 4), 0.25)]:
        assert m[i + nxp * (j + nyp * k)] == pytest.approx(factor * vol, rel=1e-15)
    assert m.sum() == pytest.approx(c.Lx * c.Ly * c.Lz, rel=1e-14)


# ------------------------------------------------------------------------------------------------
# Manufactured solutions: Neumann problem -div(D grad u) = f, D grad u . n = g, zero-mean u.
def _solve_neumann(A, b, m):
    """Solve the singular consistent system by pinning node 0, then remove the m-weighted mean."""
    n = A.shape[0]
    A = A.tolil()
    A[0, :] = 0.0
    A[0, 0] = 1.0
    b = b.copy()
    b[0] = 0.0
    u = spla.spsolve(A.tocsc(), b)
    return u - (m @ u) / m.sum()


def _errors(case, A, load, u_exact):
    m = fem.lumped_mass(case)
    uh = _solve_neumann(A, load, m)
    ue = u_exact - (m @ u_exact) / m.sum()
    return np.max(np.abs(uh - ue)), math.sqrt(m @ (uh - ue) ** 2)


def _boundary_load(case, flux):
    """int over boundary faces of g phi_p, 2x2 Gauss per face; flux(x, y, z, nvec) -> g."""
    nxp, nyp = case.nx + 1, case.ny + 1
    hx, hy, hz = case.h
    b = np.zeros(case.n)
    g1 = fem.GAUSS_1D
    def add_face(axis, side):
        dims = [case.nx, case.ny, case.nz]
        hs = [hx, hy, hz]
        t1, t2 = [d for d in range(3) if d != axis]
        nvec = np.zeros(3)
        nvec[axis] = 1.0 if side else -1.0
        for e1 in range(dims[t1]):
            for e2 in range(dims[t2]):
                for s1 in g1:
                    for s2 in g1:
                        X = np.zeros(3)
                        X[axis] = side * [case.Lx, case.Ly, case.Lz][axis]
                        X[t1] = (e1 + s1) * hs[t1]
                        X[t2] = (e2 + s2) * hs[t2]
                        g = flux(X, nvec) * 0.25 * hs[t1] * hs[t2]
                        for a1 in (0, 1):
                            for a2 in (0, 1):
                                w = (s1 if a1 else 1 - s1) * (s2 if a2 else 1 - s2)
                                idx = [0, 0, 0]
                                idx[axis] = side * dims[axis]
                                idx[t1] = e1 + a1
                                idx[t2] = e2 + a2
                                b[idx[0] + nxp * (idx[1] + nyp * idx[2])] += g * w
    for axis in range(3):
        for side in (0, 1):
            add_face(axis, side)
    return b


def _convergence(make, sizes):
    errs = []
    for nx, ny, nz in sizes:
        errs.append(make(nx, ny, nz))
    return errs


def _check_rates(errs, max_rate=3.6):
    for (emax0, el20), (emax1, el21) in zip(errs, errs[1:]):
        assert emax0 / emax1 >= max_rate, errs
        assert el20 / el21 >= 3.6, errs


SIZES = [(8, 8, 4), (16, 16, 8), (32, 32, 16)]


@pytest.mark.slow
def test_manufactured_aligned_anisotropic():
    """Fibers along x (no rotation): D = diag(sl, st, st); u = cos(pi x/Lx) cos(pi y/Ly) cos(pi z/Lz)
    satisfies the homogeneous Neumann condition and -div(D grad u) = kappa u."""
    sl, st = 3e-3, 3.1525e-4
    def run(nx, ny, nz):
        c = bc.SlabCase(nx, ny, nz, fiber_theta0=0.0, fiber_rotation=0.0)
        X, Y, Z = bc.node_coordinates(c)
        u = np.cos(np.pi * X / c.Lx) * np.cos(np.pi * Y / c.Ly) * np.cos(np.pi * Z / c.Lz)
        kappa = sl * (np.pi / c.Lx) ** 2 + st * (np.pi / c.Ly) ** 2 + st * (np.pi / c.Lz) ** 2
        A = fem.assemble_stiffness(c, sl, st)
        return _errors(c, A, fem.lumped_mass(c) * kappa * u, u)
    _check_rates(_convergence(run, SIZES))


@pytest.mark.slow
def test_manufactured_rotating_fibers_transmural():
    """Rotating in-plane fibers; u = cos(pi z / Lz) has D grad u = st grad u (a_l is in-plane),
    so the Neumann condition holds and -div(D grad u) = st (pi/Lz)^2 u."""
    sl, st = 2e-3, 1.3514e-3
    def run(nx, ny, nz):
        c = bc.SlabCase(nx, ny, nz)
        X, Y, Z = bc.node_coordinates(c)
        u = np.cos(np.pi * Z / c.Lz)
        A = fem.assemble_stiffness(c, sl, st)
        return _errors(c, A, fem.lumped_mass(c) * st * (np.pi / c.Lz) ** 2 * u, u)
    _check_rates(_convergence(run, SIZES))


@pytest.mark.slow
def test_manufactured_rotating_fibers_in_plane_with_flux():
    """Rotating fibers and u = cos(pi x/Lx) cos(pi y/Ly): -div(D grad u) = -st Lap u - (sl-st) a^T H a
    (a depends on z only and has no z component), with boundary flux g = n^T D grad u."""
    sl, st = 3e-3, 3.1525e-4
    def run(nx, ny, nz):
        c = bc.SlabCase(nx, ny, nz)
        kx, ky = np.pi / c.Lx, np.pi / c.Ly
        def grad(X):
            x, y = X[0], X[1]
            return np.array([-kx * math.sin(kx * x) * math.cos(ky * y), -ky * math.cos(kx * x) * math.sin(ky * y), 0.0])
        def flux(X, nvec):
            a = np.array([math.cos(c.fiber_theta0 + c.fiber_rotation * X[2] / c.Lz),
                          math.sin(c.fiber_theta0 + c.fiber_rotation * X[2] / c.Lz), 0.0])
            gu = grad(X)
            return float(nvec @ (st * gu + (sl - st) * (a @ gu) * a))
        X, Y, Z = bc.node_coordinates(c)
        u = np.cos(kx * X) * np.cos(ky * Y)
        th = c.fiber_theta0 + c.fiber_rotation * Z / c.Lz
        ax, ay = np.cos(th), np.sin(th)
        uxx = -kx * kx * u
        uyy = -ky * ky * u
        uxy = kx * ky * np.sin(kx * X) * np.sin(ky * Y)
        f = -st * (uxx + uyy) - (sl - st) * (ax * ax * uxx + 2 * ax * ay * uxy + ay * ay * uyy)
        A = fem.assemble_stiffness(c, sl, st)
        load = fem.lumped_mass(c) * f + _boundary_load(c, flux)
        return _errors(c, A, load, u)
    # The nodal max error sits on the vertical edges where two flux faces meet; with the
    # lumped-mass load its rate approaches 4 slowly (2.9, 3.06, 3.23 measured up to 64x64x32),
    # so the max-norm bar is 2.8 here; the L2 bar stays 3.6.  A wrong or dropped term gives
    # an error that does not decrease at all.
    _check_rates(_convergence(run, SIZES), max_rate=2.8)
