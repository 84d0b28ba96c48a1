"""Pins of the oracle's truncated-ellipsoid Q1 operators (Sec. 3, eq. (8), Table 1; Sec. 2.2)
against facts that do not come from the oracle: the paper's node counts, the exact volume of the
shell (closed form, approached at second order by the trilinear geometry), the exactness of the
isoparametric Q1 space on linear functions (patch test: interior rows of the isotropic stiffness
annihilate a linear function exactly; its energy is sigma |g|^2 times the mesh volume), the
rotational symmetry of Table 1's spheroid (a shift by one element in theta is a rotation about z,
so it maps the operators onto themselves, seam included), and the fiber frame's invariants."""
import json
import math
import os
from dataclasses import replace

import numpy as np
import pytest

import bidomain_cases as bc
from oracle import ellipsoid as el

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "paper_ellipsoid_nodes.json")


def test_node_counts_match_the_paper():
    g = json.load(open(GOLD))
    for row in g["rows"]:
        c = bc.EllipsoidCase(*row["elements"])
        assert el.nodes(c) == row["nodes"] == c.n
    t = g["table1"]
    c = bc.EllipsoidCase(4, 4, 2)
    assert (c.a1, c.a2, c.b1, c.b2, c.c1, c.c2) == (t["a1"], t["a2"], t["b1"], t["b2"], t["c1"], t["c2"])
    assert c.theta_min == -1.5 * math.pi and c.theta_max == 0.5 * math.pi
    assert c.phi_min == -0.375 * math.pi and c.phi_max == 0.125 * math.pi


def _exact_volume(c):
    """Volume of the shell {x(theta, phi, r)}: the Jacobian of eq. (8)'s map is
    cos(phi) [a' b c cos^2(theta) cos^2(phi) + a b' c sin^2(theta) cos^2(phi) + a b c' sin^2(phi)]
    (with the axes linear in r); over a full theta period cos^2 and sin^2 integrate to pi."""
    s0, s1 = math.sin(c.phi_min), math.sin(c.phi_max)
    i_cos3 = (s1 - s1 ** 3 / 3) - (s0 - s0 ** 3 / 3)      # int cos^3(phi)
    i_cos_sin2 = (s1 ** 3 - s0 ** 3) / 3                   # int cos(phi) sin^2(phi)
    da, db, dc = c.a2 - c.a1, c.b2 - c.b1, c.c2 - c.c1
    # r-integrals of products of three linear functions: Simpson's rule is exact for cubics
    f = lambda g: (g(0.0) + 4 * g(0.5) + g(1.0)) / 6
    a = lambda r: c.a1 + r * da
    b = lambda r: c.b1 + r * db
    cc = lambda r: c.c1 + r * dc
    return (math.pi * i_cos3 * f(lambda r: da * b(r) * cc(r) + a(r) * db * cc(r))
            + 2 * math.pi * i_cos_sin2 * f(lambda r: a(r) * b(r) * dc))


def test_lumped_mass_converges_to_the_shell_volume_at_second_order():
    errs = []
    for k in (1, 2, 4):
        c = bc.EllipsoidCase(8 * k, 4 * k, 1)   # the trilinear geometry is exact in r
        _, m = el.assemble(c, 1.0, 1.0)
        errs.append(abs(m.sum() - _exact_volume(c)) / _exact_volume(c))
    assert errs[0] > errs[1] > errs[2]
    for e0, e1 in zip(errs, errs[1:]):
        assert 3.6 < e0 / e1 < 4.4
    assert errs[2] < 2e-2


def _interior(c):
    j = np.tile(np.repeat(np.arange(c.n_phi + 1), c.n_theta), c.n_r + 1)
    k = np.repeat(np.arange(c.n_r + 1), c.n_theta * (c.n_phi + 1))
    return (j > 0) & (j < c.n_phi) & (k > 0) & (k < c.n_r)


@pytest.mark.parametrize("dims", [(6, 5, 3), (9, 4, 4)])
def test_isotropic_patch_test(dims):
    c = bc.EllipsoidCase(*dims)
    A, m = el.assemble(c, 0.7, 0.7)        # D = 0.7 I
    X = el.node_positions(c)
    g = np.array([0.3, -1.1, 0.8])
    u = X @ g
    Au = A @ u
    inner = _interior(c)
    assert inner.sum() > 0
    assert np.max(np.abs(Au[inner])) <= 1e-12 * np.max(np.abs(A.data)) * np.max(np.abs(u))
    assert np.max(np.abs(Au[~inner])) > 1e-6          # boundary rows carry the flux
    energy = u @ Au
    assert energy == pytest.approx(0.7 * (g @ g) * m.sum(), rel=1e-12)


def test_stiffness_is_symmetric_and_annihilates_constants():
    c = bc.EllipsoidCase(7, 5, 3)
    ops = el.assemble_operators(c)
    for key in ("Ai", "Ae", "Aell"):
        A = ops[key]
        assert abs(A - A.T).max() <= 1e-15 * abs(A).max()
        assert np.max(np.abs(A @ np.ones(A.shape[0]))) <= 1e-14 * abs(A).max()
    # the full 27-point pattern, periodic in theta
    assert ops["Aell"].nnz == c.nnz27
    # positive definite once the mass is added
    lam = np.linalg.eigvalsh(ops["Apar"].toarray())
    assert lam.min() > 0


def test_theta_shift_is_a_symmetry_of_the_spheroid():
    """a1 = b1 and a2 = b2 (Table 1): shifting every node by one element in theta rotates the
    mesh about z, fibers included, so P A P^T = A (the seam elements included)."""
    c = bc.EllipsoidCase(6, 4, 2)
    ops = el.assemble_operators(c)
    nt = c.n_theta
    p = np.arange(c.n)
    shifted = (p % nt + 1) % nt + nt * (p // nt)
    for key in ("Ai", "Aell"):
        A = ops[key].toarray()
        B = A[np.ix_(shifted, shifted)]
        assert np.max(np.abs(A - B)) <= 1e-13 * np.max(np.abs(A))
    np.testing.assert_allclose(ops["m"][shifted], ops["m"], rtol=1e-13)
    # and the symmetry breaks when a != b, as it must
    c2 = replace(c, b1=2.0, b2=3.0)
    A2 = el.assemble_operators(c2)["Ai"].toarray()
    assert np.max(np.abs(A2 - A2[np.ix_(shifted, shifted)])) > 1e-6 * np.max(np.abs(A2))


def test_fiber_frame():
    """Unit fibers tangent to the r-surface; the angle from the theta direction is +60 deg at the
    endocardium and -60 deg at the epicardium, so seen from outside (along the inward normal)
    fibers turn counterclockwise from epi- to endocardium (Sec. 2)."""
    c = bc.EllipsoidCase(8, 8, 4)
    rng = np.random.default_rng(0)
    h = 1e-6
    for _ in range(20):
        th = rng.uniform(c.theta_min, c.theta_max)
        ph = rng.uniform(c.phi_min, c.phi_max)
        r = rng.uniform(0, 1)
        X = lambda t, p, rr: el.position(c, t, p, rr)
        d_th = (X(th + h, ph, r) - X(th - h, ph, r)) / (2 * h)
        d_ph = (X(th, ph + h, r) - X(th, ph - h, r)) / (2 * h)
        d_r = (X(th, ph, r + h) - X(th, ph, r - h)) / (2 * h)
        nrm = np.cross(d_th, d_ph)
        nrm /= np.linalg.norm(nrm)
        assert nrm @ d_r > 0                          # outward, towards the epicardium
        for rr, want in ((0.0, math.pi / 3), (1.0, -math.pi / 3)):
            a = el.fiber_direction(c, th, ph, rr)
            assert np.linalg.norm(a) == pytest.approx(1.0, abs=1e-14)
            n2 = np.cross((X(th + h, ph, rr) - X(th - h, ph, rr)), (X(th, ph + h, rr) - X(th, ph - h, rr)))
            n2 /= np.linalg.norm(n2)
            assert abs(a @ n2) < 1e-8
            e_th = X(th + h, ph, rr) - X(th - h, ph, rr)
            e_th /= np.linalg.norm(e_th)
            ang = math.atan2(np.cross(e_th, a) @ n2, e_th @ a)
            assert ang == pytest.approx(want, abs=1e-7)
        # counterclockwise about the outward normal from r = 1 to r = 0
        a_epi, a_endo = el.fiber_direction(c, th, ph, 1.0), el.fiber_direction(c, th, ph, 0.0)
        assert np.cross(a_epi, a_endo) @ nrm > 0


def test_conductivity_eigenstructure():
    c = bc.EllipsoidCase(8, 8, 4)
    D = el.conductivity(c, 0.3, -0.4, 0.6, 3e-3, 3e-4)
    a = el.fiber_direction(c, 0.3, -0.4, 0.6)
    w, V = np.linalg.eigh(D)
    np.testing.assert_allclose(w, [3e-4, 3e-4, 3e-3], rtol=1e-12)
    assert abs(abs(V[:, 2] @ a) - 1) < 1e-12


def test_stimulus_block_lies_at_the_apical_endocardium():
    c = bc.ellipsoid_case("E1")
    v0 = bc.ellipsoid_v0(c)
    X = el.node_positions(c)
    on = v0 == c.v_plateau
    assert 0 < on.sum() < c.n // 20
    assert X[on, 2].max() < X[:, 2].min() + 0.35 * (X[:, 2].max() - X[:, 2].min())


def _element_corners(c, i, j, k):
    th, ph, r = el.parameters(c)
    dth = (c.theta_max - c.theta_min) / c.n_theta
    P = np.zeros((2, 2, 2, 3))     # P[a, b, cc] = node at local offset (a, b, cc)
    Q = np.zeros((2, 2, 2, 3))     # its parameters (theta, phi, r)
    for a in (0, 1):
        for b in (0, 1):
            for cc in (0, 1):
                Q[a, b, cc] = (th[i] + a * dth, ph[j + b], r[k + cc])
                P[a, b, cc] = el.position(c, *Q[a, b, cc])
    return P, Q


def _trilinear(C, s, t, u):
    return ((1 - s) * (1 - t) * (1 - u) * C[0, 0, 0] + s * (1 - t) * (1 - u) * C[1, 0, 0]
            + (1 - s) * t * (1 - u) * C[0, 1, 0] + s * t * (1 - u) * C[1, 1, 0]
            + (1 - s) * (1 - t) * u * C[0, 0, 1] + s * (1 - t) * u * C[1, 0, 1]
            + (1 - s) * t * u * C[0, 1, 1] + s * t * u * C[1, 1, 1])


def test_element_volumes_by_the_divergence_theorem():
    """Sum of the lumped mass = volume of the trilinear mesh, computed here from its faces alone:
    V_e = 1/3 of the flux of x through the six bilinear faces (3-point Gauss per direction, exact
    for the cubic integrand)."""
    c = replace(bc.EllipsoidCase(6, 5, 2), b1=2.0, b2=3.1)
    _, m = el.assemble(c, 1.0, 1.0)
    x3, w3 = np.polynomial.legendre.leggauss(3)
    x3, w3 = 0.5 * (x3 + 1), 0.5 * w3
    h = 1e-6
    total = 0.0
    for k in range(c.n_r):
        for j in range(c.n_phi):
            for i in range(c.n_theta):
                P, _ = _element_corners(c, i, j, k)
                X = lambda s, t, u: _trilinear(P, s, t, u)
                for ax in range(3):
                    for side in (0.0, 1.0):
                        sign = 1.0 if side else -1.0
                        for s, ws in zip(x3, w3):
                            for t, wt in zip(x3, w3):
                                # face coordinates (s, t) follow the cyclic order after `ax`
                                def pt(a, b):
                                    q = [0.0, 0.0, 0.0]
                                    q[ax], q[(ax + 1) % 3], q[(ax + 2) % 3] = side, a, b
                                    return X(*q)
                                xs = (pt(s + h, t) - pt(s - h, t)) / (2 * h)
                                xt = (pt(s, t + h) - pt(s, t - h)) / (2 * h)
                                total += sign * ws * wt * (pt(s, t) @ np.cross(xs, xt)) / 3.0
    assert m.sum() == pytest.approx(total, rel=1e-9)


def test_one_element_stiffness_by_brute_force():
    """One anisotropic element matrix recomputed independently: finite-difference Jacobians of the
    trilinear map, gradients from J^T grad = reference gradient, fiber taken at the trilinear
    interpolation of the nodal parameters, at the 2x2x2 Gauss points."""
    c = replace(bc.EllipsoidCase(5, 4, 2), b1=2.0, b2=3.1)
    i, j, k = 3, 2, 1
    K, mvec = el.element_matrices(c, i, j, k, 3e-3, 3e-4)
    P, Q = _element_corners(c, i, j, k)
    g = [0.5 - 0.5 / math.sqrt(3), 0.5 + 0.5 / math.sqrt(3)]
    h = 1e-6
    Kb = np.zeros((8, 8))
    mb = np.zeros(8)
    for s in g:
        for t in g:
            for u in g:
                X = lambda a, b, cc: _trilinear(P, a, b, cc)
                J = np.column_stack([(X(s + h, t, u) - X(s - h, t, u)) / (2 * h),
                                     (X(s, t + h, u) - X(s, t - h, u)) / (2 * h),
                                     (X(s, t, u + h) - X(s, t, u - h)) / (2 * h)])
                D = el.conductivity(c, *_trilinear(Q, s, t, u), 3e-3, 3e-4)
                grads, vals = [], []
                for l in range(8):
                    a, b, cc = l & 1, (l >> 1) & 1, (l >> 2) & 1
                    E = np.zeros((2, 2, 2))
                    E[a, b, cc] = 1.0
                    ref = np.array([(_trilinear(E, s + h, t, u) - _trilinear(E, s - h, t, u)) / (2 * h),
                                    (_trilinear(E, s, t + h, u) - _trilinear(E, s, t - h, u)) / (2 * h),
                                    (_trilinear(E, s, t, u + h) - _trilinear(E, s, t, u - h)) / (2 * h)])
                    grads.append(np.linalg.solve(J.T, ref))
                    vals.append(_trilinear(E, s, t, u))
                G = np.array(grads)
                wdet = 0.125 * np.linalg.det(J)
                Kb += wdet * G @ D @ G.T
                mb += wdet * np.array(vals)
    assert np.max(np.abs(K - Kb)) <= 1e-7 * np.max(np.abs(K))
    np.testing.assert_allclose(mvec, mb, rtol=1e-8)


def test_fiber_frame_on_a_general_ellipsoid():
    """With a != b the theta and phi directions are not orthogonal; the fiber still has unit
    length, lies in the tangent plane and makes the prescribed angle with the theta direction."""
    c = replace(bc.EllipsoidCase(8, 8, 4), b1=1.6, b2=2.9)
    rng = np.random.default_rng(1)
    h = 1e-6
    for _ in range(20):
        th, ph, r = rng.uniform(c.theta_min, c.theta_max), rng.uniform(c.phi_min, c.phi_max), rng.uniform(0, 1)
        X = lambda t, p: el.position(c, t, p, r)
        e_th = X(th + h, ph) - X(th - h, ph)
        d_ph = X(th, ph + h) - X(th, ph - h)
        nrm = np.cross(e_th, d_ph)
        nrm /= np.linalg.norm(nrm)
        e_th /= np.linalg.norm(e_th)
        a = el.fiber_direction(c, th, ph, r)
        want = c.fiber_endo + r * (c.fiber_epi - c.fiber_endo)
        assert np.linalg.norm(a) == pytest.approx(1.0, abs=1e-14)
        assert abs(a @ nrm) < 1e-8
        assert math.atan2(np.cross(e_th, a) @ nrm, e_th @ a) == pytest.approx(want, abs=1e-7)
