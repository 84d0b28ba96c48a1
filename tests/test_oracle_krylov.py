"""Pins for the oracle's smoothers, V-cycle and Krylov solvers (CPU only): the Chebyshev error
polynomial in closed form, the pseudo-inverse coarse solve, a dense two-grid operator built
from that closed form, V-cycle symmetry, PCG termination properties, exact dots against
rational arithmetic, and AMG-PCG against dense direct solves."""
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import bidomain_cases as bc
from oracle import amg, fem, krylov


def _cheb_error_factor(lam, lamhat, lo, hi):
    """T_2((theta - lam) / delta) / T_2(theta / delta) with T_2(t) = 2 t^2 - 1."""
    a, b = lo * lamhat, hi * lamhat
    theta, delta = (a + b) / 2, (b - a) / 2
    T2 = lambda t: 2 * t * t - 1
    return T2((theta - lam) / delta) / T2(theta / delta)


def test_chebyshev_error_polynomial_closed_form():
    rng = np.random.default_rng(0)
    Q = rng.standard_normal((10, 10))
    A = Q @ Q.T + 3 * np.eye(10)
    D = np.diag(np.diag(A))
    lams, Y = sla.eigh(A, D)
    lamhat = lams[-1] * 0.97
    As = sp.csr_matrix(A)
    Dinv = 1.0 / np.diag(A)
    for lam, y in zip(lams, Y.T):
        x = krylov.chebyshev(As, Dinv, A @ y, None, lamhat, 2, 0.05, 1.05)
        err = y - x
        np.testing.assert_allclose(err, _cheb_error_factor(lam, lamhat, 0.05, 1.05) * y, rtol=0,
                                   atol=1e-11 * np.abs(y).max())


def _small_hierarchy(nx, ny, nz, nullspace=True, **kw):
    c = bc.make_case(nx, ny, nz, seed=3)
    ops = fem.assemble_operators(c)
    A = ops["Aell"] if nullspace else ops["Apar"]
    opts = amg.AMGOptions(nullspace=nullspace, coarse_eq_limit=kw.pop("coarse_eq_limit", 4), **kw)
    return c, ops, A, amg.setup(A, opts)


def test_coarse_solve_is_pseudo_inverse_on_range():
    c, ops, A, h = _small_hierarchy(3, 3, 2, max_levels=1, coarse_eq_limit=1000)
    Ad = A.toarray()
    f = np.random.default_rng(1).standard_normal(Ad.shape[0])
    f -= f.mean()
    np.testing.assert_allclose(krylov.coarse_solve(h, f), np.linalg.pinv(Ad) @ f, rtol=0,
                               atol=1e-9 * np.abs(np.linalg.pinv(Ad) @ f).max())


def _vcycle_matrix(h, n):
    return np.column_stack([krylov.vcycle(h, e) for e in np.eye(n)])


def test_two_grid_matches_dense_closed_form():
    """Two levels, exact coarse solve: B = G + M - M A G with G = M + P A_c^+ R (I - A M) and
    the smoother M = q(D^{-1} A) D^{-1}, 1 - t q(t) = T_2((theta - t)/delta) / T_2(sigma)."""
    c, ops, A, h = _small_hierarchy(4, 4, 2, max_levels=2, coarse_eq_limit=4)
    assert h.nlevels == 2
    lv = h.levels[0]
    Ad = A.toarray()
    n = Ad.shape[0]
    lo, hi = h.opts.cheb_lo, h.opts.cheb_hi
    a, b = lo * lv.lam, hi * lv.lam
    theta, delta = (a + b) / 2, (b - a) / 2
    sigma = theta / delta
    T2s = 2 * sigma ** 2 - 1
    # p(t) = (2 ((theta - t)/delta)^2 - 1) / T2s = c0 + c1 t + c2 t^2 with c0 = 1; q(t) = -(c1 + c2 t)
    c1 = -4 * theta / delta ** 2 / T2s
    c2 = 2 / delta ** 2 / T2s
    S = np.diag(lv.Dinv) @ Ad
    M = -(c1 * np.eye(n) + c2 * S) @ np.diag(lv.Dinv)
    Ac = h.levels[1].A.toarray()
    P, R = lv.P.toarray(), lv.R.toarray()
    G = M + P @ np.linalg.pinv(Ac) @ R @ (np.eye(n) - Ad @ M)
    Bdense = G + M - M @ Ad @ G
    B = _vcycle_matrix(h, n)
    # compare on the range of A (the singular direction is projected by PCG anyway)
    Pi = np.eye(n) - np.ones((n, n)) / n
    np.testing.assert_allclose(B @ Pi, Bdense @ Pi, rtol=0, atol=1e-9 * np.abs(Bdense).max())


def test_vcycle_symmetric_positive():
    c, ops, A, h = _small_hierarchy(5, 5, 3, coarse_eq_limit=10, mis="greedy")
    assert h.nlevels >= 3
    n = A.shape[0]
    B = _vcycle_matrix(h, n)
    assert np.abs(B - B.T).max() <= 1e-12 * np.abs(B).max()
    Pi = np.eye(n) - np.ones((n, n)) / n
    ev = np.linalg.eigvalsh(Pi @ (0.5 * (B + B.T)) @ Pi)
    assert np.sort(ev)[1] > 0  # one zero eigenvalue along the constant, the rest positive


def test_pcg_exact_preconditioner_one_iteration():
    c, ops, A, h = _small_hierarchy(3, 3, 2, max_levels=1, coarse_eq_limit=1000)
    f = np.random.default_rng(2).standard_normal(A.shape[0])
    Apinv = np.linalg.pinv(A.toarray())
    res = krylov.pcg(A, f, lambda r: Apinv @ r, rtol=1e-10, nullspace=True)
    assert res.iterations == 1 and res.converged


def test_pcg_identity_terminates_within_n():
    rng = np.random.default_rng(4)
    n = 40
    Q = rng.standard_normal((n, n))
    A = sp.csr_matrix(Q @ Q.T / n + np.eye(n))
    res = krylov.pcg(A, rng.standard_normal(n), lambda r: r, rtol=1e-10)
    assert res.converged and res.iterations <= n


def test_fcg_equals_cg_in_double():
    c, ops, A, h = _small_hierarchy(6, 6, 3, coarse_eq_limit=20)
    f = -(ops["Ai"] @ bc.random_vector(A.shape[0], 9))
    r1 = krylov.pcg(A, f, lambda r: krylov.vcycle(h, r), rtol=1e-10, nullspace=True)
    r2 = krylov.fcg(A, f, lambda r: krylov.vcycle(h, r), rtol=1e-10, nullspace=True, lowp=np.float64)
    assert r1.iterations == r2.iterations
    np.testing.assert_allclose(r1.x, r2.x, rtol=0, atol=1e-9 * np.abs(r1.x).max())


def test_exact_dot_is_correctly_rounded():
    rng = np.random.default_rng(5)
    for n in (1, 7, 1000):
        x = rng.standard_normal(n).astype(np.float32) * np.float32(1e3)
        y = rng.standard_normal(n).astype(np.float32)
        exact = sum(Fraction(float(a)) * Fraction(float(b)) for a, b in zip(x, y))
        assert krylov.exact_dot(x, y) == float(exact)


@pytest.mark.parametrize("dims", [(2, 2, 1), (3, 3, 2), (4, 4, 2)])
def test_amg_pcg_matches_dense_pseudo_inverse_tiny(dims):
    c, ops, A, h = _small_hierarchy(*dims, coarse_eq_limit=4)
    f = -(ops["Ai"] @ bc.nodal_v0(bc.make_case(*dims, seed=3)))
    f = f + 1e-3 * bc.random_vector(A.shape[0], 1)  # make the load non-trivial on tiny meshes
    res = krylov.amg_pcg(A, f, h, rtol=1e-12, m=ops["m"])
    fh = f - f.mean()
    x = np.linalg.pinv(A.toarray()) @ fh
    x -= (ops["m"] @ x) / ops["m"].sum()
    assert np.linalg.norm(res.x - x) <= 1e-10 * np.linalg.norm(x)


@pytest.mark.slow
def test_amg_pcg_matches_dense_pseudo_inverse_c1():
    c = bc.config_case("C1")
    ops = fem.assemble_operators(c)
    A = ops["Aell"]
    h = amg.setup(A, amg.AMGOptions(nullspace=True))
    f = -(ops["Ai"] @ bc.nodal_v0(c))
    res = krylov.amg_pcg(A, f, h, rtol=1e-12, m=ops["m"])
    Ad = A.toarray()
    w, V = np.linalg.eigh(Ad)
    fh = f - f.mean()
    coef = V.T @ fh
    keep = w > 1e-12 * w[-1]
    x = V[:, keep] @ (coef[keep] / w[keep])
    x -= (ops["m"] @ x) / ops["m"].sum()
    assert np.linalg.norm(res.x - x) <= 1e-10 * np.linalg.norm(x)
    # and at the working tolerance, relative error and residual as the solver reports
    res8 = krylov.amg_pcg(A, f, h, rtol=1e-8, m=ops["m"])
    assert res8.rel_residual_true <= 1e-8
    assert np.linalg.norm(res8.x - x) <= 1e-6 * np.linalg.norm(x)


def test_parabolic_matches_dense_cholesky():
    c = bc.make_case(6, 6, 3, seed=2)
    ops = fem.assemble_operators(c)
    A = ops["Apar"]
    h = amg.setup(A, amg.AMGOptions(coarse_eq_limit=10, threshold=0.0))
    f = A @ bc.nodal_v0(c)
    res = krylov.amg_pcg(A, f, h, rtol=1e-12)
    x = sla.cho_solve(sla.cho_factor(A.toarray()), f)
    assert np.linalg.norm(res.x - x) <= 1e-10 * np.linalg.norm(x)


def test_mixed_fcg_reaches_tolerance_c1():
    c = bc.config_case("C1")
    ops = fem.assemble_operators(c)
    A = ops["Aell"]
    h = amg.setup(A, amg.AMGOptions(nullspace=True))
    f = -(ops["Ai"] @ bc.nodal_v0(c))
    r64 = krylov.amg_pcg(A, f, h, rtol=1e-8, m=ops["m"])
    r32 = krylov.amg_fcg_mixed(A, f, h, rtol=1e-8, m=ops["m"])
    assert r32.converged and r32.rel_residual_true <= 1e-8
    assert abs(r32.iterations - r64.iterations) <= 2


def _spd(n, seed):
    rng = np.random.default_rng(seed)
    Q = rng.standard_normal((n, n))
    d = rng.uniform(0.5, 50.0, n)                    # a badly scaled diagonal
    A = Q @ Q.T / n + np.diag(d)
    return sp.csr_matrix(A)


def test_diag_pcg_none_solves_and_terminates():
    """Unpreconditioned CG reaches the exact solution (dense LU) within n + a few steps."""
    n = 40
    A = _spd(n, 3)
    f = np.random.default_rng(4).standard_normal(n)
    res = krylov.diag_pcg(A, f, "none", rtol=1e-12, maxit=200)
    assert res.converged and res.iterations <= n + 5
    x = sla.solve(A.toarray(), f)
    assert np.linalg.norm(res.x - x) <= 1e-9 * np.linalg.norm(x)


@pytest.mark.parametrize("k", [1, 3, 7, 12])
def test_jacobi_pcg_is_cg_on_the_scaled_system(k):
    """k steps of Jacobi-preconditioned CG on A x = f equal k steps of plain CG on
    (D^-1/2 A D^-1/2) y = D^-1/2 f mapped back by x = D^-1/2 y (an identity of the method)."""
    n = 30
    A = _spd(n, 5)
    f = np.random.default_rng(6).standard_normal(n)
    s = 1.0 / np.sqrt(A.diagonal())
    As = sp.diags(s) @ A @ sp.diags(s)
    xj = krylov.diag_pcg(A, f, "jacobi", rtol=1e-300, maxit=k).x
    ys = krylov.diag_pcg(As, s * f, "none", rtol=1e-300, maxit=k).x
    assert np.linalg.norm(xj - s * ys) <= 1e-11 * np.linalg.norm(xj)


def test_jacobi_on_a_scaled_identity_diagonal_is_plain_cg():
    """With diag(A) = c I the Jacobi preconditioner is a scalar: the iterates are plain CG's."""
    n = 25
    rng = np.random.default_rng(7)
    Q = rng.standard_normal((n, n))
    A = Q @ Q.T / n + 3.0 * np.eye(n)
    A[np.diag_indices(n)] = 7.5                       # the same diagonal everywhere (still SPD)
    A = sp.csr_matrix(A)
    f = rng.standard_normal(n)
    for k in (2, 5, 9):
        a = krylov.diag_pcg(A, f, "jacobi", rtol=1e-300, maxit=k).x
        b = krylov.diag_pcg(A, f, "none", rtol=1e-300, maxit=k).x
        assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(b)



@pytest.mark.parametrize("degree", [1, 2, 3])
def test_jacobi_error_factor_per_eigenpair(degree):
    """Damped Jacobi with omega = 4/(3 lambda_hat) from x0 = 0: for an eigenpair (lam, y) of
    D^-1 A and f = A y, each sweep multiplies the error by (1 - omega lam), so after d sweeps
    y - x = (1 - omega lam)^d y."""
    rng = np.random.default_rng(8)
    Q = rng.standard_normal((10, 10))
    A = Q @ Q.T + 3 * np.eye(10)
    lams, Y = sla.eigh(A, np.diag(np.diag(A)))
    lamhat = lams[-1] * 1.1
    omega = 4.0 / (3.0 * lamhat)
    As, Dinv = sp.csr_matrix(A), 1.0 / np.diag(A)
    for lam, y in zip(lams, Y.T):
        x = krylov.jacobi(As, Dinv, A @ y, None, lamhat, degree)
        np.testing.assert_allclose(y - x, (1 - omega * lam) ** degree * y, rtol=0,
                                   atol=1e-12 * np.abs(y).max())


def test_smooth_dispatches_jacobi_with_degree_sweeps():
    c, ops, A, h = _small_hierarchy(3, 3, 2, smoother="jacobi", degree=3, coarse_eq_limit=4)
    lv = h.levels[0]
    f = bc.random_vector(A.shape[0], 2)
    omega = 4.0 / (3.0 * lv.lam)
    x = np.zeros_like(f)
    for _ in range(3):
        x = x + omega * lv.Dinv * (f - lv.A @ x)
    np.testing.assert_allclose(krylov.smooth(h, 0, f, None), x, rtol=0, atol=1e-14 * np.abs(x).max())


class _Recorder:
    """Wraps a matrix and records every vector it multiplies (the search directions p_k)."""

    def __init__(self, A):
        self.A, self.seen = A, []

    def __matmul__(self, v):
        self.seen.append(np.array(v, dtype=np.float64))
        return self.A @ v


def _varying_preconditioner(n, seed):
    """z = C_k r with a different random positive diagonal C_k at every call."""
    rng = np.random.default_rng(seed)
    return lambda r: rng.uniform(0.2, 5.0, n).astype(r.dtype) * r


def test_fcg_local_a_orthogonality_with_varying_preconditioner():
    """Flexible CG, FCG(1) (Notay 2000): beta_k = z_{k+1}^T (r_{k+1} - r_k) / (z_k^T r_k) makes
    consecutive directions A-orthogonal, p_{k+1}^T A p_k = 0, for any preconditioner, because
    A p_k = (r_k - r_{k+1}) / alpha_k and alpha_k = rho_k / p_k^T A p_k.  Plain CG's
    beta = z_{k+1}^T r_{k+1} / rho_k leaves p_{k+1}^T A p_k = (p_k^T A p_k) z_{k+1}^T r_k / rho_k,
    which is nonzero once the preconditioner changes between iterations."""
    n = 30
    A = _spd(n, 11)
    f = np.random.default_rng(12).standard_normal(n)

    def directions(solver):
        rec = _Recorder(A)
        solver(rec)
        return rec.seen[1:-1]                # drop the initial and final residual products

    ps = directions(lambda M: krylov.fcg(M, f, _varying_preconditioner(n, 1), rtol=1e-300,
                                         maxit=8, lowp=np.float64))
    assert len(ps) == 8
    Ad = A.toarray()
    for p0, p1 in zip(ps, ps[1:]):
        assert abs(p1 @ Ad @ p0) <= 1e-12 * np.linalg.norm(p1) * np.linalg.norm(Ad @ p0)
    # the same check separates plain CG's beta under the same varying preconditioner
    qs = directions(lambda M: krylov.pcg(M, f, _varying_preconditioner(n, 1), rtol=1e-300, maxit=8))
    worst = max(abs(p1 @ Ad @ p0) / (np.linalg.norm(p1) * np.linalg.norm(Ad @ p0))
                for p0, p1 in zip(qs, qs[1:]))
    assert worst > 1e-3


def test_fcg_two_steps_by_hand():
    """Two FCG(1) steps on a 3x3 system written out: r0 = f, z0 = C0 r0, p0 = z0,
    alpha0 = z0.r0 / p0.A p0, r1 = r0 - alpha0 A p0, z1 = C1 r1, beta0 = z1.(r1 - r0) / z0.r0,
    p1 = z1 + beta0 p0, alpha1 = z1.r1 / p1.A p1, x2 = alpha0 p0 + alpha1 p1."""
    A = np.array([[4., 1, 0], [1, 3, 1], [0, 1, 2]])
    f = np.array([1., 2, 3])
    C = [np.array([1.0, 0.5, 2.0]), np.array([0.3, 1.5, 0.7]), np.ones(3)]
    calls = iter(C)                          # the third call follows the last step, unused
    res = krylov.fcg(sp.csr_matrix(A), f, lambda r: next(calls) * r, rtol=1e-300, maxit=2,
                     lowp=np.float64)
    r0 = f.copy(); z0 = C[0] * r0; p0 = z0.copy()
    a0 = (z0 @ r0) / (p0 @ A @ p0)
    r1 = r0 - a0 * (A @ p0); z1 = C[1] * r1
    b0 = (z1 @ (r1 - r0)) / (z0 @ r0)
    p1 = z1 + b0 * p0
    a1 = (z1 @ r1) / (p1 @ A @ p1)
    np.testing.assert_allclose(res.x, a0 * p0 + a1 * p1, rtol=1e-14)
