"""Smoothers, V-cycle, coarse solve and (flexible) PCG (oracle; test infrastructure only).

Paper: Alg. 2 (MGV: mu1 pre-smoothing steps, residual, restriction, recursive call,
interpolation, correction, mu2 post-smoothing steps; direct solve on the coarsest level);
Sec. 4 (Richardson-Jacobi smoothing u <- u + omega S^{-1} (f - A u)); App. A (Chebyshev
smoother of degree 2 on Jacobi-scaled A, interval [0.05, 1.05] x lambda_max); Sec. 2.2
(PCG for the SPD parabolic and the positive semi-definite elliptic system); Sec. 2.1 (the
extracellular potential lives in the zero-mean space).

Readings:
  * mu1 = mu2 = one application of the degree-2 smoother; pre-smoothing starts from zero;
  * Chebyshev follows the three-term recurrence of Saad, Iterative Methods (2nd ed.),
    Alg. 12.1, for D^{-1} A on [a, b] = [lo * lambda, hi * lambda];
  * Jacobi variant: omega = 4 / (3 lambda), `degree` sweeps;
  * coarse solve for the singular operator: K^{-1} (f - bbar bbar^T f), projected onto
    bbar-perp, with K = A_M + abar bbar bbar^T (equals A_M^+ f for f perpendicular to bbar);
  * PCG (Saad Alg. 9.1) with Pi = I - 1 1^T / n applied to the right-hand side, initial
    guess and preconditioned residual for the elliptic system; stop on the recursive residual
    ||r|| <= rtol ||Pi f||; the returned elliptic solution is normalised to m^T x = 0
    (integral zero);
  * diagonal preconditioning (point Jacobi, z = D^{-1} r) or none stand in for the paper's
    parabolic solvers (block Jacobi on CPUs, unpreconditioned on GPUs, Sec. 5);
  * flexible CG (Notay 2000) with beta = z_{k+1}^T (r_{k+1} - r_k) / (z_k^T r_k);
  * mixed form: the V-cycle runs in float32 on a float32 copy of the hierarchy, the coarse
    solve stays float64; its inner products z.r are taken exactly (correctly rounded) here,
    which is the value a compensated float32 dot approximates within its error bound.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .amg import Hierarchy


# ---------------------------------------------------------------------------------------------
def chebyshev(A, Dinv, f, x, lam, degree, lo, hi):
    """Degree-`degree` Chebyshev iteration for D^{-1} A on [lo*lam, hi*lam] (x=None: zero guess)."""
    a, b = lo * lam, hi * lam
    theta = 0.5 * (b + a)
    delta = 0.5 * (b - a)
    sigma = theta / delta
    rho = 1.0 / sigma
    if x is None:
        x = np.zeros_like(f)
        r = f.copy()
    else:
        r = f - A @ x
    d = (Dinv * r) / theta
    for j in range(degree):
        x = x + d
        if j + 1 < degree:
            r = r - A @ d
            rho_new = 1.0 / (2.0 * sigma - rho)
            d = (rho_new * rho) * d + (2.0 * rho_new / delta) * (Dinv * r)
            rho = rho_new
    return x


def jacobi(A, Dinv, f, x, lam, degree):
    omega = 4.0 / (3.0 * lam)
    if x is None:
        x = np.zeros_like(f)
    for _ in range(degree):
        x = x + omega * Dinv * (f - A @ x)
    return x


def smooth(h: Hierarchy, k: int, f, x, lv=None):
    lv = lv or h.levels[k]
    o = h.opts
    if o.smoother == "chebyshev":
        return chebyshev(lv.A, lv.Dinv, f, x, lv.lam, o.degree, o.cheb_lo, o.cheb_hi)
    return jacobi(lv.A, lv.Dinv, f, x, lv.lam, o.degree)


def coarse_solve(h: Hierarchy, f):
    f64 = np.asarray(f, dtype=np.float64)
    if isinstance(h.coarse_factor, str):      # one-row coarsest level of the singular operator
        return np.zeros_like(f64)
    if h.coarse_bbar is not None:
        bb = h.coarse_bbar
        e = sla.cho_solve(h.coarse_factor, f64 - bb * (bb @ f64))
        return e - bb * (bb @ e)
    return sla.cho_solve(h.coarse_factor, f64)


def vcycle(h: Hierarchy, f, k: int = 0, levels=None):
    """Alg. 2 with mu1 = mu2 = 1 and zero initial guess."""
    levels = levels or h.levels
    if k == len(levels) - 1:
        if h.coarse_factor is None:          # oversized coarsest level: smoother relaxation
            return smooth(h, k, f, None, levels[k])
        return coarse_solve(h, f).astype(f.dtype)
    lv = levels[k]
    x = smooth(h, k, f, None, lv)
    r = f - lv.A @ x
    e = vcycle(h, lv.R @ r, k + 1, levels)
    x = x + lv.P @ e
    x = smooth(h, k, f, x, lv)
    return x


def float32_levels(h: Hierarchy):
    """A float32 copy of every level's matrices for the mixed-precision V-cycle."""
    from copy import copy
    out = []
    for lv in h.levels:
        c = copy(lv)
        c.A = lv.A.astype(np.float32)
        c.Dinv = lv.Dinv.astype(np.float32)
        c.P = None if lv.P is None else lv.P.astype(np.float32)
        c.R = None if lv.R is None else lv.R.astype(np.float32)
        out.append(c)
    return out


# ---------------------------------------------------------------------------------------------
def exact_dot(x, y) -> float:
    """Correctly rounded x . y for float32 operands: every product is exact in float64 and
    math.fsum returns the correctly rounded sum."""
    return math.fsum((np.asarray(x, np.float64) * np.asarray(y, np.float64)).tolist())


@dataclass
class SolveResult:
    x: np.ndarray
    iterations: int
    converged: bool
    rel_residual_true: float
    rel_residual_rec: float
    status: str = "ok"


def _project(v, on):
    return v - v.mean() if on else v


def _finish(A, fh, nf, x, r, it, converged, status, nullspace, m):
    rec = float(np.linalg.norm(r)) / nf
    true = float(np.linalg.norm(fh - A @ x)) / nf
    if nullspace and m is not None:
        x = x - (m @ x) / m.sum()          # integral-zero normalisation (Sec. 2.1)
    if status == "ok" and not converged:
        status = "not_converged"
    return SolveResult(x, it, converged, true, rec, status)


def pcg(A, f, precond, x0=None, rtol=1e-8, maxit=500, nullspace=False, m=None):
    """Preconditioned CG (Saad Alg. 9.1) on A x = f.

    nullspace: A has the constant kernel; f, x0 and every preconditioned residual are
    projected with Pi = I - 1 1^T / n.  m: lumped mass for the final m^T x = 0 normalisation.
    The iteration count is the number of products A p.
    """
    fh = _project(np.asarray(f, np.float64), nullspace)
    nf = float(np.linalg.norm(fh))
    n = fh.size
    if nf == 0.0:
        return SolveResult(np.zeros(n), 0, True, 0.0, 0.0)
    x = np.zeros(n) if x0 is None else _project(np.array(x0, np.float64), nullspace)
    r = fh - A @ x
    it, status = 0, "ok"
    converged = bool(np.linalg.norm(r) <= rtol * nf)
    if not converged:
        z = _project(np.asarray(precond(r), np.float64), nullspace)
        p = z.copy()
        rho = float(r @ z)
        while it < maxit:
            q = A @ p
            pq = float(p @ q)
            if not (pq > 0.0 and rho > 0.0):
                status = "breakdown"
                break
            alpha = rho / pq
            x = x + alpha * p
            r = r - alpha * q
            it += 1
            if np.linalg.norm(r) <= rtol * nf:
                converged = True
                break
            z = _project(np.asarray(precond(r), np.float64), nullspace)
            rho_new = float(r @ z)
            p = z + (rho_new / rho) * p
            rho = rho_new
    return _finish(A, fh, nf, x, r, it, converged, status, nullspace, m)


def fcg(A, f, precond_lo, x0=None, rtol=1e-8, maxit=500, nullspace=False, m=None,
        lowp=np.float32, dot=None):
    """Flexible CG, FCG(1) (Notay 2000), around a preconditioner working in precision `lowp`.

    precond_lo maps r_lo = fl_lowp(r) to z_lo (dtype lowp).  The search direction uses the
    float64 projected z = Pi fl64(z_lo).  The preconditioned-residual inner products are
    taken on the low-precision operands:  rho_k = z_lo_k . r_lo_k  and
    beta_k = (z_lo_{k+1} . r_lo_{k+1} - z_lo_{k+1} . r_lo_k) / rho_k.
    `dot` defaults to the correctly rounded dot for float32 operands (the value a compensated
    float32 dot approximates within its error bound) and to the float64 dot otherwise.
    Without the projection these equal the projected-z values up to the rounding of 1^T r.
    """
    if dot is None:
        dot = exact_dot if lowp == np.float32 else (lambda a, b: float(np.dot(a, b)))
    fh = _project(np.asarray(f, np.float64), nullspace)
    nf = float(np.linalg.norm(fh))
    n = fh.size
    if nf == 0.0:
        return SolveResult(np.zeros(n), 0, True, 0.0, 0.0)
    x = np.zeros(n) if x0 is None else _project(np.array(x0, np.float64), nullspace)
    r = fh - A @ x
    it, status = 0, "ok"
    converged = bool(np.linalg.norm(r) <= rtol * nf)
    if not converged:
        r_lo = r.astype(lowp)
        z_lo = precond_lo(r_lo)
        p = _project(z_lo.astype(np.float64), nullspace)
        rho = dot(z_lo, r_lo)
        while it < maxit:
            q = A @ p
            pq = float(p @ q)
            if not (pq > 0.0 and rho > 0.0):
                status = "breakdown"
                break
            alpha = rho / pq
            x = x + alpha * p
            r = r - alpha * q
            it += 1
            if np.linalg.norm(r) <= rtol * nf:
                converged = True
                break
            r_lo_old = r_lo
            r_lo = r.astype(lowp)
            z_lo = precond_lo(r_lo)
            rho_new = dot(z_lo, r_lo)
            beta = (rho_new - dot(z_lo, r_lo_old)) / rho
            p = _project(z_lo.astype(np.float64), nullspace) + beta * p
            rho = rho_new
    return _finish(A, fh, nf, x, r, it, converged, status, nullspace, m)


def amg_pcg(A, f, h: Hierarchy, x0=None, rtol=1e-8, maxit=500, m=None):
    return pcg(A, f, lambda r: vcycle(h, r), x0, rtol, maxit, h.opts.nullspace, m)


def amg_fcg_mixed(A, f, h: Hierarchy, x0=None, rtol=1e-8, maxit=500, m=None):
    """FCG(1) in float64 around a float32 V-cycle with a float64 coarse solve."""
    lv32 = float32_levels(h)
    return fcg(A, f, lambda r32: vcycle(h, r32, 0, lv32), x0, rtol, maxit, h.opts.nullspace, m)


def diag_pcg(A, f, kind, x0=None, rtol=1e-8, maxit=5000, nullspace=False, m=None):
    """CG with a diagonal preconditioner or none.  The paper solves the parabolic system with
    unpreconditioned CG on GPUs and with block-Jacobi-preconditioned CG on CPUs (Sec. 5).
    kind "jacobi": z = D^{-1} r with D = diag(A) (point Jacobi); kind "none": z = r."""
    if kind == "jacobi":
        dinv = 1.0 / A.diagonal()
        precond = lambda r: dinv * r
    elif kind == "none":
        precond = lambda r: r
    else:
        raise ValueError(kind)
    return pcg(A, f, precond, x0, rtol, maxit, nullspace, m)

