"""Membrane model and the decoupled IMEX Bidomain step (oracle; test infrastructure only).

Paper: eq. (1) (parabolic-elliptic Bidomain system), eqs. (4)-(7) (IMEX step: gating update,
elliptic solve with A_i + A_e, parabolic solve with c_m/dt M + A_i), Sec. 2.2 (PCG for both).

Readings:
  * membrane model: the two-variable Aliev-Panfilov model (Aliev & Panfilov, Chaos Solitons
    Fractals 7 (1996) 293-301) stands in for TP06, with its published parameters k = 8,
    a = 0.15, eps0 = 0.002, mu1 = 0.2, mu2 = 0.3 and time unit 12.9 ms; the potential maps as
    u = (v + 85) / 105, so rest is u = 0 and a +20 mV plateau is u = 1;
  * gating update semi-implicit as in eq. (4) with the sign read as w^{n+1} - dt R = w^n:
    w^{n+1} = (w^n + dt' eps^n (-k u (u - a - 1))) / (1 + dt' eps^n),
    eps^n = eps0 + mu1 w^n / (u^n + mu2), dt' = dt / 12.9;
  * I_ion = -c_m (105 / 12.9) [k u (u - a)(1 - u) - u w^{n+1}] (mA/cm^3), entering the
    parabolic right-hand side as -M I_ion (eq. (1) has I_ion on the left-hand side);
  * the parabolic hierarchy defaults to strength threshold 0 (the paper sets no AMG options for
    that system; its mass term weakens the couplings below 0.06 on coarse meshes);
  * order within a step: membrane, parabolic (with u_e^n), elliptic (with v^{n+1}); this is
    the recurrence of eqs. (4)-(7) shifted by half a step, and u_e^0 comes from an elliptic
    solve with v^0.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import amg, ellipsoid, fem, krylov

AP_K = 8.0
AP_A = 0.15
AP_EPS0 = 0.002
AP_MU1 = 0.2
AP_MU2 = 0.3
AP_TUNIT_MS = 12.9
AP_VSCALE_MV = 105.0
AP_VREST_MV = -85.0


AP_PUBLISHED = (AP_K, AP_A, AP_EPS0, AP_MU1, AP_MU2, AP_TUNIT_MS, AP_VSCALE_MV, AP_VREST_MV)


def case_ap_params(case):
    """The case's membrane parameters (k, a, eps0, mu1, mu2, time unit, potential scale, rest)."""
    names = ("ap_k", "ap_a", "ap_eps0", "ap_mu1", "ap_mu2", "ap_t_unit", "ap_v_scale", "ap_v_rest")
    return tuple(getattr(case, nm, dflt) for nm, dflt in zip(names, AP_PUBLISHED))


def aliev_panfilov(v, w, dt, cm, params=AP_PUBLISHED):
    """One membrane step: returns (w^{n+1}, I_ion)."""
    k, a, eps0, mu1, mu2, t_unit, v_scale, v_rest = params
    u = (v - v_rest) / v_scale
    dtp = dt / t_unit
    eps = eps0 + mu1 * w / (u + mu2)
    w_new = (w + dtp * eps * (-k * u * (u - a - 1.0))) / (1.0 + dtp * eps)
    iion = -cm * (v_scale / t_unit) * (k * u * (u - a) * (1.0 - u) - u * w_new)
    return w_new, iion


@dataclass
class Sim:
    case: object
    ops: dict
    h_ell: amg.Hierarchy
    h_par: amg.Hierarchy
    v: np.ndarray
    ue: np.ndarray
    w: np.ndarray
    rtol: float
    mixed: bool = False
    it_par: int = 0
    it_ell: int = 0


def _solve(A, f, h, x0, rtol, m, mixed):
    if mixed:
        return krylov.amg_fcg_mixed(A, f, h, x0=x0, rtol=rtol, m=m)
    return krylov.amg_pcg(A, f, h, x0=x0, rtol=rtol, m=m)


def assemble(case):
    """The case's operators: the truncated ellipsoid (a case with n_theta) or the slab."""
    return ellipsoid.assemble_operators(case) if hasattr(case, "n_theta") else fem.assemble_operators(case)


def create(case, v0, w0=None, rtol=1e-8, ell_opts=None, par_opts=None, mixed=False, ops=None):
    """ops: the case's operators when already assembled (assemble(case))."""
    ops = ops if ops is not None else assemble(case)
    ell_opts = ell_opts or amg.AMGOptions(nullspace=True)
    par_opts = par_opts or amg.AMGOptions(nullspace=False, threshold=0.0)
    h_ell = amg.setup(ops["Aell"], ell_opts)
    h_par = amg.setup(ops["Apar"], par_opts)
    v = np.array(v0, np.float64)
    w = np.zeros_like(v) if w0 is None else np.array(w0, np.float64)
    res = _solve(ops["Aell"], -(ops["Ai"] @ v), h_ell, None, rtol, ops["m"], mixed)
    return Sim(case, ops, h_ell, h_par, v, res.x, w, rtol, mixed)


def step(sim: Sim, iapp=None):
    """Eqs. (4)-(7): membrane update, parabolic solve, elliptic solve."""
    c, o = sim.case, sim.ops
    m = o["m"]
    w_new, iion = aliev_panfilov(sim.v, sim.w, c.dt, c.cm, case_ap_params(c))
    rhs = (c.cm / c.dt) * (m * sim.v) - o["Ai"] @ sim.ue - m * iion
    if iapp is not None:
        rhs = rhs + m * iapp
    rp = _solve(o["Apar"], rhs, sim.h_par, sim.v, sim.rtol, None, sim.mixed)
    re = _solve(o["Aell"], -(o["Ai"] @ rp.x), sim.h_ell, sim.ue, sim.rtol, m, sim.mixed)
    sim.w, sim.v, sim.ue = w_new, rp.x, re.x
    sim.it_par, sim.it_ell = rp.iterations, re.iterations
    return rp, re
