"""Pins for the oracle's membrane model and IMEX step (CPU only): fixed points and the
excitation threshold of the cubic Aliev-Panfilov current, reduction of the PDE step to the
single-cell ODE for spatially uniform states, and charge conservation without currents."""
import numpy as np
import pytest

import bidomain_cases as bc
from oracle import bidomain, fem


def test_membrane_fixed_points():
    # rest (u = 0, w = 0) is an equilibrium: no current, gating unchanged
    w, iion = bidomain.aliev_panfilov(np.array([-85.0]), np.array([0.0]), 0.05, 1.0)
    assert w[0] == 0.0 and iion[0] == 0.0
    # u = a and u = 1 are the other roots of the cubic k u (u - a)(1 - u): zero current at w = 0
    # (dt = 0 keeps the gate at w = 0 so that only the cubic remains)
    for u in (bidomain.AP_A, 1.0):
        v = bidomain.AP_VREST_MV + bidomain.AP_VSCALE_MV * u
        _, iion = bidomain.aliev_panfilov(np.array([v]), np.array([0.0]), 0.0, 1.0)
        assert abs(iion[0]) < 1e-12


def _single_cell(v0, steps, dt=0.05, cm=1.0):
    v, w = np.array([v0]), np.array([0.0])
    out = []
    for _ in range(steps):
        w, iion = bidomain.aliev_panfilov(v, w, dt, cm)
        v = v - dt / cm * iion
        out.append(v[0])
    return np.array(out)


def test_excitation_threshold():
    a = bidomain.AP_A
    v_above = bidomain.AP_VREST_MV + bidomain.AP_VSCALE_MV * (a + 0.05)
    v_below = bidomain.AP_VREST_MV + bidomain.AP_VSCALE_MV * (a - 0.05)
    up = _single_cell(v_above, 2000)        # 100 ms
    down = _single_cell(v_below, 2000)
    assert up.max() > bidomain.AP_VREST_MV + 0.9 * bidomain.AP_VSCALE_MV   # fires to the plateau
    assert down[-1] < bidomain.AP_VREST_MV + 0.01 * bidomain.AP_VSCALE_MV   # decays to rest


def test_plateau_repolarises():
    v = _single_cell(20.0, 20000)  # 1 s of a cell starting on the plateau
    assert v[0] > 0.0 and v[-1] < -80.0


def test_uniform_state_reduces_to_single_cell():
    c = bc.make_case(6, 6, 3, seed=1)
    v0 = np.full(c.n, -40.0)
    sim = bidomain.create(c, v0, rtol=1e-12)
    assert np.abs(sim.ue).max() <= 1e-9  # the elliptic right-hand side -A_i v vanishes up to rounding
    ref = _single_cell(-40.0, 5)
    for s in range(5):
        bidomain.step(sim)
        assert np.abs(sim.v - ref[s]).max() <= 1e-9 * abs(ref[s])
        assert np.abs(sim.ue).max() <= 1e-9


def test_conservation_without_currents(monkeypatch):
    c = bc.make_case(8, 8, 4, seed=2)
    v0 = bc.nodal_v0(c)
    sim = bidomain.create(c, v0, rtol=1e-12)
    monkeypatch.setattr(bidomain, "aliev_panfilov", lambda v, w, dt, cm, *p: (w, np.zeros_like(v)))
    m = sim.ops["m"]
    q0 = m @ sim.v
    for _ in range(5):
        bidomain.step(sim)
    assert abs(m @ sim.v - q0) <= 1e-9 * abs(q0)
    # u_e stays in the integral-zero space
    assert abs(m @ sim.ue) <= 1e-12 * np.abs(sim.ue).max() * m.sum()
