"""Serving (continuous batching): every served case gives the same result alone and in a mix of
cases of different sizes; served results equal the standalone simulation's and match the
oracle; a tight device budget queues cases instead of failing; a case larger than the whole
budget is refused."""
import time

import numpy as np
import pytest

import bidomain_cases as bc
from oracle import bidomain

pytestmark = pytest.mark.gpu

lib = pytest.importorskip("paper_2311_13914_amd")


def _mix():
    return [bc.make_case(12, 12, 6, seed=11), bc.make_case(24, 24, 12, seed=14),
            bc.make_case(16, 16, 8, seed=12), bc.make_case(20, 16, 10, seed=13)]


_LAST_STATS = {}   # bidomain_serve_stats of the last _serve call, read after all cases finished


def _serve(cases, nsteps, budget=1 << 34, slots=8, prec=None, timeout=150, budget_fn=None, reorder=1):
    prec = lib.BD_F32 if prec is None else prec
    oe = lib.bidomain_default_opts(vcycle_precision=prec, reorder=reorder)
    op = lib.bidomain_default_opts(vcycle_precision=prec, threshold=0.0, reorder=reorder)  # the parabolic default
    if budget_fn is not None:  # size the budget from the server's own admission estimate
        probe = lib.bidomain_serve_create(1 << 40, 1, oe, op, 1e-8)
        try:
            budget = budget_fn(lambda c: lib.bidomain_serve_estimate(probe, c))
        finally:
            lib.bidomain_serve_destroy(probe)
    srv = lib.bidomain_serve_create(budget, slots, oe, op, 1e-8)
    try:
        tickets = [lib.bidomain_serve_submit(srv, c, bc.nodal_v0(c), nsteps) for c in cases]
        done, peak_running, peak_bytes = {}, 0, 0
        t_end = time.time() + timeout
        while len(done) < len(cases):
            for r in lib.bidomain_serve_poll(srv):
                done[r["ticket"]] = r
            st = lib.bidomain_serve_stats(srv)
            peak_running = max(peak_running, st["running"] + st["setting_up"])
            peak_bytes = max(peak_bytes, st["bytes_in_use"])
            assert time.time() < t_end, "serving did not finish"
        states = {t: lib.bidomain_serve_fetch(srv, t, c.n) for t, c in zip(tickets, cases)
                  if done[t]["status"] == lib.BD_OK}
        lat = lib.bidomain_serve_solve_latencies(srv)
        _LAST_STATS.clear()
        _LAST_STATS.update(lib.bidomain_serve_stats(srv))
        return tickets, done, states, peak_running, peak_bytes, lat
    finally:
        lib.bidomain_serve_destroy(srv)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_each_result_is_the_same_alone_and_in_the_mix(torch, prec):
    p = lib.BD_F32 if prec == "f32" else lib.BD_F64
    cases = _mix()
    print(f"[gpu] serve mix of {len(cases)} cases, {prec}", flush=True)
    tk, done, states, peak, _, lat = _serve(cases, 3, prec=p)
    assert peak >= 2, "the mix never ran cases together"
    assert _LAST_STATS["max_batched"] >= 2, "no round's launches advanced two solves together"
    for t in tk:
        assert done[t]["status"] == lib.BD_OK and done[t]["steps"] == 3
        assert done[t]["max_rel_residual"] <= 1e-8
    assert len(lat) == len(cases) * (1 + 2 * 3)
    for c, t in zip(cases, tk):
        tk1, done1, states1, _, _, _ = _serve([c], 3, prec=p)
        v_mix, ue_mix = states[t]
        v_one, ue_one = states1[tk1[0]]
        assert np.array_equal(v_mix, v_one) and np.array_equal(ue_mix, ue_one)
        assert (done1[tk1[0]]["it_par"], done1[tk1[0]]["it_ell"]) == (done[t]["it_par"], done[t]["it_ell"])


def test_renumbered_levels_alone_and_in_the_mix(torch):
    """With every eligible coarse level renumbered on the device (reorder = 2: these cases' levels
    are below the default's 2^26 entries), served results are the same alone and in the mix,
    and the first case matches the oracle."""
    cases = [bc.make_case(40, 40, 20, seed=21), bc.make_case(36, 30, 16, seed=22)]
    oe = lib.bidomain_default_opts(reorder=2)
    op = lib.bidomain_default_opts(threshold=0.0, reorder=2)
    v0 = torch.tensor(bc.nodal_v0(cases[0]), dtype=torch.float64, device="cuda")
    sim = lib.bidomain_sim_create(cases[0], v0, ell_opts=oe, par_opts=op)
    try:
        ren = lib.bidomain_amg_info(lib.bidomain_sim_hierarchy(sim, 0))["renumbered"]
    finally:
        lib.bidomain_sim_destroy(sim)
    print(f"[gpu] serve with renumbered levels {ren}", flush=True)
    assert any(ren)
    tk, done, states, _, _, _ = _serve(cases, 2, prec=lib.BD_F64, reorder=2)
    for c, t in zip(cases, tk):
        assert done[t]["status"] == lib.BD_OK and done[t]["max_rel_residual"] <= 1e-8
        tk1, done1, states1, _, _, _ = _serve([c], 2, prec=lib.BD_F64, reorder=2)
        assert np.array_equal(states[t][0], states1[tk1[0]][0]) and np.array_equal(states[t][1], states1[tk1[0]][1])
    ref = bidomain.create(cases[0], bc.nodal_v0(cases[0]), rtol=1e-12)
    for _ in range(2):
        bidomain.step(ref)
    v, ue = states[tk[0]]
    assert np.linalg.norm(v - ref.v) <= 1e-6 * np.linalg.norm(ref.v)
    assert np.linalg.norm(ue - ref.ue) <= 1e-6 * np.linalg.norm(ref.ue)


def test_served_case_equals_standalone_simulation(torch):
    c = bc.make_case(20, 16, 10, seed=13)
    tk, done, states, _, _, _ = _serve([c, bc.make_case(12, 12, 6, seed=11)], 3, prec=lib.BD_F64)
    v0 = torch.tensor(bc.nodal_v0(c), dtype=torch.float64, device="cuda")
    sim = lib.bidomain_sim_create(c, v0, rtol=1e-8)
    try:
        rc, info = lib.bidomain_step(sim, 3, 1e-8)
        assert rc == lib.BD_OK
        out = torch.empty(c.n, dtype=torch.float64, device="cuda")
        lib.bidomain_sim_get(sim, lib.BD_V, out)
        v = out.cpu().numpy()
        lib.bidomain_sim_get(sim, lib.BD_UE, out)
        ue = out.cpu().numpy()
    finally:
        lib.bidomain_sim_destroy(sim)
    vs, ues = states[tk[0]]
    np.testing.assert_allclose(vs, v, rtol=0, atol=1e-12 * np.abs(v).max())
    np.testing.assert_allclose(ues, ue, rtol=0, atol=1e-12 * np.abs(ue).max())


def test_served_case_matches_oracle(torch):
    c = bc.make_case(16, 16, 8, seed=12)
    tk, done, states, _, _, _ = _serve([c], 3, prec=lib.BD_F64)
    sim = bidomain.create(c, bc.nodal_v0(c), rtol=1e-12)
    for _ in range(3):
        bidomain.step(sim)
    v, ue = states[tk[0]]
    assert np.linalg.norm(v - sim.v) <= 1e-6 * np.linalg.norm(sim.v)
    assert np.linalg.norm(ue - sim.ue) <= 1e-6 * np.linalg.norm(sim.ue)


def test_tight_budget_queues_instead_of_failing(torch):
    big1, big2, small = bc.make_case(24, 24, 12, seed=14), bc.make_case(24, 24, 12, seed=15), bc.make_case(12, 12, 6, seed=11)
    tk, done, _, _, _, _ = _serve([big1], 1)
    actual = done[tk[0]]["device_bytes"]
    print(f"[gpu] 24x24x12 case holds {actual} bytes", flush=True)
    # room for one large case, not two: they must run one after the other
    tk, done, states, peak, peak_bytes, _ = _serve(
        [big1, big2, small], 2, budget_fn=lambda est: int(1.2 * max(est(big1), actual)))
    assert all(done[t]["status"] == lib.BD_OK and done[t]["steps"] == 2 for t in tk)
    a, b = done[tk[0]], done[tk[1]]
    assert a["t_done"] <= b["t_admit"] or b["t_done"] <= a["t_admit"], (a, b)


def test_slots_gate_admission(torch):
    cases = _mix()
    tk, done, _, peak, _, _ = _serve(cases, 1, slots=1)
    assert all(done[t]["status"] == lib.BD_OK for t in tk)
    assert peak == 1


def test_case_larger_than_budget_is_refused(torch):
    srv = lib.bidomain_serve_create(1 << 20, 2)
    try:
        c = bc.make_case(64, 64, 32, seed=1)
        with pytest.raises(lib.BidomainError) as e:
            lib.bidomain_serve_submit(srv, c, bc.nodal_v0(c), 1)
        assert e.value.status == lib.BD_E_BUDGET
    finally:
        lib.bidomain_serve_destroy(srv)


def test_failed_upload_retires_the_case_and_frees_its_budget(torch, monkeypatch):
    """The library's test hook makes the upload of ticket 1 report an allocation failure after
    its device memory was taken: that case must come back with BD_E_NOMEM, its slot and budget
    must be released, and the other case must still be served."""
    monkeypatch.setenv("BIDOMAIN_SERVE_FAIL_UPLOAD", "1")
    cases = [bc.make_case(12, 12, 6, seed=11), bc.make_case(16, 16, 8, seed=12)]
    print("[gpu] serve with an injected upload failure", flush=True)
    tk, done, states, _, _, _ = _serve(cases, 2, slots=1, prec=lib.BD_F64)
    assert tk[0] == 1
    assert done[tk[0]]["status"] == lib.BD_E_NOMEM and done[tk[0]]["steps"] == 0
    assert done[tk[1]]["status"] == lib.BD_OK and done[tk[1]]["steps"] == 2
    assert tk[1] in states and tk[0] not in states
    assert _LAST_STATS["bytes_in_use"] == 0 and _LAST_STATS["running"] == 0
