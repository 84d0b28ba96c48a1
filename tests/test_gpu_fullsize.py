"""Full-size parity: at 128 x 128 x 64 (float64 and float32 V-cycles), sampled rows of every
level-0 product against the oracle's own assembly, the elliptic solution against the oracle's
rtol-1e-12 solution, and properties that hold at any size -- true residuals of both solves
recomputed with the oracle's matrices, the integral-zero normalisation, charge balance of the
parabolic step, and bitwise reproducibility of a step; at 384 x 384 x 96 (the benchmarked size,
in bench.py's launch configuration), sampled rows of the fine product against rows built from the
oracle's element matrices."""
import numpy as np
import pytest

import bidomain_cases as bc
from oracle import bidomain, fem

pytestmark = pytest.mark.gpu

lib = pytest.importorskip("paper_2311_13914_amd")


@pytest.fixture(scope="module")
def c2():
    import torch
    assert torch.cuda.is_available()
    case = bc.config_case("C2")
    print(f"[gpu] C2 n={case.n}: oracle assembly", flush=True)
    ops = fem.assemble_operators(case)
    return case, ops


def _dev(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def test_fine_level_products_sampled(c2):
    import torch
    case, ops = c2
    rng = np.random.default_rng(21)
    rows = np.concatenate([[0, case.n - 1], rng.integers(0, case.n, 4000)])
    for key, nullspace in (("Aell", 1), ("Apar", 0)):
        A = ops[key]
        h = lib.bidomain_amg_setup(A, lib.bidomain_default_opts(nullspace=nullspace, max_levels=1))
        try:
            x = rng.uniform(-1, 1, case.n)
            y = torch.empty(case.n, dtype=torch.float64, device="cuda")
            lib.bidomain_amg_apply(h, lib.BD_OP_A, 0, _dev(x), y)
            ys = y.cpu().numpy()
            ref = A[rows] @ x
            assert np.max(np.abs(ys[rows] - ref)) <= 1e-13 * np.max(np.abs(ref)), key
        finally:
            lib.bidomain_amg_destroy(h)


def test_time_steps_at_full_size(c2):
    import torch
    case, ops = c2
    v0 = bc.nodal_v0(case)
    sim = lib.bidomain_sim_create(case, _dev(v0), rtol=1e-8)
    try:
        out = torch.empty(case.n, dtype=torch.float64, device="cuda")
        lib.bidomain_sim_get(sim, lib.BD_UE, out)
        ue0 = out.cpu().numpy()
        m, Ai, Aell, Apar = ops["m"], ops["Ai"], ops["Aell"], ops["Apar"]
        f0 = -(Ai @ v0)
        f0h = f0 - f0.mean()
        assert np.linalg.norm(f0h - Aell @ ue0) <= 1.0001e-8 * np.linalg.norm(f0h)
        assert abs(m @ ue0) <= 1e-12 * np.abs(ue0).max() * m.sum()
        w0 = np.zeros(case.n)
        rc, info = lib.bidomain_step(sim, 1, 1e-8)
        assert rc == lib.BD_OK, info
        print(f"[gpu] C2 step: it_par {info['it_par']} it_ell {info['it_ell']}", flush=True)
        lib.bidomain_sim_get(sim, lib.BD_V, out); v1 = out.cpu().numpy()
        lib.bidomain_sim_get(sim, lib.BD_UE, out); ue1 = out.cpu().numpy()
        lib.bidomain_sim_get(sim, lib.BD_W, out); w1 = out.cpu().numpy()
        # membrane update against the oracle's pointwise model (same inputs, same formula order)
        w_ref, iion = bidomain.aliev_panfilov(v0, w0, case.dt, case.cm)
        np.testing.assert_allclose(w1, w_ref, rtol=1e-13, atol=1e-300)
        # parabolic system (eq. (7)) solved to the tolerance with the oracle's matrices
        rhs = (case.cm / case.dt) * (m * v0) - Ai @ ue0 - m * iion
        assert np.linalg.norm(rhs - Apar @ v1) <= 1.0001e-8 * np.linalg.norm(rhs)
        # elliptic system (eq. (6)) with the new potential
        f1 = -(Ai @ v1)
        f1h = f1 - f1.mean()
        assert np.linalg.norm(f1h - Aell @ ue1) <= 1.0001e-8 * np.linalg.norm(f1h)
        assert abs(m @ ue1) <= 1e-12 * np.abs(ue1).max() * m.sum()
        # charge balance: 1^T A_par v1 = (c_m/dt) m^T v1 = 1^T rhs
        assert abs((case.cm / case.dt) * (m @ v1) - rhs.sum()) <= 1e-7 * np.abs(rhs).sum()
    finally:
        lib.bidomain_sim_destroy(sim)


def test_step_is_bitwise_reproducible(c2):
    import torch
    case, _ = c2
    v0 = _dev(bc.nodal_v0(case))
    outs = []
    for _ in range(2):
        sim = lib.bidomain_sim_create(case, v0, rtol=1e-8)
        try:
            rc, info = lib.bidomain_step(sim, 2, 1e-8)
            assert rc == lib.BD_OK
            o = torch.empty(case.n, dtype=torch.float64, device="cuda")
            lib.bidomain_sim_get(sim, lib.BD_UE, o)
            outs.append((o.cpu().numpy(), info["it_ell"], info["it_par"]))
        finally:
            lib.bidomain_sim_destroy(sim)
    assert outs[0][1:] == outs[1][1:]
    assert np.array_equal(outs[0][0], outs[1][0])


def _oracle_rows(case, rows, x):
    """(A_ell x)_p for the sampled rows p, from the oracle's element matrices alone: row p sums
    K_e[l(p), m] x[node_m(e)] over the (up to 8) elements e containing node p."""
    nxp, nyp = case.nx + 1, case.ny + 1
    K = {}
    out = np.zeros(len(rows))
    for t, p in enumerate(rows):
        i, j, k = p % nxp, (p // nxp) % nyp, p // (nxp * nyp)
        s = 0.0
        for l in range(8):
            a, b, c = fem.local_node_bits(l)
            ex, ey, ez = i - a, j - b, k - c
            if not (0 <= ex < case.nx and 0 <= ey < case.ny and 0 <= ez < case.nz):
                continue
            if ez not in K:
                K[ez] = (fem.element_stiffness(case, ez, case.sig_il, case.sig_it)
                         + fem.element_stiffness(case, ez, case.sig_el, case.sig_et))
            for m2 in range(8):
                a2, b2, c2 = fem.local_node_bits(m2)
                s += K[ez][l, m2] * x[(ex + a2) + nxp * ((ey + b2) + nyp * (ez + c2))]
        out[t] = s
    return out


def test_c5_fine_product_sampled():
    """The fine elliptic product at the largest single-GPU size bench.py runs (384 x 384 x 96
    elements, 14.4 M rows, 384 M nonzeros; the diagonal form, in its launch configuration) on
    sampled rows -- the first and last rows and 12,000 random ones -- against the same rows built
    from the oracle's element stiffness matrices."""
    import torch
    case = bc.config_case("C5")
    print(f"[gpu] C5 n={case.n}: library assembly and diagonal form", flush=True)
    rp, ci, v, _ = lib.bidomain_slab_assemble(case, lib.BD_MAT_AELL)
    h = lib.bidomain_amg_setup((rp, ci, v), lib.bidomain_default_opts(nullspace=1, max_levels=1))
    del rp, ci, v
    try:
        assert lib.bidomain_amg_info(h)["diags"][0] == 14
        rng = np.random.default_rng(5)
        x = rng.uniform(-1, 1, case.n)
        y = torch.empty(case.n, dtype=torch.float64, device="cuda")
        lib.bidomain_amg_apply(h, lib.BD_OP_A, 0, _dev(x), y)
        ys = y.cpu().numpy()
        edge = [0, 1, 2, case.nx, case.nx + 1, case.n - case.nx - 2, case.n - 2, case.n - 1]
        rows = np.concatenate([edge, rng.integers(0, case.n, 12000)])
        ref = _oracle_rows(case, rows, x)
        assert np.max(np.abs(ys[rows] - ref)) <= 1e-12 * np.max(np.abs(ref))
    finally:
        lib.bidomain_amg_destroy(h)


@pytest.mark.parametrize("reorder", [1, 2])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_c2_elliptic_solution_matches_oracle(c2, precision, reorder):
    """The 128 x 128 x 64 elliptic solve (f = -A_i v0, zero guess) against the oracle's solution
    at rtol 1e-12 on the oracle's own hierarchy: relative error <= 1e-6, true relative residual
    <= 1e-8, iteration count within 1 (float64) or 2 (float32 V-cycles) of the oracle's; with
    the default options and with levels 1 and 2 renumbered on the device (reorder = 2)."""
    import torch
    from oracle import amg, krylov
    case, ops = c2
    A, m = ops["Aell"], ops["m"]
    f = -(ops["Ai"] @ bc.nodal_v0(case))
    if "ref" not in _C2_REF:
        print("[gpu] C2 oracle setup and rtol-1e-12 solve", flush=True)
        h_or = amg.setup(A, amg.AMGOptions(nullspace=True))
        _C2_REF["ref"] = krylov.amg_pcg(A, f, h_or, rtol=1e-12, m=m).x
        _C2_REF["f64"] = krylov.amg_pcg(A, f, h_or, rtol=1e-8, m=m).iterations
        _C2_REF["f32"] = krylov.amg_fcg_mixed(A, f, h_or, rtol=1e-8, m=m).iterations
    ref = _C2_REF["ref"]
    prec = lib.BD_F32 if precision == "f32" else lib.BD_F64
    h = lib.bidomain_amg_setup(A, lib.bidomain_default_opts(nullspace=1, vcycle_precision=prec, reorder=reorder), m)
    try:
        ren = lib.bidomain_amg_info(h)["renumbered"]
        assert (sum(ren) >= 2) if reorder == 2 else not any(ren), ren
        x = torch.zeros(case.n, dtype=torch.float64, device="cuda")
        rc, info = lib.bidomain_pcg_solve(h, _dev(f), x, False, 1e-8, 500)
        assert rc == lib.BD_OK, info
        xs = x.cpu().numpy()
        fh = f - f.mean()
        assert np.linalg.norm(fh - A @ xs) <= 1e-8 * np.linalg.norm(fh) * (1 + 1e-6)
        err = np.linalg.norm(xs - ref) / np.linalg.norm(ref)
        print(f"[gpu] C2 {precision} reorder={reorder}: {info['iterations']} iterations (oracle {_C2_REF[precision]}), "
              f"error {err:.2e}", flush=True)
        assert err <= 1e-6
        assert abs(info["iterations"] - _C2_REF[precision]) <= (1 if precision == "f64" else 2)
    finally:
        lib.bidomain_amg_destroy(h)


_C2_REF = {}
