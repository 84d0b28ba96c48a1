"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the same seeded inputs.

Bars (float64 path): every V-cycle operation on every level within 1e-12 (relative, max norm)
of the oracle's operation on the oracle's own hierarchy; solves at rtol 1e-8 with true relative
residual <= 1e-8 (recomputed here with the oracle's matrix) and relative error <= 1e-6 against
the oracle's rtol-1e-12 solution; iteration counts equal to the oracle's within one.
Mixed form: the same residual bar and error <= 1e-6; iterations within two of the oracle's
float32 V-cycle.
"""
import numpy as np
import pytest

import bidomain_cases as bc
from oracle import amg, bidomain, fem, krylov

pytestmark = pytest.mark.gpu

lib = pytest.importorskip("paper_2311_13914_amd")


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def dev(torch, a, dtype=None):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype or torch.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


CASES = {
    "C1": lambda: bc.config_case("C1"),
    "ragged": lambda: bc.make_case(37, 29, 13, seed=7),   # several tiles and a ragged tail
}


def _problem(name):
    c = CASES[name]()
    ops = fem.assemble_operators(c)
    f = -(ops["Ai"] @ bc.nodal_v0(c))
    return c, ops, f


def _relerr(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


# the fine operator in the symmetric diagonal form (the default for a 27-point operator) or in
# the CSR-stream offset-dictionary form
FORMS = {"diag": (1, 14, 0), "csr": (0, 0, 1)}  # diag_form option, stored diagonals, index bytes


@pytest.mark.parametrize("form", list(FORMS))
@pytest.mark.parametrize("name", list(CASES))
def test_vcycle_operations_match_oracle(torch, name, form):
    c, ops, f = _problem(name)
    A = ops["Aell"]
    h_or = amg.setup(A, amg.AMGOptions(nullspace=True))
    print(f"[gpu] case={name} form={form} n={c.n} levels={h_or.nlevels}", flush=True)
    h = lib.bidomain_amg_setup(A, lib.bidomain_default_opts(nullspace=1, diag_form=FORMS[form][0]), ops["m"])
    try:
        info = lib.bidomain_amg_info(h)
        assert info["n"] == [lv.A.shape[0] for lv in h_or.levels]
        assert (info["diags"][0], info["col_bytes"][0]) == FORMS[form][1:]
        rng = np.random.default_rng(11)
        for k, lv in enumerate(h_or.levels):
            n = lv.A.shape[0]
            x = rng.uniform(-1, 1, n)
            out = torch.empty(n, dtype=torch.float64, device="cuda")
            lib.bidomain_amg_apply(h, lib.BD_OP_A, k, dev(torch, x), out)
            assert _relerr(host(out), lv.A @ x) <= 1e-12, f"A_{k}"
            if lv.P is not None:
                nc = lv.P.shape[1]
                e = rng.uniform(-1, 1, nc)
                out = torch.empty(n, dtype=torch.float64, device="cuda")
                lib.bidomain_amg_apply(h, lib.BD_OP_P, k, dev(torch, e), out)
                assert _relerr(host(out), lv.P @ e) <= 1e-12, f"P_{k}"
                outc = torch.empty(nc, dtype=torch.float64, device="cuda")
                lib.bidomain_amg_apply(h, lib.BD_OP_R, k, dev(torch, x), outc)
                assert _relerr(host(outc), lv.R @ x) <= 1e-12, f"R_{k}"
                out = torch.empty(n, dtype=torch.float64, device="cuda")
                lib.bidomain_amg_apply(h, lib.BD_OP_PRESMOOTH, k, dev(torch, x), out)
                assert _relerr(host(out), krylov.smooth(h_or, k, x, None)) <= 1e-12, f"S_{k}"
                fk = x - x.mean()
                out = torch.empty(n, dtype=torch.float64, device="cuda")
                lib.bidomain_amg_apply(h, lib.BD_OP_VCYCLE, k, dev(torch, fk), out)
                assert _relerr(host(out), krylov.vcycle(h_or, fk, k)) <= 1e-10, f"V_{k}"
        M = h_or.levels[-1]
        fM = rng.uniform(-1, 1, M.A.shape[0])
        fM -= fM.mean()
        out = torch.empty(M.A.shape[0], dtype=torch.float64, device="cuda")
        lib.bidomain_amg_apply(h, lib.BD_OP_COARSE, 0, dev(torch, fM), out)
        assert _relerr(host(out), krylov.coarse_solve(h_or, fM)) <= 1e-10
    finally:
        lib.bidomain_amg_destroy(h)


def test_renumbered_levels_match_oracle(torch):
    """Intermediate levels renumbered on the device (reverse Cuthill-McKee; option reorder = 2
    takes this small hierarchy's level 1, the default only levels of 2^26 entries or more): each
    V-cycle operation on every level, through the host numbering of bidomain_amg_apply, within
    1e-12 of the oracle's; solves with and without renumbering take the same iterations (within
    one) and agree to rounding, in float64 and with float32 V-cycles."""
    c = bc.make_case(64, 48, 24, seed=9)  # level 1: 3,817 rows, 1.6 % dense
    ops = fem.assemble_operators(c)
    A, m = ops["Aell"], ops["m"]
    f = -(ops["Ai"] @ bc.nodal_v0(c))
    h_or = amg.setup(A, amg.AMGOptions(nullspace=True))
    h = lib.bidomain_amg_setup(A, lib.bidomain_default_opts(nullspace=1, reorder=2), m)
    h0 = lib.bidomain_amg_setup(A, lib.bidomain_default_opts(nullspace=1), m)
    try:
        info, info0 = lib.bidomain_amg_info(h), lib.bidomain_amg_info(h0)
        print(f"[gpu] renumbered levels n={info['n']} renumbered={info['renumbered']}", flush=True)
        assert info["n"] == info0["n"] == [lv.A.shape[0] for lv in h_or.levels]
        assert info["renumbered"][0] == 0 and info["renumbered"][-1] == 0 and sum(info["renumbered"]) >= 1
        assert not any(info0["renumbered"])
        rng = np.random.default_rng(23)
        for k, lv in enumerate(h_or.levels[:-1]):
            n, nc = lv.A.shape[0], lv.P.shape[1]
            x, e = rng.uniform(-1, 1, n), rng.uniform(-1, 1, nc)
            out, outc = (torch.empty(k_, dtype=torch.float64, device="cuda") for k_ in (n, nc))
            lib.bidomain_amg_apply(h, lib.BD_OP_A, k, dev(torch, x), out)
            assert _relerr(host(out), lv.A @ x) <= 1e-12, f"A_{k}"
            lib.bidomain_amg_apply(h, lib.BD_OP_P, k, dev(torch, e), out)
            assert _relerr(host(out), lv.P @ e) <= 1e-12, f"P_{k}"
            lib.bidomain_amg_apply(h, lib.BD_OP_R, k, dev(torch, x), outc)
            assert _relerr(host(outc), lv.R @ x) <= 1e-12, f"R_{k}"
            lib.bidomain_amg_apply(h, lib.BD_OP_PRESMOOTH, k, dev(torch, x), out)
            assert _relerr(host(out), krylov.smooth(h_or, k, x, None)) <= 1e-12, f"S_{k}"
            fk = x - x.mean()
            lib.bidomain_amg_apply(h, lib.BD_OP_VCYCLE, k, dev(torch, fk), out)
            assert _relerr(host(out), krylov.vcycle(h_or, fk, k)) <= 1e-10, f"V_{k}"
    finally:
        lib.bidomain_amg_destroy(h)
        lib.bidomain_amg_destroy(h0)
    for prec in (lib.BD_F64, lib.BD_F32):
        xs = []
        for reorder in (2, 0):
            g = lib.bidomain_amg_setup(A, lib.bidomain_default_opts(nullspace=1, vcycle_precision=prec,
                                                                    reorder=reorder), m)
            try:
                x = torch.zeros(c.n, dtype=torch.float64, device="cuda")
                rc, inf = lib.bidomain_pcg_solve(g, dev(torch, f), x, False, 1e-8, 200)
                assert rc == lib.BD_OK and inf["rel_residual_true"] <= 1e-8, inf
                xs.append((inf["iterations"], host(x)))
            finally:
                lib.bidomain_amg_destroy(g)
        assert abs(xs[0][0] - xs[1][0]) <= 1
        assert np.linalg.norm(xs[0][1] - xs[1][1]) <= 1e-7 * np.linalg.norm(xs[1][1])


def _check_solution(A, f, x, m, x_ref, rtol=1e-8, err=1e-6, nullspace=True):
    fh = f - f.mean() if nullspace else f
    assert np.linalg.norm(fh - A @ x) <= rtol * np.linalg.norm(fh) * (1 + 1e-6)
    if nullspace:
        assert abs(m @ x) <= 1e-12 * np.abs(x).max() * m.sum()
    assert np.linalg.norm(x - x_ref) <= err * np.linalg.norm(x_ref)


@pytest.mark.parametrize("form", list(FORMS))
@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_elliptic_solve_matches_oracle(torch, name, precision, form):
    c, ops, f = _problem(name)
    A, m = ops["Aell"], ops["m"]
    h_or = amg.setup(A, amg.AMGOptions(nullspace=True))
    ref = krylov.amg_pcg(A, f, h_or, rtol=1e-12, m=m)
    or8 = (krylov.amg_pcg if precision == "f64" else krylov.amg_fcg_mixed)(A, f, h_or, rtol=1e-8, m=m)
    print(f"[gpu] case={name} precision={precision} form={form} oracle_its={or8.iterations}", flush=True)
    opts = lib.bidomain_default_opts(nullspace=1, vcycle_precision=lib.BD_F64 if precision == "f64" else lib.BD_F32,
                                     diag_form=FORMS[form][0])
    h = lib.bidomain_amg_setup(A, opts, m)
    try:
        assert lib.bidomain_amg_info(h)["diags"][0] == FORMS[form][1]
        x = torch.zeros(c.n, dtype=torch.float64, device="cuda")
        rc, info = lib.bidomain_pcg_solve(h, dev(torch, f), x, False, 1e-8, 200)
        assert rc == lib.BD_OK, info
        assert info["rel_residual_true"] <= 1e-8
        xs = host(x)
        _check_solution(A, f, xs, m, ref.x)
        assert abs(info["iterations"] - or8.iterations) <= (1 if precision == "f64" else 2)
        # a second solve is bitwise identical (deterministic reductions)
        x2 = torch.zeros(c.n, dtype=torch.float64, device="cuda")
        rc2, info2 = lib.bidomain_pcg_solve(h, dev(torch, f), x2, False, 1e-8, 200)
        assert info2["iterations"] == info["iterations"]
        assert np.array_equal(host(x2), xs)
    finally:
        lib.bidomain_amg_destroy(h)


@pytest.mark.parametrize("dims", [(24, 24, 12), (48, 48, 24)])
def test_parabolic_solve_matches_oracle(torch, dims):
    c = bc.make_case(*dims, seed=5)
    ops = fem.assemble_operators(c)
    A = ops["Apar"]
    f = A @ bc.nodal_v0(c) + 0.1 * ops["m"] * bc.random_vector(c.n, 2)
    h_or = amg.setup(A, amg.AMGOptions(threshold=0.0))
    ref = krylov.amg_pcg(A, f, h_or, rtol=1e-12)
    or8 = krylov.amg_pcg(A, f, h_or, rtol=1e-8)
    print(f"[gpu] parabolic dims={dims} levels={h_or.nlevels} oracle_its={or8.iterations}", flush=True)
    h = lib.bidomain_amg_setup(A, lib.bidomain_default_opts(threshold=0.0))
    try:
        x = torch.zeros(c.n, dtype=torch.float64, device="cuda")
        rc, info = lib.bidomain_pcg_solve(h, dev(torch, f), x, False, 1e-8, 200)
        assert rc == lib.BD_OK and info["rel_residual_true"] <= 1e-8
        _check_solution(A, f, host(x), None, ref.x, nullspace=False)
        assert abs(info["iterations"] - or8.iterations) <= 1
    finally:
        lib.bidomain_amg_destroy(h)


@pytest.mark.parametrize("kind", ["none", "jacobi"])
def test_diag_preconditioned_solves_match_oracle(torch, kind):
    """The paper's GPU parabolic solver (unpreconditioned CG, Sec. 5) and point-Jacobi CG:
    the parabolic system at 24 x 24 x 12, and the singular elliptic system at 16 x 16 x 8 with
    the null-space projection; iteration counts within 1 (parabolic) or 2 % (elliptic, a few
    hundred iterations) of the oracle's, solutions against a tighter oracle solve."""
    pc = {"none": lib.BD_PC_NONE, "jacobi": lib.BD_PC_JACOBI}[kind]
    c = bc.make_case(24, 24, 12, seed=5)
    ops = fem.assemble_operators(c)
    A = ops["Apar"]
    f = A @ np.random.default_rng(12).standard_normal(c.n)
    ref = krylov.diag_pcg(A, f, kind, rtol=1e-12)
    or8 = krylov.diag_pcg(A, f, kind, rtol=1e-8)
    print(f"[gpu] diagonal preconditioner {kind}: parabolic oracle_its={or8.iterations}", flush=True)
    h = lib.bidomain_amg_setup(A, lib.bidomain_default_opts(preconditioner=pc))
    try:
        assert lib.bidomain_amg_info(h)["nlevels"] == 1
        x = torch.zeros(c.n, dtype=torch.float64, device="cuda")
        rc, info = lib.bidomain_pcg_solve(h, dev(torch, f), x, False, 1e-8, 2000)
        assert rc == lib.BD_OK and info["rel_residual_true"] <= 1e-8 * (1 + 1e-6)
        _check_solution(A, f, host(x), None, ref.x, nullspace=False)
        assert abs(info["iterations"] - or8.iterations) <= 1
    finally:
        lib.bidomain_amg_destroy(h)
    c = bc.make_case(16, 16, 8, seed=9)
    ops = fem.assemble_operators(c)
    A, m = ops["Aell"], ops["m"]
    f = -(ops["Ai"] @ bc.nodal_v0(c))
    ref = krylov.diag_pcg(A, f, kind, rtol=1e-12, nullspace=True, m=m)
    or8 = krylov.diag_pcg(A, f, kind, rtol=1e-8, nullspace=True, m=m)
    print(f"[gpu] diagonal preconditioner {kind}: elliptic oracle_its={or8.iterations}", flush=True)
    h = lib.bidomain_amg_setup(A, lib.bidomain_default_opts(nullspace=1, preconditioner=pc), m)
    try:
        x = torch.zeros(c.n, dtype=torch.float64, device="cuda")
        rc, info = lib.bidomain_pcg_solve(h, dev(torch, f), x, False, 1e-8, 5000)
        assert rc == lib.BD_OK
        _check_solution(A, f, host(x), m, ref.x)
        assert abs(info["iterations"] - or8.iterations) <= max(2, 0.02 * or8.iterations)
    finally:
        lib.bidomain_amg_destroy(h)


def test_diag_preconditioner_rejects_float32_and_serving(torch):
    A = fem.assemble_operators(bc.make_case(8, 8, 4, seed=1))["Apar"]
    with pytest.raises(lib.BidomainError):
        lib.bidomain_amg_setup(A, lib.bidomain_default_opts(preconditioner=lib.BD_PC_NONE,
                                                            vcycle_precision=lib.BD_F32))
    with pytest.raises(lib.BidomainError):
        lib.bidomain_serve_create(1 << 30, 1, None, lib.bidomain_default_opts(preconditioner=lib.BD_PC_NONE))


def test_classical_hierarchy_solve(torch):
    c, ops, f = _problem("ragged")
    A, m = ops["Aell"], ops["m"]
    h_or = amg.setup(A, amg.AMGOptions(coarsening="rs", threshold=0.5, nullspace=True))
    ref = krylov.amg_pcg(A, f, h_or, rtol=1e-12, m=m)
    or8 = krylov.amg_pcg(A, f, h_or, rtol=1e-8, m=m)
    h = lib.bidomain_amg_setup(A, lib.bidomain_default_opts(nullspace=1, coarsening=lib.BD_RS, threshold=0.5), m)
    try:
        x = torch.zeros(c.n, dtype=torch.float64, device="cuda")
        rc, info = lib.bidomain_pcg_solve(h, dev(torch, f), x, False, 1e-8, 200)
        assert rc == lib.BD_OK
        _check_solution(A, f, host(x), m, ref.x)
        assert abs(info["iterations"] - or8.iterations) <= 1
    finally:
        lib.bidomain_amg_destroy(h)


def test_edge_cases(torch):
    c, ops, f = _problem("C1")
    A, m = ops["Aell"], ops["m"]
    h = lib.bidomain_amg_setup(A, lib.bidomain_default_opts(nullspace=1), m)
    try:
        x = torch.full((c.n,), 3.0, dtype=torch.float64, device="cuda")
        # zero right-hand side: x = 0, no iteration
        rc, info = lib.bidomain_pcg_solve(h, torch.zeros(c.n, dtype=torch.float64, device="cuda"), x, True)
        assert rc == lib.BD_OK and info["iterations"] == 0 and float(x.abs().max()) == 0.0
        # a constant right-hand side lies in the kernel: projected away, x = 0
        rc, info = lib.bidomain_pcg_solve(h, torch.ones(c.n, dtype=torch.float64, device="cuda"), x, False)
        assert rc == lib.BD_OK and info["iterations"] == 0
        # warm start at the solution: converged before the first iteration
        rc, info = lib.bidomain_pcg_solve(h, dev(torch, f), x, False, 1e-10)
        rc, info2 = lib.bidomain_pcg_solve(h, dev(torch, f), x, True, 1e-8)
        assert rc == lib.BD_OK and info2["iterations"] == 0
        # iteration cap
        x.zero_()
        rc, info = lib.bidomain_pcg_solve(h, dev(torch, f), x, False, 1e-12, 1)
        assert rc == lib.BD_E_NOT_CONVERGED and info["iterations"] == 1
        # non-finite input
        bad = f.copy()
        bad[5] = np.nan
        rc, info = lib.bidomain_pcg_solve(h, dev(torch, bad), x, False)
        assert rc == lib.BD_E_NONFINITE
        # wrong sizes are refused before any launch
        with pytest.raises(ValueError):
            lib.bidomain_pcg_solve(h, torch.zeros(c.n - 1, dtype=torch.float64, device="cuda"), x, False)
        # and the handle still solves correctly afterwards
        x.zero_()
        rc, info = lib.bidomain_pcg_solve(h, dev(torch, f), x, False)
        assert rc == lib.BD_OK and info["rel_residual_true"] <= 1e-8
    finally:
        lib.bidomain_amg_destroy(h)


def test_apply_rejects_vectors_of_the_wrong_precision(torch):
    """bidomain_amg_apply's vectors have the hierarchy's V-cycle precision, reported by
    bidomain_amg_info; the binding refuses the other type before any launch."""
    c, ops, f = _problem("C1")
    A = ops["Aell"]
    for prec, good, bad in ((lib.BD_F32, torch.float32, torch.float64), (lib.BD_F64, torch.float64, torch.float32)):
        h = lib.bidomain_amg_setup(A, lib.bidomain_default_opts(nullspace=1, vcycle_precision=prec), ops["m"])
        try:
            assert lib.bidomain_amg_info(h)["vcycle_precision"] == prec
            with pytest.raises(ValueError):
                lib.bidomain_amg_apply(h, lib.BD_OP_A, 0, torch.zeros(c.n, dtype=bad, device="cuda"),
                                       torch.zeros(c.n, dtype=bad, device="cuda"))
            out = torch.zeros(c.n, dtype=good, device="cuda")
            lib.bidomain_amg_apply(h, lib.BD_OP_A, 0, dev(torch, f, good), out)
            ref = A @ f.astype(np.float32 if prec == lib.BD_F32 else np.float64)
            assert _relerr(host(out).astype(np.float64), ref) <= (1e-4 if prec == lib.BD_F32 else 1e-13)
        finally:
            lib.bidomain_amg_destroy(h)


@pytest.mark.parametrize("dims", [(2, 2, 1), (3, 3, 2), (4, 4, 2)])
def test_tiny_meshes(torch, dims):
    c = bc.make_case(*dims, seed=3)
    ops = fem.assemble_operators(c)
    A, m = ops["Aell"], ops["m"]
    f = -(ops["Ai"] @ bc.nodal_v0(c)) + 1e-3 * bc.random_vector(c.n, 1)
    x_ref = np.linalg.pinv(A.toarray()) @ (f - f.mean())
    x_ref -= (m @ x_ref) / m.sum()
    h = lib.bidomain_amg_setup(A, lib.bidomain_default_opts(nullspace=1, coarse_eq_limit=4), m)
    try:
        x = torch.zeros(c.n, dtype=torch.float64, device="cuda")
        rc, info = lib.bidomain_pcg_solve(h, dev(torch, f), x, False, 1e-12, 100)
        assert rc == lib.BD_OK
        assert np.linalg.norm(host(x) - x_ref) <= 1e-10 * np.linalg.norm(x_ref)
    finally:
        lib.bidomain_amg_destroy(h)


@pytest.mark.parametrize("mixed,membrane", [(False, "published"), (True, "published"), (False, "other")])
def test_time_steps_match_oracle(torch, mixed, membrane):
    c = bc.make_case(24, 24, 12, seed=2)
    if membrane == "other":  # membrane parameters reach the kernel from the slab description
        from dataclasses import replace
        c = replace(c, ap_k=6.5, ap_a=0.12, ap_eps0=0.003, ap_mu1=0.15, ap_mu2=0.25, ap_t_unit=10.0)
    v0 = bc.nodal_v0(c)
    sim_or = bidomain.create(c, v0, rtol=1e-12)
    prec = lib.BD_F32 if mixed else lib.BD_F64
    sim = lib.bidomain_sim_create(c, dev(torch, v0), rtol=1e-10,
                                  ell_opts=lib.bidomain_default_opts(vcycle_precision=prec),
                                  par_opts=lib.bidomain_default_opts(vcycle_precision=prec, threshold=0.0))
    try:
        out = torch.empty(c.n, dtype=torch.float64, device="cuda")
        for s in range(4):
            bidomain.step(sim_or)
            rc, info = lib.bidomain_step(sim, 1, 1e-10)
            assert rc == lib.BD_OK, info
            for field, ref in ((lib.BD_V, sim_or.v), (lib.BD_UE, sim_or.ue), (lib.BD_W, sim_or.w)):
                lib.bidomain_sim_get(sim, field, out)
                err = np.linalg.norm(host(out) - ref) / np.linalg.norm(ref)
                assert err <= 1e-6, (s, field, err)
    finally:
        lib.bidomain_sim_destroy(sim)


def _far_matrix(n, far, jitter):
    """Rows i of every other block of 256 rows also couple to column i - f - (i % jitter) for f in
    far (jitter 1: a single offset per f); every third row is diagonal only, so tile boundaries
    fall at arbitrary entry alignments."""
    import scipy.sparse as sp
    rng = np.random.default_rng(17)
    rows, cols = [np.arange(n)], [np.arange(n)]
    for f in far:
        i = np.arange(f + jitter, n)
        i = i[(i % 3 != 0) & ((i // 256) % 2 == 0)]
        rows.append(i)
        cols.append(i - f - (i % jitter))
    r, c = np.concatenate(rows), np.concatenate(cols)
    v = np.where(r == c, 4.0, rng.uniform(-1.0, 1.0, r.size))
    return sp.csr_matrix((v, (r, c)), shape=(n, n))


def _product_check(torch, h, A, x, prec):
    """A x through BD_OP_A on level 0 in the handle's precision: float64 within 1e-13 of the
    product; float32 within 2e-5 (max norm, relative) of the float64 product of the float32
    matrix and vector."""
    if prec == lib.BD_F64:
        out = torch.empty(A.shape[0], dtype=torch.float64, device="cuda")
        lib.bidomain_amg_apply(h, lib.BD_OP_A, 0, dev(torch, x), out)
        assert _relerr(host(out), A @ x) <= 1e-13
    else:
        x32 = x.astype(np.float32)
        out = torch.empty(A.shape[0], dtype=torch.float32, device="cuda")
        lib.bidomain_amg_apply(h, lib.BD_OP_A, 0, dev(torch, x32, torch.float32), out)
        A32 = A.astype(np.float32).astype(np.float64)
        assert _relerr(host(out).astype(np.float64), A32 @ x32.astype(np.float64)) <= 2e-5


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n,far,jitter,col_bytes", [(131072, (60000,), 1, 1), (131072, (60000,), 600, 2),
                                                     (131072, (60000, 120000), 600, 3),
                                                     ((1 << 24) + (1 << 16), (60000, 120000), 600, 4)])
def test_product_index_forms(torch, n, far, jitter, col_bytes, prec):
    """The product in each column-index form: an offset dictionary (two distinct column - row
    offsets), 16-bit per-tile offsets (~400 distinct offsets, tiles spanning < 65,536 columns),
    24-bit indices (tiles spanning more, at most 2^24 columns) and 32-bit indices (more than
    2^24 columns).  In the 16-bit case the 256-row tiles alternate between column bases
    ~60,000 apart, so near the end of the matrix the previous tile's entries that an aligned
    chunk picks up decode past the last column unless they are clamped; every result must
    still be exact."""
    A = _far_matrix(n, far, jitter)
    A.sort_indices()
    p = lib.BD_F64 if prec == "f64" else lib.BD_F32
    h = lib.bidomain_amg_setup(A, lib.bidomain_default_opts(max_levels=1, nullspace=0, vcycle_precision=p))
    try:
        info = lib.bidomain_amg_info(h)
        print(f"[gpu] product index forms n={n} far={far} jitter={jitter} {prec} col_bytes={info['col_bytes'][0]} "
              f"tiles={info['tiles'][0]}", flush=True)
        assert info["col_bytes"][0] == col_bytes and info["tiles"][0] > 0
        _product_check(torch, h, A, np.random.default_rng(5).standard_normal(n), p)
    finally:
        lib.bidomain_amg_destroy(h)


def _long_row_matrix(n, base, long_rows, seed):
    """Rows of 0..base-1 entries plus `long_rows` rows of 4,029..12,000 entries (longer than a
    stream tile holds, so the lane-group kernel takes the matrix), row lengths ragged around
    the kernel's trips (256 entries a 64-lane group in float64, 1,024 in float32); columns (7 i + k s_i) mod n with odd s_i, distinct within a
    row since n is a power of two; a diagonal added to every row."""
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    L = rng.integers(0, base, n)
    pick = rng.choice(n, long_rows, replace=False)
    L[pick] = rng.integers(4029, 12001, long_rows)
    L[pick[:4]] = [4029, 4096, 5121, 8191][: min(4, long_rows)]
    step = rng.integers(0, n // 2, n) * 2 + 1
    r = np.repeat(np.arange(n), L)
    k = np.arange(r.size) - np.repeat(np.cumsum(L) - L, L)
    c = (7 * r + k * step[r]) % n
    v = rng.uniform(-1.0, 1.0, r.size)
    d = np.arange(n)
    return sp.csr_matrix((np.concatenate([v, np.full(n, 4.0)]),
                          (np.concatenate([r, d]), np.concatenate([c, d]))), shape=(n, n))


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("n,base,long_rows,col_bytes", [(16384, 400, 64, 2), (16384, 100, 3, 4)])
def test_long_rows_lane_group(torch, n, base, long_rows, col_bytes, prec):
    """Rows longer than a stream tile (coarse levels of the largest slabs reach ~12,000 entries)
    go to the lane-group kernel: 64 lanes a row, with 16-bit column indices, when the mean row
    is long (and there are at most 65,536 columns), fewer lanes and 32-bit indices otherwise;
    the product must still be exact to rounding, in float64 and in float32 (16 entries a lane
    a trip there)."""
    A = _long_row_matrix(n, base, long_rows, seed=23)
    A.sort_indices()
    p = lib.BD_F64 if prec == "f64" else lib.BD_F32
    h = lib.bidomain_amg_setup(A, lib.bidomain_default_opts(max_levels=1, nullspace=0, vcycle_precision=p))
    try:
        info = lib.bidomain_amg_info(h)
        print(f"[gpu] long rows n={n} base={base} long={long_rows} {prec} nnz={A.nnz} "
              f"tiles={info['tiles'][0]}", flush=True)
        assert info["tiles"][0] == 0 and info["col_bytes"][0] == col_bytes
        _product_check(torch, h, A, np.random.default_rng(6).standard_normal(n), p)
    finally:
        lib.bidomain_amg_destroy(h)


def _diag_cases():
    """(name, matrix, expected stored diagonals): the symmetric diagonal form is taken only for
    an exactly symmetric matrix with at most 14 offsets >= 0 that it stores in fewer bytes."""
    import scipy.sparse as sp
    c = bc.make_case(21, 19, 11, seed=3)            # n = 22 * 20 * 12 = 5280
    A = fem.assemble_operators(c)["Aell"].tocsr()
    A.sort_indices()
    out = [("27-point", A, 14)]
    B = A.copy()
    k = B.indptr[100] + 3                            # one value no longer equals its mirror
    B.data[k] = np.nextafter(B.data[k], np.inf)
    out.append(("one value off", B, 0))
    C = A.tolil()
    i = 2000
    j = int(A.indices[A.indptr[i]])                  # drop one mirror entry: pattern asymmetric
    C[j, i] = 0.0
    C = C.tocsr()
    C.eliminate_zeros()
    out.append(("one mirror missing", C, 0))
    n = A.shape[0]
    e = np.ones(n)
    L = sp.diags([-e[1:], 2 * e, -e[1:]], [-1, 0, 1], format="csr")   # 3 nonzeros a row
    out.append(("three-point", L, 0))
    return out


@pytest.mark.parametrize("case", range(4))
def test_diag_form_selection(torch, case):
    name, A, nd = _diag_cases()[case]
    h = lib.bidomain_amg_setup(A, lib.bidomain_default_opts(max_levels=1, nullspace=0))
    try:
        info = lib.bidomain_amg_info(h)
        print(f"[gpu] diagonal form case={name} diags={info['diags'][0]} col_bytes={info['col_bytes'][0]}", flush=True)
        assert info["diags"][0] == nd
        x = np.random.default_rng(8).standard_normal(A.shape[0])
        out = torch.empty(A.shape[0], dtype=torch.float64, device="cuda")
        lib.bidomain_amg_apply(h, lib.BD_OP_A, 0, dev(torch, x), out)
        assert _relerr(host(out), A @ x) <= 1e-14
    finally:
        lib.bidomain_amg_destroy(h)


@pytest.mark.parametrize("dims,coarsening", [((16, 16, 8), "sa"), ((37, 29, 13), "sa"), ((32, 32, 16), "sa"),
                                              ((32, 32, 16), "rs"), ((37, 29, 13), "pmis")])
def test_device_galerkin_equals_host(torch, dims, coarsening):
    """Galerkin products as sparse device products (forced on every level) give the host's
    hierarchy bit for bit: the same levels, patterns and values."""
    c = bc.make_case(*dims, seed=9)
    ops = fem.assemble_operators(c)
    A = ops["Aell"]
    kw = dict(nullspace=1, coarsening={"sa": lib.BD_SA, "rs": lib.BD_RS, "pmis": lib.BD_PMIS}[coarsening])
    if coarsening != "sa":
        kw["threshold"] = 0.5
    hd = lib.bidomain_amg_setup(A, lib.bidomain_default_opts(galerkin_device=2, **kw), ops["m"])
    hh = lib.bidomain_amg_build_host(A, lib.bidomain_default_opts(**kw))
    try:
        idd, ih = lib.bidomain_amg_info(hd), lib.bidomain_amg_info(hh)
        print(f"[gpu] device Galerkin dims={dims} {coarsening} levels={idd['n']}", flush=True)
        assert idd["n"] == ih["n"] and idd["nnz"] == ih["nnz"] and idd["p_nnz"] == ih["p_nnz"]
        for k in range(idd["nlevels"]):
            for which in ([0, 1] if k + 1 < idd["nlevels"] else [0]):
                rd, cd, vd, _ = lib.bidomain_amg_export(hd, k, which)
                rh, ch, vh, _ = lib.bidomain_amg_export(hh, k, which)
                assert np.array_equal(rd, rh) and np.array_equal(cd, ch), (k, which)
                assert np.array_equal(vd, vh), (k, which, np.max(np.abs(vd - vh)))
    finally:
        lib.bidomain_amg_destroy(hd)
        lib.bidomain_amg_destroy(hh)


def _long_row_operands(n, nc, a_per_row, p_per_row, spread, seed, hub=0):
    """A symmetric n x n matrix with about a_per_row entries a row in a band, and a random
    n x nc interpolation with p_per_row entries a row within nc / spread of the diagonal; with
    hub > 0, that many random rows also interpolate from column 0 (so row 0 of the product is
    far longer than the rest)."""
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(n), a_per_row // 2)
    cols = np.clip(rows + rng.integers(-4 * a_per_row, 4 * a_per_row, rows.size), 0, n - 1)
    B = sp.csr_matrix((rng.uniform(-1, 1, rows.size), (rows, cols)), shape=(n, n))
    A = (B + B.T + sp.diags(np.full(n, 4.0 * a_per_row))).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    pr = np.repeat(np.arange(n), p_per_row)
    pc = (pr * nc // n + rng.integers(-nc // spread, nc // spread, pr.size)) % nc
    if hub:
        hr = rng.choice(n, hub, replace=False)
        pr, pc = np.concatenate([pr, hr]), np.concatenate([pc, np.zeros(hub, pc.dtype)])
    P = sp.csr_matrix((rng.uniform(0.1, 1, pr.size), (pr, pc)), shape=(n, nc))
    P.sum_duplicates()
    P.sort_indices()
    return A, P


@pytest.mark.parametrize("n,nc,a_per_row,p_per_row,spread,hub", [(3000, 700, 20, 4, 8, 0), (10000, 9000, 60, 16, 2, 0),
                                                                   (100000, 70000, 20, 2, 1, 5000)])
def test_galerkin_product_device_equals_host(torch, n, nc, a_per_row, p_per_row, spread, hub):
    """The device product on rows of every kind: few partial products (LDS hash); many, with at
    most 65,536 product columns (LDS bitmap, dense accumulation windows, rows longer than one
    window) or more (mark arrays; sorted in LDS, or with more than 8192 distinct columns by an
    ordered scan of the marks, the hub row); equal to the host product bit for bit and to sparse
    algebra within rounding."""
    A, P = _long_row_operands(n, nc, a_per_row, p_per_row, spread, seed=1, hub=hub)
    Cd = lib.bidomain_galerkin(A, P, on_device=True)
    Ch = lib.bidomain_galerkin(A, P, on_device=False)
    longest = int(np.diff(Cd.indptr).max())
    print(f"[gpu] Galerkin n={n} nc={nc}: nnz {Cd.nnz}, longest row {longest}", flush=True)
    assert np.array_equal(Cd.indptr, Ch.indptr) and np.array_equal(Cd.indices, Ch.indices)
    assert np.array_equal(Cd.data, Ch.data)
    R = (P.T @ A @ P).tocsr()
    ref = 0.5 * (R + R.T)
    assert abs(Cd - ref).max() <= 1e-12 * abs(ref).max()
    if n >= 10000:
        assert longest > 8192
    if n <= 65536 and nc <= 65536:
        Cm = lib.bidomain_galerkin(A, P, on_device=2)     # dense MFMA form: same pattern
        assert np.array_equal(Cm.indptr, Ch.indptr) and np.array_equal(Cm.indices, Ch.indices)
        assert np.max(np.abs(Cm.data - Ch.data)) <= 1e-12 * np.max(np.abs(Ch.data))


@pytest.mark.parametrize("dims", [(24, 24, 12), (40, 36, 20)])
def test_dense_device_galerkin_hierarchy(torch, dims):
    """Every level's Galerkin product in the dense MFMA form (galerkin_device = 3): the host's
    levels and patterns, values within rounding of the host's, and a solve that converges like
    the host hierarchy's."""
    c = bc.make_case(*dims, seed=9)
    ops = fem.assemble_operators(c)
    A = ops["Aell"]
    hd = lib.bidomain_amg_setup(A, lib.bidomain_default_opts(nullspace=1, galerkin_device=3), ops["m"])
    hh = lib.bidomain_amg_build_host(A, lib.bidomain_default_opts(nullspace=1))
    try:
        idd, ih = lib.bidomain_amg_info(hd), lib.bidomain_amg_info(hh)
        print(f"[gpu] dense device Galerkin dims={dims} levels={idd['n']}", flush=True)
        assert idd["n"] == ih["n"] and idd["nnz"] == ih["nnz"]
        for k in range(1, idd["nlevels"]):
            rd, cd, vd, _ = lib.bidomain_amg_export(hd, k, 0)
            rh, ch, vh, _ = lib.bidomain_amg_export(hh, k, 0)
            assert np.array_equal(rd, rh) and np.array_equal(cd, ch), k
            assert np.max(np.abs(vd - vh)) <= 1e-11 * np.max(np.abs(vh)), k
    finally:
        lib.bidomain_amg_destroy(hd)
        lib.bidomain_amg_destroy(hh)



@pytest.mark.parametrize("case,kw", [("slab", dict(nullspace=1)), ("ragged", dict(nullspace=1, square_graph_levels=2)),
                                     ("parabolic", dict(threshold=0.0)), ("ellipsoid", dict(nullspace=1))])
def test_device_coarsening_equals_host(torch, case, kw):
    """Strength graph, parallel independent set, aggregation and prolongator smoothing on the
    device (aggregate_device = 1, with the sparse device Galerkin products) give the host
    setup's hierarchy with the same independent set bit for bit: every level's A, P and R."""
    from oracle import ellipsoid
    if case == "ellipsoid":
        ops = ellipsoid.assemble_operators(bc.EllipsoidCase(24, 16, 8))
    else:
        dims = {"slab": (24, 24, 12), "ragged": (37, 29, 13), "parabolic": (32, 32, 16)}[case]
        ops = fem.assemble_operators(bc.make_case(*dims, seed=9))
    A = ops["Apar"] if case == "parabolic" else ops["Aell"]
    base = dict(independent_set=lib.BD_MIS_LUBY, seed=3, **kw)
    hd = lib.bidomain_amg_setup(A, lib.bidomain_default_opts(aggregate_device=1, galerkin_device=2, **base))
    hh = lib.bidomain_amg_build_host(A, lib.bidomain_default_opts(**base))
    try:
        idd, ih = lib.bidomain_amg_info(hd), lib.bidomain_amg_info(hh)
        print(f"[gpu] device coarsening {case}: levels {idd['n']} (host {ih['n']})", flush=True)
        assert idd["n"] == ih["n"] and idd["nnz"] == ih["nnz"] and idd["p_nnz"] == ih["p_nnz"]
        for k in range(idd["nlevels"]):
            for which in ([0, 1, 2] if k + 1 < idd["nlevels"] else [0]):
                rd, cd, vd, _ = lib.bidomain_amg_export(hd, k, which)
                rh, ch, vh, _ = lib.bidomain_amg_export(hh, k, which)
                assert np.array_equal(rd, rh) and np.array_equal(cd, ch), (k, which)
                assert np.array_equal(vd, vh), (k, which, np.max(np.abs(vd - vh)))
        assert np.array_equal(idd["lam"], ih["lam"], equal_nan=True)
    finally:
        lib.bidomain_amg_destroy(hd)
        lib.bidomain_amg_destroy(hh)
