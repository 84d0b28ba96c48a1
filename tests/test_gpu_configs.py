"""GPU parity for configurations beyond the default path, each against the CPU oracle on the same
seeded inputs (through the C ABI):

* the other smoothers of Alg. 2 / App. A: damped Jacobi (degree 2, 3) and Chebyshev of degree 1
  and 3 -- every level's pre-smoothing and V-cycle, and a full solve;
* the lane-group product (rows longer than a CSR-stream tile holds, as on the coarse levels of
  the largest slabs) inside the V-cycle and the CG: its fused smoothing, residual and reduction
  epilogues, with 16-bit and 32-bit column indices;
* the mixed-precision form (float32 V-cycle inside float64 flexible CG) with smoothed-aggregation,
  classical (first-pass) and PMIS hierarchies on an aspect-2 slab with eight stimulus ellipsoids
  (the stimulus law and element shape of the 256 x 256 x 64 and 384 x 384 x 96 workloads), large
  enough that the classical hierarchies' first coarse level has more than 65,536 rows.

Bars as in test_gpu_solve: level operations 1e-12 (V-cycle 1e-10) relative to the oracle's on the
oracle's own hierarchy; solves reach the true relative residual 1e-8, relative error <= 1e-6
against the oracle's rtol-1e-12 float64 solution, iteration counts within 1 (float64) or 2
(float32 V-cycles) of the oracle's.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import bidomain_cases as bc
from oracle import amg, fem, krylov

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


def _relerr(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def _level_ops(torch, h, h_or, levels, rng, null):
    """Every level's pre-smoothing and V-cycle against the oracle's."""
    for k in levels:
        lv = h_or.levels[k]
        n = lv.A.shape[0]
        x = rng.uniform(-1, 1, n)
        out = torch.empty(n, dtype=torch.float64, device="cuda")
        lib.bidomain_amg_apply(h, lib.BD_OP_A, k, dev(torch, x), out)
        assert _relerr(host(out), lv.A @ x) <= 1e-12, f"A_{k}"
        if lv.P is None:
            continue
        out = torch.empty(n, dtype=torch.float64, device="cuda")
        lib.bidomain_amg_apply(h, lib.BD_OP_PRESMOOTH, k, dev(torch, x), out)
        assert _relerr(host(out), krylov.smooth(h_or, k, x, None)) <= 1e-12, f"S_{k}"
        fk = x - x.mean() if null else x
        out = torch.empty(n, dtype=torch.float64, device="cuda")
        lib.bidomain_amg_apply(h, lib.BD_OP_VCYCLE, k, dev(torch, fk), out)
        assert _relerr(host(out), krylov.vcycle(h_or, fk, k)) <= 1e-10, f"V_{k}"


def _solve_and_check(torch, h, A, f, m, ref, or_its, null, slack):
    n = A.shape[0]
    x = torch.zeros(n, dtype=torch.float64, device="cuda")
    rc, info = lib.bidomain_pcg_solve(h, dev(torch, f), x, False, 1e-8, 500)
    assert rc == lib.BD_OK, info
    xs = host(x)
    fh = f - f.mean() if null else f
    assert np.linalg.norm(fh - A @ xs) <= 1e-8 * np.linalg.norm(fh) * (1 + 1e-6)
    if null:
        assert abs(m @ xs) <= 1e-12 * np.abs(xs).max() * m.sum()
    assert np.linalg.norm(xs - ref) <= 1e-6 * np.linalg.norm(ref)
    assert abs(info["iterations"] - or_its) <= slack, (info["iterations"], or_its)
    return info


SMOOTHERS = {"jacobi2": ("jacobi", lib.BD_JACOBI, 2), "jacobi3": ("jacobi", lib.BD_JACOBI, 3),
             "cheb1": ("chebyshev", lib.BD_CHEBYSHEV, 1), "cheb3": ("chebyshev", lib.BD_CHEBYSHEV, 3)}


@pytest.mark.parametrize("smoother", list(SMOOTHERS))
def test_smoother_variants_match_oracle(torch, smoother):
    name, code, deg = SMOOTHERS[smoother]
    c = bc.make_case(37, 29, 13, seed=7)
    ops = fem.assemble_operators(c)
    A, m = ops["Aell"], ops["m"]
    f = -(ops["Ai"] @ bc.nodal_v0(c))
    h_or = amg.setup(A, amg.AMGOptions(nullspace=True, smoother=name, degree=deg))
    ref = krylov.amg_pcg(A, f, h_or, rtol=1e-12, m=m)
    or8 = krylov.amg_pcg(A, f, h_or, rtol=1e-8, m=m)
    print(f"[gpu] smoother={smoother} levels={h_or.nlevels} oracle_its={or8.iterations}", flush=True)
    h = lib.bidomain_amg_setup(A, lib.bidomain_default_opts(nullspace=1, smoother=code, smoother_degree=deg), m)
    try:
        assert lib.bidomain_amg_info(h)["n"] == [lv.A.shape[0] for lv in h_or.levels]
        _level_ops(torch, h, h_or, range(h_or.nlevels), np.random.default_rng(3), True)
        _solve_and_check(torch, h, A, f, m, ref.x, or8.iterations, True, 1)
    finally:
        lib.bidomain_amg_destroy(h)
    # the float32 V-cycle with the same smoother
    h = lib.bidomain_amg_setup(A, lib.bidomain_default_opts(nullspace=1, smoother=code, smoother_degree=deg,
                                                            vcycle_precision=lib.BD_F32), m)
    try:
        or32 = krylov.amg_fcg_mixed(A, f, h_or, rtol=1e-8, m=m)
        _solve_and_check(torch, h, A, f, m, ref.x, or32.iterations, True, 2)
    finally:
        lib.bidomain_amg_destroy(h)


def _long_row_spd(n, base, long_rows, seed):
    """A symmetric positive definite matrix with rows of up to `base` random couplings plus
    `long_rows` rows of 4,029..9,000 (longer than a CSR-stream tile holds) and their mirrors;
    diagonal 0.55 x the absolute row sum + 1 (strictly diagonally dominant)."""
    rng = np.random.default_rng(seed)
    L = rng.integers(0, base, n)
    pick = rng.choice(n, long_rows, replace=False)
    L[pick] = rng.integers(4029, 9000, long_rows)
    step = rng.integers(0, n // 2, n) * 2 + 1
    r = np.repeat(np.arange(n), L)
    k = np.arange(r.size) - np.repeat(np.cumsum(L) - L, L)
    col = (7 * r + k * step[r]) % n
    S = sp.csr_matrix((rng.uniform(-1.0, 1.0, r.size), (r, col)), shape=(n, n))
    S = S - sp.diags(S.diagonal())
    A = (S + S.T).tocsr()
    A.eliminate_zeros()
    A = (A + sp.diags(np.asarray(abs(A).sum(axis=1)).ravel() * 0.55 + 1.0)).tocsr()
    A.sort_indices()
    return A


@pytest.mark.parametrize("base,long_rows,col_bytes", [(400, 64, 2), (100, 3, 4)])
def test_lane_group_vcycle_matches_oracle(torch, base, long_rows, col_bytes):
    n = 16384
    A = _long_row_spd(n, base, long_rows, 23)
    opts = dict(threshold=0.0, square_graph_levels=0)
    h_or = amg.setup(A, amg.AMGOptions(**opts))
    x_true = np.random.default_rng(4).standard_normal(n)
    f = A @ x_true
    ref = krylov.amg_pcg(A, f, h_or, rtol=1e-12)
    or8 = krylov.amg_pcg(A, f, h_or, rtol=1e-8)
    print(f"[gpu] lane group base={base} long={long_rows} levels={[lv.A.shape[0] for lv in h_or.levels]} "
          f"oracle_its={or8.iterations}", flush=True)
    for prec in (lib.BD_F64, lib.BD_F32):
        h = lib.bidomain_amg_setup(A, lib.bidomain_default_opts(nullspace=0, vcycle_precision=prec, **opts))
        try:
            info = lib.bidomain_amg_info(h)
            assert info["n"] == [lv.A.shape[0] for lv in h_or.levels]
            assert info["tiles"][0] == 0 and info["col_bytes"][0] == col_bytes   # the lane-group kernel
            if prec == lib.BD_F64:
                _level_ops(torch, h, h_or, [0], np.random.default_rng(5), False)
                _solve_and_check(torch, h, A, f, None, ref.x, or8.iterations, False, 1)
            else:
                or32 = krylov.amg_fcg_mixed(A, f, h_or, rtol=1e-8)
                _solve_and_check(torch, h, A, f, None, ref.x, or32.iterations, False, 2)
        finally:
            lib.bidomain_amg_destroy(h)


@pytest.fixture(scope="module")
def aspect2():
    c = bc.make_case(96, 96, 24, seed=3, n_ellipsoids=8)   # h_z = 2 h_x, as in the larger workloads
    ops = fem.assemble_operators(c)
    f = -(ops["Ai"] @ bc.nodal_v0(c))
    return c, ops, f


@pytest.mark.parametrize("coarsening", ["sa", "rs", "pmis"])
def test_mixed_form_on_aspect2_slab(torch, aspect2, coarsening):
    c, ops, f = aspect2
    A, m = ops["Aell"], ops["m"]
    thr = 0.06 if coarsening == "sa" else 0.5
    h_or = amg.setup(A, amg.AMGOptions(nullspace=True, coarsening=coarsening, threshold=thr))
    ref = krylov.amg_pcg(A, f, h_or, rtol=1e-12, m=m)
    or64 = krylov.amg_pcg(A, f, h_or, rtol=1e-8, m=m)
    or32 = krylov.amg_fcg_mixed(A, f, h_or, rtol=1e-8, m=m)
    sizes = [lv.A.shape[0] for lv in h_or.levels]
    print(f"[gpu] aspect-2 slab n={c.n} {coarsening} levels={sizes} oracle_its f64={or64.iterations} "
          f"f32={or32.iterations}", flush=True)
    if coarsening != "sa":
        assert sizes[1] > 65536
    code = {"sa": lib.BD_SA, "rs": lib.BD_RS, "pmis": lib.BD_PMIS}[coarsening]
    for prec, its, slack in ((lib.BD_F64, or64.iterations, 1), (lib.BD_F32, or32.iterations, 2)):
        h = lib.bidomain_amg_setup(A, lib.bidomain_default_opts(nullspace=1, coarsening=code, threshold=thr,
                                                                vcycle_precision=prec), m)
        try:
            info = lib.bidomain_amg_info(h)
            assert info["n"] == sizes and info["nnz"] == [lv.A.nnz for lv in h_or.levels]
            _solve_and_check(torch, h, A, f, m, ref.x, its, True, slack)
        finally:
            lib.bidomain_amg_destroy(h)
