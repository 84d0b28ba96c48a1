"""Pins for the oracle's AMG setup (CPU only): published generator outputs, hand-derived
aggregates and C/F splittings, exact Ritz values, and the algebraic invariants of the
smoothed-aggregation and classical hierarchies."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import bidomain_cases as bc
from oracle import amg, fem


def test_splitmix64_published_outputs():
    # first two outputs of SplitMix64 seeded with 0 (reference values of the published generator)
    out = amg.splitmix64(0, 2)
    assert int(out[0]) == 0xE220A8397B1DCDAF
    assert int(out[1]) == 0x6E789E6AA1B965F4
    u = amg.splitmix_uniform(7, 10000)
    assert u.min() >= -1.0 and u.max() < 1.0 and abs(u.mean()) < 0.05


def _path_laplacian(n):
    A = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tolil()
    A[0, 0] = A[n - 1, n - 1] = 1.0
    return A.tocsr()


def test_mis_and_aggregates_on_a_path():
    A = _path_laplacian(10)
    G = amg.sa_strength(A, 0.06)
    roots = amg.greedy_mis(G, square=False)
    assert np.flatnonzero(roots).tolist() == [0, 2, 4, 6, 8]
    agg = amg.sa_aggregate(G, roots)
    # weights of an interior node's two root neighbours are equal up to rounding, lowest index wins
    assert agg.tolist() == [0, 0, 1, 1, 2, 2, 3, 3, 4, 4]
    roots2 = amg.greedy_mis(G, square=True)
    assert np.flatnonzero(roots2).tolist() == [0, 3, 6, 9]
    agg2 = amg.sa_aggregate(G, roots2)
    assert agg2.tolist() == [0, 0, 1, 1, 1, 2, 2, 2, 3, 3]


def test_aggregation_second_pass():
    # path 0 - 1 - 2 with distance-2 MIS: 0 is the only root; node 2 has no root neighbour, so
    # pass 1 leaves it out and pass 2 joins it to the aggregate of its assigned neighbour 1
    A = _path_laplacian(3)
    G = amg.sa_strength(A, 0.06)
    roots = amg.greedy_mis(G, square=True)
    assert np.flatnonzero(roots).tolist() == [0]
    assert amg.sa_aggregate(G, roots).tolist() == [0, 0, 0]
    # without squaring node 2 is a root of its own
    roots1 = amg.greedy_mis(G, square=False)
    assert np.flatnonzero(roots1).tolist() == [0, 2]
    assert amg.sa_aggregate(G, roots1).tolist() == [0, 0, 1]


def test_ritz_value_is_exact_after_full_krylov_space():
    rng = np.random.default_rng(3)
    Q = rng.standard_normal((8, 8))
    A = sp.csr_matrix(Q @ Q.T + 8 * np.eye(8))
    Dinv = 1.0 / A.diagonal()
    lam = amg.estimate_lambda_max(A, Dinv, 10, seed=5)
    exact = sla.eigh(A.toarray(), np.diag(A.diagonal()), eigvals_only=True)[-1]
    assert lam == pytest.approx(exact, rel=1e-10)


def test_ritz_value_bounds_on_slab():
    c = bc.make_case(6, 6, 3, seed=1)
    A = fem.assemble_operators(c)["Aell"]
    Dinv = 1.0 / A.diagonal()
    lam = amg.estimate_lambda_max(A, Dinv, 10, seed=0)
    exact = sla.eigh(A.toarray(), np.diag(A.diagonal()), eigvals_only=True)[-1]
    assert 0.8 * exact <= lam <= exact * (1 + 1e-12)


@pytest.fixture(scope="module")
def c1_sa():
    c = bc.config_case("C1")
    ops = fem.assemble_operators(c)
    return c, ops, amg.setup(ops["Aell"], amg.AMGOptions(nullspace=True))


def test_sa_invariants(c1_sa):
    c, ops, h = c1_sa
    assert h.levels[-1].A.shape[0] <= 100
    for k, lv in enumerate(h.levels[:-1]):
        n, nc = lv.P.shape
        # aggregates partition the nodes and every aggregate is non-empty
        assert lv.agg.min() == 0 and lv.agg.max() == nc - 1
        assert np.all(np.bincount(lv.agg, minlength=nc) >= 1)
        Pt, Bc = amg.tentative_prolongator(lv.agg, lv.B, nc)
        assert np.array_equal(Bc, h.levels[k + 1].B)
        np.testing.assert_allclose(Pt @ Bc, lv.B, rtol=1e-15)
        # smoothing keeps the near-null vector because A B = 0
        np.testing.assert_allclose(lv.P @ Bc, lv.B, rtol=0, atol=1e-13 * np.abs(lv.B).max())
        Ac = h.levels[k + 1].A
        assert abs(Ac - Ac.T).max() == 0.0
        assert np.abs(Ac @ Bc).max() <= 1e-13 * np.abs(Ac.data).max() * np.abs(Bc).max()
        # R is the transpose of P
        assert abs(lv.R - lv.P.T).max() == 0.0


def test_sa_level_one_is_unsmoothed_aggregate_size(c1_sa):
    c, ops, h = c1_sa
    lv = h.levels[0]
    nc = lv.P.shape[1]
    Pt, _ = amg.tentative_prolongator(lv.agg, lv.B, nc)
    sizes = np.bincount(lv.agg, minlength=nc)
    # level 0 has B = 1, so P_t[i, j] = |C_j|^{-1/2} (Sec. 4)
    np.testing.assert_allclose(Pt.data, sizes[lv.agg] ** -0.5, rtol=1e-15)


def test_rs_on_a_path():
    A = _path_laplacian(9)
    S = amg.rs_strength(A, 0.5)
    cpts = amg.rs_first_pass(S)
    assert np.flatnonzero(cpts).tolist() == [1, 3, 5, 7]
    P = amg.rs_direct_interpolation(A, S, cpts).toarray()
    expect = np.zeros((9, 4))
    expect[0, 0] = 1.0
    for c_idx, i in enumerate([1, 3, 5, 7]):
        expect[i, c_idx] = 1.0
    for i, (l, r) in {2: (0, 1), 4: (1, 2), 6: (2, 3)}.items():
        expect[i, l] = expect[i, r] = 0.5
    expect[8, 3] = 1.0
    np.testing.assert_allclose(P, expect, rtol=0, atol=1e-15)


def test_rs_invariants_on_c1():
    c = bc.config_case("C1")
    A = fem.assemble_operators(c)["Aell"]
    h = amg.setup(A, amg.AMGOptions(coarsening="rs", threshold=0.5, nullspace=True))
    for k, lv in enumerate(h.levels[:-1]):
        A_k = lv.A
        S = amg.rs_strength(A_k, 0.5)
        cp = lv.cpts.astype(bool)
        P = lv.P
        # every F point interpolates from at least one strong C neighbour
        for i in np.flatnonzero(~cp):
            strong = S.indices[S.indptr[i]:S.indptr[i + 1]]
            assert cp[strong].any()
            assert P.indptr[i + 1] > P.indptr[i]
        # direct interpolation reproduces constants on zero-row-sum rows
        rs = np.abs(A_k @ np.ones(A_k.shape[0])) <= 1e-13 * np.abs(A_k).max()
        np.testing.assert_allclose((P @ np.ones(P.shape[1]))[rs], 1.0, rtol=0, atol=1e-13)
        Ac = h.levels[k + 1].A
        assert abs(Ac - Ac.T).max() == 0.0


def test_coarsening_stops_on_weakly_coupled_operator():
    c = bc.make_case(16, 16, 8, seed=1)
    Apar = fem.assemble_operators(c)["Apar"]
    h = amg.setup(Apar, amg.AMGOptions())
    # the mass term dominates on this coarse mesh: no edge reaches theta, no coarsening, and the
    # oversized coarsest level is relaxed by its smoother rather than factorised
    assert h.nlevels == 1 and h.coarse_factor is None and np.isfinite(h.levels[0].lam)


def test_smoothed_prolongator_hand_derived_neumann_path():
    """P = (I - omega D^-1 A) P_t with omega = 4 / (3 lambda), written out by hand.

    Path of four nodes with Neumann ends, A = [[1,-1,0,0],[-1,2,-1,0],[0,-1,2,-1],[0,0,-1,1]],
    D = diag(1, 2, 2, 1); aggregates {0, 1}, {2, 3}, s = 2^-1/2.  A P_t = s [[0,0],[1,-1],[-1,1],[0,0]],
    D^-1 A P_t = s [[0,0],[1/2,-1/2],[-1/2,1/2],[0,0]].  D^-1 A has eigenvalues 1 - cos(k pi/3),
    so lambda = 2 and omega = 2/3: P = s [[1,0],[2/3,1/3],[1/3,2/3],[0,1]].
    """
    A = _path_laplacian(4)
    s = 2.0 ** -0.5
    Pt = sp.csr_matrix(np.array([[s, 0], [s, 0], [0, s], [0, s]]))
    P = amg.smooth_prolongator(A, 1.0 / A.diagonal(), Pt, 2.0, 1).toarray()
    expect = s * np.array([[1, 0], [2 / 3, 1 / 3], [1 / 3, 2 / 3], [0, 1]])
    np.testing.assert_allclose(P, expect, rtol=0, atol=1e-15)


def test_smoothed_prolongator_in_setup_dirichlet_path():
    """The same product inside setup(), with lambda from the eigenvalue estimate.

    A = tridiag(-1, 2, -1) on four nodes (SPD), D = 2 I.  D^-1 A has eigenvalues 1 - cos(k pi/5),
    k = 1..4, so after a complete Krylov space lambda = 1 + cos(pi/5) = (5 + 5^1/2)/4 and
    omega = 4/(3 lambda) = 4 (5 - 5^1/2)/15.  All couplings have weight 1/2; node 1 ties between
    roots 0 and 2 and joins 0 (greedy independent set in index order), so the aggregates are
    {0, 1}, {2, 3}.  D^-1 A P_t =
    (s/2) [[1,0],[1,-1],[-1,1],[0,1]], hence P = s [[1-w,0],[1-w,w],[w,1-w],[0,1-w]], w = omega/2.
    """
    A = sp.csr_matrix(np.array([[2., -1, 0, 0], [-1, 2, -1, 0], [0, -1, 2, -1], [0, 0, -1, 2]]))
    h = amg.setup(A, amg.AMGOptions(coarse_eq_limit=2, square_graph_levels=0, mis="greedy"))
    lv = h.levels[0]
    assert lv.agg.tolist() == [0, 0, 1, 1]
    assert lv.lam == pytest.approx((5 + 5 ** 0.5) / 4, rel=1e-14)
    w = 2 * (5 - 5 ** 0.5) / 15
    s = 2.0 ** -0.5
    expect = s * np.array([[1 - w, 0], [1 - w, w], [w, 1 - w], [0, 1 - w]])
    np.testing.assert_allclose(lv.P.toarray(), expect, rtol=0, atol=1e-14)


def _rs_star():
    """Centre 0 (diagonal 10) coupled to 1 (-4), 2 (+3), 3 (-2), 4 (-1), 5 (+1); each leaf is
    coupled to the centre only."""
    off = {1: -4.0, 2: 3.0, 3: -2.0, 4: -1.0, 5: 1.0}
    A = np.zeros((6, 6))
    A[0, 0] = 10.0
    for j, a in off.items():
        A[0, j] = A[j, 0] = a
        A[j, j] = 5.0
    return sp.csr_matrix(A)


def test_rs_strength_eq10_cuts_and_keeps_positive_couplings():
    """Eq. (10) with alpha = 0.5: row 0 has max |a_0k| = 4, so |a| >= 2 is strong: 1 (-4), 2 (+3),
    3 (-2) strong; 4 (-1) and 5 (+1) weak.  A leaf's only coupling is its own maximum."""
    S = amg.rs_strength(_rs_star(), 0.5)
    strong = {i: S.indices[S.indptr[i]:S.indptr[i + 1]].tolist() for i in range(6)}
    assert strong == {0: [1, 2, 3], 1: [0], 2: [0], 3: [0], 4: [0], 5: [0]}
    # a smaller alpha keeps the weak couplings too; a larger one cuts 3 and then 2
    assert amg.rs_strength(_rs_star(), 0.25).indices[:5].tolist() == [1, 2, 3, 4, 5]
    row0 = lambda al: amg.rs_strength(_rs_star(), al)[0].indices.tolist()
    assert row0(0.6) == [1, 2] and row0(0.8) == [1]


def test_rs_direct_interpolation_both_sign_classes():
    """F point 0 of the star with C points {1, 2}: P_0 = C cap S_0 = {1, 2}.
    Sums over all neighbours: negative -4 - 2 - 1 = -7, positive 3 + 1 = 4; over P_0: -4 and 3.
    alpha_0 = 7/4, beta_0 = 4/3, abar = a_00 = 10 (both classes interpolate).
    w_01 = -(7/4)(-4)/10 = 0.7, w_02 = -(4/3)(3)/10 = -0.4."""
    A = _rs_star()
    S = amg.rs_strength(A, 0.5)
    cpts = np.array([0, 1, 1, 0, 0, 0], dtype=np.int8)
    P = amg.rs_direct_interpolation(A, S, cpts).toarray()
    expect = np.zeros((6, 2))
    expect[0] = [0.7, -0.4]
    expect[1, 0] = expect[2, 1] = 1.0           # C points inject; leaves 3-5 have no strong C point
    np.testing.assert_allclose(P, expect, rtol=0, atol=1e-15)


def test_rs_direct_interpolation_lumps_a_class_without_interpolatory_member():
    """F point 0 with a_00 = 6, a_01 = -3 (C), a_02 = +2 (F, strong).  No positive coupling
    interpolates, so it is lumped: abar = 6 + 2 = 8; alpha_0 = -3/-3 = 1; w_01 = 3/8."""
    A = sp.csr_matrix(np.array([[6., -3, 2], [-3, 4, 0], [2, 0, 4]]))
    S = amg.rs_strength(A, 0.5)
    assert S[0].indices.tolist() == [1, 2]
    P = amg.rs_direct_interpolation(A, S, np.array([0, 1, 0], dtype=np.int8)).toarray()
    np.testing.assert_allclose(P, [[3 / 8], [1.0], [0.0]], rtol=0, atol=1e-15)


def test_sa_strength_uses_absolute_scaled_coupling():
    """w_ij = |a_ij| / sqrt(a_ii a_jj) (Sec. 4, with the absolute value of reading R8):
    star of _rs_star with diagonals 10 and 5: w = 4/sqrt(50) = 0.566, 3/sqrt(50) = 0.424,
    0.283, 0.141, 0.141.  theta = 0.2 keeps 1, 2, 3 (positive coupling 2 included) and cuts 4, 5;
    theta = 0.3 cuts 3 as well."""
    A = _rs_star()
    G = amg.sa_strength(A, 0.2)
    assert G[0].indices.tolist() == [1, 2, 3]
    np.testing.assert_allclose(G[0].data, np.array([4, 3, 2]) / 50 ** 0.5, rtol=1e-15)
    assert G[2].indices.tolist() == [0]         # symmetric: the positive edge is kept both ways
    assert amg.sa_strength(A, 0.3)[0].indices.tolist() == [1, 2]


def _digraph(rows):
    n = len(rows)
    A = np.zeros((n, n))
    for i, js in enumerate(rows):
        A[i, js] = 1.0
    return sp.csr_matrix(A)


def test_pmis_on_a_path_follows_the_measures():
    """Symmetric path 0-1-2-3-4: |S_i^T| = 1, 2, 2, 2, 1.
    Draws (.1, .5, .3, .9, .2): measures 1.1, 2.5, 2.3, 2.9, 1.2; points 1 and 3 beat all their
    neighbours and become C in the first round, and 0, 2, 4 (each depending on one of them) F.
    Draws (.9, .1, .8, .2, .7): measures 1.9, 2.1, 2.8, 2.2, 1.7; round 1 selects 2 and makes 1, 3
    F; in round 2, 0 and 4 have no undecided neighbour left and become C."""
    S = _digraph([[1], [0, 2], [1, 3], [2, 4], [3]])
    assert amg.pmis_split(S, np.array([0.1, 0.5, 0.3, 0.9, 0.2])).tolist() == [0, 1, 0, 1, 0]
    assert amg.pmis_split(S, np.array([0.9, 0.1, 0.8, 0.2, 0.7])).tolist() == [1, 0, 1, 0, 1]


def test_pmis_independence_uses_both_directions():
    """S: 0 depends on 1, 2, 4; 1 and 2 on 0; 4 on 2, 3; 3 on nothing.  |S^T| = 2, 1, 2, 1, 1;
    draws (.45, .85, .25, .35, .95): measures 2.45, 1.85, 2.25, 1.35, 1.95.
    Round 1: 0 beats its neighbours 1, 2, 4 in S + S^T (4 is a neighbour only through 0 -> 4) and
    becomes C; 1 and 2 depend on 0 and become F; 4 does not depend on 0 and stays.  Round 2: 4
    beats 3 and becomes C (3 depends on nothing, so it stays).  Round 3: 3 has no undecided
    neighbour and becomes C.  C = {0, 3, 4}: later C points may influence earlier ones.  Taking
    only S_i (not S_i^T) as the neighbourhood would let 4 into round 1's set next to 0."""
    S = _digraph([[1, 2, 4], [0], [0], [], [2, 3]])
    assert amg.pmis_split(S, np.array([0.45, 0.85, 0.25, 0.35, 0.95])).tolist() == [1, 0, 0, 1, 1]


def test_pmis_f_points_are_those_depending_on_a_new_c_point():
    """S: 0 -> 2, 1 -> 0, 2 -> 1, 3, 3 -> 1, 4 -> 1, 3.  |S^T| = 1, 3, 1, 2, 0, so 4 is F from
    the start.  Draws (.25, .55, .85, .25, .15): measures 1.25, 3.55, 1.85, 2.25.  Round 1: 1 is C;
    2 and 3 depend on 1 and become F; 0 only influences 1 (1 -> 0) and stays.  Round 2: 0 has no
    undecided neighbour and becomes C.  C = {0, 1}; marking every neighbour of a new C point F
    (instead of its dependants) would leave C = {1}."""
    S = _digraph([[2], [0], [1, 3], [1], [1, 3]])
    assert amg.pmis_split(S, np.array([0.25, 0.55, 0.85, 0.25, 0.15])).tolist() == [1, 1, 0, 0, 0]


def test_pmis_invariants_on_c1():
    c = bc.config_case("C1")
    A = fem.assemble_operators(c)["Aell"]
    h = amg.setup(A, amg.AMGOptions(coarsening="pmis", threshold=0.5, nullspace=True))
    assert h.nlevels >= 2
    for k, lv in enumerate(h.levels[:-1]):
        S = amg.rs_strength(lv.A, 0.5)
        ST = S.T.tocsr()
        cp = lv.cpts.astype(bool)
        influence = np.diff(ST.indptr)
        for i in np.flatnonzero(~cp):
            # an F point either influences nobody or depends strongly on a C point
            strong = S.indices[S.indptr[i]:S.indptr[i + 1]]
            assert influence[i] == 0 or cp[strong].any()
        # the draws are the documented SplitMix64 stream, and the split is what they give
        r = amg.pmis_random(0, k, lv.A.shape[0])
        assert 0.0 <= r.min() and r.max() < 1.0
        assert np.array_equal(amg.pmis_split(S, r), lv.cpts)


def test_luby_order_on_a_path_by_hand():
    """Path 0 - 1 - 2 - 3 - 4, priorities (5, 9, 1, 7, 3): unsquared, 1 (9) takes 0 and 2, then 3
    (7) takes 4 -> roots {1, 3}; squared, 1 takes 0, 2 and 3, and 4 (distance 3 from 1) becomes
    a root -> roots {1, 4}."""
    A = _path_laplacian(5)
    G = amg.sa_strength(A, 0.06)
    keys = np.array([5, 9, 1, 7, 3], dtype=np.uint64)
    order = np.argsort(keys)[::-1]
    assert np.flatnonzero(amg.greedy_mis(G, square=False, order=order)).tolist() == [1, 3]
    assert np.flatnonzero(amg.greedy_mis(G, square=True, order=order)).tolist() == [1, 4]


def _parallel_rounds(G, keys, square):
    """The parallel (Luby-type) independent set written as its rounds: every free node whose key
    beats all free nodes within reach becomes a root; the free nodes within reach of a new root
    are taken.  Reach = neighbours in G, or nodes within distance 2 when squared."""
    n = G.shape[0]
    R = (G + sp.eye(n)).tocsr()
    if square:
        R = (R @ R).tocsr()
    R = (R != 0).astype(np.int8).tocsr()
    rows = np.repeat(np.arange(n), np.diff(R.indptr))
    cols = R.indices
    FREE, ROOT, TAKEN = 0, 1, 2
    st = np.zeros(n, dtype=np.int8)
    kf = keys.astype(object)
    while np.any(st == FREE):
        free = st == FREE
        best = np.zeros(n, dtype=object)
        for r, c in zip(rows.tolist(), cols.tolist()):
            if free[c] and kf[c] > best[r]:
                best[r] = kf[c]
        new = free & np.array([best[i] == kf[i] for i in range(n)])
        assert new.any()
        st[new] = ROOT
        reach = (R @ new.astype(np.int64)) > 0
        st[(st == FREE) & reach] = TAKEN
    return st == ROOT


@pytest.mark.parametrize("square", [False, True])
def test_luby_order_equals_the_parallel_rounds(square):
    """With fixed priorities the parallel rounds end in the greedy set taken in decreasing
    priority order (the oracle's 'luby' variant): checked on random graphs and on a slab's
    strength graph, against the rounds written out above."""
    rng = np.random.default_rng(11)
    graphs = []
    for n in (30, 60):
        M = sp.random(n, n, density=0.08, random_state=rng, format="csr")
        M = ((M + M.T) != 0).astype(np.float64)
        M.setdiag(0)
        M.eliminate_zeros()
        graphs.append(M.tocsr())
    A = fem.assemble_operators(bc.make_case(5, 4, 3, seed=1))["Aell"]
    graphs.append(amg.sa_strength(A, 0.06))
    for G in graphs:
        n = G.shape[0]
        keys = amg.luby_keys(7, 2, n)
        mis = amg.greedy_mis(G, square=square, order=np.argsort(keys)[::-1])
        assert np.array_equal(mis, _parallel_rounds(G, keys, square))


def test_luby_keys_are_distinct_and_follow_the_stream():
    keys = amg.luby_keys(5, 3, 1000)
    assert len(set(keys.tolist())) == 1000
    z = amg.splitmix64(5 + amg.LUBY_SEED_OFFSET + 3, 1000)
    assert np.array_equal(keys >> np.uint64(32), z >> np.uint64(32))
    assert np.array_equal(keys & np.uint64(0xFFFFFFFF), np.arange(1000, dtype=np.uint64))


def test_luby_hierarchy_invariants_on_c1():
    """The SA hierarchy with the parallel independent set keeps the SA invariants: roots
    independent within distance 2 on the first level, every node aggregated, P B_c = B."""
    c = bc.config_case("C1")
    A = fem.assemble_operators(c)["Aell"]
    h = amg.setup(A, amg.AMGOptions(nullspace=True, mis="luby", seed=4))
    hg = amg.setup(A, amg.AMGOptions(nullspace=True, mis="greedy"))
    lv = h.levels[0]
    G = amg.sa_strength(A, 0.06)
    roots = amg.greedy_mis(G, square=True, order=np.argsort(amg.luby_keys(4, 0, A.shape[0]))[::-1])
    R2 = ((G + sp.eye(A.shape[0])) @ (G + sp.eye(A.shape[0]))).tocsr()
    ri = np.flatnonzero(roots)
    sub = R2[ri][:, ri]
    assert sub.nnz == ri.size                      # only the diagonal: no two roots within reach
    assert np.all((R2 @ roots.astype(float)) > 0)  # maximal
    assert lv.P.shape[1] == ri.size
    assert np.allclose(lv.P @ h.levels[1].B, lv.B)
    assert h.levels[1].A.shape != hg.levels[1].A.shape or not np.array_equal(lv.agg, hg.levels[0].agg)
