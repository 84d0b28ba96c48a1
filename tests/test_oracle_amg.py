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
