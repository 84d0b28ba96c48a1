"""AMG setup (oracle; test infrastructure only).

Paper: Alg. 1 (setup: C/F split, P^k, R^k = (P^k)^T, A^{k+1} = R^k A^k P^k, smoother setup);
Sec. 4 (smoothed aggregation: strength weights w_ij = a_ij / sqrt(a_ii a_jj), cut below the
threshold, greedy MIS, clusters C_j joined by maximal weight, P_ij = |C_j|^{-1/2}; classical
coarsening: strong set |a_ij| >= alpha max_{k != i} |a_ik|, eq. (10)); App. A (one prolongator
smoothing, coarse-equation limit 100, graph squaring on the first level, Chebyshev degree 2
on Jacobi-scaled A over [0.05, 1.05] x lambda_max estimated by 10 CG steps).

Readings where the paper is silent or ambiguous:
  * strength uses |a_ij| (the slab operators have large positive off-diagonal entries);
    an edge is kept iff w_ij >= theta (1 - 1e-12) and a_ij != 0;
  * MIS is greedy in increasing index order; a node with no strong edge is its own root;
  * aggregation: pass 1 joins each non-root to the strongly connected root of largest w;
    pass 2 (reading a snapshot of pass 1) joins each leftover node to the aggregate of its
    assigned strong neighbour of largest w; weights within 1e-12 (relative) tie and the
    lowest index wins; the coarse index of an aggregate is the rank of its root;
  * tentative prolongator with the near-null vector B normalised per aggregate,
    P_t[i, j] = B_i / ||B|_{C_j}||, B_c[j] = ||B|_{C_j}||; with B = 1 this is |C_j|^{-1/2};
  * prolongator smoothing P = (I - omega D^{-1} A) P_t with omega = 4 / (3 lambda);
  * lambda = largest Ritz value of `esteig_iters` Jacobi-preconditioned CG steps from a
    SplitMix64 start vector (seed + level), via the CG/Lanczos tridiagonal;
  * A_c = R (A P), then symmetrised (A_c + A_c^T) / 2; no dropping;
  * classical (Ruge-Stueben) first pass and Stueben's direct interpolation, with both
    positive and negative couplings interpolated separately; or the PMIS split (the parallel
    independent-set coarsening of [des06], on which BoomerAMG's GPU setup relies) with the same
    strength and interpolation, its random tie-breaking draws from SplitMix64;
  * coarsening stops once a level has at most `coarse_eq_limit` rows, at `max_levels`, or
    when it would keep more than `stagnation_ratio` of the rows (weakly coupled operators,
    e.g. the mass-dominated parabolic matrix on coarse meshes);
  * the coarsest level is solved directly (dense Cholesky) when it has at most
    `coarse_dense_max` rows (a one-row coarsest level of the singular operator gives a zero
    correction, since its b-perp space is {0}); a larger coarsest level (only reached through stagnation) is
    instead relaxed by the level's smoother from a zero guess.
"""
from __future__ import annotations

import heapq
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

TIE = 1e-12


@dataclass
class AMGOptions:
    coarsening: str = "sa"          # "sa" (smoothed aggregation), "rs" (classical, first pass)
                                    # or "pmis" (classical strength, PMIS split)
    threshold: float = 0.06         # SA theta; for "rs" the strong threshold alpha
    square_graph_levels: int = 1
    prolong_smooths: int = 1
    coarse_eq_limit: int = 100
    max_levels: int = 25
    smoother: str = "chebyshev"     # or "jacobi"
    degree: int = 2
    cheb_lo: float = 0.05
    cheb_hi: float = 1.05
    esteig_iters: int = 10
    seed: int = 0
    nullspace: bool = False         # True: pure Neumann operator with constant kernel
    stagnation_ratio: float = 0.9   # stop coarsening when n_c > ratio * n_k
    coarse_dense_max: int = 2048    # larger coarsest levels are relaxed by their smoother
    mis: str = "luby"               # SA independent set: "luby" (random priorities, the
                                    # parallel algorithm's outcome) or "greedy" (index order)


@dataclass
class Level:
    A: sp.csr_matrix
    B: np.ndarray
    Dinv: np.ndarray
    lam: float = float("nan")
    P: Optional[sp.csr_matrix] = None
    R: Optional[sp.csr_matrix] = None
    agg: Optional[np.ndarray] = None     # SA: aggregate of each fine node
    cpts: Optional[np.ndarray] = None    # RS: C/F marker (1 = C)


@dataclass
class Hierarchy:
    levels: List[Level]
    opts: AMGOptions
    coarse_factor: object = None
    coarse_bbar: Optional[np.ndarray] = None

    @property
    def nlevels(self):
        return len(self.levels)


# ---------------------------------------------------------------------------------------------
# SplitMix64 (Steele, Lea & Flood, OOPSLA 2014), counter form: output i of the stream seeded
# with s is mix(s + (i + 1) * GAMMA).
_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, count: int) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (np.arange(1, count + 1, dtype=np.uint64) * _GAMMA)
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def splitmix_uniform(seed: int, count: int) -> np.ndarray:
    """Uniform doubles in [-1, 1): 2 * (top 53 bits / 2^53) - 1."""
    u = (splitmix64(seed, count) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return 2.0 * u - 1.0


# ---------------------------------------------------------------------------------------------
def estimate_lambda_max(A: sp.csr_matrix, Dinv: np.ndarray, iters: int, seed: int) -> float:
    """Largest Ritz value of D^{-1} A from `iters` steps of Jacobi-preconditioned CG.

    CG on A x = b, x0 = 0, b from SplitMix64; alpha_j = rho_j / p_j^T A p_j, beta_j =
    rho_{j+1} / rho_j; the Lanczos tridiagonal is T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1},
    T_{j,j+1} = sqrt(beta_j) / alpha_j (Saad, Iterative Methods, Sec. 6.7.3).
    """
    b = splitmix_uniform(seed, A.shape[0])
    r = b.copy()
    z = Dinv * r
    p = z.copy()
    rho = r @ z
    rho0 = rho
    alphas, betas = [], []
    for j in range(iters):
        q = A @ p
        pq = p @ q
        if not pq > 0.0:
            break
        alpha = rho / pq
        alphas.append(alpha)
        if j == iters - 1:
            break
        r = r - alpha * q
        z = Dinv * r
        rho_new = r @ z
        if not rho_new > 1e-28 * rho0:
            break
        betas.append(rho_new / rho)
        p = z + (rho_new / rho) * p
        rho = rho_new
    m = len(alphas)
    if m == 0:
        return float(np.max(Dinv * A.diagonal()))
    T = np.zeros((m, m))
    for j in range(m):
        T[j, j] = 1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
        if j + 1 < m:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(betas[j]) / alphas[j]
    return float(np.linalg.eigvalsh(T)[-1])


# ---------------------------------------------------------------------------------------------
# Smoothed aggregation (Sec. 4).
def sa_strength(A: sp.csr_matrix, theta: float) -> sp.csr_matrix:
    """Strength graph: edge (i, j), j != i, kept iff |a_ij| / sqrt(a_ii a_jj) >= theta and a_ij != 0.

    The returned matrix stores the weight w_ij on every kept edge.
    """
    n = A.shape[0]
    d = A.diagonal()
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    cols = A.indices
    w = np.abs(A.data) / np.sqrt(d[rows] * d[cols])
    keep = (rows != cols) & (A.data != 0.0) & (w >= theta * (1.0 - TIE))
    G = sp.csr_matrix((w[keep], (rows[keep], cols[keep])), shape=(n, n))
    G.sort_indices()
    return G


LUBY_SEED_OFFSET = 0x4C554259   # keeps these draws apart from the other SplitMix64 streams


def luby_keys(seed: int, level: int, n: int) -> np.ndarray:
    """Priorities of the parallel independent set of a level: the top 32 bits of the SplitMix64
    stream seeded with seed + LUBY_SEED_OFFSET + level, above the node index (so all differ)."""
    z = splitmix64(seed + LUBY_SEED_OFFSET + level, n)
    return ((z >> np.uint64(32)) << np.uint64(32)) | np.arange(n, dtype=np.uint64)


def greedy_mis(G: sp.csr_matrix, square: bool, order=None) -> np.ndarray:
    """Greedy maximal independent set on G (or on G^2, distance <= 2), visiting the nodes in
    index order, or in the given order.

    Sec. 4 allows the greedy MIS or its parallel form (Luby): in rounds, every free node whose
    priority exceeds that of every free node within reach (distance 1, or 2 on a squared level)
    becomes a root and the free nodes within its reach are taken.  With fixed priorities that
    parallel process ends in the greedy set taken in decreasing priority order, which is how the
    "luby" variant is computed here (order = nodes by decreasing luby_keys)."""
    n = G.shape[0]
    indptr, indices = G.indptr, G.indices
    state = bytearray(n)  # 0 free, 1 root, 2 taken by a root
    for i in (range(n) if order is None else (int(v) for v in order)):
        if state[i]:
            continue
        state[i] = 1
        nb = indices[indptr[i]:indptr[i + 1]]
        if square and nb.size:
            nb = np.concatenate([nb] + [indices[indptr[j]:indptr[j + 1]] for j in nb])
        for j in nb.tolist():
            if state[j] == 0:
                state[j] = 2
    return np.frombuffer(bytes(state), dtype=np.uint8) == 1


def _pick_best(rows, cols, w, n):
    """For each row, the column of largest w; weights within TIE of the max tie, lowest column wins."""
    best = np.full(n, -np.inf)
    np.maximum.at(best, rows, w)
    cand = w >= best[rows] * (1.0 - TIE)
    choice = np.full(n, -1, dtype=np.int64)
    big = np.iinfo(np.int64).max
    tmp = np.full(n, big, dtype=np.int64)
    np.minimum.at(tmp, rows[cand], cols[cand])
    has = tmp != big
    choice[has] = tmp[has]
    return choice


def sa_aggregate(G: sp.csr_matrix, roots: np.ndarray) -> np.ndarray:
    """Aggregate index of every node (coarse index = rank of the root)."""
    n = G.shape[0]
    agg = np.full(n, -1, dtype=np.int64)
    root_ids = np.flatnonzero(roots)
    agg[root_ids] = np.arange(root_ids.size)
    rows = np.repeat(np.arange(n), np.diff(G.indptr))
    cols = G.indices.astype(np.int64)
    w = G.data
    # pass 1: non-roots join the strongly connected root of largest weight
    m = roots[cols] & ~roots[rows]
    choice = _pick_best(rows[m], cols[m], w[m], n)
    sel = (choice >= 0) & ~roots
    agg[sel] = agg[choice[sel]]
    # pass 2: leftovers join the aggregate of their assigned neighbour of largest weight,
    # reading the pass-1 assignment only
    snap = agg.copy()
    left = snap < 0
    m2 = left[rows] & (snap[cols] >= 0)
    choice2 = _pick_best(rows[m2], cols[m2], w[m2], n)
    sel2 = left & (choice2 >= 0)
    agg[sel2] = snap[choice2[sel2]]
    if np.any(agg < 0):
        raise RuntimeError("aggregation left nodes unassigned")
    return agg


def tentative_prolongator(agg: np.ndarray, B: np.ndarray, nc: int):
    """P_t[i, agg_i] = B_i / ||B restricted to the aggregate||; B_c = the aggregate norms."""
    norms = np.sqrt(np.bincount(agg, weights=B * B, minlength=nc))
    n = agg.size
    Pt = sp.csr_matrix((B / norms[agg], agg, np.arange(n + 1)), shape=(n, nc))
    return Pt, norms


def smooth_prolongator(A, Dinv, Pt, lam, nsmooth):
    P = Pt
    omega = 4.0 / (3.0 * lam)
    for _ in range(nsmooth):
        P = (P - sp.diags(omega * Dinv) @ (A @ P)).tocsr()
    P.sort_indices()
    return P


# ---------------------------------------------------------------------------------------------
# Classical coarsening (Sec. 4, eq. (10)) with direct interpolation.
def rs_strength(A: sp.csr_matrix, alpha: float) -> sp.csr_matrix:
    """S[i, j] = 1 iff j != i, a_ij != 0 and |a_ij| >= alpha * max_{k != i} |a_ik| (eq. (10))."""
    n = A.shape[0]
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    cols = A.indices
    off = rows != cols
    mag = np.where(off, np.abs(A.data), 0.0)
    rowmax = np.zeros(n)
    np.maximum.at(rowmax, rows, mag)
    keep = off & (A.data != 0.0) & (mag >= alpha * rowmax[rows] * (1.0 - TIE))
    S = sp.csr_matrix((np.ones(keep.sum()), (rows[keep], cols[keep])), shape=(n, n))
    S.sort_indices()
    return S


def rs_first_pass(S: sp.csr_matrix) -> np.ndarray:
    """Classical C/F splitting (first pass). Returns 1 for C points, 0 for F points."""
    n = S.shape[0]
    ST = S.T.tocsr()
    ST.sort_indices()
    UND, CPT, FPT = 0, 1, 2
    state = np.zeros(n, dtype=np.int8)
    lam = np.diff(ST.indptr).astype(np.int64)     # |S_i^T| = how many points depend on i
    isolated = (np.diff(S.indptr) == 0) & (lam == 0)
    state[isolated] = FPT
    heap = [(-int(lam[i]), i) for i in range(n) if state[i] == UND]
    heapq.heapify(heap)
    while heap:
        negl, i = heapq.heappop(heap)
        if state[i] != UND or -negl != lam[i]:
            continue
        state[i] = CPT
        for j in ST.indices[ST.indptr[i]:ST.indptr[i + 1]]:
            if state[j] == UND:
                state[j] = FPT
                for l in S.indices[S.indptr[j]:S.indptr[j + 1]]:
                    if state[l] == UND:
                        lam[l] += 1
                        heapq.heappush(heap, (-int(lam[l]), int(l)))
        for l in S.indices[S.indptr[i]:S.indptr[i + 1]]:
            if state[l] == UND:
                lam[l] -= 1
                heapq.heappush(heap, (-int(lam[l]), int(l)))
    return (state == CPT).astype(np.int8)


def pmis_random(seed: int, level: int, n: int) -> np.ndarray:
    """The PMIS tie-breaking draws of a level: uniform in [0, 1) from the SplitMix64 stream seeded
    with seed + PMIS_SEED_OFFSET + level (top 53 bits / 2^53)."""
    z = splitmix64(seed + PMIS_SEED_OFFSET + level, n)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


PMIS_SEED_OFFSET = 0x504D4953   # keeps these draws apart from the eigenvalue estimates' (seed + k)


def pmis_split(S: sp.csr_matrix, rand: np.ndarray) -> np.ndarray:
    """Parallel modified independent set (PMIS; De Sterck, Yang & Heys, SIAM J. Matrix Anal.
    Appl. 27 (2006), the independent-set coarsening behind the HMIS of [des06]).

    Measure lam_i = |S_i^T| + rand_i.  Points that influence no other point (|S_i^T| = 0) are F
    points from the start.  Then, in rounds until every point is decided: an undecided point
    whose measure exceeds that of every undecided neighbour in the symmetrised strength graph
    S + S^T (equal measures: the lower index wins) becomes a C point, and the undecided points
    that depend strongly on one of the new C points become F points.  Measures never change.
    Returns 1 for C points, 0 for F points."""
    n = S.shape[0]
    ST = S.T.tocsr()
    influence = np.diff(ST.indptr)
    lam = influence + rand
    N = (abs(S) + abs(ST)).tocsr()
    rows = np.repeat(np.arange(n), np.diff(N.indptr))
    cols = N.indices
    off = rows != cols
    rows, cols = rows[off], cols[off]
    UND, CPT, FPT = 0, 1, 2
    state = np.zeros(n, dtype=np.int8)
    state[influence == 0] = FPT
    while np.any(state == UND):
        und = state == UND
        e = und[rows] & und[cols]
        beats = (lam[cols] > lam[rows]) | ((lam[cols] == lam[rows]) & (cols < rows))
        loses = np.zeros(n, dtype=bool)
        loses[rows[e & beats]] = True
        new_c = und & ~loses
        state[new_c] = CPT
        dep = (S @ new_c.astype(np.float64)) > 0
        state[und & ~new_c & dep] = FPT
    return (state == CPT).astype(np.int8)


def rs_direct_interpolation(A: sp.csr_matrix, S: sp.csr_matrix, cpts: np.ndarray) -> sp.csr_matrix:
    """Direct interpolation (Stueben): for F point i with interpolatory set P_i = C cap S_i,
    w_ij = -alpha_i a_ij / abar_ii (a_ij < 0), -beta_i a_ij / abar_ii (a_ij > 0), where
    alpha_i = sum_{N_i} a^- / sum_{P_i} a^-, beta_i = sum_{N_i} a^+ / sum_{P_i} a^+, and a sign
    class with no member in P_i is lumped into the diagonal abar_ii."""
    n = A.shape[0]
    cidx = np.cumsum(cpts) - 1
    nc = int(cpts.sum())
    prow, pcol, pval = [], [], []
    for i in range(n):
        if cpts[i]:
            prow.append(i); pcol.append(cidx[i]); pval.append(1.0)
            continue
        cols = A.indices[A.indptr[i]:A.indptr[i + 1]]
        vals = A.data[A.indptr[i]:A.indptr[i + 1]]
        strong = set(S.indices[S.indptr[i]:S.indptr[i + 1]].tolist())
        aii = 0.0
        neg_N = pos_N = neg_P = pos_P = 0.0
        interp = []
        for j, a in zip(cols.tolist(), vals.tolist()):
            if j == i:
                aii = a
                continue
            if a < 0:
                neg_N += a
            else:
                pos_N += a
            if j in strong and cpts[j]:
                interp.append((j, a))
                if a < 0:
                    neg_P += a
                else:
                    pos_P += a
        if not interp:
            continue  # no strong C neighbour: empty row
        abar = aii
        if neg_P == 0.0:
            abar += neg_N
        if pos_P == 0.0:
            abar += pos_N
        al = neg_N / neg_P if neg_P != 0.0 else 0.0
        be = pos_N / pos_P if pos_P != 0.0 else 0.0
        for j, a in interp:
            prow.append(i); pcol.append(cidx[j])
            pval.append(-(al if a < 0 else be) * a / abar)
    P = sp.csr_matrix((pval, (prow, pcol)), shape=(n, nc))
    P.sort_indices()
    return P


# ---------------------------------------------------------------------------------------------
def galerkin(A, P):
    R = P.T.tocsr()
    R.sort_indices()
    Ac = (R @ (A @ P)).tocsr()
    Ac = (0.5 * (Ac + Ac.T)).tocsr()
    Ac.sort_indices()
    return R, Ac


def setup(A: sp.csr_matrix, opts: AMGOptions) -> Hierarchy:
    """Alg. 1: build levels until the coarse-equation limit, stagnation, or max_levels."""
    A = A.tocsr()
    B = np.ones(A.shape[0])
    levels: List[Level] = []
    k = 0
    while True:
        lvl = Level(A=A, B=B, Dinv=1.0 / A.diagonal())
        n = A.shape[0]
        if n <= opts.coarse_eq_limit or k == opts.max_levels - 1:
            levels.append(lvl)
            break
        lvl.lam = estimate_lambda_max(A, lvl.Dinv, opts.esteig_iters, opts.seed + k)
        if opts.coarsening == "sa":
            G = sa_strength(A, opts.threshold)
            order = None
            if opts.mis == "luby":
                order = np.argsort(luby_keys(opts.seed, k, n))[::-1]
            roots = greedy_mis(G, square=k < opts.square_graph_levels, order=order)
            agg = sa_aggregate(G, roots)
            nc = int(roots.sum())
            Pt, Bc = tentative_prolongator(agg, B, nc)
            P = smooth_prolongator(A, lvl.Dinv, Pt, lvl.lam, opts.prolong_smooths)
            lvl.agg = agg
        elif opts.coarsening in ("rs", "pmis"):
            S = rs_strength(A, opts.threshold)
            if opts.coarsening == "rs":
                cpts = rs_first_pass(S)
            else:
                cpts = pmis_split(S, pmis_random(opts.seed, k, n))
            P = rs_direct_interpolation(A, S, cpts)
            nc = P.shape[1]
            Bc = np.ones(nc)
            lvl.cpts = cpts
        else:
            raise ValueError(opts.coarsening)
        if nc > opts.stagnation_ratio * n or nc == 0:
            lvl.agg = lvl.cpts = None        # keep lam: the level may be relaxed as coarsest
            levels.append(lvl)
            break
        R, Ac = galerkin(A, P)
        lvl.P, lvl.R = P, R
        levels.append(lvl)
        A, B = Ac, Bc
        k += 1
    h = Hierarchy(levels=levels, opts=opts)
    _setup_coarse(h)
    return h


def _setup_coarse(h: Hierarchy):
    """Coarsest level: Cholesky of A_M (SPD), or of A_M + abar bbar bbar^T with bbar = B_M / ||B_M||
    and abar = mean(diag A_M) when A_M carries the constant kernel (Alg. 2, direct solve)."""
    L = h.levels[-1]
    if L.A.shape[0] > h.opts.coarse_dense_max:
        if not np.isfinite(L.lam):
            L.lam = estimate_lambda_max(L.A, L.Dinv, h.opts.esteig_iters, h.opts.seed + len(h.levels) - 1)
        h.coarse_factor = None            # relaxed by the smoother (see module notes)
        return
    Ad = L.A.toarray()
    if h.opts.nullspace and Ad.shape[0] == 1:
        # b-perp is {0}: the pseudo-inverse on it is zero
        h.coarse_bbar = np.ones(1)
        h.coarse_factor = "zero"
        return
    if h.opts.nullspace:
        bbar = L.B / np.linalg.norm(L.B)
        abar = float(np.mean(np.diag(Ad)))
        K = Ad + abar * np.outer(bbar, bbar)
        h.coarse_bbar = bbar
    else:
        K = Ad
    h.coarse_factor = sla.cho_factor(K, lower=True)


def complexity(h: Hierarchy):
    nnz = [lv.A.nnz for lv in h.levels]
    ns = [lv.A.shape[0] for lv in h.levels]
    return dict(n=ns, nnz=nnz, operator_complexity=sum(nnz) / nnz[0], grid_complexity=sum(ns) / ns[0])
