// AMG setup phase on the host (Alg. 1 of the paper; Sec. 4 and App. A for the components).
//
// Smoothed aggregation: strength graph from w_ij = |a_ij| / sqrt(a_ii a_jj) >= theta, maximal
// independent set taken greedily in decreasing random priority (the set the parallel Luby-type
// rounds reach; option independent_set) or in index order, on the squared graph for the first
// `square_graph_levels` levels,
// clusters formed around the MIS roots by largest weight, tentative prolongator normalised
// per cluster (|C_j|^{-1/2} for the constant near-null vector), one Jacobi smoothing of the
// prolongator, Galerkin coarse operator R A P with R = P^T.  Classical coarsening: strong
// set of eq. (10), first-pass C/F splitting, direct interpolation.  The coarsest level gets
// a dense inverse (pseudo-inverse on the complement of the constant when the operator is
// singular).  Tie and threshold rules are spelled out where they are applied; they make the
// hierarchy independent of the rounding of the matrix entries.
#include <algorithm>
#include <functional>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <queue>
#include <string>
#include <vector>

#include <omp.h>

#include "bd_host.hpp"

namespace bd {

namespace {
constexpr double kTie = 1e-12;  // relative width of a tie / threshold band
}

// ------------------------------------------------------------------------------------------
Csr transpose(const Csr& A) {
  // Threads take consecutive row blocks of A (balanced by entries) and scatter them in order
  // through per-thread column offsets, so every output row is sorted, as in a serial pass.
  Csr T;
  T.nrows = A.ncols;
  T.ncols = A.nrows;
  T.rp.assign((size_t)T.nrows + 1, 0);
  T.ci.resize(A.ci.size());
  T.v.resize(A.v.size());
  const int64_t nnz = (int64_t)A.ci.size();
  int nt = std::max(1, std::min(omp_get_max_threads(), (int)(nnz >> 16) + 1));
  while (nt > 1 && (int64_t)nt * T.nrows > (int64_t(1) << 28)) --nt;  // counts stay within 1 GiB
  std::vector<int32_t> r0(nt + 1, A.nrows);
  for (int t = 0; t < nt; ++t)
    r0[t] = (int32_t)(std::lower_bound(A.rp.begin(), A.rp.end(), (int32_t)(nnz * t / nt)) - A.rp.begin());
  r0[0] = 0;
  std::vector<int32_t> off((size_t)nt * T.nrows, 0);  // counts, then each thread's next slot
#pragma omp parallel num_threads(nt)
  {
    const int t = omp_get_thread_num();
    int32_t* c = off.data() + (size_t)t * T.nrows;
    for (int32_t k = A.rp[r0[t]]; k < A.rp[r0[t + 1]]; ++k) c[A.ci[k]]++;
#pragma omp barrier
#pragma omp for schedule(static)
    for (int32_t col = 0; col < T.nrows; ++col) {
      int32_t sum = 0;
      for (int u = 0; u < nt; ++u) {
        const int32_t n_u = off[(size_t)u * T.nrows + col];
        off[(size_t)u * T.nrows + col] = sum;
        sum += n_u;
      }
      T.rp[col + 1] = sum;
    }
#pragma omp single
    for (int32_t col = 0; col < T.nrows; ++col) T.rp[col + 1] += T.rp[col];
    for (int32_t i = r0[t]; i < r0[t + 1]; ++i)
      for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
        const int32_t col = A.ci[k];
        const int32_t pos = T.rp[col] + c[col]++;
        T.ci[pos] = i;
        T.v[pos] = A.v[k];
      }
  }
  return T;
}

// C = A B with products accumulated in the order of A's row, then B's rows, into a dense
// accumulator with a row-stamped marker.  Sparse products (a few partial products per entry
// of A) take a symbolic pass for the row sizes and write C in place.  Dense ones (the coarse
// levels of smoothed aggregation, where rows of A P fill most of the coarse columns) take one
// numeric pass into per-thread buffers, since a symbolic pass would repeat the whole product;
// their rows accumulate without a branch and are emitted by a scan of the marker.
namespace {
Csr spgemm_sparse(const Csr& A, const Csr& B) {
  Csr C;
  C.nrows = A.nrows;
  C.ncols = B.ncols;
  C.rp.assign((size_t)C.nrows + 1, 0);
#pragma omp parallel
  {
    std::vector<int32_t> mk(B.ncols, -1);
#pragma omp for schedule(dynamic, 16)
    for (int32_t i = 0; i < A.nrows; ++i) {
      int32_t cnt = 0;
      for (int32_t ka = A.rp[i]; ka < A.rp[i + 1]; ++ka) {
        const int32_t k = A.ci[ka];
        for (int32_t kb = B.rp[k]; kb < B.rp[k + 1]; ++kb)
          if (mk[B.ci[kb]] != i) {
            mk[B.ci[kb]] = i;
            ++cnt;
          }
      }
      C.rp[i + 1] = cnt;
    }
  }
  for (int32_t i = 0; i < C.nrows; ++i) C.rp[i + 1] += C.rp[i];
  C.ci.resize(C.rp[C.nrows]);
  C.v.resize(C.rp[C.nrows]);
#pragma omp parallel
  {
    std::vector<int32_t> mk(B.ncols, -1);
    std::vector<double> acc(B.ncols, 0.0);
    std::vector<int32_t> cols;
#pragma omp for schedule(dynamic, 16)
    for (int32_t i = 0; i < A.nrows; ++i) {
      cols.clear();
      for (int32_t ka = A.rp[i]; ka < A.rp[i + 1]; ++ka) {
        const int32_t k = A.ci[ka];
        const double a = A.v[ka];
        for (int32_t kb = B.rp[k]; kb < B.rp[k + 1]; ++kb) {
          const int32_t j = B.ci[kb];
          if (mk[j] != i) {
            mk[j] = i;
            acc[j] = a * B.v[kb];
            cols.push_back(j);
          } else {
            acc[j] += a * B.v[kb];
          }
        }
      }
      std::sort(cols.begin(), cols.end());
      int32_t pos = C.rp[i];
      for (int32_t j : cols) {
        C.ci[pos] = j;
        C.v[pos] = acc[j];
        ++pos;
      }
    }
  }
  return C;
}

Csr spgemm_dense(const Csr& A, const Csr& B) {
  Csr C;
  C.nrows = A.nrows;
  C.ncols = B.ncols;
  C.rp.assign((size_t)C.nrows + 1, 0);
  const int nt = omp_get_max_threads();
  std::vector<std::vector<int32_t>> bci(nt);
  std::vector<std::vector<double>> bv(nt);
  std::vector<int64_t> row_off(C.nrows);  // row start in its thread's buffer
  std::vector<int32_t> row_thr(C.nrows);
#pragma omp parallel
  {
    const int tid = omp_get_thread_num();
    std::vector<int32_t> mk(B.ncols, -1);
    std::vector<double> acc(B.ncols, 0.0);  // zero outside the row being accumulated
    std::vector<int32_t>& oc = bci[tid];
    std::vector<double>& ov = bv[tid];
#pragma omp for schedule(dynamic, 4)
    for (int32_t i = 0; i < A.nrows; ++i) {
      for (int32_t ka = A.rp[i]; ka < A.rp[i + 1]; ++ka) {
        const int32_t k = A.ci[ka];
        const double a = A.v[ka];
        for (int32_t kb = B.rp[k]; kb < B.rp[k + 1]; ++kb) {
          const int32_t j = B.ci[kb];
          acc[j] += a * B.v[kb];
          mk[j] = i;
        }
      }
      row_off[i] = (int64_t)oc.size();
      row_thr[i] = tid;
      for (int32_t j = 0; j < B.ncols; ++j)
        if (mk[j] == i) {
          oc.push_back(j);
          ov.push_back(acc[j]);
          acc[j] = 0.0;
        }
      C.rp[i + 1] = (int32_t)((int64_t)oc.size() - row_off[i]);
    }
  }
  for (int32_t i = 0; i < C.nrows; ++i) C.rp[i + 1] += C.rp[i];
  C.ci.resize(C.rp[C.nrows]);
  C.v.resize(C.rp[C.nrows]);
#pragma omp parallel for schedule(static, 256)
  for (int32_t i = 0; i < C.nrows; ++i) {
    const int64_t len = C.rp[i + 1] - C.rp[i];
    std::copy_n(bci[row_thr[i]].data() + row_off[i], len, C.ci.data() + C.rp[i]);
    std::copy_n(bv[row_thr[i]].data() + row_off[i], len, C.v.data() + C.rp[i]);
  }
  return C;
}
}  // namespace

Csr spgemm(const Csr& A, const Csr& B) {
  // partial products per row, on average, against the output width
  int64_t flops = 0;
#pragma omp parallel for reduction(+ : flops) schedule(static, 4096)
  for (int32_t i = 0; i < A.nrows; ++i)
    for (int32_t ka = A.rp[i]; ka < A.rp[i + 1]; ++ka) flops += B.rp[A.ci[ka] + 1] - B.rp[A.ci[ka]];
  const bool dense = A.nrows > 0 && (double)flops / A.nrows > 0.25 * (double)B.ncols;
  return dense ? spgemm_dense(A, B) : spgemm_sparse(A, B);
}

std::vector<double> diagonal(const Csr& A) {
  std::vector<double> d(A.nrows, 0.0);
#pragma omp parallel for schedule(static, 4096)
  for (int32_t i = 0; i < A.nrows; ++i)
    for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
      if (A.ci[k] == i) d[i] = A.v[k];
  return d;
}

std::string validate(const Csr& A) {
  if (A.nrows <= 0 || A.nrows != A.ncols) return "matrix must be square with n > 0";
  if ((int64_t)A.rp.size() != (int64_t)A.nrows + 1 || A.rp[0] != 0) return "row_ptr must start at 0";
  for (int32_t i = 0; i < A.nrows; ++i)
    if (A.rp[i + 1] < A.rp[i]) return "row_ptr must be non-decreasing";
  if ((int64_t)A.rp[A.nrows] != A.nnz()) return "row_ptr[n] must equal nnz";
  // rows checked in parallel; the message names the first bad row and its first problem
  enum : uint8_t { OK = 0, RANGE, ORDER, NONFINITE, DIAG_SIGN, NO_DIAG };
  std::vector<uint8_t> bad(A.nrows, OK);
#pragma omp parallel for schedule(static, 4096)
  for (int32_t i = 0; i < A.nrows; ++i) {
    bool diag = false;
    uint8_t b = OK;
    for (int32_t k = A.rp[i]; k < A.rp[i + 1] && b == OK; ++k) {
      if (A.ci[k] < 0 || A.ci[k] >= A.ncols) b = RANGE;
      else if (k > A.rp[i] && A.ci[k] <= A.ci[k - 1]) b = ORDER;
      else if (!std::isfinite(A.v[k])) b = NONFINITE;
      else if (A.ci[k] == i) {
        diag = true;
        if (!(A.v[k] > 0.0)) b = DIAG_SIGN;
      }
    }
    bad[i] = b != OK ? b : (diag ? OK : NO_DIAG);
  }
  for (int32_t i = 0; i < A.nrows; ++i) {
    if (bad[i] == OK) continue;
    const std::string row = std::to_string(i);
    switch (bad[i]) {
      case RANGE: return "column index out of range in row " + row;
      case ORDER: return "columns must be sorted and unique in row " + row;
      case NONFINITE: return "non-finite value in row " + row;
      case DIAG_SIGN: return "diagonal must be positive in row " + row;
      default: return "missing diagonal in row " + row;
    }
  }
  return "";
}

// ------------------------------------------------------------------------------------------
// Eigenvalue estimate for the Chebyshev interval and the prolongator damping.
namespace {

uint64_t splitmix64_at(uint64_t seed, uint64_t i) {
  // output i (0-based) of SplitMix64 seeded with `seed`: the state advances by the golden
  // gamma before each output, then the published finaliser is applied
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// Priority of node i in the parallel independent set of level k: the top 32 bits of the level's
// SplitMix64 draw above the node index (all distinct).
uint64_t luby_key(uint64_t seed, int level, int32_t i) {
  return ((splitmix64_at(seed + kLubySeedOffset + (uint64_t)level, (uint64_t)i) >> 32) << 32) | (uint64_t)(uint32_t)i;
}

// Largest eigenvalue of the symmetric tridiagonal (diag a, off-diagonal b) by bisection on
// the Sturm sequence count.
double tridiag_max_eig(const std::vector<double>& a, const std::vector<double>& b) {
  const int m = (int)a.size();
  double lo = a[0], hi = a[0];
  for (int i = 0; i < m; ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  auto count_below = [&](double x) {  // number of eigenvalues < x
    int cnt = 0;
    double q = a[0] - x;
    if (q < 0) ++cnt;
    for (int i = 1; i < m; ++i) {
      if (q == 0.0) q = 1e-300;
      q = (a[i] - x) - b[i - 1] * b[i - 1] / q;
      if (q < 0) ++cnt;
    }
    return cnt;
  };
  for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(std::fabs(lo), std::fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (count_below(mid) == m) hi = mid; else lo = mid;
  }
  return 0.5 * (lo + hi);
}

}  // namespace

namespace {
// Dot product in a fixed order independent of the thread count: 4096-entry blocks summed in
// parallel, then the block sums in index order.
double fixed_dot(const std::vector<double>& a, const std::vector<double>& b) {
  const int64_t n = (int64_t)a.size(), nb = (n + kDotBlock - 1) / kDotBlock;
  std::vector<double> part(nb, 0.0);
#pragma omp parallel for schedule(static)
  for (int64_t blk = 0; blk < nb; ++blk) {
    double s = 0.0;
    for (int64_t i = blk * kDotBlock; i < std::min(n, (blk + 1) * kDotBlock); ++i) s += a[i] * b[i];
    part[blk] = s;
  }
  double s = 0.0;
  for (double v : part) s += v;
  return s;
}
}  // namespace

double lambda_estimate(const Csr& A, const std::vector<double>& Dinv, int iters, uint64_t seed) {
  const int32_t n = A.nrows;
  std::vector<double> r(n), z(n), p(n), q(n);
#pragma omp parallel for schedule(static)
  for (int32_t i = 0; i < n; ++i) {
    r[i] = 2.0 * ((double)(splitmix64_at(seed, (uint64_t)i) >> 11) * 0x1.0p-53) - 1.0;
    z[i] = Dinv[i] * r[i];
    p[i] = z[i];
  }
  double rho = fixed_dot(r, z);
  const double rho0 = rho;
  std::vector<double> alpha, beta;
  for (int j = 0; j < iters; ++j) {
#pragma omp parallel for schedule(dynamic, 256)
    for (int32_t i = 0; i < n; ++i) {
      double s = 0.0;
      for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) s += A.v[k] * p[A.ci[k]];
      q[i] = s;
    }
    const double pq = fixed_dot(p, q);
    if (!(pq > 0.0)) break;
    const double al = rho / pq;
    alpha.push_back(al);
    if (j == iters - 1) break;
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) {
      r[i] -= al * q[i];
      z[i] = Dinv[i] * r[i];
    }
    const double rn = fixed_dot(r, z);
    if (!(rn > 1e-28 * rho0)) break;
    const double be = rn / rho;
    beta.push_back(be);
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) p[i] = z[i] + be * p[i];
    rho = rn;
  }
  return ritz_from_cg(A, Dinv, alpha, beta);
}

double ritz_from_cg(const Csr& A, const std::vector<double>& Dinv, const std::vector<double>& alpha,
                    const std::vector<double>& beta) {
  const int32_t n = A.nrows;
  const int m = (int)alpha.size();
  if (m == 0) {
    double mx = 0.0;
    for (int32_t i = 0; i < n; ++i)
      for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
        if (A.ci[k] == i) mx = std::max(mx, Dinv[i] * A.v[k]);
    return mx;
  }
  // CG/Lanczos relation: T_jj = 1/alpha_j + beta_{j-1}/alpha_{j-1}, T_{j,j+1} = sqrt(beta_j)/alpha_j
  std::vector<double> td(m), to(std::max(m - 1, 0));
  for (int j = 0; j < m; ++j) {
    td[j] = 1.0 / alpha[j] + (j > 0 ? beta[j - 1] / alpha[j - 1] : 0.0);
    if (j + 1 < m) to[j] = std::sqrt(beta[j]) / alpha[j];
  }
  return tridiag_max_eig(td, to);
}

// ------------------------------------------------------------------------------------------
// Smoothed aggregation.
namespace {

struct Graph {
  std::vector<int32_t> rp, ci;
  std::vector<double> w;
};

Graph sa_strength(const Csr& A, const std::vector<double>& d, double theta) {
  Graph G;
  const int32_t n = A.nrows;
  G.rp.assign(n + 1, 0);
  const double cut = theta * (1.0 - kTie);
  auto strong = [&](int32_t i, int32_t k, double& w) {
    const int32_t j = A.ci[k];
    if (j == i || A.v[k] == 0.0) return false;
    w = std::fabs(A.v[k]) / std::sqrt(d[i] * d[j]);
    return w >= cut;
  };
#pragma omp parallel for schedule(static, 4096)
  for (int32_t i = 0; i < n; ++i) {
    int32_t c = 0;
    double w;
    for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) c += strong(i, k, w);
    G.rp[i + 1] = c;
  }
  for (int32_t i = 0; i < n; ++i) G.rp[i + 1] += G.rp[i];
  G.ci.resize(G.rp[n]);
  G.w.resize(G.rp[n]);
#pragma omp parallel for schedule(static, 4096)
  for (int32_t i = 0; i < n; ++i) {
    int32_t pos = G.rp[i];
    double w;
    for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
      if (strong(i, k, w)) {
        G.ci[pos] = A.ci[k];
        G.w[pos] = w;
        ++pos;
      }
  }
  return G;
}

// Greedy MIS in index order, or in the order `order` (a permutation); with `square`, a new root
// also takes its distance-2 nodes.
std::vector<uint8_t> greedy_mis(const Graph& G, int32_t n, bool square, const std::vector<int32_t>* order = nullptr) {
  std::vector<uint8_t> st(n, 0);  // 0 free, 1 root, 2 taken
  for (int32_t q = 0; q < n; ++q) {
    const int32_t i = order ? (*order)[q] : q;
    if (st[i]) continue;
    st[i] = 1;
    for (int32_t k = G.rp[i]; k < G.rp[i + 1]; ++k) {
      const int32_t j = G.ci[k];
      if (st[j] == 0) st[j] = 2;
      if (square)
        for (int32_t l = G.rp[j]; l < G.rp[j + 1]; ++l)
          if (st[G.ci[l]] == 0) st[G.ci[l]] = 2;
    }
  }
  return st;
}

// Among the neighbours j of i accepted by `ok`, the one of largest weight; weights within the
// tie band of the largest are equal and the lowest index wins.  -1 if none.
template <class Ok>
int32_t best_neighbour(const Graph& G, int32_t i, Ok ok) {
  double best = -1.0;
  for (int32_t k = G.rp[i]; k < G.rp[i + 1]; ++k)
    if (ok(G.ci[k]) && G.w[k] > best) best = G.w[k];
  if (best < 0.0) return -1;
  int32_t pick = -1;
  for (int32_t k = G.rp[i]; k < G.rp[i + 1]; ++k) {
    const int32_t j = G.ci[k];
    if (ok(j) && G.w[k] >= best * (1.0 - kTie) && (pick < 0 || j < pick)) pick = j;
  }
  return pick;
}

// Returns the number of aggregates; agg[i] = aggregate of node i (rank of its root).
int32_t sa_aggregate(const Graph& G, const std::vector<uint8_t>& st, std::vector<int32_t>& agg) {
  const int32_t n = (int32_t)st.size();
  agg.assign(n, -1);
  int32_t nc = 0;
  for (int32_t i = 0; i < n; ++i)
    if (st[i] == 1) agg[i] = nc++;
  for (int32_t i = 0; i < n; ++i) {  // pass 1: strongly connected root of largest weight
    if (st[i] == 1) continue;
    const int32_t j = best_neighbour(G, i, [&](int32_t c) { return st[c] == 1; });
    if (j >= 0) agg[i] = agg[j];
  }
  const std::vector<int32_t> snap(agg);
  for (int32_t i = 0; i < n; ++i) {  // pass 2: assigned neighbour of largest weight (snapshot)
    if (snap[i] >= 0) continue;
    const int32_t j = best_neighbour(G, i, [&](int32_t c) { return snap[c] >= 0; });
    if (j >= 0) agg[i] = snap[j];
  }
  for (int32_t i = 0; i < n; ++i)
    if (agg[i] < 0) return -1;
  return nc;
}

Csr sa_prolongator(const Csr& A, const std::vector<double>& Dinv, const std::vector<double>& B,
                   const std::vector<int32_t>& agg, int32_t nc, double lam, int nsmooth,
                   std::vector<double>& Bc) {
  const int32_t n = A.nrows;
  Csr P = tentative_prolongator(B, agg, nc, Bc);
  const double omega = prolongator_damping(lam);
  for (int s = 0; s < nsmooth; ++s) {
    Csr AP = spgemm(A, P);  // pattern(AP) contains pattern(P): every diagonal a_ii is stored
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) {
      const double sc = omega * Dinv[i];
      int32_t kp = P.rp[i];
      for (int32_t k = AP.rp[i]; k < AP.rp[i + 1]; ++k) {
        double pij = 0.0;
        while (kp < P.rp[i + 1] && P.ci[kp] < AP.ci[k]) ++kp;
        if (kp < P.rp[i + 1] && P.ci[kp] == AP.ci[k]) pij = P.v[kp];
        AP.v[k] = pij - sc * AP.v[k];
      }
    }
    P = std::move(AP);
  }
  return P;
}

// ------------------------------------------------------------------------------------------
// Classical coarsening.
constexpr uint64_t kPmisSeedOffset = 0x504D4953;  // PMIS draws: seed + offset + level
Csr rs_strength(const Csr& A, double alpha) {
  Csr S;
  const int32_t n = A.nrows;
  S.nrows = S.ncols = n;
  S.rp.assign(n + 1, 0);
  std::vector<double> cut(n);
#pragma omp parallel for schedule(static, 4096)
  for (int32_t i = 0; i < n; ++i) {
    double mx = 0.0;
    for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
      if (A.ci[k] != i) mx = std::max(mx, std::fabs(A.v[k]));
    cut[i] = alpha * mx * (1.0 - kTie);
    int32_t c = 0;
    for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
      c += A.ci[k] != i && A.v[k] != 0.0 && std::fabs(A.v[k]) >= cut[i];
    S.rp[i + 1] = c;
  }
  for (int32_t i = 0; i < n; ++i) S.rp[i + 1] += S.rp[i];
  S.ci.resize(S.rp[n]);
  S.v.assign(S.rp[n], 1.0);
#pragma omp parallel for schedule(static, 4096)
  for (int32_t i = 0; i < n; ++i) {
    int32_t pos = S.rp[i];
    for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
      if (A.ci[k] != i && A.v[k] != 0.0 && std::fabs(A.v[k]) >= cut[i]) S.ci[pos++] = A.ci[k];
  }
  return S;
}

// First pass: repeatedly make the undecided point of largest measure (lowest index on ties)
// a C point; the undecided points depending on it become F points, and measures are updated.
std::vector<uint8_t> rs_split(const Csr& S) {
  const int32_t n = S.nrows;
  const Csr ST = transpose(S);
  enum : uint8_t { UND = 0, CP = 1, FP = 2 };
  std::vector<uint8_t> st(n, UND);
  std::vector<int32_t> lam(n);
  for (int32_t i = 0; i < n; ++i) {
    lam[i] = ST.rp[i + 1] - ST.rp[i];
    if (lam[i] == 0 && S.rp[i + 1] == S.rp[i]) st[i] = FP;  // no strong connection at all
  }
  std::priority_queue<std::pair<int32_t, int32_t>> pq;  // (measure, -index)
  for (int32_t i = 0; i < n; ++i)
    if (st[i] == UND) pq.push({lam[i], -i});
  while (!pq.empty()) {
    const auto top = pq.top();
    pq.pop();
    const int32_t i = -top.second;
    if (st[i] != UND || top.first != lam[i]) continue;
    st[i] = CP;
    for (int32_t k = ST.rp[i]; k < ST.rp[i + 1]; ++k) {
      const int32_t j = ST.ci[k];
      if (st[j] != UND) continue;
      st[j] = FP;
      for (int32_t l = S.rp[j]; l < S.rp[j + 1]; ++l) {
        const int32_t m = S.ci[l];
        if (st[m] == UND) pq.push({++lam[m], -m});
      }
    }
    for (int32_t l = S.rp[i]; l < S.rp[i + 1]; ++l) {
      const int32_t m = S.ci[l];
      if (st[m] == UND) pq.push({--lam[m], -m});
    }
  }
  return st;
}

// PMIS split (De Sterck, Yang & Heys 2006, the independent-set coarsening of the HMIS the paper
// cites): measure lam_i = |S_i^T| + r_i with r_i uniform in [0, 1) from SplitMix64; points that
// influence no other point are F points; then in rounds, every undecided point whose measure
// beats all undecided neighbours in S + S^T (equal measures: lower index wins) becomes C, and the
// undecided points depending strongly on a new C point become F.  Each round reads the previous
// round's states only, so its loops run in parallel and the result does not depend on order.
std::vector<uint8_t> pmis_split(const Csr& S, uint64_t seed) {
  const int32_t n = S.nrows;
  const Csr ST = transpose(S);
  enum : uint8_t { UND = 0, CP = 1, FP = 2 };
  std::vector<double> lam(n);
  std::vector<uint8_t> st(n, UND), newc(n, 0);
#pragma omp parallel for schedule(static, 4096)
  for (int32_t i = 0; i < n; ++i) {
    const int32_t infl = ST.rp[i + 1] - ST.rp[i];
    lam[i] = (double)infl + (double)(splitmix64_at(seed, (uint64_t)i) >> 11) * 0x1.0p-53;
    if (infl == 0) st[i] = FP;
  }
  auto beats = [&](int32_t j, int32_t i) { return lam[j] > lam[i] || (lam[j] == lam[i] && j < i); };
  for (;;) {
    int64_t undecided = 0;
#pragma omp parallel for schedule(static, 4096) reduction(+ : undecided)
    for (int32_t i = 0; i < n; ++i) {
      newc[i] = 0;
      if (st[i] != UND) continue;
      ++undecided;
      bool best = true;
      for (int32_t k = S.rp[i]; k < S.rp[i + 1] && best; ++k) {
        const int32_t j = S.ci[k];
        if (j != i && st[j] == UND && beats(j, i)) best = false;
      }
      for (int32_t k = ST.rp[i]; k < ST.rp[i + 1] && best; ++k) {
        const int32_t j = ST.ci[k];
        if (j != i && st[j] == UND && beats(j, i)) best = false;
      }
      newc[i] = best;
    }
    if (undecided == 0) break;
#pragma omp parallel for schedule(static, 4096)
    for (int32_t i = 0; i < n; ++i) {
      if (st[i] != UND || newc[i]) continue;
      for (int32_t k = S.rp[i]; k < S.rp[i + 1]; ++k)
        if (newc[S.ci[k]]) {
          st[i] = FP;
          break;
        }
    }
#pragma omp parallel for schedule(static, 4096)
    for (int32_t i = 0; i < n; ++i)
      if (newc[i]) st[i] = CP;
  }
  return st;
}

// Direct interpolation: an F point interpolates from its strong C neighbours, scaling the
// negative and positive couplings separately so that row sums are preserved; a sign class
// with no interpolatory member is added to the diagonal.
Csr rs_interpolation(const Csr& A, const Csr& S, const std::vector<uint8_t>& st) {
  const int32_t n = A.nrows;
  std::vector<int32_t> cidx(n, -1);
  int32_t nc = 0;
  for (int32_t i = 0; i < n; ++i)
    if (st[i] == 1) cidx[i] = nc++;
  Csr P;
  P.nrows = n;
  P.ncols = nc;
  P.rp.assign(n + 1, 0);
  std::vector<uint8_t> strong(n, 0);
  for (int32_t i = 0; i < n; ++i) {
    if (st[i] == 1) {
      P.ci.push_back(cidx[i]);
      P.v.push_back(1.0);
      P.rp[i + 1] = (int32_t)P.ci.size();
      continue;
    }
    for (int32_t l = S.rp[i]; l < S.rp[i + 1]; ++l) strong[S.ci[l]] = 1;
    double aii = 0.0, negN = 0.0, posN = 0.0, negP = 0.0, posP = 0.0;
    bool any = false;
    for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      const int32_t j = A.ci[k];
      const double a = A.v[k];
      if (j == i) { aii = a; continue; }
      if (a < 0) negN += a; else posN += a;
      if (strong[j] && st[j] == 1) {
        any = true;
        if (a < 0) negP += a; else posP += a;
      }
    }
    if (any) {
      double abar = aii;
      if (negP == 0.0) abar += negN;
      if (posP == 0.0) abar += posN;
      const double al = negP != 0.0 ? negN / negP : 0.0;
      const double be = posP != 0.0 ? posN / posP : 0.0;
      for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
        const int32_t j = A.ci[k];
        if (j == i || !strong[j] || st[j] != 1) continue;
        const double a = A.v[k];
        P.ci.push_back(cidx[j]);
        P.v.push_back(-(a < 0 ? al : be) * a / abar);
      }
    }
    for (int32_t l = S.rp[i]; l < S.rp[i + 1]; ++l) strong[S.ci[l]] = 0;
    P.rp[i + 1] = (int32_t)P.ci.size();
  }
  return P;  // columns ascend with the fine index, so rows are sorted
}

// ------------------------------------------------------------------------------------------
// (A + A^T) / 2.  The Galerkin product R A P with R = P^T has a symmetric pattern (A's is), so
// every entry's mirror is found by a binary search in the mirror row; rows are independent.
Csr symmetrize(const Csr& A) {
  Csr C = A;
  {  // a structurally symmetric matrix (the Galerkin products): a_ji from the transpose
    const Csr T = transpose(A);
    if (T.rp == A.rp && T.ci == A.ci) {
#pragma omp parallel for schedule(static, 4096)
      for (int64_t k = 0; k < (int64_t)A.v.size(); ++k) C.v[k] = 0.5 * (A.v[k] + T.v[k]);
      return C;
    }
  }
#pragma omp parallel for schedule(dynamic, 64)
  for (int32_t i = 0; i < A.nrows; ++i)
    for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) {
      const int32_t j = A.ci[k];
      const int32_t* lo = A.ci.data() + A.rp[j];
      const int32_t* hi = A.ci.data() + A.rp[j + 1];
      const int32_t* m = std::lower_bound(lo, hi, i);
      const double aji = (m != hi && *m == i) ? A.v[m - A.ci.data()] : 0.0;
      C.v[k] = 0.5 * (A.v[k] + aji);
    }
  return C;
}

bool cholesky(std::vector<double>& K, int n) {  // in place, lower triangle, row-major
  for (int j = 0; j < n; ++j) {
    double s = K[(size_t)j * n + j];
    for (int k = 0; k < j; ++k) s -= K[(size_t)j * n + k] * K[(size_t)j * n + k];
    if (!(s > 0.0)) return false;
    const double d = std::sqrt(s);
    K[(size_t)j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double t = K[(size_t)i * n + j];
      for (int k = 0; k < j; ++k) t -= K[(size_t)i * n + k] * K[(size_t)j * n + k];
      K[(size_t)i * n + j] = t / d;
    }
  }
  return true;
}

// Inverse of an SPD matrix from its Cholesky factor L: solve L L^T X = I column by column.
std::vector<double> spd_inverse(const std::vector<double>& L, int n) {
  std::vector<double> X((size_t)n * n, 0.0);
#pragma omp parallel for schedule(dynamic, 4)
  for (int c = 0; c < n; ++c) {
    std::vector<double> y(n, 0.0);
    for (int i = 0; i < n; ++i) {
      double t = (i == c) ? 1.0 : 0.0;
      for (int k = 0; k < i; ++k) t -= L[(size_t)i * n + k] * y[k];
      y[i] = t / L[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double t = y[i];
      for (int k = i + 1; k < n; ++k) t -= L[(size_t)k * n + i] * y[k];
      y[i] = t / L[(size_t)i * n + i];
    }
    for (int i = 0; i < n; ++i) X[(size_t)i * n + c] = y[i];
  }
  return X;
}

// Coarsest-level operator G: A_M^{-1}; for the singular operator, the pseudo-inverse on the
// complement of bbar = B_M / ||B_M||, obtained as Pi K^{-1} Pi with K = A_M + abar bbar bbar^T
// and abar = mean(diag A_M), Pi = I - bbar bbar^T.
int coarse_operator(const HostLevel& L, bool nullspace, std::vector<double>& G, std::string& err) {
  const int n = L.A.nrows;
  G.assign((size_t)n * n, 0.0);
  if (nullspace && n == 1) return BD_OK;  // b-perp = {0}: zero correction
  std::vector<double> K((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int32_t k = L.A.rp[i]; k < L.A.rp[i + 1]; ++k) K[(size_t)i * n + L.A.ci[k]] = L.A.v[k];
  std::vector<double> bb;
  if (nullspace) {
    double nb = 0.0, md = 0.0;
    for (int i = 0; i < n; ++i) { nb += L.B[i] * L.B[i]; md += K[(size_t)i * n + i]; }
    nb = std::sqrt(nb);
    md /= n;
    bb.resize(n);
    for (int i = 0; i < n; ++i) bb[i] = L.B[i] / nb;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) K[(size_t)i * n + j] += md * bb[i] * bb[j];
  }
  if (!cholesky(K, n)) {
    err = "coarsest-level operator is not positive definite";
    return BD_E_INVALID;
  }
  G = spd_inverse(K, n);
  if (nullspace) {
    std::vector<double> u(n, 0.0);  // u = K^{-1} bbar
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) u[i] += G[(size_t)i * n + j] * bb[j];
    double c = 0.0;
    for (int i = 0; i < n; ++i) c += bb[i] * u[i];
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j)
        G[(size_t)i * n + j] += -u[i] * bb[j] - bb[i] * u[j] + c * bb[i] * bb[j];
  }
  return BD_OK;
}

}  // namespace

Csr symmetrized(const Csr& A) { return symmetrize(A); }

Csr tentative_prolongator(const std::vector<double>& B, const std::vector<int32_t>& agg, int32_t nc,
                          std::vector<double>& Bc) {
  const int32_t n = (int32_t)agg.size();
  std::vector<double> norm2(nc, 0.0);
  for (int32_t i = 0; i < n; ++i) norm2[agg[i]] += B[i] * B[i];
  Bc.resize(nc);
  for (int32_t c = 0; c < nc; ++c) Bc[c] = std::sqrt(norm2[c]);
  Csr P;
  P.nrows = n;
  P.ncols = nc;
  P.rp.resize(n + 1);
  P.ci.resize(n);
  P.v.resize(n);
  for (int32_t i = 0; i <= n; ++i) P.rp[i] = i;
  for (int32_t i = 0; i < n; ++i) {
    P.ci[i] = agg[i];
    P.v[i] = B[i] / Bc[agg[i]];
  }
  return P;
}

double prolongator_damping(double lam) { return 4.0 / (3.0 * lam); }

std::vector<int32_t> rcm_order(const Csr& A) {
  const int32_t n = A.nrows;
  std::vector<int32_t> deg(n);
  for (int32_t i = 0; i < n; ++i) deg[i] = A.rp[i + 1] - A.rp[i];
  auto lighter = [&](int32_t a, int32_t b) { return deg[a] != deg[b] ? deg[a] < deg[b] : a < b; };
  // component starts: nodes by increasing degree, the first unvisited one each time
  std::vector<int32_t> starts(n);
  for (int32_t i = 0; i < n; ++i) starts[i] = i;
  std::sort(starts.begin(), starts.end(), lighter);
  std::vector<uint8_t> seen(n, 0);
  std::vector<int32_t> order;
  order.reserve(n);
  std::vector<int32_t> nb;
  size_t next_start = 0;
  while ((int32_t)order.size() < n) {
    while (seen[starts[next_start]]) ++next_start;
    const int32_t s0 = starts[next_start];
    seen[s0] = 1;
    order.push_back(s0);
    for (size_t head = order.size() - 1; head < order.size(); ++head) {
      const int32_t u = order[head];
      nb.clear();
      for (int32_t k = A.rp[u]; k < A.rp[u + 1]; ++k) {
        const int32_t c = A.ci[k];
        if (!seen[c]) {
          seen[c] = 1;
          nb.push_back(c);
        }
      }
      std::sort(nb.begin(), nb.end(), lighter);
      order.insert(order.end(), nb.begin(), nb.end());
    }
  }
  std::reverse(order.begin(), order.end());
  return order;
}

Csr renumbered(const Csr& M, const int32_t* rows, const int32_t* cols) {
  Csr R;
  R.nrows = M.nrows;
  R.ncols = M.ncols;
  R.rp.assign(M.nrows + 1, 0);
  for (int32_t i = 0; i < M.nrows; ++i) {
    const int32_t o = rows ? rows[i] : i;
    R.rp[i + 1] = R.rp[i] + (M.rp[o + 1] - M.rp[o]);
  }
  R.ci.resize(M.ci.size());
  R.v.resize(M.v.size());
#pragma omp parallel
  {
    std::vector<uint64_t> key;  // new column in the high word, position in the row in the low
#pragma omp for schedule(dynamic, 256)
    for (int32_t i = 0; i < M.nrows; ++i) {
      const int32_t o = rows ? rows[i] : i, b = M.rp[o], len = M.rp[o + 1] - b;
      key.resize(len);
      bool sorted = true;
      for (int32_t j = 0; j < len; ++j) {
        const uint32_t c = (uint32_t)(cols ? cols[M.ci[b + j]] : M.ci[b + j]);
        key[j] = (uint64_t)c << 32 | (uint32_t)j;
        sorted = sorted && (j == 0 || key[j] > key[j - 1]);
      }
      if (!sorted) std::sort(key.begin(), key.end());
      const int32_t q = R.rp[i];
      for (int32_t j = 0; j < len; ++j) {
        R.ci[q + j] = (int32_t)(key[j] >> 32);
        R.v[q + j] = M.v[b + (int32_t)(key[j] & 0xffffffffu)];
      }
    }
  }
  return R;
}

double strength_cut(double theta) { return theta * (1.0 - kTie); }
double tie_keep() { return 1.0 - kTie; }

// ------------------------------------------------------------------------------------------
// With BIDOMAIN_SETUP_LOG set in the environment, one line per level goes to stderr as the
// setup proceeds (large hierarchies take minutes on the host).
int build_hierarchy(Csr A0, const bd_amg_opts& o, HostHierarchy& H, std::string& err,
                    const GalerkinOffload* offload, const AggregateOffload* agg_offload) {
  const bool log = std::getenv("BIDOMAIN_SETUP_LOG") != nullptr;
  const auto t_start = std::chrono::steady_clock::now();
  auto elapsed = [&] { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count(); };
  auto stamp = [&](int k, const char* what) {
    if (log) std::fprintf(stderr, "[setup] level %d: %s (%.2f s)\n", k, what, elapsed());
  };
  H.lv.clear();
  HostLevel cur;
  cur.B.assign(A0.nrows, 1.0);
  cur.A = std::move(A0);
  for (int k = 0;; ++k) {
    const std::vector<double> d = diagonal(cur.A);
    cur.Dinv.resize(d.size());
    bool positive = true;
    for (size_t i = 0; i < d.size(); ++i) {
      positive = positive && d[i] > 0.0;
      cur.Dinv[i] = 1.0 / d[i];
    }
    const int32_t n = cur.A.nrows;
    const std::string bad_diag = "level " + std::to_string(k) + " has a non-positive diagonal entry";
    if (n <= o.coarse_eq_limit || k == o.max_levels - 1 || k == BD_MAX_LEVELS - 1) {
      // a directly solved coarsest level is never Jacobi-scaled (a one-row level of the
      // singular operator is zero up to rounding)
      if (!positive && n > o.coarse_dense_max) {
        err = bad_diag;
        return BD_E_INVALID;
      }
      H.lv.push_back(std::move(cur));
      break;
    }
    if (!positive) {
      err = bad_diag;
      return BD_E_INVALID;
    }
    Csr P;
    std::vector<double> Bc;
    int32_t nc = 0;
    bool on_device = false;
    if (o.coarsening == BD_SA && agg_offload && o.independent_set == BD_MIS_LUBY) {
      on_device = (*agg_offload)(cur.A, d, cur.Dinv, cur.B, k, cur.lam, P, Bc, nc);
      if (on_device) stamp(k, "eigenvalue estimate, strength, independent set, aggregates and prolongator on the device");
    }
    if (!on_device) {
      cur.lam = lambda_estimate(cur.A, cur.Dinv, o.esteig_iters, o.seed + (uint64_t)k);
      stamp(k, "eigenvalue estimate");
    }
    if (o.coarsening == BD_SA) {
      if (!on_device) {
        const Graph G = sa_strength(cur.A, d, o.threshold);
        stamp(k, "strength graph");
        std::vector<int32_t> order;
        if (o.independent_set == BD_MIS_LUBY) {  // decreasing priority (the index in the low bits)
          std::vector<uint64_t> key(n);
#pragma omp parallel for schedule(static, 4096)
          for (int32_t i = 0; i < n; ++i) key[i] = luby_key(o.seed, k, i);
          std::sort(key.begin(), key.end(), std::greater<uint64_t>());
          order.resize(n);
          for (int32_t q = 0; q < n; ++q) order[q] = (int32_t)(key[q] & 0xFFFFFFFFu);
        }
        const std::vector<uint8_t> st =
            greedy_mis(G, n, k < o.square_graph_levels, o.independent_set == BD_MIS_LUBY ? &order : nullptr);
        stamp(k, "independent set");
        std::vector<int32_t> agg;
        nc = sa_aggregate(G, st, agg);
        if (nc < 0) {
          err = "aggregation left nodes unassigned";
          return BD_E_INVALID;
        }
        P = sa_prolongator(cur.A, cur.Dinv, cur.B, agg, nc, cur.lam, o.prolong_smooths, Bc);
        stamp(k, "aggregates and smoothed prolongator");
      }
    } else {
      const Csr S = rs_strength(cur.A, o.threshold);
      const std::vector<uint8_t> st =
          o.coarsening == BD_PMIS ? pmis_split(S, o.seed + kPmisSeedOffset + (uint64_t)k) : rs_split(S);
      P = rs_interpolation(cur.A, S, st);
      nc = P.ncols;
      Bc.assign(nc, 1.0);
    }
    if (nc == 0 || (double)nc > o.stagnation_ratio * n) {
      H.lv.push_back(std::move(cur));  // keep lam: this level may be relaxed as coarsest
      break;
    }
    Csr R = transpose(P);
    Csr Ac;
    bool done = false;
    if (offload) {
      int64_t flops = 0;
#pragma omp parallel for reduction(+ : flops) schedule(static, 4096)
      for (int32_t i = 0; i < n; ++i)
        for (int32_t ka = cur.A.rp[i]; ka < cur.A.rp[i + 1]; ++ka) flops += P.rp[cur.A.ci[ka] + 1] - P.rp[cur.A.ci[ka]];
      done = (*offload)(cur.A, P, R, flops, Ac);
      if (done && log) std::fprintf(stderr, "[setup] level %d: Galerkin product on the device (%.1f s)\n", k, elapsed());
    }
    if (!done) {
      Csr AP = spgemm(cur.A, P);
      if (log) std::fprintf(stderr, "[setup] level %d: A P has %zu nonzeros (%.1f s)\n", k, AP.v.size(), elapsed());
      Csr RAP = spgemm(R, AP);
      stamp(k, "R (A P)");
      Ac = symmetrize(RAP);
    }
    if (log)
      std::fprintf(stderr, "[setup] level %d: %d rows, %zu nonzeros -> %d rows, %zu nonzeros (%.1f s)\n", k, n,
                   cur.A.v.size(), Ac.nrows, Ac.v.size(), elapsed());
    cur.P = std::move(P);
    cur.R = std::move(R);
    HostLevel next;
    next.A = std::move(Ac);
    next.B = std::move(Bc);
    H.lv.push_back(std::move(cur));
    cur = std::move(next);
  }
  HostLevel& L = H.lv.back();
  if (L.A.nrows > o.coarse_dense_max) {
    H.coarse_mode = 1;
    if (!std::isfinite(L.lam))
      L.lam = lambda_estimate(L.A, L.Dinv, o.esteig_iters, o.seed + (uint64_t)(H.lv.size() - 1));
    H.G.clear();
    return BD_OK;
  }
  H.coarse_mode = 0;
  return coarse_operator(L, o.nullspace == BD_NULL_CONSTANT, H.G, err);
}

}  // namespace bd

// The App. A defaults (declared in bidomain.h; host code, so the setup can run without HIP).
extern "C" void bidomain_default_opts(bd_amg_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->coarsening = BD_SA;
  o->threshold = 0.06;
  o->square_graph_levels = 1;
  o->prolong_smooths = 1;
  o->coarse_eq_limit = 100;
  o->max_levels = 25;
  o->smoother = BD_CHEBYSHEV;
  o->smoother_degree = 2;
  o->cheb_lo = 0.05;
  o->cheb_hi = 1.05;
  o->esteig_iters = 10;
  o->seed = 0;
  o->vcycle_precision = BD_F64;
  o->nullspace = BD_NULL_NONE;
  o->stagnation_ratio = 0.9;
  o->coarse_dense_max = 2048;
  o->galerkin_device = 1;
  o->diag_form = 1;
  o->preconditioner = BD_PC_AMG;
  o->independent_set = BD_MIS_LUBY;
  o->aggregate_device = 1;
  o->reorder = 1;
}
