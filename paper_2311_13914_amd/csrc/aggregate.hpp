// Smoothed-aggregation coarsening of a level on the device (Alg. 1, Sec. 4): the strength graph,
// the parallel independent set (Luby-type rounds with fixed priorities), the two aggregation
// passes and the prolongator smoothing's combination step.  Every decision uses the host's
// arithmetic (the same weight |a_ij| / sqrt(a_ii a_jj), the same tie band) so the aggregates are
// the host's; the priorities are the host's SplitMix64 keys.
//
// The independent set runs in rounds.  Within reach means a neighbour in the strength graph S,
// or a node within distance 2 on a squared level (App. A squares the first level's graph).  Each
// round: m1(i) = the largest key among the free nodes of {i} + S(i); on a squared level
// m2(i) = the largest m1 over {i} + S(i), i.e. over the free nodes within distance 2; a free node
// whose own key is that maximum becomes a root; then the free nodes within reach of a new root
// are taken.  With fixed priorities the rounds end in the greedy set taken in decreasing priority,
// the set the host computes sequentially.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bd {
namespace ag {

__device__ inline uint64_t splitmix64_at(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

// key[i] = top 32 bits of the stream's draw i above i; st[i] = 0 (free).  stream = seed +
// offset + level.
__global__ void k_ag_keys(int n, uint64_t stream, uint64_t* __restrict__ key, uint8_t* __restrict__ st) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    key[i] = ((splitmix64_at(stream, (uint64_t)i) >> 32) << 32) | (uint64_t)(uint32_t)i;
    st[i] = 0;
  }
}

// Strength graph: j != i with a_ij != 0 and w = |a_ij| / sqrt(a_ii a_jj) >= cut.  MODE 0 counts
// the strong entries of each row into cnt; MODE 1 writes them (columns in A's order) and their
// weights at srp[i].  One thread per row.
template <int MODE>
__global__ void k_ag_strength(const int* __restrict__ rp, const int* __restrict__ ci, const double* __restrict__ v,
                              const double* __restrict__ d, int n, double cut, int* __restrict__ cnt,
                              const int* __restrict__ srp, int* __restrict__ sci, double* __restrict__ sw) {
#pragma clang fp contract(off)
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    int c = 0, pos = MODE == 1 ? srp[i] : 0;
    const double di = d[i];
    for (int k = rp[i]; k < rp[i + 1]; ++k) {
      const int j = ci[k];
      if (j == i || v[k] == 0.0) continue;
      const double w = fabs(v[k]) / sqrt(di * d[j]);
      if (w >= cut) {
        if (MODE == 1) {
          sci[pos] = j;
          sw[pos] = w;
          ++pos;
        } else {
          ++c;
        }
      }
    }
    if (MODE == 0) cnt[i] = c;
  }
}

// out[i] = max over j in {i} + S(i) of in[j], where in[j] is key[j] for free j and 0 otherwise
// (FREE = true), or m[j] (FREE = false).
template <bool FREE>
__global__ void k_ag_max(const int* __restrict__ srp, const int* __restrict__ sci, int n,
                         const uint64_t* __restrict__ in, const uint8_t* __restrict__ st, uint64_t* __restrict__ out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    uint64_t m = (!FREE || st[i] == 0) ? in[i] : 0;
    for (int k = srp[i]; k < srp[i + 1]; ++k) {
      const int j = sci[k];
      const uint64_t x = (!FREE || st[j] == 0) ? in[j] : 0;
      m = x > m ? x : m;
    }
    out[i] = m;
  }
}

// A free node whose key is the maximum within its reach becomes a root (st = 1, mark = 1).
__global__ void k_ag_select(int n, const uint64_t* __restrict__ m, const uint64_t* __restrict__ key,
                            uint8_t* __restrict__ st, uint8_t* __restrict__ mark) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const bool root = st[i] == 0 && m[i] == key[i];
    if (root) st[i] = 1;
    mark[i] = root ? 1 : 0;
  }
}

// out[i] = in[i] or any in[j], j in S(i).
__global__ void k_ag_reach(const int* __restrict__ srp, const int* __restrict__ sci, int n,
                           const uint8_t* __restrict__ in, uint8_t* __restrict__ out) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    uint8_t r = in[i];
    for (int k = srp[i]; k < srp[i + 1] && !r; ++k) r = in[sci[k]];
    out[i] = r;
  }
}

// Free nodes within reach of a new root are taken (st = 2); *nfree counts those still free.
__global__ void k_ag_take(int n, const uint8_t* __restrict__ reach, uint8_t* __restrict__ st, int* __restrict__ nfree) {
  int c = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    if (st[i] == 0 && reach[i]) st[i] = 2;
    c += st[i] == 0;
  }
  for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off);
  if ((threadIdx.x & 63) == 0 && c) atomicAdd(nfree, c);
}

// Among the neighbours j of i with ok(j), the one of largest weight; weights within the tie band
// of the largest are equal and the lowest index wins; -1 if none (the host's rule).
template <class Ok>
__device__ inline int best_neighbour(const int* __restrict__ srp, const int* __restrict__ sci,
                                     const double* __restrict__ sw, int i, double keep, Ok ok) {
#pragma clang fp contract(off)
  double best = -1.0;
  for (int k = srp[i]; k < srp[i + 1]; ++k)
    if (ok(sci[k]) && sw[k] > best) best = sw[k];
  if (best < 0.0) return -1;
  const double lo = best * keep;
  int pick = -1;
  for (int k = srp[i]; k < srp[i + 1]; ++k) {
    const int j = sci[k];
    if (ok(j) && sw[k] >= lo && (pick < 0 || j < pick)) pick = j;
  }
  return pick;
}

// Pass 1: root[i] = i for roots; a non-root joins the strongly connected root of largest weight
// (root[i] = that root), else root[i] = -1.  keep = 1 - tie.
__global__ void k_ag_pass1(const int* __restrict__ srp, const int* __restrict__ sci, const double* __restrict__ sw,
                           int n, const uint8_t* __restrict__ st, double keep, int* __restrict__ root) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    if (st[i] == 1) {
      root[i] = i;
      continue;
    }
    root[i] = best_neighbour(srp, sci, sw, i, keep, [&](int j) { return st[j] == 1; });
  }
}

// Pass 2 on the snapshot root1: a node left out joins the aggregate of its assigned neighbour of
// largest weight.
__global__ void k_ag_pass2(const int* __restrict__ srp, const int* __restrict__ sci, const double* __restrict__ sw,
                           int n, const int* __restrict__ root1, double keep, int* __restrict__ root2) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int r = root1[i];
    if (r >= 0) {
      root2[i] = r;
      continue;
    }
    const int j = best_neighbour(srp, sci, sw, i, keep, [&](int q) { return root1[q] >= 0; });
    root2[i] = j >= 0 ? root1[j] : -1;
  }
}

// Prolongator smoothing, P_new = P - (omega D^{-1}) (A P) on the pattern of A P (which contains
// P's): v[k] of row i of A P becomes p_i(col) - (omega dinv_i) v[k], the host's operations.
__global__ void k_ag_smooth(const int* __restrict__ prp, const int* __restrict__ pci, const double* __restrict__ pv,
                            const int* __restrict__ crp, const int* __restrict__ cci, double* __restrict__ cv,
                            const double* __restrict__ dinv, double omega, int n) {
#pragma clang fp contract(off)
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double sc = omega * dinv[i];
    int kp = prp[i];
    const int kpe = prp[i + 1];
    for (int k = crp[i]; k < crp[i + 1]; ++k) {
      while (kp < kpe && pci[kp] < cci[k]) ++kp;
      const double pij = (kp < kpe && pci[kp] == cci[k]) ? pv[kp] : 0.0;
      cv[k] = pij - sc * cv[k];
    }
  }
}

// ---- eigenvalue estimate: Jacobi-CG on D^{-1} A in the host's operation order -------------

// r = the start vector (uniform in [-1, 1) from the stream `seed`), z = D^{-1} r, p = z.
__global__ void k_lam_init(int n, uint64_t seed, const double* __restrict__ dinv, double* __restrict__ r,
                           double* __restrict__ z, double* __restrict__ p) {
#pragma clang fp contract(off)
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double ri = 2.0 * ((double)(splitmix64_at(seed, (uint64_t)i) >> 11) * 0x1.0p-53) - 1.0;
    r[i] = ri;
    z[i] = dinv[i] * ri;
    p[i] = z[i];
  }
}

// q = A p, each row summed in order.
__global__ void k_lam_spmv(const int* __restrict__ rp, const int* __restrict__ ci, const double* __restrict__ v,
                           const double* __restrict__ p, int n, double* __restrict__ q) {
#pragma clang fp contract(off)
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int k = rp[i]; k < rp[i + 1]; ++k) s = s + v[k] * p[ci[k]];
    q[i] = s;
  }
}

// part[b] = sum of a[i] b[i] over block b of DB consecutive entries, in order: the block's
// products are staged in LDS by 64 lanes, then added one by one.
template <int DB>
__global__ __launch_bounds__(64) void k_lam_dot_blocks(const double* __restrict__ a, const double* __restrict__ b,
                                                       int64_t n, double* __restrict__ part) {
#pragma clang fp contract(off)
  __shared__ double prod[DB];
  const int64_t nb = (n + DB - 1) / DB;
  for (int64_t blk = blockIdx.x; blk < nb; blk += gridDim.x) {
    const int64_t i0 = blk * DB;
    const int len = (int)(n - i0 < DB ? n - i0 : DB);
    for (int t = threadIdx.x; t < len; t += 64) prod[t] = a[i0 + t] * b[i0 + t];
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int t = 0; t < len; ++t) s = s + prod[t];
      part[blk] = s;
    }
    __syncthreads();
  }
}

// r -= alpha q; z = D^{-1} r.
__global__ void k_lam_update_r(int n, double alpha, const double* __restrict__ q, const double* __restrict__ dinv,
                               double* __restrict__ r, double* __restrict__ z) {
#pragma clang fp contract(off)
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    z[i] = dinv[i] * ri;
  }
}

// p = z + beta p.
__global__ void k_lam_update_p(int n, double beta, const double* __restrict__ z, double* __restrict__ p) {
#pragma clang fp contract(off)
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = z[i] + beta * p[i];
}

}  // namespace ag
}  // namespace bd
