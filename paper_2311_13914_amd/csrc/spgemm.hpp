// Sparse matrix products of the setup phase on the device: the Galerkin product R (A P) of
// Alg. 1 as two products C = A B of CSR matrices, and the symmetrisation (C + C^T) / 2.
//
// Row-wise, in two passes.  Symbolic: the distinct columns of row i of C are the union of the
// columns of the rows B(k), k in A(i); rows with few partial products collect them in an LDS
// hash table (one 64-lane block per row), the others with a per-block mark array over C's
// columns in device memory (one 256-thread block per row); a first pass counts them (the host
// turns the counts into row offsets), a second pass writes them sorted (bitonic sort in LDS, or
// an ordered scan of the marks for rows with very many columns).  Numeric: the row's sorted
// columns and their accumulators sit in LDS (in windows of kWindow columns for long rows); the
// block walks A(i) in order and adds a_ik b_kj for B(k)'s entries in parallel -- one B row holds
// a column at most once, so no two threads touch the same accumulator within a step, and a
// barrier between steps fixes the order: every entry of C is summed in the order of A(i), with
// separately rounded products and sums.  That is the host product's order, so the two agree bit
// for bit.  No floating-point atomics anywhere.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>

namespace bd {
namespace sg {

constexpr int kSmallBlock = 64;      // one wave per small row
constexpr int kSmallProducts = 512;  // partial products of a small row (so at most 512 columns)
constexpr int kSmallHash = 1024;     // LDS hash slots of a small row (load <= 1/2)
constexpr int kBigBlock = 256;       // one block per big row
constexpr int kBigSort = 8192;       // columns of a big row sorted in LDS; more: ordered mark scan
constexpr int kWindow = 4096;        // output columns of a big row accumulated in LDS at a time

__device__ inline uint32_t hash_slot(int32_t c) {
  return ((uint32_t)c * 0x9E3779B1u) >> (32 - 10);  // kSmallHash = 2^10 slots
}

// First index of a[0..len) (ascending) that is >= key.
__device__ inline int lower_bound(const int* a, int len, int key) {
  int lo = 0, hi = len;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// Ascending bitonic sort of a[0..P) in LDS (P a power of two) by the whole block.
__device__ inline void bitonic_sort(int* a, int P, int t, int nt) {
  for (int k = 2; k <= P; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int idx = t; idx < P; idx += nt) {
        const int ixj = idx ^ j;
        if (ixj > idx) {
          const int x = a[idx], y = a[ixj];
          if ((x > y) == ((idx & k) == 0)) {
            a[idx] = y;
            a[ixj] = x;
          }
        }
      }
      __syncthreads();
    }
}

// u[i] = number of partial products of row i of A B (saturated at INT_MAX).
__global__ void k_sg_products(const int* __restrict__ arp, const int* __restrict__ aci, const int* __restrict__ brp,
                              int n, int* __restrict__ u) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    int64_t s = 0;
    for (int k = arp[i]; k < arp[i + 1]; ++k) {
      const int c = aci[k];
      s += brp[c + 1] - brp[c];
    }
    u[i] = (int)(s < INT_MAX ? s : INT_MAX);
  }
}

// Rows with at most kSmallProducts partial products, one 64-lane block each.  MODE 0: cnt[i] =
// number of distinct columns; MODE 1: the columns, ascending, at cci[crp[i]...].
template <int MODE>
__global__ __launch_bounds__(kSmallBlock) void k_sg_small(const int* __restrict__ arp, const int* __restrict__ aci,
                                                          const int* __restrict__ brp, const int* __restrict__ bci,
                                                          const int* __restrict__ u, int n, int* __restrict__ cnt,
                                                          const int* __restrict__ crp, int* __restrict__ cci) {
  __shared__ int hs[kSmallHash];
  __shared__ int list[kSmallProducts];
  __shared__ int nlist;
  const int t = threadIdx.x;
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    if (u[i] > kSmallProducts) continue;  // the same for every thread of the block
    for (int s = t; s < kSmallHash; s += kSmallBlock) hs[s] = -1;
    if (t == 0) nlist = 0;
    __syncthreads();
    const int a1 = arp[i + 1];
    for (int ka = arp[i]; ka < a1; ++ka) {
      const int k = aci[ka];
      const int b1 = brp[k + 1];
      for (int kb = brp[k] + t; kb < b1; kb += kSmallBlock) {
        const int c = bci[kb];
        uint32_t h = hash_slot(c);
        while (true) {
          const int prev = atomicCAS(&hs[h], -1, c);
          if (prev == -1) {
            list[atomicAdd(&nlist, 1)] = c;
            break;
          }
          if (prev == c) break;
          h = (h + 1) & (kSmallHash - 1);
        }
      }
    }
    __syncthreads();
    const int m = nlist;
    if (MODE == 0) {
      if (t == 0) cnt[i] = m;
    } else {
      int P = 1;
      while (P < m) P <<= 1;
      for (int s = m + t; s < P; s += kSmallBlock) list[s] = INT_MAX;
      __syncthreads();
      bitonic_sort(list, P, t, kSmallBlock);
      const int c0 = crp[i];
      for (int s = t; s < m; s += kSmallBlock) cci[c0 + s] = list[s];
    }
    __syncthreads();
  }
}

// Rows with more partial products (the list `big`), one 256-thread block each, with a mark array
// of p ints per block (marks + blockIdx.x * p, all -1 before the first pass).  A column is new to
// the row when the block swaps its tag (pass * n + row) into the column's mark.  MODE as above.
template <int MODE>
__global__ __launch_bounds__(kBigBlock) void k_sg_big(const int* __restrict__ arp, const int* __restrict__ aci,
                                                      const int* __restrict__ brp, const int* __restrict__ bci,
                                                      const int* __restrict__ big, int nbig, int n, int p,
                                                      int* __restrict__ marks_all, int* __restrict__ cnt,
                                                      const int* __restrict__ crp, int* __restrict__ cci) {
  __shared__ int list[kBigSort];
  __shared__ int nlist;
  __shared__ int wsum[kBigBlock / 64];
  const int t = threadIdx.x;
  int* marks = marks_all + (int64_t)blockIdx.x * p;
  for (int b = blockIdx.x; b < nbig; b += gridDim.x) {
    const int i = big[b];
    const int tag = MODE * n + i;
    if (t == 0) nlist = 0;
    __syncthreads();
    const int a1 = arp[i + 1];
    for (int ka = arp[i]; ka < a1; ++ka) {
      const int k = aci[ka];
      const int b1 = brp[k + 1];
      for (int kb = brp[k] + t; kb < b1; kb += kBigBlock) {
        const int c = bci[kb];
        if (atomicExch(&marks[c], tag) != tag) {
          const int s = atomicAdd(&nlist, 1);
          if (s < kBigSort) list[s] = c;
        }
      }
    }
    __syncthreads();
    const int m = nlist;
    if (MODE == 0) {
      if (t == 0) cnt[i] = m;
    } else if (m <= kBigSort) {
      int P = 1;
      while (P < m) P <<= 1;
      for (int s = m + t; s < P; s += kBigBlock) list[s] = INT_MAX;
      __syncthreads();
      bitonic_sort(list, P, t, kBigBlock);
      const int c0 = crp[i];
      for (int s = t; s < m; s += kBigBlock) cci[c0 + s] = list[s];
    } else {
      // very many columns: scan the marks in column order
      const int lane = t & 63, wv = t >> 6;
      int base = crp[i];
      for (int c0 = 0; c0 < p; c0 += kBigBlock) {
        const int c = c0 + t;
        const bool f = c < p && __hip_atomic_load(&marks[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == tag;
        const uint64_t bal = __ballot(f);
        if (lane == 0) wsum[wv] = __popcll(bal);
        __syncthreads();
        int off = 0, tot = 0;
        for (int w = 0; w < kBigBlock / 64; ++w) {
          off += w < wv ? wsum[w] : 0;
          tot += wsum[w];
        }
        if (f) cci[base + off + __popcll(bal & ((1ull << lane) - 1))] = c;
        base += tot;
        __syncthreads();
      }
    }
    __syncthreads();
  }
}

// Numeric pass of the small rows: C(i, :) accumulated in LDS in the order of A(i).
__global__ __launch_bounds__(kSmallBlock) void k_sg_num_small(const int* __restrict__ arp, const int* __restrict__ aci,
                                                              const double* __restrict__ av,
                                                              const int* __restrict__ brp, const int* __restrict__ bci,
                                                              const double* __restrict__ bv, const int* __restrict__ u,
                                                              int n, const int* __restrict__ crp,
                                                              const int* __restrict__ cci, double* __restrict__ cv) {
#pragma clang fp contract(off)  // product and sum rounded separately, as on the host
  __shared__ int cols[kSmallProducts];
  __shared__ double acc[kSmallProducts];
  const int t = threadIdx.x;
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    if (u[i] > kSmallProducts) continue;
    const int c0 = crp[i], m = crp[i + 1] - c0;
    for (int s = t; s < m; s += kSmallBlock) {
      cols[s] = cci[c0 + s];
      acc[s] = 0.0;
    }
    __syncthreads();
    const int a1 = arp[i + 1];
    for (int ka = arp[i]; ka < a1; ++ka) {
      const int k = aci[ka];
      const double a = av[ka];
      const int b1 = brp[k + 1];
      for (int kb = brp[k] + t; kb < b1; kb += kSmallBlock) {
        const int pos = lower_bound(cols, m, bci[kb]);
        acc[pos] = acc[pos] + a * bv[kb];
      }
      __syncthreads();
    }
    for (int s = t; s < m; s += kSmallBlock) cv[c0 + s] = acc[s];
    __syncthreads();
  }
}

// Numeric pass of the big rows, kWindow output columns at a time.
__global__ __launch_bounds__(kBigBlock) void k_sg_num_big(const int* __restrict__ arp, const int* __restrict__ aci,
                                                          const double* __restrict__ av, const int* __restrict__ brp,
                                                          const int* __restrict__ bci, const double* __restrict__ bv,
                                                          const int* __restrict__ big, int nbig,
                                                          const int* __restrict__ crp, const int* __restrict__ cci,
                                                          double* __restrict__ cv) {
#pragma clang fp contract(off)  // product and sum rounded separately, as on the host
  __shared__ int cols[kWindow];
  __shared__ double acc[kWindow];
  const int t = threadIdx.x;
  for (int b = blockIdx.x; b < nbig; b += gridDim.x) {
    const int i = big[b];
    const int r0 = crp[i], m = crp[i + 1] - r0;
    for (int w0 = 0; w0 < m; w0 += kWindow) {
      const int wl = m - w0 < kWindow ? m - w0 : kWindow;
      for (int s = t; s < wl; s += kBigBlock) {
        cols[s] = cci[r0 + w0 + s];
        acc[s] = 0.0;
      }
      __syncthreads();
      const int lo = cols[0], hi = cols[wl - 1];
      const int a1 = arp[i + 1];
      for (int ka = arp[i]; ka < a1; ++ka) {
        const int k = aci[ka];
        const double a = av[ka];
        const int b1 = brp[k + 1];
        for (int kb = brp[k] + t; kb < b1; kb += kBigBlock) {
          const int c = bci[kb];
          if (c < lo || c > hi) continue;
          const int pos = lower_bound(cols, wl, c);
          acc[pos] = acc[pos] + a * bv[kb];
        }
        __syncthreads();
      }
      for (int s = t; s < wl; s += kBigBlock) cv[r0 + w0 + s] = acc[s];
      __syncthreads();
    }
  }
}

// Big rows of a product with at most kDenseCols output columns (the filled coarse levels).  The
// row's partial products are walked kGroup entries of A(i) at a time, flattened: each thread
// takes products by index through the prefix of the group's B-row lengths, so short B rows do
// not serialise the row.  Symbolic: a bitmap over all p columns in LDS.  Numeric: kChunk
// products at a time are sorted by (column, product index) in LDS and each column's run is added,
// in that order, to a dense accumulator of p doubles in device memory owned by the block; chunks
// follow each other behind a barrier, so every column is summed in the order of A(i).
constexpr int kDenseCols = 65536;
constexpr int kGroup = kBigBlock;  // one A entry per thread
constexpr int kChunk = 2048;       // products sorted at a time (11 bits of the sort key)

// Exclusive prefix sum of v over the block (kBigBlock threads); *total gets the sum.
__device__ inline int block_exclusive_scan(int v, int* sh, int* total) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < kBigBlock; off <<= 1) {
    const int add = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += add;
    __syncthreads();
  }
  const int incl = sh[t];
  *total = sh[kBigBlock - 1];
  __syncthreads();
  return incl - v;
}

// Entries [g0, min(g0 + kGroup, a1)) of A(i) into LDS: their B-row start, the exclusive prefix of
// the B-row lengths and (with av) the A value; returns the group's number of partial products.
__device__ inline int load_group(const int* __restrict__ aci, const double* __restrict__ av,
                                 const int* __restrict__ brp, int g0, int a1, int* gbs, int* goff, double* ga,
                                 int* sh) {
  const int t = threadIdx.x, ka = g0 + t;
  int bs = 0, bl = 0;
  double a = 0.0;
  if (ka < a1) {
    const int k = aci[ka];
    bs = brp[k];
    bl = brp[k + 1] - bs;
    if (av) a = av[ka];
  }
  int total;
  const int off = block_exclusive_scan(bl, sh, &total);
  gbs[t] = bs;
  goff[t] = off;
  if (ga) ga[t] = a;
  __syncthreads();
  return total;
}

// The group entry that holds product j (0 <= j < total): the last g with goff[g] <= j.
__device__ inline int group_entry(const int* goff, int j) {
  int lo = 0, hi = kGroup - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (goff[mid] <= j) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <int MODE>
__global__ __launch_bounds__(kBigBlock) void k_sg_dense_sym(const int* __restrict__ arp, const int* __restrict__ aci,
                                                            const int* __restrict__ brp, const int* __restrict__ bci,
                                                            const int* __restrict__ big, int nbig, int p,
                                                            int* __restrict__ cnt, const int* __restrict__ crp,
                                                            int* __restrict__ cci) {
  __shared__ uint32_t bm[kDenseCols / 32];
  __shared__ int sh[kBigBlock];
  __shared__ int gbs[kGroup], goff[kGroup];
  const int t = threadIdx.x;
  const int words = (p + 31) / 32;
  for (int b = blockIdx.x; b < nbig; b += gridDim.x) {
    const int i = big[b];
    for (int w = t; w < words; w += kBigBlock) bm[w] = 0u;
    __syncthreads();
    const int a1 = arp[i + 1];
    for (int g0 = arp[i]; g0 < a1; g0 += kGroup) {
      const int total = load_group(aci, nullptr, brp, g0, a1, gbs, goff, nullptr, sh);
      for (int j = t; j < total; j += kBigBlock) {
        const int g = group_entry(goff, j);
        const int c = bci[gbs[g] + j - goff[g]];
        atomicOr(&bm[c >> 5], 1u << (c & 31));
      }
      __syncthreads();
    }
    int base = MODE == 1 ? crp[i] : 0;
    for (int w0 = 0; w0 < words; w0 += kBigBlock) {
      const int w = w0 + t;
      const uint32_t bits = w < words ? bm[w] : 0u;
      int total;
      const int off = block_exclusive_scan(__popc(bits), sh, &total);
      if (MODE == 1) {
        uint32_t x = bits;
        int q = base + off;
        while (x) {
          cci[q++] = w * 32 + (__ffs(x) - 1);
          x &= x - 1;
        }
      }
      base += total;
    }
    if (MODE == 0 && t == 0) cnt[i] = base;
    __syncthreads();
  }
}

// accg_all: p doubles per block, zero before the launch (each row leaves its columns zero).
__global__ __launch_bounds__(kBigBlock) void k_sg_dense_num(const int* __restrict__ arp, const int* __restrict__ aci,
                                                            const double* __restrict__ av,
                                                            const int* __restrict__ brp, const int* __restrict__ bci,
                                                            const double* __restrict__ bv, const int* __restrict__ big,
                                                            int nbig, int p, double* __restrict__ accg_all,
                                                            const int* __restrict__ crp, const int* __restrict__ cci,
                                                            double* __restrict__ cv) {
#pragma clang fp contract(off)  // product and sum rounded separately, as on the host
  __shared__ int key[kChunk];
  __shared__ double val[kChunk];
  __shared__ int sh[kBigBlock];
  __shared__ int gbs[kGroup], goff[kGroup];
  __shared__ double ga[kGroup];
  const int t = threadIdx.x;
  double* accg = accg_all + (int64_t)blockIdx.x * p;
  for (int b = blockIdx.x; b < nbig; b += gridDim.x) {
    const int i = big[b];
    const int a1 = arp[i + 1];
    for (int g0 = arp[i]; g0 < a1; g0 += kGroup) {
      const int total = load_group(aci, av, brp, g0, a1, gbs, goff, ga, sh);
      for (int c0 = 0; c0 < total; c0 += kChunk) {
        const int cn = total - c0 < kChunk ? total - c0 : kChunk;
        int P = 1;
        while (P < cn) P <<= 1;
        for (int s = t; s < P; s += kBigBlock) {
          if (s < cn) {
            const int j = c0 + s;
            const int g = group_entry(goff, j);
            const int kb = gbs[g] + j - goff[g];
            key[s] = (bci[kb] << 11) | s;
            val[s] = ga[g] * bv[kb];
          } else {
            key[s] = INT_MAX;
          }
        }
        __syncthreads();
        bitonic_sort(key, P, t, kBigBlock);
        for (int s = t; s < cn; s += kBigBlock) {
          const int col = key[s] >> 11;
          if (s == 0 || (key[s - 1] >> 11) != col) {
            double acc = accg[col];
            for (int q = s; q < cn && (key[q] >> 11) == col; ++q) acc = acc + val[key[q] & (kChunk - 1)];
            accg[col] = acc;
          }
        }
        __syncthreads();
      }
    }
    for (int e = crp[i] + t; e < crp[i + 1]; e += kBigBlock) {
      const int c = cci[e];
      cv[e] = accg[c];
      accg[c] = 0.0;
    }
    __syncthreads();
  }
}

// out = (C + C^T) / 2 on C's pattern (a mirror entry that does not exist counts as zero); one
// 64-lane group per row.
__global__ void k_sg_symmetrize(const int* __restrict__ crp, const int* __restrict__ cci,
                                const double* __restrict__ cv, int n, double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int stride = gridDim.x * (blockDim.x / 64);
  for (int i = blockIdx.x * (blockDim.x / 64) + (int)(threadIdx.x / 64); i < n; i += stride)
    for (int k = crp[i] + lane; k < crp[i + 1]; k += 64) {
      const int j = cci[k];
      const int lo = crp[j], len = crp[j + 1] - lo;
      const int q = lower_bound(cci + lo, len, i);
      const double mirror = (q < len && cci[lo + q] == i) ? cv[lo + q] : 0.0;
      out[k] = __dmul_rn(0.5, __dadd_rn(cv[k], mirror));
    }
}

}  // namespace sg
}  // namespace bd
