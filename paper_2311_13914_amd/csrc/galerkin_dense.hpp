// Galerkin products of the filled coarse levels on the matrix cores.  Smoothed aggregation fills
// its coarse operators in (a 21,403-row level of the 384 x 384 x 96 slab keeps 59 % of its
// entries), and R (A P) there is a dense contraction: 10^12 partial products as a sparse product
// against ~10^13 flops as a dense one.  So the operands are expanded to dense row-major matrices
// (zero padded to whole tiles) and multiplied by a float64 MFMA kernel that skips every 128 x 16
// tile of the left operand holding no entry (R's tiles are mostly empty, A's band leaves many);
// the structural pattern of the product, which the sparse product keeps entry for entry, comes
// from bitmaps: the columns of row i of A P are the OR of the column bitmaps of P's rows k in
// A(i), and likewise for R (A P).  The values then equal the sparse product up to rounding order.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bd {
namespace gd {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kTile = 128;  // block tile of the product (rows and columns); dimensions padded to it
constexpr int kKStep = 16;  // k extent of one staged tile pair
constexpr int kAStride = kKStep + 1;  // LDS row stride of the left tile (doubles), against bank conflicts

// out[i * ld + ci[k]] = v[k] for the CSR rows (out zero beforehand); one block per row.
__global__ void k_gd_densify(const int* __restrict__ rp, const int* __restrict__ ci, const double* __restrict__ v,
                             int nrows, int64_t ld, double* __restrict__ out) {
  for (int i = blockIdx.x; i < nrows; i += gridDim.x)
    for (int k = rp[i] + (int)threadIdx.x; k < rp[i + 1]; k += blockDim.x) out[(int64_t)i * ld + ci[k]] = v[k];
}

// occ[(i / kTile) * nkt + c / kKStep] = 1 for every entry (i, c) (occ zero beforehand).
__global__ void k_gd_occupancy(const int* __restrict__ rp, const int* __restrict__ ci, int nrows, int nkt,
                               uint8_t* __restrict__ occ) {
  for (int i = blockIdx.x; i < nrows; i += gridDim.x)
    for (int k = rp[i] + (int)threadIdx.x; k < rp[i + 1]; k += blockDim.x)
      occ[(int64_t)(i / kTile) * nkt + ci[k] / kKStep] = 1;
}

// C = A B for row-major A (M x K, ld lda), B (K x N, ldb), C (M x N, ldc), with M and N multiples
// of kTile and K of kKStep; grid (N / kTile, M / kTile), 256 threads.  Each wave computes a 64 x 64
// quarter of the block tile as 4 x 4 MFMA tiles of 16 x 16 (v_mfma_f64_16x16x4: lane l holds
// A(l % 16, l / 16), B(l / 16, l % 16) and D(4 i + l / 16, l % 16), i < 4).  occ (M / kTile rows of
// nkt = K / kKStep bytes): left tiles to multiply; an all-zero tile is skipped.
__global__ __launch_bounds__(256) void k_gd_gemm(const double* __restrict__ A, int64_t lda,
                                                 const double* __restrict__ B, int64_t ldb, double* __restrict__ C,
                                                 int64_t ldc, int nkt, const uint8_t* __restrict__ occ) {
  __shared__ double As[kTile * kAStride];
  __shared__ double Bs[kKStep * kTile];
  const int t = threadIdx.x, l = t & 63, w = t >> 6;
  const int m0 = blockIdx.y * kTile, n0 = blockIdx.x * kTile;
  const int wm = (w >> 1) * 64, wn = (w & 1) * 64;
  d4 acc[4][4];
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) acc[a][b] = d4{0.0, 0.0, 0.0, 0.0};
  const uint8_t* orow = occ + (int64_t)blockIdx.y * nkt;
  for (int kt = 0; kt < nkt; ++kt) {
    if (!orow[kt]) continue;  // the same for the whole block
    const int k0 = kt * kKStep;
    {  // left tile 128 x 16: thread t takes row t / 2, columns 8 (t % 2) .. + 7
      const double* ap = A + (int64_t)(m0 + (t >> 1)) * lda + k0 + (t & 1) * 8;
      double* as = As + (t >> 1) * kAStride + (t & 1) * 8;
      for (int j = 0; j < 8; j += 2) {
        const double2 x = *(const double2*)(ap + j);
        as[j] = x.x;
        as[j + 1] = x.y;
      }
      // right tile 16 x 128: thread t takes row t / 16, columns 8 (t % 16) .. + 7
      const double* bp = B + (int64_t)(k0 + (t >> 4)) * ldb + n0 + (t & 15) * 8;
      double* bs = Bs + (t >> 4) * kTile + (t & 15) * 8;
      for (int j = 0; j < 8; j += 2) *(double2*)(bs + j) = *(const double2*)(bp + j);
    }
    __syncthreads();
    for (int kk = 0; kk < kKStep / 4; ++kk) {
      double av[4], bv[4];
      for (int a = 0; a < 4; ++a) av[a] = As[(wm + a * 16 + (l & 15)) * kAStride + kk * 4 + (l >> 4)];
      for (int b = 0; b < 4; ++b) bv[b] = Bs[(kk * 4 + (l >> 4)) * kTile + wn + b * 16 + (l & 15)];
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    __syncthreads();
  }
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b)
      for (int i = 0; i < 4; ++i)
        C[(int64_t)(m0 + wm + a * 16 + 4 * i + (l >> 4)) * ldc + n0 + wn + b * 16 + (l & 15)] = acc[a][b][i];
}

// bits[i * W + c / 32] has bit c % 32 set for every entry (i, c) (bits zero beforehand).
__global__ void k_gd_row_bits(const int* __restrict__ rp, const int* __restrict__ ci, int nrows, int W,
                              uint32_t* __restrict__ bits) {
  for (int i = blockIdx.x; i < nrows; i += gridDim.x)
    for (int k = rp[i] + (int)threadIdx.x; k < rp[i + 1]; k += blockDim.x)
      atomicOr(&bits[(int64_t)i * W + (ci[k] >> 5)], 1u << (ci[k] & 31));
}

// out row i = OR of in rows k over the entries (i, k) of the CSR matrix; one block per row.
__global__ void k_gd_or_rows(const int* __restrict__ rp, const int* __restrict__ ci, int nrows, int W,
                             const uint32_t* __restrict__ in, uint32_t* __restrict__ out) {
  for (int i = blockIdx.x; i < nrows; i += gridDim.x)
    for (int w = threadIdx.x; w < W; w += blockDim.x) {
      uint32_t x = 0u;
      for (int k = rp[i]; k < rp[i + 1]; ++k) x |= in[(int64_t)ci[k] * W + w];
      out[(int64_t)i * W + w] = x;
    }
}

// cnt[i] = number of bits set in row i; one block (kBlock threads) per row.
__global__ void k_gd_count(const uint32_t* __restrict__ bits, int nrows, int W, int* __restrict__ cnt) {
  __shared__ int part[1024 / 64];
  for (int i = blockIdx.x; i < nrows; i += gridDim.x) {
    int s = 0;
    for (int w = threadIdx.x; w < W; w += blockDim.x) s += __popc(bits[(int64_t)i * W + w]);
    for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
      int tot = 0;
      for (int q = 0; q < (int)(blockDim.x >> 6); ++q) tot += part[q];
      cnt[i] = tot;
    }
    __syncthreads();
  }
}

// Column indices of row i, ascending, at ci[rp[i]...]; one 256-thread block per row.
__global__ __launch_bounds__(256) void k_gd_extract(const uint32_t* __restrict__ bits, int nrows, int W,
                                                    const int* __restrict__ rp, int* __restrict__ ci) {
  __shared__ int sh[256];
  const int t = threadIdx.x;
  for (int i = blockIdx.x; i < nrows; i += gridDim.x) {
    int base = rp[i];
    for (int w0 = 0; w0 < W; w0 += 256) {
      const int w = w0 + t;
      const uint32_t x0 = w < W ? bits[(int64_t)i * W + w] : 0u;
      const int c = __popc(x0);
      sh[t] = c;
      __syncthreads();
      for (int off = 1; off < 256; off <<= 1) {
        const int add = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
      }
      int q = base + sh[t] - c;
      const int tot = sh[255];
      uint32_t x = x0;
      while (x) {
        ci[q++] = w * 32 + (__ffs(x) - 1);
        x &= x - 1;
      }
      base += tot;
      __syncthreads();
    }
  }
}

// out[e] = (D(i, c) + D(c, i)) / 2 for the entries e = (i, c) of the pattern; one 64-lane group
// per row.
__global__ void k_gd_values(const int* __restrict__ rp, const int* __restrict__ ci, int nrows,
                            const double* __restrict__ D, int64_t ld, double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int stride = gridDim.x * (blockDim.x / 64);
  for (int i = blockIdx.x * (blockDim.x / 64) + (int)(threadIdx.x / 64); i < nrows; i += stride)
    for (int e = rp[i] + lane; e < rp[i + 1]; e += 64) {
      const int c = ci[e];
      out[e] = 0.5 * (D[(int64_t)i * ld + c] + D[(int64_t)c * ld + i]);
    }
}

}  // namespace gd
}  // namespace bd
