// Device kernels of the AMG-PCG solve phase for gfx950 (CDNA4, wave64).
//
// Everything here is bandwidth-bound streaming: CSR products with a fused epilogue (the
// V-cycle steps of Alg. 2 and the CG product q = A p), pointwise CG vector updates, and
// deterministic reductions.  No matrix-core (MFMA) work: nothing on this path is a dense
// contraction (the coarsest-level matrix-vector product has at most a few thousand rows).
//
// Conventions:
//  * a block has 256 threads (4 waves); products run as the symmetric diagonal kernel (the fine
//    27-point operators stored as their 14 diagonals of offset >= 0), the CSR-stream kernel (a
//    block owns a tile of consecutive rows whose entries it streams through LDS; column indices
//    as 8-bit offset-dictionary entries, 16-bit per-tile offsets, 24-bit or 32-bit indices), or,
//    for rows longer than the staging buffer, as the lane-group kernel (a row per group of G
//    lanes, G a power of two chosen from the mean row length, rows_per_block = 256 / G * TPB);
//  * consecutive passes over one matrix walk its tiles in alternating order, so each pass
//    starts on what the previous one left in the memory-side Infinity Cache;
//  * the block -> row-tile map is XCD-aware: the hardware deals blocks round-robin over the
//    8 XCDs, so consecutive block ids are remapped to one contiguous row range per XCD, which
//    keeps each XCD's L2 working on neighbouring rows (and their shared x entries);
//  * reductions are deterministic and atomic-free: each block stores a partial from a
//    fixed-order tree, and a one-block finalize kernel sums the partials in a fixed order and
//    derives the solver scalars on the device.  (A "last block finishes" scheme would need a
//    device-scope release fence per block, which on CDNA writes back the XCD's L2 each time;
//    the kernel boundary gives the same visibility once.)
//  * every solve kernel first reads the solve's `done` flag and returns at once when it is set,
//    so iterations enqueued past convergence cost only their launch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bd {

constexpr int kBlock = 256;
constexpr int kXcds = 8;

// Device scalar slots (double) and flag slots (int) of one solve.
enum Scalar : int {
  S_RHO = 0,      // current r^T z (or its compensated float analogue)
  S_PQ,           // p^T A p
  S_ALPHA,
  S_BETA,
  S_RNORM2,       // ||r||^2 (recursive residual)
  S_FNORM2,       // ||b^||^2
  S_TOL2,         // rtol^2 ||b^||^2
  S_MU_B,         // mean of b (projection)
  S_MU_X,         // mean of the initial guess
  S_MU_Z,         // mean of the preconditioned residual
  S_RTOL2,        // rtol^2 (input)
  S_TRUE2,        // ||b^ - A x||^2 at exit
  S_WX,           // w^T x (normalisation)
  S_WSUM,         // sum of w
  S_COUNT
};
enum Flag : int {
  F_DONE = 0,     // 1 once converged / failed / capped
  F_ITERS,        // completed iterations
  F_STATUS,       // BD_* status
  F_FIRST,        // 1 before the first direction is formed
  F_MAXIT,
  F_NULLSPACE,
  F_COUNT
};
// Finalize kinds (one-block kernels that turn block partials into solver scalars).
enum Fin : int { FIN_CGQ = 0, FIN_UPDATE, FIN_VC64, FIN_VC32, FIN_INIT, FIN_TRUE, FIN_MEANS, FIN_NORM };

struct Solve {
  double* sc;          // S_COUNT scalars
  int* fl;             // F_COUNT flags
  double* part;        // block partials
  int* host_flags;     // pinned host mirror of (done, iters, status), may be null
  long n;              // fine-level rows
};

__device__ __forceinline__ int xcd_tile(int b, int nb) {
  // bijection of [0, nb): block b runs on XCD b % 8; XCD x gets one contiguous tile range
  const int x = b % kXcds, idx = b / kXcds;
  const int per = nb / kXcds, rem = nb % kXcds;
  return x * per + (x < rem ? x : rem) + idx;
}

__device__ __forceinline__ bool solve_done(const Solve& s) {
  return __hip_atomic_load(&s.fl[F_DONE], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// ---------------------------------------------------------------------------------------
// Reductions.
// Sum over a block of NT threads (NT / 64 waves, a power of two): wave shuffles, then a fixed
// pairwise tree over the waves; every thread returns the totals.
template <int NV, int NT = kBlock>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* lds /* NV * NT / 64 */) {
  constexpr int W = NT / 64;
  static_assert(W >= 1 && (W & (W - 1)) == 0, "a power-of-two number of waves");
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double t = v[k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
    v[k] = t;
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) lds[k * W + wave] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double t[W];
#pragma unroll
    for (int w = 0; w < W; ++w) t[w] = lds[k * W + w];
#pragma unroll
    for (int st = 1; st < W; st *= 2)
#pragma unroll
      for (int w = 0; w < W; w += 2 * st) t[w] += t[w + st];
    v[k] = t[0];
  }
  __syncthreads();
}

// Fixed-order sum of NV partial arrays (stride nb) by the whole block.  Each thread keeps
// kSumLanes independent accumulators so that that many loads are in flight at once (a single
// chain would wait out one memory latency per partial).
constexpr int kSumLanes = 8;
template <int NV, int NT = kBlock>
__device__ __forceinline__ void sum_partials(const double* part, int nb, double (&out)[NV], double* lds) {
  double acc[NV][kSumLanes];
#pragma unroll
  for (int k = 0; k < NV; ++k)
#pragma unroll
    for (int u = 0; u < kSumLanes; ++u) acc[k][u] = 0.0;
  int i = threadIdx.x;
  for (; i + (kSumLanes - 1) * NT < nb; i += kSumLanes * NT)
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
      for (int u = 0; u < kSumLanes; ++u) acc[k][u] += part[(long)k * nb + i + u * NT];
#pragma unroll
  for (int u = 0; u < kSumLanes; ++u)
    if (i + u * NT < nb)
#pragma unroll
      for (int k = 0; k < NV; ++k) acc[k][u] += part[(long)k * nb + i + u * NT];
#pragma unroll
  for (int k = 0; k < NV; ++k)
    out[k] = ((acc[k][0] + acc[k][1]) + (acc[k][2] + acc[k][3])) + ((acc[k][4] + acc[k][5]) + (acc[k][6] + acc[k][7]));
  block_sum<NV, NT>(out, lds);
}
static_assert(kSumLanes == 8, "the combining tree above is written for 8 lanes");

// Compensated float arithmetic (Ogita, Rump & Oishi, SIAM J. Sci. Comput. 26 (2005)):
// TwoSum (Knuth) and TwoProduct with a fused multiply-add.
__device__ __forceinline__ void two_sum(float a, float b, float& s, float& e) {
  s = a + b;
  const float bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}
__device__ __forceinline__ void two_prod(float a, float b, float& p, float& e) {
  p = a * b;
  e = __builtin_fmaf(a, b, -p);
}
// (p, s) accumulator of Dot2: p the running sum, s the accumulated error terms.
struct Dot2 {
  float p = 0.f, s = 0.f;
  __device__ __forceinline__ void add(float x, float y) {
    float h, r, q;
    two_prod(x, y, h, r);
    two_sum(p, h, p, q);
    s += q + r;
  }
  __device__ __forceinline__ void merge(float op, float os) {
    float q;
    two_sum(p, op, p, q);
    s += os + q;
  }
};

template <int NV, int NT = kBlock>
__device__ __forceinline__ void block_dot2(Dot2 (&v)[NV], float* lds /* NV * 2 * NT / 64 */) {
  constexpr int W = NT / 64;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const float op = __shfl_xor(v[k].p, off, 64), os = __shfl_xor(v[k].s, off, 64);
      // both lanes of a pair combine in the same order so that they hold identical values
      Dot2 a, b;
      const bool lo = (threadIdx.x & off) == 0;
      a.p = lo ? v[k].p : op; a.s = lo ? v[k].s : os;
      b.p = lo ? op : v[k].p; b.s = lo ? os : v[k].s;
      a.merge(b.p, b.s);
      v[k] = a;
    }
  }
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < NV; ++k) { lds[k * 2 * W + wave * 2] = v[k].p; lds[k * 2 * W + wave * 2 + 1] = v[k].s; }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    Dot2 a;
    a.p = lds[k * 2 * W + 0]; a.s = lds[k * 2 * W + 1];
    for (int w = 1; w < W; ++w) a.merge(lds[k * 2 * W + 2 * w], lds[k * 2 * W + 2 * w + 1]);
    v[k] = a;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------------------
// CSR row product by a group of G lanes; every lane of the group returns the row sum.  U
// strided entries per lane per trip (consecutive lanes on consecutive entries, so each gather
// instruction reads the x values of a run of sorted columns), with indices clamped into the
// row so that the U column loads and the U x gathers are issued together (entries past the
// row end are gathered but multiplied by zero).  Column indices of type I: int, or uint16_t
// for a matrix of at most 65,536 columns.
template <typename T, int G, typename I = int, int U = 4>
__device__ __forceinline__ T row_product(const int* __restrict__ rp, const I* __restrict__ ci,
                                         const T* __restrict__ av, const T* __restrict__ x, int row,
                                         int lane) {
  T s = T(0);
  const int beg = rp[row], end = rp[row + 1];
  if (end > beg) {
    for (int k = beg + lane; k < end; k += U * G) {
      int kk[U], c[U];
      T v[U], xv[U];
#pragma unroll
      for (int j = 0; j < U; ++j) kk[j] = min(k + j * G, end - 1);
#pragma unroll
      for (int j = 0; j < U; ++j) { c[j] = (int)ci[kk[j]]; v[j] = av[kk[j]]; }
#pragma unroll
      for (int j = 0; j < U; ++j) xv[j] = x[c[j]];
#pragma unroll
      for (int j = 0; j < U; ++j) s += (k + j * G < end) ? v[j] * xv[j] : T(0);
    }
  }
#pragma unroll
  for (int off = G / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, G);
  return s;
}

// Operations fused into the CSR product (epilogue at row i, s = (A x)_i, x the product input):
enum SpOp : int {
  OP_Y = 0,        // y = s
  OP_ADDY,         // y += s                                   (prolongation + correction)
  OP_RESID,        // y = f - s                                (residual)
  OP_RESTRICT,     // y = s; y2 = c0 dinv2 s; xs = y2 if set   (restriction + first smoothing
                   //                                           step of the next level)
  OP_CHEB_FIRST,   // r1 = f - s; dn = c1 x + c2 dinv r1; xs = x + dn; [r = r1; y2 = dn]
                   //                                          (pre-smoothing from zero, step 1)
  OP_CHEB_POST0,   // r = f - s; y2 = c0 dinv r                (post-smoothing, step 0)
  OP_CHEB_STEP,    // r1 = r - s; dn = c1 x + c2 dinv r1; xs += [x] + dn; [r = r1; y2 = dn]
  OP_JACOBI,       // y = x + c0 dinv (f - s)                  (Richardson-Jacobi sweep)
  OP_CG_Q,         // y = s; partial x^T s; last block: alpha  (outer CG product q = A p)
  OP_INIT_RESID,   // y = (b - mu_b) - s; partials |b^|^2, |y|^2 (initial residual)
  OP_TRUE_RESID,   // partial |(b - mu_b) - s|^2               (true residual at exit)
};

// Level-0 reductions fused into the last V-cycle kernel (OP_CHEB_STEP) or run alone.
enum VcRed : int { RED_NONE = 0, RED_F64 = 1, RED_F32 = 2 };

// Stored diagonals of the symmetric diagonal form: offset 0 and the 13 positive column - row
// offsets of a 27-point stencil.
constexpr int kDiagK = 14;

template <typename T>
struct SpArgs {
  const int* rp;
  const int* ci;          // 32-bit column indices (null when cs is used)
  const uint16_t* cs;     // CSR-stream only: column - cbase[tile], or null
  const int* cbase;       // CSR-stream only: per-tile column base, with cs
  const uint32_t* c24;    // CSR-stream only: 24-bit column indices (entries 4q.. in words 3q..), or null
  const uint8_t* cd;      // CSR-stream only: index into dict of column - row, or null
  const int* dict;        // the distinct column - row offsets (at most 256), with cd
  int ndict;
  int ncols;
  const T* av;
  int nrows;
  int tpb;           // row tiles per block (row-group kernel); chunks per plane S (diagonal form)
  const T* x;        // product input (also the pointwise direction d of the Chebyshev steps)
  T* y;              // output
  T* y2;             // second output
  const T* f;        // right-hand side
  T* r;              // residual in/out
  T* xs;             // iterate in/out
  const T* dinv;     // 1 / diag of this matrix's level
  const T* dinv2;    // OP_RESTRICT: 1 / diag of the next level
  T c0, c1, c2;
  int add_d;         // OP_CHEB_STEP: also add x_i (the deferred step 0 of post-smoothing)
  int store_rd;      // OP_CHEB_FIRST / OP_CHEB_STEP: store r1 into r and dn into y2
  int rev;           // walk the tiles in reverse order (single-matrix product kernels; see k_spmv_sdia)
  Solve sv;
  int red;           // VcRed (OP_CHEB_STEP only)
  const double* b;   // OP_INIT_RESID / OP_TRUE_RESID: the caller's right-hand side
  const double* r64;     // RED_F64: the CG residual (level-0 right-hand side)
  const float* r32;      // RED_F32: current level-0 right-hand side
  const float* r32_old;  // RED_F32: previous level-0 right-hand side
  // symmetric diagonal form only: diagonal o (offset doff[o] >= 0) at dv + o * ds
  const T* dv;
  int64_t ds;
  int doff[kDiagK];
};

template <typename T>
struct VcAcc {
  double acc[3] = {0.0, 0.0, 0.0};
  Dot2 dd[2];
  // z: the V-cycle output at a row; rr: the CG residual there (RED_F64); r32 / r32o: the
  // current and previous level-0 right-hand sides (RED_F32)
  __device__ __forceinline__ void add(int red, double z64, float z32, double rr, float r32, float r32o) {
    if (red == RED_F64) {
      acc[0] += z64;
      acc[1] += rr * z64;
      acc[2] += rr;
    } else if (red == RED_F32) {
      dd[0].add(z32, r32);
      dd[1].add(z32, r32o);
      acc[0] += (double)z32;
    }
  }
};

template <typename T>
__device__ void vc_partials(VcAcc<T>& v, int red, const Solve& sv, int bi, int nb, double* lds, float* lds32);

// Row operands of the fused epilogue, read right after the gathers so that their latency
// overlaps the product's.  Every field an OP uses is read from a valid address whatever the
// run-time flags (unused reduction operands read solve scalar 0), so the reads are
// unconditional and never split the kernel's load sequence into branches.
template <typename T>
struct RowIn {
  T f = T(0), x = T(0), dinv = T(0), r = T(0), xs = T(0), y = T(0);
  double r64 = 0.0, b = 0.0;
  float r32 = 0.f, r32o = 0.f;
};

template <typename T, int OP>
__device__ __forceinline__ RowIn<T> row_fetch(const SpArgs<T>& a, int row) {
  RowIn<T> in;
  if constexpr (OP == OP_ADDY) {
    in.y = a.y[row];
  } else if constexpr (OP == OP_RESID) {
    in.f = a.f[row];
  } else if constexpr (OP == OP_RESTRICT) {
    in.dinv = a.dinv2[row];
  } else if constexpr (OP == OP_CHEB_FIRST || OP == OP_JACOBI) {
    in.f = a.f[row];
    in.x = a.x[row];
    in.dinv = a.dinv[row];
  } else if constexpr (OP == OP_CHEB_POST0) {
    in.f = a.f[row];
    in.dinv = a.dinv[row];
  } else if constexpr (OP == OP_CHEB_STEP) {
    in.r = a.r[row];
    in.x = a.x[row];
    in.dinv = a.dinv[row];
    in.xs = a.xs[row];
    const bool f64 = a.red == RED_F64, f32 = a.red == RED_F32;
    const float* s32 = reinterpret_cast<const float*>(a.sv.sc);
    in.r64 = (f64 ? a.r64 : a.sv.sc)[f64 ? row : 0];
    in.r32 = (f32 ? a.r32 : s32)[f32 ? row : 0];
    in.r32o = (f32 ? a.r32_old : s32)[f32 ? row : 0];
  } else if constexpr (OP == OP_CG_Q) {
    in.x = a.x[row];
  } else if constexpr (OP == OP_INIT_RESID || OP == OP_TRUE_RESID) {
    in.b = a.b[row];
  }
  return in;
}

// Fused epilogue of one row (s = (A x)_row, in = row_fetch of the same row); reduction terms
// accumulate in acc / vc.  The reduction operands are never stored by the same launch (the
// host does not combine store_rd with a level-0 reduction), so reading them first is exact.
template <typename T, int OP>
__device__ __forceinline__ void row_apply(const SpArgs<T>& a, int row, T s, const RowIn<T>& in, double (&acc)[3],
                                          VcAcc<T>& vc) {
  if constexpr (OP == OP_Y) {
    a.y[row] = s;
  } else if constexpr (OP == OP_ADDY) {
    a.y[row] = in.y + s;
  } else if constexpr (OP == OP_RESID) {
    a.y[row] = in.f - s;
  } else if constexpr (OP == OP_RESTRICT) {
    a.y[row] = s;
    const T d = a.c0 * in.dinv * s;
    a.y2[row] = d;
    if (a.xs) a.xs[row] = d;
  } else if constexpr (OP == OP_CHEB_FIRST) {
    const T r1 = in.f - s;
    const T d = in.x;
    const T dn = a.c1 * d + a.c2 * in.dinv * r1;
    a.xs[row] = d + dn;
    if (a.store_rd) { a.r[row] = r1; a.y2[row] = dn; }
  } else if constexpr (OP == OP_CHEB_POST0) {
    const T r0 = in.f - s;
    a.r[row] = r0;
    a.y2[row] = a.c0 * in.dinv * r0;
  } else if constexpr (OP == OP_CHEB_STEP) {
    const T r1 = in.r - s;
    const T d = in.x;
    const T dn = a.c1 * d + a.c2 * in.dinv * r1;
    const T xn = in.xs + (a.add_d ? d + dn : dn);
    a.xs[row] = xn;
    if (a.store_rd) { a.r[row] = r1; a.y2[row] = dn; }
    vc.add(a.red, (double)xn, (float)xn, in.r64, in.r32, in.r32o);
  } else if constexpr (OP == OP_JACOBI) {
    a.y[row] = in.x + a.c0 * in.dinv * (in.f - s);
  } else if constexpr (OP == OP_CG_Q) {
    a.y[row] = s;
    acc[0] += (double)in.x * (double)s;
  } else if constexpr (OP == OP_INIT_RESID) {
    const double bh = in.b - a.sv.sc[S_MU_B];
    const double rr = bh - (double)s;
    a.y[row] = (T)rr;
    acc[0] += bh * bh;
    acc[1] += rr * rr;
  } else if constexpr (OP == OP_TRUE_RESID) {
    const double rr = (in.b - a.sv.sc[S_MU_B]) - (double)s;
    acc[0] += rr * rr;
  }
}

template <typename T, int OP>
__device__ __forceinline__ void row_epilogue(const SpArgs<T>& a, int row, T s, double (&acc)[3], VcAcc<T>& vc) {
  row_apply<T, OP>(a, row, s, row_fetch<T, OP>(a, row), acc, vc);
}

// Block partials of the reducing ops (finalized by k_finalize).  Called by every thread.
template <typename T, int OP>
__device__ __forceinline__ void block_tail(const SpArgs<T>& a, double (&acc)[3], VcAcc<T>& vc, int bi, int nb,
                                           double* lds, float* lds32) {
  if constexpr (OP == OP_CG_Q || OP == OP_TRUE_RESID) {
    block_sum<1>(*reinterpret_cast<double(*)[1]>(acc), lds);
    if (threadIdx.x == 0) a.sv.part[bi] = acc[0];
  } else if constexpr (OP == OP_INIT_RESID) {
    block_sum<2>(*reinterpret_cast<double(*)[2]>(acc), lds);
    if (threadIdx.x == 0) { a.sv.part[bi] = acc[0]; a.sv.part[nb + bi] = acc[1]; }
  } else if constexpr (OP == OP_CHEB_STEP) {
    if (a.red != RED_NONE) vc_partials<T>(vc, a.red, a.sv, bi, nb, lds, lds32);
  }
}

// Row-group kernel: G lanes per row, TPB consecutive 256/G-row tiles per block.  Used for
// matrices with a row longer than the CSR-stream staging buffer (kStreamCap entries); IX16:
// 16-bit column indices (cs) for a matrix of at most 65,536 columns.  In float32, rows averaging
// more than 256 entries (G = 64: the filled coarse levels, thousands of entries a row) keep 16
// entries a lane in flight per trip; measured at 11,408 rows of 8,000 entries: 128 us a product
// against 142 us with 4 and 136 us with 8.  Float64 products gained nothing from it (within
// +-3 %) and keep 4.
template <typename T, int G, int OP, int IX = 0>
__global__ __launch_bounds__(kBlock) void k_spmv(SpArgs<T> a) {
  if (solve_done(a.sv)) return;
  __shared__ double lds[16];
  __shared__ float lds32[24];
  constexpr int RPT = kBlock / G;  // rows per tile
  const int nb = gridDim.x;
  const int bt = a.rev ? nb - 1 - xcd_tile(blockIdx.x, nb) : xcd_tile(blockIdx.x, nb);
  const int tile0 = bt * a.tpb;
  const int grp = threadIdx.x / G, lane = threadIdx.x % G;
  double acc[3] = {0.0, 0.0, 0.0};
  VcAcc<T> vc;
  for (int t = 0; t < a.tpb; ++t) {
    const int row = (tile0 + t) * RPT + grp;
    if (row >= a.nrows) break;
    T s;
    constexpr int U = G == 64 && sizeof(T) == 4 ? 16 : 4;
    if constexpr (IX == 1) s = row_product<T, G, uint16_t, U>(a.rp, a.cs, a.av, a.x, row, lane);
    else s = row_product<T, G, int, U>(a.rp, a.ci, a.av, a.x, row, lane);
    if (lane == 0) row_epilogue<T, OP>(a, row, s, acc, vc);
  }
  block_tail<T, OP>(a, acc, vc, bt, nb, lds, lds32);
}

// CSR-stream kernel (after Greathouse & Daga, SC'14): tile b owns rows [blk[b], blk[b+1]),
// at most kStreamRows rows whose nonzeros fit in kStreamCap.  Phase 1 streams the tile's
// contiguous value/column range with consecutive lanes on consecutive entries (every load
// instruction covers one contiguous span) and stages the products a_k x_{c_k} in LDS;
// phase 2 reduces each row from LDS with a power-of-two lane group (or, in a tile of more than
// kBlock rows, one thread for two rows) and applies the epilogue.
// 4028 entries: the staging buffer (kStageLen doubles) plus the reduction scratch stay within
// 32 KiB of LDS, so five blocks fit a CU's 160 KiB (4 aligned 4-entry chunks per thread)
constexpr int kStreamCap = 4028;
// Rows of a tile: up to two a thread in phase 2 (one thread a row, each taking a second row
// kBlock further on) -- a prolongator's rows of ~7 entries fill 512-row tiles to 90 % of the
// staging buffer, 256-row ones to 45 % (the 14.4 M-row fine prolongator of the
// 384 x 384 x 96 slab: 266 -> 242 us a product).  Dictionary tiles keep a lane group a row.
constexpr int kStreamRows = 2 * kBlock;
constexpr int kStreamRowsD = kBlock;
constexpr int kStreamPad = 4;   // value/column arrays carry this many padding entries
// aligned 4-entry chunks spanned by kStreamCap entries at the worst alignment, per thread
constexpr int kStreamChunks = ((kStreamCap + 2) / 4 + 1 + kBlock - 1) / kBlock;
static_assert((kStreamCap + 2) / 4 + 1 <= kStreamChunks * kBlock, "chunks must cover an unaligned tile");

// Four consecutive matrix entries with 16-byte loads (entry index a multiple of 4).
__device__ __forceinline__ void load4(const double* p, double (&v)[4]) {
  const double2 a = *reinterpret_cast<const double2*>(p);
  const double2 b = *reinterpret_cast<const double2*>(p + 2);
  v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
}
__device__ __forceinline__ void load4(const float* p, float (&v)[4]) {
  const float4 a = *reinterpret_cast<const float4*>(p);
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
}

// Rows and entry range of one tile, plus the row-offset pair of this thread's phase-2 row.
struct Tile {
  int r0, r1, beg, end;
  int cb;      // column base of the tile's 16-bit column offsets (0 with 32-bit indices)
  int k0;      // beg rounded down to a multiple of 4: LDS slot 0 holds entry k0
  int lo, hi;  // rp[row], rp[row + 1] of this thread's phase-2 row
  int g;       // lanes per row in phase 2: a power of two, at most 64
};

// Matrix entries of one tile held in registers between phase 1's loads and its gathers:
// four 32-bit column indices per chunk, (16-bit offsets) two words of two offsets each, or
// (24-bit indices) the three words that pack the chunk's four indices.
template <typename T>
struct TileRegs {
  int c[kStreamChunks][4];
  T v[kStreamChunks][4];
};

// LDS entries of the product staging buffer: slot k - k0 of every chunk a tile of at most
// kStreamCap entries spans at the worst alignment (clamped chunks reuse the last slot).
constexpr int kStageLen = 4 * ((kStreamCap + 2) / 4 + 1);
static_assert(kStageLen <= kStreamChunks * 4 * kBlock, "every spanned chunk has a thread");

// Column index forms of a CSR-stream matrix: 32-bit indices; 16-bit offsets from a per-tile
// base; for matrices whose column - row offsets take at most 256 distinct values (the
// stencil operators of a structured mesh), an 8-bit index into that offset dictionary; or,
// where tiles span too many columns for 16-bit offsets and the matrix has at most 2^24
// columns, 24-bit column indices (four entries in three 32-bit words).
// SDIA: the symmetric diagonal form (k_spmv_sdia), no column indices at all.
enum IdxForm : int { IX32 = 0, IX16 = 1, IXD8 = 2, IX24 = 3, SDIA = 4, kForms = 5 };
constexpr int kMaxCols24 = 1 << 24;

// Three 32-bit words at 4-byte alignment (one load of 12 bytes): the 24-bit indices of four
// consecutive entries, entry j in bits 24 j .. 24 j + 23 of the 96-bit little-endian word.
struct __attribute__((aligned(4))) Words3 {
  uint32_t w0, w1, w2;
};
// Dictionary tiles stage values, index bytes and the dictionary in LDS: a smaller cap keeps
// the float64 total within the other forms' staging buffer.
constexpr int kStreamCapD = 3450;
constexpr int kStageLenD = 4 * ((kStreamCapD + 2) / 4 + 1);
constexpr int kDictMax = 256;
static_assert(kStageLenD <= kStreamChunks * 4 * kBlock, "every spanned chunk has a thread");
static_assert(kDictMax <= kBlock, "one thread per dictionary entry");
template <typename T>
constexpr int smem_bytes() {
  const int a = kStageLen * (int)sizeof(T);
  const int b = kStageLenD * ((int)sizeof(T) + 1) + kDictMax * 4;
  return a > b ? a : b;
}

template <int IX>
__device__ __forceinline__ Tile tile_open(const int* __restrict__ rp, const int* __restrict__ blk,
                                          const int* __restrict__ cbase, int b) {
  Tile t;
  t.r0 = blk[b];
  t.r1 = blk[b + 1];
  t.beg = rp[t.r0];
  t.end = rp[t.r1];
  t.cb = IX == IX16 ? cbase[b] : 0;
  t.k0 = t.beg & ~3;
  const int nrow = t.r1 - t.r0;
  int g = kBlock / (nrow > 0 ? nrow : 1);
  t.g = g >= 64 ? 64 : (g >= 32 ? 32 : (g >= 16 ? 16 : (g >= 8 ? 8 : (g >= 4 ? 4 : (g >= 2 ? 2 : 1)))));
  // this thread's phase-2 row, clamped into the tile so that the reads are unconditional
  const int row = min(t.r0 + (int)threadIdx.x / t.g, t.r1 - 1);
  t.lo = rp[row];
  t.hi = rp[row + 1];
  return t;
}

// Phase 1, loads: the 4-entry chunks (aligned to 4) spanning the tile's entries [beg, end).
// Branch-free so that every chunk load is in flight at once: chunk positions past the tile are
// clamped to its last chunk.  Entries outside [beg, end) are neighbouring rows' or the zero
// padding of the arrays (kStreamPad entries past nnz), so every 32-bit column index is valid;
// IX16 (16-bit offsets): offsets of a neighbouring tile decode against this tile's base and are
// clamped into [0, ncols) at the gather.  The index form is a template parameter: a run-time
// branch around the loads made the compiler wait for them at the join.
template <typename T, int IX>
__device__ __forceinline__ void tile_load(const SpArgs<T>& a, const Tile& t, TileRegs<T>& R) {
  const int klast = max(t.k0, (t.end - 1) & ~3);
#pragma unroll
  for (int c = 0; c < kStreamChunks; ++c) {
    const int k = min(t.k0 + 4 * ((int)threadIdx.x + kBlock * c), klast);
    if constexpr (IX == IX16) {
      const uint2 cc = *reinterpret_cast<const uint2*>(a.cs + k);
      R.c[c][0] = (int)cc.x; R.c[c][1] = (int)cc.y;
    } else if constexpr (IX == IX24) {
      const Words3 cc = *reinterpret_cast<const Words3*>(a.c24 + 3 * (k >> 2));
      R.c[c][0] = (int)cc.w0; R.c[c][1] = (int)cc.w1; R.c[c][2] = (int)cc.w2;
    } else {
      const int4 cc = *reinterpret_cast<const int4*>(a.ci + k);
      R.c[c][0] = cc.x; R.c[c][1] = cc.y; R.c[c][2] = cc.z; R.c[c][3] = cc.w;
    }
    load4(a.av + k, R.v[c]);
  }
}

// Phase 1, gathers of x at the loaded columns (issued together).
template <typename T, int IX>
__device__ __forceinline__ void tile_gather(const SpArgs<T>& a, const Tile& t, const TileRegs<T>& R,
                                            T (&xv)[kStreamChunks][4]) {
  if constexpr (IX == IX16) {
    const int cmax = a.ncols - 1;
#pragma unroll
    for (int c = 0; c < kStreamChunks; ++c) {
      const unsigned w0 = (unsigned)R.c[c][0], w1 = (unsigned)R.c[c][1];
      xv[c][0] = a.x[min(t.cb + (int)(w0 & 0xffffu), cmax)];
      xv[c][1] = a.x[min(t.cb + (int)(w0 >> 16), cmax)];
      xv[c][2] = a.x[min(t.cb + (int)(w1 & 0xffffu), cmax)];
      xv[c][3] = a.x[min(t.cb + (int)(w1 >> 16), cmax)];
    }
  } else if constexpr (IX == IX24) {
    // every packed index is a column of the matrix (neighbouring rows' or the zero padding)
#pragma unroll
    for (int c = 0; c < kStreamChunks; ++c) {
      const unsigned w0 = (unsigned)R.c[c][0], w1 = (unsigned)R.c[c][1], w2 = (unsigned)R.c[c][2];
      xv[c][0] = a.x[w0 & 0xffffffu];
      xv[c][1] = a.x[(w0 >> 24) | ((w1 & 0xffffu) << 8)];
      xv[c][2] = a.x[(w1 >> 16) | ((w2 & 0xffu) << 16)];
      xv[c][3] = a.x[w2 >> 8];
    }
  } else {
#pragma unroll
    for (int c = 0; c < kStreamChunks; ++c)
#pragma unroll
      for (int j = 0; j < 4; ++j) xv[c][j] = a.x[R.c[c][j]];
  }
}

// Phase 1, products a_k x_{c_k} into LDS slot k - k0.  Every chunk is stored whole: entries of
// neighbouring rows land in slots phase 2 does not read, and a clamped chunk rewrites the
// tile's last chunk with identical values.
template <typename T>
__device__ __forceinline__ void tile_stage(const Tile& t, const TileRegs<T>& R, const T (&xv)[kStreamChunks][4],
                                           T* prod) {
  const int klast = max(t.k0, (t.end - 1) & ~3);
#pragma unroll
  for (int c = 0; c < kStreamChunks; ++c) {
    const int k = min(t.k0 + 4 * ((int)threadIdx.x + kBlock * c), klast) - t.k0;
#pragma unroll
    for (int j = 0; j < 4; ++j) prod[k + j] = R.v[c][j] * xv[c][j];
  }
}

// This thread's phase-2 row (clamped into the tile) and its epilogue operands.
template <typename T, int OP>
__device__ __forceinline__ RowIn<T> tile_fetch(const SpArgs<T>& a, const Tile& t) {
  return row_fetch<T, OP>(a, min(t.r0 + (int)threadIdx.x / t.g, t.r1 - 1));
}

// Phase 2 tail: the lane group's row sum s (every lane holds it after the shuffles), the fused
// epilogue, and the tile's reduction partials (slot bi of nb).  Called by every thread.
template <typename T, int OP>
__device__ __forceinline__ void tile_finish(const SpArgs<T>& a, const Tile& t, const RowIn<T>& in, T s, int bi,
                                            int nb, double* lds, float* lds32) {
  const int grp = threadIdx.x / t.g, lane = threadIdx.x % t.g;
  double acc[3] = {0.0, 0.0, 0.0};
  VcAcc<T> vc;
  for (int off = t.g / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, t.g);
  if (grp < t.r1 - t.r0 && lane == 0) row_apply<T, OP>(a, t.r0 + grp, s, in, acc, vc);
  block_tail<T, OP>(a, acc, vc, bi, nb, lds, lds32);
}

// Phase 2: row sums of the staged products, then tile_finish.  Called by every thread after a
// barrier that follows tile_stage.
template <typename T, int OP>
__device__ __forceinline__ void tile_reduce(const SpArgs<T>& a, const Tile& t, const RowIn<T>& in, int bi, int nb,
                                            const T* prod, double* lds, float* lds32) {
  const int grp = threadIdx.x / t.g, lane = threadIdx.x % t.g;
  const int hi = grp < t.r1 - t.r0 ? t.hi - t.k0 : 0;
  // four independent partial sums: a row of 27 entries on one lane is 7 LDS round trips, not 27
  T s0 = T(0), s1 = T(0), s2 = T(0), s3 = T(0);
  int k = t.lo - t.k0 + lane;
  for (; k + 3 * t.g < hi; k += 4 * t.g) {
    s0 += prod[k];
    s1 += prod[k + t.g];
    s2 += prod[k + 2 * t.g];
    s3 += prod[k + 3 * t.g];
  }
  for (; k < hi; k += t.g) s0 += prod[k];
  if (t.r1 - t.r0 > kBlock) {  // the same for the whole block: rows r0 + tid and r0 + tid + kBlock
    double acc[3] = {0.0, 0.0, 0.0};
    VcAcc<T> vc;
    row_apply<T, OP>(a, t.r0 + (int)threadIdx.x, (s0 + s1) + (s2 + s3), in, acc, vc);
    const int row2 = t.r0 + (int)threadIdx.x + kBlock;
    if (row2 < t.r1) {
      const RowIn<T> in2 = row_fetch<T, OP>(a, row2);
      const int hi2 = a.rp[row2 + 1] - t.k0;
      T u0 = T(0), u1 = T(0), u2 = T(0), u3 = T(0);
      int q = a.rp[row2] - t.k0;
      for (; q + 3 < hi2; q += 4) {
        u0 += prod[q];
        u1 += prod[q + 1];
        u2 += prod[q + 2];
        u3 += prod[q + 3];
      }
      for (; q < hi2; ++q) u0 += prod[q];
      row_apply<T, OP>(a, row2, (u0 + u1) + (u2 + u3), in2, acc, vc);
    }
    block_tail<T, OP>(a, acc, vc, bi, nb, lds, lds32);
    return;
  }
  tile_finish<T, OP>(a, t, in, (s0 + s1) + (s2 + s3), bi, nb, lds, lds32);
}

// Dictionary form.  Phase 1 streams the tile's values and index bytes into LDS (no gathers:
// an entry's row is not known there); phase 2 runs a lane group per row, so lanes on
// consecutive rows gather x at the same offset from their rows -- consecutive addresses.
// Only the rows' own entries are read, so every gather is in bounds.
template <typename T>
__device__ __forceinline__ void dict_stage(const SpArgs<T>& a, const Tile& t, T* vals, uint8_t* idxs, int* dict) {
  const int klast = max(t.k0, (t.end - 1) & ~3);
  // the dictionary entry is read first and stored last, so no wait for it holds the chunk
  // loads back
  const int dv = a.dict[min((int)threadIdx.x, a.ndict - 1)];
  T v[kStreamChunks][4];
  uint32_t ix[kStreamChunks];
#pragma unroll
  for (int c = 0; c < kStreamChunks; ++c) {
    const int k = min(t.k0 + 4 * ((int)threadIdx.x + kBlock * c), klast);
    ix[c] = *reinterpret_cast<const uint32_t*>(a.cd + k);
    load4(a.av + k, v[c]);
  }
#pragma unroll
  for (int c = 0; c < kStreamChunks; ++c) {
    const int k = min(t.k0 + 4 * ((int)threadIdx.x + kBlock * c), klast) - t.k0;
#pragma unroll
    for (int j = 0; j < 4; ++j) vals[k + j] = v[c][j];
    *reinterpret_cast<uint32_t*>(idxs + k) = ix[c];
  }
  if ((int)threadIdx.x < a.ndict) dict[threadIdx.x] = dv;
}

// Entries per lane whose index, offset and x reads are issued together in phase 2.
constexpr int kDictBatch = 16;

template <typename T, int OP>
__device__ __forceinline__ void dict_reduce(const SpArgs<T>& a, const Tile& t, const RowIn<T>& in, int bi, int nb,
                                            const T* vals, const uint8_t* idxs, const int* dict, double* lds,
                                            float* lds32) {
  const int grp = threadIdx.x / t.g, lane = threadIdx.x % t.g;
  const int row = t.r0 + grp;
  const int hi = grp < t.r1 - t.r0 ? t.hi - t.k0 : 0;
  const T* __restrict__ x = a.x;
  T acc[4] = {T(0), T(0), T(0), T(0)};
  for (int kb = t.lo - t.k0 + lane; kb < hi; kb += kDictBatch * t.g) {
    // positions past the row's end are clamped to its last entry (a valid column) and weighted 0
    T v[kDictBatch];
    int off[kDictBatch];
#pragma unroll
    for (int u = 0; u < kDictBatch; ++u) {
      const int k = kb + u * t.g;
      const int kc = min(k, hi - 1);
      v[u] = k < hi ? vals[kc] : T(0);
      off[u] = idxs[kc];
    }
#pragma unroll
    for (int u = 0; u < kDictBatch; ++u) off[u] = dict[off[u]];
    T xv[kDictBatch];
#pragma unroll
    for (int u = 0; u < kDictBatch; ++u) xv[u] = x[row + off[u]];
#pragma unroll
    for (int u = 0; u < kDictBatch; ++u) acc[u & 3] += v[u] * xv[u];
  }
  tile_finish<T, OP>(a, t, in, (acc[0] + acc[1]) + (acc[2] + acc[3]), bi, nb, lds, lds32);
}

// Body of the CSR-stream product for row tile b of nb (b also indexes the block partials), in
// index form IX; smem holds smem_bytes<T>() bytes of staging.
// (Testing the solve's done flag only after the tile's vector reads are issued measured
// slower: the branch keeps every loaded register live across it.)
template <typename T, int OP, int IX>
__device__ __forceinline__ void stream_body(const SpArgs<T>& a, const int* __restrict__ blk, int b, int nb,
                                            unsigned char* smem, double* lds, float* lds32) {
  // The done flag (written by an earlier kernel, so a plain load sees it) is read together
  // with the tile bounds and tested before any vector load: one scalar round trip fewer.
  const int done = a.sv.fl[F_DONE];
  const Tile t = tile_open<IX>(a.rp, blk, a.cbase, b);
  if (done) return;
  if constexpr (IX == IXD8) {
    T* vals = reinterpret_cast<T*>(smem);
    uint8_t* idxs = reinterpret_cast<uint8_t*>(vals + kStageLenD);
    int* dict = reinterpret_cast<int*>(idxs + kStageLenD);
    const RowIn<T> in = tile_fetch<T, OP>(a, t);  // first: phase 1 has no gathers to hide it behind
    dict_stage(a, t, vals, idxs, dict);
    __syncthreads();
    dict_reduce<T, OP>(a, t, in, b, nb, vals, idxs, dict, lds, lds32);
  } else {
    T* prod = reinterpret_cast<T*>(smem);
    TileRegs<T> R;
    T xv[kStreamChunks][4];
    tile_load<T, IX>(a, t, R);
    tile_gather<T, IX>(a, t, R, xv);
    const RowIn<T> in = tile_fetch<T, OP>(a, t);
    tile_stage(t, R, xv, prod);
    __syncthreads();
    tile_reduce<T, OP>(a, t, in, b, nb, prod, lds, lds32);
  }
}

template <typename T, int OP, int IX>
__global__ __launch_bounds__(kBlock) void k_spmv_stream(SpArgs<T> a, const int* __restrict__ blk) {
  __shared__ double lds[16];
  __shared__ float lds32[24];
  __shared__ __align__(16) unsigned char smem[smem_bytes<T>()];
  const int b = xcd_tile(blockIdx.x, gridDim.x);
  stream_body<T, OP, IX>(a, blk, a.rev ? (int)gridDim.x - 1 - b : b, gridDim.x, smem, lds, lds32);
}

// ---------------------------------------------------------------------------------------
// Symmetric diagonal product.  A matrix equal to its transpose whose column - row offsets
// take at most 2 kDiagK - 1 values, symmetric about zero (27 for the 27-point stencil of a
// structured hexahedral mesh), is stored as its diagonals of offset d_o >= 0 only:
// dv[o * ds + i] = a(i, i + d_o), zero where that entry does not exist.  Row i takes
// a(i, i + d_o) from dv[o][i] and a(i, i - d_o) = a(i - d_o, i) from dv[o][i - d_o].  One row
// per lane: the value streams are contiguous across a wave's consecutive rows, so the product
// reads no column indices or row pointers, stages nothing in LDS, and moves 14 values per row
// from HBM instead of 27; the shifted second read of each diagonal comes from cache (a lane's
// own rows or those of recent blocks of the same XCD).  Indices past either end are clamped and
// their terms weighted by zero (the stored value there is zero; each diagonal holds at least
// one zero slot past row n - 1).
//
// The 27 gathers of x fall into 9 triples x[i + C - 1], x[i + C], x[i + C + 1] around the
// centres C = 0, +-C_1 .. +-C_4 (the plan accepts the form only for offsets
// {0, 1, C_t - 1, C_t, C_t + 1}).  Each lane loads x[i + C] only; its neighbours are the values
// of the adjacent lanes (rows i - 1, i + 1), moved by DPP wave shifts, and the two that fall
// outside the wave come from scalar loads at wave-uniform addresses.  Likewise a(i, i - 1) is
// the previous lane's a(i - 1, i).  That leaves 35 vector loads a row instead of 54 (the form
// with 54 kept the texture units busy 96 % of the kernel).  Halving them again -- two rows a
// lane, 8-byte float32 loads -- measured only 3 % faster on a 14.4 M-row grid (16 % where the
// diagonals are cache-resident), so at scale the 27 offset streams' memory latency, not the
// instruction count, keeps the product below a plain stream's rate.
template <typename T, int CTRL>
__device__ __forceinline__ T lane_move(T v) {
  if constexpr (sizeof(T) == 8) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
  } else {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
  }
}
constexpr int kDppFromPrev = 0x138;  // wave_shr:1, lane l receives lane l - 1
constexpr int kDppFromNext = 0x130;  // wave_shl:1, lane l receives lane l + 1

__device__ __forceinline__ int clamp_index(long v, int n) { return (int)(v < 0 ? 0 : (v > n - 1 ? n - 1 : v)); }

// An empty asm statement that takes v as an input: v must be computed at this point of the
// program (no code is emitted for the statement itself).
template <typename T>
__device__ __forceinline__ void pin_value(T v) {
  __asm__ volatile("" ::"v"(v));
}
template <typename T>
__device__ __forceinline__ void pin_row(const RowIn<T>& in) {
  pin_value(in.f); pin_value(in.x); pin_value(in.dinv); pin_value(in.r); pin_value(in.xs); pin_value(in.y);
  pin_value(in.r64); pin_value(in.b); pin_value(in.r32); pin_value(in.r32o);
}

// Called by every lane of the wave (rows past n included: the lane shifts need all 64), which
// stores only for rows below n.
template <typename T, int OP>
__device__ __forceinline__ void sdia_row(const SpArgs<T>& a, int row, double (&acc)[3], VcAcc<T>& vc) {
  const int n = a.nrows;
  const int lane = (int)threadIdx.x & 63;
  const int wb = __builtin_amdgcn_readfirstlane(row - lane);  // the wave's first row
  const T* __restrict__ dv = a.dv;
  const T* __restrict__ x = a.x;
  const int64_t ds = a.ds;
  T vu[kDiagK], vl[kDiagK];
  const int ru = min(row, n);
#pragma unroll
  for (int o = 0; o < kDiagK; ++o) vu[o] = dv[o * ds + ru];
#pragma unroll
  for (int o = 2; o < kDiagK; ++o) {
    // before the first row (and past the last) the index points at the zero slot n, so every
    // term is a plain product (a select on the product let the compiler sink loads into a branch)
    const int j = row - a.doff[o];
    vl[o] = dv[o * ds + (j < 0 ? n : min(j, n))];
  }
  // centres 0, +C_1, -C_1, ..., +C_4, -C_4 (C_t = doff[3 t])
  T xm[9], xe0[9], xe1[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    const int cen = t == 0 ? 0 : ((t & 1) ? a.doff[3 * ((t + 1) / 2)] : -a.doff[3 * (t / 2)]);
    xm[t] = x[clamp_index((long)row + cen, n)];
    xe0[t] = x[clamp_index((long)wb + cen - 1, n)];   // row wb - 1 + C: lane 0's left neighbour
    xe1[t] = x[clamp_index((long)wb + 64 + cen, n)];  // row wb + 64 + C: lane 63's right neighbour
  }
  const T vl1e = dv[ds + (wb >= 1 ? min(wb - 1, n) : n)];
  const RowIn<T> in = row_fetch<T, OP>(a, min(row, n - 1));
  T xl[9], xr[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    const T pl = lane_move<T, kDppFromPrev>(xm[t]), pr = lane_move<T, kDppFromNext>(xm[t]);
    xl[t] = lane == 0 ? xe0[t] : pl;
    xr[t] = lane == 63 ? xe1[t] : pr;
  }
  {
    const T p1 = lane_move<T, kDppFromPrev>(vu[1]);
    vl[1] = lane == 0 ? vl1e : p1;
  }
  // d = 0, 1 and the mirror of 1; then per centre C_t the offsets C_t - 1, C_t, C_t + 1 above
  // (left, middle, right of +C_t) and below (right, middle, left of -C_t)
  T s[4] = {vu[0] * xm[0], vu[1] * xr[0], T(0), vl[1] * xl[0]};
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int o = 2 + 3 * t, cu = 1 + 2 * t, cl = 2 + 2 * t;
    s[(o + 0) & 3] += vu[o] * xl[cu];
    s[(o + 1) & 3] += vu[o + 1] * xm[cu];
    s[(o + 2) & 3] += vu[o + 2] * xr[cu];
    s[(o + 2) & 3] += vl[o] * xr[cl];
    s[(o + 3) & 3] += vl[o + 1] * xm[cl];
    s[(o + 0) & 3] += vl[o + 2] * xl[cl];
  }
  const T sum = (s[0] + s[1]) + (s[2] + s[3]);
  // Only rows below n store.  Pinning the sum and the row operands here keeps their loads ahead
  // of that branch: the compiler otherwise sinks them into it and waits for each group in turn.
  pin_value(sum);
  pin_row(in);
  if (row < n) row_apply<T, OP>(a, row, sum, in, acc, vc);
}

// Block order: 256-row chunks form a grid of Z "planes" of S chunks (S chunks span at least the
// largest offset).  The sequence takes the planes in segments of kZseg, and within a segment
// walks the columns (c fixed, z increasing): a chunk's far rows i - d_o lie in the chunks
// (z - 1, c) and (z - 1, c + 1), loaded one block earlier and a few blocks later in the same
// XCD, so their second read hits that XCD's L2 (measured at C2: 143 MB fetched per product
// against 130 MB of algorithmic reads; plain row order 194 MB).  Rows stay consecutive across
// a wave: two-dimensional tiles of a grid plane fetch no less and run slower.
constexpr int kZseg = 8;

template <typename T, int OP>
__device__ __forceinline__ void sdia_body(const SpArgs<T>& a, int b, int nb, double* lds, float* lds32) {
  if (a.sv.fl[F_DONE]) return;  // written by an earlier kernel: a plain load sees it
  const int S = a.tpb, Z = nb / S;
  const int Zs = min(kZseg, Z), zseg = b / (S * Zs), z0 = zseg * Zs, Zl = min(Zs, Z - z0);
  const int rem = b - zseg * S * Zs, c = rem / Zl, z = z0 + rem % Zl;
  const int row = (z * S + c) * kBlock + (int)threadIdx.x;
  double acc[3] = {0.0, 0.0, 0.0};
  VcAcc<T> vc;
  sdia_row<T, OP>(a, row, acc, vc);
  block_tail<T, OP>(a, acc, vc, b, nb, lds, lds32);
}

// Consecutive passes over the same matrix alternate direction (rev; the CSR-stream and lane-group
// kernels do the same): the tiles a pass reads last -- still in the memory-side Infinity Cache --
// are the ones the next pass reads first.  Each tile keeps its partial-sum slot, so the order
// changes no result.  Measured on the 384 x 384 x 96 slab: 5.435 -> 5.39 ms an elliptic
// iteration with the level-0 passes alternating.
template <typename T, int OP>
__global__ __launch_bounds__(kBlock) void k_spmv_sdia(SpArgs<T> a) {
  __shared__ double lds[16];
  __shared__ float lds32[24];
  const int b = xcd_tile(blockIdx.x, gridDim.x);
  sdia_body<T, OP>(a, a.rev ? (int)gridDim.x - 1 - b : b, gridDim.x, lds, lds32);
}

// Block partials of the level-0 reductions: 1^T z, r^T z, 1^T r (RED_F64) or the two Dot2
// pairs z32.r32, z32.r32_old and 1^T z (RED_F32).
template <typename T>
__device__ void vc_partials(VcAcc<T>& v, int red, const Solve& sv, int bi, int nb, double* lds, float* lds32) {
  if (red == RED_F64) {
    block_sum<3>(v.acc, lds);
    if (threadIdx.x == 0) {
      sv.part[bi] = v.acc[0];
      sv.part[nb + bi] = v.acc[1];
      sv.part[2 * nb + bi] = v.acc[2];
    }
  } else {
    block_dot2<2>(v.dd, lds32);
    block_sum<1>(*reinterpret_cast<double(*)[1]>(v.acc), lds);
    if (threadIdx.x == 0) {
      float* pf = reinterpret_cast<float*>(sv.part + nb);
      pf[4 * bi + 0] = v.dd[0].p;
      pf[4 * bi + 1] = v.dd[0].s;
      pf[4 * bi + 2] = v.dd[1].p;
      pf[4 * bi + 3] = v.dd[1].s;
      sv.part[bi] = v.acc[0];
    }
  }
}

// The level-0 reductions on their own, for V-cycles whose last kernel is not a fused
// Chebyshev step (single-level hierarchies, Jacobi smoothing).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_vc_reduce(SpArgs<T> a, const T* __restrict__ z) {
  if (solve_done(a.sv)) return;
  __shared__ double lds[16];
  __shared__ float lds32[24];
  VcAcc<T> vc;
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < a.nrows; i += (long)gridDim.x * kBlock) {
    double rr = 0.0;
    float r32 = 0.f, r32o = 0.f;
    if (a.red == RED_F64) {
      rr = a.r64[i];
    } else if (a.red == RED_F32) {
      r32 = a.r32[i];
      r32o = a.r32_old[i];
    }
    vc.add(a.red, (double)z[i], (float)z[i], rr, r32, r32o);
  }
  vc_partials<T>(vc, a.red, a.sv, blockIdx.x, gridDim.x, lds, lds32);
}

// Diagonal preconditioners of a solve without a hierarchy: z = D^{-1} r (Jacobi) or z = r
// (none: plain CG), with the reductions of the preconditioned residual (RED_F64) fused.
__global__ __launch_bounds__(kBlock) void k_pc_diag(SpArgs<double> a, double* __restrict__ z) {
  if (solve_done(a.sv)) return;
  __shared__ double lds[16];
  __shared__ float lds32[24];
  VcAcc<double> vc;
  for (long i = (long)blockIdx.x * kBlock + threadIdx.x; i < a.nrows; i += (long)gridDim.x * kBlock) {
    const double r = a.r64[i];
    const double zi = a.dinv ? a.dinv[i] * r : r;
    z[i] = zi;
    vc.add(RED_F64, zi, 0.f, r, 0.f, 0.f);
  }
  vc_partials<double>(vc, RED_F64, a.sv, blockIdx.x, gridDim.x, lds, lds32);
}

// One block: sums the partials of the preceding kernel (nb blocks) in a fixed order and
// updates the solver scalars and flags.
//   FIN_CGQ    p^T q -> alpha = rho / p^T q            (breakdown if p^T q <= 0)
//   FIN_UPDATE ||r||^2 -> convergence / cap / non-finite, iteration count, host mirror
//   FIN_VC64   mu_z = 1^T z / n, rho = r^T (z - mu_z 1), beta = rho / rho_old
//   FIN_VC32   rho = Dot2(z32, r32), beta = (rho - Dot2(z32, r32_old)) / rho_old (flexible CG)
//   FIN_INIT   ||b^||^2, ||r0||^2 -> tolerance, early exit
//   FIN_TRUE   ||b^ - A x||^2
//   FIN_MEANS  means of b and of the initial guess (projection)
//   FIN_NORM   w^T x and 1^T w (normalisation)
template <int NT>
__device__ __forceinline__ void finalize_body(const Solve& sv, int kind, int nb, double* lds, float* lds32) {
  const bool guarded = kind == FIN_CGQ || kind == FIN_UPDATE || kind == FIN_VC64 || kind == FIN_VC32;
  // Flags and scalars are read before the partial sums so that every read is in flight at
  // once; a solve that was already done skips the updates (its partials are stale but valid
  // memory).
  const bool was_done = guarded && sv.fl[F_DONE] != 0;
  const int iters = sv.fl[F_ITERS], maxit = sv.fl[F_MAXIT];
  const bool first = sv.fl[F_FIRST] != 0, ns = sv.fl[F_NULLSPACE] != 0;
  const double rho_old = sv.sc[S_RHO], tol2_in = sv.sc[S_TOL2], rtol2 = sv.sc[S_RTOL2];
  double tot[3] = {0.0, 0.0, 0.0};
  Dot2 c[2];
  if (kind == FIN_VC64) {
    sum_partials<3, NT>(sv.part, nb, tot, lds);
  } else if (kind == FIN_INIT || kind == FIN_MEANS || kind == FIN_NORM) {
    sum_partials<2, NT>(sv.part, nb, *reinterpret_cast<double(*)[2]>(tot), lds);
  } else {
    sum_partials<1, NT>(sv.part, nb, *reinterpret_cast<double(*)[1]>(tot), lds);
  }
  if (kind == FIN_VC32) {
    // fixed order per thread (i, i + NT, ...), then a fixed tree; loads in batches
    const float* pf = reinterpret_cast<const float*>(sv.part + nb);
    for (int i0 = threadIdx.x; i0 < nb; i0 += kSumLanes * NT) {
      float v[kSumLanes][4];
#pragma unroll
      for (int u = 0; u < kSumLanes; ++u) {
        const int i = min(i0 + u * NT, nb - 1);
#pragma unroll
        for (int j = 0; j < 4; ++j) v[u][j] = pf[4 * i + j];
      }
#pragma unroll
      for (int u = 0; u < kSumLanes; ++u)
        if (i0 + u * NT < nb) {
          c[0].merge(v[u][0], v[u][1]);
          c[1].merge(v[u][2], v[u][3]);
        }
    }
    block_dot2<2, NT>(c, lds32);
  }
  const bool t0 = threadIdx.x == 0;
  if (was_done) {
    if (t0 && sv.host_flags)
      __hip_atomic_store(&sv.host_flags[0], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    return;
  }
  int iters_out = iters, done_out = 0;
  if (t0) {
    if (kind == FIN_CGQ) {
      const double pq = tot[0];
      sv.sc[S_PQ] = pq;
      if (!(pq > 0.0) || !isfinite(pq)) {
        sv.fl[F_STATUS] = isfinite(pq) ? -4 : -5;
        done_out = 1;
      } else {
        sv.sc[S_ALPHA] = rho_old / pq;
      }
    } else if (kind == FIN_UPDATE) {
      const double r2 = tot[0];
      sv.sc[S_RNORM2] = r2;
      iters_out = iters + 1;
      sv.fl[F_ITERS] = iters_out;
      if (!isfinite(r2)) { sv.fl[F_STATUS] = -5; done_out = 1; }
      else if (r2 <= tol2_in) { done_out = 1; }
      else if (iters_out >= maxit) { sv.fl[F_STATUS] = 1; done_out = 1; }
    } else if (kind == FIN_VC64 || kind == FIN_VC32) {
      double sz, rz, num;
      if (kind == FIN_VC64) {
        const double mu = ns ? tot[0] / (double)sv.n : 0.0;
        sz = tot[0];
        rz = tot[1] - mu * tot[2];
        num = rz;
      } else {
        sz = tot[0];
        rz = (double)c[0].p + (double)c[0].s;
        num = rz - ((double)c[1].p + (double)c[1].s);
      }
      sv.sc[S_MU_Z] = ns ? sz / (double)sv.n : 0.0;
      sv.sc[S_BETA] = first ? 0.0 : num / rho_old;
      sv.sc[S_RHO] = rz;
      if (!(rz > 0.0) || !isfinite(rz)) {
        sv.fl[F_STATUS] = isfinite(rz) ? -4 : -5;
        done_out = 1;
      }
    } else if (kind == FIN_INIT) {
      sv.sc[S_FNORM2] = tot[0];
      sv.sc[S_RNORM2] = tot[1];
      const double tol2 = rtol2 * tot[0];
      sv.sc[S_TOL2] = tol2;
      if (!isfinite(tot[0]) || !isfinite(tot[1])) {
        sv.fl[F_STATUS] = -5;
        done_out = 1;
      } else if (tot[0] == 0.0 || tot[1] <= tol2) {
        done_out = 1;
      }
    } else if (kind == FIN_TRUE) {
      sv.sc[S_TRUE2] = tot[0];
    } else if (kind == FIN_MEANS) {
      sv.sc[S_MU_B] = ns ? tot[0] / (double)sv.n : 0.0;
      sv.sc[S_MU_X] = ns ? tot[1] / (double)sv.n : 0.0;
    } else if (kind == FIN_NORM) {
      sv.sc[S_WX] = tot[0];
      sv.sc[S_WSUM] = tot[1];
    }
    if (done_out) sv.fl[F_DONE] = 1;
    // pinned host mirror of (done, iterations) for the solve loops' convergence polling
    if (sv.host_flags && (guarded || kind == FIN_INIT)) {
      __hip_atomic_store(&sv.host_flags[1], iters_out, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __hip_atomic_store(&sv.host_flags[0], done_out, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
  }
}

// One block of kFinBlock threads: the partials are few thousand values spread over the XCDs'
// caches, so the sum is bound by memory latency and wants many reads in flight.
constexpr int kFinBlock = 1024;
__global__ __launch_bounds__(kFinBlock) void k_finalize(Solve sv, int kind, int nb) {
  __shared__ double lds[3 * kFinBlock / 64];
  __shared__ float lds32[2 * 2 * kFinBlock / 64];
  finalize_body<kFinBlock>(sv, kind, nb, lds, lds32);
}

// ---------------------------------------------------------------------------------------
// Pointwise kernels.
__device__ __forceinline__ long gtid() { return (long)blockIdx.x * kBlock + threadIdx.x; }

// x += alpha p; r -= alpha q; partial ||r||^2 (convergence test in FIN_UPDATE).  Optionally writes the level-0
// right-hand side of the float V-cycle (r32 = fl32(r)) and the first pre-smoothing step of
// level 0 (d0 = c0 dinv0 f0; also x0 = d0 when x0 is given).
template <typename T>
__device__ __forceinline__ void cg_update_body(const Solve& sv, double* __restrict__ x, double* __restrict__ r,
                                               const double* __restrict__ p, const double* __restrict__ q,
                                               float* __restrict__ r32, const T* __restrict__ dinv0,
                                               T* __restrict__ d0, T* __restrict__ x0, T c0, long n, int bi, int nb,
                                               double* lds) {
  const double alpha = sv.sc[S_ALPHA];
  double acc[1] = {0.0};
  for (long i = (long)bi * kBlock + threadIdx.x; i < n; i += (long)nb * kBlock) {
    x[i] += alpha * p[i];
    const double rn = r[i] - alpha * q[i];
    r[i] = rn;
    acc[0] += rn * rn;
    T f0;
    if (r32) { const float rf = (float)rn; r32[i] = rf; f0 = (T)rf; } else { f0 = (T)rn; }
    if (d0) {
      const T d = c0 * dinv0[i] * f0;
      d0[i] = d;
      if (x0) x0[i] = d;
    }
  }
  block_sum<1>(acc, lds);
  if (threadIdx.x == 0) sv.part[bi] = acc[0];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_cg_update(Solve sv, double* __restrict__ x, double* __restrict__ r,
                                                      const double* __restrict__ p, const double* __restrict__ q,
                                                      float* __restrict__ r32, const T* __restrict__ dinv0,
                                                      T* __restrict__ d0, T* __restrict__ x0, T c0, long n) {
  if (solve_done(sv)) return;
  __shared__ double lds[4];
  cg_update_body<T>(sv, x, r, p, q, r32, dinv0, d0, x0, c0, n, blockIdx.x, gridDim.x, lds);
}

// p = (z - mu_z) + beta p   (p = z - mu_z for the first direction).
template <typename T>
__device__ __forceinline__ void cg_direction_body(const Solve& sv, double* __restrict__ p, const T* __restrict__ z, long n,
                                                  int bi, int nb) {
  const double mu = sv.sc[S_MU_Z], beta = sv.sc[S_BETA];
  const int first = sv.fl[F_FIRST];
  for (long i = (long)bi * kBlock + threadIdx.x; i < n; i += (long)nb * kBlock) {
    const double zi = (double)z[i] - mu;
    p[i] = first ? zi : zi + beta * p[i];
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_cg_direction(Solve sv, double* __restrict__ p, const T* __restrict__ z, long n) {
  if (solve_done(sv)) return;
  cg_direction_body<T>(sv, p, z, n, blockIdx.x, gridDim.x);
}

// Marks the first direction as formed (a separate launch, so that every block of
// k_cg_direction has read the flag before it changes).
__global__ void k_clear_first(Solve sv) {
  if (threadIdx.x == 0) sv.fl[F_FIRST] = 0;
}

// Solve-state control from the device queue: mode 0 starts a solve (flags, iteration cap,
// null-space switch, rtol^2), mode 1 clears `done` (exit-phase kernels then run).
__global__ void k_solve_control(Solve sv, int mode, int maxit, int nullspace, double rtol2) {
  if (threadIdx.x != 0) return;
  if (mode == 0) {
    for (int f = 0; f < F_COUNT; ++f) sv.fl[f] = 0;
    sv.fl[F_FIRST] = 1;
    sv.fl[F_MAXIT] = maxit;
    sv.fl[F_NULLSPACE] = nullspace;
    sv.sc[S_RTOL2] = rtol2;
  } else {
    sv.fl[F_DONE] = 0;
  }
}

// d = c0 dinv f, and x = d when x is given (first smoothing step from a zero guess, when it
// is not fused into the kernel that produced f).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cheb_pre0(Solve sv, const T* __restrict__ f, const T* __restrict__ dinv,
                                                      T* __restrict__ d, T* __restrict__ x, T c0, long n) {
  if (solve_done(sv)) return;
  for (long i = gtid(); i < n; i += (long)gridDim.x * kBlock) {
    const T v = c0 * dinv[i] * f[i];
    d[i] = v;
    if (x) x[i] = v;
  }
}

// x = 0 (a fill kernel rather than a memset node, so that the call is safe under stream capture).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_fill_zero(T* __restrict__ x, long n) {
  for (long i = gtid(); i < n; i += (long)gridDim.x * kBlock) x[i] = T(0);
}

// x = 0 when the solve's projected right-hand side is zero (its norm is a device scalar).
__global__ __launch_bounds__(kBlock) void k_zero_if_zero_rhs(Solve sv, double* __restrict__ x, long n) {
  if (sv.sc[S_FNORM2] != 0.0) return;
  for (long i = gtid(); i < n; i += (long)gridDim.x * kBlock) x[i] = 0.0;
}

// x += d   (degree-1 post-smoothing completion); x = d when `assign`.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_add(Solve sv, T* __restrict__ x, const T* __restrict__ d, int assign, long n) {
  if (solve_done(sv)) return;
  for (long i = gtid(); i < n; i += (long)gridDim.x * kBlock) x[i] = assign ? d[i] : x[i] + d[i];
}

// Coarsest level: x = G f with the dense float64 operator G (one wave per row).
template <typename T>
__device__ __forceinline__ void coarse_gemv_body(const double* __restrict__ G, const T* __restrict__ f, T* __restrict__ x,
                                                 int n, int bi) {
  const int row = bi * (kBlock / 64) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  double s = 0.0;
  for (int j = lane; j < n; j += 64) s += G[(long)row * n + j] * (double)f[j];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
  if (lane == 0) x[row] = (T)s;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_coarse_gemv(Solve sv, const double* __restrict__ G, const T* __restrict__ f,
                                                        T* __restrict__ x, int n) {
  if (solve_done(sv)) return;
  coarse_gemv_body<T>(G, f, x, n, blockIdx.x);
}


// ---------------------------------------------------------------------------------------
// Setup / exit kernels of a solve.
// Partial sums of b (and of the initial guess) for the projection means (FIN_MEANS).
__global__ __launch_bounds__(kBlock) void k_init_means(Solve sv, const double* __restrict__ b, const double* __restrict__ x,
                                                       long n) {
  __shared__ double lds[8];
  double acc[2] = {0.0, 0.0};
  for (long i = gtid(); i < n; i += (long)gridDim.x * kBlock) {
    acc[0] += b[i];
    if (x) acc[1] += x[i];
  }
  block_sum<2>(acc, lds);
  const int nb = gridDim.x;
  if (threadIdx.x == 0) { sv.part[blockIdx.x] = acc[0]; sv.part[nb + blockIdx.x] = acc[1]; }
}

// x = x - mu_x (guess) or 0; with no guess also r = b - mu_b and the norms of b^.
__global__ __launch_bounds__(kBlock) void k_init_guess(Solve sv, double* __restrict__ x, int guess, long n) {
  const double mu = sv.sc[S_MU_X];
  for (long i = gtid(); i < n; i += (long)gridDim.x * kBlock) x[i] = guess ? x[i] - mu : 0.0;
}

// Weighted normalisation x -= (w^T x / sum w) 1: partials (FIN_NORM), then the update.
__global__ __launch_bounds__(kBlock) void k_norm_sums(Solve sv, const double* __restrict__ w, const double* __restrict__ x,
                                                      long n) {
  __shared__ double lds[8];
  double acc[2] = {0.0, 0.0};
  for (long i = gtid(); i < n; i += (long)gridDim.x * kBlock) {
    const double wi = w ? w[i] : 1.0;
    acc[0] += wi * x[i];
    acc[1] += wi;
  }
  block_sum<2>(acc, lds);
  const int nb = gridDim.x;
  if (threadIdx.x == 0) { sv.part[blockIdx.x] = acc[0]; sv.part[nb + blockIdx.x] = acc[1]; }
}

__global__ __launch_bounds__(kBlock) void k_norm_apply(Solve sv, double* __restrict__ x, long n) {
  const double s = sv.sc[S_WX] / sv.sc[S_WSUM];
  for (long i = gtid(); i < n; i += (long)gridDim.x * kBlock) x[i] -= s;
}

// ---------------------------------------------------------------------------------------
// Multi-task launches (batched solves): one launch serves several independent solves.  Each
// task owns the contiguous block range [off, off + nb) of the grid; a block finds its task,
// reads the task's arguments (uniform per block) and runs the single-solve body with its
// local block index, so every solve computes exactly what it computes alone.
template <typename Task>
__device__ __forceinline__ int task_of(const Task* __restrict__ tasks, int ntasks) {
  __shared__ int t_sh;
  if (threadIdx.x == 0) {
    int t = 0;
    while (t + 1 < ntasks && tasks[t + 1].off <= (int)blockIdx.x) ++t;
    t_sh = t;
  }
  __syncthreads();
  return t_sh;
}

template <typename T>
struct SpTask {
  SpArgs<T> a;
  const int* blk;
  int nb, off;
};

template <typename T, int OP, int IX>
__global__ __launch_bounds__(kBlock) void k_spmv_stream_multi(const SpTask<T>* __restrict__ tasks, int ntasks) {
  __shared__ double lds[16];
  __shared__ float lds32[24];
  __shared__ __align__(16) unsigned char smem[smem_bytes<T>()];
  const SpTask<T>& tk = tasks[task_of(tasks, ntasks)];
  const SpArgs<T> a = tk.a;
  stream_body<T, OP, IX>(a, tk.blk, xcd_tile((int)blockIdx.x - tk.off, tk.nb), tk.nb, smem, lds, lds32);
}

template <typename T, int OP>
__global__ __launch_bounds__(kBlock) void k_spmv_sdia_multi(const SpTask<T>* __restrict__ tasks, int ntasks) {
  __shared__ double lds[16];
  __shared__ float lds32[24];
  const SpTask<T>& tk = tasks[task_of(tasks, ntasks)];
  const SpArgs<T> a = tk.a;
  sdia_body<T, OP>(a, xcd_tile((int)blockIdx.x - tk.off, tk.nb), tk.nb, lds, lds32);
}

template <typename T>
struct UpdTask {
  Solve sv;
  double *x, *r;
  const double *p, *q;
  float* r32;
  const T* dinv0;
  T *d0, *x0;
  T c0;
  long n;
  int nb, off;
};

template <typename T>
__global__ __launch_bounds__(kBlock) void k_cg_update_multi(const UpdTask<T>* __restrict__ tasks, int ntasks) {
  __shared__ double lds[4];
  const UpdTask<T>& k = tasks[task_of(tasks, ntasks)];
  if (solve_done(k.sv)) return;
  cg_update_body<T>(k.sv, k.x, k.r, k.p, k.q, k.r32, k.dinv0, k.d0, k.x0, k.c0, k.n, (int)blockIdx.x - k.off, k.nb, lds);
}

template <typename T>
struct DirTask {
  Solve sv;
  double* p;
  const T* z;
  long n;
  int nb, off;
};

template <typename T>
__global__ __launch_bounds__(kBlock) void k_cg_direction_multi(const DirTask<T>* __restrict__ tasks, int ntasks) {
  const DirTask<T>& k = tasks[task_of(tasks, ntasks)];
  if (solve_done(k.sv)) return;
  cg_direction_body<T>(k.sv, k.p, k.z, k.n, (int)blockIdx.x - k.off, k.nb);
}

template <typename T>
struct GemvTask {
  Solve sv;
  const double* G;
  const T* f;
  T* x;
  int n;
  int nb, off;
};

template <typename T>
__global__ __launch_bounds__(kBlock) void k_coarse_gemv_multi(const GemvTask<T>* __restrict__ tasks, int ntasks) {
  const GemvTask<T>& k = tasks[task_of(tasks, ntasks)];
  if (solve_done(k.sv)) return;
  coarse_gemv_body<T>(k.G, k.f, k.x, k.n, (int)blockIdx.x - k.off);
}

struct FinTask {
  Solve sv;
  int kind, nb_part;
  int nb, off;  // one block per task
};

__global__ __launch_bounds__(kBlock) void k_finalize_multi(const FinTask* __restrict__ tasks, int ntasks) {
  __shared__ double lds[16];
  __shared__ float lds32[24];
  const FinTask& k = tasks[task_of(tasks, ntasks)];
  finalize_body<kBlock>(k.sv, k.kind, k.nb_part, lds, lds32);
}

// ---------------------------------------------------------------------------------------
// Vector utilities.
template <typename S, typename D>
__global__ __launch_bounds__(kBlock) void k_convert(const S* __restrict__ s, D* __restrict__ d, long n) {
  for (long i = gtid(); i < n; i += (long)gridDim.x * kBlock) d[i] = (D)s[i];
}

}  // namespace bd
