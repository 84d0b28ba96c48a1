// Device side of the library: the AMG hierarchy in HBM, the V-cycle (Alg. 2) as a sequence
// of fused kernels, PCG / flexible CG with all scalars kept on the device, the Bidomain
// time step (eqs. (4)-(7)) and the C ABI declared in bidomain.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <type_traits>
#include <vector>

#include "bd_host.hpp"
#include "bidomain.h"
#include "kernels.hpp"
#include "spgemm.hpp"
#include "galerkin_dense.hpp"
#include "aggregate.hpp"

namespace bd {

// ------------------------------------------------------------------------------------------
// Errors: internal code throws Failure; every C entry point converts it to a status code.
struct Failure {
  int code;
  std::string msg;
};
thread_local std::string g_last_error;

#define HIPCHK(expr)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      throw Failure{e_ == hipErrorOutOfMemory ? BD_E_NOMEM : BD_E_DEVICE,                 \
                    std::string(#expr) + ": " + hipGetErrorString(e_)};                   \
  } while (0)

template <class F>
int guarded(F&& f) {
  try {
    return f();
  } catch (const Failure& e) {
    g_last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return BD_E_NOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return BD_E_INVALID;
  }
}

// ------------------------------------------------------------------------------------------
// Device memory owned by a handle.
struct Arena {
  std::vector<void*> ptrs;
  int64_t bytes = 0;
  template <typename T>
  T* alloc(size_t count) {
    if (count == 0) count = 1;
    void* p = nullptr;
    HIPCHK(hipMalloc(&p, count * sizeof(T)));
    ptrs.push_back(p);
    bytes += (int64_t)(count * sizeof(T));
    return static_cast<T*>(p);
  }
  ~Arena() {
    for (void* p : ptrs) (void)hipFree(p);
  }
};

// Sparsity pattern of a device matrix and its launch plan (shared by matrices with the same
// pattern, e.g. the float64 and float32 copies of the fine operator).
struct DPat {
  int n = 0, ncols = 0;
  int64_t nnz = 0;
  const int* rp = nullptr;
  const int* ci = nullptr;        // 32-bit column indices, or null when only cs is kept
  const uint16_t* cs = nullptr;   // column - cbase[tile] (stream) or the column (lane group) in 16 bits, or null
  const int* cbase = nullptr;     // CSR-stream: per-tile column base, with cs
  const uint32_t* c24 = nullptr;  // CSR-stream: 24-bit column indices, four in three words, or null
  const uint8_t* cd = nullptr;    // CSR-stream: index into dict of column - row, or null
  const int* dict = nullptr;      // the distinct column - row offsets, with cd
  int ndict = 0;
  int G = 8;    // lanes per row (row-group kernel)
  int tpb = 1;  // row tiles per block (row-group kernel); chunks per plane (diagonal form)
  int nb = 0;   // blocks of a product launch
  const int* blk = nullptr;  // CSR-stream row tiles (nb + 1 row boundaries), or null
  int nd = 0;                // symmetric diagonal form: stored diagonals (kDiagK), or 0
  int64_t ds = 0;            // with nd: stride between the diagonals
  int doff[kDiagK] = {};     // with nd: their column - row offsets (>= 0)
  int col_bytes() const { return nd ? 0 : (cd ? 1 : (cs ? 2 : (c24 ? 3 : 4))); }
  int form() const { return nd ? SDIA : (cd ? IXD8 : (cs ? IX16 : (c24 ? IX24 : IX32))); }
};

template <typename T>
struct DCsr : DPat {
  T* v = nullptr;   // CSR values (null in the symmetric diagonal form)
  T* dv = nullptr;  // with nd: the nd diagonals, ds apart
};

int lanes_for(double mean_row) {
  int g = 2;
  while (g < 64 && g * 4 < mean_row) g *= 2;
  return g;
}

// Greedy packing of consecutive rows into tiles of at most max_rows rows and max_nnz entries
// (row boundaries, nb + 1 of them).
std::vector<int> pack_tiles(const Csr& H, int max_rows, int64_t max_nnz) {
  std::vector<int> blk(1, 0);
  int32_t r = 0;
  while (r < H.nrows) {
    const int32_t start = r;
    int64_t cnt = 0;
    while (r < H.nrows && r - start < max_rows && cnt + (H.rp[r + 1] - H.rp[r]) <= max_nnz) {
      cnt += H.rp[r + 1] - H.rp[r];
      ++r;
    }
    blk.push_back(r);
  }
  return blk;
}

// Row tiles of the CSR-stream kernel (nb + 1 row boundaries).  Matrices whose every row fits
// the staging buffer use it (measured faster than the lane-group kernel on every level of the
// slab hierarchies, short and long rows alike); longer rows fall back to the lane-group kernel
// (empty result).  Tiles hold at most cap entries and max_rows rows (149 rows of a 27-point
// operator, 512 of a prolongator), so that every tile streams a few thousand entries.
// (Capping long-row tiles at 128 rows, for two lanes per row in phase 2, measured slower; so
// did shrinking tiles until their count fills whole rounds of resident blocks.)
std::vector<int> stream_blocks(const Csr& H, int cap, int max_rows) {
  if (H.nrows == 0) return {};
  for (int32_t i = 0; i < H.nrows; ++i)
    if (H.rp[i + 1] - H.rp[i] > cap) return {};
  return pack_tiles(H, max_rows, cap);
}

// Offset dictionary: if the matrix's column - row offsets take at most kDictMax distinct values
// (27 for the slab's 27-point operators), each entry stores its offset's index in one byte.
bool dict_columns(const Csr& H, std::vector<uint8_t>& cd, std::vector<int>& dict) {
  std::vector<int64_t> offs;
  std::atomic<bool> fits{true};
#pragma omp parallel
  {
    std::vector<int64_t> mine;
#pragma omp for schedule(static, 4096)
    for (int32_t i = 0; i < H.nrows; ++i) {
      if (!fits.load(std::memory_order_relaxed)) continue;
      for (int32_t k = H.rp[i]; k < H.rp[i + 1]; ++k) {
        const int64_t o = (int64_t)H.ci[k] - i;
        if (std::find(mine.begin(), mine.end(), o) == mine.end()) {
          mine.push_back(o);
          if ((int)mine.size() > kDictMax) {
            fits.store(false, std::memory_order_relaxed);
            break;
          }
        }
      }
    }
#pragma omp critical
    offs.insert(offs.end(), mine.begin(), mine.end());
  }
  if (!fits) return false;
  std::sort(offs.begin(), offs.end());
  offs.erase(std::unique(offs.begin(), offs.end()), offs.end());
  if ((int)offs.size() > kDictMax) return false;
  dict.assign(offs.begin(), offs.end());
  cd.assign(H.ci.size(), 0);
#pragma omp parallel for schedule(static, 4096)
  for (int32_t i = 0; i < H.nrows; ++i)
    for (int32_t k = H.rp[i]; k < H.rp[i + 1]; ++k)
      cd[k] = (uint8_t)(std::lower_bound(offs.begin(), offs.end(), (int64_t)H.ci[k] - i) - offs.begin());
  return true;
}

void configure(DPat& M, int max_blocks) {
  M.G = lanes_for(M.n ? (double)M.nnz / M.n : 1.0);
  const int rpt = kBlock / M.G;
  const int64_t tiles = (M.n + rpt - 1) / rpt;
  M.tpb = (int)std::max<int64_t>(1, (tiles + max_blocks - 1) / max_blocks);
  M.nb = (int)std::max<int64_t>(1, (tiles + M.tpb - 1) / M.tpb);
}

// Per-tile 16-bit column offsets: every tile's columns span fewer than 65,536 values (a
// 27-point stencil spans two grid planes around a tile's rows), so each entry stores
// column - cbase[tile] in 16 bits instead of a 32-bit index.  Empty result if some tile spans
// more (the matrix then keeps 32-bit indices).
bool compact_columns(const Csr& H, const std::vector<int>& blk, std::vector<uint16_t>& cs, std::vector<int>& cbase) {
  const int nb = (int)blk.size() - 1;
  cbase.assign(nb, 0);
  cs.assign(H.ci.size(), 0);
  for (int t = 0; t < nb; ++t) {
    const int32_t beg = H.rp[blk[t]], end = H.rp[blk[t + 1]];
    if (end == beg) continue;
    int32_t lo = H.ci[beg], hi = H.ci[beg];
    for (int32_t k = beg; k < end; ++k) {
      lo = std::min(lo, H.ci[k]);
      hi = std::max(hi, H.ci[k]);
    }
    if (hi - lo > 65535) return false;
    cbase[t] = lo;
    for (int32_t k = beg; k < end; ++k) cs[k] = (uint16_t)(H.ci[k] - lo);
  }
  return true;
}

// 24-bit column indices for a CSR-stream matrix of at most 2^24 columns: entries 4q .. 4q + 3
// (zero past nnz) in words 3q .. 3q + 2, entry j in bits 24 j .. 24 j + 23 of the 96 bits.
void pack_columns24(const Csr& H, std::vector<uint32_t>& c24) {
  const int64_t nnz = H.nnz(), nq = (nnz + 3) / 4;
  c24.assign((size_t)(3 * nq), 0u);
#pragma omp parallel for schedule(static, 65536)
  for (int64_t q = 0; q < nq; ++q) {
    uint32_t c[4];
    for (int j = 0; j < 4; ++j) c[j] = 4 * q + j < nnz ? (uint32_t)H.ci[4 * q + j] : 0u;
    c24[3 * q] = c[0] | c[1] << 24;
    c24[3 * q + 1] = c[1] >> 8 | c[2] << 16;
    c24[3 * q + 2] = c[2] >> 16 | c[3] << 8;
  }
}

// Host values in the device precision: the vector itself for float64, a copy converted in
// parallel for float32.
template <typename T>
const std::vector<double>& as_type(const std::vector<double>& v,
                                   typename std::enable_if<std::is_same<T, double>::value>::type* = nullptr) {
  return v;
}
template <typename T>
std::vector<float> as_type(const std::vector<double>& v,
                           typename std::enable_if<std::is_same<T, float>::value>::type* = nullptr) {
  std::vector<float> f(v.size());
#pragma omp parallel for schedule(static, 65536)
  for (int64_t i = 0; i < (int64_t)v.size(); ++i) f[i] = (float)v[i];
  return f;
}

template <typename U>
U* upload_padded(Arena& ar, const U* src, size_t count, hipStream_t st) {
  U* d = ar.alloc<U>(count + kStreamPad);  // padded for 4-entry vector loads
  HIPCHK(hipMemsetAsync(d + count, 0, kStreamPad * sizeof(U), st));
  if (count) HIPCHK(hipMemcpyAsync(d, src, count * sizeof(U), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  return d;
}

}  // namespace bd

// Host half of a product's launch plan: the symmetric diagonal form, or the CSR-stream row
// tiles and column index encoding.  Built on whichever thread runs the setup (a serving
// worker, not the serving thread), so that the upload itself is copies only.
struct StreamPlan {
  int nd = 0;                   // symmetric diagonal form: stored diagonals, or 0
  int64_t ds = 0;               // stride between the diagonals
  int doff[bd::kDiagK] = {};    // their column - row offsets (>= 0; 0 pads unused ones)
  std::vector<double> dval;     // nd * ds values, zero where an entry does not exist
  std::vector<int> blk;         // row tiles, or empty (lane-group kernel)
  std::vector<uint8_t> cd;      // offset-dictionary indices, or empty
  std::vector<int> dict;
  std::vector<uint16_t> cs;     // 16-bit per-tile offsets (stream) or column indices (lane group), or empty
  std::vector<int> cbase;
  std::vector<uint32_t> c24;    // 24-bit column indices (stream), or empty
  std::shared_ptr<bd::Csr> mat;  // the renumbered matrix the plan is for (uploaded instead of the
                                // host's; released after the upload), or null
};

namespace bd {

// Symmetric diagonal form: taken where the matrix is square and equal to its transpose (every
// entry a(i, j) has an entry a(j, i) of the same value, no duplicates), its column - row
// offsets d >= 0 are those of a 27-point stencil ({0, 1} and four triples C - 1, C, C + 1), and
// the kDiagK diagonals (8 bytes a slot) move fewer bytes than the offset-dictionary form's
// values and index bytes (9 bytes an entry).  Square matrices with too many offsets (coarse
// levels) are rejected after a few rows.
bool sym_diagonals(const Csr& H, StreamPlan& P) {
  const int32_t n = H.nrows;
  if (n == 0 || H.ncols != n) return false;
  if ((int64_t)kDiagK * n * 8 >= H.nnz() * 9 + 4 * (int64_t)n) return false;
  std::vector<int> offs{0};
  std::atomic<bool> ok{true};
#pragma omp parallel
  {
    std::vector<int> mine;
#pragma omp for schedule(static, 4096)
    for (int32_t i = 0; i < n; ++i) {
      if (!ok.load(std::memory_order_relaxed)) continue;
      for (int32_t k = H.rp[i]; k < H.rp[i + 1]; ++k) {
        const int d = H.ci[k] - i;
        if (d < 0 || std::find(mine.begin(), mine.end(), d) != mine.end()) continue;
        mine.push_back(d);
        if ((int)mine.size() > kDiagK) {
          ok.store(false, std::memory_order_relaxed);
          break;
        }
      }
    }
#pragma omp critical
    offs.insert(offs.end(), mine.begin(), mine.end());
  }
  if (!ok) return false;
  std::sort(offs.begin(), offs.end());
  offs.erase(std::unique(offs.begin(), offs.end()), offs.end());
  const int nu = (int)offs.size();
  if (nu != kDiagK) return false;
  // the product gathers x in triples around the centres 0, C_1 .. C_4: the offsets must be
  // {0, 1, C_t - 1, C_t, C_t + 1} (a 27-point stencil of a grid at least 2 nodes wide in x)
  if (offs[1] != 1) return false;
  for (int t = 0; t < 4; ++t)
    if (offs[3 + 3 * t] - offs[2 + 3 * t] != 1 || offs[4 + 3 * t] - offs[3 + 3 * t] != 1) return false;
  for (int o = 0; o < kDiagK; ++o) P.doff[o] = offs[o];
  auto slot = [&](int d) {
    for (int o = 0; o < nu; ++o)
      if (P.doff[o] == d) return o;
    return -1;
  };
  P.ds = ((int64_t)n + 1 + 63) / 64 * 64;  // at least one zero slot past the last row
  P.dval.assign((size_t)kDiagK * P.ds, 0.0);
  std::vector<uint16_t> up(n, 0), lo(n, 0);  // slots filled by row i's own and mirrored entries
  int64_t nup = 0, nlo = 0;
  // entries on and above the diagonal: row i's own slots (no duplicates)
#pragma omp parallel for schedule(static, 4096) reduction(+ : nup)
  for (int32_t i = 0; i < n; ++i)
    for (int32_t k = H.rp[i]; k < H.rp[i + 1]; ++k) {
      const int d = H.ci[k] - i;
      if (d < 0) continue;
      const int o = slot(d);
      if (up[i] >> o & 1) ok.store(false, std::memory_order_relaxed);
      up[i] |= (uint16_t)(1u << o);
      P.dval[(size_t)o * P.ds + i] = H.v[k];
      if (d > 0) ++nup;
    }
  // entries below: each the mirror of a distinct stored entry, with the same value
#pragma omp parallel for schedule(static, 4096) reduction(+ : nlo)
  for (int32_t i = 0; i < n; ++i)
    for (int32_t k = H.rp[i]; k < H.rp[i + 1]; ++k) {
      const int32_t c = H.ci[k];
      const int o = c < i ? slot(i - c) : -1;
      if (c >= i) continue;
      if (o < 0 || !(up[c] >> o & 1) || (lo[i] >> o & 1) || !(P.dval[(size_t)o * P.ds + c] == H.v[k])) {
        ok.store(false, std::memory_order_relaxed);
        continue;
      }
      lo[i] |= (uint16_t)(1u << o);
      ++nlo;
    }
  if (!ok || nlo != nup) {
    P.dval.clear();
    P.dval.shrink_to_fit();
    return false;
  }
  P.nd = kDiagK;
  return true;
}

StreamPlan plan_stream(const Csr& H, bool diag_form) {
  StreamPlan P;
  if (diag_form && sym_diagonals(H, P)) return P;
  // index form: offset dictionary, else 16-bit per-tile offsets, else 32-bit indices
  P.blk = stream_blocks(H, kStreamCapD, kStreamRowsD);
  const bool dictf = !P.blk.empty() && dict_columns(H, P.cd, P.dict);
  if (!dictf) {
    P.cd.clear();
    P.dict.clear();
    P.blk = stream_blocks(H, kStreamCap, kStreamRows);
    if (!P.blk.empty() && !compact_columns(H, P.blk, P.cs, P.cbase)) {
      P.cs.clear();
      P.cbase.clear();
      if (H.ncols <= kMaxCols24) pack_columns24(H, P.c24);
    }
    // rows too long for a stream tile, 64 lanes a row: 16-bit column indices where they fit
    if (P.blk.empty() && H.nrows > 0 && H.ncols <= 65536 && lanes_for((double)H.nnz() / H.nrows) == 64)
      P.cs.assign(H.ci.begin(), H.ci.end());
  }
  return P;
}

// Levels renumbered on the device (option reorder): the intermediate ones -- not the fine
// level, whose numbering is the caller's, nor the coarsest, solved through its dense inverse --
// of more than 256 rows and at most 10 % dense, and (reorder = 1) with at least 2^26 stored
// entries.  Reverse Cuthill-McKee order clusters a row's columns: on the 384 x 384 x 96 slab the
// 128-byte lines of x a row of level 2 touches fall from 261 to 95 and its product from 431 to
// 302 us (level 1: 64 -> 24 lines, 177 -> 148 us), both levels' tiles then fit 16-bit offsets,
// and level 3 (8 % dense) gains too.  The renumbering costs the setup ~10 ns an entry on the
// host, in large allocations; with a 2^24-entry floor the serving stream's larger cases were
// renumbered too, on the setup workers, and the serving thread's p99 solve latency rose from
// ~55 to ~140 ms, so smaller hierarchies keep the aggregate order by default.
bool renumber_level(const HostHierarchy& H, int k, int reorder) {
  const int M = (int)H.lv.size() - 1;
  const Csr& A = H.lv[k].A;
  return reorder > 0 && k >= 1 && k < M && A.nrows > 256 &&
         (double)A.nnz() <= 0.1 * (double)A.nrows * (double)A.nrows && (reorder == 2 || A.nnz() >= (int64_t(1) << 26));
}// Launch plans of every matrix of a host hierarchy (levels' A, P, R), with the renumbered
// copies where a level is renumbered (reorder).
void plan_hierarchy(HostHierarchy& H, bool diag_form, int reorder) {
  const int nl = (int)H.lv.size();
  std::vector<std::vector<int32_t>> inv(nl);  // old -> new, per renumbered level
  for (int k = 0; k < nl; ++k) {
    HostLevel& L = H.lv[k];
    L.perm.clear();
    if (renumber_level(H, k, reorder)) {
      L.perm = rcm_order(L.A);
      inv[k].resize(L.perm.size());
      for (int32_t i = 0; i < (int32_t)L.perm.size(); ++i) inv[k][L.perm[i]] = i;
    }
  }
  auto plan = [&](const Csr& M, const std::vector<int32_t>& rows, const std::vector<int32_t>& cols, bool diag) {
    if (rows.empty() && cols.empty()) return std::make_shared<StreamPlan>(plan_stream(M, diag));
    auto mat = std::make_shared<Csr>(renumbered(M, rows.empty() ? nullptr : rows.data(),
                                                cols.empty() ? nullptr : cols.data()));
    auto P = std::make_shared<StreamPlan>(plan_stream(*mat, diag));
    P->mat = std::move(mat);
    return P;
  };
  const std::vector<int32_t> none;
  for (int k = 0; k < nl; ++k) {
    HostLevel& L = H.lv[k];
    L.plan_a = plan(L.A, L.perm, inv[k], diag_form);
    // P_k: rows on level k, columns on level k + 1; R_k the other way round
    if (L.P.nrows) L.plan_p = plan(L.P, L.perm, k + 1 < nl ? inv[k + 1] : none, false);
    if (L.R.nrows) L.plan_r = plan(L.R, k + 1 < nl ? H.lv[k + 1].perm : none, inv[k], false);
  }
}

// Host copies of the renumbered matrices are needed only until they are on the device.
void release_plan_matrices(HostHierarchy& H) {
  for (HostLevel& L : H.lv)
    for (auto* p : {&L.plan_a, &L.plan_p, &L.plan_r})
      if (*p) (*p)->mat.reset();
}

template <typename U>
const U* upload_small(Arena& ar, const std::vector<U>& h, hipStream_t st) {
  U* d = ar.alloc<U>(h.size());
  HIPCHK(hipMemcpyAsync(d, h.data(), h.size() * sizeof(U), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  return d;
}

// Device copy of H with values of type T.  share: a pattern uploaded before for the same H
// (reused as is), or null.  plan: H's launch plan (built here if null).  need_ci: keep the
// 32-bit column indices even where the product reads a compressed form (for kernels outside
// the product that read them).
template <typename T>
DCsr<T> upload(Arena& ar, const Csr& H0, const DPat* share, const StreamPlan* plan, bool need_ci, hipStream_t st,
               int max_blocks) {
  const Csr& H = plan && plan->mat ? *plan->mat : H0;  // a renumbered level's matrix
  DCsr<T> M;
  if (share) {
    static_cast<DPat&>(M) = *share;
  } else {
    StreamPlan local;
    if (!plan) {
      local = plan_stream(H, false);
      plan = &local;
    }
    M.n = H.nrows;
    M.ncols = H.ncols;
    M.nnz = H.nnz();
    M.rp = upload_small<int>(ar, H.rp, st);
    configure(M, max_blocks);
    if (plan->nd) {
      M.nd = plan->nd;
      M.ds = plan->ds;
      std::copy(plan->doff, plan->doff + kDiagK, M.doff);
      // block grid of the diagonal kernel: Z planes of S 256-row chunks (tpb holds S)
      const int chunks = (M.n + kBlock - 1) / kBlock;
      const int dmax = *std::max_element(M.doff, M.doff + kDiagK);
      M.tpb = std::max(1, std::min(chunks, (dmax + kBlock - 1) / kBlock));
      M.nb = M.tpb * ((chunks + M.tpb - 1) / M.tpb);
    }
    if (!plan->blk.empty()) {
      M.blk = upload_small<int>(ar, plan->blk, st);
      M.nb = (int)plan->blk.size() - 1;
    }
    if (!plan->cd.empty()) {
      M.cd = upload_padded<uint8_t>(ar, plan->cd.data(), plan->cd.size(), st);
      M.dict = upload_small<int>(ar, plan->dict, st);
      M.ndict = (int)plan->dict.size();
    }
    if (!plan->cs.empty()) {
      M.cs = upload_padded<uint16_t>(ar, plan->cs.data(), plan->cs.size(), st);
      if (!plan->cbase.empty()) M.cbase = upload_small<int>(ar, plan->cbase, st);
    }
    if (!plan->c24.empty()) M.c24 = upload_padded<uint32_t>(ar, plan->c24.data(), plan->c24.size(), st);
    if ((!M.nd && !M.cd && !M.cs && !M.c24) || need_ci) M.ci = upload_padded<int>(ar, H.ci.data(), H.ci.size(), st);
  }
  if (M.nd && !(plan && plan->nd == M.nd)) {
    // a matrix sharing a diagonal-form pattern without diagonals of its own (a simulation's
    // A_i): CSR only, read by kernels outside the product (which keep the column indices)
    M.nd = 0;
    configure(M, max_blocks);
    if (!M.ci) throw std::runtime_error("device matrix without a usable form");
  }
  if (M.nd) {
    M.dv = ar.alloc<T>(plan->dval.size());
    const auto& dv = as_type<T>(plan->dval);
    HIPCHK(hipMemcpyAsync(M.dv, dv.data(), dv.size() * sizeof(T), hipMemcpyHostToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
  } else {
    M.v = upload_padded<T>(ar, as_type<T>(H.v).data(), H.v.size(), st);
  }
  return M;
}

template <typename T>
T* upload_vec(Arena& ar, const std::vector<double>& h, hipStream_t st) {
  T* d = ar.alloc<T>(h.size());
  std::vector<T> tmp(h.begin(), h.end());
  HIPCHK(hipMemcpyAsync(d, tmp.data(), tmp.size() * sizeof(T), hipMemcpyHostToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  return d;
}

template <typename T>
struct DLevel {
  int n = 0;
  DCsr<T> A, P, R;
  const int* perm = nullptr;  // device numbering of the level's unknowns, new -> old (null: the host's)
  int dir = 0;                // direction of the next pass over A (diagonal form), alternating
  T* dinv = nullptr;
  T* f = nullptr;  // right-hand side (level 0: set per call)
  T *x = nullptr, *r = nullptr, *da = nullptr, *db = nullptr;
  double lam = 0.0;
  T c0 = 0;                 // first smoothing step coefficient (Chebyshev 1/theta, Jacobi omega)
  std::vector<T> c1, c2;    // Chebyshev step j = 1 .. degree-1
};

constexpr int kMaxBlocksSpmv = 8192;
constexpr int kMaxBlocksVec = 2048;

int vec_blocks(int64_t n) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + kBlock - 1) / kBlock, kMaxBlocksVec));
}

// Profiling of the fine-level outer product (see bidomain_profile_enable).
struct Prof {
  std::mutex mu;
  bool on = false;
  double total_ms = 0.0;
  int64_t launches = 0;
} g_prof;

}  // namespace bd

using namespace bd;

struct bd_amg {
  bd_amg_opts o{};
  HostHierarchy H;
  Arena ar;
  int n = 0;
  int M = 0;  // index of the coarsest level
  bool mixed = false;
  bool host_only = false;   // hierarchy on the host only (bidomain_amg_build_host)
  // outer (float64) fine operator
  DCsr<double> A0;
  std::vector<DLevel<double>> L64;
  std::vector<DLevel<float>> L32;
  double* G = nullptr;  // coarsest dense operator (float64)
  int nM = 0;
  // CG state
  double *r = nullptr, *p = nullptr, *q = nullptr, *w = nullptr;
  float* r32[2] = {nullptr, nullptr};
  Solve sv{};
  Solve sv_apply{};     // flags that never say "done", for bidomain_amg_apply
  int64_t part_len = 0;
  int* host_flags = nullptr;  // pinned
  int last_iters = 8;
  // events of a solve (created with the solve state, so that a solve creates none): start and
  // stop of the timed region, and the two alternating "update kernel finished" markers
  hipEvent_t ev_start = nullptr, ev_stop = nullptr, ev_iter[2] = {nullptr, nullptr};
  ~bd_amg() {
    if (host_flags) (void)hipHostFree(host_flags);
    for (hipEvent_t e : {ev_start, ev_stop, ev_iter[0], ev_iter[1]})
      if (e) (void)hipEventDestroy(e);
  }
};

namespace bd {

// ------------------------------------------------------------------------------------------
// Kernel launch helpers.
// The matrix fields of a product's arguments.
template <typename T>
void bind(SpArgs<T>& a, const DCsr<T>& M) {
  a.rp = M.rp;
  a.ci = M.ci;
  a.cs = M.cs;
  a.cbase = M.cbase;
  a.c24 = M.c24;
  a.cd = M.cd;
  a.dict = M.dict;
  a.ndict = M.ndict;
  a.ncols = M.ncols;
  a.av = M.v;
  a.nrows = M.n;
  a.tpb = M.tpb;
  a.dv = M.dv;
  a.ds = M.ds;
  for (int o = 0; o < kDiagK; ++o) a.doff[o] = M.doff[o];
}

template <typename T, int OP>
void launch_spmv(const DCsr<T>& M, SpArgs<T> a, hipStream_t st) {
  bind(a, M);
  if (M.n == 0) return;
  if (M.nd) {
    k_spmv_sdia<T, OP><<<M.nb, kBlock, 0, st>>>(a);
    HIPCHK(hipGetLastError());
    return;
  }
  if (M.blk) {
    switch (M.form()) {
      case IXD8: k_spmv_stream<T, OP, IXD8><<<M.nb, kBlock, 0, st>>>(a, M.blk); break;
      case IX16: k_spmv_stream<T, OP, IX16><<<M.nb, kBlock, 0, st>>>(a, M.blk); break;
      case IX24: k_spmv_stream<T, OP, IX24><<<M.nb, kBlock, 0, st>>>(a, M.blk); break;
      default: k_spmv_stream<T, OP, IX32><<<M.nb, kBlock, 0, st>>>(a, M.blk); break;
    }
    HIPCHK(hipGetLastError());
    return;
  }
  if (M.cs && M.G == 64) {  // 16-bit column indices (plan_stream takes them only with 64 lanes)
    k_spmv<T, 64, OP, IX16><<<M.nb, kBlock, 0, st>>>(a);
    HIPCHK(hipGetLastError());
    return;
  }
  switch (M.G) {
    case 2: k_spmv<T, 2, OP><<<M.nb, kBlock, 0, st>>>(a); break;
    case 4: k_spmv<T, 4, OP><<<M.nb, kBlock, 0, st>>>(a); break;
    case 8: k_spmv<T, 8, OP><<<M.nb, kBlock, 0, st>>>(a); break;
    case 16: k_spmv<T, 16, OP><<<M.nb, kBlock, 0, st>>>(a); break;
    case 32: k_spmv<T, 32, OP><<<M.nb, kBlock, 0, st>>>(a); break;
    default: k_spmv<T, 64, OP><<<M.nb, kBlock, 0, st>>>(a); break;
  }
  HIPCHK(hipGetLastError());
}

void finalize(const Solve& sv, int kind, int nb, hipStream_t st) {
  k_finalize<<<1, kFinBlock, 0, st>>>(sv, kind, nb);
  HIPCHK(hipGetLastError());
}

template <typename T>
SpArgs<T> args(const Solve& sv) {
  SpArgs<T> a{};
  a.sv = sv;
  return a;
}

template <typename T>
std::vector<DLevel<T>>& levels(bd_amg* h);
template <>
std::vector<DLevel<double>>& levels<double>(bd_amg* h) { return h->L64; }
template <>
std::vector<DLevel<float>>& levels<float>(bd_amg* h) { return h->L32; }

// First smoothing step from a zero guess can be folded into the producer of f_k when level k
// is smoothed (every level but a directly solved coarsest one).
bool smoothed_level(const bd_amg* h, int k) { return k < h->M || h->H.coarse_mode == 1; }

// Pre-smoothing from a zero guess: x_k = S_k(f_k).  `d_ready`: d = c0 dinv f (and x = d for
// degree 1 / Jacobi) were already written by the producer of f_k.
template <typename T>
void smooth_pre(bd_amg* h, DLevel<T>& L, const Solve& sv, bool d_ready, hipStream_t st) {
  const int deg = h->o.smoother_degree;
  const bool jac = h->o.smoother == BD_JACOBI;
  if (!d_ready) {
    k_cheb_pre0<T><<<vec_blocks(L.n), kBlock, 0, st>>>(sv, L.f, L.dinv, L.da, (deg == 1 || jac) ? L.x : nullptr,
                                                      L.c0, L.n);
    HIPCHK(hipGetLastError());
  }
  if (jac) {
    T* cur = L.x;
    T* oth = L.da;
    for (int j = 1; j < deg; ++j) {
      SpArgs<T> a = args<T>(sv);
      a.x = cur; a.y = oth; a.f = L.f; a.dinv = L.dinv; a.c0 = L.c0;
      launch_spmv<T, OP_JACOBI>(L.A, a, st);
      std::swap(cur, oth);
    }
    if (cur != L.x) {
      k_add<T><<<vec_blocks(L.n), kBlock, 0, st>>>(sv, L.x, cur, 1, L.n);
      HIPCHK(hipGetLastError());
    }
    return;
  }
  if (deg < 2) return;
  SpArgs<T> a = args<T>(sv);
  a.x = L.da; a.xs = L.x; a.f = L.f; a.dinv = L.dinv; a.c1 = L.c1[0]; a.c2 = L.c2[0];
  a.store_rd = deg > 2; a.r = L.r; a.y2 = L.db; a.rev = L.dir ^= 1;
  launch_spmv<T, OP_CHEB_FIRST>(L.A, a, st);
  T* dcur = L.db;
  T* doth = L.da;
  for (int j = 2; j < deg; ++j) {
    SpArgs<T> b = args<T>(sv);
    b.x = dcur; b.xs = L.x; b.r = L.r; b.dinv = L.dinv; b.c1 = L.c1[j - 1]; b.c2 = L.c2[j - 1];
    b.add_d = 0; b.store_rd = j < deg - 1; b.y2 = doth; b.rev = L.dir ^= 1;
    launch_spmv<T, OP_CHEB_STEP>(L.A, b, st);
    std::swap(dcur, doth);
  }
}

struct RedSpec {
  int red = RED_NONE;
  const double* r64 = nullptr;
  const float* r32 = nullptr;
  const float* r32_old = nullptr;
};

// Post-smoothing from the current x_k.  Returns true if the level-0 reductions were fused
// into its last kernel.
template <typename T>
bool smooth_post(bd_amg* h, DLevel<T>& L, const Solve& sv, const RedSpec& red, hipStream_t st) {
  const int deg = h->o.smoother_degree;
  if (h->o.smoother == BD_JACOBI) {
    T* cur = L.x;
    T* oth = L.da;
    for (int j = 0; j < deg; ++j) {
      SpArgs<T> a = args<T>(sv);
      a.x = cur; a.y = oth; a.f = L.f; a.dinv = L.dinv; a.c0 = L.c0;
      launch_spmv<T, OP_JACOBI>(L.A, a, st);
      std::swap(cur, oth);
    }
    if (cur != L.x) {
      k_add<T><<<vec_blocks(L.n), kBlock, 0, st>>>(sv, L.x, cur, 1, L.n);
      HIPCHK(hipGetLastError());
    }
    return false;
  }
  SpArgs<T> a = args<T>(sv);
  a.x = L.x; a.f = L.f; a.r = L.r; a.y2 = L.da; a.dinv = L.dinv; a.c0 = L.c0; a.rev = L.dir ^= 1;
  launch_spmv<T, OP_CHEB_POST0>(L.A, a, st);
  if (deg == 1) {
    k_add<T><<<vec_blocks(L.n), kBlock, 0, st>>>(sv, L.x, L.da, 0, L.n);
    HIPCHK(hipGetLastError());
    return false;
  }
  T* dcur = L.da;
  T* doth = L.db;
  bool fused = false;
  for (int j = 1; j < deg; ++j) {
    SpArgs<T> b = args<T>(sv);
    b.x = dcur; b.xs = L.x; b.r = L.r; b.dinv = L.dinv; b.c1 = L.c1[j - 1]; b.c2 = L.c2[j - 1];
    b.add_d = j == 1; b.store_rd = j < deg - 1; b.y2 = doth; b.rev = L.dir ^= 1;
    if (j == deg - 1 && red.red != RED_NONE) {
      b.red = red.red; b.r64 = red.r64; b.r32 = red.r32; b.r32_old = red.r32_old;
      fused = true;
    }
    launch_spmv<T, OP_CHEB_STEP>(L.A, b, st);
    std::swap(dcur, doth);
  }
  return fused;
}

template <typename T>
void coarse_solve(bd_amg* h, DLevel<T>& L, const Solve& sv, bool d_ready, hipStream_t st) {
  if (h->H.coarse_mode == 1) {
    smooth_pre<T>(h, L, sv, d_ready, st);
    return;
  }
  k_coarse_gemv<T><<<(h->nM + 3) / 4, kBlock, 0, st>>>(sv, h->G, L.f, L.x, h->nM);
  HIPCHK(hipGetLastError());
}

// V-cycle from level k (Alg. 2, mu1 = mu2 = 1): x_k = V(f_k).  Returns true if the level-0
// reductions were fused.
template <typename T>
bool vcycle(bd_amg* h, int k, const Solve& sv, bool d_ready, const RedSpec& red, hipStream_t st) {
  auto& L = levels<T>(h);
  DLevel<T>& Lk = L[k];
  if (k == h->M) {
    coarse_solve<T>(h, Lk, sv, d_ready, st);
    return false;
  }
  smooth_pre<T>(h, Lk, sv, d_ready, st);
  {  // residual
    SpArgs<T> a = args<T>(sv);
    a.x = Lk.x; a.f = Lk.f; a.y = Lk.r; a.rev = Lk.dir ^= 1;
    launch_spmv<T, OP_RESID>(Lk.A, a, st);
  }
  DLevel<T>& Ln = L[k + 1];
  const bool fuse = smoothed_level(h, k + 1);
  {  // restriction (+ first smoothing step of the next level)
    SpArgs<T> a = args<T>(sv);
    a.x = Lk.r; a.y = Ln.f;
    if (fuse) {
      a.y2 = Ln.da; a.dinv2 = Ln.dinv; a.c0 = Ln.c0;
      a.xs = (h->o.smoother == BD_JACOBI || h->o.smoother_degree == 1) ? Ln.x : nullptr;
      launch_spmv<T, OP_RESTRICT>(Lk.R, a, st);
    } else {
      launch_spmv<T, OP_Y>(Lk.R, a, st);
    }
  }
  vcycle<T>(h, k + 1, sv, fuse, RedSpec{}, st);
  {  // prolongation and correction
    SpArgs<T> a = args<T>(sv);
    a.x = Ln.x; a.y = Lk.x;
    launch_spmv<T, OP_ADDY>(Lk.P, a, st);
  }
  return smooth_post<T>(h, Lk, sv, k == 0 ? red : RedSpec{}, st);
}

// Runs the V-cycle on level 0 and makes sure the level-0 reductions happen.
template <typename T>
void precondition(bd_amg* h, const Solve& sv, bool d_ready, const RedSpec& red, hipStream_t st) {
  auto& L = levels<T>(h);
  if constexpr (std::is_same<T, double>::value) {
    if (h->o.preconditioner != BD_PC_AMG) {  // Jacobi or none: one pointwise kernel
      SpArgs<double> a = args<double>(sv);
      a.nrows = L[0].n;
      a.r64 = red.r64;
      a.dinv = h->o.preconditioner == BD_PC_JACOBI ? L[0].dinv : nullptr;
      const int nb = vec_blocks(L[0].n);
      k_pc_diag<<<nb, kBlock, 0, st>>>(a, L[0].x);
      HIPCHK(hipGetLastError());
      finalize(sv, FIN_VC64, nb, st);
      return;
    }
  }
  const bool fused = vcycle<T>(h, 0, sv, d_ready, red, st);
  if (red.red == RED_NONE) return;
  int nb = L[0].A.nb;
  if (!fused) {
    SpArgs<T> a = args<T>(sv);
    a.nrows = L[0].n;
    a.red = red.red; a.r64 = red.r64; a.r32 = red.r32; a.r32_old = red.r32_old;
    nb = vec_blocks(L[0].n);
    k_vc_reduce<T><<<nb, kBlock, 0, st>>>(a, L[0].x);
    HIPCHK(hipGetLastError());
  }
  finalize(sv, red.red == RED_F64 ? FIN_VC64 : FIN_VC32, nb, st);
}

// ------------------------------------------------------------------------------------------
template <typename T>
void build_levels(bd_amg* h, hipStream_t st) {
  auto& L = levels<T>(h);
  const auto& HL = h->H.lv;
  const int nl = (int)HL.size();
  L.resize(nl);
  const int deg = std::max(1, h->o.smoother_degree);
  for (int k = 0; k < nl; ++k) {
    DLevel<T>& D = L[k];
    D.n = HL[k].A.nrows;
    if constexpr (std::is_same<T, double>::value) {
      if (k == 0) D.A = h->A0;  // level 0 of the float64 V-cycle is the outer operator itself
    }
    if (D.A.n == 0)
      D.A = upload<T>(h->ar, HL[k].A, k == 0 ? &h->A0 : nullptr, HL[k].plan_a.get(), false, st, kMaxBlocksSpmv);
    if (k < nl - 1) {
      D.P = upload<T>(h->ar, HL[k].P, nullptr, HL[k].plan_p.get(), false, st, kMaxBlocksSpmv);
      D.R = upload<T>(h->ar, HL[k].R, nullptr, HL[k].plan_r.get(), false, st, kMaxBlocksSpmv);
    }
    if (HL[k].perm.empty()) {
      D.dinv = upload_vec<T>(h->ar, HL[k].Dinv, st);
    } else {
      std::vector<double> dp(HL[k].perm.size());
      for (size_t i = 0; i < dp.size(); ++i) dp[i] = HL[k].Dinv[HL[k].perm[i]];
      D.dinv = upload_vec<T>(h->ar, dp, st);
      D.perm = upload_small<int>(h->ar, HL[k].perm, st);
    }
    if (k > 0) D.f = h->ar.alloc<T>(D.n);
    D.x = h->ar.alloc<T>(D.n);
    D.r = h->ar.alloc<T>(D.n);
    D.da = h->ar.alloc<T>(D.n);
    D.db = h->ar.alloc<T>(D.n);
    D.lam = HL[k].lam;
    if (smoothed_level(h, k)) {
      if (h->o.smoother == BD_JACOBI) {
        D.c0 = (T)(4.0 / (3.0 * D.lam));
      } else {
        // Chebyshev three-term recurrence on [lo, hi] * lambda (Saad, Iterative Methods, Alg. 12.1)
        const double a = h->o.cheb_lo * D.lam, b = h->o.cheb_hi * D.lam;
        const double theta = 0.5 * (a + b), delta = 0.5 * (b - a), sigma = theta / delta;
        double rho = 1.0 / sigma;
        D.c0 = (T)(1.0 / theta);
        for (int j = 1; j < deg; ++j) {
          const double rn = 1.0 / (2.0 * sigma - rho);
          D.c1.push_back((T)(rn * rho));
          D.c2.push_back((T)(2.0 * rn / delta));
          rho = rn;
        }
      }
    }
  }
}

// dst[i] = src[perm[i]] (into a renumbered level's device numbering, TO_DEVICE) or
// dst[perm[i]] = src[i] (back to the host's numbering).
template <typename T, bool TO_DEVICE>
__global__ void k_renumber(const T* __restrict__ src, T* __restrict__ dst, const int* __restrict__ perm, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    if (TO_DEVICE) dst[i] = src[perm[i]];
    else dst[perm[i]] = src[i];
  }
}

void alloc_solve_state(bd_amg* h, hipStream_t st) {
  Arena& ar = h->ar;
  const int n = h->n;
  h->r = ar.alloc<double>(n);
  h->p = ar.alloc<double>(n);
  h->q = ar.alloc<double>(n);
  if (h->mixed) {
    h->r32[0] = ar.alloc<float>(n);
    h->r32[1] = ar.alloc<float>(n);
  }
  int64_t maxnb = vec_blocks(n);
  auto upd = [&](int nb) { maxnb = std::max<int64_t>(maxnb, nb); };
  upd(h->A0.nb);
  if (h->mixed) upd(h->L32[0].A.nb); else upd(h->L64[0].A.nb);
  h->part_len = 4 * maxnb + 16;
  for (Solve* s : {&h->sv, &h->sv_apply}) {
    s->sc = ar.alloc<double>(S_COUNT);
    s->fl = ar.alloc<int>(F_COUNT);
    s->part = ar.alloc<double>(h->part_len);
    s->n = n;
    HIPCHK(hipMemsetAsync(s->sc, 0, S_COUNT * sizeof(double), st));
    HIPCHK(hipMemsetAsync(s->fl, 0, F_COUNT * sizeof(int), st));
  }
  // fine-grained (coherent) pinned memory: the update kernel's system-scope stores are seen
  // by the host as soon as the event after that kernel completes
  HIPCHK(hipHostMalloc(&h->host_flags, 4 * sizeof(int), hipHostMallocCoherent | hipHostMallocMapped));
  std::memset(h->host_flags, 0, 4 * sizeof(int));
  int* dflags = nullptr;
  HIPCHK(hipHostGetDevicePointer((void**)&dflags, h->host_flags, 0));
  h->sv.host_flags = dflags;
  h->sv_apply.host_flags = nullptr;
  HIPCHK(hipEventCreate(&h->ev_start));
  HIPCHK(hipEventCreate(&h->ev_stop));
  HIPCHK(hipEventCreateWithFlags(&h->ev_iter[0], hipEventDisableTiming));
  HIPCHK(hipEventCreateWithFlags(&h->ev_iter[1], hipEventDisableTiming));
  HIPCHK(hipStreamSynchronize(st));
}

// ------------------------------------------------------------------------------------------
// The solve.  sv: the solve state (scalars, flags, block partials) the kernels use: the
// handle's own (h->sv), or the same layout in the library's static scratch array.  profile:
// allow the per-launch timing events of bidomain_profile_enable (they are created per call).
template <typename T>
int pcg(bd_amg* h, const Solve& sv, const double* b, double* x, int guess, double rtol, int maxit, hipStream_t st,
        bd_solve_info* info, bool profile = true) {
  const int n = h->n;
  auto& L = levels<T>(h);
  hipEvent_t t0 = h->ev_start, t1 = h->ev_stop;
  HIPCHK(hipEventRecord(t0, st));

  // solve state: flags, iteration cap, null-space switch and rtol^2, set on the device queue
  k_solve_control<<<1, 64, 0, st>>>(sv, 0, std::max(1, maxit), h->o.nullspace == BD_NULL_CONSTANT, rtol * rtol);
  HIPCHK(hipGetLastError());
  h->host_flags[0] = h->host_flags[1] = 0;

  const int vb = vec_blocks(n);
  k_init_means<<<vb, kBlock, 0, st>>>(sv, b, guess ? x : nullptr, n);
  HIPCHK(hipGetLastError());
  finalize(sv, FIN_MEANS, vb, st);
  k_init_guess<<<vb, kBlock, 0, st>>>(sv, x, guess, n);
  HIPCHK(hipGetLastError());
  {
    SpArgs<double> a = args<double>(sv);
    a.x = x; a.y = h->r; a.b = b;
    launch_spmv<double, OP_INIT_RESID>(h->A0, a, st);
    finalize(sv, FIN_INIT, h->A0.nb, st);
  }
  int flags[F_COUNT];
  HIPCHK(hipMemcpyAsync(flags, sv.fl, sizeof(flags), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));

  if (!flags[F_DONE]) {
    const bool mixed = h->mixed;
    // level-0 right-hand side of the V-cycle
    int cur = 0;
    RedSpec red;
    if (mixed) {
      k_convert<double, float><<<vb, kBlock, 0, st>>>(h->r, h->r32[0], n);
      HIPCHK(hipGetLastError());
      L[0].f = (T*)h->r32[0];
      red.red = RED_F32; red.r32 = h->r32[0]; red.r32_old = h->r32[0];
    } else {
      L[0].f = (T*)h->r;
      red.red = RED_F64; red.r64 = h->r;
    }
    precondition<T>(h, sv, false, red, st);
    k_cg_direction<T><<<vb, kBlock, 0, st>>>(sv, h->p, L[0].x, n);
    k_clear_first<<<1, 64, 0, st>>>(sv);
    HIPCHK(hipGetLastError());

    const bool fuse0 = smoothed_level(h, 0) && h->o.preconditioner == BD_PC_AMG;
    const bool x0_too = h->o.smoother == BD_JACOBI || h->o.smoother_degree == 1;
    hipEvent_t* ev = h->ev_iter;
    std::unique_lock<std::mutex> plock(g_prof.mu, std::defer_lock);
    if (profile) plock.lock();
    const bool prof = profile && g_prof.on;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pev;
    int enq = 0;
    for (;;) {
      // q = A p, alpha
      SpArgs<double> a = args<double>(sv);
      a.x = h->p; a.y = h->q;
      if (prof) {
        hipEvent_t e0, e1;
        HIPCHK(hipEventCreate(&e0));
        HIPCHK(hipEventCreate(&e1));
        HIPCHK(hipEventRecord(e0, st));
        launch_spmv<double, OP_CG_Q>(h->A0, a, st);
        HIPCHK(hipEventRecord(e1, st));
        pev.push_back({e0, e1});
      } else {
        launch_spmv<double, OP_CG_Q>(h->A0, a, st);
      }
      finalize(sv, FIN_CGQ, h->A0.nb, st);
      // x, r update, convergence test, next V-cycle right-hand side
      float* r32n = mixed ? h->r32[cur ^ 1] : nullptr;
      T* f0 = mixed ? (T*)r32n : (T*)h->r;
      k_cg_update<T><<<vb, kBlock, 0, st>>>(sv, x, h->r, h->p, h->q, r32n, L[0].dinv, fuse0 ? L[0].da : nullptr,
                                           (fuse0 && x0_too) ? L[0].x : nullptr, L[0].c0, n);
      HIPCHK(hipGetLastError());
      finalize(sv, FIN_UPDATE, vb, st);
      HIPCHK(hipEventRecord(ev[enq & 1], st));
      if (mixed) {
        red.r32_old = h->r32[cur];
        red.r32 = r32n;
        cur ^= 1;
      }
      L[0].f = f0;
      precondition<T>(h, sv, fuse0, red, st);
      k_cg_direction<T><<<vb, kBlock, 0, st>>>(sv, h->p, L[0].x, n);
      HIPCHK(hipGetLastError());
      ++enq;
      // look one iteration behind: the update of iteration enq-1 has finished (or will soon)
      if (enq >= 2 || enq > maxit) {
        HIPCHK(hipEventSynchronize(ev[(enq - 2) & 1]));  // update kernel of iteration enq - 1
        const int done = __atomic_load_n(&h->host_flags[0], __ATOMIC_ACQUIRE);
        if (done || enq > maxit) break;
      }
    }
    HIPCHK(hipStreamSynchronize(st));
    if (prof) {
      // launch j computes q for iteration j + 1; the launches enqueued after the converging
      // iteration found the done flag set and returned at once, so only the first
      // `iterations` launches did the product
      HIPCHK(hipMemcpyAsync(flags, sv.fl, sizeof(flags), hipMemcpyDeviceToHost, st));
      HIPCHK(hipStreamSynchronize(st));
      const size_t worked = std::min<size_t>(pev.size(), (size_t)std::max(0, flags[F_ITERS]));
      for (size_t j = 0; j < pev.size(); ++j) {
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, pev[j].first, pev[j].second));
        (void)hipEventDestroy(pev[j].first);
        (void)hipEventDestroy(pev[j].second);
        if (j < worked) g_prof.total_ms += ms;
      }
      g_prof.launches += (int64_t)worked;
    }
  } else if (flags[F_STATUS] == 0) {
    // b^ = 0 gives x = 0; a converged initial guess is kept
  }

  double sc[S_COUNT];
  HIPCHK(hipMemcpyAsync(sc, sv.sc, sizeof(sc), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(flags, sv.fl, sizeof(flags), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const bool zero_rhs = sc[S_FNORM2] == 0.0;
  if (zero_rhs) {
    k_fill_zero<double><<<vec_blocks(n), kBlock, 0, st>>>(x, n);
    HIPCHK(hipGetLastError());
  }
  // true residual, then the null-space normalisation (the exit kernels run once `done` is clear)
  Solve svx = sv;
  k_solve_control<<<1, 64, 0, st>>>(sv, 1, 0, 0, 0.0);
  HIPCHK(hipGetLastError());
  if (!zero_rhs) {
    SpArgs<double> a = args<double>(svx);
    a.x = x; a.b = b;
    launch_spmv<double, OP_TRUE_RESID>(h->A0, a, st);
    finalize(svx, FIN_TRUE, h->A0.nb, st);
  }
  if (h->o.nullspace == BD_NULL_CONSTANT && !zero_rhs) {
    k_norm_sums<<<vb, kBlock, 0, st>>>(svx, h->w, x, n);
    HIPCHK(hipGetLastError());
    finalize(svx, FIN_NORM, vb, st);
    k_norm_apply<<<vb, kBlock, 0, st>>>(svx, x, n);
    HIPCHK(hipGetLastError());
  }
  HIPCHK(hipEventRecord(t1, st));
  HIPCHK(hipMemcpyAsync(sc, sv.sc, sizeof(sc), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, t0, t1));

  int status = flags[F_STATUS];
  const double fn = sc[S_FNORM2];
  bd_solve_info inf{};
  inf.iterations = flags[F_ITERS];
  inf.rel_residual_rec = fn > 0 ? std::sqrt(sc[S_RNORM2] / fn) : 0.0;
  inf.rel_residual_true = fn > 0 ? std::sqrt(sc[S_TRUE2] / fn) : 0.0;
  inf.seconds = ms * 1e-3;
  if (status == 0 && !std::isfinite(inf.rel_residual_true)) status = BD_E_NONFINITE;
  inf.status = status;
  if (info) *info = inf;
  h->last_iters = std::max(1, inf.iterations);
  if (status == BD_E_BREAKDOWN) g_last_error = "CG breakdown (p^T A p <= 0 or r^T z <= 0)";
  if (status == BD_E_NONFINITE) g_last_error = "non-finite value in the right-hand side or an iterate";
  if (status == BD_E_NOT_CONVERGED) g_last_error = "iteration cap reached before convergence";
  return status;
}

}  // namespace bd

namespace bd {
// Aliev-Panfilov parameters of a case (bd_slab, bd_ellipsoid; published values k = 8, a = 0.15,
// eps0 = 0.002, mu1 = 0.2, mu2 = 0.3, one model time unit = 12.9 ms, u = (v + 85) / 105).
struct ApParams {
  double k, a, eps0, mu1, mu2, t_unit, v_scale, v_rest;
};
template <typename Case>
inline ApParams ap_params(const Case& s) {
  return ApParams{s.ap_k, s.ap_a, s.ap_eps0, s.ap_mu1, s.ap_mu2, s.ap_t_unit, s.ap_v_scale, s.ap_v_rest};
}
// What a time step needs of a case beyond its operators.
struct SimPhysics {
  double cm = 0, dt = 0;
  ApParams ap{};
};
template <typename Case>
inline SimPhysics sim_physics(const Case& s) {
  return SimPhysics{s.cm, s.dt, ap_params(s)};
}
}  // namespace bd

// ==========================================================================================
// Simulation handle.
struct bd_sim {
  bd::SimPhysics ph{};
  int n = 0;
  bd_amg* hell = nullptr;
  bd_amg* hpar = nullptr;
  Arena ar;
  DCsr<double> Ai;
  double *v = nullptr, *ue = nullptr, *w = nullptr, *m = nullptr, *rhs = nullptr, *fell = nullptr;
  ~bd_sim() {
    delete hell;
    delete hpar;
  }
};

namespace bd {


// One membrane step and the parabolic right-hand side (eqs. (4), (7)):
//   w <- (w + dt' eps (-k u (u - a - 1))) / (1 + dt' eps),   eps = eps0 + mu1 w / (u + mu2),
//   I_ion = -cm (105 / 12.9) [k u (u - a)(1 - u) - u w_new],
//   rhs = (cm / dt) m v - (A_i u_e) - m I_ion.
template <int G>
__global__ __launch_bounds__(kBlock) void k_membrane_rhs(const int* __restrict__ rp, const int* __restrict__ ci,
                                                         const double* __restrict__ av, const double* __restrict__ ue,
                                                         const double* __restrict__ v, double* __restrict__ w,
                                                         const double* __restrict__ m, double* __restrict__ rhs,
                                                         double dt, double cm, ApParams ap, int n) {
  constexpr int RPT = kBlock / G;
  const int row = xcd_tile(blockIdx.x, gridDim.x) * RPT + threadIdx.x / G;
  const int lane = threadIdx.x % G;
  if (row >= n) return;
  const double s = row_product<double, G>(rp, ci, av, ue, row, lane);
  if (lane != 0) return;
  const double u = (v[row] - ap.v_rest) / ap.v_scale;
  const double dtp = dt / ap.t_unit;
  const double wo = w[row];
  const double eps = ap.eps0 + ap.mu1 * wo / (u + ap.mu2);
  const double wn = (wo + dtp * eps * (-ap.k * u * (u - ap.a - 1.0))) / (1.0 + dtp * eps);
  w[row] = wn;
  const double iion = -cm * (ap.v_scale / ap.t_unit) * (ap.k * u * (u - ap.a) * (1.0 - u) - u * wn);
  rhs[row] = (cm / dt) * m[row] * v[row] - s - m[row] * iion;
}

// y = -A x (right-hand side of the elliptic system, eq. (6)).
template <int G>
__global__ __launch_bounds__(kBlock) void k_neg_spmv(const int* __restrict__ rp, const int* __restrict__ ci,
                                                     const double* __restrict__ av, const double* __restrict__ x,
                                                     double* __restrict__ y, int n) {
  constexpr int RPT = kBlock / G;
  const int row = xcd_tile(blockIdx.x, gridDim.x) * RPT + threadIdx.x / G;
  const int lane = threadIdx.x % G;
  if (row >= n) return;
  const double s = row_product<double, G>(rp, ci, av, x, row, lane);
  if (lane == 0) y[row] = -s;
}

// Second half of the setup phase: copy a host-built hierarchy into HBM and allocate the
// solve state.  weights: n host doubles (normalisation weights) or null.
// need_ci: keep the fine operator's 32-bit column indices (a simulation's A_i shares its
// pattern and the step kernels read them).
void device_upload(bd_amg* h, const double* weights, bool need_ci, hipStream_t st) {
  h->A0 = upload<double>(h->ar, h->H.lv[0].A, nullptr, h->H.lv[0].plan_a.get(), need_ci, st, kMaxBlocksSpmv);
  if (h->mixed) build_levels<float>(h, st);
  else build_levels<double>(h, st);
  if (h->H.coarse_mode == 0) {
    h->nM = h->H.lv.back().A.nrows;
    h->G = upload_vec<double>(h->ar, h->H.G, st);
  }
  if (h->o.nullspace == BD_NULL_CONSTANT && weights) {
    std::vector<double> wv(weights, weights + h->n);
    h->w = upload_vec<double>(h->ar, wv, st);
  }
  alloc_solve_state(h, st);
  release_plan_matrices(h->H);
  h->host_only = false;
}

// ------------------------------------------------------------------------------------------
// Sparse Galerkin products on the device (setup phase): A_c = (R (A P) + (R (A P))^T) / 2 with
// this library's product kernels (spgemm.hpp).  They sum every entry in the host product's
// order with separately rounded operations, so the hierarchy is the host's bit for bit.

std::mutex g_galerkin_mu;  // one device Galerkin product at a time (its buffers are large)

// Device memory a setup may take for transient buffers: reserve(bytes) returns false when the
// bytes are not available (the product then runs on the host); release(bytes) gives them back.
struct TransientBudget {
  std::function<bool(int64_t)> reserve;
  std::function<void(int64_t)> release;
};

namespace {

struct DevCsr {
  int n = 0, ncols = 0;
  int64_t nnz = 0;
  int *rp = nullptr, *ci = nullptr;
  double* v = nullptr;
};

// Transient buffers of one Galerkin product: each allocation must fit in half the free device
// memory and, with a budget, be reserved from it first; all are freed (and the reservations
// given back) when the scope ends.  `ok` turns false at the first refusal.
struct DevScratch {
  const TransientBudget* tb = nullptr;
  std::vector<void*> bufs;
  int64_t reserved = 0;
  bool ok = true;
  ~DevScratch() {
    for (void* q : bufs) (void)hipFree(q);
    if (tb && reserved) tb->release(reserved);
  }
  template <typename T>
  T* alloc(int64_t count) {
    if (!ok) return nullptr;
    const int64_t bytes = std::max<int64_t>(1, count) * (int64_t)sizeof(T);
    size_t freeb = 0, total = 0;
    if (hipMemGetInfo(&freeb, &total) != hipSuccess || bytes > (int64_t)(freeb / 2)) {
      ok = false;
      return nullptr;
    }
    if (tb) {
      if (!tb->reserve(bytes)) {
        ok = false;
        return nullptr;
      }
      reserved += bytes;
    }
    void* q = nullptr;
    if (hipMalloc(&q, bytes) != hipSuccess) {
      (void)hipGetLastError();
      ok = false;
      return nullptr;
    }
    bufs.push_back(q);
    return (T*)q;
  }
  void check(hipError_t e) {
    if (e != hipSuccess) {
      (void)hipGetLastError();
      ok = false;
    }
  }
};

DevCsr upload_csr(DevScratch& s, const Csr& H, hipStream_t st) {
  DevCsr D;
  D.n = H.nrows;
  D.ncols = H.ncols;
  D.nnz = H.nnz();
  D.rp = s.alloc<int>(D.n + 1);
  D.ci = s.alloc<int>(D.nnz);
  D.v = s.alloc<double>(D.nnz);
  if (!s.ok) return D;
  s.check(hipMemcpyAsync(D.rp, H.rp.data(), sizeof(int) * (D.n + 1), hipMemcpyHostToDevice, st));
  if (D.nnz) {
    s.check(hipMemcpyAsync(D.ci, H.ci.data(), sizeof(int) * D.nnz, hipMemcpyHostToDevice, st));
    s.check(hipMemcpyAsync(D.v, H.v.data(), sizeof(double) * D.nnz, hipMemcpyHostToDevice, st));
  }
  return D;
}

int grid_for(int64_t units, int per_block, int cap) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(cap, (units + per_block - 1) / per_block));
}

// C = A B on the device (C's buffers from s); false when memory is refused or a call fails.
// log: print the time of each pass.
bool device_spgemm(DevScratch& s, const DevCsr& A, const DevCsr& B, DevCsr& C, hipStream_t st, bool log) {
  using namespace sg;
  const int n = A.n, p = B.ncols;
  const auto t0 = std::chrono::steady_clock::now();
  auto lap = [&](const char* what) {
    if (!log) return;
    s.check(hipStreamSynchronize(st));
    std::fprintf(stderr, "[setup]   product %d x %d (B %d cols, nnz A %lld B %lld): %s at %.3f s\n", n, A.ncols, p,
                 (long long)A.nnz, (long long)B.nnz, what,
                 std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
  };
  int* u = s.alloc<int>(n);
  int* cnt = s.alloc<int>(n);
  if (!s.ok) return false;
  k_sg_products<<<grid_for(n, kBlock, 4096), kBlock, 0, st>>>(A.rp, A.ci, B.rp, n, u);
  s.check(hipGetLastError());
  std::vector<int> hv(n);
  s.check(hipMemcpyAsync(hv.data(), u, sizeof(int) * n, hipMemcpyDeviceToHost, st));
  s.check(hipStreamSynchronize(st));
  if (!s.ok) return false;
  std::vector<int> big;
  int64_t products = 0;
  for (int i = 0; i < n; ++i) {
    products += hv[i];
    if (hv[i] > kSmallProducts) big.push_back(i);
  }
  const int nbig = (int)big.size();
  if (log) std::fprintf(stderr, "[setup]   product: %lld partial products, %d big rows\n", (long long)products, nbig);
  // big rows: a column bitmap in LDS when C has at most kDenseCols columns, else mark arrays of
  // p ints per block (at most 4 GiB together)
  // (dense accumulators of p doubles per block, at most 2 GiB together)
  const bool dense = p <= kDenseCols;
  const int gbig = !nbig ? 0
                   : dense ? (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)nbig, 2048, (1LL << 28) / std::max(1, p)}))
                           : (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)nbig, 1024, (1LL << 30) / std::max(1, p)}));
  int* dbig = nbig ? s.alloc<int>(nbig) : nullptr;
  int* marks = nbig && !dense ? s.alloc<int>((int64_t)gbig * p) : nullptr;
  double* accg = nbig && dense ? s.alloc<double>((int64_t)gbig * p) : nullptr;
  if (!s.ok) return false;
  if (nbig) s.check(hipMemcpyAsync(dbig, big.data(), sizeof(int) * nbig, hipMemcpyHostToDevice, st));
  if (marks) s.check(hipMemsetAsync(marks, 0xff, sizeof(int) * (size_t)gbig * p, st));  // -1
  if (accg) s.check(hipMemsetAsync(accg, 0, sizeof(double) * (size_t)gbig * p, st));
  const int gsmall = grid_for(n, 1, 65536);
  k_sg_small<0><<<gsmall, kSmallBlock, 0, st>>>(A.rp, A.ci, B.rp, B.ci, u, n, cnt, nullptr, nullptr);
  if (nbig && dense) k_sg_dense_sym<0><<<gbig, kBigBlock, 0, st>>>(A.rp, A.ci, B.rp, B.ci, dbig, nbig, p, cnt, nullptr, nullptr);
  if (nbig && !dense) k_sg_big<0><<<gbig, kBigBlock, 0, st>>>(A.rp, A.ci, B.rp, B.ci, dbig, nbig, n, p, marks, cnt, nullptr, nullptr);
  s.check(hipGetLastError());
  lap("counted");
  s.check(hipMemcpyAsync(hv.data(), cnt, sizeof(int) * n, hipMemcpyDeviceToHost, st));
  s.check(hipStreamSynchronize(st));
  if (!s.ok) return false;
  std::vector<int> rp(n + 1, 0);
  int64_t total = 0;
  for (int i = 0; i < n; ++i) {
    total += hv[i];
    if (total > INT32_MAX) return false;
    rp[i + 1] = (int)total;
  }
  C.n = n;
  C.ncols = p;
  C.nnz = total;
  C.rp = s.alloc<int>(n + 1);
  C.ci = s.alloc<int>(total);
  C.v = s.alloc<double>(total);
  if (!s.ok) return false;
  s.check(hipMemcpyAsync(C.rp, rp.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice, st));
  k_sg_small<1><<<gsmall, kSmallBlock, 0, st>>>(A.rp, A.ci, B.rp, B.ci, u, n, nullptr, C.rp, C.ci);
  if (nbig && dense) k_sg_dense_sym<1><<<gbig, kBigBlock, 0, st>>>(A.rp, A.ci, B.rp, B.ci, dbig, nbig, p, nullptr, C.rp, C.ci);
  if (nbig && !dense) k_sg_big<1><<<gbig, kBigBlock, 0, st>>>(A.rp, A.ci, B.rp, B.ci, dbig, nbig, n, p, marks, nullptr, C.rp, C.ci);
  lap("columns");
  k_sg_num_small<<<gsmall, kSmallBlock, 0, st>>>(A.rp, A.ci, A.v, B.rp, B.ci, B.v, u, n, C.rp, C.ci, C.v);
  if (nbig && dense) k_sg_dense_num<<<gbig, kBigBlock, 0, st>>>(A.rp, A.ci, A.v, B.rp, B.ci, B.v, dbig, nbig, p, accg, C.rp, C.ci, C.v);
  if (nbig && !dense) k_sg_num_big<<<gbig, kBigBlock, 0, st>>>(A.rp, A.ci, A.v, B.rp, B.ci, B.v, dbig, nbig, C.rp, C.ci, C.v);
  s.check(hipGetLastError());
  s.check(hipStreamSynchronize(st));
  lap("values");
  return s.ok;
}

// A_c = sym(R (A P)) as block-sparse MFMA products of dense expansions (galerkin_dense.hpp), the
// pattern from row bitmaps; fills Ac on the host.  false when memory is refused or a call fails.
bool dense_galerkin_dev(DevScratch& s, const DevCsr& A, const DevCsr& P, const DevCsr& R, Csr& Ac, hipStream_t st,
                        bool log) {
  using namespace gd;
  const auto t0 = std::chrono::steady_clock::now();
  const int n = A.n, nc = P.ncols;
  const int64_t np = (n + kTile - 1) / kTile * kTile, ncp = (nc + kTile - 1) / kTile * kTile;
  const int W = (nc + 31) / 32;
  double* dA = s.alloc<double>(np * np);
  double* dP = s.alloc<double>(np * ncp);
  double* dR = s.alloc<double>(ncp * np);
  double* dAP = s.alloc<double>(np * ncp);
  double* dRAP = s.alloc<double>(ncp * ncp);
  const int nkt = (int)(np / kKStep);
  uint8_t* occA = s.alloc<uint8_t>(np / kTile * nkt);
  uint8_t* occR = s.alloc<uint8_t>(ncp / kTile * nkt);
  uint32_t* bP = s.alloc<uint32_t>((int64_t)n * W);
  uint32_t* bAP = s.alloc<uint32_t>((int64_t)n * W);
  uint32_t* bRAP = s.alloc<uint32_t>((int64_t)nc * W);
  int* cnt = s.alloc<int>(nc);
  if (!s.ok) return false;
  s.check(hipMemsetAsync(dA, 0, sizeof(double) * np * np, st));
  s.check(hipMemsetAsync(dP, 0, sizeof(double) * np * ncp, st));
  s.check(hipMemsetAsync(dR, 0, sizeof(double) * ncp * np, st));
  s.check(hipMemsetAsync(occA, 0, np / kTile * nkt, st));
  s.check(hipMemsetAsync(occR, 0, ncp / kTile * nkt, st));
  s.check(hipMemsetAsync(bP, 0, sizeof(uint32_t) * n * W, st));
  const int g = grid_for(std::max(n, nc), 1, 65536);
  k_gd_densify<<<g, kBlock, 0, st>>>(A.rp, A.ci, A.v, n, np, dA);
  k_gd_densify<<<g, kBlock, 0, st>>>(P.rp, P.ci, P.v, n, ncp, dP);
  k_gd_densify<<<g, kBlock, 0, st>>>(R.rp, R.ci, R.v, nc, np, dR);
  k_gd_occupancy<<<g, kBlock, 0, st>>>(A.rp, A.ci, n, nkt, occA);
  k_gd_occupancy<<<g, kBlock, 0, st>>>(R.rp, R.ci, nc, nkt, occR);
  k_gd_row_bits<<<g, kBlock, 0, st>>>(P.rp, P.ci, n, W, bP);
  k_gd_or_rows<<<g, kBlock, 0, st>>>(A.rp, A.ci, n, W, bP, bAP);
  k_gd_or_rows<<<g, kBlock, 0, st>>>(R.rp, R.ci, nc, W, bAP, bRAP);
  k_gd_count<<<g, kBlock, 0, st>>>(bRAP, nc, W, cnt);
  k_gd_gemm<<<dim3((unsigned)(ncp / kTile), (unsigned)(np / kTile)), 256, 0, st>>>(dA, np, dP, ncp, dAP, ncp, nkt, occA);
  k_gd_gemm<<<dim3((unsigned)(ncp / kTile), (unsigned)(ncp / kTile)), 256, 0, st>>>(dR, np, dAP, ncp, dRAP, ncp, nkt, occR);
  s.check(hipGetLastError());
  std::vector<int> hc(nc);
  s.check(hipMemcpyAsync(hc.data(), cnt, sizeof(int) * nc, hipMemcpyDeviceToHost, st));
  s.check(hipStreamSynchronize(st));
  if (!s.ok) return false;
  Ac = Csr();
  Ac.nrows = Ac.ncols = nc;
  Ac.rp.assign(nc + 1, 0);
  for (int i = 0; i < nc; ++i) {
    if ((int64_t)Ac.rp[i] + hc[i] > INT32_MAX) return false;
    Ac.rp[i + 1] = Ac.rp[i] + hc[i];
  }
  const int64_t nnz = Ac.rp[nc];
  int* crp = s.alloc<int>(nc + 1);
  int* cci = s.alloc<int>(nnz);
  double* cv = s.alloc<double>(nnz);
  if (!s.ok) return false;
  s.check(hipMemcpyAsync(crp, Ac.rp.data(), sizeof(int) * (nc + 1), hipMemcpyHostToDevice, st));
  k_gd_extract<<<grid_for(nc, 1, 65536), 256, 0, st>>>(bRAP, nc, W, crp, cci);
  k_gd_values<<<grid_for(nc, kBlock / 64, 8192), kBlock, 0, st>>>(crp, cci, nc, dRAP, ncp, cv);
  s.check(hipGetLastError());
  Ac.ci.resize(nnz);
  Ac.v.resize(nnz);
  if (nnz) {
    s.check(hipMemcpyAsync(Ac.ci.data(), cci, sizeof(int) * nnz, hipMemcpyDeviceToHost, st));
    s.check(hipMemcpyAsync(Ac.v.data(), cv, sizeof(double) * nnz, hipMemcpyDeviceToHost, st));
  }
  s.check(hipStreamSynchronize(st));
  if (log)
    std::fprintf(stderr, "[setup]   dense product %d x %d -> %d: %.3f s\n", n, n, nc,
                 std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
  return s.ok;
}

}  // namespace

// Galerkin product A_c = sym(R (A P)) on the device.  mode 0: never.  1: levels with at least 5e7
// partial products in A P (smaller ones are as fast on the host); those of at most 65,536 rows
// and columns whose dense contraction is within 1000 times the partial products of A P (the
// filled coarse levels) as MFMA products (equal to the host's up to rounding order), the others
// as sparse products (equal bit for bit).  2: every level, sparse.  3: every level of at most
// 65,536 rows and columns dense, the others sparse.  Returns false (the host computes the
// product) when the device memory or the budget is not available.
bool sparse_galerkin(const Csr& A, const Csr& P, const Csr& R, int64_t sparse_flops, int mode, bool log, Csr& Ac,
                     const TransientBudget* tb) {
  if (mode == 0 || A.nrows == 0 || P.ncols == 0) return false;
  if (mode == 1 && sparse_flops < 50000000LL) return false;
  const double n = A.nrows, nc = P.ncols;
  const bool fits = n <= sg::kDenseCols && nc <= sg::kDenseCols;
  const bool dense = fits && (mode == 3 || (mode == 1 && 2.0 * n * n * nc + 2.0 * nc * n * nc <= 1000.0 * (double)sparse_flops));
  std::lock_guard<std::mutex> lock(g_galerkin_mu);
  hipStream_t st = nullptr;
  if (hipStreamCreate(&st) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  bool ok = false;
  for (int attempt = dense ? 0 : 1; attempt < 2 && !ok; ++attempt) {
    DevScratch s;
    s.tb = tb;
    const DevCsr dA = upload_csr(s, A, st), dP = upload_csr(s, P, st), dR = upload_csr(s, R, st);
    if (!s.ok) continue;
    if (attempt == 0) {
      ok = dense_galerkin_dev(s, dA, dP, dR, Ac, st, log);
      if (!ok && log) std::fprintf(stderr, "[setup] dense device Galerkin product unavailable, trying the sparse one\n");
      continue;
    }
    DevCsr AP, RAP;
    if (device_spgemm(s, dA, dP, AP, st, log) && device_spgemm(s, dR, AP, RAP, st, log)) {
      double* sym = s.alloc<double>(RAP.nnz);
      if (s.ok) {
        sg::k_sg_symmetrize<<<grid_for(RAP.n, kBlock / 64, 8192), kBlock, 0, st>>>(RAP.rp, RAP.ci, RAP.v, RAP.n, sym);
        s.check(hipGetLastError());
        Ac = Csr();
        Ac.nrows = RAP.n;
        Ac.ncols = RAP.ncols;
        Ac.rp.resize(RAP.n + 1);
        Ac.ci.resize(RAP.nnz);
        Ac.v.resize(RAP.nnz);
        s.check(hipMemcpyAsync(Ac.rp.data(), RAP.rp, sizeof(int) * (RAP.n + 1), hipMemcpyDeviceToHost, st));
        if (RAP.nnz) {
          s.check(hipMemcpyAsync(Ac.ci.data(), RAP.ci, sizeof(int) * RAP.nnz, hipMemcpyDeviceToHost, st));
          s.check(hipMemcpyAsync(Ac.v.data(), sym, sizeof(double) * RAP.nnz, hipMemcpyDeviceToHost, st));
        }
        s.check(hipStreamSynchronize(st));
        ok = s.ok;
      }
    }
  }
  (void)hipStreamDestroy(st);
  if (!ok && log) std::fprintf(stderr, "[setup] device Galerkin product unavailable, using the host\n");
  return ok;
}

// SA coarsening of a level on the device (aggregate.hpp): eigenvalue estimate, strength graph,
// parallel independent set, aggregation passes and the prolongator smoothing's product and
// combination; the O(n)
// bookkeeping between them (aggregate ranks, the tentative prolongator's norms in index order)
// on the host with the host's own routine.  The result is the host setup's bit for bit (tests
// compare whole hierarchies).  false (the host builds the level) when memory is refused or a
// call fails.
bool device_sa_level(const Csr& A, const std::vector<double>& d, const std::vector<double>& Dinv,
                     const std::vector<double>& B, int level, const bd_amg_opts& o, bool log, double& lam, Csr& P,
                     std::vector<double>& Bc, int32_t& nc, const TransientBudget* tb) {
  using namespace ag;
  const int n = A.nrows;
  const bool square = level < o.square_graph_levels;
  std::lock_guard<std::mutex> lock(g_galerkin_mu);
  hipStream_t st = nullptr;
  if (hipStreamCreate(&st) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  bool ok = false;
  {
    DevScratch s;
    s.tb = tb;
    const auto t0 = std::chrono::steady_clock::now();
    const DevCsr dA = upload_csr(s, A, st);
    double* dd = s.alloc<double>(n);
    double* ddinv = s.alloc<double>(n);
    int* cnt = s.alloc<int>(n);
    if (!s.ok) goto done;
    s.check(hipMemcpyAsync(dd, d.data(), sizeof(double) * n, hipMemcpyHostToDevice, st));
    s.check(hipMemcpyAsync(ddinv, Dinv.data(), sizeof(double) * n, hipMemcpyHostToDevice, st));
    {  // eigenvalue estimate: the host's Jacobi-CG steps and dot-product order
      const int g = grid_for(n, kBlock, 8192);
      double *r = s.alloc<double>(n), *z = s.alloc<double>(n), *p = s.alloc<double>(n), *q = s.alloc<double>(n);
      const int64_t nb = (n + kDotBlock - 1) / kDotBlock;
      double* part = s.alloc<double>(nb);
      if (!s.ok) goto done;
      std::vector<double> hp(nb);
      auto dot = [&](const double* a, const double* b) {
        k_lam_dot_blocks<kDotBlock><<<(int)std::min<int64_t>(nb, 65536), 64, 0, st>>>(a, b, n, part);
        s.check(hipMemcpyAsync(hp.data(), part, sizeof(double) * nb, hipMemcpyDeviceToHost, st));
        s.check(hipStreamSynchronize(st));
        double acc = 0.0;
        for (double v : hp) acc += v;
        return acc;
      };
      k_lam_init<<<g, kBlock, 0, st>>>(n, o.seed + (uint64_t)level, ddinv, r, z, p);
      double rho = dot(r, z);
      const double rho0 = rho;
      std::vector<double> alpha, beta;
      for (int j = 0; j < o.esteig_iters && s.ok; ++j) {
        k_lam_spmv<<<g, kBlock, 0, st>>>(dA.rp, dA.ci, dA.v, p, n, q);
        const double pq = dot(p, q);
        if (!(pq > 0.0)) break;
        const double al = rho / pq;
        alpha.push_back(al);
        if (j == o.esteig_iters - 1) break;
        k_lam_update_r<<<g, kBlock, 0, st>>>(n, al, q, ddinv, r, z);
        const double rn = dot(r, z);
        if (!(rn > 1e-28 * rho0)) break;
        const double be = rn / rho;
        beta.push_back(be);
        k_lam_update_p<<<g, kBlock, 0, st>>>(n, be, z, p);
        rho = rn;
      }
      s.check(hipGetLastError());
      if (!s.ok) goto done;
      lam = ritz_from_cg(A, Dinv, alpha, beta);
    }
    {
      const int g = grid_for(n, kBlock, 8192);
      const double cut = strength_cut(o.threshold), keep = tie_keep();
      k_ag_strength<0><<<g, kBlock, 0, st>>>(dA.rp, dA.ci, dA.v, dd, n, cut, cnt, nullptr, nullptr, nullptr);
      std::vector<int> hv(n), srp(n + 1, 0);
      s.check(hipMemcpyAsync(hv.data(), cnt, sizeof(int) * n, hipMemcpyDeviceToHost, st));
      s.check(hipStreamSynchronize(st));
      if (!s.ok) goto done;
      for (int i = 0; i < n; ++i) srp[i + 1] = srp[i] + hv[i];
      int* dsrp = s.alloc<int>(n + 1);
      int* dsci = s.alloc<int>(srp[n]);
      double* dsw = s.alloc<double>(srp[n]);
      uint64_t* key = s.alloc<uint64_t>(n);
      uint64_t* m1 = s.alloc<uint64_t>(n);
      uint64_t* m2 = s.alloc<uint64_t>(n);
      uint8_t* stt = s.alloc<uint8_t>(n);
      uint8_t* mark = s.alloc<uint8_t>(n);
      uint8_t* r1 = s.alloc<uint8_t>(n);
      uint8_t* r2 = s.alloc<uint8_t>(n);
      int* nfree = s.alloc<int>(1);
      int* root1 = s.alloc<int>(n);
      int* root2 = s.alloc<int>(n);
      if (!s.ok) goto done;
      s.check(hipMemcpyAsync(dsrp, srp.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice, st));
      k_ag_strength<1><<<g, kBlock, 0, st>>>(dA.rp, dA.ci, dA.v, dd, n, cut, nullptr, dsrp, dsci, dsw);
      k_ag_keys<<<g, kBlock, 0, st>>>(n, o.seed + kLubySeedOffset + (uint64_t)level, key, stt);
      int rounds = 0, free_left = n;
      while (free_left > 0 && s.ok) {
        // every round makes at least the largest free key a root, and random priorities finish
        // in O(log n) rounds; a run past 1000 rounds is handed to the host
        if (++rounds > 1000) goto done;
        s.check(hipMemsetAsync(nfree, 0, sizeof(int), st));
        k_ag_max<true><<<g, kBlock, 0, st>>>(dsrp, dsci, n, key, stt, m1);
        if (square) k_ag_max<false><<<g, kBlock, 0, st>>>(dsrp, dsci, n, m1, stt, m2);
        k_ag_select<<<g, kBlock, 0, st>>>(n, square ? m2 : m1, key, stt, mark);
        k_ag_reach<<<g, kBlock, 0, st>>>(dsrp, dsci, n, mark, r1);
        if (square) k_ag_reach<<<g, kBlock, 0, st>>>(dsrp, dsci, n, r1, r2);
        k_ag_take<<<g, kBlock, 0, st>>>(n, square ? r2 : r1, stt, nfree);
        s.check(hipGetLastError());
        s.check(hipMemcpyAsync(&free_left, nfree, sizeof(int), hipMemcpyDeviceToHost, st));
        s.check(hipStreamSynchronize(st));
      }
      k_ag_pass1<<<g, kBlock, 0, st>>>(dsrp, dsci, dsw, n, stt, keep, root1);
      k_ag_pass2<<<g, kBlock, 0, st>>>(dsrp, dsci, dsw, n, root1, keep, root2);
      s.check(hipGetLastError());
      s.check(hipMemcpyAsync(hv.data(), root2, sizeof(int) * n, hipMemcpyDeviceToHost, st));
      s.check(hipStreamSynchronize(st));
      if (!s.ok) goto done;
      // aggregate = rank of the root (index order)
      std::vector<int32_t> rank(n, -1), agg(n);
      nc = 0;
      for (int i = 0; i < n; ++i)
        if (hv[i] == i) rank[i] = nc++;
      for (int i = 0; i < n; ++i) {
        if (hv[i] < 0 || rank[hv[i]] < 0) goto done;  // left out (the host reports it)
        agg[i] = rank[hv[i]];
      }
      if (log)
        std::fprintf(stderr, "[setup]   level %d on the device: %d rounds, %d aggregates (%.3f s)\n", level, rounds, nc,
                     std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
      P = tentative_prolongator(B, agg, nc, Bc);
      const double omega = prolongator_damping(lam);
      for (int sm = 0; sm < o.prolong_smooths; ++sm) {
        DevScratch s2;
        s2.tb = tb;
        const DevCsr dP = upload_csr(s2, P, st);
        DevCsr AP;
        if (!s2.ok || !device_spgemm(s2, dA, dP, AP, st, false)) goto done;
        k_ag_smooth<<<grid_for(n, kBlock, 8192), kBlock, 0, st>>>(dP.rp, dP.ci, dP.v, AP.rp, AP.ci, AP.v, ddinv,
                                                                  omega, n);
        s2.check(hipGetLastError());
        Csr Q;
        Q.nrows = n;
        Q.ncols = nc;
        Q.rp.resize(n + 1);
        Q.ci.resize(AP.nnz);
        Q.v.resize(AP.nnz);
        s2.check(hipMemcpyAsync(Q.rp.data(), AP.rp, sizeof(int) * (n + 1), hipMemcpyDeviceToHost, st));
        if (AP.nnz) {
          s2.check(hipMemcpyAsync(Q.ci.data(), AP.ci, sizeof(int) * AP.nnz, hipMemcpyDeviceToHost, st));
          s2.check(hipMemcpyAsync(Q.v.data(), AP.v, sizeof(double) * AP.nnz, hipMemcpyDeviceToHost, st));
        }
        s2.check(hipStreamSynchronize(st));
        if (!s2.ok) goto done;
        P = std::move(Q);
      }
      ok = s.ok;
    }
  done:;
  }
  (void)hipStreamDestroy(st);
  if (!ok && log) std::fprintf(stderr, "[setup] device coarsening of level %d unavailable, using the host\n", level);
  return ok;
}

// host_only: build the hierarchy but do not upload it; use_device: the setup may run its
// Galerkin products on the device (option galerkin_device); plan: build the launch plans (for a
// hierarchy that will be uploaded).
int setup_impl(const bd_csr* A, const bd_amg_opts* opts, const double* weights, hipStream_t st, bd_amg** out,
               bool host_only = false, bool use_device = true, bool plan = true,
               const TransientBudget* tb = nullptr) {
  if (!A || !out) throw Failure{BD_E_INVALID, "null argument"};
  bd_amg_opts o;
  bidomain_default_opts(&o);
  if (opts) o = *opts;
  if (o.smoother_degree < 1 || o.coarse_eq_limit < 1 || o.max_levels < 1 || !(o.cheb_hi > o.cheb_lo) ||
      !(o.cheb_lo >= 0.0) || o.esteig_iters < 1 || !(o.threshold >= 0.0) || !(o.stagnation_ratio > 0.0) ||
      o.coarse_dense_max < 1 || (o.coarsening != BD_SA && o.coarsening != BD_RS && o.coarsening != BD_PMIS) ||
      o.galerkin_device < 0 || o.galerkin_device > 3 || o.diag_form < 0 || o.diag_form > 1 ||
      o.preconditioner < BD_PC_AMG || o.preconditioner > BD_PC_NONE ||
      (o.independent_set != BD_MIS_GREEDY && o.independent_set != BD_MIS_LUBY) || o.aggregate_device < 0 ||
      o.aggregate_device > 1 || o.reorder < 0 || o.reorder > 2 ||
      (o.preconditioner != BD_PC_AMG && o.vcycle_precision != BD_F64) ||
      (o.smoother != BD_CHEBYSHEV && o.smoother != BD_JACOBI) ||
      (o.vcycle_precision != BD_F64 && o.vcycle_precision != BD_F32))
    throw Failure{BD_E_INVALID, "invalid AMG options"};
  if (o.preconditioner != BD_PC_AMG) {
    o.max_levels = 1;        // the fine level only (operator, D^{-1}, work vectors)
    o.coarse_dense_max = 1;  // no dense coarse inverse of it
  }
  Csr H;
  H.nrows = H.ncols = A->n;
  if (A->n <= 0 || A->nnz < 0 || A->nnz > INT32_MAX || !A->row_ptr || !A->col_idx || !A->val)
    throw Failure{BD_E_INVALID, "invalid CSR arguments"};
  H.rp.assign(A->row_ptr, A->row_ptr + A->n + 1);
  if (H.rp[A->n] != A->nnz) throw Failure{BD_E_INVALID, "row_ptr[n] must equal nnz"};
  H.ci.assign(A->col_idx, A->col_idx + A->nnz);
  H.v.assign(A->val, A->val + A->nnz);
  const std::string bad = validate(H);
  if (!bad.empty()) throw Failure{BD_E_INVALID, bad};

  std::unique_ptr<bd_amg> h(new bd_amg());
  h->o = o;
  h->n = A->n;
  h->mixed = o.vcycle_precision == BD_F32;
  std::string err;
  const bool log = std::getenv("BIDOMAIN_SETUP_LOG") != nullptr;
  const AggregateOffload agg_offload = [&](const Csr& Ak, const std::vector<double>& dk, const std::vector<double>& Dk,
                                           const std::vector<double>& Bk, int level, double& lam, Csr& Pk,
                                           std::vector<double>& Bc, int32_t& nc) {
    return device_sa_level(Ak, dk, Dk, Bk, level, o, log, lam, Pk, Bc, nc, tb);
  };
  const GalerkinOffload offload = [&](const Csr& Ak, const Csr& Pk, const Csr& Rk, int64_t flops, Csr& Ac) {
    return sparse_galerkin(Ak, Pk, Rk, flops, o.galerkin_device, log, Ac, tb);
  };
  const auto t0 = std::chrono::steady_clock::now();
  const int rc = build_hierarchy(std::move(H), o, h->H, err, use_device && o.galerkin_device != 0 ? &offload : nullptr,
                                 use_device && o.aggregate_device == 1 ? &agg_offload : nullptr);
  if (rc != BD_OK) throw Failure{rc, err};
  const auto t1 = std::chrono::steady_clock::now();
  if (plan) plan_hierarchy(h->H, o.diag_form != 0, o.reorder);  // launch plans, on this (possibly worker) thread
  if (log)
    std::fprintf(stderr, "[setup] hierarchy %.2f s, launch plans (with renumbered levels) %.2f s\n",
                 std::chrono::duration<double>(t1 - t0).count(),
                 std::chrono::duration<double>(std::chrono::steady_clock::now() - t1).count());
  h->M = (int)h->H.lv.size() - 1;
  h->host_only = true;
  if (!host_only) device_upload(h.get(), weights, false, st);
  *out = h.release();
  return BD_OK;
}

// Host half of a simulation: assembled operators and host-built hierarchies.  With
// device_galerkin false the setup does no device work at all; with it true the filled levels'
// Galerkin products may run on the device (option galerkin_device) in transient buffers of up to
// half the free device memory, each first reserved from `tb` when given (a server counts them
// against its budget while the setup runs on a worker thread).
struct SimHost {
  SimPhysics ph{};
  Csr Ai;
  std::vector<double> m;
  bd_amg* hell = nullptr;
  bd_amg* hpar = nullptr;
  ~SimHost() {
    delete hell;
    delete hpar;
  }
};

// Hierarchies of a case from its assembled A_i, A_e (same pattern) and lumped mass.
std::unique_ptr<SimHost> build_sim_host_ops(Csr Ai, const Csr& Ae, std::vector<double> m, const SimPhysics& ph,
                                            const bd_amg_opts* ell, const bd_amg_opts* par, bool device_galerkin,
                                            const TransientBudget* tb) {
  std::unique_ptr<SimHost> H(new SimHost());
  H->ph = ph;
  H->Ai = std::move(Ai);
  H->m = std::move(m);
  const int n = H->Ai.nrows;
  Csr Aell = H->Ai, Apar = H->Ai;
#pragma omp parallel for schedule(static, 4096)
  for (int32_t i = 0; i < n; ++i)
    for (int32_t k = Aell.rp[i]; k < Aell.rp[i + 1]; ++k) {
      Aell.v[k] += Ae.v[k];
      if (Apar.ci[k] == i) Apar.v[k] += ph.cm / ph.dt * H->m[i];
    }
  bd_amg_opts oe, op;
  bidomain_default_opts(&oe);
  bidomain_default_opts(&op);
  op.threshold = 0.0;  // parabolic default: see bidomain_sim_create
  if (ell) oe = *ell;
  if (par) op = *par;
  oe.nullspace = BD_NULL_CONSTANT;
  op.nullspace = BD_NULL_NONE;
  bd_csr ce{n, Aell.nnz(), Aell.rp.data(), Aell.ci.data(), Aell.v.data()};
  bd_csr cp{n, Apar.nnz(), Apar.rp.data(), Apar.ci.data(), Apar.v.data()};
  setup_impl(&ce, &oe, nullptr, nullptr, &H->hell, true, device_galerkin, true, tb);
  setup_impl(&cp, &op, nullptr, nullptr, &H->hpar, true, device_galerkin, true, tb);
  return H;
}

std::unique_ptr<SimHost> build_sim_host(const bd_slab& s, const bd_amg_opts* ell, const bd_amg_opts* par,
                                        bool device_galerkin, const TransientBudget* tb = nullptr) {
  const bool log = std::getenv("BIDOMAIN_SETUP_LOG") != nullptr;
  const auto t0 = std::chrono::steady_clock::now();
  Csr Ai, Ae;
  std::vector<double> m;
  assemble_slab_stiffness(s, s.sig_il, s.sig_it, Ai);
  assemble_slab_stiffness(s, s.sig_el, s.sig_et, Ae);
  slab_lumped_mass(s, m);
  if (log)
    std::fprintf(stderr, "[setup] slab operators assembled: %.2f s\n",
                 std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
  return build_sim_host_ops(std::move(Ai), Ae, std::move(m), sim_physics(s), ell, par, device_galerkin, tb);
}

// Device half: hierarchies, A_i, the lumped mass and the state vectors in HBM (takes the
// hierarchies from H).  v0 / w0: n doubles on the device or the host (w0 may be null: w = 0).
std::unique_ptr<bd_sim> upload_sim(SimHost& H, const double* v0, bool v0_dev, const double* w0, bool w0_dev,
                                   hipStream_t st) {
  std::unique_ptr<bd_sim> S(new bd_sim());
  S->ph = H.ph;
  S->n = H.Ai.nrows;
  const int n = S->n;
  S->hell = H.hell;
  S->hpar = H.hpar;
  H.hell = H.hpar = nullptr;
  device_upload(S->hell, H.m.data(), true, st);
  device_upload(S->hpar, nullptr, false, st);
  S->Ai = upload<double>(S->ar, H.Ai, &S->hell->A0, nullptr, false, st, kMaxBlocksSpmv);
  S->v = S->ar.alloc<double>(n);
  S->ue = S->ar.alloc<double>(n);
  S->w = S->ar.alloc<double>(n);
  S->rhs = S->ar.alloc<double>(n);
  S->fell = S->ar.alloc<double>(n);
  S->m = upload_vec<double>(S->ar, H.m, st);
  HIPCHK(hipMemcpyAsync(S->v, v0, sizeof(double) * n, v0_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
  if (w0) HIPCHK(hipMemcpyAsync(S->w, w0, sizeof(double) * n, w0_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
  else HIPCHK(hipMemsetAsync(S->w, 0, sizeof(double) * n, st));
  HIPCHK(hipMemsetAsync(S->ue, 0, sizeof(double) * n, st));
  HIPCHK(hipStreamSynchronize(st));
  return S;
}

int64_t sim_device_bytes(const bd_sim* S) { return S->ar.bytes + S->hell->ar.bytes + S->hpar->ar.bytes; }

// ------------------------------------------------------------------------------------------
// Solve state of bidomain_pcg_solve_noalloc in a file-scope device array instead of the
// handle: scalars at [0, S_COUNT), flags (int) at [kNoAllocFlags, +F_COUNT / 2 + 1), block
// partials from kNoAllocPart on.  Each device holds its own copy for the life of the process;
// every call on a device shares it (the last call's contents stay), so calls that overlap on
// one device race.
constexpr int64_t kNoAllocScratchBytes = int64_t(4) << 20;
constexpr int kNoAllocFlags = 16, kNoAllocPart = 32;
static_assert(S_COUNT <= kNoAllocFlags && kNoAllocFlags + (F_COUNT + 1) / 2 <= kNoAllocPart, "scratch layout");
static __device__ __align__(256) double scratch[kNoAllocScratchBytes / 8];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// The device address of the current device's scratch array, looked up once per device (with
// that device current); the array's name in host code is only a host-side stand-in.
double* scratch_address() {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) throw Failure{BD_E_DEVICE, "device ordinal out of range"};
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  return g_scratch_ptr[dev];
}

// A solve state in the scratch array for a solve of h, cleared on the stream (scalars, flags
// and partials start at zero as in a freshly set-up handle).  Rejects a hierarchy whose block
// partials do not fit.  The environment variable BIDOMAIN_NOALLOC_SCRATCH_BYTES may lower
// (never raise) the limit, so that the rejection can be tested.
Solve noalloc_solve_state(bd_amg* h, hipStream_t st) {
  int64_t limit = kNoAllocScratchBytes;
  if (const char* e = std::getenv("BIDOMAIN_NOALLOC_SCRATCH_BYTES"))
    limit = std::min<int64_t>(limit, std::max<int64_t>(0, std::strtoll(e, nullptr, 10)));
  const int64_t need = (int64_t)(kNoAllocPart + h->part_len) * 8;
  if (need > limit)
    throw Failure{BD_E_INVALID, "the solve needs " + std::to_string(need) + " bytes of scratch, more than the " +
                                    std::to_string(limit) + " the no-allocation entry point has"};
  double* base = scratch_address();
  k_fill_zero<double><<<vec_blocks(need / 8), kBlock, 0, st>>>(base, need / 8);
  HIPCHK(hipGetLastError());
  Solve sv = h->sv;
  sv.sc = base;
  sv.fl = reinterpret_cast<int*>(base + kNoAllocFlags);
  sv.part = base + kNoAllocPart;
  return sv;
}

}  // namespace bd

// ==========================================================================================
// C ABI
extern "C" {

const char* bidomain_last_error(void) { return g_last_error.c_str(); }

int bidomain_amg_setup(const bd_csr* A, const bd_amg_opts* opts, const double* null_weights, void* stream,
                       bd_amg** out) {
  return guarded([&] { return setup_impl(A, opts, null_weights, (hipStream_t)stream, out); });
}

int bidomain_amg_build_host(const bd_csr* A, const bd_amg_opts* opts, bd_amg** out) {
  return guarded([&] { return setup_impl(A, opts, nullptr, nullptr, out, true, false, false); });
}

int bidomain_pcg_solve(bd_amg* h, const double* b_dev, double* x_dev, int x_is_guess, double rtol, int maxit,
                       void* stream, bd_solve_info* info) {
  return guarded([&] {
    if (h && h->host_only) throw Failure{BD_E_INVALID, "host-only hierarchy"};
    if (!h || !b_dev || !x_dev || !(rtol > 0.0) || maxit < 1) throw Failure{BD_E_INVALID, "invalid solve arguments"};
    hipStream_t st = (hipStream_t)stream;
    return h->mixed ? pcg<float>(h, h->sv, b_dev, x_dev, x_is_guess, rtol, maxit, st, info)
                    : pcg<double>(h, h->sv, b_dev, x_dev, x_is_guess, rtol, maxit, st, info);
  });
}

int bidomain_pcg_solve_noalloc(bd_amg* h, const double* b_dev, double* x_dev, int x_is_guess, double rtol,
                               int maxit, void* stream, bd_solve_info* info) {
  return guarded([&] {
    if (h && h->host_only) throw Failure{BD_E_INVALID, "host-only hierarchy"};
    if (!h || !b_dev || !x_dev || !(rtol > 0.0) || maxit < 1) throw Failure{BD_E_INVALID, "invalid solve arguments"};
    hipStream_t st = (hipStream_t)stream;
    const Solve sv = noalloc_solve_state(h, st);
    return h->mixed ? pcg<float>(h, sv, b_dev, x_dev, x_is_guess, rtol, maxit, st, info, false)
                    : pcg<double>(h, sv, b_dev, x_dev, x_is_guess, rtol, maxit, st, info, false);
  });
}

int bidomain_amg_info(const bd_amg* h, bd_amg_stats* s) {
  return guarded([&] {
    if (!h || !s) throw Failure{BD_E_INVALID, "null argument"};
    std::memset(s, 0, sizeof(*s));
    const auto& L = h->H.lv;
    s->nlevels = (int)L.size();
    double nnz = 0, nn = 0;
    for (size_t k = 0; k < L.size() && k < BD_MAX_LEVELS; ++k) {
      s->n[k] = L[k].A.nrows;
      s->nnz[k] = L[k].A.nnz();
      s->p_nnz[k] = L[k].P.nnz();
      s->lambda[k] = L[k].lam;
      nnz += (double)L[k].A.nnz();
      nn += L[k].A.nrows;
    }
    if (!h->host_only) {
      for (size_t k = 0; k < L.size() && k < BD_MAX_LEVELS; ++k) {
        const DPat& M = k == 0 ? static_cast<const DPat&>(h->A0)
                               : (h->mixed ? static_cast<const DPat&>(h->L32[k].A) : static_cast<const DPat&>(h->L64[k].A));
        s->col_bytes[k] = M.col_bytes();
        s->tiles[k] = M.blk ? M.nb : 0;
        s->diags[k] = M.nd;
        s->renumbered[k] = L[k].perm.empty() ? 0 : 1;
        if (k + 1 < L.size()) {
          const DPat& P = h->mixed ? static_cast<const DPat&>(h->L32[k].P) : static_cast<const DPat&>(h->L64[k].P);
          const DPat& R = h->mixed ? static_cast<const DPat&>(h->L32[k].R) : static_cast<const DPat&>(h->L64[k].R);
          s->col_bytes_p[k] = P.col_bytes();
          s->col_bytes_r[k] = R.col_bytes();
        }
      }
    }
    s->coarse_mode = h->H.coarse_mode;
    s->vcycle_precision = h->o.vcycle_precision;
    s->operator_complexity = nnz / (double)L[0].A.nnz();
    s->grid_complexity = nn / (double)L[0].A.nrows;
    s->device_bytes = h->ar.bytes;
    return BD_OK;
  });
}

void bidomain_amg_destroy(bd_amg* h) { delete h; }

int bidomain_amg_export(const bd_amg* h, int level, int which, int32_t* rows, int32_t* cols, int64_t* nnz,
                        int32_t* row_ptr, int32_t* col_idx, double* val) {
  return guarded([&] {
    if (!h || level < 0 || level >= (int)h->H.lv.size() || which < 0 || which > 2 || !rows || !cols || !nnz)
      throw Failure{BD_E_INVALID, "invalid export arguments"};
    const HostLevel& L = h->H.lv[level];
    const Csr& M = which == 0 ? L.A : (which == 1 ? L.P : L.R);
    *rows = M.nrows;
    *cols = M.ncols;
    *nnz = M.nnz();
    if (row_ptr) std::copy(M.rp.begin(), M.rp.end(), row_ptr);
    if (col_idx) std::copy(M.ci.begin(), M.ci.end(), col_idx);
    if (val) std::copy(M.v.begin(), M.v.end(), val);
    return BD_OK;
  });
}

int bidomain_galerkin(int32_t n, int32_t nc, const int32_t* a_row_ptr, const int32_t* a_col_idx, const double* a_val,
                      const int32_t* p_row_ptr, const int32_t* p_col_idx, const double* p_val, int on_device,
                      int64_t capacity, int32_t* c_row_ptr, int32_t* c_col_idx, double* c_val, int64_t* c_nnz) {
  return guarded([&] {
    if (n <= 0 || nc <= 0 || !a_row_ptr || !a_col_idx || !a_val || !p_row_ptr || !p_col_idx || !p_val || !c_nnz ||
        on_device < 0 || on_device > 2 || (on_device == 2 && (n > sg::kDenseCols || nc > sg::kDenseCols)))
      throw Failure{BD_E_INVALID, "invalid Galerkin arguments"};
    Csr A, P;
    A.nrows = A.ncols = n;
    A.rp.assign(a_row_ptr, a_row_ptr + n + 1);
    if (A.rp[0] != 0 || A.rp[n] < 0) throw Failure{BD_E_INVALID, "A: row_ptr must start at 0"};
    A.ci.assign(a_col_idx, a_col_idx + A.rp[n]);
    A.v.assign(a_val, a_val + A.rp[n]);
    const std::string err = validate(A);
    if (!err.empty()) throw Failure{BD_E_INVALID, "A: " + err};
    P.nrows = n;
    P.ncols = nc;
    P.rp.assign(p_row_ptr, p_row_ptr + n + 1);
    if (P.rp[0] != 0) throw Failure{BD_E_INVALID, "P: row_ptr must start at 0"};
    for (int32_t i = 0; i < n; ++i)
      if (P.rp[i + 1] < P.rp[i]) throw Failure{BD_E_INVALID, "P: row_ptr must be non-decreasing"};
    P.ci.assign(p_col_idx, p_col_idx + P.rp[n]);
    P.v.assign(p_val, p_val + P.rp[n]);
    for (int32_t c : P.ci)
      if (c < 0 || c >= nc) throw Failure{BD_E_INVALID, "P: column index out of range"};
    const Csr R = transpose(P);
    int64_t flops = 0;
    for (int32_t i = 0; i < n; ++i)
      for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) flops += P.rp[A.ci[k] + 1] - P.rp[A.ci[k]];
    Csr Ac;
    if (on_device) {
      if (!sparse_galerkin(A, P, R, flops, on_device == 1 ? 2 : 3, false, Ac, nullptr))
        throw Failure{BD_E_NOMEM, "device Galerkin product: device memory not available"};
    } else {
      Ac = symmetrized(spgemm(R, spgemm(A, P)));
    }
    *c_nnz = Ac.nnz();
    if (c_row_ptr) std::copy(Ac.rp.begin(), Ac.rp.end(), c_row_ptr);
    if (c_col_idx || c_val) {
      if (capacity < Ac.nnz()) throw Failure{BD_E_INVALID, "output capacity below the product's nonzeros"};
      if (c_col_idx) std::copy(Ac.ci.begin(), Ac.ci.end(), c_col_idx);
      if (c_val) std::copy(Ac.v.begin(), Ac.v.end(), c_val);
    }
    return BD_OK;
  });
}

int bidomain_amg_apply(bd_amg* h, int op, int level, const void* in_dev, void* out_dev, void* stream) {
  return guarded([&] {
    if (!h || h->host_only || !in_dev || !out_dev || level < 0 || level > h->M)
      throw Failure{BD_E_INVALID, "invalid apply arguments"};
    hipStream_t st = (hipStream_t)stream;
    auto run = [&](auto tag) {
      using T = decltype(tag);
      auto& L = levels<T>(h);
      const Solve& sv = h->sv_apply;
      const T* in = (const T*)in_dev;
      T* out = (T*)out_dev;
      DLevel<T>& Lk = L[level];
      // the caller's vectors are in the host numbering; a renumbered level's input goes through
      // its work vector da and its output through db
      auto to_device = [&](const DLevel<T>& Lv, const T* src) -> const T* {
        if (!Lv.perm) return src;
        k_renumber<T, true><<<vec_blocks(Lv.n), kBlock, 0, st>>>(src, Lv.da, Lv.perm, Lv.n);
        return Lv.da;
      };
      auto from_device = [&](const DLevel<T>& Lv, const T* src, T* dst) {
        if (Lv.perm) k_renumber<T, false><<<vec_blocks(Lv.n), kBlock, 0, st>>>(src, dst, Lv.perm, Lv.n);
        else HIPCHK(hipMemcpyAsync(dst, src, sizeof(T) * Lv.n, hipMemcpyDeviceToDevice, st));
      };
      switch (op) {
        case BD_OP_A: {
          SpArgs<T> a = args<T>(sv); a.x = to_device(Lk, in); a.y = Lk.perm ? Lk.db : out;
          launch_spmv<T, OP_Y>(Lk.A, a, st);
          if (Lk.perm) from_device(Lk, Lk.db, out);
          break;
        }
        case BD_OP_P:
        case BD_OP_R: {
          if (level >= h->M) throw Failure{BD_E_INVALID, "the coarsest level has no transfer operators"};
          const DLevel<T>& Lin = op == BD_OP_P ? L[level + 1] : Lk;
          const DLevel<T>& Lout = op == BD_OP_P ? Lk : L[level + 1];
          SpArgs<T> a = args<T>(sv); a.x = to_device(Lin, in); a.y = Lout.perm ? Lout.db : out;
          launch_spmv<T, OP_Y>(op == BD_OP_P ? Lk.P : Lk.R, a, st);
          if (Lout.perm) from_device(Lout, Lout.db, out);
          break;
        }
        case BD_OP_PRESMOOTH:
        case BD_OP_VCYCLE:
        case BD_OP_COARSE: {
          const int k = op == BD_OP_COARSE ? h->M : level;
          DLevel<T>& Lx = L[k];
          T* saved = Lx.f;
          if (k == 0) {
            Lx.f = (T*)in;
          } else if (Lx.perm) {
            k_renumber<T, true><<<vec_blocks(Lx.n), kBlock, 0, st>>>(in, Lx.f, Lx.perm, Lx.n);
          } else {
            HIPCHK(hipMemcpyAsync(Lx.f, in, sizeof(T) * Lx.n, hipMemcpyDeviceToDevice, st));
          }
          if (op == BD_OP_PRESMOOTH) {
            if (!smoothed_level(h, k)) throw Failure{BD_E_INVALID, "the coarsest level is solved directly"};
            smooth_pre<T>(h, Lx, sv, false, st);
          } else if (op == BD_OP_COARSE) {
            coarse_solve<T>(h, Lx, sv, false, st);
          } else {
            vcycle<T>(h, k, sv, false, RedSpec{}, st);
          }
          from_device(Lx, Lx.x, out);
          if (k == 0) Lx.f = saved;
          break;
        }
        default:
          throw Failure{BD_E_INVALID, "unknown operation"};
      }
      HIPCHK(hipStreamSynchronize(st));
    };
    if (h->mixed) run(float{}); else run(double{});
    return BD_OK;
  });
}

static int64_t bd_slab_nnz27(const bd_slab* s) {
  return (int64_t)(3 * s->nx + 1) * (3 * s->ny + 1) * (3 * s->nz + 1);
}

static void check_membrane(const bd::ApParams& p, const char* what) {
  if (!(p.k > 0) || !(p.eps0 > 0) || !(p.mu2 > 0) || !(p.t_unit > 0) || !(p.v_scale > 0) || !std::isfinite(p.k) ||
      !std::isfinite(p.a) || !std::isfinite(p.eps0) || !std::isfinite(p.mu1) || !std::isfinite(p.mu2) ||
      !std::isfinite(p.t_unit) || !std::isfinite(p.v_scale) || !std::isfinite(p.v_rest))
    throw Failure{BD_E_INVALID, std::string("invalid Aliev-Panfilov parameters in the ") + what + " description"};
}

static void check_slab(const bd_slab* s) {
  if (!s || s->nx < 1 || s->ny < 1 || s->nz < 1 || !(s->Lx > 0) || !(s->Ly > 0) || !(s->Lz > 0) || !(s->dt > 0) ||
      !(s->cm > 0) || !(s->sig_it > 0) || !(s->sig_il > 0) || !(s->sig_et > 0) || !(s->sig_el > 0))
    throw Failure{BD_E_INVALID, "invalid slab description"};
  check_membrane(ap_params(*s), "slab");
  if (bd::slab_nodes(*s) > INT32_MAX || bd_slab_nnz27(s) > INT32_MAX)
    throw Failure{BD_E_INVALID, "slab too large for 32-bit CSR indices"};
}

static void check_ellipsoid(const bd_ellipsoid* e) {
  const double pi = 3.14159265358979323846;
  auto finite_pos = [](double v) { return std::isfinite(v) && v > 0; };
  if (!e || e->n_theta < 3 || e->n_phi < 1 || e->n_r < 1 || !finite_pos(e->a1) || !finite_pos(e->a2) ||
      !finite_pos(e->b1) || !finite_pos(e->b2) || !finite_pos(e->c1) || !finite_pos(e->c2) || !finite_pos(e->dt) ||
      !finite_pos(e->cm) || !finite_pos(e->sig_il) || !finite_pos(e->sig_it) || !finite_pos(e->sig_el) ||
      !finite_pos(e->sig_et) || !std::isfinite(e->fiber_endo) || !std::isfinite(e->fiber_epi) ||
      !std::isfinite(e->theta_min) || !std::isfinite(e->theta_max))
    throw Failure{BD_E_INVALID, "invalid ellipsoid description"};
  if (!(std::fabs((e->theta_max - e->theta_min) - 2 * pi) <= 1e-12 * 2 * pi))
    throw Failure{BD_E_INVALID, "the ellipsoid mesh is periodic in theta: theta_max - theta_min must be 2 pi"};
  if (!(e->phi_min > -0.5 * pi && e->phi_min < e->phi_max && e->phi_max < 0.5 * pi))
    throw Failure{BD_E_INVALID, "ellipsoid phi range must satisfy -pi/2 < phi_min < phi_max < pi/2"};
  check_membrane(ap_params(*e), "ellipsoid");
  if (bd::ellipsoid_nodes(*e) > INT32_MAX || bd::ellipsoid_nnz(*e) > INT32_MAX)
    throw Failure{BD_E_INVALID, "ellipsoid too large for 32-bit CSR indices"};
}

static void ellipsoid_operator(const bd_ellipsoid& e, double sl, double st, Csr& A, std::vector<double>* m) {
  if (!bd::assemble_ellipsoid(e, sl, st, A, m))
    throw Failure{BD_E_INVALID, "ellipsoid element with a non-positive Jacobian"};
}

// A_i, A_e and the lumped mass: one of the operators the assemble calls return.
static void pick_operator(int which, Csr&& Ai, const Csr& Ae, const std::vector<double>& m, double cm, double dt,
                          int32_t* row_ptr, int32_t* col_idx, double* val) {
  Csr A = std::move(Ai);
  if (which == BD_MAT_AE) {
    A.v = Ae.v;
  } else if (which == BD_MAT_AELL) {
    for (size_t k = 0; k < A.v.size(); ++k) A.v[k] += Ae.v[k];
  } else if (which == BD_MAT_APAR) {
    for (int32_t i = 0; i < A.nrows; ++i)
      for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k)
        if (A.ci[k] == i) A.v[k] += cm / dt * m[i];
  }
  std::copy(A.rp.begin(), A.rp.end(), row_ptr);
  std::copy(A.ci.begin(), A.ci.end(), col_idx);
  std::copy(A.v.begin(), A.v.end(), val);
}

int bidomain_ellipsoid_assemble(const bd_ellipsoid* e, int which, int32_t* row_ptr, int32_t* col_idx, double* val,
                                double* mass) {
  return guarded([&] {
    check_ellipsoid(e);
    if (which < BD_MAT_AI || which > BD_MAT_APAR || !row_ptr || !col_idx || !val)
      throw Failure{BD_E_INVALID, "invalid assemble arguments"};
    Csr Ai, Ae;
    std::vector<double> m;
    ellipsoid_operator(*e, e->sig_il, e->sig_it, Ai, &m);
    if (which == BD_MAT_AE || which == BD_MAT_AELL) ellipsoid_operator(*e, e->sig_el, e->sig_et, Ae, nullptr);
    pick_operator(which, std::move(Ai), Ae, m, e->cm, e->dt, row_ptr, col_idx, val);
    if (mass) std::copy(m.begin(), m.end(), mass);
    return BD_OK;
  });
}

int bidomain_slab_assemble(const bd_slab* s, int which, int32_t* row_ptr, int32_t* col_idx, double* val,
                           double* mass) {
  return guarded([&] {
    check_slab(s);
    if (which < BD_MAT_AI || which > BD_MAT_APAR || !row_ptr || !col_idx || !val)
      throw Failure{BD_E_INVALID, "invalid assemble arguments"};
    Csr Ai, Ae;
    std::vector<double> m;
    slab_lumped_mass(*s, m);
    assemble_slab_stiffness(*s, s->sig_il, s->sig_it, Ai);
    if (which == BD_MAT_AE || which == BD_MAT_AELL) assemble_slab_stiffness(*s, s->sig_el, s->sig_et, Ae);
    pick_operator(which, std::move(Ai), Ae, m, s->cm, s->dt, row_ptr, col_idx, val);
    if (mass) std::copy(m.begin(), m.end(), mass);
    return BD_OK;
  });
}

static void launch_membrane(bd_sim* S, hipStream_t st) {
  const int G = S->Ai.G;
  const int rpt = kBlock / G;
  const int nb = (S->n + rpt - 1) / rpt;
  switch (G) {
    case 4: k_membrane_rhs<4><<<nb, kBlock, 0, st>>>(S->Ai.rp, S->Ai.ci, S->Ai.v, S->ue, S->v, S->w, S->m, S->rhs, S->ph.dt, S->ph.cm, S->ph.ap, S->n); break;
    case 8: k_membrane_rhs<8><<<nb, kBlock, 0, st>>>(S->Ai.rp, S->Ai.ci, S->Ai.v, S->ue, S->v, S->w, S->m, S->rhs, S->ph.dt, S->ph.cm, S->ph.ap, S->n); break;
    default: k_membrane_rhs<16><<<nb, kBlock, 0, st>>>(S->Ai.rp, S->Ai.ci, S->Ai.v, S->ue, S->v, S->w, S->m, S->rhs, S->ph.dt, S->ph.cm, S->ph.ap, S->n); break;
  }
  HIPCHK(hipGetLastError());
}

static void launch_neg_spmv(bd_sim* S, const double* x, double* y, hipStream_t st) {
  const int G = S->Ai.G;
  const int rpt = kBlock / G;
  const int nb = (S->n + rpt - 1) / rpt;
  switch (G) {
    case 4: k_neg_spmv<4><<<nb, kBlock, 0, st>>>(S->Ai.rp, S->Ai.ci, S->Ai.v, x, y, S->n); break;
    case 8: k_neg_spmv<8><<<nb, kBlock, 0, st>>>(S->Ai.rp, S->Ai.ci, S->Ai.v, x, y, S->n); break;
    default: k_neg_spmv<16><<<nb, kBlock, 0, st>>>(S->Ai.rp, S->Ai.ci, S->Ai.v, x, y, S->n); break;
  }
  HIPCHK(hipGetLastError());
}

// Uploads a case's hierarchies and state and solves for u_e^0 from v^0 (eq. (6)).
static int start_sim(SimHost& H, const double* v0_dev, const double* w0_dev, double rtol, hipStream_t st,
                     bd_sim** out) {
  std::unique_ptr<bd_sim> S = upload_sim(H, v0_dev, true, w0_dev, true, st);
  launch_neg_spmv(S.get(), S->v, S->fell, st);
  bd_solve_info inf;
  const int rc = S->hell->mixed ? pcg<float>(S->hell, S->hell->sv, S->fell, S->ue, 0, rtol, 1000, st, &inf)
                                : pcg<double>(S->hell, S->hell->sv, S->fell, S->ue, 0, rtol, 1000, st, &inf);
  if (rc < 0) return rc;
  *out = S.release();
  return BD_OK;
}

int bidomain_sim_create(const bd_slab* s, const bd_amg_opts* ell, const bd_amg_opts* par, const double* v0_dev,
                        const double* w0_dev, double rtol, void* stream, bd_sim** out) {
  return guarded([&] {
    check_slab(s);
    if (!v0_dev || !out || !(rtol > 0)) throw Failure{BD_E_INVALID, "invalid simulation arguments"};
    std::unique_ptr<SimHost> H = build_sim_host(*s, ell, par, true);
    return start_sim(*H, v0_dev, w0_dev, rtol, (hipStream_t)stream, out);
  });
}

int bidomain_ellipsoid_sim_create(const bd_ellipsoid* e, const bd_amg_opts* ell, const bd_amg_opts* par,
                                  const double* v0_dev, const double* w0_dev, double rtol, void* stream,
                                  bd_sim** out) {
  return guarded([&] {
    check_ellipsoid(e);
    if (!v0_dev || !out || !(rtol > 0)) throw Failure{BD_E_INVALID, "invalid simulation arguments"};
    Csr Ai, Ae;
    std::vector<double> m;
    ellipsoid_operator(*e, e->sig_il, e->sig_it, Ai, &m);
    ellipsoid_operator(*e, e->sig_el, e->sig_et, Ae, nullptr);
    std::unique_ptr<SimHost> H =
        build_sim_host_ops(std::move(Ai), Ae, std::move(m), sim_physics(*e), ell, par, true, nullptr);
    return start_sim(*H, v0_dev, w0_dev, rtol, (hipStream_t)stream, out);
  });
}

int bidomain_step(bd_sim* S, int nsteps, double rtol, void* stream, bd_step_info* info) {
  return guarded([&] {
    if (!S || nsteps < 0 || !(rtol > 0)) throw Failure{BD_E_INVALID, "invalid step arguments"};
    hipStream_t st = (hipStream_t)stream;
    bd_step_info inf{};
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    int status = BD_OK;
    for (int s = 0; s < nsteps; ++s) {
      HIPCHK(hipEventRecord(e0, st));
      launch_membrane(S, st);
      HIPCHK(hipEventRecord(e1, st));
      HIPCHK(hipEventSynchronize(e1));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, e0, e1));
      inf.ms_memb += ms;
      bd_solve_info ip, ie;
      int rc = S->hpar->mixed ? pcg<float>(S->hpar, S->hpar->sv, S->rhs, S->v, 1, rtol, 1000, st, &ip)
                              : pcg<double>(S->hpar, S->hpar->sv, S->rhs, S->v, 1, rtol, 1000, st, &ip);
      if (rc != BD_OK) status = rc;
      launch_neg_spmv(S, S->v, S->fell, st);
      rc = S->hell->mixed ? pcg<float>(S->hell, S->hell->sv, S->fell, S->ue, 1, rtol, 1000, st, &ie)
                          : pcg<double>(S->hell, S->hell->sv, S->fell, S->ue, 1, rtol, 1000, st, &ie);
      if (rc != BD_OK && status == BD_OK) status = rc;
      inf.steps++;
      inf.it_par += ip.iterations;
      inf.it_ell += ie.iterations;
      inf.ms_par += ip.seconds * 1e3;
      inf.ms_ell += ie.seconds * 1e3;
      inf.rel_res_par = ip.rel_residual_true;
      inf.rel_res_ell = ie.rel_residual_true;
      if (status < 0) break;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    inf.status = status;
    if (info) *info = inf;
    return status;
  });
}

int bidomain_sim_get(bd_sim* S, int field, double* out_dev, void* stream) {
  return guarded([&] {
    if (!S || !out_dev || field < BD_V || field > BD_W) throw Failure{BD_E_INVALID, "invalid get arguments"};
    hipStream_t st = (hipStream_t)stream;
    const double* src = field == BD_V ? S->v : (field == BD_UE ? S->ue : S->w);
    HIPCHK(hipMemcpyAsync(out_dev, src, sizeof(double) * S->n, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipStreamSynchronize(st));
    return BD_OK;
  });
}

bd_amg* bidomain_sim_hierarchy(bd_sim* S, int which) { return S ? (which == 0 ? S->hell : S->hpar) : nullptr; }

void bidomain_sim_destroy(bd_sim* S) { delete S; }

void bidomain_profile_enable(int on) {
  std::lock_guard<std::mutex> g(g_prof.mu);
  g_prof.on = on != 0;
}

void bidomain_profile_read(double* total_ms, int64_t* launches, int reset) {
  std::lock_guard<std::mutex> g(g_prof.mu);
  if (total_ms) *total_ms = g_prof.total_ms;
  if (launches) *launches = g_prof.launches;
  if (reset) {
    g_prof.total_ms = 0.0;
    g_prof.launches = 0;
  }
}

}  // extern "C"

// ==========================================================================================
// Serving: continuous batching of many Bidomain cases.
#include <array>
#include <chrono>
#include <deque>
#include <functional>
#include <future>
#include <map>
#include <thread>

#include <omp.h>

namespace bd {

// Task tables of the multi-task launches: each launch copies its table from a pinned host ring
// into the same slice of a device buffer.
struct Staging {
  char* host = nullptr;
  char* dev = nullptr;
  size_t cap = 0, used = 0, lo = 0, hi = 0;
  // Rounds alternate between the two halves: a round's tables are rewritten only after the
  // round before it (which used the other half) is known complete, and the round that used this
  // half two rounds ago is complete by then too.
  void begin(int parity) {
    lo = parity ? cap / 2 : 0;
    hi = parity ? cap : cap / 2;
    used = lo;
  }
  void init(size_t bytes) {
    HIPCHK(hipHostMalloc(&host, bytes, hipHostMallocDefault));
    HIPCHK(hipMalloc(&dev, bytes));
    cap = bytes;
  }
  ~Staging() {
    if (host) (void)hipHostFree(host);
    if (dev) (void)hipFree(dev);
  }
  template <class Task>
  const Task* push(const std::vector<Task>& v, hipStream_t st) {
    const size_t bytes = v.size() * sizeof(Task);
    const size_t off = std::max(lo, (used + 255) & ~size_t(255));
    if (off + bytes > hi) throw Failure{BD_E_NOMEM, "serving task staging buffer exhausted"};
    std::memcpy(host + off, v.data(), bytes);
    HIPCHK(hipMemcpyAsync(dev + off, host + off, bytes, hipMemcpyHostToDevice, st));
    used = off + bytes;
    return reinterpret_cast<const Task*>(dev + off);
  }
};

template <class Task, class Launch>
void launch_tasks(std::vector<Task>& v, hipStream_t st, Staging& stg, Launch launch) {
  if (v.empty()) return;
  int off = 0;
  for (auto& t : v) {
    t.off = off;
    off += t.nb;
  }
  const Task* d = stg.push(v, st);
  launch(d, (int)v.size(), off);
  HIPCHK(hipGetLastError());
  v.clear();
}

// One sub-step of a round across all solves: the ops it collects are independent.
template <typename T>
struct Batch {
  // products by index form (IdxForm) and op
  std::vector<SpTask<T>> sp[kForms][OP_TRUE_RESID + 1];
  std::vector<SpTask<double>> cgq[kForms];  // outer products (always float64)
  std::vector<UpdTask<T>> upd;
  std::vector<DirTask<T>> dir;
  std::vector<GemvTask<T>> gemv;
  std::vector<FinTask> fin;
  std::vector<std::function<void()>> single;  // ops without a multi-task kernel, launched alone

  template <int OP>
  void add(const DCsr<T>& M, SpArgs<T> a, hipStream_t st) {
    if (M.n == 0) return;
    if (!M.blk && !M.nd) {  // rows longer than the staging buffer: lane-group kernel, one launch
      single.push_back([=] { launch_spmv<T, OP>(M, a, st); });
      return;
    }
    bind(a, M);
    SpTask<T> t;
    t.a = a;
    t.blk = M.blk;
    t.nb = M.nb;
    t.off = 0;
    sp[M.form()][OP].push_back(t);
  }

  void flush(hipStream_t st, Staging& stg) {
    for (auto& f : single) f();
    single.clear();
#define BD_SPL(OPV)                                                                                      \
  launch_tasks(sp[IX32][OPV], st, stg, [&](const SpTask<T>* d, int n, int nb) {                          \
    k_spmv_stream_multi<T, OPV, IX32><<<nb, kBlock, 0, st>>>(d, n);                                      \
  });                                                                                                    \
  launch_tasks(sp[IX16][OPV], st, stg, [&](const SpTask<T>* d, int n, int nb) {                          \
    k_spmv_stream_multi<T, OPV, IX16><<<nb, kBlock, 0, st>>>(d, n);                                      \
  });                                                                                                    \
  launch_tasks(sp[IXD8][OPV], st, stg, [&](const SpTask<T>* d, int n, int nb) {                          \
    k_spmv_stream_multi<T, OPV, IXD8><<<nb, kBlock, 0, st>>>(d, n);                                      \
  });                                                                                                    \
  launch_tasks(sp[IX24][OPV], st, stg, [&](const SpTask<T>* d, int n, int nb) {                          \
    k_spmv_stream_multi<T, OPV, IX24><<<nb, kBlock, 0, st>>>(d, n);                                      \
  });                                                                                                    \
  launch_tasks(sp[SDIA][OPV], st, stg, [&](const SpTask<T>* d, int n, int nb) {                          \
    k_spmv_sdia_multi<T, OPV><<<nb, kBlock, 0, st>>>(d, n);                                              \
  });
    BD_SPL(OP_Y)
    BD_SPL(OP_ADDY)
    BD_SPL(OP_RESID)
    BD_SPL(OP_RESTRICT)
    BD_SPL(OP_CHEB_FIRST)
    BD_SPL(OP_CHEB_POST0)
    BD_SPL(OP_CHEB_STEP)
#undef BD_SPL
    launch_tasks(cgq[IX32], st, stg, [&](const SpTask<double>* d, int n, int nb) {
      k_spmv_stream_multi<double, OP_CG_Q, IX32><<<nb, kBlock, 0, st>>>(d, n);
    });
    launch_tasks(cgq[IX16], st, stg, [&](const SpTask<double>* d, int n, int nb) {
      k_spmv_stream_multi<double, OP_CG_Q, IX16><<<nb, kBlock, 0, st>>>(d, n);
    });
    launch_tasks(cgq[IXD8], st, stg, [&](const SpTask<double>* d, int n, int nb) {
      k_spmv_stream_multi<double, OP_CG_Q, IXD8><<<nb, kBlock, 0, st>>>(d, n);
    });
    launch_tasks(cgq[IX24], st, stg, [&](const SpTask<double>* d, int n, int nb) {
      k_spmv_stream_multi<double, OP_CG_Q, IX24><<<nb, kBlock, 0, st>>>(d, n);
    });
    launch_tasks(cgq[SDIA], st, stg, [&](const SpTask<double>* d, int n, int nb) {
      k_spmv_sdia_multi<double, OP_CG_Q><<<nb, kBlock, 0, st>>>(d, n);
    });
    launch_tasks(upd, st, stg, [&](const UpdTask<T>* d, int n, int nb) { k_cg_update_multi<T><<<nb, kBlock, 0, st>>>(d, n); });
    launch_tasks(dir, st, stg, [&](const DirTask<T>* d, int n, int nb) { k_cg_direction_multi<T><<<nb, kBlock, 0, st>>>(d, n); });
    launch_tasks(gemv, st, stg, [&](const GemvTask<T>* d, int n, int nb) { k_coarse_gemv_multi<T><<<nb, kBlock, 0, st>>>(d, n); });
    launch_tasks(fin, st, stg, [&](const FinTask* d, int n, int nb) { k_finalize_multi<<<nb, kBlock, 0, st>>>(d, n); });
  }
};

// One PCG / FCG solve in flight on a hierarchy.
struct BInst {
  bd_amg* h = nullptr;
  const double* b = nullptr;
  double* x = nullptr;
  int guess = 0;
  double rtol = 1e-8;
  int maxit = 1000;
  int state = -1;  // -1 idle, 0 new (initial phase enqueued this round), 1 running
  int cur = 0;     // float right-hand-side buffer in use (mixed form)
  RedSpec red;
  std::chrono::steady_clock::time_point t0;
};

FinTask fin_task(const Solve& sv, int kind, int nb_part) {
  FinTask f;
  f.sv = sv;
  f.kind = kind;
  f.nb_part = nb_part;
  f.nb = 1;
  f.off = 0;
  return f;
}

// Initial phase of a solve (as in pcg(), without the host synchronisation).
template <typename T>
void inst_begin(BInst& I, hipStream_t st) {
  bd_amg* h = I.h;
  const Solve& sv = h->sv;
  const int n = h->n;
  const int vb = vec_blocks(n);
  h->host_flags[0] = h->host_flags[1] = 0;
  k_solve_control<<<1, 64, 0, st>>>(sv, 0, I.maxit, h->o.nullspace == BD_NULL_CONSTANT, I.rtol * I.rtol);
  k_init_means<<<vb, kBlock, 0, st>>>(sv, I.b, I.guess ? I.x : nullptr, n);
  HIPCHK(hipGetLastError());
  finalize(sv, FIN_MEANS, vb, st);
  k_init_guess<<<vb, kBlock, 0, st>>>(sv, I.x, I.guess, n);
  HIPCHK(hipGetLastError());
  SpArgs<double> a = args<double>(sv);
  a.x = I.x;
  a.y = h->r;
  a.b = I.b;
  launch_spmv<double, OP_INIT_RESID>(h->A0, a, st);
  finalize(sv, FIN_INIT, h->A0.nb, st);
  auto& L = levels<T>(h);
  I.cur = 0;
  I.red = RedSpec{};
  if (h->mixed) {
    k_convert<double, float><<<vb, kBlock, 0, st>>>(h->r, h->r32[0], n);
    HIPCHK(hipGetLastError());
    L[0].f = (T*)h->r32[0];
    I.red.red = RED_F32;
    I.red.r32 = h->r32[0];
    I.red.r32_old = h->r32[0];
  } else {
    L[0].f = (T*)h->r;
    I.red.red = RED_F64;
    I.red.r64 = h->r;
  }
  I.state = 0;
}

// V-cycles of several solves at once (Alg. 2), levels aligned: the down sweep visits level k
// of every solve whose hierarchy reaches it (a solve whose coarsest level is k solves there),
// then the up sweep returns.  Chebyshev degree 2.
template <typename T>
void batched_vcycle(std::vector<BInst*>& I, Batch<T>& B, hipStream_t st, Staging& stg) {
  int maxM = 0;
  for (BInst* i : I) maxM = std::max(maxM, i->h->M);
  for (int k = 0; k <= maxM; ++k) {
    if (k == 0)
      for (BInst* i : I) {
        bd_amg* h = i->h;
        DLevel<T>& L0 = levels<T>(h)[0];
        if (i->state == 0 && smoothed_level(h, 0)) {
          const Solve sv = h->sv;
          B.single.push_back([=] {
            k_cheb_pre0<T><<<vec_blocks(L0.n), kBlock, 0, st>>>(sv, L0.f, L0.dinv, L0.da, nullptr, L0.c0, L0.n);
          });
        }
      }
    B.flush(st, stg);
    for (BInst* i : I) {  // pre-smoothing step 1, or the coarsest solve
      bd_amg* h = i->h;
      if (k > h->M) continue;
      DLevel<T>& Lk = levels<T>(h)[k];
      if (k == h->M && h->H.coarse_mode == 0) {
        GemvTask<T> g;
        g.sv = h->sv; g.G = h->G; g.f = Lk.f; g.x = Lk.x; g.n = h->nM; g.nb = (h->nM + 3) / 4; g.off = 0;
        B.gemv.push_back(g);
      } else {
        SpArgs<T> a = args<T>(h->sv);
        a.x = Lk.da; a.xs = Lk.x; a.f = Lk.f; a.dinv = Lk.dinv; a.c1 = Lk.c1[0]; a.c2 = Lk.c2[0];
        a.store_rd = 0; a.r = Lk.r; a.y2 = Lk.db;
        B.template add<OP_CHEB_FIRST>(Lk.A, a, st);
      }
    }
    B.flush(st, stg);
    for (BInst* i : I) {  // residual
      bd_amg* h = i->h;
      if (k >= h->M) continue;
      DLevel<T>& Lk = levels<T>(h)[k];
      SpArgs<T> a = args<T>(h->sv);
      a.x = Lk.x; a.f = Lk.f; a.y = Lk.r;
      B.template add<OP_RESID>(Lk.A, a, st);
    }
    B.flush(st, stg);
    for (BInst* i : I) {  // restriction (+ first smoothing step of the next level)
      bd_amg* h = i->h;
      if (k >= h->M) continue;
      auto& L = levels<T>(h);
      DLevel<T>& Lk = L[k];
      DLevel<T>& Ln = L[k + 1];
      SpArgs<T> a = args<T>(h->sv);
      a.x = Lk.r; a.y = Ln.f;
      if (smoothed_level(h, k + 1)) {
        a.y2 = Ln.da; a.dinv2 = Ln.dinv; a.c0 = Ln.c0; a.xs = nullptr;
        B.template add<OP_RESTRICT>(Lk.R, a, st);
      } else {
        B.template add<OP_Y>(Lk.R, a, st);
      }
    }
    B.flush(st, stg);
  }
  for (int k = maxM - 1; k >= 0; --k) {
    for (BInst* i : I) {  // prolongation and correction
      bd_amg* h = i->h;
      if (k >= h->M) continue;
      auto& L = levels<T>(h);
      SpArgs<T> a = args<T>(h->sv);
      a.x = L[k + 1].x; a.y = L[k].x;
      B.template add<OP_ADDY>(L[k].P, a, st);
    }
    B.flush(st, stg);
    for (BInst* i : I) {  // post-smoothing step 0
      bd_amg* h = i->h;
      if (k >= h->M) continue;
      DLevel<T>& Lk = levels<T>(h)[k];
      SpArgs<T> a = args<T>(h->sv);
      a.x = Lk.x; a.f = Lk.f; a.r = Lk.r; a.y2 = Lk.da; a.dinv = Lk.dinv; a.c0 = Lk.c0;
      B.template add<OP_CHEB_POST0>(Lk.A, a, st);
    }
    B.flush(st, stg);
    for (BInst* i : I) {  // post-smoothing step 1 (+ level-0 CG reductions)
      bd_amg* h = i->h;
      if (k >= h->M) continue;
      DLevel<T>& Lk = levels<T>(h)[k];
      SpArgs<T> a = args<T>(h->sv);
      a.x = Lk.da; a.xs = Lk.x; a.r = Lk.r; a.dinv = Lk.dinv; a.c1 = Lk.c1[0]; a.c2 = Lk.c2[0];
      a.add_d = 1; a.store_rd = 0; a.y2 = Lk.db;
      if (k == 0) {
        a.red = i->red.red; a.r64 = i->red.r64; a.r32 = i->red.r32; a.r32_old = i->red.r32_old;
      }
      B.template add<OP_CHEB_STEP>(Lk.A, a, st);
    }
    B.flush(st, stg);
  }
}

// One round: one CG iteration of every running solve, and the first V-cycle of every new one.
template <typename T>
void batched_round(std::vector<BInst*>& I, hipStream_t st, Staging& stg) {
  Batch<T> B;
  std::vector<BInst*> run;
  for (BInst* i : I)
    if (i->state == 1) run.push_back(i);
  for (BInst* i : run) {  // q = A p
    const DCsr<double>& M = i->h->A0;
    SpArgs<double> a = args<double>(i->h->sv);
    a.x = i->h->p; a.y = i->h->q;
    if (M.blk || M.nd) {
      bind(a, M);
      SpTask<double> t;
      t.a = a; t.blk = M.blk; t.nb = M.nb; t.off = 0;
      B.cgq[M.form()].push_back(t);
    } else {
      const DCsr<double> Mc = M;
      B.single.push_back([=] { launch_spmv<double, OP_CG_Q>(Mc, a, st); });
    }
  }
  B.flush(st, stg);
  for (BInst* i : run) B.fin.push_back(fin_task(i->h->sv, FIN_CGQ, i->h->A0.nb));
  B.flush(st, stg);
  for (BInst* i : run) {  // x, r update and the next V-cycle's right-hand side
    bd_amg* h = i->h;
    auto& L = levels<T>(h);
    const bool fuse0 = smoothed_level(h, 0);
    UpdTask<T> u;
    u.sv = h->sv; u.x = i->x; u.r = h->r; u.p = h->p; u.q = h->q;
    u.r32 = h->mixed ? h->r32[i->cur ^ 1] : nullptr;
    u.dinv0 = L[0].dinv; u.d0 = fuse0 ? L[0].da : nullptr; u.x0 = nullptr; u.c0 = L[0].c0;
    u.n = h->n; u.nb = vec_blocks(h->n); u.off = 0;
    B.upd.push_back(u);
    if (h->mixed) {
      i->red.r32_old = h->r32[i->cur];
      i->red.r32 = h->r32[i->cur ^ 1];
      L[0].f = (T*)h->r32[i->cur ^ 1];
      i->cur ^= 1;
    }
  }
  B.flush(st, stg);
  for (BInst* i : run) B.fin.push_back(fin_task(i->h->sv, FIN_UPDATE, vec_blocks(i->h->n)));
  B.flush(st, stg);
  batched_vcycle<T>(I, B, st, stg);
  for (BInst* i : I) {  // level-0 reductions -> rho, beta
    bd_amg* h = i->h;
    const int kind = i->red.red == RED_F64 ? FIN_VC64 : FIN_VC32;
    if (h->M == 0) {  // no fused post-smoothing on level 0
      DLevel<T>& L0 = levels<T>(h)[0];
      SpArgs<T> a = args<T>(h->sv);
      a.nrows = L0.n; a.red = i->red.red; a.r64 = i->red.r64; a.r32 = i->red.r32; a.r32_old = i->red.r32_old;
      const int nb = vec_blocks(L0.n);
      const T* z = L0.x;
      B.single.push_back([=] { k_vc_reduce<T><<<nb, kBlock, 0, st>>>(a, z); });
      B.flush(st, stg);
      B.fin.push_back(fin_task(h->sv, kind, nb));
    } else {
      B.fin.push_back(fin_task(h->sv, kind, levels<T>(h)[0].A.nb));
    }
  }
  B.flush(st, stg);
  for (BInst* i : I) {
    DirTask<T> d;
    d.sv = i->h->sv; d.p = i->h->p; d.z = levels<T>(i->h)[0].x; d.n = i->h->n; d.nb = vec_blocks(i->h->n); d.off = 0;
    B.dir.push_back(d);
  }
  B.flush(st, stg);
  for (BInst* i : I)
    if (i->state == 0) {
      k_clear_first<<<1, 64, 0, st>>>(i->h->sv);
      HIPCHK(hipGetLastError());
      i->state = 1;
    }
}

// Exit phase of a finished solve: true residual and null-space normalisation.
void inst_exit(BInst& I, hipStream_t st) {
  bd_amg* h = I.h;
  const Solve& sv = h->sv;
  const int vb = vec_blocks(h->n);
  k_solve_control<<<1, 64, 0, st>>>(sv, 1, 0, 0, 0.0);
  k_zero_if_zero_rhs<<<vb, kBlock, 0, st>>>(sv, I.x, h->n);  // b^ = 0 gives x = 0
  HIPCHK(hipGetLastError());
  SpArgs<double> a = args<double>(sv);
  a.x = I.x;
  a.b = I.b;
  launch_spmv<double, OP_TRUE_RESID>(h->A0, a, st);
  finalize(sv, FIN_TRUE, h->A0.nb, st);
  if (h->o.nullspace == BD_NULL_CONSTANT) {
    k_norm_sums<<<vb, kBlock, 0, st>>>(sv, h->w, I.x, h->n);
    HIPCHK(hipGetLastError());
    finalize(sv, FIN_NORM, vb, st);
    k_norm_apply<<<vb, kBlock, 0, st>>>(sv, I.x, h->n);
    HIPCHK(hipGetLastError());
  }
}

}  // namespace bd

// Scalars and flags of a finished solve, copied to pinned host memory after its exit phase.
struct ExitSlot {
  double sc[bd::S_COUNT];
  int fl[bd::F_COUNT];
};
struct PendingExit {
  int slot = 0;
  int stage = 0;
  int64_t ready_round = 0;  // complete once the event of this round has been reached
};
constexpr int kExitSlots = 4;

struct ServedCase {
  uint64_t ticket = 0;
  bd_slab s{};
  int nsteps = 0;
  std::vector<double> v0;
  double t_submit = 0, t_admit = 0, t_ready = 0, t_done = 0;
  int state = 0;  // 0 queued, 1 host setup, 2 running, 3 done, 4 fetched
  int64_t est = 0, bytes = 0;
  std::future<std::unique_ptr<SimHost>> fut;
  std::unique_ptr<bd_sim> sim;
  int stage = 0;  // 0 initial elliptic solve, 1 parabolic, 2 elliptic
  int steps_done = 0;
  BInst inst;
  int it_par = 0, it_ell = 0;
  double max_res = 0.0;
  int status = BD_OK;
  std::vector<double> v_out, ue_out;
  ExitSlot* slots = nullptr;  // pinned, kExitSlots
  std::deque<PendingExit> exits;
  int next_slot = 0;
  ~ServedCase() {
    if (slots) (void)hipHostFree(slots);
  }
};

struct bd_server {
  int64_t budget = 0, used = 0;
  // device memory held by setup workers' transient buffers (device Galerkin products), counted
  // against the budget with `used`; both are read and written under budget_mu
  int64_t transient = 0;
  std::mutex budget_mu;
  bd::TransientBudget tbudget;
  int max_slots = 1, admitted = 0, setups = 0;
  bd_amg_opts oe{}, op{};
  double rtol = 1e-8;
  hipStream_t st = nullptr;
  bool mixed = false;
  std::deque<ServedCase*> queue;
  std::vector<std::unique_ptr<ServedCase>> cases;
  std::map<uint64_t, ServedCase*> by_ticket;
  std::vector<ServedCase*> live;
  std::deque<ServedCase*> unreported;
  Staging stg;
  std::vector<double> solve_lat;
  int64_t rounds = 0, solves = 0, max_batched = 0;
  hipEvent_t ev[2] = {nullptr, nullptr};  // end of the last two rounds (alternating)
  int64_t ev_round[2] = {0, 0};
  int parity = 0;
  int64_t pending_exits = 0;
  double t_enqueue = 0.0, t_wait = 0.0, t_exit = 0.0;  // host seconds spent per round phase
  // test hook (environment BIDOMAIN_SERVE_FAIL_UPLOAD=<ticket>): the upload of that case
  // reports an allocation failure after its device memory was taken, exercising the cleanup
  uint64_t fail_upload_ticket = 0;
  uint64_t next_ticket = 1;
  std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
  double now() const { return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count(); }
  ~bd_server() {
    for (auto& c : cases)
      if (c->fut.valid()) c->fut.wait();
    if (st) (void)hipStreamSynchronize(st);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
  }
};

namespace bd {

constexpr int kMaxConcurrentSetups = 3;

// OpenMP threads of one host-setup worker: the workers share the cores and leave two for the
// serving thread, which enqueues the rounds.
int setup_threads() {
  const int hw = (int)std::max(1u, std::thread::hardware_concurrency());
  return std::max(1, (hw - 2) / kMaxConcurrentSetups);
}

// Device footprint estimate used for admission: 85 bytes per 27-point nonzero of the fine mesh
// (both hierarchies, A_i and the state vectors; 63-76 measured with float32 V-cycles from
// 32x32x16 to 160x160x64); replaced by the measured footprint once the case is on the device.
int64_t case_estimate(const bd_slab& s) { return (int64_t)85 * ((int64_t)(3 * s.nx + 1) * (3 * s.ny + 1) * (3 * s.nz + 1)); }

void start_solve(bd_server* S, ServedCase* c, bd_amg* h, const double* b, double* x, int guess) {
  c->inst = BInst{};
  c->inst.h = h;
  c->inst.b = b;
  c->inst.x = x;
  c->inst.guess = guess;
  c->inst.rtol = S->rtol;
  c->inst.maxit = 1000;
  c->inst.t0 = std::chrono::steady_clock::now();
  if (S->mixed) inst_begin<float>(c->inst, S->st);
  else inst_begin<double>(c->inst, S->st);
}

// A case's last solve is done (or it failed): wait for its work, take its results, copy its
// final state to the host and release its device memory, slot and budget.
void finish_case(bd_server* S, ServedCase* c) {
  hipStream_t st = S->st;
  HIPCHK(hipStreamSynchronize(st));
  while (!c->exits.empty()) {
    const PendingExit e = c->exits.front();
    c->exits.pop_front();
    S->pending_exits--;
    const ExitSlot& r = c->slots[e.slot];
    const double fn = r.sc[S_FNORM2];
    c->max_res = std::max(c->max_res, fn > 0 ? std::sqrt(r.sc[S_TRUE2] / fn) : 0.0);
    if (r.fl[F_STATUS] != 0 && c->status == BD_OK) c->status = r.fl[F_STATUS];
    if (e.stage == 1) c->it_par += r.fl[F_ITERS]; else c->it_ell += r.fl[F_ITERS];
  }
  bd_sim* sim = c->sim.get();
  c->v_out.resize(sim->n);
  c->ue_out.resize(sim->n);
  HIPCHK(hipMemcpyAsync(c->v_out.data(), sim->v, sizeof(double) * sim->n, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(c->ue_out.data(), sim->ue, sizeof(double) * sim->n, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  c->sim.reset();
  c->inst.state = -1;
  {
    std::lock_guard<std::mutex> g(S->budget_mu);
    S->used -= c->bytes;
  }
  S->admitted--;
  c->state = 3;
  c->t_done = S->now();
  S->unreported.push_back(c);
}

int serve_poll(bd_server* S, bd_case_result* results, int max_results, int* n_results) {
  hipStream_t st = S->st;
  // admission in arrival order, against free slots and the device budget
  while (!S->queue.empty() && S->admitted < S->max_slots && S->setups < kMaxConcurrentSetups) {
    ServedCase* c = S->queue.front();
    {
      std::lock_guard<std::mutex> g(S->budget_mu);
      if (S->used + S->transient + c->est > S->budget) break;
      S->used += c->est;
    }
    S->queue.pop_front();
    S->admitted++;
    S->setups++;
    c->state = 1;
    c->t_admit = S->now();
    const bd_slab slab = c->s;
    const bd_amg_opts oe = S->oe, op = S->op;
    const int nthr = setup_threads();
    const TransientBudget* tb = &S->tbudget;
    c->fut = std::async(std::launch::async, [slab, oe, op, nthr, tb] {
      omp_set_num_threads(nthr);
      return build_sim_host(slab, &oe, &op, true, tb);  // device products within the budget
    });
    S->live.push_back(c);
  }
  // cases whose host setup finished: upload and start the initial elliptic solve
  for (ServedCase* c : S->live) {
    if (c->state != 1 || c->fut.wait_for(std::chrono::seconds(0)) != std::future_status::ready) continue;
    S->setups--;
    std::unique_ptr<SimHost> H;
    try {
      H = c->fut.get();
    } catch (const Failure& e) {
      c->status = e.code;
    } catch (...) {
      c->status = BD_E_INVALID;
    }
    if (!H) {  // host setup failed: retire the case
      {
        std::lock_guard<std::mutex> g(S->budget_mu);
        S->used -= c->est;
      }
      S->admitted--;
      c->state = 3;
      c->t_done = S->now();
      S->unreported.push_back(c);
      continue;
    }
    try {
      if (!c->slots) HIPCHK(hipHostMalloc((void**)&c->slots, sizeof(ExitSlot) * kExitSlots, hipHostMallocDefault));
      c->sim = upload_sim(*H, c->v0.data(), false, nullptr, false, st);
      if (S->fail_upload_ticket == c->ticket)
        throw Failure{BD_E_NOMEM, "upload failure injected for ticket " + std::to_string(c->ticket)};
      launch_neg_spmv(c->sim.get(), c->sim->v, c->sim->fell, st);
      c->stage = 0;
      start_solve(S, c, c->sim->hell, c->sim->fell, c->sim->ue, 0);
    } catch (const Failure& e) {
      // out of device memory (or a HIP error) while bringing the case onto the device: retire
      // it with that status and give back its slot and budget, as for a failed host setup
      c->status = e.code;
      (void)hipStreamSynchronize(st);
      c->sim.reset();
      {
        std::lock_guard<std::mutex> g(S->budget_mu);
        S->used -= c->est;
      }
      S->admitted--;
      c->state = 3;
      c->t_done = S->now();
      S->unreported.push_back(c);
      continue;
    }
    c->bytes = sim_device_bytes(c->sim.get());
    {
      std::lock_guard<std::mutex> g(S->budget_mu);
      S->used += c->bytes - c->est;
    }
    c->state = 2;
    c->t_ready = S->now();
  }
  // One round: one CG iteration of every running solve, enqueued as multi-task launches.  The
  // host does not wait for this round: it waits for the previous one (so the GPU always has a
  // round queued while the host reads flags and enqueues the next), then finishes the solves
  // that round (or an earlier one) completed.  A solve that converged in round r - 1 still has
  // its round-r launches queued; they find the done flag set and return at once.
  std::vector<BInst*> act;
  for (ServedCase* c : S->live)
    if (c->state == 2 && c->inst.state >= 0) act.push_back(&c->inst);
  const auto ta = std::chrono::steady_clock::now();
  bool recorded = false;
  if (!act.empty()) {
    S->max_batched = std::max<int64_t>(S->max_batched, (int64_t)act.size());
    S->stg.begin(S->parity);
    if (S->mixed) batched_round<float>(act, st, S->stg);
    else batched_round<double>(act, st, S->stg);
    HIPCHK(hipEventRecord(S->ev[S->parity], st));
    S->ev_round[S->parity] = S->rounds;
    S->rounds++;
    recorded = true;
  }
  const auto tb = std::chrono::steady_clock::now();
  int64_t completed = -1;  // rounds known complete: every launch enqueued before that round's event
  if (recorded && S->rounds >= 2) {
    HIPCHK(hipEventSynchronize(S->ev[S->parity ^ 1]));  // the previous round
    completed = S->ev_round[S->parity ^ 1];
  } else if (recorded || S->pending_exits > 0) {
    HIPCHK(hipStreamSynchronize(st));  // the first round, or no round left to overlap with
    completed = INT64_MAX;
  }
  if (recorded) S->parity ^= 1;
  const auto tc = std::chrono::steady_clock::now();
  S->t_enqueue += std::chrono::duration<double>(tb - ta).count();
  S->t_wait += std::chrono::duration<double>(tc - tb).count();
  const auto td = std::chrono::steady_clock::now();
  // exit phases whose results have arrived (they were enqueued before a completed round)
  for (ServedCase* c : S->live) {
    if (c->state != 2) continue;
    while (!c->exits.empty() && c->exits.front().ready_round <= completed) {
      const PendingExit e = c->exits.front();
      c->exits.pop_front();
      S->pending_exits--;
      const ExitSlot& r = c->slots[e.slot];
      const double fn = r.sc[S_FNORM2];
      c->max_res = std::max(c->max_res, fn > 0 ? std::sqrt(r.sc[S_TRUE2] / fn) : 0.0);
      if (r.fl[F_STATUS] != 0 && c->status == BD_OK) c->status = r.fl[F_STATUS];
      if (e.stage == 1) c->it_par += r.fl[F_ITERS]; else c->it_ell += r.fl[F_ITERS];
    }
  }
  // solves found finished (their pinned flag; possibly set by the round still running, whose
  // remaining launches for that solve return at once): enqueue the exit phase and copy its
  // scalars back asynchronously, then start the case's next solve at once
  const auto tnow = std::chrono::steady_clock::now();
  for (ServedCase* c : S->live) {
    if (c->state != 2 || c->inst.state < 0) continue;
    if (!__atomic_load_n(&c->inst.h->host_flags[0], __ATOMIC_ACQUIRE)) continue;
    BInst& I = c->inst;
    inst_exit(I, st);
    const int slot = c->next_slot;
    c->next_slot = (c->next_slot + 1) % kExitSlots;
    if ((int)c->exits.size() >= kExitSlots) throw Failure{BD_E_DEVICE, "serving: exit result slots exhausted"};
    HIPCHK(hipMemcpyAsync(c->slots[slot].sc, I.h->sv.sc, sizeof(double) * S_COUNT, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(c->slots[slot].fl, I.h->sv.fl, sizeof(int) * F_COUNT, hipMemcpyDeviceToHost, st));
    c->exits.push_back(PendingExit{slot, c->stage, S->rounds});
    S->pending_exits++;
    S->solves++;
    S->solve_lat.push_back(std::chrono::duration<double>(tnow - I.t0).count());
    I.state = -1;
    bd_sim* sim = c->sim.get();
    if (c->stage == 0 || c->stage == 2) {
      if (c->stage == 2) c->steps_done++;
      if (c->steps_done >= c->nsteps) {
        finish_case(S, c);
        continue;
      }
      c->stage = 1;  // next step: membrane update + parabolic solve (eqs. (4), (7))
      launch_membrane(sim, st);
      start_solve(S, c, sim->hpar, sim->rhs, sim->v, 1);
    } else {
      c->stage = 2;  // elliptic solve with the new potential (eq. (6))
      launch_neg_spmv(sim, sim->v, sim->fell, st);
      start_solve(S, c, sim->hell, sim->fell, sim->ue, 1);
    }
  }
  // a case whose solve failed stops at the next solve boundary it reaches (its status is known
  // once the exit results arrive)
  for (ServedCase* c : S->live)
    if (c->state == 2 && c->status < 0 && c->exits.empty()) finish_case(S, c);
  S->t_exit += std::chrono::duration<double>(std::chrono::steady_clock::now() - td).count();
  if (act.empty() && S->setups > 0)
    std::this_thread::sleep_for(std::chrono::microseconds(200));  // only host setups in flight
  {
    std::vector<ServedCase*> keep;
    for (ServedCase* c : S->live)
      if (c->state != 3) keep.push_back(c);
    S->live.swap(keep);
  }
  int k = 0;
  while (k < max_results && !S->unreported.empty()) {
    ServedCase* c = S->unreported.front();
    S->unreported.pop_front();
    bd_case_result& r = results[k++];
    r.ticket = c->ticket;
    r.status = c->status;
    r.steps = c->steps_done;
    r.it_par = c->it_par;
    r.it_ell = c->it_ell;
    r.t_submit = c->t_submit;
    r.t_admit = c->t_admit;
    r.t_ready = c->t_ready;
    r.t_done = c->t_done;
    r.max_rel_residual = c->max_res;
    r.device_bytes = c->bytes;
  }
  if (n_results) *n_results = k;
  return BD_OK;
}

}  // namespace bd

extern "C" {

int bidomain_serve_create(int64_t budget_bytes, int32_t max_slots, const bd_amg_opts* ell, const bd_amg_opts* par,
                          double rtol, void* stream, bd_server** out) {
  return guarded([&] {
    if (!out || budget_bytes <= 0 || max_slots < 1 || !(rtol > 0)) throw Failure{BD_E_INVALID, "invalid server arguments"};
    std::unique_ptr<bd_server> S(new bd_server());
    bidomain_default_opts(&S->oe);
    bidomain_default_opts(&S->op);
    if (ell) S->oe = *ell;
    if (par) S->op = *par;
    for (const bd_amg_opts* o : {&S->oe, &S->op}) {
      if (o->smoother != BD_CHEBYSHEV || o->smoother_degree != 2)
        throw Failure{BD_E_INVALID, "serving needs the Chebyshev smoother of degree 2"};
      if (o->preconditioner != BD_PC_AMG) throw Failure{BD_E_INVALID, "serving needs the AMG preconditioner"};
    }
    if (S->oe.vcycle_precision != S->op.vcycle_precision)
      throw Failure{BD_E_INVALID, "both systems must use the same V-cycle precision when served"};
    S->mixed = S->oe.vcycle_precision == BD_F32;
    S->budget = budget_bytes;
    S->max_slots = max_slots;
    S->rtol = rtol;
    S->st = (hipStream_t)stream;
    S->stg.init(size_t(32) << 20);
    bd_server* srv = S.get();
    S->tbudget.reserve = [srv](int64_t b) {
      std::lock_guard<std::mutex> g(srv->budget_mu);
      if (srv->used + srv->transient + b > srv->budget) return false;
      srv->transient += b;
      return true;
    };
    S->tbudget.release = [srv](int64_t b) {
      std::lock_guard<std::mutex> g(srv->budget_mu);
      srv->transient -= b;
    };
    HIPCHK(hipEventCreateWithFlags(&S->ev[0], hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&S->ev[1], hipEventDisableTiming));
    if (const char* f = std::getenv("BIDOMAIN_SERVE_FAIL_UPLOAD")) S->fail_upload_ticket = std::strtoull(f, nullptr, 10);
    *out = S.release();
    return BD_OK;
  });
}

int bidomain_serve_submit(bd_server* S, const bd_slab* slab, const double* v0_host, int32_t nsteps, uint64_t* ticket) {
  return guarded([&] {
    if (!S || !v0_host || nsteps < 0 || !ticket) throw Failure{BD_E_INVALID, "invalid submit arguments"};
    check_slab(slab);
    const int64_t est = case_estimate(*slab);
    if (est > S->budget) {
      g_last_error = "the case needs more device memory than the whole budget";
      return BD_E_BUDGET;
    }
    std::unique_ptr<ServedCase> c(new ServedCase());
    c->ticket = S->next_ticket++;
    c->s = *slab;
    c->nsteps = nsteps;
    c->v0.assign(v0_host, v0_host + slab_nodes(*slab));
    c->est = est;
    c->t_submit = S->now();
    *ticket = c->ticket;
    S->by_ticket[c->ticket] = c.get();
    S->queue.push_back(c.get());
    S->cases.push_back(std::move(c));
    return BD_OK;
  });
}

int bidomain_serve_estimate(const bd_server* S, const bd_slab* slab, int64_t* bytes) {
  return guarded([&] {
    if (!S || !bytes) throw Failure{BD_E_INVALID, "null argument"};
    check_slab(slab);
    *bytes = case_estimate(*slab);
    return BD_OK;
  });
}

int bidomain_serve_poll(bd_server* S, bd_case_result* results, int32_t max_results, int32_t* n_results) {
  return guarded([&] {
    if (!S || (max_results > 0 && !results)) throw Failure{BD_E_INVALID, "invalid poll arguments"};
    return serve_poll(S, results, max_results, n_results);
  });
}

int bidomain_serve_fetch(bd_server* S, uint64_t ticket, double* v_host, double* ue_host) {
  return guarded([&] {
    auto it = S ? S->by_ticket.find(ticket) : decltype(S->by_ticket)::iterator();
    if (!S || it == S->by_ticket.end() || it->second->state != 3) throw Failure{BD_E_INVALID, "no completed case with that ticket"};
    ServedCase* c = it->second;
    if (v_host) std::copy(c->v_out.begin(), c->v_out.end(), v_host);
    if (ue_host) std::copy(c->ue_out.begin(), c->ue_out.end(), ue_host);
    std::vector<double>().swap(c->v_out);
    std::vector<double>().swap(c->ue_out);
    c->state = 4;
    return BD_OK;
  });
}

int bidomain_serve_stats(const bd_server* S, bd_serve_stats* st) {
  return guarded([&] {
    if (!S || !st) throw Failure{BD_E_INVALID, "null argument"};
    std::memset(st, 0, sizeof(*st));
    for (const auto& c : S->cases) {
      if (c->state == 0) st->queued++;
      else if (c->state == 1) st->setting_up++;
      else if (c->state == 2) st->running++;
      else st->done++;
    }
    {
      std::lock_guard<std::mutex> g(const_cast<bd_server*>(S)->budget_mu);
      st->bytes_in_use = S->used + S->transient;
    }
    st->budget = S->budget;
    st->rounds = S->rounds;
    st->solves = S->solves;
    st->host_enqueue_s = S->t_enqueue;
    st->host_wait_s = S->t_wait;
    st->host_exit_s = S->t_exit;
    st->max_batched = S->max_batched;
    return BD_OK;
  });
}

int bidomain_serve_solve_latencies(const bd_server* S, double* out, int32_t cap, int32_t* count) {
  return guarded([&] {
    if (!S || !count || (cap > 0 && !out)) throw Failure{BD_E_INVALID, "invalid arguments"};
    const int n = (int)std::min<size_t>(S->solve_lat.size(), (size_t)std::max(cap, 0));
    std::copy(S->solve_lat.begin(), S->solve_lat.begin() + n, out);
    *count = (int)S->solve_lat.size();
    return BD_OK;
  });
}

void bidomain_serve_destroy(bd_server* S) { delete S; }

}  // extern "C"
