// Host-side self-check of the library's setup code (Q1 assembly and the AMG setup phase), built
// with AddressSanitizer and UndefinedBehaviorSanitizer by `python -m paper_2311_13914_amd.build
// --host-check`: every host routine runs on small and ragged slabs with each coarsening,
// smoother and null-space option, and on small periodic ellipsoid meshes, and the results are checked against the identities they
// must satisfy (exact symmetry, zero row sums of the stiffness, the lumped mass summing to the
// volume, R = P^T, P B_c = B and A_c B_c = 0 for smoothed aggregation, P 1 = 1 on zero-row-sum
// rows for classical coarsening).  Exit status 0 when every check passes.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "bd_host.hpp"

using namespace bd;

static int g_fail = 0;
#define CHECK(cond, ...)                        \
  do {                                          \
    if (!(cond)) {                              \
      std::fprintf(stderr, "FAIL: " __VA_ARGS__); \
      std::fprintf(stderr, "\n");               \
      ++g_fail;                                 \
    }                                           \
  } while (0)

static bd_slab slab(int nx, int ny, int nz) {
  bd_slab s{};
  s.nx = nx; s.ny = ny; s.nz = nz;
  s.Lx = 1.0; s.Ly = 1.0; s.Lz = 0.5;
  s.sig_il = 3.0e-3; s.sig_it = 3.1525e-4; s.sig_el = 2.0e-3; s.sig_et = 1.3514e-3;
  s.fiber_theta0 = -M_PI / 3.0; s.fiber_rotation = 2.0 * M_PI / 3.0;
  s.cm = 1.0; s.dt = 0.05;
  s.ap_k = 8.0; s.ap_a = 0.15; s.ap_eps0 = 0.002; s.ap_mu1 = 0.2; s.ap_mu2 = 0.3;
  s.ap_t_unit = 12.9; s.ap_v_scale = 105.0; s.ap_v_rest = -85.0;
  return s;
}

static double max_abs(const Csr& A) {
  double m = 0.0;
  for (double v : A.v) m = std::max(m, std::fabs(v));
  return m;
}

static std::vector<double> matvec(const Csr& A, const std::vector<double>& x) {
  std::vector<double> y(A.nrows, 0.0);
  for (int32_t i = 0; i < A.nrows; ++i)
    for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) y[i] += A.v[k] * x[A.ci[k]];
  return y;
}

// exact transpose equality of the value arrays (the setup symmetrises every coarse operator)
static bool exactly_symmetric(const Csr& A) {
  const Csr T = transpose(A);
  return T.rp == A.rp && T.ci == A.ci && T.v == A.v;
}

static void check_hierarchy(const HostHierarchy& H, const bd_amg_opts& o, const char* what) {
  CHECK(!H.lv.empty(), "%s: empty hierarchy", what);
  for (size_t k = 0; k < H.lv.size(); ++k) {
    const HostLevel& L = H.lv[k];
    // a one-row coarsest level of the pure Neumann operator is zero up to rounding (the
    // constant spans it; its correction is zero), so its diagonal need not be positive
    const bool null_row = o.nullspace == BD_NULL_CONSTANT && k > 0 && L.A.nrows == 1;
    CHECK(null_row || validate(L.A).empty(), "%s: level %zu operator: %s", what, k, validate(L.A).c_str());
    CHECK(k == 0 || exactly_symmetric(L.A), "%s: level %zu not symmetric", what, k);
    CHECK((int)L.Dinv.size() == L.A.nrows, "%s: level %zu Dinv size", what, k);
    if (k + 1 == H.lv.size()) break;
    const Csr& P = L.P;
    const Csr& R = L.R;
    const HostLevel& C = H.lv[k + 1];
    CHECK(P.nrows == L.A.nrows && P.ncols == C.A.nrows, "%s: level %zu P shape", what, k);
    const Csr Pt = transpose(P);
    CHECK(Pt.rp == R.rp && Pt.ci == R.ci && Pt.v == R.v, "%s: level %zu R != P^T", what, k);
    CHECK(C.A.nrows < L.A.nrows, "%s: level %zu does not coarsen", what, k);
    if (o.coarsening == BD_SA && o.nullspace == BD_NULL_CONSTANT) {  // A B = 0, so P B_c = B
      const std::vector<double> PB = matvec(P, C.B);
      double err = 0.0, ref = 0.0;
      for (int32_t i = 0; i < P.nrows; ++i) {
        err = std::max(err, std::fabs(PB[i] - L.B[i]));
        ref = std::max(ref, std::fabs(L.B[i]));
      }
      CHECK(err <= 1e-12 * ref, "%s: level %zu P B_c != B (%g)", what, k, err / ref);
      if (C.A.nrows > 1) {
        const std::vector<double> AB = matvec(C.A, C.B);
        double e = 0.0, bmax = 0.0;
        for (size_t i = 0; i < AB.size(); ++i) e = std::max(e, std::fabs(AB[i]));
        for (double b : C.B) bmax = std::max(bmax, std::fabs(b));
        CHECK(e <= 1e-12 * max_abs(C.A) * bmax, "%s: level %zu A_c B_c != 0", what, k + 1);
      }
    } else if (o.coarsening == BD_RS) {
      const std::vector<double> one(P.ncols, 1.0), ones_f(L.A.nrows, 1.0);
      const std::vector<double> P1 = matvec(P, one), A1 = matvec(L.A, ones_f);
      for (int32_t i = 0; i < P.nrows; ++i)
        if (std::fabs(A1[i]) <= 1e-13 * max_abs(L.A) && P.rp[i + 1] > P.rp[i])
          CHECK(std::fabs(P1[i] - 1.0) <= 1e-13, "%s: level %zu row %d P 1 = %g", what, k, i, P1[i]);
    }
  }
  if (H.coarse_mode == 0) {
    const int nM = H.lv.back().A.nrows;
    CHECK((int64_t)H.G.size() == (int64_t)nM * nM, "%s: coarse inverse size", what);
    for (double g : H.G) CHECK(std::isfinite(g), "%s: non-finite coarse inverse", what);
  }
}

int main() {
  const int dims[][3] = {{1, 1, 1}, {2, 2, 1}, {5, 4, 3}, {16, 16, 8}, {23, 19, 9}};
  for (const auto& d : dims) {
    const bd_slab s = slab(d[0], d[1], d[2]);
    Csr Ai, Ae;
    assemble_slab_stiffness(s, s.sig_il, s.sig_it, Ai);
    assemble_slab_stiffness(s, s.sig_el, s.sig_et, Ae);
    std::vector<double> m;
    slab_lumped_mass(s, m);
    const int64_t n = slab_nodes(s);
    CHECK(Ai.nrows == n && (int64_t)m.size() == n, "slab %dx%dx%d sizes", d[0], d[1], d[2]);
    CHECK(validate(Ai).empty(), "slab %dx%dx%d CSR: %s", d[0], d[1], d[2], validate(Ai).c_str());
    CHECK(exactly_symmetric(Ai), "slab %dx%dx%d A_i not symmetric", d[0], d[1], d[2]);
    double vol = 0.0;
    for (double x : m) vol += x;
    CHECK(std::fabs(vol - 0.5) <= 1e-13, "slab %dx%dx%d mass sum %g", d[0], d[1], d[2], vol);
    const std::vector<double> r = matvec(Ai, std::vector<double>(n, 1.0));
    for (double x : r) CHECK(std::fabs(x) <= 1e-13 * max_abs(Ai), "slab %dx%dx%d A_i 1 != 0", d[0], d[1], d[2]);
    Csr Aell = Ai, Apar = Ai;
    for (int32_t i = 0; i < Aell.nrows; ++i)
      for (int32_t k = Aell.rp[i]; k < Aell.rp[i + 1]; ++k) {
        Aell.v[k] += Ae.v[k];
        if (Apar.ci[k] == i) Apar.v[k] += s.cm / s.dt * m[i];
      }
    for (int variant = 0; variant < 6; ++variant) {
      bd_amg_opts o;
      bidomain_default_opts(&o);
      o.coarse_eq_limit = n < 200 ? 4 : 100;
      o.galerkin_device = 0;
      const char* what = "sa";
      Csr A = Aell;
      o.nullspace = BD_NULL_CONSTANT;
      if (variant == 1) { o.square_graph_levels = 0; what = "sa-unsquared"; }
      if (variant == 2) { o.coarsening = BD_RS; o.threshold = 0.5; what = "rs"; }
      if (variant == 3) { o.smoother = BD_JACOBI; o.smoother_degree = 3; what = "sa-jacobi"; }
      if (variant == 4) { A = Apar; o.nullspace = BD_NULL_NONE; o.threshold = 0.0; what = "parabolic"; }
      if (variant == 5) { o.coarsening = BD_PMIS; o.threshold = 0.5; o.seed = 7; what = "pmis"; }
      HostHierarchy H;
      std::string err;
      const int rc = build_hierarchy(A, o, H, err);
      CHECK(rc == BD_OK, "slab %dx%dx%d %s: setup failed: %s", d[0], d[1], d[2], what, err.c_str());
      if (rc == BD_OK) check_hierarchy(H, o, what);
    }
  }
  // the theta-periodic truncated ellipsoid (n_theta = 3 is the smallest periodic ring)
  const int edims[][3] = {{3, 1, 1}, {4, 2, 1}, {7, 5, 3}, {16, 12, 6}};
  for (const auto& d : edims) {
    bd_ellipsoid e{};
    e.n_theta = d[0]; e.n_phi = d[1]; e.n_r = d[2];
    e.a1 = 2.2; e.a2 = 3.3; e.b1 = 2.0; e.b2 = 3.1; e.c1 = 5.9; e.c2 = 6.4;
    e.theta_min = -1.5 * M_PI; e.theta_max = 0.5 * M_PI; e.phi_min = -0.375 * M_PI; e.phi_max = 0.125 * M_PI;
    e.sig_il = 3.0e-3; e.sig_it = 3.1525e-4; e.sig_el = 2.0e-3; e.sig_et = 1.3514e-3;
    e.fiber_endo = M_PI / 3.0; e.fiber_epi = -M_PI / 3.0;
    Csr A;
    std::vector<double> m;
    const bool ok = assemble_ellipsoid(e, e.sig_il + e.sig_el, e.sig_it + e.sig_et, A, &m);
    CHECK(ok, "ellipsoid %dx%dx%d: non-positive Jacobian", d[0], d[1], d[2]);
    if (!ok) continue;
    CHECK(A.nrows == ellipsoid_nodes(e) && A.nnz() == ellipsoid_nnz(e), "ellipsoid %dx%dx%d sizes", d[0], d[1], d[2]);
    CHECK(validate(A).empty(), "ellipsoid %dx%dx%d CSR: %s", d[0], d[1], d[2], validate(A).c_str());
    CHECK(exactly_symmetric(A), "ellipsoid %dx%dx%d not symmetric", d[0], d[1], d[2]);
    for (double x : m) CHECK(x > 0, "ellipsoid %dx%dx%d non-positive mass", d[0], d[1], d[2]);
    const std::vector<double> r = matvec(A, std::vector<double>(A.nrows, 1.0));
    for (double x : r) CHECK(std::fabs(x) <= 1e-13 * max_abs(A), "ellipsoid %dx%dx%d A 1 != 0", d[0], d[1], d[2]);
    bd_amg_opts o;
    bidomain_default_opts(&o);
    o.coarse_eq_limit = A.nrows < 200 ? 4 : 100;
    o.galerkin_device = 0;
    o.nullspace = BD_NULL_CONSTANT;
    HostHierarchy H;
    std::string err;
    const int rc = build_hierarchy(A, o, H, err);
    CHECK(rc == BD_OK, "ellipsoid %dx%dx%d: setup failed: %s", d[0], d[1], d[2], err.c_str());
    if (rc == BD_OK) check_hierarchy(H, o, "ellipsoid sa");
  }
  // reverse Cuthill-McKee numbering: a permutation; a shuffled path (and a graph of several
  // paths and isolated nodes) gets bandwidth 1 back; renumbered() is the permuted matrix
  {
    auto bandwidth = [](const Csr& A) {
      int32_t b = 0;
      for (int32_t i = 0; i < A.nrows; ++i)
        for (int32_t k = A.rp[i]; k < A.rp[i + 1]; ++k) b = std::max(b, std::abs(A.ci[k] - i));
      return b;
    };
    auto is_perm = [](const std::vector<int32_t>& q, int32_t n) {
      std::vector<int> hit(n, 0);
      if ((int32_t)q.size() != n) return false;
      for (int32_t v : q) {
        if (v < 0 || v >= n || hit[v]) return false;
        hit[v] = 1;
      }
      return true;
    };
    for (int comps = 1; comps <= 3; ++comps) {
      const int32_t n = 997;
      std::vector<int32_t> lab(n);  // node at path position i
      for (int32_t i = 0; i < n; ++i) lab[i] = i;
      uint64_t z = 12345 + comps;
      for (int32_t i = n - 1; i > 0; --i) {  // Fisher-Yates with a fixed LCG
        z = z * 6364136223846793005ull + 1442695040888963407ull;
        std::swap(lab[i], lab[(int32_t)((z >> 33) % (uint64_t)(i + 1))]);
      }
      std::vector<std::vector<int32_t>> adj(n);
      for (int32_t i = 0; i + 1 < n; ++i) {
        if (comps > 1 && (i % (n / comps) == n / comps - 1)) continue;  // cut into components
        if (comps == 3 && i % 97 == 0) continue;                         // and a few isolated pieces
        adj[lab[i]].push_back(lab[i + 1]);
        adj[lab[i + 1]].push_back(lab[i]);
      }
      Csr A;
      A.nrows = A.ncols = n;
      A.rp.assign(n + 1, 0);
      for (int32_t i = 0; i < n; ++i) {
        adj[i].push_back(i);
        std::sort(adj[i].begin(), adj[i].end());
        A.rp[i + 1] = A.rp[i] + (int32_t)adj[i].size();
        for (int32_t c : adj[i]) {
          A.ci.push_back(c);
          A.v.push_back(c == i ? 2.0 + 0.001 * i : -1.0 - 0.001 * (i + c));
        }
      }
      const std::vector<int32_t> q = rcm_order(A);
      CHECK(is_perm(q, n), "rcm (%d components): not a permutation", comps);
      if (!is_perm(q, n)) continue;
      std::vector<int32_t> inv(n);
      for (int32_t i = 0; i < n; ++i) inv[q[i]] = i;
      const Csr B = renumbered(A, q.data(), inv.data());
      CHECK(validate(B).empty(), "rcm (%d components): renumbered CSR: %s", comps, validate(B).c_str());
      CHECK(bandwidth(B) == 1, "rcm (%d components): bandwidth %d, not 1", comps, bandwidth(B));
      std::vector<double> x(n);
      for (int32_t i = 0; i < n; ++i) x[i] = std::sin(0.37 * i);
      std::vector<double> xb(n);
      for (int32_t i = 0; i < n; ++i) xb[i] = x[q[i]];
      const std::vector<double> y = matvec(A, x), yb = matvec(B, xb);
      for (int32_t i = 0; i < n; ++i)
        CHECK(std::fabs(yb[i] - y[q[i]]) <= 1e-14 * (1.0 + std::fabs(y[q[i]])), "rcm: renumbered product row %d", i);
    }
    // on a coarse SA level of a slab: a permutation, and no wider than the aggregate numbering
    const bd_slab s = slab(23, 19, 9);
    Csr Ai;
    assemble_slab_stiffness(s, s.sig_il, s.sig_it, Ai);
    bd_amg_opts o;
    bidomain_default_opts(&o);
    o.coarse_eq_limit = 100;
    o.galerkin_device = 0;
    o.nullspace = BD_NULL_CONSTANT;
    HostHierarchy H;
    std::string err;
    CHECK(build_hierarchy(Ai, o, H, err) == BD_OK && H.lv.size() > 2, "rcm: slab hierarchy: %s", err.c_str());
    if (H.lv.size() > 2) {
      const Csr& A1 = H.lv[1].A;
      const std::vector<int32_t> q = rcm_order(A1);
      CHECK(is_perm(q, A1.nrows), "rcm: level 1 not a permutation");
      if (is_perm(q, A1.nrows)) {
        std::vector<int32_t> inv(A1.nrows);
        for (int32_t i = 0; i < A1.nrows; ++i) inv[q[i]] = i;
        const Csr B = renumbered(A1, q.data(), inv.data());
        CHECK(B.nnz() == A1.nnz() && validate(B).empty(), "rcm: level 1 renumbered CSR");
        CHECK(bandwidth(B) <= bandwidth(A1), "rcm: level 1 bandwidth %d > %d", bandwidth(B), bandwidth(A1));
      }
    }
  }
  // malformed input is rejected, not read out of bounds
  Csr bad;
  bad.nrows = bad.ncols = 3;
  bad.rp = {0, 2, 3, 5};
  bad.ci = {1, 0, 1, 2, 2};
  bad.v = {1, 1, 1, 1, 1};
  CHECK(!validate(bad).empty(), "unsorted columns accepted");
  std::printf(g_fail ? "host check: %d failures\n" : "host check ok\n", g_fail);
  return g_fail ? 1 : 0;
}
