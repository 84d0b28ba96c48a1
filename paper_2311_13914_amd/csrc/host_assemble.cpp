// Q1 finite-element operators of the Bidomain slab (Sec. 2.2; conductivity of eq. (2)).
//
// The stiffness entry a_pq = sum over elements e that contain p and q of
// int_e grad(phi_q)^T D grad(phi_p), computed row by row: each row gathers the (up to eight)
// elements around its node, so rows are independent and assembled in parallel.  Element
// matrices depend on the element layer only (D varies with z), and are integrated with the
// 2x2x2 Gauss rule with D taken at each Gauss point.  Fibers lie in the xy-plane at angle
// theta(z) = theta0 + rotation * z / Lz; tissue is axisymmetric (sigma_n = sigma_t), so
// D = sigma_t I + (sigma_l - sigma_t) a a^T.
#include <array>
#include <cmath>

#include "bd_host.hpp"

namespace bd {

int64_t slab_nodes(const bd_slab& s) {
  return (int64_t)(s.nx + 1) * (s.ny + 1) * (s.nz + 1);
}

namespace {

using Mat8 = std::array<double, 64>;

// Element matrix of layer ez.  Local node l = a + 2b + 4c at offset (a, b, c).
Mat8 layer_element(const bd_slab& s, int ez, double sl, double st) {
  const double hx = s.Lx / s.nx, hy = s.Ly / s.ny, hz = s.Lz / s.nz;
  const double g[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
  const double wq = 0.125 * hx * hy * hz;  // product of the 1-D weights (1/2 each) times |J|
  Mat8 K{};
  for (int qz = 0; qz < 2; ++qz) {
    const double th = s.fiber_theta0 + s.fiber_rotation * ((ez + g[qz]) * hz) / s.Lz;
    const double ax = std::cos(th), ay = std::sin(th);
    const double dl = sl - st;
    const double D[3][3] = {{st + dl * ax * ax, dl * ax * ay, 0.0},
                            {dl * ax * ay, st + dl * ay * ay, 0.0},
                            {0.0, 0.0, st}};
    for (int qy = 0; qy < 2; ++qy)
      for (int qx = 0; qx < 2; ++qx) {
        const double t[3] = {g[qx], g[qy], g[qz]};
        const double h[3] = {hx, hy, hz};
        double grad[8][3];
        for (int l = 0; l < 8; ++l) {
          const int bit[3] = {l & 1, (l >> 1) & 1, (l >> 2) & 1};
          double val[3], der[3];
          for (int d = 0; d < 3; ++d) {
            val[d] = bit[d] ? t[d] : 1.0 - t[d];
            der[d] = (bit[d] ? 1.0 : -1.0) / h[d];
          }
          grad[l][0] = der[0] * val[1] * val[2];
          grad[l][1] = val[0] * der[1] * val[2];
          grad[l][2] = val[0] * val[1] * der[2];
        }
        for (int l = 0; l < 8; ++l) {
          double Dg[3];
          for (int a = 0; a < 3; ++a) Dg[a] = D[a][0] * grad[l][0] + D[a][1] * grad[l][1] + D[a][2] * grad[l][2];
          for (int m = l; m < 8; ++m)
            K[l * 8 + m] += wq * (Dg[0] * grad[m][0] + Dg[1] * grad[m][1] + Dg[2] * grad[m][2]);
        }
      }
  }
  for (int l = 0; l < 8; ++l)
    for (int m = 0; m < l; ++m) K[l * 8 + m] = K[m * 8 + l];
  return K;
}

}  // namespace

void assemble_slab_stiffness(const bd_slab& s, double sl, double st, Csr& A) {
  const int nxp = s.nx + 1, nyp = s.ny + 1, nzp = s.nz + 1;
  const int64_t n = slab_nodes(s);
  std::vector<Mat8> Kz(s.nz);
  for (int ez = 0; ez < s.nz; ++ez) Kz[ez] = layer_element(s, ez, sl, st);

  A.nrows = A.ncols = (int32_t)n;
  A.rp.assign(n + 1, 0);
  auto span = [](int i, int np) { return (i > 0 ? 1 : 0) + 1 + (i + 1 < np ? 1 : 0); };
  for (int64_t p = 0; p < n; ++p) {
    const int i = (int)(p % nxp), j = (int)((p / nxp) % nyp), k = (int)(p / ((int64_t)nxp * nyp));
    A.rp[p + 1] = span(i, nxp) * span(j, nyp) * span(k, nzp);
  }
  for (int64_t p = 0; p < n; ++p) A.rp[p + 1] += A.rp[p];
  A.ci.resize(A.rp[n]);
  A.v.resize(A.rp[n]);

#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < n; ++p) {
    const int i = (int)(p % nxp), j = (int)((p / nxp) % nyp), k = (int)(p / ((int64_t)nxp * nyp));
    int64_t pos = A.rp[p];
    for (int dk = -1; dk <= 1; ++dk) {
      if (k + dk < 0 || k + dk >= nzp) continue;
      for (int dj = -1; dj <= 1; ++dj) {
        if (j + dj < 0 || j + dj >= nyp) continue;
        for (int di = -1; di <= 1; ++di) {
          if (i + di < 0 || i + di >= nxp) continue;
          double a = 0.0;
          // elements (ex, ey, ez) containing both p and q = p + (di, dj, dk)
          for (int ez = k - 1; ez <= k; ++ez) {
            if (ez < 0 || ez >= s.nz || k + dk < ez || k + dk > ez + 1) continue;
            for (int ey = j - 1; ey <= j; ++ey) {
              if (ey < 0 || ey >= s.ny || j + dj < ey || j + dj > ey + 1) continue;
              for (int ex = i - 1; ex <= i; ++ex) {
                if (ex < 0 || ex >= s.nx || i + di < ex || i + di > ex + 1) continue;
                const int lp = (i - ex) + 2 * (j - ey) + 4 * (k - ez);
                const int lq = (i + di - ex) + 2 * (j + dj - ey) + 4 * (k + dk - ez);
                a += Kz[ez][lp * 8 + lq];
              }
            }
          }
          A.ci[pos] = (int32_t)(p + di + (int64_t)nxp * dj + (int64_t)nxp * nyp * dk);
          A.v[pos] = a;
          ++pos;
        }
      }
    }
  }
}

void slab_lumped_mass(const bd_slab& s, std::vector<double>& m) {
  const int nxp = s.nx + 1, nyp = s.ny + 1, nzp = s.nz + 1;
  const double vol8 = (s.Lx / s.nx) * (s.Ly / s.ny) * (s.Lz / s.nz) / 8.0;
  m.resize(slab_nodes(s));
  auto cnt = [](int i, int np) { return (i == 0 || i == np - 1) ? 1.0 : 2.0; };
#pragma omp parallel for schedule(static)
  for (int64_t p = 0; p < (int64_t)m.size(); ++p) {
    const int i = (int)(p % nxp), j = (int)((p / nxp) % nyp), k = (int)(p / ((int64_t)nxp * nyp));
    m[p] = cnt(i, nxp) * cnt(j, nyp) * cnt(k, nzp) * vol8;  // elements around p, each |e| / 8
  }
}

}  // namespace bd
