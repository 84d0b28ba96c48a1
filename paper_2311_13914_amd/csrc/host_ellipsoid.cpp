// Q1 finite-element operators of the truncated ellipsoid, the idealised left ventricle of Sec. 3
// (eq. (8), Table 1), with the conductivities of eq. (2) and the Q1 space of Sec. 2.2.
//
// Geometry.  A point of parameters (theta, phi, r) sits at
//   x = a(r) cos(theta) cos(phi),  y = b(r) sin(theta) cos(phi),  z = c(r) sin(phi),
// a(r) = a1 + r (a2 - a1) and likewise b(r), c(r); r = 0 is the endocardium, r = 1 the
// epicardium.  (Eq. (8) prints cos(theta) sin(phi) in y, which would flatten every theta-line
// into a plane; the ellipsoid has sin(theta) cos(phi).)  theta spans one full period, so the
// mesh is periodic in theta: node p = i + n_theta (j + (n_phi + 1) k) at (theta_i, phi_j, r_k)
// on uniform grids, i taken mod n_theta.  Elements are isoparametric trilinear hexahedra: inside
// element (i, j, k) the position is the trilinear interpolation of its eight nodes' positions
// (local node l = a + 2b + 4c at (i + a mod n_theta, j + b, k + c)), and every integral uses
// the 2x2x2 Gauss rule on the reference cube.
//
// Fibers lie in the tangent plane of the r-surfaces, a_l = cos(alpha) e_theta + sin(alpha) e_phi
// with e_theta the unit d/dtheta direction and e_phi the unit part of d/dphi orthogonal to it;
// alpha(r) = alpha_endo + r (alpha_epi - alpha_endo) turns counterclockwise (seen from outside)
// from the epicardium to the endocardium, as Sec. 2 describes.  Each Gauss point takes the
// fiber at its own (theta, phi, r), the trilinear interpolation of the element's nodal
// parameters; tissue is axisymmetric (sigma_n = sigma_t in eq. (2)).
//
// Assembly runs layer by layer in r: the element matrices of layers k - 1 and k are held (two
// layers of n_theta n_phi 8x8 matrices, whatever the mesh depth), and the rows of node layer k
// gather their entries from the elements around each node, in parallel over rows.  The pattern
// is the full 27-point one (3 theta x up to 3 phi x up to 3 r neighbours), structural zeros
// kept, columns sorted.
#include <algorithm>
#include <array>
#include <atomic>
#include <cmath>
#include <utility>

#include "bd_host.hpp"

namespace bd {

int64_t ellipsoid_nodes(const bd_ellipsoid& e) {
  return (int64_t)e.n_theta * (e.n_phi + 1) * (e.n_r + 1);
}

int64_t ellipsoid_nnz(const bd_ellipsoid& e) {
  return 3 * (int64_t)e.n_theta * (3 * (int64_t)e.n_phi + 1) * (3 * (int64_t)e.n_r + 1);
}

namespace {

using Mat8 = std::array<double, 64>;

struct Vec3 {
  double x, y, z;
};

double theta_at(const bd_ellipsoid& e, double i) {
  return e.theta_min + (e.theta_max - e.theta_min) * i / e.n_theta;
}
double phi_at(const bd_ellipsoid& e, double j) {
  return e.phi_min + (e.phi_max - e.phi_min) * j / e.n_phi;
}

Vec3 point(const bd_ellipsoid& e, double th, double ph, double r) {
  const double a = e.a1 + r * (e.a2 - e.a1), b = e.b1 + r * (e.b2 - e.b1), c = e.c1 + r * (e.c2 - e.c1);
  return {a * std::cos(th) * std::cos(ph), b * std::sin(th) * std::cos(ph), c * std::sin(ph)};
}

// Fiber direction at parameters (th, ph, r).
Vec3 fiber(const bd_ellipsoid& e, double th, double ph, double r) {
  const double a = e.a1 + r * (e.a2 - e.a1), b = e.b1 + r * (e.b2 - e.b1), c = e.c1 + r * (e.c2 - e.c1);
  const double ct = std::cos(th), st = std::sin(th), cp = std::cos(ph), sp = std::sin(ph);
  Vec3 t{-a * st * cp, b * ct * cp, 0.0};        // d position / d theta
  const Vec3 f{-a * ct * sp, -b * st * sp, c * cp};  // d position / d phi
  const double tn = std::sqrt(t.x * t.x + t.y * t.y);
  t = {t.x / tn, t.y / tn, 0.0};
  const double ft = f.x * t.x + f.y * t.y;
  Vec3 q{f.x - ft * t.x, f.y - ft * t.y, f.z};
  const double qn = std::sqrt(q.x * q.x + q.y * q.y + q.z * q.z);
  q = {q.x / qn, q.y / qn, q.z / qn};
  const double al = e.fiber_endo + r * (e.fiber_epi - e.fiber_endo);
  const double ca = std::cos(al), sa = std::sin(al);
  return {ca * t.x + sa * q.x, ca * t.y + sa * q.y, ca * t.z + sa * q.z};
}

// Stiffness (sig_l, sig_t) and the integrals of the basis functions over element (i, j, k).
// Returns false if the interpolated geometry has a non-positive Jacobian at a Gauss point.
bool element(const bd_ellipsoid& e, int i, int j, int k, double sl, double sg, Mat8& K, double* mi) {
  const double g[2] = {0.5 - 0.5 / std::sqrt(3.0), 0.5 + 0.5 / std::sqrt(3.0)};
  const double th0 = theta_at(e, i), dth = (e.theta_max - e.theta_min) / e.n_theta;
  const double ph0 = phi_at(e, j), dph = phi_at(e, j + 1) - ph0;
  const double r0 = (double)k / e.n_r, dr = (double)(k + 1) / e.n_r - r0;
  Vec3 X[8];
  for (int l = 0; l < 8; ++l)
    X[l] = point(e, th0 + (l & 1) * dth, phi_at(e, j + ((l >> 1) & 1)), (double)(k + ((l >> 2) & 1)) / e.n_r);
  K.fill(0.0);
  for (int l = 0; l < 8; ++l) mi[l] = 0.0;
  for (int qz = 0; qz < 2; ++qz)
    for (int qy = 0; qy < 2; ++qy)
      for (int qx = 0; qx < 2; ++qx) {
        const double t[3] = {g[qx], g[qy], g[qz]};
        double N[8], dN[8][3];
        for (int l = 0; l < 8; ++l) {
          const int bit[3] = {l & 1, (l >> 1) & 1, (l >> 2) & 1};
          double f[3], s[3];
          for (int d = 0; d < 3; ++d) {
            f[d] = bit[d] ? t[d] : 1.0 - t[d];
            s[d] = bit[d] ? 1.0 : -1.0;
          }
          N[l] = f[0] * f[1] * f[2];
          dN[l][0] = s[0] * f[1] * f[2];
          dN[l][1] = f[0] * s[1] * f[2];
          dN[l][2] = f[0] * f[1] * s[2];
        }
        // J[d][q] = d x_d / d xi_q of the trilinear geometry
        double J[3][3] = {};
        for (int l = 0; l < 8; ++l) {
          const double xl[3] = {X[l].x, X[l].y, X[l].z};
          for (int d = 0; d < 3; ++d)
            for (int q = 0; q < 3; ++q) J[d][q] += xl[d] * dN[l][q];
        }
        // inverse through the cofactors: Jinv[q][d] = cof(J)[d][q] / det
        double C[3][3];
        for (int d = 0; d < 3; ++d)
          for (int q = 0; q < 3; ++q) {
            const int d1 = (d + 1) % 3, d2 = (d + 2) % 3, q1 = (q + 1) % 3, q2 = (q + 2) % 3;
            C[d][q] = J[d1][q1] * J[d2][q2] - J[d1][q2] * J[d2][q1];
          }
        const double det = J[0][0] * C[0][0] + J[0][1] * C[0][1] + J[0][2] * C[0][2];
        if (!(det > 0.0)) return false;
        // physical gradients G[l][d] = sum_q dN[l][q] Jinv[q][d]
        double G[8][3];
        for (int l = 0; l < 8; ++l)
          for (int d = 0; d < 3; ++d)
            G[l][d] = (dN[l][0] * C[d][0] + dN[l][1] * C[d][1] + dN[l][2] * C[d][2]) / det;
        const Vec3 a = fiber(e, th0 + t[0] * dth, ph0 + t[1] * dph, r0 + t[2] * dr);
        const double av[3] = {a.x, a.y, a.z};
        double D[3][3];
        for (int p = 0; p < 3; ++p)
          for (int q = 0; q < 3; ++q) D[p][q] = (sl - sg) * av[p] * av[q] + (p == q ? sg : 0.0);
        const double w = 0.125 * det;  // product of the 1-D weights (1/2 each) times det J
        for (int l = 0; l < 8; ++l) {
          double Dg[3];
          for (int p = 0; p < 3; ++p) Dg[p] = D[p][0] * G[l][0] + D[p][1] * G[l][1] + D[p][2] * G[l][2];
          for (int m = l; m < 8; ++m) K[l * 8 + m] += w * (Dg[0] * G[m][0] + Dg[1] * G[m][1] + Dg[2] * G[m][2]);
          mi[l] += w * N[l];
        }
      }
  for (int l = 0; l < 8; ++l)
    for (int m = 0; m < l; ++m) K[l * 8 + m] = K[m * 8 + l];
  return true;
}

}  // namespace

bool assemble_ellipsoid(const bd_ellipsoid& e, double sl, double sg, Csr& A, std::vector<double>* mass) {
  const int nt = e.n_theta, np = e.n_phi + 1, nr = e.n_r + 1;
  const int64_t n = ellipsoid_nodes(e);
  const int64_t ring = (int64_t)nt * np;  // nodes of one r-layer
  A.nrows = A.ncols = (int32_t)n;
  A.rp.assign(n + 1, 0);
  auto span = [](int v, int cnt) { return (v > 0 ? 1 : 0) + 1 + (v + 1 < cnt ? 1 : 0); };
  for (int64_t p = 0; p < n; ++p) {
    const int j = (int)((p / nt) % np), k = (int)(p / ring);
    A.rp[p + 1] = 3 * span(j, np) * span(k, nr);
  }
  for (int64_t p = 0; p < n; ++p) A.rp[p + 1] += A.rp[p];
  A.ci.resize(A.rp[n]);
  A.v.resize(A.rp[n]);
  if (mass) mass->assign(n, 0.0);

  const int64_t nel = (int64_t)nt * e.n_phi;  // elements of one r-layer
  std::vector<Mat8> K[2] = {std::vector<Mat8>(nel), std::vector<Mat8>(nel)};
  std::vector<std::array<double, 8>> M[2] = {std::vector<std::array<double, 8>>(nel),
                                              std::vector<std::array<double, 8>>(nel)};
  std::atomic<bool> ok{true};
  for (int k = 0; k < nr; ++k) {
    if (k < e.n_r) {
      std::vector<Mat8>& Kk = K[k & 1];
      std::vector<std::array<double, 8>>& Mk = M[k & 1];
#pragma omp parallel for schedule(static)
      for (int64_t q = 0; q < nel; ++q)
        if (!element(e, (int)(q % nt), (int)(q / nt), k, sl, sg, Kk[q], Mk[q].data()))
          ok.store(false, std::memory_order_relaxed);
    }
    if (!ok) return false;
#pragma omp parallel for schedule(static)
    for (int64_t pr = 0; pr < ring; ++pr) {
      const int i = (int)(pr % nt), j = (int)(pr / nt);
      const int64_t p = pr + ring * k;
      std::pair<int32_t, double> ent[27];
      int cnt = 0;
      double mp = 0.0;
      for (int dk = -1; dk <= 1; ++dk) {
        if (k + dk < 0 || k + dk >= nr) continue;
        for (int dj = -1; dj <= 1; ++dj) {
          if (j + dj < 0 || j + dj >= np) continue;
          for (int di = -1; di <= 1; ++di) {
            const int iq = (i + di + nt) % nt;
            double a = 0.0;
            // elements (ei, ej, ek) around p; local offsets of p and q inside them
            for (int ek = k - 1; ek <= k; ++ek) {
              if (ek < 0 || ek >= e.n_r || k + dk < ek || k + dk > ek + 1) continue;
              for (int ej = j - 1; ej <= j; ++ej) {
                if (ej < 0 || ej >= e.n_phi || j + dj < ej || j + dj > ej + 1) continue;
                for (int si = -1; si <= 0; ++si) {  // element i + si (mod n_theta)
                  const int ap = -si, aq = di - si;
                  if (aq < 0 || aq > 1) continue;
                  const int ei = (i + si + nt) % nt;
                  const int lp = ap + 2 * (j - ej) + 4 * (k - ek);
                  const int lq = aq + 2 * (j + dj - ej) + 4 * (k + dk - ek);
                  const int64_t q = ei + (int64_t)nt * ej;
                  a += K[ek & 1][q][lp * 8 + lq];
                  if (dk == 0 && dj == 0 && di == 0) mp += M[ek & 1][q][lp];
                }
              }
            }
            ent[cnt++] = {(int32_t)(iq + (int64_t)nt * (j + dj) + ring * (k + dk)), a};
          }
        }
      }
      std::sort(ent, ent + cnt, [](const auto& x, const auto& y) { return x.first < y.first; });
      int64_t pos = A.rp[p];
      for (int c = 0; c < cnt; ++c, ++pos) {
        A.ci[pos] = ent[c].first;
        A.v[pos] = ent[c].second;
      }
      if (mass) (*mass)[p] = mp;
    }
  }
  return true;
}

}  // namespace bd
