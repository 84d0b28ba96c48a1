// Host-side data structures of the library: CSR matrices, the AMG level hierarchy as built
// on the host, and the setup/assembly routines (setup phase, Alg. 1; Q1 assembly, Sec. 2.2).
#pragma once

#include <cmath>
#include <cstdint>
#include <limits>
#include <memory>
#include <functional>
#include <string>
#include <vector>

#include "bidomain.h"

namespace bd {

struct Csr {
  int32_t nrows = 0, ncols = 0;
  std::vector<int32_t> rp;  // nrows + 1
  std::vector<int32_t> ci;  // nnz, sorted within each row
  std::vector<double> v;    // nnz
  int64_t nnz() const { return (int64_t)ci.size(); }
};

// C = A^T (columns sorted).
Csr transpose(const Csr& A);
// C = A B on the structural pattern of the product (no value is dropped); every entry summed in
// the order of A's row, each product and sum rounded separately.
Csr spgemm(const Csr& A, const Csr& B);
// (A + A^T) / 2 on A's pattern (a mirror entry that does not exist counts as zero).
Csr symmetrized(const Csr& A);
// Reverse Cuthill-McKee numbering of the graph of a square matrix with a symmetric pattern
// (Cuthill & McKee, 1969; reversed after George, 1971): each connected component is walked
// breadth-first from a node of least degree (ties: lowest index), the unvisited neighbours of a
// node queued by increasing degree (ties: index); the visit order, reversed, is returned as
// new -> old.
std::vector<int32_t> rcm_order(const Csr& A);
// Row- and column-renumbered copy of M: row i of the result is row rows[i] of M (rows: new ->
// old, or null to keep the order), column c becomes cols[c] (cols: old -> new, or null); each row
// sorted by its new column.
Csr renumbered(const Csr& M, const int32_t* rows, const int32_t* cols);
// Tentative SA prolongator: P(i, agg[i]) = B_i / |B restricted to the aggregate| (norms summed in
// index order); Bc receives the norms (the coarse near-null vector).
Csr tentative_prolongator(const std::vector<double>& B, const std::vector<int32_t>& agg, int32_t nc,
                          std::vector<double>& Bc);
// Damping of the prolongator smoothing, 4 / (3 lambda).
double prolongator_damping(double lam);
// SA strength: a coupling is strong when its weight is >= strength_cut(theta); weights >=
// tie_keep() times the largest tie in the aggregation passes.
double strength_cut(double theta);
double tie_keep();
std::vector<double> diagonal(const Csr& A);
// Checks the boundary's CSR contract; returns an empty string when valid.
std::string validate(const Csr& A);

}  // namespace bd
struct StreamPlan;  // device launch plan of a matrix (filled by the device library)
namespace bd {

struct HostLevel {
  Csr A;                        // level operator
  Csr P, R;                     // prolongator to this level from the next, and its transpose
  std::shared_ptr<StreamPlan> plan_a, plan_p, plan_r;  // launch plans, once planned
  std::vector<double> B;        // near-null vector on this level
  std::vector<double> Dinv;     // 1 / diag(A)
  double lam = std::numeric_limits<double>::quiet_NaN();  // lambda_max(D^{-1} A) estimate
  // Numbering of this level's unknowns on the device, new -> old (empty: the host's); set with
  // the launch plans, which then hold the renumbered matrices.
  std::vector<int32_t> perm;
};

struct HostHierarchy {
  std::vector<HostLevel> lv;
  int coarse_mode = 0;          // 0: dense G on the coarsest level, 1: smoother relaxation
  std::vector<double> G;        // n_M x n_M row-major: A_M^{-1}, or the pseudo-inverse on b-perp
};

// Galerkin product on another engine: given A_k, P_k, R_k = P_k^T and the number of partial
// products of A_k P_k, either fills A_c = symmetrized R_k (A_k P_k) exactly as the host would
// and returns true, or returns false and the host computes it.
using GalerkinOffload = std::function<bool(const Csr& A, const Csr& P, const Csr& R, int64_t sparse_flops, Csr& Ac)>;

// The SA coarsening of a level on another engine (independent set BD_MIS_LUBY): given A_k, its
// diagonal d and D^{-1}, the near-null vector B_k and the level index, either fills lambda, P_k,
// B_{k+1} and the number of aggregates exactly as the host would and returns true, or returns
// false and the host builds them.
using AggregateOffload = std::function<bool(const Csr& A, const std::vector<double>& d, const std::vector<double>& Dinv,
                                            const std::vector<double>& B, int level, double& lam, Csr& P,
                                            std::vector<double>& Bc, int32_t& nc)>;

// SplitMix64 stream offset of the parallel independent set's priorities (seed + offset + level).
constexpr uint64_t kLubySeedOffset = 0x4C554259;

// Setup phase: returns BD_OK or a BD_E_* code with a message in err.
int build_hierarchy(Csr A, const bd_amg_opts& o, HostHierarchy& H, std::string& err,
                    const GalerkinOffload* offload = nullptr, const AggregateOffload* agg_offload = nullptr);

// Largest Ritz value of D^{-1} A after `iters` Jacobi-CG steps from a SplitMix64 vector.  Dot
// products: blocks of kDotBlock entries summed in order, then the block sums in order.
double lambda_estimate(const Csr& A, const std::vector<double>& Dinv, int iters, uint64_t seed);
// The same from the CG coefficients (alpha, beta) such a run produced (the CG/Lanczos relation);
// without any step, the largest diagonal entry of D^{-1} A.
double ritz_from_cg(const Csr& A, const std::vector<double>& Dinv, const std::vector<double>& alpha,
                    const std::vector<double>& beta);
constexpr int kDotBlock = 4096;

// Q1 slab operators (27-point pattern, structural zeros kept).
void assemble_slab_stiffness(const bd_slab& s, double sig_l, double sig_t, Csr& A);
void slab_lumped_mass(const bd_slab& s, std::vector<double>& m);
int64_t slab_nodes(const bd_slab& s);

// Q1 operators of the theta-periodic truncated ellipsoid (isoparametric, 27-point pattern,
// structural zeros kept).  Returns false if an element's interpolated geometry has a non-positive
// Jacobian at a Gauss point.  mass (may be null): integral of each basis function.
bool assemble_ellipsoid(const bd_ellipsoid& e, double sig_l, double sig_t, Csr& A, std::vector<double>* mass);
int64_t ellipsoid_nodes(const bd_ellipsoid& e);
int64_t ellipsoid_nnz(const bd_ellipsoid& e);

}  // namespace bd
