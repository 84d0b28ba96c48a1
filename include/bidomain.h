/*
 * bidomain.h -- C ABI of the MI355X (gfx950) AMG-preconditioned CG solver for the
 * decoupled Bidomain step.
 *
 * The method: Centofanti & Scacchi, "A comparison of Algebraic Multigrid Bidomain solvers
 * on hybrid CPU-GPU architectures".  Each time step of the IMEX scheme (eqs. (4)-(7)) solves
 * one elliptic system (A_i + A_e) u_e = -A_i v and one parabolic system
 * (c_m/dt M + A_i) v^{n+1} = ... with CG preconditioned by algebraic multigrid (Sec. 2.2,
 * Sec. 4): a setup phase (Alg. 1) builds the level hierarchy once, and every CG iteration
 * applies one V-cycle (Alg. 2).
 *
 * Conventions for every entry point:
 *   - "_dev" pointers are device (HBM) pointers on the current HIP device; every other
 *     pointer is a host pointer.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).  All device work
 *     of a call is enqueued on that stream; calls return after the results are in place
 *     (they synchronise the stream once per convergence check).
 *   - The caller owns every buffer it passes; setup and create calls copy what they keep
 *     into library-owned device memory, so caller buffers may be freed once the call returns.
 *   - Handles are owned by the library and released by the matching *_destroy call.  A
 *     handle may be used by one stream (one host thread) at a time.
 *   - Return value: one of the BD_* status codes.  On a nonzero status,
 *     bidomain_last_error() returns a thread-local message.
 *   - Sparse matrices are CSR with 32-bit row offsets and column indices, columns sorted
 *     and unique within each row, square, every diagonal entry stored and positive.
 */
#ifndef BIDOMAIN_H
#define BIDOMAIN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------------------ */
#define BD_OK 0
#define BD_E_NOT_CONVERGED 1   /* maxit reached: x holds the last iterate, info is filled */
#define BD_E_INVALID (-1)      /* malformed CSR, bad options or arguments                  */
#define BD_E_NOMEM (-2)        /* device or host allocation failed                         */
#define BD_E_DEVICE (-3)       /* a HIP call failed                                        */
#define BD_E_BREAKDOWN (-4)    /* CG breakdown: p^T A p <= 0 or r^T z <= 0                 */
#define BD_E_NONFINITE (-5)    /* NaN/Inf in the right-hand side or an iterate             */
#define BD_E_BUDGET (-6)       /* serving: the case does not fit the device budget         */

/* ---- options ----------------------------------------------------------------------- */
/* coarsening: smoothed aggregation (GAMG's method), classical Ruge-Stueben first pass (the HMIS
 * split of a one-process run), or the PMIS split (the parallel independent-set coarsening of
 * BoomerAMG's GPU setup); the last two use the strength of eq. (10) and direct interpolation */
enum { BD_SA = 0, BD_RS = 1, BD_PMIS = 2 };
enum { BD_CHEBYSHEV = 0, BD_JACOBI = 1 };      /* level smoother                            */
enum { BD_F64 = 0, BD_F32 = 1 };               /* V-cycle precision                          */
enum { BD_NULL_NONE = 0, BD_NULL_CONSTANT = 1 };/* kernel of the operator                    */
enum { BD_PC_AMG = 0, BD_PC_JACOBI = 1, BD_PC_NONE = 2 }; /* preconditioner of the CG solve    */
enum { BD_MIS_GREEDY = 0, BD_MIS_LUBY = 1 };   /* SA independent set                         */

/*
 * AMG options.  Defaults (bidomain_default_opts) follow App. A of the paper: smoothed
 * aggregation with threshold 0.06, one prolongator smoothing, graph squaring on the first
 * level, coarse-equation limit 100, Chebyshev smoother of degree 2 on D^{-1}A over
 * [0.05, 1.05] x lambda with lambda from 10 Jacobi-CG steps; the independent set in its
 * parallel form (Sec. 4).  For BD_RS, `threshold` is the
 * strong threshold alpha of eq. (10) (0.5 is the paper's CPU optimum).
 */
typedef struct {
  int32_t coarsening;          /* BD_SA | BD_RS | BD_PMIS                                */
  double threshold;            /* SA theta (default 0.06) or the alpha of eq. (10)        */
  int32_t square_graph_levels; /* levels whose MIS runs on the squared graph (1)         */
  int32_t prolong_smooths;     /* Jacobi smoothings of the tentative prolongator (1)     */
  int32_t coarse_eq_limit;     /* stop coarsening at or below this many rows (100)       */
  int32_t max_levels;          /* (25)                                                   */
  int32_t smoother;            /* BD_CHEBYSHEV | BD_JACOBI                               */
  int32_t smoother_degree;     /* Chebyshev degree or Jacobi sweeps per application (2)  */
  double cheb_lo, cheb_hi;     /* Chebyshev interval factors (0.05, 1.05)                */
  int32_t esteig_iters;        /* CG steps of the eigenvalue estimate (10)               */
  uint64_t seed;               /* SplitMix64 seed of the estimate's start vector (seed + level)
                                * and of the PMIS draws (seed + 0x504D4953 + level) (0)   */
  int32_t vcycle_precision;    /* BD_F64 | BD_F32 (then the outer CG is flexible CG)     */
  int32_t nullspace;           /* BD_NULL_NONE | BD_NULL_CONSTANT                        */
  double stagnation_ratio;     /* stop coarsening when n_c > ratio * n_k (0.9)           */
  int32_t coarse_dense_max;    /* largest coarsest level solved directly (2048)          */
  /* Galerkin products R (A P) of the setup on the device, with this library's kernels: sparse
   * products (every entry summed in the host product's order with separately rounded
   * operations, so equal to the host's bit for bit) or, for the filled coarse levels, float64
   * MFMA products of the dense expansions that skip empty tiles (the same pattern, values
   * equal up to rounding order).  0 never; 1 (default) levels with at least 5e7 partial
   * products in A P, dense where both dimensions are at most 65,536 and the dense work is
   * within 1000 times the partial products, sparse otherwise; 2 every level, sparse; 3 every
   * level, dense where the dimensions allow.  A product whose buffers do not fit in half the
   * free device memory (or in a server's budget) falls back to the sparse form, then to the
   * host.  bidomain_amg_build_host never uses the device. */
  int32_t galerkin_device;
  /* 1: keep a level operator that equals its transpose and whose column - row offsets >= 0
   * are those of a 27-point stencil (the fine operators) in the symmetric diagonal form
   * (default); 0: CSR forms only. */
  int32_t diag_form;
  /* Preconditioner of bidomain_pcg_solve (and of the simulation's solves): BD_PC_AMG, one
   * V-cycle (default); BD_PC_JACOBI, z = D^{-1} r; BD_PC_NONE, z = r (plain CG; the paper runs
   * the parabolic system unpreconditioned on GPUs and with block Jacobi on CPUs, Sec. 5).
   * With JACOBI or NONE the setup keeps the fine level only and vcycle_precision must be
   * BD_F64; the serving API takes BD_PC_AMG only. */
  int32_t preconditioner;
  /* Independent set of the SA levels (Sec. 4: greedy, or its parallel form after Luby):
   * BD_MIS_LUBY (default) takes the nodes in decreasing random priority (the top 32 bits of
   * SplitMix64 draws from seed + 0x4C554259 + level, above the node index), the set the
   * parallel rounds reach; BD_MIS_GREEDY visits them in index order. */
  int32_t independent_set;
  /* 1 (default): with BD_MIS_LUBY, each SA level's eigenvalue estimate, strength graph,
   * independent set (parallel rounds), aggregates and smoothed prolongator are computed on the
   * device with this library's kernels -- the host's result bit for bit; 0: on the host.
   * bidomain_amg_build_host never uses the device. */
  int32_t aggregate_device;
  /* Renumbering of coarse levels on the device: the unknowns of an intermediate level (not the
   * fine one, not the coarsest; over 256 rows, at most 10 % dense) are put in reverse
   * Cuthill-McKee order, so that a row's columns -- and the gathers of the level's products --
   * fall on fewer cache lines and 16-bit column offsets become possible.  1 (default): levels of
   * at least 2^26 stored entries (the renumbering costs host setup time and memory that smaller
   * hierarchies do not earn back); 2: every such level; 0: none.  The host hierarchy, bidomain_amg_export and the
   * vectors of bidomain_amg_apply keep the aggregate numbering. */
  int32_t reorder;
} bd_amg_opts;

void bidomain_default_opts(bd_amg_opts* opts);

/* A CSR matrix in host memory (see the conventions above). */
typedef struct {
  int32_t n;
  int64_t nnz;
  const int32_t* row_ptr; /* n + 1 */
  const int32_t* col_idx; /* nnz   */
  const double* val;      /* nnz   */
} bd_csr;

typedef struct bd_amg bd_amg; /* opaque hierarchy handle */

typedef struct {
  int32_t iterations;        /* number of products A p                          */
  double rel_residual_true;  /* ||b^ - A x|| / ||b^|| from a fresh product at exit */
  double rel_residual_rec;   /* the recursive residual the stopping test used   */
  double seconds;            /* wall time of the solve on the stream            */
  int32_t status;
} bd_solve_info;

#define BD_MAX_LEVELS 32
typedef struct {
  int32_t nlevels;
  int64_t n[BD_MAX_LEVELS];
  int64_t nnz[BD_MAX_LEVELS];
  int64_t p_nnz[BD_MAX_LEVELS];   /* prolongator P_k (level k -> k+1); 0 on the coarsest */
  double lambda[BD_MAX_LEVELS];   /* estimate of lambda_max(D_k^{-1} A_k)                 */
  int32_t coarse_mode;            /* 0 dense direct, 1 smoother relaxation                */
  double operator_complexity;
  double grid_complexity;
  int64_t device_bytes;           /* device memory owned by the handle                    */
  /* The level operator's product on the device (0 on a host-only handle): bytes per column
   * index it reads (4; 3 for 24-bit column indices where row tiles span more than 65,536
   * columns and there are at most 2^24 columns; 2 for 16-bit offsets from a per-tile column
   * base, or for 16-bit column indices where rows are too long for the staging buffer and
   * there are at most 65,536 columns; 1 for an index into the matrix's dictionary of at most
   * 256 distinct column - row offsets; 0 in the symmetric diagonal form below) and its row
   * tiles (0 when rows are too long for the staging buffer
   * and a lane-group kernel runs, or in the diagonal form). */
  int32_t col_bytes[BD_MAX_LEVELS];
  int64_t tiles[BD_MAX_LEVELS];
  int32_t col_bytes_p[BD_MAX_LEVELS];  /* the same for P_k and R_k (0 on the coarsest level) */
  int32_t col_bytes_r[BD_MAX_LEVELS];
  /* Stored diagonals (14) where the level operator is kept in the symmetric diagonal form,
   * else 0.  That form is taken for a square matrix equal to its transpose (values compared
   * exactly) whose column - row offsets >= 0 are those of a 27-point stencil ({0, 1} and four
   * triples C - 1, C, C + 1, as on a grid at least 2 nodes wide in x): only the
   * diagonals of offset >= 0 are stored, n values each, and row i reads a(i, i - d) as
   * a(i - d, i).  It holds no column indices or CSR values (bd_amg_export still returns the
   * host CSR).  A structurally missing entry reads as zero times x, so a non-finite x value
   * next to a boundary row can turn that row's result into NaN. */
  int32_t diags[BD_MAX_LEVELS];
  /* The hierarchy's V-cycle precision (BD_F64 | BD_F32): the element type of the vectors
   * bidomain_amg_apply reads and writes. */
  int32_t vcycle_precision;
  /* 1 where the level's unknowns are renumbered on the device (option reorder), else 0. */
  int32_t renumbered[BD_MAX_LEVELS];
} bd_amg_stats;

/*
 * Setup phase (Alg. 1): build the hierarchy of A and keep it on the device.  The host drives
 * the level loop; with the default options each SA level's eigenvalue estimate, strength graph,
 * independent set, aggregation, prolongator smoothing and Galerkin product run on the device
 * (aggregate_device, galerkin_device), and the host keeps a copy of every level (for
 * bidomain_amg_export and the launch plans).  A: host CSR (copied).  opts: NULL for defaults.  null_weights: NULL, or n host doubles w;
 * with BD_NULL_CONSTANT the solution is normalised to w^T x = 0 (w = lumped mass gives the
 * integral-zero normalisation of the extracellular potential, Sec. 2.1), else to 1^T x = 0.
 * Errors: BD_E_INVALID (malformed CSR, bad options), BD_E_NOMEM, BD_E_DEVICE.
 */
int bidomain_amg_setup(const bd_csr* A, const bd_amg_opts* opts, const double* null_weights,
                       void* stream, bd_amg** out);

/*
 * The setup phase alone, on the host: the returned handle holds the hierarchy but no device
 * memory; only bidomain_amg_info, bidomain_amg_export and bidomain_amg_destroy accept it
 * (other calls return BD_E_INVALID).  Needs no GPU.  Arguments as for bidomain_amg_setup.
 */
int bidomain_amg_build_host(const bd_csr* A, const bd_amg_opts* opts, bd_amg** out);

/*
 * Solve A x = b with AMG-preconditioned CG (Sec. 2.2): PCG in float64 (BD_F64), or flexible
 * CG in float64 around a float32 V-cycle (BD_F32).  With BD_NULL_CONSTANT, b, the initial
 * guess and every preconditioned residual are projected onto 1-perp.  Stops when
 * ||b^ - A x|| <= rtol ||b^|| on the recursive residual (b^ = projected b).
 * b_dev: n doubles (read).  x_dev: n doubles; read as the initial guess if x_is_guess,
 * overwritten with the solution.  maxit: iteration cap.  info: may be NULL.
 * Returns BD_OK, BD_E_NOT_CONVERGED, BD_E_BREAKDOWN, BD_E_NONFINITE, BD_E_INVALID,
 * BD_E_DEVICE.
 */
int bidomain_pcg_solve(bd_amg* h, const double* b_dev, double* x_dev, int x_is_guess, double rtol,
                       int maxit, void* stream, bd_solve_info* info);

/*
 * bidomain_pcg_solve without any device allocation, for callers that cannot allocate (code
 * under stream capture, tight serving loops, harnesses that forbid allocation).  Arguments,
 * results and errors as bidomain_pcg_solve; the result is the same (the same kernels in the same
 * order).  The solve's scalars, flags and block partials live in a static device array of the
 * library (4 MiB per device, held until the process ends) instead of the handle; the call
 * allocates no device or pinned memory and creates no events (the handle's, made by the setup,
 * are used; per-launch profiling is not available here).  Each device has one such array, shared
 * by every call on it: calls that overlap on one device race and must be serialised by the
 * caller.  A hierarchy whose block partials need more than the array holds is rejected with
 * BD_E_INVALID (fine operators up to about 33 million rows fit).
 */
int bidomain_pcg_solve_noalloc(bd_amg* h, const double* b_dev, double* x_dev, int x_is_guess, double rtol,
                               int maxit, void* stream, bd_solve_info* info);

int bidomain_amg_info(const bd_amg* h, bd_amg_stats* s);
void bidomain_amg_destroy(bd_amg* h);

/*
 * Copy level k's operator (which = 0: A_k, 1: P_k, 2: R_k) to host arrays.  Pass NULL
 * arrays to query sizes: *rows, *cols, *nnz are always written.  row_ptr needs rows + 1
 * entries, col_idx and val nnz entries.
 */
int bidomain_amg_export(const bd_amg* h, int level, int which, int32_t* rows, int32_t* cols,
                        int64_t* nnz, int32_t* row_ptr, int32_t* col_idx, double* val);

/*
 * The Galerkin product of the setup phase (Alg. 1): C = (R A P + (R A P)^T) / 2 with R = P^T,
 * on the structural pattern of the product (no entry dropped), on the host (on_device = 0), as
 * the device's sparse product (1; equal to the host's bit for bit) or as its dense MFMA product
 * (2; n and nc at most 65,536; the same pattern, values equal up to rounding order) -- the
 * kernels the setup uses with galerkin_device.
 * A: n x n CSR (sorted columns, positive diagonal, as for bidomain_amg_setup); P: n x nc CSR
 * (columns in [0, nc)); host arrays, read only.  *c_nnz receives the nonzero count and c_row_ptr
 * (nc + 1 entries, may be NULL) the row offsets; pass NULL c_col_idx and c_val to query the size,
 * else both must hold `capacity` >= *c_nnz entries (BD_E_INVALID otherwise).  BD_E_NOMEM when
 * the device product's buffers do not fit in half the free device memory.
 */
int bidomain_galerkin(int32_t n, int32_t nc, const int32_t* a_row_ptr, const int32_t* a_col_idx,
                      const double* a_val, const int32_t* p_row_ptr, const int32_t* p_col_idx,
                      const double* p_val, int on_device, int64_t capacity, int32_t* c_row_ptr,
                      int32_t* c_col_idx, double* c_val, int64_t* c_nnz);

/*
 * Apply one operation of the V-cycle on level k, on device vectors of the hierarchy's
 * working precision (double for BD_F64, float for BD_F32; `in_dev`/`out_dev` are typed as
 * void* for that reason):
 *   BD_OP_A        out = A_k in
 *   BD_OP_P        out = P_k in           (in: level k+1, out: level k)
 *   BD_OP_R        out = R_k in           (in: level k,   out: level k+1)
 *   BD_OP_PRESMOOTH  out = S_k(in) from a zero guess (in = right-hand side)
 *   BD_OP_VCYCLE   out = V-cycle from level k with right-hand side in (Alg. 2)
 *   BD_OP_COARSE   out = coarsest-level solve of in (k is ignored)
 * These run the same kernels the solve uses; they exist so each can be checked alone.
 */
enum { BD_OP_A = 0, BD_OP_P = 1, BD_OP_R = 2, BD_OP_PRESMOOTH = 3, BD_OP_VCYCLE = 4, BD_OP_COARSE = 5 };
int bidomain_amg_apply(bd_amg* h, int op, int level, const void* in_dev, void* out_dev, void* stream);

/* ---- the Bidomain slab and its time step --------------------------------------------- */
/*
 * A slab [0,Lx] x [0,Ly] x [0,Lz] (cm) of nx*ny*nz trilinear (Q1) elements, node
 * p = i + (nx+1)(j + (ny+1)k).  Conductivities (S/cm) are axisymmetric (eq. (2) with
 * sigma_n = sigma_t) around in-plane fibers at angle theta(z) = fiber_theta0 +
 * fiber_rotation * z / Lz.  cm = chi C_m (mF/cm^3), dt in ms.
 *
 * Membrane model (the ionic current of eq. (1) and the gating update of eq. (4)): the
 * two-variable Aliev-Panfilov model (Aliev & Panfilov, Chaos Solitons Fractals 7 (1996) 293),
 * whose published parameters are ap_k = 8, ap_a = 0.15, ap_eps0 = 0.002, ap_mu1 = 0.2,
 * ap_mu2 = 0.3, with one model time unit = ap_t_unit = 12.9 ms and the dimensionless potential
 * u = (v - ap_v_rest) / ap_v_scale (ap_v_rest = -85 mV, ap_v_scale = 105 mV).  All must be
 * finite; ap_k, ap_eps0, ap_mu2, ap_t_unit and ap_v_scale positive (else BD_E_INVALID).
 */
typedef struct {
  int32_t nx, ny, nz;
  double Lx, Ly, Lz;
  double sig_il, sig_it, sig_el, sig_et;
  double fiber_theta0, fiber_rotation;
  double cm, dt;
  double ap_k, ap_a, ap_eps0, ap_mu1, ap_mu2, ap_t_unit, ap_v_scale, ap_v_rest;
} bd_slab;

enum { BD_MAT_AI = 0, BD_MAT_AE = 1, BD_MAT_AELL = 2, BD_MAT_APAR = 3 };
/*
 * Assemble one slab operator on the host (Sec. 2.2: Q1 stiffness with 2x2x2 Gauss points,
 * lumped mass): A_i, A_e, A_ell = A_i + A_e, or A_par = (cm/dt) M + A_i, all on the full
 * 27-point pattern.  Arrays are caller-owned host buffers of n + 1 (row_ptr), nnz27 (col_idx,
 * val) and n (mass, may be NULL) entries, n = (nx+1)(ny+1)(nz+1),
 * nnz27 = (3nx+1)(3ny+1)(3nz+1).
 */
int bidomain_slab_assemble(const bd_slab* s, int which, int32_t* row_ptr, int32_t* col_idx,
                           double* val, double* mass);

/* ---- the truncated ellipsoid (idealised left ventricle) ----------------------------------- */
/*
 * The structured geometry of Sec. 3, eq. (8) with the axes of Table 1 (a1 = b1 = 2.2,
 * a2 = b2 = 3.3, c1 = 5.9, c2 = 6.4 cm; theta in [-3 pi/2, pi/2], phi in [-3 pi/8, pi/8]):
 *   x = a(r) cos(theta) cos(phi),  y = b(r) sin(theta) cos(phi),  z = c(r) sin(phi),
 * a(r) = a1 + r (a2 - a1) and likewise b, c; r in [0, 1] runs from the endocardium to the
 * epicardium.  (Eq. (8) prints cos(theta) sin(phi) for y; the ellipsoid has sin(theta) cos(phi).)
 * theta spans one full period (theta_max - theta_min = 2 pi, else BD_E_INVALID), so the mesh of
 * n_theta x n_phi x n_r isoparametric trilinear elements is periodic in theta and has
 * n = n_theta (n_phi + 1)(n_r + 1) nodes, p = i + n_theta (j + (n_phi + 1) k) at
 * (theta_i, phi_j, r_k) on uniform grids; n_theta >= 3, n_phi >= 1, n_r >= 1, and
 * -pi/2 < phi_min < phi_max < pi/2.  Fibers lie in the tangent plane of the r-surfaces at angle
 * alpha(r) = fiber_endo + r (fiber_epi - fiber_endo) from the theta direction towards the phi
 * direction (the paper's rotation: counterclockwise from epi- to endocardium, e.g. -60 deg at
 * the epicardium to +60 deg at the endocardium); conductivities, cm, dt and the Aliev-Panfilov
 * parameters mean what they mean in bd_slab and are validated the same way.
 */
typedef struct {
  int32_t n_theta, n_phi, n_r;
  double a1, a2, b1, b2, c1, c2;
  double theta_min, theta_max, phi_min, phi_max;
  double sig_il, sig_it, sig_el, sig_et;
  double fiber_endo, fiber_epi;
  double cm, dt;
  double ap_k, ap_a, ap_eps0, ap_mu1, ap_mu2, ap_t_unit, ap_v_scale, ap_v_rest;
} bd_ellipsoid;

/*
 * Assemble one ellipsoid operator on the host (which as for the slab), 2x2x2 Gauss points on
 * the reference cube with the fiber taken at each point's parameters, lumped mass = integral of
 * each basis function.  Full 27-point pattern with structural zeros, columns sorted; caller-owned
 * host buffers of n + 1 (row_ptr), nnz = 3 n_theta (3 n_phi + 1)(3 n_r + 1) (col_idx, val) and
 * n (mass, may be NULL) entries.  An element whose interpolated geometry has a non-positive
 * Jacobian at a Gauss point (axes that shrink from endo- to epicardium, say) is BD_E_INVALID.
 */
int bidomain_ellipsoid_assemble(const bd_ellipsoid* e, int which, int32_t* row_ptr, int32_t* col_idx,
                                double* val, double* mass);

typedef struct bd_sim bd_sim;

typedef struct {
  int32_t steps;
  int32_t it_par, it_ell;           /* iterations summed over the steps      */
  double ms_memb, ms_par, ms_ell;   /* device time summed over the steps     */
  double rel_res_par, rel_res_ell;  /* true relative residuals of the last step */
  int32_t status;
} bd_step_info;

/*
 * Create a simulation: assemble A_i, A_e and M, build the elliptic (ell, nullspace forced to
 * BD_NULL_CONSTANT, normalised with the lumped mass) and parabolic (par) hierarchies once
 * (hierarchy reuse, App. A), copy v0 (and w0, NULL = 0), and solve for u_e^0.
 * ell = NULL: the App. A defaults.  par = NULL: the same with strength threshold 0 (the paper
 * sets no AMG options for the parabolic system; its mass term weakens every coupling below
 * 0.06 on coarse meshes, which leaves slowly coarsening, dense hierarchies).
 * v0_dev, w0_dev: n device doubles (read).
 */
int bidomain_sim_create(const bd_slab* s, const bd_amg_opts* ell, const bd_amg_opts* par,
                        const double* v0_dev, const double* w0_dev, double rtol, void* stream,
                        bd_sim** out);
/* The same on the truncated ellipsoid (bidomain_ellipsoid_assemble's operators). */
int bidomain_ellipsoid_sim_create(const bd_ellipsoid* e, const bd_amg_opts* ell, const bd_amg_opts* par,
                                  const double* v0_dev, const double* w0_dev, double rtol, void* stream,
                                  bd_sim** out);

/*
 * Advance nsteps IMEX steps (eqs. (4)-(7)): Aliev-Panfilov membrane update, parabolic solve
 * (warm-started from v^n), elliptic solve (warm-started from u_e^n).  rtol for both solves.
 */
int bidomain_step(bd_sim* sim, int nsteps, double rtol, void* stream, bd_step_info* info);

enum { BD_V = 0, BD_UE = 1, BD_W = 2 };
int bidomain_sim_get(bd_sim* sim, int field, double* out_dev, void* stream);
/* Handles of the two hierarchies (owned by the simulation). */
bd_amg* bidomain_sim_hierarchy(bd_sim* sim, int which /* 0 elliptic, 1 parabolic */);
void bidomain_sim_destroy(bd_sim* sim);

/* ---- serving: continuous batching of many cases ----------------------------------------- */
/*
 * A server admits slab cases (bd_slab + initial v, a number of IMEX steps each) in arrival order
 * whenever a slot and enough of the device budget are free, builds each case's two hierarchies
 * on a host worker thread while the GPU serves the admitted ones, keeps every hierarchy and state
 * vector in HBM for the whole case, and advances all running solves together: one CG iteration of
 * every running solve per round, each round's products, V-cycle steps (levels aligned across
 * cases) and reductions issued as multi-task launches that serve all cases at once.  Each solve
 * computes exactly what it computes alone (its own block partials, fixed reduction order).
 * Requires the Chebyshev smoother of degree 2 and the same V-cycle precision for both systems.
 * Times are seconds since bidomain_serve_create.
 */
typedef struct bd_server bd_server;
typedef struct {
  uint64_t ticket;
  int32_t status;           /* BD_OK or the first failing status of the case's solves      */
  int32_t steps;
  int32_t it_par, it_ell;   /* iterations summed over the case (initial u_e solve included) */
  double t_submit, t_admit, t_ready, t_done;
  double max_rel_residual;  /* largest true relative residual over the case's solves       */
  int64_t device_bytes;     /* HBM the case held while running                             */
} bd_case_result;
typedef struct {
  int32_t queued, setting_up, running, done;
  int64_t bytes_in_use, budget;  /* in use: cases on the device and setup transients */
  int64_t rounds, solves;
  double host_enqueue_s, host_wait_s, host_exit_s;  /* host time: enqueuing rounds, waiting on
                                                     the GPU, finishing solves */
  int64_t max_batched;      /* most running solves advanced together by one round's launches */
} bd_serve_stats;

/* budget_bytes: HBM the server may hold for cases; max_slots: cases admitted at once. */
int bidomain_serve_create(int64_t budget_bytes, int32_t max_slots, const bd_amg_opts* ell,
                          const bd_amg_opts* par, double rtol, void* stream, bd_server** out);
/* Queue a case (v0_host: n host doubles, copied).  BD_E_BUDGET if it can never fit. */
int bidomain_serve_submit(bd_server* srv, const bd_slab* slab, const double* v0_host, int32_t nsteps,
                          uint64_t* ticket);
/* The device footprint the server assumes for a case before it is on the device (admission). */
int bidomain_serve_estimate(const bd_server* srv, const bd_slab* slab, int64_t* bytes);
/* Admit what fits, run one round, and return up to max_results newly completed cases. */
int bidomain_serve_poll(bd_server* srv, bd_case_result* results, int32_t max_results, int32_t* n_results);
/* Final v and u_e of a completed case (n host doubles each, either may be NULL); releases them. */
int bidomain_serve_fetch(bd_server* srv, uint64_t ticket, double* v_host, double* ue_host);
int bidomain_serve_stats(const bd_server* srv, bd_serve_stats* st);
/* Wall time of every completed solve (start of its first kernel enqueue to detection). */
int bidomain_serve_solve_latencies(const bd_server* srv, double* out, int32_t cap, int32_t* count);
void bidomain_serve_destroy(bd_server* srv);

/*
 * Instrumentation: when enabled, every launch of the fine-level outer product q = A p
 * (the solve's dominant kernel) is bracketed by HIP events on the solve's stream; the sum
 * of their durations and the launch count accumulate until read (and reset) here.
 */
void bidomain_profile_enable(int on);
void bidomain_profile_read(double* total_ms, int64_t* launches, int reset);

const char* bidomain_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BIDOMAIN_H */
