/*
 * chns.h -- C-ABI of the MI355X (gfx950) solver library for the linear systems
 * of one semi-implicit finite-element time step of the Cahn-Hilliard /
 * Allen-Cahn / Navier-Stokes drying model of arXiv 2501.11767
 * ("Preconditioning for a Cahn-Hilliard-Navier-Stokes model for morphology
 * formation in organic solar cells").
 *
 * Problem statement (paper, sections "Spatial & temporal discretization" and
 * "Iterative solvers and preconditioning"): a triangulation, the fields
 * phi_i^k, mu_i^k, Phi_v^k, v^k, p^k and the parameters go in; the step-(k+1)
 * fields come out.  Each step solves
 *   - per Cahn-Hilliard phase eq. (CH_linear):
 *       [[M + tau C, tau g K], [tau g K, -(tau g / beta) M]] [phi; mu]
 *         = [M phi^k; -(tau g / beta) f^k],
 *   - the Allen-Cahn system (M + tau delta_v K + tau C) Phi = M Phi^k - tau g_v f_v^k,
 *   - the Oseen saddle point eq. (linearnav) [[A, B^T], [B, 0]] [v; p] = [..; 0],
 * with FGMRES and the paper's block-diagonal preconditioners.
 *
 * Conventions shared by every entry point
 *   - Mesh: periodic square of side `length` (default 1), n cells per side
 *     (n even, 8 <= n <= 8192), each cell split along its (i,j)-(i+1,j+1)
 *     diagonal.  P1 node (i, j) has id i + n*j.  P2 velocity nodes: the n*n
 *     vertices, then the midpoints of horizontal, vertical and diagonal edges,
 *     each block numbered i + n*j; a velocity field is 2 * 4n^2 doubles, x
 *     components first.  Or the closed square [0, length]^2
 *     (CHNS_BOUNDARY_NOFLUX): the same cells, (n+1)^2 vertices numbered
 *     i + (n+1)*j, P1 fields of N = (n+1)^2 doubles; P2 ids in the same four
 *     blocks of N ids each numbered i + (n+1)*j (ids with i = n in the first
 *     and third edge block or j = n in the second and third name no edge), a
 *     velocity field 2 * 4N doubles.
 *   - Parameter reading: beta = eps^2, gamma = mobility, gamma_v = evap_rate,
 *     delta_v = evap_rate * eps^2, beta_v = eps^2, rho and alpha as given.
 *   - Every "d_" pointer is device memory owned by the caller, FP64 unless
 *     stated, contiguous, not aliased with another argument unless stated.
 *     Every "h_" pointer is host memory owned by the caller.
 *   - "stream" is a hipStream_t (NULL = the default stream).  Calls are
 *     asynchronous on that stream unless documented as synchronising.
 *   - The context owns all matrices, multigrid levels and Krylov workspace;
 *     it allocates device memory only in chns_create, through the caller's
 *     allocator when one is given.  A context is not thread-safe; use one
 *     context per stream.
 *   - Return values: CHNS_OK, the warning CHNS_WNOCONV (outputs written with
 *     the best iterate), or a negative error.  Invalid arguments are rejected
 *     with CHNS_EINVAL before anything is launched; chns_last_error() then
 *     describes the problem.
 */
#ifndef CHNS_H
#define CHNS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CHNS_API __attribute__((visibility("default")))

typedef struct chns_ctx chns_ctx;

enum {
  CHNS_OK = 0,
  CHNS_WNOCONV = 1,      /* tolerance not reached within maxiter: best iterate written */
  CHNS_EINVAL = -1,      /* invalid argument (shape, null pointer, NaN/Inf parameter) */
  CHNS_ENOMEM = -2,      /* device allocation failed in chns_create */
  CHNS_EHIP = -3,        /* a HIP runtime call failed */
  CHNS_ESTATE = -4,      /* call not valid in the context's current state */
  CHNS_EUNSUPPORTED = -5 /* operation not available for this model */
};

/* Models: which fields a step advances. */
enum {
  CHNS_MODEL_CH = 0,      /* one CH phase, double-well potential phi^2 (1-phi)^2 */
  CHNS_MODEL_CH_AC = 1,   /* one CH phase + vapour field, liquid/gas interpolated potential */
  CHNS_MODEL_TERNARY = 2, /* polymer + NFA CH phases (solvent = 1 - sum), vapour, Oseen */
  CHNS_MODEL_QUATERNARY = 3 /* the paper's full system: polymer, NFA, solvent CH phases with the
                               air eliminated (phi_a = 1 - sum, section "Numerical results"), the
                               fitted quartic of eq. (appPotential) with its air terms, a gradient
                               coefficient per phase (beta_phase), mu_a from eq. (airdisc),
                               vapour, Oseen with all four phases in the Korteweg force and the
                               convecting field */
};

/* Linear systems (blocks) of a step. */
enum { CHNS_BLOCK_CH = 0, CHNS_BLOCK_AC = 1, CHNS_BLOCK_NS = 2 };

/* Operators for chns_spmv / chns_get_matrix.  N is the P1 node count: n^2 on
 * the periodic square, (n+1)^2 on the closed one (CHNS_BOUNDARY_*); the sizes
 * below are written for the periodic square (n^2 = N). */
enum {
  CHNS_OP_M = 0,       /* P1 mass, n^2 x n^2 */
  CHNS_OP_K = 1,       /* P1 stiffness */
  CHNS_OP_C = 2,       /* P1 convection C(v^k) from the last chns_assemble */
  CHNS_OP_CH = 3,      /* CH 2x2 block operator on [phi; mu], 2n^2 x 2n^2 */
  CHNS_OP_AC = 4,      /* Allen-Cahn matrix M + tau delta_v K + tau C */
  CHNS_OP_X = 5,       /* matching factor tau g K + sqrt(tau g / beta) M */
  CHNS_OP_L = 6,       /* CH (1,1) block M + tau C */
  CHNS_OP_NS = 7,      /* Oseen saddle point on [v_x; v_y; p], 9n^2 x 9n^2 (ternary model) */
  CHNS_OP_VX = 8,      /* velocity block A_xx = (rho/tau) M + J(w) + K_sym,xx on P2, 4n^2 x 4n^2 */
  CHNS_OP_AP = 9       /* pressure convection-diffusion matrix (rho/tau) M + eta K + N(w), P1 */
};

/* Arithmetic of the preconditioner: all FP64, or FP32 multigrid inside an
 * FP64 flexible Krylov method (residuals, dots, Hessenberg in FP64). */
enum { CHNS_F64 = 0, CHNS_MIXED = 1 };

/* Domain boundary (section "Model", eq. (bc); section "Numerical results"
 * for the square of side 10). */
enum {
  CHNS_BOUNDARY_PERIODIC = 0, /* periodic square, n*n vertices i + n*j at (i h, j h) */
  CHNS_BOUNDARY_NOFLUX = 1    /* closed square [0, length]^2 with the natural (no-flux)
                                 conditions of the phase fields, chemical potentials and
                                 vapour field and the no-slip walls of the velocity: (n+1)^2
                                 vertices i + (n+1)*j at (i h, j h), 0 <= i, j <= n.  The
                                 Oseen operator holds the no-slip set (wall nodes and the ids
                                 of no edge) with identity rows no other row couples to and
                                 zero right-hand side rows; a convecting velocity given to
                                 chns_assemble must vanish there; the adjoint step's
                                 transposed Oseen solve holds it the same way */
};

typedef struct {
  int32_t n;        /* cells per side (even, 8..8192; 8..128 on the cube) */
  int32_t model;    /* CHNS_MODEL_* */
  int32_t boundary; /* CHNS_BOUNDARY_*; 0 = periodic */
  int32_t dim;      /* 2 (0 means 2): the square; 3: the cube [0, length]^3 (section
                       "Numerical results", three-dimensional runs), each cell split into
                       the six Kuhn tetrahedra along its main diagonal (P1 rows of 15
                       entries): periodic with n^3 vertices i + n j + n^2 k at (i h, j h,
                       k h), or with CHNS_BOUNDARY_NOFLUX closed with (n+1)^3 vertices
                       i + (n+1) j + (n+1)^2 k and the top-face flux (top_flux on the face
                       z = length, phi read at its centre); the binary models only, no
                       convecting velocity */
  double length;    /* side of the square or cube (h = length / n); 0 means 1 */
} chns_mesh;

/* Local free-energy density of the ternary model. */
enum {
  CHNS_POT_QUARTIC = 0,        /* the fitted quartic of eq. (appPotential), air = 0 */
  CHNS_POT_FLORY_HUGGINS = 1   /* Flory-Huggins liquid and ideal-gas densities (section "Free
                                  energy functional") with every phi ln phi replaced by its
                                  degree-4 Taylor polynomial about 1/2 (section "Numerical
                                  results"), air = 0 */
};

typedef struct {
  double eps;        /* interface parameter: beta = beta_v = eps^2 */
  double tau;        /* time step */
  double mobility;   /* gamma_i (all phases) */
  double evap_rate;  /* gamma_v; delta_v = evap_rate * eps^2 */
  double viscosity;  /* eta */
  double alpha;      /* alpha_i in the Oseen convecting field */
  double rho;        /* density (rho = 1 when all pure densities are 1) */
  /* ternary model only (else CHNS_POT_QUARTIC and truncate 0): */
  int32_t potential;     /* CHNS_POT_* */
  int32_t truncate;      /* 1: the density's terms are evaluated at the truncated fields
                            clip(phi, 0, 1) of eq. (truncateCH) (solvent: clip(1 - phi_p - phi_N)) */
  double fh_nsize[3];    /* Flory-Huggins molar sizes N_p, N_NFA, N_s (> 0) */
  double fh_chi[3];      /* interaction parameters chi_(p,NFA), chi_(p,s), chi_(NFA,s) */
  double fh_phisat[3];   /* saturated vapour fractions of p, NFA, s, in (0, 1] */
  /* ternary model only (else 0): */
  int32_t var_density;   /* 1: the Oseen step's density is the field rho^k = sum_i rho_pure[i]
                            phi_i^k of eq. (matrixns) (polymer, NFA, solvent phi_s = 1 - phi_p -
                            phi_N, air zero): the velocity mass int rho^k psi_m psi_n, the
                            convecting field the P2 interpolant of the nodal rho^k v^k, and the
                            PCD matrix's mass weighted alike; 0: the constant rho above */
  int32_t ns_picard;     /* Oseen solves per step (<= 1: one, the linear scheme): solve m convects
                            with the velocity of solve m - 1 (the outer iteration the remark on
                            Newton schemes after eq. (linearnav) implies); 1..100 */
  double rho_pure[3];    /* pure densities of polymer, NFA, solvent (> 0) when var_density */
  double ns_picard_tol;  /* stop the solves once ||v^(m) - v^(m-1)||_2 <= tol ||v^(m)||_2 (>= 0) */
  /* closed square only (CHNS_BOUNDARY_NOFLUX; else 0): evaporation at the top
     wall (eq. (bc), Hertz-Knudsen outflux): d phi / dn = j_out = top_flux *
     (phi^k(x_ref) - flux_inf) on y = length, x_ref the wall's midpoint (vertex
     n/2 + (n+1) n); it loads the mu equation (eq. (weakch)) with -beta j_out
     int_top w ds, i.e. the CH right-hand side's second block with
     + tau gamma j_out int_top phi_i ds.  top_flux lumps the flow rate, the
     square root and P_0 of the flux law into one finite coefficient. */
  double top_flux;
  double flux_inf;
  /* quaternary model only (else 0): the gradient coefficients beta_p, beta_N,
     beta_s, beta_a (each > 0) of the CH phases and of the eliminated air; the
     vapour field keeps beta_v = eps^2 and delta_v = evap_rate * eps^2.  Each
     CH solve forms its block with its phase's beta (the second row's
     -(tau g / beta_i) M and X = tau g K + sqrt(tau g / beta_i) M); between
     steps the CH operators hold the polymer's. */
  double beta_phase[4];
} chns_params;

typedef struct {
  double rtol, atol;    /* stop when ||b - A x||_2 <= max(rtol ||b||_2, atol) */
  int32_t restart;      /* FGMRES restart length m (1..64) */
  int32_t maxiter;      /* total Arnoldi steps allowed */
  int32_t precision;    /* CHNS_F64 or CHNS_MIXED */
  int32_t mg_cycles;    /* V-cycles per inner solve (>= 1) */
  int32_t mg_pre;       /* Chebyshev pre-smoothing steps (>= 1) */
  int32_t mg_post;      /* Chebyshev post-smoothing steps (>= 0) */
  int32_t mg_coarse;    /* Chebyshev steps on a coarse cut level (>= 1) */
  double mg_lmax;       /* upper bound of the spectrum of D^{-1}A (smoothing on [lmax/4, lmax]) */
  double mg_rho_cut;    /* cut the hierarchy at the first level with 8 b n_l^2 / a <= rho_cut */
} chns_solve_opts;

typedef struct {
  int32_t iters;      /* Arnoldi steps taken */
  int32_t restarts;   /* cycles started */
  int32_t converged;  /* 1 if the true residual met the tolerance */
  int32_t status;     /* CHNS_OK or CHNS_WNOCONV */
  double bnorm;       /* ||b||_2 */
  double res0;        /* ||b - A x0||_2 */
  double res_true;    /* ||b - A x||_2 of the returned iterate (recomputed) */
  double ms;          /* wall time of the solve in milliseconds (hipEvent) */
  int32_t passes;     /* Oseen solve with ns_picard > 1: solves made (iters, restarts and ms
                         summed over them, converged of all, the rest of the last); else 1 */
  double change;      /* the last solve's ||v^(m) - v^(m-1)||_2 / ||v^(m)||_2 (Oseen, else 0) */
} chns_solve_info;

/* Field set at one time level (device pointers; NULL where the model has no
 * such field).  phi[0], phi[1]: CH phases (n^2 each); mu[0..1] their chemical
 * potentials; mu[2] the eliminated solvent's potential (ternary); quaternary:
 * phi[0..2] polymer, NFA, solvent, mu[0..2] theirs and mu[3] the eliminated
 * air's; Phi_v: vapour field (n^2); vel: P2 velocity (2 * 4n^2); p: pressure
 * (n^2, mean zero). */
typedef struct {
  double* phi[3];
  double* mu[4];
  double* Phi_v;
  double* vel;
  double* p;
} chns_fields;

/* Defaults: rtol 1e-8, atol 0, restart 40, maxiter 600, F64, 1 V(2,2) cycle,
 * 8 coarse steps, lmax 2.1, rho_cut 0.25.
 *
 * The inner cycle for an operator A = a M + b K (+ c C): Galerkin levels
 * n, n/2, ... (nested P1 interpolation) down to the first level where
 * 8 b n_l^2 / a <= rho_cut or the last level (size >= 4); Chebyshev smoothing
 * of D^{-1}A on [lmax/4, lmax]; on the cut level Chebyshev steps on
 * [0.45 / (1 + 8 b n_l^2 / a), lmax] (mg_coarse of them on a coarse level,
 * mg_pre + mg_post when the operator is cut on the finest level). */
CHNS_API void chns_default_opts(chns_solve_opts* opts);

/* Device allocator supplied by the caller: alloc(bytes, alloc_ctx) returns
 * device memory aligned to at least 256 bytes, or NULL on failure;
 * free_(ptr, alloc_ctx) releases it.  A caching allocator (PyTorch's, for
 * example) may hand the memory out again as soon as free_ returns: the library
 * calls free_ only after synchronising the device. */
typedef void* (*chns_alloc_fn)(size_t bytes, void* alloc_ctx);
typedef void (*chns_free_fn)(void* ptr, void* alloc_ctx);

/* Set up a context for the discretisation of section "Spatial & temporal
 * discretization" (P1 phase fields, potentials and vapour field, Taylor-Hood
 * P2-P1 velocity and pressure on the triangulated box) with the parameters
 * of the nondimensional model (section "Nondimensionalized governing
 * equations", eq. (model)):
 * build the mesh tables, sparsity patterns (CSR -> SELL-C-sigma), multigrid
 * hierarchy and Krylov workspace, and assemble M and K on the device
 * (coloured element scatter).  Every device buffer of the context comes from
 * alloc (freed through free_ by chns_destroy); alloc and free_ both NULL
 * means hipMalloc / hipFree, exactly one of them NULL is CHNS_EINVAL.  A
 * 128-byte pinned host slot for the solver's residual read-back is the only
 * host allocation (hipHostMalloc).  No later call allocates device memory.
 * Synchronising.  *out is NULL on failure; CHNS_ENOMEM when alloc returns
 * NULL. */
CHNS_API int chns_create(const chns_mesh* mesh, const chns_params* params, chns_alloc_fn alloc,
                         chns_free_fn free_, void* alloc_ctx, chns_ctx** out);

/* Synchronise the device, then release every buffer of the context (through
 * the caller's free_ when chns_create was given an allocator). */
CHNS_API int chns_destroy(chns_ctx* ctx);

/* Replace the parameters and re-form every parameter-dependent operator
 * (on all multigrid levels).  Also forgets the solver's history: FGMRES
 * predicts from the mean residual reduction per step of the block's last
 * solve when the next residual estimate may meet the tolerance (and reads it
 * before enqueuing more work); after chns_set_params the first solve of each
 * block runs without that prediction.  Synchronising on return. */
CHNS_API int chns_set_params(chns_ctx* ctx, const chns_params* params);

/* Variable density (eq. (matrixns), ternary contexts with var_density): form
 * rho^k = sum_i rho_pure[i] phi_i^k from the device fields d_phi_p, d_phi_n
 * (N each; phi_s = 1 - phi_p - phi_N) and the density-weighted velocity and
 * pressure masses; the next chns_assemble convects with rho^k v.
 * chns_timestep calls it on its input state.  CHNS_EINVAL for other
 * contexts or NULL fields. */
CHNS_API int chns_set_density(chns_ctx* ctx, const double* d_phi_p, const double* d_phi_n, void* stream);

/* Per-step assembly (paper: C(v^k) of eq. (CH_linear); J(w^k) and the PCD
 * matrix A_p(w^k) for the Oseen step): coloured element scatter of the
 * convection matrix from the P2 velocity d_vel (NULL means v = 0; required
 * for the ternary model), Galerkin refresh of every coarse level, and
 * re-forming of the block values.  d_mu: for the ternary model the three
 * chemical potentials (polymer, NFA, solvent) entering the convecting field
 * w = rho v - alpha sum_i grad mu_i, for the quaternary model four (polymer,
 * NFA, solvent, air) (an entry or the array may be NULL for mu = 0); ignored
 * otherwise. */
CHNS_API int chns_assemble(chns_ctx* ctx, const double* d_vel, const double* const* d_mu,
                           void* stream);

/* Transposed operators (differentiation form, ternary model): assemble at the
 * state (d_vel, d_mu) exactly as chns_assemble, then replace each
 * state-dependent convection part by its transpose (C -> C^T in the CH and AC
 * blocks, J -> J^T in the Oseen velocity block, N_p -> N_p^T in the PCD
 * matrix; values moved to the slots of the transposed entries of the
 * symmetric patterns) before the coarse levels and block values are formed.
 * M, K, K_sym and the mass terms are symmetric and B enters the Oseen
 * operator as [[A, B^T], [B, 0]], so chns_spmv, chns_precond_apply and
 * chns_krylov_solve then act on the transposed systems with the transposed
 * block preconditioner: with mg_pre == mg_post each V-cycle on the transposed
 * matrix is the exact transpose of the forward one (same Chebyshev polynomial
 * before and after the Galerkin coarse correction, R = P^T), and the PCD
 * factors are applied in reverse order.  chns_assemble restores the forward
 * operators.  CHNS_EUNSUPPORTED for the binary models. */
CHNS_API int chns_assemble_transposed(chns_ctx* ctx, const double* d_vel, const double* const* d_mu,
                                      void* stream);

/* Shape of an assembled operator (host query, no device work). */
CHNS_API int chns_matrix_shape(chns_ctx* ctx, int32_t op, int64_t* nrows, int64_t* ncols,
                               int64_t* nnz);

/* Copy an assembled operator back as sorted CSR with explicit zeros kept:
 * h_rowptr[nrows+1], h_col[nnz], h_val[nnz] (any may be NULL to skip).
 * Synchronising. */
CHNS_API int chns_get_matrix(chns_ctx* ctx, int32_t op, int32_t* h_rowptr, int32_t* h_col,
                             double* h_val, void* stream);

/* y = alpha * op(A) x + beta * y for A in CHNS_OP_* (the matrices of section
 * "Iterative solvers and preconditioning": M, K, C(v^k) and the blocks of
 * eq. (CH_linear), the Allen-Cahn matrix, the matching factor X, and the
 * Oseen saddle point of eq. (linearnav)), op(A) = A for transpose == 0 and
 * A^T for transpose == 1.  The transposed product reads the transposed
 * operators that chns_assemble_transposed leaves in the context; operators
 * equal to their transpose in the current state (M, K, X always; C, L, AC and
 * the CH block when no velocity is assembled) accept either value, any other
 * mismatch between transpose and the context's orientation returns
 * CHNS_ESTATE.  precision CHNS_F64: x, y double; CHNS_MIXED: x, y float with
 * FP32 matrix values (not for CHNS_OP_NS).  x and y must not overlap.  With
 * beta == 0, y is not read. */
CHNS_API int chns_spmv(chns_ctx* ctx, int32_t op, int32_t precision, int32_t transpose, double alpha,
                       const void* d_x, double beta, void* d_y, void* stream);

/* z = P^{-1} r for a block (section "Iterative solvers and preconditioning":
 * CH diag(L, X M^{-1} X) with L ~ M + tau C and X = tau g K + sqrt(tau g /
 * beta) M, the matching approximation of eq. (schurCH); AC multigrid on its
 * matrix; NS diag(A^, M_p^{-1} A_p K_p^{-1}) with A^ = diag of the two
 * velocity component blocks and K_p^{-1} applied to mean-zero pressures).
 * Inner inverses are opts->mg_cycles geometric V-cycles in the precision
 * opts->precision (the velocity blocks start on their P2 level and continue
 * on the P1 levels); r and z are FP64 and must not overlap.  transpose == 1
 * applies the preconditioner built on the transposed operators of
 * chns_assemble_transposed, which is (P^{-1})^T when mg_pre == mg_post (each
 * V-cycle then the transpose of the forward one, the PCD factors in reverse
 * order); the orientation rule of chns_spmv applies (the CH and AC blocks
 * accept either value when no velocity is assembled). */
CHNS_API int chns_precond_apply(chns_ctx* ctx, int32_t block, int32_t transpose,
                                const chns_solve_opts* opts, const double* d_r, double* d_z,
                                void* stream);

/* Solve op(block) x = b (the systems of eq. (CH_linear), the Allen-Cahn
 * system and eq. (linearnav)) by right-preconditioned restarted FGMRES with
 * the block preconditioner of chns_precond_apply: Gram-Schmidt by delayed
 * classical Gram-Schmidt with reorthogonalisation (two passes over the basis
 * per step), Givens least squares on the device, stopping rule ||b - A x|| <=
 * max(rtol ||b||, atol) on the recomputed true residual (section "Numerical
 * results" states the same rule for its GMRES).  op and the orientation rule
 * as in chns_spmv.  d_x holds the initial guess and receives the solution.
 * Synchronising (the host reads the residual estimate once per Arnoldi
 * step).  h_info may be NULL.  For CHNS_BLOCK_NS the returned pressure is
 * projected to mean zero. */
CHNS_API int chns_krylov_solve(chns_ctx* ctx, int32_t block, int32_t transpose, const double* d_b,
                               double* d_x, const chns_solve_opts* opts, chns_solve_info* h_info,
                               void* stream);

/* Diagnostics of a field set, in FP64 on the GPU (synchronises the stream):
 * the discrete mass 1^T M u of every phase field and the discrete free energy
 * of the paper's functional (section "Free energy functional"; mass
 * conservation of the Cahn-Hilliard phases).  h_out[0]: 1^T M phi (binary) or
 * 1^T M phi_p (ternary, quaternary); h_out[1]: 1^T M phi_N (ternary,
 * quaternary, else 0); h_out[2]: 1^T M phi_s (quaternary; ternary: of the
 * eliminated solvent phi_s = 1 - phi_p - phi_N; else 0); h_out[3]: 1^T M Phi_v
 * (models with a vapour field, else 0);
 * h_out[4]: E_h = sum_i beta/2 phi_i^T K phi_i + sum_j (M 1)_j f(x_j), the
 * phases i of the model (ternary: polymer, NFA and solvent), f the model's
 * local density (binary: double-well, interpolated with the gas form by
 * p(Phi_v) when there is a vapour field; ternary: the fitted quartic with
 * air = 0; quaternary: eq. (appPotential) with the air eliminated and the
 * gradient sum over the four phases with beta_phase) at the nodal values,
 * beta = eps^2.  Fields: phi[0] (and phi[1] for the flow models, phi[2] for
 * the quaternary; Phi_v for models with a vapour field) are device
 * pointers of n^2 doubles; other members are ignored.  h_out: 5 doubles on
 * the host.  CHNS_EINVAL for a missing field or output. */
CHNS_API int chns_diagnostics(chns_ctx* ctx, const chns_fields* f, double* h_out, void* stream);

/* chns_diagnostics for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same results, bit for bit, from the same kernels, with the reduction's
 * per-block partials and results in a library-owned static device array of
 * 5 * 1025 doubles per GPU (held until the process ends) instead of the
 * context's workspace.  Allocates nothing (no hipMalloc, hipFree or allocating
 * library routine).  Every call on one GPU shares that GPU's array, which
 * keeps the last call's contents: calls that overlap on one GPU (several
 * streams, threads or contexts) race and must be serialised by the caller.
 * Must be called with the context's GPU current (CHNS_ESTATE otherwise);
 * CHNS_EINVAL for a reduction that would not fit the array (none does for n
 * <= 8192) and for a missing field or output.  Synchronises the stream. */
CHNS_API int chns_diagnostics_noalloc(chns_ctx* ctx, const chns_fields* f, double* h_out, void* stream);

/* Right-hand sides of one step from the level-k fields (paper: [M phi^k;
 * -(tau g/beta) f^k] per CH phase with f^k = M f'(phi^k) nodal, the AC
 * right-hand side, and for the ternary model (rho/tau) M v^k + F^k with the
 * Korteweg force F = int G : grad, G = beta sum_i grad phi_i (x) grad phi_i
 * + beta_v grad Phi (x) grad Phi over polymer, NFA and solvent, and zero
 * pressure rows; quaternary: beta_i per phase, the Korteweg sum over polymer,
 * NFA, solvent and air).  d_rhs_ch: 2n^2 per CH phase, phases consecutive
 * (quaternary: the second row of phase i scaled by -(tau g / beta_i));
 * d_rhs_ac: n^2 (required for models with a vapour field); d_rhs_ns: 9n^2
 * (required for the flow models). */
CHNS_API int chns_step_rhs(chns_ctx* ctx, const chns_fields* in, double* d_rhs_ch,
                           double* d_rhs_ac, double* d_rhs_ns, void* stream);

/* Advance nsteps steps of the semi-implicit scheme of section "Spatial &
 * temporal discretization" (linear terms implicit, potential terms explicit,
 * the Navier-Stokes convection lagged; every coupling at level k) from *in to
 * *out (both field sets complete for the model; in and out may be the same
 * set).  Per step: assemble C(v^k) (and J(w^k), A_p(w^k)), the right-hand
 * sides of chns_step_rhs, one FGMRES solve of eq. (CH_linear) per CH phase,
 * the AC solve, the Oseen solve of eq. (linearnav), and the closure of the
 * eliminated phase (section "Numerical results": the air for the quaternary
 * model, mu_a = f_a^k + beta_a M^{-1} K phi_a^{k+1}; the same procedure
 * applied to the solvent for the ternary model).  h_info (may be NULL)
 * receives one entry per solve, in the order CH phases, AC, NS, per step.
 * Synchronising. */
CHNS_API int chns_timestep(chns_ctx* ctx, const chns_fields* in, const chns_fields* out,
                           int32_t nsteps, const chns_solve_opts* opts,
                           chns_solve_info* h_info, void* stream);

/* Adjoint of one ternary step (differentiation form; the discrete adjoint of
 * the scheme of section "Spatial & temporal discretization").  in: the state
 * s^k; out: the state s^{k+1} that chns_timestep computes from it (the caller
 * recomputes it from a checkpoint); lam_out: the adjoint lambda^{k+1} = dL/ds^{k+1}
 * (phi[2], mu[3], Phi_v, vel; its pressure is ignored: the pressure enters no
 * later step); lam_in: receives lambda^k = (ds^{k+1}/ds^k)^T lambda^{k+1}
 * (pressure adjoint 0) and may coincide with lam_out; h_dtheta[3] +=
 * (ds^{k+1}/dtheta)^T lambda^{k+1} for theta = (eps, mobility, evaporation
 * rate), with beta = eps^2, delta_v = evap_rate eps^2 and Korteweg
 * coefficients eps^2.  The four transposed systems (CH for each phase, AC,
 * Oseen) are solved by FGMRES on the operators of chns_assemble_transposed at
 * s^k; h_info (4 entries, may be NULL) receives their reports.  The initial
 * state of a run is data (independent of theta).  Leaves the context holding
 * the transposed operators.  Returns CHNS_WNOCONV if a solve did not
 * converge; CHNS_EUNSUPPORTED for the binary and quaternary models and for
 * var_density or ns_picard > 1 (the reverse step covers the linear
 * constant-density ternary scheme).
 * Synchronising. */
CHNS_API int chns_timestep_adjoint(chns_ctx* ctx, const chns_fields* in, const chns_fields* out,
                                   const chns_fields* lam_out, const chns_fields* lam_in,
                                   double* h_dtheta, const chns_solve_opts* opts,
                                   chns_solve_info* h_info, void* stream);

/* Kernel classes of the measurement ledger. */
enum {
  CHNS_KERNEL_CHEB32 = 0,      /* FP32 Chebyshev sweep of the P1 stencil kernel (every level) */
  CHNS_KERNEL_CHEB64 = 1,      /* FP64 Chebyshev sweep of the P1 stencil kernel */
  CHNS_KERNEL_CH_BLOCK = 2,    /* FP64 CH block operator inside FGMRES */
  CHNS_KERNEL_DCGS_DOTS = 3,   /* Gram-Schmidt dot pass */
  CHNS_KERNEL_DCGS_UPDATE = 4, /* Gram-Schmidt update pass */
  CHNS_KERNEL_MG_FINE = 5      /* tiled multigrid passes on the finest level (down, up, steps from zero) */
};

/* Measurement ledger.  chns_ledger_start(kernel) clears the ledger and from
 * then on brackets every launch of that kernel class on this context by a
 * pair of HIP events recorded on the stream it is launched on, recording the
 * launch's algorithmic bytes (what the method must move: matrix values,
 * vectors read once, vectors written; computed indices excluded); -1 stops.
 * chns_ledger_read returns the launches, summed bytes and summed event time
 * in ms since the start (synchronising).  The events add a few microseconds
 * of host work per bracketed launch. */
CHNS_API int chns_ledger_start(chns_ctx* ctx, int32_t kernel);
CHNS_API int chns_ledger_read(chns_ctx* ctx, int64_t* launches, double* bytes, double* ms);

/* Message of the last error on this context (never NULL). */
CHNS_API const char* chns_last_error(const chns_ctx* ctx);

/* ---------------------------------------------------------------- batched form
 * Many independent instances of the CH + AC model (CHNS_MODEL_CH_AC, v = 0),
 * each with its own mesh size and parameters, advanced together: every stage
 * of a step (right-hand sides, operator products, multigrid sweeps, Krylov
 * reductions) is one launch covering all instances.  Fields are packed: the
 * nodes of instance i occupy [off[i], off[i+1]) of each field array
 * (off from chns_batch_offsets, off[i+1] - off[i] = n_i^2). */
typedef struct chns_batch chns_batch;

/* count instances of the CH + AC systems (eq. (CH_linear) and the Allen-Cahn
 * system of section "Iterative solvers and preconditioning", v = 0) with
 * sizes h_n[i] (multiples of 32 in 32..2048) and parameters h_params[i]
 * (read as in chns_create).  Device memory comes from alloc / free_ as in
 * chns_create (both NULL: hipMalloc / hipFree); no later call allocates.
 * Synchronising.  *out is NULL on failure. */
CHNS_API int chns_batch_create(int32_t count, const int32_t* h_n, const chns_params* h_params,
                               chns_alloc_fn alloc, chns_free_fn free_, void* alloc_ctx,
                               chns_batch** out);
/* Synchronise the device and release the batch's buffers and graphs. */
CHNS_API int chns_batch_destroy(chns_batch* b);
/* h_offsets[count + 1]: node offsets of the instances in the packed fields. */
CHNS_API int chns_batch_offsets(const chns_batch* b, int64_t* h_offsets);
/* Advance all instances nsteps steps (packed FP64 fields): the first step
 * reads in_*, every later step reads the previous step's output d_* (or
 * in_* again when each_from_input != 0, which repeats the first step's
 * systems); outputs go to d_*, which may equal in_* (in-place).  Each block
 * (the stacked CH blocks, then the stacked AC matrices) is solved by
 * right-preconditioned FGMRES with per-instance Krylov scalars on the device;
 * an instance freezes once its estimated residual meets its own tolerance and
 * every kernel then skips its rows.  opts->mg_cycles must be 1.
 * use_graph == 0 (eager): FGMRES(restart) up to maxiter Arnoldi steps, ending
 * as soon as every instance has converged (activity read back every few
 * steps).  use_graph != 0: each step variant (from in_*, from d_*) is captured
 * once on the given non-default stream into a hipGraph and replayed; the graph
 * runs a fixed budget B = min(maxiter, graph budget of the block) of Arnoldi
 * steps in cycles of min(restart, B) (chns_batch_set_graph_budget), so an
 * instance that needs more than B steps is reported as not converged.
 * Fails with CHNS_EUNSUPPORTED if one step's graph would exceed 100000 kernel
 * launches.  h_iters (2*count, may be NULL): Arnoldi steps of the last step,
 * CH then AC; h_conv (2*count, may be NULL): 1 where the recomputed true
 * residual met the tolerance; h_ms: device time of the nsteps steps (graph
 * capture excluded).  Returns CHNS_WNOCONV if any instance did not converge.
 * Synchronising. */
CHNS_API int chns_batch_timestep(chns_batch* b, const double* in_phi, const double* in_mu,
                                 const double* in_Phi, double* d_phi, double* d_mu, double* d_Phi,
                                 int32_t nsteps, int32_t each_from_input,
                                 const chns_solve_opts* opts, int32_t use_graph, int32_t* h_iters,
                                 int32_t* h_conv, double* h_ms, void* stream);
/* Autotuner (the batched form's launch shapes): time the batched smoothing
 * kernel on every level in rows-per-thread {1, 2, 4} x workgroup {128, 256,
 * 512, 1024}, the Gram-Schmidt update pass with 256, 512 or 1024 threads per
 * 1024-row chunk and the Gram-Schmidt dot pass with 8 or 16 basis vectors per
 * launch, on this batch's stacked sizes, and keep the fastest of each.
 * cache_path (may be NULL): a text file "gfx950" followed by "level rows rpt
 * block", "update rows threads" and "dots rows group" lines, read when
 * present (cached entries are not timed) and rewritten with the choices.
 * Changes the arithmetic order of the Gram-Schmidt reductions only.  Uses the
 * Krylov workspace: do not call it while a step runs.  Synchronising. */
CHNS_API int chns_batch_tune(chns_batch* b, const char* cache_path, void* stream);
/* Work-list form of the batched multigrid passes: with grid > 0 every
 * tiled pass (one per level and role) launches a fixed grid of at most `grid`
 * workgroups (at least 8) that take the tiles of all instances from per-XCD
 * atomic counters, instead of one workgroup per tile (grid 0, the default).
 * Same arithmetic, same results.  Synchronising when the form changes. */
CHNS_API int chns_batch_set_worklist(chns_batch* b, int32_t grid);
/* The Gram-Schmidt launch shapes in use: update-pass threads per chunk and
 * dot-pass vectors per launch (host outputs, either may be NULL). */
CHNS_API int chns_batch_tuned(const chns_batch* b, int32_t* h_update_threads, int32_t* h_dots_group);
/* Arnoldi-step budgets of the graph mode for the CH and the AC block (0: use
 * maxiter), typically the largest iteration counts of an eager step plus a
 * margin.  Changing them makes the next graph-mode call capture anew. */
CHNS_API int chns_batch_set_graph_budget(chns_batch* b, int32_t ch_iters, int32_t ac_iters);
/* One application of the batched block preconditioner (the paper's block
 * preconditioners with geometric multigrid, Sec. 3) of block CHNS_BLOCK_CH
 * (r, z: [phi_all; mu_all], 2 * off[count] doubles) or CHNS_BLOCK_AC (off[count]
 * doubles) to every instance: z = P^{-1} r with opts' multigrid settings and
 * precision, the same operator as the one inside chns_batch_timestep.  r and z
 * are device arrays and must not overlap.  Asynchronous on `stream`. */
CHNS_API int chns_batch_precond_apply(chns_batch* b, int32_t block, const double* d_r, double* d_z,
                                      const chns_solve_opts* opts, void* stream);
CHNS_API const char* chns_batch_last_error(const chns_batch* b);

#ifdef __cplusplus
}
#endif

#endif /* CHNS_H */
