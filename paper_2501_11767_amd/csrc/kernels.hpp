// Launchers of the gfx950 kernels (definitions in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace chns {

// Device view of a SELL-C-sigma pattern with C = 64 (one wavefront per slice).
struct DSell {
  int nrows = 0, nslices = 0, width = 0;  // width: slice width when uniform
  int uniform = 0;                        // all slices width `width`, identity permutation
  const int* slice_ptr = nullptr;
  const int* slice_w = nullptr;
  const int* col = nullptr;
  const int* perm = nullptr;              // lane position -> row (-1 padding)
  int side = 0;  // > 0: periodic side x side P1 pattern in neighbour order (columns computed)
  int cube = 0;  // > 0: periodic cube P1 pattern of this side in neighbour order (columns computed)
};

// Optional start/stop events taken by the dispatch itself (the kernel's own
// start and end timestamps), for the measurement ledger.
struct LaunchEv {
  hipEvent_t start = nullptr, stop = nullptr;
};

// Operator modes of the fused stencil kernel (uniform width-7 P1 patterns).
enum StencilMode { ST_SPMV = 0, ST_RESID = 1, ST_CHEB = 2 };

// Chebyshev step coefficients: step i updates d <- c1[i] d + c2[i] D^{-1}(b - A x),
// x <- x + d (c1[0] = 0).
constexpr int MAXCHEB = 64;
template <typename T>
struct ChebCoef {
  T c1[MAXCHEB];
  T c2[MAXCHEB];
  int steps;
};

// y = alpha A x + beta y on any SELL pattern (beta == 0: y not read).
template <typename T, typename TV>
void spmv(const DSell& A, const TV* val, const T* x, T* y, T alpha, T beta, hipStream_t s);

// Uniform P1 operators: mode ST_RESID: y = b - A x;
// ST_CHEB: d <- c1 d + c2 dinv (b - A x) (d not read when c1 == 0), y = x + d.
template <typename T, typename TV>
void stencil(const DSell& A, const TV* val, int mode, const T* x, const T* b, const T* dinv,
             T* d, T c1, T c2, T* y, hipStream_t s, LaunchEv ev = {});

// Fused steps on the periodic P1 levels (A.side > 0):
// cheb01: the first two Chebyshev steps from x = 0 (x0 = d0 = c20 dinv b formed on
//   the fly): d = c11 d0 + c21 dinv (b - A x0), y = x0 + d.
// pcheb: coarse-grid correction x' = x + P e (P1 interpolation from the side/2
//   mesh) with the first post-smoothing step: d = c2 dinv (b - A x'), y = x' + d.
template <typename T, typename TV>
void cheb01(const DSell& A, const TV* val, const T* b, const T* dinv, T c20, T c11, T c21, T* d, T* y,
            hipStream_t s);
template <typename T, typename TV>
void pcheb(const DSell& A, const TV* val, const T* x, const T* e, const T* b, const T* dinv, T c2, T* d,
           T* y, hipStream_t s);

// First Chebyshev step from x = 0: x = d = c2 dinv b.
template <typename T>
void cheb0(int n, const T* dinv, const T* b, T c2, T* d, T* x, hipStream_t s);

// Chebyshev steps from x = 0 in one workgroup (nrows <= 1024, uniform
// width-7 pattern), for the cut level of a cycle.
template <typename T, typename TV>
void coarse_cheb(const DSell& A, const TV* val, const T* dinv, const T* b, const ChebCoef<T>& cc,
                 T* x, hipStream_t s);

// The small levels of a V-cycle in one workgroup (periodic P1 levels only):
// levels 0..nlev-1 of `a` are consecutive levels of the hierarchy, the last one
// the cut level.  Each smoothing level takes `pre` Chebyshev steps from zero,
// restricts its residual (R = P^T), recurses, adds the P1 interpolation of the
// coarse iterate and takes `post` steps; the cut level takes coarse.steps steps
// from zero.  x = V b on the first level.  Every level's vectors live in LDS:
// tail_fits() says whether a chain of levels fits.
constexpr int TAIL_MAXLEV = 8;
constexpr int TAIL_MAXSM = 32;
constexpr int TAIL_THREADS = 1024;
template <typename T>
struct TailArgs {
  int inst;  // batched: the instance (activity check)
  int roff;  // batched: row offset of b and x in the launch's base vectors
  int nlev;
  int side[TAIL_MAXLEV];
  const T* val[TAIL_MAXLEV];
  const T* dinv[TAIL_MAXLEV];
  const T* b;
  T* x;
  int pre, post;
  T pre_c1[TAIL_MAXSM], pre_c2[TAIL_MAXSM];
  T post_c1[TAIL_MAXSM], post_c2[TAIL_MAXSM];
  ChebCoef<T> coarse;
};
// sides: the chain's level sides (each even side halves into the next).
template <typename T>
bool tail_fits(const int* sides, int nlev);
template <typename T>
void vtail(const TailArgs<T>& a, hipStream_t s);
// Batched: n workgroups, workgroup w runs list[idx[w]] (device arrays) with
// b = bbase + roff and x = xbase + roff (the entries' own b and x unused);
// tails of instances with act[inst] == 0 (act may be null) do nothing.
template <typename T>
void bvtail(int n, const TailArgs<T>* list, const int* idx, const int* act, const T* bbase, T* xbase,
            hipStream_t s);

// Tiled multigrid kernels on one periodic P1 level: one workgroup per square
// tile of the level's grid plus a halo of H rings, every dependent step of the
// level run in LDS (the halo is recomputed by both tiles that touch it).
//   TILE_ZERO: `steps` Chebyshev steps from x = 0 (H = steps - 1); x written.
//   TILE_DOWN: `steps` pre-smoothing steps from zero, the residual and its
//              restriction (H = steps + 1); x (pre-smoothed) and bc (coarse
//              right-hand side, side/2 grid) written.
//   TILE_UP:   x' = xin + P e (e on the side/2 grid), then `steps`
//              post-smoothing steps (H = steps); x written (x != xin).
// c1/c2: the Chebyshev coefficients of the steps (c1[0] unused).
//   TILE_UPM:  as TILE_UP over one more halo ring (H = steps + 1), then writes
//              M x (mval: the values of M, same pattern) instead of x.
enum TileMode { TILE_ZERO = 0, TILE_DOWN = 1, TILE_UP = 2, TILE_UPM = 3 };
constexpr int TILE_MAXSTEPS = 9;
template <typename T>
struct TileArgs {
  int side = 0, steps = 0;
  const T* val = nullptr;
  const T* dinv = nullptr;
  const T* b = nullptr;
  const T* xin = nullptr;
  const T* e = nullptr;
  T* x = nullptr;
  T* bc = nullptr;
  T c1[TILE_MAXSTEPS] = {};
  T c2[TILE_MAXSTEPS] = {};
  // FP64 boundary of an FP32 cycle: when b64 is given the right-hand side is
  // read from it (converted on load) instead of b; when x64 is given the
  // result goes there as FP64, multiplied by xs[0] when xs is given, instead
  // of into x
  const double* b64 = nullptr;
  double* x64 = nullptr;
  const double* xs = nullptr;
  const T* mval = nullptr;  // TILE_UPM: values of the matrix applied to the result
};
// Tile side of a level: float levels of side >= 1024 take 64 x 64 tiles
// (256 or more tiles), levels of side <= 256 take 16 x 16 tiles (256-thread
// workgroups), the others 32 x 32.
constexpr int TILE64_MIN_SIDE = 1024;
constexpr int TILE16_MAX_SIDE = 256;
template <typename T>
inline int tile_side(int side) {
  if (sizeof(T) == 4 && side >= TILE64_MIN_SIDE) return 64;
  return side <= TILE16_MAX_SIDE ? 16 : 32;
}
// Whether a level of this side takes the tiled kernel of `mode` with `steps`.
template <typename T>
bool tile_fits(int mode, int side, int steps);
template <typename T>
void vtile(int mode, const TileArgs<T>& a, hipStream_t s, LaunchEv ev = {});

// Two consecutive smoothing levels in one launch (32 x 32 fine tiles, the
// 16 x 16 coarse tile under each):
//   down2: pre-smoothing, residual and restriction on the fine level over a
//     halo of 3 pre + 3 rings, then on the coarse region it restricts to
//     (halo pre + 1); writes the fine and coarse pre-smoothed iterates (xf,
//     xc), the coarse right-hand side (bc) and that of the level below (bcc).
//   up2: coarse correction by e (level below) and post-smoothing on a coarse
//     region of halo (post + 1) / 2 + 1 + post, then the fine correction and
//     post-smoothing; writes the fine result xf.
// The rows computed are those of the level-by-level kernels (the halos
// recomputed by every tile that touches them).
template <typename T>
struct Tile2Args {
  int side = 0, steps = 0;  // fine side; pre (down2) or post (up2) steps
  const T* valf = nullptr;
  const T* dinvf = nullptr;
  const T* bf = nullptr;
  const T* xinf = nullptr;  // up2: fine pre-smoothed iterate
  T* xf = nullptr;
  const T* valc = nullptr;
  const T* dinvc = nullptr;
  T* bc = nullptr;          // down2 writes, up2 reads
  T* xc = nullptr;          // down2 writes, up2 reads (pre-smoothed coarse iterate)
  T* bcc = nullptr;         // down2: right-hand side of the level below
  const T* e = nullptr;     // up2: result of the level below
  T c1[TILE_MAXSTEPS] = {};
  T c2[TILE_MAXSTEPS] = {};
  // up2 with csteps > 0: the level below the pair is the cut level; every
  // workgroup takes its csteps Chebyshev steps from zero (coefficients cc1,
  // cc2; operator valcc, dinvcc; right-hand side bcc) itself on the region its
  // interpolation reads, and e is not read
  int csteps = 0;
  const T* valcc = nullptr;
  const T* dinvcc = nullptr;
  T cc1[TILE_MAXSTEPS] = {};
  T cc2[TILE_MAXSTEPS] = {};
};
// Whether two levels (fine side `side`) take the paired kernels with pre and
// post steps.
bool tile2_fits(int side, int pre, int post);
// Whether vup2 can solve the cut level below the pair (side / 4) itself with
// `steps` steps from zero.
bool tile2_cut_fits(int side, int post, int steps);
template <typename T>
void vdown2(const Tile2Args<T>& a, hipStream_t s);
template <typename T>
void vup2(const Tile2Args<T>& a, hipStream_t s);

// Batched tiled kernels (32 x 32 tiles): one workgroup per entry of a tile
// list; each entry names its instance, its tile, the instance's level side and
// its row offsets on the level (roff) and on the next coarser level (croff).
// Tiles of instances with act[inst] == 0 (act may be null) do nothing.
// Coefficients: c1/c2 for every instance, or per instance from cc1/cc2
// ([step * count + inst]) when those are given.
struct BTile {
  int inst, tile, side, roff, croff;
};
template <typename T>
struct BTileLaunch {
  const BTile* tiles = nullptr;
  const int* act = nullptr;
  int count = 0, steps = 0;
  const T* val = nullptr;
  const T* dinv = nullptr;
  const T* b = nullptr;
  const T* xin = nullptr;
  const T* e = nullptr;
  T* x = nullptr;
  T* bc = nullptr;
  T c1[TILE_MAXSTEPS] = {};
  T c2[TILE_MAXSTEPS] = {};
  const T* cc1 = nullptr;
  const T* cc2 = nullptr;
  // FP64 boundary (as in TileArgs), offset per instance like b and x; xs per
  // instance (xs[inst])
  const double* b64 = nullptr;
  double* x64 = nullptr;
  const double* xs = nullptr;
  const T* mval = nullptr;  // TILE_UPM (as in TileArgs), offset per instance like val
};
bool btile_fits(int mode, int side, int steps);
int btile_count(int side);  // tiles of one instance level
// wl_grid > 0 with wl_ctr (16 ints, zero between launches): the work-list
// form, a grid of at most wl_grid workgroups taking tiles from per-XCD
// atomic counters; else one workgroup per tile.
template <typename T>
void bvtile(int mode, int ntiles, const BTileLaunch<T>& a, hipStream_t s, int wl_grid = 0,
            int* wl_ctr = nullptr);

// CH block on [x1; x2] with value streams L = M + tau C, K, M (uniform P1):
//   y1 = alpha (L x1 + c12 K x2) + beta u1,  y2 = alpha (c12 K x1 + c22 M x2) + beta u2
// with u = yin when given (of the size of y, not overlapping it), else u = y.
template <typename T, typename TV>
void ch_block(const DSell& A, const TV* L, const TV* K, const TV* M, T c12, T c22, const T* x,
              T alpha, T beta, T* y, hipStream_t s, LaunchEv ev = {}, const T* yin = nullptr);

// Vector kernels.
template <typename T>
void axpby(int64_t n, T a, const T* x, T b, T* y, hipStream_t s);
template <typename TI, typename TO>
void convert(int64_t n, const TI* x, TO* y, hipStream_t s);
void scale_by_inv(int64_t n, const double* x, const double* inv, double* y, hipStream_t s);
// x <- x * inv[0] in place and y = float(x) (input stage of an FP32 preconditioner).
void convert_scaled(int64_t n, double* x, const double* inv, float* y, hipStream_t s);
// y = double(x) * inv[0] (inv may be null) (output stage of an FP32 preconditioner).
void convert_out(int64_t n, const float* x, const double* inv, double* y, hipStream_t s);

// Krylov reductions (FP64).  Partial sums per workgroup go to `part`
// (reduce_blocks(n) * cols doubles); reduce_* finish them deterministically.
int reduce_blocks(int64_t n);
// Delayed classical Gram-Schmidt with reorthogonalisation (DCGS2) at Arnoldi
// step j, basis V (columns of length n, stride ld): V_j holds the vector used
// for this step (orthogonalised once), V_{j+1} the new vector w = A z_j.
// dots: partials of V_i . V_j, V_i . w (i < j), V_j . V_j, V_j . w, w . w
// (2j + 3 slots of dcgs_dot_blocks(n) partials).
int dcgs_dot_blocks(int64_t n);
// Device state of one FGMRES cycle used by the two passes: slot partials
// (2j + 3 slots of dcgs_dot_blocks(n)) and their sums, |w|^2 partials
// (reduce_blocks(n)), raw Hessenberg H and its rotated form HR (ld m + 1),
// rotations, g, gp, coefficients and scal.
struct DcgsState {
  double *part = nullptr, *red = nullptr, *nrm_part = nullptr;
  double *H = nullptr, *HR = nullptr, *cs = nullptr, *sn = nullptr;
  double *g = nullptr, *gp = nullptr, *scal = nullptr;
  // V_j as stored times vscale[0] is the step's vector (may be null: 1); the
  // passes scale it on load and the update pass stores it normalised
  const double* vscale = nullptr;
  int m = 0;
};
// Dot pass and slot sums (into red: V_i . v_j, V_i . w for i < j, then
// v_j . v_j, v_j . w, w . w); the update pass forms the coefficients.
void dcgs_dots(int64_t n, const double* V, int64_t ld, int j, const DcgsState& st, hipStream_t s,
               LaunchEv ev = {});
// The CH block operator (as ch_block with alpha = 1, beta = 0; L == M
// selects the convection-free form) applied to z into V_{j+1} and the dot pass
// of step j in one launch, then the slot sums as dcgs_dots;
// for j with ch_dots_fits(j) (j < 16).
bool ch_dots_fits(int j);
void ch_dcgs_dots(const DSell& A, const double* Lv, const double* Kv, const double* Mv, double c12, double c22,
                  const double* z, double* V, int64_t ld, int j, const DcgsState& st, hipStream_t s,
                  LaunchEv ev = {});
// Update pass: the reorthogonalisation coefficients of V_j and the projection
// coefficients of w from the slot sums (and the correction of Hessenberg
// column j-1 and column j of H); V_j <- its reorthogonalised, normalised form
// (j > 0), w <- w projected out of the final basis; then one workgroup sets
// h_{j+1,j} = |w|,
// takes the final Givens rotation of column j-1 into HR and g, a provisional
// rotation of column j into HR and gp, and scal = (|gp_{j+1}|, 1/|w|, |w|)
// (also into pinned host memory `host` when given, followed, behind a
// system-scope fence, by host[3] = tag; w itself is not scaled).
void dcgs_update(int64_t n, double* V, int64_t ld, int j, const DcgsState& st, double* host, double tag,
                 hipStream_t s, LaunchEv ev = {});
// Least squares back-substitution for k columns: y = R^{-1} g.
void lsq_solve(int k, int m, const double* H, const double* g, double* y, hipStream_t s);
// x += Z y (k columns).
void xupdate(int64_t n, const double* Z, int64_t ldz, int k, const double* y, double* x,
             hipStream_t s);
// ||w||: partials then scal[0..2] = (norm, 1/norm (0 if norm == 0), norm),
// g = [norm, 0...] when given; the three values also into pinned host memory
// `host` when given, then, behind a system-scope fence, host[3] = tag.
void norm_partial(int64_t n, const double* w, double* part, hipStream_t s);
void norm_finish(int nblk, const double* part, double* scal, double* g, int m, hipStream_t s,
                 double* host = nullptr, double tag = 0.0);

// Assembly: coloured element scatter into a SELL value array.  kind 0: P1
// mass, 1: P1 stiffness, 2: P1 convection by a P2 velocity vel (2 x n2 nodes),
// 3: P1 mass weighted by the vertex field rho (int rho phi_i phi_j, exact).
void assemble_p1(int kind, int e0, int e1, const int* ep2, const int* etype, const int* eslot,
                 double h, const double* vel, int64_t n2, double* val, hipStream_t s,
                 const double* rho = nullptr);

// P1 on the periodic Kuhn tetrahedral mesh, one colour [e0, e1): kind 0 mass
// (|T| (1 + delta_ab) / 20), 1 stiffness; eslot16: 16 SELL slots per element.
void assemble_p1_tet(int kind, int e0, int e1, const int* etype, const int* eslot16, double h, double* val,
                     hipStream_t s);

// coarse[s] = sum_k w_k fine[src_k] over the Galerkin map.
void galerkin(int64_t nslots, const int* ptr, const int* src, const double* w, const double* fine,
              double* coarse, hipStream_t s);
// out = a A + b B + c C (C may be null) with FP32 copy; dinv from diagonal slots.
void combine(int64_t nslots, double a, const double* A, double b, const double* B, double c,
             const double* C, double* out64, float* out32, hipStream_t s);
// The three preconditioner operators of every P1 level in one launch.
// Operator o of a level: values a[o] M (+ b[o] K if useK[o]) (+ c[o] C if
// useC[o] and conv) on every SELL slot, FP64 and FP32, and 1/diagonal (0 where
// the diagonal is 0) in both precisions; work items of level l are
// [begin, begin + ns + N): first the slots, then the rows.
struct FormLevel {
  int64_t begin = 0, ns = 0;
  int N = 0;
  const int* diag = nullptr;
  const double *M = nullptr, *K = nullptr, *C = nullptr;
  double* v64[3] = {};
  float* v32[3] = {};
  double* d64[3] = {};
  float* d32[3] = {};
};
struct FormCoef {
  double a[3], b[3], c[3];
  int useK[3], useC[3];
};
void form_ops(int nlev, const FormLevel* tab, int64_t total, const FormCoef& k, bool conv, hipStream_t s);
void diag_inverse(int nrows, const int* diag, const double* val, double* d64, float* d32,
                  hipStream_t s);

// Right-hand sides of the binary models (uniform P1 pattern of M):
// rhs_ch = [M phi; -(tau g/beta) M f'(phi, Phi)], rhs_ac = M Phi - tau g_v M f_v(phi, Phi).
// Phi == nullptr selects the pure double-well (no vapour field).
// Masses and discrete energy of a field set on the finest P1 level (uniform
// width-7 pattern; M and K values): out[0..4] as chns_diagnostics documents,
// through per-block partials (part: 5 x reduce_blocks(n)) and one summing
// workgroup.  p1 (ternary second phase) and Phi may be null.
// Coefficients of the ternary density (definitions with the device
// functions in device_util.hpp): fh = 0 the fitted quartic, 1 Flory-Huggins;
// trunc: evaluate at the truncated fields.
struct PotCoef {
  int fh = 0, trunc = 0;
  double t4[5] = {0, 0, 0, 0, 0};  // Taylor coefficients of x ln x about 1/2
  double invN[3] = {1, 1, 1};
  double chi[3] = {0, 0, 0};       // (p, n), (p, s), (n, s)
  double lsat[3] = {0, 0, 0};      // ln phi_sat
};
// Gradient coefficients of the phases (in the order of the fields given, the
// eliminated phase last) and of the vapour field.
struct KorBeta {
  double b[4];
  double bv;
};

// Three per-phase scalars passed by value.
struct Coef3 {
  double v[3];
};

constexpr int NDIAG = 5;
int diag_part_blocks(int64_t n);  // per-block partial sums diagnostics() writes per quantity
// [mass p0, mass p1, mass of the third phase (p2, or 1 - p0 - p1 when p2 is
// null), mass Phi, energy]; the energy's gradient part sums kb.b[i]/2 u_i^T K u_i
// over p0, p1, p2 (if given) and the eliminated phase, in that order.
void diagnostics(const DSell& A, const double* M, const double* K, const double* p0, const double* p1,
                 const double* p2, const double* Phi, bool ternary, const KorBeta& kb, const PotCoef& pc,
                 double* part, double* out, hipStream_t s);
// a[idx[i]] = v (and a32[idx[i]] when a32 is given), i < n.
void set_slots(int64_t n, const int* idx, double v, double* a, float* a32, hipStream_t s);
// Quaternary right-hand sides (polymer, NFA, solvent; air eliminated):
// rhs_ch holds three CH blocks [M phi_i; c_mu[i] M d_i] of 2n each, rhs_ac the
// AC block, fa the unreduced air derivative per vertex.
void rhs_quaternary(const DSell& A, const double* Mv, const double* php, const double* phn, const double* phs,
                    const double* Phi, const Coef3& c_mu, double c_ac, double* rhs_ch, double* rhs_ac,
                    double* fa, hipStream_t s);
// Evaporation load of the closed square's top wall or the closed cube's top
// face: rows top0 .. nrows-1 (the vertices on y = length, resp. z = length)
// gain coef * (phi[ref] - phi_inf) * w_i in the CH right-hand side's second
// block, w_i = int_top phi_i: w[i - top0] when w is given (the cube), else h
// (h/2 at the corners; the square).  coef = 0: no load.
struct TopFlux {
  double coef = 0.0, phi_inf = 0.0, h = 0.0;
  int top0 = 0, ref = 0;
  const double* w = nullptr;
};
void rhs_binary(const DSell& A, const double* Mv, const double* phi, const double* Phi,
                double c_mu, double c_ac, const TopFlux& tf, double* rhs_ch, double* rhs_ac, hipStream_t s);

// Library-owned device scratch of the allocation-free diagnostics entry
// point: a file-scope device array (one copy per GPU) of STATIC_SCRATCH
// doubles, the per-block partials (NDIAG x at most 1024 blocks) and the NDIAG
// results.  static_scratch_init() resolves the array's device address on the
// current device once and caches it; static_scratch(device) returns the
// cached address (null before the init on that device).
constexpr int64_t STATIC_SCRATCH = int64_t(NDIAG) * (1024 + 1);
hipError_t static_scratch_init();
double* static_scratch(int device);

// ------------------------------------------------------------ Taylor-Hood / ternary

// General SELL operator forms (any pattern): ST_RESID and ST_CHEB as in stencil().
template <typename T, typename TV>
void sell_op(const DSell& A, const TV* val, int mode, const T* x, const T* b, const T* dinv, T* d,
             T c1, T c2, T* y, hipStream_t s);

// Device copy of the exact P2 reference tables (see host_mesh.hpp).
struct DP2Tables {
  const double* MM;   // [6][6]
  const double* S;    // [6][3][6][3]
  const double* T3;   // [6][6][6][3]
  const double* T2;   // [6][6][3]
  const double* TB;   // [3][6][3]
  const double* TI;   // [6][3]
  const double* MW;   // [3][6][6]
};

// Per-element gradient sources for the constant part of the convecting field
// w = rho v - alpha sum_i grad mu_i (mu: up to 4 P1 fields, each may be null).
struct MuGrad {
  const double* mu[4];
  double alpha;
};

// P2 element scatter (one colour [e0, e1)).  kind 0: mass into out[0];
// kind 1: symmetric-gradient blocks eta (2G^xx + G^yy), eta G^yx, eta G^xy,
// eta (G^xx + 2G^yy) into out[0..3]; kind 2: convection by w = wscale * vel
// (rho * vel at the P2 nodes when rho, a P2 field, is given) + w_const(mu)
// into out[0]; kind 3: mass weighted by the vertex field rho (int rho psi_i
// psi_j, exact) into out[0].  eslot36: 36 P2 SELL slots per element.
void assemble_p2(int kind, int e0, int e1, const int* ep1, const int* ep2, const int* etype,
                 const int* eslot36, double h, DP2Tables tb, double eta, const double* vel,
                 double wscale, int64_t n2, MuGrad mg, double* const* out, hipStream_t s,
                 const double* rho = nullptr);
// B_e[q][c,k] = -int d_c psi_k lambda_q into the B SELL (36 slots per element).
void assemble_b(int e0, int e1, const int* etype, const int* eslotb, double h, DP2Tables tb,
                double* out, hipStream_t s);
// P1 convection by w = wscale * vel + w_const(mu) (kind-2 P1 assembly with a
// constant part), into a P1 SELL value array.
void assemble_p1_conv(int e0, int e1, const int* ep1, const int* ep2, const int* etype,
                      const int* eslot, double h, const double* vel, double wscale, int64_t n2,
                      MuGrad mg, double* val, hipStream_t s, const double* rho = nullptr);
// (rho: the P2 nodal field that replaces wscale in w = rho v - alpha sum grad mu)
// Variable density: rho1 = sum_i rpure[i] phi_i at the vertices (phi_s = 1 -
// phi_p - phi_n), rho2 its P1 interpolant at the P2 nodes (4N; box: the
// closed square's padded numbering, 0 at the ids of no edge).
void density_fields(int n, bool box, const double* pp, const double* pn, const double* rpure, double* rho1,
                    double* rho2, hipStream_t s);
void fill(int64_t n, double v, double* out, hipStream_t s);
// out[0] = ||v - w||_2, out[1] = ||v||_2; part holds 2 * 256 partial sums.
void diff_norms(int64_t n, const double* v, const double* w, double* part, double* out, hipStream_t s);
// Korteweg load F_(c,k) += int G : grad(psi_k e_c), G = sum_i b_i grad phi_i
// (x) grad phi_i over the given phases (phi_p, phi_N and, when phs is not
// null, phi_s) and the eliminated one (one minus their sum: the solvent, or
// the air when the solvent is given), coefficients kb.b in that order, plus
// kb.bv grad Phi (x) grad Phi; out has 2 x n2 entries.
void korteweg(int e0, int e1, const int* ep1, const int* ep2, const int* etype, double h,
              DP2Tables tb, const double* php, const double* phn, const double* phs, const double* Phi,
              const KorBeta& kb, int64_t n2, double* out, hipStream_t s);

// Oseen operator values from the streams: kind 0 cm Mv + J + Kxx, 1 Kxy,
// 2 Kyx, 3 cm Mv + J + Kyy (src: P2 slot), 4 B (src: B slot), -1 zero.
void form_ns(int64_t nslots, const int8_t* kind, const int* src, double cm, const double* Mv,
             const double* J, const double* Kxx, const double* Kxy, const double* Kyx,
             const double* Kyy, const double* B, double* out, hipStream_t s);

// Right-hand sides of the ternary model (fitted quartic, air = 0, solvent
// eliminated), P1 pattern of M: rhs_p = [M phi_p; c_mu M f'_p], rhs_n likewise,
// rhs_ac = M Phi + c_ac M f_v; fs = d f / d phi_s at the nodes (for the closure).
void rhs_ternary(const DSell& A, const double* Mv, const double* php, const double* phn,
                 const double* Phi, double c_mu, double c_ac, const PotCoef& pc, double* rhs_p, double* rhs_n,
                 double* rhs_ac, double* fs, hipStream_t s);

// Mean-zero projection: partial sums (double) then x -= sum / n.
template <typename T>
void sum_partial(int64_t n, const T* x, double* part, hipStream_t s);
template <typename T>
void sub_mean(int64_t n, int nblk, const double* part, T* x, hipStream_t s, double total = 0.0);
// x -= (sum_i w_i x_i) / wtotal (the mean with weights w; wtotal = sum_i w_i).
void wmean_zero(int64_t n, const double* w, double wtotal, double* x, double* part, hipStream_t s);

// Elementwise helpers of the ternary closure.
void one_minus_sum(int64_t n, const double* a, const double* b, double* out, hipStream_t s);
void axpy_into(int64_t n, double a, const double* x, const double* y, double* out, hipStream_t s);

}  // namespace chns
