// Launchers of the batched kernels (definitions in kernels_batch.hip).
//
// Batched layout: every instance's level-l P1 matrix is a uniform width-7
// SELL-C-64 block; the blocks of all instances present on level l are
// stacked (columns offset by the instance's row offset), so one launch covers
// every instance.  Instance row counts are multiples of 1024, so a 1024-row
// chunk (and a 64-row slice) never straddles two instances.  Per-slice masks
// select the instances an operation applies to on a level; per-slice
// instance ids look up per-instance scalars.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace chns {

constexpr int BCHUNK = 1024;  // rows per reduction chunk

struct BStencil {
  int nrows = 0;
  const int* col = nullptr;
  const int* sinst = nullptr;     // slice -> instance
  // slice -> (instance's level side, instance's first row): when given, the
  // kernels compute the P1 columns (periodic side x side block in neighbour
  // order) instead of reading col; only for levels without padding rows
  const int2* geo = nullptr;
  int rpt = 1;                    // rows per thread (1, 2, 4)
  int block = 256;                // workgroup size
};

// Modes: 0 SPMV (y = p0 A x + p1 y), 1 RESID (y = b - A x),
// 2 CHEB (d <- c1 d + c2 dinv (b - A x), y = x + d; per-instance c1/c2 when
// cc1/cc2 are given, else p0/p1), 3 CHEB0 (x = d = c2 dinv b).
// mask (per slice, may be null): rows of slices with mask 0 are skipped;
// act (per instance, may be null): rows of instances with act 0 are skipped.
template <typename T>
void bstencil(const BStencil& A, const T* val, int mode, const T* x, const T* b, const T* dinv,
              T* d, T p0, T p1, const T* cc1, const T* cc2, const uint8_t* mask, const int* act,
              T* y, hipStream_t s);

// General uniform-width SELL product with a per-slice mask of output rows and
// per-instance activity (sinst: slice -> instance of the output rows).
template <typename T>
void bspmv_uniform(int nrows, int width, const int* col, const T* val, const uint8_t* mask,
                   const int* sinst, const int* act, const T* x, T* y, T alpha, T beta,
                   hipStream_t s);

// Stacked CH block on [phi_all; mu_all]: per-instance c12, c22; act may be null.
template <typename T>
void bch_block(const BStencil& A, const T* L, const T* K, const T* M, const T* c12, const T* c22,
               const int* act, const T* x, T alpha, T beta, T* y, hipStream_t s);

// Precision conversion on chunks of active instances (cinst: chunk -> instance).
template <typename TI, typename TO>
void bconvert(int64_t n, const TI* x, TO* y, const int* cinst, const int* act, hipStream_t s);

// Right-hand sides with per-instance c_mu, c_ac.
void brhs_binary(const BStencil& A, const double* Mv, const double* phi, const double* Phi,
                 const double* c_mu, const double* c_ac, double* rhs_ch, double* rhs_ac,
                 hipStream_t s);

// Per-instance combine: out = a_i A + b_i B (coefficients per slice instance).
void bcombine(int64_t nslots, const int* sinst, const double* a, const double* A, const double* b,
              const double* B, double* out64, float* out32, hipStream_t s);

// ---------------------------------------------------------------- batched Krylov
// Block vectors of length n (multiple of BCHUNK); chunk c belongs to
// instance cinst[c].  Per-instance arrays are indexed [inst * stride + j].

// Chunks of instances with act 0 (act may be null) are skipped by the chunked
// kernels below; their partials and outputs keep stale values.

// Delayed classical Gram-Schmidt with reorthogonalisation (DCGS2) at Arnoldi
// step j, per instance: V_j (vt) holds the vector of this step orthogonalised
// once, V_{j+1} (w) the new vector.  Chunk partials of V_i.vt, V_i.w (i < j),
// vt.vt, vt.w, w.w go to part[slot * nchunk + c] (slots 2j + 3; chunks of
// inactive instances skipped).
// vs (may be null): V_j as stored times vs[inst] is the step's vector.
// group: basis vectors per launch (8 or 16; the autotuner picks it).
void bdcgs_dots(int64_t n, const double* V, int64_t ld, int j, double* part, const int* cinst,
                const int* act, const double* vs, hipStream_t s, int group = 16);
// red[i * rs + k] = slot k summed over instance i's chunks [cr[2i], cr[2i+1])
// and, when half != 0, the same range shifted by half; active instances only.
void bslot_reduce(int count, int nchunk, int nslots, const double* part, const int* cr, int half,
                  double* red, int rs, const int* act, hipStream_t s);
// Per instance: reorthogonalisation coefficients of V_j, correction of
// Hessenberg column j-1 (H per instance, (m+1) x m, column-major ld m+1) and
// projection coefficients of w, into coef[i * cstride ..].
void bdcgs_coef(int count, int j, int m, const double* red, int rs, double* H, double* coef, int cstride,
                const int* act, hipStream_t s);
// Per chunk: V_j <- its reorthogonalised, normalised form (j > 0), w <- w
// projected out of the final basis; chunk partials of |w|^2 into nrm_part.
// threads: workgroup size per 1024-row chunk (256, 512 or 1024; autotuned).
void bdcgs_update(int64_t n, double* V, int64_t ld, int j, const double* coef, int cstride,
                  double* nrm_part, const int* cinst, const int* act, const double* vs, hipStream_t s,
                  int threads = 256);
// Per active instance: h_{j+1,j} = |w|, final rotation of column j-1 into HR
// and g, provisional rotation of column j into HR and gp, iteration count,
// activity (estimate |gp_{j+1}| <= tol_i, |w| == 0 or non-finite: inactive with
// kcols = j + 1), inv = 1/|w| (0 for inactive instances).
void bdcgs_finish(int count, int nchunk, const double* part2, const int* cr, int half, int j, int m,
                  double* H, double* HR, double* cs, double* sn, double* g, double* gp, double* inv,
                  const double* tol, int* active, int* kcols, int* iters, hipStream_t s);
// y = double(x) * inv[inst] (inv may be null), on chunks of active instances.
void bconvert_out(int64_t n, const float* x, const double* inv, double* y, const int* cinst, const int* act,
                  hipStream_t s);
// v = w * inv[inst] (v may alias w).
void bscale(int64_t n, const double* w, const double* inv, const int* cinst, const int* act,
            double* v, hipStream_t s);
// Per instance: y = R^{-1} g on its kcols columns (rest 0).
void blsq(int count, int m, const double* H, const double* g, const int* kcols, double* y,
          hipStream_t s);
// x += Z y_inst over the instance's first kcols columns (the rest of Z is not read).
void bxupdate(int64_t n, const double* Z, int64_t ldz, int m, const double* y, double* x,
              const int* cinst, const int* kcols, hipStream_t s);
// Per-instance norms: part[c] = sum w^2 over chunk c; then norm_i, inv_i,
// g_i = [norm, 0..]; first: tol_i = max(rtol norm_i, atol), active_i = 1;
// else active_i = (norm_i > tol_i) and kcols_i = m.
void bnorm_partial(int64_t n, const double* w, double* part, hipStream_t s);
void bnorm_finish(int count, int nchunk, const double* part, const int* cr, int half, int m,
                  int first, double rtol, double atol, double* nrm, double* inv, double* g,
                  double* tol, int* active, int* kcols, hipStream_t s);

// Plain copy and fill kernels (kept out of runtime memset/memcpy so that a
// captured graph holds kernel nodes only).
void dcopy(int64_t n, const double* x, double* y, hipStream_t s);
void dfill_int(int64_t n, int v, int* x, hipStream_t s);

}  // namespace chns
