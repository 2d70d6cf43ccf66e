// C-ABI entry points of chns.h: context set-up, assembly, operators,
// block preconditioners, flexible GMRES and the time step.
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <cstring>
#include <string>
#include <type_traits>
#include <utility>

#include "context.hpp"

using namespace chns;

namespace {

#define HIPCHK(ctx, expr)                                                      \
  do {                                                                         \
    hipError_t e_ = (expr);                                                    \
    if (e_ != hipSuccess) {                                                    \
      (ctx)->err = std::string(#expr) + ": " + hipGetErrorString(e_);          \
      return CHNS_EHIP;                                                        \
    }                                                                          \
  } while (0)

#define TRY(expr)              \
  do {                         \
    int rc_ = (expr);          \
    if (rc_ < 0) return rc_;   \
  } while (0)

thread_local std::string g_create_err;

int fail(chns_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

template <typename T>
int dalloc(chns_ctx* c, T** p, size_t n) {
  *p = nullptr;
  if (n == 0) return CHNS_OK;
  void* q = nullptr;
  hipError_t e = hipMalloc(&q, n * sizeof(T));
  if (e != hipSuccess) {
    c->err = std::string("hipMalloc: ") + hipGetErrorString(e);
    return CHNS_ENOMEM;
  }
  c->allocs.push_back(q);
  *p = static_cast<T*>(q);
  return CHNS_OK;
}

template <typename T>
int upload(chns_ctx* c, T** p, const std::vector<T>& h) {
  TRY(dalloc(c, p, h.size()));
  if (!h.empty()) HIPCHK(c, hipMemcpy(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return CHNS_OK;
}

int upload_sell(chns_ctx* c, const Sell& S, DSell& d) {
  d.nrows = S.nrows;
  d.nslices = S.nslices;
  d.width = S.width_max;
  d.uniform = S.uniform ? 1 : 0;
  int *sp, *sw, *col, *perm;
  TRY(upload(c, &sp, S.slice_ptr));
  TRY(upload(c, &sw, S.slice_w));
  TRY(upload(c, &col, S.col));
  TRY(upload(c, &perm, S.perm));
  d.slice_ptr = sp;
  d.slice_w = sw;
  d.col = col;
  d.perm = perm;
  return CHNS_OK;
}

bool is_finite(double v) { return std::isfinite(v); }

int check_params(chns_ctx* c, const chns_params* p) {
  if (!p) return fail(c, CHNS_EINVAL, "params is NULL");
  const double v[] = {p->eps, p->tau, p->mobility, p->evap_rate, p->viscosity, p->alpha, p->rho};
  for (double x : v)
    if (!is_finite(x)) return fail(c, CHNS_EINVAL, "parameter is NaN or Inf");
  if (p->eps <= 0 || p->tau <= 0 || p->mobility <= 0)
    return fail(c, CHNS_EINVAL, "eps, tau and mobility must be positive");
  if (p->evap_rate < 0 || p->viscosity <= 0 || p->rho <= 0)
    return fail(c, CHNS_EINVAL, "evap_rate must be >= 0, viscosity and rho > 0");
  return CHNS_OK;
}

int check_opts(chns_ctx* c, const chns_solve_opts* o) {
  if (!o) return fail(c, CHNS_EINVAL, "opts is NULL");
  if (!is_finite(o->rtol) || !is_finite(o->atol) || o->rtol < 0 || o->atol < 0)
    return fail(c, CHNS_EINVAL, "rtol/atol must be finite and >= 0");
  if (o->restart < 1 || o->restart > MAX_RESTART)
    return fail(c, CHNS_EINVAL, "restart must be in 1..64");
  if (o->maxiter < 1) return fail(c, CHNS_EINVAL, "maxiter must be >= 1");
  if (o->precision != CHNS_F64 && o->precision != CHNS_MIXED)
    return fail(c, CHNS_EINVAL, "unknown precision");
  if (o->mg_cycles < 1 || o->mg_pre < 1 || o->mg_post < 0 || o->mg_coarse < 1 || o->mg_cycles > 64 ||
      o->mg_pre > 32 || o->mg_post > 32 || o->mg_coarse > MAXCHEB)
    return fail(c, CHNS_EINVAL, "multigrid step counts out of range (pre 1..32, post 0..32, coarse 1..64)");
  if (!(o->mg_lmax > 0.0 && o->mg_lmax < 100.0)) return fail(c, CHNS_EINVAL, "mg_lmax must be in (0, 100)");
  if (!(o->mg_rho_cut >= 0.0 && is_finite(o->mg_rho_cut))) return fail(c, CHNS_EINVAL, "mg_rho_cut must be >= 0");
  return CHNS_OK;
}

// ------------------------------------------------------------------ operators

// Re-form L = M + tau C, X = tau g K + sqrt(tau g / beta) M and the AC matrix
// M + tau delta_v K + tau C on every level, with FP32 copies and 1/diag.
int form_operators(chns_ctx* c, hipStream_t s) {
  const auto& p = c->prm;
  const double beta = p.eps * p.eps, tg = p.tau * p.mobility;
  const double smatch = std::sqrt(tg / beta);
  const double delta_v = p.evap_rate * p.eps * p.eps;
  c->coefL[0] = 1.0;
  c->coefL[1] = 0.0;
  c->coefX[0] = smatch;
  c->coefX[1] = tg;
  c->coefAC[0] = 1.0;
  c->coefAC[1] = p.tau * delta_v;
  for (auto& L : c->lv) {
    const int64_t ns = L.sell.slots();
    const double* C = c->has_conv ? L.C : nullptr;
    combine(ns, 1.0, L.M, 0.0, nullptr, p.tau, C, L.L.v64, L.L.v32, s);
    combine(ns, smatch, L.M, tg, L.K, 0.0, nullptr, L.X.v64, L.X.v32, s);
    combine(ns, 1.0, L.M, p.tau * delta_v, L.K, p.tau, C, L.AC.v64, L.AC.v32, s);
    diag_inverse(L.N, L.diag, L.L.v64, L.L.d64, L.L.d32, s);
    diag_inverse(L.N, L.diag, L.X.v64, L.X.d64, L.X.d32, s);
    diag_inverse(L.N, L.diag, L.AC.v64, L.AC.d64, L.AC.d32, s);
  }
  HIPCHK(c, hipGetLastError());
  return CHNS_OK;
}

// Galerkin refresh of one base stream from level 0 down.
void galerkin_down(chns_ctx* c, double* Level::*stream, float* Level::*copy32, hipStream_t s) {
  for (size_t l = 0; l + 1 < c->lv.size(); ++l) {
    Level& F = c->lv[l];
    Level& G = c->lv[l + 1];
    galerkin(G.sell.slots(), F.gptr, F.gsrc, F.gw, F.*stream, G.*stream, s);
  }
  for (auto& L : c->lv) convert<double, float>(L.sell.slots(), L.*stream, L.*copy32, s);
}

int assemble_base(chns_ctx* c, int kind, double* val, const double* vel, hipStream_t s) {
  Level& L0 = c->lv[0];
  HIPCHK(c, hipMemsetAsync(val, 0, L0.sell.slots() * sizeof(double), s));
  const int64_t n2 = 4 * int64_t(c->N);
  for (int col = 0; col < 8; ++col)
    assemble_p1(kind, c->el.colour_ptr[col], c->el.colour_ptr[col + 1], c->ep2, c->etype, c->eslot,
                1.0 / c->mesh.n, vel, n2, val, s);
  HIPCHK(c, hipGetLastError());
  return CHNS_OK;
}

// ------------------------------------------------------------------ multigrid

template <typename T> struct Sel;
template <> struct Sel<double> {
  static const double* v(const OpVals& o) { return o.v64; }
  static const double* d(const OpVals& o) { return o.d64; }
  static double* b(Level& L) { return L.b64; }
  static double* x(Level& L) { return L.x64; }
  static double* t(Level& L) { return L.t64; }
  static double* r(Level& L) { return L.r64; }
  static double* e(Level& L) { return L.e64; }
  static double* dd(Level& L) { return L.d64; }
  static const double* P(Level& L) { return L.P64; }
  static const double* R(Level& L) { return L.R64; }
  static const double* M(Level& L) { return L.M; }
};
template <> struct Sel<float> {
  static const float* v(const OpVals& o) { return o.v32; }
  static const float* d(const OpVals& o) { return o.d32; }
  static float* b(Level& L) { return L.b32; }
  static float* x(Level& L) { return L.x32; }
  static float* t(Level& L) { return L.t32; }
  static float* r(Level& L) { return L.r32; }
  static float* e(Level& L) { return L.e32; }
  static float* dd(Level& L) { return L.d32; }
  static const float* P(Level& L) { return L.P32; }
  static const float* R(Level& L) { return L.R32; }
  static const float* M(Level& L) { return L.M32; }
};

// Chebyshev coefficients for `steps` steps on [lo, hi] (first kind):
// d_0 = r_0 / theta; d_i = rho_i rho_{i-1} d_{i-1} + (2 rho_i / delta) r_i.
template <typename T>
ChebCoef<T> cheb_coef(double lo, double hi, int steps) {
  ChebCoef<T> cc{};
  const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
  double rho_prev = 1.0 / sigma;
  cc.steps = steps;
  cc.c1[0] = T(0);
  cc.c2[0] = T(1.0 / theta);
  for (int i = 1; i < steps; ++i) {
    const double rho_i = 1.0 / (2.0 * sigma - rho_prev);
    cc.c1[i] = T(rho_i * rho_prev);
    cc.c2[i] = T(2.0 * rho_i / delta);
    rho_prev = rho_i;
  }
  return cc;
}

// Level where the cycle of a M + b K stops: first l with 8 b n_l^2 / a <= rho_cut.
size_t cut_level(chns_ctx* c, const double* coef, double rho_cut) {
  for (size_t l = 0; l < c->lv.size(); ++l) {
    const double nl = c->lv[l].n;
    if (8.0 * coef[1] * nl * nl / coef[0] <= rho_cut) return l;
  }
  return c->lv.size() - 1;
}

const double* coef_of(chns_ctx* c, OpVals Level::*op) {
  if (op == &Level::L) return c->coefL;
  if (op == &Level::X) return c->coefX;
  return c->coefAC;
}

// Chebyshev steps from x = 0 (cur/oth ping-pong so that the result lands in x).
template <typename T>
void cheb_from_zero(Level& L, const OpVals& A, const T* b, T* x, const ChebCoef<T>& cc,
                    hipStream_t s) {
  if (L.N <= 1024) {
    coarse_cheb<T, T>(L.d, Sel<T>::v(A), Sel<T>::d(A), b, cc, x, s);
    return;
  }
  T* cur = ((cc.steps - 1) % 2 == 0) ? x : Sel<T>::t(L);
  T* oth = (cur == x) ? Sel<T>::t(L) : x;
  T* d = Sel<T>::dd(L);
  cheb0<T>(L.N, Sel<T>::d(A), b, cc.c2[0], d, cur, s);
  for (int k = 1; k < cc.steps; ++k) {
    stencil<T, T>(L.d, Sel<T>::v(A), ST_CHEB, cur, b, Sel<T>::d(A), d, cc.c1[k], cc.c2[k], oth, s);
    std::swap(cur, oth);
  }
}

// One V(pre, post) cycle from x = 0 on level l (down to the cut level):
// x = V b.  `x` and `b` may be external buffers on level 0; the level's t, r
// and d vectors are scratch.
template <typename T>
void vcycle(chns_ctx* c, OpVals Level::*op, size_t l, size_t cut, const T* b, T* x,
            const chns_solve_opts& o, hipStream_t s) {
  Level& L = c->lv[l];
  const OpVals& A = L.*op;
  const double lmax = o.mg_lmax;
  if (l == cut) {
    const double* cf = coef_of(c, op);
    const double nl = L.n;
    const double rho = 8.0 * cf[1] * nl * nl / cf[0];
    const int steps = (l > 0) ? o.mg_coarse : o.mg_pre + o.mg_post;
    cheb_from_zero<T>(L, A, b, x, cheb_coef<T>(0.45 / (1.0 + rho), lmax, std::min(steps, MAXCHEB)), s);
    return;
  }
  const ChebCoef<T> pre = cheb_coef<T>(lmax / 4.0, lmax, o.mg_pre);
  const int swaps_post = o.mg_post;
  // pre-smoothing from zero: result must end in `cur`, then the post steps
  // alternate; choose the start buffer so that the final iterate is `x`.
  T* cur = ((o.mg_pre - 1 + swaps_post) % 2 == 0) ? x : Sel<T>::t(L);
  T* oth = (cur == x) ? Sel<T>::t(L) : x;
  T* d = Sel<T>::dd(L);
  cheb0<T>(L.N, Sel<T>::d(A), b, pre.c2[0], d, cur, s);
  for (int k = 1; k < o.mg_pre; ++k) {
    stencil<T, T>(L.d, Sel<T>::v(A), ST_CHEB, cur, b, Sel<T>::d(A), d, pre.c1[k], pre.c2[k], oth, s);
    std::swap(cur, oth);
  }
  T* r = Sel<T>::r(L);
  stencil<T, T>(L.d, Sel<T>::v(A), ST_RESID, cur, b, nullptr, nullptr, T(0), T(0), r, s);
  Level& G = c->lv[l + 1];
  spmv<T, T>(L.dR, Sel<T>::R(L), r, Sel<T>::b(G), T(1), T(0), s);
  vcycle<T>(c, op, l + 1, cut, Sel<T>::b(G), Sel<T>::x(G), o, s);
  spmv<T, T>(L.dP, Sel<T>::P(L), Sel<T>::x(G), cur, T(1), T(1), s);
  if (o.mg_post > 0) {
    const ChebCoef<T> post = cheb_coef<T>(lmax / 4.0, lmax, o.mg_post);
    for (int k = 0; k < o.mg_post; ++k) {
      stencil<T, T>(L.d, Sel<T>::v(A), ST_CHEB, cur, b, Sel<T>::d(A), d, post.c1[k], post.c2[k],
                    oth, s);
      std::swap(cur, oth);
    }
  }
}

// mg_cycles V-cycles as a stationary iteration from x = 0 on level 0.
template <typename T>
void mg_solve(chns_ctx* c, OpVals Level::*op, const T* b, T* x, const chns_solve_opts& o,
              hipStream_t s) {
  const size_t cut = cut_level(c, coef_of(c, op), o.mg_rho_cut);
  vcycle<T>(c, op, 0, cut, b, x, o, s);
  Level& L = c->lv[0];
  for (int k = 1; k < o.mg_cycles; ++k) {
    T* res = Sel<T>::e(L);
    stencil<T, T>(L.d, Sel<T>::v(L.*op), ST_RESID, x, b, nullptr, nullptr, T(0), T(0), res, s);
    T* corr = std::is_same<T, double>::value ? (T*)c->w64c : (T*)c->w32c;
    vcycle<T>(c, op, 0, cut, res, corr, o, s);
    axpby<T>(L.N, T(1), corr, T(1), x, s);
  }
}

template <typename T>
void ch_precond_t(chns_ctx* c, const T* r, T* z, T* tmp1, T* tmp2, const chns_solve_opts& o,
                  hipStream_t s) {
  const int N = c->N;
  Level& L0 = c->lv[0];
  mg_solve<T>(c, &Level::L, r, z, o, s);
  mg_solve<T>(c, &Level::X, r + N, tmp1, o, s);
  spmv<T, T>(L0.d, Sel<T>::M(L0), tmp1, tmp2, T(1), T(0), s);
  mg_solve<T>(c, &Level::X, tmp2, z + N, o, s);
}

int precond(chns_ctx* c, int block, const chns_solve_opts& o, const double* r, double* z,
            hipStream_t s) {
  const int N = c->N;
  if (block == CHNS_BLOCK_CH) {
    if (o.precision == CHNS_F64) {
      ch_precond_t<double>(c, r, z, c->w64a, c->w64b, o, s);
    } else {
      convert<double, float>(2 * int64_t(N), r, c->r32, s);
      ch_precond_t<float>(c, c->r32, c->z32, c->w32a, c->w32b, o, s);
      convert<float, double>(2 * int64_t(N), c->z32, z, s);
    }
  } else if (block == CHNS_BLOCK_AC) {
    if (c->mesh.model == CHNS_MODEL_CH) return fail(c, CHNS_EUNSUPPORTED, "model has no AC block");
    if (o.precision == CHNS_F64) {
      mg_solve<double>(c, &Level::AC, r, z, o, s);
    } else {
      convert<double, float>(N, r, c->r32, s);
      mg_solve<float>(c, &Level::AC, c->r32, c->z32, o, s);
      convert<float, double>(N, c->z32, z, s);
    }
  } else {
    return fail(c, CHNS_EUNSUPPORTED, "block not available");
  }
  HIPCHK(c, hipGetLastError());
  return CHNS_OK;
}

int64_t block_size(chns_ctx* c, int block) {
  if (block == CHNS_BLOCK_CH) return 2 * int64_t(c->N);
  if (block == CHNS_BLOCK_AC) return c->N;
  return 0;
}

// y = alpha A x + beta y for a block operator (FP64).
int apply_block(chns_ctx* c, int block, const double* x, double* y, double alpha, double beta,
                hipStream_t s) {
  const auto& p = c->prm;
  Level& L0 = c->lv[0];
  if (block == CHNS_BLOCK_CH) {
    const double tg = p.tau * p.mobility, beta_ = p.eps * p.eps;
    const double* Lv = c->has_conv ? L0.L.v64 : L0.M;
    ch_block<double, double>(L0.d, Lv, L0.K, L0.M, tg, -tg / beta_, x, alpha, beta, y, s);
  } else if (block == CHNS_BLOCK_AC) {
    spmv<double, double>(L0.d, L0.AC.v64, x, y, alpha, beta, s);
  } else {
    return fail(c, CHNS_EUNSUPPORTED, "block not available");
  }
  HIPCHK(c, hipGetLastError());
  return CHNS_OK;
}

// ------------------------------------------------------------------ FGMRES

int read_scal(chns_ctx* c, hipStream_t s, int count) {
  HIPCHK(c, hipMemcpyAsync(c->kr.host, c->kr.scal, count * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  return CHNS_OK;
}

int fgmres(chns_ctx* c, int block, const double* b, double* x, const chns_solve_opts& o,
           chns_solve_info* info, hipStream_t s) {
  Krylov& K = c->kr;
  const int64_t n = block_size(c, block);
  const int m = o.restart;
  const int nblk = reduce_blocks(n);
  const int64_t ld = n;  // basis vectors stored contiguously with stride n
  chns_solve_info inf{};
  HIPCHK(c, hipEventRecord(c->ev0, s));
  norm_partial(n, b, K.nrm_part, s);
  norm_finish(nblk, K.nrm_part, K.scal, nullptr, m, s);
  TRY(read_scal(c, s, 3));
  inf.bnorm = K.host[0];
  const double tol = std::fmax(o.rtol * inf.bnorm, o.atol);
  int iters = 0;
  bool first = true;
  while (true) {
    // V0 = b - A x, beta = ||V0||, g = beta e1
    HIPCHK(c, hipMemcpyAsync(K.V, b, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    TRY(apply_block(c, block, x, K.V, -1.0, 1.0, s));
    norm_partial(n, K.V, K.nrm_part, s);
    norm_finish(nblk, K.nrm_part, K.scal, K.g, m, s);
    TRY(read_scal(c, s, 3));
    const double beta = K.host[0];
    if (first) inf.res0 = beta;
    first = false;
    inf.res_true = beta;
    if (beta <= tol) {
      inf.converged = 1;
      break;
    }
    if (iters >= o.maxiter || !std::isfinite(beta)) break;
    inf.restarts++;
    scale_by_inv(n, K.V, K.scal + 1, K.V, s);
    int k = 0;
    for (int j = 0; j < m; ++j) {
      double* vj = K.V + j * ld;
      double* vn = K.V + (j + 1) * ld;
      double* zj = K.Z + j * ld;
      double* hcol = K.H + int64_t(j) * (m + 1);
      TRY(precond(c, block, o, vj, zj, s));
      TRY(apply_block(c, block, zj, vn, 1.0, 0.0, s));
      // classical Gram-Schmidt; the first multi-dot also gives ||w||^2 (w is
      // basis slot j+1), the update gives ||w'||^2, and a second pass runs
      // only when ||w'||^2 < ||w||^2 / 2 (decided on the device).
      mdot_partial(n, K.V, ld, j + 2, vn, K.part, nullptr, s);
      mdot_reduce(nblk, j + 2, K.part, K.htmp, hcol, 0, nullptr, s);
      maxpy(n, K.V, ld, j + 1, K.htmp, vn, K.nrm_part, nullptr, s);
      reorth_decide(nblk, K.nrm_part, K.htmp + j + 1, K.flag, K.scal, s);
      mdot_partial(n, K.V, ld, j + 1, vn, K.part, K.flag, s);
      mdot_reduce(nblk, j + 1, K.part, K.htmp, hcol, 1, K.flag, s);
      maxpy(n, K.V, ld, j + 1, K.htmp, vn, K.nrm_part2, K.flag, s);
      arnoldi_finish(nblk, K.nrm_part2, K.flag, j, m, K.H, K.cs, K.sn, K.g, K.scal, s);
      scale_by_inv(n, vn, K.scal + 1, vn, s);
      HIPCHK(c, hipGetLastError());
      k = j + 1;
      ++iters;
      TRY(read_scal(c, s, 3));
      const double est = K.host[0], hnext = K.host[2];
      if (est <= tol || hnext == 0.0 || iters >= o.maxiter || !std::isfinite(est)) break;
    }
    lsq_solve(k, m, K.H, K.g, K.y, s);
    xupdate(n, K.Z, ld, k, K.y, x, s);
    HIPCHK(c, hipGetLastError());
  }
  HIPCHK(c, hipEventRecord(c->ev1, s));
  HIPCHK(c, hipEventSynchronize(c->ev1));
  float ms = 0.f;
  HIPCHK(c, hipEventElapsedTime(&ms, c->ev0, c->ev1));
  inf.ms = ms;
  inf.iters = iters;
  inf.status = inf.converged ? CHNS_OK : CHNS_WNOCONV;
  if (info) *info = inf;
  return inf.status;
}

// ------------------------------------------------------------------ set-up

int build(chns_ctx* c) {
  const int n = c->mesh.n;
  c->N = n * n;
  // levels n, n/2, ... while even and the next size is >= 4
  std::vector<int> sizes{n};
  while (sizes.back() % 2 == 0 && sizes.back() / 2 >= 4) sizes.push_back(sizes.back() / 2);
  c->lv.resize(sizes.size());
  for (size_t l = 0; l < sizes.size(); ++l) {
    Level& L = c->lv[l];
    L.n = sizes[l];
    L.N = L.n * L.n;
    Elements E = make_elements(L.n);
    L.csr = pattern_from_elements(L.N, L.N, E.ne, E.v.data(), 3, E.v.data(), 3);
    L.sell = make_sell(L.csr, 64, 1);
    if (!L.sell.uniform || L.sell.width_max != 7)
      return fail(c, CHNS_EINVAL, "P1 pattern is not the uniform 7-point stencil");
    TRY(upload_sell(c, L.sell, L.d));
    TRY(upload(c, &L.diag, L.sell.diag));
    if (l == 0) {
      c->el = std::move(E);
      std::vector<int> slot(size_t(c->el.ne) * 9);
      for (int e = 0; e < c->el.ne; ++e)
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) {
            const int q = L.csr.find(c->el.v[e * 3 + a], c->el.v[e * 3 + b]);
            slot[size_t(e) * 9 + a * 3 + b] = L.sell.csr2sell[q];
          }
      TRY(upload(c, &c->ep2, c->el.p2));
      TRY(upload(c, &c->etype, c->el.type));
      TRY(upload(c, &c->eslot, slot));
    }
  }
  for (size_t l = 0; l + 1 < c->lv.size(); ++l) {
    Level& F = c->lv[l];
    Level& G = c->lv[l + 1];
    p1_prolongation(F.n, F.Pcsr, F.Pval);
    csr_transpose(F.Pcsr, F.Pval, F.Rcsr, F.Rval);
    F.Psell = make_sell(F.Pcsr, 64, 1);
    F.Rsell = make_sell(F.Rcsr, 64, 1);
    TRY(upload_sell(c, F.Psell, F.dP));
    TRY(upload_sell(c, F.Rsell, F.dR));
    auto sell_vals = [](const Sell& S, const Csr& A, const std::vector<double>& v) {
      std::vector<double> out(S.slots(), 0.0);
      for (int64_t q = 0; q < A.nnz(); ++q) out[S.csr2sell[q]] = v[q];
      return out;
    };
    auto pv = sell_vals(F.Psell, F.Pcsr, F.Pval), rv = sell_vals(F.Rsell, F.Rcsr, F.Rval);
    std::vector<float> pv32(pv.begin(), pv.end()), rv32(rv.begin(), rv.end());
    TRY(upload(c, &F.P64, pv));
    TRY(upload(c, &F.R64, rv));
    TRY(upload(c, &F.P32, pv32));
    TRY(upload(c, &F.R32, rv32));
    std::string gerr;
    GalerkinMap gm = make_galerkin(F.csr, F.sell, F.Pcsr, F.Pval, G.csr, G.sell, &gerr);
    if (!gerr.empty()) return fail(c, CHNS_EINVAL, gerr);
    TRY(upload(c, &F.gptr, gm.ptr));
    TRY(upload(c, &F.gsrc, gm.src));
    TRY(upload(c, &F.gw, gm.w));
  }
  // values and work vectors
  for (auto& L : c->lv) {
    const size_t ns = L.sell.slots(), N = L.N;
    TRY(dalloc(c, &L.M, ns));
    TRY(dalloc(c, &L.K, ns));
    TRY(dalloc(c, &L.C, ns));
    TRY(dalloc(c, &L.M32, ns));
    TRY(dalloc(c, &L.K32, ns));
    TRY(dalloc(c, &L.C32, ns));
    for (OpVals* o : {&L.L, &L.X, &L.AC}) {
      TRY(dalloc(c, &o->v64, ns));
      TRY(dalloc(c, &o->v32, ns));
      TRY(dalloc(c, &o->d64, N));
      TRY(dalloc(c, &o->d32, N));
    }
    for (double** v : {&L.b64, &L.x64, &L.t64, &L.r64, &L.e64, &L.d64}) TRY(dalloc(c, v, N));
    for (float** v : {&L.b32, &L.x32, &L.t32, &L.r32, &L.e32, &L.d32}) TRY(dalloc(c, v, N));
    HIPCHK(c, hipMemset(L.C, 0, ns * sizeof(double)));
    HIPCHK(c, hipMemset(L.C32, 0, ns * sizeof(float)));
  }
  const size_t N1 = size_t(c->N), N2 = 2 * N1;
  for (double** v : {&c->w64a, &c->w64b, &c->w64c, &c->rhs_ac}) TRY(dalloc(c, v, N1));
  for (double** v : {&c->rhs_ch, &c->xch}) TRY(dalloc(c, v, N2));
  for (float** v : {&c->r32, &c->z32}) TRY(dalloc(c, v, N2));
  for (float** v : {&c->w32a, &c->w32b, &c->w32c}) TRY(dalloc(c, v, N1));
  // Krylov workspace, sized for the largest block
  Krylov& K = c->kr;
  K.nmax = int64_t(N2);
  TRY(dalloc(c, &K.V, size_t(MAX_RESTART + 1) * K.nmax));
  TRY(dalloc(c, &K.Z, size_t(MAX_RESTART) * K.nmax));
  TRY(dalloc(c, &K.H, size_t(MAX_RESTART + 1) * MAX_RESTART));
  TRY(dalloc(c, &K.cs, MAX_RESTART + 1));
  TRY(dalloc(c, &K.sn, MAX_RESTART + 1));
  TRY(dalloc(c, &K.g, MAX_RESTART + 2));
  TRY(dalloc(c, &K.y, MAX_RESTART + 1));
  TRY(dalloc(c, &K.scal, 8));
  TRY(dalloc(c, &K.htmp, MAX_RESTART + 2));
  TRY(dalloc(c, &K.part, size_t(1024) * (MAX_RESTART + 2)));
  TRY(dalloc(c, &K.nrm_part, 1024));
  TRY(dalloc(c, &K.nrm_part2, 1024));
  TRY(dalloc(c, &K.flag, 4));
  HIPCHK(c, hipHostMalloc((void**)&K.host, 8 * sizeof(double), hipHostMallocDefault));
  HIPCHK(c, hipEventCreate(&c->ev0));
  HIPCHK(c, hipEventCreate(&c->ev1));
  // M and K on the finest level by coloured scatter, then Galerkin down
  hipStream_t s = nullptr;
  Level& L0 = c->lv[0];
  TRY(assemble_base(c, 0, L0.M, nullptr, s));
  TRY(assemble_base(c, 1, L0.K, nullptr, s));
  galerkin_down(c, &Level::M, &Level::M32, s);
  galerkin_down(c, &Level::K, &Level::K32, s);
  TRY(form_operators(c, s));
  HIPCHK(c, hipDeviceSynchronize());
  return CHNS_OK;
}

void release(chns_ctx* c) {
  if (!c) return;
  for (void* p : c->allocs) (void)hipFree(p);
  c->allocs.clear();
  if (c->kr.host) (void)hipHostFree(c->kr.host);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
}

const DSell* op_pattern(chns_ctx* c, int op) {
  if (op >= CHNS_OP_M && op <= CHNS_OP_L) return &c->lv[0].d;
  return nullptr;
}

}  // namespace

// ================================================================== C-ABI

extern "C" {

void chns_default_opts(chns_solve_opts* o) {
  if (!o) return;
  o->rtol = 1e-8;
  o->atol = 0.0;
  o->restart = 40;
  o->maxiter = 600;
  o->precision = CHNS_F64;
  o->mg_cycles = 1;
  o->mg_pre = 2;
  o->mg_post = 2;
  o->mg_coarse = 8;
  o->mg_lmax = 2.1;
  o->mg_rho_cut = 0.25;
}

int chns_create(const chns_mesh* mesh, const chns_params* params, chns_ctx** out) {
  if (!out) return CHNS_EINVAL;
  *out = nullptr;
  if (!mesh) {
    g_create_err = "mesh is NULL";
    return CHNS_EINVAL;
  }
  if (mesh->n < 8 || mesh->n > 8192 || mesh->n % 2 != 0) {
    g_create_err = "n must be even and in 8..8192";
    return CHNS_EINVAL;
  }
  if (mesh->model < CHNS_MODEL_CH || mesh->model > CHNS_MODEL_TERNARY) {
    g_create_err = "unknown model";
    return CHNS_EINVAL;
  }
  if (mesh->model == CHNS_MODEL_TERNARY) {
    g_create_err = "the ternary model (Oseen block) is not available in this build";
    return CHNS_EUNSUPPORTED;
  }
  chns_ctx tmp;
  if (check_params(&tmp, params) != CHNS_OK) {
    g_create_err = tmp.err;
    return CHNS_EINVAL;
  }
  chns_ctx* c = new chns_ctx();
  c->mesh = *mesh;
  c->prm = *params;
  const int rc = build(c);
  if (rc < 0) {
    g_create_err = c->err;
    release(c);
    delete c;
    return rc;
  }
  *out = c;
  return CHNS_OK;
}

int chns_destroy(chns_ctx* c) {
  if (!c) return CHNS_EINVAL;
  (void)hipDeviceSynchronize();
  release(c);
  delete c;
  return CHNS_OK;
}

int chns_set_params(chns_ctx* c, const chns_params* p) {
  if (!c) return CHNS_EINVAL;
  TRY(check_params(c, p));
  c->prm = *p;
  TRY(form_operators(c, nullptr));
  HIPCHK(c, hipDeviceSynchronize());
  return CHNS_OK;
}

int chns_assemble(chns_ctx* c, const double* d_vel, const double* const* d_mu, void* stream) {
  if (!c) return CHNS_EINVAL;
  (void)d_mu;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Level& L0 = c->lv[0];
  if (d_vel) {
    TRY(assemble_base(c, 2, L0.C, d_vel, s));
    galerkin_down(c, &Level::C, &Level::C32, s);
    c->has_conv = true;
  } else {
    for (auto& L : c->lv) {
      HIPCHK(c, hipMemsetAsync(L.C, 0, L.sell.slots() * sizeof(double), s));
      HIPCHK(c, hipMemsetAsync(L.C32, 0, L.sell.slots() * sizeof(float), s));
    }
    c->has_conv = false;
  }
  return form_operators(c, s);
}

int chns_matrix_shape(chns_ctx* c, int32_t op, int64_t* nrows, int64_t* ncols, int64_t* nnz) {
  if (!c) return CHNS_EINVAL;
  const Level& L0 = c->lv[0];
  int64_t r, k, z;
  if (op >= CHNS_OP_M && op <= CHNS_OP_L && op != CHNS_OP_CH) {
    r = k = L0.N;
    z = L0.csr.nnz();
  } else if (op == CHNS_OP_CH) {
    r = k = 2 * int64_t(L0.N);
    z = 4 * L0.csr.nnz();
  } else {
    return fail(c, CHNS_EINVAL, "unknown operator");
  }
  if (nrows) *nrows = r;
  if (ncols) *ncols = k;
  if (nnz) *nnz = z;
  return CHNS_OK;
}

int chns_get_matrix(chns_ctx* c, int32_t op, int32_t* h_rowptr, int32_t* h_col, double* h_val,
                    void* stream) {
  if (!c) return CHNS_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  Level& L0 = c->lv[0];
  const int64_t ns = L0.sell.slots(), nnz = L0.csr.nnz();
  auto fetch = [&](const double* d, std::vector<double>& csrv) -> int {
    std::vector<double> sv(ns);
    HIPCHK(c, hipMemcpyAsync(sv.data(), d, ns * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    csrv.resize(nnz);
    for (int64_t q = 0; q < nnz; ++q) csrv[q] = sv[L0.sell.csr2sell[q]];
    return CHNS_OK;
  };
  const double* src = nullptr;
  switch (op) {
    case CHNS_OP_M: src = L0.M; break;
    case CHNS_OP_K: src = L0.K; break;
    case CHNS_OP_C: src = L0.C; break;
    case CHNS_OP_AC: src = L0.AC.v64; break;
    case CHNS_OP_X: src = L0.X.v64; break;
    case CHNS_OP_L: src = L0.L.v64; break;
    case CHNS_OP_CH: break;
    default: return fail(c, CHNS_EINVAL, "unknown operator");
  }
  const int N = L0.N;
  if (op != CHNS_OP_CH) {
    std::vector<double> v;
    if (h_val) {
      TRY(fetch(src, v));
      std::memcpy(h_val, v.data(), nnz * sizeof(double));
    }
    if (h_rowptr) std::memcpy(h_rowptr, L0.csr.rowptr.data(), (N + 1) * sizeof(int));
    if (h_col) std::memcpy(h_col, L0.csr.col.data(), nnz * sizeof(int));
    return CHNS_OK;
  }
  // CH block [[L, tg K], [tg K, -(tg/beta) M]] assembled on the host from the device streams
  std::vector<double> Lv, Kv, Mv;
  const double tg = c->prm.tau * c->prm.mobility, beta = c->prm.eps * c->prm.eps;
  if (h_val) {
    TRY(fetch(c->has_conv ? L0.L.v64 : L0.M, Lv));
    TRY(fetch(L0.K, Kv));
    TRY(fetch(L0.M, Mv));
  }
  int64_t q = 0;
  if (h_rowptr) h_rowptr[0] = 0;
  for (int blockrow = 0; blockrow < 2; ++blockrow)
    for (int r = 0; r < N; ++r) {
      for (int half = 0; half < 2; ++half)
        for (int p = L0.csr.rowptr[r]; p < L0.csr.rowptr[r + 1]; ++p) {
          if (h_col) h_col[q] = L0.csr.col[p] + half * N;
          if (h_val) {
            double v;
            if (blockrow == 0) v = half == 0 ? Lv[p] : tg * Kv[p];
            else v = half == 0 ? tg * Kv[p] : -(tg / beta) * Mv[p];
            h_val[q] = v;
          }
          ++q;
        }
      if (h_rowptr) h_rowptr[blockrow * N + r + 1] = int32_t(q);
    }
  return CHNS_OK;
}

int chns_spmv(chns_ctx* c, int32_t op, int32_t precision, double alpha, const void* d_x, double beta,
              void* d_y, void* stream) {
  if (!c) return CHNS_EINVAL;
  if (!d_x || !d_y) return fail(c, CHNS_EINVAL, "x or y is NULL");
  if (d_x == d_y) return fail(c, CHNS_EINVAL, "x and y must not overlap");
  if (precision != CHNS_F64 && precision != CHNS_MIXED) return fail(c, CHNS_EINVAL, "unknown precision");
  if (!is_finite(alpha) || !is_finite(beta)) return fail(c, CHNS_EINVAL, "alpha/beta not finite");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Level& L0 = c->lv[0];
  const auto& p = c->prm;
  const double tg = p.tau * p.mobility, be = p.eps * p.eps;
  if (op == CHNS_OP_CH) {
    if (precision == CHNS_F64) {
      ch_block<double, double>(L0.d, c->has_conv ? L0.L.v64 : L0.M, L0.K, L0.M, tg, -tg / be,
                               (const double*)d_x, alpha, beta, (double*)d_y, s);
    } else {
      ch_block<float, float>(L0.d, c->has_conv ? L0.L.v32 : L0.M32, L0.K32, L0.M32, float(tg),
                             float(-tg / be), (const float*)d_x, float(alpha), float(beta),
                             (float*)d_y, s);
    }
    HIPCHK(c, hipGetLastError());
    return CHNS_OK;
  }
  const double* v64 = nullptr;
  const float* v32 = nullptr;
  switch (op) {
    case CHNS_OP_M: v64 = L0.M; v32 = L0.M32; break;
    case CHNS_OP_K: v64 = L0.K; v32 = L0.K32; break;
    case CHNS_OP_C: v64 = L0.C; v32 = L0.C32; break;
    case CHNS_OP_AC: v64 = L0.AC.v64; v32 = L0.AC.v32; break;
    case CHNS_OP_X: v64 = L0.X.v64; v32 = L0.X.v32; break;
    case CHNS_OP_L: v64 = L0.L.v64; v32 = L0.L.v32; break;
    default: return fail(c, CHNS_EINVAL, "unknown operator");
  }
  if (precision == CHNS_F64)
    spmv<double, double>(L0.d, v64, (const double*)d_x, (double*)d_y, alpha, beta, s);
  else
    spmv<float, float>(L0.d, v32, (const float*)d_x, (float*)d_y, float(alpha), float(beta), s);
  HIPCHK(c, hipGetLastError());
  return CHNS_OK;
}

int chns_precond_apply(chns_ctx* c, int32_t block, const chns_solve_opts* opts, const double* d_r,
                       double* d_z, void* stream) {
  if (!c) return CHNS_EINVAL;
  TRY(check_opts(c, opts));
  if (!d_r || !d_z) return fail(c, CHNS_EINVAL, "r or z is NULL");
  if (d_r == d_z) return fail(c, CHNS_EINVAL, "r and z must not overlap");
  if (block != CHNS_BLOCK_CH && block != CHNS_BLOCK_AC) return fail(c, CHNS_EUNSUPPORTED, "block not available");
  return precond(c, block, *opts, d_r, d_z, static_cast<hipStream_t>(stream));
}

int chns_krylov_solve(chns_ctx* c, int32_t block, const double* d_b, double* d_x,
                      const chns_solve_opts* opts, chns_solve_info* h_info, void* stream) {
  if (!c) return CHNS_EINVAL;
  TRY(check_opts(c, opts));
  if (!d_b || !d_x) return fail(c, CHNS_EINVAL, "b or x is NULL");
  if (block != CHNS_BLOCK_CH && block != CHNS_BLOCK_AC) return fail(c, CHNS_EUNSUPPORTED, "block not available");
  if (block == CHNS_BLOCK_AC && c->mesh.model == CHNS_MODEL_CH)
    return fail(c, CHNS_EUNSUPPORTED, "model has no AC block");
  return fgmres(c, block, d_b, d_x, *opts, h_info, static_cast<hipStream_t>(stream));
}

int chns_step_rhs(chns_ctx* c, const chns_fields* in, double* d_rhs_ch, double* d_rhs_ac, double* d_rhs_ns,
                  void* stream) {
  if (!c) return CHNS_EINVAL;
  if (!in || !in->phi[0] || !d_rhs_ch) return fail(c, CHNS_EINVAL, "missing field or output");
  (void)d_rhs_ns;
  const bool ac = c->mesh.model == CHNS_MODEL_CH_AC;
  if (ac && !in->Phi_v) return fail(c, CHNS_EINVAL, "model needs Phi_v");
  const auto& p = c->prm;
  const double beta = p.eps * p.eps;
  rhs_binary(c->lv[0].d, c->lv[0].M, in->phi[0], ac ? in->Phi_v : nullptr,
             -(p.tau * p.mobility / beta), -p.tau * p.evap_rate, d_rhs_ch, ac ? d_rhs_ac : nullptr,
             static_cast<hipStream_t>(stream));
  HIPCHK(c, hipGetLastError());
  return CHNS_OK;
}

int chns_timestep(chns_ctx* c, const chns_fields* in, const chns_fields* out, int32_t nsteps,
                  const chns_solve_opts* opts, chns_solve_info* h_info, void* stream) {
  if (!c) return CHNS_EINVAL;
  TRY(check_opts(c, opts));
  if (!in || !out || nsteps < 1) return fail(c, CHNS_EINVAL, "bad fields or nsteps");
  const bool ac = c->mesh.model == CHNS_MODEL_CH_AC;
  if (!in->phi[0] || !in->mu[0] || !out->phi[0] || !out->mu[0])
    return fail(c, CHNS_EINVAL, "phi[0] and mu[0] are required");
  if (ac && (!in->Phi_v || !out->Phi_v)) return fail(c, CHNS_EINVAL, "model needs Phi_v");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int N = c->N;
  const size_t bytes = size_t(N) * sizeof(double);
  TRY(chns_assemble(c, in->vel, nullptr, s));
  int worst = CHNS_OK;
  chns_fields cur = *in;
  for (int k = 0; k < nsteps; ++k) {
    TRY(chns_step_rhs(c, &cur, c->rhs_ch, c->rhs_ac, nullptr, s));
    double* xch = c->xch;
    HIPCHK(c, hipMemcpyAsync(xch, cur.phi[0], bytes, hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipMemcpyAsync(xch + N, cur.mu[0], bytes, hipMemcpyDeviceToDevice, s));
    chns_solve_info inf{};
    int rc = fgmres(c, CHNS_BLOCK_CH, c->rhs_ch, xch, *opts, &inf, s);
    if (rc < 0) return rc;
    if (rc > worst) worst = rc;
    if (h_info) *h_info++ = inf;
    if (ac) {
      if (out->Phi_v != cur.Phi_v)
        HIPCHK(c, hipMemcpyAsync(out->Phi_v, cur.Phi_v, bytes, hipMemcpyDeviceToDevice, s));
      rc = fgmres(c, CHNS_BLOCK_AC, c->rhs_ac, out->Phi_v, *opts, &inf, s);
      if (rc < 0) return rc;
      if (rc > worst) worst = rc;
      if (h_info) *h_info++ = inf;
    }
    HIPCHK(c, hipMemcpyAsync(out->phi[0], xch, bytes, hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipMemcpyAsync(out->mu[0], xch + N, bytes, hipMemcpyDeviceToDevice, s));
    cur = *out;
  }
  HIPCHK(c, hipStreamSynchronize(s));
  return worst;
}

const char* chns_last_error(const chns_ctx* c) {
  if (!c) return g_create_err.c_str();
  return c->err.c_str();
}

}  // extern "C"
