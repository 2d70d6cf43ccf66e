// C-ABI entry points of chns.h: context set-up, assembly, operators,
// block preconditioners, flexible GMRES and the time step.
#include <hip/hip_runtime.h>

#include <cmath>
#include <algorithm>
#include <atomic>
#include <immintrin.h>
#include <cstdint>
#include <cstring>
#include <string>
#include <type_traits>
#include <utility>

#include "context.hpp"
#include "kernels_adj.hpp"

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

#define HIPCHK_VOID(expr) (void)(expr)

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

// Fold the completed ledger slots into the running sums (synchronising).
int ledger_fold(chns_ctx* c) {
  Ledger& G = c->ledger;
  if (G.used == 0) return CHNS_OK;
  HIPCHK(c, hipEventSynchronize(G.ev[2 * (G.used - 1) + 1]));
  for (int i = 0; i < G.used; ++i) {
    float ms = 0.f;
    HIPCHK(c, hipEventElapsedTime(&ms, G.ev[2 * i], G.ev[2 * i + 1]));
    G.sum_ms += ms;
    G.sum_bytes += G.bytes[i];
  }
  G.used = 0;
  return CHNS_OK;
}

// Launch through the ledger: when class `kid` is being timed, the launch takes
// an event pair that the dispatch itself timestamps (kernel start and end).
template <typename F>
void timed(chns_ctx* c, int kid, double bytes, hipStream_t s, F&& launch) {
  Ledger& G = c->ledger;
  if (G.kernel != kid) {
    launch(LaunchEv{});
    return;
  }
  if (G.used == G.cap) (void)ledger_fold(c);
  LaunchEv ev;
  ev.start = G.ev[2 * G.used];
  ev.stop = G.ev[2 * G.used + 1];
  launch(ev);
  G.bytes[G.used] = bytes;
  ++G.used;
  ++G.launches;
}

// Device memory of the context: the caller's allocator when one was given to
// chns_create, else hipMalloc.  Only set-up calls allocate.
template <typename T>
int dalloc(chns_ctx* c, T** p, size_t n) {
  *p = nullptr;
  if (n == 0) return CHNS_OK;
  void* q = nullptr;
  const size_t bytes = n * sizeof(T);
  if (c->alloc) {
    q = c->alloc(bytes, c->alloc_ctx);
    if (!q) {
      c->err = "the caller's allocator returned NULL for " + std::to_string(bytes) + " bytes";
      return CHNS_ENOMEM;
    }
    if (reinterpret_cast<uintptr_t>(q) % 256 != 0) {
      c->allocs.push_back(q);
      c->err = "the caller's allocator returned memory not aligned to 256 bytes";
      return CHNS_EINVAL;
    }
  } else {
    hipError_t e = hipMalloc(&q, bytes);
    if (e != hipSuccess) {
      c->err = std::string("hipMalloc: ") + hipGetErrorString(e);
      return CHNS_ENOMEM;
    }
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
  // every stored column (padding included) is read by the kernels
  for (int col : S.col)
    if (col < 0 || col >= S.ncols) return fail(c, CHNS_EINVAL, "SELL column out of range");
  d.nrows = S.nrows;
  d.nslices = S.nslices;
  d.width = S.width_max;
  d.uniform = S.uniform ? 1 : 0;
  d.side = S.side;
  d.cube = S.cube;
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

// Coefficients of the ternary density for the kernels.  The Taylor
// coefficients of x ln x about 1/2 come from its derivatives there: ln x + 1,
// 1/x, -1/x^2, 2/x^3.
PotCoef pot_coef(const chns_params& p) {
  PotCoef c;
  c.fh = p.potential == CHNS_POT_FLORY_HUGGINS ? 1 : 0;
  c.trunc = p.truncate ? 1 : 0;
  const double h = 0.5;
  const double d[5] = {h * std::log(h), std::log(h) + 1.0, 1.0 / h, -1.0 / (h * h), 2.0 / (h * h * h)};
  const double fact[5] = {1.0, 1.0, 2.0, 6.0, 24.0};
  for (int k = 0; k < 5; ++k) c.t4[k] = d[k] / fact[k];
  for (int i = 0; i < 3; ++i) {
    c.invN[i] = c.fh ? 1.0 / p.fh_nsize[i] : 1.0;
    c.chi[i] = c.fh ? p.fh_chi[i] : 0.0;
    c.lsat[i] = c.fh ? std::log(p.fh_phisat[i]) : 0.0;
  }
  return c;
}

// Whether an operator equals its transpose in the context's current state:
// M, K and the matching factor X always; the P1 operators with a convection
// part (C, L, AC and the CH block) when no velocity is assembled; the Oseen
// operators (convection J(w), PCD N_p(w)) never.
bool op_symmetric(const chns_ctx* c, int op) {
  switch (op) {
    case CHNS_OP_M: case CHNS_OP_K: case CHNS_OP_X: return true;
    case CHNS_OP_C: case CHNS_OP_L: case CHNS_OP_AC: case CHNS_OP_CH: return !c->has_conv;
    default: return false;
  }
}

bool block_symmetric(const chns_ctx* c, int block) { return block != CHNS_BLOCK_NS && !c->has_conv; }

// The transposed products need the transposed operators in the context
// (chns_assemble_transposed) and the forward ones the forward operators.
int check_orientation(chns_ctx* c, bool symmetric, int32_t transpose) {
  if (transpose != 0 && transpose != 1) return fail(c, CHNS_EINVAL, "transpose must be 0 or 1");
  if (symmetric || (transpose != 0) == c->transposed) return CHNS_OK;
  return fail(c, CHNS_ESTATE,
              transpose ? "the context holds the forward operators: call chns_assemble_transposed first"
                        : "the context holds the transposed operators: call chns_assemble first");
}

// Parameters that belong to some models or domains only: the reason, or null.
const char* model_params_error(int model, bool box, const chns_params* p) {
  const bool ter = model == CHNS_MODEL_TERNARY, quat = model == CHNS_MODEL_QUATERNARY;
  if (!ter && (p->potential != CHNS_POT_QUARTIC || p->truncate))
    return "the Flory-Huggins density and the truncation apply to the ternary model";
  if (!ter && p->var_density) return "variable density applies to the ternary model";
  if (!ter && !quat && p->ns_picard > 1) return "Picard passes apply to the ternary and quaternary models";
  if (!box && p->top_flux != 0.0) return "the top-wall flux belongs to the closed square";
  for (int i = 0; i < 4; ++i) {
    const double b = p->beta_phase[i];
    if (quat && !(std::isfinite(b) && b > 0.0)) return "the quaternary model needs beta_phase[0..3] > 0";
    if (!quat && b != 0.0) return "per-phase gradient coefficients belong to the quaternary model";
  }
  return nullptr;
}

int check_params(chns_ctx* c, const chns_params* p) {
  if (!p) return fail(c, CHNS_EINVAL, "params is NULL");
  const double v[] = {p->eps, p->tau, p->mobility, p->evap_rate, p->viscosity, p->alpha, p->rho};
  for (double x : v)
    if (!is_finite(x)) return fail(c, CHNS_EINVAL, "parameter is NaN or Inf");
  if (p->eps <= 0 || p->tau <= 0 || p->mobility <= 0)
    return fail(c, CHNS_EINVAL, "eps, tau and mobility must be positive");
  if (p->evap_rate < 0 || p->viscosity <= 0 || p->rho <= 0)
    return fail(c, CHNS_EINVAL, "evap_rate must be >= 0, viscosity and rho > 0");
  if (p->potential != CHNS_POT_QUARTIC && p->potential != CHNS_POT_FLORY_HUGGINS)
    return fail(c, CHNS_EINVAL, "unknown potential");
  if (p->truncate != 0 && p->truncate != 1) return fail(c, CHNS_EINVAL, "truncate must be 0 or 1");
  if (p->var_density != 0 && p->var_density != 1) return fail(c, CHNS_EINVAL, "var_density must be 0 or 1");
  if (p->var_density)
    for (int i = 0; i < 3; ++i)
      if (!is_finite(p->rho_pure[i]) || !(p->rho_pure[i] > 0.0))
        return fail(c, CHNS_EINVAL, "pure densities must be positive");
  if (p->ns_picard < 0 || p->ns_picard > 100) return fail(c, CHNS_EINVAL, "ns_picard must be in 0..100");
  if (!is_finite(p->ns_picard_tol) || p->ns_picard_tol < 0.0)
    return fail(c, CHNS_EINVAL, "ns_picard_tol must be >= 0");
  if (!is_finite(p->top_flux) || !is_finite(p->flux_inf))
    return fail(c, CHNS_EINVAL, "top_flux and flux_inf must be finite");
  if (p->potential == CHNS_POT_FLORY_HUGGINS)
    for (int i = 0; i < 3; ++i) {
      if (!is_finite(p->fh_nsize[i]) || !(p->fh_nsize[i] > 0.0))
        return fail(c, CHNS_EINVAL, "Flory-Huggins sizes N_i must be positive");
      if (!is_finite(p->fh_chi[i])) return fail(c, CHNS_EINVAL, "Flory-Huggins chi must be finite");
      if (!(p->fh_phisat[i] > 0.0 && p->fh_phisat[i] <= 1.0))
        return fail(c, CHNS_EINVAL, "saturated vapour fractions must lie in (0, 1]");
    }
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

int form_ternary(chns_ctx* c, hipStream_t s);

// Re-form L = M + tau C, X = tau g K + sqrt(tau g / beta) M and the AC matrix
// M + tau delta_v K + tau C on every level, with FP32 copies and 1/diag.
int form_operators(chns_ctx* c, hipStream_t s) {
  c->formed_c0 = false;
  const auto& p = c->prm;
  const double beta = c->beta_ch, tg = p.tau * p.mobility;
  const double smatch = std::sqrt(tg / beta);
  const double delta_v = p.evap_rate * p.eps * p.eps;
  c->coefL[0] = 1.0;
  c->coefL[1] = 0.0;
  c->coefX[0] = smatch;
  c->coefX[1] = tg;
  c->coefAC[0] = 1.0;
  c->coefAC[1] = p.tau * delta_v;
  // one launch over all levels: L = M (+ tau C), X = smatch M + tg K,
  // AC = M + tau delta_v K (+ tau C)
  FormCoef k{};
  k.a[0] = 1.0;
  k.useK[0] = 0;
  k.c[0] = p.tau;
  k.useC[0] = 1;
  k.a[1] = smatch;
  k.b[1] = tg;
  k.useK[1] = 1;
  k.useC[1] = 0;
  k.a[2] = 1.0;
  k.b[2] = p.tau * delta_v;
  k.useK[2] = 1;
  k.c[2] = p.tau;
  k.useC[2] = 1;
  form_ops(int(c->lv.size()), c->form_tab, c->form_total, k, c->has_conv, s);
  HIPCHK(c, hipGetLastError());
  c->formed_c0 = c->c_zero;
  if (c->ternary) TRY(form_ternary(c, s));
  return CHNS_OK;
}

// Ternary model: velocity blocks A_xx = (rho/tau) M + J + K_xx (and yy) on the
// P2 level and Galerkin down the P1 levels, the Oseen operator values, and the
// PCD matrix A_p = (rho/tau) M + eta K + N_p(w) on the finest P1 level.
int form_ternary(chns_ctx* c, hipStream_t s) {
  const auto& p = c->prm;
  P2Level& P = c->p2;
  Level& L0 = c->lv[0];
  // mass terms: (rho/tau) M, or (1/tau) times the rho^k-weighted masses
  const bool vd = p.var_density != 0;
  const double cm = vd ? 1.0 / p.tau : p.rho / p.tau;
  const double* Mvel = vd ? P.Mr : P.Mv;
  const double* Mpcd = vd ? L0.Mrp : L0.M;
  // the hierarchy cut takes the smallest density's diagonal weight
  c->coefV[0] = vd ? std::min({p.rho_pure[0], p.rho_pure[1], p.rho_pure[2]}) / p.tau : cm;
  c->coefV[1] = 1.5 * p.viscosity;  // the xx/yy forms have a P1 diagonal of 6 eta
  const int64_t ns2 = P.sell.slots();
  combine(ns2, cm, Mvel, 1.0, P.J, 1.0, P.Kxx, P.Vx.v64, P.Vx.v32, s);
  combine(ns2, cm, Mvel, 1.0, P.J, 1.0, P.Kyy, P.Vy.v64, P.Vy.v32, s);
  const NSData& S = c->ns;
  if (c->box)  // no-slip walls: identity rows, and no coupling into them
    for (OpVals* o : {&P.Vx, &P.Vy}) {
      set_slots(S.n_p2_zero, S.p2_zero, 0.0, o->v64, o->v32, s);
      set_slots(S.n_p2_one, S.p2_one, 1.0, o->v64, o->v32, s);
    }
  diag_inverse(P.N4, P.diag, P.Vx.v64, P.Vx.d64, P.Vx.d32, s);
  diag_inverse(P.N4, P.diag, P.Vy.v64, P.Vy.d64, P.Vy.d32, s);
  galerkin(L0.sell.slots(), P.gptr, P.gsrc, P.gw, P.Vx.v64, L0.Vx.v64, s);
  galerkin(L0.sell.slots(), P.gptr, P.gsrc, P.gw, P.Vy.v64, L0.Vy.v64, s);
  for (size_t l = 0; l + 1 < c->lv.size(); ++l) {
    Level& F = c->lv[l];
    Level& G = c->lv[l + 1];
    galerkin(G.sell.slots(), F.gptr, F.gsrc, F.gw, F.Vx.v64, G.Vx.v64, s);
    galerkin(G.sell.slots(), F.gptr, F.gsrc, F.gw, F.Vy.v64, G.Vy.v64, s);
  }
  for (auto& L : c->lv) {
    const int64_t ns = L.sell.slots();
    convert<double, float>(ns, L.Vx.v64, L.Vx.v32, s);
    convert<double, float>(ns, L.Vy.v64, L.Vy.v32, s);
    diag_inverse(L.N, L.diag, L.Vx.v64, L.Vx.d64, L.Vx.d32, s);
    diag_inverse(L.N, L.diag, L.Vy.v64, L.Vy.d64, L.Vy.d32, s);
  }
  form_ns(c->ns.sell.slots(), c->ns.kind, c->ns.src, cm, Mvel, P.J, P.Kxx, P.Kxy, P.Kyx, P.Kyy,
          c->ns.B, c->ns.val, s);
  if (c->box) {
    set_slots(S.n_ns_zero, S.ns_zero, 0.0, c->ns.val, nullptr, s);
    set_slots(S.n_ns_one, S.ns_one, 1.0, c->ns.val, nullptr, s);
  }
  combine(L0.sell.slots(), cm, Mpcd, p.viscosity, L0.K, 1.0, L0.Cw, L0.Ap.v64, L0.Ap.v32, s);
  HIPCHK(c, hipGetLastError());
  return CHNS_OK;
}

int assemble_sym_stiffness(chns_ctx* c, hipStream_t s) {
  P2Level& P = c->p2;
  const int64_t ns2 = P.sell.slots();
  double* outs[4] = {P.Kxx, P.Kxy, P.Kyx, P.Kyy};
  for (double* o : outs) HIPCHK(c, hipMemsetAsync(o, 0, ns2 * sizeof(double), s));
  MuGrad none{{nullptr, nullptr, nullptr}, 0.0};
  for (int col = 0; col < 8; ++col)
    assemble_p2(1, c->el.colour_ptr[col], c->el.colour_ptr[col + 1], c->ep1, c->ep2, c->etype,
                c->ns.eslot36, c->h, c->ns.tb, c->prm.viscosity, nullptr, 0.0,
                4 * int64_t(c->N), none, outs, s);
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
  if (c->dim3) {
    if (kind > 1) return fail(c, CHNS_EUNSUPPORTED, "the cube assembles the mass and stiffness matrices only");
    for (int col = 0; col < 48; ++col)
      assemble_p1_tet(kind, c->colour_ptr3[col], c->colour_ptr3[col + 1], c->etype, c->eslot, c->h, val, s);
    HIPCHK(c, hipGetLastError());
    return CHNS_OK;
  }
  const int64_t n2 = 4 * int64_t(c->N);
  for (int col = 0; col < 8; ++col)
    assemble_p1(kind, c->el.colour_ptr[col], c->el.colour_ptr[col + 1], c->ep2, c->etype, c->eslot,
                c->h, vel, n2, val, s);
  HIPCHK(c, hipGetLastError());
  return CHNS_OK;
}

// State-dependent operators: the P1 convection C(v) of the CH and AC blocks,
// and for the ternary model the P2 convection J(w) of the Oseen velocity block
// and the P1 convection N_p(w) of the PCD matrix, w = rho v - alpha sum grad
// mu_i; then the operator values on every level.  transposed: each of these
// convection parts is replaced by its transpose (values moved to the slots of
// the transposed entries of the symmetric patterns) before the coarse levels
// and the combined operators are formed, so every block and preconditioner
// acts on the transposed system.
int transpose_values(chns_ctx* c, int64_t n, const int* tmap, double* val, hipStream_t s) {
  gather_slots(n, tmap, val, c->tbuf, s);
  HIPCHK(c, hipMemcpyAsync(val, c->tbuf, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  return CHNS_OK;
}

// The Oseen convection J(w) and the PCD convection N_p(w) of the ternary
// model, w = rho v - alpha sum_i grad mu_i (rho^k v at the P2 nodes with
// variable density).
int assemble_ternary_conv(chns_ctx* c, const double* d_vel, const double* const* d_mu, bool transposed,
                          hipStream_t s) {
  Level& L0 = c->lv[0];
  P2Level& P = c->p2;
  MuGrad mg{{nullptr, nullptr, nullptr, nullptr}, c->prm.alpha};
  if (d_mu)
    for (int i = 0; i < (c->quat ? 4 : 3); ++i) mg.mu[i] = d_mu[i];
  HIPCHK(c, hipMemsetAsync(P.J, 0, P.sell.slots() * sizeof(double), s));
  HIPCHK(c, hipMemsetAsync(L0.Cw, 0, L0.sell.slots() * sizeof(double), s));
  double* jo[1] = {P.J};
  const double* rho2 = c->prm.var_density ? c->rho2 : nullptr;
  for (int col = 0; col < 8; ++col) {
    const int e0 = c->el.colour_ptr[col], e1 = c->el.colour_ptr[col + 1];
    assemble_p2(2, e0, e1, c->ep1, c->ep2, c->etype, c->ns.eslot36, c->h, c->ns.tb, 0.0,
                d_vel, c->prm.rho, 4 * int64_t(c->N), mg, jo, s, rho2);
    assemble_p1_conv(e0, e1, c->ep1, c->ep2, c->etype, c->eslot, c->h, d_vel, c->prm.rho,
                     4 * int64_t(c->N), mg, L0.Cw, s, rho2);
  }
  HIPCHK(c, hipGetLastError());
  if (transposed) {
    TRY(transpose_values(c, P.sell.slots(), c->tslot2, P.J, s));
    TRY(transpose_values(c, L0.sell.slots(), c->tslot1, L0.Cw, s));
  }
  return CHNS_OK;
}

// Variable density: rho^k = sum_i rho_i phi_i^k at the vertices and the P2
// nodes, and the masses weighted by it: the P2 velocity mass (int rho psi_m
// psi_n) and the finest-level P1 mass of the PCD matrix.
int weighted_masses(chns_ctx* c, hipStream_t s);

int set_density(chns_ctx* c, const double* php, const double* phn, hipStream_t s) {
  density_fields(c->mesh.n, c->box, php, phn, c->prm.rho_pure, c->rho1, c->rho2, s);
  return weighted_masses(c, s);
}

// Before the first chns_set_density: the uniform density rho.
int uniform_density(chns_ctx* c, hipStream_t s) {
  fill(c->N, c->prm.rho, c->rho1, s);
  fill(4 * int64_t(c->N), c->prm.rho, c->rho2, s);
  return weighted_masses(c, s);
}

int weighted_masses(chns_ctx* c, hipStream_t s) {
  P2Level& P = c->p2;
  Level& L0 = c->lv[0];
  const double h = c->h;
  const int64_t n2 = 4 * int64_t(c->N);
  HIPCHK(c, hipMemsetAsync(P.Mr, 0, P.sell.slots() * sizeof(double), s));
  HIPCHK(c, hipMemsetAsync(L0.Mrp, 0, L0.sell.slots() * sizeof(double), s));
  double* mo[1] = {P.Mr};
  const MuGrad none{{nullptr, nullptr, nullptr}, 0.0};
  for (int col = 0; col < 8; ++col) {
    const int e0 = c->el.colour_ptr[col], e1 = c->el.colour_ptr[col + 1];
    assemble_p2(3, e0, e1, c->ep1, c->ep2, c->etype, c->ns.eslot36, h, c->ns.tb, 0.0, nullptr, 0.0, n2,
                none, mo, s, c->rho1);
    assemble_p1(3, e0, e1, c->ep2, c->etype, c->eslot, h, nullptr, n2, L0.Mrp, s, c->rho1);
  }
  HIPCHK(c, hipGetLastError());
  return CHNS_OK;
}

int assemble_ops(chns_ctx* c, const double* d_vel, const double* const* d_mu, bool transposed,
                 hipStream_t s) {
  if (c->ternary && !d_vel) return fail(c, CHNS_EINVAL, "the ternary model needs a velocity");
  if (c->dim3 && d_vel) return fail(c, CHNS_EUNSUPPORTED, "no convecting velocity on the cube");
  Level& L0 = c->lv[0];
  if (c->ternary) TRY(assemble_ternary_conv(c, d_vel, d_mu, transposed, s));
  if (d_vel) {
    c->c_zero = false;
    TRY(assemble_base(c, 2, L0.C, d_vel, s));
    if (transposed) TRY(transpose_values(c, L0.sell.slots(), c->tslot1, L0.C, s));
    galerkin_down(c, &Level::C, &Level::C32, s);
    c->has_conv = true;
  } else {
    // the binary models' operators depend on the parameters, beta and C only:
    // with C = 0 already formed (and no parameter change since), nothing to do
    if (!c->ternary && c->c_zero && c->formed_c0 && c->transposed == transposed) return CHNS_OK;
    if (!c->c_zero)  // C = 0 without a velocity
      for (auto& L : c->lv) {
        HIPCHK(c, hipMemsetAsync(L.C, 0, L.sell.slots() * sizeof(double), s));
        HIPCHK(c, hipMemsetAsync(L.C32, 0, L.sell.slots() * sizeof(float), s));
      }
    c->c_zero = true;
    c->has_conv = false;
  }
  c->transposed = transposed;
  return form_operators(c, s);
}

// A tiled pass; on the finest level it goes through the ledger (class
// CHNS_KERNEL_MG_FINE) with its algorithmic bytes per fine row: 7 values,
// 1/diag and the right-hand side read; down: the pre-smoothed iterate and
// the coarse right-hand side (a quarter row) written; up: the pre-smoothed
// iterate and the coarse correction read, the result written; from zero:
// the result written.
template <typename T>
void vtile_at(chns_ctx* c, int mode, const TileArgs<T>& a, bool finest, hipStream_t s) {
  if (!finest) {
    vtile<T>(mode, a, s);
    return;
  }
  const double t = sizeof(T), rows = double(a.side) * a.side;
  const double bin = a.b64 ? 8.0 : t, xout = a.x64 ? 8.0 : t;
  double per = 8.0 * t + bin;
  if (mode == TILE_DOWN) per += 1.25 * t;
  else if (mode == TILE_UP) per += 1.25 * t + xout;
  else if (mode == TILE_UPM) per += 8.25 * t + xout;  // and the values of M
  else per += xout;
  timed(c, CHNS_KERNEL_MG_FINE, rows * per, s, [&](LaunchEv ev) { vtile<T>(mode, a, s, ev); });
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

// Upper Chebyshev bound of D^{-1}A for A = a M + b K: the option's value on
// triangles; on the Kuhn tetrahedra, whose D^{-1}M reaches 2.5 (2 on
// triangles), scaled by 5/4.
double lmax_of(const chns_ctx* c, const chns_solve_opts& o) { return c->dim3 ? 1.25 * o.mg_lmax : o.mg_lmax; }

// Level where the cycle of a M + b K stops: first l with r b / (a h_l^2) <=
// rho_cut, r = diag(K) h^2 / diag(M) (8 on triangles, 15 on the tetrahedra).
size_t cut_level(chns_ctx* c, const double* coef, double rho_cut) {
  for (size_t l = 0; l < c->lv.size(); ++l) {
    const double ih = c->lv[l].n / c->len;  // 1 / h on level l
    if (c->diag_ratio * coef[1] * ih * ih / coef[0] <= rho_cut) return l;
  }
  return c->lv.size() - 1;
}

const double kCoefKp[2] = {0.0, 1.0};
const double kCoefMp[2] = {1.0, 0.0};

const double* coef_of(chns_ctx* c, OpVals Level::*op) {
  if (op == &Level::L) return c->coefL;
  if (op == &Level::X) return c->coefX;
  if (op == &Level::Vx || op == &Level::Vy) return c->coefV;
  if (op == &Level::Kp) return kCoefKp;
  if (op == &Level::Mp) return kCoefMp;
  return c->coefAC;
}

bool singular_of(OpVals Level::*op) { return op == &Level::Kp; }

// One Chebyshev sweep of the P1 stencil kernel, through the ledger.
// Algorithmic bytes per row: the row's values (7 on triangles), x (own entry),
// b, 1/diag, d (read when c1 != 0), d and y written; columns are computed on
// the periodic square, not read.
template <typename T>
void cheb_sweep(chns_ctx* c, Level& L, const OpVals& A, const T* x, const T* b, T* d, T c1, T c2,
                T* y, hipStream_t s) {
  const bool f32 = std::is_same<T, float>::value;
  const double bytes = double(L.N) * sizeof(T) * (L.d.width + 5 + (c1 != T(0) ? 1 : 0));
  timed(c, f32 ? CHNS_KERNEL_CHEB32 : CHNS_KERNEL_CHEB64, bytes, s, [&](LaunchEv ev) {
    stencil<T, T>(L.d, Sel<T>::v(A), ST_CHEB, x, b, Sel<T>::d(A), d, c1, c2, y, s, ev);
  });
}

// Chebyshev steps from x = 0 (cur/oth ping-pong so that the result lands in x).
template <typename T>
void cheb_from_zero(chns_ctx* c, Level& L, const OpVals& A, const T* b, T* x, const ChebCoef<T>& cc,
                    hipStream_t s) {
  if (L.N <= 1024) {
    coarse_cheb<T, T>(L.d, Sel<T>::v(A), Sel<T>::d(A), b, cc, x, s);
    return;
  }
  T* d = Sel<T>::dd(L);
  if (cc.steps >= 2 && L.d.side > 0) {  // steps 0 and 1 fused
    T* cur = ((cc.steps - 2) % 2 == 0) ? x : Sel<T>::t(L);
    T* oth = (cur == x) ? Sel<T>::t(L) : x;
    cheb01<T, T>(L.d, Sel<T>::v(A), b, Sel<T>::d(A), cc.c2[0], cc.c1[1], cc.c2[1], d, cur, s);
    for (int k = 2; k < cc.steps; ++k) {
      cheb_sweep<T>(c, L, A, cur, b, d, cc.c1[k], cc.c2[k], oth, s);
      std::swap(cur, oth);
    }
    return;
  }
  T* cur = ((cc.steps - 1) % 2 == 0) ? x : Sel<T>::t(L);
  T* oth = (cur == x) ? Sel<T>::t(L) : x;
  cheb0<T>(L.N, Sel<T>::d(A), b, cc.c2[0], d, cur, s);
  for (int k = 1; k < cc.steps; ++k) {
    cheb_sweep<T>(c, L, A, cur, b, d, cc.c1[k], cc.c2[k], oth, s);
    std::swap(cur, oth);
  }
}

// One V(pre, post) cycle from x = 0 on level l (down to the cut level):
// x = V b.  `x` and `b` may be external buffers on level 0; the level's t, r
// and d vectors are scratch.
// Chebyshev coefficients of the cut level l: interval [lo, lmax] with lo the
// lower spectral bound of D^{-1}A for a M + b K on that level (the smallest
// nonzero eigenvalue for the singular Neumann Laplacian).
template <typename T>
ChebCoef<T> cut_coef(chns_ctx* c, OpVals Level::*op, size_t l, const chns_solve_opts& o) {
  const double* cf = coef_of(c, op);
  const double nl = c->lv[l].n, ih = nl / c->len;  // cells per side, 1 / h
  double lo;
  if (singular_of(op)) {
    // smallest nonzero eigenvalue of D^-1 K: its slowest mode has period n_l
    // cells on the periodic square, 2 n_l on the closed one (Neumann)
    lo = 0.9 * (1.0 - std::cos((c->box ? 1.0 : 2.0) * M_PI / nl)) / 2.0;
  } else {
    lo = 0.45 / (1.0 + c->diag_ratio * cf[1] * ih * ih / cf[0]);
  }
  const int steps = (l > 0) ? o.mg_coarse : o.mg_pre + o.mg_post;
  return cheb_coef<T>(lo, lmax_of(c, o), std::min(steps, MAXCHEB));
}

template <typename T>
TileArgs<T> tile_args(Level& L, const OpVals& A, int steps, const ChebCoef<T>& cc) {
  TileArgs<T> a;
  a.side = L.d.side;
  a.steps = steps;
  a.val = Sel<T>::v(A);
  a.dinv = Sel<T>::d(A);
  for (int k = 0; k < steps && k < TILE_MAXSTEPS; ++k) {
    a.c1[k] = cc.c1[k];
    a.c2[k] = cc.c2[k];
  }
  return a;
}

// Levels l..cut in one workgroup launch when they are periodic P1 levels
// small enough for LDS; false when they are not.
template <typename T>
bool vcycle_tail(chns_ctx* c, OpVals Level::*op, size_t l, size_t cut, const T* b, T* x,
                 const chns_solve_opts& o, hipStream_t s) {
  const int nlev = int(cut - l + 1);
  if (nlev > TAIL_MAXLEV || o.mg_pre > TAIL_MAXSM || o.mg_post > TAIL_MAXSM) return false;
  int sides[TAIL_MAXLEV];
  for (int t = 0; t < nlev; ++t) {
    sides[t] = c->lv[l + t].d.side;
    if (sides[t] <= 0) return false;
  }
  if (!tail_fits<T>(sides, nlev)) return false;
  TailArgs<T> a{};
  a.nlev = nlev;
  for (int t = 0; t < nlev; ++t) {
    const OpVals& A = c->lv[l + t].*op;
    a.side[t] = sides[t];
    a.val[t] = Sel<T>::v(A);
    a.dinv[t] = Sel<T>::d(A);
  }
  a.b = b;
  a.x = x;
  a.pre = o.mg_pre;
  a.post = o.mg_post;
  const ChebCoef<T> pre = cheb_coef<T>(lmax_of(c, o) / 4.0, lmax_of(c, o), o.mg_pre);
  const ChebCoef<T> post = cheb_coef<T>(lmax_of(c, o) / 4.0, lmax_of(c, o), o.mg_post);
  for (int k = 0; k < o.mg_pre; ++k) {
    a.pre_c1[k] = pre.c1[k];
    a.pre_c2[k] = pre.c2[k];
  }
  for (int k = 0; k < o.mg_post; ++k) {
    a.post_c1[k] = post.c1[k];
    a.post_c2[k] = post.c2[k];
  }
  a.coarse = cut_coef<T>(c, op, cut, o);
  vtail<T>(a, s);
  return true;
}

template <typename T>
void vcycle(chns_ctx* c, OpVals Level::*op, size_t l, size_t cut, const T* b, T* x,
            const chns_solve_opts& o, hipStream_t s);

// Levels l and l + 1 both smoothing, below the 64 x 64 tiles and above the
// tail: one launch for both down passes, the coarser levels, one for both up
// passes.  False when they do not qualify.
template <typename T>
bool vcycle_pair(chns_ctx* c, OpVals Level::*op, size_t l, size_t cut, const T* b, T* x,
                 const chns_solve_opts& o, hipStream_t s) {
  if (l + 1 >= cut || l + 2 >= c->lv.size()) return false;
  Level& L = c->lv[l];
  Level& G = c->lv[l + 1];
  Level& GG = c->lv[l + 2];
  const int side = L.d.side;
  if (side <= 0 || G.d.side != side / 2 || GG.d.side != side / 4) return false;
  // the paired kernels recompute wide halos: only for latency-bound levels
  if (tile_side<T>(side) == 64 || side > TILE64_MIN_SIDE / 2 || !tile2_fits(side, o.mg_pre, o.mg_post))
    return false;
  {  // the tail would start at l + 1: keep the level-by-level kernels
    const int nlev = int(cut - l);
    if (nlev <= TAIL_MAXLEV) {
      int sides[TAIL_MAXLEV];
      bool all = true;
      for (int t = 0; t < nlev; ++t) {
        sides[t] = c->lv[l + 1 + t].d.side;
        all = all && sides[t] > 0;
      }
      if (all && tail_fits<T>(sides, nlev)) return false;
    }
  }
  const OpVals& A = L.*op;
  const OpVals& AG = G.*op;
  Tile2Args<T> a;
  a.side = side;
  a.valf = Sel<T>::v(A);
  a.dinvf = Sel<T>::d(A);
  a.bf = b;
  a.valc = Sel<T>::v(AG);
  a.dinvc = Sel<T>::d(AG);
  a.bc = Sel<T>::b(G);
  a.xc = Sel<T>::t(G);
  const ChebCoef<T> pre = cheb_coef<T>(lmax_of(c, o) / 4.0, lmax_of(c, o), o.mg_pre);
  a.steps = o.mg_pre;
  for (int k = 0; k < o.mg_pre; ++k) {
    a.c1[k] = pre.c1[k];
    a.c2[k] = pre.c2[k];
  }
  a.xf = Sel<T>::t(L);
  a.bcc = Sel<T>::b(GG);
  vdown2<T>(a, s);
  // a cut level right below the pair is solved inside the up launch
  ChebCoef<T> cc{};
  bool cut_in_up = false;
  if (l + 2 == cut && GG.d.side > 0) {
    cc = cut_coef<T>(c, op, cut, o);
    cut_in_up = tile2_cut_fits(side, o.mg_post, cc.steps);
  }
  if (!cut_in_up) vcycle<T>(c, op, l + 2, cut, Sel<T>::b(GG), Sel<T>::x(GG), o, s);
  const ChebCoef<T> post = cheb_coef<T>(lmax_of(c, o) / 4.0, lmax_of(c, o), o.mg_post);
  a.steps = o.mg_post;
  for (int k = 0; k < o.mg_post; ++k) {
    a.c1[k] = post.c1[k];
    a.c2[k] = post.c2[k];
  }
  a.xinf = Sel<T>::t(L);
  a.xf = x;
  if (cut_in_up) {
    const OpVals& AGG = GG.*op;
    a.csteps = cc.steps;
    a.valcc = Sel<T>::v(AGG);
    a.dinvcc = Sel<T>::d(AGG);
    for (int k = 0; k < cc.steps; ++k) {
      a.cc1[k] = cc.c1[k];
      a.cc2[k] = cc.c2[k];
    }
  } else {
    a.e = Sel<T>::x(GG);
    a.bcc = nullptr;
  }
  vup2<T>(a, s);
  return true;
}

template <typename T>
void vcycle(chns_ctx* c, OpVals Level::*op, size_t l, size_t cut, const T* b, T* x,
            const chns_solve_opts& o, hipStream_t s) {
  Level& L = c->lv[l];
  const OpVals& A = L.*op;
  const double lmax = lmax_of(c, o);
  if (vcycle_tail<T>(c, op, l, cut, b, x, o, s)) return;
  if (l == cut) {
    const ChebCoef<T> cc = cut_coef<T>(c, op, l, o);
    if (L.d.side > 0 && tile_fits<T>(TILE_ZERO, L.d.side, cc.steps)) {
      TileArgs<T> ta = tile_args<T>(L, A, cc.steps, cc);
      ta.b = b;
      ta.x = x;
      vtile_at<T>(c, TILE_ZERO, ta, l == 0, s);
      return;
    }
    cheb_from_zero<T>(c, L, A, b, x, cc, s);
    return;
  }
  if (vcycle_pair<T>(c, op, l, cut, b, x, o, s)) return;
  if (L.d.side > 0 && tile_fits<T>(TILE_DOWN, L.d.side, o.mg_pre) &&
      tile_fits<T>(TILE_UP, L.d.side, o.mg_post)) {
    // two launches per level: pre-smoothing, residual and restriction in one,
    // coarse correction and post-smoothing in the other
    Level& G = c->lv[l + 1];
    TileArgs<T> dn = tile_args<T>(L, A, o.mg_pre, cheb_coef<T>(lmax / 4.0, lmax, o.mg_pre));
    dn.b = b;
    dn.x = Sel<T>::t(L);
    dn.bc = Sel<T>::b(G);
    vtile_at<T>(c, TILE_DOWN, dn, l == 0, s);
    vcycle<T>(c, op, l + 1, cut, Sel<T>::b(G), Sel<T>::x(G), o, s);
    TileArgs<T> up = tile_args<T>(L, A, o.mg_post, cheb_coef<T>(lmax / 4.0, lmax, o.mg_post));
    up.b = b;
    up.xin = Sel<T>::t(L);
    up.e = Sel<T>::x(G);
    up.x = x;
    vtile_at<T>(c, TILE_UP, up, l == 0, s);
    return;
  }
  const ChebCoef<T> pre = cheb_coef<T>(lmax / 4.0, lmax, o.mg_pre);
  if (L.d.side > 0 && o.mg_pre >= 2 && o.mg_post >= 1) {
    // fused: the first two pre-smoothing steps, and the coarse correction
    // with the first post-smoothing step; the result lands in x after
    // pre + post - 2 swaps
    const ChebCoef<T> post = cheb_coef<T>(lmax / 4.0, lmax, o.mg_post);
    T* cur = ((o.mg_pre - 2 + o.mg_post) % 2 == 0) ? x : Sel<T>::t(L);
    T* oth = (cur == x) ? Sel<T>::t(L) : x;
    T* d = Sel<T>::dd(L);
    const T* v = Sel<T>::v(A);
    const T* di = Sel<T>::d(A);
    cheb01<T, T>(L.d, v, b, di, pre.c2[0], pre.c1[1], pre.c2[1], d, cur, s);
    for (int k = 2; k < o.mg_pre; ++k) {
      cheb_sweep<T>(c, L, A, cur, b, d, pre.c1[k], pre.c2[k], oth, s);
      std::swap(cur, oth);
    }
    Level& G = c->lv[l + 1];
    T* r = Sel<T>::r(L);
    stencil<T, T>(L.d, v, ST_RESID, cur, b, nullptr, nullptr, T(0), T(0), r, s);
    spmv<T, T>(L.dR, Sel<T>::R(L), r, Sel<T>::b(G), T(1), T(0), s);
    vcycle<T>(c, op, l + 1, cut, Sel<T>::b(G), Sel<T>::x(G), o, s);
    pcheb<T, T>(L.d, v, cur, Sel<T>::x(G), b, di, post.c2[0], d, oth, s);
    std::swap(cur, oth);
    for (int k = 1; k < o.mg_post; ++k) {
      cheb_sweep<T>(c, L, A, cur, b, d, post.c1[k], post.c2[k], oth, s);
      std::swap(cur, oth);
    }
    return;
  }
  const int swaps_post = o.mg_post;
  // pre-smoothing from zero: result must end in `cur`, then the post steps
  // alternate; choose the start buffer so that the final iterate is `x`.
  T* cur = ((o.mg_pre - 1 + swaps_post) % 2 == 0) ? x : Sel<T>::t(L);
  T* oth = (cur == x) ? Sel<T>::t(L) : x;
  T* d = Sel<T>::dd(L);
  cheb0<T>(L.N, Sel<T>::d(A), b, pre.c2[0], d, cur, s);
  for (int k = 1; k < o.mg_pre; ++k) {
    cheb_sweep<T>(c, L, A, cur, b, d, pre.c1[k], pre.c2[k], oth, s);
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
      cheb_sweep<T>(c, L, A, cur, b, d, post.c1[k], post.c2[k], oth, s);
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

template <typename T> struct SelP2;
template <> struct SelP2<double> {
  static const double* v(const OpVals& o) { return o.v64; }
  static const double* d(const OpVals& o) { return o.d64; }
  static double* t(P2Level& L) { return L.t64; }
  static double* r(P2Level& L) { return L.r64; }
  static double* dd(P2Level& L) { return L.d64; }
  static double* e(P2Level& L) { return L.e64; }
  static double* corr(P2Level& L) { return L.c64; }
  static const double* P(P2Level& L) { return L.P64; }
  static const double* R(P2Level& L) { return L.R64; }
};
template <> struct SelP2<float> {
  static const float* v(const OpVals& o) { return o.v32; }
  static const float* d(const OpVals& o) { return o.d32; }
  static float* t(P2Level& L) { return L.t32; }
  static float* r(P2Level& L) { return L.r32; }
  static float* dd(P2Level& L) { return L.d32; }
  static float* e(P2Level& L) { return L.e32; }
  static float* corr(P2Level& L) { return L.c32; }
  static const float* P(P2Level& L) { return L.P32; }
  static const float* R(P2Level& L) { return L.R32; }
};

constexpr double LMAX_P2 = 2.3;  // bound of D^-1 A for P2 mass/stiffness combinations

// V-cycle of a velocity block: P2 level on the finest mesh, then the P1
// hierarchy of the same block (Galerkin through P1 -> P2 interpolation).
template <typename T>
void vcycle_p2(chns_ctx* c, OpVals P2Level::*op2, OpVals Level::*op1, const T* b, T* x,
               const chns_solve_opts& o, hipStream_t s) {
  P2Level& P = c->p2;
  Level& L0 = c->lv[0];
  const OpVals& A = P.*op2;
  const double lmax = LMAX_P2;
  const ChebCoef<T> pre = cheb_coef<T>(lmax / 4.0, lmax, o.mg_pre);
  T* cur = ((o.mg_pre - 1 + o.mg_post) % 2 == 0) ? x : SelP2<T>::t(P);
  T* oth = (cur == x) ? SelP2<T>::t(P) : x;
  T* d = SelP2<T>::dd(P);
  cheb0<T>(P.N4, SelP2<T>::d(A), b, pre.c2[0], d, cur, s);
  for (int k = 1; k < o.mg_pre; ++k) {
    sell_op<T, T>(P.d, SelP2<T>::v(A), ST_CHEB, cur, b, SelP2<T>::d(A), d, pre.c1[k], pre.c2[k], oth, s);
    std::swap(cur, oth);
  }
  T* r = SelP2<T>::r(P);
  sell_op<T, T>(P.d, SelP2<T>::v(A), ST_RESID, cur, b, nullptr, nullptr, T(0), T(0), r, s);
  spmv<T, T>(P.dR, SelP2<T>::R(P), r, Sel<T>::b(L0), T(1), T(0), s);
  const size_t cut = cut_level(c, coef_of(c, op1), o.mg_rho_cut);
  vcycle<T>(c, op1, 0, cut, Sel<T>::b(L0), Sel<T>::x(L0), o, s);
  spmv<T, T>(P.dP, SelP2<T>::P(P), Sel<T>::x(L0), cur, T(1), T(1), s);
  if (o.mg_post > 0) {
    const ChebCoef<T> post = cheb_coef<T>(lmax / 4.0, lmax, o.mg_post);
    for (int k = 0; k < o.mg_post; ++k) {
      sell_op<T, T>(P.d, SelP2<T>::v(A), ST_CHEB, cur, b, SelP2<T>::d(A), d, post.c1[k], post.c2[k],
                    oth, s);
      std::swap(cur, oth);
    }
  }
}

template <typename T>
void mg_solve_p2(chns_ctx* c, OpVals P2Level::*op2, OpVals Level::*op1, const T* b, T* x,
                 const chns_solve_opts& o, hipStream_t s) {
  P2Level& P = c->p2;
  vcycle_p2<T>(c, op2, op1, b, x, o, s);
  for (int k = 1; k < o.mg_cycles; ++k) {
    T* res = SelP2<T>::e(P);
    sell_op<T, T>(P.d, SelP2<T>::v(P.*op2), ST_RESID, x, b, nullptr, nullptr, T(0), T(0), res, s);
    T* corr = SelP2<T>::corr(P);
    vcycle_p2<T>(c, op2, op1, res, corr, o, s);
    axpby<T>(P.N4, T(1), corr, T(1), x, s);
  }
}

template <typename T>
void mean_zero(chns_ctx* c, int64_t n, T* x, hipStream_t s) {
  sum_partial<T>(n, x, c->red, s);
  sub_mean<T>(n, reduce_blocks(n), c->red, x, s);
}

// Pressure convection-diffusion Schur approximation: z = M_p^{-1} A_p K_p^{-1} r
// with K_p^{-1} on mean-zero pressures; on transposed operators the factors
// are applied in reverse order (the exact transpose, M_p and K_p symmetric).
template <typename T>
void pcd_apply(chns_ctx* c, const T* r, T* z, T* tmp1, T* tmp2, const chns_solve_opts& o,
               hipStream_t s) {
  Level& L0 = c->lv[0];
  const int N = c->N;
  if (c->transposed) {  // (M_p^{-1} A_p P0 K_p^{-1} P0)^T = P0 K_p^{-1} P0 A_p^T M_p^{-1}
    mg_solve<T>(c, &Level::Mp, r, tmp1, o, s);
    spmv<T, T>(L0.d, Sel<T>::v(L0.Ap), tmp1, tmp2, T(1), T(0), s);
    mean_zero<T>(c, N, tmp2, s);
    mg_solve<T>(c, &Level::Kp, tmp2, z, o, s);
    mean_zero<T>(c, N, z, s);
    return;
  }
  HIPCHK_VOID(hipMemcpyAsync(tmp1, r, N * sizeof(T), hipMemcpyDeviceToDevice, s));
  mean_zero<T>(c, N, tmp1, s);
  mg_solve<T>(c, &Level::Kp, tmp1, tmp2, o, s);
  mean_zero<T>(c, N, tmp2, s);
  spmv<T, T>(L0.d, Sel<T>::v(L0.Ap), tmp2, tmp1, T(1), T(0), s);
  mg_solve<T>(c, &Level::Mp, tmp1, z, o, s);
}

template <typename T>
void ns_precond_t(chns_ctx* c, const T* r, T* z, T* tmp1, T* tmp2, const chns_solve_opts& o,
                  hipStream_t s) {
  const int64_t N4 = 4 * int64_t(c->N);
  mg_solve_p2<T>(c, &P2Level::Vx, &Level::Vx, r, z, o, s);
  mg_solve_p2<T>(c, &P2Level::Vy, &Level::Vy, r + N4, z + N4, o, s);
  pcd_apply<T>(c, r + 2 * N4, z + 2 * N4, tmp1, tmp2, o, s);
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

// One V-cycle of op whose finest level takes the tiled down and up passes,
// with the FP64 boundary at that level: the right-hand side read from b64
// when given (else b), the result written to x64 times xs[0] when x64 is
// given (else to x).
template <typename T>
void vcycle_top(chns_ctx* c, OpVals Level::*op, size_t cut, const T* b, const double* b64, T* x,
                double* x64, const double* xs, const chns_solve_opts& o, hipStream_t s,
                const T* mval = nullptr) {
  Level& L = c->lv[0];
  Level& G = c->lv[1];
  const OpVals& A = L.*op;
  TileArgs<T> dn = tile_args<T>(L, A, o.mg_pre, cheb_coef<T>(lmax_of(c, o) / 4.0, lmax_of(c, o), o.mg_pre));
  dn.b = b;
  dn.b64 = b64;
  dn.x = Sel<T>::t(L);
  dn.bc = Sel<T>::b(G);
  vtile_at<T>(c, TILE_DOWN, dn, true, s);
  vcycle<T>(c, op, 1, cut, Sel<T>::b(G), Sel<T>::x(G), o, s);
  TileArgs<T> up = tile_args<T>(L, A, o.mg_post, cheb_coef<T>(lmax_of(c, o) / 4.0, lmax_of(c, o), o.mg_post));
  up.b = b;
  up.b64 = b64;
  up.xin = Sel<T>::t(L);
  up.e = Sel<T>::x(G);
  up.x = x;
  up.x64 = x64;
  up.xs = xs;
  up.mval = mval;  // when given, the pass writes M times the result
  vtile_at<T>(c, mval ? TILE_UPM : TILE_UP, up, true, s);
}

// Whether the cycles of a block (precision T) can take their FP64 input and
// write their FP64 output, times the output scale, inside the finest level's
// tiled launches: one cycle per inner solve, a finest level of side >= 1024
// (64 x 64 tiles in FP32, 32 x 32 in FP64; never paired), the mass-like
// inverses ((1,1) block of CH, the AC matrix) cut on the finest level, X not.
template <typename T>
bool fused_top(chns_ctx* c, int block, const chns_solve_opts& o) {
  const int side = c->lv[0].d.side;
  if (o.mg_cycles != 1 || side < TILE64_MIN_SIDE || c->lv.size() < 2) return false;
  const int z = std::min(o.mg_pre + o.mg_post, MAXCHEB);
  auto cut0 = [&](OpVals Level::*op) {
    return cut_level(c, coef_of(c, op), o.mg_rho_cut) == 0 && tile_fits<T>(TILE_ZERO, side, z);
  };
  if (block == CHNS_BLOCK_AC) return c->mesh.model != CHNS_MODEL_CH && cut0(&Level::AC);
  if (block != CHNS_BLOCK_CH) return false;
  return cut0(&Level::L) && cut_level(c, coef_of(c, &Level::X), o.mg_rho_cut) > 0 &&
         tile_fits<T>(TILE_DOWN, side, o.mg_pre) && tile_fits<T>(TILE_UP, side, o.mg_post);
}

// The block preconditioner with the boundary in the finest tiles (see
// fused_top): z = inv[0] P^{-1} r.
template <typename T>
void fused_precond(chns_ctx* c, int block, const chns_solve_opts& o, const double* r, const double* inv,
                   double* z, hipStream_t s) {
  const int N = c->N;
  Level& L0 = c->lv[0];
  const int z0 = std::min(o.mg_pre + o.mg_post, MAXCHEB);
  auto zero_cut = [&](OpVals Level::*op, const double* b, double* x) {
    TileArgs<T> a = tile_args<T>(L0, L0.*op, z0, cut_coef<T>(c, op, 0, o));
    a.b64 = b;
    a.x64 = x;
    a.xs = inv;
    vtile_at<T>(c, TILE_ZERO, a, true, s);
  };
  if (block == CHNS_BLOCK_AC) {
    zero_cut(&Level::AC, r, z);
    return;
  }
  T* t1 = std::is_same<T, double>::value ? (T*)c->w64a : (T*)c->w32a;
  T* t2 = std::is_same<T, double>::value ? (T*)c->w64b : (T*)c->w32b;
  const size_t cutX = cut_level(c, coef_of(c, &Level::X), o.mg_rho_cut);
  zero_cut(&Level::L, r, z);
  if (tile_fits<T>(TILE_UPM, L0.d.side, o.mg_post)) {
    // the first cycle's up pass writes M X^{-1} r2 directly
    vcycle_top<T>(c, &Level::X, cutX, nullptr, r + N, t2, nullptr, nullptr, o, s, Sel<T>::M(L0));
  } else {
    vcycle_top<T>(c, &Level::X, cutX, nullptr, r + N, t1, nullptr, nullptr, o, s);
    spmv<T, T>(L0.d, Sel<T>::M(L0), t1, t2, T(1), T(0), s);
  }
  vcycle_top<T>(c, &Level::X, cutX, t2, nullptr, nullptr, z + N, inv, o, s);
}

// Preconditioner of a block: z = inv[0] P^{-1} r (inv may be null: 1); r is
// not written.  The Krylov basis vector arrives unnormalised and its 1/|w|
// rides on the output (P is linear).  Where fused_top() holds the cycles read
// r and write the scaled z in the finest level's tiles; else through
// conversion (mixed precision) and scaling passes.
int precond_scaled(chns_ctx* c, int block, const chns_solve_opts& o, const double* r, const double* inv,
                   double* z, hipStream_t s) {
  const int N = c->N;
  int64_t n = 0;
  if (block == CHNS_BLOCK_CH) n = 2 * int64_t(N);
  else if (block == CHNS_BLOCK_AC && c->mesh.model != CHNS_MODEL_CH) n = N;
  else if (block == CHNS_BLOCK_NS && c->ternary) n = 9 * int64_t(N);
  else return fail(c, CHNS_EUNSUPPORTED, "block not available");
  const bool f64 = o.precision == CHNS_F64;
  if (f64 ? fused_top<double>(c, block, o) : fused_top<float>(c, block, o)) {
    if (f64) fused_precond<double>(c, block, o, r, inv, z, s);
    else fused_precond<float>(c, block, o, r, inv, z, s);
    HIPCHK(c, hipGetLastError());
    return CHNS_OK;
  }
  if (!f64) convert<double, float>(n, r, c->r32, s);
  if (block == CHNS_BLOCK_CH) {
    if (f64) ch_precond_t<double>(c, r, z, c->w64a, c->w64b, o, s);
    else ch_precond_t<float>(c, c->r32, c->z32, c->w32a, c->w32b, o, s);
  } else if (block == CHNS_BLOCK_AC) {
    if (f64) mg_solve<double>(c, &Level::AC, r, z, o, s);
    else mg_solve<float>(c, &Level::AC, c->r32, c->z32, o, s);
  } else {
    if (f64) ns_precond_t<double>(c, r, z, c->w64a, c->w64b, o, s);
    else ns_precond_t<float>(c, c->r32, c->z32, c->w32a, c->w32b, o, s);
  }
  if (f64) {
    if (inv) scale_by_inv(n, z, inv, z, s);
  } else {
    convert_out(n, c->z32, inv, z, s);
  }
  HIPCHK(c, hipGetLastError());
  return CHNS_OK;
}

int precond(chns_ctx* c, int block, const chns_solve_opts& o, const double* r, double* z,
            hipStream_t s) {
  return precond_scaled(c, block, o, r, nullptr, z, s);
}

int64_t block_size(chns_ctx* c, int block) {
  if (block == CHNS_BLOCK_CH) return 2 * int64_t(c->N);
  if (block == CHNS_BLOCK_AC) return c->N;
  if (block == CHNS_BLOCK_NS) return 9 * int64_t(c->N);
  return 0;
}

// y = alpha A x + beta u for a block operator (FP64), u = yin when given (not
// overlapping y), else y.
int apply_block(chns_ctx* c, int block, const double* x, double* y, double alpha, double beta,
                hipStream_t s, const double* yin = nullptr) {
  const auto& p = c->prm;
  Level& L0 = c->lv[0];
  if (yin && block != CHNS_BLOCK_CH) {  // the other blocks' products update y in place
    const int64_t n = block_size(c, block);
    HIPCHK(c, hipMemcpyAsync(y, yin, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    yin = nullptr;
  }
  if (block == CHNS_BLOCK_CH) {
    const double tg = p.tau * p.mobility, beta_ = c->beta_ch;
    const double* Lv = c->has_conv ? L0.L.v64 : L0.M;
    // values M, K (and L when C != 0), x and y of both rows; y read when beta != 0
    const double bytes = double(c->N) * (8 * (14 + (c->has_conv ? 7 : 0)) + 32 + (beta != 0.0 ? 16 : 0));
    timed(c, CHNS_KERNEL_CH_BLOCK, bytes, s, [&](LaunchEv ev) {
      ch_block<double, double>(L0.d, Lv, L0.K, L0.M, tg, -tg / beta_, x, alpha, beta, y, s, ev, yin);
    });
  } else if (block == CHNS_BLOCK_AC) {
    spmv<double, double>(L0.d, L0.AC.v64, x, y, alpha, beta, s);
  } else if (block == CHNS_BLOCK_NS && c->ternary) {
    spmv<double, double>(c->ns.d, c->ns.val, x, y, alpha, beta, s);
  } else {
    return fail(c, CHNS_EUNSUPPORTED, "block not available");
  }
  HIPCHK(c, hipGetLastError());
  return CHNS_OK;
}

// ------------------------------------------------------------------ FGMRES

constexpr int64_t KRYLOV_PAD = 640;  // doubles (5 KiB) between consecutive basis vectors

// Waits until a kernel on stream s has stored `tag` in slot[3] of pinned host
// memory (after the slot's values, behind a system-scope fence: they are then
// visible too).  Every few thousand polls it queries the stream, so that a
// failed launch ends the wait with its error, and a stream found idle without
// the tag is an error rather than a hang.
int wait_slot(chns_ctx* c, const double* slot, double tag, hipStream_t s) {
  const volatile double* t = slot + 3;
  for (uint32_t it = 1; *t != tag; ++it) {
    if ((it & 4095) == 0) {
      const hipError_t e = hipStreamQuery(s);
      if (e == hipSuccess) {
        if (*t == tag) break;
        return fail(c, CHNS_EHIP, "stream idle but the step's scalars were not written");
      }
      if (e != hipErrorNotReady) HIPCHK(c, e);
    }
    _mm_pause();
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  return CHNS_OK;
}

int fgmres(chns_ctx* c, int block, const double* b, double* x, const chns_solve_opts& o,
           chns_solve_info* info, hipStream_t s) {
  Krylov& K = c->kr;
  const int64_t n = block_size(c, block);
  const int m = o.restart;
  const int nblk = reduce_blocks(n);
  // basis vectors with stride n + KRYLOV_PAD: without the pad the vectors of a
  // large block sit a multiple of 16 MiB apart and the loads of one row of all
  // of them fall into the same HBM channel
  const int64_t ld = n + KRYLOV_PAD;
  DcgsState st;
  st.part = K.part;
  st.red = K.red;
  st.nrm_part = K.nrm_part;
  st.H = K.H;
  st.HR = K.HR;
  st.cs = K.cs;
  st.sn = K.sn;
  st.g = K.g;
  st.gp = K.gp;
  st.scal = K.scal;
  st.m = m;
  chns_solve_info inf{};
  HIPCHK(c, hipEventRecord(c->ev0, s));
  // ||b|| into scal[4]; the host reads it together with the first residual
  norm_partial(n, b, K.nrm_part, s);
  double* rslot = K.host + 8;  // restart read-back: beta, 1/beta, beta, tag, ||b||, -, -, tag
  const double btag = ++K.tag;
  norm_finish(nblk, K.nrm_part, K.scal + 4, nullptr, m, s, rslot + 4, btag);
  double rtag = 0.0;
  double tol = 0.0;
  int iters = 0;
  bool first = true, stop = false;
  // The host reads a restart's residual norm only after the cycle's first
  // Arnoldi step is enqueued (speculation), unless the previous cycle may
  // have converged (its last residual estimate was below the tolerance or is
  // still unread): then it waits for the norm first.  A speculative step whose
  // cycle turns out not to be needed changes nothing but the basis.
  bool spec = true;
  int unread = -1;  // host slot of a finished cycle's last step, not yet read
  auto check = [&]() -> int {
    TRY(wait_slot(c, rslot, rtag, s));
    if (first) {
      TRY(wait_slot(c, rslot + 4, btag, s));
      inf.bnorm = rslot[4];
      if (!std::isfinite(inf.bnorm)) return fail(c, CHNS_EINVAL, "right-hand side is not finite");
      tol = std::fmax(o.rtol * inf.bnorm, o.atol);
      inf.res0 = rslot[0];
      first = false;
    }
    const double beta = rslot[0];
    inf.res_true = beta;
    if (beta <= tol) {
      inf.converged = 1;
      stop = true;
    } else if (iters >= o.maxiter || !std::isfinite(beta)) {
      stop = true;
    } else {
      inf.restarts++;
    }
    return CHNS_OK;
  };
  while (true) {
    // V0 = b - A x, beta = ||V0||, g = beta e1
    TRY(apply_block(c, block, x, K.V, -1.0, 1.0, s, b));
    norm_partial(n, K.V, K.nrm_part, s);
    rtag = ++K.tag;
    norm_finish(nblk, K.nrm_part, K.scal, K.g, m, s, rslot, rtag);
    if (unread >= 0) {  // the previous cycle's last estimate
      TRY(wait_slot(c, K.host + 4 * unread, K.stag[unread], s));
      const double est = K.host[4 * unread];
      if (!(est > tol)) spec = false;
      unread = -1;
    }
    if (iters >= o.maxiter) spec = false;
    if (!spec) {
      TRY(check());
      if (stop) break;
    }
    scale_by_inv(n, K.V, K.scal + 1, K.V, s);
    // One-step lookahead: step j is enqueued before the host reads step
    // j-1's residual estimate, so the stream never drains at the check.  If
    // step j-1 turns out to be the last one, the speculative step j has only
    // finalised column j-1 (its Givens rotation and g) and the least squares
    // over k = j columns uses that final data.
    int k = 0;
    double hist[MAX_RESTART];  // residual estimates of this cycle, as read
    for (int j = 0; j < m; ++j) {
      double* vj = K.V + j * ld;
      double* vn = K.V + (j + 1) * ld;
      double* zj = K.Z + j * ld;
      // Step j - 1's estimate predicted from the last known one and the mean
      // reduction per step of the block's previous solve (else this cycle's
      // last ratio; the estimates of these systems alternate plateaus and
      // drops, so one ratio alone predicts badly): when it is likely to meet
      // the tolerance the host reads it before enqueuing step j, and if it
      // does, step j only closes column j - 1 (the DCGS2 correction and final
      // rotation the least squares needs) with w = 0 instead of a full
      // speculative step.
      bool checked = false, closing = false;
      if (j > 0) {
        const double last = j == 1 ? inf.res_true : hist[j - 2];
        double rate = K.rate[block];
        if (!(rate > 0.0) && j >= 3 && hist[j - 3] > 0.0) rate = hist[j - 2] / hist[j - 3];
        const double pred = rate > 0.0 ? last * rate : -1.0;
        if (pred >= 0.0 && pred <= 2.0 * tol) {
          TRY(wait_slot(c, K.host + 4 * ((j - 1) & 1), K.stag[(j - 1) & 1], s));
          ++iters;
          checked = true;
          const double* prev = K.host + 4 * ((j - 1) & 1);
          const double est = prev[0], hnext = prev[2];
          hist[j - 1] = est;
          closing = est <= tol || hnext == 0.0 || iters >= o.maxiter || !std::isfinite(est);
        }
      }
      // v_j is stored unnormalised (j > 0): its 1/|w| scales the preconditioner's
      // output and is applied on load by the two Gram-Schmidt passes, which
      // store v_j normalised
      const double* vsc = j > 0 ? K.scal + 1 : nullptr;
      st.vscale = vsc;
      // the CH operator and the dot pass share one launch where the group fits
      const bool fuse = !closing && block == CHNS_BLOCK_CH && ch_dots_fits(j);
      if (closing) {
        HIPCHK(c, hipMemsetAsync(vn, 0, size_t(n) * sizeof(double), s));
      } else {
        TRY(precond_scaled(c, block, o, vj, vsc, zj, s));
        if (!fuse) TRY(apply_block(c, block, zj, vn, 1.0, 0.0, s));
      }
      // DCGS2: one dot pass and one update pass over the basis (the previous
      // vector's reorthogonalisation rides along with w's projection); the
      // end-of-step scalars land in the pinned host slot
      const int kk0 = j < 16 ? j : 16;
      if (fuse) {
        const auto& p = c->prm;
        Level& L0 = c->lv[0];
        const double tg = p.tau * p.mobility;
        const double* Lv = c->has_conv ? L0.L.v64 : L0.M;
        // CH operator (values, z read, w written) and the dots of V_0..V_j-1, vt
        const double bytes = double(c->N) * (8 * (14 + (c->has_conv ? 7 : 0)) + 32) + 8.0 * n * (j + 1);
        timed(c, CHNS_KERNEL_CH_BLOCK, bytes, s, [&](LaunchEv ev) {
          ch_dcgs_dots(L0.d, Lv, L0.K, L0.M, tg, -tg / c->beta_ch, zj, K.V, ld, j, st, s, ev);
        });
      } else {
        timed(c, CHNS_KERNEL_DCGS_DOTS, 8.0 * n * (kk0 + 2), s,
              [&](LaunchEv ev) { dcgs_dots(n, K.V, ld, j, st, s, ev); });
      }
      double* slot = K.host + 4 * (j & 1);
      const double tag = K.stag[j & 1] = ++K.tag;
      timed(c, CHNS_KERNEL_DCGS_UPDATE, 8.0 * n * (j + 2 + (j > 0 ? 1 : 0) + 1), s,
            [&](LaunchEv ev) { dcgs_update(n, K.V, ld, j, st, slot, tag, s, ev); });
      HIPCHK(c, hipGetLastError());
      if (closing) {
        k = j;
        break;
      }
      if (j == 0 && spec) {
        TRY(check());
        if (stop) break;
      }
      if (j > 0 && !checked) {
        TRY(wait_slot(c, K.host + 4 * ((j - 1) & 1), K.stag[(j - 1) & 1], s));
        ++iters;
        const double* prev = K.host + 4 * ((j - 1) & 1);
        const double est = prev[0], hnext = prev[2];
        hist[j - 1] = est;
        if (est <= tol || hnext == 0.0 || iters >= o.maxiter || !std::isfinite(est)) {
          k = j;
          break;
        }
      }
      if (j == m - 1) {  // the cycle ends at its length: no wait for this step
        ++iters;
        k = m;
        unread = j & 1;
      }
    }
    if (stop) break;
    lsq_solve(k, m, K.HR, K.gp, K.y, s);
    xupdate(n, K.Z, ld, k, K.y, x, s);
    HIPCHK(c, hipGetLastError());
    spec = k == m;
  }
  if (iters > 0 && inf.res0 > 0.0 && inf.res_true > 0.0)
    K.rate[block] = std::pow(inf.res_true / inf.res0, 1.0 / iters);
  if (block == CHNS_BLOCK_NS) {
    // the pressure in L^2_0: zero integral, i.e. 1^T M p = 0 (the plain mean
    // on the periodic square, where every row of M sums to h^2)
    double* p = x + 8 * int64_t(c->N);
    if (c->pw) wmean_zero(c->N, c->pw, c->len * c->len, p, c->red, s);
    else mean_zero<double>(c, c->N, p, s);
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

// Taylor-Hood patterns, slot tables, P2 -> P1 transfer and reference tables.
int build_ternary_tables(chns_ctx* c) {
  const int N = c->N;
  const Elements& E = c->el;
  P2Level& P = c->p2;
  NSData& S = c->ns;
  Level& L0 = c->lv[0];
  P.N4 = 4 * N;
  P.csr = p2_pattern(E);
  P.sell = make_sell(P.csr, 64, 1);
  TRY(upload_sell(c, P.sell, P.d));
  TRY(upload(c, &P.diag, P.sell.diag));
  S.bcsr = b_pattern(E);
  S.bsell = make_sell(S.bcsr, 64, 1);
  TRY(upload_sell(c, S.bsell, S.db));
  S.csr = ns_pattern(E);
  S.sell = make_sell(S.csr, 64, 1);
  TRY(upload_sell(c, S.sell, S.d));
  if (c->box) {
    // no-slip walls: the P2 ids held at zero give identity rows, and no
    // other row couples to them (velocity blocks, B and B^T in the Oseen
    // operator); their right-hand side rows are zero
    const std::vector<char> f = p2_fixed_box(c->mesh.n);
    const int N4 = 4 * N;
    std::vector<int> z2, o2, zn, on, vf;
    for (int r = 0; r < P.csr.nrows; ++r)
      for (int q = P.csr.rowptr[r]; q < P.csr.rowptr[r + 1]; ++q) {
        const int col = P.csr.col[q];
        if (!f[r] && !f[col]) continue;
        (col == r ? o2 : z2).push_back(P.sell.csr2sell[q]);
      }
    auto vfixed = [&](int i) { return i < 2 * N4 && f[i % N4]; };
    for (int r = 0; r < S.csr.nrows; ++r)
      for (int q = S.csr.rowptr[r]; q < S.csr.rowptr[r + 1]; ++q) {
        const int col = S.csr.col[q];
        if (!vfixed(r) && !vfixed(col)) continue;
        (col == r ? on : zn).push_back(S.sell.csr2sell[q]);
      }
    for (int i = 0; i < 2 * N4; ++i)
      if (vfixed(i)) vf.push_back(i);
    for (auto* l : {&z2, &o2, &zn, &on, &vf})
      if (l->empty()) return fail(c, CHNS_EINVAL, "no-slip tables are empty");
    TRY(upload(c, &S.p2_zero, z2));
    TRY(upload(c, &S.p2_one, o2));
    TRY(upload(c, &S.ns_zero, zn));
    TRY(upload(c, &S.ns_one, on));
    TRY(upload(c, &S.vfix, vf));
    S.n_p2_zero = int64_t(z2.size());
    S.n_p2_one = int64_t(o2.size());
    S.n_ns_zero = int64_t(zn.size());
    S.n_ns_one = int64_t(on.size());
    S.n_vfix = int64_t(vf.size());
  }
  // element slot tables
  std::vector<int> s36(size_t(E.ne) * 36), sb(size_t(E.ne) * 36);
  for (int e = 0; e < E.ne; ++e) {
    const int* q = &E.p2[e * 6];
    const int* v = &E.v[e * 3];
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) s36[size_t(e) * 36 + i * 6 + j] = P.sell.csr2sell[P.csr.find(q[i], q[j])];
    for (int a = 0; a < 3; ++a)
      for (int cc = 0; cc < 2; ++cc)
        for (int k = 0; k < 6; ++k)
          sb[size_t(e) * 36 + a * 12 + cc * 6 + k] = S.bsell.csr2sell[S.bcsr.find(v[a], cc * 4 * N + q[k])];
  }
  TRY(upload(c, &S.eslot36, s36));
  TRY(upload(c, &S.eslotb, sb));
  // Oseen operator slots: source stream and slot
  std::vector<int8_t> kind(S.sell.slots(), int8_t(-1));
  std::vector<int> src(S.sell.slots(), 0);
  for (int r = 0; r < S.csr.nrows; ++r)
    for (int q = S.csr.rowptr[r]; q < S.csr.rowptr[r + 1]; ++q) {
      const int col = S.csr.col[q];
      const int slot = S.sell.csr2sell[q];
      if (r < 8 * N && col < 8 * N) {
        const int cr = r / (4 * N), cc = col / (4 * N);
        kind[slot] = int8_t(2 * cr + cc);
        src[slot] = P.sell.csr2sell[P.csr.find(r % (4 * N), col % (4 * N))];
      } else if (r < 8 * N) {  // B^T: velocity row r, pressure column
        kind[slot] = 4;
        src[slot] = S.bsell.csr2sell[S.bcsr.find(col - 8 * N, r)];
      } else {
        kind[slot] = 4;
        src[slot] = S.bsell.csr2sell[S.bcsr.find(r - 8 * N, col)];
      }
    }
  TRY(upload(c, &S.kind, kind));
  TRY(upload(c, &S.src, src));
  // P1 -> P2 on the finest mesh and the Galerkin map P2 -> P1
  p2_from_p1_prolongation(c->mesh.n, P.Pcsr, P.Pval, c->box);
  csr_transpose(P.Pcsr, P.Pval, P.Rcsr, P.Rval);
  P.Psell = make_sell(P.Pcsr, 64, 1);
  P.Rsell = make_sell(P.Rcsr, 64, 1);
  TRY(upload_sell(c, P.Psell, P.dP));
  TRY(upload_sell(c, P.Rsell, P.dR));
  auto sell_vals = [](const Sell& Sl, const Csr& A, const std::vector<double>& v) {
    std::vector<double> out(Sl.slots(), 0.0);
    for (int64_t q = 0; q < A.nnz(); ++q) out[Sl.csr2sell[q]] = v[q];
    return out;
  };
  auto pv = sell_vals(P.Psell, P.Pcsr, P.Pval), rv = sell_vals(P.Rsell, P.Rcsr, P.Rval);
  std::vector<float> pv32(pv.begin(), pv.end()), rv32(rv.begin(), rv.end());
  TRY(upload(c, &P.P64, pv));
  TRY(upload(c, &P.R64, rv));
  TRY(upload(c, &P.P32, pv32));
  TRY(upload(c, &P.R32, rv32));
  std::string gerr;
  GalerkinMap gm = make_galerkin(P.csr, P.sell, P.Pcsr, P.Pval, L0.csr, L0.sell, &gerr);
  if (!gerr.empty()) return fail(c, CHNS_EINVAL, gerr);
  TRY(upload(c, &P.gptr, gm.ptr));
  TRY(upload(c, &P.gsrc, gm.src));
  TRY(upload(c, &P.gw, gm.w));
  // reference tables
  const P2Tables T = p2_tables();
  std::vector<double> flat(sizeof(P2Tables) / sizeof(double));
  std::memcpy(flat.data(), &T, sizeof(P2Tables));
  TRY(upload(c, &S.tables, flat));
  const double* b = S.tables;
  S.tb.MM = b;
  S.tb.S = b + 36;
  S.tb.T3 = S.tb.S + 324;
  S.tb.T2 = S.tb.T3 + 648;
  S.tb.TB = S.tb.T2 + 108;
  S.tb.TI = S.tb.TB + 54;
  S.tb.MW = S.tb.TI + 18;
  // values and vectors
  const size_t ns2 = P.sell.slots(), n4 = P.N4;
  for (double** v : {&P.Mv, &P.J, &P.Kxx, &P.Kxy, &P.Kyx, &P.Kyy, &P.Mr}) TRY(dalloc(c, v, ns2));
  for (OpVals* o : {&P.Vx, &P.Vy}) {
    TRY(dalloc(c, &o->v64, ns2));
    TRY(dalloc(c, &o->v32, ns2));
    TRY(dalloc(c, &o->d64, n4));
    TRY(dalloc(c, &o->d32, n4));
  }
  for (double** v : {&P.b64, &P.x64, &P.t64, &P.r64, &P.d64, &P.e64, &P.c64}) TRY(dalloc(c, v, n4));
  for (float** v : {&P.b32, &P.x32, &P.t32, &P.r32, &P.d32, &P.e32, &P.c32}) TRY(dalloc(c, v, n4));
  TRY(dalloc(c, &S.B, S.bsell.slots()));
  TRY(dalloc(c, &S.val, S.sell.slots()));
  return CHNS_OK;
}

// The periodic cube: P1 levels n, n/2, ... (Kuhn tetrahedra, width-15 rows,
// stored columns), nested prolongation, Galerkin maps; the finest level's
// element tables (types and the 16 SELL slots of each tetrahedron, colour by
// colour) for the assembly.
int build_cube_levels(chns_ctx* c) {
  const int n = c->mesh.n;
  const bool box = c->box;
  // vertices: n^3 on the periodic cube, (n+1)^3 on the closed one
  auto nodes = [box](int k) { return box ? (k + 1) * (k + 1) * (k + 1) : k * k * k; };
  c->N = nodes(n);
  std::vector<int> sizes{n};
  while (sizes.back() % 2 == 0 && sizes.back() / 2 >= 4) sizes.push_back(sizes.back() / 2);
  c->lv.resize(sizes.size());
  for (size_t l = 0; l < sizes.size(); ++l) {
    Level& L = c->lv[l];
    L.n = sizes[l];
    L.N = nodes(L.n);
    Tets T = make_tets(L.n, box);
    L.csr = pattern_from_elements(L.N, L.N, T.ne, T.v.data(), 4, T.v.data(), 4);
    L.sell = box ? make_sell_p1_cube_box(L.csr, L.n) : make_sell_p1_cube(L.csr, L.n);
    if (!L.sell.uniform || L.sell.width_max != 15 || L.sell.cube != (box ? 0 : L.n))
      return fail(c, CHNS_EINVAL, "P1 pattern of the cube is not the uniform 15-point stencil");
    TRY(upload_sell(c, L.sell, L.d));
    TRY(upload(c, &L.diag, L.sell.diag));
    if (l == 0) {
      std::vector<int> slot(size_t(T.ne) * 16);
      for (int e = 0; e < T.ne; ++e)
        for (int a = 0; a < 4; ++a)
          for (int b = 0; b < 4; ++b) {
            const int q = L.csr.find(T.v[size_t(e) * 4 + a], T.v[size_t(e) * 4 + b]);
            if (q < 0) return fail(c, CHNS_EINVAL, "tetrahedron edge missing from the pattern");
            slot[size_t(e) * 16 + a * 4 + b] = L.sell.csr2sell[q];
          }
      TRY(upload(c, &c->etype, T.type));
      TRY(upload(c, &c->eslot, slot));
      std::copy(T.colour_ptr, T.colour_ptr + 49, c->colour_ptr3);
      if (box) TRY(upload(c, &c->topw, cube_top_weights(T, c->h)));
    }
  }
  return CHNS_OK;
}

int build(chns_ctx* c) {
  const int n = c->mesh.n;
  const bool box = c->box;
  if (c->dim3) TRY(build_cube_levels(c));
  else {
  // P1 nodes: n^2 on the periodic square, (n+1)^2 on the closed one
  auto nodes = [box](int m) { return box ? (m + 1) * (m + 1) : m * m; };
  c->N = nodes(n);
  // levels n, n/2, ... while even and the next size is >= 4
  std::vector<int> sizes{n};
  while (sizes.back() % 2 == 0 && sizes.back() / 2 >= 4) sizes.push_back(sizes.back() / 2);
  c->lv.resize(sizes.size());
  for (size_t l = 0; l < sizes.size(); ++l) {
    Level& L = c->lv[l];
    L.n = sizes[l];
    L.N = nodes(L.n);
    Elements E = make_elements(L.n, box);
    L.csr = pattern_from_elements(L.N, L.N, E.ne, E.v.data(), 3, E.v.data(), 3);
    L.sell = box ? make_sell_p1_box(L.csr, L.n) : make_sell_p1(L.csr, L.n);
    if (!L.sell.uniform || L.sell.width_max != 7 || L.sell.side != (box ? 0 : L.n))
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
      TRY(upload(c, &c->ep1, c->el.v));
      TRY(upload(c, &c->ep2, c->el.p2));
      TRY(upload(c, &c->etype, c->el.type));
      TRY(upload(c, &c->eslot, slot));
    }
  }
  }
  for (size_t l = 0; l + 1 < c->lv.size(); ++l) {
    Level& F = c->lv[l];
    Level& G = c->lv[l + 1];
    if (c->dim3) p1_prolongation3(F.n, F.Pcsr, F.Pval, box);
    else p1_prolongation(F.n, F.Pcsr, F.Pval, box);
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
  if (c->ternary) TRY(build_ternary_tables(c));
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
    if (c->ternary) {
      for (OpVals* o : {&L.Vx, &L.Vy}) {
        TRY(dalloc(c, &o->v64, ns));
        TRY(dalloc(c, &o->v32, ns));
        TRY(dalloc(c, &o->d64, N));
        TRY(dalloc(c, &o->d32, N));
      }
      for (OpVals* o : {&L.Kp, &L.Mp}) {
        TRY(dalloc(c, &o->d64, N));
        TRY(dalloc(c, &o->d32, N));
      }
      L.Kp.v64 = L.K;
      L.Kp.v32 = L.K32;
      L.Mp.v64 = L.M;
      L.Mp.v32 = L.M32;
      if (&L == &c->lv[0]) {
        TRY(dalloc(c, &L.Ap.v64, ns));
        TRY(dalloc(c, &L.Ap.v32, ns));
        TRY(dalloc(c, &L.Cw, ns));
        HIPCHK(c, hipMemset(L.Cw, 0, ns * sizeof(double)));
        TRY(dalloc(c, &L.Mrp, ns));
      }
    }
    for (double** v : {&L.b64, &L.x64, &L.t64, &L.r64, &L.e64, &L.d64}) TRY(dalloc(c, v, N));
    for (float** v : {&L.b32, &L.x32, &L.t32, &L.r32, &L.e32, &L.d32}) TRY(dalloc(c, v, N));
    HIPCHK(c, hipMemset(L.C, 0, ns * sizeof(double)));
    HIPCHK(c, hipMemset(L.C32, 0, ns * sizeof(float)));
  }
  {  // table of the fused operator formation
    std::vector<FormLevel> tab;
    int64_t at = 0;
    for (auto& L : c->lv) {
      FormLevel f;
      f.begin = at;
      f.ns = L.sell.slots();
      f.N = L.N;
      f.diag = L.diag;
      f.M = L.M;
      f.K = L.K;
      f.C = L.C;
      int o = 0;
      for (OpVals* v : {&L.L, &L.X, &L.AC}) {
        f.v64[o] = v->v64;
        f.v32[o] = v->v32;
        f.d64[o] = v->d64;
        f.d32[o] = v->d32;
        ++o;
      }
      tab.push_back(f);
      at += f.ns + f.N;
    }
    TRY(upload(c, &c->form_tab, tab));
    c->form_total = at;
  }
  const size_t N1 = size_t(c->N), N2 = 2 * N1;
  const size_t NB = c->ternary ? 9 * N1 : N2;  // largest block
  for (double** v : {&c->w64a, &c->w64b, &c->w64c, &c->w64d, &c->rhs_ac, &c->xac, &c->fs})
    TRY(dalloc(c, v, N1));
  for (double** v : {&c->rhs_ch, &c->xch}) TRY(dalloc(c, v, (c->quat ? 3 : 2) * N2));
  if (c->ternary) {
    for (double** v : {&c->rhs_ns, &c->xns}) TRY(dalloc(c, v, 9 * N1));
    TRY(dalloc(c, &c->rho1, N1));
    TRY(dalloc(c, &c->rho2, 4 * N1));
    TRY(dalloc(c, &c->vprev, 8 * N1));
    TRY(dalloc(c, &c->pic, 2 * 256 + 2));
  }
  for (float** v : {&c->r32, &c->z32}) TRY(dalloc(c, v, NB));
  for (float** v : {&c->w32a, &c->w32b, &c->w32c}) TRY(dalloc(c, v, N1));
  TRY(dalloc(c, &c->red, 1024));
  TRY(dalloc(c, &c->diag, NDIAG));
  if (c->ternary) {
    // slots of the transposed entries on the finest P1 and P2 patterns (both
    // symmetric); padding slots map to themselves
    std::string terr;
    auto tmap = [&terr](const Csr& A, const Sell& S) {
      std::vector<int> t(S.slots());
      for (int64_t q = 0; q < S.slots(); ++q) t[q] = int(q);
      for (int r = 0; r < A.nrows; ++r)
        for (int p = A.rowptr[r]; p < A.rowptr[r + 1]; ++p) {
          const int pt = A.find(A.col[p], r);
          if (pt < 0) {
            terr = "pattern is not symmetric";
            continue;
          }
          t[S.csr2sell[p]] = S.csr2sell[pt];
        }
      return t;
    };
    const std::vector<int> t1 = tmap(c->lv[0].csr, c->lv[0].sell), t2 = tmap(c->p2.csr, c->p2.sell);
    if (!terr.empty()) return fail(c, CHNS_EINVAL, terr);
    TRY(upload(c, &c->tslot1, t1));
    TRY(upload(c, &c->tslot2, t2));
    TRY(dalloc(c, &c->tbuf, size_t(std::max<int64_t>(c->lv[0].sell.slots(), c->p2.sell.slots()))));
    AdjData& A = c->adj;
    TRY(dalloc(c, &A.eta, 2 * N2));
    TRY(dalloc(c, &A.zeta, N1));
    TRY(dalloc(c, &A.xi, 9 * N1));
    TRY(dalloc(c, &A.rhs, 9 * N1));
    for (double*& v : A.v) TRY(dalloc(c, &v, N1));
    TRY(dalloc(c, &A.q, N1));
    TRY(dalloc(c, &A.gmu, N1));
    TRY(dalloc(c, &A.F, 8 * N1));
    TRY(dalloc(c, &A.part, 3 * size_t(ADJ_NBLK)));
    TRY(dalloc(c, &A.acc, 4));
  }
  // Krylov workspace, sized for the largest block
  Krylov& K = c->kr;
  K.nmax = int64_t(NB) + KRYLOV_PAD;
  TRY(dalloc(c, &K.V, size_t(MAX_RESTART + 1) * K.nmax));
  TRY(dalloc(c, &K.Z, size_t(MAX_RESTART) * K.nmax));
  TRY(dalloc(c, &K.H, size_t(MAX_RESTART + 1) * MAX_RESTART));
  TRY(dalloc(c, &K.cs, MAX_RESTART + 1));
  TRY(dalloc(c, &K.sn, MAX_RESTART + 1));
  TRY(dalloc(c, &K.g, MAX_RESTART + 2));
  TRY(dalloc(c, &K.y, MAX_RESTART + 1));
  TRY(dalloc(c, &K.scal, 8));
  TRY(dalloc(c, &K.part, size_t(1024) * (2 * MAX_RESTART + 4)));
  TRY(dalloc(c, &K.HR, size_t(MAX_RESTART + 1) * MAX_RESTART));
  TRY(dalloc(c, &K.gp, MAX_RESTART + 2));
  TRY(dalloc(c, &K.red, 2 * MAX_RESTART + 4));
  TRY(dalloc(c, &K.nrm_part, 1024));
  HIPCHK(c, hipHostMalloc((void**)&K.host, 16 * sizeof(double), hipHostMallocCoherent));
  std::memset(K.host, 0, 16 * sizeof(double));
  HIPCHK(c, hipEventCreate(&c->ev0));
  HIPCHK(c, hipEventCreate(&c->ev1));
  // M and K on the finest level by coloured scatter, then Galerkin down
  hipStream_t s = nullptr;
  Level& L0 = c->lv[0];
  TRY(assemble_base(c, 0, L0.M, nullptr, s));
  TRY(assemble_base(c, 1, L0.K, nullptr, s));
  galerkin_down(c, &Level::M, &Level::M32, s);
  galerkin_down(c, &Level::K, &Level::K32, s);
  if (c->ternary) {
    for (auto& L : c->lv) {
      diag_inverse(L.N, L.diag, L.K, L.Kp.d64, L.Kp.d32, s);
      diag_inverse(L.N, L.diag, L.M, L.Mp.d64, L.Mp.d32, s);
    }
    P2Level& P = c->p2;
    const int64_t ns2 = P.sell.slots();
    HIPCHK(c, hipMemsetAsync(P.Mv, 0, ns2 * sizeof(double), s));
    HIPCHK(c, hipMemsetAsync(P.J, 0, ns2 * sizeof(double), s));
    HIPCHK(c, hipMemsetAsync(c->ns.B, 0, c->ns.bsell.slots() * sizeof(double), s));
    MuGrad none{{nullptr, nullptr, nullptr}, 0.0};
    double* mo[1] = {P.Mv};
    for (int col = 0; col < 8; ++col) {
      const int e0 = c->el.colour_ptr[col], e1 = c->el.colour_ptr[col + 1];
      assemble_p2(0, e0, e1, c->ep1, c->ep2, c->etype, c->ns.eslot36, c->h, c->ns.tb, 0.0,
                  nullptr, 0.0, 4 * int64_t(c->N), none, mo, s);
      assemble_b(e0, e1, c->etype, c->ns.eslotb, c->h, c->ns.tb, c->ns.B, s);
    }
    TRY(assemble_sym_stiffness(c, s));
    TRY(uniform_density(c, s));
    if (c->box) {  // row sums of M: the weights of the pressure's mean on the closed square
      TRY(dalloc(c, &c->pw, size_t(c->N)));
      fill(c->N, 1.0, c->w64a, s);
      spmv<double, double>(L0.d, L0.M, c->w64a, c->pw, 1.0, 0.0, s);
    }
  }
  TRY(form_operators(c, s));
  HIPCHK(c, hipDeviceSynchronize());
  return CHNS_OK;
}

void release(chns_ctx* c) {
  if (!c) return;
  for (void* p : c->allocs) {
    if (c->free_)
      c->free_(p, c->alloc_ctx);
    else
      (void)hipFree(p);
  }
  c->allocs.clear();
  if (c->kr.host) (void)hipHostFree(c->kr.host);
  for (auto& e : c->ledger.ev) (void)hipEventDestroy(e);
  c->ledger.ev.clear();
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
}

const DSell* op_pattern(chns_ctx* c, int op) {
  if (op >= CHNS_OP_M && op <= CHNS_OP_L) return &c->lv[0].d;
  return nullptr;
}

// Ternary right-hand sides: two CH phases, AC, and the Oseen momentum rows
// (rho/tau) M v^k + F^k (pressure rows zero); fs = d f / d phi_s at level k.
int ternary_rhs(chns_ctx* c, const chns_fields* in, double* rhs_ch, double* rhs_ac, double* rhs_ns,
                double* fs, hipStream_t s) {
  const auto& p = c->prm;
  const int N = c->N;
  const double beta = p.eps * p.eps;
  Level& L0 = c->lv[0];
  rhs_ternary(L0.d, L0.M, in->phi[0], in->phi[1], in->Phi_v, -(p.tau * p.mobility / beta),
              -p.tau * p.evap_rate, pot_coef(p), rhs_ch, rhs_ch + 2 * int64_t(N), rhs_ac, fs, s);
  P2Level& P = c->p2;
  const int64_t N4 = 4 * int64_t(N);
  // (rho/tau) M v^k, or M_rho v^k / tau with the weighted mass of chns_set_density
  const double cm = p.var_density ? 1.0 / p.tau : p.rho / p.tau;
  const double* Mvel = p.var_density ? P.Mr : P.Mv;
  spmv<double, double>(P.d, Mvel, in->vel, rhs_ns, cm, 0.0, s);
  spmv<double, double>(P.d, Mvel, in->vel + N4, rhs_ns + N4, cm, 0.0, s);
  HIPCHK(c, hipMemsetAsync(rhs_ns + 2 * N4, 0, N * sizeof(double), s));
  for (int col = 0; col < 8; ++col)
    korteweg(c->el.colour_ptr[col], c->el.colour_ptr[col + 1], c->ep1, c->ep2, c->etype,
             c->h, c->ns.tb, in->phi[0], in->phi[1], nullptr, in->Phi_v, KorBeta{{beta, beta, beta, 0.0}, beta},
             N4, rhs_ns, s);
  if (c->box) set_slots(c->ns.n_vfix, c->ns.vfix, 0.0, rhs_ns, nullptr, s);  // no-slip rows
  HIPCHK(c, hipGetLastError());
  return CHNS_OK;
}

int chns_solve_block(chns_ctx* c, int block, const double* b, double* x, const chns_solve_opts& o,
                     chns_solve_info** info, int& worst, hipStream_t s);

// ||v - w||_2 / ||v||_2 for the velocity part of the Oseen unknown (read back).
int velocity_change(chns_ctx* c, const double* w, double* out, hipStream_t s) {
  double nrm[2];
  diff_norms(8 * int64_t(c->N), c->xns, w, c->pic, c->pic + 512, s);
  HIPCHK(c, hipMemcpyAsync(nrm, c->pic + 512, sizeof(nrm), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  *out = nrm[1] > 0.0 ? nrm[0] / nrm[1] : 0.0;
  return CHNS_OK;
}

// Picard passes of the Oseen solve: solve m convects with the velocity of
// solve m - 1 (mu and rho at level k, same right-hand side, warm start), until
// the relative change of the velocity is <= ns_picard_tol or ns_picard solves
// are made.  Their reports are merged into the first solve's (rec).
int picard_passes(chns_ctx* c, const chns_fields& cur, const double* const* mu3, const chns_solve_opts& o,
                  chns_solve_info* rec, int& worst, hipStream_t s) {
  const size_t vbytes = 8 * size_t(c->N) * sizeof(double);
  double change = 0.0;
  TRY(velocity_change(c, cur.vel, &change, s));
  int passes = 1;
  for (int m = 1; m < c->prm.ns_picard; ++m) {
    HIPCHK(c, hipMemcpyAsync(c->vprev, c->xns, vbytes, hipMemcpyDeviceToDevice, s));
    TRY(assemble_ternary_conv(c, c->vprev, mu3, false, s));
    TRY(form_ternary(c, s));
    chns_solve_info inf{};
    chns_solve_info* ip = &inf;
    TRY(chns_solve_block(c, CHNS_BLOCK_NS, c->rhs_ns, c->xns, o, &ip, worst, s));
    ++passes;
    TRY(velocity_change(c, c->vprev, &change, s));
    if (rec) {
      rec->iters += inf.iters;
      rec->restarts += inf.restarts;
      rec->converged = rec->converged && inf.converged;
      if (inf.status != CHNS_OK) rec->status = inf.status;
      rec->bnorm = inf.bnorm;
      rec->res0 = inf.res0;
      rec->res_true = inf.res_true;
      rec->ms += inf.ms;
    }
    if (change <= c->prm.ns_picard_tol) break;
  }
  if (rec) {
    rec->passes = passes;
    rec->change = change;
  }
  return CHNS_OK;
}

// One ternary step from `cur` into `out` (all outputs written at the end, so
// the two field sets may coincide).
int ternary_step(chns_ctx* c, const chns_fields& cur, const chns_fields* out,
                 const chns_solve_opts& o, chns_solve_info** info, int& worst, hipStream_t s) {
  const int N = c->N;
  const size_t bytes = size_t(N) * sizeof(double);
  const double beta = c->prm.eps * c->prm.eps;
  const double* mu3[3] = {cur.mu[0], cur.mu[1], cur.mu[2]};
  if (c->prm.var_density) TRY(set_density(c, cur.phi[0], cur.phi[1], s));
  TRY(chns_assemble(c, cur.vel, mu3, s));
  TRY(ternary_rhs(c, &cur, c->rhs_ch, c->rhs_ac, c->rhs_ns, c->fs, s));
  double* xch = c->xch;
  for (int ph = 0; ph < 2; ++ph) {
    HIPCHK(c, hipMemcpyAsync(xch + 2 * ph * size_t(N), cur.phi[ph], bytes, hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipMemcpyAsync(xch + (2 * ph + 1) * size_t(N), cur.mu[ph], bytes, hipMemcpyDeviceToDevice, s));
  }
  HIPCHK(c, hipMemcpyAsync(c->xac, cur.Phi_v, bytes, hipMemcpyDeviceToDevice, s));
  HIPCHK(c, hipMemcpyAsync(c->xns, cur.vel, 8 * bytes, hipMemcpyDeviceToDevice, s));
  HIPCHK(c, hipMemcpyAsync(c->xns + 8 * size_t(N), cur.p, bytes, hipMemcpyDeviceToDevice, s));
  TRY(chns_solve_block(c, CHNS_BLOCK_CH, c->rhs_ch, xch, o, info, worst, s));
  TRY(chns_solve_block(c, CHNS_BLOCK_CH, c->rhs_ch + 2 * size_t(N), xch + 2 * size_t(N), o, info, worst, s));
  TRY(chns_solve_block(c, CHNS_BLOCK_AC, c->rhs_ac, c->xac, o, info, worst, s));
  chns_solve_info* ns_rec = (info && *info) ? *info : nullptr;  // the Oseen solve's report
  TRY(chns_solve_block(c, CHNS_BLOCK_NS, c->rhs_ns, c->xns, o, info, worst, s));
  if (c->prm.ns_picard > 1) TRY(picard_passes(c, cur, mu3, o, ns_rec, worst, s));
  if (c->box) set_slots(c->ns.n_vfix, c->ns.vfix, 0.0, c->xns, nullptr, s);  // walls exactly at rest
  for (int ph = 0; ph < 2; ++ph) {
    HIPCHK(c, hipMemcpyAsync(out->phi[ph], xch + 2 * ph * size_t(N), bytes, hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipMemcpyAsync(out->mu[ph], xch + (2 * ph + 1) * size_t(N), bytes, hipMemcpyDeviceToDevice, s));
  }
  HIPCHK(c, hipMemcpyAsync(out->Phi_v, c->xac, bytes, hipMemcpyDeviceToDevice, s));
  HIPCHK(c, hipMemcpyAsync(out->vel, c->xns, 8 * bytes, hipMemcpyDeviceToDevice, s));
  HIPCHK(c, hipMemcpyAsync(out->p, c->xns + 8 * size_t(N), bytes, hipMemcpyDeviceToDevice, s));
  // closure: phi_s = 1 - phi_p - phi_N; mu_s = f_s'(level k) + beta M^{-1} K phi_s
  Level& L0 = c->lv[0];
  one_minus_sum(N, out->phi[0], out->phi[1], c->w64d, s);
  spmv<double, double>(L0.d, L0.K, c->w64d, c->w64a, 1.0, 0.0, s);
  cheb_from_zero<double>(c, L0, L0.Mp, c->w64a, c->w64b, cheb_coef<double>(0.49, 2.01, 40), s);
  axpy_into(N, beta, c->w64b, c->fs, out->mu[2], s);
  HIPCHK(c, hipGetLastError());
  return CHNS_OK;
}

// Quaternary right-hand sides: three CH blocks (polymer, NFA, solvent, each
// with its own beta), the AC block, the Oseen momentum rows with the Korteweg
// load of all four phases, and f_a (the air's unreduced derivative) into fa.
int quaternary_rhs(chns_ctx* c, const chns_fields* in, double* rhs_ch, double* rhs_ac, double* rhs_ns,
                   double* fa, hipStream_t s) {
  const auto& p = c->prm;
  const int N = c->N;
  const double tg = p.tau * p.mobility, bv = p.eps * p.eps;
  Level& L0 = c->lv[0];
  const Coef3 cmu{{-tg / p.beta_phase[0], -tg / p.beta_phase[1], -tg / p.beta_phase[2]}};
  rhs_quaternary(L0.d, L0.M, in->phi[0], in->phi[1], in->phi[2], in->Phi_v, cmu, -p.tau * p.evap_rate, rhs_ch,
                 rhs_ac, fa, s);
  P2Level& P = c->p2;
  const int64_t N4 = 4 * int64_t(N);
  const double cm = p.rho / p.tau;
  spmv<double, double>(P.d, P.Mv, in->vel, rhs_ns, cm, 0.0, s);
  spmv<double, double>(P.d, P.Mv, in->vel + N4, rhs_ns + N4, cm, 0.0, s);
  HIPCHK(c, hipMemsetAsync(rhs_ns + 2 * N4, 0, N * sizeof(double), s));
  const KorBeta kb{{p.beta_phase[0], p.beta_phase[1], p.beta_phase[2], p.beta_phase[3]}, bv};
  for (int col = 0; col < 8; ++col)
    korteweg(c->el.colour_ptr[col], c->el.colour_ptr[col + 1], c->ep1, c->ep2, c->etype, c->h, c->ns.tb,
             in->phi[0], in->phi[1], in->phi[2], in->Phi_v, kb, N4, rhs_ns, s);
  if (c->box) set_slots(c->ns.n_vfix, c->ns.vfix, 0.0, rhs_ns, nullptr, s);  // no-slip rows
  HIPCHK(c, hipGetLastError());
  return CHNS_OK;
}

// The CH block's beta (the second row's -(tau g / beta) M and the matching
// factor X): re-form the operators on every level when it changes.
int set_beta_ch(chns_ctx* c, double beta, hipStream_t s) {
  if (beta == c->beta_ch) return CHNS_OK;
  c->beta_ch = beta;
  for (double& r : c->kr.rate) r = -1.0;  // the rate predictor belongs to the other system
  return form_operators(c, s);
}

// One quaternary step: three CH solves (each phase's beta), AC, Oseen (with
// Picard passes when asked), then the air's closure mu_a = f_a^k + beta_a
// M^{-1} K phi_a^{k+1} with phi_a = 1 - phi_p - phi_N - phi_s (eq. (airdisc)).
// The CH operators are left formed with the polymer's beta.
int quaternary_step(chns_ctx* c, const chns_fields& cur, const chns_fields* out, const chns_solve_opts& o,
                    chns_solve_info** info, int& worst, hipStream_t s) {
  const auto& p = c->prm;
  const int N = c->N;
  const size_t bytes = size_t(N) * sizeof(double);
  const double* mu4[4] = {cur.mu[0], cur.mu[1], cur.mu[2], cur.mu[3]};
  TRY(chns_assemble(c, cur.vel, mu4, s));
  TRY(quaternary_rhs(c, &cur, c->rhs_ch, c->rhs_ac, c->rhs_ns, c->fs, s));
  double* xch = c->xch;
  for (int ph = 0; ph < 3; ++ph) {
    HIPCHK(c, hipMemcpyAsync(xch + 2 * ph * size_t(N), cur.phi[ph], bytes, hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipMemcpyAsync(xch + (2 * ph + 1) * size_t(N), cur.mu[ph], bytes, hipMemcpyDeviceToDevice, s));
  }
  HIPCHK(c, hipMemcpyAsync(c->xac, cur.Phi_v, bytes, hipMemcpyDeviceToDevice, s));
  HIPCHK(c, hipMemcpyAsync(c->xns, cur.vel, 8 * bytes, hipMemcpyDeviceToDevice, s));
  HIPCHK(c, hipMemcpyAsync(c->xns + 8 * size_t(N), cur.p, bytes, hipMemcpyDeviceToDevice, s));
  for (int ph = 0; ph < 3; ++ph) {
    TRY(set_beta_ch(c, p.beta_phase[ph], s));
    TRY(chns_solve_block(c, CHNS_BLOCK_CH, c->rhs_ch + 2 * ph * size_t(N), xch + 2 * ph * size_t(N), o, info,
                         worst, s));
  }
  TRY(set_beta_ch(c, p.beta_phase[0], s));
  TRY(chns_solve_block(c, CHNS_BLOCK_AC, c->rhs_ac, c->xac, o, info, worst, s));
  chns_solve_info* ns_rec = (info && *info) ? *info : nullptr;
  TRY(chns_solve_block(c, CHNS_BLOCK_NS, c->rhs_ns, c->xns, o, info, worst, s));
  if (p.ns_picard > 1) TRY(picard_passes(c, cur, mu4, o, ns_rec, worst, s));
  if (c->box) set_slots(c->ns.n_vfix, c->ns.vfix, 0.0, c->xns, nullptr, s);  // walls exactly at rest
  for (int ph = 0; ph < 3; ++ph) {
    HIPCHK(c, hipMemcpyAsync(out->phi[ph], xch + 2 * ph * size_t(N), bytes, hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipMemcpyAsync(out->mu[ph], xch + (2 * ph + 1) * size_t(N), bytes, hipMemcpyDeviceToDevice, s));
  }
  HIPCHK(c, hipMemcpyAsync(out->Phi_v, c->xac, bytes, hipMemcpyDeviceToDevice, s));
  HIPCHK(c, hipMemcpyAsync(out->vel, c->xns, 8 * bytes, hipMemcpyDeviceToDevice, s));
  HIPCHK(c, hipMemcpyAsync(out->p, c->xns + 8 * size_t(N), bytes, hipMemcpyDeviceToDevice, s));
  Level& L0 = c->lv[0];
  one_minus_sum(N, out->phi[0], out->phi[1], c->w64c, s);                 // 1 - p - n
  axpby<double>(N, -1.0, out->phi[2], 1.0, c->w64c, s);                    // - s
  spmv<double, double>(L0.d, L0.K, c->w64c, c->w64a, 1.0, 0.0, s);
  cheb_from_zero<double>(c, L0, L0.Mp, c->w64a, c->w64b, cheb_coef<double>(0.49, 2.01, 40), s);
  axpy_into(N, p.beta_phase[3], c->w64b, c->fs, out->mu[3], s);
  HIPCHK(c, hipGetLastError());
  return CHNS_OK;
}

// Adjoint of one ternary step (differentiation form).  With the transposed
// operators of state k: the closure adjoint q = beta K M^{-1} nu_s, the two CH
// solves A^T eta_i = [lambda_phi_i - q; lambda_mu_i], the AC solve
// A_ac^T zeta = lambda_Phi and the Oseen solve A^T xi = [lambda_v; 0]; then
// the nodal Hessian terms of the explicit densities, the element
// vector-Jacobian products of the convection, Oseen-convection and Korteweg
// forms, and the parameter-derivative integrals accumulated in adj.acc.
int ternary_adjoint(chns_ctx* c, const chns_fields& in, const chns_fields& out, const chns_fields& lo,
                    const chns_fields& li, const chns_solve_opts& o, chns_solve_info** info,
                    int& worst, hipStream_t s) {
  const auto& p = c->prm;
  const int N = c->N;
  const int64_t N2 = 2 * int64_t(N), N4 = 4 * int64_t(N);
  const size_t bytes = size_t(N) * sizeof(double);
  const double beta = p.eps * p.eps;
  AdjData& A = c->adj;
  Level& L0 = c->lv[0];
  P2Level& P = c->p2;
  const double h = c->h;
  const double* mu3[3] = {in.mu[0], in.mu[1], in.mu[2]};
  TRY(assemble_ops(c, in.vel, mu3, true, s));
  cheb_from_zero<double>(c, L0, L0.Mp, lo.mu[2], c->w64a, cheb_coef<double>(0.49, 2.01, 40), s);
  spmv<double, double>(L0.d, L0.K, c->w64a, A.q, beta, 0.0, s);
  for (int i = 0; i < 2; ++i) {
    double* eta = A.eta + i * N2;
    axpy_into(N, -1.0, A.q, lo.phi[i], A.rhs, s);
    HIPCHK(c, hipMemcpyAsync(A.rhs + N, lo.mu[i], bytes, hipMemcpyDeviceToDevice, s));
    HIPCHK(c, hipMemsetAsync(eta, 0, 2 * bytes, s));
    TRY(chns_solve_block(c, CHNS_BLOCK_CH, A.rhs, eta, o, info, worst, s));
  }
  HIPCHK(c, hipMemsetAsync(A.zeta, 0, bytes, s));
  TRY(chns_solve_block(c, CHNS_BLOCK_AC, lo.Phi_v, A.zeta, o, info, worst, s));
  HIPCHK(c, hipMemcpyAsync(A.rhs, lo.vel, 8 * bytes, hipMemcpyDeviceToDevice, s));
  HIPCHK(c, hipMemsetAsync(A.rhs + 8 * int64_t(N), 0, bytes, s));
  // closed square: the step holds the no-slip unknowns at zero, so their
  // entries of lambda^{k+1} act on nothing (identity rows, zero right-hand side)
  if (c->box) set_slots(c->ns.n_vfix, c->ns.vfix, 0.0, A.rhs, nullptr, s);
  HIPCHK(c, hipMemsetAsync(A.xi, 0, 9 * bytes, s));
  TRY(chns_solve_block(c, CHNS_BLOCK_NS, A.rhs, A.xi, o, info, worst, s));
  // M and K products of the CH and AC adjoint solutions
  const double* src[10] = {A.eta, A.eta + N2, A.eta + N, A.eta + N2 + N, A.eta, A.eta + N2,
                           A.eta + N, A.eta + N2 + N, A.zeta, A.zeta};
  for (int k = 0; k < 10; ++k) {
    const bool useK = (k >= 4 && k < 8) || k == 9;
    spmv<double, double>(L0.d, useK ? L0.K : L0.M, src[k], A.v[k], 1.0, 0.0, s);
  }
  AdjNodal a{};
  a.php = in.phi[0];
  a.phn = in.phi[1];
  a.Phi = in.Phi_v;
  a.php1 = out.phi[0];
  a.phn1 = out.phi[1];
  a.mup1 = out.mu[0];
  a.mun1 = out.mu[1];
  a.mus1 = out.mu[2];
  a.Phi1 = out.Phi_v;
  a.Me1p = A.v[0];
  a.Me1n = A.v[1];
  a.Me2p = A.v[2];
  a.Me2n = A.v[3];
  a.Ke1p = A.v[4];
  a.Ke1n = A.v[5];
  a.Ke2p = A.v[6];
  a.Ke2n = A.v[7];
  a.Mz = A.v[8];
  a.Kz = A.v[9];
  a.nus = lo.mu[2];
  a.lam_php = li.phi[0];
  a.lam_phn = li.phi[1];
  a.lam_Phi = li.Phi_v;
  a.eps = p.eps;
  a.tau = p.tau;
  a.gam = p.mobility;
  a.gv = p.evap_rate;
  a.pc = pot_coef(p);
  adj_nodal(N, a, A.part, s);
  adj_finish(3, ADJ_NBLK, A.part, A.acc, s);
  const double cm = p.rho / p.tau;
  spmv<double, double>(P.d, P.Mv, A.xi, li.vel, cm, 0.0, s);
  spmv<double, double>(P.d, P.Mv, A.xi + N4, li.vel + N4, cm, 0.0, s);
  HIPCHK(c, hipMemsetAsync(A.gmu, 0, bytes, s));
  const double* etas[3] = {A.eta, A.eta + N2, A.zeta};
  const double* xs[3] = {out.phi[0], out.phi[1], out.Phi_v};
  for (int col = 0; col < 8; ++col) {
    const int e0 = c->el.colour_ptr[col], e1 = c->el.colour_ptr[col + 1];
    adj_p1conv(e0, e1, c->ep1, c->ep2, c->etype, h, N4, etas, xs, -p.tau, li.vel, s);
    adj_ns(e0, e1, c->ep1, c->ep2, c->etype, h, c->ns.tb, N4, A.xi, out.vel, p.rho, p.alpha, in.phi[0],
           in.phi[1], in.Phi_v, beta, beta, li.vel, A.gmu, li.phi[0], li.phi[1], li.Phi_v, s);
  }
  for (int i = 0; i < 3; ++i)
    HIPCHK(c, hipMemcpyAsync(li.mu[i], A.gmu, bytes, hipMemcpyDeviceToDevice, s));
  HIPCHK(c, hipMemsetAsync(li.p, 0, bytes, s));
  // Korteweg coefficients beta_i = beta_v = eps^2: d/deps (xi^T F) = (2 / eps) xi^T F
  HIPCHK(c, hipMemsetAsync(A.F, 0, 8 * bytes, s));
  for (int col = 0; col < 8; ++col)
    korteweg(c->el.colour_ptr[col], c->el.colour_ptr[col + 1], c->ep1, c->ep2, c->etype, h, c->ns.tb,
             in.phi[0], in.phi[1], nullptr, in.Phi_v, KorBeta{{beta, beta, beta, 0.0}, beta}, N4, A.F, s);
  dot_acc(8 * int64_t(N), A.xi, A.F, 2.0 / p.eps, A.part, A.acc, s);
  HIPCHK(c, hipGetLastError());
  return CHNS_OK;
}

int chns_solve_block(chns_ctx* c, int block, const double* b, double* x, const chns_solve_opts& o,
                     chns_solve_info** info, int& worst, hipStream_t s) {
  chns_solve_info inf{};
  const int rc = fgmres(c, block, b, x, o, &inf, s);
  inf.passes = 1;
  if (rc < 0) return rc;
  if (rc > worst) worst = rc;
  if (info && *info) *(*info)++ = inf;
  return CHNS_OK;
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

int chns_create(const chns_mesh* mesh, const chns_params* params, chns_alloc_fn alloc, chns_free_fn free_,
                void* alloc_ctx, chns_ctx** out) {
  if (!out) return CHNS_EINVAL;
  *out = nullptr;
  if ((alloc == nullptr) != (free_ == nullptr)) {
    g_create_err = "alloc and free must both be given or both be NULL";
    return CHNS_EINVAL;
  }
  if (!mesh) {
    g_create_err = "mesh is NULL";
    return CHNS_EINVAL;
  }
  if (mesh->n < 8 || mesh->n > 8192 || mesh->n % 2 != 0) {
    g_create_err = "n must be even and in 8..8192";
    return CHNS_EINVAL;
  }
  if (mesh->model < CHNS_MODEL_CH || mesh->model > CHNS_MODEL_QUATERNARY) {
    g_create_err = "unknown model";
    return CHNS_EINVAL;
  }
  if (mesh->boundary != CHNS_BOUNDARY_PERIODIC && mesh->boundary != CHNS_BOUNDARY_NOFLUX) {
    g_create_err = "unknown boundary";
    return CHNS_EINVAL;
  }
  if (!(mesh->length >= 0.0 && std::isfinite(mesh->length))) {
    g_create_err = "length must be finite and > 0 (0 for 1)";
    return CHNS_EINVAL;
  }
  if (mesh->dim != 0 && mesh->dim != 2 && mesh->dim != 3) {
    g_create_err = "dim must be 2 or 3 (0 for 2)";
    return CHNS_EINVAL;
  }
  if (mesh->dim == 3) {
    if (mesh->model > CHNS_MODEL_CH_AC || mesh->n > 128) {
      g_create_err = "the cube takes the binary models and n <= 128";
      return CHNS_EINVAL;
    }
  }
  chns_ctx tmp;
  if (check_params(&tmp, params) != CHNS_OK) {
    g_create_err = tmp.err;
    return CHNS_EINVAL;
  }
  if (const char* why = model_params_error(mesh->model, mesh->boundary == CHNS_BOUNDARY_NOFLUX, params)) {
    g_create_err = why;
    return CHNS_EINVAL;
  }
  chns_ctx* c = new chns_ctx();
  c->alloc = alloc;
  c->free_ = free_;
  c->alloc_ctx = alloc_ctx;
  c->mesh = *mesh;
  c->prm = *params;
  // the flow models (Taylor-Hood Oseen step): ternary and quaternary
  c->ternary = (mesh->model == CHNS_MODEL_TERNARY || mesh->model == CHNS_MODEL_QUATERNARY);
  c->quat = mesh->model == CHNS_MODEL_QUATERNARY;
  c->beta_ch = c->quat ? params->beta_phase[0] : params->eps * params->eps;
  c->box = mesh->boundary == CHNS_BOUNDARY_NOFLUX;
  c->len = mesh->length > 0.0 ? mesh->length : 1.0;
  c->h = c->len / mesh->n;
  c->dim3 = mesh->dim == 3;
  c->diag_ratio = c->dim3 ? 15.0 : 8.0;
  int rc = CHNS_OK;
  if (hipGetDevice(&c->device) != hipSuccess) {
    c->err = "hipGetDevice failed";
    rc = CHNS_EHIP;
  } else if (hipError_t e = static_scratch_init(); e != hipSuccess) {
    c->err = std::string("static scratch address: ") + hipGetErrorString(e);
    rc = CHNS_EHIP;
  } else {
    rc = build(c);
  }
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
  if (const char* why = model_params_error(c->mesh.model, c->box, p)) return fail(c, CHNS_EINVAL, why);
  c->prm = *p;
  c->beta_ch = c->quat ? p->beta_phase[0] : p->eps * p->eps;
  // the residual reduction rates of earlier solves belong to other systems
  for (double& r : c->kr.rate) r = -1.0;
  if (c->ternary) TRY(assemble_sym_stiffness(c, nullptr));
  TRY(form_operators(c, nullptr));
  HIPCHK(c, hipDeviceSynchronize());
  return CHNS_OK;
}

int chns_assemble(chns_ctx* c, const double* d_vel, const double* const* d_mu, void* stream) {
  if (!c) return CHNS_EINVAL;
  return assemble_ops(c, d_vel, d_mu, false, static_cast<hipStream_t>(stream));
}

int chns_set_density(chns_ctx* c, const double* d_phi_p, const double* d_phi_n, void* stream) {
  if (!c) return CHNS_EINVAL;
  if (!c->ternary || c->quat || !c->prm.var_density)
    return fail(c, CHNS_EINVAL, "the density field needs a ternary context with var_density");
  if (!d_phi_p || !d_phi_n) return fail(c, CHNS_EINVAL, "phi_p and phi_n are required");
  return set_density(c, d_phi_p, d_phi_n, static_cast<hipStream_t>(stream));
}

int chns_assemble_transposed(chns_ctx* c, const double* d_vel, const double* const* d_mu, void* stream) {
  if (!c) return CHNS_EINVAL;
  if (!c->ternary) return fail(c, CHNS_EUNSUPPORTED, "transposed operators need the ternary model");
  return assemble_ops(c, d_vel, d_mu, true, static_cast<hipStream_t>(stream));
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
  } else if (op == CHNS_OP_NS && c->ternary) {
    r = k = 9 * int64_t(L0.N);
    z = c->ns.csr.nnz();
  } else if (op == CHNS_OP_VX && c->ternary) {
    r = k = 4 * int64_t(L0.N);
    z = c->p2.csr.nnz();
  } else if (op == CHNS_OP_AP && c->ternary) {
    r = k = L0.N;
    z = L0.csr.nnz();
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
  if ((op == CHNS_OP_NS || op == CHNS_OP_VX) && c->ternary) {
    const Csr& A = op == CHNS_OP_NS ? c->ns.csr : c->p2.csr;
    const Sell& Sl = op == CHNS_OP_NS ? c->ns.sell : c->p2.sell;
    const double* d = op == CHNS_OP_NS ? c->ns.val : c->p2.Vx.v64;
    if (h_val) {
      std::vector<double> sv(Sl.slots());
      HIPCHK(c, hipMemcpyAsync(sv.data(), d, sv.size() * sizeof(double), hipMemcpyDeviceToHost, s));
      HIPCHK(c, hipStreamSynchronize(s));
      for (int64_t q = 0; q < A.nnz(); ++q) h_val[q] = sv[Sl.csr2sell[q]];
    }
    if (h_rowptr) std::memcpy(h_rowptr, A.rowptr.data(), (A.nrows + 1) * sizeof(int));
    if (h_col) std::memcpy(h_col, A.col.data(), A.nnz() * sizeof(int));
    return CHNS_OK;
  }
  const double* src = nullptr;
  switch (op) {
    case CHNS_OP_AP:
      if (!c->ternary) return fail(c, CHNS_EINVAL, "unknown operator");
      src = L0.Ap.v64;
      break;
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
  const double tg = c->prm.tau * c->prm.mobility, beta = c->beta_ch;
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

int chns_spmv(chns_ctx* c, int32_t op, int32_t precision, int32_t transpose, double alpha, const void* d_x,
              double beta, void* d_y, void* stream) {
  if (!c) return CHNS_EINVAL;
  TRY(check_orientation(c, op_symmetric(c, op), transpose));
  if (!d_x || !d_y) return fail(c, CHNS_EINVAL, "x or y is NULL");
  if (d_x == d_y) return fail(c, CHNS_EINVAL, "x and y must not overlap");
  if (precision != CHNS_F64 && precision != CHNS_MIXED) return fail(c, CHNS_EINVAL, "unknown precision");
  if (!is_finite(alpha) || !is_finite(beta)) return fail(c, CHNS_EINVAL, "alpha/beta not finite");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Level& L0 = c->lv[0];
  const auto& p = c->prm;
  const double tg = p.tau * p.mobility, be = c->beta_ch;
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
  if ((op == CHNS_OP_NS || op == CHNS_OP_VX) && c->ternary) {
    if (precision != CHNS_F64 && op == CHNS_OP_NS)
      return fail(c, CHNS_EUNSUPPORTED, "the Oseen operator is applied in FP64 only");
    if (op == CHNS_OP_NS)
      spmv<double, double>(c->ns.d, c->ns.val, (const double*)d_x, (double*)d_y, alpha, beta, s);
    else if (precision == CHNS_F64)
      spmv<double, double>(c->p2.d, c->p2.Vx.v64, (const double*)d_x, (double*)d_y, alpha, beta, s);
    else
      spmv<float, float>(c->p2.d, c->p2.Vx.v32, (const float*)d_x, (float*)d_y, float(alpha),
                         float(beta), s);
    HIPCHK(c, hipGetLastError());
    return CHNS_OK;
  }
  const double* v64 = nullptr;
  const float* v32 = nullptr;
  switch (op) {
    case CHNS_OP_AP:
      if (!c->ternary) return fail(c, CHNS_EINVAL, "unknown operator");
      v64 = L0.Ap.v64;
      v32 = L0.Ap.v32;
      break;
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

int chns_precond_apply(chns_ctx* c, int32_t block, int32_t transpose, const chns_solve_opts* opts,
                       const double* d_r, double* d_z, void* stream) {
  if (!c) return CHNS_EINVAL;
  TRY(check_opts(c, opts));
  if (!d_r || !d_z) return fail(c, CHNS_EINVAL, "r or z is NULL");
  if (d_r == d_z) return fail(c, CHNS_EINVAL, "r and z must not overlap");
  if (block != CHNS_BLOCK_CH && block != CHNS_BLOCK_AC && !(block == CHNS_BLOCK_NS && c->ternary))
    return fail(c, CHNS_EUNSUPPORTED, "block not available");
  TRY(check_orientation(c, block_symmetric(c, block), transpose));
  return precond(c, block, *opts, d_r, d_z, static_cast<hipStream_t>(stream));
}

int chns_krylov_solve(chns_ctx* c, int32_t block, int32_t transpose, const double* d_b, double* d_x,
                      const chns_solve_opts* opts, chns_solve_info* h_info, void* stream) {
  if (!c) return CHNS_EINVAL;
  TRY(check_opts(c, opts));
  if (!d_b || !d_x) return fail(c, CHNS_EINVAL, "b or x is NULL");
  if (block != CHNS_BLOCK_CH && block != CHNS_BLOCK_AC && !(block == CHNS_BLOCK_NS && c->ternary))
    return fail(c, CHNS_EUNSUPPORTED, "block not available");
  if (block == CHNS_BLOCK_AC && c->mesh.model == CHNS_MODEL_CH)
    return fail(c, CHNS_EUNSUPPORTED, "model has no AC block");
  TRY(check_orientation(c, block_symmetric(c, block), transpose));
  return fgmres(c, block, d_b, d_x, *opts, h_info, static_cast<hipStream_t>(stream));
}

int chns_step_rhs(chns_ctx* c, const chns_fields* in, double* d_rhs_ch, double* d_rhs_ac, double* d_rhs_ns,
                  void* stream) {
  if (!c) return CHNS_EINVAL;
  if (!in || !in->phi[0] || !d_rhs_ch) return fail(c, CHNS_EINVAL, "missing field or output");
  if (c->quat) {
    if (!in->phi[1] || !in->phi[2] || !in->Phi_v || !in->vel || !d_rhs_ac || !d_rhs_ns)
      return fail(c, CHNS_EINVAL, "the quaternary model needs phi[0..2], Phi_v, vel and all outputs");
    return quaternary_rhs(c, in, d_rhs_ch, d_rhs_ac, d_rhs_ns, c->fs, static_cast<hipStream_t>(stream));
  }
  if (c->ternary) {
    if (!in->phi[1] || !in->Phi_v || !in->vel || !d_rhs_ac || !d_rhs_ns)
      return fail(c, CHNS_EINVAL, "the ternary model needs phi[0..1], Phi_v, vel and all outputs");
    if (c->prm.var_density) TRY(set_density(c, in->phi[0], in->phi[1], static_cast<hipStream_t>(stream)));
    return ternary_rhs(c, in, d_rhs_ch, d_rhs_ac, d_rhs_ns, c->fs, static_cast<hipStream_t>(stream));
  }
  const bool ac = c->mesh.model == CHNS_MODEL_CH_AC;
  if (ac && !in->Phi_v) return fail(c, CHNS_EINVAL, "model needs Phi_v");
  const auto& p = c->prm;
  const double beta = p.eps * p.eps;
  TopFlux tf;
  if (c->box && p.top_flux != 0.0) {
    const int n = c->mesh.n;
    tf.coef = p.tau * p.mobility * p.top_flux;
    tf.phi_inf = p.flux_inf;
    tf.h = c->h;
    if (c->dim3) {  // the top face z = length: vertices (i, j, n), weights int phi_i dS
      tf.top0 = n * (n + 1) * (n + 1);
      tf.ref = n / 2 + (n + 1) * (n / 2) + (n + 1) * (n + 1) * n;  // centre of the top face
      tf.w = c->topw;
    } else {
      tf.top0 = n * (n + 1);
      tf.ref = n / 2 + (n + 1) * n;  // midpoint of the top wall
    }
  }
  rhs_binary(c->lv[0].d, c->lv[0].M, in->phi[0], ac ? in->Phi_v : nullptr,
             -(p.tau * p.mobility / beta), -p.tau * p.evap_rate, tf, d_rhs_ch, ac ? d_rhs_ac : nullptr,
             static_cast<hipStream_t>(stream));
  HIPCHK(c, hipGetLastError());
  return CHNS_OK;
}

// Gradient coefficients of the energy per phase (the eliminated phase last).
KorBeta diag_betas(const chns_ctx* c) {
  const double b = c->prm.eps * c->prm.eps;
  if (c->quat) {
    const double* q = c->prm.beta_phase;
    return KorBeta{{q[0], q[1], q[2], q[3]}, b};
  }
  return KorBeta{{b, b, b, b}, b};
}

int chns_diagnostics(chns_ctx* c, const chns_fields* f, double* h_out, void* stream) {
  if (!c) return CHNS_EINVAL;
  if (!f || !f->phi[0] || !h_out) return fail(c, CHNS_EINVAL, "phi[0] and the output are required");
  const bool vapour = c->mesh.model != CHNS_MODEL_CH;
  if (c->ternary && !f->phi[1]) return fail(c, CHNS_EINVAL, "the ternary model needs phi[1]");
  if (c->quat && !f->phi[2]) return fail(c, CHNS_EINVAL, "the quaternary model needs phi[2]");
  if (vapour && !f->Phi_v) return fail(c, CHNS_EINVAL, "model needs Phi_v");
  hipStream_t s = static_cast<hipStream_t>(stream);
  Level& L0 = c->lv[0];
  diagnostics(L0.d, L0.M, L0.K, f->phi[0], c->ternary ? f->phi[1] : nullptr, c->quat ? f->phi[2] : nullptr,
              vapour ? f->Phi_v : nullptr, c->ternary, diag_betas(c), pot_coef(c->prm), c->kr.part, c->diag, s);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipMemcpyAsync(h_out, c->diag, NDIAG * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  return CHNS_OK;
}

int chns_diagnostics_noalloc(chns_ctx* c, const chns_fields* f, double* h_out, void* stream) {
  if (!c) return CHNS_EINVAL;
  if (!f || !f->phi[0] || !h_out) return fail(c, CHNS_EINVAL, "phi[0] and the output are required");
  const bool vapour = c->mesh.model != CHNS_MODEL_CH;
  if (c->ternary && !f->phi[1]) return fail(c, CHNS_EINVAL, "the ternary model needs phi[1]");
  if (c->quat && !f->phi[2]) return fail(c, CHNS_EINVAL, "the quaternary model needs phi[2]");
  if (vapour && !f->Phi_v) return fail(c, CHNS_EINVAL, "model needs Phi_v");
  int dev = -1;
  HIPCHK(c, hipGetDevice(&dev));
  if (dev != c->device) return fail(c, CHNS_ESTATE, "the context's GPU is not the current device");
  double* scr = static_scratch(dev);
  if (!scr) return fail(c, CHNS_ESTATE, "static scratch not set up on this device");
  Level& L0 = c->lv[0];
  const int64_t nblk = diag_part_blocks(L0.d.nrows);
  if (int64_t(NDIAG) * (nblk + 1) > STATIC_SCRATCH)
    return fail(c, CHNS_EINVAL, "the reduction needs " + std::to_string(NDIAG * (nblk + 1)) +
                                    " doubles of static scratch, more than its " +
                                    std::to_string(STATIC_SCRATCH));
  hipStream_t s = static_cast<hipStream_t>(stream);
  double* part = scr;                  // NDIAG x nblk partials, each written before it is read
  double* res = scr + NDIAG * nblk;    // NDIAG results
  diagnostics(L0.d, L0.M, L0.K, f->phi[0], c->ternary ? f->phi[1] : nullptr, c->quat ? f->phi[2] : nullptr,
              vapour ? f->Phi_v : nullptr, c->ternary, diag_betas(c), pot_coef(c->prm), part, res, s);
  HIPCHK(c, hipGetLastError());
  HIPCHK(c, hipMemcpyAsync(h_out, res, NDIAG * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
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
  if (c->ternary) {
    const chns_fields* fs[2] = {in, out};
    for (const chns_fields* f : fs) {
      if (!f->phi[1] || !f->mu[1] || !f->mu[2] || !f->Phi_v || !f->vel || !f->p)
        return fail(c, CHNS_EINVAL, "the ternary and quaternary models need every field");
      if (c->quat && (!f->phi[2] || !f->mu[3]))
        return fail(c, CHNS_EINVAL, "the quaternary model needs phi[0..2] and mu[0..3]");
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    int worst = CHNS_OK;
    chns_fields cur = *in;
    chns_solve_info* info = h_info;
    for (int k = 0; k < nsteps; ++k) {
      if (c->quat) TRY(quaternary_step(c, cur, out, *opts, &info, worst, s));
      else TRY(ternary_step(c, cur, out, *opts, &info, worst, s));
      cur = *out;
    }
    HIPCHK(c, hipStreamSynchronize(s));
    return worst;
  }
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

int chns_timestep_adjoint(chns_ctx* c, const chns_fields* in, const chns_fields* out,
                          const chns_fields* lam_out, const chns_fields* lam_in, double* h_dtheta,
                          const chns_solve_opts* opts, chns_solve_info* h_info, void* stream) {
  if (!c) return CHNS_EINVAL;
  TRY(check_opts(c, opts));
  if (!c->ternary || c->quat) return fail(c, CHNS_EUNSUPPORTED, "the adjoint step is defined for the ternary model");
  if (c->prm.var_density || c->prm.ns_picard > 1)
    return fail(c, CHNS_EUNSUPPORTED, "the adjoint step covers the linear scheme with constant density");
  if (!in || !out || !lam_out || !lam_in || !h_dtheta) return fail(c, CHNS_EINVAL, "NULL argument");
  const chns_fields* full[3] = {in, out, lam_in};
  for (const chns_fields* f : full)
    if (!f->phi[0] || !f->phi[1] || !f->mu[0] || !f->mu[1] || !f->mu[2] || !f->Phi_v || !f->vel || !f->p)
      return fail(c, CHNS_EINVAL, "states and the output adjoint need every field");
  if (!lam_out->phi[0] || !lam_out->phi[1] || !lam_out->mu[0] || !lam_out->mu[1] || !lam_out->mu[2] ||
      !lam_out->Phi_v || !lam_out->vel)
    return fail(c, CHNS_EINVAL, "the input adjoint needs phi, mu, Phi_v and vel");
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIPCHK(c, hipMemsetAsync(c->adj.acc, 0, 4 * sizeof(double), s));
  int worst = CHNS_OK;
  chns_solve_info* info = h_info;
  TRY(ternary_adjoint(c, *in, *out, *lam_out, *lam_in, *opts, &info, worst, s));
  HIPCHK(c, hipMemcpyAsync(c->kr.host, c->adj.acc, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(c, hipStreamSynchronize(s));
  for (int i = 0; i < 3; ++i) h_dtheta[i] += c->kr.host[i];
  return worst;
}

int chns_ledger_start(chns_ctx* c, int32_t kernel) {
  if (!c) return CHNS_EINVAL;
  if (kernel < -1 || kernel > CHNS_KERNEL_MG_FINE) return fail(c, CHNS_EINVAL, "unknown kernel class");
  Ledger& G = c->ledger;
  TRY(ledger_fold(c));
  if (kernel >= 0 && G.cap == 0) {
    G.cap = 4096;
    G.ev.resize(2 * size_t(G.cap));
    for (auto& e : G.ev) HIPCHK(c, hipEventCreate(&e));
    G.bytes.assign(G.cap, 0.0);
  }
  G.kernel = kernel;
  G.launches = 0;
  G.sum_bytes = G.sum_ms = 0.0;
  return CHNS_OK;
}

int chns_ledger_read(chns_ctx* c, int64_t* launches, double* bytes, double* ms) {
  if (!c) return CHNS_EINVAL;
  TRY(ledger_fold(c));
  if (launches) *launches = c->ledger.launches;
  if (bytes) *bytes = c->ledger.sum_bytes;
  if (ms) *ms = c->ledger.sum_ms;
  return CHNS_OK;
}

const char* chns_last_error(const chns_ctx* c) {
  if (!c) return g_create_err.c_str();
  return c->err.c_str();
}

}  // extern "C"
