// Batched form: many independent CH + AC instances (uneven mesh sizes and
// parameters) advanced together.  Every stage is one launch over all
// instances: stacked per-level operators, stacked Krylov vectors, per-instance
// Krylov scalars on the device, and an autotuned launch shape per level.
// Converged instances freeze: inside the Arnoldi loop every kernel skips their
// rows.  The eager mode reads the activity flags back now and then and stops
// when every instance has converged; the graph mode runs a fixed budget of
// Arnoldi steps per block without host synchronisation, captured once per
// step variant and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/chns.h"
#include "host_mesh.hpp"
#include "kernels.hpp"
#include "kernels_batch.hpp"

using namespace chns;

namespace {

constexpr int NOPS = 3;  // 0: L = M, 1: X = s M + tau g K, 2: AC = M + tau delta_v K
constexpr int BMAX_RESTART = 64;
constexpr int64_t KRYLOV_PAD = 640;  // doubles between consecutive basis vectors (HBM channel spread)
constexpr size_t GRAPH_MAX_NODES = 100000;  // refuse to instantiate larger step graphs
constexpr int GRAPH_CACHE = 4;              // step graphs kept per batch
constexpr int GRAPH_STEPS = 10;             // time steps captured in one graph
constexpr int EAGER_CHECK = 4;              // eager mode: Arnoldi steps between activity readbacks

struct GraphEntry {
  std::string key;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

struct SizeTables {  // host tables of one mesh size, all its levels
  std::vector<int> n;
  std::vector<Csr> csr;
  std::vector<Sell> sell;
  std::vector<Csr> P, R;
  std::vector<std::vector<double>> Pv, Rv;
  std::vector<Sell> Psell, Rsell;
  std::vector<GalerkinMap> gm;
  Elements el;
  std::vector<int> eslot;
  int *d_ep2 = nullptr, *d_etype = nullptr, *d_eslot = nullptr;
};

template <typename T>
struct Vec2 {
  T* p[2] = {nullptr, nullptr};
};

struct BLevel {
  int nrows = 0, nslices = 0;
  std::vector<int> roff;  // per instance, -1 when absent
  BStencil st;
  int *col = nullptr, *sinst = nullptr, *diag = nullptr;
  int *Pcol = nullptr, *Rcol = nullptr;  // transfer to the next level
  double *P64 = nullptr, *R64 = nullptr;
  float *P32 = nullptr, *R32 = nullptr;
  int *gptr = nullptr, *gsrc = nullptr;
  double* gw = nullptr;
  int64_t slots = 0;
  double *M = nullptr, *K = nullptr;
  float* M32 = nullptr;
  double* v64[NOPS] = {};
  float* v32[NOPS] = {};
  double* d64[NOPS] = {};
  float* d32[NOPS] = {};
  double *b64 = nullptr, *x64 = nullptr, *t64 = nullptr, *r64 = nullptr, *dd64 = nullptr;
  float *b32 = nullptr, *x32 = nullptr, *t32 = nullptr, *r32 = nullptr, *dd32 = nullptr;
  // per op: masks (per slice) and counts, coarse Chebyshev coefficients [step][inst]
  uint8_t *smooth[NOPS] = {}, *coarse[NOPS] = {}, *present[NOPS] = {};
  int nsmooth[NOPS] = {}, ncoarse[NOPS] = {}, npresent[NOPS] = {};
  double* cc64[NOPS][2] = {};
  float* cc32[NOPS][2] = {};
  double* aco[NOPS][2] = {};  // per-instance a, b of each op
  // tiled cycle, per op: tiles of the instances smoothing on this level
  // (down/up pass) and of those cut here, and the instances whose
  // one-workgroup tail starts on this level (indices into the tail tables)
  BTile* tdown[NOPS] = {};
  BTile* tzero[NOPS] = {};
  int* tail_idx[NOPS] = {};
  int ntdown[NOPS] = {}, ntzero[NOPS] = {}, ntail[NOPS] = {};
  size_t tile_cap = 0;  // tiles of every instance present on this level
};

}  // namespace

struct chns_batch {
  int count = 0;
  std::vector<int> n;
  std::vector<chns_params> prm;
  std::vector<int64_t> off;  // node offsets (level 0)
  int64_t Ntot = 0;
  std::vector<BLevel> lv;
  std::map<int, std::unique_ptr<SizeTables>> sizes;
  // per-instance scalars
  double *c12 = nullptr, *c22 = nullptr, *cmu = nullptr, *cac = nullptr;
  float *c12f = nullptr, *c22f = nullptr;
  int* cinst = nullptr;      // chunk -> instance over [phi_all; mu_all]
  int *cr = nullptr;         // chunk ranges per instance (first half)
  int nchunk1 = 0;
  // Krylov (DCGS2): basis and preconditioned vectors with stride ld, per
  // instance Hessenberg (raw H, rotated HR), rotations, g, gp, slot sums and
  // coefficients
  int64_t ld = 0;
  double *V = nullptr, *Z = nullptr, *H = nullptr, *HR = nullptr, *cs = nullptr, *sn = nullptr;
  double *g = nullptr, *gp = nullptr, *y = nullptr, *red = nullptr, *coef = nullptr;
  double *inv = nullptr, *nrm = nullptr, *tol = nullptr;
  double *part = nullptr, *part2 = nullptr;
  int *active = nullptr, *kcols = nullptr;
  int *iters[2] = {}, *conv[2] = {};
  // step buffers
  double *rhs_ch = nullptr, *rhs_ac = nullptr, *xch = nullptr, *xac = nullptr;
  double *w64a = nullptr, *w64b = nullptr;
  float *r32 = nullptr, *z32 = nullptr, *w32a = nullptr, *w32b = nullptr;
  // graph mode: Arnoldi budget per block (0: maxiter) and cached step graphs
  int budget[2] = {0, 0};
  std::vector<GraphEntry> graphs;
  // current coarse-coefficient opts; whether they run the tiled cycle, and
  // its tail tables (per op, one entry per instance)
  std::string opts_key;
  bool tiled = false;
  TailArgs<float>* tails32[NOPS] = {};
  TailArgs<double>* tails64[NOPS] = {};
  // work-list form of the tiled multigrid passes: grid (0: one workgroup per
  // tile) and the per-XCD tile counters
  int wl_grid = 0;
  int* wl_ctr = nullptr;
  // autotuned launch shapes of the Gram-Schmidt passes
  int upd_threads = 256;  // workgroup size of the update pass per 1024-row chunk
  int dots_group = 16;    // basis vectors per dot-pass launch
  std::vector<void*> allocs;
  // device allocator of the caller (chns_batch_create), or hipMalloc/hipFree when NULL
  chns_alloc_fn alloc = nullptr;
  chns_free_fn free_ = nullptr;
  void* alloc_ctx = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  std::string err;
};

namespace {

thread_local std::string g_batch_err;

int fail_cap(chns_batch* b) {
  b->err = "internal: an options table exceeds its buffer";
  return CHNS_EINVAL;
}

#define BCHK(b, expr)                                                  \
  do {                                                                 \
    hipError_t e_ = (expr);                                            \
    if (e_ != hipSuccess) {                                            \
      (b)->err = std::string(#expr) + ": " + hipGetErrorString(e_);    \
      return CHNS_EHIP;                                                \
    }                                                                  \
  } while (0)
#define BTRY(expr)            \
  do {                        \
    int rc_ = (expr);         \
    if (rc_ < 0) return rc_;  \
  } while (0)

template <typename T>
int balloc(chns_batch* b, T** p, size_t n) {
  *p = nullptr;
  if (n == 0) return CHNS_OK;
  void* q = nullptr;
  if (b->alloc) {
    q = b->alloc(n * sizeof(T), b->alloc_ctx);
    if (!q) {
      b->err = "the caller's allocator returned NULL";
      return CHNS_ENOMEM;
    }
    b->allocs.push_back(q);
    if (reinterpret_cast<uintptr_t>(q) % 256 != 0) {
      b->err = "the caller's allocator returned memory not aligned to 256 bytes";
      return CHNS_EINVAL;
    }
  } else {
    if (hipMalloc(&q, n * sizeof(T)) != hipSuccess) {
      b->err = "hipMalloc failed";
      return CHNS_ENOMEM;
    }
    b->allocs.push_back(q);
  }
  *p = static_cast<T*>(q);
  return CHNS_OK;
}

// Copy a host table into a buffer allocated at creation (tables that depend
// on the solve options are rewritten in place, never reallocated).
template <typename T>
int bput(chns_batch* b, T* dst, const std::vector<T>& h, size_t cap) {
  if (h.size() > cap) return fail_cap(b);
  if (!h.empty()) BCHK(b, hipMemcpy(dst, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return CHNS_OK;
}

template <typename T>
int bupload(chns_batch* b, T** p, const std::vector<T>& h) {
  BTRY(balloc(b, p, h.size()));
  if (!h.empty()) BCHK(b, hipMemcpy(*p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return CHNS_OK;
}

int fail(chns_batch* b, int code, const std::string& m) {
  if (b) b->err = m;
  return code;
}

SizeTables* tables_for(chns_batch* b, int n) {
  auto it = b->sizes.find(n);
  if (it != b->sizes.end()) return it->second.get();
  auto T = std::make_unique<SizeTables>();
  std::vector<int> sz{n};
  while (sz.back() % 2 == 0 && sz.back() / 2 >= 4) sz.push_back(sz.back() / 2);
  T->n = sz;
  for (int nl : sz) {
    Elements E = make_elements(nl);
    T->csr.push_back(pattern_from_elements(nl * nl, nl * nl, E.ne, E.v.data(), 3, E.v.data(), 3));
    T->sell.push_back(make_sell_p1(T->csr.back(), nl));
    if (nl == n) T->el = std::move(E);
  }
  for (size_t l = 0; l + 1 < sz.size(); ++l) {
    Csr P, R;
    std::vector<double> Pv, Rv;
    p1_prolongation(sz[l], P, Pv);
    csr_transpose(P, Pv, R, Rv);
    T->Psell.push_back(make_sell(P, 64, 1));
    T->Rsell.push_back(make_sell(R, 64, 1));
    T->gm.push_back(make_galerkin(T->csr[l], T->sell[l], P, Pv, T->csr[l + 1], T->sell[l + 1], nullptr));
    T->P.push_back(std::move(P));
    T->R.push_back(std::move(R));
    T->Pv.push_back(std::move(Pv));
    T->Rv.push_back(std::move(Rv));
  }
  const Csr& A = T->csr[0];
  T->eslot.resize(size_t(T->el.ne) * 9);
  for (int e = 0; e < T->el.ne; ++e)
    for (int a = 0; a < 3; ++a)
      for (int c = 0; c < 3; ++c)
        T->eslot[size_t(e) * 9 + a * 3 + c] = T->sell[0].csr2sell[A.find(T->el.v[e * 3 + a], T->el.v[e * 3 + c])];
  SizeTables* raw = T.get();
  b->sizes[n] = std::move(T);
  return raw;
}

// Stack the per-instance level structures.
int build_levels(chns_batch* b) {
  int Lmax = 0;
  std::vector<SizeTables*> tab(b->count);
  for (int i = 0; i < b->count; ++i) {
    tab[i] = tables_for(b, b->n[i]);
    Lmax = std::max(Lmax, int(tab[i]->n.size()));
  }
  b->lv.resize(Lmax);
  for (int l = 0; l < Lmax; ++l) {
    BLevel& L = b->lv[l];
    L.roff.assign(b->count, -1);
    int rows = 0;
    for (int i = 0; i < b->count; ++i)
      if (l < int(tab[i]->n.size())) {
        L.roff[i] = rows;
        const int nl = tab[i]->n[l];
        rows += ((nl * nl + 63) / 64) * 64;  // slice-aligned
      }
    L.nrows = rows;
    L.nslices = rows / 64;
    L.slots = int64_t(rows) * 7;
    std::vector<int> col(L.slots, 0), sinst(L.nslices, 0), diag(rows, 0);
    for (int i = 0; i < b->count; ++i) {
      if (L.roff[i] < 0) continue;
      const Sell& S = tab[i]->sell[l];
      const int r0 = L.roff[i];
      for (int64_t q = 0; q < S.slots(); ++q) col[int64_t(r0) * 7 + q] = S.col[q] + r0;
      for (int r = 0; r < S.nrows; ++r) diag[r0 + r] = int(int64_t(r0) * 7 + S.diag[r]);
      // padding rows of a partial last slice keep diag at their own slot 0
      for (int r = S.nrows; r < S.nslices * 64; ++r) diag[r0 + r] = int(int64_t(r0) * 7 + (r / 64) * 448 + (r % 64));
      for (int s = 0; s < S.nslices; ++s) sinst[r0 / 64 + s] = i;
    }
    BTRY(bupload(b, &L.col, col));
    BTRY(bupload(b, &L.sinst, sinst));
    BTRY(bupload(b, &L.diag, diag));
    L.st.nrows = L.nrows;
    L.st.col = L.col;
    L.st.sinst = L.sinst;
    // computed columns where no instance block has padding rows
    bool whole = true;
    std::vector<int2> geo(L.nslices);
    for (int i = 0; i < b->count; ++i) {
      if (L.roff[i] < 0) continue;
      const int nl = tab[i]->n[l];
      if ((nl * nl) % 64 != 0) whole = false;
      for (int s0 = L.roff[i] / 64, s = s0; s < s0 + (nl * nl + 63) / 64; ++s) geo[s] = make_int2(nl, L.roff[i]);
    }
    if (whole) {
      int2* dgeo = nullptr;
      BTRY(bupload(b, &dgeo, geo));
      L.st.geo = dgeo;
    }
  }
  // transfers and Galerkin maps between l and l+1
  for (int l = 0; l + 1 < Lmax; ++l) {
    BLevel& F = b->lv[l];
    BLevel& G = b->lv[l + 1];
    std::vector<int> Pcol(int64_t(F.nrows) * 2, 0), Rcol(int64_t(G.nrows) * 7, 0);
    std::vector<double> Pval(int64_t(F.nrows) * 2, 0.0), Rval(int64_t(G.nrows) * 7, 0.0);
    std::vector<int> gptr(G.slots + 1, 0), gsrc;
    std::vector<double> gw;
    std::vector<std::vector<std::pair<int, double>>> lists(G.slots);
    for (int i = 0; i < b->count; ++i) {
      if (G.roff[i] < 0) continue;
      SizeTables* T = tab[i];
      const int rf = F.roff[i], rc = G.roff[i];
      const Sell& Ps = T->Psell[l];
      const Sell& Rs = T->Rsell[l];
      std::vector<double> pv(Ps.slots(), 0.0), rv(Rs.slots(), 0.0);
      for (int64_t q = 0; q < T->P[l].nnz(); ++q) pv[Ps.csr2sell[q]] = T->Pv[l][q];
      for (int64_t q = 0; q < T->R[l].nnz(); ++q) rv[Rs.csr2sell[q]] = T->Rv[l][q];
      if (Ps.width_max != 2 || !Ps.uniform || Rs.width_max != 7 || !Rs.uniform)
        return fail(b, CHNS_EINVAL, "unexpected transfer layout");
      for (int64_t q = 0; q < Ps.slots(); ++q) {
        Pcol[int64_t(rf) * 2 + q] = Ps.col[q] + rc;
        Pval[int64_t(rf) * 2 + q] = pv[q];
      }
      for (int64_t q = 0; q < Rs.slots(); ++q) {
        Rcol[int64_t(rc) * 7 + q] = Rs.col[q] + rf;
        Rval[int64_t(rc) * 7 + q] = rv[q];
      }
      const GalerkinMap& gm = T->gm[l];
      for (int64_t s = 0; s + 1 < int64_t(gm.ptr.size()); ++s)
        for (int k = gm.ptr[s]; k < gm.ptr[s + 1]; ++k)
          lists[int64_t(rc) * 7 + s].push_back({int(int64_t(rf) * 7 + gm.src[k]), gm.w[k]});
    }
    for (int64_t s = 0; s < G.slots; ++s) {
      gptr[s + 1] = gptr[s] + int(lists[s].size());
      for (auto& e : lists[s]) {
        gsrc.push_back(e.first);
        gw.push_back(e.second);
      }
    }
    std::vector<float> P32(Pval.begin(), Pval.end()), R32(Rval.begin(), Rval.end());
    BTRY(bupload(b, &F.Pcol, Pcol));
    BTRY(bupload(b, &F.Rcol, Rcol));
    BTRY(bupload(b, &F.P64, Pval));
    BTRY(bupload(b, &F.R64, Rval));
    BTRY(bupload(b, &F.P32, P32));
    BTRY(bupload(b, &F.R32, R32));
    BTRY(bupload(b, &F.gptr, gptr));
    BTRY(bupload(b, &F.gsrc, gsrc));
    BTRY(bupload(b, &F.gw, gw));
  }
  return CHNS_OK;
}

double op_a(const chns_params& p, int op) {
  if (op == 1) return std::sqrt(p.tau * p.mobility / (p.eps * p.eps));
  return 1.0;
}
double op_b(const chns_params& p, int op) {
  if (op == 1) return p.tau * p.mobility;
  if (op == 2) return p.tau * p.evap_rate * p.eps * p.eps;
  return 0.0;
}

int ninst_levels(chns_batch* b, int i) {
  int c = 0;
  for (auto& L : b->lv)
    if (L.roff[i] >= 0) ++c;
  return c;
}

template <typename T>
std::vector<T> cheb_seq(double lo, double hi, int steps, bool first) {
  // first ? c2 sequence : c1 sequence
  std::vector<T> out(steps);
  const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
  double rho_prev = 1.0 / sigma;
  out[0] = first ? T(1.0 / theta) : T(0);
  for (int i = 1; i < steps; ++i) {
    const double rho_i = 1.0 / (2.0 * sigma - rho_prev);
    out[i] = first ? T(2.0 * rho_i / delta) : T(rho_i * rho_prev);
    rho_prev = rho_i;
  }
  return out;
}

template <typename T> struct BSel;
template <> struct BSel<double> {
  static double* v(BLevel& L, int op) { return L.v64[op]; }
  static double* d(BLevel& L, int op) { return L.d64[op]; }
  static double* cc(BLevel& L, int op, int w) { return L.cc64[op][w]; }
  static double* b(BLevel& L) { return L.b64; }
  static double* x(BLevel& L) { return L.x64; }
  static double* t(BLevel& L) { return L.t64; }
  static double* r(BLevel& L) { return L.r64; }
  static double* dd(BLevel& L) { return L.dd64; }
  static double* P(BLevel& L) { return L.P64; }
  static double* R(BLevel& L) { return L.R64; }
  static double* M(BLevel& L) { return L.M; }
};
template <> struct BSel<float> {
  static float* v(BLevel& L, int op) { return L.v32[op]; }
  static float* d(BLevel& L, int op) { return L.d32[op]; }
  static float* cc(BLevel& L, int op, int w) { return L.cc32[op][w]; }
  static float* b(BLevel& L) { return L.b32; }
  static float* x(BLevel& L) { return L.x32; }
  static float* t(BLevel& L) { return L.t32; }
  static float* r(BLevel& L) { return L.r32; }
  static float* dd(BLevel& L) { return L.dd32; }
  static float* P(BLevel& L) { return L.P32; }
  static float* R(BLevel& L) { return L.R32; }
  static float* M(BLevel& L) { return L.M32; }
};

// Tail table entry of instance i from level ts to its cut level c.
template <typename T>
TailArgs<T> tail_entry(chns_batch* b, const chns_solve_opts& o, int op, int i, int ts, int c) {
  TailArgs<T> a{};
  a.inst = i;
  a.roff = b->lv[ts].roff[i];
  a.nlev = c - ts + 1;
  for (int t = 0; t < a.nlev; ++t) {
    BLevel& L = b->lv[ts + t];
    const int64_t r = L.roff[i];
    a.side[t] = b->n[i] >> (ts + t);
    a.val[t] = BSel<T>::v(L, op) + r * 7;
    a.dinv[t] = BSel<T>::d(L, op) + r;
  }
  a.pre = o.mg_pre;
  a.post = o.mg_post;
  auto p1 = cheb_seq<T>(o.mg_lmax / 4.0, o.mg_lmax, o.mg_pre, false);
  auto p2 = cheb_seq<T>(o.mg_lmax / 4.0, o.mg_lmax, o.mg_pre, true);
  for (int k = 0; k < o.mg_pre; ++k) {
    a.pre_c1[k] = p1[k];
    a.pre_c2[k] = p2[k];
  }
  auto q1 = cheb_seq<T>(o.mg_lmax / 4.0, o.mg_lmax, o.mg_post, false);
  auto q2 = cheb_seq<T>(o.mg_lmax / 4.0, o.mg_lmax, o.mg_post, true);
  for (int k = 0; k < o.mg_post; ++k) {
    a.post_c1[k] = q1[k];
    a.post_c2[k] = q2[k];
  }
  const double aa = op_a(b->prm[i], op), bb = op_b(b->prm[i], op);
  const double nl = double(b->n[i] >> c);
  const double lo = 0.45 / (1.0 + 8.0 * bb * nl * nl / aa);
  const int steps = std::min(c > 0 ? o.mg_coarse : o.mg_pre + o.mg_post, MAXCHEB);
  auto c1 = cheb_seq<T>(lo, o.mg_lmax, steps, false);
  auto c2 = cheb_seq<T>(lo, o.mg_lmax, steps, true);
  a.coarse.steps = steps;
  for (int k = 0; k < steps; ++k) {
    a.coarse.c1[k] = c1[k];
    a.coarse.c2[k] = c2[k];
  }
  return a;
}

// Tiled cycle of operator op: per instance, the levels above its tail take
// tiles (down/up on smoothing levels, from-zero steps on its cut level), the
// tail (one workgroup) takes the rest.  `tiled` turns false when a level does
// not fit the tiled kernels with these options.
int prepare_tiles(chns_batch* b, const chns_solve_opts& o, int op, const std::vector<int>& cut, bool& tiled) {
  const int Lmax = int(b->lv.size());
  const bool f32 = o.precision == CHNS_MIXED;
  std::vector<std::vector<BTile>> down(Lmax), zero(Lmax);
  std::vector<std::vector<int>> tails(Lmax);
  std::vector<TailArgs<float>> t32(b->count);
  std::vector<TailArgs<double>> t64(b->count);
  for (int i = 0; i < b->count; ++i) {
    const int c = cut[i];
    int ts = -1;
    for (int l = 0; l <= c && ts < 0; ++l) {
      int sides[TAIL_MAXLEV];
      const int nlev = c - l + 1;
      if (nlev > TAIL_MAXLEV) continue;
      for (int t = 0; t < nlev; ++t) sides[t] = b->n[i] >> (l + t);
      if (f32 ? tail_fits<float>(sides, nlev) : tail_fits<double>(sides, nlev)) ts = l;
    }
    const int lend = ts < 0 ? c + 1 : ts;
    for (int l = 0; l < lend; ++l) {
      const int side = b->n[i] >> l;
      const int roff = b->lv[l].roff[i];
      if (l < c) {
        if (!btile_fits(TILE_DOWN, side, o.mg_pre) || !btile_fits(TILE_UP, side, o.mg_post)) tiled = false;
        const int croff = b->lv[l + 1].roff[i];
        for (int t = 0; t < btile_count(side); ++t) down[l].push_back({i, t, side, roff, croff});
      } else {
        const int zs = l > 0 ? o.mg_coarse : o.mg_pre + o.mg_post;
        if (!btile_fits(TILE_ZERO, side, zs)) tiled = false;
        for (int t = 0; t < btile_count(side); ++t) zero[l].push_back({i, t, side, roff, 0});
      }
    }
    if (ts >= 0) {
      tails[ts].push_back(i);
      t32[i] = tail_entry<float>(b, o, op, i, ts, c);
      t64[i] = tail_entry<double>(b, o, op, i, ts, c);
    }
  }
  for (int l = 0; l < Lmax; ++l) {
    BLevel& L = b->lv[l];
    L.ntdown[op] = int(down[l].size());
    L.ntzero[op] = int(zero[l].size());
    L.ntail[op] = int(tails[l].size());
    BTRY(bput(b, L.tdown[op], down[l], L.tile_cap));
    BTRY(bput(b, L.tzero[op], zero[l], L.tile_cap));
    BTRY(bput(b, L.tail_idx[op], tails[l], size_t(b->count)));
  }
  BTRY(bput(b, b->tails32[op], t32, size_t(b->count)));
  BTRY(bput(b, b->tails64[op], t64, size_t(b->count)));
  return CHNS_OK;
}

void drop_graphs(chns_batch* b);

// Masks and coarse Chebyshev coefficients for the given options.
int prepare_cycles(chns_batch* b, const chns_solve_opts& o) {
  char key[256];
  std::snprintf(key, sizeof key, "%d/%d/%d/%.17g/%.17g/%d", o.mg_pre, o.mg_post, o.mg_coarse, o.mg_lmax,
                o.mg_rho_cut, o.precision);
  if (b->opts_key == key) return CHNS_OK;
  // the tables are rewritten in place: no launch may still read them, and no
  // captured graph may keep launching with the old ones
  BCHK(b, hipDeviceSynchronize());
  drop_graphs(b);
  b->opts_key.clear();
  const int Lmax = int(b->lv.size());
  bool tiled = o.mg_pre <= TAIL_MAXSM && o.mg_post <= TAIL_MAXSM;
  for (int op = 0; op < NOPS; ++op) {
    std::vector<int> cut(b->count);
    for (int i = 0; i < b->count; ++i) {
      const double a = op_a(b->prm[i], op), bb = op_b(b->prm[i], op);
      const int Li = ninst_levels(b, i);
      cut[i] = Li - 1;
      int nl = b->n[i];
      for (int l = 0; l < Li; ++l, nl /= 2)
        if (8.0 * bb * double(nl) * nl / a <= o.mg_rho_cut) {
          cut[i] = l;
          break;
        }
    }
    for (int l = 0; l < Lmax; ++l) {
      BLevel& L = b->lv[l];
      std::vector<uint8_t> sm(L.nslices, 0), co(L.nslices, 0), pr(L.nslices, 0);
      L.nsmooth[op] = L.ncoarse[op] = L.npresent[op] = 0;
      const int steps = (l > 0) ? o.mg_coarse : o.mg_pre + o.mg_post;
      std::vector<double> c1(size_t(steps) * b->count, 0.0), c2(size_t(steps) * b->count, 1.0);
      for (int i = 0; i < b->count; ++i) {
        if (L.roff[i] < 0 || l > cut[i]) continue;
        const int nl = b->n[i] >> l;
        const int s0 = L.roff[i] / 64, s1 = s0 + (nl * nl + 63) / 64;
        const uint8_t role = (l < cut[i]) ? 1 : 2;
        for (int s = s0; s < s1; ++s) {
          pr[s] = 1;
          (role == 1 ? sm : co)[s] = 1;
        }
        L.npresent[op]++;
        if (role == 1) {
          L.nsmooth[op]++;
        } else {
          L.ncoarse[op]++;
          const double a = op_a(b->prm[i], op), bb = op_b(b->prm[i], op);
          const double lo = 0.45 / (1.0 + 8.0 * bb * double(nl) * nl / a);
          auto s1v = cheb_seq<double>(lo, o.mg_lmax, steps, false);
          auto s2v = cheb_seq<double>(lo, o.mg_lmax, steps, true);
          for (int s = 0; s < steps; ++s) {
            c1[size_t(s) * b->count + i] = s1v[s];
            c2[size_t(s) * b->count + i] = s2v[s];
          }
        }
      }
      std::vector<float> c1f(c1.begin(), c1.end()), c2f(c2.begin(), c2.end());
      const size_t ns = size_t(L.nslices), nc = size_t(MAXCHEB) * b->count;
      BTRY(bput(b, L.smooth[op], sm, ns));
      BTRY(bput(b, L.coarse[op], co, ns));
      BTRY(bput(b, L.present[op], pr, ns));
      BTRY(bput(b, L.cc64[op][0], c1, nc));
      BTRY(bput(b, L.cc64[op][1], c2, nc));
      BTRY(bput(b, L.cc32[op][0], c1f, nc));
      BTRY(bput(b, L.cc32[op][1], c2f, nc));
    }
    BTRY(prepare_tiles(b, o, op, cut, tiled));
  }
  b->tiled = tiled;
  b->opts_key = key;
  return CHNS_OK;
}

// Batched V-cycle of operator `op` on level l: instances with their cut
// below l smooth and recurse, instances cut at l take Chebyshev steps.  Rows of
// instances with act 0 (act may be null) are skipped.
template <typename T>
void bvcycle(chns_batch* b, int op, int l, const T* rhs, T* x, const int* act,
             const chns_solve_opts& o, hipStream_t s) {
  BLevel& L = b->lv[l];
  const T* v = BSel<T>::v(L, op);
  const T* di = BSel<T>::d(L, op);
  T* d = BSel<T>::dd(L);
  T* t = BSel<T>::t(L);
  const double lmax = o.mg_lmax;
  if (L.nsmooth[op] > 0) {
    auto pc1 = cheb_seq<T>(lmax / 4.0, lmax, o.mg_pre, false);
    auto pc2 = cheb_seq<T>(lmax / 4.0, lmax, o.mg_pre, true);
    const uint8_t* m = L.smooth[op];
    T* cur = ((o.mg_pre - 1 + o.mg_post) % 2 == 0) ? x : t;
    T* oth = (cur == x) ? t : x;
    bstencil<T>(L.st, v, 3, nullptr, rhs, di, d, T(0), pc2[0], nullptr, nullptr, m, act, cur, s);
    for (int k = 1; k < o.mg_pre; ++k) {
      bstencil<T>(L.st, v, 2, cur, rhs, di, d, pc1[k], pc2[k], nullptr, nullptr, m, act, oth, s);
      std::swap(cur, oth);
    }
    T* r = BSel<T>::r(L);
    bstencil<T>(L.st, v, 1, cur, rhs, nullptr, nullptr, T(0), T(0), nullptr, nullptr, m, act, r, s);
    BLevel& G = b->lv[l + 1];
    bspmv_uniform<T>(G.nrows, 7, L.Rcol, BSel<T>::R(L), G.present[op], G.sinst, act, r,
                     BSel<T>::b(G), T(1), T(0), s);
    bvcycle<T>(b, op, l + 1, BSel<T>::b(G), BSel<T>::x(G), act, o, s);
    bspmv_uniform<T>(L.nrows, 2, L.Pcol, BSel<T>::P(L), m, L.sinst, act, BSel<T>::x(G), cur, T(1),
                     T(1), s);
    if (o.mg_post > 0) {
      auto qc1 = cheb_seq<T>(lmax / 4.0, lmax, o.mg_post, false);
      auto qc2 = cheb_seq<T>(lmax / 4.0, lmax, o.mg_post, true);
      for (int k = 0; k < o.mg_post; ++k) {
        bstencil<T>(L.st, v, 2, cur, rhs, di, d, qc1[k], qc2[k], nullptr, nullptr, m, act, oth, s);
        std::swap(cur, oth);
      }
    }
  }
  if (L.ncoarse[op] > 0) {
    const int steps = (l > 0) ? o.mg_coarse : o.mg_pre + o.mg_post;
    const uint8_t* m = L.coarse[op];
    const T* c1 = BSel<T>::cc(L, op, 0);
    const T* c2 = BSel<T>::cc(L, op, 1);
    T* cur = ((steps - 1) % 2 == 0) ? x : t;
    T* oth = (cur == x) ? t : x;
    bstencil<T>(L.st, v, 3, nullptr, rhs, di, d, T(0), T(0), c1, c2, m, act, cur, s);
    for (int k = 1; k < steps; ++k) {
      bstencil<T>(L.st, v, 2, cur, rhs, di, d, T(0), T(0), c1 + size_t(k) * b->count,
                  c2 + size_t(k) * b->count, m, act, oth, s);
      std::swap(cur, oth);
    }
  }
}

template <typename T> TailArgs<T>* btails(chns_batch* b, int op);
template <> TailArgs<float>* btails<float>(chns_batch* b, int op) { return b->tails32[op]; }
template <> TailArgs<double>* btails<double>(chns_batch* b, int op) { return b->tails64[op]; }

template <typename T>
void set_cheb(BTileLaunch<T>& a, double lmax, int steps) {
  auto c1 = cheb_seq<T>(lmax / 4.0, lmax, steps, false);
  auto c2 = cheb_seq<T>(lmax / 4.0, lmax, steps, true);
  a.steps = steps;
  for (int k = 0; k < steps && k < TILE_MAXSTEPS; ++k) {
    a.c1[k] = c1[k];
    a.c2[k] = c2[k];
  }
}

// Tiled batched V-cycle of operator op from level l: on each level one launch
// per role (the smoothing instances' down pass, the instances cut here, the
// instances whose one-workgroup tail starts here), the coarser levels, then
// the smoothing instances' up pass.
// b64 / x64 / xs (level 0 only, no tails there): the FP64 boundary of the
// cycle, as in the single-instance tiles (right-hand side read as FP64,
// result written as FP64 times xs[inst]).
template <typename T>
void bvcycle_tiled(chns_batch* b, int op, int l, const T* rhs, T* x, const int* act,
                   const chns_solve_opts& o, hipStream_t s, const double* b64 = nullptr,
                   double* x64 = nullptr, const double* xs = nullptr, const T* mval = nullptr) {
  BLevel& L = b->lv[l];
  const T* v = BSel<T>::v(L, op);
  const T* di = BSel<T>::d(L, op);
  if (L.ntzero[op] > 0) {
    BTileLaunch<T> a;
    a.tiles = L.tzero[op];
    a.act = act;
    a.count = b->count;
    a.steps = l > 0 ? o.mg_coarse : o.mg_pre + o.mg_post;
    a.val = v;
    a.dinv = di;
    a.b = rhs;
    a.x = x;
    a.b64 = b64;
    a.x64 = x64;
    a.xs = xs;
    a.cc1 = BSel<T>::cc(L, op, 0);
    a.cc2 = BSel<T>::cc(L, op, 1);
    bvtile<T>(TILE_ZERO, L.ntzero[op], a, s, b->wl_grid, b->wl_ctr);
  }
  if (L.ntail[op] > 0) bvtail<T>(L.ntail[op], btails<T>(b, op), L.tail_idx[op], act, rhs, x, s);
  if (L.ntdown[op] == 0) return;
  BLevel& G = b->lv[l + 1];
  BTileLaunch<T> a;
  a.tiles = L.tdown[op];
  a.act = act;
  a.count = b->count;
  a.val = v;
  a.dinv = di;
  a.b = rhs;
  a.b64 = b64;
  set_cheb<T>(a, o.mg_lmax, o.mg_pre);
  a.x = BSel<T>::t(L);
  a.bc = BSel<T>::b(G);
  bvtile<T>(TILE_DOWN, L.ntdown[op], a, s, b->wl_grid, b->wl_ctr);
  bvcycle_tiled<T>(b, op, l + 1, BSel<T>::b(G), BSel<T>::x(G), act, o, s);
  set_cheb<T>(a, o.mg_lmax, o.mg_post);
  a.xin = BSel<T>::t(L);
  a.e = BSel<T>::x(G);
  a.x = x;
  a.x64 = x64;
  a.xs = xs;
  a.bc = nullptr;
  a.mval = mval;  // when given (level 0), the up pass writes M times the result
  bvtile<T>(mval ? TILE_UPM : TILE_UP, L.ntdown[op], a, s, b->wl_grid, b->wl_ctr);
}

template <typename T>
void bcycle(chns_batch* b, int op, const T* rhs, T* x, const int* act, const chns_solve_opts& o,
            hipStream_t s) {
  if (b->tiled) bvcycle_tiled<T>(b, op, 0, rhs, x, act, o, s);
  else bvcycle<T>(b, op, 0, rhs, x, act, o, s);
}

template <typename T>
void bprecond_t(chns_batch* b, int block, const T* r, T* z, T* tmp1, T* tmp2, const int* act,
                const chns_solve_opts& o, hipStream_t s) {
  const int64_t N = b->Ntot;
  BLevel& L0 = b->lv[0];
  if (block == CHNS_BLOCK_CH) {
    bcycle<T>(b, 0, r, z, act, o, s);
    bcycle<T>(b, 1, r + N, tmp1, act, o, s);
    bstencil<T>(L0.st, BSel<T>::M(L0), 0, tmp1, nullptr, nullptr, nullptr, T(1), T(0), nullptr,
                nullptr, nullptr, act, tmp2, s);
    bcycle<T>(b, 1, tmp2, z + N, act, o, s);
  } else {
    bcycle<T>(b, 2, r, z, act, o, s);
  }
}

// Whether the FP32 cycles of a block take their FP64 input and write their
// FP64 output in the finest level's tiles: the tiled cycle, and on level 0
// no tails, the mass-like inverses cut there for every instance and X cut
// there for none.
bool bfused(chns_batch* b, int block, const chns_solve_opts& o) {
  if (o.precision == CHNS_F64 || !b->tiled) return false;
  const BLevel& L0 = b->lv[0];
  for (int op = 0; op < NOPS; ++op)
    if (L0.ntail[op] > 0) return false;
  if (block == CHNS_BLOCK_AC) return L0.ntdown[2] == 0;
  return L0.ntdown[0] == 0 && L0.ntzero[1] == 0;
}

// z = inv[inst] P^{-1} r for every active instance (inv may be null: 1); r is
// not written.  The Krylov basis vector arrives unnormalised and its 1/|w|
// rides on the output (P is linear).
void bprecond(chns_batch* b, int block, const double* r, const double* inv, double* z, const int* act,
              const chns_solve_opts& o, hipStream_t s) {
  const int64_t N = b->Ntot;
  const int64_t n = (block == CHNS_BLOCK_CH ? 2 : 1) * N;
  if (bfused(b, block, o)) {
    if (block == CHNS_BLOCK_AC) {
      bvcycle_tiled<float>(b, 2, 0, nullptr, nullptr, act, o, s, r, z, inv);
    } else {
      BLevel& L0 = b->lv[0];
      bvcycle_tiled<float>(b, 0, 0, nullptr, nullptr, act, o, s, r, z, inv);
      if (btile_fits(TILE_UPM, 64, o.mg_post)) {  // the first cycle's up pass writes M X^{-1} r2
        bvcycle_tiled<float>(b, 1, 0, nullptr, b->w32b, act, o, s, r + N, nullptr, nullptr, L0.M32);
      } else {
        bvcycle_tiled<float>(b, 1, 0, nullptr, b->w32a, act, o, s, r + N, nullptr, nullptr);
        bstencil<float>(L0.st, L0.M32, 0, b->w32a, nullptr, nullptr, nullptr, 1.0f, 0.0f, nullptr, nullptr,
                        nullptr, act, b->w32b, s);
      }
      bvcycle_tiled<float>(b, 1, 0, b->w32b, nullptr, act, o, s, nullptr, z + N, inv);
    }
    return;
  }
  if (o.precision == CHNS_F64) {
    bprecond_t<double>(b, block, r, z, b->w64a, b->w64b, act, o, s);
    if (inv) bscale(n, z, inv, b->cinst, act, z, s);
  } else {
    bconvert<double, float>(n, r, b->r32, b->cinst, act, s);
    bprecond_t<float>(b, block, b->r32, b->z32, b->w32a, b->w32b, act, o, s);
    bconvert_out(n, b->z32, inv, z, b->cinst, act, s);
  }
}

void bapply(chns_batch* b, int block, const double* x, double* y, double alpha, double beta,
            const int* act, hipStream_t s) {
  BLevel& L0 = b->lv[0];
  if (block == CHNS_BLOCK_CH)
    bch_block<double>(L0.st, L0.M, L0.K, L0.M, b->c12, b->c22, act, x, alpha, beta, y, s);
  else
    bstencil<double>(L0.st, L0.v64[2], 0, x, nullptr, nullptr, nullptr, alpha, beta, nullptr,
                     nullptr, nullptr, act, y, s);
}

int any_active(chns_batch* b, hipStream_t s, bool& any) {
  std::vector<int> act(b->count);
  BCHK(b, hipMemcpyAsync(act.data(), b->active, b->count * sizeof(int), hipMemcpyDeviceToHost, s));
  BCHK(b, hipStreamSynchronize(s));
  any = false;
  for (int a : act) any = any || a;
  return CHNS_OK;
}

__global__ void k_not_into(int n, const int* __restrict__ a, int* __restrict__ o) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) o[i] = a[i] ? 0 : 1;
}

// Batched right-preconditioned FGMRES.  Eager mode: FGMRES(restart) up to
// maxiter Arnoldi steps, stopping once every instance has converged (activity
// read back every EAGER_CHECK steps and after each cycle).  Graph mode: a fixed
// budget B = min(maxiter, budget of the block) of Arnoldi steps in cycles of
// min(restart, B) steps, with no host synchronisation; an instance that
// converges within the first cycle takes exactly the eager iterations.
int bfgmres(chns_batch* b, int block, const double* rhs, double* x, const chns_solve_opts& o,
            bool eager, hipStream_t s) {
  const int bi = block == CHNS_BLOCK_CH ? 0 : 1;
  int budget = o.maxiter;
  if (!eager && b->budget[bi] > 0) budget = std::min(budget, b->budget[bi]);
  const int m = eager ? o.restart : std::min(o.restart, budget);
  const int cycles = (budget + m - 1) / m;
  const int64_t n = (block == CHNS_BLOCK_CH ? 2 : 1) * b->Ntot;
  const int nchunk = int(n / BCHUNK);
  const int half = (block == CHNS_BLOCK_CH) ? b->nchunk1 : 0;
  const int* act = b->active;
  double* V = b->V;
  const int64_t ld = b->ld;
  const int rs = 2 * BMAX_RESTART + 3, cstride = 2 * BMAX_RESTART + 2;
  dfill_int(b->count, 0, b->iters[bi], s);
  bnorm_partial(n, rhs, b->part, s);
  bnorm_finish(b->count, nchunk, b->part, b->cr, half, m, 1, o.rtol, o.atol, b->nrm, b->inv, b->g,
               b->tol, b->active, b->kcols, s);
  for (int cyc = 0; cyc <= cycles; ++cyc) {
    // true residual of every instance decides its activity for this cycle
    dcopy(n, rhs, V, s);
    bapply(b, block, x, V, -1.0, 1.0, nullptr, s);
    bnorm_partial(n, V, b->part, s);
    bnorm_finish(b->count, nchunk, b->part, b->cr, half, m, 0, o.rtol, o.atol, b->nrm, b->inv,
                 b->g, b->tol, b->active, b->kcols, s);
    if (cyc == cycles) break;  // final true residual only
    if (eager) {
      bool any = false;
      BTRY(any_active(b, s, any));
      if (!any) break;
    }
    bscale(n, V, b->inv, b->cinst, act, V, s);
    for (int j = 0; j < m; ++j) {
      double* vj = V + int64_t(j) * ld;
      double* vn = V + int64_t(j + 1) * ld;
      double* zj = b->Z + int64_t(j) * ld;
      // v_j is stored unnormalised (j > 0): its 1/|w| scales the
      // preconditioner's output and is applied on load by the two passes,
      // which store v_j normalised
      const double* vs = j > 0 ? b->inv : nullptr;
      bprecond(b, block, vj, vs, zj, act, o, s);
      bapply(b, block, zj, vn, 1.0, 0.0, act, s);
      // DCGS2: one dot pass and one update pass over each instance's basis
      bdcgs_dots(n, V, ld, j, b->part, b->cinst, act, vs, s, b->dots_group);
      bslot_reduce(b->count, nchunk, 2 * j + 3, b->part, b->cr, half, b->red, rs, act, s);
      bdcgs_coef(b->count, j, m, b->red, rs, b->H, b->coef, cstride, act, s);
      bdcgs_update(n, V, ld, j, b->coef, cstride, b->part2, b->cinst, act, vs, s, b->upd_threads);
      bdcgs_finish(b->count, nchunk, b->part2, b->cr, half, j, m, b->H, b->HR, b->cs, b->sn, b->g,
                   b->gp, b->inv, b->tol, b->active, b->kcols, b->iters[bi], s);
      if (eager && (j + 1) % EAGER_CHECK == 0 && j + 1 < m) {
        bool any = false;
        BTRY(any_active(b, s, any));
        if (!any) break;
      }
    }
    blsq(b->count, m, b->HR, b->gp, b->kcols, b->y, s);
    bxupdate(n, b->Z, ld, m, b->y, x, b->cinst, b->kcols, s);
  }
  hipLaunchKernelGGL(k_not_into, dim3((b->count + 63) / 64), dim3(64), 0, s, b->count, b->active,
                     b->conv[bi]);
  BCHK(b, hipGetLastError());
  return CHNS_OK;
}

// One step from (phi, mu, Phi) into (ophi, omu, oPhi); the sources are read
// before any output is written, so the two sets may coincide.
int bstep(chns_batch* b, const double* phi, const double* mu, const double* Phi, double* ophi,
          double* omu, double* oPhi, const chns_solve_opts& o, bool eager, hipStream_t s) {
  const int64_t N = b->Ntot;
  BLevel& L0 = b->lv[0];
  brhs_binary(L0.st, L0.M, phi, Phi, b->cmu, b->cac, b->rhs_ch, b->rhs_ac, s);
  dcopy(N, phi, b->xch, s);
  dcopy(N, mu, b->xch + N, s);
  dcopy(N, Phi, b->xac, s);
  BTRY(bfgmres(b, CHNS_BLOCK_CH, b->rhs_ch, b->xch, o, eager, s));
  BTRY(bfgmres(b, CHNS_BLOCK_AC, b->rhs_ac, b->xac, o, eager, s));
  dcopy(N, b->xch, ophi, s);
  dcopy(N, b->xch + N, omu, s);
  dcopy(N, b->xac, oPhi, s);
  BCHK(b, hipGetLastError());
  return CHNS_OK;
}

int bbuild(chns_batch* b) {
  BTRY(build_levels(b));
  const int64_t N = b->lv[0].nrows;
  b->Ntot = N;
  b->off.assign(b->count + 1, 0);
  for (int i = 0; i < b->count; ++i) b->off[i + 1] = b->off[i] + int64_t(b->n[i]) * b->n[i];
  for (int i = 0; i < b->count; ++i)
    if (b->lv[0].roff[i] != b->off[i]) return fail(b, CHNS_EINVAL, "instance offsets not packed");
  // per-instance scalars
  std::vector<double> c12(b->count), c22(b->count), cmu(b->count), cac(b->count);
  for (int i = 0; i < b->count; ++i) {
    const auto& p = b->prm[i];
    const double tg = p.tau * p.mobility, be = p.eps * p.eps;
    c12[i] = tg;
    c22[i] = -tg / be;
    cmu[i] = -tg / be;
    cac[i] = -p.tau * p.evap_rate;
  }
  BTRY(bupload(b, &b->c12, c12));
  BTRY(bupload(b, &b->c22, c22));
  BTRY(bupload(b, &b->cmu, cmu));
  BTRY(bupload(b, &b->cac, cac));
  // chunks
  b->nchunk1 = int(N / BCHUNK);
  std::vector<int> cinst(2 * b->nchunk1), cr(2 * b->count);
  for (int i = 0; i < b->count; ++i) {
    cr[2 * i] = int(b->off[i] / BCHUNK);
    cr[2 * i + 1] = int(b->off[i + 1] / BCHUNK);
    for (int c = cr[2 * i]; c < cr[2 * i + 1]; ++c) cinst[c] = cinst[c + b->nchunk1] = i;
  }
  BTRY(bupload(b, &b->cinst, cinst));
  BTRY(bupload(b, &b->cr, cr));
  // values and vectors per level
  for (size_t l = 0; l < b->lv.size(); ++l) {
    BLevel& L = b->lv[l];
    const size_t ns = L.slots, nr = L.nrows;
    BTRY(balloc(b, &L.M, ns));
    BTRY(balloc(b, &L.K, ns));
    BTRY(balloc(b, &L.M32, ns));
    for (int op = 0; op < NOPS; ++op) {
      BTRY(balloc(b, &L.v64[op], ns));
      BTRY(balloc(b, &L.v32[op], ns));
      BTRY(balloc(b, &L.d64[op], nr));
      BTRY(balloc(b, &L.d32[op], nr));
      std::vector<double> a(b->count), bb(b->count);
      for (int i = 0; i < b->count; ++i) {
        a[i] = op_a(b->prm[i], op);
        bb[i] = op_b(b->prm[i], op);
      }
      BTRY(bupload(b, &L.aco[op][0], a));
      BTRY(bupload(b, &L.aco[op][1], bb));
    }
    for (double** v : {&L.b64, &L.x64, &L.t64, &L.r64, &L.dd64}) BTRY(balloc(b, v, nr));
    for (float** v : {&L.b32, &L.x32, &L.t32, &L.r32, &L.dd32}) BTRY(balloc(b, v, nr));
    // tables of the options-dependent cycle (masks, coarse Chebyshev
    // coefficients, tile and tail lists), rewritten when the options change
    L.tile_cap = 0;
    for (int i = 0; i < b->count; ++i)
      if (L.roff[i] >= 0) L.tile_cap += size_t(btile_count(b->n[i] >> l));
    const size_t nc = size_t(MAXCHEB) * b->count;
    for (int op = 0; op < NOPS; ++op) {
      BTRY(balloc(b, &L.smooth[op], size_t(L.nslices)));
      BTRY(balloc(b, &L.coarse[op], size_t(L.nslices)));
      BTRY(balloc(b, &L.present[op], size_t(L.nslices)));
      BTRY(balloc(b, &L.cc64[op][0], nc));
      BTRY(balloc(b, &L.cc64[op][1], nc));
      BTRY(balloc(b, &L.cc32[op][0], nc));
      BTRY(balloc(b, &L.cc32[op][1], nc));
      BTRY(balloc(b, &L.tdown[op], std::max<size_t>(L.tile_cap, 1)));
      BTRY(balloc(b, &L.tzero[op], std::max<size_t>(L.tile_cap, 1)));
      BTRY(balloc(b, &L.tail_idx[op], size_t(b->count)));
    }
    BCHK(b, hipMemset(L.M, 0, ns * sizeof(double)));
    BCHK(b, hipMemset(L.K, 0, ns * sizeof(double)));
    // padding rows (partial slices of tiny levels): unit diagonal keeps 1/diag finite
    BCHK(b, hipMemset(L.b64, 0, nr * sizeof(double)));
  }
  // assembly of M and K on the finest level, instance by instance
  BLevel& L0 = b->lv[0];
  for (int i = 0; i < b->count; ++i) {
    SizeTables* T = tables_for(b, b->n[i]);
    if (!T->d_eslot) {
      BTRY(bupload(b, &T->d_ep2, T->el.p2));
      BTRY(bupload(b, &T->d_etype, T->el.type));
      BTRY(bupload(b, &T->d_eslot, T->eslot));
    }
    const int64_t so = int64_t(L0.roff[i]) * 7;
    for (int col = 0; col < 8; ++col) {
      assemble_p1(0, T->el.colour_ptr[col], T->el.colour_ptr[col + 1], T->d_ep2, T->d_etype,
                  T->d_eslot, 1.0 / b->n[i], nullptr, 0, L0.M + so, nullptr);
      assemble_p1(1, T->el.colour_ptr[col], T->el.colour_ptr[col + 1], T->d_ep2, T->d_etype,
                  T->d_eslot, 1.0 / b->n[i], nullptr, 0, L0.K + so, nullptr);
    }
  }
  for (size_t l = 0; l + 1 < b->lv.size(); ++l) {
    BLevel& F = b->lv[l];
    BLevel& G = b->lv[l + 1];
    galerkin(G.slots, F.gptr, F.gsrc, F.gw, F.M, G.M, nullptr);
    galerkin(G.slots, F.gptr, F.gsrc, F.gw, F.K, G.K, nullptr);
  }
  for (auto& L : b->lv) {
    convert<double, float>(L.slots, L.M, L.M32, nullptr);
    for (int op = 0; op < NOPS; ++op) {
      bcombine(L.slots, L.sinst, L.aco[op][0], L.M, L.aco[op][1], L.K, L.v64[op], L.v32[op], nullptr);
      diag_inverse(L.nrows, L.diag, L.v64[op], L.d64[op], L.d32[op], nullptr);
    }
  }
  BCHK(b, hipGetLastError());
  // Krylov workspace for the CH block (2N) with restart <= BMAX_RESTART
  const size_t n2 = 2 * size_t(N), cnt = size_t(b->count), m = BMAX_RESTART;
  b->ld = int64_t(n2) + KRYLOV_PAD;
  BTRY(balloc(b, &b->V, (m + 1) * size_t(b->ld)));
  BTRY(balloc(b, &b->Z, m * size_t(b->ld)));
  BTRY(balloc(b, &b->H, cnt * (m + 1) * m));
  BTRY(balloc(b, &b->HR, cnt * (m + 1) * m));
  BTRY(balloc(b, &b->cs, cnt * (m + 1)));
  BTRY(balloc(b, &b->sn, cnt * (m + 1)));
  BTRY(balloc(b, &b->g, cnt * (m + 2)));
  BTRY(balloc(b, &b->gp, cnt * (m + 2)));
  BTRY(balloc(b, &b->y, cnt * (m + 1)));
  BTRY(balloc(b, &b->red, cnt * (2 * m + 3)));
  BTRY(balloc(b, &b->coef, cnt * (2 * m + 2)));
  for (int op = 0; op < NOPS; ++op) {
    BTRY(balloc(b, &b->tails32[op], cnt));
    BTRY(balloc(b, &b->tails64[op], cnt));
  }
  BTRY(balloc(b, &b->wl_ctr, 16));
  BCHK(b, hipMemset(b->wl_ctr, 0, 16 * sizeof(int)));
  for (double** v : {&b->inv, &b->nrm, &b->tol}) BTRY(balloc(b, v, cnt));
  for (int** v : {&b->active, &b->kcols, &b->iters[0], &b->iters[1], &b->conv[0], &b->conv[1]})
    BTRY(balloc(b, v, cnt));
  BTRY(balloc(b, &b->part, (2 * m + 3) * n2 / BCHUNK));
  BTRY(balloc(b, &b->part2, n2 / BCHUNK));
  for (double** v : {&b->rhs_ch, &b->xch}) BTRY(balloc(b, v, n2));
  for (double** v : {&b->rhs_ac, &b->xac, &b->w64a, &b->w64b}) BTRY(balloc(b, v, size_t(N)));
  for (float** v : {&b->r32, &b->z32}) BTRY(balloc(b, v, n2));
  for (float** v : {&b->w32a, &b->w32b}) BTRY(balloc(b, v, size_t(N)));
  BCHK(b, hipEventCreate(&b->ev0));
  BCHK(b, hipEventCreate(&b->ev1));
  BCHK(b, hipDeviceSynchronize());
  return CHNS_OK;
}

void drop_graphs(chns_batch* b) {
  for (auto& g : b->graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
  }
  b->graphs.clear();
}

// Kernel launches of one V-cycle of operator op from level l (mirrors bvcycle
// and bvcycle_tiled).
size_t vcycle_launches(const chns_batch* b, int op, int l, const chns_solve_opts& o) {
  const BLevel& L = b->lv[l];
  size_t c = 0;
  if (b->tiled) {
    c += (L.ntzero[op] > 0 ? 1 : 0) + (L.ntail[op] > 0 ? 1 : 0);
    if (L.ntdown[op] > 0) c += 2 + vcycle_launches(b, op, l + 1, o);
    return c;
  }
  if (L.nsmooth[op] > 0) c += size_t(o.mg_pre) + 3 + o.mg_post + vcycle_launches(b, op, l + 1, o);
  if (L.ncoarse[op] > 0) c += size_t(l > 0 ? o.mg_coarse : o.mg_pre + o.mg_post);
  return c;
}

// Kernel launches of one graph-mode step (mirrors bstep and bfgmres), so that an
// oversized graph is refused before it is captured.
size_t step_launches(const chns_batch* b, const chns_solve_opts& o) {
  size_t total = 1 + 3 + 3;  // right-hand sides, input copies, output copies
  for (int bi = 0; bi < 2; ++bi) {
    int budget = o.maxiter;
    if (b->budget[bi] > 0) budget = std::min(budget, b->budget[bi]);
    const int m = std::min(o.restart, budget);
    const size_t cycles = size_t((budget + m - 1) / m);
    const size_t pre = bi == 0 ? 3 * vcycle_launches(b, 0, 0, o) + 1 : vcycle_launches(b, 2, 0, o);
    // input stage (convert or scale) and output conversion, operator, dot
    // launches, slot sums, coefficients, update, finish
    const size_t arnoldi = pre + (o.precision == CHNS_MIXED ? 2 : 1) + 1 + (1 + size_t(m - 1) / 16) + 4;
    total += 3 + cycles * (4 + 1 + size_t(m) * arnoldi + 2) + 4 + 1;
  }
  return total;
}

// Executable graph of `ksteps` consecutive steps, captured on first use and
// cached by pointers, stream, options and step count: the first step reads
// (phi, mu, Phi), each later one the previous step's output (or the inputs
// again when each_from_input), every step writes the output fields.
int step_graph(chns_batch* b, const double* phi, const double* mu, const double* Phi, double* ophi,
               double* omu, double* oPhi, int ksteps, bool each_from_input, const chns_solve_opts& o,
               hipStream_t s, hipGraphExec_t* out) {
  char key[512];
  std::snprintf(key, sizeof key, "%p/%p/%p/%p/%p/%p/%p/%s/%d/%d/%d/%.17g/%.17g/%d/%d/%d/%d", (const void*)phi,
                (const void*)mu, (const void*)Phi, (void*)ophi, (void*)omu, (void*)oPhi, (void*)s,
                b->opts_key.c_str(), o.restart, o.maxiter, o.precision, o.rtol, o.atol, b->budget[0],
                b->budget[1], ksteps, each_from_input ? 1 : 0);
  for (size_t i = 0; i < b->graphs.size(); ++i)
    if (b->graphs[i].key == key) {  // most recently used goes last
      GraphEntry g = b->graphs[i];
      b->graphs.erase(b->graphs.begin() + i);
      b->graphs.push_back(g);
      *out = g.exec;
      return CHNS_OK;
    }
  const size_t expect = step_launches(b, o) * size_t(ksteps);
  if (expect > GRAPH_MAX_NODES)
    return fail(b, CHNS_EUNSUPPORTED,
                "a graph of " + std::to_string(expect) + " kernels exceeds " +
                    std::to_string(GRAPH_MAX_NODES) + "; set a smaller graph budget or maxiter");
  BCHK(b, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
  int rc = CHNS_OK;
  for (int k = 0; k < ksteps && rc >= 0; ++k) {
    const bool from_in = k == 0 || each_from_input;
    rc = bstep(b, from_in ? phi : ophi, from_in ? mu : omu, from_in ? Phi : oPhi, ophi, omu, oPhi, o, false, s);
  }
  hipGraph_t gr = nullptr;
  const hipError_t e = hipStreamEndCapture(s, &gr);
  if (rc < 0) {
    if (gr) (void)hipGraphDestroy(gr);
    return rc;
  }
  if (e != hipSuccess) return fail(b, CHNS_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  size_t nodes = 0;
  const hipError_t en = hipGraphGetNodes(gr, nullptr, &nodes);
  if (en != hipSuccess || nodes > GRAPH_MAX_NODES) {
    (void)hipGraphDestroy(gr);
    if (en != hipSuccess) return fail(b, CHNS_EHIP, std::string("hipGraphGetNodes: ") + hipGetErrorString(en));
    return fail(b, CHNS_EUNSUPPORTED, "captured " + std::to_string(nodes) + " graph nodes, over " +
                                          std::to_string(GRAPH_MAX_NODES));
  }
  GraphEntry g;
  g.key = key;
  g.graph = gr;
  const hipError_t ei = hipGraphInstantiate(&g.exec, gr, nullptr, nullptr, 0);
  if (ei != hipSuccess) {
    (void)hipGraphDestroy(gr);
    return fail(b, CHNS_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
  }
  if (int(b->graphs.size()) >= GRAPH_CACHE) {
    (void)hipGraphExecDestroy(b->graphs.front().exec);
    (void)hipGraphDestroy(b->graphs.front().graph);
    b->graphs.erase(b->graphs.begin());
  }
  b->graphs.push_back(g);
  *out = g.exec;
  return CHNS_OK;
}

void brelease(chns_batch* b) {
  drop_graphs(b);
  for (void* p : b->allocs) {
    if (b->free_)
      b->free_(p, b->alloc_ctx);
    else
      (void)hipFree(p);
  }
  b->allocs.clear();
  if (b->ev0) (void)hipEventDestroy(b->ev0);
  if (b->ev1) (void)hipEventDestroy(b->ev1);
}

int check_bopts(chns_batch* b, const chns_solve_opts* o) {
  if (!o) return fail(b, CHNS_EINVAL, "opts is NULL");
  if (!(o->rtol >= 0) || !(o->atol >= 0) || !std::isfinite(o->rtol) || !std::isfinite(o->atol))
    return fail(b, CHNS_EINVAL, "rtol/atol must be finite and >= 0");
  if (o->restart < 1 || o->restart > BMAX_RESTART) return fail(b, CHNS_EINVAL, "restart must be in 1..64");
  if (o->maxiter < 1 || o->maxiter > 4096) return fail(b, CHNS_EINVAL, "maxiter must be in 1..4096");
  if (o->precision != CHNS_F64 && o->precision != CHNS_MIXED) return fail(b, CHNS_EINVAL, "unknown precision");
  if (o->mg_cycles != 1) return fail(b, CHNS_EUNSUPPORTED, "the batched form runs one cycle per inner solve");
  if (o->mg_pre < 1 || o->mg_pre > 32 || o->mg_post < 0 || o->mg_post > 32 || o->mg_coarse < 1 ||
      o->mg_coarse > MAXCHEB || o->mg_pre + o->mg_post > MAXCHEB)
    return fail(b, CHNS_EINVAL, "multigrid step counts out of range");
  if (!(o->mg_lmax > 0.0 && o->mg_lmax < 100.0) || !(o->mg_rho_cut >= 0.0))
    return fail(b, CHNS_EINVAL, "bad mg_lmax / mg_rho_cut");
  return CHNS_OK;
}

}  // namespace

extern "C" {

int chns_batch_create(int32_t count, const int32_t* h_n, const chns_params* h_params, chns_alloc_fn alloc,
                      chns_free_fn free_, void* alloc_ctx, chns_batch** out) {
  if (!out) return CHNS_EINVAL;
  *out = nullptr;
  if ((alloc == nullptr) != (free_ == nullptr)) {
    g_batch_err = "alloc and free must both be given or both be NULL";
    return CHNS_EINVAL;
  }
  if (count < 1 || count > 4096 || !h_n || !h_params) {
    g_batch_err = "count must be in 1..4096 with sizes and parameters";
    return CHNS_EINVAL;
  }
  for (int i = 0; i < count; ++i) {
    if (h_n[i] < 32 || h_n[i] > 2048 || h_n[i] % 32 != 0) {
      g_batch_err = "each n must be a multiple of 32 in 32..2048";
      return CHNS_EINVAL;
    }
    const chns_params& p = h_params[i];
    const double v[] = {p.eps, p.tau, p.mobility, p.evap_rate};
    for (double x : v)
      if (!std::isfinite(x)) {
        g_batch_err = "parameter is NaN or Inf";
        return CHNS_EINVAL;
      }
    if (p.eps <= 0 || p.tau <= 0 || p.mobility <= 0 || p.evap_rate < 0) {
      g_batch_err = "eps, tau, mobility must be positive and evap_rate >= 0";
      return CHNS_EINVAL;
    }
    if (p.top_flux != 0.0) {  // instances live on periodic squares
      g_batch_err = "the top-wall flux belongs to the closed square";
      return CHNS_EINVAL;
    }
    if (p.beta_phase[0] != 0.0 || p.beta_phase[1] != 0.0 || p.beta_phase[2] != 0.0 || p.beta_phase[3] != 0.0) {
      g_batch_err = "per-phase gradient coefficients belong to the quaternary model";
      return CHNS_EINVAL;
    }
  }
  chns_batch* b = new chns_batch();
  b->alloc = alloc;
  b->free_ = free_;
  b->alloc_ctx = alloc_ctx;
  b->count = count;
  b->n.assign(h_n, h_n + count);
  b->prm.assign(h_params, h_params + count);
  const int rc = bbuild(b);
  if (rc < 0) {
    g_batch_err = b->err;
    brelease(b);
    delete b;
    return rc;
  }
  *out = b;
  return CHNS_OK;
}

int chns_batch_destroy(chns_batch* b) {
  if (!b) return CHNS_EINVAL;
  (void)hipDeviceSynchronize();
  brelease(b);
  delete b;
  return CHNS_OK;
}

int chns_batch_offsets(const chns_batch* b, int64_t* h_offsets) {
  if (!b || !h_offsets) return CHNS_EINVAL;
  std::memcpy(h_offsets, b->off.data(), (b->count + 1) * sizeof(int64_t));
  return CHNS_OK;
}

int chns_batch_timestep(chns_batch* b, const double* in_phi, const double* in_mu, const double* in_Phi,
                        double* d_phi, double* d_mu, double* d_Phi, int32_t nsteps,
                        int32_t each_from_input, const chns_solve_opts* opts, int32_t use_graph,
                        int32_t* h_iters, int32_t* h_conv, double* h_ms, void* stream) {
  if (!b) return CHNS_EINVAL;
  BTRY(check_bopts(b, opts));
  if (!in_phi || !in_mu || !in_Phi || !d_phi || !d_mu || !d_Phi || nsteps < 1 || nsteps > 1000)
    return fail(b, CHNS_EINVAL, "fields must be non-NULL and nsteps in 1..1000");
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (use_graph && !s) return fail(b, CHNS_EINVAL, "graph capture needs a non-default stream");
  BTRY(prepare_cycles(b, *opts));
  // graph mode: graphs of G = min(nsteps, GRAPH_STEPS) steps (fewer if a
  // graph would exceed the node limit), the first reading the inputs, the
  // others continuing from the outputs, and one more graph for a remainder
  hipGraphExec_t first = nullptr, cont = nullptr, rest = nullptr;
  int G = 1, full = 0, rem = 0;
  if (use_graph) {
    const size_t per = std::max<size_t>(step_launches(b, *opts), 1);
    G = int(std::min<size_t>({size_t(nsteps), size_t(GRAPH_STEPS), std::max<size_t>(GRAPH_MAX_NODES / per, 1)}));
    full = nsteps / G;
    rem = nsteps - full * G;
    const bool efi = each_from_input != 0;
    BTRY(step_graph(b, in_phi, in_mu, in_Phi, d_phi, d_mu, d_Phi, G, efi, *opts, s, &first));
    if (full > 1)
      BTRY(efi ? step_graph(b, in_phi, in_mu, in_Phi, d_phi, d_mu, d_Phi, G, true, *opts, s, &cont)
               : step_graph(b, d_phi, d_mu, d_Phi, d_phi, d_mu, d_Phi, G, false, *opts, s, &cont));
    if (rem > 0)
      BTRY(efi ? step_graph(b, in_phi, in_mu, in_Phi, d_phi, d_mu, d_Phi, rem, true, *opts, s, &rest)
               : step_graph(b, d_phi, d_mu, d_Phi, d_phi, d_mu, d_Phi, rem, false, *opts, s, &rest));
  }
  BCHK(b, hipEventRecord(b->ev0, s));
  if (use_graph) {
    for (int k = 0; k < full; ++k) BCHK(b, hipGraphLaunch(k == 0 ? first : cont, s));
    if (rem > 0) BCHK(b, hipGraphLaunch(rest, s));
  } else {
    for (int k = 0; k < nsteps; ++k) {
      const bool from_in = (k == 0) || each_from_input;
      BTRY(bstep(b, from_in ? in_phi : d_phi, from_in ? in_mu : d_mu, from_in ? in_Phi : d_Phi, d_phi,
                 d_mu, d_Phi, *opts, true, s));
    }
  }
  BCHK(b, hipEventRecord(b->ev1, s));
  BCHK(b, hipEventSynchronize(b->ev1));
  float ms = 0.f;
  BCHK(b, hipEventElapsedTime(&ms, b->ev0, b->ev1));
  if (h_ms) *h_ms = ms;
  if (h_iters) {
    BCHK(b, hipMemcpy(h_iters, b->iters[0], b->count * sizeof(int), hipMemcpyDeviceToHost));
    BCHK(b, hipMemcpy(h_iters + b->count, b->iters[1], b->count * sizeof(int), hipMemcpyDeviceToHost));
  }
  int worst = CHNS_OK;
  std::vector<int> c0(b->count), c1(b->count);
  BCHK(b, hipMemcpy(c0.data(), b->conv[0], b->count * sizeof(int), hipMemcpyDeviceToHost));
  BCHK(b, hipMemcpy(c1.data(), b->conv[1], b->count * sizeof(int), hipMemcpyDeviceToHost));
  for (int i = 0; i < b->count; ++i) {
    if (!c0[i] || !c1[i]) worst = CHNS_WNOCONV;
    if (h_conv) {
      h_conv[i] = c0[i];
      h_conv[b->count + i] = c1[i];
    }
  }
  return worst;
}

int chns_batch_tune(chns_batch* b, const char* cache_path, void* stream) {
  if (!b) return CHNS_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  // cache lines: "level rows rpt block" (smoothing kernel per level size),
  // "update threads" and "dots group" (Gram-Schmidt passes, keyed by the
  // batch's stacked size: "update rows threads", "dots rows group")
  std::map<int, std::pair<int, int>> cache, upd, dots;
  if (cache_path) {
    if (FILE* f = std::fopen(cache_path, "r")) {
      char arch[64], line[256];
      if (std::fscanf(f, "%63s\n", arch) == 1 && std::string(arch) == "gfx950")
        while (std::fgets(line, sizeof line, f)) {
          int a, c, d;
          if (std::sscanf(line, "level %d %d %d", &a, &c, &d) == 3) cache[a] = {c, d};
          else if (std::sscanf(line, "update %d %d", &a, &c) == 2) upd[a] = {c, 0};
          else if (std::sscanf(line, "dots %d %d", &a, &c) == 2) dots[a] = {c, 0};
        }
      std::fclose(f);
    }
  }
  auto time_ms = [&](auto&& launch, int reps, float& ms) -> int {
    for (int w = 0; w < 2; ++w) launch();
    BCHK(b, hipEventRecord(b->ev0, s));
    for (int w = 0; w < reps; ++w) launch();
    BCHK(b, hipEventRecord(b->ev1, s));
    BCHK(b, hipEventSynchronize(b->ev1));
    BCHK(b, hipEventElapsedTime(&ms, b->ev0, b->ev1));
    return CHNS_OK;
  };
  const int rpts[3] = {1, 2, 4};
  const int blocks[4] = {128, 256, 512, 1024};
  for (auto& L : b->lv) {
    auto it = cache.find(L.nrows);
    if (it != cache.end()) {
      L.st.rpt = it->second.first;
      L.st.block = it->second.second;
      continue;
    }
    float best = 1e30f;
    int br = 1, bb = 256;
    for (int rpt : rpts)
      for (int blk : blocks) {
        BStencil st = L.st;
        st.rpt = rpt;
        st.block = blk;
        float ms = 0.f;
        BTRY(time_ms([&] {
          bstencil<float>(st, L.v32[1], 2, L.x32, L.b32, L.d32[1], L.dd32, 0.5f, 0.5f, nullptr, nullptr,
                          nullptr, nullptr, L.t32, s);
        }, 10, ms));
        if (ms < best) {
          best = ms;
          br = rpt;
          bb = blk;
        }
      }
    L.st.rpt = br;
    L.st.block = bb;
    cache[L.nrows] = {br, bb};
  }
  // Gram-Schmidt passes on the stacked CH vectors (2 Ntot rows), at a
  // mid-cycle step: the update pass's workgroup per chunk, the dot pass's
  // vectors per launch.  The workspace holds no solve yet: its contents are
  // only timed, and the coefficients are zeroed first.
  const int64_t n2 = 2 * b->Ntot;
  const int key = int(std::min<int64_t>(n2, INT32_MAX));
  const int cstride = 2 * BMAX_RESTART + 2;
  BCHK(b, hipMemsetAsync(b->coef, 0, size_t(b->count) * cstride * sizeof(double), s));
  if (auto it = upd.find(key); it != upd.end()) {
    b->upd_threads = it->second.first;
  } else {
    float best = 1e30f;
    for (int nt : {256, 512, 1024}) {
      float ms = 0.f;
      BTRY(time_ms([&] {
        bdcgs_update(n2, b->V, b->ld, 16, b->coef, cstride, b->part2, b->cinst, nullptr, nullptr, s, nt);
      }, 5, ms));
      if (ms < best) {
        best = ms;
        b->upd_threads = nt;
      }
    }
  }
  if (auto it = dots.find(key); it != dots.end()) {
    b->dots_group = it->second.first;
  } else {
    float best = 1e30f;
    for (int g : {8, 16}) {
      float ms = 0.f;
      BTRY(time_ms([&] { bdcgs_dots(n2, b->V, b->ld, 32, b->part, b->cinst, nullptr, nullptr, s, g); }, 5, ms));
      if (ms < best) {
        best = ms;
        b->dots_group = g;
      }
    }
  }
  upd[key] = {b->upd_threads, 0};
  dots[key] = {b->dots_group, 0};
  if (cache_path) {
    if (FILE* f = std::fopen(cache_path, "w")) {
      std::fprintf(f, "gfx950\n");
      for (auto& e : cache) std::fprintf(f, "level %d %d %d\n", e.first, e.second.first, e.second.second);
      for (auto& e : upd) std::fprintf(f, "update %d %d\n", e.first, e.second.first);
      for (auto& e : dots) std::fprintf(f, "dots %d %d\n", e.first, e.second.first);
      std::fclose(f);
    }
  }
  BCHK(b, hipStreamSynchronize(s));
  drop_graphs(b);  // launch shapes changed
  return CHNS_OK;
}

int chns_batch_set_worklist(chns_batch* b, int32_t grid) {
  if (!b) return CHNS_EINVAL;
  if (grid < 0 || grid > 65536) return fail(b, CHNS_EINVAL, "work-list grid must be in 0..65536");
  if (grid != b->wl_grid) {
    BCHK(b, hipDeviceSynchronize());
    drop_graphs(b);  // the captured launches have the old shape
  }
  b->wl_grid = grid;
  return CHNS_OK;
}

// Launch shapes the autotuner chose (or the defaults).
int chns_batch_tuned(const chns_batch* b, int32_t* h_update_threads, int32_t* h_dots_group) {
  if (!b) return CHNS_EINVAL;
  if (h_update_threads) *h_update_threads = b->upd_threads;
  if (h_dots_group) *h_dots_group = b->dots_group;
  return CHNS_OK;
}

int chns_batch_set_graph_budget(chns_batch* b, int32_t ch_iters, int32_t ac_iters) {
  if (!b) return CHNS_EINVAL;
  if (ch_iters < 0 || ch_iters > 4096 || ac_iters < 0 || ac_iters > 4096)
    return fail(b, CHNS_EINVAL, "graph budgets must be in 0..4096");
  b->budget[0] = ch_iters;
  b->budget[1] = ac_iters;
  return CHNS_OK;
}

int chns_batch_precond_apply(chns_batch* b, int32_t block, const double* d_r, double* d_z,
                             const chns_solve_opts* opts, void* stream) {
  if (!b) return CHNS_EINVAL;
  BTRY(check_bopts(b, opts));
  if (block != CHNS_BLOCK_CH && block != CHNS_BLOCK_AC) return fail(b, CHNS_EINVAL, "block must be CH or AC");
  if (!d_r || !d_z) return fail(b, CHNS_EINVAL, "r and z must be non-NULL");
  const int64_t n = (block == CHNS_BLOCK_CH ? 2 : 1) * b->Ntot;
  if (d_r < d_z + n && d_z < d_r + n) return fail(b, CHNS_EINVAL, "r and z overlap");
  hipStream_t s = static_cast<hipStream_t>(stream);
  BTRY(prepare_cycles(b, *opts));
  bprecond(b, block, d_r, nullptr, d_z, nullptr, *opts, s);
  BCHK(b, hipGetLastError());
  return CHNS_OK;
}

const char* chns_batch_last_error(const chns_batch* b) {
  if (!b) return g_batch_err.c_str();
  return b->err.c_str();
}

}  // extern "C"
