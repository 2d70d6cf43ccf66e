// Solver context: device-resident matrices, multigrid levels and Krylov
// workspace behind the C-ABI of chns.h.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/chns.h"
#include "host_mesh.hpp"
#include "kernels.hpp"

namespace chns {

constexpr int MAX_RESTART = 64;

// Values of one operator on one level, FP64 plus FP32 copy, and 1/diag.
struct OpVals {
  double* v64 = nullptr;
  float* v32 = nullptr;
  double* d64 = nullptr;
  float* d32 = nullptr;
};

struct Level {
  int n = 0, N = 0;
  Csr csr;
  Sell sell;
  DSell d;
  int* diag = nullptr;
  // transfer to the next coarser level
  Csr Pcsr, Rcsr;
  std::vector<double> Pval, Rval;
  Sell Psell, Rsell;
  DSell dP, dR;
  double *P64 = nullptr, *R64 = nullptr;
  float *P32 = nullptr, *R32 = nullptr;
  int *gptr = nullptr, *gsrc = nullptr;
  double* gw = nullptr;
  // base value streams
  double *M = nullptr, *K = nullptr, *C = nullptr;
  float *M32 = nullptr, *K32 = nullptr, *C32 = nullptr;
  // preconditioner operators
  OpVals L, X, AC;
  // ternary model: velocity blocks (Galerkin from P2), pressure Laplacian and
  // mass (values = K, M), and on the finest level the PCD matrix A_p and the
  // P1 convection by the Oseen convecting field
  OpVals Vx, Vy, Kp, Mp, Ap;
  double* Cw = nullptr;
  double* Mrp = nullptr;  // finest level: P1 mass weighted by rho^k (the PCD matrix's)
  // multigrid work vectors (per precision)
  double *b64 = nullptr, *x64 = nullptr, *t64 = nullptr, *r64 = nullptr, *e64 = nullptr;
  float *b32 = nullptr, *x32 = nullptr, *t32 = nullptr, *r32 = nullptr, *e32 = nullptr;
  double* d64 = nullptr;  // Chebyshev direction
  float* d32 = nullptr;
};

// The P2 velocity level on the finest mesh (ternary model).
struct P2Level {
  int N4 = 0;
  Csr csr;
  Sell sell;
  DSell d;
  Csr Pcsr, Rcsr;  // P1 -> P2 on the same mesh, and its transpose
  std::vector<double> Pval, Rval;
  Sell Psell, Rsell;
  DSell dP, dR;
  double *P64 = nullptr, *R64 = nullptr;
  float *P32 = nullptr, *R32 = nullptr;
  int *gptr = nullptr, *gsrc = nullptr;  // Galerkin map P2 -> P1 finest level
  double* gw = nullptr;
  int* diag = nullptr;
  double *Mv = nullptr, *J = nullptr, *Kxx = nullptr, *Kxy = nullptr, *Kyx = nullptr, *Kyy = nullptr;
  double* Mr = nullptr;  // mass weighted by rho^k (variable density)
  OpVals Vx, Vy;
  double *b64 = nullptr, *x64 = nullptr, *t64 = nullptr, *r64 = nullptr, *d64 = nullptr,
         *e64 = nullptr, *c64 = nullptr;
  float *b32 = nullptr, *x32 = nullptr, *t32 = nullptr, *r32 = nullptr, *d32 = nullptr,
        *e32 = nullptr, *c32 = nullptr;
};

// Divergence matrix, the Oseen operator and the element slot tables.
struct NSData {
  Csr bcsr, csr;
  Sell bsell, sell;
  DSell db, d;
  double *B = nullptr, *val = nullptr;
  int8_t* kind = nullptr;
  int* src = nullptr;
  int *eslot36 = nullptr, *eslotb = nullptr;
  double* tables = nullptr;
  DP2Tables tb{};
  // closed square: the no-slip set's slots (zeroed; the diagonal set to 1) in
  // the P2 and Oseen SELL value arrays, and its rows of the 8N velocity
  int *p2_zero = nullptr, *p2_one = nullptr, *ns_zero = nullptr, *ns_one = nullptr, *vfix = nullptr;
  int64_t n_p2_zero = 0, n_p2_one = 0, n_ns_zero = 0, n_ns_one = 0, n_vfix = 0;
};

struct Krylov {
  int64_t nmax = 0;
  double *V = nullptr, *Z = nullptr;
  double *H = nullptr, *cs = nullptr, *sn = nullptr, *g = nullptr, *y = nullptr;
  double *scal = nullptr, *part = nullptr, *nrm_part = nullptr;
  double *HR = nullptr, *gp = nullptr, *red = nullptr;  // DCGS2
  // pinned readback: two 4-double slots for the lookahead, two for restarts
  // (the residual norm, ||b||); a kernel writes a slot's three values, then,
  // behind a system-scope fence, the slot's tag into its fourth entry
  double* host = nullptr;
  double tag = 0.0;                 // last tag issued
  double stag[2] = {0.0, 0.0};      // tag awaited in each lookahead slot
  double rate[3] = {-1.0, -1.0, -1.0};  // per block: mean residual reduction per step of the last solve
};

// Work vectors of the adjoint step (ternary contexts).
struct AdjData {
  double *eta = nullptr;   // two CH adjoint solutions, 2N each
  double *zeta = nullptr;  // AC adjoint solution, N
  double *xi = nullptr;    // Oseen adjoint solution, 9N
  double *rhs = nullptr;   // staged right-hand side, 9N
  double* v[10] = {};      // M and K products of the adjoint solutions, N each
  double *q = nullptr, *gmu = nullptr;
  double *F = nullptr;     // Korteweg load, 8N
  double *part = nullptr;  // reduction partials
  double *acc = nullptr;   // dL/d(eps, mobility, evaporation rate)
};

// Measurement ledger: launches of one kernel class bracketed by event pairs
// on their stream, with the algorithmic bytes of each launch.
struct Ledger {
  int kernel = -1;  // class being timed, -1 off
  int cap = 0, used = 0;
  std::vector<hipEvent_t> ev;  // 2 per slot
  std::vector<double> bytes;
  int64_t launches = 0;
  double sum_bytes = 0.0, sum_ms = 0.0;
  hipStream_t stream = nullptr;
};

}  // namespace chns

struct chns_ctx {
  chns_mesh mesh{};
  chns_params prm{};
  int device = 0;       // the GPU current at chns_create
  int N = 0;            // P1 nodes
  bool box = false;     // closed square (no-flux boundaries) instead of the periodic one
  double len = 1.0;     // side of the square
  double h = 0.0;       // finest mesh width len / n
  bool dim3 = false;    // the periodic cube (Kuhn tetrahedra, binary models)
  double diag_ratio = 8.0;  // diag(K) h^2 / diag(M): 8 on triangles, 15 on the tetrahedra
  bool has_conv = false;
  bool c_zero = true;   // C and C32 hold zeros on every level
  bool formed_c0 = false;  // the formed operators (L, X, AC) are those of the current
                           // parameters and beta with C = 0
  bool ternary = false;  // a flow model (ternary or quaternary): Taylor-Hood Oseen step
  bool quat = false;     // the quaternary model (three CH phases, air eliminated)
  double beta_ch = 0.0;  // the gradient coefficient the CH operators are formed with
  // device table of the fused operator formation (one entry per level)
  chns::FormLevel* form_tab = nullptr;
  int64_t form_total = 0;
  chns::P2Level p2;
  chns::NSData ns;
  double coefV[2] = {1, 0};
  // multigrid: operator coefficients a M + b K for the level cut
  double coefL[2] = {1, 0}, coefX[2] = {1, 0}, coefAC[2] = {1, 0};
  std::vector<chns::Level> lv;
  chns::Elements el;
  int *ep1 = nullptr, *ep2 = nullptr, *etype = nullptr, *eslot = nullptr;
  int colour_ptr3[49] = {0};  // the cube: colour ranges of the tetrahedra (48 colours)
  double* topw = nullptr;     // closed cube: int phi_i dS of the top-face vertices
  chns::Krylov kr;
  // differentiation form: operators hold the transposed convection parts;
  // slot maps of the transposed entries (finest P1 and P2 patterns)
  bool transposed = false;
  int *tslot1 = nullptr, *tslot2 = nullptr;
  double* tbuf = nullptr;
  chns::AdjData adj;
  chns::Ledger ledger;
  // scratch: FP64 tmp1/tmp2/corr (N each), FP32 r/z (2N each) and
  // tmp1/tmp2/corr (N each), right-hand sides and the CH unknown [phi; mu]
  double *w64a = nullptr, *w64b = nullptr, *w64c = nullptr;
  double *rhs_ch = nullptr, *rhs_ac = nullptr, *xch = nullptr;
  double *rhs_ns = nullptr, *xns = nullptr, *xac = nullptr, *fs = nullptr, *w64d = nullptr;
  double* red = nullptr;  // reduction partials for mean projections
  double* pw = nullptr;   // closed square, flow models: M 1, the weights of the pressure's mean
  // variable density and Picard passes (ternary): rho^k at the vertices and
  // at the P2 nodes, the previous velocity iterate, norm partials and results
  double *rho1 = nullptr, *rho2 = nullptr, *vprev = nullptr, *pic = nullptr;
  double* diag = nullptr;  // diagnostics results (NDIAG)
  float *r32 = nullptr, *z32 = nullptr, *w32a = nullptr, *w32b = nullptr, *w32c = nullptr;
  std::vector<void*> allocs;
  // device allocator of the caller (chns_create), or hipMalloc/hipFree when NULL
  chns_alloc_fn alloc = nullptr;
  chns_free_fn free_ = nullptr;
  void* alloc_ctx = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  std::string err;
};
