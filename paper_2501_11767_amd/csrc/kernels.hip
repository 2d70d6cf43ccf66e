// gfx950 kernels of the solver: SELL-C-sigma sparse products (plain, residual
// and Jacobi forms, the shared-pattern Cahn-Hilliard block), coloured element
// assembly, Galerkin refresh of the coarse levels, and the FP64 reductions of
// flexible GMRES.
//
// Everything here is bandwidth-bound (about 0.1-0.2 flop per byte), so the
// kernels are written for coalesced HBM streams: SELL slices are 64 rows wide
// (one wavefront, one row per lane, entry k of all 64 rows contiguous), all
// loads of a row are issued before the arithmetic, and workgroups are
// remapped so each of the 8 XCDs works on a contiguous range of rows (its L2
// then also holds the neighbouring rows that the column gathers touch).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <mutex>

#include "device_util.hpp"
#include "kernels.hpp"

namespace chns {

namespace {

constexpr int BS = 256;   // workgroup size (4 wavefronts)
constexpr int W7 = 7;     // width of every P1 row on a triangle mesh
constexpr int W15 = 15;   // width of every P1 row on the Kuhn tetrahedral mesh
constexpr int MAXRED = 1024;

inline int ceil_div(int64_t a, int64_t b) { return int((a + b - 1) / b); }

// ------------------------------------------------------------------ SpMV

template <typename T, typename TV>
__global__ __launch_bounds__(BS) void k_spmv_sell(int nslices, int nrows, const int* __restrict__ sptr,
                                                  const int* __restrict__ sw,
                                                  const int* __restrict__ col,
                                                  const TV* __restrict__ val,
                                                  const int* __restrict__ perm,
                                                  const T* __restrict__ x, T* __restrict__ y,
                                                  T alpha, T beta) {
  const int b = xcd_block(blockIdx.x, gridDim.x);
  const int pos = b * BS + threadIdx.x;
  const int slice = pos >> 6, lane = pos & 63;
  if (slice >= nslices) return;
  const int row = perm ? perm[pos] : pos;
  if (row < 0 || row >= nrows) return;
  const int w = sw[slice];
  const int base = sptr[slice] + lane;
  T sum = T(0);
  for (int k = 0; k < w; ++k) {
    const int q = base + k * 64;
    sum += T(val[q]) * x[col[q]];
  }
  y[row] = (beta == T(0)) ? alpha * sum : alpha * sum + beta * y[row];
}

// Uniform width-7 patterns (P1): identity permutation, slice s = rows 64s..64s+63.
template <typename T, typename TV, int MODE, int W>
__global__ __launch_bounds__(BS) void k_stencil(int nrows, int side, const int* __restrict__ col,
                                                 const TV* __restrict__ val,
                                                 const T* __restrict__ x,
                                                 const T* __restrict__ b,
                                                 const T* __restrict__ dinv,
                                                 T* __restrict__ d, T p0, T p1,
                                                 T* __restrict__ y) {
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int row = blk * BS + threadIdx.x;
  if (row >= nrows) return;
  const size_t base = size_t(row >> 6) * (64 * W) + (row & 63);
  int c[W];
  TV v[W];
  row_cols<W>(row, side, col, base, c);
#pragma unroll
  for (int k = 0; k < W; ++k) v[k] = val[base + k * 64];
  T sum = T(0);
#pragma unroll
  for (int k = 0; k < W; ++k) sum += T(v[k]) * x[c[k]];
  if (MODE == ST_SPMV) {  // p0 = alpha, p1 = beta
    y[row] = (p1 == T(0)) ? p0 * sum : p0 * sum + p1 * y[row];
  } else if (MODE == ST_RESID) {
    y[row] = b[row] - sum;
  } else {  // ST_CHEB, p0 = c1, p1 = c2
    const T r = dinv[row] * (b[row] - sum);
    const T dn = (p0 == T(0)) ? p1 * r : p0 * d[row] + p1 * r;
    d[row] = dn;
    y[row] = x[row] + dn;
  }
}

// Fused multigrid steps on the periodic P1 levels (structured columns).

// First two Chebyshev steps from x = 0 in one pass: x0 = d0 = c20 D^{-1} b is
// formed on the fly at the row and its neighbours, then
// d = c11 d0 + c21 D^{-1} (b - A x0), y = x0 + d.
template <typename T, typename TV>
__global__ __launch_bounds__(BS) void k_cheb01(int nrows, int side, const TV* __restrict__ val,
                                               const T* __restrict__ b, const T* __restrict__ dinv,
                                               T c20, T c11, T c21, T* __restrict__ d,
                                               T* __restrict__ y) {
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int row = blk * BS + threadIdx.x;
  if (row >= nrows) return;
  const size_t base = size_t(row >> 6) * (64 * W7) + (row & 63);
  int c[W7];
  TV v[W7];
  p1_cols(row, side, c);
#pragma unroll
  for (int k = 0; k < W7; ++k) v[k] = val[base + k * 64];
  T sum = T(0);
#pragma unroll
  for (int k = 0; k < W7; ++k) sum += T(v[k]) * (c20 * (dinv[c[k]] * b[c[k]]));
  const T di = dinv[row], br = b[row];
  const T x0 = c20 * (di * br);
  const T dn = c11 * x0 + c21 * (di * (br - sum));
  d[row] = dn;
  y[row] = x0 + dn;
}

// P1 interpolation from the coarse periodic side-nc mesh at fine vertex
// (fi, fj): vertices copy, edge midpoints (horizontal, vertical, diagonal)
// average their two coarse ends.
template <typename T>
__device__ __forceinline__ T p1_interp(const T* __restrict__ e, int fi, int fj, int nc) {
  const int I = fi >> 1, J = fj >> 1;
  const T a = e[I + nc * J];
  if (!((fi | fj) & 1)) return a;
  const int I1 = (fi & 1) ? (I + 1 == nc ? 0 : I + 1) : I;
  const int J1 = (fj & 1) ? (J + 1 == nc ? 0 : J + 1) : J;
  return T(0.5) * (a + e[I1 + nc * J1]);
}

// Coarse-grid correction and the first post-smoothing step in one pass:
// x' = x + P e at the row and its neighbours, d = c2 D^{-1} (b - A x'),
// y = x' + d.
template <typename T, typename TV>
__global__ __launch_bounds__(BS) void k_pcheb(int nrows, int side, const TV* __restrict__ val,
                                              const T* __restrict__ x, const T* __restrict__ e,
                                              const T* __restrict__ b, const T* __restrict__ dinv,
                                              T c2, T* __restrict__ d, T* __restrict__ y) {
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int row = blk * BS + threadIdx.x;
  if (row >= nrows) return;
  const size_t base = size_t(row >> 6) * (64 * W7) + (row & 63);
  const int nc = side >> 1;
  const int j = row / side, i = row - j * side;
  TV v[W7];
#pragma unroll
  for (int k = 0; k < W7; ++k) v[k] = val[base + k * 64];
  constexpr int DI[W7] = {0, -1, 0, -1, 1, 0, 1};
  constexpr int DJ[W7] = {0, -1, -1, 0, 0, 1, 1};
  T sum = T(0), xs = T(0);
#pragma unroll
  for (int k = 0; k < W7; ++k) {
    int fi = i + DI[k], fj = j + DJ[k];
    fi = fi < 0 ? fi + side : (fi >= side ? fi - side : fi);
    fj = fj < 0 ? fj + side : (fj >= side ? fj - side : fj);
    const T xn = x[fi + side * fj] + p1_interp(e, fi, fj, nc);
    sum += T(v[k]) * xn;
    if (k == 0) xs = xn;
  }
  const T dn = c2 * (dinv[row] * (b[row] - sum));
  d[row] = dn;
  y[row] = xs + dn;
}

template <typename T>
__global__ __launch_bounds__(BS) void k_cheb0(int n, const T* __restrict__ dinv,
                                              const T* __restrict__ b, T c2, T* __restrict__ d,
                                              T* __restrict__ x) {
  const int i = blockIdx.x * BS + threadIdx.x;
  if (i < n) {
    const T v = c2 * (dinv[i] * b[i]);
    d[i] = v;
    x[i] = v;
  }
}

// Chebyshev steps from x = 0 on a level of at most 1024 rows: one workgroup,
// one row per thread, the row kept in registers, x in LDS.
template <typename T, typename TV, int W>
__global__ __launch_bounds__(1024) void k_coarse_cheb(int nrows, int side, const int* __restrict__ col,
                                                      const TV* __restrict__ val,
                                                      const T* __restrict__ dinv,
                                                      const T* __restrict__ b, ChebCoef<T> cc,
                                                      T* __restrict__ x) {
  __shared__ T xa[1024], xb[1024];
  const int r = threadIdx.x;
  T* cur = xa;
  T* nxt = xb;
  int c[W];
  TV v[W];
  T di = T(0), br = T(0), dd = T(0);
  if (r < nrows) {
    const size_t base = size_t(r >> 6) * (64 * W) + (r & 63);
    row_cols<W>(r, side, col, base, c);
#pragma unroll
    for (int k = 0; k < W; ++k) v[k] = val[base + k * 64];
    di = dinv[r];
    br = b[r];
    dd = cc.c2[0] * (di * br);
    cur[r] = dd;
  }
  __syncthreads();
  for (int s = 1; s < cc.steps; ++s) {
    if (r < nrows) {
      T sum = T(0);
#pragma unroll
      for (int k = 0; k < W; ++k) sum += T(v[k]) * cur[c[k]];
      dd = cc.c1[s] * dd + cc.c2[s] * (di * (br - sum));
      nxt[r] = cur[r] + dd;
    }
    __syncthreads();
    T* t = cur;
    cur = nxt;
    nxt = t;
  }
  if (r < nrows) x[r] = cur[r];
}

// ------------------------------------------------------------------ tiled levels

// Tiled multigrid kernels: tile interior side TT, rows per thread RPT (1024
// threads cover the tile and a halo of up to HMAX rings).  A row's 7 values,
// 1/diag, right-hand side and Chebyshev direction are held by its thread for
// all steps of the launch; the iterates, which the neighbours gather, sit in
// two LDS buffers.  Large levels take 64 x 64 tiles (less halo traffic),
// smaller ones 32 x 32 tiles (more workgroups, fewer rows per thread: these
// levels are latency-bound; their halo may reach 8 rings, enough for the
// Chebyshev steps of a cut level).
constexpr int TILE_THREADS = 1024;
template <int TT> struct TileCfg;
template <> struct TileCfg<64> { static constexpr int HMAX = 4, RPT = 6, NTH = 1024; };
template <> struct TileCfg<32> { static constexpr int HMAX = 8, RPT = 3, NTH = 1024; };
template <> struct TileCfg<16> { static constexpr int HMAX = 8, RPT = 4, NTH = 256; };

__device__ __forceinline__ int wrap_once(int x, int s) { return x < 0 ? x + s : (x >= s ? x - s : x); }

// Halo rings of a tiled launch.
__host__ __device__ constexpr int tile_halo(int mode, int steps) {
  return mode == TILE_ZERO ? steps - 1 : (mode == TILE_DOWN || mode == TILE_UPM ? steps + 1 : steps);
}

// One tile of a level (tile index `tile` of the side x side grid, row-major
// over ceil(side / TT)^2 tiles).  Pointers address the level (or, batched,
// one instance's block of it); c1/c2 the step coefficients.
template <typename T, int MODE, int TT>
__device__ __forceinline__ void vtile_body(int s, int steps, const T* __restrict__ val,
                                           const T* __restrict__ dinv, const T* __restrict__ b,
                                           const T* __restrict__ xin, const T* __restrict__ e,
                                           T* __restrict__ x, T* __restrict__ bc, const T* c1s,
                                           const T* c2s, int tile, T* xa, T* xb,
                                           const double* __restrict__ b64 = nullptr,
                                           double* __restrict__ x64 = nullptr,
                                           const double* __restrict__ xs = nullptr,
                                           const T* __restrict__ mval = nullptr) {
  constexpr int RPT = TileCfg<TT>::RPT, NTH = TileCfg<TT>::NTH;
  constexpr bool UPLIKE = MODE == TILE_UP || MODE == TILE_UPM;
  const int H = tile_halo(MODE, steps);
  const int W = TT + 2 * H, R = W * W;
  const int nt = (s + TT - 1) / TT;
  const int ty = tile / nt, tx = tile - ty * nt;
  const int i0 = tx * TT - H, j0 = ty * TT - H;
  const int tid = threadIdx.x;
  // neighbour offsets in the tile, in the order of the stored values:
  // self, (-1,-1), (0,-1), (-1,0), (1,0), (0,1), (1,1)
  const int off[W7] = {0, -W - 1, -W, -1, 1, W, W + 1};
  T v[RPT][W7], di[RPT], bb[RPT], d[RPT];
  int gr[RPT], ring[RPT];
  bool own[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int idx = tid + q * NTH;
    ring[q] = -1;
    own[q] = false;
    if (idx < R) {
      const int rj = idx / W, ri = idx - rj * W;
      const int gi = wrap_once(i0 + ri, s), gj = wrap_once(j0 + rj, s);
      const int row = gi + s * gj;
      gr[q] = row;
      ring[q] = min(min(ri, rj), min(W - 1 - ri, W - 1 - rj));
      own[q] = ring[q] >= H && tx * TT + (ri - H) < s && ty * TT + (rj - H) < s;
      const size_t base = size_t(row >> 6) * (64 * W7) + (row & 63);
      // ring 0 is never updated by a step with neighbours (its rows only take
      // the first step from zero, and in the up pass not even that): no values
      // there, nor 1/diag and right-hand side in the up pass
      const bool upd = ring[q] >= 1;
#pragma unroll
      for (int k = 0; k < W7; ++k) v[q][k] = upd ? val[base + k * 64] : T(0);
      if (UPLIKE && !upd) {
        di[q] = T(0);
        bb[q] = T(0);
      } else {
        di[q] = dinv[row];
        bb[q] = b64 ? T(b64[row]) : b[row];
      }
      if (UPLIKE) xa[idx] = xin[row] + p1_interp(e, gi, gj, s >> 1);
    }
  }
  // up pass with the M product: the values of M for the own rows, taken in
  // a direct map (interior row o = tid + p NTH of the TT x TT tile), are
  // loaded here, after every other load, so that they arrive during the
  // sweeps instead of after them
  constexpr int NOWN = MODE == TILE_UPM ? TT * TT / NTH : 1;
  static_assert(MODE != TILE_UPM || NOWN * NTH == TT * TT, "interior rows per thread");
  T mv[NOWN][W7];
  int orow[NOWN], oidx[NOWN];
  if constexpr (MODE == TILE_UPM) {
#pragma unroll
    for (int p = 0; p < NOWN; ++p) {
      const int o = tid + p * NTH;
      const int oj = o / TT, oi = o - oj * TT;
      const int gi = tx * TT + oi, gj = ty * TT + oj;
      const bool in = gi < s && gj < s;  // ragged last tiles
      orow[p] = in ? gi + s * gj : -1;
      oidx[p] = (oi + H) + W * (oj + H);
      const int rr = in ? orow[p] : tx * TT + s * (ty * TT);
      const size_t base = size_t(rr >> 6) * (64 * W7) + (rr & 63);
#pragma unroll
      for (int k = 0; k < W7; ++k) mv[p][k] = mval[base + k * 64];
    }
  }
  if (!UPLIKE) {  // first step from zero: x = d = c2 D^{-1} b
    const T c20 = c2s[0];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int idx = tid + q * NTH;
      if (idx < R) {
        d[q] = c20 * (di[q] * bb[q]);
        xa[idx] = d[q];
      }
    }
  }
  __syncthreads();
  T* cur = xa;
  T* nxt = xb;
  // Chebyshev steps k0.. on shrinking rings: step k is valid at ring >= k - k0 + 1
  const int k0 = UPLIKE ? 0 : 1;
  for (int k = k0; k < steps; ++k) {
    const T c1 = c1s[k], c2 = c2s[k];
    const int rmin = k - k0 + 1;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int idx = tid + q * NTH;
      if (ring[q] >= rmin) {
        T sum = T(0);
#pragma unroll
        for (int m = 0; m < W7; ++m) sum += v[q][m] * cur[idx + off[m]];
        const T r = di[q] * (bb[q] - sum);
        const T dn = (k == 0) ? c2 * r : c1 * d[q] + c2 * r;
        d[q] = dn;
        nxt[idx] = cur[idx] + dn;
      }
    }
    __syncthreads();
    T* t = cur;
    cur = nxt;
    nxt = t;
  }
  if constexpr (MODE == TILE_UPM) {
    // the result is valid at ring >= steps, so on every neighbour of an own row
#pragma unroll
    for (int p = 0; p < NOWN; ++p) {
      if (orow[p] >= 0) {
        T y = T(0);
#pragma unroll
        for (int k = 0; k < W7; ++k) y += mv[p][k] * cur[oidx[p] + off[k]];
        if (x64) x64[orow[p]] = double(y) * (xs ? xs[0] : 1.0);
        else x[orow[p]] = y;
      }
    }
  } else if (x64) {
    const double sc = xs ? xs[0] : 1.0;
#pragma unroll
    for (int q = 0; q < RPT; ++q)
      if (own[q]) x64[gr[q]] = double(cur[tid + q * NTH]) * sc;
  } else {
#pragma unroll
    for (int q = 0; q < RPT; ++q)
      if (own[q]) x[gr[q]] = cur[tid + q * NTH];
  }
  if (MODE == TILE_DOWN) {
    // residual on ring >= steps, then R = P^T into the coarse rows whose fine
    // vertex lies in the tile interior
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int idx = tid + q * NTH;
      if (ring[q] >= steps) {
        T sum = T(0);
#pragma unroll
        for (int m = 0; m < W7; ++m) sum += v[q][m] * cur[idx + off[m]];
        nxt[idx] = bb[q] - sum;
      }
    }
    __syncthreads();
    constexpr int TC = TT / 2;
    const int nc = s >> 1;
    if (tid < TC * TC) {
      const int lj = tid / TC, li = tid - lj * TC;
      const int cI = tx * TC + li, cJ = ty * TC + lj;
      if (cI < nc && cJ < nc) {
        const int idx = (2 * li + H) + W * (2 * lj + H);
        T sm = T(0);
#pragma unroll
        for (int m = 1; m < W7; ++m) sm += nxt[idx + off[m]];
        bc[cI + nc * cJ] = nxt[idx] + T(0.5) * sm;
      }
    }
  }
}

template <typename T, int MODE, int TT>
__global__ __launch_bounds__(TileCfg<TT>::NTH) void k_vtile(TileArgs<T> a) {
  constexpr int WMAX = TT + 2 * TileCfg<TT>::HMAX;
  __shared__ T xa[WMAX * WMAX], xb[WMAX * WMAX];
  vtile_body<T, MODE, TT>(a.side, a.steps, a.val, a.dinv, a.b, a.xin, a.e, a.x, a.bc, a.c1, a.c2,
                          xcd_block(blockIdx.x, gridDim.x), xa, xb, a.b64, a.x64, a.xs, a.mval);
}

// Software-pipelined form of the 64 x 64 FP32 tile pass (the finest level
// of the mixed-precision cycles).  The region's rows are cut into bands of
// NTH consecutive region indices (one row of each band per thread; a band
// spans more than one region line, so a stencil reaches only the adjacent
// bands).  Stage t issues the loads of band t + LA (all bands up to LA ahead
// are in flight), initialises band t - 1 (x = c2 D^{-1} b from zero, or x +
// P e in the up pass), runs sweep k of band t - 1 - 2k and stores the result
// of band t - 2 - 2S: every band's sweep k comes one stage after sweep k - 1
// of its lower neighbour band and after its upper neighbour's, and the loads
// of the bands still ahead are in flight during the sweeps of the bands
// behind.  The number of sweeps S, the halo and the FP64 boundary are
// compile-time, so that every band's registers are fixed and the waits for
// its loads name only those loads; the right-hand side stays in its load
// type until the band's initialisation.  The arithmetic per row and sweep is
// k_vtile's.
constexpr int PIPE_LA = 1;  // bands loaded ahead of the band being initialised

template <typename T, int MODE, int S, int IO>
struct PipeTile {
  static constexpr int TT = 64, NTH = 1024;
  static constexpr bool UPLIKE = MODE == TILE_UP || MODE == TILE_UPM;
  static constexpr bool BIN64 = (IO & 1) != 0, XOUT64 = (IO & 2) != 0;
  static constexpr int STEPS = UPLIKE ? S : S + 1;
  static constexpr int H = tile_halo(MODE, STEPS);
  static constexpr int W = TT + 2 * H, R = W * W;
  static constexpr int NB = (R + NTH - 1) / NTH;
  static constexpr int NOWN = MODE == TILE_UPM ? TT * TT / NTH : 1;
  // last stage: the result stores of the last band (DOWN: its residual, one later)
  static constexpr int NST = NB + 2 + 2 * S + (MODE == TILE_DOWN ? 1 : 0);
  using BIn = typename std::conditional<BIN64, double, T>::type;
  const TileArgs<T>& a;
  T* buf0;
  T* buf1;
  int s, tx, ty, i0, j0, tid, row_safe;
  T v[NB][W7], di[NB], d[NB], xin[NB], ea[NB], eb[NB];
  BIn bl[NB];
  T bb[NB];
  int ring[NB], gr[NB];
  bool own[NB], odd[NB];
  T mv[NOWN][W7];
  int orow[NOWN], oidx[NOWN];
  double xsc = 1.0;  // the FP64 output's scale
  __device__ __forceinline__ PipeTile(const TileArgs<T>& a_, T* b0, T* b1) : a(a_), buf0(b0), buf1(b1) {}
  template <int K> __device__ __forceinline__ T* B() { return (K & 1) ? buf1 : buf0; }

  template <int q> __device__ __forceinline__ void load() {
    const int idx = tid + q * NTH;
    const bool in = idx < R;
    const int ic = in ? idx : W + 1;
    const int rj = ic / W, ri = ic - rj * W;
    const int gi = wrap_once(i0 + ri, s), gj = wrap_once(j0 + rj, s);
    const int row = gi + s * gj;
    const int rg = min(min(ri, rj), min(W - 1 - ri, W - 1 - rj));
    ring[q] = in ? rg : -1;
    own[q] = in && rg >= H && tx * TT + (ri - H) < s && ty * TT + (rj - H) < s;
    gr[q] = row;
    const bool upd = in && rg >= 1;
    const int rv = upd ? row : row_safe;
    const int rd = (UPLIKE && !upd) ? row_safe : row;
    const size_t base = size_t(rv >> 6) * (64 * W7) + (rv & 63);
#pragma unroll
    for (int k = 0; k < W7; ++k) v[q][k] = a.val[base + k * 64];
    di[q] = a.dinv[rd];
    if constexpr (BIN64) bl[q] = a.b64[rd];
    else bl[q] = a.b[rd];
    if constexpr (UPLIKE) {
      const int nc = s >> 1, I = gi >> 1, J = gj >> 1;
      const int I1 = (gi & 1) ? (I + 1 == nc ? 0 : I + 1) : I;
      const int J1 = (gj & 1) ? (J + 1 == nc ? 0 : J + 1) : J;
      odd[q] = ((gi | gj) & 1) != 0;
      xin[q] = a.xin[row];
      ea[q] = a.e[I + nc * J];
      eb[q] = a.e[I1 + nc * J1];
    }
  }

  __device__ __forceinline__ void load_m() {
    if constexpr (MODE == TILE_UPM) {
#pragma unroll
      for (int p = 0; p < NOWN; ++p) {
        const int o = tid + p * NTH;
        const int oj = o / TT, oi = o - oj * TT;
        const int gi = tx * TT + oi, gj = ty * TT + oj;
        const bool in = gi < s && gj < s;
        orow[p] = in ? gi + s * gj : -1;
        oidx[p] = (oi + H) + W * (oj + H);
        const int rr = in ? orow[p] : tx * TT + s * (ty * TT);
        const size_t base = size_t(rr >> 6) * (64 * W7) + (rr & 63);
#pragma unroll
        for (int k = 0; k < W7; ++k) mv[p][k] = a.mval[base + k * 64];
      }
    }
  }

  template <int q> __device__ __forceinline__ void init() {
    const int idx = tid + q * NTH;
    bb[q] = T(bl[q]);
    d[q] = T(0);
    if (idx < R) {
      if constexpr (UPLIKE) {
        buf0[idx] = xin[q] + (odd[q] ? T(0.5) * (ea[q] + eb[q]) : ea[q]);
      } else {
        d[q] = a.c2[0] * (di[q] * bb[q]);
        buf0[idx] = d[q];
      }
    }
  }

  template <int q, int k> __device__ __forceinline__ void sweep() {
    // valid at ring >= k after sweep k
    constexpr int ci = UPLIKE ? k - 1 : k;
    const T c1 = a.c1[ci], c2 = a.c2[ci];
    T* cur = B<k - 1>();
    T* nxt = B<k>();
    const int idx = tid + q * NTH;
    if (ring[q] >= k) {
      T sum = T(0);
#pragma unroll
      for (int m = 0; m < W7; ++m) sum += v[q][m] * cur[idx + off(m)];
      const T r = di[q] * (bb[q] - sum);
      const T dn = (UPLIKE && k == 1) ? c2 * r : c1 * d[q] + c2 * r;
      d[q] = dn;
      nxt[idx] = cur[idx] + dn;
    }
  }

  template <int q> __device__ __forceinline__ void store() {
    if constexpr (MODE != TILE_UPM) {
      const int idx = tid + q * NTH;
      if (own[q]) {
        const T y = B<S>()[idx];
        if constexpr (XOUT64) a.x64[gr[q]] = double(y) * xsc;
        else a.x[gr[q]] = y;
      }
    }
  }

  template <int q> __device__ __forceinline__ void resid() {
    if constexpr (MODE == TILE_DOWN) {
      // residual on ring >= steps, into the buffer the last sweep did not write
      T* cur = B<S>();
      T* nxt = B<S + 1>();
      const int idx = tid + q * NTH;
      if (ring[q] >= STEPS) {
        T sum = T(0);
#pragma unroll
        for (int m = 0; m < W7; ++m) sum += v[q][m] * cur[idx + off(m)];
        nxt[idx] = bb[q] - sum;
      }
    }
  }

  static __device__ __forceinline__ constexpr int off(int m) {
    return m == 0 ? 0 : m == 1 ? -W - 1 : m == 2 ? -W : m == 3 ? -1 : m == 4 ? 1 : m == 5 ? W : W + 1;
  }

  template <int t, int k> __device__ __forceinline__ void sweeps_at() {
    if constexpr (k <= S) {
      constexpr int q = t - 1 - 2 * k;
      if constexpr (q >= 0 && q < NB) sweep<q, k>();
      sweeps_at<t, k + 1>();
    }
  }

  template <int t, int q> __device__ __forceinline__ void loads_at() {
    if constexpr (q < NB) {
      constexpr int ls = q - PIPE_LA < 0 ? 0 : q - PIPE_LA;  // stage that issues band q's loads
      if constexpr (ls == t) load<q>();
      loads_at<t, q + 1>();
    }
  }

  template <int t> __device__ __forceinline__ void stage() {
    loads_at<t, 0>();
    constexpr int lastls = NB - 1 - PIPE_LA < 0 ? 0 : NB - 1 - PIPE_LA;
    if constexpr (t == lastls) load_m();
    if constexpr (t - 1 >= 0 && t - 1 < NB) init<t - 1>();
    sweeps_at<t, 1>();
    constexpr int qs = t - 2 - 2 * S;
    if constexpr (qs >= 0 && qs < NB) store<qs>();
    constexpr int qr = t - 3 - 2 * S;
    if constexpr (qr >= 0 && qr < NB) resid<qr>();
    __syncthreads();
  }

  template <int t> __device__ __forceinline__ void run_from() {
    if constexpr (t < NST) {
      stage<t>();
      run_from<t + 1>();
    }
  }

  __device__ __forceinline__ void run(int tile) {
    s = a.side;
    const int nt = (s + TT - 1) / TT;
    ty = tile / nt;
    tx = tile - ty * nt;
    i0 = tx * TT - H;
    j0 = ty * TT - H;
    tid = threadIdx.x;
    row_safe = wrap_once(i0 + 1, s) + s * wrap_once(j0 + 1, s);
    if constexpr (XOUT64) xsc = a.xs ? a.xs[0] : 1.0;
    run_from<0>();
    if constexpr (MODE == TILE_UPM) {
      T* cur = B<S>();
#pragma unroll
      for (int p = 0; p < NOWN; ++p) {
        if (orow[p] >= 0) {
          T y = T(0);
#pragma unroll
          for (int k = 0; k < W7; ++k) y += mv[p][k] * cur[oidx[p] + off(k)];
          if constexpr (XOUT64) a.x64[orow[p]] = double(y) * xsc;
          else a.x[orow[p]] = y;
        }
      }
    }
    if constexpr (MODE == TILE_DOWN) {
      // R = P^T of the residual into the coarse rows whose fine vertex lies
      // in the tile interior
      const T* res = B<S + 1>();
      constexpr int TC = TT / 2;
      const int nc = s >> 1;
      if (tid < TC * TC) {
        const int lj = tid / TC, lc = tid - lj * TC;
        const int cI = tx * TC + lc, cJ = ty * TC + lj;
        if (cI < nc && cJ < nc) {
          const int idx = (2 * lc + H) + W * (2 * lj + H);
          T sm = T(0);
#pragma unroll
          for (int m = 1; m < W7; ++m) sm += res[idx + off(m)];
          a.bc[cI + nc * cJ] = res[idx] + T(0.5) * sm;
        }
      }
    }
  }
};

template <typename T, int MODE, int S, int IO>
__global__ __launch_bounds__(1024) void k_vtile_pipe(TileArgs<T> a) {
  using P = PipeTile<T, MODE, S, IO>;
  __shared__ T b0[P::R], b1[P::R];
  P p(a, b0, b1);
  p.run(xcd_block(blockIdx.x, gridDim.x));
}

// Batched: workgroup -> (instance, tile) from the tile list; the launch's
// pointers address the stacked level, offset per instance by its row offsets
// (values by 7 slots per row); c1/c2 shared, or per instance ([step][count]).
template <typename T, int MODE, int TT>
__global__ __launch_bounds__(TileCfg<TT>::NTH) void k_bvtile(BTileLaunch<T> a) {
  constexpr int WMAX = TT + 2 * TileCfg<TT>::HMAX;
  __shared__ T xa[WMAX * WMAX], xb[WMAX * WMAX];
  __shared__ T c1s[TILE_MAXSTEPS], c2s[TILE_MAXSTEPS];
  const BTile t = a.tiles[xcd_block(blockIdx.x, gridDim.x)];
  if (a.act && !a.act[t.inst]) return;
  if (threadIdx.x < a.steps) {
    const int k = threadIdx.x;
    c1s[k] = a.cc1 ? a.cc1[k * a.count + t.inst] : a.c1[k];
    c2s[k] = a.cc2 ? a.cc2[k * a.count + t.inst] : a.c2[k];
  }
  __syncthreads();
  const int64_t r = t.roff, rc = t.croff;
  vtile_body<T, MODE, TT>(t.side, a.steps, a.val + r * W7, a.dinv + r, a.b ? a.b + r : nullptr,
                          a.xin ? a.xin + r : nullptr, a.e ? a.e + rc : nullptr, a.x ? a.x + r : nullptr,
                          a.bc ? a.bc + rc : nullptr, c1s, c2s, t.tile, xa, xb, a.b64 ? a.b64 + r : nullptr,
                          a.x64 ? a.x64 + r : nullptr, a.xs ? a.xs + t.inst : nullptr,
                          a.mval ? a.mval + r * W7 : nullptr);
}

// Work-list form of k_bvtile: a fixed grid (CUs x k workgroups, a multiple of
// 8) instead of one workgroup per tile.  The tile list is cut into 8
// contiguous ranges, one per XCD (workgroup b runs on XCD b mod 8, so a range
// of neighbouring tiles shares that XCD's L2); the workgroups of XCD x take
// tiles of range x from the atomic counter ctr[2x] until it runs past the
// range, then count themselves in ctr[2x + 1]; the last one resets both for
// the next launch.  Every workgroup leaves after at most (its range's size)
// tiles, so the grid always drains.  The per-tile arithmetic is k_bvtile's.
template <typename T, int MODE, int TT>
__global__ __launch_bounds__(TileCfg<TT>::NTH) void k_bvtile_wl(BTileLaunch<T> a, int ntiles,
                                                                 int* __restrict__ ctr) {
  constexpr int WMAX = TT + 2 * TileCfg<TT>::HMAX;
  __shared__ T xa[WMAX * WMAX], xb[WMAX * WMAX];
  __shared__ T c1s[TILE_MAXSTEPS], c2s[TILE_MAXSTEPS];
  __shared__ int tsh;
  const int x = blockIdx.x & 7;
  const int nwg = int(gridDim.x);
  const int wg_x = nwg / 8 + (x < nwg % 8 ? 1 : 0);  // workgroups on XCD x (nwg >= 8)
  const int lo = int(int64_t(x) * ntiles / 8), hi = int(int64_t(x + 1) * ntiles / 8);
  for (;;) {
    if (threadIdx.x == 0) tsh = lo + atomicAdd(&ctr[2 * x], 1);
    __syncthreads();
    const int ti = tsh;
    __syncthreads();
    if (ti >= hi) break;
    const BTile t = a.tiles[ti];
    if (a.act && !a.act[t.inst]) continue;
    if (threadIdx.x < a.steps) {
      const int k = threadIdx.x;
      c1s[k] = a.cc1 ? a.cc1[k * a.count + t.inst] : a.c1[k];
      c2s[k] = a.cc2 ? a.cc2[k * a.count + t.inst] : a.c2[k];
    }
    __syncthreads();
    const int64_t r = t.roff, rc = t.croff;
    vtile_body<T, MODE, TT>(t.side, a.steps, a.val + r * W7, a.dinv + r, a.b ? a.b + r : nullptr,
                            a.xin ? a.xin + r : nullptr, a.e ? a.e + rc : nullptr, a.x ? a.x + r : nullptr,
                            a.bc ? a.bc + rc : nullptr, c1s, c2s, t.tile, xa, xb, a.b64 ? a.b64 + r : nullptr,
                            a.x64 ? a.x64 + r : nullptr, a.xs ? a.xs + t.inst : nullptr,
                            a.mval ? a.mval + r * W7 : nullptr);
    __syncthreads();  // the LDS buffers and coefficients are reused by the next tile
  }
  if (threadIdx.x == 0) {
    __threadfence();
    if (atomicAdd(&ctr[2 * x + 1], 1) == wg_x - 1) {  // the last of XCD x: every take is done
      atomicExch(&ctr[2 * x], 0);
      atomicExch(&ctr[2 * x + 1], 0);
    }
  }
}

// ------------------------------------------------------------------ paired levels

// Two consecutive smoothing levels per launch: a 32 x 32 fine tile and the
// 16 x 16 coarse tile under it.  Region sizes for up to T2_PMAX pre / post
// steps; every workgroup has 1024 threads.
constexpr int T2_TT = 32, T2_TC = 16, T2_PMAX = 3;
constexpr int T2_WF = T2_TT + 2 * (3 * T2_PMAX + 3);                  // down2 fine region side
constexpr int T2_WC = T2_TC + 2 * (T2_PMAX + 1);                      // down2 coarse region side
constexpr int T2_WCU = T2_TC + 2 * ((T2_PMAX + 1) / 2 + 1 + T2_PMAX);  // up2 coarse region side
constexpr int T2_WFU = T2_TT + 2 * T2_PMAX;                           // up2 fine region side
constexpr int T2_RPTF = (T2_WF * T2_WF + 1023) / 1024;
constexpr int T2_RPTU = (T2_WFU * T2_WFU + 1023) / 1024;
static_assert(T2_WC * T2_WC <= 1024 && T2_WCU * T2_WCU <= 1024, "one coarse row per thread");

// down2: fine pre-smoothing from zero over a halo of Hf = 3P + 3 rings (the
// residual must hold on the fine points restricted into the coarse region),
// coarse right-hand side on the coarse region (halo Hc = P + 1), coarse
// pre-smoothing, residual and restriction to the level below.
template <typename T>
__global__ __launch_bounds__(1024) void k_vdown2(Tile2Args<T> a) {
  __shared__ T fx[T2_WF * T2_WF], fy[T2_WF * T2_WF];
  __shared__ T cx[T2_WC * T2_WC], cy[T2_WC * T2_WC];
  const int s = a.side, sc = s >> 1, scc = sc >> 1, P = a.steps;
  const int Hc = P + 1, Hf = 3 * P + 3;
  const int Wf = T2_TT + 2 * Hf, Rf = Wf * Wf;
  const int Wc = T2_TC + 2 * Hc, Rc = Wc * Wc;
  const int nt = (s + T2_TT - 1) / T2_TT;
  const int tile = xcd_block(blockIdx.x, gridDim.x);
  const int ty = tile / nt, tx = tile - ty * nt;
  const int i0 = tx * T2_TT - Hf, j0 = ty * T2_TT - Hf;
  const int ci0 = tx * T2_TC - Hc, cj0 = ty * T2_TC - Hc;
  const int tid = threadIdx.x;
  const int offf[W7] = {0, -Wf - 1, -Wf, -1, 1, Wf, Wf + 1};
  const int offc[W7] = {0, -Wc - 1, -Wc, -1, 1, Wc, Wc + 1};
  T v[T2_RPTF][W7], di[T2_RPTF], bb[T2_RPTF], d[T2_RPTF];
  int gr[T2_RPTF], ring[T2_RPTF];
  bool own[T2_RPTF];
#pragma unroll
  for (int q = 0; q < T2_RPTF; ++q) {
    const int idx = tid + q * 1024;
    ring[q] = -1;
    own[q] = false;
    if (idx < Rf) {
      const int rj = idx / Wf, ri = idx - rj * Wf;
      const int gi = wrap_once(i0 + ri, s), gj = wrap_once(j0 + rj, s);
      const int row = gi + s * gj;
      gr[q] = row;
      ring[q] = min(min(ri, rj), min(Wf - 1 - ri, Wf - 1 - rj));
      own[q] = ring[q] >= Hf && tx * T2_TT + (ri - Hf) < s && ty * T2_TT + (rj - Hf) < s;
      const size_t base = size_t(row >> 6) * (64 * W7) + (row & 63);
#pragma unroll
      for (int k = 0; k < W7; ++k) v[q][k] = a.valf[base + k * 64];
      di[q] = a.dinvf[row];
      bb[q] = a.bf[row];
    }
  }
  // this thread's coarse row, loaded with the fine rows
  T cv[W7], cdi = T(0), cd = T(0), cbv = T(0);
  int cring = -1, crow = 0;
  bool cown = false;
  int cri = 0, crj = 0;
  if (tid < Rc) {
    crj = tid / Wc;
    cri = tid - crj * Wc;
    const int cgi = wrap_once(ci0 + cri, sc), cgj = wrap_once(cj0 + crj, sc);
    crow = cgi + sc * cgj;
    cring = min(min(cri, crj), min(Wc - 1 - cri, Wc - 1 - crj));
    cown = cring >= Hc && tx * T2_TC + (cri - Hc) < sc && ty * T2_TC + (crj - Hc) < sc;
    const size_t base = size_t(crow >> 6) * (64 * W7) + (crow & 63);
#pragma unroll
    for (int k = 0; k < W7; ++k) cv[k] = a.valc[base + k * 64];
    cdi = a.dinvc[crow];
  }
  // fine pre-smoothing from zero on shrinking rings
  {
    const T c20 = a.c2[0];
#pragma unroll
    for (int q = 0; q < T2_RPTF; ++q) {
      const int idx = tid + q * 1024;
      if (idx < Rf) {
        d[q] = c20 * (di[q] * bb[q]);
        fx[idx] = d[q];
      }
    }
  }
  __syncthreads();
  T* cur = fx;
  T* nxt = fy;
  for (int k = 1; k < P; ++k) {
    const T c1 = a.c1[k], c2 = a.c2[k];
#pragma unroll
    for (int q = 0; q < T2_RPTF; ++q) {
      const int idx = tid + q * 1024;
      if (ring[q] >= k) {
        T sum = T(0);
#pragma unroll
        for (int m = 0; m < W7; ++m) sum += v[q][m] * cur[idx + offf[m]];
        const T r = di[q] * (bb[q] - sum);
        const T dn = c1 * d[q] + c2 * r;
        d[q] = dn;
        nxt[idx] = cur[idx] + dn;
      }
    }
    __syncthreads();
    T* t = cur;
    cur = nxt;
    nxt = t;
  }
#pragma unroll
  for (int q = 0; q < T2_RPTF; ++q)
    if (own[q]) a.xf[gr[q]] = cur[tid + q * 1024];
#pragma unroll
  for (int q = 0; q < T2_RPTF; ++q) {
    const int idx = tid + q * 1024;
    if (ring[q] >= P) {
      T sum = T(0);
#pragma unroll
      for (int m = 0; m < W7; ++m) sum += v[q][m] * cur[idx + offf[m]];
      nxt[idx] = bb[q] - sum;
    }
  }
  __syncthreads();
  // coarse right-hand side (R = P^T) on the coarse region: the fine vertex
  // of coarse point (cri, crj) sits at fine-region column P + 1 + 2 cri
  if (tid < Rc) {
    const int f = (P + 1 + 2 * cri) + Wf * (P + 1 + 2 * crj);
    T sm = T(0);
#pragma unroll
    for (int m = 1; m < W7; ++m) sm += nxt[f + offf[m]];
    cbv = nxt[f] + T(0.5) * sm;
    if (cown) a.bc[crow] = cbv;
    cd = a.c2[0] * (cdi * cbv);
    cx[tid] = cd;
  }
  __syncthreads();
  T* ccur = cx;
  T* cnxt = cy;
  for (int k = 1; k < P; ++k) {
    if (cring >= k) {
      T sum = T(0);
#pragma unroll
      for (int m = 0; m < W7; ++m) sum += cv[m] * ccur[tid + offc[m]];
      const T r = cdi * (cbv - sum);
      cd = a.c1[k] * cd + a.c2[k] * r;
      cnxt[tid] = ccur[tid] + cd;
    }
    __syncthreads();
    T* t = ccur;
    ccur = cnxt;
    cnxt = t;
  }
  if (cown) a.xc[crow] = ccur[tid];
  if (cring >= P) {
    T sum = T(0);
#pragma unroll
    for (int m = 0; m < W7; ++m) sum += cv[m] * ccur[tid + offc[m]];
    cnxt[tid] = cbv - sum;
  }
  __syncthreads();
  constexpr int TCC = T2_TC / 2;
  if (tid < TCC * TCC) {
    const int lj = tid / TCC, li = tid - lj * TCC;
    const int I = tx * TCC + li, J = ty * TCC + lj;
    if (I < scc && J < scc) {
      const int q = (2 * li + Hc) + Wc * (2 * lj + Hc);
      T sm = T(0);
#pragma unroll
      for (int m = 1; m < W7; ++m) sm += cnxt[q + offc[m]];
      a.bcc[I + scc * J] = cnxt[q] + T(0.5) * sm;
    }
  }
}

// Side of the cut-level region vup2 solves: the cut-level nodes its coarse
// region's interpolation reads (coarse region side wc starting at a coarse
// column of parity p), widened by steps - 1 rings (a step from zero at ring
// r >= k stays exact after k + 1 steps).
__host__ __device__ constexpr int t2_cut_side(int wc, int p, int steps) {
  return ((wc - 1 + p) >> 1) + 2 + 2 * (steps - 1);
}

// up2: coarse correction x_c + P e and post-smoothing on a coarse region of
// halo Hcu = D + Q (D = (Q + 1) / 2 + 1 coarse rings feed the fine
// interpolation), then the fine correction and post-smoothing (halo Q).
// With a.csteps > 0, e comes from the cut level solved in LDS first.
template <typename T>
__global__ __launch_bounds__(1024) void k_vup2(Tile2Args<T> a) {
  __shared__ T fx[T2_WFU * T2_WFU], fy[T2_WFU * T2_WFU];
  __shared__ T cx[T2_WCU * T2_WCU], cy[T2_WCU * T2_WCU];
  const int s = a.side, sc = s >> 1, scc = sc >> 1, Q = a.steps;
  const int D = (Q + 1) / 2 + 1, Hcu = D + Q;
  const int W = T2_TT + 2 * Q, R = W * W;
  const int Wc = T2_TC + 2 * Hcu, Rc = Wc * Wc;
  const int nt = (s + T2_TT - 1) / T2_TT;
  const int tile = xcd_block(blockIdx.x, gridDim.x);
  const int ty = tile / nt, tx = tile - ty * nt;
  const int i0 = tx * T2_TT - Q, j0 = ty * T2_TT - Q;
  const int ci0 = tx * T2_TC - Hcu, cj0 = ty * T2_TC - Hcu;
  const int tid = threadIdx.x;
  const int off[W7] = {0, -W - 1, -W, -1, 1, W, W + 1};
  const int offc[W7] = {0, -Wc - 1, -Wc, -1, 1, Wc, Wc + 1};
  // fine rows: operands loaded early (before the cut-level steps when there
  // are any, else before the coarse smoothing), corrections after it
  T v[T2_RPTU][W7], di[T2_RPTU], bb[T2_RPTU], d[T2_RPTU], xi[T2_RPTU];
  int gr[T2_RPTU], ring[T2_RPTU];
  bool own[T2_RPTU];
  auto load_fine = [&]() {
#pragma unroll
    for (int q = 0; q < T2_RPTU; ++q) {
      const int idx = tid + q * 1024;
      ring[q] = -1;
      own[q] = false;
      if (idx < R) {
        const int rj = idx / W, ri = idx - rj * W;
        const int gi = wrap_once(i0 + ri, s), gj = wrap_once(j0 + rj, s);
        const int row = gi + s * gj;
        gr[q] = row;
        ring[q] = min(min(ri, rj), min(W - 1 - ri, W - 1 - rj));
        own[q] = ring[q] >= Q && tx * T2_TT + (ri - Q) < s && ty * T2_TT + (rj - Q) < s;
        const size_t base = size_t(row >> 6) * (64 * W7) + (row & 63);
#pragma unroll
        for (int k = 0; k < W7; ++k) v[q][k] = a.valf[base + k * 64];
        di[q] = a.dinvf[row];
        bb[q] = a.bf[row];
        xi[q] = a.xinf[row];
      }
    }
  };
  // coarse row: corrected iterate into LDS
  T cv[W7], cdi = T(0), cd = T(0), cbv = T(0), cxv = T(0);
  int cring = -1, crow = 0, cri = 0, crj = 0;
  if (tid < Rc) {
    crj = tid / Wc;
    cri = tid - crj * Wc;
    const int cgi = wrap_once(ci0 + cri, sc), cgj = wrap_once(cj0 + crj, sc);
    crow = cgi + sc * cgj;
    cring = min(min(cri, crj), min(Wc - 1 - cri, Wc - 1 - crj));
    const size_t base = size_t(crow >> 6) * (64 * W7) + (crow & 63);
#pragma unroll
    for (int k = 0; k < W7; ++k) cv[k] = a.valc[base + k * 64];
    cdi = a.dinvc[crow];
    cbv = a.bc[crow];
    cxv = a.xc[crow];
    if (a.csteps == 0) cx[tid] = cxv + p1_interp(a.e, cgi, cgj, scc);
  }
  if (a.csteps == 0) load_fine();
  if (a.csteps > 0) {
    // the cut level (side scc) from zero on the region the interpolation
    // reads (origin floor(ci0 / 2) - (S - 1)), in the fine buffers, which
    // are free until the fine correction
    const int S = a.csteps, pi = ci0 & 1, pj = cj0 & 1;
    const int We = t2_cut_side(Wc, pi, S), Re = We * We;
    const int ei0 = ((ci0 + 2 * Hcu) >> 1) - Hcu - (S - 1), ej0 = ((cj0 + 2 * Hcu) >> 1) - Hcu - (S - 1);
    const int offe[W7] = {0, -We - 1, -We, -1, 1, We, We + 1};
    T ev[W7], edi = T(0), eb = T(0), ed = T(0);
    int ering = -1;
    if (tid < Re) {
      const int erj = tid / We, eri = tid - erj * We;
      const int row = wrap_once(ei0 + eri, scc) + scc * wrap_once(ej0 + erj, scc);
      ering = min(min(eri, erj), min(We - 1 - eri, We - 1 - erj));
      const size_t base = size_t(row >> 6) * (64 * W7) + (row & 63);
#pragma unroll
      for (int k = 0; k < W7; ++k) ev[k] = a.valcc[base + k * 64];
      edi = a.dinvcc[row];
      eb = a.bcc[row];
    }
    // the fine rows' operands are in flight during the cut-level steps
    load_fine();
    T* ecur = fx;
    T* enxt = fy;
    for (int k = 0; k < S; ++k) {
      if (ering >= k) {
        T sum = T(0);
        if (k > 0) {
#pragma unroll
          for (int m = 0; m < W7; ++m) sum += ev[m] * ecur[tid + offe[m]];
        }
        const T r = edi * (eb - sum);
        ed = (k == 0) ? a.cc2[0] * r : a.cc1[k] * ed + a.cc2[k] * r;
        enxt[tid] = (k == 0) ? ed : ecur[tid] + ed;
      }
      __syncthreads();
      T* t = ecur;
      ecur = enxt;
      enxt = t;
    }
    // P1 interpolation from the region (coarse column ci0 + cri maps to
    // region column S - 1 + floor((cri + pi) / 2))
    if (tid < Rc) {
      const int I = S - 1 + ((cri + pi) >> 1), J = S - 1 + ((crj + pj) >> 1);
      const int oi = (cri + pi) & 1, oj = (crj + pj) & 1;
      const T e0 = ecur[I + We * J];
      cx[tid] = cxv + ((oi | oj) ? T(0.5) * (e0 + ecur[(I + oi) + We * (J + oj)]) : e0);
    }
  }
  __syncthreads();
  T* ccur = cx;
  T* cnxt = cy;
  for (int k = 0; k < Q; ++k) {
    if (cring >= k + 1) {
      T sum = T(0);
#pragma unroll
      for (int m = 0; m < W7; ++m) sum += cv[m] * ccur[tid + offc[m]];
      const T r = cdi * (cbv - sum);
      cd = (k == 0) ? a.c2[0] * r : a.c1[k] * cd + a.c2[k] * r;
      cnxt[tid] = ccur[tid] + cd;
    }
    __syncthreads();
    T* t = ccur;
    ccur = cnxt;
    cnxt = t;
  }
  // fine correction: P1 interpolation of the coarse result (fine-region
  // column ri maps to coarse-region column floor((ri - Q) / 2) + Hcu)
#pragma unroll
  for (int q = 0; q < T2_RPTU; ++q) {
    const int idx = tid + q * 1024;
    if (idx < R) {
      const int rj = idx / W, ri = idx - rj * W;
      const int ai = ri - Q, aj = rj - Q;
      const int qi = ((ai + 2 * Q) >> 1) - Q + Hcu, qj = ((aj + 2 * Q) >> 1) - Q + Hcu;
      const int oi = ai & 1, oj = aj & 1;
      const T e0 = ccur[qi + Wc * qj];
      const T val = (oi | oj) ? T(0.5) * (e0 + ccur[(qi + oi) + Wc * (qj + oj)]) : e0;
      fx[idx] = xi[q] + val;
    }
  }
  __syncthreads();
  T* cur = fx;
  T* nxt = fy;
  for (int k = 0; k < Q; ++k) {
    const T c1 = a.c1[k], c2 = a.c2[k];
#pragma unroll
    for (int q = 0; q < T2_RPTU; ++q) {
      const int idx = tid + q * 1024;
      if (ring[q] >= k + 1) {
        T sum = T(0);
#pragma unroll
        for (int m = 0; m < W7; ++m) sum += v[q][m] * cur[idx + off[m]];
        const T r = di[q] * (bb[q] - sum);
        const T dn = (k == 0) ? c2 * r : c1 * d[q] + c2 * r;
        d[q] = dn;
        nxt[idx] = cur[idx] + dn;
      }
    }
    __syncthreads();
    T* t = cur;
    cur = nxt;
    nxt = t;
  }
#pragma unroll
  for (int q = 0; q < T2_RPTU; ++q)
    if (own[q]) a.xf[gr[q]] = cur[tid + q * 1024];
}

// ------------------------------------------------------------------ V-cycle tail

// Rows per thread of the tail kernel and its LDS budget (three vectors per
// level: two iterate buffers, the second also holding the residual, and the
// right-hand side).
template <typename T> struct TailCfg;
template <> struct TailCfg<float> { static constexpr int RPT = 1; };
template <> struct TailCfg<double> { static constexpr int RPT = 2; };
constexpr size_t TAIL_LDS = 65536;

__device__ __forceinline__ int tail_off(const int* side, int t) {
  int o = 0;
  for (int u = 0; u < t; ++u) o += 3 * side[u] * side[u];
  return o;
}

// The tail levels of one V-cycle in one workgroup (see vtail).  Each thread
// owns rows tid + q * 1024; a row's 7 values, 1/diag, right-hand side and
// Chebyshev direction stay in registers while its level is being smoothed,
// the iterates (which neighbours gather) in LDS.  Between the level's
// dependent steps only a workgroup barrier is needed, where each step of the
// launch-per-step cycle pays a kernel launch.
template <typename T, int RPT>
__device__ __forceinline__ void vtail_body(const TailArgs<T>* ka, const T* bbase, T* xbase) {
  __shared__ T lds[TAIL_LDS / sizeof(T)];
  __shared__ TailArgs<T> a;
  const int tid = threadIdx.x;
  {
    // the arguments to LDS in one parallel copy: the cycle reads level
    // descriptors and step coefficients at every step, and each scalar load
    // of a fresh argument buffer would wait for memory
    const unsigned* src = reinterpret_cast<const unsigned*>(ka);
    unsigned* dst = reinterpret_cast<unsigned*>(&a);
    for (int i = tid; i < int(sizeof(TailArgs<T>) / 4); i += TAIL_THREADS) dst[i] = src[i];
    __syncthreads();
  }
  // right-hand side and result of the first level
  const T* b0 = bbase ? bbase + a.roff : a.b;
  T* x0 = xbase ? xbase + a.roff : a.x;
  const int last = a.nlev - 1;
  unsigned in_y = 0;  // bit t: level t's iterate is in its second buffer
  T v[RPT][W7], di[RPT], br[RPT], d[RPT];
  int c[RPT][W7];

  // Registers of level t: values, 1/diag, columns and the right-hand side
  // (from LDS, or from global memory on the first level).
  auto load_level = [&](int t, const T* B) {
    const int side = a.side[t], rows = side * side;
    const T* val = a.val[t];
    const T* dv = a.dinv[t];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int row = tid + q * TAIL_THREADS;
      if (row < rows) {
        const size_t base = size_t(row >> 6) * (64 * W7) + (row & 63);
#pragma unroll
        for (int k = 0; k < W7; ++k) v[q][k] = val[base + k * 64];
        p1_cols(row, side, c[q]);
        di[q] = dv[row];
        br[q] = B[row];
      }
    }
  };
  // One Chebyshev step on level t: d <- c1 d + c2 D^{-1} (b - A cur), nxt = cur + d
  // (c1 == 0: d not read).
  auto sweep = [&](int rows, const T* cur, T* nxt, T c1, T c2) {
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int row = tid + q * TAIL_THREADS;
      if (row < rows) {
        T sum = T(0);
#pragma unroll
        for (int k = 0; k < W7; ++k) sum += v[q][k] * cur[c[q][k]];
        const T r = di[q] * (br[q] - sum);
        const T dn = (c1 == T(0)) ? c2 * r : c1 * d[q] + c2 * r;
        d[q] = dn;
        nxt[row] = cur[row] + dn;
      }
    }
    __syncthreads();
  };
  // Chebyshev steps from zero with coefficients (c1, c2)[0..steps); returns
  // whether the iterate ends in the second buffer.
  auto from_zero = [&](int rows, T* X, T* Y, const T* c1, const T* c2, int steps) {
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int row = tid + q * TAIL_THREADS;
      if (row < rows) {
        d[q] = c2[0] * (di[q] * br[q]);
        X[row] = d[q];
      }
    }
    __syncthreads();
    T* cur = X;
    T* nxt = Y;
    for (int k = 1; k < steps; ++k) {
      sweep(rows, cur, nxt, c1[k], c2[k]);
      T* t = cur;
      cur = nxt;
      nxt = t;
    }
    return cur == Y;
  };

  // down: pre-smoothing, residual and restriction on each smoothing level
  for (int t = 0; t < last; ++t) {
    const int side = a.side[t], rows = side * side;
    T* X = lds + tail_off(a.side, t);
    T* Y = X + rows;
    T* B = Y + rows;
    load_level(t, t == 0 ? b0 : B);
    const bool y = from_zero(rows, X, Y, a.pre_c1, a.pre_c2, a.pre);
    if (y) in_y |= 1u << t;
    const T* cur = y ? Y : X;
    T* res = y ? X : Y;
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int row = tid + q * TAIL_THREADS;
      if (row < rows) {
        T sum = T(0);
#pragma unroll
        for (int k = 0; k < W7; ++k) sum += v[q][k] * cur[c[q][k]];
        res[row] = br[q] - sum;
      }
    }
    __syncthreads();
    // R = P^T: a coarse vertex collects its fine vertex and, with weight 1/2,
    // the six edge midpoints around it (the neighbours of the fine vertex)
    const int nc = side >> 1, rows_c = nc * nc;
    T* Bc = lds + tail_off(a.side, t + 1) + 2 * rows_c;
    for (int rc = tid; rc < rows_c; rc += TAIL_THREADS) {
      const int J = rc / nc, I = rc - J * nc;
      int cf[W7];
      p1_cols(2 * I + side * (2 * J), side, cf);
      T s = T(0);
#pragma unroll
      for (int k = 1; k < W7; ++k) s += res[cf[k]];
      Bc[rc] = res[cf[0]] + T(0.5) * s;
    }
    __syncthreads();
  }
  // the cut level
  {
    const int side = a.side[last], rows = side * side;
    T* X = lds + tail_off(a.side, last);
    T* Y = X + rows;
    T* B = Y + rows;
    load_level(last, last == 0 ? b0 : B);
    if (from_zero(rows, X, Y, a.coarse.c1, a.coarse.c2, a.coarse.steps)) in_y |= 1u << last;
  }
  // up: interpolation of the coarse iterate and post-smoothing
  for (int t = last - 1; t >= 0; --t) {
    const int side = a.side[t], rows = side * side, nc = side >> 1;
    T* X = lds + tail_off(a.side, t);
    T* Y = X + rows;
    T* B = Y + rows;
    const T* E = lds + tail_off(a.side, t + 1) + ((in_y >> (t + 1)) & 1u ? nc * nc : 0);
    T* cur = (in_y >> t) & 1u ? Y : X;
    T* nxt = (cur == X) ? Y : X;
    load_level(t, t == 0 ? b0 : B);
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int row = tid + q * TAIL_THREADS;
      if (row < rows) {
        const int j = row / side, i = row - j * side;
        cur[row] += p1_interp(E, i, j, nc);
      }
    }
    __syncthreads();
    for (int k = 0; k < a.post; ++k) {
      sweep(rows, cur, nxt, a.post_c1[k], a.post_c2[k]);
      T* tmp = cur;
      cur = nxt;
      nxt = tmp;
    }
    if (t == 0) {
      in_y = (cur == Y) ? 1u : 0u;
    } else {
      in_y = (in_y & ~(1u << t)) | ((cur == Y ? 1u : 0u) << t);
    }
  }
  // result of the first level
  {
    const int rows = a.side[0] * a.side[0];
    const T* src = lds + (in_y & 1u ? rows : 0);
    for (int row = tid; row < rows; row += TAIL_THREADS) x0[row] = src[row];
  }
}

template <typename T, int RPT>
__global__ __launch_bounds__(TAIL_THREADS) void k_vtail(TailArgs<T> ka) {
  vtail_body<T, RPT>(&ka, nullptr, nullptr);
}

// Batched: workgroup w runs the tail described by list[idx[w]] (skipped when
// its instance is inactive), with right-hand side and result at row offset
// roff of bbase and xbase.
template <typename T, int RPT>
__global__ __launch_bounds__(TAIL_THREADS) void k_bvtail(const TailArgs<T>* __restrict__ list,
                                                         const int* __restrict__ idx,
                                                         const int* __restrict__ act, const T* bbase,
                                                         T* xbase) {
  const TailArgs<T>* t = list + idx[blockIdx.x];
  if (act && !act[t->inst]) return;
  vtail_body<T, RPT>(t, bbase, xbase);
}

template <typename T, typename TV, bool L_IS_M, int W>
__global__ __launch_bounds__(BS) void k_ch_block(int n, int side, const int* __restrict__ col,
                                                 const TV* __restrict__ Lv,
                                                 const TV* __restrict__ Kv,
                                                 const TV* __restrict__ Mv, T c12, T c22,
                                                 const T* __restrict__ x, T alpha, T beta,
                                                 T* y, const T* yin) {
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int row = blk * BS + threadIdx.x;
  if (row >= n) return;
  const size_t base = size_t(row >> 6) * (64 * W) + (row & 63);
  const T* x1 = x;
  const T* x2 = x + n;
  int c[W];
  TV kv[W], mv[W], lv[W];
  row_cols<W>(row, side, col, base, c);
#pragma unroll
  for (int k = 0; k < W; ++k) {
    kv[k] = Kv[base + k * 64];
    mv[k] = Mv[base + k * 64];
    if (!L_IS_M) lv[k] = Lv[base + k * 64];
  }
  T sl = T(0), sk1 = T(0), sk2 = T(0), sm = T(0);
#pragma unroll
  for (int k = 0; k < W; ++k) {
    const T a = x1[c[k]], bb = x2[c[k]];
    sl += T(L_IS_M ? mv[k] : lv[k]) * a;
    sk1 += T(kv[k]) * a;
    sk2 += T(kv[k]) * bb;
    sm += T(mv[k]) * bb;
  }
  const T y1 = alpha * (sl + c12 * sk2);
  const T y2 = alpha * (c12 * sk1 + c22 * sm);
  if (beta == T(0)) {
    y[row] = y1;
    y[n + row] = y2;
  } else {
    const T* yb = yin ? yin : y;
    y[row] = y1 + beta * yb[row];
    y[n + row] = y2 + beta * yb[n + row];
  }
}

// ------------------------------------------------------------------ vectors

template <typename T>
__global__ __launch_bounds__(BS) void k_axpby(int64_t n, T a, const T* __restrict__ x, T b,
                                              T* __restrict__ y) {
  const int64_t i = int64_t(blockIdx.x) * BS + threadIdx.x;
  if (i < n) y[i] = (b == T(0)) ? a * x[i] : a * x[i] + b * y[i];
}

template <typename TI, typename TO>
__global__ __launch_bounds__(BS) void k_convert(int64_t n, const TI* __restrict__ x,
                                                TO* __restrict__ y) {
  const int64_t i = int64_t(blockIdx.x) * BS + threadIdx.x;
  if (i < n) y[i] = TO(x[i]);
}

// y = double(x) * inv[0] (inv may be null: plain conversion).
__global__ __launch_bounds__(BS) void k_convert_out(int64_t n, const float* __restrict__ x,
                                                    const double* __restrict__ inv,
                                                    double* __restrict__ y) {
  const int64_t i = int64_t(blockIdx.x) * BS + threadIdx.x;
  if (i < n) y[i] = inv ? double(x[i]) * inv[0] : double(x[i]);
}

// x <- x * inv[0] (written back) and y = float(x * inv[0]).
__global__ __launch_bounds__(BS) void k_convert_scaled(int64_t n, double* __restrict__ x,
                                                       const double* __restrict__ inv,
                                                       float* __restrict__ y) {
  const int64_t i = int64_t(blockIdx.x) * BS + threadIdx.x;
  if (i < n) {
    const double v = x[i] * inv[0];
    x[i] = v;
    y[i] = float(v);
  }
}

__global__ __launch_bounds__(BS) void k_scale_by_inv(int64_t n, const double* __restrict__ x,
                                                     const double* __restrict__ inv,
                                                     double* __restrict__ y) {
  const int64_t i = int64_t(blockIdx.x) * BS + threadIdx.x;
  if (i < n) y[i] = x[i] * inv[0];
}

// ------------------------------------------------------------------ Krylov reductions

// Delayed classical Gram-Schmidt with reorthogonalisation (DCGS2): at Arnoldi
// step j the stored vector V_j (= vt) is orthogonalised once; one pass over
// V_0..V_{j-1} gives both its reorthogonalisation dots and the projection dots
// of the new vector w = V_{j+1}, one pass applies both updates.

constexpr int DG = 16;  // basis vectors per group of the dot pass

// One workgroup per slot: red[k] = sum of slot k's nblk partials
// (part[k * nblk + b]), in a fixed order.
__global__ __launch_bounds__(BS) void k_slot_reduce(int nblk, const double* __restrict__ part,
                                                    double* __restrict__ red) {
  __shared__ double sh[4];
  const int k = blockIdx.x;
  double a = 0.0;
  for (int b = threadIdx.x; b < nblk; b += BS) a += part[int64_t(k) * nblk + b];
  a = block_sum(a, sh);
  if (threadIdx.x == 0) red[k] = a;
}

// Coefficients of step j from the reduced dots, formed by the first wavefront
// of a workgroup into LDS.  j >= 1: vt = sum c_i V_i + r v_j with
// r = sqrt(vt.vt - |c|^2); column j-1 of the raw Hessenberg H (whose last entry
// multiplied vt) becomes h_i += h_j c_i, h_j *= r.  Projection of w on the
// final basis: a_i = V_i . w (i < j), b = (vt . w - c . a) / r; so
// w' = w - sum (a_i - b c_i / r) V_i - (b / r) vt and v_j = (vt - sum c_i V_i) / r.
// cf: [0, j) c_i, [j, 2j+1) the w coefficients (last one multiplies vt),
// 2j+1: 1/r.  H is written only when write_h (one workgroup of the launch).
// j < 64.
__device__ void form_coefs(int j, int m, const double* __restrict__ red, double* __restrict__ H,
                           double* __restrict__ cf, bool write_h) {
  const int t = threadIdx.x, ld = m + 1;
  const double c = t < j ? red[t] : 0.0;
  const double a = t < j ? red[j + t] : 0.0;
  const double cc = wave_sum(c * c), ca = wave_sum(c * a);
  const double nu = red[2 * j], tw = red[2 * j + 1];
  const double r = j > 0 ? sqrt(fmax(nu - cc, 0.0)) : 1.0;
  const double inv = r > 0.0 ? 1.0 / r : 0.0;
  const double b = (tw - ca) * inv;
  if (t < j) {
    cf[t] = c;
    cf[j + t] = a - b * c * inv;
  }
  if (t == 0) {
    cf[2 * j] = b * inv;
    cf[2 * j + 1] = inv;
  }
  if (!write_h) return;
  const double hj = j > 0 ? H[int64_t(j - 1) * ld + j] : 0.0;
  if (j > 0 && t <= j) {
    double* hp = H + int64_t(j - 1) * ld;
    hp[t] = (t < j) ? hp[t] + hj * c : hj * r;
  }
  double* h = H + int64_t(j) * ld;
  if (t < j) h[t] = a;
  if (t == 0) h[j] = b;
}

// The CH block product w = A z (both block rows of node r: y1 = L z1 + c12 K
// z2, y2 = c12 K z1 + c22 M z2, as k_ch_block with alpha = 1, beta = 0) fused
// with the dot pass of Arnoldi step j = KK < DG: w is written once and its dots
// are taken from registers (the separate pass would read it back).  Slots as
// k_dcgs_dots with LAST; partials per block, grid-stride over the nodes.
template <int KK, bool L_IS_M, int W>
__global__ __launch_bounds__(BS) void k_ch_dots(int N, int side, const int* __restrict__ col,
                                                const double* __restrict__ Lv, const double* __restrict__ Kv,
                                                const double* __restrict__ Mv, double c12, double c22,
                                                const double* __restrict__ z, double* __restrict__ V,
                                                int64_t ld, double* __restrict__ part,
                                                const double* __restrict__ vscale) {
  constexpr int NV = 2 * KK + 3;
  constexpr int j = KK;
  __shared__ double sh[4][NV];
  const double* vt = V + int64_t(j) * ld;
  double* w = V + int64_t(j + 1) * ld;
  const double sv = vscale ? vscale[0] : 1.0;
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.0;
  const int stride = gridDim.x * BS;
  // XCD-contiguous blocks: the mesh lines above and below a block's rows are
  // mostly read through the same XCD's L2
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  for (int row = blk * BS + threadIdx.x; row < N; row += stride) {
    const size_t base = size_t(row >> 6) * (64 * W) + (row & 63);
    int c[W];
    row_cols<W>(row, side, col, base, c);
    double sl = 0.0, sk1 = 0.0, sk2 = 0.0, sm = 0.0;
#pragma unroll
    for (int k = 0; k < W; ++k) {
      const double kv = Kv[base + k * 64], mv = Mv[base + k * 64];
      const double lv = L_IS_M ? mv : Lv[base + k * 64];
      const double a = z[c[k]], bb = z[N + c[k]];
      sl += lv * a;
      sk1 += kv * a;
      sk2 += kv * bb;
      sm += mv * bb;
    }
    const double y[2] = {sl + c12 * sk2, c12 * sk1 + c22 * sm};
    w[row] = y[0];
    w[N + row] = y[1];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t e = row + int64_t(h) * N;
      const double t = vt[e] * sv, wr = y[h];
      double v[KK > 0 ? KK : 1];
#pragma unroll
      for (int i = 0; i < KK; ++i) v[i] = __builtin_nontemporal_load(V + i * ld + e);
#pragma unroll
      for (int i = 0; i < KK; ++i) {
        acc[i] += v[i] * t;
        acc[KK + i] += v[i] * wr;
      }
      acc[2 * KK] += t * t;
      acc[2 * KK + 1] += t * wr;
      acc[2 * KK + 2] += wr * wr;
    }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int sbase = 0, lim = NV;
  WaveRS<NV, 32>::run(acc, lane, sbase, lim);
  if (lim >= 1) sh[wid][sbase] = acc[0];
  __syncthreads();
  const int t = threadIdx.x;
  if (t < NV) {
    const double sum = (sh[0][t] + sh[1][t]) + (sh[2][t] + sh[3][t]);
    const int64_t slot = t < KK ? t : (t < 2 * KK ? j + (t - KK) : 2 * j + (t - 2 * KK));
    part[slot * gridDim.x + blockIdx.x] = sum;
  }
}

// Dots of KK basis vectors V_g0 .. V_{g0+KK-1} against vt and w, and with
// LAST also vt . vt, vt . w, w . w.  Slots (per block partial, stride
// gridDim.x): [0, j) V_i . vt, [j, 2j) V_i . w, then 2j, 2j+1, 2j+2.  KK is a
// compile-time count so that every load of a row is issued before its FMAs;
// the epilogue reduces the accumulators per wavefront by a reduce-scatter and
// then across the 4 wavefronts with one barrier.
template <int KK, bool LAST>
__global__ __launch_bounds__(BS) void k_dcgs_dots(int64_t n, const double* __restrict__ V, int64_t ld,
                                                  int j, int g0, double* __restrict__ part,
                                                  const double* __restrict__ vscale) {
  constexpr int NV = 2 * KK + (LAST ? 3 : 0);
  __shared__ double sh[4][NV > 0 ? NV : 1];
  const double* vt = V + int64_t(j) * ld;
  const double* w = V + int64_t(j + 1) * ld;
  const double sv = vscale ? vscale[0] : 1.0;
  double acc[NV > 0 ? NV : 1];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.0;
  const int64_t stride = int64_t(gridDim.x) * BS;
  for (int64_t r = int64_t(blockIdx.x) * BS + threadIdx.x; r < n; r += stride) {
    const double t = vt[r] * sv, wr = w[r];
    double v[KK > 0 ? KK : 1];
#pragma unroll
    // basis vectors: non-temporal loads, so that the streamed basis does not
    // evict the operator values the preconditioner and the matrix product reuse
    // from the last-level cache
    for (int i = 0; i < KK; ++i) v[i] = __builtin_nontemporal_load(V + (g0 + i) * ld + r);
#pragma unroll
    for (int i = 0; i < KK; ++i) {
      acc[i] += v[i] * t;
      acc[KK + i] += v[i] * wr;
    }
    if (LAST) {
      acc[2 * KK] += t * t;
      acc[2 * KK + 1] += t * wr;
      acc[2 * KK + 2] += wr * wr;
    }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if constexpr (NV > 0) {
    int base = 0, lim = NV;
    WaveRS<NV, 32>::run(acc, lane, base, lim);
    if (lim >= 1) sh[wid][base] = acc[0];
  }
  __syncthreads();
  const int t = threadIdx.x;
  if (t < NV) {
    const double s = (sh[0][t] + sh[1][t]) + (sh[2][t] + sh[3][t]);
    int64_t slot;
    if (t < KK) slot = g0 + t;
    else if (t < 2 * KK) slot = j + g0 + (t - KK);
    else slot = 2 * j + (t - 2 * KK);
    part[slot * gridDim.x + blockIdx.x] = s;
  }
}


__device__ __forceinline__ void givens(double a, double b, double& c, double& s) {
  if (b == 0.0) {
    c = 1.0;
    s = 0.0;
  } else if (fabs(b) > fabs(a)) {
    const double t = a / b;
    s = 1.0 / sqrt(1.0 + t * t);
    c = t * s;
  } else {
    const double t = b / a;
    c = 1.0 / sqrt(1.0 + t * t);
    s = t * c;
  }
}

// Rotations 0..upto-1 applied in order to x[0..upto] (x[upto+1..] untouched):
// rotation i maps (x_i, x_{i+1}) to (c_i x_i + s_i x_{i+1}, -s_i x_i + c_i x_{i+1}).
__device__ __forceinline__ void apply_rotations(double* x, int upto, const double* c, const double* s) {
  double carry = x[0];
  for (int i = 0; i < upto; ++i) {
    const double b = x[i + 1];
    x[i] = c[i] * carry + s[i] * b;
    carry = -s[i] * carry + c[i] * b;
  }
  x[upto] = carry;
}

// End of step j, by one workgroup: h_{j+1,j} = |w'| (provisional until the
// next step corrects it); column j-1 is final now: rotate it into HR, fix
// rotation j-1 and the right-hand side g.  Column j gets a provisional
// rotation: HR column j and gp (g with the provisional rotation) serve the
// residual estimate and, if the cycle ends here, the least-squares solve.
// scal = (estimate, 1/|w'|, |w'|), also written to `host` (pinned host memory)
// when given.  The columns, rotations and g are staged in LDS (their loads in
// flight with those of the norm partials) so that the serial rotation chain
// runs at LDS latency.
__global__ __launch_bounds__(BS) void k_dcgs_finish(int nblk, const double* __restrict__ nrm_part, int j,
                                                    int m, double* __restrict__ H, double* __restrict__ HR,
                                                    double* __restrict__ cs, double* __restrict__ sn,
                                                    double* __restrict__ g, double* __restrict__ gp,
                                                    double* __restrict__ scal, double* __restrict__ host,
                                                    double tag) {
  __shared__ double hp[66], hc[66], cs_s[64], sn_s[64], g_s[66], res[3];
  __shared__ double sh[4];
  const int ld = m + 1, t = threadIdx.x;
  if (t <= j) hc[t] = H[int64_t(j) * ld + t];
  if (j > 0 && t <= j) hp[t] = H[int64_t(j - 1) * ld + t];
  if (t + 1 < j) {
    cs_s[t] = cs[t];
    sn_s[t] = sn[t];
  }
  if (t <= j) g_s[t] = g[t];
  double a = 0.0;
  for (int b = t; b < nblk; b += BS) a += nrm_part[b];
  const double nrm = sqrt(block_sum(a, sh));  // valid in thread 0, which alone uses it
  if (t == 0) {
    hc[j + 1] = nrm;
    if (j > 0) {
      apply_rotations(hp, j - 1, cs_s, sn_s);
      double c, s;
      givens(hp[j - 1], hp[j], c, s);
      cs_s[j - 1] = c;
      sn_s[j - 1] = s;
      hp[j - 1] = c * hp[j - 1] + s * hp[j];
      hp[j] = 0.0;
      g_s[j] = -s * g_s[j - 1];
      g_s[j - 1] = c * g_s[j - 1];
    }
    apply_rotations(hc, j, cs_s, sn_s);
    double c, s;
    givens(hc[j], hc[j + 1], c, s);
    hc[j] = c * hc[j] + s * hc[j + 1];
    hc[j + 1] = 0.0;
    res[0] = c * g_s[j];
    res[1] = -s * g_s[j];
    res[2] = nrm;
  }
  __syncthreads();
  const double nr = res[2];
  if (t == 0) H[int64_t(j) * ld + j + 1] = nr;
  if (t <= j + 1) HR[int64_t(j) * ld + t] = hc[t];
  if (j > 0 && t <= j) HR[int64_t(j - 1) * ld + t] = hp[t];
  if (j > 0 && t == 0) {
    cs[j - 1] = cs_s[j - 1];
    sn[j - 1] = sn_s[j - 1];
    g[j - 1] = g_s[j - 1];
    g[j] = g_s[j];
  }
  if (t < j) gp[t] = g_s[t];
  if (t == 0) {
    gp[j] = res[0];
    gp[j + 1] = res[1];
    const double sv[3] = {fabs(res[1]), nr > 0.0 ? 1.0 / nr : 0.0, nr};
    for (int i = 0; i < 3; ++i) scal[i] = sv[i];
    if (host) {
      for (int i = 0; i < 3; ++i) host[i] = sv[i];
      __threadfence_system();
      host[3] = tag;
      __threadfence_system();
    }
  }
}

// w <- w - sum_{i<j} cf[j+i] V_i - cf[2j] vt; vt <- (vt - sum_{i<j} cf[i] V_i) / r
// (j > 0); per-block partials of |w'|^2.
// Every workgroup forms the coefficients from the slot sums `red` itself
// (form_coefs); workgroup 0 also corrects H.
__global__ __launch_bounds__(BS) void k_dcgs_update(int64_t n, double* __restrict__ V, int64_t ld, int j,
                                                    int m, const double* __restrict__ red,
                                                    double* __restrict__ H, double* __restrict__ nrm_part,
                                                    const double* __restrict__ vscale) {
  __shared__ double cs_l[2 * 64 + 2];
  __shared__ double sh[4];
  if (threadIdx.x < 64) form_coefs(j, m, red, H, cs_l, blockIdx.x == 0);
  __syncthreads();
  double* vt = V + int64_t(j) * ld;
  double* w = V + int64_t(j + 1) * ld;
  const double inv = cs_l[2 * j + 1], wt = cs_l[2 * j];
  const double sv = vscale ? vscale[0] : 1.0;
  double acc = 0.0;
  const int64_t stride = int64_t(gridDim.x) * BS;
  for (int64_t r = int64_t(blockIdx.x) * BS + threadIdx.x; r < n; r += stride) {
    const double t = vt[r] * sv;
    double wn = w[r] - wt * t, vn = t;
    int i = 0;
    // groups of 8: all loads issued before the FMAs; basis vectors loaded
    // non-temporally (last use in this step)
    for (; i + 8 <= j; i += 8) {
      double v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = __builtin_nontemporal_load(V + (i + q) * ld + r);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        vn -= cs_l[i + q] * v[q];
        wn -= cs_l[j + i + q] * v[q];
      }
    }
    const int rem = j - i;
    if (rem > 0) {  // the rest (< 8): all loads issued before the FMAs
      double v[7];
#pragma unroll
      for (int q = 0; q < 7; ++q)
        if (q < rem) v[q] = __builtin_nontemporal_load(V + (i + q) * ld + r);
#pragma unroll
      for (int q = 0; q < 7; ++q)
        if (q < rem) {
          vn -= cs_l[i + q] * v[q];
          wn -= cs_l[j + i + q] * v[q];
        }
    }
    if (j > 0) vt[r] = vn * inv;
    w[r] = wn;
    acc += wn * wn;
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) nrm_part[blockIdx.x] = s;
}

__device__ double sum_partials_wave(int nblk, const double* part) {
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  for (int b = lane; b < nblk; b += 64) s += part[b];
  return wave_sum(s);
}

// y = R^{-1} g for the k x k upper triangle R of H (column-major, ld m + 1):
// the triangle and g are staged in LDS by the whole workgroup, then one
// thread back-substitutes at LDS latency.
__global__ __launch_bounds__(BS) void k_lsq_solve(int k, int m, const double* __restrict__ H,
                                                  const double* __restrict__ g, double* __restrict__ y) {
  __shared__ double R[64 * 65], gs[64], ys[64];
  const int ld = m + 1;
  for (int q = threadIdx.x; q < k * k; q += BS) {
    const int l = q / k, i = q - l * k;  // column l, row i
    if (i <= l) R[l * 65 + i] = H[int64_t(l) * ld + i];
  }
  for (int i = threadIdx.x; i < k; i += BS) gs[i] = g[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = k - 1; i >= 0; --i) {
      double s = gs[i];
      for (int l = i + 1; l < k; ++l) s -= R[l * 65 + i] * ys[l];
      ys[i] = s / R[i * 65 + i];
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < k; i += BS) y[i] = ys[i];
}

__global__ __launch_bounds__(BS) void k_xupdate(int64_t n, const double* __restrict__ Z,
                                                int64_t ldz, int k, const double* __restrict__ y,
                                                double* __restrict__ x) {
  __shared__ double ys[257];
  for (int i = threadIdx.x; i < k; i += BS) ys[i] = y[i];
  __syncthreads();
  const int64_t r = int64_t(blockIdx.x) * BS + threadIdx.x;
  if (r >= n) return;
  double s = x[r];
  for (int i = 0; i < k; ++i) s += ys[i] * __builtin_nontemporal_load(Z + i * ldz + r);  // last use of Z
  x[r] = s;
}

__global__ __launch_bounds__(BS) void k_norm_partial(int64_t n, const double* __restrict__ w,
                                                     double* __restrict__ part) {
  __shared__ double sh[4];
  double acc = 0.0;
  const int64_t stride = int64_t(gridDim.x) * BS;
  for (int64_t r = int64_t(blockIdx.x) * BS + threadIdx.x; r < n; r += stride) acc += w[r] * w[r];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_norm_finish(int nblk, const double* __restrict__ part, double* __restrict__ scal,
                              double* __restrict__ g, int m, double* __restrict__ host, double tag) {
  const double nrm = sqrt(sum_partials_wave(nblk, part));
  if (threadIdx.x == 0) {
    const double sv[3] = {nrm, nrm > 0.0 ? 1.0 / nrm : 0.0, nrm};
    for (int i = 0; i < 3; ++i) scal[i] = sv[i];
    if (g) {
      g[0] = nrm;
      for (int i = 1; i <= m; ++i) g[i] = 0.0;
    }
    if (host) {
      for (int i = 0; i < 3; ++i) host[i] = sv[i];
      __threadfence_system();
      host[3] = tag;
      __threadfence_system();
    }
  }
}

// ------------------------------------------------------------------ assembly

__global__ __launch_bounds__(BS) void k_assemble_p1(int kind, int e0, int e1,
                                                    const int* __restrict__ ep2,
                                                    const int* __restrict__ etype,
                                                    const int* __restrict__ eslot, double h,
                                                    const double* __restrict__ vel, int64_t n2,
                                                    double* __restrict__ val,
                                                    const double* __restrict__ rho) {
  const int e = e0 + blockIdx.x * BS + threadIdx.x;
  if (e >= e1) return;
  // local vertex coordinates relative to the first vertex
  double x1, y1, x2, y2;
  if (etype[e] == 0) {  // (i,j), (i+1,j), (i+1,j+1)
    x1 = h; y1 = 0.0; x2 = h; y2 = h;
  } else {              // (i,j), (i+1,j+1), (i,j+1)
    x1 = h; y1 = h; x2 = 0.0; y2 = h;
  }
  const double det = x1 * y2 - x2 * y1;
  const double area = 0.5 * fabs(det);
  double gx[3], gy[3];
  gx[1] = y2 / det;  gy[1] = -x2 / det;
  gx[2] = -y1 / det; gy[2] = x1 / det;
  gx[0] = -gx[1] - gx[2];
  gy[0] = -gy[1] - gy[2];
  double loc[9];
  if (kind == 0) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) loc[a * 3 + b] = area / 12.0 * (a == b ? 2.0 : 1.0);
  } else if (kind == 3) {
    // int rho lambda_a lambda_b, rho = sum_c rho_c lambda_c: int lambda_a lambda_b
    // lambda_c = |T| / 10 (all equal), / 30 (two equal), / 60 (all distinct)
    double r[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) r[c] = rho[ep2[e * 6 + c]];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const int eq = (a == b) + (b == c) + (a == c);  // 3: all equal, 1: two equal, 0: distinct
          acc += r[c] * (eq == 3 ? 1.0 / 10.0 : (eq == 1 ? 1.0 / 30.0 : 1.0 / 60.0));
        }
        loc[a * 3 + b] = area * acc;
      }
  } else if (kind == 1) {
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) loc[a * 3 + b] = area * (gx[a] * gx[b] + gy[a] * gy[b]);
  } else {
    double vx[6], vy[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const int node = ep2[e * 6 + k];
      vx[k] = vel[node];
      vy[k] = vel[n2 + node];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double Va_x = 0.0, Va_y = 0.0;
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        const double wk = w_p2p1(k, a);
        Va_x += wk * vx[k];
        Va_y += wk * vy[k];
      }
#pragma unroll
      for (int b = 0; b < 3; ++b) loc[a * 3 + b] = area * (Va_x * gx[b] + Va_y * gy[b]);
    }
  }
#pragma unroll
  for (int q = 0; q < 9; ++q) val[eslot[e * 9 + q]] += loc[q];
}

__global__ __launch_bounds__(BS) void k_galerkin(int64_t nslots, const int* __restrict__ ptr,
                                                 const int* __restrict__ src,
                                                 const double* __restrict__ w,
                                                 const double* __restrict__ fine,
                                                 double* __restrict__ coarse) {
  const int64_t s = int64_t(blockIdx.x) * BS + threadIdx.x;
  if (s >= nslots) return;
  double acc = 0.0;
  for (int q = ptr[s]; q < ptr[s + 1]; ++q) acc += w[q] * fine[src[q]];
  coarse[s] = acc;
}

__global__ __launch_bounds__(BS) void k_combine(int64_t n, double a, const double* __restrict__ A,
                                                double b, const double* __restrict__ B, double c,
                                                const double* __restrict__ C,
                                                double* __restrict__ o64, float* __restrict__ o32) {
  const int64_t i = int64_t(blockIdx.x) * BS + threadIdx.x;
  if (i >= n) return;
  double v = a * A[i];
  if (B) v += b * B[i];
  if (C) v += c * C[i];
  o64[i] = v;
  if (o32) o32[i] = float(v);
}

__global__ __launch_bounds__(BS) void k_diag_inverse(int n, const int* __restrict__ diag,
                                                     const double* __restrict__ val,
                                                     double* __restrict__ d64,
                                                     float* __restrict__ d32) {
  const int i = blockIdx.x * BS + threadIdx.x;
  if (i >= n) return;
  const double v = val[diag[i]];
  const double d = (v != 0.0) ? 1.0 / v : 0.0;  // padding rows of stacked levels hold zeros
  d64[i] = d;
  if (d32) d32[i] = float(d);
}

__device__ __forceinline__ double form_value(const FormCoef& k, int o, bool conv, double m, double kk,
                                             double cc) {
  double v = k.a[o] * m;
  if (k.useK[o]) v += k.b[o] * kk;
  if (conv && k.useC[o]) v += k.c[o] * cc;
  return v;
}

__global__ __launch_bounds__(BS) void k_form_ops(int nlev, const FormLevel* __restrict__ tab, int64_t total,
                                                 FormCoef k, int conv) {
  const int64_t i = int64_t(blockIdx.x) * BS + threadIdx.x;
  if (i >= total) return;
  int l = 0;
  while (l + 1 < nlev && i >= tab[l + 1].begin) ++l;
  const FormLevel& t = tab[l];
  int64_t q = i - t.begin;
  if (q < t.ns) {
    const double m = t.M[q], kk = t.K[q], cc = conv ? t.C[q] : 0.0;
#pragma unroll
    for (int o = 0; o < 3; ++o) {
      const double v = form_value(k, o, conv, m, kk, cc);
      t.v64[o][q] = v;
      if (t.v32[o]) t.v32[o][q] = float(v);
    }
  } else {
    q -= t.ns;
    if (q >= t.N) return;
    const int ds = t.diag[q];
    const double m = t.M[ds], kk = t.K[ds], cc = conv ? t.C[ds] : 0.0;
#pragma unroll
    for (int o = 0; o < 3; ++o) {
      const double v = form_value(k, o, conv, m, kk, cc);
      const double d = (v != 0.0) ? 1.0 / v : 0.0;
      t.d64[o][q] = d;
      if (t.d32[o]) t.d32[o][q] = float(d);
    }
  }
}

// ------------------------------------------------------------------ diagnostics

// Local free-energy densities: the binary double-well phi^2 (1 - phi)^2 for the
// liquid and phi^2 + (1 - phi)^2 for the gas, interpolated by p(Phi) =
// Phi^2 (3 - 2 Phi) (no vapour field: the liquid form alone); the ternary
// fitted quartic with air = 0 and phi_s = 1 - phi_p - phi_N.
__device__ __forceinline__ double density_binary(double phi, const double* Phi, int j) {
  const double om = 1.0 - phi;
  const double liq = phi * phi * om * om;
  if (!Phi) return liq;
  const double P = Phi[j], p = P * P * (3.0 - 2.0 * P);
  return (1.0 - p) * liq + p * (phi * phi + om * om);
}



// Per row: the row sum of M (the nodal weight), the masses weight * u, the
// gradient terms u (K u) of each phase and weight * density; per block the
// five sums.
template <int W>
__global__ __launch_bounds__(BS) void k_diag(int n, int side, const int* __restrict__ col,
                                             const double* __restrict__ Mv, const double* __restrict__ Kv,
                                             const double* __restrict__ p0, const double* __restrict__ p1,
                                             const double* __restrict__ p2,
                                             const double* __restrict__ Phi, int ternary, KorBeta kb,
                                             PotCoef pc, double* __restrict__ part) {
  __shared__ double sh[4];
  double acc[NDIAG] = {0.0, 0.0, 0.0, 0.0, 0.0};
  const int stride = gridDim.x * BS;
  for (int row = blockIdx.x * BS + threadIdx.x; row < n; row += stride) {
    const size_t base = size_t(row >> 6) * (64 * W) + (row & 63);
    int c[W];
    row_cols<W>(row, side, col, base, c);
    // K-weighted sums of the phases and of the eliminated one
    double w = 0.0, k0 = 0.0, k1 = 0.0, k2 = 0.0, k3 = 0.0;
#pragma unroll
    for (int k = 0; k < W; ++k) {
      const double kv = Kv[base + k * 64], a = p0[c[k]];
      w += Mv[base + k * 64];
      k0 += kv * a;
      if (ternary) {
        const double b = p1[c[k]], d = p2 ? p2[c[k]] : 0.0;
        k1 += kv * b;
        if (p2) k2 += kv * d;
        k3 += kv * (1.0 - a - b - d);
      }
    }
    const double u0 = p0[row];
    double grad = kb.b[0] * u0 * k0, f;
    acc[0] += w * u0;
    if (ternary) {
      const double u1 = p1[row], u2 = p2 ? p2[row] : 0.0, ue = 1.0 - u0 - u1 - u2;
      acc[1] += w * u1;
      if (p2) {  // quaternary: polymer, NFA, solvent given, air eliminated
        acc[2] += w * u2;
        grad += kb.b[1] * u1 * k1 + kb.b[2] * u2 * k2 + kb.b[3] * ue * k3;
        f = density_quaternary(u0, u1, u2, Phi ? Phi[row] : 0.0);
      } else {   // ternary: the solvent eliminated
        acc[2] += w * ue;
        grad += kb.b[1] * u1 * k1 + kb.b[2] * ue * k3;
        f = density_ternary(u0, u1, Phi ? Phi[row] : 0.0, pc);
      }
    } else {
      f = density_binary(u0, Phi, row);
    }
    if (Phi) acc[3] += w * Phi[row];
    acc[4] += 0.5 * grad + w * f;
  }
#pragma unroll
  for (int q = 0; q < NDIAG; ++q) {
    const double v = block_sum(acc[q], sh);
    if (threadIdx.x == 0) part[q * gridDim.x + blockIdx.x] = v;
  }
}

__global__ __launch_bounds__(BS) void k_diag_finish(int nblk, const double* __restrict__ part,
                                                    double* __restrict__ out) {
  __shared__ double sh[4];
  for (int q = 0; q < NDIAG; ++q) {
    double a = 0.0;
    for (int b = threadIdx.x; b < nblk; b += BS) a += part[q * nblk + b];
    a = block_sum(a, sh);
    if (threadIdx.x == 0) out[q] = a;
  }
}

// ------------------------------------------------------------------ right-hand sides

__device__ __forceinline__ void binary_terms(double phi, const double* Phi, int j, double& fp,
                                             double& fv) {
  const double om = 1.0 - phi;
  const double dliq = 2.0 * phi * om * om - 2.0 * phi * phi * om;
  if (!Phi) {
    fp = dliq;
    fv = 0.0;
    return;
  }
  const double P = Phi[j];
  const double p = P * P * (3.0 - 2.0 * P);
  const double dgas = 2.0 * phi - 2.0 * om;
  fp = (1.0 - p) * dliq + p * dgas;
  const double fliq = phi * phi * om * om, fgas = phi * phi + om * om;
  fv = 6.0 * P * (1.0 - P) * (fgas - fliq);
}

template <int W>
__global__ __launch_bounds__(BS) void k_rhs_binary(int n, int side, const int* __restrict__ col,
                                                   const double* __restrict__ Mv,
                                                   const double* __restrict__ phi,
                                                   const double* __restrict__ Phi, double c_mu,
                                                   double c_ac, TopFlux tf, double* __restrict__ rhs_ch,
                                                   double* __restrict__ rhs_ac) {
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int row = blk * BS + threadIdx.x;
  if (row >= n) return;
  const size_t base = size_t(row >> 6) * (64 * W) + (row & 63);
  double s_phi = 0.0, s_fp = 0.0, s_Phi = 0.0, s_fv = 0.0;
  int cc[W];
  row_cols<W>(row, side, col, base, cc);
#pragma unroll
  for (int k = 0; k < W; ++k) {
    const int j = cc[k];
    const double m = Mv[base + k * 64];
    const double ph = phi[j];
    double fp, fv;
    binary_terms(ph, Phi, j, fp, fv);
    s_phi += m * ph;
    s_fp += m * fp;
    if (Phi) {
      s_Phi += m * Phi[j];
      s_fv += m * fv;
    }
  }
  rhs_ch[row] = s_phi;
  double second = c_mu * s_fp;
  if (tf.coef != 0.0 && row >= tf.top0) {
    const double w = tf.w ? tf.w[row - tf.top0] : ((row == tf.top0 || row == n - 1) ? 0.5 * tf.h : tf.h);
    second += tf.coef * (phi[tf.ref] - tf.phi_inf) * w;
  }
  rhs_ch[n + row] = second;
  if (rhs_ac) rhs_ac[row] = s_Phi + c_ac * s_fv;
}

// ------------------------------------------------------------------ Taylor-Hood

template <typename T, typename TV, int MODE>
__global__ __launch_bounds__(BS) void k_sell_op(int nslices, int nrows, const int* __restrict__ sptr,
                                                const int* __restrict__ sw,
                                                const int* __restrict__ col,
                                                const TV* __restrict__ val,
                                                const int* __restrict__ perm,
                                                const T* __restrict__ x, const T* __restrict__ b,
                                                const T* __restrict__ dinv, T* __restrict__ d,
                                                T c1, T c2, T* __restrict__ y) {
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int pos = blk * BS + threadIdx.x;
  const int slice = pos >> 6, lane = pos & 63;
  if (slice >= nslices) return;
  const int row = perm ? perm[pos] : pos;
  if (row < 0 || row >= nrows) return;
  const int w = sw[slice];
  const int base = sptr[slice] + lane;
  T sum = T(0);
  for (int k = 0; k < w; ++k) {
    const int q = base + k * 64;
    sum += T(val[q]) * x[col[q]];
  }
  if (MODE == ST_RESID) {
    y[row] = b[row] - sum;
  } else {
    const T r = dinv[row] * (b[row] - sum);
    const T dn = (c1 == T(0)) ? c2 * r : c1 * d[row] + c2 * r;
    d[row] = dn;
    y[row] = x[row] + dn;
  }
}

__global__ __launch_bounds__(BS) void k_assemble_p2(int kind, int e0, int e1,
                                                    const int* __restrict__ ep1,
                                                    const int* __restrict__ ep2,
                                                    const int* __restrict__ etype,
                                                    const int* __restrict__ eslot, double h,
                                                    DP2Tables tb, double eta,
                                                    const double* __restrict__ vel, double wscale,
                                                    int64_t n2, MuGrad mg, double* o0, double* o1,
                                                    double* o2, double* o3,
                                                    const double* __restrict__ rho) {
  const int e = e0 + blockIdx.x * BS + threadIdx.x;
  if (e >= e1) return;
  const ElemGeo g = elem_geo(etype[e], h);
  const int* slot = eslot + size_t(e) * 36;
  if (kind == 0) {
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) o0[slot[i * 6 + j]] += g.area * tb.MM[i * 6 + j];
    return;
  }
  if (kind == 3) {  // int rho psi_i psi_j, rho the P1 field at the vertices
    double r[3];
    for (int a = 0; a < 3; ++a) r[a] = rho[ep2[e * 6 + a]];
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j)
        o0[slot[i * 6 + j]] +=
            g.area * (r[0] * tb.MW[i * 6 + j] + r[1] * tb.MW[36 + i * 6 + j] + r[2] * tb.MW[72 + i * 6 + j]);
    return;
  }
  if (kind == 1) {
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) {
        double gxx = 0, gxy = 0, gyx = 0, gyy = 0;  // G^{cd}[i][j] = int d_c psi_i d_d psi_j
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) {
            const double sv = tb.S[((i * 3 + a) * 6 + j) * 3 + b];
            gxx += g.gx[a] * g.gx[b] * sv;
            gxy += g.gx[a] * g.gy[b] * sv;
            gyx += g.gy[a] * g.gx[b] * sv;
            gyy += g.gy[a] * g.gy[b] * sv;
          }
        const int q = slot[i * 6 + j];
        o0[q] += eta * g.area * (2.0 * gxx + gyy);
        o1[q] += eta * g.area * gyx;
        o2[q] += eta * g.area * gxy;
        o3[q] += eta * g.area * (gxx + 2.0 * gyy);
      }
    return;
  }
  // convection J_e[m][n] = |T| sum_a (sum_k (w_k . g_a) T3[m][k][n][a] + (w_c . g_a) T2[m][n][a])
  double wg[6][3];
  for (int k = 0; k < 6; ++k) {
    const int node = ep2[e * 6 + k];
    const double ws = rho ? rho[node] : wscale;  // rho v at the P2 nodes
    const double wx = ws * vel[node], wy = ws * vel[n2 + node];
    for (int a = 0; a < 3; ++a) wg[k][a] = wx * g.gx[a] + wy * g.gy[a];
  }
  double cx, cy;
  mu_const(mg, ep1 + size_t(e) * 3, g, cx, cy);
  double cg[3];
  for (int a = 0; a < 3; ++a) cg[a] = cx * g.gx[a] + cy * g.gy[a];
  for (int m = 0; m < 6; ++m)
    for (int n = 0; n < 6; ++n) {
      double acc = 0.0;
      for (int a = 0; a < 3; ++a) {
        double t = cg[a] * tb.T2[(m * 6 + n) * 3 + a];
        for (int k = 0; k < 6; ++k) t += wg[k][a] * tb.T3[((m * 6 + k) * 6 + n) * 3 + a];
        acc += t;
      }
      o0[slot[m * 6 + n]] += g.area * acc;
    }
}

__global__ __launch_bounds__(BS) void k_assemble_b(int e0, int e1, const int* __restrict__ etype,
                                                   const int* __restrict__ eslot, double h,
                                                   DP2Tables tb, double* __restrict__ out) {
  const int e = e0 + blockIdx.x * BS + threadIdx.x;
  if (e >= e1) return;
  const ElemGeo g = elem_geo(etype[e], h);
  const int* slot = eslot + size_t(e) * 36;  // [q][c*6 + k]
  for (int q = 0; q < 3; ++q)
    for (int k = 0; k < 6; ++k) {
      double bx = 0.0, by = 0.0;
      for (int a = 0; a < 3; ++a) {
        const double t = tb.TB[(q * 6 + k) * 3 + a];
        bx += g.gx[a] * t;
        by += g.gy[a] * t;
      }
      out[slot[q * 12 + k]] += -g.area * bx;
      out[slot[q * 12 + 6 + k]] += -g.area * by;
    }
}

__global__ __launch_bounds__(BS) void k_assemble_p1_conv(int e0, int e1, const int* __restrict__ ep1,
                                                         const int* __restrict__ ep2,
                                                         const int* __restrict__ etype,
                                                         const int* __restrict__ eslot, double h,
                                                         const double* __restrict__ vel,
                                                         double wscale, int64_t n2, MuGrad mg,
                                                         double* __restrict__ val,
                                                         const double* __restrict__ rho) {
  const int e = e0 + blockIdx.x * BS + threadIdx.x;
  if (e >= e1) return;
  const ElemGeo g = elem_geo(etype[e], h);
  double vx[6], vy[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const int node = ep2[e * 6 + k];
    const double ws = rho ? rho[node] : wscale;  // rho v at the P2 nodes
    vx[k] = ws * vel[node];
    vy[k] = ws * vel[n2 + node];
  }
  double cx, cy;
  mu_const(mg, ep1 + size_t(e) * 3, g, cx, cy);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    // int w lambda_a / |T| = sum_k W[k][a] w_k + w_c / 3
    double Vx = cx / 3.0, Vy = cy / 3.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      const double wk = w_p2p1(k, a);
      Vx += wk * vx[k];
      Vy += wk * vy[k];
    }
#pragma unroll
    for (int b = 0; b < 3; ++b) val[eslot[e * 9 + a * 3 + b]] += g.area * (Vx * g.gx[b] + Vy * g.gy[b]);
  }
}

__global__ __launch_bounds__(BS) void k_korteweg(int e0, int e1, const int* __restrict__ ep1,
                                                 const int* __restrict__ ep2,
                                                 const int* __restrict__ etype, double h,
                                                 DP2Tables tb, const double* __restrict__ php,
                                                 const double* __restrict__ phn,
                                                 const double* __restrict__ phs,
                                                 const double* __restrict__ Phi, KorBeta kb, int64_t n2,
                                                 double* __restrict__ out) {
  const int e = e0 + blockIdx.x * BS + threadIdx.x;
  if (e >= e1) return;
  const ElemGeo g = elem_geo(etype[e], h);
  const int* v = ep1 + size_t(e) * 3;
  double gp[2] = {0, 0}, gn[2] = {0, 0}, gs[2] = {0, 0}, gv[2] = {0, 0};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    gp[0] += php[v[a]] * g.gx[a];
    gp[1] += php[v[a]] * g.gy[a];
    gn[0] += phn[v[a]] * g.gx[a];
    gn[1] += phn[v[a]] * g.gy[a];
    if (phs) {
      gs[0] += phs[v[a]] * g.gx[a];
      gs[1] += phs[v[a]] * g.gy[a];
    }
    gv[0] += Phi[v[a]] * g.gx[a];
    gv[1] += Phi[v[a]] * g.gy[a];
  }
  // the eliminated phase, one minus the given ones (solvent, or air when the
  // solvent is given)
  const double ge[2] = {-gp[0] - gn[0] - gs[0], -gp[1] - gn[1] - gs[1]};
  double G[2][2];
  for (int c = 0; c < 2; ++c)
    for (int d = 0; d < 2; ++d) {
      double t = kb.b[0] * gp[c] * gp[d] + kb.b[1] * gn[c] * gn[d] + kb.bv * gv[c] * gv[d];
      if (phs) t += kb.b[2] * gs[c] * gs[d] + kb.b[3] * ge[c] * ge[d];
      else t += kb.b[2] * ge[c] * ge[d];
      G[c][d] = t;
    }
  for (int k = 0; k < 6; ++k) {
    const int node = ep2[e * 6 + k];
    for (int c = 0; c < 2; ++c) {
      double acc = 0.0;
      for (int a = 0; a < 3; ++a) acc += tb.TI[k * 3 + a] * (g.gx[a] * G[c][0] + g.gy[a] * G[c][1]);
      out[c * n2 + node] += g.area * acc;
    }
  }
}

__global__ __launch_bounds__(BS) void k_form_ns(int64_t n, const int8_t* __restrict__ kind,
                                                const int* __restrict__ src, double cm,
                                                const double* __restrict__ Mv,
                                                const double* __restrict__ J,
                                                const double* __restrict__ Kxx,
                                                const double* __restrict__ Kxy,
                                                const double* __restrict__ Kyx,
                                                const double* __restrict__ Kyy,
                                                const double* __restrict__ B,
                                                double* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * BS + threadIdx.x;
  if (i >= n) return;
  const int k = kind[i], s = src[i];
  double v = 0.0;
  if (k == 0) v = cm * Mv[s] + J[s] + Kxx[s];
  else if (k == 1) v = Kxy[s];
  else if (k == 2) v = Kyx[s];
  else if (k == 3) v = cm * Mv[s] + J[s] + Kyy[s];
  else if (k == 4) v = B[s];
  out[i] = v;
}

__global__ __launch_bounds__(BS) void k_rhs_ternary(int n, int side, const int* __restrict__ col,
                                                    const double* __restrict__ Mv,
                                                    const double* __restrict__ php,
                                                    const double* __restrict__ phn,
                                                    const double* __restrict__ Phi, double c_mu,
                                                    double c_ac, PotCoef pc, double* __restrict__ rhs_p,
                                                    double* __restrict__ rhs_n,
                                                    double* __restrict__ rhs_ac,
                                                    double* __restrict__ fs_out) {
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int row = blk * BS + threadIdx.x;
  if (row >= n) return;
  const size_t base = size_t(row >> 6) * (64 * W7) + (row & 63);
  double s_p = 0, s_n = 0, s_dp = 0, s_dn = 0, s_P = 0, s_fv = 0;
  int cc[W7];
  row_cols7(row, side, col, base, cc);
#pragma unroll
  for (int k = 0; k < W7; ++k) {
    const int j = cc[k];
    const double m = Mv[base + k * 64];
    const double a = php[j], b = phn[j], P = Phi[j];
    double dp, dn, fv, fs;
    ternary_terms(a, b, P, pc, dp, dn, fv, fs);
    s_p += m * a;
    s_n += m * b;
    s_dp += m * dp;
    s_dn += m * dn;
    s_P += m * P;
    s_fv += m * fv;
  }
  rhs_p[row] = s_p;
  rhs_p[n + row] = c_mu * s_dp;
  rhs_n[row] = s_n;
  rhs_n[n + row] = c_mu * s_dn;
  rhs_ac[row] = s_P + c_ac * s_fv;
  double dp, dn, fv, fs;
  ternary_terms(php[row], phn[row], Phi[row], pc, dp, dn, fv, fs);
  fs_out[row] = fs;
}

// Quaternary right-hand sides: per CH phase i (polymer, NFA, solvent) the
// blocks M phi_i and c_mu[i] M d_i (d_i the derivative along the air's
// elimination), the AC block M Phi + c_ac M f_v, and the unreduced air
// derivative f_a at each vertex (closure of mu_a).
__global__ __launch_bounds__(BS) void k_rhs_quaternary(int n, int side, const int* __restrict__ col,
                                                       const double* __restrict__ Mv,
                                                       const double* __restrict__ php,
                                                       const double* __restrict__ phn,
                                                       const double* __restrict__ phs,
                                                       const double* __restrict__ Phi, Coef3 c_mu,
                                                       double c_ac, double* __restrict__ rhs_ch,
                                                       double* __restrict__ rhs_ac,
                                                       double* __restrict__ fa_out) {
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int row = blk * BS + threadIdx.x;
  if (row >= n) return;
  const size_t base = size_t(row >> 6) * (64 * W7) + (row & 63);
  double s_p = 0, s_n = 0, s_s = 0, s_dp = 0, s_dn = 0, s_ds = 0, s_P = 0, s_fv = 0;
  int cc[W7];
  row_cols7(row, side, col, base, cc);
#pragma unroll
  for (int k = 0; k < W7; ++k) {
    const int j = cc[k];
    const double m = Mv[base + k * 64];
    const double a = php[j], b = phn[j], c = phs[j], P = Phi[j];
    double dp, dn, ds, fa, fv;
    quaternary_terms(a, b, c, P, dp, dn, ds, fa, fv);
    s_p += m * a;
    s_n += m * b;
    s_s += m * c;
    s_dp += m * dp;
    s_dn += m * dn;
    s_ds += m * ds;
    s_P += m * P;
    s_fv += m * fv;
  }
  const int64_t N = n;
  rhs_ch[row] = s_p;
  rhs_ch[N + row] = c_mu.v[0] * s_dp;
  rhs_ch[2 * N + row] = s_n;
  rhs_ch[3 * N + row] = c_mu.v[1] * s_dn;
  rhs_ch[4 * N + row] = s_s;
  rhs_ch[5 * N + row] = c_mu.v[2] * s_ds;
  rhs_ac[row] = s_P + c_ac * s_fv;
  double dp, dn, ds, fa, fv;
  quaternary_terms(php[row], phn[row], phs[row], Phi[row], dp, dn, ds, fa, fv);
  fa_out[row] = fa;
}

template <typename T>
__global__ __launch_bounds__(BS) void k_sum_partial(int64_t n, const T* __restrict__ x,
                                                    double* __restrict__ part) {
  __shared__ double sh[4];
  double acc = 0.0;
  const int64_t stride = int64_t(gridDim.x) * BS;
  for (int64_t r = int64_t(blockIdx.x) * BS + threadIdx.x; r < n; r += stride) acc += double(x[r]);
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// Per-block partials of sum_i w_i x_i.
__global__ __launch_bounds__(BS) void k_wsum_partial(int64_t n, const double* __restrict__ w,
                                                     const double* __restrict__ x, double* __restrict__ part) {
  __shared__ double sh[4];
  double acc = 0.0;
  const int64_t stride = int64_t(gridDim.x) * BS;
  for (int64_t r = int64_t(blockIdx.x) * BS + threadIdx.x; r < n; r += stride) acc += w[r] * x[r];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

template <typename T>
__global__ __launch_bounds__(BS) void k_sub_mean(int64_t n, int nblk, const double* __restrict__ part,
                                                 double total, T* __restrict__ x) {
  __shared__ double sh[4];
  __shared__ double mean;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += BS) s += part[b];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) mean = s / total;
  __syncthreads();
  const int64_t i = int64_t(blockIdx.x) * BS + threadIdx.x;
  if (i < n) x[i] = T(double(x[i]) - mean);
}

__global__ __launch_bounds__(BS) void k_one_minus_sum(int64_t n, const double* __restrict__ a,
                                                      const double* __restrict__ b,
                                                      double* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * BS + threadIdx.x;
  if (i < n) out[i] = 1.0 - a[i] - b[i];
}

__global__ __launch_bounds__(BS) void k_axpy_into(int64_t n, double a, const double* __restrict__ x,
                                                  const double* __restrict__ y,
                                                  double* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * BS + threadIdx.x;
  if (i < n) out[i] = a * x[i] + y[i];
}

}  // namespace

// ================================================================== launchers

// Launch, with the dispatch's own start/stop timestamps into ev when given.
#define LAUNCH_EV(ev, kern, grid, block, shm, st, ...)                                           \
  do {                                                                                           \
    if ((ev).start)                                                                              \
      hipExtLaunchKernelGGL(kern, grid, block, shm, st, (ev).start, (ev).stop, 0, __VA_ARGS__); \
    else                                                                                         \
      hipLaunchKernelGGL(kern, grid, block, shm, st, __VA_ARGS__);                               \
  } while (0)

template <typename T, typename TV>
void spmv(const DSell& A, const TV* val, const T* x, T* y, T alpha, T beta, hipStream_t s) {
  if (A.uniform && A.width == W7) {
    hipLaunchKernelGGL((k_stencil<T, TV, ST_SPMV, W7>), dim3(ceil_div(A.nrows, BS)), dim3(BS), 0, s,
                       A.nrows, A.side, A.col, val, x, (const T*)nullptr, (const T*)nullptr, (T*)nullptr,
                       alpha, beta, y);
  } else if (A.uniform && A.width == W15) {
    hipLaunchKernelGGL((k_stencil<T, TV, ST_SPMV, W15>), dim3(ceil_div(A.nrows, BS)), dim3(BS), 0, s,
                       A.nrows, A.cube, A.col, val, x, (const T*)nullptr, (const T*)nullptr, (T*)nullptr,
                       alpha, beta, y);
  } else {
    const int npos = A.nslices * 64;
    hipLaunchKernelGGL((k_spmv_sell<T, TV>), dim3(ceil_div(npos, BS)), dim3(BS), 0, s, A.nslices,
                       A.nrows, A.slice_ptr, A.slice_w, A.col, val, A.uniform ? nullptr : A.perm, x,
                       y, alpha, beta);
  }
}

template <typename T, typename TV>
void stencil(const DSell& A, const TV* val, int mode, const T* x, const T* b, const T* dinv, T* d,
             T c1, T c2, T* y, hipStream_t s, LaunchEv ev) {
  const dim3 g(ceil_div(A.nrows, BS)), blk(BS);
  if (A.width == W15) {
    if (mode == ST_RESID)
      LAUNCH_EV(ev, (k_stencil<T, TV, ST_RESID, W15>), g, blk, 0, s, A.nrows, A.cube, A.col, val, x, b, dinv,
                d, c1, c2, y);
    else
      LAUNCH_EV(ev, (k_stencil<T, TV, ST_CHEB, W15>), g, blk, 0, s, A.nrows, A.cube, A.col, val, x, b, dinv,
                d, c1, c2, y);
    return;
  }
  if (mode == ST_RESID)
    LAUNCH_EV(ev, (k_stencil<T, TV, ST_RESID, W7>), g, blk, 0, s, A.nrows, A.side, A.col, val, x, b, dinv,
              d, c1, c2, y);
  else
    LAUNCH_EV(ev, (k_stencil<T, TV, ST_CHEB, W7>), g, blk, 0, s, A.nrows, A.side, A.col, val, x, b, dinv,
              d, c1, c2, y);
}

template <typename T>
void cheb0(int n, const T* dinv, const T* b, T c2, T* d, T* x, hipStream_t s) {
  hipLaunchKernelGGL((k_cheb0<T>), dim3(ceil_div(n, BS)), dim3(BS), 0, s, n, dinv, b, c2, d, x);
}

template <typename T, typename TV>
void cheb01(const DSell& A, const TV* val, const T* b, const T* dinv, T c20, T c11, T c21, T* d, T* y,
            hipStream_t s) {
  hipLaunchKernelGGL((k_cheb01<T, TV>), dim3(ceil_div(A.nrows, BS)), dim3(BS), 0, s, A.nrows, A.side, val,
                     b, dinv, c20, c11, c21, d, y);
}

template <typename T, typename TV>
void pcheb(const DSell& A, const TV* val, const T* x, const T* e, const T* b, const T* dinv, T c2, T* d,
           T* y, hipStream_t s) {
  hipLaunchKernelGGL((k_pcheb<T, TV>), dim3(ceil_div(A.nrows, BS)), dim3(BS), 0, s, A.nrows, A.side, val, x,
                     e, b, dinv, c2, d, y);
}

template <typename T, typename TV>
void coarse_cheb(const DSell& A, const TV* val, const T* dinv, const T* b, const ChebCoef<T>& cc,
                 T* x, hipStream_t s) {
  if (A.width == W15)
    hipLaunchKernelGGL((k_coarse_cheb<T, TV, W15>), dim3(1), dim3(1024), 0, s, A.nrows, A.cube, A.col, val,
                       dinv, b, cc, x);
  else
    hipLaunchKernelGGL((k_coarse_cheb<T, TV, W7>), dim3(1), dim3(1024), 0, s, A.nrows, A.side, A.col, val,
                       dinv, b, cc, x);
}

template <typename T>
bool tile_fits(int mode, int side, int steps) {
  const int H = tile_halo(mode, steps);
  const int TT = tile_side<T>(side);
  const int hmax = TT == 64 ? TileCfg<64>::HMAX : (TT == 32 ? TileCfg<32>::HMAX : TileCfg<16>::HMAX);
  if (steps < (mode == TILE_UP || mode == TILE_UPM ? 0 : 1) || steps > TILE_MAXSTEPS || H < 0 || H > hmax)
    return false;
  if (side < TT + hmax) return false;  // one wrap reaches every halo row
  return mode != TILE_DOWN || side % 2 == 0;
}

template <typename T, int TT>
void vtile_tt(int mode, const TileArgs<T>& a, hipStream_t s, LaunchEv ev) {
  const int nt = (a.side + TT - 1) / TT;
  const dim3 g(nt * nt), b(TileCfg<TT>::NTH);
  if (mode == TILE_ZERO) LAUNCH_EV(ev, (k_vtile<T, TILE_ZERO, TT>), g, b, 0, s, a);
  else if (mode == TILE_DOWN) LAUNCH_EV(ev, (k_vtile<T, TILE_DOWN, TT>), g, b, 0, s, a);
  else if (mode == TILE_UPM) LAUNCH_EV(ev, (k_vtile<T, TILE_UPM, TT>), g, b, 0, s, a);
  else LAUNCH_EV(ev, (k_vtile<T, TILE_UP, TT>), g, b, 0, s, a);
}

// The pipelined 64 x 64 pass for the modes, sweep counts and FP64 boundary
// combinations of the mixed-precision cycles; false for the others.
template <int MODE, int S, int IO>
bool vpipe_io(const TileArgs<float>& a, hipStream_t s, LaunchEv ev) {
  const int nt = (a.side + 63) / 64;
  LAUNCH_EV(ev, (k_vtile_pipe<float, MODE, S, IO>), dim3(nt * nt), dim3(1024), 0, s, a);
  return true;
}

template <int MODE, int S>
bool vpipe_s(const TileArgs<float>& a, hipStream_t s, LaunchEv ev) {
  const int io = (a.b64 ? 1 : 0) | (a.x64 ? 2 : 0);
  if (io == 0) return vpipe_io<MODE, S, 0>(a, s, ev);
  if constexpr (MODE == TILE_ZERO) {
    if (io == 3) return vpipe_io<MODE, S, 3>(a, s, ev);
  } else if constexpr (MODE == TILE_UP) {
    if (io == 2) return vpipe_io<MODE, S, 2>(a, s, ev);
  } else {
    if (io == 1) return vpipe_io<MODE, S, 1>(a, s, ev);
  }
  return false;
}

template <int MODE>
bool vpipe_mode(const TileArgs<float>& a, hipStream_t s, LaunchEv ev) {
  constexpr bool UPLIKE = MODE == TILE_UP || MODE == TILE_UPM;
  const int S = UPLIKE ? a.steps : a.steps - 1;
  // the halo fits the 64 x 64 tiles' (tile_fits) and the sweeps are few
  switch (S) {
    case 0: return vpipe_s<MODE, 0>(a, s, ev);
    case 1: return vpipe_s<MODE, 1>(a, s, ev);
    case 2: return tile_halo(MODE, UPLIKE ? 2 : 3) <= TileCfg<64>::HMAX && vpipe_s<MODE, 2>(a, s, ev);
    case 3: return tile_halo(MODE, UPLIKE ? 3 : 4) <= TileCfg<64>::HMAX && vpipe_s<MODE, 3>(a, s, ev);
    default: return false;
  }
}

bool vtile_pipe(int mode, const TileArgs<float>& a, hipStream_t s, LaunchEv ev) {
  if (mode == TILE_ZERO) return vpipe_mode<TILE_ZERO>(a, s, ev);
  if (mode == TILE_DOWN) return vpipe_mode<TILE_DOWN>(a, s, ev);
  if (mode == TILE_UP) return vpipe_mode<TILE_UP>(a, s, ev);
  return vpipe_mode<TILE_UPM>(a, s, ev);
}

template <typename T>
void vtile(int mode, const TileArgs<T>& a, hipStream_t s, LaunchEv ev) {
  const int tt = tile_side<T>(a.side);
  if constexpr (sizeof(T) == 4) {
    if (tt == 64) {
      if (!vtile_pipe(mode, a, s, ev)) vtile_tt<T, 64>(mode, a, s, ev);
      return;
    }
  }
  if (tt == 16) vtile_tt<T, 16>(mode, a, s, ev);
  else vtile_tt<T, 32>(mode, a, s, ev);
}

bool tile2_cut_fits(int side, int post, int steps) {
  const int scc = side / 4, Q = post;
  const int wc = T2_TC + 2 * ((Q + 1) / 2 + 1 + Q);
  const int w = std::max(t2_cut_side(wc, 0, steps), t2_cut_side(wc, 1, steps));
  // one node per thread in buffers of T2_WFU^2; one wrap reaches every row
  return steps >= 1 && steps <= TILE_MAXSTEPS && w * w <= 1024 && w * w <= T2_WFU * T2_WFU && w <= scc;
}

bool tile2_fits(int side, int pre, int post) {
  // both levels even (the coarse one restricts again); one wrap reaches
  // every halo row of both regions
  return side % 4 == 0 && side >= 64 && pre >= 1 && pre <= T2_PMAX && post >= 0 && post <= T2_PMAX;
}

template <typename T>
void vdown2(const Tile2Args<T>& a, hipStream_t s) {
  const int nt = (a.side + T2_TT - 1) / T2_TT;
  hipLaunchKernelGGL((k_vdown2<T>), dim3(nt * nt), dim3(1024), 0, s, a);
}

template <typename T>
void vup2(const Tile2Args<T>& a, hipStream_t s) {
  const int nt = (a.side + T2_TT - 1) / T2_TT;
  hipLaunchKernelGGL((k_vup2<T>), dim3(nt * nt), dim3(1024), 0, s, a);
}

bool btile_fits(int mode, int side, int steps) {
  const int H = tile_halo(mode, steps);
  if (steps < (mode == TILE_UP || mode == TILE_UPM ? 0 : 1) || steps > TILE_MAXSTEPS || H < 0 ||
      H > TileCfg<32>::HMAX)
    return false;
  if (side < 32 + TileCfg<32>::HMAX) return false;
  return mode != TILE_DOWN || side % 2 == 0;
}

int btile_count(int side) {
  const int nt = (side + 31) / 32;
  return nt * nt;
}

template <typename T>
void bvtile(int mode, int ntiles, const BTileLaunch<T>& a, hipStream_t s, int wl_grid, int* wl_ctr) {
  if (ntiles <= 0) return;
  const dim3 b(TILE_THREADS);
  if (wl_grid > 0 && wl_ctr) {
    // work-list launch: at most wl_grid workgroups, at least 8 (one per XCD)
    int g = std::min(ntiles, wl_grid);
    g = std::max(8, (g + 7) / 8 * 8);
    if (mode == TILE_ZERO) hipLaunchKernelGGL((k_bvtile_wl<T, TILE_ZERO, 32>), dim3(g), b, 0, s, a, ntiles, wl_ctr);
    else if (mode == TILE_DOWN) hipLaunchKernelGGL((k_bvtile_wl<T, TILE_DOWN, 32>), dim3(g), b, 0, s, a, ntiles, wl_ctr);
    else if (mode == TILE_UPM) hipLaunchKernelGGL((k_bvtile_wl<T, TILE_UPM, 32>), dim3(g), b, 0, s, a, ntiles, wl_ctr);
    else hipLaunchKernelGGL((k_bvtile_wl<T, TILE_UP, 32>), dim3(g), b, 0, s, a, ntiles, wl_ctr);
    return;
  }
  const dim3 g(ntiles);
  if (mode == TILE_ZERO) hipLaunchKernelGGL((k_bvtile<T, TILE_ZERO, 32>), g, b, 0, s, a);
  else if (mode == TILE_DOWN) hipLaunchKernelGGL((k_bvtile<T, TILE_DOWN, 32>), g, b, 0, s, a);
  else if (mode == TILE_UPM) hipLaunchKernelGGL((k_bvtile<T, TILE_UPM, 32>), g, b, 0, s, a);
  else hipLaunchKernelGGL((k_bvtile<T, TILE_UP, 32>), g, b, 0, s, a);
}

template <typename T>
bool tail_fits(const int* sides, int nlev) {
  if (nlev < 1 || nlev > TAIL_MAXLEV) return false;
  size_t rows = 0;
  for (int t = 0; t < nlev; ++t) {
    if (sides[t] < 3) return false;
    if (t + 1 < nlev && (sides[t] % 2 != 0 || sides[t + 1] != sides[t] / 2)) return false;
    rows += size_t(sides[t]) * sides[t];
  }
  return size_t(sides[0]) * sides[0] <= size_t(TailCfg<T>::RPT) * TAIL_THREADS &&
         3 * rows * sizeof(T) <= TAIL_LDS;
}

template <typename T>
void bvtail(int n, const TailArgs<T>* list, const int* idx, const int* act, const T* bbase, T* xbase,
            hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL((k_bvtail<T, TailCfg<T>::RPT>), dim3(n), dim3(TAIL_THREADS), 0, s, list, idx, act,
                     bbase, xbase);
}

template <typename T>
void vtail(const TailArgs<T>& a, hipStream_t s) {
  hipLaunchKernelGGL((k_vtail<T, TailCfg<T>::RPT>), dim3(1), dim3(TAIL_THREADS), 0, s, a);
}

template <typename T, typename TV>
void ch_block(const DSell& A, const TV* L, const TV* K, const TV* M, T c12, T c22, const T* x,
              T alpha, T beta, T* y, hipStream_t s, LaunchEv ev, const T* yin) {
  const dim3 g(ceil_div(A.nrows, BS)), blk(BS);
  if (A.width == W15) {
    if (L == M)
      LAUNCH_EV(ev, (k_ch_block<T, TV, true, W15>), g, blk, 0, s, A.nrows, A.cube, A.col, L, K, M, c12, c22,
                x, alpha, beta, y, yin);
    else
      LAUNCH_EV(ev, (k_ch_block<T, TV, false, W15>), g, blk, 0, s, A.nrows, A.cube, A.col, L, K, M, c12, c22,
                x, alpha, beta, y, yin);
    return;
  }
  if (L == M)
    LAUNCH_EV(ev, (k_ch_block<T, TV, true, W7>), g, blk, 0, s, A.nrows, A.side, A.col, L, K, M, c12, c22, x,
              alpha, beta, y, yin);
  else
    LAUNCH_EV(ev, (k_ch_block<T, TV, false, W7>), g, blk, 0, s, A.nrows, A.side, A.col, L, K, M, c12, c22, x,
              alpha, beta, y, yin);
}

template <typename T>
void axpby(int64_t n, T a, const T* x, T b, T* y, hipStream_t s) {
  hipLaunchKernelGGL((k_axpby<T>), dim3(ceil_div(n, BS)), dim3(BS), 0, s, n, a, x, b, y);
}

template <typename TI, typename TO>
void convert(int64_t n, const TI* x, TO* y, hipStream_t s) {
  hipLaunchKernelGGL((k_convert<TI, TO>), dim3(ceil_div(n, BS)), dim3(BS), 0, s, n, x, y);
}

void convert_out(int64_t n, const float* x, const double* inv, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_convert_out, dim3(ceil_div(n, BS)), dim3(BS), 0, s, n, x, inv, y);
}

void convert_scaled(int64_t n, double* x, const double* inv, float* y, hipStream_t s) {
  hipLaunchKernelGGL(k_convert_scaled, dim3(ceil_div(n, BS)), dim3(BS), 0, s, n, x, inv, y);
}

void scale_by_inv(int64_t n, const double* x, const double* inv, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_by_inv, dim3(ceil_div(n, BS)), dim3(BS), 0, s, n, x, inv, y);
}

int reduce_blocks(int64_t n) {
  const int64_t b = (n + 4 * BS - 1) / (4 * BS);
  return int(b < 1 ? 1 : (b > MAXRED ? MAXRED : b));
}

int dcgs_dot_blocks(int64_t n) { return reduce_blocks(n); }

template <int KK, bool LAST>
static void launch_dots(int64_t n, const double* V, int64_t ld, int j, int g0, const DcgsState& st,
                        hipStream_t s, LaunchEv ev) {
  LAUNCH_EV(ev, (k_dcgs_dots<KK, LAST>), dim3(dcgs_dot_blocks(n)), dim3(BS), 0, s, n, V, ld, j, g0, st.part,
            st.vscale);
}

template <bool LAST>
static void launch_dots_kk(int kk, int64_t n, const double* V, int64_t ld, int j, int g0,
                           const DcgsState& st, hipStream_t s, LaunchEv ev) {
  switch (kk) {
#define CHNS_DOTS_CASE(K) \
  case K: launch_dots<K, LAST>(n, V, ld, j, g0, st, s, ev); break;
    CHNS_DOTS_CASE(0) CHNS_DOTS_CASE(1) CHNS_DOTS_CASE(2) CHNS_DOTS_CASE(3) CHNS_DOTS_CASE(4)
    CHNS_DOTS_CASE(5) CHNS_DOTS_CASE(6) CHNS_DOTS_CASE(7) CHNS_DOTS_CASE(8) CHNS_DOTS_CASE(9)
    CHNS_DOTS_CASE(10) CHNS_DOTS_CASE(11) CHNS_DOTS_CASE(12) CHNS_DOTS_CASE(13) CHNS_DOTS_CASE(14)
    CHNS_DOTS_CASE(15) CHNS_DOTS_CASE(16)
#undef CHNS_DOTS_CASE
    default: break;
  }
}

// Full groups of DG vectors, then the remainder group with vt . vt, vt . w,
// w . w (one launch when j < DG), then the slot sums.
void dcgs_dots(int64_t n, const double* V, int64_t ld, int j, const DcgsState& st, hipStream_t s,
               LaunchEv ev) {
  const int full = j / DG, rem = j - full * DG;
  for (int g = 0; g < full; ++g)
    launch_dots_kk<false>(DG, n, V, ld, j, g * DG, st, s, g == 0 ? ev : LaunchEv{});
  launch_dots_kk<true>(rem, n, V, ld, j, full * DG, st, s, full == 0 ? ev : LaunchEv{});
  hipLaunchKernelGGL(k_slot_reduce, dim3(2 * j + 3), dim3(BS), 0, s, dcgs_dot_blocks(n), st.part, st.red);
}

template <bool LM, int W>
static void launch_ch_dots(int j, int N, const DSell& A, const double* Lv, const double* Kv, const double* Mv,
                           double c12, double c22, const double* z, double* V, int64_t ld, const DcgsState& st,
                           hipStream_t s, LaunchEv ev) {
  const dim3 g(dcgs_dot_blocks(2 * int64_t(N))), b(BS);
  const int side = W == W15 ? A.cube : A.side;  // computed columns
  switch (j) {
#define CHNS_CHD_CASE(K)                                                                                 \
  case K:                                                                                                 \
    LAUNCH_EV(ev, (k_ch_dots<K, LM, W>), g, b, 0, s, N, side, A.col, Lv, Kv, Mv, c12, c22, z, V, ld, st.part, \
              st.vscale);                                                                                 \
    break;
    CHNS_CHD_CASE(0) CHNS_CHD_CASE(1) CHNS_CHD_CASE(2) CHNS_CHD_CASE(3) CHNS_CHD_CASE(4) CHNS_CHD_CASE(5)
    CHNS_CHD_CASE(6) CHNS_CHD_CASE(7) CHNS_CHD_CASE(8) CHNS_CHD_CASE(9) CHNS_CHD_CASE(10) CHNS_CHD_CASE(11)
    CHNS_CHD_CASE(12) CHNS_CHD_CASE(13) CHNS_CHD_CASE(14) CHNS_CHD_CASE(15)
#undef CHNS_CHD_CASE
    default: break;
  }
}

bool ch_dots_fits(int j) { return j >= 0 && j < DG; }

void ch_dcgs_dots(const DSell& A, const double* Lv, const double* Kv, const double* Mv, double c12, double c22,
                  const double* z, double* V, int64_t ld, int j, const DcgsState& st, hipStream_t s, LaunchEv ev) {
  const int N = A.nrows;
  if (A.width == W15) {
    if (Lv == Mv) launch_ch_dots<true, W15>(j, N, A, Lv, Kv, Mv, c12, c22, z, V, ld, st, s, ev);
    else launch_ch_dots<false, W15>(j, N, A, Lv, Kv, Mv, c12, c22, z, V, ld, st, s, ev);
  } else {
    if (Lv == Mv) launch_ch_dots<true, W7>(j, N, A, Lv, Kv, Mv, c12, c22, z, V, ld, st, s, ev);
    else launch_ch_dots<false, W7>(j, N, A, Lv, Kv, Mv, c12, c22, z, V, ld, st, s, ev);
  }
  hipLaunchKernelGGL(k_slot_reduce, dim3(2 * j + 3), dim3(BS), 0, s, dcgs_dot_blocks(2 * int64_t(N)), st.part,
                     st.red);
}

void dcgs_update(int64_t n, double* V, int64_t ld, int j, const DcgsState& st, double* host, double tag,
                 hipStream_t s, LaunchEv ev) {
  LAUNCH_EV(ev, k_dcgs_update, dim3(reduce_blocks(n)), dim3(BS), 0, s, n, V, ld, j, st.m, st.red, st.H,
            st.nrm_part, st.vscale);
  hipLaunchKernelGGL(k_dcgs_finish, dim3(1), dim3(BS), 0, s, reduce_blocks(n), st.nrm_part, j, st.m, st.H,
                     st.HR, st.cs, st.sn, st.g, st.gp, st.scal, host, tag);
}

void lsq_solve(int k, int m, const double* H, const double* g, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_lsq_solve, dim3(1), dim3(BS), 0, s, k, m, H, g, y);
}

void xupdate(int64_t n, const double* Z, int64_t ldz, int k, const double* y, double* x,
             hipStream_t s) {
  hipLaunchKernelGGL(k_xupdate, dim3(ceil_div(n, BS)), dim3(BS), 0, s, n, Z, ldz, k, y, x);
}

void norm_partial(int64_t n, const double* w, double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_norm_partial, dim3(reduce_blocks(n)), dim3(BS), 0, s, n, w, part);
}

void norm_finish(int nblk, const double* part, double* scal, double* g, int m, hipStream_t s, double* host,
                 double tag) {
  hipLaunchKernelGGL(k_norm_finish, dim3(1), dim3(64), 0, s, nblk, part, scal, g, m, host, tag);
}

// Kuhn tetrahedron of type t: vertices 0, h e_a, h (e_a + e_b), h (1, 1, 1)
// with (a, b, c) the t-th ordering of the axes; its barycentric gradients are
// the rows of the inverse of the edge matrix [v1 v2 v3] (columns), the first
// one minus their sum.
__global__ __launch_bounds__(BS) void k_assemble_p1_tet(int kind, int e0, int e1,
                                                        const int* __restrict__ etype,
                                                        const int* __restrict__ eslot16, double h,
                                                        double* __restrict__ val) {
  const int e = e0 + blockIdx.x * BS + threadIdx.x;
  if (e >= e1) return;
  constexpr int ORD[6][2] = {{0, 1}, {0, 2}, {1, 0}, {1, 2}, {2, 0}, {2, 1}};
  const int t = etype[e], a = ORD[t][0], b = ORD[t][1];
  double E[3][3];  // E[r][c]: component r of edge vector c
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    E[r][0] = r == a ? h : 0.0;
    E[r][1] = (r == a || r == b) ? h : 0.0;
    E[r][2] = h;
  }
  const double det = E[0][0] * (E[1][1] * E[2][2] - E[1][2] * E[2][1]) -
                     E[0][1] * (E[1][0] * E[2][2] - E[1][2] * E[2][0]) +
                     E[0][2] * (E[1][0] * E[2][1] - E[1][1] * E[2][0]);
  const double vol = fabs(det) / 6.0;
  double loc[16];
  if (kind == 0) {
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int q = 0; q < 4; ++q) loc[p * 4 + q] = vol / 20.0 * (p == q ? 2.0 : 1.0);
  } else {
    // rows of E^{-1}: the cofactors of E transposed, over det
    double g[4][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int r1 = (c + 1) % 3, r2 = (c + 2) % 3, c1 = (r + 1) % 3, c2 = (r + 2) % 3;
        g[r + 1][c] = (E[r1][c1] * E[r2][c2] - E[r1][c2] * E[r2][c1]) / det;
      }
#pragma unroll
    for (int c = 0; c < 3; ++c) g[0][c] = -(g[1][c] + g[2][c] + g[3][c]);
#pragma unroll
    for (int p = 0; p < 4; ++p)
#pragma unroll
      for (int q = 0; q < 4; ++q) loc[p * 4 + q] = vol * (g[p][0] * g[q][0] + g[p][1] * g[q][1] + g[p][2] * g[q][2]);
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) val[eslot16[int64_t(e) * 16 + q]] += loc[q];
}

void assemble_p1_tet(int kind, int e0, int e1, const int* etype, const int* eslot16, double h, double* val,
                     hipStream_t s) {
  if (e1 <= e0) return;
  hipLaunchKernelGGL(k_assemble_p1_tet, dim3(ceil_div(e1 - e0, BS)), dim3(BS), 0, s, kind, e0, e1, etype,
                     eslot16, h, val);
}

void assemble_p1(int kind, int e0, int e1, const int* ep2, const int* etype, const int* eslot,
                 double h, const double* vel, int64_t n2, double* val, hipStream_t s, const double* rho) {
  if (e1 <= e0) return;
  hipLaunchKernelGGL(k_assemble_p1, dim3(ceil_div(e1 - e0, BS)), dim3(BS), 0, s, kind, e0, e1, ep2,
                     etype, eslot, h, vel, n2, val, rho);
}

void galerkin(int64_t nslots, const int* ptr, const int* src, const double* w, const double* fine,
              double* coarse, hipStream_t s) {
  hipLaunchKernelGGL(k_galerkin, dim3(ceil_div(nslots, BS)), dim3(BS), 0, s, nslots, ptr, src, w,
                     fine, coarse);
}

void combine(int64_t nslots, double a, const double* A, double b, const double* B, double c,
             const double* C, double* out64, float* out32, hipStream_t s) {
  hipLaunchKernelGGL(k_combine, dim3(ceil_div(nslots, BS)), dim3(BS), 0, s, nslots, a, A, b, B, c,
                     C, out64, out32);
}

void diag_inverse(int nrows, const int* diag, const double* val, double* d64, float* d32,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_diag_inverse, dim3(ceil_div(nrows, BS)), dim3(BS), 0, s, nrows, diag, val,
                     d64, d32);
}

void form_ops(int nlev, const FormLevel* tab, int64_t total, const FormCoef& k, bool conv, hipStream_t s) {
  if (total <= 0) return;
  hipLaunchKernelGGL(k_form_ops, dim3(ceil_div(total, BS)), dim3(BS), 0, s, nlev, tab, total, k, conv ? 1 : 0);
}

int diag_part_blocks(int64_t n) { return reduce_blocks(n); }

void diagnostics(const DSell& A, const double* M, const double* K, const double* p0, const double* p1,
                 const double* p2, const double* Phi, bool ternary, const KorBeta& kb, const PotCoef& pc,
                 double* part, double* out, hipStream_t s) {
  const int nblk = reduce_blocks(A.nrows);
  if (A.width == W15)
    hipLaunchKernelGGL(k_diag<W15>, dim3(nblk), dim3(BS), 0, s, A.nrows, A.cube, A.col, M, K, p0, p1, p2, Phi,
                       ternary ? 1 : 0, kb, pc, part);
  else
    hipLaunchKernelGGL(k_diag<W7>, dim3(nblk), dim3(BS), 0, s, A.nrows, A.side, A.col, M, K, p0, p1, p2, Phi,
                       ternary ? 1 : 0, kb, pc, part);
  hipLaunchKernelGGL(k_diag_finish, dim3(1), dim3(BS), 0, s, nblk, part, out);
}

__global__ __launch_bounds__(BS) void k_set_slots(int64_t n, const int* __restrict__ idx, double v,
                                                  double* __restrict__ a, float* __restrict__ a32) {
  const int64_t i = int64_t(blockIdx.x) * BS + threadIdx.x;
  if (i >= n) return;
  const int q = idx[i];
  a[q] = v;
  if (a32) a32[q] = float(v);
}

void set_slots(int64_t n, const int* idx, double v, double* a, float* a32, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_set_slots, dim3(ceil_div(n, BS)), dim3(BS), 0, s, n, idx, v, a, a32);
}

void rhs_quaternary(const DSell& A, const double* Mv, const double* php, const double* phn, const double* phs,
                    const double* Phi, const Coef3& c_mu, double c_ac, double* rhs_ch, double* rhs_ac,
                    double* fa, hipStream_t s) {
  hipLaunchKernelGGL(k_rhs_quaternary, dim3(ceil_div(A.nrows, BS)), dim3(BS), 0, s, A.nrows, A.side, A.col,
                     Mv, php, phn, phs, Phi, c_mu, c_ac, rhs_ch, rhs_ac, fa);
}

void rhs_binary(const DSell& A, const double* Mv, const double* phi, const double* Phi, double c_mu,
                double c_ac, const TopFlux& tf, double* rhs_ch, double* rhs_ac, hipStream_t s) {
  if (A.width == W15)
    hipLaunchKernelGGL(k_rhs_binary<W15>, dim3(ceil_div(A.nrows, BS)), dim3(BS), 0, s, A.nrows, A.cube, A.col,
                       Mv, phi, Phi, c_mu, c_ac, tf, rhs_ch, rhs_ac);
  else
    hipLaunchKernelGGL(k_rhs_binary<W7>, dim3(ceil_div(A.nrows, BS)), dim3(BS), 0, s, A.nrows, A.side, A.col,
                       Mv, phi, Phi, c_mu, c_ac, tf, rhs_ch, rhs_ac);
}

template <typename T, typename TV>
void sell_op(const DSell& A, const TV* val, int mode, const T* x, const T* b, const T* dinv, T* d,
             T c1, T c2, T* y, hipStream_t s) {
  const int npos = A.nslices * 64;
  const int* perm = A.uniform ? nullptr : A.perm;
  if (mode == ST_RESID)
    hipLaunchKernelGGL((k_sell_op<T, TV, ST_RESID>), dim3(ceil_div(npos, BS)), dim3(BS), 0, s,
                       A.nslices, A.nrows, A.slice_ptr, A.slice_w, A.col, val, perm, x, b, dinv, d,
                       c1, c2, y);
  else
    hipLaunchKernelGGL((k_sell_op<T, TV, ST_CHEB>), dim3(ceil_div(npos, BS)), dim3(BS), 0, s,
                       A.nslices, A.nrows, A.slice_ptr, A.slice_w, A.col, val, perm, x, b, dinv, d,
                       c1, c2, y);
}

void assemble_p2(int kind, int e0, int e1, const int* ep1, const int* ep2, const int* etype,
                 const int* eslot36, double h, DP2Tables tb, double eta, const double* vel,
                 double wscale, int64_t n2, MuGrad mg, double* const* out, hipStream_t s,
                 const double* rho) {
  if (e1 <= e0) return;
  hipLaunchKernelGGL(k_assemble_p2, dim3(ceil_div(e1 - e0, BS)), dim3(BS), 0, s, kind, e0, e1, ep1,
                     ep2, etype, eslot36, h, tb, eta, vel, wscale, n2, mg, out[0],
                     kind == 1 ? out[1] : nullptr, kind == 1 ? out[2] : nullptr,
                     kind == 1 ? out[3] : nullptr, rho);
}

void assemble_b(int e0, int e1, const int* etype, const int* eslotb, double h, DP2Tables tb,
                double* out, hipStream_t s) {
  if (e1 <= e0) return;
  hipLaunchKernelGGL(k_assemble_b, dim3(ceil_div(e1 - e0, BS)), dim3(BS), 0, s, e0, e1, etype,
                     eslotb, h, tb, out);
}

void assemble_p1_conv(int e0, int e1, const int* ep1, const int* ep2, const int* etype,
                      const int* eslot, double h, const double* vel, double wscale, int64_t n2,
                      MuGrad mg, double* val, hipStream_t s, const double* rho) {
  if (e1 <= e0) return;
  hipLaunchKernelGGL(k_assemble_p1_conv, dim3(ceil_div(e1 - e0, BS)), dim3(BS), 0, s, e0, e1, ep1,
                     ep2, etype, eslot, h, vel, wscale, n2, mg, val, rho);
}

// rho = rp phi_p + rn phi_n + rs (1 - phi_p - phi_n) at the vertices, and its
// P1 interpolant at the P2 nodes (vertices; horizontal, vertical and diagonal
// edge midpoints i + n j between (i,j) and (i+1,j), (i,j+1), (i+1,j+1)).
// box: the closed square ((n+1)^2 vertices, no wrap); the P2 ids of edges
// that do not exist (i = n for the horizontal and diagonal blocks, j = n for
// the vertical and diagonal ones) get 0 (no element reads them).
__global__ __launch_bounds__(BS) void k_density(int n, int box, const double* __restrict__ pp,
                                                const double* __restrict__ pn, double rp, double rn,
                                                double rs, double* __restrict__ rho1,
                                                double* __restrict__ rho2) {
  const int m = box ? n + 1 : n;  // vertices per side
  const int N = m * m;
  const int v = blockIdx.x * BS + threadIdx.x;
  if (v >= N) return;
  const int j = v / m, i = v - j * m;
  auto r = [&](int k) { return rp * pp[k] + rn * pn[k] + rs * (1.0 - pp[k] - pn[k]); };
  const double r0 = r(v);
  rho1[v] = r0;
  rho2[v] = r0;
  if (box) {
    const bool ie = i < n, je = j < n;
    rho2[N + v] = ie ? 0.5 * (r0 + r(v + 1)) : 0.0;
    rho2[2 * N + v] = je ? 0.5 * (r0 + r(v + m)) : 0.0;
    rho2[3 * N + v] = (ie && je) ? 0.5 * (r0 + r(v + m + 1)) : 0.0;
    return;
  }
  const int i1 = i + 1 == n ? 0 : i + 1, j1 = j + 1 == n ? 0 : j + 1;
  rho2[N + v] = 0.5 * (r0 + r(i1 + n * j));
  rho2[2 * N + v] = 0.5 * (r0 + r(i + n * j1));
  rho2[3 * N + v] = 0.5 * (r0 + r(i1 + n * j1));
}

__global__ __launch_bounds__(BS) void k_fill(int64_t n, double v, double* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * BS + threadIdx.x;
  if (i < n) out[i] = v;
}

void fill(int64_t n, double v, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(ceil_div(n, BS)), dim3(BS), 0, s, n, v, out);
}

void density_fields(int n, bool box, const double* pp, const double* pn, const double* rpure, double* rho1,
                    double* rho2, hipStream_t s) {
  const int m = box ? n + 1 : n;
  hipLaunchKernelGGL(k_density, dim3(ceil_div(m * m, BS)), dim3(BS), 0, s, n, box ? 1 : 0, pp, pn, rpure[0],
                     rpure[1], rpure[2], rho1, rho2);
}

// ||v - w||_2 and ||v||_2 into out[0..1] (fixed grid, deterministic order).
constexpr int DIFF_NBLK = 256;
__global__ __launch_bounds__(BS) void k_diff_norms(int64_t n, const double* __restrict__ v,
                                                   const double* __restrict__ w, double* __restrict__ part) {
  __shared__ double sh[4];
  double dd = 0.0, vv = 0.0;
  for (int64_t i = blockIdx.x * int64_t(BS) + threadIdx.x; i < n; i += int64_t(gridDim.x) * BS) {
    const double d = v[i] - w[i];
    dd += d * d;
    vv += v[i] * v[i];
  }
  const double a = block_sum(dd, sh);
  const double b = block_sum(vv, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = a;
    part[DIFF_NBLK + blockIdx.x] = b;
  }
}

__global__ void k_diff_norms_finish(const double* __restrict__ part, double* __restrict__ out) {
  const double a = sum_partials_wave(DIFF_NBLK, part), b = sum_partials_wave(DIFF_NBLK, part + DIFF_NBLK);
  if (threadIdx.x == 0) {
    out[0] = sqrt(a);
    out[1] = sqrt(b);
  }
}

void diff_norms(int64_t n, const double* v, const double* w, double* part, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_diff_norms, dim3(DIFF_NBLK), dim3(BS), 0, s, n, v, w, part);
  hipLaunchKernelGGL(k_diff_norms_finish, dim3(1), dim3(64), 0, s, part, out);
}

void korteweg(int e0, int e1, const int* ep1, const int* ep2, const int* etype, double h,
              DP2Tables tb, const double* php, const double* phn, const double* phs, const double* Phi,
              const KorBeta& kb, int64_t n2, double* out, hipStream_t s) {
  if (e1 <= e0) return;
  hipLaunchKernelGGL(k_korteweg, dim3(ceil_div(e1 - e0, BS)), dim3(BS), 0, s, e0, e1, ep1, ep2,
                     etype, h, tb, php, phn, phs, Phi, kb, n2, out);
}

void form_ns(int64_t nslots, const int8_t* kind, const int* src, double cm, const double* Mv,
             const double* J, const double* Kxx, const double* Kxy, const double* Kyx,
             const double* Kyy, const double* B, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_form_ns, dim3(ceil_div(nslots, BS)), dim3(BS), 0, s, nslots, kind, src, cm,
                     Mv, J, Kxx, Kxy, Kyx, Kyy, B, out);
}

void rhs_ternary(const DSell& A, const double* Mv, const double* php, const double* phn,
                 const double* Phi, double c_mu, double c_ac, const PotCoef& pc, double* rhs_p, double* rhs_n,
                 double* rhs_ac, double* fs, hipStream_t s) {
  hipLaunchKernelGGL(k_rhs_ternary, dim3(ceil_div(A.nrows, BS)), dim3(BS), 0, s, A.nrows, A.side, A.col, Mv,
                     php, phn, Phi, c_mu, c_ac, pc, rhs_p, rhs_n, rhs_ac, fs);
}

template <typename T>
void sum_partial(int64_t n, const T* x, double* part, hipStream_t s) {
  hipLaunchKernelGGL((k_sum_partial<T>), dim3(reduce_blocks(n)), dim3(BS), 0, s, n, x, part);
}

template <typename T>
void sub_mean(int64_t n, int nblk, const double* part, T* x, hipStream_t s, double total) {
  hipLaunchKernelGGL((k_sub_mean<T>), dim3(ceil_div(n, BS)), dim3(BS), 0, s, n, nblk, part,
                     total > 0.0 ? total : double(n), x);
}

void wmean_zero(int64_t n, const double* w, double wtotal, double* x, double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_wsum_partial, dim3(reduce_blocks(n)), dim3(BS), 0, s, n, w, x, part);
  sub_mean<double>(n, reduce_blocks(n), part, x, s, wtotal);
}

void one_minus_sum(int64_t n, const double* a, const double* b, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_one_minus_sum, dim3(ceil_div(n, BS)), dim3(BS), 0, s, n, a, b, out);
}

void axpy_into(int64_t n, double a, const double* x, const double* y, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy_into, dim3(ceil_div(n, BS)), dim3(BS), 0, s, n, a, x, y, out);
}

// explicit instantiations
template void spmv<double, double>(const DSell&, const double*, const double*, double*, double,
                                   double, hipStream_t);
template void spmv<float, float>(const DSell&, const float*, const float*, float*, float, float,
                                 hipStream_t);
template void cheb01<double, double>(const DSell&, const double*, const double*, const double*, double,
                                     double, double, double*, double*, hipStream_t);
template void cheb01<float, float>(const DSell&, const float*, const float*, const float*, float, float,
                                   float, float*, float*, hipStream_t);
template void pcheb<double, double>(const DSell&, const double*, const double*, const double*,
                                    const double*, const double*, double, double*, double*, hipStream_t);
template void pcheb<float, float>(const DSell&, const float*, const float*, const float*, const float*,
                                  const float*, float, float*, float*, hipStream_t);
template void stencil<double, double>(const DSell&, const double*, int, const double*,
                                      const double*, const double*, double*, double, double,
                                      double*, hipStream_t, LaunchEv);
template void stencil<float, float>(const DSell&, const float*, int, const float*, const float*,
                                    const float*, float*, float, float, float*, hipStream_t, LaunchEv);
template void cheb0<double>(int, const double*, const double*, double, double*, double*,
                            hipStream_t);
template void cheb0<float>(int, const float*, const float*, float, float*, float*, hipStream_t);
template void coarse_cheb<double, double>(const DSell&, const double*, const double*,
                                          const double*, const ChebCoef<double>&, double*,
                                          hipStream_t);
template void coarse_cheb<float, float>(const DSell&, const float*, const float*, const float*,
                                        const ChebCoef<float>&, float*, hipStream_t);
template void bvtile<double>(int, int, const BTileLaunch<double>&, hipStream_t, int, int*);
template void bvtile<float>(int, int, const BTileLaunch<float>&, hipStream_t, int, int*);
template void bvtail<double>(int, const TailArgs<double>*, const int*, const int*, const double*, double*,
                             hipStream_t);
template void bvtail<float>(int, const TailArgs<float>*, const int*, const int*, const float*, float*,
                            hipStream_t);
template void vdown2<double>(const Tile2Args<double>&, hipStream_t);
template void vdown2<float>(const Tile2Args<float>&, hipStream_t);
template void vup2<double>(const Tile2Args<double>&, hipStream_t);
template void vup2<float>(const Tile2Args<float>&, hipStream_t);
template bool tile_fits<double>(int, int, int);
template bool tile_fits<float>(int, int, int);
template void vtile<double>(int, const TileArgs<double>&, hipStream_t, LaunchEv);
template void vtile<float>(int, const TileArgs<float>&, hipStream_t, LaunchEv);
template bool tail_fits<double>(const int*, int);
template bool tail_fits<float>(const int*, int);
template void vtail<double>(const TailArgs<double>&, hipStream_t);
template void vtail<float>(const TailArgs<float>&, hipStream_t);
template void ch_block<double, double>(const DSell&, const double*, const double*, const double*,
                                       double, double, const double*, double, double, double*,
                                       hipStream_t, LaunchEv, const double*);
template void ch_block<float, float>(const DSell&, const float*, const float*, const float*, float,
                                     float, const float*, float, float, float*, hipStream_t, LaunchEv,
                                     const float*);
template void axpby<double>(int64_t, double, const double*, double, double*, hipStream_t);
template void axpby<float>(int64_t, float, const float*, float, float*, hipStream_t);
template void convert<double, float>(int64_t, const double*, float*, hipStream_t);
template void convert<float, double>(int64_t, const float*, double*, hipStream_t);
template void sell_op<double, double>(const DSell&, const double*, int, const double*, const double*,
                                      const double*, double*, double, double, double*, hipStream_t);
template void sell_op<float, float>(const DSell&, const float*, int, const float*, const float*,
                                    const float*, float*, float, float, float*, hipStream_t);
template void sum_partial<double>(int64_t, const double*, double*, hipStream_t);
template void sum_partial<float>(int64_t, const float*, double*, hipStream_t);
template void sub_mean<double>(int64_t, int, const double*, double*, hipStream_t, double);
template void sub_mean<float>(int64_t, int, const double*, float*, hipStream_t, double);

}  // namespace chns

// ------------------------------------------------------------------ static scratch
// Device memory of the allocation-free diagnostics entry point.  Each GPU the
// library runs on holds its own copy until the process ends.  In host code
// `scratch` names a host-side stand-in, not the device array: host code uses
// only the address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) double scratch[chns::STATIC_SCRATCH];
static_assert(chns::STATIC_SCRATCH >= int64_t(chns::NDIAG) * (chns::MAXRED + 1),
              "static scratch holds the partials of the largest reduction grid and the results");

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch[MAX_DEVICES] = {};
}  // namespace

namespace chns {

hipError_t static_scratch_init() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[dev]) return hipSuccess;
  double* p = nullptr;
  e = hipGetSymbolAddress(reinterpret_cast<void**>(&p), HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch[dev] = p;
  return hipSuccess;
}

double* static_scratch(int device) {
  if (device < 0 || device >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch[device];
}

}  // namespace chns
