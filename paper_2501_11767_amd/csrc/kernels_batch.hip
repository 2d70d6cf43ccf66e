// Batched kernels: every launch covers all instances of the batch (stacked
// per-level P1 operators, stacked Krylov vectors with per-instance scalars).
#include <hip/hip_runtime.h>

#include "device_util.hpp"
#include "kernels_batch.hpp"

namespace chns {

namespace {

constexpr int BS = 256;
constexpr int W7 = 7;

inline int ceil_div(int64_t a, int64_t b) { return int((a + b - 1) / b); }

// Sum over the workgroup (any multiple of 64 up to 1024); valid in thread 0.
__device__ __forceinline__ double block_sum_any(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < int(blockDim.x >> 6); ++w) r += sh[w];
  __syncthreads();
  return r;
}

// Columns of a uniform width-7 row of the stacked level: computed from the
// slice's (side, first row) when geo is given, else read.
__device__ __forceinline__ void bcols7(int row, const int* __restrict__ col, const int2* __restrict__ geo,
                                       size_t base, int* c) {
  if (geo) {
    const int2 g = geo[row >> 6];
    p1_cols(row - g.y, g.x, c);
#pragma unroll
    for (int k = 0; k < W7; ++k) c[k] += g.y;
  } else {
#pragma unroll
    for (int k = 0; k < W7; ++k) c[k] = col[base + k * 64];
  }
}

template <typename T, int MODE, int RPT>
__global__ void k_bstencil(int nrows, const int* __restrict__ col, const int2* __restrict__ geo,
                           const T* __restrict__ val,
                           const T* __restrict__ x, const T* __restrict__ b,
                           const T* __restrict__ dinv, T* __restrict__ d, T p0, T p1,
                           const T* __restrict__ cc1, const T* __restrict__ cc2,
                           const uint8_t* __restrict__ mask, const int* __restrict__ act,
                           const int* __restrict__ sinst, T* __restrict__ y) {
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int row0 = blk * blockDim.x * RPT + threadIdx.x;
#pragma unroll
  for (int rr = 0; rr < RPT; ++rr) {
    const int row = row0 + rr * blockDim.x;
    if (row >= nrows) continue;
    const int slice = row >> 6;
    if (mask && !mask[slice]) continue;
    if (act && !act[sinst[slice]]) continue;
    T c1 = p0, c2 = p1;
    if (cc1) {
      const int inst = sinst[slice];
      c1 = cc1[inst];
      c2 = cc2[inst];
    }
    if (MODE == 3) {
      const T v = c2 * (dinv[row] * b[row]);
      d[row] = v;
      y[row] = v;
      continue;
    }
    const size_t base = size_t(slice) * (64 * W7) + (row & 63);
    int c[W7];
    T v[W7];
    bcols7(row, col, geo, base, c);
#pragma unroll
    for (int k = 0; k < W7; ++k) v[k] = val[base + k * 64];
    T sum = T(0);
#pragma unroll
    for (int k = 0; k < W7; ++k) sum += v[k] * x[c[k]];
    if (MODE == 0) {
      y[row] = (c2 == T(0)) ? c1 * sum : c1 * sum + c2 * y[row];
    } else if (MODE == 1) {
      y[row] = b[row] - sum;
    } else {
      const T r = dinv[row] * (b[row] - sum);
      const T dn = (c1 == T(0)) ? c2 * r : c1 * d[row] + c2 * r;
      d[row] = dn;
      y[row] = x[row] + dn;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(BS) void k_bspmv_uniform(int nrows, int width, const int* __restrict__ col,
                                                      const T* __restrict__ val,
                                                      const uint8_t* __restrict__ mask,
                                                      const int* __restrict__ sinst,
                                                      const int* __restrict__ act,
                                                      const T* __restrict__ x, T* __restrict__ y,
                                                      T alpha, T beta) {
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int row = blk * BS + threadIdx.x;
  if (row >= nrows) return;
  const int slice = row >> 6;
  if (mask && !mask[slice]) return;
  if (act && !act[sinst[slice]]) return;
  const size_t base = size_t(slice) * 64 * width + (row & 63);
  T sum = T(0);
  for (int k = 0; k < width; ++k) sum += val[base + k * 64] * x[col[base + k * 64]];
  y[row] = (beta == T(0)) ? alpha * sum : alpha * sum + beta * y[row];
}

template <typename T, bool L_IS_M>
__global__ __launch_bounds__(BS) void k_bch_block(int n, const int* __restrict__ col,
                                                  const int2* __restrict__ geo,
                                                  const int* __restrict__ sinst,
                                                  const int* __restrict__ act,
                                                  const T* __restrict__ Lv, const T* __restrict__ Kv,
                                                  const T* __restrict__ Mv,
                                                  const T* __restrict__ c12a,
                                                  const T* __restrict__ c22a,
                                                  const T* __restrict__ x, T alpha, T beta,
                                                  T* __restrict__ y) {
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int row = blk * BS + threadIdx.x;
  if (row >= n) return;
  const int inst = sinst[row >> 6];
  if (act && !act[inst]) return;
  const T c12 = c12a[inst], c22 = c22a[inst];
  const size_t base = size_t(row >> 6) * (64 * W7) + (row & 63);
  const T* x1 = x;
  const T* x2 = x + n;
  int c[W7];
  T kv[W7], mv[W7], lv[W7];
  bcols7(row, col, geo, base, c);
#pragma unroll
  for (int k = 0; k < W7; ++k) {
    kv[k] = Kv[base + k * 64];
    mv[k] = Mv[base + k * 64];
    if (!L_IS_M) lv[k] = Lv[base + k * 64];
  }
  T sl = T(0), sk1 = T(0), sk2 = T(0), sm = T(0);
#pragma unroll
  for (int k = 0; k < W7; ++k) {
    const T a = x1[c[k]], bb = x2[c[k]];
    sl += (L_IS_M ? mv[k] : lv[k]) * a;
    sk1 += kv[k] * a;
    sk2 += kv[k] * bb;
    sm += mv[k] * bb;
  }
  const T y1 = alpha * (sl + c12 * sk2);
  const T y2 = alpha * (c12 * sk1 + c22 * sm);
  if (beta == T(0)) {
    y[row] = y1;
    y[n + row] = y2;
  } else {
    y[row] = y1 + beta * y[row];
    y[n + row] = y2 + beta * y[n + row];
  }
}

__global__ __launch_bounds__(BS) void k_brhs_binary(int n, const int* __restrict__ col,
                                                    const int2* __restrict__ geo,
                                                    const int* __restrict__ sinst,
                                                    const double* __restrict__ Mv,
                                                    const double* __restrict__ phi,
                                                    const double* __restrict__ Phi,
                                                    const double* __restrict__ c_mu,
                                                    const double* __restrict__ c_ac,
                                                    double* __restrict__ rhs_ch,
                                                    double* __restrict__ rhs_ac) {
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int row = blk * BS + threadIdx.x;
  if (row >= n) return;
  const int inst = sinst[row >> 6];
  const size_t base = size_t(row >> 6) * (64 * W7) + (row & 63);
  double s_phi = 0.0, s_fp = 0.0, s_Phi = 0.0, s_fv = 0.0;
  int cc[W7];
  bcols7(row, col, geo, base, cc);
#pragma unroll
  for (int k = 0; k < W7; ++k) {
    const int j = cc[k];
    const double m = Mv[base + k * 64];
    const double ph = phi[j], P = Phi[j];
    const double om = 1.0 - ph;
    const double dliq = 2.0 * ph * om * om - 2.0 * ph * ph * om;
    const double p = P * P * (3.0 - 2.0 * P);
    const double dgas = 2.0 * ph - 2.0 * om;
    const double fp = (1.0 - p) * dliq + p * dgas;
    const double fv = 6.0 * P * (1.0 - P) * ((ph * ph + om * om) - ph * ph * om * om);
    s_phi += m * ph;
    s_fp += m * fp;
    s_Phi += m * P;
    s_fv += m * fv;
  }
  rhs_ch[row] = s_phi;
  rhs_ch[n + row] = c_mu[inst] * s_fp;
  rhs_ac[row] = s_Phi + c_ac[inst] * s_fv;
}

__global__ __launch_bounds__(BS) void k_bcombine(int64_t n, const int* __restrict__ sinst,
                                                 const double* __restrict__ a,
                                                 const double* __restrict__ A,
                                                 const double* __restrict__ b,
                                                 const double* __restrict__ B,
                                                 double* __restrict__ o64, float* __restrict__ o32) {
  const int64_t i = int64_t(blockIdx.x) * BS + threadIdx.x;
  if (i >= n) return;
  const int inst = sinst[i / (64 * W7)];
  const double v = a[inst] * A[i] + b[inst] * B[i];
  o64[i] = v;
  if (o32) o32[i] = float(v);
}

// ---------------------------------------------------------------- Krylov

constexpr int RPC = BCHUNK / BS;  // rows per thread in a chunk
constexpr int BDG = 16;          // basis vectors per dot launch

// Delayed classical Gram-Schmidt with reorthogonalisation (DCGS2), batched:
// per 1024-row chunk partial sums, reduced per instance over its chunk list
// ([cr[2i], cr[2i+1]) and, for the CH block, the same range shifted by half).

// Dots of one chunk: KK basis vectors V_g0.. against vt = V_j and w = V_{j+1},
// and with LAST vt.vt, vt.w, w.w; slot s of chunk c goes to
// part[s * nchunk + c] (slots [0, j) V_i.vt, [j, 2j) V_i.w, then 2j, 2j+1,
// 2j+2).  The accumulators are reduced by a wavefront reduce-scatter, then
// across the 4 wavefronts.  Chunks of inactive instances are skipped.  vs
// (may be null): vt is V_j as stored times vs[inst].
template <int KK, bool LAST>
__global__ __launch_bounds__(BS) void k_bdots(const double* __restrict__ V, int64_t ld, int j, int g0,
                                              double* __restrict__ part, const int* __restrict__ cinst,
                                              const int* __restrict__ act, const double* __restrict__ vs) {
  constexpr int NV = 2 * KK + (LAST ? 3 : 0);
  const int c = blockIdx.x;
  if (act && !act[cinst[c]]) return;
  const double sv = vs ? vs[cinst[c]] : 1.0;
  __shared__ double sh[4][NV];
  const double* vt = V + int64_t(j) * ld;
  const double* w = V + int64_t(j + 1) * ld;
  double acc[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) acc[i] = 0.0;
#pragma unroll
  for (int rr = 0; rr < RPC; ++rr) {
    const int64_t r = int64_t(c) * BCHUNK + rr * BS + threadIdx.x;
    const double t = vt[r] * sv, wr = w[r];
    double v[KK > 0 ? KK : 1];
#pragma unroll
    for (int i = 0; i < KK; ++i) v[i] = __builtin_nontemporal_load(V + (g0 + i) * ld + r);  // last use this step
#pragma unroll
    for (int i = 0; i < KK; ++i) {
      acc[i] += v[i] * t;
      acc[KK + i] += v[i] * wr;
    }
    if constexpr (LAST) {
      acc[2 * KK] += t * t;
      acc[2 * KK + 1] += t * wr;
      acc[2 * KK + 2] += wr * wr;
    }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int base = 0, lim = NV;
  WaveRS<NV, 32>::run(acc, lane, base, lim);
  if (lim >= 1) sh[wid][base] = acc[0];
  __syncthreads();
  const int t = threadIdx.x;
  if (t < NV) {
    int64_t slot;
    if (t < KK) slot = g0 + t;
    else if (t < 2 * KK) slot = j + g0 + (t - KK);
    else slot = 2 * j + (t - 2 * KK);
    part[slot * gridDim.x + c] = (sh[0][t] + sh[1][t]) + (sh[2][t] + sh[3][t]);
  }
}

// One wavefront per (slot, instance): red[i * rs + k] = slot k summed over the
// instance's chunks.
__global__ __launch_bounds__(64) void k_bslot_reduce(int nchunk, const double* __restrict__ part,
                                                     const int* __restrict__ cr, int half,
                                                     double* __restrict__ red, int rs,
                                                     const int* __restrict__ act) {
  const int k = blockIdx.x, i = blockIdx.y;
  if (act && !act[i]) return;
  const double* p = part + int64_t(k) * nchunk;
  double a = 0.0;
  for (int c = cr[2 * i] + int(threadIdx.x); c < cr[2 * i + 1]; c += 64) {
    a += p[c];
    if (half) a += p[c + half];
  }
  a = wave_sum(a);
  if (threadIdx.x == 0) red[int64_t(i) * rs + k] = a;
}

// One wavefront per instance: coefficients of step j from its reduced dots
// (the per-instance form of the FGMRES coefficient stage): c_i = V_i.vt,
// a_i = V_i.w, r = sqrt(vt.vt - |c|^2); column j-1 of the raw Hessenberg H
// becomes h_i += h_j c_i, h_j *= r; column j: a_i and b = (vt.w - c.a) / r;
// coef: [0, j) c_i, [j, 2j) a_i - b c_i / r, 2j: b / r, 2j+1: 1/r.
__global__ __launch_bounds__(64) void k_bdcgs_coef(int j, int m, const double* __restrict__ red, int rs,
                                                   double* __restrict__ H, double* __restrict__ coef,
                                                   int cstride, const int* __restrict__ act) {
  const int i = blockIdx.x;
  if (act && !act[i]) return;
  const double* ri = red + int64_t(i) * rs;
  double* Hi = H + int64_t(i) * (m + 1) * m;
  double* ci = coef + int64_t(i) * cstride;
  const int t = threadIdx.x, ld = m + 1;
  const double c = t < j ? ri[t] : 0.0;
  const double a = t < j ? ri[j + t] : 0.0;
  const double hj = j > 0 ? Hi[int64_t(j - 1) * ld + j] : 0.0;
  const double cc = wave_sum(c * c), ca = wave_sum(c * a);
  const double nu = ri[2 * j], tw = ri[2 * j + 1];
  const double r = j > 0 ? sqrt(fmax(nu - cc, 0.0)) : 1.0;
  const double inv = r > 0.0 ? 1.0 / r : 0.0;
  const double b = (tw - ca) * inv;
  if (j > 0 && t <= j) {
    double* hp = Hi + int64_t(j - 1) * ld;
    hp[t] = (t < j) ? hp[t] + hj * c : hj * r;
  }
  double* h = Hi + int64_t(j) * ld;
  if (t < j) {
    h[t] = a;
    ci[t] = c;
    ci[j + t] = a - b * c * inv;
  }
  if (t == 0) {
    h[j] = b;
    ci[2 * j] = b * inv;
    ci[2 * j + 1] = inv;
  }
}

// Update of one chunk with its instance's coefficients: w <- w - sum coef[j+i]
// V_i - coef[2j] vt, vt <- (vt - sum coef[i] V_i) / r (j > 0); chunk partial
// of |w'|^2.  vs (may be null): vt is V_j as stored times vs[inst].
// NT threads per 1024-row chunk (BCHUNK / NT rows each; the autotuner picks NT).
template <int NT>
__global__ __launch_bounds__(NT) void k_bdcgs_update(double* __restrict__ V, int64_t ld, int j,
                                                     const double* __restrict__ coef, int cstride,
                                                     double* __restrict__ nrm_part,
                                                     const int* __restrict__ cinst,
                                                     const int* __restrict__ act,
                                                     const double* __restrict__ vs) {
  constexpr int RPT = BCHUNK / NT;
  const int c = blockIdx.x;
  const int inst = cinst[c];
  if (act && !act[inst]) return;
  const double sv = vs ? vs[inst] : 1.0;
  __shared__ double cl[2 * 64 + 2];
  __shared__ double sh[16];
  for (int i = threadIdx.x; i < 2 * j + 2; i += NT) cl[i] = coef[int64_t(inst) * cstride + i];
  __syncthreads();
  double* vt = V + int64_t(j) * ld;
  double* w = V + int64_t(j + 1) * ld;
  const double inv = cl[2 * j + 1], wt = cl[2 * j];
  double acc = 0.0;
#pragma unroll
  for (int rr = 0; rr < RPT; ++rr) {
    const int64_t r = int64_t(c) * BCHUNK + rr * NT + threadIdx.x;
    const double t = vt[r] * sv;
    double wn = w[r] - wt * t, vn = t;
    int i = 0;
    for (; i + 8 <= j; i += 8) {
      double v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = __builtin_nontemporal_load(V + (i + q) * ld + r);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        vn -= cl[i + q] * v[q];
        wn -= cl[j + i + q] * v[q];
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
          vn -= cl[i + q] * v[q];
          wn -= cl[j + i + q] * v[q];
        }
    }
    if (j > 0) vt[r] = vn * inv;
    w[r] = wn;
    acc += wn * wn;
  }
  const double s = block_sum_any(acc, sh);
  if (threadIdx.x == 0) nrm_part[c] = s;
}

__device__ __forceinline__ void bgivens(double a, double b, double& c, double& s) {
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

// Rotations 0..upto-1 applied in order to x[0..upto].
__device__ __forceinline__ void brotate(double* x, int upto, const double* c, const double* s) {
  double carry = x[0];
  for (int i = 0; i < upto; ++i) {
    const double b = x[i + 1];
    x[i] = c[i] * carry + s[i] * b;
    carry = -s[i] * carry + c[i] * b;
  }
  x[upto] = carry;
}

// One wavefront per instance, end of step j: h_{j+1,j} = |w'| (provisional),
// column j-1 rotated into HR with its final rotation (and g), column j with a
// provisional one into HR and gp; the residual estimate |gp_{j+1}| decides
// the activity (an instance that stops keeps j + 1 columns); inv = 1/|w'|.
// The columns, rotations and g are staged in LDS for the serial chain.
__global__ __launch_bounds__(64) void k_bdcgs_finish(int nchunk, const double* __restrict__ part2,
                                                     const int* __restrict__ cr, int half, int j, int m,
                                                     double* __restrict__ H, double* __restrict__ HR,
                                                     double* __restrict__ cs, double* __restrict__ sn,
                                                     double* __restrict__ g, double* __restrict__ gp,
                                                     double* __restrict__ inv,
                                                     const double* __restrict__ tol,
                                                     int* __restrict__ active, int* __restrict__ kcols,
                                                     int* __restrict__ iters) {
  const int i = blockIdx.x, t = threadIdx.x;
  if (!active[i]) {
    if (t == 0) inv[i] = 0.0;
    return;
  }
  __shared__ double hp[66], hc[66], cs_s[64], sn_s[64], g_s[66], res[3];
  const int ld = m + 1;
  double* Hi = H + int64_t(i) * (m + 1) * m;
  double* HRi = HR + int64_t(i) * (m + 1) * m;
  double* csi = cs + int64_t(i) * (m + 1);
  double* sni = sn + int64_t(i) * (m + 1);
  double* gi = g + int64_t(i) * (m + 2);
  double* gpi = gp + int64_t(i) * (m + 2);
  for (int q = t; q <= j; q += 64) {
    hc[q] = Hi[int64_t(j) * ld + q];
    if (j > 0) hp[q] = Hi[int64_t(j - 1) * ld + q];
    g_s[q] = gi[q];
    if (q + 1 < j) {
      cs_s[q] = csi[q];
      sn_s[q] = sni[q];
    }
  }
  double a = 0.0;
  for (int c = cr[2 * i] + t; c < cr[2 * i + 1]; c += 64) {
    a += part2[c];
    if (half) a += part2[c + half];
  }
  const double nrm = sqrt(wave_sum(a));
  __syncthreads();
  if (t == 0) {
    hc[j + 1] = nrm;
    if (j > 0) {
      brotate(hp, j - 1, cs_s, sn_s);
      double c, s;
      bgivens(hp[j - 1], hp[j], c, s);
      cs_s[j - 1] = c;
      sn_s[j - 1] = s;
      hp[j - 1] = c * hp[j - 1] + s * hp[j];
      hp[j] = 0.0;
      g_s[j] = -s * g_s[j - 1];
      g_s[j - 1] = c * g_s[j - 1];
    }
    brotate(hc, j, cs_s, sn_s);
    double c, s;
    bgivens(hc[j], hc[j + 1], c, s);
    hc[j] = c * hc[j] + s * hc[j + 1];
    hc[j + 1] = 0.0;
    res[0] = c * g_s[j];
    res[1] = -s * g_s[j];
    Hi[int64_t(j) * ld + j + 1] = nrm;
    iters[i] += 1;
    const double est = fabs(res[1]);
    if (!(est > tol[i]) || nrm == 0.0 || !isfinite(est)) {
      active[i] = 0;
      kcols[i] = j + 1;
    }
    inv[i] = nrm > 0.0 ? 1.0 / nrm : 0.0;
  }
  __syncthreads();
  for (int q = t; q <= j + 1; q += 64) {
    HRi[int64_t(j) * ld + q] = hc[q];
    if (j > 0 && q <= j) HRi[int64_t(j - 1) * ld + q] = hp[q];
    if (q < j) gpi[q] = g_s[q];
  }
  if (t == 0) {
    if (j > 0) {
      csi[j - 1] = cs_s[j - 1];
      sni[j - 1] = sn_s[j - 1];
      gi[j - 1] = g_s[j - 1];
      gi[j] = g_s[j];
    }
    gpi[j] = res[0];
    gpi[j + 1] = res[1];
  }
}

// y = double(x) * inv[inst] (inv may be null) on chunks of active instances.
__global__ __launch_bounds__(BS) void k_bconvert_out(int64_t n, const float* __restrict__ x,
                                                     const double* __restrict__ inv,
                                                     double* __restrict__ y,
                                                     const int* __restrict__ cinst,
                                                     const int* __restrict__ act) {
  const int64_t r = int64_t(blockIdx.x) * BS + threadIdx.x;
  if (r >= n) return;
  const int inst = cinst[r / BCHUNK];
  if (act && act[inst] == 0) return;
  const double v = double(x[r]);
  y[r] = inv ? v * inv[inst] : v;
}

__global__ __launch_bounds__(BS) void k_bscale(int64_t n, const double* __restrict__ w,
                                               const double* __restrict__ inv,
                                               const int* __restrict__ cinst,
                                               const int* __restrict__ act,
                                               double* __restrict__ v) {
  const int64_t r = int64_t(blockIdx.x) * BS + threadIdx.x;
  if (r >= n) return;
  const int inst = cinst[r / BCHUNK];
  if (act && act[inst] == 0) return;
  v[r] = w[r] * inv[inst];
}

__global__ void k_blsq(int count, int m, const double* __restrict__ H, const double* __restrict__ g,
                       const int* __restrict__ kcols, double* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const int k = kcols[i];
  const int ld = m + 1;
  const double* Hi = H + int64_t(i) * (m + 1) * m;
  const double* gi = g + i * (m + 2);
  double* yi = y + i * (m + 1);
  for (int l = k; l < m; ++l) yi[l] = 0.0;
  for (int l = k - 1; l >= 0; --l) {
    double s = gi[l];
    for (int q = l + 1; q < k; ++q) s -= Hi[int64_t(q) * ld + l] * yi[q];
    yi[l] = s / Hi[int64_t(l) * ld + l];
  }
}

__global__ __launch_bounds__(BS) void k_bxupdate(int64_t n, const double* __restrict__ Z,
                                                 int64_t ldz, int m, const double* __restrict__ y,
                                                 double* __restrict__ x,
                                                 const int* __restrict__ cinst,
                                                 const int* __restrict__ kcols) {
  const int c = blockIdx.x;
  const int inst = cinst[c];
  const int k = kcols[inst];
  if (k == 0) return;
  __shared__ double ys[80];
  for (int i = threadIdx.x; i < k; i += BS) ys[i] = y[inst * (m + 1) + i];
  __syncthreads();
#pragma unroll
  for (int rr = 0; rr < RPC; ++rr) {
    const int64_t r = int64_t(c) * BCHUNK + rr * BS + threadIdx.x;
    double s = x[r];
    for (int i = 0; i < k; ++i) s += ys[i] * __builtin_nontemporal_load(Z + i * ldz + r);  // last use of Z
    x[r] = s;
  }
}

__global__ __launch_bounds__(BS) void k_bnorm_partial(int64_t n, const double* __restrict__ w,
                                                      double* __restrict__ part) {
  const int c = blockIdx.x;
  __shared__ double sh[16];
  double acc = 0.0;
#pragma unroll
  for (int rr = 0; rr < RPC; ++rr) {
    const double v = w[int64_t(c) * BCHUNK + rr * BS + threadIdx.x];
    acc += v * v;
  }
  const double s = block_sum_any(acc, sh);
  if (threadIdx.x == 0) part[c] = s;
}

__device__ double chunk_sum(const double* part, const int* cr, int half, int i) {
  double s = 0.0;
  for (int c = cr[2 * i] + int(threadIdx.x); c < cr[2 * i + 1]; c += blockDim.x) {
    s += part[c];
    if (half) s += part[c + half];
  }
  return s;
}

__global__ __launch_bounds__(BS) void k_bnorm_finish(int nchunk, const double* __restrict__ part,
                                                     const int* __restrict__ cr, int half, int m,
                                                     int first, double rtol, double atol,
                                                     double* __restrict__ nrm,
                                                     double* __restrict__ inv,
                                                     double* __restrict__ g,
                                                     double* __restrict__ tol,
                                                     int* __restrict__ active,
                                                     int* __restrict__ kcols) {
  const int i = blockIdx.x;
  __shared__ double sh[16];
  const double s = block_sum_any(chunk_sum(part, cr, half, i), sh);
  if (threadIdx.x != 0) return;
  const double v = sqrt(s);
  nrm[i] = v;
  if (first) {
    tol[i] = fmax(rtol * v, atol);
    return;
  }
  const int act = (v > tol[i]) && isfinite(v);
  active[i] = act;
  kcols[i] = act ? m : 0;
  inv[i] = (act && v > 0.0) ? 1.0 / v : 0.0;
  double* gi = g + i * (m + 2);
  gi[0] = v;
  for (int l = 1; l < m + 2; ++l) gi[l] = 0.0;
}

template <typename TI, typename TO>
__global__ __launch_bounds__(BS) void k_bconvert(int64_t n, const TI* __restrict__ x, TO* __restrict__ y,
                                                 const int* __restrict__ cinst,
                                                 const int* __restrict__ act) {
  const int64_t i = int64_t(blockIdx.x) * BS + threadIdx.x;
  if (i >= n) return;
  if (act && !act[cinst[i / BCHUNK]]) return;
  y[i] = TO(x[i]);
}

__global__ __launch_bounds__(BS) void k_dcopy(int64_t n, const double* __restrict__ x,
                                              double* __restrict__ y) {
  const int64_t i = int64_t(blockIdx.x) * BS + threadIdx.x;
  if (i < n) y[i] = x[i];
}

__global__ __launch_bounds__(BS) void k_dfill_int(int64_t n, int v, int* __restrict__ x) {
  const int64_t i = int64_t(blockIdx.x) * BS + threadIdx.x;
  if (i < n) x[i] = v;
}

}  // namespace

// ================================================================== launchers

template <typename T, int MODE>
static void launch_bstencil(const BStencil& A, const T* val, const T* x, const T* b, const T* dinv,
                            T* d, T p0, T p1, const T* cc1, const T* cc2, const uint8_t* mask,
                            const int* act, T* y, hipStream_t s) {
  const int rows_per_block = A.block * A.rpt;
  const dim3 g(ceil_div(A.nrows, rows_per_block)), blk(A.block);
  if (A.rpt == 4)
    hipLaunchKernelGGL((k_bstencil<T, MODE, 4>), g, blk, 0, s, A.nrows, A.col, A.geo, val, x, b, dinv, d,
                       p0, p1, cc1, cc2, mask, act, A.sinst, y);
  else if (A.rpt == 2)
    hipLaunchKernelGGL((k_bstencil<T, MODE, 2>), g, blk, 0, s, A.nrows, A.col, A.geo, val, x, b, dinv, d,
                       p0, p1, cc1, cc2, mask, act, A.sinst, y);
  else
    hipLaunchKernelGGL((k_bstencil<T, MODE, 1>), g, blk, 0, s, A.nrows, A.col, A.geo, val, x, b, dinv, d,
                       p0, p1, cc1, cc2, mask, act, A.sinst, y);
}

template <typename T>
void bstencil(const BStencil& A, const T* val, int mode, const T* x, const T* b, const T* dinv,
              T* d, T p0, T p1, const T* cc1, const T* cc2, const uint8_t* mask, const int* act,
              T* y, hipStream_t s) {
  switch (mode) {
    case 0: launch_bstencil<T, 0>(A, val, x, b, dinv, d, p0, p1, cc1, cc2, mask, act, y, s); break;
    case 1: launch_bstencil<T, 1>(A, val, x, b, dinv, d, p0, p1, cc1, cc2, mask, act, y, s); break;
    case 2: launch_bstencil<T, 2>(A, val, x, b, dinv, d, p0, p1, cc1, cc2, mask, act, y, s); break;
    default: launch_bstencil<T, 3>(A, val, x, b, dinv, d, p0, p1, cc1, cc2, mask, act, y, s); break;
  }
}

template <typename T>
void bspmv_uniform(int nrows, int width, const int* col, const T* val, const uint8_t* mask,
                   const int* sinst, const int* act, const T* x, T* y, T alpha, T beta,
                   hipStream_t s) {
  hipLaunchKernelGGL((k_bspmv_uniform<T>), dim3(ceil_div(nrows, BS)), dim3(BS), 0, s, nrows, width,
                     col, val, mask, sinst, act, x, y, alpha, beta);
}

template <typename T>
void bch_block(const BStencil& A, const T* L, const T* K, const T* M, const T* c12, const T* c22,
               const int* act, const T* x, T alpha, T beta, T* y, hipStream_t s) {
  const dim3 g(ceil_div(A.nrows, BS)), blk(BS);
  if (L == M)
    hipLaunchKernelGGL((k_bch_block<T, true>), g, blk, 0, s, A.nrows, A.col, A.geo, A.sinst, act, L, K, M,
                       c12, c22, x, alpha, beta, y);
  else
    hipLaunchKernelGGL((k_bch_block<T, false>), g, blk, 0, s, A.nrows, A.col, A.geo, A.sinst, act, L, K, M,
                       c12, c22, x, alpha, beta, y);
}

template <typename TI, typename TO>
void bconvert(int64_t n, const TI* x, TO* y, const int* cinst, const int* act, hipStream_t s) {
  hipLaunchKernelGGL((k_bconvert<TI, TO>), dim3(ceil_div(n, BS)), dim3(BS), 0, s, n, x, y, cinst, act);
}

void brhs_binary(const BStencil& A, const double* Mv, const double* phi, const double* Phi,
                 const double* c_mu, const double* c_ac, double* rhs_ch, double* rhs_ac,
                 hipStream_t s) {
  hipLaunchKernelGGL(k_brhs_binary, dim3(ceil_div(A.nrows, BS)), dim3(BS), 0, s, A.nrows, A.col, A.geo,
                     A.sinst, Mv, phi, Phi, c_mu, c_ac, rhs_ch, rhs_ac);
}

void bcombine(int64_t nslots, const int* sinst, const double* a, const double* A, const double* b,
              const double* B, double* out64, float* out32, hipStream_t s) {
  hipLaunchKernelGGL(k_bcombine, dim3(ceil_div(nslots, BS)), dim3(BS), 0, s, nslots, sinst, a, A,
                     b, B, out64, out32);
}

// The last group (kk < BDG vectors plus the vt, w products).
static void launch_bdots_last(int kk, int nchunk, const double* V, int64_t ld, int j, int g0, double* part,
                              const int* cinst, const int* act, const double* vs, hipStream_t s) {
  switch (kk) {
#define CHNS_BDOTS_CASE(K)                                                                        \
  case K:                                                                                          \
    hipLaunchKernelGGL((k_bdots<K, true>), dim3(nchunk), dim3(BS), 0, s, V, ld, j, g0, part, cinst, \
                       act, vs);                                                                   \
    break;
    CHNS_BDOTS_CASE(0) CHNS_BDOTS_CASE(1) CHNS_BDOTS_CASE(2) CHNS_BDOTS_CASE(3) CHNS_BDOTS_CASE(4)
    CHNS_BDOTS_CASE(5) CHNS_BDOTS_CASE(6) CHNS_BDOTS_CASE(7) CHNS_BDOTS_CASE(8) CHNS_BDOTS_CASE(9)
    CHNS_BDOTS_CASE(10) CHNS_BDOTS_CASE(11) CHNS_BDOTS_CASE(12) CHNS_BDOTS_CASE(13)
    CHNS_BDOTS_CASE(14) CHNS_BDOTS_CASE(15)
#undef CHNS_BDOTS_CASE
    default: break;
  }
}

void bdcgs_dots(int64_t n, const double* V, int64_t ld, int j, double* part, const int* cinst,
                const int* act, const double* vs, hipStream_t s, int group) {
  const int nchunk = int(n / BCHUNK);
  const int bdg = group == 8 ? 8 : BDG;
  const int full = j / bdg, rem = j - full * bdg;
  for (int g = 0; g < full; ++g) {
    if (bdg == 8)
      hipLaunchKernelGGL((k_bdots<8, false>), dim3(nchunk), dim3(BS), 0, s, V, ld, j, g * bdg, part, cinst,
                         act, vs);
    else
      hipLaunchKernelGGL((k_bdots<BDG, false>), dim3(nchunk), dim3(BS), 0, s, V, ld, j, g * bdg, part, cinst,
                         act, vs);
  }
  launch_bdots_last(rem, nchunk, V, ld, j, full * bdg, part, cinst, act, vs, s);
}

void bslot_reduce(int count, int nchunk, int nslots, const double* part, const int* cr, int half,
                  double* red, int rs, const int* act, hipStream_t s) {
  hipLaunchKernelGGL(k_bslot_reduce, dim3(nslots, count), dim3(64), 0, s, nchunk, part, cr, half, red, rs,
                     act);
}

void bdcgs_coef(int count, int j, int m, const double* red, int rs, double* H, double* coef, int cstride,
                const int* act, hipStream_t s) {
  hipLaunchKernelGGL(k_bdcgs_coef, dim3(count), dim3(64), 0, s, j, m, red, rs, H, coef, cstride, act);
}

void bdcgs_update(int64_t n, double* V, int64_t ld, int j, const double* coef, int cstride,
                  double* nrm_part, const int* cinst, const int* act, const double* vs, hipStream_t s,
                  int threads) {
  const dim3 g(int(n / BCHUNK));
  if (threads == 1024)
    hipLaunchKernelGGL(k_bdcgs_update<1024>, g, dim3(1024), 0, s, V, ld, j, coef, cstride, nrm_part, cinst,
                       act, vs);
  else if (threads == 512)
    hipLaunchKernelGGL(k_bdcgs_update<512>, g, dim3(512), 0, s, V, ld, j, coef, cstride, nrm_part, cinst,
                       act, vs);
  else
    hipLaunchKernelGGL(k_bdcgs_update<BS>, g, dim3(BS), 0, s, V, ld, j, coef, cstride, nrm_part, cinst,
                       act, vs);
}

void bdcgs_finish(int count, int nchunk, const double* part2, const int* cr, int half, int j, int m,
                  double* H, double* HR, double* cs, double* sn, double* g, double* gp, double* inv,
                  const double* tol, int* active, int* kcols, int* iters, hipStream_t s) {
  hipLaunchKernelGGL(k_bdcgs_finish, dim3(count), dim3(64), 0, s, nchunk, part2, cr, half, j, m, H, HR, cs,
                     sn, g, gp, inv, tol, active, kcols, iters);
}

void bconvert_out(int64_t n, const float* x, const double* inv, double* y, const int* cinst, const int* act,
                  hipStream_t s) {
  hipLaunchKernelGGL(k_bconvert_out, dim3(ceil_div(n, BS)), dim3(BS), 0, s, n, x, inv, y, cinst, act);
}

void bscale(int64_t n, const double* w, const double* inv, const int* cinst, const int* act,
            double* v, hipStream_t s) {
  hipLaunchKernelGGL(k_bscale, dim3(ceil_div(n, BS)), dim3(BS), 0, s, n, w, inv, cinst, act, v);
}

void blsq(int count, int m, const double* H, const double* g, const int* kcols, double* y,
          hipStream_t s) {
  hipLaunchKernelGGL(k_blsq, dim3(ceil_div(count, 64)), dim3(64), 0, s, count, m, H, g, kcols, y);
}

void bxupdate(int64_t n, const double* Z, int64_t ldz, int m, const double* y, double* x,
              const int* cinst, const int* kcols, hipStream_t s) {
  hipLaunchKernelGGL(k_bxupdate, dim3(int(n / BCHUNK)), dim3(BS), 0, s, n, Z, ldz, m, y, x, cinst,
                     kcols);
}

void bnorm_partial(int64_t n, const double* w, double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_bnorm_partial, dim3(int(n / BCHUNK)), dim3(BS), 0, s, n, w, part);
}

void bnorm_finish(int count, int nchunk, const double* part, const int* cr, int half, int m,
                  int first, double rtol, double atol, double* nrm, double* inv, double* g,
                  double* tol, int* active, int* kcols, hipStream_t s) {
  hipLaunchKernelGGL(k_bnorm_finish, dim3(count), dim3(BS), 0, s, nchunk, part, cr, half, m, first,
                     rtol, atol, nrm, inv, g, tol, active, kcols);
}

void dcopy(int64_t n, const double* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_dcopy, dim3(ceil_div(n, BS)), dim3(BS), 0, s, n, x, y);
}

void dfill_int(int64_t n, int v, int* x, hipStream_t s) {
  hipLaunchKernelGGL(k_dfill_int, dim3(ceil_div(n, BS)), dim3(BS), 0, s, n, v, x);
}

template void bstencil<double>(const BStencil&, const double*, int, const double*, const double*,
                               const double*, double*, double, double, const double*,
                               const double*, const uint8_t*, const int*, double*, hipStream_t);
template void bstencil<float>(const BStencil&, const float*, int, const float*, const float*,
                              const float*, float*, float, float, const float*, const float*,
                              const uint8_t*, const int*, float*, hipStream_t);
template void bspmv_uniform<double>(int, int, const int*, const double*, const uint8_t*, const int*,
                                    const int*, const double*, double*, double, double, hipStream_t);
template void bspmv_uniform<float>(int, int, const int*, const float*, const uint8_t*, const int*,
                                   const int*, const float*, float*, float, float, hipStream_t);
template void bch_block<double>(const BStencil&, const double*, const double*, const double*,
                                const double*, const double*, const int*, const double*, double,
                                double, double*, hipStream_t);
template void bconvert<double, float>(int64_t, const double*, float*, const int*, const int*,
                                      hipStream_t);
template void bconvert<float, double>(int64_t, const float*, double*, const int*, const int*,
                                      hipStream_t);

}  // namespace chns
