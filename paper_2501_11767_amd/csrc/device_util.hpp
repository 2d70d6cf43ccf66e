// Device helpers shared by the kernel files: the XCD-contiguous workgroup
// remap, wavefront and workgroup sums, the P1 element geometry of the periodic
// right-diagonal mesh, the P2-by-P1 mass weights, the elementwise constant part
// of the convecting field and the nodal terms of the ternary density.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace chns {

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b runs on
// XCD b % 8).  Map them so that XCD x processes one contiguous range.
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int per = nb >> 3, rem = nb & 7;
  const int x = b & 7, k = b >> 3;
  return x * per + (x < rem ? x : rem) + k;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Reduce-scatter over the wavefront by recursive halving: every lane holds C
// values v[0..C); at the step with lane offset O each lane keeps one half of
// its values (the upper half when its bit O is set; an odd count pads the
// upper half with a zero), adds the partner's copy of that half and sends the
// other half, one shuffle per kept value.  base tracks the index of the
// lane's first kept value and lim how many of its kept values are real.
// After the steps O = 32 .. 1 (C <= 64), a lane with lim >= 1 holds in v[0]
// the wavefront total of value index base; every index is held by exactly
// one lane.  About C shuffles in all, where C separate wavefront sums take 6 C.
template <int C, int O>
struct WaveRS {
  static __device__ __forceinline__ void run(double* v, int lane, int& base, int& lim) {
    constexpr int HH = (C + 1) / 2;
    const bool up = (lane & O) != 0;
#pragma unroll
    for (int i = 0; i < HH; ++i) {
      const double lo = v[i];
      const double hi = (i + HH < C) ? v[(i + HH < C) ? i + HH : 0] : 0.0;
      v[i] = (up ? hi : lo) + __shfl_xor(up ? lo : hi, O, 64);
    }
    if (up) {
      base += HH;
      lim = lim > HH ? lim - HH : 0;
    } else {
      lim = lim < HH ? lim : HH;
    }
    WaveRS<HH, O / 2>::run(v, lane, base, lim);
  }
};
template <int C>
struct WaveRS<C, 0> {
  static __device__ __forceinline__ void run(double*, int, int&, int&) {}
};

// Sum over a 256-thread workgroup (sh: 4 doubles); result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double* sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) sh[wid] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return r;
}

// int psi_k lambda_a / |T| for the P2 basis psi_k (vertices, then edge nodes
// opposite vertices 0, 1, 2) against the P1 basis lambda_a, from the monomial
// integrals int l0^a l1^b l2^c = 2|T| a! b! c! / (a+b+c+2)!.
__device__ __forceinline__ double w_p2p1(int k, int a) {
  if (k < 3) return (k == a) ? (1.0 / 30.0) : (-1.0 / 60.0);
  return ((k - 3) == a) ? (1.0 / 15.0) : (2.0 / 15.0);
}

// Columns of P1 row `row` of the periodic side x side mesh, in the neighbour
// order of the P1 storage: self, (-1,-1), (0,-1), (-1,0), (1,0), (0,1), (1,1).
__device__ __forceinline__ void p1_cols(int row, int side, int* c) {
  const int j = row / side, i = row - j * side;
  const int im = (i == 0) ? side - 1 : i - 1, ip = (i == side - 1) ? 0 : i + 1;
  const int jm = (j == 0) ? side - 1 : j - 1, jp = (j == side - 1) ? 0 : j + 1;
  const int rj = side * j, rm = side * jm, rp = side * jp;
  c[0] = row;
  c[1] = im + rm;
  c[2] = i + rm;
  c[3] = im + rj;
  c[4] = ip + rj;
  c[5] = i + rp;
  c[6] = ip + rp;
}

// Columns of a uniform width-7 row: computed when side > 0, else loaded.
__device__ __forceinline__ void row_cols7(int row, int side, const int* __restrict__ col, size_t base,
                                          int* c) {
  if (side > 0) {
    p1_cols(row, side, c);
  } else {
#pragma unroll
    for (int k = 0; k < 7; ++k) c[k] = col[base + k * 64];
  }
}

struct ElemGeo {
  double area;
  double gx[3], gy[3];
};

__device__ __forceinline__ ElemGeo elem_geo(int type, double h) {
  double x1, y1, x2, y2;
  if (type == 0) {
    x1 = h; y1 = 0.0; x2 = h; y2 = h;
  } else {
    x1 = h; y1 = h; x2 = 0.0; y2 = h;
  }
  const double det = x1 * y2 - x2 * y1;
  ElemGeo g;
  g.area = 0.5 * fabs(det);
  g.gx[1] = y2 / det;  g.gy[1] = -x2 / det;
  g.gx[2] = -y1 / det; g.gy[2] = x1 / det;
  g.gx[0] = -g.gx[1] - g.gx[2];
  g.gy[0] = -g.gy[1] - g.gy[2];
  return g;
}

// w_const = -alpha sum_i grad mu_i on the element (P1 gradients are constant).
__device__ __forceinline__ void mu_const(const MuGrad& mg, const int* vtx, const ElemGeo& g,
                                         double& wx, double& wy) {
  wx = 0.0;
  wy = 0.0;
  for (int i = 0; i < 3; ++i) {
    if (!mg.mu[i]) continue;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const double m = mg.mu[i][vtx[a]];
      wx += m * g.gx[a];
      wy += m * g.gy[a];
    }
  }
  wx *= -mg.alpha;
  wy *= -mg.alpha;
}

__device__ __forceinline__ void ternary_terms(double pp, double pn, double P, double& dp, double& dn,
                                              double& fv, double& fs) {
  const double ps = 1.0 - pp - pn;
  const double p = P * P * (3.0 - 2.0 * P);
  dp = (1.0 - p) * (7.0 * pp * pn * pn - 0.6 * ps) + p * (7.0 * pp - 4.0 * ps);
  dn = (1.0 - p) * (7.0 * pp * pp * pn - 0.6 * ps) + p * (7.0 * pn - 4.0 * ps);
  const double liq = 3.5 * pp * pp * pn * pn + 0.3 * ps * ps;
  const double gas = 3.5 * pp * pp + 3.5 * pn * pn + 2.0 * ps * ps;
  fv = 6.0 * P * (1.0 - P) * (gas - liq);
  fs = (1.0 - p) * 0.6 * ps + p * 4.0 * ps;
}

}  // namespace chns
