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

// Columns of a row of the periodic cube's 15-entry P1 pattern (side n,
// vertex i + n j + n^2 k): the vertex, then the neighbours at -d and +d for
// the edge directions (1,0,0), (0,1,0), (0,0,1), (1,1,0), (1,0,1), (0,1,1),
// (1,1,1) in turn.
__device__ __forceinline__ void p1_cols_cube(int row, int n, int* c) {
  const int nn = n * n;
  const int k = row / nn, rem = row - k * nn;
  const int j = rem / n, i = rem - j * n;
  const int x[3] = {i == 0 ? n - 1 : i - 1, i, i == n - 1 ? 0 : i + 1};
  const int y[3] = {(j == 0 ? n - 1 : j - 1) * n, j * n, (j == n - 1 ? 0 : j + 1) * n};
  const int z[3] = {(k == 0 ? n - 1 : k - 1) * nn, k * nn, (k == n - 1 ? 0 : k + 1) * nn};
  c[0] = row;
  c[1] = x[0] + y[1] + z[1];
  c[2] = x[2] + y[1] + z[1];
  c[3] = x[1] + y[0] + z[1];
  c[4] = x[1] + y[2] + z[1];
  c[5] = x[1] + y[1] + z[0];
  c[6] = x[1] + y[1] + z[2];
  c[7] = x[0] + y[0] + z[1];
  c[8] = x[2] + y[2] + z[1];
  c[9] = x[0] + y[1] + z[0];
  c[10] = x[2] + y[1] + z[2];
  c[11] = x[1] + y[0] + z[0];
  c[12] = x[1] + y[2] + z[2];
  c[13] = x[0] + y[0] + z[0];
  c[14] = x[2] + y[2] + z[2];
}

// Columns of a row of a uniform width-W pattern: width 7 (triangles; computed
// on the periodic square, side > 0), width 15 (tetrahedra; computed on the
// periodic cube, side > 0 its side); otherwise loaded.
template <int W>
__device__ __forceinline__ void row_cols(int row, int side, const int* __restrict__ col, size_t base, int* c) {
  if constexpr (W == 7) {
    row_cols7(row, side, col, base, c);
  } else {
    static_assert(W == 15, "rows of 7 or 15 entries");
    if (side > 0) {
      p1_cols_cube(row, side, c);
    } else {
#pragma unroll
      for (int k = 0; k < W; ++k) c[k] = col[base + k * 64];
    }
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
  for (int i = 0; i < 4; ++i) {
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

// ---------------------------------------------------------------- ternary densities
// Liquid and gas densities of polymer p, NFA n and solvent s (air = 0) in
// unreduced form with first and second partial derivatives, interpolated by
// p(Phi) = Phi^2 (3 - 2 Phi); the reduced density follows from s = 1 - p - n.
//   fitted quartic (eq. (appPotential)): liq = 3.5 p^2 n^2 + 0.3 s^2,
//     gas = 3.5 p^2 + 3.5 n^2 + 2 s^2;
//   Flory-Huggins (section "Free energy functional", x ln x by its degree-4
//     Taylor polynomial T4 about 1/2, section "Numerical results"):
//     liq = sum_i T4(x_i) / N_i + chi_pn p n + chi_ps p s + chi_ns n s,
//     gas = sum_i (T4(x_i) - x_i ln phi_sat(i)).
// trunc: the fields enter as clip(x, 0, 1) (eq. (truncateCH)) and the chain
// rule carries the clip's derivative (1 inside [0, 1], else 0).
// Every member is a named scalar assigned on both branches: an earlier form
// kept the partials in 3x3 arrays with some entries stored per branch, and on
// gfx950 one of those stores was lost (the gas d2/dn2 of the quartic read 0).
struct TerParts {
  double liq, gas;
  double lp, ln, ls, gp, gn, gs;                    // first partials (liquid, gas)
  double lpp, lnn, lss, lpn, lps, lns, gpp, gnn, gss;  // second partials (the gas part is diagonal)
};

__device__ __forceinline__ void t4_eval(const double* c, double x, double& g, double& g1, double& g2) {
  const double u = x - 0.5;
  g = c[0] + u * (c[1] + u * (c[2] + u * (c[3] + u * c[4])));
  g1 = c[1] + u * (2.0 * c[2] + u * (3.0 * c[3] + u * 4.0 * c[4]));
  g2 = 2.0 * c[2] + u * (6.0 * c[3] + u * 12.0 * c[4]);
}

__device__ __forceinline__ TerParts ter_parts(double p, double n, double s, const PotCoef& c) {
  TerParts t;
  if (!c.fh) {
    t.liq = 3.5 * p * p * n * n + 0.3 * s * s;
    t.gas = 3.5 * p * p + 3.5 * n * n + 2.0 * s * s;
    t.lp = 7.0 * p * n * n;
    t.ln = 7.0 * p * p * n;
    t.ls = 0.6 * s;
    t.gp = 7.0 * p;
    t.gn = 7.0 * n;
    t.gs = 4.0 * s;
    t.lpp = 7.0 * n * n;
    t.lnn = 7.0 * p * p;
    t.lss = 0.6;
    t.lpn = 14.0 * p * n;
    t.lps = 0.0;
    t.lns = 0.0;
    t.gpp = 7.0;
    t.gnn = 7.0;
    t.gss = 4.0;
    return t;
  }
  double ap, ap1, ap2, an, an1, an2, as, as1, as2;
  t4_eval(c.t4, p, ap, ap1, ap2);
  t4_eval(c.t4, n, an, an1, an2);
  t4_eval(c.t4, s, as, as1, as2);
  t.liq = ap * c.invN[0] + an * c.invN[1] + as * c.invN[2] + c.chi[0] * p * n + c.chi[1] * p * s +
          c.chi[2] * n * s;
  t.gas = (ap - p * c.lsat[0]) + (an - n * c.lsat[1]) + (as - s * c.lsat[2]);
  t.lp = ap1 * c.invN[0] + c.chi[0] * n + c.chi[1] * s;
  t.ln = an1 * c.invN[1] + c.chi[0] * p + c.chi[2] * s;
  t.ls = as1 * c.invN[2] + c.chi[1] * p + c.chi[2] * n;
  t.gp = ap1 - c.lsat[0];
  t.gn = an1 - c.lsat[1];
  t.gs = as1 - c.lsat[2];
  t.lpp = ap2 * c.invN[0];
  t.lnn = an2 * c.invN[1];
  t.lss = as2 * c.invN[2];
  t.lpn = c.chi[0];
  t.lps = c.chi[1];
  t.lns = c.chi[2];
  t.gpp = ap2;
  t.gnn = an2;
  t.gss = as2;
  return t;
}

// The point where the density is evaluated (p, n, s = 1 - p - n, each
// clipped to [0, 1] when the fields are truncated) and the clip's derivatives.
struct TerPoint {
  double p, n, s, cp, cn, cs;  // cp, cn, cs: the clip's derivatives
};

__device__ __forceinline__ void clip01(bool on, double v, double& x, double& d) {
  x = on ? fmin(fmax(v, 0.0), 1.0) : v;
  d = (!on || (v >= 0.0 && v <= 1.0)) ? 1.0 : 0.0;
}

__device__ __forceinline__ TerPoint ter_point(double pp, double pn, const PotCoef& c) {
  TerPoint x;
  const bool on = c.trunc != 0;
  clip01(on, pp, x.p, x.cp);
  clip01(on, pn, x.n, x.cn);
  clip01(on, 1.0 - pp - pn, x.s, x.cs);
  return x;
}

// Nodal terms of the reduced density: dp, dn (d f / d phi_p, d phi_N along
// phi_s = 1 - phi_p - phi_N), fv = d f / d Phi_v, fs = the unreduced d f / d phi_s
// (the closure of the eliminated phase).
__device__ __forceinline__ void ternary_terms(double pp, double pn, double P, const PotCoef& c, double& dp,
                                              double& dn, double& fv, double& fs) {
  const TerPoint x = ter_point(pp, pn, c);
  const TerParts t = ter_parts(x.p, x.n, x.s, c);
  const double ip = P * P * (3.0 - 2.0 * P), q = 1.0 - ip;
  const double F0 = q * t.lp + ip * t.gp, F1 = q * t.ln + ip * t.gn, F2 = q * t.ls + ip * t.gs;
  dp = F0 * x.cp - F2 * x.cs;
  dn = F1 * x.cn - F2 * x.cs;
  fv = 6.0 * P * (1.0 - P) * (t.gas - t.liq);
  fs = F2;
}

__device__ __forceinline__ double density_ternary(double pp, double pn, double P, const PotCoef& c) {
  const TerPoint x = ter_point(pp, pn, c);
  const TerParts t = ter_parts(x.p, x.n, x.s, c);
  const double ip = P * P * (3.0 - 2.0 * P);
  return (1.0 - ip) * t.liq + ip * t.gas;
}

// Quaternary model: eq. (appPotential) in all four phases with the air
// eliminated, a = 1 - p - n - s.  Liquid 3.5 p^2 n^2 + 0.3 s^2 + 0.3 a^2 -
// 10 s a, gas 3.5 p^2 + 3.5 n^2 + 2 s^2 + 0.1 a^2, interpolated by
// P = Phi^2 (3 - 2 Phi).  dp, dn, ds: derivatives along the elimination (the
// unreduced partial minus the air's); fa: the unreduced air partial (closure
// of mu_a); fv: d f / d Phi.
__device__ __forceinline__ void quaternary_terms(double p, double n, double s, double P, double& dp,
                                                 double& dn, double& ds, double& fa, double& fv) {
  const double a = 1.0 - p - n - s;
  const double ip = P * P * (3.0 - 2.0 * P), q = 1.0 - ip;
  const double Fp = q * (7.0 * p * n * n) + ip * (7.0 * p);
  const double Fn = q * (7.0 * p * p * n) + ip * (7.0 * n);
  const double Fs = q * (0.6 * s - 10.0 * a) + ip * (4.0 * s);
  const double Fa = q * (0.6 * a - 10.0 * s) + ip * (0.2 * a);
  dp = Fp - Fa;
  dn = Fn - Fa;
  ds = Fs - Fa;
  fa = Fa;
  const double liq = 3.5 * p * p * n * n + 0.3 * s * s + 0.3 * a * a - 10.0 * s * a;
  const double gas = 3.5 * p * p + 3.5 * n * n + 2.0 * s * s + 0.1 * a * a;
  fv = 6.0 * P * (1.0 - P) * (gas - liq);
}

__device__ __forceinline__ double density_quaternary(double p, double n, double s, double P) {
  const double a = 1.0 - p - n - s;
  const double ip = P * P * (3.0 - 2.0 * P);
  const double liq = 3.5 * p * p * n * n + 0.3 * s * s + 0.3 * a * a - 10.0 * s * a;
  const double gas = 3.5 * p * p + 3.5 * n * n + 2.0 * s * s + 0.1 * a * a;
  return (1.0 - ip) * liq + ip * gas;
}

}  // namespace chns
