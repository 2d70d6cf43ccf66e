// Adjoint kernels of the differentiation form (the transposed solves reuse
// the forward solver on transposed operator values).
//
// The element kernels mirror the forward assembly: one thread per triangle,
// launched per colour of the 8-colouring (triangles of one colour share no
// vertex, hence no P2 node), so the scatters need no atomics.
#include <hip/hip_runtime.h>

#include "device_util.hpp"
#include "kernels_adj.hpp"

namespace chns {

namespace {

constexpr int BS = 256;

inline int ceil_div(int64_t a, int64_t b) { return int((a + b - 1) / b); }

__global__ __launch_bounds__(BS) void k_gather_slots(int64_t n, const int* __restrict__ tmap,
                                                     const double* __restrict__ in,
                                                     double* __restrict__ out) {
  const int64_t i = int64_t(blockIdx.x) * BS + threadIdx.x;
  if (i < n) out[i] = in[tmap[i]];
}

// Second derivatives of the reduced ternary density at one node (the
// derivatives of the nodal f_p', f_N', f_v' and of the closure f_s'), from the
// unreduced partials by the chain rule along phi_s = 1 - phi_p - phi_N (with
// the clip's derivative when the fields are truncated).
struct Hess {
  double pp, pn, nn, pP, nP, vP, sp, sn, sP;
};

__device__ __forceinline__ Hess hess_ter(double pp, double pn, double P, const PotCoef& c) {
  const TerPoint x = ter_point(pp, pn, c);
  const TerParts t = ter_parts(x.p, x.n, x.s, c);
  const double ip = P * P * (3.0 - 2.0 * P), q = 1.0 - ip;
  const double dip = 6.0 * P * (1.0 - P), ddip = 6.0 - 12.0 * P;
  // second partials of the interpolated unreduced density
  const double Fpp = q * t.lpp + ip * t.gpp, Fnn = q * t.lnn + ip * t.gnn, Fss = q * t.lss + ip * t.gss;
  const double Fpn = q * t.lpn, Fps = q * t.lps, Fns = q * t.lns;
  const double Dp = dip * (t.gp - t.lp), Dn = dip * (t.gn - t.ln), Ds = dip * (t.gs - t.ls);
  const double Ip = x.cp, In = x.cn, Is = x.cs;
  Hess h;
  h.pp = Fpp * Ip - 2.0 * Fps * Ip * Is + Fss * Is;
  h.nn = Fnn * In - 2.0 * Fns * In * Is + Fss * Is;
  h.pn = Fpn * Ip * In - Fps * Ip * Is - Fns * In * Is + Fss * Is;
  h.pP = Dp * Ip - Ds * Is;
  h.nP = Dn * In - Ds * Is;
  h.vP = ddip * (t.gas - t.liq);
  h.sp = Fps * Ip - Fss * Is;
  h.sn = Fns * In - Fss * Is;
  h.sP = Ds;
  return h;
}

__global__ __launch_bounds__(BS) void k_adj_nodal(int n, AdjNodal a, double* __restrict__ part) {
  __shared__ double sh[4];
  const double beta = a.eps * a.eps;
  const double c = a.tau * a.gam / beta;
  double sg = 0.0, se = 0.0, sv = 0.0;
  for (int i = blockIdx.x * BS + threadIdx.x; i < n; i += gridDim.x * BS) {
    const double pp = a.php[i], pn = a.phn[i], P = a.Phi[i];
    double fp, fn, fv, fs;
    ternary_terms(pp, pn, P, a.pc, fp, fn, fv, fs);
    const Hess H = hess_ter(pp, pn, P, a.pc);
    const double gp = -c * a.Me2p[i], gn = -c * a.Me2n[i], gvv = -a.tau * a.gv * a.Mz[i];
    const double nu = a.nus[i];
    a.lam_php[i] = a.Me1p[i] + H.pp * gp + H.pn * gn + H.pP * gvv + H.sp * nu;
    a.lam_phn[i] = a.Me1n[i] + H.pn * gp + H.nn * gn + H.nP * gvv + H.sn * nu;
    a.lam_Phi[i] = a.Mz[i] + H.pP * gp + H.nP * gn + H.vP * gvv + H.sP * nu;
    const double mp = a.mup1[i], mn = a.mun1[i];
    const double sch = a.Me2p[i] * (fp - mp) + a.Me2n[i] * (fn - mn);
    sg += -(a.tau / beta) * sch - a.tau * (a.Ke1p[i] * mp + a.Ke1n[i] * mn) -
          a.tau * (a.Ke2p[i] * a.php1[i] + a.Ke2n[i] * a.phn1[i]);
    se += (2.0 * a.tau * a.gam / (beta * a.eps)) * sch - 2.0 * a.tau * a.gv * a.eps * a.Kz[i] * a.Phi1[i] +
          (2.0 / a.eps) * nu * (a.mus1[i] - fs);
    sv += -a.tau * a.Mz[i] * fv - a.tau * beta * a.Kz[i] * a.Phi1[i];
  }
  const double rg = block_sum(sg, sh);
  const double re = block_sum(se, sh);
  const double rv = block_sum(sv, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = re;
    part[gridDim.x + blockIdx.x] = rg;
    part[2 * gridDim.x + blockIdx.x] = rv;
  }
}

__global__ __launch_bounds__(BS) void k_adj_finish(int count, int nblk, const double* __restrict__ part,
                                                   double* __restrict__ acc) {
  __shared__ double sh[4];
  for (int i = 0; i < count; ++i) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += BS) s += part[i * nblk + b];
    s = block_sum(s, sh);
    if (threadIdx.x == 0) acc[i] += s;
  }
}

__global__ __launch_bounds__(BS) void k_dot_partial(int64_t n, const double* __restrict__ x,
                                                    const double* __restrict__ y,
                                                    double* __restrict__ part) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * BS + threadIdx.x; i < n; i += int64_t(gridDim.x) * BS)
    s += x[i] * y[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(BS) void k_dot_finish(int nblk, const double* __restrict__ part,
                                                   double coef, double* __restrict__ acc) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += BS) s += part[b];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) acc[0] += coef * s;
}

struct Ptr3 {
  const double* p[3];
};

__global__ __launch_bounds__(BS) void k_adj_p1conv(int e0, int e1, const int* __restrict__ ep1,
                                                   const int* __restrict__ ep2,
                                                   const int* __restrict__ etype, double h,
                                                   int64_t n2, Ptr3 eta, Ptr3 x, double coef,
                                                   double* __restrict__ vel_out) {
  const int e = e0 + blockIdx.x * BS + threadIdx.x;
  if (e >= e1) return;
  const ElemGeo g = elem_geo(etype[e], h);
  const int* v = ep1 + size_t(e) * 3;
  double ox[6] = {0, 0, 0, 0, 0, 0}, oy[6] = {0, 0, 0, 0, 0, 0};
  for (int t = 0; t < 3; ++t) {
    if (!eta.p[t]) continue;
    double et[3], gxv = 0.0, gyv = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      et[a] = eta.p[t][v[a]];
      const double xa = x.p[t][v[a]];
      gxv += xa * g.gx[a];
      gyv += xa * g.gy[a];
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      // int eta psi_k / |T| = sum_a eta_a int psi_k lambda_a / |T|
      double w = 0.0;
#pragma unroll
      for (int a = 0; a < 3; ++a) w += w_p2p1(k, a) * et[a];
      ox[k] += w * gxv;
      oy[k] += w * gyv;
    }
  }
  const double f = coef * g.area;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const int node = ep2[size_t(e) * 6 + k];
    vel_out[node] += f * ox[k];
    vel_out[n2 + node] += f * oy[k];
  }
}

__global__ __launch_bounds__(BS) void k_adj_ns(int e0, int e1, const int* __restrict__ ep1,
                                               const int* __restrict__ ep2,
                                               const int* __restrict__ etype, double h,
                                               DP2Tables tb, int64_t n2,
                                               const double* __restrict__ xi,
                                               const double* __restrict__ u, double rho,
                                               double alpha, const double* __restrict__ php,
                                               const double* __restrict__ phn,
                                               const double* __restrict__ Phi, double beta,
                                               double beta_v, double* __restrict__ vel_out,
                                               double* __restrict__ gmu_out,
                                               double* __restrict__ php_out,
                                               double* __restrict__ phn_out,
                                               double* __restrict__ Phi_out) {
  const int e = e0 + blockIdx.x * BS + threadIdx.x;
  if (e >= e1) return;
  const ElemGeo g = elem_geo(etype[e], h);
  const int* v = ep1 + size_t(e) * 3;
  const int* q = ep2 + size_t(e) * 6;
  double xx[6], xy[6];
  double P[6][6];  // P[m][n] = sum_c xi_c[m] u_c[n]
  {
    double ux[6], uy[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      xx[k] = xi[q[k]];
      xy[k] = xi[n2 + q[k]];
      ux[k] = u[q[k]];
      uy[k] = u[n2 + q[k]];
    }
    for (int m = 0; m < 6; ++m)
      for (int nn = 0; nn < 6; ++nn) P[m][nn] = xx[m] * ux[nn] + xy[m] * uy[nn];
  }
  // convection: d/dw_k = |T| sum_a grad lambda_a Q[k][a], Q = T3 : P;
  // constant part: |T| sum_a grad lambda_a R[a], R = T2 : P
  double R[3] = {0, 0, 0};
  for (int a = 0; a < 3; ++a)
    for (int m = 0; m < 6; ++m)
      for (int nn = 0; nn < 6; ++nn) R[a] += tb.T2[(m * 6 + nn) * 3 + a] * P[m][nn];
  for (int k = 0; k < 6; ++k) {
    double Qa[3] = {0, 0, 0};
    for (int m = 0; m < 6; ++m)
      for (int nn = 0; nn < 6; ++nn) {
        const double* t = tb.T3 + ((m * 6 + k) * 6 + nn) * 3;
        const double pv = P[m][nn];
        Qa[0] += t[0] * pv;
        Qa[1] += t[1] * pv;
        Qa[2] += t[2] * pv;
      }
    double wx = 0.0, wy = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      wx += g.gx[a] * Qa[a];
      wy += g.gy[a] * Qa[a];
    }
    vel_out[q[k]] += -rho * g.area * wx;
    vel_out[n2 + q[k]] += -rho * g.area * wy;
  }
  if (alpha != 0.0) {
    double cx = 0.0, cy = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cx += g.gx[a] * R[a];
      cy += g.gy[a] * R[a];
    }
    cx *= g.area;
    cy *= g.area;
#pragma unroll
    for (int b = 0; b < 3; ++b) gmu_out[v[b]] += alpha * (cx * g.gx[b] + cy * g.gy[b]);
  }
  // Korteweg: xi^T F = sum_{c,d} G[c][d] Y[c][d], Y[c][d] = |T| sum_k xi_c[k] sum_a TI[k][a] d_d lambda_a
  double Y[2][2] = {{0, 0}, {0, 0}};
  for (int k = 0; k < 6; ++k) {
    double ix = 0.0, iy = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      ix += tb.TI[k * 3 + a] * g.gx[a];
      iy += tb.TI[k * 3 + a] * g.gy[a];
    }
    Y[0][0] += xx[k] * ix;
    Y[0][1] += xx[k] * iy;
    Y[1][0] += xy[k] * ix;
    Y[1][1] += xy[k] * iy;
  }
  const double s00 = 2.0 * Y[0][0] * g.area, s11 = 2.0 * Y[1][1] * g.area;
  const double s01 = (Y[0][1] + Y[1][0]) * g.area;
  double gp[2] = {0, 0}, gn[2] = {0, 0}, gv[2] = {0, 0};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    gp[0] += php[v[a]] * g.gx[a];
    gp[1] += php[v[a]] * g.gy[a];
    gn[0] += phn[v[a]] * g.gx[a];
    gn[1] += phn[v[a]] * g.gy[a];
    gv[0] += Phi[v[a]] * g.gx[a];
    gv[1] += Phi[v[a]] * g.gy[a];
  }
  const double gs[2] = {-gp[0] - gn[0], -gp[1] - gn[1]};
  // (Y + Y^T) g for each field; the solvent gradient depends on phi_p and phi_N with sign -1
  auto ys = [&](const double* w, double* o) {
    o[0] = s00 * w[0] + s01 * w[1];
    o[1] = s01 * w[0] + s11 * w[1];
  };
  double yp[2], yn[2], yss[2], yv[2];
  ys(gp, yp);
  ys(gn, yn);
  ys(gs, yss);
  ys(gv, yv);
  const double dp[2] = {beta * (yp[0] - yss[0]), beta * (yp[1] - yss[1])};
  const double dn[2] = {beta * (yn[0] - yss[0]), beta * (yn[1] - yss[1])};
  const double dv[2] = {beta_v * yv[0], beta_v * yv[1]};
#pragma unroll
  for (int b = 0; b < 3; ++b) {
    php_out[v[b]] += dp[0] * g.gx[b] + dp[1] * g.gy[b];
    phn_out[v[b]] += dn[0] * g.gx[b] + dn[1] * g.gy[b];
    Phi_out[v[b]] += dv[0] * g.gx[b] + dv[1] * g.gy[b];
  }
}

}  // namespace

void gather_slots(int64_t n, const int* tmap, const double* in, double* out, hipStream_t s) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_gather_slots, dim3(ceil_div(n, BS)), dim3(BS), 0, s, n, tmap, in, out);
}

void adj_nodal(int n, const AdjNodal& a, double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_nodal, dim3(ADJ_NBLK), dim3(BS), 0, s, n, a, part);
}

void adj_finish(int count, int nblk, const double* part, double* acc, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_finish, dim3(1), dim3(BS), 0, s, count, nblk, part, acc);
}

void dot_acc(int64_t n, const double* x, const double* y, double coef, double* part, double* acc,
             hipStream_t s) {
  hipLaunchKernelGGL(k_dot_partial, dim3(ADJ_NBLK), dim3(BS), 0, s, n, x, y, part);
  hipLaunchKernelGGL(k_dot_finish, dim3(1), dim3(BS), 0, s, ADJ_NBLK, part, coef, acc);
}

void adj_p1conv(int e0, int e1, const int* ep1, const int* ep2, const int* etype, double h,
                int64_t n2, const double* const* eta, const double* const* x, double coef,
                double* vel_out, hipStream_t s) {
  if (e1 <= e0) return;
  Ptr3 pe{{eta[0], eta[1], eta[2]}}, px{{x[0], x[1], x[2]}};
  hipLaunchKernelGGL(k_adj_p1conv, dim3(ceil_div(e1 - e0, BS)), dim3(BS), 0, s, e0, e1, ep1, ep2, etype,
                     h, n2, pe, px, coef, vel_out);
}

void adj_ns(int e0, int e1, const int* ep1, const int* ep2, const int* etype, double h,
            DP2Tables tb, int64_t n2, const double* xi, const double* u, double rho, double alpha,
            const double* php, const double* phn, const double* Phi, double beta, double beta_v,
            double* vel_out, double* gmu_out, double* php_out, double* phn_out, double* Phi_out,
            hipStream_t s) {
  if (e1 <= e0) return;
  hipLaunchKernelGGL(k_adj_ns, dim3(ceil_div(e1 - e0, BS)), dim3(BS), 0, s, e0, e1, ep1, ep2, etype, h,
                     tb, n2, xi, u, rho, alpha, php, phn, Phi, beta, beta_v, vel_out, gmu_out, php_out,
                     phn_out, Phi_out);
}

}  // namespace chns
