// Launchers of the adjoint kernels (definitions in kernels_adj.hip): the
// transposition of values stored on a symmetric pattern, the nodal adjoint of
// the explicit ternary terms with the parameter-derivative integrands, the
// element vector-Jacobian products of the P1 convection, the Oseen convection
// and the Korteweg load, and deterministic dot products.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace chns {

// out[q] = in[tmap[q]]: tmap[q] is the slot of the transposed entry of slot q
// (padding slots map to themselves).
void gather_slots(int64_t n, const int* tmap, const double* in, double* out, hipStream_t s);

// Nodal part of one adjoint step of the ternary scheme (all arrays P1, n).
// State k: php, phn, Phi.  State k+1: php1, phn1, mup1, mun1, mus1, Phi1.
// Adjoint solutions mapped by M and K: Me1p/Me1n = M eta_i (phi rows),
// Me2p/Me2n = M eta_i (mu rows), Ke1p/Ke1n, Ke2p/Ke2n likewise with K,
// Mz = M zeta, Kz = K zeta; nus = adjoint of mu_s^{k+1}.
// Writes lam_php, lam_phn, lam_Phi (= M eta_i1 / M zeta plus the Hessian
// terms of f', f_v' and the closure density) and per-block partial sums of
// the integrands of dL/d(eps, mobility, evaporation rate) into part[3][nblk].
struct AdjNodal {
  const double *php, *phn, *Phi;
  const double *php1, *phn1, *mup1, *mun1, *mus1, *Phi1;
  const double *Me1p, *Me1n, *Me2p, *Me2n, *Ke1p, *Ke1n, *Ke2p, *Ke2n, *Mz, *Kz, *nus;
  double *lam_php, *lam_phn, *lam_Phi;
  double eps, tau, gam, gv;
  PotCoef pc;  // the ternary density
};
constexpr int ADJ_NBLK = 512;  // fixed grid of the reductions (deterministic order)
void adj_nodal(int n, const AdjNodal& a, double* part, hipStream_t s);
// acc[i] += sum_b part[i * nblk + b] for i < count (one workgroup).
void adj_finish(int count, int nblk, const double* part, double* acc, hipStream_t s);
// acc[0] += coef * x . y (partials in part[ADJ_NBLK]).
void dot_acc(int64_t n, const double* x, const double* y, double coef, double* part, double* acc,
             hipStream_t s);

// vel_out (2 x n2, P2 nodes) += coef * d/dv [sum_t eta_t^T C(v) x_t] over one
// colour [e0, e1); C_ij = int (v . grad phi_j) phi_i; up to three (eta, x)
// pairs, unused ones null.
void adj_p1conv(int e0, int e1, const int* ep1, const int* ep2, const int* etype, double h,
                int64_t n2, const double* const* eta, const double* const* x, double coef,
                double* vel_out, hipStream_t s);

// Oseen part of one adjoint step over one colour, with xi the velocity part
// of the transposed Oseen solve and u = v^{k+1}:
//   vel_out += -rho d/dw [sum_c xi_c^T J(w) u_c]   (w = rho v^k + w_const)
//   gmu_out += alpha grad^T(d/dw_const [...])      (w_const = -alpha sum grad mu_i)
//   php_out, phn_out, Phi_out += d/dphi [xi^T F(phi^k, Phi^k)] (Korteweg load)
void adj_ns(int e0, int e1, const int* ep1, const int* ep2, const int* etype, double h,
            DP2Tables tb, int64_t n2, const double* xi, const double* u, double rho, double alpha,
            const double* php, const double* phn, const double* Phi, double beta, double beta_v,
            double* vel_out, double* gmu_out, double* php_out, double* phn_out, double* Phi_out,
            hipStream_t s);

}  // namespace chns
