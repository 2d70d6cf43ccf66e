// Host-only view of the mesh tables, SELL layouts and Galerkin maps that the
// library builds, exported for CPU tests of the indexing (no device code).
#include <cstdint>
#include <cstring>
#include <string>

#include "host_mesh.hpp"

using namespace chns;

namespace {

void copy_out(const std::vector<int>& v, int32_t* dst) {
  if (dst) std::memcpy(dst, v.data(), v.size() * sizeof(int));
}

// vertices of the periodic (n^2) or closed ((n+1)^2) square
int nodes(int n, bool box) { return box ? (n + 1) * (n + 1) : n * n; }

Csr p1_pattern(const Elements& E, int n, bool box) {
  const int N = nodes(n, box);
  return pattern_from_elements(N, N, E.ne, E.v.data(), 3, E.v.data(), 3);
}

Sell p1_sell(const Csr& A, int n, bool box) { return box ? make_sell_p1_box(A, n) : make_sell_p1(A, n); }

int probe_galerkin(int nf, bool box, const double* fine_csr, double* coarse_csr) {
  Elements Ef = make_elements(nf, box), Ec = make_elements(nf / 2, box);
  Csr Af = p1_pattern(Ef, nf, box), Ac = p1_pattern(Ec, nf / 2, box);
  Sell Sf = p1_sell(Af, nf, box), Sc = p1_sell(Ac, nf / 2, box);
  Csr P;
  std::vector<double> Pv;
  p1_prolongation(nf, P, Pv, box);
  std::string err;
  GalerkinMap G = make_galerkin(Af, Sf, P, Pv, Ac, Sc, &err);
  if (!err.empty()) return -1;
  std::vector<double> fs(Sf.slots(), 0.0), cs(Sc.slots(), 0.0);
  for (int64_t q = 0; q < Af.nnz(); ++q) fs[Sf.csr2sell[q]] = fine_csr[q];
  for (int64_t s = 0; s < Sc.slots(); ++s)
    for (int k = G.ptr[s]; k < G.ptr[s + 1]; ++k) cs[s] += G.w[k] * fs[G.src[k]];
  for (int64_t q = 0; q < Ac.nnz(); ++q) coarse_csr[q] = cs[Sc.csr2sell[q]];
  // slots outside the coarse pattern (padding) must receive nothing
  std::vector<char> used(Sc.slots(), 0);
  for (int64_t q = 0; q < Ac.nnz(); ++q) used[Sc.csr2sell[q]] = 1;
  for (int64_t s = 0; s < Sc.slots(); ++s)
    if (!used[s] && G.ptr[s + 1] != G.ptr[s]) return -2;
  return 0;
}

Csr cube_pattern(const Tets& T) {
  const int m = T.box ? T.n + 1 : T.n, N = m * m * m;
  return pattern_from_elements(N, N, T.ne, T.v.data(), 4, T.v.data(), 4);
}

Sell cube_sell(const Csr& A, int n, bool box) { return box ? make_sell_p1_cube_box(A, n) : make_sell_p1_cube(A, n); }

}  // namespace

extern "C" {

// The periodic cube: tetrahedra in colour order (v[ne*4], type[ne],
// colour_ptr[49]); returns ne.
__attribute__((visibility("default"))) int chns_probe_cube_tets(int n, int box, int32_t* v, int32_t* type,
                                                                int32_t* colour_ptr) {
  Tets T = make_tets(n, box != 0);
  copy_out(T.v, v);
  copy_out(T.type, type);
  if (colour_ptr) std::memcpy(colour_ptr, T.colour_ptr, sizeof(T.colour_ptr));
  return T.ne;
}

// Its P1 pattern (CSR; returns nnz) and SELL-C-64 layout as the library
// builds it: sell_col[slots], csr2sell[nnz], diag[N], flags (uniform, width,
// slots, side of the computed columns), and the 16 SELL slots of each tetrahedron (eslot[ne*16], -1 for a
// pair missing from the pattern).
__attribute__((visibility("default"))) int64_t chns_probe_cube_p1(int n, int box, int32_t* rowptr, int32_t* col,
                                                                  int32_t* sell_col, int32_t* csr2sell,
                                                                  int32_t* diag, int32_t* flags,
                                                                  int32_t* eslot) {
  Tets T = make_tets(n, box != 0);
  Csr A = cube_pattern(T);
  Sell S = cube_sell(A, n, box != 0);
  copy_out(A.rowptr, rowptr);
  copy_out(A.col, col);
  copy_out(S.col, sell_col);
  copy_out(S.csr2sell, csr2sell);
  copy_out(S.diag, diag);
  if (flags) {
    flags[0] = S.uniform;
    flags[1] = S.width_max;
    flags[2] = int(S.slots());
    flags[3] = S.cube;
  }
  if (eslot)
    for (int e = 0; e < T.ne; ++e)
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
          const int q = A.find(T.v[size_t(e) * 4 + a], T.v[size_t(e) * 4 + b]);
          eslot[size_t(e) * 16 + a * 4 + b] = q < 0 ? -1 : S.csr2sell[q];
        }
  return A.nnz();
}

// The closed cube's top-face weights int phi_i dS ((n+1)^2 values).
__attribute__((visibility("default"))) int chns_probe_cube_top_weights(int n, double h, double* w) {
  const std::vector<double> v = cube_top_weights(make_tets(n, true), h);
  if (w) std::memcpy(w, v.data(), v.size() * sizeof(double));
  return int(v.size());
}

// Nested prolongation n/2 -> n on the cube (returns nnz).
__attribute__((visibility("default"))) int chns_probe_cube_prolongation(int nf, int box, int32_t* rowptr,
                                                                        int32_t* col, double* val) {
  Csr P;
  std::vector<double> Pv;
  p1_prolongation3(nf, P, Pv, box != 0);
  copy_out(P.rowptr, rowptr);
  copy_out(P.col, col);
  if (val) std::memcpy(val, Pv.data(), Pv.size() * sizeof(double));
  return int(P.nnz());
}

// Galerkin coarsening of fine CSR values on the cube through the library's
// slot map: coarse CSR values; -1 when the map cannot be built, -2 when a
// padding slot would receive a value, -3 when a source slot is out of range.
__attribute__((visibility("default"))) int chns_probe_cube_galerkin(int nf, int box, const double* fine_csr,
                                                                    double* coarse_csr) {
  Tets Tf = make_tets(nf, box != 0), Tc = make_tets(nf / 2, box != 0);
  Csr Af = cube_pattern(Tf), Ac = cube_pattern(Tc);
  Sell Sf = cube_sell(Af, nf, box != 0), Sc = cube_sell(Ac, nf / 2, box != 0);
  Csr P;
  std::vector<double> Pv;
  p1_prolongation3(nf, P, Pv, box != 0);
  std::string err;
  GalerkinMap G = make_galerkin(Af, Sf, P, Pv, Ac, Sc, &err);
  if (!err.empty()) return -1;
  std::vector<double> fs(Sf.slots(), 0.0), cs(Sc.slots(), 0.0);
  for (int64_t q = 0; q < Af.nnz(); ++q) fs[Sf.csr2sell[q]] = fine_csr[q];
  for (int64_t s = 0; s < Sc.slots(); ++s)
    for (int k = G.ptr[s]; k < G.ptr[s + 1]; ++k) {
      if (G.src[k] < 0 || G.src[k] >= Sf.slots()) return -3;
      cs[s] += G.w[k] * fs[G.src[k]];
    }
  for (int64_t q = 0; q < Ac.nnz(); ++q) coarse_csr[q] = cs[Sc.csr2sell[q]];
  std::vector<char> used(Sc.slots(), 0);
  for (int64_t q = 0; q < Ac.nnz(); ++q) used[Sc.csr2sell[q]] = 1;
  for (int64_t s = 0; s < Sc.slots(); ++s)
    if (!used[s] && G.ptr[s + 1] != G.ptr[s]) return -2;
  return 0;
}

__attribute__((visibility("default"))) int64_t chns_probe_p1_nnz(int n) {
  Elements E = make_elements(n);
  return pattern_from_elements(n * n, n * n, E.ne, E.v.data(), 3, E.v.data(), 3).nnz();
}

// P1 pattern (CSR) and its SELL-C-64 layout: sell_col[slots], csr2sell[nnz],
// diag[N], and the flags (uniform, width).
__attribute__((visibility("default"))) int chns_probe_p1(int n, int32_t* rowptr, int32_t* col,
                                                         int32_t* sell_col, int32_t* csr2sell,
                                                         int32_t* diag, int32_t* flags) {
  Elements E = make_elements(n);
  Csr A = pattern_from_elements(n * n, n * n, E.ne, E.v.data(), 3, E.v.data(), 3);
  Sell S = make_sell_p1(A, n);
  copy_out(A.rowptr, rowptr);
  copy_out(A.col, col);
  copy_out(S.col, sell_col);
  copy_out(S.csr2sell, csr2sell);
  copy_out(S.diag, diag);
  if (flags) {
    flags[0] = S.uniform;
    flags[1] = S.width_max;
    flags[2] = int(S.slots());
  }
  return 0;
}

// Element tables in colour order: v[ne*3], p2[ne*6], type[ne], colour_ptr[9].
__attribute__((visibility("default"))) int chns_probe_elements(int n, int32_t* v, int32_t* p2,
                                                               int32_t* type, int32_t* cptr) {
  Elements E = make_elements(n);
  copy_out(E.v, v);
  copy_out(E.p2, p2);
  copy_out(E.type, type);
  if (cptr) std::memcpy(cptr, E.colour_ptr, 9 * sizeof(int));
  return 0;
}

// Apply the Galerkin map of level nf -> nf/2 to fine values given in CSR
// order; coarse values returned in CSR order.
__attribute__((visibility("default"))) int chns_probe_galerkin(int nf, const double* fine_csr,
                                                               double* coarse_csr) {
  return probe_galerkin(nf, false, fine_csr, coarse_csr);
}

// Prolongation nf -> nf/2 as CSR (rowptr[nf^2+1], col, val) and the SELL
// layout flags of P and R = P^T: flags = {P uniform, P width, R uniform, R width}.
__attribute__((visibility("default"))) int chns_probe_prolongation(int nf, int32_t* rowptr,
                                                                   int32_t* col, double* val,
                                                                   int32_t* flags) {
  Csr P, R;
  std::vector<double> Pv, Rv;
  p1_prolongation(nf, P, Pv);
  csr_transpose(P, Pv, R, Rv);
  copy_out(P.rowptr, rowptr);
  copy_out(P.col, col);
  if (val) std::memcpy(val, Pv.data(), Pv.size() * sizeof(double));
  if (flags) {
    Sell Ps = make_sell(P, 64, 1), Rs = make_sell(R, 64, 1);
    flags[0] = Ps.uniform;
    flags[1] = Ps.width_max;
    flags[2] = Rs.uniform;
    flags[3] = Rs.width_max;
  }
  return int(P.nnz());
}

// P2 reference tables, flattened in declaration order (MM, S, T3, T2, TB, TI).
__attribute__((visibility("default"))) int chns_probe_p2_tables(double* out) {
  P2Tables T = p2_tables();
  std::memcpy(out, &T, sizeof(P2Tables));
  return int(sizeof(P2Tables) / sizeof(double));
}

// Taylor-Hood patterns: which = 0 scalar P2, 1 B, 2 Oseen.  Returns nnz; fills
// rowptr/col when non-null.
__attribute__((visibility("default"))) int64_t chns_probe_th_pattern(int n, int which, int32_t* rowptr,
                                                                     int32_t* col) {
  Elements E = make_elements(n);
  Csr A = which == 0 ? p2_pattern(E) : which == 1 ? b_pattern(E) : ns_pattern(E);
  copy_out(A.rowptr, rowptr);
  copy_out(A.col, col);
  return A.nnz();
}

// The closed square [0, L]^2 ((n+1)^2 vertices i + (n+1) j): P1 pattern and
// its padded SELL layout (as chns_probe_p1, flags[3] = side), element tables
// (v, type, colour_ptr), the Galerkin map nf -> nf/2 (-2 when a padding slot
// would receive a contribution) and the prolongation (returns nnz).
__attribute__((visibility("default"))) int64_t chns_probe_box_p1_nnz(int n) {
  return p1_pattern(make_elements(n, true), n, true).nnz();
}

__attribute__((visibility("default"))) int chns_probe_box_p1(int n, int32_t* rowptr, int32_t* col,
                                                             int32_t* sell_col, int32_t* csr2sell,
                                                             int32_t* diag, int32_t* flags) {
  Csr A = p1_pattern(make_elements(n, true), n, true);
  Sell S = make_sell_p1_box(A, n);
  copy_out(A.rowptr, rowptr);
  copy_out(A.col, col);
  copy_out(S.col, sell_col);
  copy_out(S.csr2sell, csr2sell);
  copy_out(S.diag, diag);
  if (flags) {
    flags[0] = S.uniform;
    flags[1] = S.width_max;
    flags[2] = int(S.slots());
    flags[3] = S.side;
  }
  return 0;
}

__attribute__((visibility("default"))) int chns_probe_box_elements(int n, int32_t* v, int32_t* type,
                                                                   int32_t* cptr) {
  Elements E = make_elements(n, true);
  copy_out(E.v, v);
  copy_out(E.type, type);
  if (cptr) std::memcpy(cptr, E.colour_ptr, 9 * sizeof(int));
  return int(E.p2.size());
}

__attribute__((visibility("default"))) int chns_probe_box_galerkin(int nf, const double* fine_csr,
                                                                   double* coarse_csr) {
  return probe_galerkin(nf, true, fine_csr, coarse_csr);
}

__attribute__((visibility("default"))) int chns_probe_box_prolongation(int nf, int32_t* rowptr,
                                                                       int32_t* col, double* val) {
  Csr P;
  std::vector<double> Pv;
  p1_prolongation(nf, P, Pv, true);
  copy_out(P.rowptr, rowptr);
  copy_out(P.col, col);
  if (val) std::memcpy(val, Pv.data(), Pv.size() * sizeof(double));
  return int(P.nnz());
}

// Taylor-Hood patterns of the closed square (which: 0 scalar P2, 1 B, 2 Oseen;
// returns nnz), its P1 -> P2 transfer (returns nnz) and the no-slip flags.
__attribute__((visibility("default"))) int64_t chns_probe_box_th_pattern(int n, int which, int32_t* rowptr,
                                                                         int32_t* col) {
  Elements E = make_elements(n, true);
  Csr A = which == 0 ? p2_pattern(E) : which == 1 ? b_pattern(E) : ns_pattern(E);
  copy_out(A.rowptr, rowptr);
  copy_out(A.col, col);
  return A.nnz();
}

__attribute__((visibility("default"))) int chns_probe_box_p2_transfer(int n, int32_t* rowptr, int32_t* col,
                                                                      double* val) {
  Csr P;
  std::vector<double> Pv;
  p2_from_p1_prolongation(n, P, Pv, true);
  copy_out(P.rowptr, rowptr);
  copy_out(P.col, col);
  if (val) std::memcpy(val, Pv.data(), Pv.size() * sizeof(double));
  return int(P.nnz());
}

// Stored columns outside [0, ncols) in the SELL layouts of the closed
// square's P1 -> P2 transfer and of its transpose (padding included).
__attribute__((visibility("default"))) int chns_probe_box_p2_transfer_sell_bad(int n) {
  Csr P, R;
  std::vector<double> Pv, Rv;
  p2_from_p1_prolongation(n, P, Pv, true);
  csr_transpose(P, Pv, R, Rv);
  int bad = 0;
  for (const Sell& S : {make_sell(P, 64, 1), make_sell(R, 64, 1)})
    for (int col : S.col) bad += col < 0 || col >= S.ncols;
  return bad;
}

__attribute__((visibility("default"))) int chns_probe_box_p2_fixed(int n, int8_t* out) {
  const std::vector<char> f = p2_fixed_box(n);
  for (size_t i = 0; i < f.size(); ++i) out[i] = int8_t(f[i]);
  return int(f.size());
}

__attribute__((visibility("default"))) int chns_probe_box_p2_elements(int n, int32_t* p2) {
  Elements E = make_elements(n, true);
  copy_out(E.p2, p2);
  return int(E.p2.size());
}

}  // extern "C"
