// Host-side mesh tables, sparsity patterns and SELL-C-sigma layouts.
//
// Mesh: periodic square with n cells per side, each cell (i, j) split by
// its (i,j)-(i+1,j+1) diagonal into a lower triangle ((i,j),(i+1,j),(i+1,j+1))
// and an upper triangle ((i,j),(i+1,j+1),(i,j+1)).  P1 node (i, j) = i + n*j;
// P2 nodes: vertices, then horizontal, vertical and diagonal edge midpoints.
// The closed square (box) has the same cells and (n+1)^2 vertices
// i + (n+1)*j, 0 <= i, j <= n; its P2 ids pad the four blocks to (n+1)^2
// each (edge ids i + (n+1)*j with i = n, j = n, or either, name no edge).
// P2 local order on a triangle (v0, v1, v2): vertices, then the nodes of the
// edges (v1,v2), (v0,v2), (v0,v1).
//
// Elements are grouped in 8 colours, colour = (i mod 2) + 2 (j mod 2) + 4 type
// (type 0 = lower, 1 = upper); for even n no two triangles of one colour share
// a vertex or an edge, so a colour can be scattered without atomics.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace chns {

struct Csr {
  int nrows = 0, ncols = 0;
  std::vector<int> rowptr, col;
  int64_t nnz() const { return rowptr.empty() ? 0 : rowptr.back(); }
  // position of (r, c) in col[], or -1
  int find(int r, int c) const;
};

// SELL-C-sigma: rows sorted by length inside windows of sigma rows (stable,
// longest first), cut into slices of C rows; slice s stores its entries
// column-major (entry k of the slice's lane l at slice_ptr[s] + k*C + l),
// padded to the slice's longest row with value 0 and a valid column.
struct Sell {
  int nrows = 0, ncols = 0, C = 64, sigma = 1, nslices = 0, width_max = 0;
  bool uniform = false;          // every slice has width width_max and perm is identity
  std::vector<int> slice_ptr;    // nslices + 1
  std::vector<int> slice_w;      // nslices
  std::vector<int> col;          // slice_ptr[nslices]
  std::vector<int> perm;         // nslices*C: row stored at that lane position (-1 = none)
  std::vector<int> csr2sell;     // CSR entry -> SELL slot
  std::vector<int> diag;         // per row: SELL slot of the diagonal entry (-1 if absent)
  int side = 0;                  // > 0: P1 pattern of the periodic side x side mesh stored in
                                 // the fixed neighbour order of p1_offset (columns computable)
  int cube = 0;                  // > 0: P1 pattern of the periodic cube of this side in the
                                 // neighbour order of CUBE_DIRS (columns computable)
  int64_t slots() const { return slice_ptr.empty() ? 0 : slice_ptr.back(); }
};

struct Elements {
  int n = 0, ne = 0;
  std::vector<int> v;            // ne*3 P1 vertex ids, colour-sorted
  std::vector<int> p2;           // ne*6 P2 node ids (empty on the closed square)
  std::vector<int> type;         // 0 lower, 1 upper
  int colour_ptr[9] = {0};
  bool box = false;
  int nodes() const { return box ? (n + 1) * (n + 1) : n * n; }  // P1 nodes N
};

Elements make_elements(int n, bool box = false);

// Periodic unit cube with n cells per side (n even): vertex (i, j, k) has id
// i + n j + n^2 k; each cell is split into the six Kuhn tetrahedra sharing its
// main diagonal, type t taking the axes in the order KUHN_ORDER[t]: vertices
// v0, v0 + e_a, v0 + e_a + e_b, v0 + (1, 1, 1).  48 colours,
// (i mod 2) + 2 (j mod 2) + 4 (k mod 2) + 8 type: no two tetrahedra of a colour
// share a vertex.
constexpr int KUHN_ORDER[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
// Neighbour order of the cube's 15-entry P1 rows in the library's SELL
// layout: the vertex itself, then for each edge direction d of
// CUBE_DIRS the neighbours at -d and +d (entries 2m + 1 and 2m + 2).
constexpr int CUBE_DIRS[7][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}, {1, 1, 0}, {1, 0, 1}, {0, 1, 1}, {1, 1, 1}};
struct Tets {
  int n = 0, ne = 0;
  bool box = false;
  std::vector<int> v;     // ne*4 vertex ids, colour-sorted
  std::vector<int> type;  // 0..5
  int colour_ptr[49] = {0};
};
// box: the closed cube, (n+1)^3 vertices i + (n+1) j + (n+1)^2 k (no wrap;
// the same 48 colours).
Tets make_tets(int n, bool box = false);
// Closed cube: int_{z = L} phi_i dS of the top-face vertices (k = n), in the
// order i + (n+1) j, from the faces of the tetrahedra lying on that face.
std::vector<double> cube_top_weights(const Tets& T, double h);
// Nested P1 prolongation on the periodic cube from n/2 to n: coarse vertex
// (I, J, K) at fine (2I, 2J, 2K); the other fine vertices are midpoints of
// the coarse edges in the directions (a, b, c) in {0, 1}^3 (values 1 or 1/2).
void p1_prolongation3(int nf, Csr& P, std::vector<double>& val, bool box = false);
// SELL-C-64 layout of the cube's P1 pattern with entry k of every row at the
// fixed neighbour of the order above (columns computable from the row index:
// Sell::cube = n); an empty Sell when the pattern is not that stencil.
Sell make_sell_p1_cube(const Csr& A, int n);
// The closed cube's P1 pattern ((n+1)^3 rows) in the same neighbour order,
// a neighbour outside the cube stored as the row's own column (value 0);
// columns stored (Sell::cube = 0).
Sell make_sell_p1_cube_box(const Csr& A, int n);

// Node-pair pattern of an element list: rows from `rn` (per element nr ids),
// columns from `cn` (nc ids), sorted, duplicates merged.
Csr pattern_from_elements(int nrows, int ncols, int ne, const int* rn, int nr, const int* cn,
                          int nc);

Sell make_sell(const Csr& A, int C, int sigma);

// Neighbour offsets (di, dj) of a P1 row of the periodic right-diagonal mesh,
// in the storage order of make_sell_p1: self, (-1,-1), (0,-1), (-1,0), (1,0),
// (0,1), (1,1).
constexpr int P1_DI[7] = {0, -1, 0, -1, 1, 0, 1};
constexpr int P1_DJ[7] = {0, -1, -1, 0, 0, 1, 1};

// SELL-C-64 of the P1 pattern of the periodic n x n mesh (vertex i + n j) with
// entry k of every row at neighbour offset k (no padding, identity
// permutation), so a kernel can compute the columns from the row index.
Sell make_sell_p1(const Csr& A, int n);

// The same layout on the closed square with n cells per side ((n+1)^2 rows):
// a neighbour outside the square is stored as the row's own column with value
// 0 (never in the CSR pattern); side = 0, so kernels read the columns.
Sell make_sell_p1_box(const Csr& A, int n);

// Nested P1 prolongation from size n/2 to n (values: 1 or 1/2), periodic or
// on the closed square.
void p1_prolongation(int nf, Csr& P, std::vector<double>& val, bool box = false);

// Galerkin map A_c = P^T A_f P on fixed patterns: for each coarse SELL slot,
// the list of (fine SELL slot, weight).  ptr has Sc.slots()+1 entries.
struct GalerkinMap {
  std::vector<int> ptr, src;
  std::vector<double> w;
};
GalerkinMap make_galerkin(const Csr& Af, const Sell& Sf, const Csr& P, const std::vector<double>& Pv,
                          const Csr& Ac, const Sell& Sc, std::string* err);

// Transpose of a CSR pattern with values.
void csr_transpose(const Csr& A, const std::vector<double>& av, Csr& T, std::vector<double>& tv);

// P1 on mesh n into P2 on mesh n (vertex nodes copy, edge midpoints average);
// on the closed square the rows of p2_fixed_box are empty (the velocity's
// no-slip set receives no coarse correction).
void p2_from_p1_prolongation(int n, Csr& P, std::vector<double>& val, bool box = false);

// The closed square's P2 ids held at zero by the no-slip walls: the wall
// vertices and wall edges, and the ids of no edge (4 (n+1)^2 flags).
std::vector<char> p2_fixed_box(int n);

// Taylor-Hood patterns on mesh n (N = n^2 vertices, or (n+1)^2 on the closed
// square; 4N P2 ids, every row with its diagonal):
//   scalar P2 (4N x 4N), B (N x 8N: pressure rows, [x; y] velocity columns),
//   the Oseen operator (9N x 9N: rows/cols [v_x; v_y; p], no p-p block).
Csr p2_pattern(const Elements& E);
Csr b_pattern(const Elements& E);
Csr ns_pattern(const Elements& E);

// Exact integrals over a triangle T divided by |T|, in barycentric form, for
// the P2 basis psi_k (vertices, then the nodes of edges (1,2), (0,2), (0,1))
// and the P1 basis lambda_a; dpsi[k][a] = d psi_k / d lambda_a (psi written
// as a polynomial in the three barycentrics).
struct P2Tables {
  double MM[6][6];           // int psi_i psi_j
  double S[6][3][6][3];      // int dpsi[i][a] dpsi[j][b]
  double T3[6][6][6][3];     // int psi_m psi_k dpsi[n][a]
  double T2[6][6][3];        // int psi_m dpsi[n][a]
  double TB[3][6][3];        // int lambda_q dpsi[k][a]
  double TI[6][3];           // int dpsi[k][a]
  double MW[3][6][6];        // int lambda_a psi_i psi_j (P1-weighted mass)
};
P2Tables p2_tables();

}  // namespace chns
