#include "host_mesh.hpp"

#include <algorithm>
#include <cmath>
#include <array>
#include <map>
#include <numeric>

namespace chns {

int Csr::find(int r, int c) const {
  auto b = col.begin() + rowptr[r], e = col.begin() + rowptr[r + 1];
  auto it = std::lower_bound(b, e, c);
  return (it != e && *it == c) ? int(it - col.begin()) : -1;
}

Elements make_elements(int n, bool box) {
  Elements E;
  E.n = n;
  E.box = box;
  E.ne = 2 * n * n;
  const int N = E.nodes();
  auto id = [n, box](int i, int j) {
    return box ? i + (n + 1) * j : ((i % n + n) % n) + n * ((j % n + n) % n);
  };
  E.v.reserve(E.ne * 3);
  E.p2.reserve(E.ne * 6);
  E.type.reserve(E.ne);
  int count = 0;
  for (int colour = 0; colour < 8; ++colour) {
    E.colour_ptr[colour] = count;
    const int pi = colour & 1, pj = (colour >> 1) & 1, ty = colour >> 2;
    for (int j = pj; j < n; j += 2)
      for (int i = pi; i < n; i += 2) {
        const int a = id(i, j), b = id(i + 1, j), c = id(i + 1, j + 1), d = id(i, j + 1);
        if (ty == 0) {
          const int loc[3] = {a, b, c};
          const int e2[3] = {2 * N + id(i + 1, j), 3 * N + id(i, j), N + id(i, j)};
          E.v.insert(E.v.end(), loc, loc + 3);
          E.p2.insert(E.p2.end(), loc, loc + 3);
          E.p2.insert(E.p2.end(), e2, e2 + 3);
        } else {
          const int loc[3] = {a, c, d};
          const int e2[3] = {N + id(i, j + 1), 2 * N + id(i, j), 3 * N + id(i, j)};
          E.v.insert(E.v.end(), loc, loc + 3);
          E.p2.insert(E.p2.end(), loc, loc + 3);
          E.p2.insert(E.p2.end(), e2, e2 + 3);
        }
        E.type.push_back(ty);
        ++count;
      }
  }
  E.colour_ptr[8] = count;
  return E;
}

Tets make_tets(int n, bool box) {
  Tets T;
  T.n = n;
  T.box = box;
  T.ne = 6 * n * n * n;
  const int m = box ? n + 1 : n;
  auto id = [n, m, box](int i, int j, int k) {
    if (box) return i + m * j + m * m * k;
    return ((i % n + n) % n) + n * ((j % n + n) % n) + n * n * ((k % n + n) % n);
  };
  T.v.reserve(size_t(T.ne) * 4);
  T.type.reserve(T.ne);
  int count = 0;
  for (int colour = 0; colour < 48; ++colour) {
    T.colour_ptr[colour] = count;
    const int pi = colour & 1, pj = (colour >> 1) & 1, pk = (colour >> 2) & 1, ty = colour >> 3;
    for (int k = pk; k < n; k += 2)
      for (int j = pj; j < n; j += 2)
        for (int i = pi; i < n; i += 2) {
          int o[3] = {i, j, k};
          T.v.push_back(id(o[0], o[1], o[2]));
          for (int s = 0; s < 3; ++s) {
            ++o[KUHN_ORDER[ty][s]];
            T.v.push_back(id(o[0], o[1], o[2]));
          }
          T.type.push_back(ty);
          ++count;
        }
  }
  T.colour_ptr[48] = count;
  return T;
}

void p1_prolongation3(int nf, Csr& P, std::vector<double>& val, bool box) {
  const int nc = nf / 2;
  // vertices per side: n on the periodic cube, n + 1 on the closed one
  const int mf = box ? nf + 1 : nf, mc = box ? nc + 1 : nc;
  auto fid = [nf, mf, box](int i, int j, int k) {
    if (box) return i + mf * j + mf * mf * k;
    return ((i % nf + nf) % nf) + nf * ((j % nf + nf) % nf) + nf * nf * ((k % nf + nf) % nf);
  };
  auto cid = [nc, mc, box](int i, int j, int k) {
    if (box) return i + mc * j + mc * mc * k;
    return ((i % nc + nc) % nc) + nc * ((j % nc + nc) % nc) + nc * nc * ((k % nc + nc) % nc);
  };
  const int64_t Nf = int64_t(mf) * mf * mf;
  std::vector<std::vector<std::pair<int, double>>> rows(Nf);
  for (int K = 0; K < mc; ++K)
    for (int J = 0; J < mc; ++J)
      for (int I = 0; I < mc; ++I)
        for (int d = 0; d < 8; ++d) {
          const int a = d & 1, b = (d >> 1) & 1, c = (d >> 2) & 1;
          // closed cube: the midpoints of edges leaving the last coarse layer do not exist
          if (box && ((a && I == nc) || (b && J == nc) || (c && K == nc))) continue;
          auto& row = rows[fid(2 * I + a, 2 * J + b, 2 * K + c)];
          if (d == 0) {
            row.push_back({cid(I, J, K), 1.0});
          } else {
            row.push_back({cid(I, J, K), 0.5});
            row.push_back({cid(I + a, J + b, K + c), 0.5});
          }
        }
  P.nrows = int(Nf);
  P.ncols = mc * mc * mc;
  P.rowptr.assign(P.nrows + 1, 0);
  P.col.clear();
  val.clear();
  for (int r = 0; r < P.nrows; ++r) {
    auto& row = rows[r];
    std::sort(row.begin(), row.end());
    for (auto& e : row) {
      P.col.push_back(e.first);
      val.push_back(e.second);
    }
    P.rowptr[r + 1] = int(P.col.size());
  }
}

Sell make_sell_p1_cube(const Csr& A, int n) {
  Sell S;
  const int N = n * n * n;
  constexpr int W = 15;
  S.nrows = N;
  S.ncols = N;
  S.C = 64;
  S.sigma = 1;
  S.cube = n;
  S.nslices = (N + 63) / 64;
  S.width_max = W;
  S.uniform = true;
  S.perm.assign(size_t(S.nslices) * 64, -1);
  for (int r = 0; r < N; ++r) S.perm[r] = r;
  S.slice_ptr.resize(S.nslices + 1);
  for (int s = 0; s <= S.nslices; ++s) S.slice_ptr[s] = s * 64 * W;
  S.slice_w.assign(S.nslices, W);
  S.col.assign(size_t(S.nslices) * 64 * W, 0);
  S.csr2sell.assign(A.nnz(), -1);
  S.diag.assign(N, -1);
  auto wrap = [n](int a) { return ((a % n) + n) % n; };
  auto neighbour = [&](int r, int k) {
    const int i = r % n, j = (r / n) % n, l = r / (n * n);
    if (k == 0) return r;
    const int* d = CUBE_DIRS[(k - 1) / 2];
    const int sg = (k % 2 == 1) ? -1 : 1;
    return wrap(i + sg * d[0]) + n * wrap(j + sg * d[1]) + n * n * wrap(l + sg * d[2]);
  };
  for (int r = 0; r < S.nslices * 64; ++r)
    for (int k = 0; k < W; ++k)  // padding lanes of a partial slice: column 0, value 0
      S.col[size_t(r >> 6) * 64 * W + k * 64 + (r & 63)] = r < N ? neighbour(r, k) : 0;
  for (int r = 0; r < N; ++r)
    for (int q = A.rowptr[r]; q < A.rowptr[r + 1]; ++q) {
      int k = -1;
      for (int t = 0; t < W; ++t)
        if (neighbour(r, t) == A.col[q]) k = t;
      if (k < 0) return Sell{};  // not the 15-point stencil
      const int slot = (r >> 6) * 64 * W + k * 64 + (r & 63);
      S.csr2sell[q] = slot;
      if (A.col[q] == r) S.diag[r] = slot;
    }
  return S;
}

Sell make_sell_p1_cube_box(const Csr& A, int n) {
  Sell S;
  const int m = n + 1, N = m * m * m;
  constexpr int W = 15;
  S.nrows = N;
  S.ncols = N;
  S.C = 64;
  S.sigma = 1;
  S.cube = 0;  // columns are stored, not computed
  S.nslices = (N + 63) / 64;
  S.width_max = W;
  S.uniform = true;
  S.perm.assign(size_t(S.nslices) * 64, -1);
  for (int r = 0; r < N; ++r) S.perm[r] = r;
  S.slice_ptr.resize(S.nslices + 1);
  for (int s = 0; s <= S.nslices; ++s) S.slice_ptr[s] = s * 64 * W;
  S.slice_w.assign(S.nslices, W);
  S.col.assign(size_t(S.nslices) * 64 * W, 0);
  S.csr2sell.assign(A.nnz(), -1);
  S.diag.assign(N, -1);
  // neighbour k of row r, or -1 outside the cube
  auto neighbour = [m](int r, int k) {
    if (k == 0) return r;
    const int i = r % m, j = (r / m) % m, l = r / (m * m);
    const int* d = CUBE_DIRS[(k - 1) / 2];
    const int sg = (k % 2 == 1) ? -1 : 1;
    const int a = i + sg * d[0], b = j + sg * d[1], c = l + sg * d[2];
    if (a < 0 || a >= m || b < 0 || b >= m || c < 0 || c >= m) return -1;
    return a + m * b + m * m * c;
  };
  for (int r = 0; r < S.nslices * 64; ++r)
    for (int k = 0; k < W; ++k) {
      // padding lanes of a partial slice: column 0; a missing neighbour: the row itself
      const int c = r < N ? neighbour(r, k) : 0;
      S.col[size_t(r >> 6) * 64 * W + k * 64 + (r & 63)] = c < 0 ? r : c;
    }
  for (int r = 0; r < N; ++r)
    for (int q = A.rowptr[r]; q < A.rowptr[r + 1]; ++q) {
      int k = -1;
      for (int t = 0; t < W; ++t)
        if (neighbour(r, t) == A.col[q]) k = t;
      if (k < 0) return Sell{};  // not the 15-point stencil
      const int slot = (r >> 6) * 64 * W + k * 64 + (r & 63);
      S.csr2sell[q] = slot;
      if (A.col[q] == r) S.diag[r] = slot;
    }
  return S;
}

std::vector<double> cube_top_weights(const Tets& T, double h) {
  const int n = T.n, m = n + 1;
  std::vector<double> w(size_t(m) * m, 0.0);
  const int top0 = n * m * m;  // first vertex of the layer k = n
  for (int e = 0; e < T.ne; ++e) {
    int on[4], cnt = 0;
    for (int a = 0; a < 4; ++a) {
      const int v = T.v[size_t(e) * 4 + a];
      if (v >= top0) on[cnt++] = v;
    }
    if (cnt != 3) continue;
    // the face's corners in the layer's (i, j) coordinates, area by the cross product
    double xy[3][2];
    for (int t = 0; t < 3; ++t) {
      const int q = on[t] - top0;
      xy[t][0] = (q % m) * h;
      xy[t][1] = (q / m) * h;
    }
    const double area = 0.5 * std::fabs((xy[1][0] - xy[0][0]) * (xy[2][1] - xy[0][1]) -
                                        (xy[2][0] - xy[0][0]) * (xy[1][1] - xy[0][1]));
    for (int t = 0; t < 3; ++t) w[on[t] - top0] += area / 3.0;
  }
  return w;
}

Csr pattern_from_elements(int nrows, int ncols, int ne, const int* rn, int nr, const int* cn,
                          int nc) {
  std::vector<std::vector<int>> rows(nrows);
  for (int e = 0; e < ne; ++e)
    for (int a = 0; a < nr; ++a)
      for (int b = 0; b < nc; ++b) rows[rn[e * nr + a]].push_back(cn[e * nc + b]);
  Csr A;
  A.nrows = nrows;
  A.ncols = ncols;
  A.rowptr.assign(nrows + 1, 0);
  for (int r = 0; r < nrows; ++r) {
    auto& v = rows[r];
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    A.rowptr[r + 1] = A.rowptr[r] + int(v.size());
  }
  A.col.reserve(A.rowptr[nrows]);
  for (int r = 0; r < nrows; ++r) A.col.insert(A.col.end(), rows[r].begin(), rows[r].end());
  return A;
}

Sell make_sell_p1(const Csr& A, int n) {
  Sell S;
  const int N = n * n;
  S.nrows = N;
  S.ncols = N;
  S.C = 64;
  S.sigma = 1;
  S.side = n;
  S.nslices = (N + 63) / 64;
  S.width_max = 7;
  S.uniform = true;
  S.perm.assign(size_t(S.nslices) * 64, -1);
  for (int r = 0; r < N; ++r) S.perm[r] = r;
  S.slice_ptr.resize(S.nslices + 1);
  for (int s = 0; s <= S.nslices; ++s) S.slice_ptr[s] = s * 448;
  S.slice_w.assign(S.nslices, 7);
  S.col.assign(size_t(S.nslices) * 448, 0);
  S.csr2sell.assign(A.nnz(), -1);
  S.diag.assign(N, -1);
  for (int r = 0; r < S.nslices * 64; ++r) {
    const int rr = r < N ? r : 0;  // padding lanes of a partial slice: valid column, value 0
    const int i = rr % n, j = rr / n;
    for (int k = 0; k < 7; ++k) {
      const int ci = (i + P1_DI[k] + n) % n, cj = (j + P1_DJ[k] + n) % n;
      S.col[size_t(r >> 6) * 448 + k * 64 + (r & 63)] = ci + n * cj;
    }
  }
  for (int r = 0; r < N; ++r) {
    const int i = r % n, j = r / n;
    for (int q = A.rowptr[r]; q < A.rowptr[r + 1]; ++q) {
      const int c = A.col[q], ci = c % n, cj = c / n;
      const int di = (ci - i + n + 1) % n - 1, dj = (cj - j + n + 1) % n - 1;
      int k = -1;
      for (int t = 0; t < 7; ++t)
        if (P1_DI[t] == di && P1_DJ[t] == dj) k = t;
      if (k < 0) return Sell{};  // not the periodic 7-point pattern
      const int slot = (r >> 6) * 448 + k * 64 + (r & 63);
      S.csr2sell[q] = slot;
      if (c == r) S.diag[r] = slot;
    }
  }
  return S;
}

Sell make_sell(const Csr& A, int C, int sigma) {
  Sell S;
  S.nrows = A.nrows;
  S.ncols = A.ncols;
  S.C = C;
  S.sigma = sigma;
  S.nslices = (A.nrows + C - 1) / C;
  const int npos = S.nslices * C;
  std::vector<int> order(A.nrows);
  std::iota(order.begin(), order.end(), 0);
  auto len = [&](int r) { return A.rowptr[r + 1] - A.rowptr[r]; };
  if (sigma > 1)
    for (int w0 = 0; w0 < A.nrows; w0 += sigma) {
      const int w1 = std::min(A.nrows, w0 + sigma);
      std::stable_sort(order.begin() + w0, order.begin() + w1,
                       [&](int x, int y) { return len(x) > len(y); });
    }
  S.perm.assign(npos, -1);
  for (int p = 0; p < A.nrows; ++p) S.perm[p] = order[p];
  S.slice_ptr.assign(S.nslices + 1, 0);
  S.slice_w.assign(S.nslices, 0);
  for (int s = 0; s < S.nslices; ++s) {
    int w = 0;
    for (int l = 0; l < C; ++l) {
      const int r = S.perm[s * C + l];
      if (r >= 0) w = std::max(w, len(r));
    }
    S.slice_w[s] = w;
    S.slice_ptr[s + 1] = S.slice_ptr[s] + w * C;
    S.width_max = std::max(S.width_max, w);
  }
  S.col.assign(S.slice_ptr[S.nslices], 0);
  S.csr2sell.assign(A.nnz(), -1);
  S.diag.assign(A.nrows, -1);
  bool uniform = true;
  for (int s = 0; s < S.nslices; ++s) {
    if (S.slice_w[s] != S.width_max) uniform = false;
    for (int l = 0; l < C; ++l) {
      const int p = s * C + l, r = S.perm[p];
      if (r >= 0 && r != p) uniform = false;
      for (int k = 0; k < S.slice_w[s]; ++k) {
        const int slot = S.slice_ptr[s] + k * C + l;
        if (r < 0) {
          S.col[slot] = 0;
          continue;
        }
        const int L = len(r);
        if (k < L) {
          const int q = A.rowptr[r] + k;
          S.col[slot] = A.col[q];
          S.csr2sell[q] = slot;
          if (A.col[q] == r) S.diag[r] = slot;
        } else {
          // padding: a valid column (the row's first, or 0 for an empty row), value stays 0
          S.col[slot] = L > 0 ? A.col[A.rowptr[r]] : 0;
        }
      }
    }
  }
  S.uniform = uniform;
  return S;
}

Sell make_sell_p1_box(const Csr& A, int n) {
  Sell S;
  const int m = n + 1, N = m * m;
  S.nrows = N;
  S.ncols = N;
  S.C = 64;
  S.sigma = 1;
  S.side = 0;  // columns are stored, not computed
  S.nslices = (N + 63) / 64;
  S.width_max = 7;
  S.uniform = true;
  S.perm.assign(size_t(S.nslices) * 64, -1);
  for (int r = 0; r < N; ++r) S.perm[r] = r;
  S.slice_ptr.resize(S.nslices + 1);
  for (int s = 0; s <= S.nslices; ++s) S.slice_ptr[s] = s * 448;
  S.slice_w.assign(S.nslices, 7);
  S.col.assign(size_t(S.nslices) * 448, 0);
  S.csr2sell.assign(A.nnz(), -1);
  S.diag.assign(N, -1);
  for (int r = 0; r < S.nslices * 64; ++r) {
    const bool pad = r >= N;  // padding lanes of a partial slice: column 0, value 0
    const int i = r % m, j = r / m;
    for (int k = 0; k < 7; ++k) {
      const int ci = i + P1_DI[k], cj = j + P1_DJ[k];
      const bool in = !pad && ci >= 0 && ci < m && cj >= 0 && cj < m;
      // a neighbour outside the square: the row's own column, value 0
      S.col[size_t(r >> 6) * 448 + k * 64 + (r & 63)] = pad ? 0 : (in ? ci + m * cj : r);
    }
  }
  for (int r = 0; r < N; ++r) {
    const int i = r % m, j = r / m;
    for (int q = A.rowptr[r]; q < A.rowptr[r + 1]; ++q) {
      const int c = A.col[q], di = c % m - i, dj = c / m - j;
      int k = -1;
      for (int t = 0; t < 7; ++t)
        if (P1_DI[t] == di && P1_DJ[t] == dj) k = t;
      if (k < 0) return Sell{};  // not the 7-point pattern
      const int slot = (r >> 6) * 448 + k * 64 + (r & 63);
      S.csr2sell[q] = slot;
      if (c == r) S.diag[r] = slot;
    }
  }
  return S;
}

void p1_prolongation(int nf, Csr& P, std::vector<double>& val, bool box) {
  const int nc = nf / 2;
  // vertices per side: n on the periodic square, n + 1 on the closed one
  const int vf = box ? nf + 1 : nf, vc = box ? nc + 1 : nc;
  auto fid = [nf, vf, box](int i, int j) {
    return box ? i + vf * j : ((i % nf + nf) % nf) + nf * ((j % nf + nf) % nf);
  };
  auto cid = [nc, vc, box](int i, int j) {
    return box ? i + vc * j : ((i % nc + nc) % nc) + nc * ((j % nc + nc) % nc);
  };
  std::vector<std::vector<std::pair<int, double>>> rows(size_t(vf) * vf);
  for (int J = 0; J < vc; ++J)
    for (int I = 0; I < vc; ++I) {
      rows[fid(2 * I, 2 * J)].push_back({cid(I, J), 1.0});
      const int d[3][2] = {{1, 0}, {0, 1}, {1, 1}};
      for (auto& o : d) {
        // on the closed square the last coarse row and column have no
        // midpoints beyond them
        if (box && ((o[0] && I == nc) || (o[1] && J == nc))) continue;
        auto& row = rows[fid(2 * I + o[0], 2 * J + o[1])];
        row.push_back({cid(I, J), 0.5});
        row.push_back({cid(I + o[0], J + o[1]), 0.5});
      }
    }
  P.nrows = vf * vf;
  P.ncols = vc * vc;
  P.rowptr.assign(P.nrows + 1, 0);
  P.col.clear();
  val.clear();
  for (int r = 0; r < P.nrows; ++r) {
    auto& row = rows[r];
    std::sort(row.begin(), row.end());
    for (auto& e : row) {
      P.col.push_back(e.first);
      val.push_back(e.second);
    }
    P.rowptr[r + 1] = int(P.col.size());
  }
}

GalerkinMap make_galerkin(const Csr& Af, const Sell& Sf, const Csr& P, const std::vector<double>& Pv,
                          const Csr& Ac, const Sell& Sc, std::string* err) {
  // contributions to coarse entry (I, J) from fine entry (a, b): P[a,I] P[b,J]
  std::vector<std::vector<std::pair<int, double>>> lists(Sc.slots());
  for (int a = 0; a < Af.nrows; ++a)
    for (int q = Af.rowptr[a]; q < Af.rowptr[a + 1]; ++q) {
      const int b = Af.col[q];
      const int fslot = Sf.csr2sell[q];
      for (int pa = P.rowptr[a]; pa < P.rowptr[a + 1]; ++pa)
        for (int pb = P.rowptr[b]; pb < P.rowptr[b + 1]; ++pb) {
          const int I = P.col[pa], J = P.col[pb];
          const int cq = Ac.find(I, J);
          if (cq < 0) {
            if (err) *err = "Galerkin product leaves the coarse pattern";
            return {};
          }
          lists[Sc.csr2sell[cq]].push_back({fslot, Pv[pa] * Pv[pb]});
        }
    }
  GalerkinMap G;
  G.ptr.assign(Sc.slots() + 1, 0);
  for (size_t s = 0; s < lists.size(); ++s) {
    auto& l = lists[s];
    std::sort(l.begin(), l.end());  // fixed summation order
    G.ptr[s + 1] = G.ptr[s] + int(l.size());
    for (auto& e : l) {
      G.src.push_back(e.first);
      G.w.push_back(e.second);
    }
  }
  return G;
}

void csr_transpose(const Csr& A, const std::vector<double>& av, Csr& T, std::vector<double>& tv) {
  T.nrows = A.ncols;
  T.ncols = A.nrows;
  T.rowptr.assign(T.nrows + 1, 0);
  for (int c : A.col) T.rowptr[c + 1]++;
  for (int r = 0; r < T.nrows; ++r) T.rowptr[r + 1] += T.rowptr[r];
  T.col.assign(A.nnz(), 0);
  tv.assign(A.nnz(), 0.0);
  std::vector<int> fill(T.rowptr.begin(), T.rowptr.end() - 1);
  for (int r = 0; r < A.nrows; ++r)
    for (int q = A.rowptr[r]; q < A.rowptr[r + 1]; ++q) {
      const int p = fill[A.col[q]]++;
      T.col[p] = r;
      tv[p] = av[q];
    }
}

void p2_from_p1_prolongation(int n, Csr& P, std::vector<double>& val, bool box) {
  const int m = box ? n + 1 : n, N = m * m;
  auto id = [n, m, box](int i, int j) { return box ? i + m * j : ((i % n + n) % n) + n * ((j % n + n) % n); };
  P.nrows = 4 * N;
  P.ncols = N;
  P.rowptr.assign(P.nrows + 1, 0);
  P.col.clear();
  val.clear();
  std::vector<std::vector<std::pair<int, double>>> rows(P.nrows);
  const std::vector<char> fixed = box ? p2_fixed_box(n) : std::vector<char>(size_t(4) * N, 0);
  for (int j = 0; j < m; ++j)
    for (int i = 0; i < m; ++i) {
      if (!fixed[id(i, j)]) rows[id(i, j)].push_back({id(i, j), 1.0});
      const int d[3][2] = {{1, 0}, {0, 1}, {1, 1}};
      for (int blk = 0; blk < 3; ++blk) {
        const int r = (blk + 1) * N + id(i, j);
        if (fixed[r]) continue;  // a wall node or an id of no edge: no interpolation
        rows[r].push_back({id(i, j), 0.5});
        rows[r].push_back({id(i + d[blk][0], j + d[blk][1]), 0.5});
      }
    }
  for (int r = 0; r < P.nrows; ++r) {
    auto& row = rows[r];
    std::sort(row.begin(), row.end());
    for (auto& e : row) {
      P.col.push_back(e.first);
      val.push_back(e.second);
    }
    P.rowptr[r + 1] = int(P.col.size());
  }
}

std::vector<char> p2_fixed_box(int n) {
  const int m = n + 1, N = m * m;
  std::vector<char> f(size_t(4) * N, 0);
  for (int j = 0; j < m; ++j)
    for (int i = 0; i < m; ++i) {
      const bool side = i == 0 || i == n, tb = j == 0 || j == n;
      const int v = i + m * j;
      f[v] = side || tb;                           // wall vertices
      f[N + v] = i == n || tb;                     // (i,j)-(i+1,j): none at i = n, walls at j = 0, n
      f[2 * N + v] = j == n || side;               // (i,j)-(i,j+1): none at j = n, walls at i = 0, n
      f[3 * N + v] = i == n || j == n;             // diagonals: none on the last row or column
    }
  return f;
}

// Every row keeps its diagonal entry, also a row no element touches (the
// unused ids of the closed square's padded P2 numbering).
static Csr with_diagonal(const Csr& A) {
  Csr B;
  B.nrows = A.nrows;
  B.ncols = A.ncols;
  B.rowptr.assign(A.nrows + 1, 0);
  for (int r = 0; r < A.nrows; ++r) {
    const int* b = A.col.data() + A.rowptr[r];
    const int* e = A.col.data() + A.rowptr[r + 1];
    const bool has = std::binary_search(b, e, r);
    for (const int* q = b; q < e; ++q) {
      if (!has && *q > r && (q == b || q[-1] < r)) B.col.push_back(r);
      B.col.push_back(*q);
    }
    if (!has && (b == e || e[-1] < r)) B.col.push_back(r);
    B.rowptr[r + 1] = int(B.col.size());
  }
  return B;
}

Csr p2_pattern(const Elements& E) {
  const int N = E.nodes();
  return with_diagonal(pattern_from_elements(4 * N, 4 * N, E.ne, E.p2.data(), 6, E.p2.data(), 6));
}

Csr b_pattern(const Elements& E) {
  const int N = E.nodes();
  std::vector<int> vel(size_t(E.ne) * 12);
  for (int e = 0; e < E.ne; ++e)
    for (int k = 0; k < 6; ++k) {
      vel[size_t(e) * 12 + k] = E.p2[e * 6 + k];
      vel[size_t(e) * 12 + 6 + k] = 4 * N + E.p2[e * 6 + k];
    }
  return pattern_from_elements(N, 8 * N, E.ne, E.v.data(), 3, vel.data(), 12);
}

Csr ns_pattern(const Elements& E) {
  // velocity rows couple to both velocity components and to pressure;
  // pressure rows couple to both velocity components only; a velocity row no
  // element touches keeps its diagonal.
  const int N = E.nodes();
  std::vector<std::vector<int>> rows(9 * N);
  for (int r = 0; r < 8 * N; ++r) rows[r].push_back(r);
  for (int e = 0; e < E.ne; ++e) {
    const int* q = &E.p2[e * 6];
    const int* v = &E.v[e * 3];
    for (int c = 0; c < 2; ++c)
      for (int a = 0; a < 6; ++a) {
        auto& r = rows[c * 4 * N + q[a]];
        for (int d = 0; d < 2; ++d)
          for (int b = 0; b < 6; ++b) r.push_back(d * 4 * N + q[b]);
        for (int b = 0; b < 3; ++b) r.push_back(8 * N + v[b]);
      }
    for (int a = 0; a < 3; ++a) {
      auto& r = rows[8 * N + v[a]];
      for (int d = 0; d < 2; ++d)
        for (int b = 0; b < 6; ++b) r.push_back(d * 4 * N + q[b]);
    }
  }
  Csr A;
  A.nrows = A.ncols = 9 * N;
  A.rowptr.assign(A.nrows + 1, 0);
  for (int r = 0; r < A.nrows; ++r) {
    auto& v = rows[r];
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    A.rowptr[r + 1] = A.rowptr[r] + int(v.size());
  }
  for (auto& v : rows) A.col.insert(A.col.end(), v.begin(), v.end());
  return A;
}

namespace {

// Polynomials in the barycentrics (l0, l1, l2), integrated over a triangle by
// int l0^a l1^b l2^c = 2|T| a! b! c! / (a+b+c+2)!.
using Mono = std::array<int, 3>;
using Poly = std::map<Mono, double>;

Poly mul(const Poly& p, const Poly& q) {
  Poly r;
  for (auto& [mp, cp] : p)
    for (auto& [mq, cq] : q) r[{mp[0] + mq[0], mp[1] + mq[1], mp[2] + mq[2]}] += cp * cq;
  return r;
}

double fact(int k) {
  double f = 1;
  for (int i = 2; i <= k; ++i) f *= i;
  return f;
}

double integrate(const Poly& p) {  // divided by |T|
  double s = 0;
  for (auto& [m, c] : p) s += c * 2.0 * fact(m[0]) * fact(m[1]) * fact(m[2]) / fact(m[0] + m[1] + m[2] + 2);
  return s;
}

Poly lam(int a) {
  Mono m{0, 0, 0};
  m[a] = 1;
  return Poly{{m, 1.0}};
}

}  // namespace

P2Tables p2_tables() {
  // psi_k and d psi_k / d lambda_a as polynomials
  Poly psi[6], dpsi[6][3];
  const int edge[3][2] = {{1, 2}, {0, 2}, {0, 1}};
  for (int k = 0; k < 3; ++k) {
    Poly p = mul(lam(k), lam(k));
    for (auto& t : p) t.second *= 2.0;
    p[{k == 0, k == 1, k == 2}] -= 1.0;  // 2 l_k^2 - l_k
    psi[k] = p;
    for (int a = 0; a < 3; ++a) {
      Poly d;
      if (a == k) {
        d = lam(k);
        for (auto& t : d) t.second *= 4.0;
        d[{0, 0, 0}] = -1.0;  // 4 l_k - 1
      }
      dpsi[k][a] = d;
    }
  }
  for (int e = 0; e < 3; ++e) {
    const int k = edge[e][0], l = edge[e][1];
    Poly p = mul(lam(k), lam(l));
    for (auto& t : p) t.second *= 4.0;
    psi[3 + e] = p;
    for (int a = 0; a < 3; ++a) {
      Poly d;
      if (a == k) d = lam(l);
      if (a == l) d = lam(k);
      for (auto& t : d) t.second *= 4.0;
      dpsi[3 + e][a] = d;
    }
  }
  P2Tables T{};
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) T.MM[i][j] = integrate(mul(psi[i], psi[j]));
  for (int i = 0; i < 6; ++i)
    for (int a = 0; a < 3; ++a)
      for (int j = 0; j < 6; ++j)
        for (int b = 0; b < 3; ++b) T.S[i][a][j][b] = integrate(mul(dpsi[i][a], dpsi[j][b]));
  for (int m = 0; m < 6; ++m)
    for (int k = 0; k < 6; ++k) {
      const Poly pk = mul(psi[m], psi[k]);
      for (int n = 0; n < 6; ++n)
        for (int a = 0; a < 3; ++a) T.T3[m][k][n][a] = integrate(mul(pk, dpsi[n][a]));
    }
  for (int m = 0; m < 6; ++m)
    for (int n = 0; n < 6; ++n)
      for (int a = 0; a < 3; ++a) T.T2[m][n][a] = integrate(mul(psi[m], dpsi[n][a]));
  for (int q = 0; q < 3; ++q)
    for (int k = 0; k < 6; ++k)
      for (int a = 0; a < 3; ++a) T.TB[q][k][a] = integrate(mul(lam(q), dpsi[k][a]));
  for (int k = 0; k < 6; ++k)
    for (int a = 0; a < 3; ++a) T.TI[k][a] = integrate(dpsi[k][a]);
  for (int a = 0; a < 3; ++a)
    for (int i = 0; i < 6; ++i)
      for (int j = 0; j < 6; ++j) T.MW[a][i][j] = integrate(mul(lam(a), mul(psi[i], psi[j])));
  return T;
}

}  // namespace chns
