#include "host_mesh.hpp"

#include <algorithm>
#include <numeric>

namespace chns {

int Csr::find(int r, int c) const {
  auto b = col.begin() + rowptr[r], e = col.begin() + rowptr[r + 1];
  auto it = std::lower_bound(b, e, c);
  return (it != e && *it == c) ? int(it - col.begin()) : -1;
}

Elements make_elements(int n) {
  Elements E;
  E.n = n;
  E.ne = 2 * n * n;
  const int N = n * n;
  auto id = [n](int i, int j) { return ((i % n + n) % n) + n * ((j % n + n) % n); };
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
          S.col[slot] = A.col[A.rowptr[r]];  // padding: valid column, value stays 0
        }
      }
    }
  }
  S.uniform = uniform;
  return S;
}

void p1_prolongation(int nf, Csr& P, std::vector<double>& val) {
  const int nc = nf / 2;
  auto fid = [nf](int i, int j) { return ((i % nf + nf) % nf) + nf * ((j % nf + nf) % nf); };
  auto cid = [nc](int i, int j) { return ((i % nc + nc) % nc) + nc * ((j % nc + nc) % nc); };
  std::vector<std::vector<std::pair<int, double>>> rows(nf * nf);
  for (int J = 0; J < nc; ++J)
    for (int I = 0; I < nc; ++I) {
      rows[fid(2 * I, 2 * J)].push_back({cid(I, J), 1.0});
      const int d[3][2] = {{1, 0}, {0, 1}, {1, 1}};
      for (auto& o : d) {
        auto& row = rows[fid(2 * I + o[0], 2 * J + o[1])];
        row.push_back({cid(I, J), 0.5});
        row.push_back({cid(I + o[0], J + o[1]), 0.5});
      }
    }
  P.nrows = nf * nf;
  P.ncols = nc * nc;
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

}  // namespace chns
