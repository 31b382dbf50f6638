// Oracle: partition, overlap, reverse Cuthill-McKee, subdomain matrices, block ILU(0),
// restricted additive Schwarz and the block sparse product (test infrastructure only).
//
// Paper §3: the mesh is split into np submeshes, each extended by delta layers of mesh
// points; R_i^delta selects the unknowns of an extended submesh (eq. (14)); the
// subdomain matrix is R_i^delta J (R_i^delta)^T (eq. (15), read with the transposes in
// the standard place); the restricted Schwarz preconditioner is
// B^{-1} = sum_i (R_i^0)^T (J_i^delta)^{-1} R_i^delta (eq. (16)) with an incomplete LU
// subdomain solve.  §4.5: subdomain matrices are reordered (RCM).  §4.3: ILU(l) keeps l
// levels of fill; ILU(0) keeps the sparsity of the subdomain matrix.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <numeric>

#include "core.hpp"

namespace fsio {

// Recursive coordinate bisection (a deterministic stand-in for the paper's hierarchical
// partition): split the longest bounding-box axis at the rank floor(|S| * nl / np),
// vertices ordered by (coordinate, id).
static void rcb_rec(const fsio_solver& s, std::vector<int> ids, int p0, int np, std::vector<int>& part) {
  if (np == 1) {
    for (int v : ids) part[v] = p0;
    return;
  }
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int v : ids)
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::min(lo[k], s.X[3 * (size_t)v + k]);
      hi[k] = std::max(hi[k], s.X[3 * (size_t)v + k]);
    }
  int ax = 0;
  for (int k = 1; k < 3; ++k)
    if (hi[k] - lo[k] > hi[ax] - lo[ax]) ax = k;
  std::sort(ids.begin(), ids.end(), [&](int a, int b) {
    double xa = s.X[3 * (size_t)a + ax], xb = s.X[3 * (size_t)b + ax];
    return xa < xb || (xa == xb && a < b);
  });
  int nl = np / 2;
  size_t cut = (size_t)(((long long)ids.size() * nl) / np);
  rcb_rec(s, std::vector<int>(ids.begin(), ids.begin() + cut), p0, nl, part);
  rcb_rec(s, std::vector<int>(ids.begin() + cut, ids.end()), p0 + nl, np - nl, part);
}

void rcb_partition(const fsio_solver& s, int nsub, std::vector<int>& part) {
  part.assign(s.V, 0);
  std::vector<int> ids(s.V);
  std::iota(ids.begin(), ids.end(), 0);
  rcb_rec(s, ids, 0, nsub, part);
}

// ---------------------------------------------------------------------------------------
// Reverse Cuthill-McKee on the vertex graph induced by a vertex set.
// Start node: George-Liu pseudo-peripheral search from the unvisited vertex of minimum
// (degree, id); neighbours are visited in ascending (degree, id); the final sequence is
// reversed.
// ---------------------------------------------------------------------------------------
struct Induced {
  const fsio_solver* s;
  std::vector<int> loc;     // global -> position in the set, -1 outside
  std::vector<int> deg;     // degree inside the set, by global id
  bool in(int v) const { return loc[v] >= 0; }
};

static void bfs_levels(const Induced& G, int root, std::vector<std::vector<int>>& levels) {
  const fsio_solver& s = *G.s;
  levels.clear();
  std::vector<char> seen(s.V, 0);
  std::vector<int> cur = {root};
  seen[root] = 1;
  while (!cur.empty()) {
    levels.push_back(cur);
    std::vector<int> nxt;
    for (int x : cur)
      for (int k = s.J.rowptr[x]; k < s.J.rowptr[x + 1]; ++k) {
        int y = s.J.colind[k];
        if (y == x || !G.in(y) || seen[y]) continue;
        seen[y] = 1;
        nxt.push_back(y);
      }
    cur.swap(nxt);
  }
}

static bool less_dg(const Induced& G, int a, int b) {
  return G.deg[a] < G.deg[b] || (G.deg[a] == G.deg[b] && a < b);
}

static int pseudo_peripheral(const Induced& G, int r) {
  std::vector<std::vector<int>> L;
  bfs_levels(G, r, L);
  while (true) {
    const std::vector<int>& last = L.back();
    int x = last[0];
    for (int v : last)
      if (less_dg(G, v, x)) x = v;
    std::vector<std::vector<int>> Lx;
    bfs_levels(G, x, Lx);
    if (Lx.size() > L.size()) {
      r = x;
      L.swap(Lx);
    } else {
      return r;
    }
  }
}

static std::vector<int> rcm_order(const fsio_solver& s, const std::vector<int>& set) {
  Induced G;
  G.s = &s;
  G.loc.assign(s.V, -1);
  for (size_t i = 0; i < set.size(); ++i) G.loc[set[i]] = (int)i;
  G.deg.assign(s.V, 0);
  for (int v : set)
    for (int k = s.J.rowptr[v]; k < s.J.rowptr[v + 1]; ++k) {
      int y = s.J.colind[k];
      if (y != v && G.in(y)) G.deg[v]++;
    }
  std::vector<char> vis(s.V, 0);
  std::vector<int> order;
  while (order.size() < set.size()) {
    int start = -1;
    for (int v : set)
      if (!vis[v] && (start < 0 || less_dg(G, v, start))) start = v;
    int r = pseudo_peripheral(G, start);
    std::deque<int> q = {r};
    vis[r] = 1;
    order.push_back(r);
    while (!q.empty()) {
      int x = q.front();
      q.pop_front();
      std::vector<int> nb;
      for (int k = s.J.rowptr[x]; k < s.J.rowptr[x + 1]; ++k) {
        int y = s.J.colind[k];
        if (y != x && G.in(y) && !vis[y]) nb.push_back(y);
      }
      std::sort(nb.begin(), nb.end(), [&](int a, int b) { return less_dg(G, a, b); });
      for (int y : nb) {
        vis[y] = 1;
        order.push_back(y);
        q.push_back(y);
      }
    }
  }
  std::reverse(order.begin(), order.end());
  return order;
}

// ---------------------------------------------------------------------------------------
// One-way dissection (§4.5, Table 4) on the vertex graph induced by a vertex set.  Each
// connected piece, taken in the order RCM takes them, gets the level structure rooted at
// RCM's pseudo-peripheral vertex, L_0 .. L_{h-1}.  Levels L_j with (j + 1) % sep == 0 and
// j < h - 1 are separators.  The remaining vertices split into connected blocks; blocks
// come first, in order of their smallest (degree, id) vertex, each ordered by RCM on its
// own vertices; the separator levels follow in ascending j, each ordered by RCM on its
// vertices.  Blocks do not touch each other, so their rows are independent.
// ---------------------------------------------------------------------------------------
static std::vector<int> onewd_order(const fsio_solver& s, const std::vector<int>& set, int sep) {
  Induced G;
  G.s = &s;
  G.loc.assign(s.V, -1);
  for (size_t i = 0; i < set.size(); ++i) G.loc[set[i]] = (int)i;
  G.deg.assign(s.V, 0);
  for (int v : set)
    for (int k = s.J.rowptr[v]; k < s.J.rowptr[v + 1]; ++k) {
      int y = s.J.colind[k];
      if (y != v && G.in(y)) G.deg[v]++;
    }
  std::vector<char> vis(s.V, 0);
  std::vector<int> order;
  while (order.size() < set.size()) {
    int start = -1;
    for (int v : set)
      if (!vis[v] && (start < 0 || less_dg(G, v, start))) start = v;
    int r = pseudo_peripheral(G, start);
    std::vector<std::vector<int>> L;
    bfs_levels(G, r, L);
    const int h = (int)L.size();
    std::vector<char> is_sep(s.V, 0);
    std::vector<int> comp;
    for (int j = 0; j < h; ++j)
      for (int v : L[j]) {
        vis[v] = 1;
        comp.push_back(v);
        if ((j + 1) % sep == 0 && j < h - 1) is_sep[v] = 1;
      }
    // blocks: connected pieces of the non-separator vertices, by smallest (degree, id)
    std::vector<int> cand;
    for (int v : comp)
      if (!is_sep[v]) cand.push_back(v);
    std::sort(cand.begin(), cand.end(), [&](int a, int b) { return less_dg(G, a, b); });
    std::vector<char> taken(s.V, 0);
    for (int v0 : cand) {
      if (taken[v0]) continue;
      std::vector<int> blk = {v0};
      taken[v0] = 1;
      for (size_t q = 0; q < blk.size(); ++q) {
        int x = blk[q];
        for (int k = s.J.rowptr[x]; k < s.J.rowptr[x + 1]; ++k) {
          int y = s.J.colind[k];
          if (y != x && G.in(y) && !is_sep[y] && !taken[y]) { taken[y] = 1; blk.push_back(y); }
        }
      }
      std::sort(blk.begin(), blk.end());
      std::vector<int> o = rcm_order(s, blk);
      order.insert(order.end(), o.begin(), o.end());
    }
    for (int j = sep - 1; j < h - 1; j += sep) {
      std::vector<int> lv(L[j]);
      std::sort(lv.begin(), lv.end());
      std::vector<int> o = rcm_order(s, lv);
      order.insert(order.end(), o.begin(), o.end());
    }
  }
  return order;
}

// Extended submeshes (§3): owned vertices plus delta rings of vertex-graph neighbours,
// reordered by RCM or 1WD, with the sub-block pattern of R J R^T and its source blocks.
int build_subdomains(fsio_solver& s) {
  const int ns = s.opts.nsub;
  s.subs.assign(ns, Sub());
  for (int i = 0; i < ns; ++i) {
    Sub& S = s.subs[i];
    std::vector<char> in(s.V, 0);
    std::vector<int> set, frontier;
    for (int v = 0; v < s.V; ++v)
      if (s.part[v] == i) { in[v] = 1; set.push_back(v); frontier.push_back(v); }
    for (int ring = 0; ring < s.opts.overlap; ++ring) {
      std::vector<int> nxt;
      for (int x : frontier)
        for (int k = s.J.rowptr[x]; k < s.J.rowptr[x + 1]; ++k) {
          int y = s.J.colind[k];
          if (!in[y]) { in[y] = 1; nxt.push_back(y); set.push_back(y); }
        }
      frontier.swap(nxt);
    }
    std::sort(set.begin(), set.end());
    if (s.opts.ordering == 1) {
      // separators every ilu_level + 3 levels: a fill path between two separators crosses
      // ilu_level + 2 block levels and so exceeds the kept fill level
      S.verts = onewd_order(s, set, s.opts.ilu_level + 3);
    } else {
      S.verts = rcm_order(s, set);
    }
    const int m = (int)S.verts.size();
    std::vector<int> loc(s.V, -1);
    for (int l = 0; l < m; ++l) loc[S.verts[l]] = l;
    S.owned.assign(m, 0);
    S.nowned = 0;
    for (int l = 0; l < m; ++l)
      if (s.part[S.verts[l]] == i) { S.owned[l] = 1; S.nowned++; }
    S.rowptr.assign(m + 1, 0);
    S.colind.clear();
    S.src.clear();
    S.diag.assign(m, -1);
    // Symbolic ILU(k) by levels of fill (§4.3: ILU(l) keeps l layers of extra entries):
    // lev(i,j) = 0 on the pattern of J_i^delta, and a fill entry (i,j) created through a
    // pivot k < min(i,j) gets lev(i,k) + lev(k,j) + 1; entries above level k are dropped.
    // Rows are processed in order, pivots of a row in ascending column order.
    const int K = s.opts.ilu_level;
    std::vector<std::vector<std::pair<int, int>>> rows(m);  // final (col, level), sorted
    for (int l = 0; l < m; ++l) {
      int g = S.verts[l];
      std::map<int, int> lev;     // column -> level
      std::map<int, int> srcof;   // column -> global block of J
      for (int k = s.J.rowptr[g]; k < s.J.rowptr[g + 1]; ++k) {
        int h = s.J.colind[k];
        if (loc[h] >= 0) { lev[loc[h]] = 0; srcof[loc[h]] = k; }
      }
      if (K > 0) {
        for (auto it = lev.begin(); it != lev.end() && it->first < l; ++it) {
          int kcol = it->first, lik = it->second;
          for (const auto& kj : rows[kcol]) {
            if (kj.first <= kcol) continue;
            int nl = lik + kj.second + 1;
            if (nl > K) continue;
            auto f = lev.find(kj.first);
            if (f == lev.end()) lev[kj.first] = nl;
            else if (nl < f->second) f->second = nl;
          }
        }
      }
      for (const auto& c : lev) {
        rows[l].push_back(c);
        if (c.first == l) S.diag[l] = (int)S.colind.size();
        S.colind.push_back(c.first);
        auto f = srcof.find(c.first);
        S.src.push_back(f == srcof.end() ? -1 : f->second);
      }
      S.rowptr[l + 1] = (int)S.colind.size();
    }
    // level count of the lower-triangular dependency graph (reported, not used)
    std::vector<int> lev(m, 0);
    int nl = 0;
    for (int l = 0; l < m; ++l) {
      int lv = 0;
      for (int k = S.rowptr[l]; k < S.rowptr[l + 1]; ++k)
        if (S.colind[k] < l) lv = std::max(lv, lev[S.colind[k]] + 1);
      lev[l] = lv;
      nl = std::max(nl, lv + 1);
    }
    S.nlevels = nl;
  }
  return FSIO_OK;
}

// 7x7 inverse by Gauss-Jordan elimination with partial pivoting (first maximum wins),
// applied to the equilibrated block.  A pivot block of the FSI matrix mixes momentum,
// continuity (PSPG, entries near 1e-10) and kinematic or wall rows (up to 1e4), so it is
// first scaled by powers of two, rows then columns, to a largest entry in [1, 2) in each
// row and column: Ah = R A C with R = diag(r), C = diag(c).  Then A^{-1} = C Ah^{-1} R.  The
// scalings are exact, so in exact arithmetic this is the same inverse and the same block
// ILU (§3, §4.3); only the rounding of the elimination changes.
static double pow2_below(double x) {  // the power of two 2^e with 2^e <= x < 2^(e+1)
  int e;
  std::frexp(x, &e);
  return std::ldexp(1.0, e - 1);
}

int invert7(const double* A, double* Ainv) {
  double M[7][7], I[7][7], r[7], c[7];
  for (int i = 0; i < 7; ++i) {
    double mx = 0.0;
    for (int j = 0; j < 7; ++j) mx = std::max(mx, std::fabs(A[7 * i + j]));
    if (!(mx > 0.0) || !std::isfinite(mx)) return FSIO_ERR_ZERO_PIVOT;
    r[i] = 1.0 / pow2_below(mx);
  }
  for (int j = 0; j < 7; ++j) {
    double mx = 0.0;
    for (int i = 0; i < 7; ++i) mx = std::max(mx, std::fabs(A[7 * i + j]) * r[i]);
    if (!(mx > 0.0)) return FSIO_ERR_ZERO_PIVOT;
    c[j] = 1.0 / pow2_below(mx);
  }
  for (int i = 0; i < 7; ++i)
    for (int j = 0; j < 7; ++j) { M[i][j] = r[i] * A[7 * i + j] * c[j]; I[i][j] = (i == j) ? 1.0 : 0.0; }
  for (int p = 0; p < 7; ++p) {
    int piv = p;
    for (int i = p + 1; i < 7; ++i)
      if (std::fabs(M[i][p]) > std::fabs(M[piv][p])) piv = i;
    if (!(std::fabs(M[piv][p]) > 0.0) || !std::isfinite(M[piv][p])) return FSIO_ERR_ZERO_PIVOT;
    if (piv != p)
      for (int j = 0; j < 7; ++j) { std::swap(M[p][j], M[piv][j]); std::swap(I[p][j], I[piv][j]); }
    double pv = M[p][p];
    for (int j = 0; j < 7; ++j) { M[p][j] /= pv; I[p][j] /= pv; }
    for (int i = 0; i < 7; ++i) {
      if (i == p) continue;
      double f = M[i][p];
      for (int j = 0; j < 7; ++j) { M[i][j] -= f * M[p][j]; I[i][j] -= f * I[p][j]; }
    }
  }
  // I now holds Ah^{-1}; A^{-1} = C Ah^{-1} R
  for (int i = 0; i < 7; ++i)
    for (int j = 0; j < 7; ++j) Ainv[7 * i + j] = c[i] * I[i][j] * r[j];
  return FSIO_OK;
}

// C = A B.  Each entry's sum runs over m in ascending order from 0, every term added to the
// running sum with a single rounding (a fused multiply-add).  The paper states the
// factorization in exact arithmetic; this fixes one rounding order, which any other
// implementation can reproduce exactly.
static void mm7(const double* A, const double* B, double* C) {
  for (int r = 0; r < 7; ++r)
    for (int c = 0; c < 7; ++c) {
      double s = 0.0;
      for (int m = 0; m < 7; ++m) s = std::fma(A[7 * r + m], B[7 * m + c], s);
      C[7 * r + c] = s;
    }
}

// Block ILU(0) in IKJ order on the subdomain pattern: for each block row i, for each
// k < i in the row, A_ik <- A_ik D_k and A_ij -= A_ik A_kj for j > k present in row i;
// then D_i = A_ii^{-1} replaces the diagonal block.
int pc_setup(fsio_solver& s) {
  if (!s.jac_ready) { s.err = "pc_setup before jacobian"; return FSIO_ERR_ARG; }
  for (size_t si = 0; si < s.subs.size(); ++si) {
    Sub& S = s.subs[si];
    const int m = (int)S.verts.size();
    S.f.assign(S.colind.size() * 49, 0.0);
    for (size_t k = 0; k < S.colind.size(); ++k)
      if (S.src[k] >= 0) std::memcpy(&S.f[49 * k], &s.J.vals[49 * (size_t)S.src[k]], 49 * sizeof(double));
    S.udiag.assign((size_t)m * 49, 0.0);
    double tmp[49];
    for (int i = 0; i < m; ++i) {
      for (int pk = S.rowptr[i]; pk < S.rowptr[i + 1]; ++pk) {
        int k = S.colind[pk];
        if (k >= i) break;
        mm7(&S.f[49 * (size_t)pk], &S.f[49 * (size_t)S.diag[k]], tmp);
        std::memcpy(&S.f[49 * (size_t)pk], tmp, sizeof(tmp));
        for (int pj = S.diag[k] + 1; pj < S.rowptr[k + 1]; ++pj) {
          int j = S.colind[pj];
          int pij = -1;
          for (int q = S.rowptr[i]; q < S.rowptr[i + 1]; ++q)
            if (S.colind[q] == j) { pij = q; break; }
          if (pij < 0) continue;
          mm7(&S.f[49 * (size_t)pk], &S.f[49 * (size_t)pj], tmp);
          for (int t = 0; t < 49; ++t) S.f[49 * (size_t)pij + t] -= tmp[t];
        }
      }
      double* Dii = &S.f[49 * (size_t)S.diag[i]];
      std::memcpy(&S.udiag[49 * (size_t)i], Dii, 49 * sizeof(double));
      if (invert7(&S.udiag[49 * (size_t)i], Dii) != FSIO_OK) {
        s.err = "zero pivot in subdomain " + std::to_string(si) + " row " + std::to_string(i);
        return FSIO_ERR_ZERO_PIVOT;
      }
    }
  }
  s.pc_ready = true;
  return FSIO_OK;
}

// z = sum_i (R_i^0)^T (L_i U_i)^{-1} R_i^delta v
void pc_apply(const fsio_solver& s, const double* v, double* z) {
  for (const Sub& S : s.subs) {
    const int m = (int)S.verts.size();
    std::vector<double> y((size_t)m * 7), x((size_t)m * 7);
    for (int i = 0; i < m; ++i) {
      double acc[7];
      for (int r = 0; r < 7; ++r) acc[r] = v[7 * (size_t)S.verts[i] + r];
      for (int p = S.rowptr[i]; p < S.diag[i]; ++p) {
        const double* L = &S.f[49 * (size_t)p];
        const double* yk = &y[7 * (size_t)S.colind[p]];
        for (int r = 0; r < 7; ++r)
          for (int c = 0; c < 7; ++c) acc[r] -= L[7 * r + c] * yk[c];
      }
      for (int r = 0; r < 7; ++r) y[7 * (size_t)i + r] = acc[r];
    }
    for (int i = m - 1; i >= 0; --i) {
      double acc[7];
      for (int r = 0; r < 7; ++r) acc[r] = y[7 * (size_t)i + r];
      for (int p = S.diag[i] + 1; p < S.rowptr[i + 1]; ++p) {
        const double* U = &S.f[49 * (size_t)p];
        const double* xj = &x[7 * (size_t)S.colind[p]];
        for (int r = 0; r < 7; ++r)
          for (int c = 0; c < 7; ++c) acc[r] -= U[7 * r + c] * xj[c];
      }
      const double* D = &S.f[49 * (size_t)S.diag[i]];
      for (int r = 0; r < 7; ++r) {
        double t = 0.0;
        for (int c = 0; c < 7; ++c) t += D[7 * r + c] * acc[c];
        x[7 * (size_t)i + r] = t;
      }
      if (S.owned[i])
        for (int r = 0; r < 7; ++r) z[7 * (size_t)S.verts[i] + r] = x[7 * (size_t)i + r];
    }
  }
}

void spmv(const fsio_solver& s, const double* x, double* y) {
  for (int a = 0; a < s.V; ++a) {
    double acc[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int k = s.J.rowptr[a]; k < s.J.rowptr[a + 1]; ++k) {
      const double* A = &s.J.vals[49 * (size_t)k];
      const double* xb = &x[7 * (size_t)s.J.colind[k]];
      for (int r = 0; r < 7; ++r)
        for (int c = 0; c < 7; ++c) acc[r] += A[7 * r + c] * xb[c];
    }
    for (int r = 0; r < 7; ++r) y[7 * (size_t)a + r] = acc[r];
  }
}

}  // namespace fsio
