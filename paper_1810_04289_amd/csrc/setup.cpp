// Host-side setup of the HIP FSI library: interface reconstruction, vertex and row
// classes, the block pattern, element scatter maps, partition, overlapping subdomains,
// reverse Cuthill-McKee, the ILU(l) fill pattern, level schedules and the factorization
// work lists.  All of it runs once per mesh; the products are uploaded to HBM.
#include <algorithm>
#include <atomic>
#include <climits>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <numeric>
#include <queue>
#include <thread>

#include "fsi_internal.hpp"

namespace fsi {

// Host threads of the set-up: every threaded step computes per-item results that do not
// depend on the thread count, so the products are the same for any count.  The count is the
// hardware's, at most 16, unless FSI_SETUP_THREADS (1 to 64) sets it.
static int setup_threads() {
  if (const char* e = std::getenv("FSI_SETUP_THREADS")) {
    const int t = std::atoi(e);
    if (t >= 1 && t <= 64) return t;
  }
  const unsigned hw = std::thread::hardware_concurrency();
  return (int)std::max(1u, std::min(hw, 16u));
}

// f(begin, end) over [0, n) in one contiguous range per thread
template <class F>
static void parallel_ranges(int64_t n, F&& f) {
  const int T = setup_threads();
  if (T <= 1 || n < 4096) {
    f(int64_t(0), n);
    return;
  }
  std::vector<std::thread> th;
  for (int t = 0; t < T; ++t) th.emplace_back([&f, n, t, T] { f(n * t / T, n * (t + 1) / T); });
  for (auto& x : th) x.join();
}

// Outward faces of a positively oriented tetrahedron.
static const int kTetFace[4][3] = {{1, 2, 3}, {0, 3, 2}, {0, 1, 3}, {0, 2, 1}};

std::string build_topology(HostSetup& h) {
  const int V = h.V, E = h.E;
  // ---- vertex -> (e*4 + local) in ascending element order; the residual's gather map, and
  // the incidence lists the steps below search
  h.vinc_ptr.assign(V + 1, 0);
  for (int e = 0; e < E; ++e)
    for (int k = 0; k < 4; ++k) h.vinc_ptr[h.tets[4 * (size_t)e + k] + 1]++;
  for (int v = 0; v < V; ++v) h.vinc_ptr[v + 1] += h.vinc_ptr[v];
  h.vinc.resize((size_t)E * 4);
  {
    std::vector<int32_t> fill(h.vinc_ptr.begin(), h.vinc_ptr.end() - 1);
    for (int e = 0; e < E; ++e)
      for (int k = 0; k < 4; ++k) h.vinc[fill[h.tets[4 * (size_t)e + k]]++] = e * 4 + k;
  }
  // ---- Algorithm 1 (§4.8): interface triangles.  The element across a face is the other
  // element holding all three of its vertices, found among the elements of its first
  // vertex; a fluid face whose twin belongs to a wall element is an interface triangle.
  std::vector<int32_t> twin((size_t)E * 4, -1);  // element across each face
  std::atomic<bool> bad_face{false};
  parallel_ranges(E, [&](int64_t e0, int64_t e1) {
    bool bad = false;
    for (int64_t e = e0; e < e1; ++e)
      for (int f = 0; f < 4; ++f) {
        const int32_t a = h.tets[4 * e + kTetFace[f][0]], b = h.tets[4 * e + kTetFace[f][1]],
                      c = h.tets[4 * e + kTetFace[f][2]];
        int found = 0;
        for (int p = h.vinc_ptr[a]; p < h.vinc_ptr[a + 1]; ++p) {
          const int32_t o = h.vinc[p] >> 2;
          if (o == e) continue;
          const int32_t* t = &h.tets[4 * (size_t)o];
          const bool hb = t[0] == b || t[1] == b || t[2] == b || t[3] == b;
          const bool hc = t[0] == c || t[1] == c || t[2] == c || t[3] == c;
          if (hb && hc) {
            twin[4 * e + f] = o;
            ++found;
          }
        }
        if (found > 1) bad = true;
      }
    if (bad) bad_face.store(true);
  });
  if (bad_face.load()) return "a face is shared by more than two elements";
  h.iface.clear();
  for (int e = 0; e < E; ++e) {
    if (h.dom[e] != 0) continue;
    for (int f = 0; f < 4; ++f) {
      int o = twin[4 * (size_t)e + f];
      if (o >= 0 && h.dom[o] == 1)
        for (int k = 0; k < 3; ++k) h.iface.push_back(h.tets[4 * e + kTetFace[f][k]]);
    }
  }
  // ---- vertex classes (strong coupling, §2.2 eqs. (6)-(7))
  std::vector<uint8_t> touch(V, 0);  // bit0 fluid, bit1 wall, bit2 interface triangle
  for (int e = 0; e < E; ++e)
    for (int k = 0; k < 4; ++k) touch[h.tets[4 * e + k]] |= (h.dom[e] == 0) ? 1 : 2;
  for (int32_t v : h.iface) touch[v] |= 4;
  h.vkind.resize(V);
  for (int v = 0; v < V; ++v) {
    uint8_t t = touch[v];
    if ((t & 3) == 0) return "a vertex belongs to no element";
    if (t & 4) h.vkind[v] = VK_IFACE;
    else if ((t & 3) == 3) return "a vertex touches fluid and wall elements but no interface triangle";
    else h.vkind[v] = (t & 1) ? VK_FLUID : VK_SOLID;
  }
  // ---- row classes and Dirichlet rows (§2.1 eqs. (1)-(3))
  const size_t n = 7 * (size_t)V;
  h.rowkind_base.assign(n, RK_ELEM);
  h.forced_zero.assign(n, 0);
  std::vector<uint8_t> bc(V, 0);  // bit0 inlet, bit1 outlet, bit2 ring
  for (int b = 0; b < h.B; ++b) {
    int tag = h.btag[b];
    uint8_t bit = tag == FSI_TAG_FLUID_INLET ? 1 : tag == FSI_TAG_FLUID_OUTLET ? 2
                  : (tag == FSI_TAG_SOLID_RING_IN || tag == FSI_TAG_SOLID_RING_OUT) ? 4 : 0;
    for (int k = 0; k < 3; ++k) bc[h.bfaces[3 * b + k]] |= bit;
  }
  for (int v = 0; v < V; ++v) {
    uint8_t* rk = &h.rowkind_base[7 * (size_t)v];
    if (h.vkind[v] != VK_FLUID) rk[4] = rk[5] = rk[6] = RK_KIN;
    if (h.vkind[v] == VK_SOLID) rk[3] = RK_DUMMY;
    static const int uvd[6] = {0, 1, 2, 4, 5, 6};
    if (bc[v] & 4) {
      for (int c : uvd) { rk[c] = RK_DIR; h.forced_zero[7 * (size_t)v + c] = 1; }
    } else if (bc[v] & 1) {
      for (int c : uvd) rk[c] = RK_DIR;
    } else if (bc[v] & 2) {
      rk[4] = rk[5] = rk[6] = RK_DIR;
    }
  }
  // ---- block pattern: row v holds v and every vertex of an element holding v, ascending
  h.rowptr.assign(V + 1, 0);
  auto row_cols = [&](int v, std::vector<int32_t>& cols) {
    cols.clear();
    cols.push_back(v);
    for (int p = h.vinc_ptr[v]; p < h.vinc_ptr[v + 1]; ++p) {
      const int32_t* t = &h.tets[4 * (size_t)(h.vinc[p] >> 2)];
      cols.insert(cols.end(), t, t + 4);
    }
    std::sort(cols.begin(), cols.end());
    cols.erase(std::unique(cols.begin(), cols.end()), cols.end());
  };
  parallel_ranges(V, [&](int64_t v0, int64_t v1) {
    std::vector<int32_t> cols;
    for (int64_t v = v0; v < v1; ++v) {
      row_cols((int)v, cols);
      h.rowptr[v + 1] = (int32_t)cols.size();
    }
  });
  for (int v = 0; v < V; ++v) {
    if ((int64_t)h.rowptr[v + 1] + h.rowptr[v] > INT_MAX) return "block pattern exceeds 2^31 blocks";
    h.rowptr[v + 1] += h.rowptr[v];
  }
  h.colind.resize(h.rowptr[V]);
  parallel_ranges(V, [&](int64_t v0, int64_t v1) {
    std::vector<int32_t> cols;
    for (int64_t v = v0; v < v1; ++v) {
      row_cols((int)v, cols);
      std::copy(cols.begin(), cols.end(), h.colind.begin() + h.rowptr[v]);
    }
  });
  // ---- Jacobian scatter: the block of every (element, local row vertex, local column vertex)
  h.elem_blk.resize((size_t)E * 16);
  parallel_ranges(E, [&](int64_t e0, int64_t e1) {
    for (int64_t e = e0; e < e1; ++e)
      for (int a = 0; a < 4; ++a) {
        int va = h.tets[4 * e + a];
        const int32_t* c0 = &h.colind[h.rowptr[va]];
        const int32_t* c1 = &h.colind[0] + h.rowptr[va + 1];
        for (int b = 0; b < 4; ++b) {
          const int32_t* q = std::lower_bound(c0, c1, h.tets[4 * e + b]);
          h.elem_blk[16 * e + 4 * a + b] = (int32_t)(q - h.colind.data());
        }
      }
  });
  // ---- element colours, per kind: greedy in ascending element order, the least colour no
  // element sharing a vertex holds yet.  Elements of one colour touch disjoint block rows
  // and columns, so one launch per colour adds their element matrices into J without
  // atomics; colour order fixes the order of the sums.
  auto colour = [&](int kind, std::vector<int32_t>& elems, std::vector<int32_t>& col) {
    std::vector<int32_t> ids;
    for (int e = 0; e < E; ++e)
      if ((h.dom[e] == 0) == (kind == 0)) ids.push_back(e);
    int words = 1;
    std::vector<int32_t> c(ids.size());
    for (;;) {
      std::vector<uint64_t> used((size_t)V * words, 0);
      bool ok = true;
      for (size_t t = 0; t < ids.size() && ok; ++t) {
        const int32_t* tv = &h.tets[4 * (size_t)ids[t]];
        int cc = -1;
        for (int w = 0; w < words && cc < 0; ++w) {
          uint64_t u = 0;
          for (int k = 0; k < 4; ++k) u |= used[(size_t)tv[k] * words + w];
          if (~u) cc = 64 * w + __builtin_ctzll(~u);
        }
        if (cc < 0) { ok = false; break; }
        c[t] = cc;
        for (int k = 0; k < 4; ++k) used[(size_t)tv[k] * words + cc / 64] |= uint64_t(1) << (cc % 64);
      }
      if (ok) break;
      words *= 2;
    }
    int nc = 0;
    for (int x : c) nc = std::max(nc, x + 1);
    col.assign(nc + 1, 0);
    for (int x : c) col[x + 1]++;
    for (int k = 0; k < nc; ++k) col[k + 1] += col[k];
    elems.assign(ids.size(), 0);
    std::vector<int32_t> fill(col.begin(), col.end() - 1);
    for (size_t t = 0; t < ids.size(); ++t) elems[fill[c[t]]++] = ids[t];
  };
  colour(0, h.fluid_celems, h.fluid_col);
  colour(1, h.solid_celems, h.solid_col);
  h.fluid_elems.clear();
  h.solid_elems.clear();
  for (int e = 0; e < E; ++e) (h.dom[e] == 0 ? h.fluid_elems : h.solid_elems).push_back(e);
  return "";
}

// ---------------------------------------------------------------------------------------
// Partition: recursive coordinate bisection.  A set of vertices is cut along the longest
// side of its bounding box (first axis on ties); the first floor(|S| nl / np) vertices
// in (coordinate, id) order go to the lower nl = np/2 parts.
// ---------------------------------------------------------------------------------------
static void rcb(const HostSetup& h, std::vector<int32_t>& ids, size_t lo, size_t hi, int p0, int np,
                std::vector<int32_t>& part) {
  if (np == 1) {
    for (size_t i = lo; i < hi; ++i) part[ids[i]] = p0;
    return;
  }
  double mn[3], mx[3];
  for (int k = 0; k < 3; ++k) { mn[k] = 1e300; mx[k] = -1e300; }
  for (size_t i = lo; i < hi; ++i)
    for (int k = 0; k < 3; ++k) {
      double x = h.X[3 * (size_t)ids[i] + k];
      if (x < mn[k]) mn[k] = x;
      if (x > mx[k]) mx[k] = x;
    }
  int ax = 0;
  if (mx[1] - mn[1] > mx[ax] - mn[ax]) ax = 1;
  if (mx[2] - mn[2] > mx[ax] - mn[ax]) ax = 2;
  const int nl = np / 2;
  const size_t cut = lo + (size_t)(((int64_t)(hi - lo) * nl) / np);
  auto key_less = [&](int32_t a, int32_t b) {
    double xa = h.X[3 * (size_t)a + ax], xb = h.X[3 * (size_t)b + ax];
    return xa < xb || (xa == xb && a < b);
  };
  if (cut > lo && cut < hi) std::nth_element(ids.begin() + lo, ids.begin() + cut, ids.begin() + hi, key_less);
  rcb(h, ids, lo, cut, p0, nl, part);
  rcb(h, ids, cut, hi, p0 + nl, np - nl, part);
}

// ---------------------------------------------------------------------------------------
// Reverse Cuthill-McKee on an induced subgraph (§4.5).  Vertices compare by (degree in
// the subgraph, global id).  Each connected piece starts from the smallest unvisited
// vertex, moved to a pseudo-peripheral vertex by the George-Liu search (repeat: take the
// smallest vertex of the deepest BFS level; keep it while its level structure is deeper).
// ---------------------------------------------------------------------------------------
struct SubGraph {
  const HostSetup* h;
  std::vector<int32_t> deg;     // by global id; -1 = not in the set
  bool has(int v) const { return deg[v] >= 0; }
  bool before(int a, int b) const { return deg[a] != deg[b] ? deg[a] < deg[b] : a < b; }
};

// BFS depth (number of levels) from r and the smallest vertex of its last level.
static int bfs_depth(const SubGraph& G, int r, std::vector<int32_t>& stamp, int tag, int* last_min) {
  const HostSetup& h = *G.h;
  std::vector<int32_t> cur(1, r), nxt;
  stamp[r] = tag;
  int depth = 0;
  int best = r;
  while (!cur.empty()) {
    ++depth;
    best = cur[0];
    for (int v : cur)
      if (G.before(v, best)) best = v;
    nxt.clear();
    for (int v : cur)
      for (int k = h.rowptr[v]; k < h.rowptr[v + 1]; ++k) {
        int u = h.colind[k];
        if (u != v && G.has(u) && stamp[u] != tag) { stamp[u] = tag; nxt.push_back(u); }
      }
    cur.swap(nxt);
  }
  *last_min = best;
  return depth;
}

static void rcm(const HostSetup& h, const std::vector<int32_t>& set, std::vector<int32_t>& out) {
  SubGraph G;
  G.h = &h;
  G.deg.assign(h.V, -1);
  for (int v : set) G.deg[v] = 0;
  for (int v : set)
    for (int k = h.rowptr[v]; k < h.rowptr[v + 1]; ++k) {
      int u = h.colind[k];
      if (u != v && G.has(u)) G.deg[v]++;
    }
  std::vector<int32_t> stamp(h.V, -1);
  std::vector<uint8_t> done(h.V, 0);
  int tag = 0;
  std::vector<int32_t> seq;
  seq.reserve(set.size());
  std::vector<int32_t> sorted_set(set);
  std::sort(sorted_set.begin(), sorted_set.end(), [&](int a, int b) { return G.before(a, b); });
  size_t scan = 0;
  while (seq.size() < set.size()) {
    while (done[sorted_set[scan]]) ++scan;
    int r = sorted_set[scan];
    int cand;
    int dr = bfs_depth(G, r, stamp, ++tag, &cand);
    for (;;) {
      int cand2;
      int dc = bfs_depth(G, cand, stamp, ++tag, &cand2);
      if (dc > dr) { r = cand; dr = dc; cand = cand2; }
      else break;
    }
    size_t head = seq.size();
    seq.push_back(r);
    done[r] = 1;
    std::vector<int32_t> nb;
    while (head < seq.size()) {
      int v = seq[head++];
      nb.clear();
      for (int k = h.rowptr[v]; k < h.rowptr[v + 1]; ++k) {
        int u = h.colind[k];
        if (u != v && G.has(u) && !done[u]) nb.push_back(u);
      }
      std::sort(nb.begin(), nb.end(), [&](int a, int b) { return G.before(a, b); });
      for (int u : nb) { done[u] = 1; seq.push_back(u); }
    }
  }
  out.assign(seq.rbegin(), seq.rend());
}

// ---------------------------------------------------------------------------------------
// One-way dissection (§4.5, Table 4).  Connected pieces are found as in rcm() (smallest
// unfinished vertex by (degree, id), moved to the same pseudo-peripheral vertex).  The
// piece's BFS levels from that vertex are 0 .. h-1; level j is a separator when
// (j + 1) % sep == 0 and j < h - 1.  The other vertices of the piece fall into connected
// blocks, taken in ascending (degree, id) of their first vertex; each block is ordered by
// rcm() on its own vertices, then each separator level, in ascending j, by rcm() on its
// vertices.  Rows of different blocks never meet, so the triangular sweeps run them side
// by side; the separators come last, after every block they border.
// ---------------------------------------------------------------------------------------
static void onewd(const HostSetup& h, const std::vector<int32_t>& set, int sep, std::vector<int32_t>& out) {
  SubGraph G;
  G.h = &h;
  G.deg.assign(h.V, -1);
  for (int v : set) G.deg[v] = 0;
  for (int v : set)
    for (int k = h.rowptr[v]; k < h.rowptr[v + 1]; ++k) {
      int u = h.colind[k];
      if (u != v && G.has(u)) G.deg[v]++;
    }
  std::vector<int32_t> stamp(h.V, -1), level(h.V, -1), blockof(h.V, -1);
  std::vector<uint8_t> done(h.V, 0);
  int tag = 0;
  std::vector<int32_t> sorted_set(set);
  std::sort(sorted_set.begin(), sorted_set.end(), [&](int a, int b) { return G.before(a, b); });
  out.clear();
  out.reserve(set.size());
  size_t scan = 0;
  std::vector<int32_t> piece, cur, nxt, blk, part_out;
  while (out.size() < set.size()) {
    while (done[sorted_set[scan]]) ++scan;
    int r = sorted_set[scan];
    int cand;
    int dr = bfs_depth(G, r, stamp, ++tag, &cand);
    for (;;) {
      int cand2;
      int dc = bfs_depth(G, cand, stamp, ++tag, &cand2);
      if (dc > dr) { r = cand; dr = dc; cand = cand2; }
      else break;
    }
    // levels of the piece
    piece.assign(1, r);
    level[r] = 0;
    done[r] = 1;
    for (size_t q = 0; q < piece.size(); ++q) {
      int v = piece[q];
      for (int k = h.rowptr[v]; k < h.rowptr[v + 1]; ++k) {
        int u = h.colind[k];
        if (u != v && G.has(u) && !done[u]) { done[u] = 1; level[u] = level[v] + 1; piece.push_back(u); }
      }
    }
    const int depth = level[piece.back()] + 1;
    auto is_sep = [&](int v) { return (level[v] + 1) % sep == 0 && level[v] < depth - 1; };
    // blocks, seeded in ascending (degree, id)
    std::vector<int32_t> seeds;
    for (int v : piece)
      if (!is_sep(v)) seeds.push_back(v);
    std::sort(seeds.begin(), seeds.end(), [&](int a, int b) { return G.before(a, b); });
    int nblk = 0;
    for (int v0 : seeds) {
      if (blockof[v0] >= 0) continue;
      blk.assign(1, v0);
      blockof[v0] = nblk;
      for (size_t q = 0; q < blk.size(); ++q) {
        int v = blk[q];
        for (int k = h.rowptr[v]; k < h.rowptr[v + 1]; ++k) {
          int u = h.colind[k];
          if (u != v && G.has(u) && !is_sep(u) && blockof[u] < 0) { blockof[u] = nblk; blk.push_back(u); }
        }
      }
      ++nblk;
      rcm(h, blk, part_out);
      out.insert(out.end(), part_out.begin(), part_out.end());
    }
    // separator levels, ascending
    for (int j = sep - 1; j < depth - 1; j += sep) {
      cur.clear();
      for (int v : piece)
        if (level[v] == j) cur.push_back(v);
      rcm(h, cur, part_out);
      out.insert(out.end(), part_out.begin(), part_out.end());
    }
  }
}

// One subdomain's part of the concatenated set-up arrays, with its rows, blocks, levels
// and map entries counted from zero; the parts are appended in subdomain order.
struct SubPart {
  std::vector<int32_t> lglob;
  std::vector<uint8_t> lowned;
  int nowned = 0;
  std::vector<int32_t> lrowptr{0}, lcol, lsrc, ldiag;
  std::vector<int32_t> fwd_sub_lvl{0}, fwd_lvl_ptr{0}, fwd_rows;
  std::vector<int32_t> bwd_sub_lvl{0}, bwd_lvl_ptr{0}, bwd_rows;
  std::vector<int32_t> kent_ptr{0}, piv, umap;
  std::vector<int64_t> umap_row{0};
  std::vector<int32_t> fwd_qslot, bwd_qslot, lslot;
  int nslots = 0;
  std::string err;
};

// Subdomain s: overlap rings, ordering, ILU(l) pattern, level schedules, factorization work
// lists and sweep slots.  mark and loc are the calling thread's [V] arrays (mark may hold
// other subdomains' numbers; loc is -1 outside the call).
static void build_one(const HostSetup& h, const fsi_opts& o, int s, const std::vector<int32_t>& members,
                      std::vector<int32_t>& mark, std::vector<int32_t>& loc, SubPart& P) {
  const int L = o.ilu_level;
  // extended set: delta rings of vertex-graph neighbours around the owned vertices
  std::vector<int32_t> set = members;
  for (int v : set) mark[v] = s;
  size_t ring_begin = 0;
  for (int d = 0; d < o.overlap; ++d) {
    size_t ring_end = set.size();
    for (size_t i = ring_begin; i < ring_end; ++i) {
      int v = set[i];
      for (int k = h.rowptr[v]; k < h.rowptr[v + 1]; ++k) {
        int u = h.colind[k];
        if (mark[u] != s) { mark[u] = s; set.push_back(u); }
      }
    }
    ring_begin = ring_end;
  }
  std::vector<int32_t> order;
  if (o.ordering == FSI_ORDER_1WD)
    onewd(h, set, o.ilu_level + 3, order);  // separators beyond the kept fill level apart
  else
    rcm(h, set, order);
  const int m = (int)order.size();
  const int base = (int)P.lglob.size();
  for (int l = 0; l < m; ++l) loc[order[l]] = l;
  for (int l = 0; l < m; ++l) {
    P.lglob.push_back(order[l]);
    uint8_t own = h.part[order[l]] == s;
    P.lowned.push_back(own);
    P.nowned += own;
  }
  // ILU(l) pattern by levels of fill: row by row, pivots in ascending order through a
  // min-heap; lev(i,j) = min over pivots k of lev(i,k) + lev(k,j) + 1, kept if <= l.
  std::vector<std::vector<std::pair<int32_t, int32_t>>> rowpat(m);  // (col, level), sorted
  std::vector<int32_t> lev(m, INT_MAX);
  std::vector<int32_t> srcb(m, -1);
  for (int i = 0; i < m; ++i) {
    int g = order[i];
    std::vector<int32_t> cols;
    std::priority_queue<int32_t, std::vector<int32_t>, std::greater<int32_t>> heap;
    for (int k = h.rowptr[g]; k < h.rowptr[g + 1]; ++k) {
      int u = h.colind[k];
      if (mark[u] != s) continue;
      int c = loc[u];
      lev[c] = 0;
      srcb[c] = k;
      cols.push_back(c);
      if (c < i) heap.push(c);
    }
    int last = -1;
    while (L > 0 && !heap.empty()) {
      int k = heap.top();
      heap.pop();
      if (k == last) continue;
      last = k;
      for (const auto& kj : rowpat[k]) {
        if (kj.first <= k) continue;
        int nl = lev[k] + kj.second + 1;
        if (nl > L) continue;
        int j = kj.first;
        if (lev[j] == INT_MAX) {
          lev[j] = nl;
          cols.push_back(j);
          if (j < i) heap.push(j);
        } else if (nl < lev[j]) {
          lev[j] = nl;
        }
      }
    }
    std::sort(cols.begin(), cols.end());
    for (int c : cols) {
      rowpat[i].push_back({c, lev[c]});
      if (c == i) P.ldiag.push_back((int32_t)P.lcol.size());
      P.lcol.push_back(base + c);
      P.lsrc.push_back(srcb[c]);
    }
    for (int c : cols) { lev[c] = INT_MAX; srcb[c] = -1; }
    P.lrowptr.push_back((int32_t)P.lcol.size());
    if ((int)P.ldiag.size() != base + i + 1) { P.err = "missing diagonal block"; return; }
  }
  for (int l = 0; l < m; ++l) loc[order[l]] = -1;
  // level schedules of the two triangular sweeps
  auto rowb = [&](int i) { return P.lrowptr[base + i]; };
  auto rowe = [&](int i) { return P.lrowptr[base + i + 1]; };
  std::vector<int32_t> lf(m, 0), lb(m, 0);
  int nf = 0, nbk = 0;
  for (int i = 0; i < m; ++i) {
    int lv = 0;
    for (int p = rowb(i); p < P.ldiag[base + i]; ++p) lv = std::max(lv, lf[P.lcol[p] - base] + 1);
    lf[i] = lv;
    nf = std::max(nf, lv + 1);
  }
  for (int i = m - 1; i >= 0; --i) {
    int lv = 0;
    for (int p = P.ldiag[base + i] + 1; p < rowe(i); ++p) lv = std::max(lv, lb[P.lcol[p] - base] + 1);
    lb[i] = lv;
    nbk = std::max(nbk, lv + 1);
  }
  auto emit = [&](const std::vector<int32_t>& lv, int nlev, std::vector<int32_t>& lvl_ptr,
                  std::vector<int32_t>& rows, std::vector<int32_t>& sub_lvl) {
    std::vector<int32_t> cnt(nlev + 1, 0);
    for (int i = 0; i < m; ++i) cnt[lv[i] + 1]++;
    for (int l = 0; l < nlev; ++l) cnt[l + 1] += cnt[l];
    size_t r0 = rows.size();
    rows.resize(r0 + m);
    std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
    for (int i = 0; i < m; ++i) rows[r0 + fill[lv[i]]++] = base + i;
    for (int l = 0; l < nlev; ++l) lvl_ptr.push_back((int32_t)(r0 + cnt[l + 1]));
    sub_lvl.push_back((int32_t)lvl_ptr.size() - 1);
  };
  emit(lf, nf, P.fwd_lvl_ptr, P.fwd_rows, P.fwd_sub_lvl);
  emit(lb, nbk, P.bwd_lvl_ptr, P.bwd_rows, P.bwd_sub_lvl);
  // factorization work lists: for each row i, its L blocks (ascending k) as pivots
  // {position of A_ik in row i, D_k, length of U_k, offset of U_k's map}; the map gives,
  // for every block U_kj of row k, 1 + the position of A_ij in row i, or 0 when (i, j)
  // is not in the pattern
  for (int i = 0; i < m; ++i) {
    const int32_t* ci0 = &P.lcol[rowb(i)];
    const int32_t* ci1 = &P.lcol[0] + rowe(i);
    for (int p = rowb(i); p < P.ldiag[base + i]; ++p) {
      const int k = P.lcol[p] - base;
      const int u0 = P.ldiag[base + k] + 1, u1 = rowe(k);
      P.piv.insert(P.piv.end(), {p - rowb(i), P.ldiag[base + k], u1 - u0,
                                 (int32_t)((int64_t)P.umap.size() - P.umap_row.back())});
      const int32_t* f = ci0;
      for (int q = u0; q < u1; ++q) {  // both column lists ascend: one merge walk
        f = std::lower_bound(f, ci1, P.lcol[q]);
        P.umap.push_back(f != ci1 && *f == P.lcol[q] ? (int32_t)(f - ci0) + 1 : 0);
      }
    }
    P.kent_ptr.push_back((int32_t)(P.piv.size() / 4));
    P.umap_row.push_back((int64_t)P.umap.size());
  }
  // LDS slots for the sweeps: y_k (forward) or x_k (backward) is live from its own level
  // to the level of its last reader; slots are handed out greedily in level order and
  // returned once their last reader's level has passed (barrier in between).
  auto colour = [&](const std::vector<int32_t>& lv, bool bwd, std::vector<int32_t>& qslot,
                    const std::vector<int32_t>& lvl_ptr, const std::vector<int32_t>& rows_sched,
                    int lvl_base, int nlev) {
    std::vector<int32_t> last(m, -1);
    for (int i = 0; i < m; ++i) {
      const int pb = bwd ? P.ldiag[base + i] + 1 : rowb(i);
      const int pe = bwd ? rowe(i) : P.ldiag[base + i];
      for (int p = pb; p < pe; ++p) {
        const int k = P.lcol[p] - base;
        last[k] = std::max(last[k], lv[i]);
      }
    }
    std::vector<int32_t> slot(m, -1);
    std::vector<std::vector<int32_t>> release(nlev + 1);
    std::vector<int32_t> freel;
    int used = 0;
    for (int L = 0; L < nlev; ++L) {
      for (int sidx : release[L]) freel.push_back(sidx);
      for (int q = lvl_ptr[lvl_base + L]; q < lvl_ptr[lvl_base + L + 1]; ++q) {
        const int i = rows_sched[q] - base;
        if (last[i] < 0) continue;  // nobody in this sweep reads the row
        int sidx;
        if (!freel.empty()) { sidx = freel.back(); freel.pop_back(); }
        else sidx = used++;
        slot[i] = sidx;
        release[last[i] + 1].push_back(sidx);
      }
    }
    for (int q = lvl_ptr[lvl_base]; q < lvl_ptr[lvl_base + nlev]; ++q) qslot[q] = slot[rows_sched[q] - base];
    for (int i = 0; i < m; ++i) {
      const int pb = bwd ? P.ldiag[base + i] + 1 : rowb(i);
      const int pe = bwd ? rowe(i) : P.ldiag[base + i];
      for (int p = pb; p < pe; ++p) P.lslot[p] = slot[P.lcol[p] - base];
    }
    P.nslots = std::max(P.nslots, used);
  };
  P.lslot.resize(P.lcol.size(), -1);
  P.fwd_qslot.resize(P.fwd_rows.size(), -1);
  P.bwd_qslot.resize(P.bwd_rows.size(), -1);
  colour(lf, false, P.fwd_qslot, P.fwd_lvl_ptr, P.fwd_rows, 0, nf);
  colour(lb, true, P.bwd_qslot, P.bwd_lvl_ptr, P.bwd_rows, 0, nbk);
}

// Where part s goes in the concatenated arrays: its first row, block, schedule row, level
// pointer, pivot entry and map entry.
struct PartOffsets {
  int64_t row = 0, blk = 0, frow = 0, flvl = 0, brow = 0, blvl = 0, piv = 0, umap = 0;
};

static void copy_part(HostSetup& h, int s, const SubPart& P, const PartOffsets& O) {
  const int32_t rb = (int32_t)O.row, bb = (int32_t)O.blk;
  std::copy(P.lglob.begin(), P.lglob.end(), h.lglob.begin() + O.row);
  std::copy(P.lowned.begin(), P.lowned.end(), h.lowned.begin() + O.row);
  h.sub_nowned[s] = P.nowned;
  for (size_t i = 1; i < P.lrowptr.size(); ++i) h.lrowptr[O.row + i] = P.lrowptr[i] + bb;
  for (size_t k = 0; k < P.lcol.size(); ++k) h.lcol[O.blk + k] = P.lcol[k] + rb;
  std::copy(P.lsrc.begin(), P.lsrc.end(), h.lsrc.begin() + O.blk);
  std::copy(P.lslot.begin(), P.lslot.end(), h.lslot.begin() + O.blk);
  for (size_t i = 0; i < P.ldiag.size(); ++i) h.ldiag[O.row + i] = P.ldiag[i] + bb;
  auto levels = [&](const std::vector<int32_t>& lp, const std::vector<int32_t>& rows, const std::vector<int32_t>& qs,
                    std::vector<int32_t>& hlp, std::vector<int32_t>& hrows, std::vector<int32_t>& hqs,
                    std::vector<int32_t>& hsub, int64_t r0, int64_t l0) {
    for (size_t q = 0; q < rows.size(); ++q) hrows[r0 + q] = rows[q] + rb;
    std::copy(qs.begin(), qs.end(), hqs.begin() + r0);
    for (size_t l = 1; l < lp.size(); ++l) hlp[l0 + l] = lp[l] + (int32_t)r0;
    hsub[s + 1] = (int32_t)(l0 + lp.size() - 1);
  };
  levels(P.fwd_lvl_ptr, P.fwd_rows, P.fwd_qslot, h.fwd_lvl_ptr, h.fwd_rows, h.fwd_qslot, h.fwd_sub_lvl, O.frow, O.flvl);
  levels(P.bwd_lvl_ptr, P.bwd_rows, P.bwd_qslot, h.bwd_lvl_ptr, h.bwd_rows, h.bwd_qslot, h.bwd_sub_lvl, O.brow, O.blvl);
  for (size_t q = 0; q < P.piv.size(); q += 4) {
    int32_t* d = &h.piv[4 * O.piv + q];
    d[0] = P.piv[q];
    d[1] = P.piv[q + 1] + bb;
    d[2] = P.piv[q + 2];
    d[3] = P.piv[q + 3];
  }
  for (size_t i = 1; i < P.kent_ptr.size(); ++i) h.kent_ptr[O.row + i] = P.kent_ptr[i] + (int32_t)O.piv;
  std::copy(P.umap.begin(), P.umap.end(), h.umap.begin() + O.umap);
  for (size_t i = 1; i < P.umap_row.size(); ++i) h.umap_row[O.row + i] = P.umap_row[i] + O.umap;
  h.sub_row_off[s + 1] = (int32_t)(O.row + P.lglob.size());
}

std::string build_subdomains(HostSetup& h, const fsi_opts& o) {
  const int V = h.V, ns = o.nsub;
  h.ns = ns;
  if (o.part) {
    h.part.assign(o.part, o.part + V);
    for (int v = 0; v < V; ++v)
      if (h.part[v] < 0 || h.part[v] >= ns) return "partition entry out of range";
  } else {
    h.part.assign(V, 0);
    std::vector<int32_t> ids(V);
    std::iota(ids.begin(), ids.end(), 0);
    rcb(h, ids, 0, V, 0, ns, h.part);
  }
  h.sub_row_off.assign(ns + 1, 0);
  h.sub_nowned.assign(ns, 0);
  h.lglob.clear();
  h.lowned.clear();
  h.lrowptr.assign(1, 0);
  h.lcol.clear();
  h.lsrc.clear();
  h.ldiag.clear();
  h.fwd_sub_lvl.assign(1, 0);
  h.fwd_lvl_ptr.assign(1, 0);
  h.fwd_rows.clear();
  h.bwd_sub_lvl.assign(1, 0);
  h.bwd_lvl_ptr.assign(1, 0);
  h.bwd_rows.clear();
  h.kent_ptr.assign(1, 0);
  h.piv.clear();
  h.umap.clear();
  h.umap_row.assign(1, 0);

  std::vector<std::vector<int32_t>> members(ns);
  for (int v = 0; v < V; ++v) members[h.part[v]].push_back(v);
  // Each subdomain is built alone by a worker thread into its own part; the parts are then
  // copied into the concatenated arrays at offsets fixed by the subdomain order, so the
  // products do not depend on the thread count.
  std::vector<std::unique_ptr<SubPart>> parts(ns);
  {
    // largest subdomains first, so that the last ones to finish are small
    std::vector<int32_t> by_size(ns);
    std::iota(by_size.begin(), by_size.end(), 0);
    std::stable_sort(by_size.begin(), by_size.end(),
                     [&](int a, int b) { return members[a].size() > members[b].size(); });
    std::atomic<int> next{0};
    std::vector<std::thread> th;
    const int T = std::max(1, std::min(setup_threads(), ns));
    for (int t = 0; t < T; ++t)
      th.emplace_back([&] {
        std::vector<int32_t> mark(V, -1), loc(V, -1);
        for (int q; (q = next.fetch_add(1)) < ns;) {
          const int s = by_size[q];
          parts[s] = std::make_unique<SubPart>();
          build_one(h, o, s, members[s], mark, loc, *parts[s]);
        }
      });
    for (auto& t : th) t.join();
  }
  for (int s = 0; s < ns; ++s)
    if (!parts[s]->err.empty()) return parts[s]->err;
  std::vector<PartOffsets> off(ns + 1);
  for (int s = 0; s < ns; ++s) {
    const SubPart& P = *parts[s];
    PartOffsets& a = off[s + 1];
    a = off[s];
    a.row += P.lglob.size();
    a.blk += P.lcol.size();
    a.frow += P.fwd_rows.size();
    a.flvl += P.fwd_lvl_ptr.size() - 1;
    a.brow += P.bwd_rows.size();
    a.blvl += P.bwd_lvl_ptr.size() - 1;
    a.piv += P.piv.size() / 4;
    a.umap += P.umap.size();
    h.nslots = std::max(h.nslots, P.nslots);
  }
  const PartOffsets& tot = off[ns];
  if (tot.row > INT_MAX || tot.blk > INT_MAX || tot.piv > INT_MAX / 4)
    return "the subdomains' local rows, blocks or pivots exceed 2^31";
  h.lglob.resize(tot.row);
  h.lowned.resize(tot.row);
  h.lrowptr.assign(tot.row + 1, 0);
  h.ldiag.resize(tot.row);
  h.kent_ptr.assign(tot.row + 1, 0);
  h.umap_row.assign(tot.row + 1, 0);
  h.lcol.resize(tot.blk);
  h.lsrc.resize(tot.blk);
  h.lslot.resize(tot.blk);
  h.fwd_rows.resize(tot.frow);
  h.fwd_qslot.resize(tot.frow);
  h.fwd_lvl_ptr.assign(tot.flvl + 1, 0);
  h.fwd_sub_lvl.assign(ns + 1, 0);
  h.bwd_rows.resize(tot.brow);
  h.bwd_qslot.resize(tot.brow);
  h.bwd_lvl_ptr.assign(tot.blvl + 1, 0);
  h.bwd_sub_lvl.assign(ns + 1, 0);
  h.piv.resize(4 * tot.piv);
  h.umap.resize(tot.umap);
  {
    std::atomic<int> next{0};
    std::vector<std::thread> th;
    const int T = std::max(1, std::min(setup_threads(), ns));
    for (int t = 0; t < T; ++t)
      th.emplace_back([&] {
        for (int s; (s = next.fetch_add(1)) < ns;) {
          copy_part(h, s, *parts[s], off[s]);
          parts[s].reset();
        }
      });
    for (auto& t : th) t.join();
  }
  return "";
}

}  // namespace fsi

namespace fsi {

SweepTasks build_sweep_tasks(const HostSetup& h, bool bwd, const std::vector<int32_t>& sub_lvl,
                             const std::vector<int32_t>& lvl_ptr, const std::vector<int32_t>& rows,
                             const std::vector<int32_t>& qslot, int mb) {
  constexpr int W = kSweepWaves;
  SweepTasks st;
  st.wtask.assign((size_t)h.ns * W + 1, 0);
  st.nphase.assign(h.ns, 0);
  std::vector<std::vector<int4>> wt(W), wa(W);
  auto blocks = [&](int i, int& b0, int& b1) {
    b0 = bwd ? h.ldiag[i] + 1 : h.lrowptr[i];
    b1 = bwd ? h.lrowptr[i + 1] : h.ldiag[i];
  };
  // level (phase) of every local row in this sweep, filled per subdomain below
  std::vector<int32_t> lvl_of(h.lglob.size(), 0);
  // blocks [f, l) of row rows[q] on wavefront w, as tasks of at most mb blocks; the final
  // task, which in the backward sweep is the one starting at f, finishes the row.  Only the
  // final task writes (the row's LDS slot, its output), so only it must wait for the row's
  // own phase; an earlier task waits just for the rows it reads -- one phase past the
  // latest of them -- and so runs while the wavefront would otherwise sit at barriers.
  auto emit = [&](int w, int q, int f, int l, int phase) {
    const int i = rows[q];
    const int g = h.lglob[i] | (h.lowned[i] ? (int)0x80000000u : 0);
    const int nc = std::max(1, (l - f + mb - 1) / mb);
    for (int c = 0; c < nc; ++c) {
      const int k = bwd ? nc - 1 - c : c;
      const int cf = f + k * mb, cl = std::min(l, cf + mb);
      const int flags = (c > 0 ? kTaskCont : 0) | (c + 1 < nc ? kTaskMore : 0);
      int ph = phase;
      if (c + 1 < nc) {
        ph = 0;
        for (int p = cf; p < cl; ++p) ph = std::max(ph, lvl_of[h.lcol[p]] + 1);
      }
      wt[w].push_back(make_int4(i, g, cf, cl));
      wa[w].push_back(make_int4(c + 1 < nc ? -1 : qslot[q], ph, flags, phase));
    }
  };
  for (int sd = 0; sd < h.ns; ++sd) {
    for (int w = 0; w < W; ++w) {
      wt[w].clear();
      wa[w].clear();
    }
    // rows go to the wavefronts round-robin over the whole schedule, not per level: with
    // about one row per level, consecutive levels then fall to different wavefronts, and
    // each wavefront issues its next prefetch while the others work
    for (int L = sub_lvl[sd]; L < sub_lvl[sd + 1]; ++L)
      for (int q = lvl_ptr[L]; q < lvl_ptr[L + 1]; ++q) lvl_of[rows[q]] = L - sub_lvl[sd];
    int ph = 0, next = 0;
    for (int L = sub_lvl[sd]; L < sub_lvl[sd + 1]; ++L, ++ph)
      for (int q = lvl_ptr[L]; q < lvl_ptr[L + 1]; ++q) {
        int b0, b1;
        blocks(rows[q], b0, b1);
        emit(next++ % W, q, b0, b1, ph);
      }
    st.nphase[sd] = ph;
    for (int w = 0; w < W; ++w) {
      st.task.insert(st.task.end(), wt[w].begin(), wt[w].end());
      st.aux.insert(st.aux.end(), wa[w].begin(), wa[w].end());
      st.wtask[(size_t)sd * W + w + 1] = (int32_t)st.task.size();
    }
  }
  return st;
}

}  // namespace fsi
