// Oracle: interface reconstruction, vertex classes, row kinds and the block sparsity
// pattern (test infrastructure only).
#include <algorithm>
#include <array>
#include <map>
#include <set>

#include "core.hpp"

namespace fsio {

// Faces of a positively oriented tet, each listed with outward orientation.
static const int kFace[4][3] = {{1, 2, 3}, {0, 3, 2}, {0, 1, 3}, {0, 2, 1}};

int Bsr::find(int a, int b) const {
  for (int k = rowptr[a]; k < rowptr[a + 1]; ++k)
    if (colind[k] == b) return k;
  return -1;
}

// Algorithm 1 of §4.8 (interface mesh reconstruction): walk the fluid elements; a
// face of a fluid element is an interface triangle when the element on the other side
// of it is solid.  The face-to-element lookup is a plain ordered map.
static void interface_faces(const fsio_solver& s, std::vector<int>& out) {
  std::map<std::array<int, 3>, std::vector<int>> owners;
  for (int e = 0; e < s.E; ++e)
    for (int f = 0; f < 4; ++f) {
      std::array<int, 3> k = {s.tets[4 * e + kFace[f][0]], s.tets[4 * e + kFace[f][1]],
                              s.tets[4 * e + kFace[f][2]]};
      std::sort(k.begin(), k.end());
      owners[k].push_back(e);
    }
  out.clear();
  for (int e = 0; e < s.E; ++e) {
    if (s.dom[e] != 0) continue;
    for (int f = 0; f < 4; ++f) {
      std::array<int, 3> k = {s.tets[4 * e + kFace[f][0]], s.tets[4 * e + kFace[f][1]],
                              s.tets[4 * e + kFace[f][2]]};
      std::sort(k.begin(), k.end());
      for (int o : owners[k])
        if (o != e && s.dom[o] == 1) {
          for (int j = 0; j < 3; ++j) out.push_back(s.tets[4 * e + kFace[f][j]]);
          break;
        }
    }
  }
}

int build_topology(fsio_solver& s) {
  const int V = s.V;
  interface_faces(s, s.iface_faces);

  std::vector<char> on_iface(V, 0), tf(V, 0), ts(V, 0);
  for (int v : s.iface_faces) on_iface[v] = 1;
  for (int e = 0; e < s.E; ++e)
    for (int j = 0; j < 4; ++j) (s.dom[e] == 0 ? tf : ts)[s.tets[4 * e + j]] = 1;

  // Vertex classes of the strong coupling (§2.2, eqs. (6)-(7)): interface vertices
  // carry one shared velocity and one shared displacement.
  s.vkind.assign(V, V_FLUID);
  for (int v = 0; v < V; ++v) {
    if (!tf[v] && !ts[v]) { s.err = "vertex not used by any element"; return FSIO_ERR_MESH; }
    if (on_iface[v]) s.vkind[v] = V_IFACE;
    else if (tf[v] && ts[v]) { s.err = "vertex touches fluid and solid but no interface face"; return FSIO_ERR_MESH; }
    else s.vkind[v] = tf[v] ? V_FLUID : V_SOLID;
  }

  // Row kinds.  Fluid vertex: momentum, continuity, mesh Laplace.  Interface vertex:
  // fluid + solid momentum, continuity, kinematic d rows.  Solid vertex: solid momentum,
  // a dummy pressure row, kinematic d rows.
  s.rowkind_base.assign(7 * (size_t)V, ROW_ELEM);
  s.forced_zero.assign(7 * (size_t)V, 0);
  for (int v = 0; v < V; ++v) {
    uint8_t* rk = &s.rowkind_base[7 * (size_t)v];
    if (s.vkind[v] != V_FLUID)
      for (int c = 4; c < 7; ++c) rk[c] = ROW_KIN;
    if (s.vkind[v] == V_SOLID) rk[3] = ROW_DUMMY;
  }
  // Dirichlet rows from the boundary tags (§2.1 eqs. (1)-(3)): inlet u = v_in and d = 0,
  // outlets d = 0, solid rings clamped (u = 0, d = 0).  A clamp beats the inflow.
  std::vector<char> inlet(V, 0), outlet(V, 0), ring(V, 0);
  for (int b = 0; b < s.B; ++b) {
    int tag = s.btag[b];
    for (int j = 0; j < 3; ++j) {
      int v = s.bfaces[3 * b + j];
      if (tag == 1) inlet[v] = 1;
      if (tag == 2) outlet[v] = 1;
      if (tag == 3 || tag == 4) ring[v] = 1;
    }
  }
  for (int v = 0; v < V; ++v) {
    uint8_t* rk = &s.rowkind_base[7 * (size_t)v];
    uint8_t* fz = &s.forced_zero[7 * (size_t)v];
    if (ring[v]) {
      for (int c : {0, 1, 2, 4, 5, 6}) { rk[c] = ROW_DIR; fz[c] = 1; }
    } else if (inlet[v]) {
      for (int c : {0, 1, 2, 4, 5, 6}) rk[c] = ROW_DIR;
    } else if (outlet[v]) {
      for (int c : {4, 5, 6}) rk[c] = ROW_DIR;
    }
  }

  // Block pattern: block (a,b) exists when a and b share an element, or a == b.
  std::vector<std::set<int>> adj(V);
  for (int v = 0; v < V; ++v) adj[v].insert(v);
  for (int e = 0; e < s.E; ++e)
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) adj[s.tets[4 * e + i]].insert(s.tets[4 * e + j]);
  s.J.nb = V;
  s.J.rowptr.assign(V + 1, 0);
  s.J.colind.clear();
  for (int v = 0; v < V; ++v) {
    for (int b : adj[v]) s.J.colind.push_back(b);
    s.J.rowptr[v + 1] = (int)s.J.colind.size();
  }
  s.J.vals.assign(s.J.colind.size() * 49, 0.0);
  return FSIO_OK;
}

void set_rowkinds(fsio_solver& s, const uint8_t* extra_mask) {
  s.rowkind = s.rowkind_base;
  if (extra_mask)
    for (size_t i = 0; i < s.rowkind.size(); ++i)
      if (extra_mask[i]) s.rowkind[i] = ROW_DIR;
}

}  // namespace fsio
