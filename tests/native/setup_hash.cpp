// Test harness: runs the library's host set-up (topology, partition, subdomains) on a mesh
// file and prints a hash of every array it produces, so that runs with different thread
// counts can be compared.  Built with g++ from setup.cpp by tests/test_setup_threads.py.
// Mesh file: int32 V, E, B; then X (double[3V]), tets (int32[4E]), tet domain (int8[E]),
// boundary faces (int32[3B]) and their tags (int8[B]).
#include <cstdio>
#include <cstdlib>
#include <string>

#include "fsi_internal.hpp"

namespace fsi {
std::string build_topology(HostSetup& h);
std::string build_subdomains(HostSetup& h, const fsi_opts& o);
}  // namespace fsi

static unsigned long long g_all = 1469598103934665603ULL;

template <class T>
static void mix(const char* name, const std::vector<T>& v) {
  unsigned long long x = 1469598103934665603ULL;
  const unsigned char* p = (const unsigned char*)v.data();
  for (size_t i = 0; i < v.size() * sizeof(T); ++i) {
    x ^= p[i];
    x *= 1099511628211ULL;
  }
  std::printf("%s %zu %016llx\n", name, v.size(), x);
  g_all = (g_all ^ x) * 1099511628211ULL;
}

int main(int argc, char** argv) {
  if (argc < 6) {
    std::fprintf(stderr, "usage: setup_hash mesh nsub overlap ilu_level ordering [partition]\n");
    return 2;
  }
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  int32_t V, E, B;
  if (std::fread(&V, 4, 1, f) != 1 || std::fread(&E, 4, 1, f) != 1 || std::fread(&B, 4, 1, f) != 1) return 2;
  fsi::HostSetup h;
  h.V = V;
  h.E = E;
  h.B = B;
  h.X.resize(3 * (size_t)V);
  h.tets.resize(4 * (size_t)E);
  h.dom.resize(E);
  h.bfaces.resize(3 * (size_t)B);
  h.btag.resize(B);
  bool ok = std::fread(h.X.data(), 8, h.X.size(), f) == h.X.size() &&
            std::fread(h.tets.data(), 4, h.tets.size(), f) == h.tets.size() &&
            std::fread(h.dom.data(), 1, h.dom.size(), f) == h.dom.size() &&
            std::fread(h.bfaces.data(), 4, h.bfaces.size(), f) == h.bfaces.size() &&
            std::fread(h.btag.data(), 1, h.btag.size(), f) == h.btag.size();
  std::fclose(f);
  if (!ok) return 2;
  fsi_opts o{};
  o.nsub = std::atoi(argv[2]);
  o.overlap = std::atoi(argv[3]);
  o.ilu_level = std::atoi(argv[4]);
  o.ordering = std::atoi(argv[5]);
  std::vector<int32_t> part;
  if (argc > 6) {
    part.resize(V);
    FILE* g = std::fopen(argv[6], "rb");
    if (!g || std::fread(part.data(), 4, V, g) != (size_t)V) return 2;
    std::fclose(g);
    o.part = part.data();
  }
  std::string e = fsi::build_topology(h);
  if (e.empty()) e = fsi::build_subdomains(h, o);
  if (!e.empty()) {
    std::printf("error %s\n", e.c_str());
    return 1;
  }
  mix("iface", h.iface); mix("vkind", h.vkind); mix("rowkind", h.rowkind_base); mix("forced0", h.forced_zero);
  mix("rowptr", h.rowptr); mix("colind", h.colind); mix("fluid_celems", h.fluid_celems);
  mix("solid_celems", h.solid_celems); mix("fluid_col", h.fluid_col); mix("solid_col", h.solid_col);
  mix("vinc_ptr", h.vinc_ptr); mix("vinc", h.vinc); mix("elem_blk", h.elem_blk); mix("part", h.part);
  mix("sub_row_off", h.sub_row_off); mix("sub_nowned", h.sub_nowned); mix("lglob", h.lglob); mix("lowned", h.lowned);
  mix("lrowptr", h.lrowptr); mix("lcol", h.lcol); mix("lsrc", h.lsrc); mix("ldiag", h.ldiag);
  mix("fwd_sub_lvl", h.fwd_sub_lvl); mix("fwd_lvl_ptr", h.fwd_lvl_ptr); mix("fwd_rows", h.fwd_rows);
  mix("bwd_sub_lvl", h.bwd_sub_lvl); mix("bwd_lvl_ptr", h.bwd_lvl_ptr); mix("bwd_rows", h.bwd_rows);
  mix("kent_ptr", h.kent_ptr); mix("piv", h.piv); mix("umap", h.umap); mix("umap_row", h.umap_row);
  mix("fwd_qslot", h.fwd_qslot); mix("bwd_qslot", h.bwd_qslot); mix("lslot", h.lslot);
  std::printf("nslots %d\nall %016llx\n", h.nslots, g_all);
  return 0;
}
