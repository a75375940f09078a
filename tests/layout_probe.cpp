// Test-only C entry point around the host layout builder (compiled with g++
// by tests/test_layout_cpu.py together with sccs_layout.cpp).
#include <cstring>

#include "sccs_layout.hpp"

extern "C" int layout_probe(const sccs_problem* p, int G, int tile_nnz, int max_group, int* pb, unsigned* rp,
                            int* tile_start, long long* n_tiles, int* own, int* era_ptr, int* era_col,
                            long long* bound, int* gcol, int* n_groups, unsigned* gdesc) {
  std::string err;
  if (sccs::validate_problem(p, err) != SCCS_OK) return -1;
  sccs::Layout L;
  sccs::build_layout(p, G, L, tile_nnz, max_group);
  *n_tiles = (long long)L.tile_start.size() - 1;
  *bound = sccs::tile_bound(p->nnz, p->n_cols, G, tile_nnz) + 1;
  *n_groups = L.n_groups;
  std::memcpy(pb, L.pb.data(), L.pb.size() * 4);
  std::memcpy(rp, L.rp.data(), L.rp.size() * 4);
  if (tile_start) std::memcpy(tile_start, L.tile_start.data(), L.tile_start.size() * 4);
  std::memcpy(own, L.own.data(), L.own.size() * 4);
  std::memcpy(era_ptr, L.era_ptr.data(), L.era_ptr.size() * 4);
  std::memcpy(era_col, L.era_col.data(), L.era_col.size() * 4);
  std::memcpy(gcol, L.gcol.data(), L.gcol.size() * 4);
  if (gdesc) std::memcpy(gdesc, L.gdesc.data(), L.gdesc.size() * 4);
  return 0;
}

extern "C" int link_cols() { return sccs::kLinkCols; }

extern "C" int ytx_probe(const sccs_problem* p, double* out) {
  std::vector<double> y;
  sccs::host_ytx(p, p->patient_weight, y);
  std::memcpy(out, y.data(), y.size() * 8);
  return 0;
}
