// Host layout builder for libsccs (see sccs_layout.hpp).
#include "sccs_layout.hpp"

#include <algorithm>
#include <cstdio>
#include <limits>

namespace sccs {

static sccs_status fail(std::string& err, const char* msg, long long a = -1) {
  char buf[256];
  if (a >= 0)
    std::snprintf(buf, sizeof buf, "%s (at %lld)", msg, a);
  else
    std::snprintf(buf, sizeof buf, "%s", msg);
  err = buf;
  return SCCS_ERR_INVALID_ARG;
}

sccs_status validate_problem(const sccs_problem* p, std::string& err) {
  if (!p) return fail(err, "problem is NULL");
  if (p->n_patients < 1 || p->n_rows < 1 || p->n_cols < 1)
    return fail(err, "n_patients, n_rows and n_cols must be >= 1");
  if (p->n_rows >= (int64_t)std::numeric_limits<int32_t>::max())
    return fail(err, "n_rows must be < 2^31");
  if (p->nnz < 0 || p->nnz >= (int64_t)std::numeric_limits<int32_t>::max())
    return fail(err, "nnz must be in [0, 2^31)");
  if (!p->patient_ptr || !p->offset || !p->count || !p->col_ptr || (p->nnz > 0 && !p->row_idx))
    return fail(err, "a required array pointer is NULL");
  const int64_t N = p->n_patients, K = p->n_rows, J = p->n_cols;
  if (p->patient_ptr[0] != 0) return fail(err, "patient_ptr[0] must be 0");
  for (int64_t i = 0; i < N; ++i)
    if (p->patient_ptr[i + 1] < p->patient_ptr[i]) return fail(err, "patient_ptr must be non-decreasing", i);
  if (p->patient_ptr[N] != K) return fail(err, "patient_ptr[N] must equal n_rows");
  if (p->col_ptr[0] != 0) return fail(err, "col_ptr[0] must be 0");
  for (int64_t j = 0; j < J; ++j)
    if (p->col_ptr[j + 1] < p->col_ptr[j]) return fail(err, "col_ptr must be non-decreasing", j);
  if (p->col_ptr[J] != p->nnz) return fail(err, "col_ptr[J] must equal nnz");
  for (int64_t k = 0; k < K; ++k) {
    if (p->offset[k] < 0) return fail(err, "offset (era length) must be >= 0", k);
    if (p->count[k] < 0) return fail(err, "count must be >= 0", k);
    if (p->count[k] > 0 && p->offset[k] == 0) return fail(err, "an era with events must have positive length", k);
  }
  for (int64_t j = 0; j < J; ++j) {
    for (int64_t e = p->col_ptr[j]; e < p->col_ptr[j + 1]; ++e) {
      int32_t r = p->row_idx[e];
      if (r < 0 || r >= K) return fail(err, "row_idx out of range", e);
      if (e > p->col_ptr[j] && r <= p->row_idx[e - 1])
        return fail(err, "row_idx must be strictly increasing within a column", e);
    }
  }
  if (p->patient_weight)
    for (int64_t i = 0; i < N; ++i)
      if (p->patient_weight[i] < 0) return fail(err, "patient_weight must be >= 0", i);
  return SCCS_OK;
}

void build_layout(const sccs_problem* p, int32_t G, Layout& L) {
  const int32_t N = p->n_patients, J = p->n_cols;
  const int64_t K = p->n_rows, nnz = p->nnz;
  L.N = N; L.J = J; L.G = G; L.K = K; L.nnz = nnz;

  // patient ranges balanced by era count
  L.pb.assign(G + 1, 0);
  {
    int64_t i = 0;
    for (int32_t b = 1; b < G; ++b) {
      int64_t target = (K * (int64_t)b) / G;
      while (i < N && p->patient_ptr[i] < target) ++i;
      L.pb[b] = (int32_t)i;
    }
    L.pb[G] = N;
    for (int32_t b = 1; b <= G; ++b) L.pb[b] = std::max(L.pb[b], L.pb[b - 1]);
  }
  std::vector<int32_t> owner(N);
  for (int32_t b = 0; b < G; ++b)
    for (int32_t i = L.pb[b]; i < L.pb[b + 1]; ++i) owner[i] = b;

  L.pptr.resize((size_t)N + 1);
  std::vector<int32_t> era_pid((size_t)K);
  for (int32_t i = 0; i < N; ++i) {
    L.pptr[i] = (int32_t)p->patient_ptr[i];
    for (int64_t k = p->patient_ptr[i]; k < p->patient_ptr[i + 1]; ++k) era_pid[k] = i;
  }
  L.pptr[N] = (int32_t)K;

  L.rp.resize((size_t)nnz * 2);
  for (int64_t e = 0; e < nnz; ++e) {
    int32_t r = p->row_idx[e];
    L.rp[2 * e] = (uint32_t)r;
    L.rp[2 * e + 1] = (uint32_t)era_pid[r];
  }

  // tiles
  L.tile_start.clear();
  L.tile_start.reserve((size_t)(nnz / 32 + (int64_t)J * 4 + 16));
  L.own.assign((size_t)J * (G + 1), 0);
  L.max_tiles_per_wg = 0;
  for (int32_t j = 0; j < J; ++j) {
    int64_t e = p->col_ptr[j], end = p->col_ptr[j + 1];
    for (int32_t b = 0; b < G; ++b) {
      int32_t first = (int32_t)L.tile_start.size();
      L.own[(size_t)j * (G + 1) + b] = first;
      int64_t cur_start = -1, cur_len = 0;
      while (e < end && owner[era_pid[p->row_idx[e]]] == b) {
        // one patient segment
        int32_t pid = era_pid[p->row_idx[e]];
        int64_t s = e;
        while (e < end && era_pid[p->row_idx[e]] == pid) ++e;
        int64_t seg = e - s;
        if (seg > kTile) {
          L.tile_start.push_back((int32_t)s);  // long tile, one patient
          cur_start = -1; cur_len = 0;
        } else if (cur_start < 0 || cur_len + seg > kTile) {
          L.tile_start.push_back((int32_t)s);
          cur_start = s; cur_len = seg;
        } else {
          cur_len += seg;
        }
      }
      int32_t nt = (int32_t)L.tile_start.size() - first;
      L.max_tiles_per_wg = std::max(L.max_tiles_per_wg, nt);
    }
    L.own[(size_t)j * (G + 1) + G] = (int32_t)L.tile_start.size();
  }
  L.tile_start.push_back((int32_t)nnz);

  // compressed row storage of X (columns ascending within a row)
  L.era_ptr.assign((size_t)K + 1, 0);
  for (int64_t e = 0; e < nnz; ++e) L.era_ptr[(size_t)p->row_idx[e] + 1]++;
  for (int64_t k = 0; k < K; ++k) L.era_ptr[k + 1] += L.era_ptr[k];
  L.era_col.resize((size_t)nnz);
  std::vector<int32_t> fill(L.era_ptr.begin(), L.era_ptr.end() - 1);
  for (int32_t j = 0; j < J; ++j)
    for (int64_t e = p->col_ptr[j]; e < p->col_ptr[j + 1]; ++e)
      L.era_col[(size_t)fill[p->row_idx[e]]++] = j;
}

}  // namespace sccs
