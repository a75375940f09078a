// Host layout builder for libsccs (see sccs_layout.hpp).  Loops over
// patients, nonzeros and columns run on a few host threads (std::thread, so
// no OpenMP runtime is pulled into processes that already carry one).
#include "sccs_layout.hpp"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <limits>
#include <thread>

namespace sccs {

namespace {

int host_threads() {
  unsigned n = std::thread::hardware_concurrency();
  if (n == 0) n = 4;
  return (int)std::min(n, 16u);
}

// f(lo, hi) over [0, n) split into contiguous chunks, one per thread.
template <typename F>
void parallel_ranges(int64_t n, F f, int max_threads = 1 << 30, int64_t min_n = 1 << 16) {
  const int T = std::max(1, std::min(host_threads(), max_threads));
  if (n < min_n || T == 1) {
    f((int64_t)0, n);
    return;
  }
  std::vector<std::thread> th;
  th.reserve(T);
  for (int t = 0; t < T; ++t) {
    int64_t lo = n * t / T, hi = n * (t + 1) / T;
    th.emplace_back([=] { f(lo, hi); });
  }
  for (auto& x : th) x.join();
}

sccs_status fail(std::string& err, const char* msg, long long a = -1) {
  char buf[256];
  if (a >= 0)
    std::snprintf(buf, sizeof buf, "%s (at %lld)", msg, a);
  else
    std::snprintf(buf, sizeof buf, "%s", msg);
  err = buf;
  return SCCS_ERR_INVALID_ARG;
}

}  // namespace

sccs_status validate_problem(const sccs_problem* p, std::string& err) {
  if (!p) return fail(err, "problem is NULL");
  if (p->n_patients < 1 || p->n_rows < 1 || p->n_cols < 1)
    return fail(err, "n_patients, n_rows and n_cols must be >= 1");
  if (p->n_rows >= (int64_t)std::numeric_limits<int32_t>::max())
    return fail(err, "n_rows must be < 2^31");
  if (p->n_patients > (int32_t)kPidMask) return fail(err, "n_patients must be < 2^28");
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
  // first offending index (or -1) per check, found in parallel
  std::atomic<int64_t> bad_len{-1}, bad_cnt{-1}, bad_evt{-1};
  parallel_ranges(K, [&](int64_t lo, int64_t hi) {
    for (int64_t k = lo; k < hi; ++k) {
      if (p->offset[k] < 0) { bad_len = k; return; }
      if (p->count[k] < 0) { bad_cnt = k; return; }
      if (p->count[k] > 0 && p->offset[k] == 0) { bad_evt = k; return; }
    }
  });
  if (bad_len >= 0) return fail(err, "offset (era length) must be >= 0", bad_len);
  if (bad_cnt >= 0) return fail(err, "count must be >= 0", bad_cnt);
  if (bad_evt >= 0) return fail(err, "an era with events must have positive length", bad_evt);
  std::atomic<int64_t> bad_range{-1}, bad_order{-1};
  parallel_ranges(J, [&](int64_t lo, int64_t hi) {
    for (int64_t j = lo; j < hi; ++j) {
      for (int64_t e = p->col_ptr[j]; e < p->col_ptr[j + 1]; ++e) {
        int32_t r = p->row_idx[e];
        if (r < 0 || r >= K) { bad_range = e; return; }
        if (e > p->col_ptr[j] && r <= p->row_idx[e - 1]) { bad_order = e; return; }
      }
    }
  });
  if (bad_range >= 0) return fail(err, "row_idx out of range", bad_range);
  if (bad_order >= 0) return fail(err, "row_idx must be strictly increasing within a column", bad_order);
  if (p->patient_weight)
    for (int64_t i = 0; i < N; ++i)
      if (p->patient_weight[i] < 0) return fail(err, "patient_weight must be >= 0", i);
  if (p->value)
    for (int64_t e = 0; e < p->nnz; ++e)
      if (!std::isfinite(p->value[e])) return fail(err, "covariate values must be finite", e);
  return SCCS_OK;
}

int64_t tile_bound(int64_t nnz, int32_t J, int32_t G, int32_t tile_nnz) {
  // Within one (column, workgroup) range, two consecutive tiles hold more
  // than tile_nnz nonzeros together (greedy packing; a long tile alone
  // does), so a range with c nonzeros has fewer than 2c/tile_nnz + 2 tiles.
  const int64_t ranges = std::min<int64_t>(nnz, (int64_t)J * G);
  return 2 * nnz / tile_nnz + 2 * ranges + 1;
}

void build_layout(const sccs_problem* p, int32_t G, Layout& L, int32_t tile_nnz, int32_t max_group) {
  const int32_t N = p->n_patients, J = p->n_cols;
  const int64_t K = p->n_rows, nnz = p->nnz;
  L.N = N; L.J = J; L.G = G; L.K = K; L.nnz = nnz; L.tile_nnz = tile_nnz;
  if (max_group < 1) max_group = 1;
  if (max_group > kMaxGroup) max_group = kMaxGroup;

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

  L.pptr.resize((size_t)N + 1);
  std::vector<int32_t> era_pid((size_t)K);
  parallel_ranges(N, [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) {
      L.pptr[i] = (int32_t)p->patient_ptr[i];
      for (int64_t k = p->patient_ptr[i]; k < p->patient_ptr[i + 1]; ++k) era_pid[k] = (int32_t)i;
    }
  });
  L.pptr[N] = (int32_t)K;

  // column groups: greedy runs of pairwise patient-disjoint columns
  L.gcol.assign(1, 0);
  if (max_group == 1) {
    for (int32_t j = 1; j <= J; ++j) L.gcol.push_back(j);
  } else {
    std::vector<int32_t> stamp((size_t)N, -1);
    int32_t gid = 0, size = 0;
    for (int32_t j = 0; j < J; ++j) {
      bool clash = size >= max_group;
      for (int64_t e = p->col_ptr[j]; e < p->col_ptr[j + 1] && !clash; ++e)
        clash = stamp[era_pid[p->row_idx[e]]] == gid;
      if (clash) {
        L.gcol.push_back(j);
        ++gid;
        size = 0;
      }
      for (int64_t e = p->col_ptr[j]; e < p->col_ptr[j + 1]; ++e) stamp[era_pid[p->row_idx[e]]] = gid;
      ++size;
    }
    L.gcol.push_back(J);
  }
  const int32_t NG = (int32_t)L.gcol.size() - 1;
  L.n_groups = NG;

  // pass descriptors: which of the kLinkCols columns before group g share a
  // patient with g (blocks of groups in parallel, one patient stamp per
  // thread, at most about 256 MB of stamps)
  L.gdesc.assign((size_t)NG, 0u);
  if (J < kDescMaxCols) {
    const int stamp_threads = (int)std::max<int64_t>(1, ((int64_t)256 << 20) / (4 * (int64_t)N + 1));
    parallel_ranges(NG, [&](int64_t glo, int64_t ghi) {
      std::vector<int32_t> stamp((size_t)N, -1);
      for (int64_t g = glo; g < ghi; ++g) {
        const int32_t j0 = L.gcol[g], m = L.gcol[g + 1] - L.gcol[g];
        for (int32_t j = j0; j < j0 + m; ++j)
          for (int64_t e = p->col_ptr[j]; e < p->col_ptr[j + 1]; ++e) stamp[era_pid[p->row_idx[e]]] = (int32_t)g;
        uint32_t lmask = 0u;
        for (int32_t i = 0; i < kLinkCols; ++i) {
          const int32_t c = j0 - kLinkCols + i;
          if (c < 0) continue;
          bool hit = false;
          for (int64_t e = p->col_ptr[c]; e < p->col_ptr[c + 1] && !hit; ++e) hit = stamp[era_pid[p->row_idx[e]]] == g;
          if (hit) lmask |= 1u << i;
        }
        L.gdesc[g] = (uint32_t)j0 | ((uint32_t)m << kDescWidthShift) | (lmask << kDescLinkShift);
      }
    }, stamp_threads, 64);
  }

  // cwb[j*(G+1) + b]: first CSC position of column j at or after workgroup b's eras
  std::vector<int64_t> cwb((size_t)J * (G + 1));
  parallel_ranges(J, [&](int64_t jlo, int64_t jhi) {
    for (int64_t j = jlo; j < jhi; ++j) {
      const int32_t* r0 = p->row_idx + p->col_ptr[j];
      const int32_t* r1 = p->row_idx + p->col_ptr[j + 1];
      for (int32_t b = 0; b < G; ++b) {
        const int64_t era0 = p->patient_ptr[L.pb[b]];
        cwb[(size_t)j * (G + 1) + b] = (int64_t)(std::lower_bound(r0, r1, (int32_t)era0) - p->row_idx);
      }
      cwb[(size_t)j * (G + 1) + G] = p->col_ptr[j + 1];
    }
  });
  // start of each (group, workgroup) block in the group order
  std::vector<int64_t> bstart((size_t)NG * G + 1, 0);
  for (int32_t g = 0; g < NG; ++g)
    for (int32_t b = 0; b < G; ++b) {
      int64_t n = 0;
      for (int32_t j = L.gcol[g]; j < L.gcol[g + 1]; ++j)
        n += cwb[(size_t)j * (G + 1) + b + 1] - cwb[(size_t)j * (G + 1) + b];
      bstart[(size_t)g * G + b + 1] = bstart[(size_t)g * G + b] + n;
    }

  // (row, patient | column-in-group) in group order, and the covariate
  // values in the same order
  L.rp.resize((size_t)nnz * 2);
  if (p->value) L.val.resize((size_t)nnz);
  parallel_ranges(NG, [&](int64_t glo, int64_t ghi) {
    for (int64_t g = glo; g < ghi; ++g)
      for (int32_t b = 0; b < G; ++b) {
        int64_t pos = bstart[(size_t)g * G + b];
        for (int32_t j = L.gcol[g]; j < L.gcol[g + 1]; ++j) {
          const uint32_t c = (uint32_t)(j - L.gcol[g]) << kGroupShift;
          for (int64_t e = cwb[(size_t)j * (G + 1) + b]; e < cwb[(size_t)j * (G + 1) + b + 1]; ++e, ++pos) {
            const int32_t r = p->row_idx[e];
            L.rp[2 * pos] = (uint32_t)r;
            L.rp[2 * pos + 1] = (uint32_t)era_pid[r] | c;
            if (p->value) L.val[(size_t)pos] = p->value[e];
          }
        }
      }
  });

  // tiles, group by group in parallel: tile starts of group g, and the
  // number of tiles of each (g, b) block
  std::vector<std::vector<int32_t>> grp_tiles(NG);
  std::vector<int32_t> range_tiles((size_t)NG * G, 0);
  parallel_ranges(NG, [&](int64_t glo, int64_t ghi) {
    for (int64_t g = glo; g < ghi; ++g) {
      std::vector<int32_t>& ts = grp_tiles[g];
      for (int32_t b = 0; b < G; ++b) {
        const size_t first = ts.size();
        int64_t e = bstart[(size_t)g * G + b];
        const int64_t end = bstart[(size_t)g * G + b + 1];
        int64_t cur_len = -1;
        while (e < end) {
          const uint32_t key = L.rp[2 * e + 1];
          const int64_t s = e;
          while (e < end && L.rp[2 * e + 1] == key) ++e;
          const int64_t seg = e - s;
          if (seg > tile_nnz) {
            ts.push_back((int32_t)s);  // a segment longer than a tile: a tile of its own
            cur_len = -1;
          } else if (cur_len < 0 || cur_len + seg > tile_nnz) {
            ts.push_back((int32_t)s);
            cur_len = seg;
          } else {
            cur_len += seg;
          }
        }
        range_tiles[(size_t)g * G + b] = (int32_t)(ts.size() - first);
      }
    }
  });
  std::vector<int64_t> grp_first((size_t)NG + 1, 0);
  for (int32_t g = 0; g < NG; ++g) grp_first[g + 1] = grp_first[g] + (int64_t)grp_tiles[g].size();
  L.tile_start.resize((size_t)grp_first[NG] + 1);
  L.own.assign((size_t)NG * (G + 1), 0);
  std::atomic<int32_t> max_per_wg{0};
  parallel_ranges(NG, [&](int64_t glo, int64_t ghi) {
    int32_t mx = 0;
    for (int64_t g = glo; g < ghi; ++g) {
      std::copy(grp_tiles[g].begin(), grp_tiles[g].end(), L.tile_start.begin() + grp_first[g]);
      int64_t t = grp_first[g];
      for (int32_t b = 0; b < G; ++b) {
        L.own[(size_t)g * (G + 1) + b] = (int32_t)t;
        t += range_tiles[(size_t)g * G + b];
        mx = std::max(mx, range_tiles[(size_t)g * G + b]);
      }
      L.own[(size_t)g * (G + 1) + G] = (int32_t)t;
    }
    int32_t cur = max_per_wg.load();
    while (mx > cur && !max_per_wg.compare_exchange_weak(cur, mx)) {
    }
  });
  L.tile_start[grp_first[NG]] = (int32_t)nnz;
  L.max_tiles_per_wg = max_per_wg.load();

  // compressed row storage of X (columns ascending within a row)
  L.era_ptr.assign((size_t)K + 1, 0);
  for (int64_t e = 0; e < nnz; ++e) L.era_ptr[(size_t)p->row_idx[e] + 1]++;
  for (int64_t k = 0; k < K; ++k) L.era_ptr[k + 1] += L.era_ptr[k];
  L.era_col.resize((size_t)nnz);
  if (p->value) L.era_val.resize((size_t)nnz);
  std::vector<int32_t> fill(L.era_ptr.begin(), L.era_ptr.end() - 1);
  for (int32_t j = 0; j < J; ++j)
    for (int64_t e = p->col_ptr[j]; e < p->col_ptr[j + 1]; ++e) {
      const int32_t slot = fill[p->row_idx[e]]++;
      L.era_col[(size_t)slot] = j;
      if (p->value) L.era_val[(size_t)slot] = p->value[e];
    }
}

}  // namespace sccs

namespace sccs {

void host_ytx(const sccs_problem* p, const int32_t* weight, std::vector<double>& ytx) {
  const int32_t N = p->n_patients, J = p->n_cols;
  std::vector<int32_t> era_pid((size_t)p->n_rows);
  for (int32_t i = 0; i < N; ++i)
    for (int64_t k = p->patient_ptr[i]; k < p->patient_ptr[i + 1]; ++k) era_pid[k] = i;
  ytx.assign((size_t)J, 0.0);
  parallel_ranges(J, [&](int64_t jlo, int64_t jhi) {
    for (int64_t j = jlo; j < jhi; ++j) {
      double s = 0.0;
      for (int64_t e = p->col_ptr[j]; e < p->col_ptr[j + 1]; ++e) {
        const int32_t r = p->row_idx[e];
        const double om = weight ? (double)weight[era_pid[r]] : 1.0;
        s += p->value ? om * (double)p->count[r] * p->value[e] : om * (double)p->count[r];
      }
      ytx[j] = s;
    }
  });
}

}  // namespace sccs

namespace sccs {

void independent_order(const sccs_problem* p, int32_t width, std::vector<int32_t>& order) {
  const int32_t N = p->n_patients, J = p->n_cols;
  if (width < 1) width = 1;
  std::vector<int32_t> era_pid((size_t)p->n_rows);
  parallel_ranges(N, [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i)
      for (int64_t k = p->patient_ptr[i]; k < p->patient_ptr[i + 1]; ++k) era_pid[k] = (int32_t)i;
  });
  // distinct patients of each column (its rows are strictly increasing and
  // eras are stored patient by patient, so a column's patients come in
  // non-decreasing order: dropping repeats leaves each once), columns in
  // parallel; then per patient a slot for each column it appears in (the
  // groups it has joined so far)
  std::vector<int64_t> pat_ptr((size_t)J + 1, 0);
  parallel_ranges(J, [&](int64_t lo, int64_t hi) {
    for (int64_t j = lo; j < hi; ++j) {
      int64_t n = 0;
      int32_t last = -1;
      for (int64_t e = p->col_ptr[j]; e < p->col_ptr[j + 1]; ++e) {
        const int32_t i = era_pid[p->row_idx[e]];
        n += i != last;
        last = i;
      }
      pat_ptr[(size_t)j + 1] = n;
    }
  }, 1 << 30, 64);
  for (int32_t j = 0; j < J; ++j) pat_ptr[(size_t)j + 1] += pat_ptr[j];
  std::vector<int32_t> pats((size_t)pat_ptr[J]);
  parallel_ranges(J, [&](int64_t lo, int64_t hi) {
    for (int64_t j = lo; j < hi; ++j) {
      int64_t q = pat_ptr[j];
      int32_t last = -1;
      for (int64_t e = p->col_ptr[j]; e < p->col_ptr[j + 1]; ++e) {
        const int32_t i = era_pid[p->row_idx[e]];
        if (i != last) pats[(size_t)q++] = i;
        last = i;
      }
    }
  }, 1 << 30, 64);
  std::vector<int32_t> n_of((size_t)N, 0);
  for (const int32_t i : pats) ++n_of[i];
  std::vector<int64_t> memb_ptr((size_t)N + 1, 0);
  for (int32_t i = 0; i < N; ++i) memb_ptr[(size_t)i + 1] = memb_ptr[i] + n_of[i];
  std::vector<int32_t> memb((size_t)memb_ptr[N]);
  std::vector<int32_t> filled((size_t)N, 0);
  // visiting order: decreasing nonzeros, ties by column index
  std::vector<int32_t> visit((size_t)J);
  for (int32_t j = 0; j < J; ++j) visit[j] = j;
  std::stable_sort(visit.begin(), visit.end(), [&](int32_t x, int32_t y) {
    return p->col_ptr[x + 1] - p->col_ptr[x] > p->col_ptr[y + 1] - p->col_ptr[y];
  });
  // Columns are placed one after another (each placement depends on the
  // groups so far), but the two per-patient loops of a placement -- marking
  // the groups the column's patients are in, and recording the new
  // membership -- run on T threads over slices of the column's patients,
  // kept in step by a spinning barrier.  Thread 0 picks the group.
  std::vector<std::vector<int32_t>> groups;
  std::vector<int32_t> open;   // groups with room, in creation order
  const int T = std::max(1, std::min(host_threads(), 8));
  std::vector<std::vector<uint64_t>> bits((size_t)T);
  std::atomic<int> arrived{0}, phase{0};
  int32_t chosen = 0;
  auto barrier = [&](int& my_phase) {
    if (arrived.fetch_add(1) == T - 1) {
      arrived.store(0);
      phase.fetch_add(1);
    } else {
      while (phase.load() == my_phase) std::this_thread::yield();
    }
    ++my_phase;
  };
  auto worker = [&](int t) {
    int my_phase = 0;
    for (const int32_t j : visit) {
      const int64_t q0 = pat_ptr[j], q1 = pat_ptr[(size_t)j + 1];
      const int64_t lo = q0 + (q1 - q0) * t / T, hi = q0 + (q1 - q0) * (t + 1) / T;
      std::vector<uint64_t>& mine = bits[(size_t)t];
      mine.assign((groups.size() + 63) / 64, 0ull);
      for (int64_t q = lo; q < hi; ++q) {
        const int32_t i = pats[q];
        for (int64_t m = memb_ptr[i]; m < memb_ptr[i] + filled[i]; ++m) mine[memb[m] >> 6] |= 1ull << (memb[m] & 63);
      }
      barrier(my_phase);
      if (t == 0) {
        for (int u = 1; u < T; ++u)
          for (size_t x = 0; x < mine.size(); ++x) mine[x] |= bits[(size_t)u][x];
        int32_t g = -1;
        size_t oi = 0;
        for (; oi < open.size(); ++oi)
          if (!((mine[(size_t)open[oi] >> 6] >> (open[oi] & 63)) & 1ull)) { g = open[oi]; break; }
        if (g < 0) {
          g = (int32_t)groups.size();
          groups.emplace_back();
          open.push_back(g);
          oi = open.size() - 1;
        }
        groups[g].push_back(j);
        if ((int32_t)groups[g].size() >= width) open.erase(open.begin() + (ptrdiff_t)oi);
        chosen = g;
      }
      barrier(my_phase);
      // each patient appears once in the column: no two threads touch one list
      for (int64_t q = lo; q < hi; ++q) {
        const int32_t i = pats[q];
        memb[memb_ptr[i] + filled[i]++] = chosen;
      }
      barrier(my_phase);
    }
  };
  {
    std::vector<std::thread> th;
    for (int t = 1; t < T; ++t) th.emplace_back(worker, t);
    worker(0);
    for (auto& x : th) x.join();
  }
  order.clear();
  order.reserve((size_t)J);
  for (const auto& gr : groups) order.insert(order.end(), gr.begin(), gr.end());
}

void permute_columns(const sccs_problem* src, const std::vector<int32_t>& order, PermutedProblem& out) {
  const int32_t J = src->n_cols;
  out.col_ptr.assign((size_t)J + 1, 0);
  for (int32_t k = 0; k < J; ++k)
    out.col_ptr[(size_t)k + 1] = out.col_ptr[k] + (src->col_ptr[order[k] + 1] - src->col_ptr[order[k]]);
  out.row_idx.resize((size_t)src->nnz);
  if (src->value) out.value.resize((size_t)src->nnz);
  else out.value.clear();
  parallel_ranges(J, [&](int64_t lo, int64_t hi) {
    for (int64_t k = lo; k < hi; ++k) {
      const int64_t s0 = src->col_ptr[order[k]], n = src->col_ptr[order[k] + 1] - s0;
      std::copy(src->row_idx + s0, src->row_idx + s0 + n, out.row_idx.begin() + out.col_ptr[k]);
      if (src->value) std::copy(src->value + s0, src->value + s0 + n, out.value.begin() + out.col_ptr[k]);
    }
  }, 1 << 30, 64);
  out.p = *src;
  out.p.col_ptr = out.col_ptr.data();
  out.p.row_idx = out.row_idx.data();
  out.p.value = src->value ? out.value.data() : nullptr;
}

}  // namespace sccs
