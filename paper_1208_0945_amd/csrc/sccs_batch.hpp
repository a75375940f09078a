// Batched form: F independent fits (different outcomes, or cross-validation
// folds) advanced in lockstep by one cooperative persistent launch.
//
// All fits share the coordinate order j = 0..J-1 and the workgroup count G;
// workgroup b owns patient range b of every fit's problem.  When all fits
// share one problem (cross-validation folds, bootstrap replicates) they also
// share its column groups (consecutive, pairwise patient-disjoint columns,
// up to m columns with F m <= 64); otherwise every group is one column.  Per
// group, every workgroup computes its partials (G_fc, H_fc) for each active
// fit and column, ONE device-wide reduction carries all 2 F m partials (so
// its latency is paid once for all fits and columns), then each (fit,
// column) takes its own Newton / trust-region step (Eq. 4) and its own
// sparse update.  Each fit walks a chain of priors in
// order -- the warm starts along the prior-variance path used for
// cross-validation (Section 2.5) -- with its trust region reset at the start
// of every link; a link ends when its stopping rule holds or after
// max_sweeps sweeps, and the fit's beta and result are recorded.
#pragma once
#include <hip/hip_runtime.h>

#include "sccs.h"
#include "sccs_device.hpp"
#include "sccs_kernels.hpp"

namespace sccs {

constexpr int kMaxFits = 64;
constexpr int kBatchSlotWords = 2 * kMaxFits;   // 2 F m words per workgroup slot (F m <= 64)
// Slots of one class (group width m), both parities: level 1 and level 2.
constexpr size_t kBatchSlots1 = (size_t)2 * kMaxWorkgroups * kBatchSlotWords;
constexpr size_t kBatchSlots2 = (size_t)2 * kReplicas * kGroups * kBatchSlotWords;

// Fit of poller lane f m + c (m = 1..4, no general division).
__device__ __forceinline__ int fit_of(int lane, int m) {
  return m == 1 ? lane : m == 2 ? lane >> 1 : m == 4 ? lane >> 2 : lane / 3;
}

struct LinkResult {
  int32_t sweeps;
  int32_t converged;
  double loglik;
  double logpost;
  double heldout;   // Eq. 2 over the fit's weight-0 patients (fits with weights)
};

// Device-resident description of one fit of a batch.
struct BatchFit {
  KArgs k;                   // problem layout and this fit's w, pat, ytx
  double2* bt;               // [G][J] per-workgroup copies of (beta_j, trust_j)
  const int32_t* link_kind;  // [n_links] prior kinds
  const double* link_var;    // [n_links] prior variances
  int32_t n_links;
  int32_t pad;
  double* beta_out;          // [n_links][J]
  LinkResult* res_out;       // [n_links]
  const double* ho_n;        // [N] n_i of weight-0 patients, else 0; NULL without weights
  const double* ytx_ho;      // [J] Y'X_j over the weight-0 patients
};

struct BatchArgs {
  const BatchFit* fits;
  uint64_t* s1;              // [kMaxGroup classes][2][256][kBatchSlotWords]
  uint64_t* s2;              // [kMaxGroup classes][2][kReplicas][8][kBatchSlotWords]
  const int32_t* gcol;       // [n_groups + 1] column groups, shared by all fits (one problem, or width 1)
  int32_t n_groups;
  Ctrl* ctrl;
  int32_t F, G, J;
  int32_t max_sweeps;        // per link
  int32_t criterion;         // FIXED or REL_LOGPOST
  int32_t refresh_period;
  double tol;
};

// Poll the first nv words of n_members tagged slots, slot m at
// base + m * stride, spread over the workgroup: thread tid watches word
// tid % kBatchSlotWords of members tid / kBatchSlotWords + q * kMembersPerPass,
// keeping all of its loads in flight at once.  Decoded values go to
// stage[m * kBatchSlotWords + word].  On timeout/abort *flag is cleared.
constexpr int kMembersPerPass = kBlock / kBatchSlotWords;
constexpr int kPollPer = 32 / kMembersPerPass;   // up to 32 members per level
__device__ __forceinline__ void poll_spread(const uint64_t* base, size_t stride, int n_members, int nv, uint32_t tag,
                                            double* stage, Ctrl* ctrl, int* flag) {
  const int word = threadIdx.x % kBatchSlotWords, m0 = threadIdx.x / kBatchSlotWords;
  uint32_t need = 0;
  if (word < nv) {
#pragma unroll
    for (int q = 0; q < kPollPer; ++q)
      if (m0 + q * kMembersPerPass < n_members) need |= 1u << q;
  }
  long long spins = 0;
  while (need) {
    // issue every outstanding load of the round, then inspect them
    uint64_t x[kPollPer];
#pragma unroll
    for (int q = 0; q < kPollPer; ++q)
      x[q] = (need & (1u << q)) ? load_agent(base + (size_t)(m0 + q * kMembersPerPass) * stride + word) : 0ull;
#pragma unroll
    for (int q = 0; q < kPollPer; ++q) {
      if ((need & (1u << q)) && (uint32_t)(x[q] >> 63) == tag) {
        stage[(m0 + q * kMembersPerPass) * kBatchSlotWords + word] = tag_decode(x[q]);
        need &= ~(1u << q);
      }
    }
    if (!need) break;
    if (++spins > kSpinLimit) {
      __hip_atomic_store(&ctrl->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&ctrl->status, (int)SCCS_ERR_SYNC, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      *flag = 0;
      return;
    }
    if ((spins & 255) == 0 && load_agent_i(&ctrl->abort)) { *flag = 0; return; }
    if (kPollSleep) __builtin_amdgcn_s_sleep(kPollSleep);
  }
}

// Device-wide sum of nv (<= kBatchSlotWords) non-negative words per
// workgroup, all threads of every workgroup taking part; same two-level
// tagged scheme as allreduce2_wave.  part[] (LDS) holds the workgroup's
// words; out[] (LDS) receives the sums.  stage is LDS of 32 *
// kBatchSlotWords doubles.  Returns false in all threads on timeout/abort.
__device__ bool batch_allreduce(uint64_t* s1, uint64_t* s2, uint32_t seq, int G, int nv, Ctrl* ctrl,
                                const double* part, double* out, double* stage, int* flag) {
  const int tid = threadIdx.x, b = blockIdx.x;
  const uint32_t par = seq & 1u, tag = (seq >> 1) & 1u;
  const int ng = G < kGroups ? G : kGroups;
  uint64_t* L1 = s1 + (size_t)par * kMaxWorkgroups * kBatchSlotWords;
  uint64_t* L2 = s2 + (size_t)par * kReplicas * kGroups * kBatchSlotWords;
  if (tid == 0) *flag = 1;
  if (tid < nv) store_agent(L1 + (size_t)b * kBatchSlotWords + tid, tag_encode(part[tid], tag));
  __syncthreads();
  if (b < ng) {
    const int members = (G - b + ng - 1) / ng;
    poll_spread(L1 + (size_t)b * kBatchSlotWords, (size_t)ng * kBatchSlotWords, members, nv, tag, stage, ctrl, flag);
    __syncthreads();
    if (tid < nv && *flag) {
      double s = 0.0;
      for (int m = 0; m < members; ++m) s += stage[m * kBatchSlotWords + tid];
      for (int r = 0; r < kReplicas; ++r)
        store_agent(L2 + ((size_t)r * kGroups + b) * kBatchSlotWords + tid, tag_encode(s, tag));
    }
  }
  __syncthreads();
  if (*flag) {
    const int r = b % kReplicas;
    poll_spread(L2 + (size_t)r * kGroups * kBatchSlotWords, kBatchSlotWords, ng, nv, tag, stage, ctrl, flag);
  }
  __syncthreads();
  if (tid < nv) {
    double s = 0.0;
    for (int g = 0; g < ng; ++g) s += stage[g * kBatchSlotWords + tid];
    out[tid] = s;
  }
  __syncthreads();
  return *flag != 0;
}

// Device-wide sum of the W = 2F words of every workgroup by ONE wave (the
// poller) per workgroup; same tagged two-level scheme and slots as
// batch_allreduce, with level 1 cut into slices of kSliceWords words so that
// no lane keeps more than 8 polls in flight.  The leader of (member group g,
// slice s) is workgroup (g + ng s) mod G; it sums its group's 32 members
// over the slice (each lane four of them, then the four lanes of a word in
// fixed order) and publishes the slice of the group total to every replica.
// Every workgroup then polls the ng group totals of its replica and sums
// them in group order into out[] (LDS).  part[w] is in lane w % 64 of the
// wave at index w / 64.  Returns false (whole wave) on timeout/abort.
constexpr int kSliceWords = 16;
constexpr int kL2Per = kGroups * kBatchSlotWords / 64;   // level-2 polls per lane (16)

// Poll words base[off[q]] (q < n for this lane, n <= NQ) until their tag
// matches; decoded word q lands in dst[q * 64 + lane] (LDS).  All loads of a
// round are issued before any is inspected.  Returns false (whole wave) on
// timeout/abort.
template <int NQ>
__device__ __forceinline__ bool poll_words(const uint64_t* base, const int* off, int n, uint32_t tag, double* dst,
                                           Ctrl* ctrl) {
  const int lane = threadIdx.x & 63;
  uint32_t need = (1u << n) - 1u;
  long long spins = 0;
  bool ok = true;
  while (true) {
    uint64_t x[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) x[q] = (need & (1u << q)) ? load_agent(base + off[q]) : 0ull;
#pragma unroll
    for (int q = 0; q < NQ; ++q)
      if ((need & (1u << q)) && (uint32_t)(x[q] >> 63) == tag) {
        dst[q * 64 + lane] = tag_decode(x[q]);
        need &= ~(1u << q);
      }
    if (__ballot(need != 0) == 0ull) break;
    if (++spins > kSpinLimit) {
      if (lane == 0) {
        __hip_atomic_store(&ctrl->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&ctrl->status, (int)SCCS_ERR_SYNC, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      ok = false;
      break;
    }
    if ((spins & 255) == 0 && load_agent_i(&ctrl->abort)) { ok = false; break; }
    if (kPollSleep) __builtin_amdgcn_s_sleep(kPollSleep);
  }
  return __ballot(!ok) == 0ull;
}

// stage: LDS of at least 2 * kL2Per * 64 doubles.
__device__ bool batch_reduce_poller(uint64_t* s1, uint64_t* s2, uint32_t seq, int G, int W, Ctrl* ctrl,
                                    const double* part0, const double* part1, double* out, double* stage) {
  const int lane = threadIdx.x & 63, b = blockIdx.x;
  const uint32_t par = seq & 1u, tag = (seq >> 1) & 1u;
  const int ng = G < kGroups ? G : kGroups;
  const int S = (W + kSliceWords - 1) / kSliceWords;
  uint64_t* L1 = s1 + (size_t)par * kMaxWorkgroups * kBatchSlotWords;
  uint64_t* L2 = s2 + (size_t)par * kReplicas * kGroups * kBatchSlotWords;
  double* st1 = stage;                   // [8][64] level-1 values
  double* st2 = stage + kL2Per * 64;     // [kL2Per][64] level-2 values
  if (lane < W) store_agent(L1 + (size_t)b * kBatchSlotWords + lane, tag_encode(*part0, tag));
  if (lane + 64 < W) store_agent(L1 + (size_t)b * kBatchSlotWords + lane + 64, tag_encode(*part1, tag));
  constexpr int NQ = 8;
  int off[NQ];
  // level 1: the (group, slice) pairs this workgroup leads
  for (int pidx = b; pidx < ng * S; pidx += G) {
    const int g = pidx % ng, sl = pidx / ng;
    const int members = (G - g + ng - 1) / ng;
    const int w = sl * kSliceWords + (lane & 15);
    const int k0 = lane >> 4;
    int n = 0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int k = k0 + 4 * q;
      off[q] = (g + (k < members ? k : 0) * ng) * kBatchSlotWords + (w < W ? w : 0);
      if (w < W && k < members) n = q + 1;
    }
    if (!poll_words<NQ>(L1, off, n, tag, st1, ctrl)) return false;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    double acc = 0.0;
    for (int q = 0; q < n; ++q) acc += st1[q * 64 + lane];
    acc += __shfl_xor(acc, 16, 64);
    acc += __shfl_xor(acc, 32, 64);
    if (lane < 16 && w < W)
      for (int r = 0; r < kReplicas; ++r)
        store_agent(L2 + ((size_t)r * kGroups + g) * kBatchSlotWords + w, tag_encode(acc, tag));
  }
  // level 2: the ng group totals of this workgroup's replica
  const int r = b % kReplicas;
  const int items = ng * W;
  const uint64_t* L2r = L2 + (size_t)r * kGroups * kBatchSlotWords;
  for (int q0 = 0; q0 < items; q0 += NQ * 64) {   // passes of NQ polls per lane
    int n = 0;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const int i = q0 + lane + 64 * q;
      off[q] = i < items ? (i / W) * kBatchSlotWords + i % W : 0;
      if (i < items) n = q + 1;
    }
    if (!poll_words<NQ>(L2r, off, n, tag, st2 + q0, ctrl)) return false;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  // lane w sums word w (and w + 64) over the groups, in group order
  for (int w = lane; w < W; w += 64) {
    double t = 0.0;
    for (int g = 0; g < ng; ++g) t += st2[g * W + w];   // item g * W + w sits at st2[(i % 64) + 64 (i / 64)] = st2[i]
    out[w] = t;
  }
  return true;
}

// Waves 0..kBW-1 work on tiles; the last wave runs the device-wide reduction
// and the Newton steps, so that the workers can load the next coordinate's
// indices while it waits.
constexpr int kBW = kWaves - 1;
constexpr int kBPoller = kWaves - 1;

// Worker wave -> (fit, slice) assignment.  With F >= kBW fits each worker
// takes fits w, w + kBW, ... whole; with fewer fits, P = kBW / F workers
// share a fit and take every P-th of its tiles.
struct WaveMap {
  int P;
  __device__ WaveMap(int F) : P(F >= kBW ? 1 : kBW / F) {}
  __device__ int slice(int w) const { return P == 1 ? 0 : w % P; }
};

constexpr int kFitsPerWave = (kMaxFits + kBW - 1) / kBW;   // 10
constexpr int kChunk = 5;   // pairs whose loads a wave keeps in flight together
static_assert(kFitsPerWave % kChunk == 0, "chunks tile the pairs of a wave");

// Offset of worker w among the workers that share fit f's extra tiles.
__device__ __forceinline__ int rot(int w, int f) { return ((w - f) % kBW + kBW) % kBW; }

// Pair q of a worker wave: the fit it works on (F if none).  With P == 1 a
// worker takes fits wave, wave + kBW, ...; with P > 1 only pair 0 is used.
// Pair fits increase with q, so the first pair with f >= F ends the list.
__device__ __forceinline__ int pair_fit(const WaveMap& wm, int wave, int q, int F) {
  if (wm.P == 1) return wave + q * kBW;
  return (q == 0 && wave < F * wm.P) ? wave / wm.P : F;
}

// Index data of coordinate j for every pair of this wave, into the wave's
// LDS rows: ixs[q] = (first tile t0 + slice, end of range t1, e0, len of
// that first tile), ixrp[q][lane] = (row, patient) of its lane-th nonzero.
// Each stage (tile range, tile bounds, nonzeros) is issued for a chunk of
// pairs before any of it is waited on.
__device__ __forceinline__ void pair_index(const BatchArgs& A, const WaveMap& wm, int wave, int j,
                                           const int* s_done, int (*ixs)[4], uint2 (*ixrp)[64]) {
  const int lane = threadIdx.x & 63, b = blockIdx.x;
  const int slice = wm.slice(wave);
#pragma unroll 1
  for (int q0 = 0; q0 < kFitsPerWave; q0 += kChunk) {
    if (pair_fit(wm, wave, q0, A.F) >= A.F) break;
    int t[kChunk], t1[kChunk], e0[kChunk], len[kChunk];
#pragma unroll
    for (int c = 0; c < kChunk; ++c) {
      const int f = pair_fit(wm, wave, q0 + c, A.F);
      t[c] = 0;
      t1[c] = 0;
      if (f < A.F && !s_done[f]) {
        const size_t base = (size_t)j * (A.G + 1) + b;
        t[c] = A.fits[f].k.own[base] + slice;
        t1[c] = A.fits[f].k.own[base + 1];
      }
    }
#pragma unroll
    for (int c = 0; c < kChunk; ++c) {
      const int f = pair_fit(wm, wave, q0 + c, A.F);
      e0[c] = 0;
      len[c] = 0;
      if (f < A.F && t[c] < t1[c]) {
        e0[c] = A.fits[f].k.tile_start[t[c]];
        len[c] = A.fits[f].k.tile_start[t[c] + 1] - e0[c];
      }
    }
#pragma unroll
    for (int c = 0; c < kChunk; ++c) {
      const int f = pair_fit(wm, wave, q0 + c, A.F);
      uint2 rp = make_uint2(0u, 0xffffffffu);
      if (f < A.F && t[c] < t1[c] && len[c] <= 64 && lane < len[c]) rp = A.fits[f].k.rp[e0[c] + lane];
      ixrp[q0 + c][lane] = rp;
      if (lane == 0) {
        ixs[q0 + c][0] = t[c];
        ixs[q0 + c][1] = t1[c];
        ixs[q0 + c][2] = e0[c];
        ixs[q0 + c][3] = len[c];
      }
    }
  }
}

// Fits (bit f) whose range in this workgroup has more tiles than its first,
// read by lane f from the owner's staged indices (whole fits per wave only).
__device__ __forceinline__ uint64_t fits_with_more_tiles(const int (*const* all_ixs)[4], int F, const int* s_done) {
  const int lane = threadIdx.x & 63;
  bool more = false;
  if (lane < F && !s_done[lane]) {
    const int* ix = all_ixs[lane % kBW][lane / kBW];
    more = ix[0] + 1 < ix[1];
  }
  return __ballot(more);
}

// Wave sums of the first m columns' (G, H) of acc, added (add) or stored
// into row[2 (f m + c) + {0, 1}] by lane 0.  Column widths are unrolled
// with compile-time indices.  NC: columns per group at most (1 or
// kMaxGroup; the kernel is instantiated for both).
template <int NC>
__device__ __forceinline__ void put_pair_sums(const Acc<NC>& acc, int m, int f, double* row, bool add) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    if (c < m) {
      const double Gs = wave_sum(acc.g[c]);
      const double Hs = wave_sum(acc.h[c]);
      if (lane == 0) {
        double* r = row + 2 * (f * m + c);
        if (add) {
          r[0] += Gs;
          r[1] += Hs;
        } else {
          r[0] = Gs;
          r[1] = Hs;
        }
      }
    }
  }
}

// Phase A over this wave's pairs for column group (j0 .. j0+m-1): the first
// tiles of a chunk of pairs are gathered together from the staged indices,
// then any further tiles of the pair's range (large columns) are walked one
// by one.  Partials of fit f, column c go to words 2 (f m + c) of the
// wave's row pp[wave] (whole fits per wave) or of its slice's row.
template <typename WT, int NC>
__device__ __forceinline__ void pairs_phase_a(const BatchArgs& A, const WaveMap& wm, int wave, int m, const int* s_done,
                                              const int (*ixs)[4], const uint2 (*ixrp)[64],
                                              const int (*const* all_ixs)[4], double (*pp)[kBatchSlotWords]) {
  const int lane = threadIdx.x & 63, F = A.F;
  const int slice = wm.P == 1 ? wave : wm.slice(wave);
  double* row = pp[slice];
  if (wm.P == 1)
    for (int w = lane; w < 2 * F * m; w += 64) row[w] = 0.0;
#pragma unroll 1
  for (int q0 = 0; q0 < kFitsPerWave; q0 += kChunk) {
    if (pair_fit(wm, wave, q0, F) >= F) break;
    double wv[kChunk], den[kChunk], wn[kChunk];
    bool lead[kChunk];
    int seg_start[kChunk];
    uint32_t pid[kChunk];
#pragma unroll
    for (int c = 0; c < kChunk; ++c) {
      const int f = pair_fit(wm, wave, q0 + c, F);
      const int t = ixs[q0 + c][0], t1 = ixs[q0 + c][1], len = ixs[q0 + c][3];
      const uint2 rp = ixrp[q0 + c][lane];
      pid[c] = rp.y;
      wv[c] = 0.0;
      lead[c] = false;
      seg_start[c] = lane;
      if (f < F && t < t1 && len <= 64) {
        seg_layout(rp.y, lane, len, lead[c], seg_start[c]);
        if (lane < len) wv[c] = (double)((const WT*)A.fits[f].k.w)[rp.x];
      }
    }
#pragma unroll
    for (int c = 0; c < kChunk; ++c) {
      const int f = pair_fit(wm, wave, q0 + c, F);
      den[c] = 1.0;
      wn[c] = 0.0;
      if (lead[c]) {
        const double2 pv = A.fits[f].k.pat[pid_of(pid[c])];
        den[c] = pv.x;
        wn[c] = pv.y;
      }
    }
#pragma unroll
    for (int c = 0; c < kChunk; ++c) {
      const int f = pair_fit(wm, wave, q0 + c, F);
      const double num = seg_sum_v(wv[c], lane, seg_start[c]);
      Acc<NC> acc;
      acc.zero();
      if (lead[c]) acc.add(col_of(pid[c]), num, make_double2(den[c], wn[c]));
      if (f < F) put_pair_sums<NC>(acc, m, f, row, false);
    }
  }
  // a long first tile: its owner
#pragma unroll 1
  for (int q = 0; q < kFitsPerWave; ++q) {
    const int f = pair_fit(wm, wave, q, F);
    if (f >= F) break;
    if (s_done[f]) continue;
    const int t0 = ixs[q][0], t1 = ixs[q][1], len0 = ixs[q][3];
    Acc<NC> acc;
    acc.zero();
    bool any = false;
    if (t0 < t1 && len0 > 64) { tile_a<WT, NC, false>(A.fits[f].k, t0, acc); any = true; }
    if (wm.P > 1 && t0 + wm.P < t1) {
      tiles_a<WT, NC, false>(A.fits[f].k, t0 + wm.P, t1, wm.P, acc);
      any = true;
    }
    if (any) put_pair_sums<NC>(acc, m, f, row, true);
  }
  if (wm.P > 1) return;
  // whole fits per wave: the tiles after the first of every fit are spread
  // over all workers (tile t0 + 1 + ((w - f) mod kBW) + k kBW for worker w)
  uint64_t more = fits_with_more_tiles(all_ixs, F, s_done);
  while (more) {
    const int f = __builtin_ctzll(more);
    more &= more - 1;
    const int* ix = all_ixs[f % kBW][f / kBW];
    const int start = ix[0] + 1 + rot(wave, f);
    if (start >= ix[1]) continue;
    Acc<NC> acc;
    acc.zero();
    tiles_a<WT, NC, false>(A.fits[f].k, start, ix[1], kBW, acc);
    put_pair_sums<NC>(acc, m, f, row, true);
  }
}

// Phase B over this wave's pairs of fits with a nonzero step: the first
// tiles of a chunk are re-gathered together (the lines are still in L2 from
// phase A) and updated as tile_b does, column by column (s_ed / s_em1 at
// f m + c); further tiles follow one by one.
template <typename WT, int NC>
__device__ __forceinline__ void pairs_phase_b(const BatchArgs& A, const WaveMap& wm, int wave, int m, const int* s_done,
                                              const int (*ixs)[4], const uint2 (*ixrp)[64],
                                              const int (*const* all_ixs)[4], const int* s_fstep,
                                              const double* s_ed, const double* s_em1) {
  const int lane = threadIdx.x & 63, F = A.F;
#pragma unroll 1
  for (int q0 = 0; q0 < kFitsPerWave; q0 += kChunk) {
    if (pair_fit(wm, wave, q0, F) >= F) break;
    WT wo[kChunk];
    double den[kChunk], ed[kChunk], em1[kChunk];
    bool lead[kChunk], live[kChunk], upd[kChunk];
    int seg_start[kChunk];
#pragma unroll
    for (int c = 0; c < kChunk; ++c) {
      const int f = pair_fit(wm, wave, q0 + c, F);
      const int t = ixs[q0 + c][0], t1 = ixs[q0 + c][1], len = ixs[q0 + c][3];
      const uint2 rp = ixrp[q0 + c][lane];
      live[c] = f < F && !s_done[f] && s_fstep[f] && t < t1 && len <= 64;
      wo[c] = (WT)0;
      lead[c] = false;
      upd[c] = false;
      seg_start[c] = lane;
      ed[c] = 1.0;
      em1[c] = 0.0;
      if (live[c]) {
        seg_layout(rp.y, lane, len, lead[c], seg_start[c]);
        if (lane < len) {
          const int k = f * m + (NC == 1 ? 0 : (int)col_of(rp.y));
          ed[c] = s_ed[k];
          em1[c] = s_em1[k];
          upd[c] = em1[c] != 0.0;
          if (upd[c]) wo[c] = ((const WT*)A.fits[f].k.w)[rp.x];
        }
      }
    }
#pragma unroll
    for (int c = 0; c < kChunk; ++c) {
      const int f = pair_fit(wm, wave, q0 + c, F);
      den[c] = 0.0;
      if (lead[c] && upd[c]) den[c] = A.fits[f].k.pat[pid_of(ixrp[q0 + c][lane].y)].x;
    }
#pragma unroll
    for (int c = 0; c < kChunk; ++c) {
      if (!live[c]) continue;
      const int f = pair_fit(wm, wave, q0 + c, F);
      const uint2 rp = ixrp[q0 + c][lane];
      const WT wnew = wo[c] * (WT)ed[c];
      if (upd[c]) ((WT*)A.fits[f].k.w)[rp.x] = wnew;
      // a segment lies in one column, so its lanes agree on upd
      if (sizeof(WT) == 8) {
        const double num = seg_sum_v((double)wo[c], lane, seg_start[c]);
        if (lead[c] && upd[c]) A.fits[f].k.pat[pid_of(rp.y)].x = den[c] + num * em1[c];
      } else {
        const double sdiff = seg_sum_v((double)wnew - (double)wo[c], lane, seg_start[c]);
        if (lead[c] && upd[c]) A.fits[f].k.pat[pid_of(rp.y)].x = den[c] + sdiff;
      }
    }
  }
#pragma unroll 1
  for (int q = 0; q < kFitsPerWave; ++q) {
    const int f = pair_fit(wm, wave, q, F);
    if (f >= F) break;
    if (s_done[f] || !s_fstep[f]) continue;
    const int t0 = ixs[q][0], t1 = ixs[q][1], len0 = ixs[q][3];
    const Coef cf{s_ed + f * m, s_em1 + f * m};
    if (t0 < t1 && len0 > 64) tile_b<WT>(A.fits[f].k, t0, cf);
    if (wm.P > 1) tiles_b<WT>(A.fits[f].k, t0 + wm.P, t1, wm.P, cf);
  }
  if (wm.P > 1) return;
  // the tiles after the first of every fit, spread over all waves as in phase A
  uint64_t more = fits_with_more_tiles(all_ixs, F, s_done);
  while (more) {
    const int f = __builtin_ctzll(more);
    more &= more - 1;
    if (!s_fstep[f]) continue;
    const int* ix = all_ixs[f % kBW][f / kBW];
    const int start = ix[0] + 1 + rot(wave, f);
    if (start < ix[1]) tiles_b<WT>(A.fits[f].k, start, ix[1], kBW, Coef{s_ed + f * m, s_em1 + f * m});
  }
}

template <typename WT, int NC>
__global__ void __launch_bounds__(kBlock) k_batch(BatchArgs A) {
  __shared__ double stage[32 * kBatchSlotWords];
  __shared__ double pp[kBW][kBatchSlotWords];     // per worker or slice: word 2 (f m + c) + {0, 1}
  __shared__ double part[kBatchSlotWords], tot[kBatchSlotWords];
  __shared__ double s_ed[kMaxFits], s_em1[kMaxFits];   // e^d, e^d - 1 of (fit f, column c) at f m + c
  __shared__ int s_fstep[kMaxFits];                    // fit f took a nonzero step in this group
  __shared__ int s_gcol[kMaxJ + 1];                    // column groups (shared by all fits)
  __shared__ double lp_prev[kMaxFits], s_var[kMaxFits], s_lam[kMaxFits], s_ivar[kMaxFits];
  __shared__ int s_link[kMaxFits], s_sw[kMaxFits], s_kind[kMaxFits], s_done[kMaxFits];
  __shared__ int flag, bad_any, n_active;
  // sweeps since the last exact refresh: a register of every thread (all
  // threads count the same sweeps), so that all of them take the refresh
  // and its barrier together
  int since_refresh = 0;
  __shared__ double red[kWaves][4];
  __shared__ int s_ixs[2][kBW][kFitsPerWave][4];        // indices of coordinates j and j + 1
  __shared__ uint2 s_ixrp[2][kBW][kFitsPerWave][64];

  const int tid = threadIdx.x, b = blockIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int F = A.F, G = A.G, J = A.J;
  const WaveMap wm(F);
  // one sequence per slot class (group width m: 2 F m words); the objective
  // and held-out reductions use class 0 (2 F words)
  uint32_t gseq[kMaxGroup];
#pragma unroll
  for (int c = 0; c < kMaxGroup; ++c) gseq[c] = A.ctrl->gseq[c];
  for (int i = tid; i <= A.n_groups; i += kBlock) s_gcol[i] = A.gcol[i];
  const int NG = A.n_groups;

  auto set_link = [&](int f) {  // thread-local helper: prior of fit f's current link
    const BatchFit& bf = A.fits[f];
    int kind = bf.link_kind[s_link[f]];
    double var = bf.link_var[s_link[f]];
    s_kind[f] = kind;
    s_var[f] = kind == SCCS_PRIOR_NONE ? 1.0 : var;
    s_ivar[f] = 1.0 / s_var[f];
    s_lam[f] = kind == SCCS_PRIOR_LAPLACE ? sqrt(2.0 / var) : 0.0;
  };
  if (tid < F) {
    s_link[tid] = 0;
    s_sw[tid] = 0;
    s_done[tid] = A.fits[tid].n_links <= 0;
    if (!s_done[tid]) set_link(tid);
    lp_prev[tid] = 0.0;
  }
  if (tid == 0) bad_any = 0;
  __syncthreads();

  // objective of every fit: (sum of positive, sum of negative) parts of
  // sum_i omega_i n_i log den_i over the owned patients, reduced; then
  // L_f = beta'Y'X - (pos - neg) and P_f = L_f + log p_f(beta).
  auto objectives = [&](double* Lout, double* Pout) -> bool {
    for (int f = 0; f < F; ++f) {
      const KArgs& k = A.fits[f].k;
      const int p0 = k.pb[b], p1 = k.pb[b + 1];
      double loc[4] = {0.0, 0.0, 0.0, 0.0};
      if (!s_done[f]) {
        for (int i = p0 + tid; i < p1; i += kBlock) {
          double2 pv = k.pat[i];
          if (pv.y != 0.0) {
            double t = pv.y * log(pv.x);
            if (t > 0.0) loc[0] += t; else loc[1] -= t;
          }
        }
        const double2* bt = A.fits[f].bt + (size_t)b * J;
        for (int j = tid; j < J; j += kBlock) {
          double bj = bt[j].x;
          loc[2] += bj * k.ytx[j];
          if (s_kind[f] == SCCS_PRIOR_NORMAL) loc[3] -= bj * bj * (0.5 * s_ivar[f]);
          else if (s_kind[f] == SCCS_PRIOR_LAPLACE) loc[3] -= s_lam[f] * fabs(bj);
        }
      }
      double o[4];
      block_sum<4>(loc, o, red);
      if (tid == 0) {
        part[2 * f] = o[0];
        part[2 * f + 1] = o[1];
        Lout[f] = o[2];      // beta'Y'X for now
        Pout[f] = o[3];      // log prior for now
      }
    }
    __syncthreads();
    bool okr = batch_allreduce(A.s1, A.s2, gseq[0]++, G, 2 * F, A.ctrl, part, tot, stage, &flag);
    if (tid < F) {
      double L = Lout[tid] - (tot[2 * tid] - tot[2 * tid + 1]);
      Lout[tid] = L;
      Pout[tid] = L + Pout[tid];
    }
    __syncthreads();
    return okr;
  };

  // Eq. 2 over the weight-0 patients of every fit that has just finished a
  // link: sum_j beta_j Y'X_j(held out) - sum_i n_i log den_i, the second
  // sum split into positive and negative parts and reduced like the
  // objective.  Workgroup 0 stores it in the link's result.
  __shared__ int s_adv[kMaxFits];
  __shared__ double s_ho[kMaxFits];
  auto heldout = [&]() -> bool {
    for (int f = 0; f < F; ++f) {
      const BatchFit& bf = A.fits[f];
      double loc[3] = {0.0, 0.0, 0.0};
      if (s_adv[f] && bf.ho_n) {
        const int p0 = bf.k.pb[b], p1 = bf.k.pb[b + 1];
        for (int i = p0 + tid; i < p1; i += kBlock) {
          const double hn = bf.ho_n[i];
          if (hn != 0.0) {
            double t = hn * log(bf.k.pat[i].x);
            if (t > 0.0) loc[0] += t; else loc[1] -= t;
          }
        }
        const double2* bt = bf.bt + (size_t)b * J;
        for (int j = tid; j < J; j += kBlock) loc[2] += bt[j].x * bf.ytx_ho[j];
      }
      double o[3];
      block_sum<3>(loc, o, red);
      if (tid == 0) {
        part[2 * f] = o[0];
        part[2 * f + 1] = o[1];
        s_ho[f] = o[2];
      }
    }
    __syncthreads();
    bool okr = batch_allreduce(A.s1, A.s2, gseq[0]++, G, 2 * F, A.ctrl, part, tot, stage, &flag);
    if (okr && b == 0 && tid < F && s_adv[tid] && A.fits[tid].ho_n)
      A.fits[tid].res_out[s_link[tid]].heldout = s_ho[tid] - (tot[2 * tid] - tot[2 * tid + 1]);
    __syncthreads();
    return okr;
  };

  __shared__ double Lcur[kMaxFits], Pcur[kMaxFits];
  bool ok = true;
  int status = SCCS_OK;
  if (A.criterion == SCCS_CRIT_REL_LOGPOST) {
    ok = objectives(Lcur, Pcur);
    if (tid < F) lp_prev[tid] = Pcur[tid];
    __syncthreads();
  }
  int total_sweeps = 0;
  while (ok) {
    if (tid == 0) {
      int n = 0;
      for (int f = 0; f < F; ++f) n += !s_done[f];
      n_active = n;
    }
    __syncthreads();
    if (n_active == 0) break;
    const bool worker = wave < kBW;
    if (worker) pair_index(A, wm, wave, 0, s_done, s_ixs[0][wave], s_ixrp[0][wave]);
    __syncthreads();   // every worker's staged indices, read across waves in phase A
    // poller lane f m + c: (beta_j, trust_j) and Y'X_j of fit f, column j0 + c
    // of the next group, prefetched
    double2 bt_next = make_double2(0.0, 0.0);
    double ytx_next = 0.0;
    for (int g = 0; g < NG && ok; ++g) {
      const int cur = g & 1;
      const int j0 = s_gcol[g], m = s_gcol[g + 1] - j0;
      const int(*all_ixs[kBW])[4];
#pragma unroll
      for (int w = 0; w < kBW; ++w) all_ixs[w] = s_ixs[cur][w];
      if (worker) pairs_phase_a<WT, NC>(A, wm, wave, m, s_done, s_ixs[cur][wave], s_ixrp[cur][wave], all_ixs, pp);
      __syncthreads();
      if (worker) {
        // index data of the next group (static), in the shadow of the reduction
        if (g + 1 < NG) pair_index(A, wm, wave, g + 1, s_done, s_ixs[cur ^ 1][wave], s_ixrp[cur ^ 1][wave]);
      } else {
        // the poller: each word summed over the partial rows in fixed order,
        // the device-wide reduction (slot class m - 1), then one Newton /
        // trust-region step per (fit, column) on lane f m + c; (beta_j,
        // trust_j) and Y'X_j come from the previous group's prefetch
        const int lane = tid & 63;
        const int nslots = wm.P == 1 ? kBW : wm.P;
        const int W = 2 * F * m, FM = F * m;
        double p0 = 0.0, p1 = 0.0;
        if (lane < W)
          for (int q = 0; q < nslots; ++q) p0 += pp[q][lane];
        if (lane + 64 < W)
          for (int q = 0; q < nslots; ++q) p1 += pp[q][lane + 64];
        const int cls = m - 1;
        uint32_t sq = gseq[0];
#pragma unroll
        for (int c = 1; c < kMaxGroup; ++c)
          if (cls == c) sq = gseq[c];
        const bool okr = batch_reduce_poller(A.s1 + (size_t)cls * kBatchSlots1, A.s2 + (size_t)cls * kBatchSlots2, sq,
                                             G, W, A.ctrl, &p0, &p1, tot, stage);
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        const int f = lane < FM ? fit_of(lane, m) : 0, c = lane - f * m;
        double2 v = bt_next;
        double yv = ytx_next;
        if (g == 0 && lane < FM) {
          v = A.fits[f].bt[(size_t)b * J + j0 + c];
          yv = A.fits[f].k.ytx[j0 + c];
        }
        if (g + 1 < NG) {
          // the next group's copies: nothing writes them before its step
          const int j0n = s_gcol[g + 1], mn = s_gcol[g + 2] - j0n;
          if (lane < F * mn) {
            const int fn = fit_of(lane, mn), cn = lane - fn * mn;
            bt_next = A.fits[fn].bt[(size_t)b * J + j0n + cn];
            ytx_next = A.fits[fn].k.ytx[j0n + cn];
          }
        }
        double d = 0.0;
        if (lane < FM && !s_done[f] && okr) {
          double gg = yv - tot[2 * lane], hh = -tot[2 * lane + 1];
          if (isfinite(gg) && isfinite(hh)) {
            double dv = prior_step(s_kind[f], s_ivar[f], s_lam[f], v.x, gg, hh);
            d = fmin(fmax(dv, -v.y), v.y);
            double nb = v.x + d;
            if (isfinite(nb)) {
              A.fits[f].bt[(size_t)b * J + j0 + c] = make_double2(nb, fmax(2.0 * fabs(d), 0.5 * v.y));
            } else {
              d = 0.0;
              atomicOr(&bad_any, 1);
            }
          } else {
            atomicOr(&bad_any, 1);
          }
        }
        if (lane < FM) {
          double em1 = 0.0;   // zero steps are common once fits converge
          if (d != 0.0) em1 = expm1(d);
          s_ed[lane] = 1.0 + em1;
          s_em1[lane] = em1;
        }
        const uint64_t moved = __ballot(lane < FM && d != 0.0);
        if (lane < F) s_fstep[lane] = ((moved >> (lane * m)) & ((1ull << m) - 1ull)) != 0ull;
        if (lane == 0) flag = okr ? 1 : 0;
      }
#pragma unroll
      for (int c = 0; c < kMaxGroup; ++c)
        if (m - 1 == c) ++gseq[c];
      __syncthreads();
      if (!flag) { ok = false; break; }
      if (bad_any) { status = SCCS_ERR_NUMERIC; ok = false; break; }
      if (worker)
        pairs_phase_b<WT, NC>(A, wm, wave, m, s_done, s_ixs[cur][wave], s_ixrp[cur][wave], all_ixs, s_fstep, s_ed, s_em1);
      __syncthreads();
    }
    if (!ok) break;
    ++total_sweeps;
    if (tid < F && !s_done[tid]) s_sw[tid] += 1;
    if (A.refresh_period > 0 && ++since_refresh >= A.refresh_period) {
      for (int f = 0; f < F; ++f) {
        if (s_done[f]) continue;
        const KArgs& k = A.fits[f].k;
        refresh_range<WT>(k, (const double*)(A.fits[f].bt + (size_t)b * J), k.pb[b], k.pb[b + 1], tid, kBlock, 2);
      }
      since_refresh = 0;
      __syncthreads();
    }
    // objectives every sweep: the stopping rule and the per-link results
    const bool need_obj = A.criterion == SCCS_CRIT_REL_LOGPOST;
    ok = objectives(Lcur, Pcur);
    if (!ok) break;
    // link bookkeeping, identical in every workgroup
    if (tid < F) {
      const int f = tid;
      int adv = 0;
      if (!s_done[f]) {
        int conv = 0;
        if (!isfinite(Pcur[f])) atomicOr(&bad_any, 1);
        if (need_obj) conv = fabs(Pcur[f] - lp_prev[f]) < A.tol * fabs(Pcur[f]);
        lp_prev[f] = Pcur[f];
        if (conv || s_sw[f] >= A.max_sweeps) {
          adv = 1;
          if (b == 0) {
            LinkResult r;
            r.sweeps = s_sw[f];
            r.converged = conv;
            r.loglik = Lcur[f];
            r.logpost = Pcur[f];
            A.fits[f].res_out[s_link[f]] = r;
          }
        }
      }
      s_adv[f] = adv;
    }
    __syncthreads();
    if (bad_any) { status = SCCS_ERR_NUMERIC; ok = false; break; }
    // held-out log-likelihood at the end of a link, for fits with a held-out set
    {
      bool any = false;
      for (int f = 0; f < F; ++f) any = any || (s_adv[f] && A.fits[f].ho_n);
      if (any) {
        ok = heldout();
        if (!ok) break;
      }
    }
    // record beta of finished links (workgroup 0), reset trust, move on
    for (int f = 0; f < F; ++f) {
      if (!s_adv[f]) continue;
      const BatchFit& bf = A.fits[f];
      double2* bt = bf.bt + (size_t)b * J;
      if (b == 0)
        for (int j = tid; j < J; j += kBlock) bf.beta_out[(size_t)s_link[f] * J + j] = bt[j].x;
      for (int j = tid; j < J; j += kBlock) bt[j].y = 1.0;
    }
    __syncthreads();
    if (tid < F && s_adv[tid]) {
      s_link[tid] += 1;
      s_sw[tid] = 0;
      if (s_link[tid] >= A.fits[tid].n_links) s_done[tid] = 1;
      else set_link(tid);
    }
    __syncthreads();
    // the log posterior under the new prior is the reference of the next link
    if (need_obj) {
      bool any = false;
      for (int f = 0; f < F; ++f) any = any || (s_adv[f] && !s_done[f]);
      if (any) {
        ok = objectives(Lcur, Pcur);
        if (!ok) break;
        if (tid < F && s_adv[tid] && !s_done[tid]) lp_prev[tid] = Pcur[tid];
        __syncthreads();
      }
    }
  }
  __syncthreads();
  if (b == 0 && tid == 0) {
#pragma unroll
    for (int c = 0; c < kMaxGroup; ++c) A.ctrl->gseq[c] = gseq[c];
    A.ctrl->sweeps = total_sweeps;
    if (status != SCCS_OK) A.ctrl->status = status;
  }
}

}  // namespace sccs
