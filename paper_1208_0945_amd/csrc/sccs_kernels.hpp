// HIP kernels of libsccs for gfx950: the per-coordinate CCD step of the
// Bayesian SCCS model (Algorithm 1; Section 2.4 Steps 1-4; Eqs. 4, 7-9).
//
// One cooperative, persistent launch runs whole sweeps.  Workgroup b owns a
// fixed patient range, and with it every era of those patients, for all
// columns.  Per coordinate j:
//
//   phase A  (Step 4 and the fused transform/reduction of Listing 2's role):
//            for the tiles of column j in its range, gather w_k on the
//            column's rows, sum them per patient segment with a wave64
//            shuffle-based segmented reduction (num_ij), then accumulate
//            G = sum omega_i n_i r_i and H = sum omega_i n_i r_i (1 - r_i)
//            with r_i = num_ij / den_i over the column's patients only.
//   reduce   the two per-workgroup partials are exchanged through tagged
//            slots (below) and summed in a fixed order, identically in
//            every workgroup; g_j = Y'X_j - G, h_j = -H (Eqs. 7, 9).
//   step     every workgroup takes the same prior-regularised Newton step
//            with the trust-region bound (Eq. 4) on its LDS copy of beta.
//   phase B  (Steps 1-3, Listing 3's role) if the step d is nonzero:
//            w_k <- w_k e^d on the column's rows and
//            den_i <- den_i + num_ij (e^d - 1); a patient's den has a single
//            writer (its owner), so no atomics are needed.
//
// Because a workgroup only touches state it owns, phase B of coordinate j
// and phase A of coordinate j+1 are ordered by a workgroup barrier alone;
// the only device-wide traffic per coordinate is the exchange of two
// doubles per workgroup.  Independent coordinates share that exchange:
// column groups (consecutive columns with no patient in common), and passes
// of several consecutive groups when the columns linking them take zero
// steps (below).
//
// Tagged-slot reduction.  Both partials are sums of non-negative terms (the
// per-patient factor 1 - r_i is clamped at zero, which only matters when
// rounding makes r_i exceed one), so their sign bit is free.  Reduction
// number s writes slot (s & 1) with the sign bit set to ((s >> 1) & 1).  A
// slot read for reduction s still holds reduction s-2's value until it is
// overwritten, and that value carries the opposite tag, so readers spin on
// the tag alone: no reset, no counter, no device-scope fence.  A workgroup
// cannot write reduction s+2 before every workgroup has written s+1, which
// each does only after reading s, so a slot is never overwritten while it
// can still be read.  The objective uses a second slot set the same way.
#pragma once
#include <hip/hip_runtime.h>

#include "sccs.h"
#include "sccs_device.hpp"

namespace sccs {

// ------------------------------------------------------------ wave helpers

// Sum over the 64 lanes, returned to every lane.  Data-parallel-primitive
// (DPP) lane moves on the two 32-bit halves, so no LDS traffic and no wait
// on the LDS/scalar-memory counter: pairs, quads (quad_perm), half rows and
// rows (mirrors), then rows 0+1 and 2+3 (row_bcast:15 into rows 1 and 3)
// and all four (row_bcast:31 into rows 2 and 3); lane 63 holds the total,
// read back as a scalar.  The order of the additions is fixed.
template <int Ctrl, int RowMask>
__device__ __forceinline__ double dpp_add(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, Ctrl, RowMask, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), Ctrl, RowMask, 0xf, false);
  return v + __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double wave_sum(double v) {
  v = dpp_add<0xB1, 0xf>(v);   // quad_perm [1,0,3,2]
  v = dpp_add<0x4E, 0xf>(v);   // quad_perm [2,3,0,1]
  v = dpp_add<0x141, 0xf>(v);  // row_half_mirror
  v = dpp_add<0x140, 0xf>(v);  // row_mirror
  v = dpp_add<0x142, 0xa>(v);  // row_bcast:15 -> rows 1, 3
  v = dpp_add<0x143, 0xc>(v);  // row_bcast:31 -> rows 2, 3
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, 63);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Sum over lanes 0 .. L-1 (L = 8, 16 or 32; the other lanes hold +0),
// returned to every lane: the first three, four or five stages of wave_sum,
// read from the last lane they fill.  The stages left out would
// only add +0, so the value is wave_sum's, bit for bit.
template <int L>
__device__ __forceinline__ double wave_sum_lo(double v) {
  static_assert(L == 8 || L == 16 || L == 32, "eight, sixteen or thirty-two lanes");
  v = dpp_add<0xB1, 0xf>(v);   // quad_perm [1,0,3,2]
  v = dpp_add<0x4E, 0xf>(v);   // quad_perm [2,3,0,1]
  v = dpp_add<0x141, 0xf>(v);  // row_half_mirror
  if (L >= 16) v = dpp_add<0x140, 0xf>(v);  // row_mirror
  if (L == 32) v = dpp_add<0x142, 0xa>(v);  // row_bcast:15 -> rows 1, 3
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, L - 1);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), L - 1);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Lane l's value (l a compile-time constant), as a scalar.
__device__ __forceinline__ double readlane_d(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ uint64_t tag_encode(double v, uint32_t tag) {
  uint64_t b = (uint64_t)__double_as_longlong(v);
  return (b & ~kSign) | ((uint64_t)tag << 63);
}
__device__ __forceinline__ double tag_decode(uint64_t b) {
  return __longlong_as_double((long long)(b & ~kSign));
}

__device__ __forceinline__ void store_agent(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t load_agent(const uint64_t* p) {
  return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int load_agent_i(const int32_t* p) {
  return __hip_atomic_load(const_cast<int32_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Poll NV tagged words at src (active lanes) until all carry `tag`; the
// decoded values land in v (zeros in inactive lanes).  Returns false in the
// whole wave on timeout or if another workgroup aborted.
template <int NV>
__device__ __forceinline__ bool poll_tagged(const uint64_t* src, bool active, uint32_t tag, double* v, Ctrl* ctrl) {
  bool need = active;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = 0.0;
  long long spins = 0;
  while (true) {
    if (need) {
      bool ready = true;
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        uint64_t x = load_agent(src + i);
        ready = ready && ((uint32_t)(x >> 63) == tag);
        v[i] = tag_decode(x);
      }
      if (ready) need = false;
    }
    if (__ballot(need) == 0ull) return true;
    if (++spins > kSpinLimit) {
      if ((threadIdx.x & 63) == 0) {
        __hip_atomic_store(&ctrl->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&ctrl->status, (int)SCCS_ERR_SYNC, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      return false;
    }
    if ((spins & 255) == 0 && load_agent_i(&ctrl->abort)) return false;
    if (kPollSleep) __builtin_amdgcn_s_sleep(kPollSleep);
  }
}

// Device-wide sum of NV non-negative doubles per workgroup (member b of G;
// several fits can share a launch, each on a range of workgroups), in two levels:
// the workgroups form ng = min(8, G) groups (b mod ng, which follows the
// round-robin placement of workgroups on the eight XCDs); the leader of a
// group (workgroup g < ng) sums its members' tagged slots in member order and
// publishes the tagged group total; every workgroup then sums the ng group
// totals in group order, so every workgroup computes the same value bit for
// bit.  Each level-1 slot has a 128-byte line of its own, and the group
// totals are written in kReplicas copies (reader b polls copy b mod
// kReplicas): polling 256 workgroups on one line serialises at the memory
// side.  Must be called by all lanes of ONE wave of every workgroup, with the
// workgroup's partials in part[] of that wave's lane 0.  Returns the sums in
// out[] in all lanes of that wave.  Every reduction on one slot array must
// use the same NV: the tag a reader waits for is told apart only from the
// tag that reduction s-2 left in the same word.  (NV is a compile-time
// constant so that all polling loads of a round are issued before any is
// waited on.)
//
// Both sums are balanced pairwise trees in member (group) order, so the
// value does not depend on NV or on which of the two forms below runs: one
// lane per member, polling its NV words (allreduce2_lanes, for more than 8
// words), or one lane per (member, word) pair (allreduce2_rows, up to 8
// words), which needs fewer load instructions per polling round.
template <int NV>
__device__ bool allreduce2_lanes(uint64_t* s1, uint64_t* s2, uint32_t seq, int G, Ctrl* ctrl,
                                 const double* part, double* out, int b) {
  const int lane = threadIdx.x & 63;
  const uint32_t par = seq & 1u, tag = (seq >> 1) & 1u;
  const int ng = G < kGroups ? G : kGroups;
  uint64_t* L1 = s1 + (size_t)par * (kSlots1Words / 2);
  uint64_t* L2 = s2 + (size_t)par * kReplicas * kGroups * kSlotWords;
  if (lane == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) store_agent(L1 + (size_t)b * kSlotWords + v, tag_encode(part[v], tag));
  }
  double v[NV];
  if (b < ng) {
    const int member = b + lane * ng;
    if (!poll_tagged<NV>(L1 + (size_t)(member < G ? member : b) * kSlotWords, member < G, tag, v, ctrl)) return false;
    // members sit in lanes 0..31 (G <= 32 ng), lanes 0..15 when G <= 16 ng
    if (G <= 16 * ng) {
#pragma unroll
      for (int i = 0; i < NV; ++i) v[i] = wave_sum_lo<16>(v[i]);
    } else {
#pragma unroll
      for (int i = 0; i < NV; ++i) v[i] = wave_sum_lo<32>(v[i]);
    }
    if (lane < kReplicas) {
#pragma unroll
      for (int i = 0; i < NV; ++i)
        store_agent(L2 + ((size_t)lane * kGroups + b) * kSlotWords + i, tag_encode(v[i], tag));
    }
  }
  const int r = b % kReplicas;
  if (!poll_tagged<NV>(L2 + ((size_t)r * kGroups + (lane < ng ? lane : 0)) * kSlotWords, lane < ng, tag, v, ctrl))
    return false;
  // group totals sit in lanes 0..ng-1, ng <= 8
#pragma unroll
  for (int i = 0; i < NV; ++i) out[i] = wave_sum_lo<8>(v[i]);
  return true;
}

// Poll P tagged words per lane (word p at src[p], if act[p]) until all carry
// `tag`; decoded values in v (zeros where inactive).  Timeout and abort as
// for poll_tagged.
template <int P>
__device__ __forceinline__ bool poll_words(const uint64_t* const* src, const bool* act, uint32_t tag, double* v,
                                           Ctrl* ctrl) {
  bool need = false;
#pragma unroll
  for (int p = 0; p < P; ++p) {
    v[p] = 0.0;
    need = need || act[p];
  }
  long long spins = 0;
  while (true) {
    if (need) {
      bool ready = true;
#pragma unroll
      for (int p = 0; p < P; ++p) {
        if (act[p]) {
          const uint64_t x = load_agent(src[p]);
          ready = ready && ((uint32_t)(x >> 63) == tag);
          v[p] = tag_decode(x);
        }
      }
      if (ready) need = false;
    }
    if (__ballot(need) == 0ull) return true;
    if (++spins > kSpinLimit) {
      if ((threadIdx.x & 63) == 0) {
        __hip_atomic_store(&ctrl->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&ctrl->status, (int)SCCS_ERR_SYNC, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      return false;
    }
    if ((spins & 255) == 0 && load_agent_i(&ctrl->abort)) return false;
    if (kPollSleep) __builtin_amdgcn_s_sleep(kPollSleep);
  }
}

// Sum of the 16 lanes of each row (all lanes of a row end with the row's
// sum, a balanced tree in lane order).
__device__ __forceinline__ double row_sum16(double v) {
  v = dpp_add<0xB1, 0xf>(v);   // quad_perm [1,0,3,2]
  v = dpp_add<0x4E, 0xf>(v);   // quad_perm [2,3,0,1]
  v = dpp_add<0x141, 0xf>(v);  // row_half_mirror
  return dpp_add<0x140, 0xf>(v);  // row_mirror
}
// Sum of lanes 0..7 of each row in those lanes (balanced tree).
__device__ __forceinline__ double row_sum8(double v) {
  v = dpp_add<0xB1, 0xf>(v);
  v = dpp_add<0x4E, 0xf>(v);
  return dpp_add<0x141, 0xf>(v);
}

// One 16-lane row per word: lane (row r, column c) of word pass q handles
// word 4q + r of member 16p + c (level 1, member pass p) or of group c
// (level 2), so one load per (word pass, member pass) polls a whole round
// and the sums are row-wise DPP trees.
template <int NV>
__device__ bool allreduce2_rows(uint64_t* s1, uint64_t* s2, uint32_t seq, int G, Ctrl* ctrl,
                                const double* part, double* out, int b) {
  static_assert(NV >= 1 && NV <= 8, "one to eight words");
  static_assert(kReplicas <= 16 && kGroups <= 8, "copies and groups along a row");
  constexpr int NQ = (NV + 3) / 4;            // word passes (four rows each)
  constexpr int NL = 2 * NQ;                  // loads of a level-1 polling round (two member passes)
  const int lane = threadIdx.x & 63;
  const int row = lane >> 4, col = lane & 15;
  const uint32_t par = seq & 1u, tag = (seq >> 1) & 1u;
  const int ng = G < kGroups ? G : kGroups;
  uint64_t* L1 = s1 + (size_t)par * (kSlots1Words / 2);
  uint64_t* L2 = s2 + (size_t)par * kReplicas * kGroups * kSlotWords;
  {   // lane v stores word v of this workgroup's slot
    double mine = 0.0;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double pv = readlane_d(part[v], 0);
      if (lane == v) mine = pv;
    }
    if (lane < NV) store_agent(L1 + (size_t)b * kSlotWords + lane, tag_encode(mine, tag));
  }
  if (b < ng) {
    const int nm = (G - b + ng - 1) / ng;   // members of group b: b, b + ng, ... (at most 32)
    const uint64_t* src[NL];
    bool act[NL];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
      for (int p = 0; p < 2; ++p) {
        const int w = 4 * q + row, k = 16 * p + col;
        act[2 * q + p] = w < NV && k < nm;
        src[2 * q + p] = L1 + (size_t)(act[2 * q + p] ? b + k * ng : b) * kSlotWords + (w < NV ? w : 0);
      }
    double v[NL];
    if (!poll_words<NL>(src, act, tag, v, ctrl)) return false;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      // members 0..15 and 16..31 of word 4q + row (a pass with no member adds +0)
      const double sm = row_sum16(v[2 * q]) + row_sum16(v[2 * q + 1]);
      const int w = 4 * q + row;
      if (w < NV && col < kReplicas)   // copy col of the group total
        store_agent(L2 + ((size_t)col * kGroups + b) * kSlotWords + w, tag_encode(sm, tag));
    }
  }
  const int rr = b % kReplicas;
  const uint64_t* src2[NQ];
  bool act2[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const int w = 4 * q + row;
    act2[q] = w < NV && col < ng;
    src2[q] = L2 + ((size_t)rr * kGroups + (act2[q] ? col : 0)) * kSlotWords + (w < NV ? w : 0);
  }
  double v2[NQ];
  if (!poll_words<NQ>(src2, act2, tag, v2, ctrl)) return false;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const double t = row_sum8(v2[q]);
#pragma unroll
    for (int r = 0; r < 4; ++r)
      if (4 * q + r < NV) out[4 * q + r] = readlane_d(t, 16 * r + 7);
  }
  return true;
}

template <int NV>
__device__ __forceinline__ bool allreduce2_wave(uint64_t* s1, uint64_t* s2, uint32_t seq, int G, Ctrl* ctrl,
                                                const double* part, double* out, int b) {
  if constexpr (NV <= 8) return allreduce2_rows<NV>(s1, s2, seq, G, ctrl, part, out, b);
  else return allreduce2_lanes<NV>(s1, s2, seq, G, ctrl, part, out, b);
}

// Workgroup-level wrapper: wave 0 reduces, the result is broadcast through
// LDS.  Called by all threads with the partials valid in thread 0.
template <int NV>
__device__ bool allreduce_nonneg(uint64_t* s1, uint64_t* s2, uint32_t seq, int G, Ctrl* ctrl,
                                 const double* part, double* out, double* lds_out, int* lds_ok, int b) {
  if (threadIdx.x < 64) {
    double o[NV];
    bool ok = allreduce2_wave<NV>(s1, s2, seq, G, ctrl, part, o, b);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int v = 0; v < NV; ++v) lds_out[v] = o[v];
      *lds_ok = ok ? 1 : 0;
    }
  }
  __syncthreads();
  bool ok = *lds_ok != 0;
#pragma unroll
  for (int v = 0; v < NV; ++v) out[v] = lds_out[v];
  __syncthreads();
  return ok;
}

// Fixed-order workgroup sum: wave butterflies, then wave 0's partials summed
// in wave order by thread 0 (result valid in thread 0 only).
template <int NV, int W>
__device__ void block_sum(const double* v_in, double* out, double (*red)[W]) {
  static_assert(NV <= W, "reduction rows too narrow");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double v[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v_in[i]);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) red[wave][i] = v[i];
  }
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double s = 0.0;
      for (int q = 0; q < kWaves; ++q) s += red[q][i];
      out[i] = s;
    }
  }
  __syncthreads();
}

// Workgroup sum delivered to wave `dst`: wave sums, then the wave partials
// combined inside wave dst, eight words per round: lane 8k + q reads wave
// q's word r + k, and three butterfly stages within each group of eight
// lanes add ((w0 + w1) + (w2 + w3)) + ((w4 + w5) + (w6 + w7)).  The order
// does not depend on NV, so a column's sum is the same whether its
// reduction carries one column or several.  Result valid in all lanes of
// wave dst (scalars); one barrier.  red[] may be reused after the caller's
// next barrier.
template <int NV, int W>
__device__ __forceinline__ void block_sum_to(const double* v_in, double* out, double (*red)[W], int dst) {
  static_assert(NV <= W, "reduction rows too narrow");
  static_assert(kWaves == 8, "one butterfly over eight lanes per word");
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double v[NV];
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v_in[i]);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) red[wave][i] = v[i];
  }
  __syncthreads();
  if (wave == dst) {
#pragma unroll
    for (int r = 0; r < NV; r += 8) {
      const int i = r + (lane >> 3);
      double x = i < NV ? red[lane & 7][i] : 0.0;
      x = dpp_add<0xB1, 0xf>(x);   // quad_perm [1,0,3,2]
      x = dpp_add<0x4E, 0xf>(x);   // quad_perm [2,3,0,1]
      x = dpp_add<0x141, 0xf>(x);  // row_half_mirror
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (r + k < NV) out[r + k] = readlane_d(x, 8 * k);
    }
  }
}

// ------------------------------------------------------------ Newton step

// Eq. 4 with the prior; Laplace rules at the kink after Genkin et al.
__device__ double prior_step(int kind, double inv_var, double lambda, double b, double g, double h) {
  if (kind == SCCS_PRIOR_NORMAL) return -(g - b * inv_var) / (h - inv_var);
  double lam = (kind == SCCS_PRIOR_LAPLACE) ? lambda : 0.0;
  if (!(h < 0.0)) return 0.0;
  if (b > 0.0) {
    double d = -(g - lam) / h;
    return (b + d < 0.0) ? -b : d;
  }
  if (b < 0.0) {
    double d = -(g + lam) / h;
    return (b + d > 0.0) ? -b : d;
  }
  if (g > lam) return -(g - lam) / h;
  if (g < -lam) return -(g + lam) / h;
  return 0.0;
}

// Steps of a column group's m columns under the grouped Normal prior
// (called by the whole poller wave; gg, hh and the results are those of
// lane c for column j0 + c).  Columns of one class are coupled through the
// class sum, so the lanes take their steps one after another, in column
// order, each seeing the class sums the steps before it left (the order of
// Algorithm 1).
__device__ __forceinline__ void grouped_steps(const KArgs& a, int j0, int m, bool okr, double gg, double hh,
                                              double* sbeta, double* strust, double* ssum, double& d, int& bad) {
  const int lane = threadIdx.x & 63;
  for (int c = 0; c < m; ++c) {
    if (lane == c) {
      bad = !(isfinite(gg) && isfinite(hh));
      if (okr && !bad) {
        const int j = j0 + c, k = a.pclass[j];
        const double bj = sbeta[j], tr = strust[j], kap = a.pkappa[k];
        const double dv = -(gg - (bj - kap * ssum[k]) / a.var) / (hh - (1.0 - kap) / a.var);
        d = fmin(fmax(dv, -tr), tr);
        strust[j] = fmax(2.0 * fabs(d), 0.5 * tr);
        const double nb = bj + d;
        if (!isfinite(nb)) {
          bad = 1;
          d = 0.0;
        } else {
          sbeta[j] = nb;
          ssum[k] += d;
        }
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
}

// Class sums of the grouped prior from beta, in column order (thread 0;
// every workgroup forms the same bits).  Caller synchronises.
__device__ __forceinline__ void class_sums(const KArgs& a, const double* sbeta, double* ssum) {
  if (threadIdx.x == 0) {
    for (int c = 0; c < a.n_classes; ++c) ssum[c] = 0.0;
    for (int j = 0; j < a.J; ++j) ssum[a.pclass[j]] += sbeta[j];
  }
}

// ------------------------------------------------------------ precision traits

template <typename WT>
struct Prec;

template <>
struct Prec<double> {
  // w = l exp(eta)
  __device__ static double weight(int32_t l, double eta) { return (double)l * exp(eta); }
};

template <>
struct Prec<float> {
  // exp in FP32 after an FP64 range reduction eta = n ln2 + r, |r| <= ln2/2
  // (Cody and Waite's two-constant reduction, with ln2 split into a high
  // part whose low bits are zero, so that n times it is exact, and the
  // remainder -- the split fdlibm uses for its exp)
  __device__ static float weight(int32_t l, double eta) {
    double n = rint(eta * 1.4426950408889634);
    double r = fma(-n, 6.93147180369123816490e-01, eta);
    r = fma(-n, 1.90821492927058770002e-10, r);
    float e = expf((float)r);
    return ldexpf((float)l * e, (int)n);
  }
};

// ------------------------------------------------------------ segmented sums

// Segment layout of a tile.  The active lanes [0, len) hold (column,
// patient) keys in segments of equal keys; the lead lane of a segment is its
// last lane, seg_start the first lane of this lane's segment.  Neighbour keys
// come from DPP wave shifts by one lane (no LDS).
__device__ __forceinline__ void seg_layout(uint32_t key, int lane, int len, bool& lead, int& seg_start) {
  const uint32_t key_next = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)key, 0x130, 0xf, 0xf, false);  // wave_shl:1
  const uint32_t key_prev = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)key, 0x138, 0xf, 0xf, false);  // wave_shr:1
  const bool act = lane < len;
  lead = act && (lane == len - 1 || key_next != key);
  const bool first = act && (lane == 0 || key_prev != key);
  const uint64_t firsts = __ballot(first);
  const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1);
  seg_start = act ? 63 - (int)__builtin_clzll(firsts & upto) : lane;
}

// Inclusive prefix sum of v within this lane's segment, so that the lead
// lane holds the segment sum: a fixed-order scan with DPP row shifts by 1, 2,
// 4 and 8 inside each 16-lane row, then the carries of row_bcast:15 (into
// rows 1 and 3) and row_bcast:31 (into rows 2 and 3), each term added only
// when its source lane lies in the same segment.
template <int Ctrl, int RowMask>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, Ctrl, RowMask, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), Ctrl, RowMask, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

__device__ __forceinline__ double seg_sum_v(double v, int lane, int seg_start) {
  const int r = lane & 15;
  double o;
  o = dpp_move<0x111, 0xf>(v);  // row_shr:1
  if (r >= 1 && lane - 1 >= seg_start) v += o;
  o = dpp_move<0x112, 0xf>(v);  // row_shr:2
  if (r >= 2 && lane - 2 >= seg_start) v += o;
  o = dpp_move<0x114, 0xf>(v);  // row_shr:4
  if (r >= 4 && lane - 4 >= seg_start) v += o;
  o = dpp_move<0x118, 0xf>(v);  // row_shr:8
  if (r >= 8 && lane - 8 >= seg_start) v += o;
  o = dpp_move<0x142, 0xa>(v);  // row_bcast:15: lane 15 -> row 1, lane 47 -> row 3
  if ((lane & 16) && seg_start <= (lane & ~15) - 1) v += o;
  o = dpp_move<0x143, 0xc>(v);  // row_bcast:31: lane 31 -> rows 2 and 3
  if (lane >= 32 && seg_start <= 31) v += o;
  return v;
}

__device__ __forceinline__ double seg_sum(double v, uint32_t key, int lane, int len, bool& lead) {
  int seg_start;
  seg_layout(key, lane, len, lead, seg_start);
  return seg_sum_v(v, lane, seg_start);
}

// Contribution of one patient segment to G and H (the transform of Eq. 8
// fused with the two inner products of Eqs. 7 and 9).
__device__ __forceinline__ void accum_patient(double num, double2 pv, double& Gl, double& Hl) {
  // num = 0 gives r = 0, also for a patient whose eras all have length 0
  // (den_i = 0; such a patient has n_i = 0 and no term in Eq. 2)
  double r = num != 0.0 ? num / pv.x : 0.0;
  double tg = pv.y * r;
  Gl += tg;
  Hl += tg * fmax(1.0 - r, 0.0);
}

// Index load through the vector memory path.  A wave-uniform address would
// otherwise become a scalar load, and scalar loads share their completion
// counter with LDS operations: every later LDS access of the wave would
// wait for it.  A relaxed workgroup-scope atomic load is an ordinary cached
// vector load.
__device__ __forceinline__ int ld_idx(const int32_t* p) {
  return __hip_atomic_load(const_cast<int32_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ uint32_t ld_idx(const uint32_t* p) {
  return __hip_atomic_load(const_cast<uint32_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Column of a group (bits above the patient index of rp.y) and the patient.
__device__ __forceinline__ uint32_t col_of(uint32_t key) { return key >> kGroupShift; }
__device__ __forceinline__ uint32_t pid_of(uint32_t key) { return key & kPidMask; }

// Per-lane accumulators of G and H for the NC columns of a group; a lead
// lane adds its segment's terms to its own column's pair.
template <int NC>
struct Acc {
  double g[NC], h[NC];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int i = 0; i < NC; ++i) g[i] = h[i] = 0.0;
  }
  __device__ __forceinline__ void add(uint32_t c, double num, double2 pv) {
    const double r = num != 0.0 ? num / pv.x : 0.0;   // as in accum_patient
    const double tg = pv.y * r;
    const double th = tg * fmax(1.0 - r, 0.0);
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      const bool mine = NC == 1 || c == (uint32_t)i;
      g[i] += mine ? tg : 0.0;
      h[i] += mine ? th : 0.0;
    }
  }
};

// Per-column update factors e^d and e^d - 1 (LDS arrays indexed by column).
struct Coef {
  const double* ed;
  const double* em1;
};

// ---- one tile, loads included

// Phase A on tile t: gather w on the tile's rows, sum per (column, patient)
// segment, accumulate the segment's terms of G and H; optionally mark the
// tile's patients in the workgroup's bitmap.
template <typename WT, int NC, bool kMark>
__device__ __forceinline__ void tile_a(const KArgs& a, int t, Acc<NC>& acc, unsigned* bits = nullptr, int p0 = 0,
                                       uint32_t coff = 0) {
  const int lane = threadIdx.x & 63;
  const WT* __restrict__ w = (const WT*)a.w;
  const int e0 = ld_idx(a.tile_start + t), e1 = ld_idx(a.tile_start + t + 1);
  const int len = e1 - e0;
  if (len <= 64) {
    bool act = lane < len;
    uint2 rp = act ? a.rp[e0 + lane] : make_uint2(0u, 0xffffffffu);
    double wv = act ? (double)w[rp.x] : 0.0;
    bool lead;
    double num = seg_sum(wv, rp.y, lane, len, lead);
    if (lead) {
      acc.add(col_of(rp.y) + coff, num, a.pat[pid_of(rp.y)]);
      if (kMark) atomicOr(&bits[(pid_of(rp.y) - p0) >> 5], 1u << ((pid_of(rp.y) - p0) & 31));
    }
  } else {
    // one (column, patient) segment with more than 64 nonzeros
    double s = 0.0;
    for (int e = e0 + lane; e < e1; e += 64) s += (double)w[a.rp[e].x];
    s = wave_sum(s);
    if (lane == 0) {
      const uint32_t key = a.rp[e0].y;
      acc.add(col_of(key) + coff, s, a.pat[pid_of(key)]);
      if (kMark) atomicOr(&bits[(pid_of(key) - p0) >> 5], 1u << ((pid_of(key) - p0) & 31));
    }
  }
}

// Phase B on tile t: w_k <- w_k e^d on the tile's rows; den_i of each
// segment moves by num_i (e^d - 1) (FP64), or by the exact change of the
// stored FP32 weights summed in FP64 (mixed).  Columns with a zero step
// are left untouched (their update is the identity).
template <typename WT>
__device__ __forceinline__ void tile_b(const KArgs& a, int t, Coef cf) {
  const int lane = threadIdx.x & 63;
  WT* __restrict__ w = (WT*)a.w;
  const int e0 = ld_idx(a.tile_start + t), e1 = ld_idx(a.tile_start + t + 1);
  const int len = e1 - e0;
  if (len <= 64) {
    bool act = lane < len;
    uint2 rp = act ? a.rp[e0 + lane] : make_uint2(0u, 0xffffffffu);
    const uint32_t c = act ? col_of(rp.y) : 0u;
    const double ed = cf.ed[c], em1 = cf.em1[c];
    const bool upd = act && em1 != 0.0;
    WT wo = upd ? w[rp.x] : (WT)0;
    WT wn = wo * (WT)ed;
    if (upd) w[rp.x] = wn;
    bool lead;
    if (sizeof(WT) == 8) {
      double s = seg_sum((double)wo, rp.y, lane, len, lead);
      if (lead && upd) a.pat[pid_of(rp.y)].x += s * em1;
    } else {
      double s = seg_sum((double)wn - (double)wo, rp.y, lane, len, lead);
      if (lead && upd) a.pat[pid_of(rp.y)].x += s;
    }
  } else {
    const uint32_t key = a.rp[e0].y;
    const double ed = cf.ed[col_of(key)], em1 = cf.em1[col_of(key)];
    if (em1 == 0.0) return;
    const WT edw = (WT)ed;
    double s = 0.0;
    for (int e = e0 + lane; e < e1; e += 64) {
      uint32_t row = a.rp[e].x;
      WT wo = w[row];
      WT wn = wo * edw;
      w[row] = wn;
      s += (sizeof(WT) == 8) ? (double)wo : ((double)wn - (double)wo);
    }
    s = wave_sum(s);
    if (lane == 0) a.pat[pid_of(key)].x += (sizeof(WT) == 8) ? s * em1 : s;
  }
}

// Mark patient q (relative to the range start) in an LDS bitmap.
__device__ __forceinline__ void mark_patient(unsigned* bits, unsigned q) { atomicOr(&bits[q >> 5], 1u << (q & 31)); }

// ---- tiles t, t + stride, ... < t1 of one range, in order
//
// Software-pipelined: while a tile's gathers are in flight, the wave loads
// the (row, key) pairs of its next tile and the bounds of the tile after
// that, and the per-patient words are gathered together with w (the lead
// lanes follow from the keys alone).  A tile then waits on one round trip to
// memory instead of a chain of four (bounds, pairs, w, then the patient
// words).  The arithmetic, and its order, are those of tile_a and tile_b.

// Bounds of tile t (e0, len), or an empty tile past the range.
__device__ __forceinline__ void tile_bounds(const KArgs& a, int t, int t1, int& e0, int& len) {
  e0 = 0;
  len = 0;
  if (t < t1) {
    e0 = ld_idx(a.tile_start + t);
    len = ld_idx(a.tile_start + t + 1) - e0;
  }
}
// This lane's pair of a short tile (inactive lanes: no patient).
__device__ __forceinline__ uint2 tile_pair(const KArgs& a, int e0, int len) {
  const int lane = threadIdx.x & 63;
  return len <= 64 && lane < len ? a.rp[e0 + lane] : make_uint2(0u, 0xffffffffu);
}

template <typename WT, int NC, bool kMark>
__device__ __forceinline__ void tiles_a(const KArgs& a, int t, int t1, int stride, Acc<NC>& acc,
                                        unsigned* bits = nullptr, int p0 = 0, uint32_t coff = 0) {
  if (t >= t1) return;
  const int lane = threadIdx.x & 63;
  const WT* __restrict__ w = (const WT*)a.w;
  int e0, len, en, lenn;
  tile_bounds(a, t, t1, e0, len);
  tile_bounds(a, t + stride, t1, en, lenn);
  uint2 rp = tile_pair(a, e0, len);
  while (true) {
    uint2 rpn;
    int enn, lennn;
    if (len <= 64) {
      bool lead;
      int seg_start;
      seg_layout(rp.y, lane, len, lead, seg_start);
      const double wv = lane < len ? (double)w[rp.x] : 0.0;
      const double2 pv = lead ? a.pat[pid_of(rp.y)] : make_double2(1.0, 0.0);
      rpn = tile_pair(a, en, lenn);
      tile_bounds(a, t + 2 * stride, t1, enn, lennn);
      const double num = seg_sum_v(wv, lane, seg_start);
      if (lead) {
        acc.add(col_of(rp.y) + coff, num, pv);
        if (kMark) mark_patient(bits, pid_of(rp.y) - (unsigned)p0);
      }
    } else {
      rpn = tile_pair(a, en, lenn);
      tile_bounds(a, t + 2 * stride, t1, enn, lennn);
      tile_a<WT, NC, kMark>(a, t, acc, bits, p0, coff);
    }
    t += stride;
    if (t >= t1) break;
    rp = rpn;
    len = lenn;
    en = enn;
    lenn = lennn;
  }
}

template <typename WT>
__device__ __forceinline__ void tiles_b(const KArgs& a, int t, int t1, int stride, Coef cf) {
  if (t >= t1) return;
  const int lane = threadIdx.x & 63;
  WT* __restrict__ w = (WT*)a.w;
  int e0, len, en, lenn;
  tile_bounds(a, t, t1, e0, len);
  tile_bounds(a, t + stride, t1, en, lenn);
  uint2 rp = tile_pair(a, e0, len);
  while (true) {
    uint2 rpn;
    int enn, lennn;
    if (len <= 64) {
      const bool act = lane < len;
      const uint32_t c = act ? col_of(rp.y) : 0u;
      const double ed = cf.ed[c], em1 = cf.em1[c];
      const bool upd = act && em1 != 0.0;
      bool lead;
      int seg_start;
      seg_layout(rp.y, lane, len, lead, seg_start);
      const WT wo = upd ? w[rp.x] : (WT)0;
      const double den = lead && upd ? a.pat[pid_of(rp.y)].x : 0.0;
      rpn = tile_pair(a, en, lenn);
      tile_bounds(a, t + 2 * stride, t1, enn, lennn);
      const WT wn = wo * (WT)ed;
      if (upd) w[rp.x] = wn;
      if (sizeof(WT) == 8) {
        const double s = seg_sum_v((double)wo, lane, seg_start);
        if (lead && upd) a.pat[pid_of(rp.y)].x = den + s * em1;
      } else {
        const double s = seg_sum_v(upd ? (double)wn - (double)wo : 0.0, lane, seg_start);
        if (lead && upd) a.pat[pid_of(rp.y)].x = den + s;
      }
    } else {
      rpn = tile_pair(a, en, lenn);
      tile_bounds(a, t + 2 * stride, t1, enn, lennn);
      tile_b<WT>(a, t, cf);
    }
    t += stride;
    if (t >= t1) break;
    rp = rpn;
    len = lenn;
    en = enn;
    lenn = lennn;
  }
}

// ---- the sweep's path
//
// Coordinates are visited group by group (column groups: consecutive,
// pairwise patient-disjoint columns, whose Newton steps are independent;
// one device-wide reduction per group carries all of the group's partial
// sums).  Waves 0..kWorkers-1 ("workers") take tiles t0 + w, t0 + w +
// kWorkers, ... of the current group; the last wave runs the device-wide
// reduction.  Each worker keeps its first tile of a group in registers: the
// index data is prefetched two groups ahead, and the gathers of w and
// (den_i, omega_i n_i) are issued one group ahead, while the previous
// group's reduction is in flight.  Such a speculative gather is stale only
// where the previous group changed the state, i.e. for patients in both;
// every workgroup marks the patients of each group in an LDS bitmap over its
// own patient range, and a speculative tile that holds a marked patient is
// gathered again after the update.  The values used are therefore exactly
// those of the sequential algorithm.  The merged-pass form does the same per
// pass (one group or several): the first tiles of every group of the next
// pass are gathered ahead, and the bitmap marks the patients of the whole
// pass.

constexpr int kWorkers = kWaves - 1;

struct Pf {
  int t, t1;     // the wave's first tile; end of the workgroup's tile range
  int len;       // that tile's number of nonzeros
  uint2 rp;      // this lane's (row, patient | column)
};

struct Cache {
  double wv;     // gathered weight
  double num;    // segment sum (lead lanes)
  double den;    // den_i (lead lanes)
  double wn;     // omega_i n_i (lead lanes)
  bool lead;
  bool valid;    // gathered (possibly speculatively) for this group
};

__device__ __forceinline__ void pf_range(const KArgs& a, int g, int& t0, int& t1) {
  const size_t base = (size_t)g * (a.G + 1) + ((int)blockIdx.x - a.b0);
  t0 = ld_idx(a.own + base);
  t1 = ld_idx(a.own + base + 1);
}

// The wave's first tile of range [t0, t1) in two steps, so that the loads of
// several tiles can be in flight together: its bounds, then this lane's
// index pair.  kUniform: tile bounds in scalar registers (the merged-pass
// form holds many first tiles at once).
template <bool kUniform>
__device__ __forceinline__ void pf_bounds(const KArgs& a, int t0, int t1, Pf& p, int& e0) {
  const int wave = threadIdx.x >> 6;
  if (kUniform) {
    t0 = __builtin_amdgcn_readfirstlane(t0);
    t1 = __builtin_amdgcn_readfirstlane(t1);
  }
  p.t = wave < kWorkers ? t0 + wave : t1;
  if (kUniform) p.t = __builtin_amdgcn_readfirstlane(p.t);
  p.t1 = t1;
  p.len = 0;
  e0 = 0;
  if (p.t < t1) {
    e0 = ld_idx(a.tile_start + p.t);
    p.len = ld_idx(a.tile_start + p.t + 1) - e0;
  }
}
template <bool kUniform>
__device__ __forceinline__ void pf_rows(const KArgs& a, Pf& p, int e0) {
  const int lane = threadIdx.x & 63;
  if (kUniform) p.len = __builtin_amdgcn_readfirstlane(p.len);
  p.rp = make_uint2(0u, 0xffffffffu);
  if (p.t < p.t1 && p.len <= 64 && lane < p.len) p.rp = a.rp[e0 + lane];
}
template <bool kUniform = false>
__device__ __forceinline__ void pf_tile(const KArgs& a, int t0, int t1, Pf& p) {
  int e0;
  pf_bounds<kUniform>(a, t0, t1, p, e0);
  pf_rows<kUniform>(a, p, e0);
}

// Gather the wave's first tile (short tiles only) into registers, in two
// steps so that several tiles' loads can be in flight together: the loads of
// w and (den_i, omega_i n_i), then the segment sums.
template <typename WT>
__device__ __forceinline__ void gather_load(const KArgs& a, const Pf& p, Cache& c) {
  const int lane = threadIdx.x & 63;
  c.valid = true;
  c.lead = false;
  c.wv = 0.0;
  c.num = 0.0;
  c.den = 1.0;
  c.wn = 0.0;
  if (p.t < p.t1 && p.len <= 64) {
    const WT* __restrict__ w = (const WT*)a.w;
    bool lead;
    int seg_start;
    seg_layout(p.rp.y, lane, p.len, lead, seg_start);
    const bool act = lane < p.len;
    c.wv = act ? (double)w[p.rp.x] : 0.0;
    const double2 pv = lead ? a.pat[pid_of(p.rp.y)] : make_double2(1.0, 0.0);
    c.den = pv.x;
    c.wn = pv.y;
    c.lead = lead;
  }
}
__device__ __forceinline__ void gather_sum(const Pf& p, Cache& c) {
  const int lane = threadIdx.x & 63;
  if (p.t < p.t1 && p.len <= 64) {
    bool lead;
    int seg_start;
    seg_layout(p.rp.y, lane, p.len, lead, seg_start);
    c.num = seg_sum_v(c.wv, lane, seg_start);
  }
}
template <typename WT>
__device__ __forceinline__ void gather_first(const KArgs& a, const Pf& p, Cache& c) {
  gather_load<WT>(a, p, c);
  gather_sum(p, c);
}


// Does the wave's cached first tile hold a patient marked in bits?
__device__ __forceinline__ bool first_tile_stale(const Pf& p, const unsigned* bits, int p0) {
  const int lane = threadIdx.x & 63;
  bool hit = false;
  if (p.t < p.t1 && p.len <= 64 && lane < p.len) {
    const unsigned q = pid_of(p.rp.y) - (unsigned)p0;
    hit = (bits[q >> 5] >> (q & 31)) & 1u;
  }
  return __ballot(hit) != 0ull;
}

// Phase A of the current group for one worker wave: the cached first tile
// (validated by the caller) plus its remaining tiles.
template <typename WT, int NC>
__device__ __forceinline__ void phase_a_cached(const KArgs& a, const Pf& p, const Cache& c, Acc<NC>& acc,
                                               unsigned* bits, int p0, uint32_t coff) {
  if (p.t < p.t1) {
    if (p.len <= 64) {
      if (c.lead) {
        acc.add(col_of(p.rp.y) + coff, c.num, make_double2(c.den, c.wn));
        mark_patient(bits, pid_of(p.rp.y) - (unsigned)p0);
      }
    } else {
      tile_a<WT, NC, true>(a, p.t, acc, bits, p0, coff);
    }
  }
  tiles_a<WT, NC, true>(a, p.t + kWorkers, p.t1, kWorkers, acc, bits, p0, coff);
}

template <typename WT>
__device__ __forceinline__ void phase_b_cached(const KArgs& a, const Pf& p, const Cache& c, Coef cf) {
  const int lane = threadIdx.x & 63;
  WT* __restrict__ w = (WT*)a.w;
  if (p.t < p.t1) {
    if (p.len <= 64) {
      const bool act = lane < p.len;
      const uint32_t col = act ? col_of(p.rp.y) : 0u;
      const double ed = cf.ed[col], em1 = cf.em1[col];
      const bool upd = act && em1 != 0.0;
      const WT wo = (WT)c.wv;
      const WT wn = wo * (WT)ed;
      if (upd) w[p.rp.x] = wn;
      if (sizeof(WT) == 8) {
        if (c.lead && upd) a.pat[pid_of(p.rp.y)].x = c.den + c.num * em1;
      } else {
        bool lead;
        int seg_start;
        seg_layout(p.rp.y, lane, p.len, lead, seg_start);
        double s = seg_sum_v(upd ? (double)wn - (double)wo : 0.0, lane, seg_start);
        if (lead && upd) a.pat[pid_of(p.rp.y)].x = c.den + s;
      }
    } else {
      tile_b<WT>(a, p.t, cf);
    }
  }
  tiles_b<WT>(a, p.t + kWorkers, p.t1, kWorkers, cf);
}

// ---- passes
//
// A pass is one device-wide reduction: a column group, or up to kPassGroups
// consecutive groups (kPassCols columns at most) when each later group is
// predicted independent of the pass's earlier columns.  A group depends on
// an earlier column only if they share a patient (bit of the group's link
// mask) and only if that column takes a nonzero step: until it does, the
// state of the shared patients is untouched.  Under the Laplace prior many
// coordinates stay at zero sweep after sweep, so the prediction is "those
// columns did not move in their last visit" (bit j of a per-column bitmap,
// identical in every workgroup because every workgroup takes the same
// steps).  After the reduction the prediction is checked against the steps
// actually taken: the first group with a linked column that moved, and the
// groups after it, keep no step, and they form the next pass, from fresh
// data.  Either way every column's g_j and h_j are those of the sequential
// order, and each column's partial sums are accumulated in the same order as
// in a pass of its group alone (the other groups add exact zeros, and the
// workgroup and device-wide sums add each word in an order that does not
// depend on the pass's width).

__device__ __forceinline__ int desc_j0(uint32_t d) { return (int)(d & ((1u << kDescColBits) - 1u)); }
__device__ __forceinline__ int desc_m(uint32_t d) { return (int)((d >> kDescWidthShift) & 7u); }
// Links of the group with descriptor d to the `off` columns just before it
// (off <= kLinkCols): bit t for column j0 - off + t.
__device__ __forceinline__ uint32_t desc_links(uint32_t d, int off) {
  return (d >> (kDescLinkShift + kLinkCols - off)) & ((1u << off) - 1u);
}

// Bits [j0, j0 + m) of an LDS bitmap (m <= 8; the bitmap covers j0 + m).
__device__ __forceinline__ uint32_t get_bits(const uint32_t* bm, int j0, int m) {
  const int w = j0 >> 5, sh = j0 & 31;
  uint64_t v = bm[w];
  if (sh + m > 32) v |= (uint64_t)bm[w + 1] << 32;
  return (uint32_t)(v >> sh) & ((1u << m) - 1u);
}

// Set bits [j0, j0 + m) of an LDS bitmap to the low m bits of val (one lane).
__device__ __forceinline__ void set_bits(uint32_t* bm, int j0, int m, uint32_t val) {
  const int w = j0 >> 5, sh = j0 & 31;
  const uint32_t mask = (1u << m) - 1u;
  val &= mask;
  bm[w] = (bm[w] & ~(mask << sh)) | (val << sh);
  if (sh + m > 32) {
    const int r = 32 - sh;
    bm[w + 1] = (bm[w + 1] & ~(mask >> r)) | (val >> r);
  }
}

struct Pass {
  int s, n;                 // first group, number of groups (0: past the last group)
  uint32_t D[kPassGroups];  // descriptors of groups s, s + 1, ... (0 past the last group)
  Pf p[kPassGroups];        // the wave's first tile of each group
};

// Descriptors of groups s .. s + kPassGroups - 1 in lanes 0 .. kPassGroups-1.
__device__ __forceinline__ uint32_t ld_descs(const KArgs& a, int s) {
  const int l = threadIdx.x & 63;
  return (l < kPassGroups && s + l < a.n_groups) ? ld_idx(a.gdesc + s + l) : 0u;
}
__device__ __forceinline__ void take_descs(uint32_t dv, Pass& p) {
#pragma unroll
  for (int k = 0; k < kPassGroups; ++k) p.D[k] = (uint32_t)__builtin_amdgcn_readlane((int)dv, k);
}

// Groups in the pass that starts at group p.s: the longest run of groups
// that fits in kPassCols columns and whose links to the pass's earlier
// columns all point at columns predicted to stay put.  Uniform (scalar
// values and LDS reads of identical values).
__device__ __forceinline__ int plan_pass(const Pass& p, const uint32_t* mv, const KArgs& a) {
  if (!a.merge) return 1;
  const int j0 = desc_j0(p.D[0]);
  const uint32_t pred = get_bits(mv, j0, min(kLinkCols, a.J - j0));
  int cols = desc_m(p.D[0]), n = 1;
  bool open = true;
#pragma unroll
  for (int k = 1; k < kPassGroups; ++k) {
    if (open && p.s + k < a.n_groups) {
      const int mk = desc_m(p.D[k]);
      if (cols + mk <= kPassCols && (desc_links(p.D[k], cols) & pred) == 0u) {
        cols += mk;
        n = k + 1;
      } else {
        open = false;
      }
    }
  }
  return __builtin_amdgcn_readfirstlane(n);
}

// Columns of the first `n` groups of pass p.
__device__ __forceinline__ int pass_cols(const Pass& p, int n) {
  int cols = 0;
#pragma unroll
  for (int k = 0; k < kPassGroups; ++k)
    if (k < n) cols += desc_m(p.D[k]);
  return cols;
}

// Tile indices of every group of pass p (pipeline start).
__device__ __forceinline__ void load_pass(const KArgs& a, Pass& p) {
  int t0[kPassGroups], t1[kPassGroups];
#pragma unroll
  for (int k = 0; k < kPassGroups; ++k)
    if (k < p.n) pf_range(a, p.s + k, t0[k], t1[k]);
  int e0[kPassGroups];
#pragma unroll
  for (int k = 0; k < kPassGroups; ++k)
    if (k < p.n) pf_bounds<true>(a, t0[k], t1[k], p.p[k], e0[k]);
#pragma unroll
  for (int k = 0; k < kPassGroups; ++k)
    if (k < p.n) pf_rows<true>(a, p.p[k], e0[k]);
}

// The pass without its first r groups (a rejected tail, visited again).
__device__ __forceinline__ void drop_groups(Pass& p, int r) {
#pragma unroll
  for (int q = 1; q < kPassGroups; ++q) {
    if (q <= r) {
#pragma unroll
      for (int k = 0; k + 1 < kPassGroups; ++k) {
        p.D[k] = p.D[k + 1];
        p.p[k] = p.p[k + 1];
      }
      p.D[kPassGroups - 1] = 0u;
    }
  }
  p.s += r;
  p.n -= r;
}

// Exact recomputation of w = L x exp(X beta) and den = M w for patients
// [p0, p1) (the dense evaluation of Listing 1's role, plus Step 3).  beta_j
// is read at beta[j * stride].
template <typename WT>
__device__ __forceinline__ void refresh_range(const KArgs& a, const double* beta, int p0, int p1, int tid,
                                              int nthreads, int stride = 1) {
  WT* __restrict__ w = (WT*)a.w;
  for (int i = p0 + tid; i < p1; i += nthreads) {
    double den = 0.0;
    for (int k = a.pptr[i]; k < a.pptr[i + 1]; ++k) {
      double eta = 0.0;
      if (a.era_val)
        for (int c = a.era_ptr[k]; c < a.era_ptr[k + 1]; ++c) eta += a.era_val[c] * beta[(size_t)a.era_col[c] * stride];
      else
        for (int c = a.era_ptr[k]; c < a.era_ptr[k + 1]; ++c) eta += beta[(size_t)a.era_col[c] * stride];
      WT wk = Prec<WT>::weight(a.offset[k], eta);
      w[k] = wk;
      den += (double)wk;
    }
    a.pat[i].x = den;
  }
}

// Per-sweep objective (Section 2.4: evaluated once per cycle):
// L = sum_j beta_j Y'X_j - sum_i omega_i n_i log den_i, plus log p(beta), and
// for the change criterion sum_k |eta_k - eta_k(sweep start)| over owned eras.
// Called by all threads of every workgroup; results valid in all threads.
template <bool kGrouped = true>
__device__ __forceinline__ bool objective(const KArgs& a, const double* sbeta, const double* sprev, int p0, int p1,
                                          uint32_t oseq, double* out3, double (*red)[4], double* bc, int* bci) {
  const int tid = threadIdx.x;
  double loc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = p0 + tid; i < p1; i += kBlock) {
    double2 pv = a.pat[i];
    if (pv.y != 0.0) {
      double t = pv.y * log(pv.x);
      if (t > 0.0) loc[0] += t; else loc[1] -= t;
    }
  }
  if (a.criterion == SCCS_CRIT_ABS_DXBETA && a.mode == kModeSweep) {
    const int k0 = a.pptr[p0], k1 = a.pptr[p1];
    for (int k = k0 + tid; k < k1; k += kBlock) {
      double de = 0.0;
      for (int c = a.era_ptr[k]; c < a.era_ptr[k + 1]; ++c) {
        int jj = a.era_col[c];
        de += a.era_val ? a.era_val[c] * (sbeta[jj] - sprev[jj]) : sbeta[jj] - sprev[jj];
      }
      loc[2] += fabs(de);
    }
  }
  // beta'Y'X and the log prior, summed in the same order in every workgroup
  double bl[2] = {0.0, 0.0};
  for (int j = tid; j < a.J; j += kBlock) {
    double bj = sbeta[j];
    bl[0] += bj * a.ytx[j];
    if (a.prior_kind == SCCS_PRIOR_NORMAL || a.prior_kind == SCCS_PRIOR_GROUPED) bl[1] -= bj * bj / (2.0 * a.var);
    else if (a.prior_kind == SCCS_PRIOR_LAPLACE) bl[1] -= a.lambda * fabs(bj);
  }
  // grouped prior: + kappa_c S_c^2 / (2 var) per class (S_c kept in LDS)
  if (kGrouped && a.prior_kind == SCCS_PRIOR_GROUPED) {
    const double* ssum = (const double*)(&sbeta[0]) + a.ssum_off;
    for (int c = tid; c < a.n_classes; c += kBlock) bl[1] += a.pkappa[c] * ssum[c] * ssum[c] / (2.0 * a.var);
  }
  double part[4];
  block_sum<4>(loc, part, red);
  double bsum[2];
  block_sum<2>(bl, bsum, red);
  if (tid == 0) { bc[4] = bsum[0]; bc[5] = bsum[1]; }
  double tot[4];
  bool ok = allreduce_nonneg<4>(a.oslots, a.oslots2, oseq, a.G, a.ctrl, part, tot, bc, bci, (int)blockIdx.x - a.b0);
  out3[0] = bc[4] - (tot[0] - tot[1]);  // loglik
  out3[1] = out3[0] + bc[5];            // logpost
  out3[2] = tot[2];                     // sum |delta eta|
  __syncthreads();
  return ok;
}

// ------------------------------------------------------------ persistent kernel

template <typename WT, bool kMerge>
__device__ __forceinline__ void ccd_body(const KArgs& a) {
  extern __shared__ double lds_dyn[];
  double* sbeta = lds_dyn;              // [J]
  double* strust = lds_dyn + a.J;       // [J]
  double* sprev = lds_dyn + 2 * a.J;    // [J] beta at the start of the sweep
  __shared__ double red[kWaves][4];
  __shared__ double redg[kWaves][2 * kPassCols];
  __shared__ double bc[8];
  __shared__ int bci[4];
  __shared__ double s_ed[kPassCols], s_em1[kPassCols];

  const int tid = threadIdx.x, b = (int)blockIdx.x - a.b0;
  for (int j = tid; j < a.J; j += kBlock) {
    sbeta[j] = a.beta[j];
    strust[j] = a.trust[j];
  }
  // identical in all workgroups (written by the previous launch)
  uint32_t gseq[kSlotClasses];   // sequence number per reduction class
#pragma unroll
  for (int c = 0; c < kSlotClasses; ++c) gseq[c] = a.ctrl->gseq[c];
  uint32_t oseq = a.ctrl->oseq;
  int since_refresh = a.ctrl->since_refresh;
  __syncthreads();
  // grouped prior (never run in the merged-pass form)
  if (!kMerge && a.prior_kind == SCCS_PRIOR_GROUPED) {
    class_sums(a, sbeta, lds_dyn + a.ssum_off);
    __syncthreads();
  }

  const int p0 = a.pb[b], p1 = a.pb[b + 1];
  const int NG = a.n_groups;
  bool ok = true;
  int status = SCCS_OK;
  double lp_prev = 0.0;
  if (a.criterion == SCCS_CRIT_REL_LOGPOST) {
    double o3[3];
    ok = objective<!kMerge>(a, sbeta, sprev, p0, p1, oseq++, o3, red, bc, bci);
    lp_prev = o3[1];
  }
  int sweep = 0, converged = 0;
  double L = 0.0, P = 0.0;
  // merged passes: the wave index in a scalar register, so that the
  // worker/poller branches are uniform and so is the pass state they assign
  // (the one-pass-per-group loop measured faster without)
  const int wave = kMerge ? __builtin_amdgcn_readfirstlane(tid >> 6) : tid >> 6, lane = tid & 63;
  const bool worker = wave < kWorkers;
  unsigned* bits0 = (unsigned*)(lds_dyn + 3 * a.J);   // patients of even passes
  unsigned* bits1 = bits0 + a.nbits;                  // patients of odd passes
  uint32_t* s_mv = bits1 + a.nbits;                   // moved-column bits (identical in every workgroup)
  for (int i = tid; i < a.mv_words; i += kBlock) s_mv[i] = a.moved[i];
  double* ssum = lds_dyn + a.ssum_off;                // grouped prior: class sums (set up above)
  __shared__ uint32_t s_nn[1 + kPassGroups];   // merged passes: the pass after next (groups, descriptors), for the poller
  // poller lane 0: rejected merges and coordinate visits with an exactly
  // zero step in this launch
  int n_rej = 0, n_zero = 0;
  const Coef cf{s_ed, s_em1};
  __syncthreads();
  while (ok && sweep < a.n_sweeps) {
    if (a.criterion == SCCS_CRIT_ABS_DXBETA)
      for (int j = tid; j < a.J; j += kBlock) sprev[j] = sbeta[j];
    for (int i = tid; i < 2 * a.nbits; i += kBlock) bits0[i] = 0u;
    if constexpr (kMerge) {
      __syncthreads();
      // pipeline start: the first two passes' indices; nothing speculated
      Pass cur, nxt;
      cur.s = 0;
      take_descs(ld_descs(a, 0), cur);
      cur.n = plan_pass(cur, s_mv, a);
      load_pass(a, cur);
      nxt.s = cur.s + cur.n;
      nxt.n = 0;
      take_descs(nxt.s < NG ? ld_descs(a, nxt.s) : 0u, nxt);
      if (nxt.s < NG) {
        nxt.n = plan_pass(nxt, s_mv, a);
        load_pass(a, nxt);
      } else {
        nxt.s = NG;
      }
      // The workers and the poller run the pass sequence in loops of their
      // own, with the same barriers in the same order and the same decisions
      // (every one taken from LDS values that both sides read after a
      // barrier), so that the poller carries none of the workers' tile state
      // through the reduction.
      if (worker) {
        // descriptors of the pass after nxt (lanes 0 .. kPassGroups-1)
        uint32_t dv_nn = (nxt.n > 0 && nxt.s + nxt.n < NG) ? ld_descs(a, nxt.s + nxt.n) : 0u;
        Cache c_cur[kPassGroups], c_nxt[kPassGroups];
#pragma unroll
        for (int k = 0; k < kPassGroups; ++k) c_cur[k].valid = c_nxt[k].valid = false;
        int par = 0;
        // the previous pass changed the state (some step was nonzero): only
        // then can a speculative gather be stale
        bool prev_moved = true;
        while (cur.s < NG) {
          unsigned* bits_cur = par ? bits1 : bits0;
          unsigned* bits_prev = par ? bits0 : bits1;
          // the pass after next: the tile range of its first group is loaded
          // now; the pass is planned in the shadow of the reduction, from the
          // descriptors loaded one pass ago
          Pass nn;
          nn.s = nxt.s + nxt.n;
          nn.n = 0;
#pragma unroll
          for (int k = 0; k < kPassGroups; ++k) nn.D[k] = 0u;
          const bool nn_live = nxt.n > 0 && nn.s < NG;
          int nr0 = 0, nr1 = 0;
          uint32_t dv_nnn = 0u;
          if (nn_live) pf_range(a, nn.s, nr0, nr1);
          const int j0 = desc_j0(cur.D[0]);
          const int m = pass_cols(cur, cur.n);                       // columns of the pass
          const int cls = m <= kMaxGroup ? m - 1 : kMaxGroup;        // its reduction class

          // phase A: validate the speculative first tiles, then accumulate
          Acc<kPassCols> acc;
          acc.zero();
#pragma unroll
          for (int k = 0; k < kPassGroups; ++k) {
            if (k < cur.n) {
              if (!c_cur[k].valid || (prev_moved && first_tile_stale(cur.p[k], bits_prev, p0)))
                gather_first<WT>(a, cur.p[k], c_cur[k]);
              phase_a_cached<WT>(a, cur.p[k], c_cur[k], acc, bits_cur, p0, (uint32_t)(desc_j0(cur.D[k]) - j0));
            }
          }
          double loc[2 * kPassCols], part[2 * kPassCols];
#pragma unroll
          for (int i = 0; i < kPassCols; ++i) {
            loc[2 * i] = acc.g[i];
            loc[2 * i + 1] = acc.h[i];
          }
          switch (m) {   // sum only the words of the pass's columns (m is uniform)
            case 1: block_sum_to<2>(loc, part, redg, kPoller); break;
            case 2: block_sum_to<4>(loc, part, redg, kPoller); break;
            case 3:
            case 4: block_sum_to<8>(loc, part, redg, kPoller); break;
            default: block_sum_to<2 * kPassCols>(loc, part, redg, kPoller); break;
          }
          // in the shadow of the reduction: clear the other bitmap, gather the
          // next pass speculatively, plan the pass after it and load its
          // tile indices
          for (int i = tid; i < a.nbits; i += kWorkers * 64) bits_prev[i] = 0u;
#pragma unroll
          for (int k = 0; k < kPassGroups; ++k)
            if (k < nxt.n) gather_load<WT>(a, nxt.p[k], c_nxt[k]);
#pragma unroll
          for (int k = 0; k < kPassGroups; ++k)
            if (k < nxt.n) gather_sum(nxt.p[k], c_nxt[k]);
          if (nn_live) {
            take_descs(dv_nn, nn);
            nn.n = plan_pass(nn, s_mv, a);
            if (nn.s + nn.n < NG) dv_nnn = ld_descs(a, nn.s + nn.n);
            int t0[kPassGroups], t1[kPassGroups], e0[kPassGroups];
            t0[0] = nr0;
            t1[0] = nr1;
#pragma unroll
            for (int k = 1; k < kPassGroups; ++k)
              if (k < nn.n) pf_range(a, nn.s + k, t0[k], t1[k]);
#pragma unroll
            for (int k = 0; k < kPassGroups; ++k)
              if (k < nn.n) pf_bounds<true>(a, t0[k], t1[k], nn.p[k], e0[k]);
#pragma unroll
            for (int k = 0; k < kPassGroups; ++k)
              if (k < nn.n) pf_rows<true>(a, nn.p[k], e0[k]);
          }
          if (tid == 0) {
            s_nn[0] = (uint32_t)nn.n;
#pragma unroll
            for (int k = 0; k < kPassGroups; ++k) s_nn[1 + k] = nn.D[k];
          }
          __syncthreads();   // the poller's step is in LDS
#pragma unroll
          for (int c = 0; c < kSlotClasses; ++c)
            if (cls == c) ++gseq[c];
          if (!bci[0]) { ok = false; break; }
          if (bci[1]) { status = SCCS_ERR_NUMERIC; ok = false; break; }
          const int na = __builtin_amdgcn_readfirstlane(bci[3]);   // groups whose steps are taken
          prev_moved = __builtin_amdgcn_readfirstlane(bci[2]) != 0;
          if (prev_moved) {
#pragma unroll
            for (int k = 0; k < kPassGroups; ++k)
              if (k < na) {
                const int off = desc_j0(cur.D[k]) - j0;
                phase_b_cached<WT>(a, cur.p[k], c_cur[k], Coef{s_ed + off, s_em1 + off});
              }
          }
          __syncthreads();
          par ^= 1;
          if (na < cur.n) {
            // the rejected groups, from fresh data; nxt and the passes after
            // it stay as planned (their speculative gathers are repeated)
            drop_groups(cur, na);
#pragma unroll
            for (int k = 0; k < kPassGroups; ++k) c_cur[k].valid = false;
          } else {
            cur = nxt;
#pragma unroll
            for (int k = 0; k < kPassGroups; ++k) c_cur[k] = c_nxt[k];
            nxt = nn;
            dv_nn = dv_nnn;
            if (nxt.n == 0) nxt.s = NG;
          }
        }
      } else {
        int mv_cols = 0;        // columns whose moved bits this pass sets
        uint32_t mv_val = 0u;
        while (cur.s < NG) {
          Pass nn;
          nn.s = nxt.s + nxt.n;
          const int j0 = desc_j0(cur.D[0]);
          const int m = pass_cols(cur, cur.n);
          const int cls = m <= kMaxGroup ? m - 1 : kMaxGroup;
          const double ytx_cur = lane < m ? a.ytx[j0 + lane] : 0.0;
          double loc[2 * kPassCols], part[2 * kPassCols];
#pragma unroll
          for (int i = 0; i < 2 * kPassCols; ++i) loc[i] = part[i] = 0.0;
          switch (m) {
            case 1: block_sum_to<2>(loc, part, redg, kPoller); break;
            case 2: block_sum_to<4>(loc, part, redg, kPoller); break;
            case 3:
            case 4: block_sum_to<8>(loc, part, redg, kPoller); break;
            default: block_sum_to<2 * kPassCols>(loc, part, redg, kPoller); break;
          }
          // device-wide reduction of the pass's 2m partials, then one Newton /
          // trust-region step (Eq. 4) per column, lane c for column j0 + c
          double tot[2 * kPassCols];
          uint32_t sq = gseq[0];
#pragma unroll
          for (int c = 1; c < kSlotClasses; ++c)
            if (cls == c) sq = gseq[c];
          uint64_t* s1 = a.slots + cls * kSlots1PerClass;
          uint64_t* s2 = a.slots2 + cls * kSlots2PerClass;
#pragma unroll
          for (int i = 0; i < 2 * kPassCols; ++i) tot[i] = 0.0;
          bool okr;
          switch (cls) {   // one width per slot class, fixed at compile time
            case 0: okr = allreduce2_wave<2>(s1, s2, sq, a.G, a.ctrl, part, tot, b); break;
#if SCCS_MAX_GROUP >= 2
            case 1: okr = allreduce2_wave<4>(s1, s2, sq, a.G, a.ctrl, part, tot, b); break;
#endif
#if SCCS_MAX_GROUP >= 3
            case 2: okr = allreduce2_wave<6>(s1, s2, sq, a.G, a.ctrl, part, tot, b); break;
#endif
#if SCCS_MAX_GROUP >= 4
            case 3: okr = allreduce2_wave<8>(s1, s2, sq, a.G, a.ctrl, part, tot, b); break;
#endif
            default: okr = allreduce2_wave<2 * kPassCols>(s1, s2, sq, a.G, a.ctrl, part, tot, b); break;
          }

          double Gc = 0.0, Hc = 0.0;
#pragma unroll
          for (int i = 0; i < kPassCols; ++i)
            if (lane == i) {
              Gc = tot[2 * i];
              Hc = tot[2 * i + 1];
            }
          double d = 0.0, bj = 0.0, tr = 0.0;
          int bad = 0;
          if (lane < m) {
            const double gg = ytx_cur - Gc, hh = -Hc;
            bad = !(isfinite(gg) && isfinite(hh));
            if (okr && !bad) {
              bj = sbeta[j0 + lane];
              tr = strust[j0 + lane];
              const double dv = prior_step(a.prior_kind, a.inv_var, a.lambda, bj, gg, hh);
              d = fmin(fmax(dv, -tr), tr);
            }
          }
          // the first group of the pass with a linked column that moved, and
          // the groups after it, keep no step (their sums are discarded); they
          // are visited again in the next pass
          const uint32_t moved_all = (uint32_t)__ballot(lane < m && d != 0.0);
          int na = cur.n, mc = m;   // groups and columns whose steps are taken
          bool open = true;
#pragma unroll
          for (int k = 1; k < kPassGroups; ++k) {
            if (open && k < cur.n) {
              const int off = desc_j0(cur.D[k]) - j0;
              if (desc_links(cur.D[k], off) & moved_all) {
                na = k;
                mc = off;
                open = false;
              }
            }
          }
          if (lane >= mc) {
            d = 0.0;
            bad = 0;
          }
          if (lane < mc && okr && !bad) {
            strust[j0 + lane] = fmax(2.0 * fabs(d), 0.5 * tr);
            const double nb = bj + d;
            if (!isfinite(nb)) { bad = 1; d = 0.0; }
            else sbeta[j0 + lane] = nb;
          }
          if (lane < kPassCols) {
            double em1 = 0.0;   // most late-sweep steps are exactly zero
            if (d != 0.0) em1 = expm1(d);
            s_ed[lane] = 1.0 + em1;
            s_em1[lane] = em1;
          }
          const uint64_t moved = __ballot(lane < mc && d != 0.0);
          const bool any_bad = __ballot(bad != 0) != 0ull;
          if (lane == 0) {
            bci[0] = okr ? 1 : 0;
            bci[1] = any_bad ? 1 : 0;
            bci[2] = moved != 0ull ? 1 : 0;
            bci[3] = na;
          }
          mv_cols = okr ? mc : 0;
          mv_val = (uint32_t)moved;
          n_rej += na < cur.n ? 1 : 0;
          n_zero += mv_cols - __popcll(moved);
          __syncthreads();   // the workers' plan of the pass after next is in LDS
#pragma unroll
          for (int c = 0; c < kSlotClasses; ++c)
            if (cls == c) ++gseq[c];
          if (!bci[0]) { ok = false; break; }
          if (bci[1]) { status = SCCS_ERR_NUMERIC; ok = false; break; }
          // while the workers update: record which columns moved (no pass
          // reads these bits before the next sweep); take the plan of the
          // pass after next from the workers
          if (lane == 0 && mv_cols > 0) set_bits(s_mv, j0, mv_cols, mv_val);
          nn.n = (int)__builtin_amdgcn_readfirstlane(s_nn[0]);
#pragma unroll
          for (int k = 0; k < kPassGroups; ++k) nn.D[k] = __builtin_amdgcn_readfirstlane(s_nn[1 + k]);
          __syncthreads();
          if (na < cur.n) {
            drop_groups(cur, na);
          } else {
            cur = nxt;
            nxt = nn;
            if (nxt.n == 0) nxt.s = NG;
          }
        }
      }
    } else {
      // one pass per column group (few zero steps to exploit, or merging
      // off); the moved bits are kept up to date as well, so that a
      // following merged-pass launch starts with a prediction.  As in the
      // merged-pass form, the workers and the poller run the group sequence
      // in loops of their own with the same barriers.
      const bool worker_u = __builtin_amdgcn_readfirstlane(tid >> 6) < kWorkers;
      if (worker_u) {
        // pipeline start: indices of groups 0 and 1; nothing speculated
        Pf pf_cur, pf_next;
        {
          int t0, t1;
          pf_range(a, 0, t0, t1);
          pf_tile(a, t0, t1, pf_cur);
          pf_range(a, NG > 1 ? 1 : 0, t0, t1);
          pf_tile(a, t0, t1, pf_next);
        }
        Cache c_cur, c_next;
        c_cur.valid = false;
        // group bounds gcol[g], gcol[g+1], gcol[g+2] roll through registers,
        // each loaded two groups before it is needed
        int j0 = a.gcol[0], gc1 = a.gcol[1], gc2 = NG > 1 ? a.gcol[2] : gc1;
        int m = gc1 - j0;
        bool prev_moved = true;   // the previous group took a nonzero step
        __syncthreads();
        for (int g = 0; g < NG; ++g) {
          unsigned* bits_cur = (g & 1) ? bits1 : bits0;
          unsigned* bits_prev = (g & 1) ? bits0 : bits1;
          const bool has_next = g + 1 < NG;
          int nt0 = 0, nt1 = 0;
          if (g + 2 < NG) pf_range(a, g + 2, nt0, nt1);
          const int gc3 = g + 3 <= NG ? ld_idx(a.gcol + g + 3) : gc2;
          const int mn = has_next ? gc2 - gc1 : 0;

          // phase A: validate the speculative first tile, then accumulate
          Acc<kMaxGroup> acc;
          acc.zero();
          if (!c_cur.valid || (g > 0 && prev_moved && first_tile_stale(pf_cur, bits_prev, p0)))
            gather_first<WT>(a, pf_cur, c_cur);
          phase_a_cached<WT, kMaxGroup>(a, pf_cur, c_cur, acc, bits_cur, p0, 0u);
          double loc[2 * kMaxGroup], part[2 * kMaxGroup];
#pragma unroll
          for (int i = 0; i < kMaxGroup; ++i) {
            loc[2 * i] = acc.g[i];
            loc[2 * i + 1] = acc.h[i];
          }
          switch (m) {   // sum only the words of the group's columns (m is uniform)
            case 1: block_sum_to<2>(loc, part, redg, kPoller); break;
#if SCCS_MAX_GROUP >= 2
            case 2: block_sum_to<4>(loc, part, redg, kPoller); break;
#endif
            default: block_sum_to<2 * kMaxGroup>(loc, part, redg, kPoller); break;
          }
          // in the shadow of the reduction: clear the bitmap of group g+1,
          // gather group g+1 speculatively, load indices of group g+2
          Pf pf_next2;
          pf_next2.t = pf_next2.t1 = 0;
          c_next.valid = false;
          for (int i = tid; i < a.nbits; i += kWorkers * 64) bits_prev[i] = 0u;
          if (has_next) gather_first<WT>(a, pf_next, c_next);
          if (g + 2 < NG) pf_tile(a, nt0, nt1, pf_next2);
          __syncthreads();   // the poller's step is in LDS
#pragma unroll
          for (int c = 0; c < kMaxGroup; ++c)
            if (m - 1 == c) ++gseq[c];
          if (!bci[0]) { ok = false; break; }
          if (bci[1]) { status = SCCS_ERR_NUMERIC; ok = false; break; }
          prev_moved = __builtin_amdgcn_readfirstlane(bci[2]) != 0;
          if (prev_moved) phase_b_cached<WT>(a, pf_cur, c_cur, cf);
          __syncthreads();
          pf_cur = pf_next;
          pf_next = pf_next2;
          c_cur = c_next;
          j0 = gc1;
          m = mn;
          gc1 = gc2;
          gc2 = gc3;
        }
      } else {
        uint32_t mv_val = 0u;   // the last group's moved columns
        int j0 = a.gcol[0], gc1 = a.gcol[1], gc2 = NG > 1 ? a.gcol[2] : gc1;
        int m = gc1 - j0;
        double ytx_cur = lane < m ? a.ytx[j0 + lane] : 0.0;
        __syncthreads();
        // (the stamp is a store that the next barrier waits for: taken
        // only on request)
        const bool stamp = a.stamp && b == 0 && lane == 0;
        if (stamp) a.group_ticks[NG] = wall_clock64();
        for (int g = 0; g < NG; ++g) {
          const bool has_next = g + 1 < NG;
          const int gc3 = g + 3 <= NG ? ld_idx(a.gcol + g + 3) : gc2;
          const int j0n = gc1;
          const int mn = has_next ? gc2 - gc1 : 0;
          const double ytx_next = lane < mn ? a.ytx[j0n + lane] : 0.0;
          double loc[2 * kMaxGroup], part[2 * kMaxGroup];
#pragma unroll
          for (int i = 0; i < 2 * kMaxGroup; ++i) loc[i] = part[i] = 0.0;
          switch (m) {
            case 1: block_sum_to<2>(loc, part, redg, kPoller); break;
#if SCCS_MAX_GROUP >= 2
            case 2: block_sum_to<4>(loc, part, redg, kPoller); break;
#endif
            default: block_sum_to<2 * kMaxGroup>(loc, part, redg, kPoller); break;
          }
          // device-wide reduction of the group's 2m partials, then one
          // Newton / trust-region step (Eq. 4) per column, lane c for column
          // j0 + c (the columns are independent)
          double tot[2 * kMaxGroup];
          const int cls = m - 1;
          uint32_t sq = gseq[0];
#pragma unroll
          for (int c = 1; c < kMaxGroup; ++c)
            if (cls == c) sq = gseq[c];
          uint64_t* s1 = a.slots + cls * kSlots1PerClass;
          uint64_t* s2 = a.slots2 + cls * kSlots2PerClass;
#pragma unroll
          for (int i = 0; i < 2 * kMaxGroup; ++i) tot[i] = 0.0;
          // beta_j and Delta_j of the lane's column, read before the wait:
          // only this lane writes them, after the reduction
          const double bj_pre = lane < m ? sbeta[j0 + lane] : 0.0;
          const double tr_pre = lane < m ? strust[j0 + lane] : 1.0;
          bool okr;
          switch (m) {   // one width per slot class, fixed at compile time
            case 1: okr = allreduce2_wave<2>(s1, s2, sq, a.G, a.ctrl, part, tot, b); break;
#if SCCS_MAX_GROUP >= 2
            case 2: okr = allreduce2_wave<4>(s1, s2, sq, a.G, a.ctrl, part, tot, b); break;
#endif
#if SCCS_MAX_GROUP >= 3
            case 3: okr = allreduce2_wave<6>(s1, s2, sq, a.G, a.ctrl, part, tot, b); break;
#endif
            default: okr = allreduce2_wave<2 * kMaxGroup>(s1, s2, sq, a.G, a.ctrl, part, tot, b); break;
          }

          double Gc = 0.0, Hc = 0.0;
#pragma unroll
          for (int i = 0; i < kMaxGroup; ++i)
            if (lane == i) {
              Gc = tot[2 * i];
              Hc = tot[2 * i + 1];
            }
          double d = 0.0;
          int bad = 0;
          if (a.prior_kind == SCCS_PRIOR_GROUPED) {
            grouped_steps(a, j0, m, okr, ytx_cur - Gc, -Hc, sbeta, strust, ssum, d, bad);
          } else if (lane < m) {
            const double gg = ytx_cur - Gc, hh = -Hc;
            bad = !(isfinite(gg) && isfinite(hh));
            if (okr && !bad) {
              const int j = j0 + lane;
              const double bj = bj_pre, tr = tr_pre;
              const double dv = prior_step(a.prior_kind, a.inv_var, a.lambda, bj, gg, hh);
              d = fmin(fmax(dv, -tr), tr);
              strust[j] = fmax(2.0 * fabs(d), 0.5 * tr);
              const double nb = bj + d;
              if (!isfinite(nb)) { bad = 1; d = 0.0; }
              else sbeta[j] = nb;
            }
          }
          if (lane < kMaxGroup) {
            double em1 = 0.0;   // most late-sweep steps are exactly zero
            if (d != 0.0) em1 = expm1(d);
            s_ed[lane] = 1.0 + em1;
            s_em1[lane] = em1;
          }
          const uint64_t moved = __ballot(lane < m && d != 0.0);
          const bool any_bad = __ballot(bad != 0) != 0ull;
          if (lane == 0) {
            bci[0] = okr ? 1 : 0;
            bci[1] = any_bad ? 1 : 0;
            bci[2] = moved != 0ull ? 1 : 0;
          }
          n_zero += okr ? m - __popcll(moved) : 0;
          mv_val = (uint32_t)moved;
          if (stamp) a.group_ticks[g] = wall_clock64();
          __syncthreads();
#pragma unroll
          for (int c = 0; c < kMaxGroup; ++c)
            if (m - 1 == c) ++gseq[c];
          if (!bci[0]) { ok = false; break; }
          if (bci[1]) { status = SCCS_ERR_NUMERIC; ok = false; break; }
          if (lane == 0) set_bits(s_mv, j0, m, mv_val);   // while the workers update
          __syncthreads();
          ytx_cur = ytx_next;
          j0 = j0n;
          m = mn;
          gc1 = gc2;
          gc2 = gc3;
        }
      }
    }
    if (!ok) break;
    ++sweep;
    if (a.refresh_period > 0 && ++since_refresh >= a.refresh_period) {
      refresh_range<WT>(a, sbeta, p0, p1, tid, kBlock);
      since_refresh = 0;
      __syncthreads();
    }
    const bool need_obj = (a.criterion != SCCS_CRIT_FIXED) || (a.want_objective && sweep == a.n_sweeps);
    if (need_obj) {
      double o3[3];
      if (!objective<!kMerge>(a, sbeta, sprev, p0, p1, oseq++, o3, red, bc, bci)) { ok = false; break; }
      L = o3[0];
      P = o3[1];
      if (a.criterion == SCCS_CRIT_REL_LOGPOST) {
        if (fabs(P - lp_prev) < a.tol * fabs(P)) converged = 1;
        lp_prev = P;
      } else if (a.criterion == SCCS_CRIT_ABS_DXBETA) {
        if (o3[2] < a.tol) converged = 1;
      }
      if (!isfinite(P)) { status = SCCS_ERR_NUMERIC; ok = false; break; }
    }
    if (converged) break;
  }

  __syncthreads();
  if (b == 0) {
    for (int j = tid; j < a.J; j += kBlock) {
      a.beta[j] = sbeta[j];
      a.trust[j] = strust[j];
    }
    for (int i = tid; i < a.mv_words; i += kBlock) a.moved[i] = s_mv[i];
    if (tid == kPoller * 64) {
      a.ctrl->rejects = n_rej;
      a.ctrl->zero_steps = n_zero;
    }
    if (tid == 0) {

      a.ctrl->sweeps = sweep;
      a.ctrl->converged = converged;
      a.ctrl->loglik = L;
      a.ctrl->logpost = P;
      for (int c = 0; c < kSlotClasses; ++c) a.ctrl->gseq[c] = gseq[c];
      a.ctrl->oseq = oseq;
      a.ctrl->since_refresh = since_refresh;
      if (status != SCCS_OK) a.ctrl->status = status;
    }
  }
}

template <typename WT, bool kMerge>
__global__ void __launch_bounds__(kBlock) k_ccd(KArgs a) {
  ccd_body<WT, kMerge>(a);
}

// Several independent single fits in one cooperative launch: workgroup x
// runs fit fit_of_block[x] as that fit's workgroup x - b0 of G (its own
// layout for G workgroups, its own state, reduction slots and control
// block), so each fit advances, and stops, on its own.
template <typename WT, bool kMerge>
__global__ void __launch_bounds__(kBlock) k_ccd_multi(const KArgs* __restrict__ fits,
                                                      const int32_t* __restrict__ fit_of_block) {
  ccd_body<WT, kMerge>(fits[fit_of_block[blockIdx.x]]);
}

// Diagnostics: g_j, h_j of column diag_j (column diag_c of group diag_g) at
// the current beta (mode 1), or the objective (mode 2).  Same ownership and
// reductions as the sweep kernel.
template <typename WT>
__global__ void __launch_bounds__(kBlock) k_diag(KArgs a) {
  extern __shared__ double lds_dyn[];
  double* sbeta = lds_dyn;
  __shared__ double red[kWaves][4];
  __shared__ double bc[8];
  __shared__ int bci[4];
  const int tid = threadIdx.x, b = (int)blockIdx.x - a.b0;
  for (int j = tid; j < a.J; j += kBlock) sbeta[j] = a.beta[j];
  uint32_t seq = a.ctrl->gseq[0], oseq = a.ctrl->oseq;   // one column: reduction class 0
  __syncthreads();
  const int p0 = a.pb[b], p1 = a.pb[b + 1];
  if (a.mode == kModeObjective) {
    if (a.prior_kind == SCCS_PRIOR_GROUPED) {
      class_sums(a, sbeta, lds_dyn + a.ssum_off);
      __syncthreads();
    }
    double o3[3];
    bool ok = objective(a, sbeta, sbeta, p0, p1, oseq++, o3, red, bc, bci);
    if (b == 0 && tid == 0 && ok) { a.ctrl->loglik = o3[0]; a.ctrl->logpost = o3[1]; }
  } else {
    Acc<kMaxGroup> acc;
    acc.zero();
    int t0, t1;
    pf_range(a, a.diag_g, t0, t1);
    for (int t = t0 + (tid >> 6); t < t1; t += kWaves) tile_a<WT, kMaxGroup, false>(a, t, acc);
    double loc[2] = {0.0, 0.0}, part2[2];
#pragma unroll
    for (int i = 0; i < kMaxGroup; ++i)
      if (i == a.diag_c) {
        loc[0] = acc.g[i];
        loc[1] = acc.h[i];
      }
    block_sum<2>(loc, part2, red);
    double tot[2];
    bool ok = allreduce_nonneg<2>(a.slots, a.slots2, seq++, a.G, a.ctrl, part2, tot, bc, bci, b);
    if (b == 0 && tid == 0 && ok) { a.ctrl->g = a.ytx[a.diag_j] - tot[0]; a.ctrl->h = -tot[1]; }
  }
  __syncthreads();
  if (b == 0 && tid == 0) { a.ctrl->gseq[0] = seq; a.ctrl->oseq = oseq; }
}

// Held-out log-likelihood of one fit (Eq. 2 over its weight-0 patients):
// block partials of -sum_i hn_i log den_i over a fixed grid, then one block
// adds them and beta'Y'X(held out) (fixed order throughout).
constexpr int kHoBlocks = 1024;
__global__ void __launch_bounds__(256) k_heldout_part(const double2* pat, const double* hn, int N, double* part) {
  __shared__ double red[4];
  double s = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < N; i += kHoBlocks * 256)
    if (hn[i] != 0.0) s -= hn[i] * log(pat[i].x);
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}
__global__ void __launch_bounds__(256) k_heldout_final(const double* part, const double* beta, const double* ytx_ho,
                                                       int J, double* out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int j = threadIdx.x; j < J; j += 256) s += beta[j] * ytx_ho[j];
  for (int b = threadIdx.x; b < kHoBlocks; b += 256) s += part[b];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) *out = (red[0] + red[1]) + (red[2] + red[3]);
}

// ------------------------------------------------------------ setup kernels

__global__ void k_fill_u64(uint64_t* p, size_t n, uint64_t v) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// omega_i n_i with n_i = sum_k y_ik
__global__ void k_setup_patients(const int32_t* pptr, const int32_t* count, const int32_t* weight,
                                 double2* pat, int N) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
    long long n = 0;
    for (int k = pptr[i]; k < pptr[i + 1]; ++k) n += count[k];
    double om = weight ? (double)weight[i] : 1.0;
    pat[i].y = om * (double)n;
  }
}

// n_i of the patients whose weight is 0 (the held-out set of a cross-
// validation fold), 0 for every other patient.
__global__ void k_setup_heldout(const int32_t* pptr, const int32_t* count, const int32_t* weight, double* hn, int N) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < N; i += gridDim.x * blockDim.x) {
    long long n = 0;
    for (int k = pptr[i]; k < pptr[i + 1]; ++k) n += count[k];
    hn[i] = weight[i] == 0 ? (double)n : 0.0;
  }
}

// Y'X_j with patient weights: one workgroup per column, fixed-order sum.
// complement != 0 sums over the weight-0 patients only (held-out set).
__global__ void __launch_bounds__(256) k_setup_ytx(const int64_t* col_ptr, const uint2* rp, const int32_t* count,
                                                   const int32_t* weight, int complement, double* ytx, int J) {
  __shared__ double red[4];
  for (int j = blockIdx.x; j < J; j += gridDim.x) {
    double s = 0.0;
    for (long long e = col_ptr[j] + threadIdx.x; e < col_ptr[j + 1]; e += blockDim.x) {
      uint2 q = rp[e];
      double om = weight ? (double)weight[q.y] : 1.0;
      if (complement) om = om == 0.0 ? 1.0 : 0.0;
      s += om * (double)count[q.x];
    }
    s = wave_sum(s);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) ytx[j] = red[0] + red[1] + red[2] + red[3];
    __syncthreads();
  }
}

template <typename WT>
__global__ void k_refresh(KArgs a) {
  refresh_range<WT>(a, a.beta, 0, a.N, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

// Same, with beta taken from the x members of a (beta, trust) array.
template <typename WT>
__global__ void k_refresh_bt(KArgs a, const double2* bt) {
  refresh_range<WT>(a, (const double*)bt, 0, a.N, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x, 2);
}

template __global__ void k_ccd<double, false>(KArgs);
template __global__ void k_ccd<double, true>(KArgs);
template __global__ void k_ccd<float, false>(KArgs);
template __global__ void k_ccd<float, true>(KArgs);
template __global__ void k_ccd_multi<double, false>(const KArgs*, const int32_t*);
template __global__ void k_ccd_multi<float, false>(const KArgs*, const int32_t*);
template __global__ void k_diag<double>(KArgs);
template __global__ void k_diag<float>(KArgs);
template __global__ void k_refresh<double>(KArgs);
template __global__ void k_refresh<float>(KArgs);
template __global__ void k_refresh_bt<double>(KArgs, const double2*);
template __global__ void k_refresh_bt<float>(KArgs, const double2*);

}  // namespace sccs
