// Non-binary and dense covariates: the CCD sweep for problems whose stored
// entries carry values x_kj (Section 4 names dense covariates such as
// baseline measurements as the next extension of the model).
//
// Differentiating Eq. 2 along beta_j with eta = X beta gives, per patient i
// with A_i = M[w x X_j]_i / den_i and B_i = M[w x X_j^2]_i / den_i,
//   g_j = Y'X_j - sum_i omega_i n_i A_i,
//   h_j = -sum_i omega_i n_i (B_i - A_i^2),
// which for binary x (B = A = W) is Eqs. 7-9.  A step delta on column j
// multiplies w_k by exp(delta x_kj) on the column's rows (one exp per
// nonzero, the paper's Steps 1-2 in full) and moves den_i by the sum of the
// changes.
//
// Same ownership, tiles, column groups and tagged device-wide reduction as
// the binary sweep (sccs_kernels.hpp), without its merged passes and
// speculative gathers: every workgroup walks its tiles of a group with all
// eight waves, reduces, steps and updates.  A dense column is a column that
// stores every row; its segments are whole patients.
//
// The tagged reduction needs non-negative words, and with signed covariate
// values the sum behind g_j has either sign: each column carries three words,
// the positive and the negative parts of sum omega n A and the sum behind
// h_j (B - A^2 >= 0 by Cauchy-Schwarz; clamped at 0 against rounding).
#pragma once
#include "sccs_kernels.hpp"

namespace sccs {

constexpr int kValWords = 3;   // reduction words per column

// class sums of the grouped prior in the dynamic LDS area (sbeta is its start)
__device__ __forceinline__ double* lds_dyn_ssum(const KArgs& a, double* sbeta) { return sbeta + a.ssum_off; }
static_assert(kValWords * kMaxGroup <= kSlotWords, "one slot line per group");

// Per-lane accumulators of (positive part, negative part) of
// sum omega n A and of sum omega n (B - A^2), for the NC columns of a group.
template <int NC>
struct AccV {
  double gp[NC], gn[NC], h[NC];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int i = 0; i < NC; ++i) gp[i] = gn[i] = h[i] = 0.0;
  }
  // s1 = M[w x X_j]_i and s2 = M[w x X_j^2]_i over the segment; both zero
  // adds nothing (also for a patient whose eras all have length 0)
  __device__ __forceinline__ void add(uint32_t c, double s1, double s2, double2 pv) {
    const bool z = s1 == 0.0 && s2 == 0.0;
    const double A = z ? 0.0 : s1 / pv.x, B = z ? 0.0 : s2 / pv.x;
    const double tg = pv.y * A;
    const double th = pv.y * fmax(B - A * A, 0.0);
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      const bool mine = NC == 1 || c == (uint32_t)i;
      gp[i] += mine ? fmax(tg, 0.0) : 0.0;
      gn[i] += mine ? fmax(-tg, 0.0) : 0.0;
      h[i] += mine ? th : 0.0;
    }
  }
};

// Phase A on tile t: gather w on the tile's rows, form w x and w x^2 with
// the stored values, sum both per (column, patient) segment, and add the
// segment's terms.
template <typename WT, int NC>
__device__ __forceinline__ void tile_a_val(const KArgs& a, int t, AccV<NC>& acc) {
  const int lane = threadIdx.x & 63;
  const WT* __restrict__ w = (const WT*)a.w;
  const int e0 = ld_idx(a.tile_start + t), e1 = ld_idx(a.tile_start + t + 1);
  const int len = e1 - e0;
  if (len <= 64) {
    const bool act = lane < len;
    const uint2 rp = act ? a.rp[e0 + lane] : make_uint2(0u, 0xffffffffu);
    const double x = act ? a.val[e0 + lane] : 0.0;
    const double wx = act ? (double)w[rp.x] * x : 0.0;
    bool lead;
    int seg_start;
    seg_layout(rp.y, lane, len, lead, seg_start);
    const double s1 = seg_sum_v(wx, lane, seg_start);
    const double s2 = seg_sum_v(wx * x, lane, seg_start);
    if (lead) acc.add(col_of(rp.y), s1, s2, a.pat[pid_of(rp.y)]);
  } else {
    // one (column, patient) segment with more than 64 nonzeros
    double s1 = 0.0, s2 = 0.0;
    for (int e = e0 + lane; e < e1; e += 64) {
      const double x = a.val[e];
      const double wx = (double)w[a.rp[e].x] * x;
      s1 += wx;
      s2 += wx * x;
    }
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    if (lane == 0) {
      const uint32_t key = a.rp[e0].y;
      acc.add(col_of(key), s1, s2, a.pat[pid_of(key)]);
    }
  }
}

// New weight and its change for a step d on an entry with value x: FP64
// w e^{dx} (change w (e^{dx} - 1)); mixed: the FP32 weight times an FP32
// exp, and the exact change of the stored weight in FP64.
template <typename WT>
__device__ __forceinline__ WT val_update(WT wo, double d, double x, double& delta) {
  if constexpr (sizeof(WT) == 8) {
    const double em1 = expm1(d * x);
    delta = (double)wo * em1;
    return (WT)((double)wo * (1.0 + em1));
  } else {
    const WT wn = wo * expf((float)(d * x));
    delta = (double)wn - (double)wo;
    return wn;
  }
}

// Phase B on tile t: w_k <- w_k exp(d_c x_k) on the rows of columns with a
// nonzero step d_c, and den_i += the sum of the changes per segment.
template <typename WT>
__device__ __forceinline__ void tile_b_val(const KArgs& a, int t, const double* s_d) {
  const int lane = threadIdx.x & 63;
  WT* __restrict__ w = (WT*)a.w;
  const int e0 = ld_idx(a.tile_start + t), e1 = ld_idx(a.tile_start + t + 1);
  const int len = e1 - e0;
  if (len <= 64) {
    const bool act = lane < len;
    const uint2 rp = act ? a.rp[e0 + lane] : make_uint2(0u, 0xffffffffu);
    const double d = act ? s_d[col_of(rp.y)] : 0.0;
    const bool upd = act && d != 0.0;
    double delta = 0.0;
    if (upd) {
      const WT wo = w[rp.x];
      w[rp.x] = val_update<WT>(wo, d, a.val[e0 + lane], delta);
    }
    bool lead;
    const double s = seg_sum(delta, rp.y, lane, len, lead);
    if (lead && upd) a.pat[pid_of(rp.y)].x += s;
  } else {
    const uint32_t key = a.rp[e0].y;
    const double d = s_d[col_of(key)];
    if (d == 0.0) return;
    double s = 0.0;
    for (int e = e0 + lane; e < e1; e += 64) {
      const uint32_t row = a.rp[e].x;
      double delta;
      w[row] = val_update<WT>(w[row], d, a.val[e], delta);
      s += delta;
    }
    s = wave_sum(s);
    if (lane == 0) a.pat[pid_of(key)].x += s;
  }
}

// Tiles t, t + stride, ... < t1 in order, software-pipelined as the binary
// sweep's tile loops: the next tile's pairs and values and the bounds of
// the tile after it are loaded while this tile's gathers are in flight, and
// the patient words are gathered together with w.  The arithmetic and its
// order are those of tile_a_val and tile_b_val.
__device__ __forceinline__ double tile_value(const KArgs& a, int e0, int len) {
  const int lane = threadIdx.x & 63;
  return len <= 64 && lane < len ? a.val[e0 + lane] : 0.0;
}

template <typename WT, int NC>
__device__ __forceinline__ void tiles_a_val(const KArgs& a, int t, int t1, int stride, AccV<NC>& acc) {
  if (t >= t1) return;
  const int lane = threadIdx.x & 63;
  const WT* __restrict__ w = (const WT*)a.w;
  int e0, len, en, lenn;
  tile_bounds(a, t, t1, e0, len);
  tile_bounds(a, t + stride, t1, en, lenn);
  uint2 rp = tile_pair(a, e0, len);
  double x = tile_value(a, e0, len);
  while (true) {
    uint2 rpn;
    double xn;
    int enn, lennn;
    if (len <= 64) {
      bool lead;
      int seg_start;
      seg_layout(rp.y, lane, len, lead, seg_start);
      const bool act = lane < len;
      const double wv = act ? (double)w[rp.x] : 0.0;
      const double2 pv = lead ? a.pat[pid_of(rp.y)] : make_double2(1.0, 0.0);
      rpn = tile_pair(a, en, lenn);
      xn = tile_value(a, en, lenn);
      tile_bounds(a, t + 2 * stride, t1, enn, lennn);
      const double wx = act ? wv * x : 0.0;
      const double s1 = seg_sum_v(wx, lane, seg_start);
      const double s2 = seg_sum_v(wx * x, lane, seg_start);
      if (lead) acc.add(col_of(rp.y), s1, s2, pv);
    } else {
      rpn = tile_pair(a, en, lenn);
      xn = tile_value(a, en, lenn);
      tile_bounds(a, t + 2 * stride, t1, enn, lennn);
      tile_a_val<WT, NC>(a, t, acc);
    }
    t += stride;
    if (t >= t1) break;
    rp = rpn;
    x = xn;
    e0 = en;
    len = lenn;
    en = enn;
    lenn = lennn;
  }
}

template <typename WT>
__device__ __forceinline__ void tiles_b_val(const KArgs& a, int t, int t1, int stride, const double* s_d) {
  if (t >= t1) return;
  const int lane = threadIdx.x & 63;
  WT* __restrict__ w = (WT*)a.w;
  int e0, len, en, lenn;
  tile_bounds(a, t, t1, e0, len);
  tile_bounds(a, t + stride, t1, en, lenn);
  uint2 rp = tile_pair(a, e0, len);
  double x = tile_value(a, e0, len);
  while (true) {
    uint2 rpn;
    double xn;
    int enn, lennn;
    if (len <= 64) {
      const bool act = lane < len;
      const double d = act ? s_d[col_of(rp.y)] : 0.0;
      const bool upd = act && d != 0.0;
      bool lead;
      int seg_start;
      seg_layout(rp.y, lane, len, lead, seg_start);
      const WT wo = upd ? w[rp.x] : (WT)0;
      const double den = lead && upd ? a.pat[pid_of(rp.y)].x : 0.0;
      rpn = tile_pair(a, en, lenn);
      xn = tile_value(a, en, lenn);
      tile_bounds(a, t + 2 * stride, t1, enn, lennn);
      double delta = 0.0;
      if (upd) w[rp.x] = val_update<WT>(wo, d, x, delta);
      const double sd = seg_sum_v(delta, lane, seg_start);
      if (lead && upd) a.pat[pid_of(rp.y)].x = den + sd;
    } else {
      rpn = tile_pair(a, en, lenn);
      xn = tile_value(a, en, lenn);
      tile_bounds(a, t + 2 * stride, t1, enn, lennn);
      tile_b_val<WT>(a, t, s_d);
    }
    t += stride;
    if (t >= t1) break;
    rp = rpn;
    x = xn;
    e0 = en;
    len = lenn;
    en = enn;
    lenn = lennn;
  }
}

// Workgroup sum of a group's 3m words to the poller wave, the device-wide
// reduction on the group's slot class (m - 1), and the Newton /
// trust-region step of each column (Eq. 4 with the prior; lane c for column
// j0 + c) on the LDS copies of beta and trust.  Writes the steps to s_d and
// bci = {reduction completed, non-finite value, some step nonzero}.  Called
// by all threads; one barrier inside block_sum_to and one at the end.
template <int M>
__device__ __forceinline__ void val_group_step(const KArgs& a, const AccV<kMaxGroup>& acc, int j0, uint32_t seq,
                                               double* sbeta, double* strust, double (*redg)[kValWords * kMaxGroup],
                                               double* s_d, int* bci, int& n_zero) {
  constexpr int NV = kValWords * M;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double loc[NV], part[NV];
#pragma unroll
  for (int c = 0; c < M; ++c) {
    loc[kValWords * c] = acc.gp[c];
    loc[kValWords * c + 1] = acc.gn[c];
    loc[kValWords * c + 2] = acc.h[c];
  }
  block_sum_to<NV, kValWords * kMaxGroup>(loc, part, redg, kPoller);
  if (wave == kPoller) {
    double tot[NV];
#pragma unroll
    for (int i = 0; i < NV; ++i) tot[i] = 0.0;
    const bool okr = allreduce2_wave<NV>(a.slots + (M - 1) * kSlots1PerClass, a.slots2 + (M - 1) * kSlots2PerClass,
                                         seq, a.G, a.ctrl, part, tot, (int)blockIdx.x - a.b0);
    double Gp = 0.0, Gn = 0.0, Hc = 0.0;
#pragma unroll
    for (int c = 0; c < M; ++c)
      if (lane == c) {
        Gp = tot[kValWords * c];
        Gn = tot[kValWords * c + 1];
        Hc = tot[kValWords * c + 2];
      }
    double d = 0.0;
    int bad = 0;
    if (a.prior_kind == SCCS_PRIOR_GROUPED) {
      grouped_steps(a, j0, M, okr, a.ytx[j0 + (lane < M ? lane : 0)] - (Gp - Gn), -Hc, sbeta, strust,
                    lds_dyn_ssum(a, sbeta), d, bad);
    } else if (lane < M && okr) {
      const int j = j0 + lane;
      const double gg = a.ytx[j] - (Gp - Gn), hh = -Hc;
      bad = !(isfinite(gg) && isfinite(hh));
      if (!bad) {
        const double bj = sbeta[j], tr = strust[j];
        const double dv = prior_step(a.prior_kind, a.inv_var, a.lambda, bj, gg, hh);
        d = fmin(fmax(dv, -tr), tr);
        strust[j] = fmax(2.0 * fabs(d), 0.5 * tr);
        const double nb = bj + d;
        if (!isfinite(nb)) { bad = 1; d = 0.0; }
        else sbeta[j] = nb;
      }
    }
    if (lane < kMaxGroup) s_d[lane] = d;
    const uint64_t moved = __ballot(lane < M && d != 0.0);
    const bool any_bad = __ballot(bad != 0) != 0ull;
    if (lane == 0) {
      bci[0] = okr ? 1 : 0;
      bci[1] = any_bad ? 1 : 0;
      bci[2] = moved != 0ull ? 1 : 0;
      n_zero += okr ? M - __popcll(moved) : 0;
    }
  }
  __syncthreads();
}

// The sweep for problems with covariate values: same contract as k_ccd
// (n sweeps or a stopping rule, objective on request, beta/trust and the
// control block written back by workgroup 0).
template <typename WT>
__global__ void __launch_bounds__(kBlock) k_ccd_val(KArgs a) {
  extern __shared__ double lds_dyn[];
  double* sbeta = lds_dyn;              // [J]
  double* strust = lds_dyn + a.J;       // [J]
  double* sprev = lds_dyn + 2 * a.J;    // [J] beta at the start of the sweep
  __shared__ double red[kWaves][4];
  __shared__ double redg[kWaves][kValWords * kMaxGroup];
  __shared__ double bc[8];
  __shared__ int bci[4];
  __shared__ double s_d[kMaxGroup];

  const int tid = threadIdx.x, b = (int)blockIdx.x - a.b0, wave = tid >> 6;
  for (int j = tid; j < a.J; j += kBlock) {
    sbeta[j] = a.beta[j];
    strust[j] = a.trust[j];
  }
  uint32_t gseq[kSlotClasses];
#pragma unroll
  for (int c = 0; c < kSlotClasses; ++c) gseq[c] = a.ctrl->gseq[c];
  uint32_t oseq = a.ctrl->oseq;
  int since_refresh = a.ctrl->since_refresh;
  if (a.prior_kind == SCCS_PRIOR_GROUPED) {
    __syncthreads();
    class_sums(a, sbeta, lds_dyn_ssum(a, sbeta));
  }
  __syncthreads();

  const int p0 = a.pb[b], p1 = a.pb[b + 1];
  const int NG = a.n_groups;
  bool ok = true;
  int status = SCCS_OK;
  double lp_prev = 0.0;
  if (a.criterion == SCCS_CRIT_REL_LOGPOST) {
    double o3[3];
    ok = objective(a, sbeta, sprev, p0, p1, oseq++, o3, red, bc, bci);
    lp_prev = o3[1];
  }
  int sweep = 0, converged = 0, n_zero = 0;
  double L = 0.0, P = 0.0;
  while (ok && sweep < a.n_sweeps) {
    if (a.criterion == SCCS_CRIT_ABS_DXBETA) {
      for (int j = tid; j < a.J; j += kBlock) sprev[j] = sbeta[j];
      __syncthreads();
    }
    for (int g = 0; g < NG; ++g) {
      const int j0 = ld_idx(a.gcol + g), m = ld_idx(a.gcol + g + 1) - j0;
      const int t0 = ld_idx(a.own + (size_t)g * (a.G + 1) + b), t1 = ld_idx(a.own + (size_t)g * (a.G + 1) + b + 1);
      AccV<kMaxGroup> acc;
      acc.zero();
      tiles_a_val<WT, kMaxGroup>(a, t0 + wave, t1, kWaves, acc);
      const int cls = m - 1;
      uint32_t sq = gseq[0];
#pragma unroll
      for (int c = 1; c < kMaxGroup; ++c)
        if (cls == c) sq = gseq[c];
      switch (m) {   // one width per slot class, fixed at compile time
        case 1: val_group_step<1>(a, acc, j0, sq, sbeta, strust, redg, s_d, bci, n_zero); break;
#if SCCS_MAX_GROUP >= 2
        case 2: val_group_step<2>(a, acc, j0, sq, sbeta, strust, redg, s_d, bci, n_zero); break;
#endif
#if SCCS_MAX_GROUP >= 3
        case 3: val_group_step<3>(a, acc, j0, sq, sbeta, strust, redg, s_d, bci, n_zero); break;
#endif
        default: val_group_step<kMaxGroup>(a, acc, j0, sq, sbeta, strust, redg, s_d, bci, n_zero); break;
      }
#pragma unroll
      for (int c = 0; c < kMaxGroup; ++c)
        if (cls == c) ++gseq[c];
      if (!bci[0]) { ok = false; break; }
      if (bci[1]) { status = SCCS_ERR_NUMERIC; ok = false; break; }
      if (bci[2])
        tiles_b_val<WT>(a, t0 + wave, t1, kWaves, s_d);
      // the next group may share patients with this one
      __syncthreads();
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
      if (!objective(a, sbeta, sprev, p0, p1, oseq++, o3, red, bc, bci)) { ok = false; break; }
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
    if (tid == kPoller * 64) {
      a.ctrl->rejects = 0;
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

// g_j and h_j of one column (column diag_c of group diag_g) at the current
// beta for problems with covariate values: the group's phase A, and one
// reduction on slot class 0 with kValWords words (the width every
// reduction of class 0 has on such a handle).
template <typename WT>
__global__ void __launch_bounds__(kBlock) k_diag_val(KArgs a) {
  __shared__ double red[kWaves][4];
  __shared__ double bc[8];
  __shared__ int bci[4];
  const int tid = threadIdx.x, b = (int)blockIdx.x - a.b0;
  uint32_t seq = a.ctrl->gseq[0];
  AccV<kMaxGroup> acc;
  acc.zero();
  const int t0 = a.own[(size_t)a.diag_g * (a.G + 1) + b], t1 = a.own[(size_t)a.diag_g * (a.G + 1) + b + 1];
  tiles_a_val<WT, kMaxGroup>(a, t0 + (tid >> 6), t1, kWaves, acc);
  double loc[kValWords] = {0.0, 0.0, 0.0}, part[kValWords];
#pragma unroll
  for (int i = 0; i < kMaxGroup; ++i)
    if (i == a.diag_c) {
      loc[0] = acc.gp[i];
      loc[1] = acc.gn[i];
      loc[2] = acc.h[i];
    }
  block_sum<kValWords>(loc, part, red);
  double tot[kValWords];
  const bool ok = allreduce_nonneg<kValWords>(a.slots, a.slots2, seq++, a.G, a.ctrl, part, tot, bc, bci, b);
  if (b == 0 && tid == 0 && ok) {
    a.ctrl->g = a.ytx[a.diag_j] - (tot[0] - tot[1]);
    a.ctrl->h = -tot[2];
  }
  __syncthreads();
  if (b == 0 && tid == 0) a.ctrl->gseq[0] = seq;
}

template __global__ void k_ccd_val<double>(KArgs);
template __global__ void k_ccd_val<float>(KArgs);
template __global__ void k_diag_val<double>(KArgs);
template __global__ void k_diag_val<float>(KArgs);

}  // namespace sccs
