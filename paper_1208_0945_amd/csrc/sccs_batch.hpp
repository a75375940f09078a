// Batched form: F independent fits (different outcomes, or cross-validation
// folds) advanced in lockstep by one cooperative persistent launch.
//
// All fits share the coordinate order j = 0..J-1 and the workgroup count G;
// workgroup b owns patient range b of every fit's problem.  Per coordinate,
// every workgroup computes its partial (G_f, H_f) for each active fit, ONE
// device-wide reduction carries all 2F partials (so its latency is paid once
// for all fits), then each fit takes its own Newton / trust-region step
// (Eq. 4) and its own sparse update.  Each fit walks a chain of priors in
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
constexpr int kBatchSlotWords = 2 * kMaxFits;   // 2F words per workgroup slot

struct LinkResult {
  int32_t sweeps;
  int32_t converged;
  double loglik;
  double logpost;
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
};

struct BatchArgs {
  const BatchFit* fits;
  uint64_t* s1;              // [2][256][kBatchSlotWords]
  uint64_t* s2;              // [2][kReplicas][8][kBatchSlotWords]
  Ctrl* ctrl;
  int32_t F, G, J;
  int32_t max_sweeps;        // per link
  int32_t criterion;         // FIXED or REL_LOGPOST
  int32_t refresh_period;
  double tol;
};

// Poll n tagged words (word e at src(e)) spread over the workgroup's
// threads, every thread keeping all of its loads in flight at once; the
// decoded values go to stage[dst(e)].  Returns false on timeout/abort
// (also recorded in *flag).
template <typename Src, typename Dst>
__device__ __forceinline__ void poll_spread(int n, uint32_t tag, Src src, Dst dst, double* stage, Ctrl* ctrl,
                                            int* flag) {
  constexpr int kPer = (32 * kBatchSlotWords + kBlock - 1) / kBlock;
  uint32_t need = 0;
#pragma unroll
  for (int q = 0; q < kPer; ++q)
    if ((int)threadIdx.x + q * kBlock < n) need |= 1u << q;
  long long spins = 0;
  while (need) {
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      if (need & (1u << q)) {
        const int e = threadIdx.x + q * kBlock;
        uint64_t x = load_agent(src(e));
        if ((uint32_t)(x >> 63) == tag) {
          stage[dst(e)] = tag_decode(x);
          need &= ~(1u << q);
        }
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
    __builtin_amdgcn_s_sleep(2);
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
    poll_spread(
        members * nv, tag,
        [&](int e) { return L1 + (size_t)(b + (e / nv) * ng) * kBatchSlotWords + (e % nv); },
        [&](int e) { return (e / nv) * kBatchSlotWords + (e % nv); }, stage, ctrl, flag);
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
    poll_spread(
        ng * nv, tag, [&](int e) { return L2 + ((size_t)r * kGroups + e / nv) * kBatchSlotWords + (e % nv); },
        [&](int e) { return (e / nv) * kBatchSlotWords + (e % nv); }, stage, ctrl, flag);
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

// Wave -> (fit, slice) assignment.  With F >= kWaves fits each wave takes
// fits w, w + kWaves, ... whole; with fewer fits, P = kWaves / F waves share
// a fit and take every P-th of its tiles.
struct WaveMap {
  int P;
  __device__ WaveMap(int F) : P(F >= kWaves ? 1 : kWaves / F) {}
  __device__ int first_fit(int w, int F) const { return P == 1 ? w : (w < F * P ? w / P : F); }
  __device__ int next_fit(int f) const { return P == 1 ? f + kWaves : 1 << 30; }
  __device__ int slice(int w) const { return P == 1 ? 0 : w % P; }
};

template <typename WT>
__global__ void __launch_bounds__(kBlock) k_batch(BatchArgs A) {
  __shared__ double stage[32 * kBatchSlotWords];
  __shared__ double pp[kMaxFits][kWaves][2];      // per (fit, slice) partials
  __shared__ double part[kBatchSlotWords], tot[kBatchSlotWords];
  __shared__ double dd[kMaxFits][3];              // d, e^d, e^d - 1
  __shared__ double lp_prev[kMaxFits], s_var[kMaxFits], s_lam[kMaxFits], s_ivar[kMaxFits];
  __shared__ int s_link[kMaxFits], s_sw[kMaxFits], s_kind[kMaxFits], s_done[kMaxFits];
  __shared__ int flag, bad_any, n_active, since_refresh;
  __shared__ double red[kWaves][4];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, b = blockIdx.x;
  const int F = A.F, G = A.G, J = A.J;
  const WaveMap wm(F);
  uint32_t seq = A.ctrl->seq;

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
  if (tid == 0) { since_refresh = 0; bad_any = 0; }
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
    bool okr = batch_allreduce(A.s1, A.s2, seq++, G, 2 * F, A.ctrl, part, tot, stage, &flag);
    if (tid < F) {
      double L = Lout[tid] - (tot[2 * tid] - tot[2 * tid + 1]);
      Lout[tid] = L;
      Pout[tid] = L + Pout[tid];
    }
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
    for (int j = 0; j < J && ok; ++j) {
      // phase A for every (fit, slice) of this wave
      for (int f = wm.first_fit(wave, F); f < F; f = wm.next_fit(f)) {
        double Gl = 0.0, Hl = 0.0;
        if (!s_done[f]) {
          const KArgs& k = A.fits[f].k;
          const size_t base = (size_t)j * (G + 1) + b;
          const int t0 = k.own[base], t1 = k.own[base + 1];
          for (int t = t0 + wm.slice(wave); t < t1; t += wm.P) tile_a<WT>(k, t, Gl, Hl);
        }
        Gl = wave_sum(Gl);
        Hl = wave_sum(Hl);
        if (lane == 0) {
          pp[f][wm.slice(wave)][0] = Gl;
          pp[f][wm.slice(wave)][1] = Hl;
        }
      }
      __syncthreads();
      if (tid < F) {
        double g = 0.0, h = 0.0;
        for (int q = 0; q < wm.P; ++q) { g += pp[tid][q][0]; h += pp[tid][q][1]; }
        part[2 * tid] = g;
        part[2 * tid + 1] = h;
      }
      __syncthreads();
      if (!batch_allreduce(A.s1, A.s2, seq++, G, 2 * F, A.ctrl, part, tot, stage, &flag)) { ok = false; break; }
      // one Newton / trust-region step per fit (lanes of wave 0)
      if (tid < F) {
        const int f = tid;
        double d = 0.0;
        if (!s_done[f]) {
          const BatchFit& bf = A.fits[f];
          double2* bt = bf.bt + (size_t)b * J + j;
          double2 v = *bt;
          double g = bf.k.ytx[j] - tot[2 * f], h = -tot[2 * f + 1];
          if (isfinite(g) && isfinite(h)) {
            double dv = prior_step(s_kind[f], s_ivar[f], s_lam[f], v.x, g, h);
            d = fmin(fmax(dv, -v.y), v.y);
            double nb = v.x + d;
            if (isfinite(nb)) {
              *bt = make_double2(nb, fmax(2.0 * fabs(d), 0.5 * v.y));
            } else {
              d = 0.0;
              atomicOr(&bad_any, 1);
            }
          } else {
            atomicOr(&bad_any, 1);
          }
        }
        const double em1 = expm1(d);
        dd[f][0] = d;
        dd[f][1] = 1.0 + em1;
        dd[f][2] = em1;
      }
      __syncthreads();
      if (bad_any) { status = SCCS_ERR_NUMERIC; ok = false; break; }
      for (int f = wm.first_fit(wave, F); f < F; f = wm.next_fit(f)) {
        if (s_done[f] || dd[f][0] == 0.0) continue;
        const KArgs& k = A.fits[f].k;
        const size_t base = (size_t)j * (G + 1) + b;
        const int t0 = k.own[base], t1 = k.own[base + 1];
        for (int t = t0 + wm.slice(wave); t < t1; t += wm.P) tile_b<WT>(k, t, dd[f][1], dd[f][2]);
      }
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
    __shared__ int s_adv[kMaxFits];
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
    A.ctrl->seq = seq;
    A.ctrl->sweeps = total_sweeps;
    if (status != SCCS_OK) A.ctrl->status = status;
  }
}

}  // namespace sccs
