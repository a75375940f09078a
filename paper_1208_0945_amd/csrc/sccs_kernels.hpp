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
// doubles per workgroup.
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

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
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

// Device-wide sum of NV non-negative doubles per workgroup.  Called by all
// threads of every workgroup with the workgroup's partials valid in thread 0.
// Returns false (in all threads) if the wait timed out or another workgroup
// aborted.  out[] receives the sums (all threads).
template <int NV>
__device__ bool allreduce_nonneg(uint64_t* slots, uint32_t seq, int G, Ctrl* ctrl,
                                 const double* part, double* out, double* lds_out, int* lds_ok) {
  const int tid = threadIdx.x, lane = tid & 63;
  const uint32_t par = seq & 1u, tag = (seq >> 1) & 1u;
  uint64_t* mine = slots + ((size_t)par * G + blockIdx.x) * NV;
  if (tid == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v) store_agent(mine + v, tag_encode(part[v], tag));
  }
  if (tid < 64) {
    const uint64_t* base = slots + (size_t)par * G * NV;
    double val[kMaxSlotsPerLane][NV];
    uint32_t need = 0;
    for (int q = 0; q < kMaxSlotsPerLane; ++q)
      if (lane + 64 * q < G) need |= 1u << q;
    long long spins = 0;
    bool ok = true;
    while (true) {
#pragma unroll
      for (int q = 0; q < kMaxSlotsPerLane; ++q) {
        if (need & (1u << q)) {
          const uint64_t* s = base + (size_t)(lane + 64 * q) * NV;
          bool ready = true;
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            uint64_t x = load_agent(s + v);
            ready = ready && ((uint32_t)(x >> 63) == tag);
            val[q][v] = tag_decode(x);
          }
          if (ready) need &= ~(1u << q);
        }
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
      __builtin_amdgcn_s_sleep(1);
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < kMaxSlotsPerLane; ++q)
        if (lane + 64 * q < G) s += val[q][v];
      s = wave_sum(s);
      if (lane == 0) lds_out[v] = s;
    }
    if (lane == 0) *lds_ok = ok ? 1 : 0;
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
template <int NV>
__device__ void block_sum(const double* v_in, double* out, double (*red)[4]) {
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

// ------------------------------------------------------------ Newton step

// Eq. 4 with the prior; Laplace rules at the kink after Genkin et al.
__device__ double prior_step(int kind, double var, double lambda, double b, double g, double h) {
  if (kind == SCCS_PRIOR_NORMAL) return -(g - b / var) / (h - 1.0 / var);
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
  __device__ static float weight(int32_t l, double eta) {
    double n = rint(eta * 1.4426950408889634);
    double r = fma(-n, 6.93147180369123816490e-01, eta);
    r = fma(-n, 1.90821492927058770002e-10, r);
    float e = expf((float)r);
    return ldexpf((float)l * e, (int)n);
  }
};

// ------------------------------------------------------------ segmented sums

// Sum of v over the lanes of this lane's patient segment, valid in the
// segment's head lane.  pid is sorted ascending over the active lanes
// [0, len); inactive lanes hold v = 0.
__device__ __forceinline__ double seg_sum(double v, uint32_t pid, int lane, int len, bool& head) {
  uint32_t pid_next = __shfl_down(pid, 1, 64);
  uint32_t pid_prev = __shfl_up(pid, 1, 64);
  bool act = lane < len;
  bool tail = act && (lane == len - 1 || pid_next != pid);
  head = act && (lane == 0 || pid_prev != pid);
  uint64_t tails = __ballot(tail);
  int seg_end = act ? lane + (int)__builtin_ctzll(tails >> lane) : lane;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    double o = __shfl_down(v, d, 64);
    if (lane + d <= seg_end) v += o;
  }
  return v;
}

// Phase A over the tiles of column j owned by this workgroup; per-lane
// accumulators of G and H.
template <typename WT>
__device__ void phase_a(const KArgs& a, int j, double& Gl, double& Hl) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const size_t base = (size_t)j * (a.G + 1) + blockIdx.x;
  const int t0 = a.own[base], t1 = a.own[base + 1];
  const WT* __restrict__ w = (const WT*)a.w;
  for (int t = t0 + wave; t < t1; t += kWaves) {
    const int e0 = a.tile_start[t], e1 = a.tile_start[t + 1];
    const int len = e1 - e0;
    if (len <= 64) {
      bool act = lane < len;
      uint2 rp = act ? a.rp[e0 + lane] : make_uint2(0u, 0xffffffffu);
      double wv = act ? (double)w[rp.x] : 0.0;
      bool head;
      double num = seg_sum(wv, rp.y, lane, len, head);
      if (head) {
        double2 pv = a.pat[rp.y];
        double r = num / pv.x;
        double tg = pv.y * r;
        Gl += tg;
        Hl += tg * fmax(1.0 - r, 0.0);
      }
    } else {
      double s = 0.0;
      for (int e = e0 + lane; e < e1; e += 64) s += (double)w[a.rp[e].x];
      s = wave_sum(s);
      if (lane == 0) {
        double2 pv = a.pat[a.rp[e0].y];
        double r = s / pv.x;
        double tg = pv.y * r;
        Gl += tg;
        Hl += tg * fmax(1.0 - r, 0.0);
      }
    }
  }
}

// Phase B: w_k <- w_k e^d on the column's rows, den_i updated per segment.
// ed = e^d and em1 = e^d - 1 are computed once per coordinate by the caller.
template <typename WT>
__device__ void phase_b(const KArgs& a, int j, double ed, double em1) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const size_t base = (size_t)j * (a.G + 1) + blockIdx.x;
  const int t0 = a.own[base], t1 = a.own[base + 1];
  WT* __restrict__ w = (WT*)a.w;
  const WT edw = (WT)ed;
  for (int t = t0 + wave; t < t1; t += kWaves) {
    const int e0 = a.tile_start[t], e1 = a.tile_start[t + 1];
    const int len = e1 - e0;
    if (len <= 64) {
      bool act = lane < len;
      uint2 rp = act ? a.rp[e0 + lane] : make_uint2(0u, 0xffffffffu);
      WT wo = act ? w[rp.x] : (WT)0;
      WT wn = wo * edw;
      if (act) w[rp.x] = wn;
      bool head;
      double s;
      if (sizeof(WT) == 8) {
        s = seg_sum((double)wo, rp.y, lane, len, head);
        if (head) a.pat[rp.y].x += s * em1;
      } else {
        // mixed: track the exact change of the stored FP32 weights in FP64
        s = seg_sum((double)wn - (double)wo, rp.y, lane, len, head);
        if (head) a.pat[rp.y].x += s;
      }
    } else {
      double s = 0.0;
      for (int e = e0 + lane; e < e1; e += 64) {
        uint32_t row = a.rp[e].x;
        WT wo = w[row];
        WT wn = wo * edw;
        w[row] = wn;
        s += (sizeof(WT) == 8) ? (double)wo : ((double)wn - (double)wo);
      }
      s = wave_sum(s);
      if (lane == 0) {
        double2* pp = &a.pat[a.rp[e0].y];
        pp->x += (sizeof(WT) == 8) ? s * em1 : s;
      }
    }
  }
}

// Exact recomputation of w = L x exp(X beta) and den = M w for patients
// [p0, p1) (the dense evaluation of Listing 1's role, plus Step 3).
template <typename WT>
__device__ __forceinline__ void refresh_range(const KArgs& a, const double* beta, int p0, int p1, int tid, int nthreads) {
  WT* __restrict__ w = (WT*)a.w;
  for (int i = p0 + tid; i < p1; i += nthreads) {
    double den = 0.0;
    for (int k = a.pptr[i]; k < a.pptr[i + 1]; ++k) {
      double eta = 0.0;
      for (int c = a.era_ptr[k]; c < a.era_ptr[k + 1]; ++c) eta += beta[a.era_col[c]];
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
        de += sbeta[jj] - sprev[jj];
      }
      loc[2] += fabs(de);
    }
  }
  // beta'Y'X and the log prior, summed in the same order in every workgroup
  double bl[2] = {0.0, 0.0};
  for (int j = tid; j < a.J; j += kBlock) {
    double bj = sbeta[j];
    bl[0] += bj * a.ytx[j];
    if (a.prior_kind == SCCS_PRIOR_NORMAL) bl[1] -= bj * bj / (2.0 * a.var);
    else if (a.prior_kind == SCCS_PRIOR_LAPLACE) bl[1] -= a.lambda * fabs(bj);
  }
  double part[4];
  block_sum<4>(loc, part, red);
  double bsum[2];
  block_sum<2>(bl, bsum, red);
  if (tid == 0) { bc[4] = bsum[0]; bc[5] = bsum[1]; }
  double tot[4];
  bool ok = allreduce_nonneg<4>(a.oslots, oseq, a.G, a.ctrl, part, tot, bc, bci);
  out3[0] = bc[4] - (tot[0] - tot[1]);  // loglik
  out3[1] = out3[0] + bc[5];            // logpost
  out3[2] = tot[2];                     // sum |delta eta|
  __syncthreads();
  return ok;
}

// ------------------------------------------------------------ persistent kernel

template <typename WT>
__global__ void __launch_bounds__(kBlock) k_ccd(KArgs a) {
  extern __shared__ double lds_dyn[];
  double* sbeta = lds_dyn;              // [J]
  double* strust = lds_dyn + a.J;       // [J]
  double* sprev = lds_dyn + 2 * a.J;    // [J] beta at the start of the sweep
  __shared__ double red[kWaves][4];
  __shared__ double bc[8];
  __shared__ int bci[4];

  const int tid = threadIdx.x, b = blockIdx.x;
  for (int j = tid; j < a.J; j += kBlock) {
    sbeta[j] = a.beta[j];
    strust[j] = a.trust[j];
  }
  uint32_t seq = a.ctrl->seq;     // identical in all workgroups (written by the previous launch)
  uint32_t oseq = a.ctrl->oseq;
  int since_refresh = a.ctrl->since_refresh;
  __syncthreads();

  const int p0 = a.pb[b], p1 = a.pb[b + 1];
  bool ok = true;
  int status = SCCS_OK;
  double lp_prev = 0.0;
  if (a.criterion == SCCS_CRIT_REL_LOGPOST) {
    double o3[3];
    ok = objective(a, sbeta, sprev, p0, p1, oseq++, o3, red, bc, bci);
    lp_prev = o3[1];
  }
  int sweep = 0, converged = 0;
  double L = 0.0, P = 0.0;
  while (ok && sweep < a.n_sweeps) {
    if (a.criterion == SCCS_CRIT_ABS_DXBETA) {
      for (int j = tid; j < a.J; j += kBlock) sprev[j] = sbeta[j];
      __syncthreads();
    }
    for (int j = 0; j < a.J; ++j) {
      double ytxj = 0.0;
      if (tid == 0) ytxj = a.ytx[j];
      double Gl = 0.0, Hl = 0.0;
      phase_a<WT>(a, j, Gl, Hl);
      double loc[2] = {Gl, Hl}, part[2], tot[2];
      block_sum<2>(loc, part, red);
      if (!allreduce_nonneg<2>(a.slots, seq++, a.G, a.ctrl, part, tot, bc, bci)) { ok = false; break; }
      if (tid == 0) {
        double g = ytxj - tot[0], h = -tot[1];
        double d = 0.0;
        int bad = !(isfinite(g) && isfinite(h));
        if (!bad) {
          double bj = sbeta[j], tr = strust[j];
          double dv = prior_step(a.prior_kind, a.var, a.lambda, bj, g, h);
          d = fmin(fmax(dv, -tr), tr);
          strust[j] = fmax(2.0 * fabs(d), 0.5 * tr);
          double nb = bj + d;
          if (!isfinite(nb)) { bad = 1; d = 0.0; }
          else sbeta[j] = nb;
        }
        bc[0] = d;
        bc[1] = exp(d);
        bc[2] = expm1(d);
        bci[1] = bad;
      }
      __syncthreads();
      const double d = bc[0], ed = bc[1], em1 = bc[2];
      if (bci[1]) { status = SCCS_ERR_NUMERIC; ok = false; break; }
      if (d != 0.0) phase_b<WT>(a, j, ed, em1);
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
    if (tid == 0) {
      a.ctrl->sweeps = sweep;
      a.ctrl->converged = converged;
      a.ctrl->loglik = L;
      a.ctrl->logpost = P;
      a.ctrl->seq = seq;
      a.ctrl->oseq = oseq;
      a.ctrl->since_refresh = since_refresh;
      if (status != SCCS_OK) a.ctrl->status = status;
    }
  }
}

// Diagnostics: g_j, h_j of column diag_j at the current beta (mode 1), or the
// objective (mode 2).  Same ownership and reductions as the sweep kernel.
template <typename WT>
__global__ void __launch_bounds__(kBlock) k_diag(KArgs a) {
  extern __shared__ double lds_dyn[];
  double* sbeta = lds_dyn;
  __shared__ double red[kWaves][4];
  __shared__ double bc[8];
  __shared__ int bci[4];
  const int tid = threadIdx.x, b = blockIdx.x;
  for (int j = tid; j < a.J; j += kBlock) sbeta[j] = a.beta[j];
  uint32_t seq = a.ctrl->seq, oseq = a.ctrl->oseq;
  __syncthreads();
  const int p0 = a.pb[b], p1 = a.pb[b + 1];
  if (a.mode == kModeObjective) {
    double o3[3];
    bool ok = objective(a, sbeta, sbeta, p0, p1, oseq++, o3, red, bc, bci);
    if (b == 0 && tid == 0 && ok) { a.ctrl->loglik = o3[0]; a.ctrl->logpost = o3[1]; }
  } else {
    const int j = a.diag_j;
    double Gl = 0.0, Hl = 0.0;
    phase_a<WT>(a, j, Gl, Hl);
    double loc[2] = {Gl, Hl}, part[2], tot[2];
    block_sum<2>(loc, part, red);
    bool ok = allreduce_nonneg<2>(a.slots, seq++, a.G, a.ctrl, part, tot, bc, bci);
    if (b == 0 && tid == 0 && ok) { a.ctrl->g = a.ytx[j] - tot[0]; a.ctrl->h = -tot[1]; }
  }
  __syncthreads();
  if (b == 0 && tid == 0) { a.ctrl->seq = seq; a.ctrl->oseq = oseq; }
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

// Y'X_j with patient weights: one workgroup per column, fixed-order sum.
__global__ void __launch_bounds__(256) k_setup_ytx(const int64_t* col_ptr, const uint2* rp, const int32_t* count,
                                                   const int32_t* weight, double* ytx, int J) {
  __shared__ double red[4];
  for (int j = blockIdx.x; j < J; j += gridDim.x) {
    double s = 0.0;
    for (long long e = col_ptr[j] + threadIdx.x; e < col_ptr[j + 1]; e += blockDim.x) {
      uint2 q = rp[e];
      double om = weight ? (double)weight[q.y] : 1.0;
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

template __global__ void k_ccd<double>(KArgs);
template __global__ void k_ccd<float>(KArgs);
template __global__ void k_diag<double>(KArgs);
template __global__ void k_diag<float>(KArgs);
template __global__ void k_refresh<double>(KArgs);
template __global__ void k_refresh<float>(KArgs);

}  // namespace sccs
