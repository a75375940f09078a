// Device-side building blocks of libsccs for gfx950 (wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "sccs_limits.hpp"

namespace sccs {

constexpr int kBlock = 512;              // threads per persistent workgroup
constexpr int kWaves = kBlock / 64;      // wavefronts per workgroup
constexpr int kMaxWorkgroups = 256;       // two-level reduction: <= 32 members per group
constexpr int kGroups = 8;               // reduction groups (one per XCD under round-robin placement)
static_assert(kMaxWorkgroups <= 32 * kGroups && kGroups <= 8, "level-1 members in lanes 0..31, group totals in lanes 0..7");
constexpr int kPoller = kWaves - 1;      // wave that runs the device-wide reduction
constexpr int kSlotWords = 16;           // one 128-byte line per reduction slot
#ifndef SCCS_REPLICAS
#define SCCS_REPLICAS 8
#endif
constexpr int kReplicas = SCCS_REPLICAS;  // copies of the group totals
static_assert(kReplicas >= 1 && kReplicas <= 64, "one leader lane per copy");
constexpr int kMaxJ = 6144;              // beta, trust, beta_prev live in LDS
static_assert(kMaxJ < kDescMaxCols, "every column index fits in a pass descriptor");
constexpr uint64_t kSign = 0x8000000000000000ull;
constexpr long long kSpinLimit = 1ll << 22;  // bounded waits (about a second), then abort
#ifndef SCCS_POLL_SLEEP
#define SCCS_POLL_SLEEP 0
#endif
// s_sleep between two polls of a reduction slot (units of 64 clocks); a
// chain of reductions measured fastest with none.
constexpr int kPollSleep = SCCS_POLL_SLEEP;

// Coordinate reductions of a single fit use one slot array per width (class
// m - 1 for m <= kMaxGroup columns, 2m words; class kMaxGroup for merged
// passes of more columns, 2 * kPassCols words), each with its own sequence
// number, so that every reduction on a slot array writes and reads the same
// number of words.
constexpr int kSlotClasses = kMaxGroup + 1;
constexpr size_t kSlots1Words = (size_t)2 * kMaxWorkgroups * kSlotWords;  // one level-1 array, both parities
constexpr size_t kSlots1PerClass = kSlots1Words;
constexpr size_t kSlots2PerClass = (size_t)2 * kReplicas * kGroups * kSlotWords;

// Control block shared by all workgroups of a launch (device memory).
struct Ctrl {
  uint32_t seq;        // batched form: reduction sequence number (persists across launches)
  uint32_t oseq;       // objective-reduction sequence number
  int32_t abort;       // set by a workgroup that timed out
  int32_t status;      // SCCS_OK or an error code
  int32_t sweeps;      // sweeps run by the last launch
  int32_t converged;
  int32_t since_refresh;
  int32_t passes;      // reductions run by the last sccs_sweep_static launch
  double loglik, logpost;
  double g, h;         // diagnostic output
  uint32_t gseq[kSlotClasses];  // single fit: sequence number of each reduction class
  int32_t rejects;     // single fit, last launch: merged passes whose later groups were visited again
  int32_t zero_steps;  //   coordinate visits whose step was exactly zero
};

struct KArgs {
  const uint2* rp;            // [nnz] (row, patient)
  const int32_t* tile_start;  // [T+1]
  const int32_t* own;         // [n_groups*(G+1)]
  const int32_t* gcol;        // [n_groups+1] first column of each group
  const uint32_t* gdesc;      // [n_groups] pass descriptors (sccs_layout.hpp)
  uint32_t* moved;            // [mv_words] bit j: column j's last step was nonzero
  const int32_t* pb;          // [G+1]
  const int32_t* pptr;        // [N+1]
  const int32_t* era_ptr;     // [K+1]
  const int32_t* era_col;     // [nnz]
  const double* val;          // [nnz] covariate values in rp order, NULL for binary exposures
  const double* era_val;      // [nnz] covariate values in era_col order, NULL for binary exposures
  const int32_t* offset;      // [K]
  void* w;                    // [K] double (FP64) or float (mixed)
  double2* pat;               // [N] (den_i, omega_i n_i)
  const double* ytx;          // [J]
  double* beta;               // [J]
  double* trust;              // [J]
  uint64_t* slots;            // [kSlotClasses][2][256][16] coordinate reductions, level 1
  uint64_t* slots2;           // [kSlotClasses][2][8 replicas][8 groups][16] group totals
  uint64_t* oslots;           // objective reduction, same shapes
  uint64_t* oslots2;
  Ctrl* ctrl;
  int32_t N, J, G;
  int32_t n_groups;
  int32_t prior_kind;
  double var, inv_var, lambda;
  int32_t n_sweeps;
  int32_t criterion;
  double tol;
  int32_t refresh_period;
  int32_t want_objective;     // evaluate P after the last sweep
  int32_t mode;               // 0 sweep, 1 grad/hess of diag_j, 2 objective only
  int32_t diag_j;
  int32_t diag_g, diag_c;     // group of diag_j and its column within the group
  int32_t nbits;              // words of each per-workgroup patient bitmap (LDS)
  int32_t mv_words;           // 32-bit words of the moved-column bitmap (LDS copy of moved)
  int32_t merge;              // merge the next group into a pass when predicted independent
  // grouped Normal prior (prior_kind SCCS_PRIOR_GROUPED): class of each
  // column, kappa_c = class_var / (var + m_c class_var) per class, and the
  // offset (in doubles) of the per-class sums in the dynamic LDS area
  const int32_t* pclass;      // [J]
  const double* pkappa;       // [n_classes]
  int32_t n_classes;
  int32_t ssum_off;
  // one-pass form: wall-clock ticks at the moment each group's steps were
  // taken in the current sweep ([n_groups]) and at the sweep's start
  // ([n_groups]); written by workgroup 0 when stamp is set
  uint64_t* group_ticks;      // [n_groups + 1]
  int32_t stamp;
  // first workgroup of this fit in the launch: several single fits can share
  // one launch, fit f on workgroups [b0, b0 + G) (0 for a launch of one fit)
  int32_t b0;
};

enum { kModeSweep = 0, kModeGradHess = 1, kModeObjective = 2 };

}  // namespace sccs
