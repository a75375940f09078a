// Device-side building blocks of libsccs for gfx950 (wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace sccs {

constexpr int kBlock = 1024;             // threads per persistent workgroup
constexpr int kWaves = kBlock / 64;      // wavefronts per workgroup
constexpr int kMaxSlotsPerLane = 4;      // => at most 256 workgroups
constexpr int kMaxJ = 6144;              // beta, trust, beta_prev live in LDS
constexpr uint64_t kSign = 0x8000000000000000ull;
constexpr long long kSpinLimit = 1ll << 22;  // bounded waits (about a second), then abort

// Control block shared by all workgroups of a launch (device memory).
struct Ctrl {
  uint32_t seq;        // coordinate-reduction sequence number (persists across launches)
  uint32_t oseq;       // objective-reduction sequence number
  int32_t abort;       // set by a workgroup that timed out
  int32_t status;      // SCCS_OK or an error code
  int32_t sweeps;      // sweeps run by the last launch
  int32_t converged;
  int32_t since_refresh;
  int32_t pad;
  double loglik, logpost;
  double g, h;         // diagnostic output
};

struct KArgs {
  const uint2* rp;            // [nnz] (row, patient)
  const int32_t* tile_start;  // [T+1]
  const int32_t* own;         // [J*(G+1)]
  const int32_t* pb;          // [G+1]
  const int32_t* pptr;        // [N+1]
  const int32_t* era_ptr;     // [K+1]
  const int32_t* era_col;     // [nnz]
  const int32_t* offset;      // [K]
  void* w;                    // [K] double (FP64) or float (mixed)
  double2* pat;               // [N] (den_i, omega_i n_i)
  const double* ytx;          // [J]
  double* beta;               // [J]
  double* trust;              // [J]
  uint64_t* slots;            // [2][G][2] coordinate reduction
  uint64_t* oslots;           // [2][G][4] objective reduction
  Ctrl* ctrl;
  int32_t N, J, G;
  int32_t prior_kind;
  double var, lambda;
  int32_t n_sweeps;
  int32_t criterion;
  double tol;
  int32_t refresh_period;
  int32_t want_objective;     // evaluate P after the last sweep
  int32_t mode;               // 0 sweep, 1 grad/hess of diag_j, 2 objective only
  int32_t diag_j;
};

enum { kModeSweep = 0, kModeGradHess = 1, kModeObjective = 2 };

}  // namespace sccs
