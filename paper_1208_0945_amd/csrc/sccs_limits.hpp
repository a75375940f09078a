// Limits shared by the host layout builder and the device code of libsccs
// (plain C++, no HIP dependency).
#pragma once
#include <cstdint>

namespace sccs {

constexpr int kTile = 64;                // nonzeros per tile (one wavefront)
#ifndef SCCS_MAX_GROUP
#define SCCS_MAX_GROUP 4
#endif
constexpr int kMaxGroup = SCCS_MAX_GROUP;  // columns per group (the reduction carries 2 words per column)
constexpr int kGroupShift = 28;          // column-in-group bits above the patient index in rp.y
constexpr uint32_t kPidMask = (1u << kGroupShift) - 1;
static_assert(kMaxGroup >= 1 && kMaxGroup <= 4, "column-in-group index is 2 bits; descriptors hold 3-bit widths");
// Merged passes: up to kPassGroups consecutive groups and kPassCols columns
// share one reduction.  A group's descriptor marks which of the kLinkCols
// columns just before it share a patient with it (every column of a pass
// that precedes one of its groups lies in that window).
#ifndef SCCS_PASS_GROUPS
#define SCCS_PASS_GROUPS 3
#endif
#ifndef SCCS_PASS_COLS
#define SCCS_PASS_COLS 4
#endif
constexpr int kPassGroups = SCCS_PASS_GROUPS;
constexpr int kPassCols = SCCS_PASS_COLS;
static_assert(kPassGroups >= 2 && kPassGroups <= 4, "groups per merged pass");
constexpr int kLinkCols = kPassCols - 1;
static_assert(kPassCols >= kMaxGroup && kPassCols <= 8, "one 16-word reduction slot per pass");
constexpr int kDescColBits = 13;         // first column of a group in a pass descriptor
constexpr int32_t kDescMaxCols = 1 << kDescColBits;
constexpr int kDescWidthShift = kDescColBits;         // width: 3 bits
constexpr int kDescLinkShift = kDescColBits + 3;      // link mask: kLinkCols bits
static_assert(kDescLinkShift + kLinkCols <= 32, "pass descriptor is one 32-bit word");
// Default sweeps between exact recomputations of w and den in the mixed
// form: every sweep.  The FP32 multiplicative updates drift by about 2e-8
// (relative to max |beta|) per sweep on the mid and full workloads; a
// refresh every 10 sweeps keeps max-norm errors near 2e-7 but lets a
// coordinate near 1e-3 drift by a few parts in 1e4, so rarer refreshes are
// the caller's choice (refresh_period).
constexpr int kMixedRefresh = 1;

}  // namespace sccs
