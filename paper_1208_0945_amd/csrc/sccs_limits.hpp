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
static_assert(kMaxGroup >= 1 && kMaxGroup <= 4, "pass descriptors hold 3-bit widths and a 4-bit mask");
constexpr int kDescColBits = 13;         // first column of a group in a pass descriptor
constexpr int32_t kDescMaxCols = 1 << kDescColBits;

}  // namespace sccs
