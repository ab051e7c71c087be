// Build generations of a cell list.  Every build advances a 32-bit counter on
// the device; a recorded neighbour list or accepted-pair mask stores the
// generation it was recorded for and is used only while they match.  Two
// values are reserved and never produced by a build: 0 (a mask record that
// holds no usable record: none yet, or an overflowed row) and 0xFFFFFFFF (a
// neighbour list that was never recorded).  The counter therefore steps from
// 0xFFFFFFFE back to 1, so a stale record can only match again after 2^32 - 2
// builds, and a reserved value never matches.  Plain constexpr C++: the
// kernels and a host-compiled test use the same rule.
#pragma once

#include <stdint.h>

namespace aboria {

constexpr uint32_t kGenNone = 0u;           // mask status: no record
constexpr uint32_t kGenNeverListed = 0xFFFFFFFFu;  // list generation before the first recording

constexpr uint32_t next_generation(uint32_t g) { return g >= kGenNeverListed - 1u ? 1u : g + 1u; }

}  // namespace aboria
