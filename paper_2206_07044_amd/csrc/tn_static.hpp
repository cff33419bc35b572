// Fixed device scratch of the allocation-free compression entry point (tn_static.hip).
#pragma once

#include <stddef.h>

#include <string>

namespace tn {

// Size of each device's scratch array: 32 MiB.  Holds one compression's descriptors, the Gram
// partials of both sides (at D = 64, 512-row splits: about 260000 rows per side), the core
// workspace, the projectors and the per-tile maxima.
constexpr size_t kStaticScratchBytes = (size_t)32 << 20;

// Look up the scratch address on `device` (which must be current); once per device.
std::string static_scratch_init(int device);
// The address found by static_scratch_init on `device`, or null before it ran.
void* static_scratch(int device);

}  // namespace tn
