// kur_noalloc.hpp -- the per-device fixed scratch of the entry points that allocate nothing
// (noalloc.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace kur {

// largest n the fixed scratch serves (3 FP64 partials per chunk of 256 rows)
constexpr int64_t kNoAllocMaxN = (int64_t)1 << 24;

// Look up the scratch's device address on `device`, which must be the current device; once per
// device, later calls return the first result.
hipError_t noalloc_scratch_init(int device);
// The device address found by noalloc_scratch_init (null if it failed or was not run).
void *noalloc_scratch(int device);
size_t noalloc_scratch_bytes();
// offset, in doubles, of the three totals after the partials
int64_t noalloc_totals_offset();

}  // namespace kur
