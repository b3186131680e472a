// Internal declarations of the allocation-free solve's static device scratch.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace sp2 {

// Bytes of the static device array: the two padded X buffers of the largest
// allowed size (2 x 1024^2 doubles = 16 MiB), the partial-sum slots, and the
// chunk accumulators of the FP64 product's K split in the rest.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
// Largest N the allocation-free solve accepts.
constexpr int kStaticMaxN = 1024;

// Device address of the static scratch on `device` (looked up once per device
// with that device current, then cached).
hipError_t static_scratch_init(int device, void** out);

}  // namespace sp2
