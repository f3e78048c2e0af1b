// Workspace of the allocation-free adjoint entry point (rd_noalloc.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace rd {

// Bytes of the per-GPU workspace: 128 MiB, enough for meshes of about
// 125,000 vertices and 250,000 triangles (the adjoint needs about
// 296 B per vertex, 96 B per corner slot and 96 B per triangle).
constexpr size_t kNoallocScratchBytes = size_t(128) << 20;

// Device address of the current GPU's workspace (looked up on the first call
// on each device, with that device current, then cached).
hipError_t noalloc_scratch(void** ptr);

}  // namespace rd
