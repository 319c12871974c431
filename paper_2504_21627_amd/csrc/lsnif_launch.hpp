// Kernel launchers shared between the host runtime and the kernel units.
#pragma once
#include <hip/hip_runtime.h>

namespace lsnif {
struct QueryArgs;
struct DebugArgs;
hipError_t launch_f32(const QueryArgs &A, int feat_dtype, int F, hipStream_t s);
hipError_t launch_mma(const QueryArgs &A, int feat_dtype, int mlp_dtype, int F, hipStream_t s);
hipError_t launch_debug(const DebugArgs &D, hipStream_t s);
}  // namespace lsnif
