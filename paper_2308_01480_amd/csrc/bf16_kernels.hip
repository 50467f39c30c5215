// bfloat16 storage: streaming kernels on v_mfma_f32_16x16x32_bf16 (float32 accumulation).
#include <hip/hip_runtime.h>

#include "common.h"
#include "kernels.h"

namespace ttr {

hipError_t launch_fused_bf16(const StreamArgs&) { return hipErrorNotSupported; }
hipError_t launch_aw_bf16(const StreamArgs&) { return hipErrorNotSupported; }
hipError_t launch_atz_bf16(const StreamArgs&, void*, int, int64_t, int, int) { return hipErrorNotSupported; }
hipError_t launch_gram_bf16(const StreamArgs&, double*) { return hipErrorNotSupported; }

}  // namespace ttr
