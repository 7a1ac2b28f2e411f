// Streaming copy kernel: the achievable-bandwidth reference (the paper takes
// its b_S from the STREAM copy kernel, Sec. 4.3) and the calibration kernel of
// known traffic for the hardware fetch/write counters.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lbm.h"

namespace lbm {

// 16 bytes per access, grid-stride; 512-thread groups and a 65536-group grid
// gave the highest copy rate among the shapes tried on gfx950
constexpr int PROBE_TPB = 512;
constexpr size_t PROBE_GROUPS = 65536;

__global__ __launch_bounds__(PROBE_TPB) void k_copy_probe(const float4 *__restrict__ src, float4 *__restrict__ dst,
                                                          size_t n) {
    for (size_t i = blockIdx.x * (size_t)PROBE_TPB + threadIdx.x; i < n; i += (size_t)gridDim.x * PROBE_TPB)
        dst[i] = src[i];
}

}  // namespace lbm

extern "C" int lbm_copy_probe(const void *src, void *dst, size_t bytes, void *stream) {
    if (!src || !dst || bytes % 16 || ((uintptr_t)src & 15) || ((uintptr_t)dst & 15)) return LBM_EINVAL;
    const size_t n = bytes / 16;
    if (n == 0) return LBM_OK;
    const size_t want = (n + lbm::PROBE_TPB - 1) / lbm::PROBE_TPB;
    const unsigned groups = (unsigned)(want < lbm::PROBE_GROUPS ? want : lbm::PROBE_GROUPS);
    lbm::k_copy_probe<<<groups, lbm::PROBE_TPB, 0, (hipStream_t)stream>>>((const float4 *)src, (float4 *)dst, n);
    return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EHIP;
}
