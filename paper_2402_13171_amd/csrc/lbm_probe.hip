// Streaming copy kernel: the achievable-bandwidth reference (the paper takes
// its b_S from the STREAM copy kernel, Sec. 4.3) and the calibration kernel of
// known traffic for the hardware fetch/write counters.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/lbm.h"

namespace lbm {

// 16 bytes per access, one access per thread: 256-thread groups, as many
// groups as 16-byte elements / 256 (up to 2^22 groups, i.e. 16 GiB; a larger
// copy strides over the grid). On gfx950 this one-shot shape copied 4 GiB at
// 6.3 TB/s, against 5.4 TB/s for a 65536-group grid-stride loop and less
// again with 2, 4 or 8 elements per thread.
constexpr int PROBE_TPB = 256;
constexpr size_t PROBE_GROUPS = (size_t)1 << 22;

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
