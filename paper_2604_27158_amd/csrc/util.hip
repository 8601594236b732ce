// util.hip -- a plain streaming copy, the reference for achievable HBM bandwidth
// and for scaling the memory counters of the other kernels.
#include <hip/hip_runtime.h>

#include "common.hpp"

namespace lbmfno {

// One 16-byte element per lane, no grid-stride loop: the form that reaches the
// highest sustained bandwidth on this part.
__global__ __launch_bounds__(256) void k_stream_copy(const float4* __restrict__ src,
                                                     float4* __restrict__ dst, size_t n4) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n4) dst[i] = src[i];
}

}  // namespace lbmfno

using namespace lbmfno;

extern "C" int lbm_stream_copy(const float* d_src, float* d_dst, size_t n, void* stream) {
    if (!d_src || !d_dst) return fail(LBM_EINVAL, "NULL buffer");
    if (n % 4 != 0) return fail(LBM_EINVAL, "n = %zu is not a multiple of 4", n);
    if (((uintptr_t)d_src | (uintptr_t)d_dst) & 15) return fail(LBM_EINVAL, "buffers not 16-byte aligned");
    if (n == 0) return LBM_OK;
    const size_t n4 = n / 4;
    const size_t blocks = (n4 + 255) / 256;
    if (blocks > 0x7FFFFFFFu) return fail(LBM_EINVAL, "n = %zu too large for one launch", n);
    k_stream_copy<<<(unsigned)blocks, 256, 0, (hipStream_t)stream>>>(
        reinterpret_cast<const float4*>(d_src), reinterpret_cast<float4*>(d_dst), n4);
    LBM_HIP(hipGetLastError());
    return LBM_OK;
}
