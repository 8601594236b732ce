// Shared host/device helpers of liblbmfno: error state, HIP checks, the D2Q9
// constants of the product path, and the XCD-aware block remap.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "../../include/lbmfno.h"

namespace lbmfno {

// Thread-local message of the last failure; returned by lbm_last_error().
void set_error(const char* fmt, ...);
int fail(int code, const char* fmt, ...);

#define LBM_HIP(call)                                                              \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess)                                                      \
            return ::lbmfno::fail(LBM_EHIP, "%s failed: %s (%s:%d)", #call,       \
                                  hipGetErrorString(e_), __FILE__, __LINE__);      \
    } while (0)

// D2Q9 velocity set in the ABI's order; opposite directions; weights.
__host__ __device__ constexpr int cx_of(int q) {
    return q == 1 || q == 5 || q == 8 ? 1 : (q == 3 || q == 6 || q == 7 ? -1 : 0);
}
__host__ __device__ constexpr int cy_of(int q) {
    return q == 2 || q == 5 || q == 6 ? 1 : (q == 4 || q == 7 || q == 8 ? -1 : 0);
}
__host__ __device__ constexpr int opp_of(int q) {
    return q == 0 ? 0 : (q <= 4 ? ((q + 1) & 3) + 1 : ((q - 3) & 3) + 5);
}
__host__ __device__ constexpr float w_of(int q) {
    return q == 0 ? 4.0f / 9.0f : (q <= 4 ? 1.0f / 9.0f : 1.0f / 36.0f);
}
__host__ __device__ constexpr double w_of_d(int q) {
    return q == 0 ? 4.0 / 9.0 : (q <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
}
static_assert(opp_of(1) == 3 && opp_of(2) == 4 && opp_of(3) == 1 && opp_of(4) == 2, "opp");
static_assert(opp_of(5) == 7 && opp_of(6) == 8 && opp_of(7) == 5 && opp_of(8) == 6, "opp");

// Workgroups are dispatched round-robin over the 8 XCDs (workgroup b runs on XCD
// b % 8).  Remap so that XCD x processes one contiguous range of logical tiles:
// neighbouring tiles (which share halo rows) then share that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int nblocks) {
    const int q = nblocks >> 3, r = nblocks & 7;
    const int x = b & 7, k = b >> 3;
    return x * q + (x < r ? x : r) + k;
}

}  // namespace lbmfno
