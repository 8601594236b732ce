// fno.hip -- Fourier Neural Operator forward pass (paper Sec. 2.2, Eq. 6) for
// gfx950: bfloat16 operands on MFMA (v_mfma_f32_32x32x16_bf16), float32
// accumulation.
//
// Data layout (device workspace, per sample b):
//   v  [Hp][Wpad][CP]   bf16  activations, channels last (CP = width rounded up to
//                             32, Wpad = W' rounded up to 32; w >= W' is zero)
//   T  [m2][Hpad][CP][2] bf16 row-DFT coefficients (re, im): mode k2 of all rows
//                             one contiguous block (one column workgroup's input);
//                             row h writes one 128-byte (CP = 32) piece per mode
//   Z  [2 m2][Hp][CP]   bf16  column-inverse coefficients, row kk = 2 k2 + (re/im),
//                             channels fastest (each mode group stores whole rows)
// Every contraction is arranged so that both MFMA operands are contiguous along
// the summed index, i.e. each lane fetches its eight bf16 as one 16-byte load:
//   row forward   T[kk][c]   = sum_w  EwT[kk][w]   * vt[c][w]     (vt staged in LDS)
//   column        X[r][c]    = sum_hk EcolA[r][hk] * T[c][hk]     (per sample, k2; T of
//                                the column staged transposed into LDS)
//   mixing        Y[k][o]    = sum_i  X[k][i] R[i][o]              (complex, per mode; bf16
//                                dot products, weights with o contiguous)
//   column inv    Zc[q][o]   = sum_r  EcolB[q][r]  * Y[o][r]
//   row inverse   s[w][o]    = sum_kk BinvT[w][kk] * Z[o][kk] + sum_i v[w][i] * Wc[o][i]
//                                (Z of the row transposed into LDS, kk >= 2 m2 zero)
// followed by bias and the activation, rounded to bf16 in the epilogue.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <tuple>
#include <utility>
#include <vector>

#include "common.hpp"

namespace lbmfno {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// One 32x32 tile C += A[32 x K] * Bt[32 x K]^T, A and Bt row-major with K
// contiguous (lda, ldb multiples of 8, 16-byte aligned rows), K a multiple of 16.
// Operand layout of v_mfma_f32_32x32x16_bf16: lane l supplies A[l % 32][8 (l / 32) + e]
// and B[8 (l / 32) + e][l % 32], e = 0..7.
__device__ __forceinline__ f32x16 mma_tile(const __bf16* A, int lda, const __bf16* Bt, int ldb,
                                           int K, f32x16 acc) {
    const int lane = threadIdx.x & 63;
    const int row = lane & 31, kh = lane >> 5;
    const __bf16* a = A + row * lda + 8 * kh;
    const __bf16* b = Bt + row * ldb + 8 * kh;
    // groups of four k-steps: the next group's operands are requested before the
    // current group's products, so that at most one memory latency per group is
    // exposed (these tiles are latency-bound at batch 1: few waves per CU)
    constexpr int U = 4;
    bf16x8 av[U] = {}, bv[U] = {};   // slots past K stay defined (zero) and unused
#pragma unroll
    for (int j = 0; j < U; ++j)
        if (16 * j < K) {
            av[j] = *reinterpret_cast<const bf16x8*>(a + 16 * j);
            bv[j] = *reinterpret_cast<const bf16x8*>(b + 16 * j);
        }
    for (int k0 = 0; k0 < K; k0 += 16 * U) {
        bf16x8 an[U] = {}, bn[U] = {};
        const int k1 = k0 + 16 * U;
#pragma unroll
        for (int j = 0; j < U; ++j)
            if (k1 + 16 * j < K) {
                an[j] = *reinterpret_cast<const bf16x8*>(a + k1 + 16 * j);
                bn[j] = *reinterpret_cast<const bf16x8*>(b + k1 + 16 * j);
            }
#pragma unroll
        for (int j = 0; j < U; ++j)
            if (k0 + 16 * j < K) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[j], bv[j], acc, 0, 0, 0);
#pragma unroll
        for (int j = 0; j < U; ++j) {
            av[j] = an[j];
            bv[j] = bn[j];
        }
    }
    return acc;
}

// Accumulator element r of this lane holds C[acc_row(r)][acc_col()].
__device__ __forceinline__ int acc_row(int r) {
    return 8 * (r >> 2) + 4 * ((threadIdx.x & 63) >> 5) + (r & 3);
}
__device__ __forceinline__ int acc_col() { return threadIdx.x & 31; }

// C += A[32 x 16 KS] * Bt[32 x 16 KS]^T with KS (the number of 16-wide k-steps)
// known at compile time: every operand is requested before the first product (one
// exposed memory latency), with no loop and no unused operand slots.  Same operand
// layout and k order as mma_tile, so the two give identical results.
template <int KS>
__device__ __forceinline__ f32x16 mma_k(const __bf16* A, int lda, const __bf16* Bt, int ldb, f32x16 acc) {
    const int lane = threadIdx.x & 63;
    const __bf16* a = A + (lane & 31) * lda + 8 * (lane >> 5);
    const __bf16* b = Bt + (lane & 31) * ldb + 8 * (lane >> 5);
    bf16x8 av[KS], bv[KS];
#pragma unroll
    for (int j = 0; j < KS; ++j) {
        av[j] = *reinterpret_cast<const bf16x8*>(a + 16 * j);
        bv[j] = *reinterpret_cast<const bf16x8*>(b + 16 * j);
    }
#pragma unroll
    for (int j = 0; j < KS; ++j) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av[j], bv[j], acc, 0, 0, 0);
    return acc;
}

// One operand of a 32 x 32 tile with KS k-steps held in registers, in mma_k's
// layout (rows lane % 32, k = 8 (lane / 32) + 16 j + e), and the products of two
// such operands: mma_rows(load_rows(A), load_rows(Bt)) is exactly mma_k(A, Bt).
template <int KS>
__device__ __forceinline__ void load_rows(bf16x8 (&o)[KS], const __bf16* A, int lda) {
    const int lane = threadIdx.x & 63;
    const __bf16* a = A + (lane & 31) * lda + 8 * (lane >> 5);
#pragma unroll
    for (int j = 0; j < KS; ++j) o[j] = *reinterpret_cast<const bf16x8*>(a + 16 * j);
}
template <int KS>
__device__ __forceinline__ f32x16 mma_rows(const bf16x8 (&a)[KS], const bf16x8 (&b)[KS], f32x16 acc) {
#pragma unroll
    for (int j = 0; j < KS; ++j) acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[j], b[j], acc, 0, 0, 0);
    return acc;
}

// K = 16 KS with KS a template constant when it is 2 or 4 (KS = 0: run-time K).
template <int KS>
__device__ __forceinline__ f32x16 mma_any(const __bf16* A, int lda, const __bf16* Bt, int ldb, int K,
                                          f32x16 acc) {
    if constexpr (KS > 0) return mma_k<KS>(A, lda, Bt, ldb, acc);
    else return mma_tile(A, lda, Bt, ldb, K, acc);
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// One 16x16 tile C += A[16 x K] * Bt[16 x K]^T on v_mfma_f32_16x16x32_bf16 (K a
// multiple of 32, operands K-contiguous as for mma_tile): lane l supplies
// A[l % 16][8 (l / 16) + e] and B[8 (l / 16) + e][l % 16], e = 0..7, and holds
// C[4 (l / 16) + r][l % 16] in acc[r], r = 0..3.  Groups of four k-steps, the next
// group requested before the current group's products.
__device__ __forceinline__ f32x4 mma16_tile(const __bf16* A, int lda, const __bf16* Bt, int ldb, int K,
                                            f32x4 acc) {
    const int lane = threadIdx.x & 63;
    const __bf16* a = A + (lane & 15) * lda + 8 * (lane >> 4);
    const __bf16* b = Bt + (lane & 15) * ldb + 8 * (lane >> 4);
    constexpr int U = 4;
    bf16x8 av[U] = {}, bv[U] = {};   // slots past K stay defined (zero) and unused
#pragma unroll
    for (int j = 0; j < U; ++j)
        if (32 * j < K) {
            av[j] = *reinterpret_cast<const bf16x8*>(a + 32 * j);
            bv[j] = *reinterpret_cast<const bf16x8*>(b + 32 * j);
        }
    for (int k0 = 0; k0 < K; k0 += 32 * U) {
        bf16x8 an[U] = {}, bn[U] = {};
        const int k1 = k0 + 32 * U;
#pragma unroll
        for (int j = 0; j < U; ++j)
            if (k1 + 32 * j < K) {
                an[j] = *reinterpret_cast<const bf16x8*>(a + k1 + 32 * j);
                bn[j] = *reinterpret_cast<const bf16x8*>(b + k1 + 32 * j);
            }
#pragma unroll
        for (int j = 0; j < U; ++j)
            if (k0 + 32 * j < K) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[j], bv[j], acc, 0, 0, 0);
#pragma unroll
        for (int j = 0; j < U; ++j) {
            av[j] = an[j];
            bv[j] = bn[j];
        }
    }
    return acc;
}

// Packed round-to-nearest-even bf16 pair (lo, hi) in one 32-bit word.
__device__ __forceinline__ uint32_t pack_bf16(float lo, float hi) {
    typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
    bf16x2 p;
    p[0] = (__bf16)lo;
    p[1] = (__bf16)hi;
    return *reinterpret_cast<uint32_t*>(&p);
}

// GELU x Phi(x) = x (1 + erf(x / sqrt 2)) / 2 for the forward kernels, with erf from
// Abramowitz & Stegun, Handbook of Mathematical Functions, 7.1.26: for z >= 0,
// erf z = 1 - t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) exp(-z^2), t = 1 / (1 + p z),
// absolute error below 1.5e-7.  With z = |x| / sqrt 2 and
// q = |x| t (a1 + ...) exp(-x^2 / 2) / 2, GELU is x - q for x >= 0 and -q for x < 0,
// that is max(x, 0) - q (the halved coefficients are the a_k / 2, exactly).
// The error (a few 1e-7 of |x|) is far below the bf16 rounding that follows.
__device__ __forceinline__ float gelu_fast(float x) {
    const float ax = fabsf(x);
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f * 0.70710678118654752f, ax, 1.0f));
    const float p = t * (0.127414796f + t * (-0.142248368f + t * (0.7107068705f +
                    t * (-0.7265760135f + t * 0.5307027145f))));
    // exp(-x^2 / 2) = 2^(-x^2 log2(e) / 2)
    const float e = __builtin_amdgcn_exp2f((-0.72134752044448170368f * x) * x);
    // max(x, 0) as a median of three (one instruction; fmaxf adds a canonicalising
    // max of x with itself); equal for every finite x
    return fmaf(-(ax * p), e, __builtin_amdgcn_fmed3f(x, 0.0f, 3.402823466e38f));
}

template <int KIND>
__device__ __forceinline__ float act_t(float x) {
    if constexpr (KIND == FNO_ACT_GELU) return gelu_fast(x);
    else if constexpr (KIND == FNO_ACT_RELU) return x > 0.0f ? x : 0.0f;
    // SiLU x sigmoid(x) with the hardware exponential and reciprocal (a few ulp in
    // FP32, far below the bf16 rounding that follows every activation)
    else if constexpr (KIND == FNO_ACT_SILU) return x * __builtin_amdgcn_rcpf(1.0f + __expf(-x));
    else return x;
}

// Run-time activation choice for the cold paths.  The forward kernels take the
// activation as a template argument instead: with a run-time switch inside an
// unrolled epilogue the compiler evaluates every branch and selects.
__device__ __forceinline__ float act_f(int kind, float x) {
    switch (kind) {
        case FNO_ACT_GELU: return act_t<FNO_ACT_GELU>(x);
        case FNO_ACT_RELU: return act_t<FNO_ACT_RELU>(x);
        case FNO_ACT_SILU: return act_t<FNO_ACT_SILU>(x);
        default: return x;
    }
}

__device__ __forceinline__ __bf16 to_bf16(float x) { return (__bf16)x; }
__device__ __forceinline__ float from_bf16(__bf16 x) { return (float)x; }

struct FnoDev {
    // sizes
    int B, H, W, Hp, Wp, Wpad, Hpad, CP, width, cin, cl, half, L, m1, m2, K1, R2, KKp;
    int dec_layers, dec_size, DSP, cout, act, dec_act, coords;
    // parameters (device)
    const float *lift1w, *lift1b, *lift2w, *lift2b;  // float32
    const __bf16* Rmix;     // [L][m2][K1][CP o][CP i][2] (backward: i contiguous)
    const __bf16* RmixT;    // [L][m2][K1][CP i][CP o][2] (forward: o contiguous)
    const __bf16* Wc;       // [L][CP][CP]
    const float* bc;        // [L][CP]
    const __bf16* decw;     // per decoder layer [DSP][in_p], then out [CoutP][DSP]
    const float* decb;      // per decoder layer [DSP], then out [cout]
    const __bf16 *EwT, *BinvT, *EcolA, *EcolB;
    const __bf16* WcT;      // [L][CP][CP], WcT[i][o] = Wc[o][i] (backward)
    const __bf16* B1;       // [Wpad][KKp] unit-coefficient inverse row basis (backward)
    const __bf16* decwT;    // hidden decoder layers transposed, [din_p][DSP] each (backward)
    int DKP;                // decoder LDS row stride (bf16 elements)
    int colS;               // column kernel: parts its column DFT's K range is split into
    int ncu;                // compute units of the device (persistent row kernels)
    // workspace
    __bf16 *v0, *v1, *T, *Z;
    // training forward: saved activations (NULL in plain inference)
    float* sv_a1;     // lift pre-activation [B][H][W][32]
    float* sv_X;      // column-DFT coefficients of this layer [B][m2][R2][CP]
    float* sv_pre;    // Fourier-layer pre-activation [B][Hp][Wpad][CP]
    float* sv_dec;    // decoder pre-activations, per layer [B][H][W][DSP]
};

// Row stride (bf16 elements) of a row's transposed copy vt[c][w] in LDS: Wpad plus
// 8, so that the 32 channels a wavefront stores (or the 32 rows an MFMA operand
// load reads) at one w fall on different banks (a stride of Wpad, a multiple of 32,
// put them all on one bank); still a multiple of 8 for 16-byte loads.
__host__ __device__ __forceinline__ int vt_stride(const FnoDev& d) { return d.Wpad + 8; }


// ---------------------------------------------------------------- kernels

// Lift weights staged in LDS, zero-padded to 32 hidden units, 8 inputs and NO
// outputs, so that the point loop has no channel-count branches.
template <int NO>
struct LiftW {
    float w1[32][8];   // W1[k][c]
    float b1[32];
    float w2t[32][NO];  // w2t[k][c] = W2[c][k]
    float b2[NO];
};

template <int NO>
__device__ __forceinline__ void lift_stage_weights(const FnoDev& d, LiftW<NO>& s) {
    for (int t = threadIdx.x; t < 32 * 8; t += blockDim.x) {
        const int k = t / 8, c = t % 8;
        s.w1[k][c] = (k < d.half && c < d.cl) ? d.lift1w[k * d.cl + c] : 0.0f;
    }
    for (int t = threadIdx.x; t < 32 * NO; t += blockDim.x) {
        const int k = t / NO, c = t % NO;
        s.w2t[k][c] = (k < d.half && c < d.width) ? d.lift2w[c * d.half + k] : 0.0f;
    }
    for (int t = threadIdx.x; t < NO; t += blockDim.x) s.b2[t] = t < d.width ? d.lift2b[t] : 0.0f;
    for (int t = threadIdx.x; t < 32; t += blockDim.x) s.b1[t] = t < d.half ? d.lift1b[t] : 0.0f;
}

// Hidden layer of the lift for point (b, h, w) of this lane: hid[k] = act(b1[k] +
// sum_c W1[k][c] z[c]) for k < KH (KH = 16 when half <= 16, else 32; the padded
// units come out as exact zeros), z = the fields and the two coordinates; zeros for
// a point outside H x W.  sv (training): the pre-activations, k < half.
template <int NO, int ACT, int KH>
__device__ __forceinline__ void lift_hidden(const FnoDev& d, const LiftW<NO>& s, const float* __restrict__ x,
                                            int b, int h, int w, bool valid, float (&hid)[KH], float* sv) {
#pragma unroll
    for (int k = 0; k < KH; ++k) hid[k] = 0.0f;
    if (!valid) return;
    float z[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) z[c] = 0.0f;
#pragma unroll
    for (int c = 0; c < 6; ++c)
        if (c < d.cin) z[c] = x[(((size_t)b * d.cin + c) * d.H + h) * d.W + w];
    if (d.coords) {
        const float xc = d.W > 1 ? (float)w / (float)(d.W - 1) : 0.0f;
        const float yc = d.H > 1 ? (float)h / (float)(d.H - 1) : 0.0f;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            if (c == d.cin) z[c] = xc;
            if (c == d.cin + 1) z[c] = yc;
        }
    }
#pragma unroll
    for (int k = 0; k < KH; ++k) {
        // padded inputs carry zero weights and zero values: exact no-ops
        float a = s.b1[k];
#pragma unroll
        for (int c = 0; c < 8; ++c) a = fmaf(s.w1[k][c], z[c], a);
        if (sv && k < d.half) sv[k] = a;
        hid[k] = act_t<ACT>(a);
    }
}

// Output layer of the lift for the wave's 64 points (lane l holds the hidden units
// of point p0 + l) on the float32 matrix cores (v_mfma_f32_32x32x2_f32: lane l
// supplies A[l % 32][l / 32] and B[l / 32][l % 32], one float each, and holds the
// 32 x 32 result in the layout of the bf16 tiles).  Tile u covers points
// p0 + 32 u + (l % 32); step s sums hidden units 2 s and 2 s + 1, the half-wave
// that does not own the point receiving its unit from the other half.  acc[u][nt][r]
// = b2[o] + sum_k W2[o][k] hid[k] for channel o = 32 nt + acc_row(r).
template <int NO, int KH>
__device__ __forceinline__ void lift_output(const LiftW<NO>& s, const float (&hid)[KH], f32x16 (&acc)[2][NO / 32]) {
    const int lane = threadIdx.x & 63, p = lane & 31, g = lane >> 5;
#pragma unroll
    for (int nt = 0; nt < NO / 32; ++nt)
#pragma unroll
        for (int r = 0; r < 16; ++r) acc[0][nt][r] = acc[1][nt][r] = s.b2[32 * nt + acc_row(r)];
#pragma unroll
    for (int st = 0; st < KH / 2; ++st) {
        const float a = hid[2 * st], c = hid[2 * st + 1];
        const float sa = __shfl_xor(a, 32), sc = __shfl_xor(c, 32);
        const float b0 = g == 0 ? a : sc;   // tile 0: unit 2 st from the lower half, 2 st + 1 from the upper
        const float b1 = g == 0 ? sa : c;   // tile 1: the points of the upper half
#pragma unroll
        for (int nt = 0; nt < NO / 32; ++nt) {
            const float wa = s.w2t[2 * st + g][32 * nt + p];
            acc[0][nt] = __builtin_amdgcn_mfma_f32_32x32x2f32(wa, b0, acc[0][nt], 0, 0, 0);
            acc[1][nt] = __builtin_amdgcn_mfma_f32_32x32x2f32(wa, b1, acc[1][nt], 0, 0, 0);
        }
    }
}

// Lift: x (cin channels, float32) + coordinates -> width/2 (act) -> width, rounded
// to bf16, written channels-last; the zero-padded region and w >= W' hold zeros.
// A lane per point, a wave per 64 consecutive points.  NO = CP (32 or 64); ACT =
// d.act; KH as for lift_hidden.
template <int NO, int ACT, int KH>
__global__ __launch_bounds__(256) void k_fno_lift(FnoDev d, const float* __restrict__ x) {
    __shared__ LiftW<NO> lw;
    lift_stage_weights<NO>(d, lw);
    __syncthreads();
    // point indices fit 32 bits (B Hp Wpad CP < 2^31 is checked on the host), so
    // the index arithmetic avoids 64-bit division
    const unsigned total = (unsigned)d.B * d.Hp * d.Wpad;
    const unsigned p0 = (blockIdx.x * blockDim.x + threadIdx.x) & ~63u;   // the wave's first point
    if (p0 >= total) return;   // uniform over the wave
    const int lane = threadIdx.x & 63;
    auto locate = [&](unsigned idx, int& b, int& h, int& w) {
        const unsigned rw = idx / (unsigned)d.Wpad;
        w = (int)(idx - rw * d.Wpad);
        b = (int)(rw / (unsigned)d.Hp);
        h = (int)(rw - (unsigned)b * d.Hp);
    };
    int b, h, w;
    const unsigned idx = p0 + lane;
    locate(idx, b, h, w);
    const bool valid = idx < total && h < d.H && w < d.W;
    float hid[KH];
    lift_hidden<NO, ACT, KH>(d, lw, x, b, h, w, valid, hid,
                             d.sv_a1 && valid ? d.sv_a1 + (((size_t)b * d.H + h) * d.W + w) * 32 : nullptr);
    f32x16 acc[2][NO / 32];
    lift_output<NO, KH>(lw, hid, acc);
    const int g = lane >> 5;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const unsigned pt = p0 + 32 * u + (lane & 31);
        if (pt >= total) continue;
        int pb, ph, pw;
        locate(pt, pb, ph, pw);
        const bool live = ph < d.H && pw < d.W;
        __bf16* op = d.v0 + (size_t)pt * d.CP;
#pragma unroll
        for (int nt = 0; nt < NO / 32; ++nt)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                uint2 q;
                q.x = live ? pack_bf16(acc[u][nt][4 * j], acc[u][nt][4 * j + 1]) : 0u;
                q.y = live ? pack_bf16(acc[u][nt][4 * j + 2], acc[u][nt][4 * j + 3]) : 0u;
                *reinterpret_cast<uint2*>(op + 32 * nt + 8 * j + 4 * g) = q;
            }
    }
}

// Row forward DFT: one workgroup per (b, h), h < Hpad (rows h >= H' write zeros so
// the column transform's padded K range is exactly zero).
// Row DFT of row (b, h < Hp) from its transposed copy vt[c][w] in LDS:
// T[k2][c][ri][h] = sum_w EwT[2 k2 + ri][w] vt[c][w].
// T is laid out [B][m2][Hpad][CP] (re, im) pairs, so that the column kernel of
// (b, k2) reads one contiguous block: the CP pairs of row h, mode k2.
__device__ __forceinline__ __bf16* t_piece(const FnoDev& d, int b, int h, int k2) {
    return d.T + (((size_t)b * d.m2 + k2) * d.Hpad + h) * d.CP * 2;
}

// Rows h >= Hp of T are zero (the column transform's K range runs over Hpad rows).
__device__ __forceinline__ void t_zero_row(const FnoDev& d, int b, int h) {
    for (int i = threadIdx.x; i < d.m2 * d.CP; i += blockDim.x)
        reinterpret_cast<uint32_t*>(t_piece(d, b, h, i / d.CP))[i % d.CP] = 0u;
}

// The KKp x CP result is taken in 16 x 16 tiles, so that every wave of the
// workgroup has one (the 2 m2 <= KKp rows in use fill fewer 32-row tiles than there
// are waves).
__device__ __forceinline__ void row_dft_from_lds(const FnoDev& d, const __bf16* vt, int b, int h) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int Mt = (2 * d.m2 + 15) / 16, Nt = d.CP / 16;
    for (int t = wave; t < Mt * Nt; t += blockDim.x >> 6) {
        const int mi = t / Nt, ni = t % Nt;
        f32x4 acc = {};
        acc = mma16_tile(d.EwT + (size_t)mi * 16 * d.Wpad, d.Wpad, vt + ni * 16 * vt_stride(d), vt_stride(d),
                         d.Wpad, acc);
        // rows kk = 2 k2 + ri come in (re, im) pairs, two per lane: one packed word
        // per pair, and the 16 lanes of a quarter-wave store 16 consecutive words
        const int c = ni * 16 + (lane & 15);
        const int kk = mi * 16 + 4 * (lane >> 4);
        if (kk < 2 * d.m2) reinterpret_cast<uint32_t*>(t_piece(d, b, h, kk >> 1))[c] = pack_bf16(acc[0], acc[1]);
        if (kk + 2 < 2 * d.m2)
            reinterpret_cast<uint32_t*>(t_piece(d, b, h, (kk >> 1) + 1))[c] = pack_bf16(acc[2], acc[3]);
    }
}

// The same row DFT with the EwT operand held in registers: when the 16 x 16 tiles
// number at most one per wave and Wpad = 32 KW, each wave requests its tile's EwT
// rows at the start of the row kernel (row_dft_load), long before the transposed
// row in LDS is complete, so that after the barrier the products wait on LDS only
// (row_dft_regs).  Same products in the same order as row_dft_from_lds.
__host__ __device__ __forceinline__ int row_dft_tiles(const FnoDev& d) { return (2 * d.m2 + 15) / 16 * (d.CP / 16); }

template <int KW>
__device__ __forceinline__ void row_dft_load(const FnoDev& d, bf16x8 (&ew)[KW]) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int mi = wave / (d.CP / 16);
    const __bf16* a = d.EwT + (size_t)(mi * 16 + (lane & 15)) * d.Wpad + 8 * (lane >> 4);
#pragma unroll
    for (int j = 0; j < KW; ++j) ew[j] = *reinterpret_cast<const bf16x8*>(a + 32 * j);
}

template <int KW>
__device__ __forceinline__ void row_dft_regs(const FnoDev& d, const bf16x8 (&ew)[KW], const __bf16* vt, int b,
                                             int h) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int Nt = d.CP / 16, mi = wave / Nt, ni = wave % Nt;
    const __bf16* bp = vt + (ni * 16 + (lane & 15)) * vt_stride(d) + 8 * (lane >> 4);
    bf16x8 bv[KW];
#pragma unroll
    for (int j = 0; j < KW; ++j) bv[j] = *reinterpret_cast<const bf16x8*>(bp + 32 * j);
    f32x4 acc = {};
#pragma unroll
    for (int j = 0; j < KW; ++j) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ew[j], bv[j], acc, 0, 0, 0);
    const int c = ni * 16 + (lane & 15);
    const int kk = mi * 16 + 4 * (lane >> 4);
    if (kk < 2 * d.m2) reinterpret_cast<uint32_t*>(t_piece(d, b, h, kk >> 1))[c] = pack_bf16(acc[0], acc[1]);
    if (kk + 2 < 2 * d.m2)
        reinterpret_cast<uint32_t*>(t_piece(d, b, h, (kk >> 1) + 1))[c] = pack_bf16(acc[2], acc[3]);
}

// The row held transposed in LDS, vt[c][w], stored channels last to orow[w][c]:
// each thread assembles 8 channels of one point, and consecutive threads take
// consecutive 16-byte pieces of the row, so a wave writes 1 KB of it contiguously.
// CP is 32 or 64, so the CP / 8 pieces of a point divide the workgroup size (a
// multiple of 64): a thread keeps its channel group c0 and steps through w.
__device__ __forceinline__ void store_row_from_vt(const FnoDev& d, const __bf16* vt, __bf16* orow) {
    const int VS = vt_stride(d), ncg = d.CP / 8;
    const int c0 = 8 * (threadIdx.x % ncg), wstep = blockDim.x / ncg;
    for (int w = threadIdx.x / ncg; w < d.Wpad; w += wstep) {
        bf16x8 t;
#pragma unroll
        for (int e = 0; e < 8; ++e) t[e] = vt[(c0 + e) * VS + w];
        *reinterpret_cast<bf16x8*>(orow + w * d.CP + c0) = t;
    }
}

__global__ __launch_bounds__(256) void k_fno_rowfwd(FnoDev d, const __bf16* __restrict__ v) {
    extern __shared__ __align__(16) unsigned char smem[];
    __bf16* vt = reinterpret_cast<__bf16*>(smem);  // [CP][vt_stride]
    const int b = blockIdx.x / d.Hpad, h = blockIdx.x % d.Hpad;
    const int tid = threadIdx.x;
    if (h >= d.Hp) {
        t_zero_row(d, b, h);
        return;
    }
    const __bf16* row = v + ((size_t)b * d.Hp + h) * d.Wpad * d.CP;
    // stage the row transposed: vt[c][w] = row[w][c]
    const int nvec = d.Wpad * d.CP / 8;
    for (int i = tid; i < nvec; i += blockDim.x) {
        const bf16x8 t = *reinterpret_cast<const bf16x8*>(row + 8 * i);
        const int w = (8 * i) / d.CP, c0 = (8 * i) % d.CP;
        for (int e = 0; e < 8; ++e) vt[(c0 + e) * vt_stride(d) + w] = t[e];
    }
    __syncthreads();
    row_dft_from_lds(d, vt, b, h);
}

// Inference: the lift fused with the first layer's row DFT, one workgroup per row
// (b, h < Hpad) with a lane per point of the row (blockDim.x >= Wpad).  Each lane
// lifts its point as k_fno_lift does (same operations, same order), stores it to v
// and into the row's transposed copy in LDS, from which the row DFT is taken as in
// k_fno_rowfwd; rows h >= Hp only write T's zero rows.
template <int NO, int ACT, int KH, int KW>
__global__ __launch_bounds__(1024) void k_fno_lift_row(FnoDev d, const float* __restrict__ x) {
    __shared__ LiftW<NO> lw;
    extern __shared__ __align__(16) unsigned char smem[];
    __bf16* vt = reinterpret_cast<__bf16*>(smem);  // [CP][vt_stride]
    const int tid = threadIdx.x, lane = tid & 63, g = lane >> 5;
    const int VS = vt_stride(d);
    bf16x8 ew[KW > 0 ? KW : 1];
    const bool dft_wave = KW > 0 && (int)(tid >> 6) < row_dft_tiles(d);
    if constexpr (KW > 0)
        if (dft_wave) row_dft_load<KW>(d, ew);
    lift_stage_weights<NO>(d, lw);
    // the workgroups step through the rows (one row each when launched with a
    // workgroup per row); the weights and, with KW > 0, the row-DFT operand are
    // loaded once per workgroup
    const int rows = d.B * d.Hpad;
    for (int row = blockIdx.x; row < rows; row += gridDim.x) {
        const int b = row / d.Hpad, h = row - b * d.Hpad;
        if (h >= d.Hp) {
            t_zero_row(d, b, h);
            continue;
        }
        // the staged weights (first row); the previous row's reads of vt
        __syncthreads();
        const int w = tid, w0 = tid & ~63;   // the wave's points w0 .. w0 + 63
        float hid[KH];
        lift_hidden<NO, ACT, KH>(d, lw, x, b, h, w, h < d.H && w < d.W, hid, nullptr);
        f32x16 acc[2][NO / 32];
        lift_output<NO, KH>(lw, hid, acc);
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int wu = w0 + 32 * u + (lane & 31);
            if (wu >= d.Wpad) continue;
            const bool live = h < d.H && wu < d.W;
#pragma unroll
            for (int nt = 0; nt < NO / 32; ++nt)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    __bf16* vc = vt + (32 * nt + 8 * j + 4 * g) * VS + wu;
#pragma unroll
                    for (int i = 0; i < 4; ++i) vc[i * VS] = to_bf16(live ? acc[u][nt][4 * j + i] : 0.0f);
                }
        }
        __syncthreads();
        if constexpr (KW > 0) {
            if (dft_wave) row_dft_regs<KW>(d, ew, vt, b, h);
        } else {
            row_dft_from_lds(d, vt, b, h);
        }
        store_row_from_vt(d, vt, d.v0 + ((size_t)b * d.Hp + h) * d.Wpad * d.CP);
    }
}

// Column inverse of column k2 of sample b from Y[o][r] in LDS: Zc[q][o] =
// sum_r EcolB[q][r] Y[o][r], q = ri * Hpad + h, stored to Z rows kk = 2 k2 + ri
// (rows h < Hp).  Each tile is formed transposed, C^T[o][q], so that a lane holds
// four consecutive channels of one (ri, h) and stores them as one 8-byte quad.
__device__ __forceinline__ void z_store_column(const FnoDev& d, int b, int k2, const __bf16* ys) {
    const int wave = threadIdx.x >> 6, nw = blockDim.x >> 6, lane = threadIdx.x & 63;
    const int Mt = 2 * d.Hpad / 32, Nt = d.CP / 32;
    for (int t = wave; t < Mt * Nt; t += nw) {
        const int mi = t / Nt, ni = t % Nt;
        f32x16 acc = {};
        acc = mma_tile(ys + ni * 32 * d.R2, d.R2, d.EcolB + (size_t)mi * 32 * d.R2, d.R2, d.R2, acc);
        const int q = mi * 32 + (lane & 31);
        const int ri = q >= d.Hpad ? 1 : 0, h = q - ri * d.Hpad;
        if (h < d.Hp) {
            __bf16* zp = d.Z + (((size_t)b * 2 * d.m2 + 2 * k2 + ri) * d.Hp + h) * d.CP + ni * 32 + 4 * (lane >> 5);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                uint2 w;
                w.x = pack_bf16(acc[4 * j], acc[4 * j + 1]);
                w.y = pack_bf16(acc[4 * j + 2], acc[4 * j + 3]);
                *reinterpret_cast<uint2*>(zp + 8 * j) = w;
            }
        }
    }
}

// Z coefficients of row (b, h) transposed into LDS, zs[o][kk] with row stride
// KKp + 8, and the padded coefficient columns kk >= 2 m2 set to zero.  Reads are
// 16-byte channel vectors of whole Z rows.
__device__ __forceinline__ void stage_z(const FnoDev& d, int b, int h, __bf16* zs) {
    // (nvec = CP / 8 is 4 or 8 and divides the workgroup size, as in store_row_from_vt)
    const int KKs = d.KKp + 8, nvec = d.CP / 8;
    const int o0 = 8 * (threadIdx.x % nvec), kstep = blockDim.x / nvec;
    for (int kk = threadIdx.x / nvec; kk < d.KKp; kk += kstep) {
        bf16x8 t;
        if (kk < 2 * d.m2) {
            t = *reinterpret_cast<const bf16x8*>(d.Z + (((size_t)b * 2 * d.m2 + kk) * d.Hp + h) * d.CP + o0);
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) t[e] = to_bf16(0.0f);
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) zs[(o0 + e) * KKs + kk] = t[e];
    }
    __syncthreads();
}

// Row stride (bf16) of a column's T staged in LDS, [CP][TS], K = (ri, h) contiguous.
__host__ __device__ __forceinline__ int ts_stride(const FnoDev& d) { return 2 * d.Hpad + 8; }

// T of column k2 of sample b, staged transposed: tsl[c][ri * Hpad + h] (the MFMA
// operand layout, K contiguous).  Each row h holds the column's CP (re, im) pairs
// as one 128-byte (CP = 32) piece, read with 16-byte loads (eight lanes per piece);
// a thread takes one 16-byte slot q of four consecutive rows and writes each of its
// eight values' four rows as one 8-byte LDS store (Hpad is a multiple of 16).
// Ends with a barrier.
__device__ __forceinline__ void stage_t(const FnoDev& d, int b, int k2, __bf16* tsl) {
    const int TS = ts_stride(d), nq = d.CP / 4, ng = d.Hpad / 4;
    for (int i = threadIdx.x; i < ng * nq; i += blockDim.x) {
        const int g = i / nq, q = i - g * nq;
        bf16x8 t[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            t[u] = *reinterpret_cast<const bf16x8*>(t_piece(d, b, 4 * g + u, k2) + 8 * q);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            bf16x4 v;
            v[0] = t[0][e];
            v[1] = t[1][e];
            v[2] = t[2][e];
            v[3] = t[3][e];
            *reinterpret_cast<bf16x4*>(tsl + (4 * q + (e >> 1)) * TS + (e & 1) * d.Hpad + 4 * g) = v;
        }
    }
    __syncthreads();
}

// Column forward DFT, per-mode complex mixing and column inverse DFT for one
// (sample, k2).
// Launched with COL_THREADS threads: at batch 1 there is one workgroup per mode
// column and the kernel is a chain of memory latencies, so more waves shorten it.
constexpr int COL_THREADS = 512;

typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(COL_THREADS) void k_fno_col(FnoDev d, int layer) {
    extern __shared__ __align__(16) unsigned char smem[];
    __bf16* Ts = reinterpret_cast<__bf16*>(smem);                                // [CP][TS]
    unsigned char* sm2 = smem + (size_t)d.CP * ts_stride(d) * 2;
    float* xs = reinterpret_cast<float*>(sm2);                                   // [R2][CP]
    __bf16* ys = reinterpret_cast<__bf16*>(sm2 + sizeof(float) * d.R2 * d.CP);   // [CP][R2]
    const int b = blockIdx.x / d.m2, k2 = blockIdx.x % d.m2;
    const int tid = threadIdx.x, wave = tid >> 6, nw = blockDim.x >> 6;
    const int H2 = 2 * d.Hpad, TS = ts_stride(d);
    const int Nt = d.CP / 32;
    const int nmix = d.K1 * d.width;
    const uint32_t* R =
        reinterpret_cast<const uint32_t*>(d.RmixT + ((size_t)layer * d.m2 + k2) * d.K1 * d.CP * d.CP * 2);
    const int Mt1 = d.R2 / 32, T1 = Mt1 * Nt;
    stage_t(d, b, k2, Ts);
    float* svX = d.sv_X ? d.sv_X + ((size_t)b * d.m2 + k2) * d.R2 * d.CP : nullptr;
    // X[r][c] = sum_{ri,h} EcolA[r][ri,h] T[c][ri,h]
    if (d.colS == 1) {
        for (int t = wave; t < T1; t += nw) {
            const int mi = t / Nt, ni = t % Nt;
            f32x16 acc = {};
            acc = mma_tile(d.EcolA + (size_t)mi * 32 * H2, H2, Ts + ni * 32 * TS, TS, H2, acc);
            const int c = ni * 32 + acc_col();
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const float xv = from_bf16(to_bf16(acc[r]));
                xs[(mi * 32 + acc_row(r)) * d.CP + c] = xv;
                if (svX) svX[(mi * 32 + acc_row(r)) * d.CP + c] = xv;
            }
        }
    } else {
        // fewer tiles than waves: the K range (2 Hpad, in 16-wide steps) is split
        // into S parts, wave w taking tile w mod T1 and part w / T1.  Part 0 writes
        // xs, part s > 0 its own [R2][CP] partial after ys; the parts are then added
        // in part order (deterministic) and rounded.
        const int S = d.colS, KS = H2 / 16;
        const int tile = wave % T1, part = wave / T1;
        const int mi = tile / Nt, ni = tile % Nt;
        const int k0 = 16 * (part * KS / S), k1 = 16 * ((part + 1) * KS / S);
        float* parts = reinterpret_cast<float*>(sm2 + (size_t)d.R2 * d.CP * 6);  // [S-1][R2][CP]
        if (part < S) {
            f32x16 acc = {};
            if (k1 > k0)
                acc = mma_tile(d.EcolA + (size_t)mi * 32 * H2 + k0, H2, Ts + ni * 32 * TS + k0, TS,
                               k1 - k0, acc);
            float* dst = part == 0 ? xs : parts + (size_t)(part - 1) * d.R2 * d.CP;
            const int c = ni * 32 + acc_col();
#pragma unroll
            for (int r = 0; r < 16; ++r) dst[(mi * 32 + acc_row(r)) * d.CP + c] = acc[r];
        }
        __syncthreads();
        for (int i = tid; i < d.R2 * d.CP; i += blockDim.x) {
            float v = xs[i];
            for (int q = 1; q < S; ++q) v += parts[(size_t)(q - 1) * d.R2 * d.CP + i];
            const float xv = from_bf16(to_bf16(v));
            xs[i] = xv;
            if (svX) svX[i] = xv;
        }
    }
    __syncthreads();
    // X as the mixing's bf16 operand pairs, in place: the slot of xr = X[k][c] takes
    // (xr, -xi) and that of xi = X[K1 + k][c] takes (xi, xr), so that with a weight
    // pair w = (rr, ri), dot((xr, -xi), w) = Re(x r) and dot((xi, xr), w) = Im(x r).
    // (X is already bf16, so the packing is exact.)
    uint32_t* xu = reinterpret_cast<uint32_t*>(xs);
    for (int i = tid; i < d.K1 * d.CP; i += blockDim.x) {
        const float xr = xs[i], xi = xs[d.K1 * d.CP + i];
        xu[i] = pack_bf16(xr, -xi);
        xu[d.K1 * d.CP + i] = pack_bf16(xi, xr);
    }
    for (int i = tid; i < d.CP * d.R2; i += blockDim.x) ys[i] = to_bf16(0.0f);
    __syncthreads();
    // Y[k][o] = sum_i X[k][i] R[i][o][k][k2] (complex), k over the 2 m1 kept rows
    // Only the width real channels take part, and ys was cleared above.  A thread
    // forms one (k, o) with two bf16 dot products per i (each product exact in
    // FP32); the weights are laid out with o contiguous, so for each i the lanes of
    // a wave read consecutive (re, im) pairs of one or two weight rows, and the
    // operand pairs of X are the same for 32 lanes.
    for (int idx = tid; idx < nmix; idx += blockDim.x) {
        const int k = idx / d.width, o = idx % d.width;
        const uint32_t* p1 = xu + (size_t)k * d.CP;
        const uint32_t* p2 = xu + (size_t)(d.K1 + k) * d.CP;
        const uint32_t* Rk = R + (size_t)k * d.CP * d.CP + o;
        float sr = 0.0f, si = 0.0f;
        if (d.width <= 32) {
            // 32 channels (CP >= 32) in two groups of 16 weights requested together;
            // the padded channels' X and R are zero and add nothing
#pragma unroll
            for (int i0 = 0; i0 < 32; i0 += 16) {
                uint32_t wv[16];
#pragma unroll
                for (int j = 0; j < 16; ++j) wv[j] = Rk[(size_t)(i0 + j) * d.CP];
#pragma unroll
                for (int j = 0; j < 16; ++j) {
                    const bf16x2v w = __builtin_bit_cast(bf16x2v, wv[j]);
                    sr = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2v, p1[i0 + j]), w, sr, false);
                    si = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2v, p2[i0 + j]), w, si, false);
                }
            }
        } else {
#pragma unroll 8
            for (int i = 0; i < d.width; ++i) {
                const bf16x2v w = __builtin_bit_cast(bf16x2v, Rk[(size_t)i * d.CP]);
                sr = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2v, p1[i]), w, sr, false);
                si = __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2v, p2[i]), w, si, false);
            }
        }
        ys[o * d.R2 + k] = to_bf16(sr);
        ys[o * d.R2 + d.K1 + k] = to_bf16(si);
    }
    __syncthreads();
    z_store_column(d, b, k2, ys);
}

// Row inverse DFT + 1x1 convolution + bias (+ activation) for one (b, h).
// ACT: d.act, or the identity for the last layer.  DFT: also take the next layer's
// row DFT of the output row (kept in LDS, transposed), so the next layer needs no
// row-forward launch; rows h >= Hp of T stay the zeros the first row DFT wrote.
// KZ, KC: 16-wide k-steps of the coefficient and channel contractions (KKp / 16,
// CP / 16) as template constants, 0 for a run-time count.
//
// Each 32 x 32 output tile is formed transposed, C^T[o][w] = Z[o][:] . Binv[w][:] +
// Wc[o][:] . v[w][:]: a lane then holds the four channels o, o+1, o+2, o+3 of one
// point w in four register groups, so it stores 8-byte packed bf16 quads of the
// channels-last output row (four stores per tile), and the transposed LDS copy
// for the next row DFT is written along w (consecutive lanes, consecutive bf16).
template <int ACT, bool DFT, int KZ, int KC>
__global__ __launch_bounds__(256) void k_fno_rowinv(FnoDev d, const __bf16* __restrict__ v,
                                                    __bf16* __restrict__ vout, int layer) {
    const int b = blockIdx.x / d.Hp, h = blockIdx.x % d.Hp;
    const int tid = threadIdx.x, wave = tid >> 6, nw = blockDim.x >> 6;
    const int lane = tid & 63, wl = lane & 31, g = lane >> 5;
    const size_t rowoff = ((size_t)b * d.Hp + h) * d.Wpad * d.CP;
    const __bf16* vrow = v + rowoff;
    __bf16* orow = vout + rowoff;
    extern __shared__ __align__(16) unsigned char smem[];
    __bf16* zs = reinterpret_cast<__bf16*>(smem);  // [CP][KKp + 8]
    __bf16* vt = zs + (size_t)d.CP * (d.KKp + 8);  // [CP][vt_stride] (DFT)
    stage_z(d, b, h, zs);
    const int KKs = d.KKp + 8, VS = vt_stride(d), CP = d.CP;
    const __bf16* Wc = d.Wc + (size_t)layer * CP * CP;
    const float* bias = d.bc + (size_t)layer * CP;
    const int Mt = d.Wpad / 32, Nt = CP / 32;
    for (int t = wave; t < Mt * Nt; t += nw) {
        const int mi = t / Nt, ni = t % Nt;
        f32x16 acc = {};
        acc = mma_any<KZ>(zs + ni * 32 * KKs, KKs, d.BinvT + mi * 32 * d.KKp, d.KKp, d.KKp, acc);
        acc = mma_any<KC>(Wc + ni * 32 * CP, CP, vrow + mi * 32 * CP, CP, CP, acc);
        const int w = mi * 32 + wl;
        const bool live = w < d.Wp;
        const uint32_t lmask = live ? 0xffffffffu : 0u;
        const int ob = ni * 32 + 4 * g;  // channels of register group j: ob + 8 j + 0..3
        float val[16];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float4 bq = *reinterpret_cast<const float4*>(bias + ob + 8 * j);
            val[4 * j + 0] = acc[4 * j + 0] + bq.x;
            val[4 * j + 1] = acc[4 * j + 1] + bq.y;
            val[4 * j + 2] = acc[4 * j + 2] + bq.z;
            val[4 * j + 3] = acc[4 * j + 3] + bq.w;
        }
        if (d.sv_pre) {   // training: the pre-activation, zero beyond W'
            float* sp = d.sv_pre + rowoff + (size_t)w * CP + ob;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                *reinterpret_cast<float4*>(sp + 8 * j) =
                    live ? make_float4(val[4 * j], val[4 * j + 1], val[4 * j + 2], val[4 * j + 3])
                         : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
        __bf16* op = orow + w * CP + ob;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            uint2 q;
            // (the activations unconditionally, then the mask: see k_fno_rowinv_p)
            q.x = pack_bf16(act_t<ACT>(val[4 * j + 0]), act_t<ACT>(val[4 * j + 1])) & lmask;
            q.y = pack_bf16(act_t<ACT>(val[4 * j + 2]), act_t<ACT>(val[4 * j + 3])) & lmask;
            if constexpr (DFT) {   // the row goes out from LDS below
                __bf16* vc = vt + (ob + 8 * j) * VS + w;
                const __bf16* e = reinterpret_cast<const __bf16*>(&q);
                vc[0] = e[0];
                vc[VS] = e[1];
                vc[2 * VS] = e[2];
                vc[3 * VS] = e[3];
            } else {
                *reinterpret_cast<uint2*>(op + 8 * j) = q;
            }
        }
    }
    if constexpr (DFT) {
        __syncthreads();
        row_dft_from_lds(d, vt, b, h);
        store_row_from_vt(d, vt, orow);
    }
}

// The row inverse as a persistent kernel for row shapes whose 32 x 32 tiles number
// at most two per wave (Wpad / 32 x CP / 32 <= 8) and, with DFT, whose row-DFT tiles
// number at most one per wave, with Wpad = 32 KW: the workgroups step through the
// rows, and each wave keeps its constant operands in registers across them (the Wc
// rows of its channel tile, the BinvT rows of its two point tiles and, with DFT,
// the EwT rows of its row-DFT tile).  Per row only the activations and the row's Z
// are read, where the one-row kernel also re-reads some 50 KB of constant operands
// through the vector memory path.  Same products in the same order as k_fno_rowinv,
// so the results are identical.
template <int ACT, bool DFT, int KZ, int KC, int KW>
__global__ __launch_bounds__(256) void k_fno_rowinv_p(FnoDev d, const __bf16* __restrict__ v,
                                                      __bf16* __restrict__ vout, int layer) {
    const int tid = threadIdx.x, wave = tid >> 6, nw = blockDim.x >> 6;
    const int lane = tid & 63, wl = lane & 31, g = lane >> 5;
    extern __shared__ __align__(16) unsigned char smem[];
    __bf16* zs = reinterpret_cast<__bf16*>(smem);  // [CP][KKp + 8]
    __bf16* vt = zs + (size_t)d.CP * (d.KKp + 8);  // [CP][vt_stride] (DFT)
    const int KKs = d.KKp + 8, VS = vt_stride(d), CP = d.CP;
    const int Mt = d.Wpad / 32, Nt = CP / 32, T = Mt * Nt;
    const int ni = wave % Nt;  // both tiles of the wave (t = wave, wave + nw; nw is a multiple of Nt)
    const int ob = ni * 32 + 4 * g;  // channels of register group j: ob + 8 j + 0..3
    bf16x8 wc[KC], bi[2][KZ];
    load_rows<KC>(wc, d.Wc + ((size_t)layer * CP + ni * 32) * CP, CP);
#pragma unroll
    for (int u = 0; u < 2; ++u)
        if (wave + u * nw < T) load_rows<KZ>(bi[u], d.BinvT + ((wave + u * nw) / Nt) * 32 * d.KKp, d.KKp);
    bf16x8 ew[DFT ? KW : 1];
    const bool dft_wave = DFT && wave < row_dft_tiles(d);
    if constexpr (DFT)
        if (dft_wave) row_dft_load<KW>(d, ew);
    float4 bq[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) bq[j] = *reinterpret_cast<const float4*>(d.bc + (size_t)layer * CP + ob + 8 * j);
    const int rows = d.B * d.Hp;
    for (int row = blockIdx.x; row < rows; row += gridDim.x) {
        const int b = row / d.Hp, h = row - b * d.Hp;
        const size_t rowoff = (size_t)row * d.Wpad * CP;
        const __bf16* vrow = v + rowoff;
        __bf16* orow = vout + rowoff;
        // (with DFT, the barrier of the previous row's DFT already keeps these writes
        // of zs behind every wave's reads of it, and the barrier in stage_z keeps this
        // row's writes of vt behind every wave's reads of the previous row)
        stage_z(d, b, h, zs);
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int t = wave + u * nw;
            if (t >= T) break;
            const int mi = t / Nt;
            bf16x8 za[KZ], vb[KC];
            load_rows<KZ>(za, zs + ni * 32 * KKs, KKs);
            load_rows<KC>(vb, vrow + mi * 32 * CP, CP);
            f32x16 acc = {};
            acc = mma_rows<KZ>(za, bi[u], acc);
            acc = mma_rows<KC>(wc, vb, acc);
            const int w = mi * 32 + wl;
            const bool live = w < d.Wp;
            const uint32_t lmask = live ? 0xffffffffu : 0u;
            float val[16];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                val[4 * j + 0] = acc[4 * j + 0] + bq[j].x;
                val[4 * j + 1] = acc[4 * j + 1] + bq[j].y;
                val[4 * j + 2] = acc[4 * j + 2] + bq[j].z;
                val[4 * j + 3] = acc[4 * j + 3] + bq[j].w;
            }
            if (d.sv_pre) {   // training: the pre-activation, zero beyond W'
                float* sp = d.sv_pre + rowoff + (size_t)w * CP + ob;
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    *reinterpret_cast<float4*>(sp + 8 * j) =
                        live ? make_float4(val[4 * j], val[4 * j + 1], val[4 * j + 2], val[4 * j + 3])
                             : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            }
            __bf16* op = orow + w * CP + ob;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                uint2 q;
                // every lane evaluates the activations and a mask clears the points beyond W'
                // (a select on the packed words would put each pair behind its own branch,
                // and the sixteen evaluations could not be interleaved)
                q.x = pack_bf16(act_t<ACT>(val[4 * j + 0]), act_t<ACT>(val[4 * j + 1])) & lmask;
                q.y = pack_bf16(act_t<ACT>(val[4 * j + 2]), act_t<ACT>(val[4 * j + 3])) & lmask;
                if constexpr (DFT) {
                    __bf16* vc = vt + (ob + 8 * j) * VS + w;
                    const __bf16* e = reinterpret_cast<const __bf16*>(&q);
                    vc[0] = e[0];
                    vc[VS] = e[1];
                    vc[2 * VS] = e[2];
                    vc[3 * VS] = e[3];
                } else {
                    *reinterpret_cast<uint2*>(op + 8 * j) = q;
                }
            }
        }
        if constexpr (DFT) {
            __syncthreads();
            if (dft_wave) row_dft_regs<KW>(d, ew, vt, b, h);
            store_row_from_vt(d, vt, orow);
        } else {
            __syncthreads();  // every wave's reads of zs before the next row's stage_z
        }
    }
}

// Decoder on MFMA.  Each wave takes 32 consecutive output points; a layer's input
// (bf16, channels contiguous) sits in LDS and is multiplied by the layer's
// [DSP][din_p] weights, both operands contiguous along the input channels; bias,
// activation and the bf16 rounding run in the accumulator epilogue, which writes
// the next layer's input back to LDS.  The output layer (cout <= 8 rows) is a
// per-point dot product over the last LDS row (float32 out).
constexpr int DEC_PTS = 32;

// (point indices fit 32 bits: B Hp Wpad CP < 2^31 is checked on the host)
__device__ __forceinline__ size_t dec_point_offset(const FnoDev& d, size_t pt) {
    const unsigned p = (unsigned)pt, r = p / (unsigned)d.W, w = p - r * d.W;
    const unsigned b = r / (unsigned)d.H, h = r - b * d.H;
    return ((size_t)b * d.Hp + h) * d.Wpad + w;
}

__device__ __forceinline__ size_t dec_out_offset(const FnoDev& d, size_t pt, int o) {
    const unsigned p = (unsigned)pt, hw = (unsigned)d.H * d.W, b = p / hw;
    return ((size_t)b * d.cout + o) * hw + (p - b * hw);
}

__device__ __forceinline__ void dec_stage_input(const FnoDev& d, const __bf16* __restrict__ v,
                                                size_t pt0, size_t total, __bf16* buf, int lane) {
    const int c8n = d.CP / 8;
    for (int e = lane; e < DEC_PTS * c8n; e += 64) {
        const int pp = e / c8n, c8 = e % c8n;
        const size_t pt = pt0 + pp;
        bf16x8 t;
        if (pt < total) {
            t = *reinterpret_cast<const bf16x8*>(v + dec_point_offset(d, pt) * d.CP + 8 * c8);
        } else {
#pragma unroll
            for (int k = 0; k < 8; ++k) t[k] = to_bf16(0.0f);
        }
        *reinterpret_cast<bf16x8*>(buf + pp * d.DKP + 8 * c8) = t;
    }
}

// One hidden decoder layer for the wave's 32 points: out[pt][su] = act(W[su][:] .
// in[pt][:] + b[su]) for su < dec_size (zero for the padded units), formed
// transposed so that a lane holds four consecutive units of one point and writes
// them as one 8-byte bf16 quad.  With sv != NULL (training) the pre-activations
// go to sv[pt][su] (float, DSP per point) for points below `valid`.
// Mask of a packed bf16 pair (units u, u + 1) that keeps the units below n.
__device__ __forceinline__ uint32_t unit_mask(int u, int n) {
    return (u < n ? 0x0000ffffu : 0u) | (u + 1 < n ? 0xffff0000u : 0u);
}

template <int ACT>
__device__ __forceinline__ void dec_hidden_layer(const FnoDev& d, const __bf16* in, __bf16* outb, int KP,
                                                 const __bf16* wp, const float* bp, int din, float* sv,
                                                 int valid) {
    const int lane = threadIdx.x & 63, pt = lane & 31, g = lane >> 5;
    for (int nt = 0; nt < d.DSP / 32; ++nt) {
        f32x16 acc = {};
        const __bf16* A = wp + (size_t)nt * 32 * din;
        if (din == 32) acc = mma_k<2>(A, din, in, KP, acc);
        else if (din == 64) acc = mma_k<4>(A, din, in, KP, acc);
        else acc = mma_tile(A, din, in, KP, din, acc);
        const int sb = nt * 32 + 4 * g;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int su = sb + 8 * j;
            const float4 bq = *reinterpret_cast<const float4*>(bp + su);
            const float x0 = acc[4 * j] + bq.x, x1 = acc[4 * j + 1] + bq.y;
            const float x2 = acc[4 * j + 2] + bq.z, x3 = acc[4 * j + 3] + bq.w;
            if (sv && pt < valid) *reinterpret_cast<float4*>(sv + (size_t)pt * d.DSP + su) = make_float4(x0, x1, x2, x3);
            // the activations unconditionally, the padded units (su >= dec_size) cleared
            // by a bit mask afterwards, so that no activation sits behind a branch
            uint2 q;
            q.x = pack_bf16(act_t<ACT>(x0), act_t<ACT>(x1)) & unit_mask(su, d.dec_size);
            q.y = pack_bf16(act_t<ACT>(x2), act_t<ACT>(x3)) & unit_mask(su + 2, d.dec_size);
            *reinterpret_cast<uint2*>(outb + pt * KP + su) = q;
        }
    }
}

// Output weights of the decoder (cout <= 8 rows of din <= 64, bf16) staged in LDS
// as the A operand of one 32-row MFMA tile, rows cout..31 zero, and the output bias.
__device__ __forceinline__ int dec_stage_output(const FnoDev& d, __bf16* wo, float* bo) {
    const __bf16* wg = d.decw;
    const float* bg = d.decb;
    int dn = d.CP;
    for (int l = 0; l < d.dec_layers; ++l) {
        wg += (size_t)d.DSP * dn;
        bg += d.DSP;
        dn = d.DSP;
    }
    for (int t = threadIdx.x; t < 32 * dn; t += blockDim.x) wo[t] = t < d.cout * dn ? wg[t] : to_bf16(0.0f);
    for (int t = threadIdx.x; t < d.cout; t += blockDim.x) bo[t] = bg[t];
    return dn;
}

// Output layer for the wave's 32 points on MFMA, C^T[o][pt] = Wo[o][:] . in[pt][:]
// (bf16 operands, float32 sums, as the per-point dot products would form them up to
// the order of the sums): lane l holds outputs o = 4 (l / 32) + i of point l % 32 in
// acc[i], i = 0..3.
__device__ __forceinline__ f32x16 dec_output_layer(const __bf16* wo, const __bf16* in, int KP, int din) {
    f32x16 acc = {};
    if (din == 32) acc = mma_k<2>(wo, din, in, KP, acc);
    else if (din == 64) acc = mma_k<4>(wo, din, in, KP, acc);
    else acc = mma_tile(wo, din, in, KP, din, acc);
    return acc;
}

// ACT = d.dec_act.
template <int ACT>
__global__ __launch_bounds__(256) void k_fno_dec(FnoDev d, const __bf16* __restrict__ v,
                                                 float* __restrict__ out) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int KP = d.DKP;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __bf16* bufA = reinterpret_cast<__bf16*>(smem) + (size_t)wave * 2 * DEC_PTS * KP;
    __bf16* bufB = bufA + DEC_PTS * KP;
    const size_t total = (size_t)d.B * d.H * d.W;
    const size_t pt0 = ((size_t)blockIdx.x * 4 + wave) * DEC_PTS;
    __shared__ __align__(16) __bf16 wo[32 * 64];
    __shared__ float bo[8];
    dec_stage_output(d, wo, bo);
    dec_stage_input(d, v, pt0, total, bufA, lane);
    __syncthreads();
    int din = d.CP;
    const __bf16* wp = d.decw;
    const float* bp = d.decb;
    for (int l = 0; l < d.dec_layers; ++l) {
        dec_hidden_layer<ACT>(d, bufA, bufB, KP, wp, bp, din,
                              d.sv_dec ? d.sv_dec + ((size_t)l * total + pt0) * d.DSP : nullptr,
                              (int)(pt0 < total ? total - pt0 : 0));
        __syncthreads();
        __bf16* t = bufA; bufA = bufB; bufB = t;
        wp += (size_t)d.DSP * din;
        bp += d.DSP;
        din = d.DSP;
    }
    const f32x16 acc = dec_output_layer(wo, bufA, KP, din);
    const size_t pt = pt0 + (lane & 31);
    if (pt < total) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int o = 4 * (lane >> 5) + i;
            if (o < d.cout) out[dec_out_offset(d, pt, o)] = acc[i] + bo[o];
        }
    }
}

// Inference: the last layer's row inverse (no activation, no next row DFT) fused
// with the decoder, one workgroup per interior row (b, h < H).  The row's output,
// rounded to bf16 exactly as the separate row inverse stores it, stays in LDS
// ([Wpad][DKP]) as the decoder's input, so the last activation never goes to global
// memory and the padded rows h >= H are not formed.  The waves take the row's
// 32-point groups in turn; every wave runs the same number of rounds and layers, so
// a wave without a group still meets every barrier.
template <int DACT, int KZ, int KC>
__global__ __launch_bounds__(256) void k_fno_rowinv_dec(FnoDev d, const __bf16* __restrict__ v,
                                                        float* __restrict__ out, int layer) {
    const int b = blockIdx.x / d.H, h = blockIdx.x % d.H;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, nw = blockDim.x >> 6;
    const int KP = d.DKP;
    const size_t rowoff = ((size_t)b * d.Hp + h) * d.Wpad * d.CP;
    const __bf16* vrow = v + rowoff;
    extern __shared__ __align__(16) unsigned char smem[];
    __bf16* zs = reinterpret_cast<__bf16*>(smem);                     // [CP][KKp + 8]
    __bf16* vr = zs + (size_t)d.CP * (d.KKp + 8);                     // [Wpad][DKP]
    __bf16* own = vr + (size_t)d.Wpad * KP + (size_t)wave * DEC_PTS * KP;  // [32][DKP] per wave
    __shared__ __align__(16) __bf16 wo[32 * 64];
    __shared__ float bo[8];
    dec_stage_output(d, wo, bo);
    stage_z(d, b, h, zs);  // ends with a barrier, which also covers wo and bo
    const int KKs = d.KKp + 8;
    const __bf16* Wc = d.Wc + (size_t)layer * d.CP * d.CP;
    const float* bias = d.bc + (size_t)layer * d.CP;
    const int Mt = d.Wpad / 32, Nt = d.CP / 32;
    const int wl = lane & 31, gq = lane >> 5;
    for (int t = wave; t < Mt * Nt; t += nw) {
        const int mi = t / Nt, ni = t % Nt;
        f32x16 acc = {};
        // transposed tile C^T[o][w], as k_fno_rowinv forms it (same values)
        acc = mma_any<KZ>(zs + ni * 32 * KKs, KKs, d.BinvT + mi * 32 * d.KKp, d.KKp, d.KKp, acc);
        acc = mma_any<KC>(Wc + ni * 32 * d.CP, d.CP, vrow + mi * 32 * d.CP, d.CP, d.CP, acc);
        const int w = mi * 32 + wl;
        const bool live = w < d.Wp;
        const int ob = ni * 32 + 4 * gq;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const float4 bq = *reinterpret_cast<const float4*>(bias + ob + 8 * j);
            uint2 q;
            q.x = live ? pack_bf16(acc[4 * j] + bq.x, acc[4 * j + 1] + bq.y) : 0u;
            q.y = live ? pack_bf16(acc[4 * j + 2] + bq.z, acc[4 * j + 3] + bq.w) : 0u;
            *reinterpret_cast<uint2*>(vr + (size_t)w * KP + ob + 8 * j) = q;
        }
    }
    __syncthreads();
    const int ng = (d.W + DEC_PTS - 1) / DEC_PTS, rounds = (ng + nw - 1) / nw;
    for (int rd = 0; rd < rounds; ++rd) {
        const int g = rd * nw + wave;
        const bool live = g < ng;  // uniform over the wave
        __bf16* bufA = vr + (size_t)(live ? g : 0) * DEC_PTS * KP;
        __bf16* bufB = own;
        int din = d.CP;
        const __bf16* wp = d.decw;
        const float* bp = d.decb;
        for (int l = 0; l < d.dec_layers; ++l) {
            if (live) dec_hidden_layer<DACT>(d, bufA, bufB, KP, wp, bp, din, nullptr, 0);
            __syncthreads();
            __bf16* t = bufA; bufA = bufB; bufB = t;
            wp += (size_t)d.DSP * din;
            bp += d.DSP;
            din = d.DSP;
        }
        if (live) {
            const f32x16 acc = dec_output_layer(wo, bufA, KP, din);
            const int w = g * DEC_PTS + (lane & 31);
            if (w < d.W) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int o = 4 * (lane >> 5) + i;
                    if (o < d.cout) out[(((size_t)b * d.cout + o) * d.H + h) * d.W + w] = acc[i] + bo[o];
                }
            }
        }
        __syncthreads();  // this round's reads of own / vr before the next round's writes
    }
}

// Decoder hidden-layer weights ([DSP][din] per layer, bf16) and biases (float)
// in elements, as the persistent fused decoder stages them in LDS.
__host__ __device__ __forceinline__ int dec_hidden_weights(const FnoDev& d) {
    return d.dec_layers > 0 ? d.DSP * d.CP + (d.dec_layers - 1) * d.DSP * d.DSP : 0;
}

// The fused last row inverse + decoder as a persistent kernel (same conditions on
// the row shape as k_fno_rowinv_p): the workgroups step through the rows, the
// decoder's weights and biases are staged in LDS once per workgroup, and each wave
// keeps its row-inverse operands (Wc rows, BinvT rows of its two point tiles, the
// bias) in registers.  Same products in the same order as k_fno_rowinv_dec.
template <int DACT, int KZ, int KC>
__global__ __launch_bounds__(256) void k_fno_rowinv_dec_p(FnoDev d, const __bf16* __restrict__ v,
                                                          float* __restrict__ out, int layer) {
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, nw = blockDim.x >> 6;
    const int KP = d.DKP, CP = d.CP;
    extern __shared__ __align__(16) unsigned char smem[];
    __bf16* zs = reinterpret_cast<__bf16*>(smem);                     // [CP][KKp + 8]
    __bf16* vr = zs + (size_t)CP * (d.KKp + 8);                       // [Wpad][DKP]
    __bf16* own = vr + (size_t)d.Wpad * KP + (size_t)wave * DEC_PTS * KP;  // [32][DKP] per wave
    __bf16* dw = vr + (size_t)d.Wpad * KP + (size_t)nw * DEC_PTS * KP;    // hidden weights
    float* db = reinterpret_cast<float*>(dw + dec_hidden_weights(d));      // hidden biases
    __shared__ __align__(16) __bf16 wo[32 * 64];
    __shared__ float bo[8];
    dec_stage_output(d, wo, bo);
    for (int i = tid; i < dec_hidden_weights(d); i += blockDim.x) dw[i] = d.decw[i];
    for (int i = tid; i < d.dec_layers * d.DSP; i += blockDim.x) db[i] = d.decb[i];
    const int KKs = d.KKp + 8;
    const int Mt = d.Wpad / 32, Nt = CP / 32, T = Mt * Nt;
    const int wl = lane & 31, gq = lane >> 5;
    const int ni = wave % Nt;  // both tiles of the wave (nw is a multiple of Nt)
    const int ob = ni * 32 + 4 * gq;
    bf16x8 wc[KC], bi[2][KZ];
    load_rows<KC>(wc, d.Wc + ((size_t)layer * CP + ni * 32) * CP, CP);
#pragma unroll
    for (int u = 0; u < 2; ++u)
        if (wave + u * nw < T) load_rows<KZ>(bi[u], d.BinvT + ((wave + u * nw) / Nt) * 32 * d.KKp, d.KKp);
    const float* bias = d.bc + (size_t)layer * CP + ob;
    const int ng = (d.W + DEC_PTS - 1) / DEC_PTS, rounds = (ng + nw - 1) / nw;
    const int rows = d.B * d.H;
    for (int row = blockIdx.x; row < rows; row += gridDim.x) {
        const int b = row / d.H, h = row - b * d.H;
        const __bf16* vrow = v + ((size_t)b * d.Hp + h) * d.Wpad * CP;
        // the barrier in stage_z also covers the staged weights (first row) and keeps
        // this row's writes of vr behind every wave's reads of the previous row
        stage_z(d, b, h, zs);
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int t = wave + u * nw;
            if (t >= T) break;
            const int mi = t / Nt;
            bf16x8 za[KZ], vb[KC];
            load_rows<KZ>(za, zs + ni * 32 * KKs, KKs);
            load_rows<KC>(vb, vrow + mi * 32 * CP, CP);
            f32x16 acc = {};
            acc = mma_rows<KZ>(za, bi[u], acc);
            acc = mma_rows<KC>(wc, vb, acc);
            const int w = mi * 32 + wl;
            const bool live = w < d.Wp;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float4 bqj = *reinterpret_cast<const float4*>(bias + 8 * j);
                uint2 q;
                q.x = live ? pack_bf16(acc[4 * j] + bqj.x, acc[4 * j + 1] + bqj.y) : 0u;
                q.y = live ? pack_bf16(acc[4 * j + 2] + bqj.z, acc[4 * j + 3] + bqj.w) : 0u;
                *reinterpret_cast<uint2*>(vr + (size_t)w * KP + ob + 8 * j) = q;
            }
        }
        __syncthreads();
        for (int rd = 0; rd < rounds; ++rd) {
            const int g = rd * nw + wave;
            const bool live = g < ng;  // uniform over the wave
            __bf16* bufA = vr + (size_t)(live ? g : 0) * DEC_PTS * KP;
            __bf16* bufB = own;
            int din = CP;
            const __bf16* wp = dw;
            const float* bp = db;
            for (int l = 0; l < d.dec_layers; ++l) {
                if (live) dec_hidden_layer<DACT>(d, bufA, bufB, KP, wp, bp, din, nullptr, 0);
                __syncthreads();
                __bf16* t = bufA; bufA = bufB; bufB = t;
                wp += (size_t)d.DSP * din;
                bp += d.DSP;
                din = d.DSP;
            }
            if (live) {
                const f32x16 acc = dec_output_layer(wo, bufA, KP, din);
                const int w = g * DEC_PTS + wl;
                if (w < d.W) {
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int o = 4 * gq + i;
                        if (o < d.cout) out[(((size_t)b * d.cout + o) * d.H + h) * d.W + w] = acc[i] + bo[o];
                    }
                }
            }
            __syncthreads();  // this round's reads of own / vr before the next writes
        }
    }
}

}  // namespace lbmfno

// ------------------------------------------------------------ host side

using namespace lbmfno;

struct fno_model {
    fno_spec spec;
    FnoDev d;            // sizes and parameter pointers (workspace filled per call)
    std::vector<void*> allocs;
    int device;
    int64_t nparams;
    // device index maps: element j of a device weight array takes packed parameter
    // map[j] (or 0 when map[j] < 0); used to refresh weights from device params
    struct Map { void* dst; const int32_t* map; int64_t n; bool bf16; };
    std::vector<Map> maps;
    // replayable forward: the launches of one (input, output, B, workspace) tuple
    // captured once on a private stream
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t fwd_exec = nullptr;
    const void* g_in = nullptr;
    const void* g_out = nullptr;
    const void* g_ws = nullptr;
    int32_t g_B = 0;
};

static int rup(int x, int m) { return (x + m - 1) / m * m; }

// dynamic LDS of the decoder kernels: 4 waves x (two bf16 rows of 32 points) or
// (one bf16 + one float row of 32 points)
static size_t dec_lds(const FnoDev& d) { return (size_t)4 * 2 * DEC_PTS * d.DKP * 2; }
static size_t dec_bwd_lds(const FnoDev& d) { return (size_t)4 * DEC_PTS * d.DKP * (2 + 4); }
// Host dispatch of a run-time activation kind to the template argument A.
#define FNO_WITH_ACT(kind, ...)                                                  \
    switch (kind) {                                                              \
        case FNO_ACT_GELU: { constexpr int A = FNO_ACT_GELU; __VA_ARGS__; break; } \
        case FNO_ACT_RELU: { constexpr int A = FNO_ACT_RELU; __VA_ARGS__; break; } \
        case FNO_ACT_SILU: { constexpr int A = FNO_ACT_SILU; __VA_ARGS__; break; } \
        default: { constexpr int A = FNO_ACT_IDENTITY; __VA_ARGS__; break; }        \
    }

// The lift kernels' template arguments: NO = CP (32 or 64), KH = 16 when
// half <= 16, else 32.
#define FNO_WITH_LIFT(dev, ...)                                                                   \
    if ((dev).CP <= 32) { constexpr int NO = 32, KH = 16; __VA_ARGS__; }                         \
    else if ((dev).half <= 16) { constexpr int NO = 64, KH = 16; __VA_ARGS__; }                  \
    else { constexpr int NO = 64, KH = 32; __VA_ARGS__; }

// lift over npts padded points (a wave per 64 points)
static void launch_lift(const FnoDev& d, size_t npts, const float* d_in, hipStream_t st) {
    const unsigned grid = (unsigned)((npts + 255) / 256);
    FNO_WITH_LIFT(d, FNO_WITH_ACT(d.act, (k_fno_lift<NO, A, KH><<<grid, 256, 0, st>>>(d, d_in))));
}

// dynamic LDS of the row-inverse kernels: the row's Z transposed, [CP][KKp + 8] bf16
static size_t zs_lds(const FnoDev& d) { return (size_t)d.CP * (d.KKp + 8) * 2; }

// whether the row inverse can also hold the output row for the next row DFT in LDS
static bool fuse_row_dft(const FnoDev& d) {
    return zs_lds(d) + (size_t)d.CP * vt_stride(d) * 2 <= 64 * 1024;
}

// Host dispatch of the row-inverse contraction sizes to template constants KZ
// (KKp / 16: 2 or 4, else 0 for a run-time loop) and KC (CP / 16: 2 or 4).
#define FNO_WITH_K(dev, ...)                                                           \
    if ((dev).KKp == 32 && (dev).CP == 32) { constexpr int KZ = 2, KC = 2; __VA_ARGS__; }      \
    else if ((dev).KKp == 64 && (dev).CP == 32) { constexpr int KZ = 4, KC = 2; __VA_ARGS__; } \
    else if ((dev).KKp == 32 && (dev).CP == 64) { constexpr int KZ = 2, KC = 4; __VA_ARGS__; } \
    else if ((dev).KKp == 64 && (dev).CP == 64) { constexpr int KZ = 4, KC = 4; __VA_ARGS__; } \
    else if ((dev).CP == 32) { constexpr int KZ = 0, KC = 2; __VA_ARGS__; }                     \
    else { constexpr int KZ = 0, KC = 4; __VA_ARGS__; }

// KZ, KC both compile-time (the persistent row inverse)
#define FNO_WITH_KZC(dev, ...)                                                                  \
    if ((dev).KKp == 32 && (dev).CP == 32) { constexpr int KZ = 2, KC = 2; __VA_ARGS__; }      \
    else if ((dev).KKp == 64 && (dev).CP == 32) { constexpr int KZ = 4, KC = 2; __VA_ARGS__; } \
    else if ((dev).KKp == 32 && (dev).CP == 64) { constexpr int KZ = 2, KC = 4; __VA_ARGS__; } \
    else { constexpr int KZ = 4, KC = 4; __VA_ARGS__; }

// A persistent row kernel over `rows` rows: as many 256-thread workgroups as fit on
// the device at once (the occupancy the runtime reports for this kernel and LDS
// size, times the compute units), at most one per row.
// The runtime's occupancy query, remembered per (kernel, block size, LDS size): the
// forward asks it for every persistent launch.
static int blocks_per_cu(const void* kernel, unsigned threads, size_t lds) {
    static std::mutex mu;
    static std::vector<std::pair<std::tuple<const void*, unsigned, size_t>, int>> seen;
    const auto key = std::make_tuple(kernel, threads, lds);
    {
        std::lock_guard<std::mutex> g(mu);
        for (const auto& e : seen)
            if (e.first == key) return e.second;
    }
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, (int)threads, lds) != hipSuccess || per < 1)
        per = 1;
    std::lock_guard<std::mutex> g(mu);
    seen.emplace_back(key, per);
    return per;
}

template <typename... P, typename... Args>
static void launch_persistent(void (*kernel)(P...), const FnoDev& d, size_t lds, unsigned rows, hipStream_t st,
                              unsigned threads, Args... args) {
    const int per = blocks_per_cu(reinterpret_cast<const void*>(kernel), threads, lds);
    const unsigned grid = std::min(rows, (unsigned)(per * d.ncu));
    kernel<<<grid, threads, lds, st>>>(d, args...);
}

// whether the persistent row inverse applies: compile-time k-steps, at most two
// 32 x 32 tiles per wave and, with the fused row DFT, at most one row-DFT tile per
// wave and a row of 160 or 256 points
static bool rowinv_persistent(const FnoDev& d, bool dft) {
    const bool kzc = (d.KKp == 32 || d.KKp == 64) && (d.CP == 32 || d.CP == 64);
    const bool tiles = (d.Wpad / 32) * (d.CP / 32) <= 8;
    return kzc && tiles && (!dft || (row_dft_tiles(d) <= 4 && (d.Wpad == 256 || d.Wpad == 160)));
}

// row inverse of layer l over all (b, h) rows; the last layer has no activation,
// the others also take the next layer's row DFT when it fits (fuse_row_dft)
static void launch_rowinv(const FnoDev& d, const __bf16* v, __bf16* vout, int l, hipStream_t st) {
    const unsigned grid = (unsigned)(d.B * d.Hp);
    if (l < d.L - 1 && fuse_row_dft(d)) {
        const size_t lds = zs_lds(d) + (size_t)d.CP * vt_stride(d) * 2;
        if (rowinv_persistent(d, true) && d.Wpad == 256) {
            FNO_WITH_KZC(d, FNO_WITH_ACT(d.act, (launch_persistent(k_fno_rowinv_p<A, true, KZ, KC, 8>, d, lds, grid, st, 256u, v, vout, l))))
        } else if (rowinv_persistent(d, true) && d.Wpad == 160) {
            FNO_WITH_KZC(d, FNO_WITH_ACT(d.act, (launch_persistent(k_fno_rowinv_p<A, true, KZ, KC, 5>, d, lds, grid, st, 256u, v, vout, l))))
        } else {
            FNO_WITH_K(d, FNO_WITH_ACT(d.act, (k_fno_rowinv<A, true, KZ, KC><<<grid, 256, lds, st>>>(d, v, vout, l))))
        }
    } else if (rowinv_persistent(d, false)) {
        FNO_WITH_KZC(d, FNO_WITH_ACT(l == d.L - 1 ? FNO_ACT_IDENTITY : d.act,
                                     (launch_persistent(k_fno_rowinv_p<A, false, KZ, KC, 1>, d, zs_lds(d), grid, st,
                                                        256u, v, vout, l))))
    } else {
        FNO_WITH_K(d, FNO_WITH_ACT(l == d.L - 1 ? FNO_ACT_IDENTITY : d.act,
                                   (k_fno_rowinv<A, false, KZ, KC><<<grid, 256, zs_lds(d), st>>>(d, v, vout, l))))
    }
}

static size_t dec_lds(const FnoDev& d);

static void launch_dec(const FnoDev& d, const __bf16* v, float* out, hipStream_t st) {
    const size_t nout = (size_t)d.B * d.H * d.W;
    const unsigned grid = (unsigned)((nout + 4 * DEC_PTS - 1) / (4 * DEC_PTS));
    FNO_WITH_ACT(d.dec_act, (k_fno_dec<A><<<grid, 256, dec_lds(d), st>>>(d, v, out)))
}

// dynamic LDS of the fused last row inverse + decoder: the row's Z, its output row
// [Wpad][DKP] and one [32][DKP] buffer per wave (static: the output layer, 1 KB)
static size_t rowinv_dec_lds(const FnoDev& d) {
    return zs_lds(d) + (size_t)d.Wpad * d.DKP * 2 + (size_t)4 * DEC_PTS * d.DKP * 2;
}
static bool fuse_dec(const FnoDev& d) {
    return !d.sv_pre && !d.sv_dec && rowinv_dec_lds(d) + 32 * 64 * 2 + 64 <= 64 * 1024;
}
static void launch_rowinv_dec(const FnoDev& d, const __bf16* v, float* out, int l, hipStream_t st) {
    const unsigned grid = (unsigned)(d.B * d.H);
    const size_t lds_p = rowinv_dec_lds(d) + (size_t)dec_hidden_weights(d) * 2 + (size_t)d.dec_layers * d.DSP * 4;
    if (rowinv_persistent(d, false) && lds_p + 32 * 64 * 2 + 64 <= 64 * 1024) {
        FNO_WITH_KZC(d, FNO_WITH_ACT(d.dec_act, (launch_persistent(k_fno_rowinv_dec_p<A, KZ, KC>, d, lds_p, grid, st,
                                                                   256u, v, out, l))));
    } else {
        FNO_WITH_K(d, FNO_WITH_ACT(d.dec_act, (k_fno_rowinv_dec<A, KZ, KC><<<grid, 256, rowinv_dec_lds(d), st>>>(d, v, out, l))))
    }
}

// dynamic LDS of the column kernel: xs [R2][CP] float, ys [CP][R2] bf16 and, when
// its K range is split over spare waves, S - 1 float partials of xs
static size_t col_lds_parts(const FnoDev& d, int S) {
    return (size_t)d.CP * ts_stride(d) * 2 + (size_t)d.R2 * d.CP * (4 + 2) +
           (size_t)(S - 1) * d.R2 * d.CP * 4;
}

// K-split of the column DFT: spare waves (fewer 32 x 32 tiles than waves) take
// parts of the K range, as many as the 64 KB of LDS leave room for.
static int col_split(const FnoDev& d) {
    const int T1 = (d.R2 / 32) * (d.CP / 32), nw = COL_THREADS / 64;
    int S = T1 >= nw ? 1 : nw / T1;
    while (S > 1 && col_lds_parts(d, S) > 64 * 1024) --S;
    return S;
}

static size_t col_lds(const FnoDev& d) { return col_lds_parts(d, d.colS); }

static uint16_t host_bf16(double v) {
    float f = (float)v;
    uint32_t u;
    std::memcpy(&u, &f, 4);
    if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)(u >> 16);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

static int64_t count_params(const fno_spec* s) {
    const int64_t cl = s->cin + (s->coords ? 2 : 0), h = s->width / 2, wd = s->width;
    int64_t n = cl * h + h + h * wd + wd;
    n += (int64_t)s->layers * (4 * wd * wd * s->m1 * s->m2 + wd * wd + wd);
    int64_t din = wd;
    for (int l = 0; l < s->dec_layers; ++l) {
        n += (int64_t)s->dec_size * din + s->dec_size;
        din = s->dec_size;
    }
    n += (int64_t)s->cout * din + s->cout;
    return n;
}

static int validate_spec(const fno_spec* s) {
    if (!s) return fail(LBM_EINVAL, "spec is NULL");
    if (s->cin < 1 || s->cin > 6) return fail(LBM_EINVAL, "cin = %d (1..6)", s->cin);
    if (s->width < 2 || s->width > 64 || s->width % 2) return fail(LBM_EINVAL, "width = %d (even, 2..64)", s->width);
    if (s->layers < 1 || s->layers > 32) return fail(LBM_EINVAL, "layers = %d", s->layers);
    if (s->m1 < 1 || s->m2 < 1 || s->m1 > 64 || s->m2 > 64) return fail(LBM_EINVAL, "modes %d x %d", s->m1, s->m2);
    if (s->dec_layers < 0 || s->dec_layers > 4) return fail(LBM_EINVAL, "dec_layers = %d", s->dec_layers);
    if (s->dec_layers > 0 && (s->dec_size < 1 || s->dec_size > 64)) return fail(LBM_EINVAL, "dec_size = %d (1..64)", s->dec_size);
    if (s->cout < 1 || s->cout > 8) return fail(LBM_EINVAL, "cout = %d", s->cout);
    if (s->padding < 0 || s->padding > 64) return fail(LBM_EINVAL, "padding = %d", s->padding);
    if (s->coords != 0 && s->coords != 1) return fail(LBM_EINVAL, "coords = %d", s->coords);
    if (s->act < 0 || s->act > 3 || s->dec_act < 0 || s->dec_act > 3) return fail(LBM_EINVAL, "activation code");
    return LBM_OK;
}

extern "C" int fno_param_count(const fno_spec* spec, int64_t* count) {
    int rc = validate_spec(spec);
    if (rc) return rc;
    if (!count) return fail(LBM_EINVAL, "count is NULL");
    *count = count_params(spec);
    return LBM_OK;
}

extern "C" void fno_model_destroy(fno_model* m) {
    if (!m) return;
    if (m->fwd_exec) (void)hipGraphExecDestroy(m->fwd_exec);
    if (m->cap_stream) (void)hipStreamDestroy(m->cap_stream);
    for (void* p : m->allocs) (void)hipFree(p);
    delete m;
}

template <typename T>
static int upload(fno_model* m, const std::vector<T>& h, const T** out) {
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, std::max<size_t>(h.size(), 1) * sizeof(T));
    if (e != hipSuccess) return fail(LBM_ENOMEM, "hipMalloc: %s", hipGetErrorString(e));
    m->allocs.push_back(p);
    if (!h.empty()) {
        e = hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
        if (e != hipSuccess) return fail(LBM_EHIP, "hipMemcpy: %s", hipGetErrorString(e));
    }
    *out = reinterpret_cast<const T*>(p);
    return LBM_OK;
}

// The forward mixing layout of the spectral weights: (o, i) of every [CP][CP][2]
// block of the backward layout swapped.
template <typename T>
static std::vector<T> mix_transpose(const std::vector<T>& a, int CP) {
    std::vector<T> t(a.size());
    const size_t blk = (size_t)CP * CP * 2;
    for (size_t b0 = 0; b0 < a.size(); b0 += blk)
        for (int o = 0; o < CP; ++o)
            for (int i = 0; i < CP; ++i)
                for (int ri = 0; ri < 2; ++ri)
                    t[b0 + ((size_t)i * CP + o) * 2 + ri] = a[b0 + ((size_t)o * CP + i) * 2 + ri];
    return t;
}

static int build_param_maps(fno_model* m, const FnoDev& d) {
    const fno_spec& s = m->spec;
    const int wd = s.width, CP = d.CP, half = d.half, cl = d.cl;
    int64_t off = 0;
    const int64_t o_l1w = off; off += (int64_t)half * cl;
    const int64_t o_l1b = off; off += half;
    const int64_t o_l2w = off; off += (int64_t)wd * half;
    const int64_t o_l2b = off; off += wd;
    std::vector<int32_t> l1w(half * cl), l1b(half), l2w(wd * half), l2b(wd);
    for (int i = 0; i < half * cl; ++i) l1w[i] = (int32_t)(o_l1w + i);
    for (int i = 0; i < half; ++i) l1b[i] = (int32_t)(o_l1b + i);
    for (int i = 0; i < wd * half; ++i) l2w[i] = (int32_t)(o_l2w + i);
    for (int i = 0; i < wd; ++i) l2b[i] = (int32_t)(o_l2b + i);
    std::vector<int32_t> Rm((size_t)s.layers * s.m2 * d.K1 * CP * CP * 2, -1);
    std::vector<int32_t> Wc((size_t)s.layers * CP * CP, -1), WcT((size_t)s.layers * CP * CP, -1);
    std::vector<int32_t> bc((size_t)s.layers * CP, -1);
    const int64_t blk = (int64_t)wd * wd * s.m1 * s.m2 * 2;
    for (int l = 0; l < s.layers; ++l) {
        const int64_t top = off, bot = off + blk;
        off += 2 * blk;
        for (int i = 0; i < wd; ++i)
            for (int o = 0; o < wd; ++o)
                for (int a = 0; a < s.m1; ++a)
                    for (int k2 = 0; k2 < s.m2; ++k2)
                        for (int ri = 0; ri < 2; ++ri) {
                            const int64_t src = ((((int64_t)i * wd + o) * s.m1 + a) * s.m2 + k2) * 2 + ri;
                            for (int hf = 0; hf < 2; ++hf) {
                                const int k = hf * s.m1 + a;
                                const size_t dst = (((((size_t)l * s.m2 + k2) * d.K1 + k) * CP + o) * CP + i) * 2 + ri;
                                Rm[dst] = (int32_t)((hf ? bot : top) + src);
                            }
                        }
        for (int o = 0; o < wd; ++o)
            for (int i = 0; i < wd; ++i) {
                Wc[((size_t)l * CP + o) * CP + i] = (int32_t)(off + o * wd + i);
                WcT[((size_t)l * CP + i) * CP + o] = (int32_t)(off + o * wd + i);
            }
        off += (int64_t)wd * wd;
        for (int o = 0; o < wd; ++o) bc[(size_t)l * CP + o] = (int32_t)(off + o);
        off += wd;
    }
    std::vector<int32_t> decw, decb, decwT;
    int din = wd, dinp = CP;
    for (int l = 0; l < s.dec_layers; ++l) {
        const size_t base = decw.size();
        decw.resize(base + (size_t)d.DSP * dinp, -1);
        const size_t tb = decwT.size();
        decwT.resize(tb + (size_t)dinp * d.DSP, -1);
        for (int o = 0; o < s.dec_size; ++o)
            for (int i = 0; i < din; ++i) {
                decw[base + (size_t)o * dinp + i] = (int32_t)(off + o * din + i);
                decwT[tb + (size_t)i * d.DSP + o] = (int32_t)(off + o * din + i);
            }
        off += (int64_t)s.dec_size * din;
        const size_t bb = decb.size();
        decb.resize(bb + d.DSP, -1);
        for (int o = 0; o < s.dec_size; ++o) decb[bb + o] = (int32_t)(off + o);
        off += s.dec_size;
        din = s.dec_size;
        dinp = d.DSP;
    }
    {
        const size_t base = decw.size();
        decw.resize(base + (size_t)s.cout * dinp, -1);
        for (int o = 0; o < s.cout; ++o)
            for (int i = 0; i < din; ++i) decw[base + (size_t)o * dinp + i] = (int32_t)(off + o * din + i);
        off += (int64_t)s.cout * din;
        for (int o = 0; o < s.cout; ++o) decb.push_back((int32_t)(off + o));
        off += s.cout;
    }
    m->nparams = off;
    std::vector<int32_t> RmT = mix_transpose(Rm, CP);
    struct Item { const void* dst; std::vector<int32_t>* v; bool bf; };
    Item items[] = {{d.lift1w, &l1w, false}, {d.lift1b, &l1b, false}, {d.lift2w, &l2w, false},
                    {d.lift2b, &l2b, false}, {d.Rmix, &Rm, true}, {d.RmixT, &RmT, true}, {d.Wc, &Wc, true},
                    {d.WcT, &WcT, true}, {d.bc, &bc, false}, {d.decw, &decw, true},
                    {d.decb, &decb, false}, {d.decwT, &decwT, true}};
    for (const Item& it : items) {
        const int32_t* dm = nullptr;
        int rc = upload(m, *it.v, &dm);
        if (rc) return rc;
        m->maps.push_back({const_cast<void*>(it.dst), dm, (int64_t)it.v->size(), it.bf});
    }
    return LBM_OK;
}

// ------------------------------------------- forward without any allocation
//
// fno_forward_noalloc runs fno_forward's kernels with their workspace in a
// file-scope device array instead of a caller buffer.  Each GPU the library runs
// on holds its own copy of the array until the process ends.  In host code the
// array's name is only a host-side stand-in: kernels receive the device address
// that hipGetSymbolAddress returned for that GPU, looked up once per device when
// the first model is created there (with that device current).
static __device__ __align__(256) unsigned char scratch[FNO_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
std::atomic<void*> g_scratch_ptr[kMaxDevices];
}  // namespace

// Device address of `scratch` on `device` (the current device), looked up once.
static int scratch_setup(int device) {
    if (device < 0 || device >= kMaxDevices)
        return fail(LBM_EUNSUPPORTED, "device index %d beyond %d", device, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[device].load()) return LBM_OK;
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(LBM_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", device,
                    hipGetErrorString(e));
    g_scratch_ptr[device].store(ptr);
    return LBM_OK;
}

extern "C" int fno_model_create(fno_model** out, const fno_spec* spec, const float* h_params,
                                int64_t nparams, int32_t H, int32_t W) {
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate_spec(spec);
    if (rc) return rc;
    if (!h_params) return fail(LBM_EINVAL, "h_params is NULL");
    if (nparams != count_params(spec))
        return fail(LBM_EINVAL, "nparams = %lld, spec needs %lld", (long long)nparams,
                    (long long)count_params(spec));
    if (H < 2 || W < 2 || H > 4096 || W > 4096) return fail(LBM_EINVAL, "grid %d x %d", H, W);
    const fno_spec& s = *spec;
    FnoDev d{};
    d.H = H; d.W = W;
    d.Hp = H + s.padding; d.Wp = W + s.padding;
    if (2 * s.m1 > d.Hp || 2 * s.m2 > d.Wp) return fail(LBM_EINVAL, "modes exceed the grid");
    d.Wpad = rup(d.Wp, 32);
    d.Hpad = rup(d.Hp, 16);
    d.width = s.width;
    d.CP = rup(s.width, 32);
    d.cin = s.cin;
    d.coords = s.coords;
    d.cl = s.cin + (s.coords ? 2 : 0);
    d.half = s.width / 2;
    d.L = s.layers;
    d.m1 = s.m1; d.m2 = s.m2;
    d.K1 = 2 * s.m1;
    d.R2 = rup(2 * d.K1, 32);
    d.KKp = rup(2 * s.m2, 32);
    d.dec_layers = s.dec_layers;
    d.dec_size = s.dec_size;
    d.DSP = s.dec_layers > 0 ? rup(s.dec_size, 32) : 0;
    d.DKP = std::max(d.CP, d.DSP) + 8;
    d.cout = s.cout;
    d.act = s.act; d.dec_act = s.dec_act;
    if ((size_t)d.CP * vt_stride(d) * 2 > 64 * 1024) return fail(LBM_EUNSUPPORTED, "row of %d x %d too large for LDS", d.Wpad, d.CP);
    d.colS = col_split(d);
    {
        int dev = 0, ncu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu <= 0)
            ncu = 256;
        d.ncu = ncu;
    }
    if (col_lds(d) > 64 * 1024) return fail(LBM_EUNSUPPORTED, "mode block too large for LDS");
    if (zs_lds(d) > 64 * 1024) return fail(LBM_EUNSUPPORTED, "row coefficients too large for LDS");
    fno_model* m = new (std::nothrow) fno_model();
    if (!m) return fail(LBM_ENOMEM, "model allocation");
    m->spec = s;
    (void)hipGetDevice(&m->device);
    auto bail = [&](int code) { fno_model_destroy(m); return code; };
    // set-up of fno_forward_noalloc's workspace on this device (once per device)
    if (int rc2 = scratch_setup(m->device)) return bail(rc2);

    // ---- unpack parameters (layout documented in lbmfno.h)
    const float* p = h_params;
    const int wd = s.width, CP = d.CP, half = d.half, cl = d.cl;
    std::vector<float> l1w(p, p + (size_t)half * cl); p += (size_t)half * cl;
    std::vector<float> l1b(p, p + half); p += half;
    std::vector<float> l2w(p, p + (size_t)wd * half); p += (size_t)wd * half;
    std::vector<float> l2b(p, p + wd); p += wd;
    std::vector<uint16_t> Rmix((size_t)s.layers * s.m2 * d.K1 * CP * CP * 2, 0);
    std::vector<uint16_t> Wc((size_t)s.layers * CP * CP, 0);
    std::vector<float> bc((size_t)s.layers * CP, 0.0f);
    const size_t blk = (size_t)wd * wd * s.m1 * s.m2 * 2;
    for (int l = 0; l < s.layers; ++l) {
        const float* top = p;
        const float* bot = p + blk;
        p += 2 * blk;
        for (int i = 0; i < wd; ++i)
            for (int o = 0; o < wd; ++o)
                for (int a = 0; a < s.m1; ++a)
                    for (int k2 = 0; k2 < s.m2; ++k2)
                        for (int ri = 0; ri < 2; ++ri) {
                            const size_t src = ((((size_t)i * wd + o) * s.m1 + a) * s.m2 + k2) * 2 + ri;
                            for (int half_ = 0; half_ < 2; ++half_) {
                                const int k = half_ * s.m1 + a;  // kept-row index
                                const size_t dst =
                                    (((((size_t)l * s.m2 + k2) * d.K1 + k) * CP + o) * CP + i) * 2 + ri;
                                Rmix[dst] = host_bf16(half_ ? bot[src] : top[src]);
                            }
                        }
        for (int o = 0; o < wd; ++o)
            for (int i = 0; i < wd; ++i) Wc[((size_t)l * CP + o) * CP + i] = host_bf16(p[o * wd + i]);
        p += (size_t)wd * wd;
        for (int o = 0; o < wd; ++o) bc[(size_t)l * CP + o] = p[o];
        p += wd;
    }
    std::vector<uint16_t> WcT((size_t)s.layers * CP * CP, 0);
    for (int l = 0; l < s.layers; ++l)
        for (int o = 0; o < CP; ++o)
            for (int i = 0; i < CP; ++i)
                WcT[((size_t)l * CP + i) * CP + o] = Wc[((size_t)l * CP + o) * CP + i];
    std::vector<uint16_t> decw;
    std::vector<float> decb;
    int din = wd, dinp = CP;
    for (int l = 0; l < s.dec_layers; ++l) {
        const size_t base = decw.size();
        decw.resize(base + (size_t)d.DSP * dinp, 0);
        for (int o = 0; o < s.dec_size; ++o)
            for (int i = 0; i < din; ++i) decw[base + (size_t)o * dinp + i] = host_bf16(p[o * din + i]);
        p += (size_t)s.dec_size * din;
        const size_t bb = decb.size();
        decb.resize(bb + d.DSP, 0.0f);
        for (int o = 0; o < s.dec_size; ++o) decb[bb + o] = p[o];
        p += s.dec_size;
        din = s.dec_size;
        dinp = d.DSP;
    }
    {
        const size_t base = decw.size();
        decw.resize(base + (size_t)s.cout * dinp, 0);
        for (int o = 0; o < s.cout; ++o)
            for (int i = 0; i < din; ++i) decw[base + (size_t)o * dinp + i] = host_bf16(p[o * din + i]);
        p += (size_t)s.cout * din;
        for (int o = 0; o < s.cout; ++o) decb.push_back(p[o]);
        p += s.cout;
    }
    // hidden decoder layers transposed: [din_p][DSP] per layer
    std::vector<uint16_t> decwT;
    {
        size_t base = 0;
        int dinp2 = CP;
        for (int l = 0; l < s.dec_layers; ++l) {
            const size_t tb = decwT.size();
            decwT.resize(tb + (size_t)dinp2 * d.DSP, 0);
            for (int o = 0; o < d.DSP; ++o)
                for (int i = 0; i < dinp2; ++i) decwT[tb + (size_t)i * d.DSP + o] = decw[base + (size_t)o * dinp2 + i];
            base += (size_t)d.DSP * dinp2;
            dinp2 = d.DSP;
        }
    }
    // ---- DFT bases (angles reduced exactly in integers, values in double, RNE to bf16)
    const double two_pi = 6.283185307179586476925286766559;
    std::vector<uint16_t> EwT((size_t)d.KKp * d.Wpad, 0), BinvT((size_t)d.Wpad * d.KKp, 0),
        B1((size_t)d.Wpad * d.KKp, 0);
    const double inv_hw = 1.0 / ((double)d.Hp * d.Wp);
    for (int k2 = 0; k2 < s.m2; ++k2)
        for (int w = 0; w < d.Wp; ++w) {
            const double ph = two_pi * (double)(((int64_t)k2 * w) % d.Wp) / d.Wp;
            const double c = std::cos(ph), sn = std::sin(ph);
            EwT[(size_t)(2 * k2) * d.Wpad + w] = host_bf16(c);
            EwT[(size_t)(2 * k2 + 1) * d.Wpad + w] = host_bf16(-sn);
            const double ck = (k2 == 0 ? 1.0 : 2.0) * inv_hw;
            BinvT[(size_t)w * d.KKp + 2 * k2] = host_bf16(ck * c);
            BinvT[(size_t)w * d.KKp + 2 * k2 + 1] = host_bf16(-ck * sn);
            B1[(size_t)w * d.KKp + 2 * k2] = host_bf16(c);
            B1[(size_t)w * d.KKp + 2 * k2 + 1] = host_bf16(-sn);
        }
    const int H2 = 2 * d.Hpad;
    std::vector<uint16_t> EcolA((size_t)d.R2 * H2, 0), EcolB((size_t)H2 * d.R2, 0);
    for (int k = 0; k < d.K1; ++k) {
        const int k1 = k < s.m1 ? k : d.Hp - s.m1 + (k - s.m1);
        for (int h = 0; h < d.Hp; ++h) {
            const double th = two_pi * (double)(((int64_t)k1 * h) % d.Hp) / d.Hp;
            const uint16_t c = host_bf16(std::cos(th)), sn = host_bf16(std::sin(th)),
                           msn = host_bf16(-std::sin(th));
            EcolA[(size_t)k * H2 + h] = c;
            EcolA[(size_t)k * H2 + d.Hpad + h] = sn;
            EcolA[(size_t)(d.K1 + k) * H2 + h] = msn;
            EcolA[(size_t)(d.K1 + k) * H2 + d.Hpad + h] = c;
            EcolB[(size_t)h * d.R2 + k] = c;
            EcolB[(size_t)h * d.R2 + d.K1 + k] = msn;
            EcolB[(size_t)(d.Hpad + h) * d.R2 + k] = sn;
            EcolB[(size_t)(d.Hpad + h) * d.R2 + d.K1 + k] = c;
        }
    }
    // ---- upload
    const float *f1, *f2, *f3, *f4, *f5, *f6;
    const uint16_t *u1, *u2, *u3, *u4, *u5, *u6, *u7, *u8, *u9, *u10, *u11;
    if ((rc = upload(m, l1w, &f1)) || (rc = upload(m, l1b, &f2)) || (rc = upload(m, l2w, &f3)) ||
        (rc = upload(m, l2b, &f4)) || (rc = upload(m, bc, &f5)) || (rc = upload(m, decb, &f6)) ||
        (rc = upload(m, Rmix, &u1)) || (rc = upload(m, Wc, &u2)) || (rc = upload(m, decw, &u3)) ||
        (rc = upload(m, EwT, &u4)) || (rc = upload(m, BinvT, &u5)) || (rc = upload(m, EcolA, &u6)) ||
        (rc = upload(m, EcolB, &u7)) || (rc = upload(m, WcT, &u8)) || (rc = upload(m, B1, &u9)) ||
        (rc = upload(m, decwT, &u10)) || (rc = upload(m, mix_transpose(Rmix, CP), &u11)))
        return bail(rc);
    d.lift1w = f1; d.lift1b = f2; d.lift2w = f3; d.lift2b = f4; d.bc = f5; d.decb = f6;
    d.Rmix = reinterpret_cast<const __bf16*>(u1);
    d.RmixT = reinterpret_cast<const __bf16*>(u11);
    d.Wc = reinterpret_cast<const __bf16*>(u2);
    d.decw = reinterpret_cast<const __bf16*>(u3);
    d.EwT = reinterpret_cast<const __bf16*>(u4);
    d.BinvT = reinterpret_cast<const __bf16*>(u5);
    d.EcolA = reinterpret_cast<const __bf16*>(u6);
    d.EcolB = reinterpret_cast<const __bf16*>(u7);
    d.WcT = reinterpret_cast<const __bf16*>(u8);
    d.B1 = reinterpret_cast<const __bf16*>(u9);
    d.decwT = reinterpret_cast<const __bf16*>(u10);
    int rc2 = build_param_maps(m, d);
    if (rc2) return bail(rc2);
    m->d = d;
    *out = m;
    return LBM_OK;
}

struct WsLayout {
    size_t v, T, Z, total;
};

static WsLayout ws_layout(const FnoDev& d, int B) {
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    WsLayout L;
    L.v = al((size_t)B * d.Hp * d.Wpad * d.CP * 2);
    L.T = al((size_t)B * d.m2 * d.CP * 2 * d.Hpad * 2);
    L.Z = al((size_t)B * 2 * d.m2 * d.Hp * d.CP * 2);
    L.total = 2 * L.v + L.T + L.Z;
    return L;
}

extern "C" int fno_workspace_size(const fno_model* m, int32_t B, size_t* bytes) {
    if (!m || !bytes) return fail(LBM_EINVAL, "NULL argument");
    if (B < 1) return fail(LBM_EINVAL, "B = %d", B);
    *bytes = ws_layout(m->d, B).total;
    return LBM_OK;
}

static int check_forward(const fno_model* m, const float* d_in, float* d_out, int32_t B,
                         void* d_ws, size_t ws_bytes) {
    if (!m) return fail(LBM_EINVAL, "model is NULL");
    if (!d_in || !d_out || !d_ws) return fail(LBM_EINVAL, "NULL device buffer");
    if (B < 1 || (int64_t)B * m->d.Hp * m->d.Wpad > ((int64_t)1 << 31) / 64)
        return fail(LBM_EINVAL, "B = %d", B);
    if ((uintptr_t)d_ws % 256) return fail(LBM_EINVAL, "workspace not 256-byte aligned");
    FnoDev d = m->d;
    d.B = B;
    const WsLayout L = ws_layout(d, B);
    if (ws_bytes < L.total) return fail(LBM_EINVAL, "workspace %zu < %zu bytes", ws_bytes, L.total);
    return LBM_OK;
}

// the forward's launches (arguments already checked)
static void launch_forward(const fno_model* m, const float* d_in, float* d_out, int32_t B,
                           void* d_ws, hipStream_t st) {
    FnoDev d = m->d;
    d.B = B;
    const WsLayout L = ws_layout(d, B);
    unsigned char* ws = static_cast<unsigned char*>(d_ws);
    d.v0 = reinterpret_cast<__bf16*>(ws);
    d.v1 = reinterpret_cast<__bf16*>(ws + L.v);
    d.T = reinterpret_cast<__bf16*>(ws + 2 * L.v);
    d.Z = reinterpret_cast<__bf16*>(ws + 2 * L.v + L.T);
    const size_t npts = (size_t)B * d.Hp * d.Wpad;
    const size_t lds_row = (size_t)d.CP * vt_stride(d) * 2;
    // the lift takes the first row DFT in the same kernel when a row fits one
    // workgroup (a lane per point) and the row in LDS
    const bool flift = !d.sv_a1 && d.Wpad <= 1024 && lds_row + 12 * 1024 <= 64 * 1024;
    if (flift) {
        const unsigned threads = (unsigned)rup(d.Wpad, 64), grid = (unsigned)(B * d.Hpad);
        // with the row-DFT operand held in registers (at most one row-DFT tile per
        // wave, rows of 160 or 256 points) the workgroups are persistent
        const int kw = row_dft_tiles(d) > (int)threads / 64 ? 0 : d.Wpad == 256 ? 8 : d.Wpad == 160 ? 5 : 0;
        if (kw == 8) {
            FNO_WITH_LIFT(d, FNO_WITH_ACT(d.act, (launch_persistent(k_fno_lift_row<NO, A, KH, 8>, d, lds_row, grid,
                                                                    st, threads, d_in))));
        } else if (kw == 5) {
            FNO_WITH_LIFT(d, FNO_WITH_ACT(d.act, (launch_persistent(k_fno_lift_row<NO, A, KH, 5>, d, lds_row, grid,
                                                                    st, threads, d_in))));
        } else {
            FNO_WITH_LIFT(d, FNO_WITH_ACT(d.act, (k_fno_lift_row<NO, A, KH, 0><<<grid, threads, lds_row, st>>>(d, d_in))));
        }
    } else {
        launch_lift(d, npts, d_in, st);
    }
    __bf16* cur = d.v0;
    __bf16* nxt = d.v1;
    // the first layer's row DFT (it also writes T's zero rows h >= Hp); with
    // fuse_row_dft the row inverse of each layer produces the next layer's row DFT
    const bool fused = fuse_row_dft(d);
    // the last layer's row inverse also runs the decoder when it fits (fuse_dec)
    const bool fdec = fuse_dec(d);
    for (int l = 0; l < d.L; ++l) {
        if ((l == 0 && !flift) || (l > 0 && !fused)) k_fno_rowfwd<<<B * d.Hpad, 256, lds_row, st>>>(d, cur);
        k_fno_col<<<B * d.m2, COL_THREADS, col_lds(d), st>>>(d, l);
        if (l == d.L - 1 && fdec) {
            launch_rowinv_dec(d, cur, d_out, l, st);
            return;
        }
        launch_rowinv(d, cur, nxt, l, st);
        __bf16* t = cur; cur = nxt; nxt = t;
    }
    launch_dec(d, cur, d_out, st);
}

extern "C" int fno_forward(const fno_model* m, const float* d_in, float* d_out, int32_t B,
                           void* d_ws, size_t ws_bytes, void* stream) {
    int rc = check_forward(m, d_in, d_out, B, d_ws, ws_bytes);
    if (rc) return rc;
    launch_forward(m, d_in, d_out, B, d_ws, (hipStream_t)stream);
    LBM_HIP(hipGetLastError());
    return LBM_OK;
}

extern "C" int fno_forward_graph(fno_model* m, const float* d_in, float* d_out, int32_t B,
                                 void* d_ws, size_t ws_bytes, void* stream) {
    int rc = check_forward(m, d_in, d_out, B, d_ws, ws_bytes);
    if (rc) return rc;
    if (!m->fwd_exec || m->g_in != d_in || m->g_out != d_out || m->g_ws != d_ws || m->g_B != B) {
        if (m->fwd_exec) {
            LBM_HIP(hipGraphExecDestroy(m->fwd_exec));
            m->fwd_exec = nullptr;
        }
        if (!m->cap_stream) LBM_HIP(hipStreamCreateWithFlags(&m->cap_stream, hipStreamNonBlocking));
        hipGraph_t graph = nullptr;
        LBM_HIP(hipStreamBeginCapture(m->cap_stream, hipStreamCaptureModeThreadLocal));
        launch_forward(m, d_in, d_out, B, d_ws, m->cap_stream);
        hipError_t e = hipStreamEndCapture(m->cap_stream, &graph);
        if (e != hipSuccess) return fail(LBM_EHIP, "graph capture: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&m->fwd_exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            m->fwd_exec = nullptr;
            return fail(LBM_EHIP, "graph instantiate: %s", hipGetErrorString(e));
        }
        m->g_in = d_in;
        m->g_out = d_out;
        m->g_ws = d_ws;
        m->g_B = B;
    }
    LBM_HIP(hipGraphLaunch(m->fwd_exec, (hipStream_t)stream));
    return LBM_OK;
}

// fno_forward on the static scratch array (see the set-up above fno_model_create).
extern "C" int fno_forward_noalloc(const fno_model* m, const float* d_in, float* d_out, int32_t B,
                                   void* stream) {
    if (!m) return fail(LBM_EINVAL, "model is NULL");
    if (!d_in || !d_out) return fail(LBM_EINVAL, "NULL device buffer");
    if (B < 1 || (int64_t)B * m->d.Hp * m->d.Wpad > ((int64_t)1 << 31) / 64)
        return fail(LBM_EINVAL, "B = %d", B);
    FnoDev d = m->d;
    d.B = B;
    const size_t need = ws_layout(d, B).total;
    if (need > FNO_NOALLOC_SCRATCH_BYTES)
        return fail(LBM_EINVAL,
                    "batch %d needs %zu workspace bytes; the static scratch holds %zu "
                    "(use fno_forward with a caller workspace)",
                    B, need, (size_t)FNO_NOALLOC_SCRATCH_BYTES);
    if (m->device < 0 || m->device >= kMaxDevices) return fail(LBM_EINVAL, "model device %d", m->device);
    void* ws = g_scratch_ptr[m->device].load();
    if (!ws) return fail(LBM_EHIP, "scratch not set up on device %d", m->device);
    launch_forward(m, d_in, d_out, B, ws, (hipStream_t)stream);
    LBM_HIP(hipGetLastError());
    return LBM_OK;
}

// ================================================================ training
//
// Backward pass of the FNO (reverse order of the forward), AdamW and the device
// parameter refresh.  Spectral layer, with pre = s + Wc v + b, s = Re-inverse(R X),
// X = DFT(v):
//   dY = (c_k2 / (H'W')) DFT(dpre)              (c_0 = 1, c_k2>0 = 2)
//   dX[i] = sum_o dY[o] conj(R[i][o]),  dR[i][o] = sum_b conj(X[i]) dY[o]
//   dv = sum_k Re(dX e^{+i theta}) + Wc^T dpre  (unit-coefficient real inverse)
// The transforms reuse the forward kernels (BF16 operands on MFMA, FP32
// accumulation); pointwise backward and every weight-gradient reduction run in
// FP32 with a fixed summation order (deterministic).

namespace lbmfno {

__device__ __forceinline__ float act_grad(int kind, float x) {
    switch (kind) {
        case FNO_ACT_GELU: {
            const float cdf = 0.5f * (1.0f + erff(x * 0.70710678118654752f));
            const float pdf = 0.39894228040143268f * expf(-0.5f * x * x);
            return cdf + x * pdf;
        }
        case FNO_ACT_RELU: return x > 0.0f ? 1.0f : 0.0f;
        case FNO_ACT_SILU: {
            const float sg = 1.0f / (1.0f + expf(-x));
            return sg * (1.0f + x * (1.0f - sg));
        }
        default: return 1.0f;
    }
}

struct FnoBwd {
    float* dv;         // [B][Hp][Wpad][CP] gradient w.r.t. the current layer's output
    float* dpre;       // [B][Hp][Wpad][CP]
    __bf16* dpre_bf;   // same, bf16 (transform / MFMA operand)
    float* dY;         // [B][m2][R2][CP]
    float* dec_in;     // [dec_layers + 1][P0][MAXD]
    float* dec_da;     // [dec_layers][P0][DSP]
    float* d_out_cl;   // [P0][8] output gradient, channels last
    float* l_dv0;      // [P0][width]
    float* l_h1;       // [P0][width / 2]
    float* l_da1;      // [P0][width / 2]
    float* l_z;        // [P0][lift input channels]
    float* partials;   // reduction scratch
    float* grad;       // packed gradient (float32, parameter layout)
};

__global__ __launch_bounds__(256) void k_fill_f32(float* __restrict__ p, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

// d out = 2 (out - target) / n, and per-workgroup partial sums of (out - target)^2.
__global__ __launch_bounds__(256) void k_fno_mse(const float* __restrict__ out,
                                                 const float* __restrict__ tgt, size_t n,
                                                 float* __restrict__ dout,
                                                 double* __restrict__ partials) {
    __shared__ double red[4];
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    double e2 = 0.0;
    if (i < n) {
        const float e = out[i] - tgt[i];
        dout[i] = 2.0f * e / (float)n;
        e2 = (double)e * e;
    }
    for (int o = 32; o > 0; o >>= 1) e2 += __shfl_down(e2, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = e2;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = ((red[0] + red[1]) + red[2]) + red[3];
}

__global__ __launch_bounds__(256) void k_sum_partials(const double* __restrict__ p, int n,
                                                      double* __restrict__ out) {
    __shared__ double red[4];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += p[i];
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) *out = ((red[0] + red[1]) + red[2]) + red[3];
}

// Decoder backward, same tiling as the forward: the layer inputs are recomputed
// from the saved pre-activations (written out as float for the weight gradients),
// the output layer's transpose is a per-point sum over cout, and every hidden
// layer's input gradient dh_prev = da * W_l is an MFMA product with the
// transposed weights [din_p][DSP] (da rounded to bf16).  Writes dv (channels last).
__global__ __launch_bounds__(256) void k_fno_dec_bwd(FnoDev d, FnoBwd g, const __bf16* __restrict__ v,
                                                     const float* __restrict__ dout, int maxd) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int KP = d.DKP;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __bf16* buf = reinterpret_cast<__bf16*>(smem) + (size_t)wave * DEC_PTS * KP;
    float* dh = reinterpret_cast<float*>(smem + (size_t)4 * DEC_PTS * KP * 2) + (size_t)wave * DEC_PTS * KP;
    const size_t total = (size_t)d.B * d.H * d.W;
    const size_t pt0 = ((size_t)blockIdx.x * 4 + wave) * DEC_PTS;
    // layer inputs (float, row stride maxd) for the weight gradients
    for (int e = lane; e < DEC_PTS * maxd; e += 64) {
        const int pp = e / maxd, i = e % maxd;
        const size_t pt = pt0 + pp;
        if (pt >= total) continue;
        g.dec_in[pt * maxd + i] = i < d.CP ? from_bf16(v[dec_point_offset(d, pt) * d.CP + i]) : 0.0f;
        for (int l = 0; l < d.dec_layers; ++l) {
            float a = 0.0f;
            if (i < d.dec_size)
                a = from_bf16(to_bf16(act_f(d.dec_act, d.sv_dec[((size_t)l * total + pt) * d.DSP + i])));
            g.dec_in[((size_t)(l + 1) * total + pt) * maxd + i] = a;
        }
    }
    // output layer: d out (channels last copy) and dh = Wout^T d out
    const int dinL = d.dec_layers > 0 ? d.DSP : d.CP;
    const __bf16* wout = d.decw + (d.dec_layers > 0 ? (size_t)d.DSP * d.CP +
                                                          (size_t)(d.dec_layers - 1) * d.DSP * d.DSP : 0);
    for (int e = lane; e < DEC_PTS * 8; e += 64) {
        const int pp = e >> 3, o = e & 7;
        const size_t pt = pt0 + pp;
        if (pt < total) g.d_out_cl[pt * 8 + o] = o < d.cout ? dout[dec_out_offset(d, pt, o)] : 0.0f;
    }
    for (int e = lane; e < DEC_PTS * dinL; e += 64) {
        const int pp = e / dinL, i = e % dinL;
        const size_t pt = pt0 + pp;
        float t = 0.0f;
        if (pt < total)
            for (int o = 0; o < d.cout; ++o) t = fmaf(dout[dec_out_offset(d, pt, o)], from_bf16(wout[o * dinL + i]), t);
        dh[pp * KP + i] = t;
    }
    __syncthreads();
    for (int l = d.dec_layers - 1; l >= 0; --l) {
        for (int e = lane; e < DEC_PTS * d.DSP; e += 64) {
            const int pp = e / d.DSP, su = e % d.DSP;
            const size_t pt = pt0 + pp;
            float da = 0.0f;
            if (pt < total && su < d.dec_size)
                da = dh[pp * KP + su] * act_grad(d.dec_act, d.sv_dec[((size_t)l * total + pt) * d.DSP + su]);
            if (pt < total) g.dec_da[((size_t)l * total + pt) * d.DSP + su] = da;
            buf[pp * KP + su] = to_bf16(da);
        }
        __syncthreads();
        const int dinl = l == 0 ? d.CP : d.DSP;
        const __bf16* wt = d.decwT + (l == 0 ? 0 : (size_t)d.CP * d.DSP + (size_t)(l - 1) * d.DSP * d.DSP);
        for (int ct = 0; ct < dinl / 32; ++ct) {
            f32x16 acc = {};
            acc = mma_tile(buf, KP, wt + (size_t)ct * 32 * d.DSP, d.DSP, d.DSP, acc);
            const int c = ct * 32 + acc_col();
#pragma unroll
            for (int r = 0; r < 16; ++r) dh[acc_row(r) * KP + c] = acc[r];
        }
        __syncthreads();
    }
    // dv of the last latent layer
    for (int e = lane; e < DEC_PTS * d.CP; e += 64) {
        const int pp = e / d.CP, c = e % d.CP;
        const size_t pt = pt0 + pp;
        if (pt < total) g.dv[dec_point_offset(d, pt) * d.CP + c] = c < d.width ? dh[pp * KP + c] : 0.0f;
    }
}

// Deterministic outer-product reduction G[n][m] = sum_p A[p][n] X[p][m] (and
// bias[n] = sum_p A[p][n]) over P points, N, M <= 64.  Each workgroup takes a fixed
// set of 64-point stages (grid-stride), staged through LDS as float; a thread owns
// a 4 x 4 block of (n, m) and, when the tensor is narrow, the 256 threads form G
// groups that take every G-th point of a stage.  Group sums are combined in a fixed
// order, then one partial per workgroup is written; k_outer_final adds the
// partials in FP64 in a fixed order.
constexpr int OUT_TP = 64;
constexpr int OUT_MAX_BLOCKS = 2048;

template <typename TX>
__global__ __launch_bounds__(256) void k_outer_partial(const float* __restrict__ A, int lda,
                                                       const TX* __restrict__ X, int ldx, size_t P,
                                                       int N, int M, float* __restrict__ partials) {
    __shared__ __align__(16) float As[OUT_TP][64];
    __shared__ __align__(16) float Xs[OUT_TP][64];
    const int tid = threadIdx.x;
    const int tn = (N + 3) >> 2, tm = (M + 3) >> 2, T = tn * tm, G = 256 / T;
    const int g = tid / T, r = tid % T, ty = r / tm, tx = r % tm;
    const bool active = g < G;
    float acc[4][4] = {};
    float bacc[4] = {};
    // columns >= N (M) stay zero; only the valid columns are loaded per stage
    for (int i = tid; i < OUT_TP * 64; i += 256) {
        As[i >> 6][i & 63] = 0.0f;
        Xs[i >> 6][i & 63] = 0.0f;
    }
    const size_t nstage = (P + OUT_TP - 1) / OUT_TP;
    for (size_t st = blockIdx.x; st < nstage; st += gridDim.x) {
        const size_t p0 = st * OUT_TP;
        __syncthreads();
        for (int i = tid; i < OUT_TP * N; i += 256) {
            const int pp = i / N, c = i - pp * N;
            const size_t p = p0 + pp;
            As[pp][c] = p < P ? A[p * lda + c] : 0.0f;
        }
        for (int i = tid; i < OUT_TP * M; i += 256) {
            const int pp = i / M, c = i - pp * M;
            const size_t p = p0 + pp;
            Xs[pp][c] = p < P ? (float)X[p * ldx + c] : 0.0f;
        }
        __syncthreads();
        if (active) {
            for (int pp = g; pp < OUT_TP; pp += G) {
                const float4 a = *reinterpret_cast<const float4*>(&As[pp][4 * ty]);
                const float4 x = *reinterpret_cast<const float4*>(&Xs[pp][4 * tx]);
                const float av[4] = {a.x, a.y, a.z, a.w}, xv[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
                for (int i = 0; i < 4; ++i) {
#pragma unroll
                    for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(av[i], xv[j], acc[i][j]);
                    bacc[i] += av[i];
                }
            }
        }
    }
    // combine the G groups in a fixed order through LDS (reusing As / Xs: 2 x 16 KB)
    __syncthreads();
    float* red = &As[0][0];  // [G][T][16] <= 256 * 16 floats
    float* bred = &Xs[0][0]; // [G][T][4]
    if (active) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
            for (int j = 0; j < 4; ++j) red[((size_t)g * T + r) * 16 + i * 4 + j] = acc[i][j];
            bred[((size_t)g * T + r) * 4 + i] = bacc[i];
        }
    }
    __syncthreads();
    const int M1 = M + 1;
    float* out = partials + (size_t)blockIdx.x * N * M1;
    for (int e = tid; e < N * M1; e += 256) {
        const int n = e / M1, m = e % M1;
        const int ry = n >> 2, i = n & 3;
        float t = 0.0f;
        if (m < M) {
            const int rr = ry * tm + (m >> 2), j = m & 3;
            for (int q = 0; q < G; ++q) t += red[((size_t)q * T + rr) * 16 + i * 4 + j];
        } else {
            const int rr = ry * tm;   // bias sums: the tx = 0 thread of row block ry
            for (int q = 0; q < G; ++q) t += bred[((size_t)q * T + rr) * 4 + i];
        }
        out[e] = t;
    }
}

// Second pass: 64 outputs per workgroup, the four waves each sum a contiguous
// quarter of the partials in FP64, combined in a fixed order.
__global__ __launch_bounds__(256) void k_outer_final(const float* __restrict__ partials, int nchunks,
                                                     int N, int M, float* __restrict__ gw,
                                                     float* __restrict__ gb) {
    __shared__ double red[4][64];
    const int M1 = M + 1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int t = blockIdx.x * 64 + lane;
    const int q0 = (nchunks * wave) / 4, q1 = (nchunks * (wave + 1)) / 4;
    double s8[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (t < N * M1) {
        int c = q0;
        for (; c + 8 <= q1; c += 8) {
#pragma unroll
            for (int j = 0; j < 8; ++j) s8[j] += partials[(size_t)(c + j) * N * M1 + t];
        }
#pragma unroll
        for (int j = 0; j < 8; ++j)
            if (c + j < q1) s8[j] += partials[(size_t)(c + j) * N * M1 + t];
    }
    const double s = ((s8[0] + s8[1]) + (s8[2] + s8[3])) + ((s8[4] + s8[5]) + (s8[6] + s8[7]));
    red[wave][lane] = s;
    __syncthreads();
    if (wave == 0 && t < N * M1) {
        const double v = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
        const int n = t / M1, m = t % M1;
        if (m < M) gw[n * M + m] = (float)v;
        else if (gb) gb[n] = (float)v;
    }
}

// dpre = dv * act'(pre) (identity for the last layer); zero outside w < W'.
__global__ __launch_bounds__(256) void k_fno_act_bwd(FnoDev d, FnoBwd g, const float* __restrict__ pre,
                                                     int last) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t total = (size_t)d.B * d.Hp * d.Wpad * d.CP;
    if (i >= total) return;
    const int w = (int)(((unsigned)i / (unsigned)d.CP) % (unsigned)d.Wpad);
    float v = w < d.Wp ? g.dv[i] : 0.0f;
    if (!last) v *= act_grad(d.act, pre[i]);
    g.dpre[i] = v;
    g.dpre_bf[i] = to_bf16(v);
}

// Backward column step for one (sample, k2): dY = scale * DFT_H(T), complex
// mixing with conj(R), inverse column DFT of dX into Z.
__global__ __launch_bounds__(256) void k_fno_col_bwd(FnoDev d, FnoBwd g, int layer) {
    extern __shared__ __align__(16) unsigned char smem[];
    __bf16* Ts = reinterpret_cast<__bf16*>(smem);                                // [CP][TS]
    unsigned char* sm2 = smem + (size_t)d.CP * ts_stride(d) * 2;
    float* xs = reinterpret_cast<float*>(sm2);
    __bf16* ys = reinterpret_cast<__bf16*>(sm2 + sizeof(float) * d.R2 * d.CP);
    const int b = blockIdx.x / d.m2, k2 = blockIdx.x % d.m2;
    const int tid = threadIdx.x, wave = tid >> 6, nw = blockDim.x >> 6;
    const int H2 = 2 * d.Hpad, Nt = d.CP / 32;
    const float scale = (k2 == 0 ? 1.0f : 2.0f) / ((float)d.Hp * (float)d.Wp);
    const int TS = ts_stride(d);
    stage_t(d, b, k2, Ts);
    for (int t = wave; t < (d.R2 / 32) * Nt; t += nw) {
        const int mi = t / Nt, ni = t % Nt;
        f32x16 acc = {};
        acc = mma_tile(d.EcolA + (size_t)mi * 32 * H2, H2, Ts + ni * 32 * TS, TS, H2, acc);
        const int c = ni * 32 + acc_col();
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = mi * 32 + acc_row(r);
            const float y = acc[r] * scale;
            xs[row * d.CP + c] = y;
            g.dY[(((size_t)b * d.m2 + k2) * d.R2 + row) * d.CP + c] = y;
        }
    }
    for (int i = tid; i < d.CP * d.R2; i += blockDim.x) ys[i] = to_bf16(0.0f);
    __syncthreads();
    const __bf16* R = d.Rmix + ((size_t)layer * d.m2 + k2) * d.K1 * d.CP * d.CP * 2;
    // padded channels of R are zero: only the width real ones take part
    for (int idx = tid; idx < d.K1 * d.width; idx += blockDim.x) {
        const int k = idx / d.width, i = idx % d.width;
        const float* yr = xs + k * d.CP;
        const float* yi = xs + (d.K1 + k) * d.CP;
        float sr = 0.0f, si = 0.0f;
        for (int o = 0; o < d.width; ++o) {
            const __bf16* Rp = R + (((size_t)k * d.CP + o) * d.CP + i) * 2;
            const float rr = from_bf16(Rp[0]), rim = from_bf16(Rp[1]);
            sr = fmaf(yr[o], rr, sr);
            sr = fmaf(yi[o], rim, sr);
            si = fmaf(-yr[o], rim, si);
            si = fmaf(yi[o], rr, si);
        }
        ys[i * d.R2 + k] = to_bf16(sr);
        ys[i * d.R2 + d.K1 + k] = to_bf16(si);
    }
    __syncthreads();
    z_store_column(d, b, k2, ys);
}

// dv[w][i] = sum_kk B1[w][kk] Z[i][kk] + sum_o dpre[w][o] Wc[o][i], per (b, h) row.
__global__ __launch_bounds__(256) void k_fno_rowinv_bwd(FnoDev d, FnoBwd g, int layer) {
    const int b = blockIdx.x / d.Hp, h = blockIdx.x % d.Hp;
    const int tid = threadIdx.x, wave = tid >> 6, nw = blockDim.x >> 6;
    const size_t rowoff = ((size_t)b * d.Hp + h) * d.Wpad * d.CP;
    extern __shared__ __align__(16) unsigned char smem[];
    __bf16* zs = reinterpret_cast<__bf16*>(smem);  // [CP][KKp + 8]
    stage_z(d, b, h, zs);
    const int KKs = d.KKp + 8;
    const __bf16* WcT = d.WcT + (size_t)layer * d.CP * d.CP;
    const int Mt = d.Wpad / 32, Nt = d.CP / 32;
    for (int t = wave; t < Mt * Nt; t += nw) {
        const int mi = t / Nt, ni = t % Nt;
        f32x16 acc = {};
        acc = mma_tile(d.B1 + (size_t)mi * 32 * d.KKp, d.KKp, zs + (size_t)ni * 32 * KKs, KKs,
                       d.KKp, acc);
        acc = mma_tile(g.dpre_bf + rowoff + (size_t)mi * 32 * d.CP, d.CP, WcT + (size_t)ni * 32 * d.CP,
                       d.CP, d.CP, acc);
        const int i = ni * 32 + acc_col();
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int w = mi * 32 + acc_row(r);
            g.dv[rowoff + (size_t)w * d.CP + i] = (w < d.Wp && i < d.width) ? acc[r] : 0.0f;
        }
    }
}

// dR of one layer into the packed gradient: thread per (k2, kept row k, o, i).
__global__ __launch_bounds__(256) void k_fno_dR(FnoDev d, FnoBwd g, const float* __restrict__ X,
                                                float* __restrict__ gtop, float* __restrict__ gbot) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int wd = d.width;
    const size_t total = (size_t)d.m2 * d.K1 * wd * wd;
    if (idx >= total) return;
    const int i = (int)(idx % wd);
    const int o = (int)((idx / wd) % wd);
    const int k = (int)((idx / ((size_t)wd * wd)) % d.K1);
    const int k2 = (int)(idx / ((size_t)wd * wd * d.K1));
    double sr = 0.0, si = 0.0;
    for (int b = 0; b < d.B; ++b) {
        const size_t base = ((size_t)b * d.m2 + k2) * d.R2;
        const double xr = X[(base + k) * d.CP + i], xi = X[(base + d.K1 + k) * d.CP + i];
        const double yr = g.dY[(base + k) * d.CP + o], yi = g.dY[(base + d.K1 + k) * d.CP + o];
        sr += xr * yr + xi * yi;
        si += xr * yi - xi * yr;
    }
    const int a = k < d.m1 ? k : k - d.m1;
    float* dst = k < d.m1 ? gtop : gbot;
    const size_t off = ((((size_t)i * wd + o) * d.m1 + a) * d.m2 + k2) * 2;
    dst[off] = (float)sr;
    dst[off + 1] = (float)si;
}

// Lift backward for one input point: dh1 = P2^T dv0, da1 = dh1 act'(a1); writes
// the reduction inputs (dv0, h1, da1, z).
__global__ __launch_bounds__(256) void k_fno_lift_bwd(FnoDev d, FnoBwd g, const float* __restrict__ x) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t total = (size_t)d.B * d.H * d.W;
    if (idx >= total) return;
    const unsigned rw = (unsigned)idx / (unsigned)d.W;
    const int w = (int)((unsigned)idx - rw * d.W);
    const int b = (int)(rw / (unsigned)d.H);
    const int h = (int)(rw - (unsigned)b * d.H);
    const size_t vpt = ((size_t)b * d.Hp + h) * d.Wpad + w;
    float s[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) s[k] = 0.0f;
    for (int c = 0; c < d.width; ++c) {
        const float dv = g.dv[vpt * d.CP + c];
        g.l_dv0[idx * d.width + c] = dv;
        const float* w2 = d.lift2w + (size_t)c * d.half;
#pragma unroll
        for (int k = 0; k < 32; ++k)
            if (k < d.half) s[k] = fmaf(dv, w2[k], s[k]);
    }
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        if (k < d.half) {
            const float a1 = d.sv_a1[idx * 32 + k];
            g.l_h1[idx * d.half + k] = act_f(d.act, a1);
            g.l_da1[idx * d.half + k] = s[k] * act_grad(d.act, a1);
        }
    }
    for (int c = 0; c < d.cin; ++c) g.l_z[idx * d.cl + c] = x[(((size_t)b * d.cin + c) * d.H + h) * d.W + w];
    if (d.coords) {
        g.l_z[idx * d.cl + d.cin] = d.W > 1 ? (float)w / (float)(d.W - 1) : 0.0f;
        g.l_z[idx * d.cl + d.cin + 1] = d.H > 1 ? (float)h / (float)(d.H - 1) : 0.0f;
    }
}

__global__ __launch_bounds__(256) void k_param_map(const float* __restrict__ params,
                                                   const int32_t* __restrict__ map, int64_t n,
                                                   void* __restrict__ dst, int bf) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int32_t src = map[j];
    const float v = src >= 0 ? params[src] : 0.0f;
    if (bf) reinterpret_cast<__bf16*>(dst)[j] = to_bf16(v);
    else reinterpret_cast<float*>(dst)[j] = v;
}

__global__ __launch_bounds__(256) void k_adamw(float* __restrict__ p, const float* __restrict__ gr,
                                               float* __restrict__ m, float* __restrict__ v, int64_t n,
                                               float lr, float b1, float b2, float eps, float wd,
                                               float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = gr[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    float pi = p[i] * (1.0f - lr * wd);
    pi -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
}

}  // namespace lbmfno

// ------------------------------------------------------------ training host

struct TrainLayout {
    size_t v, pre, X, a1, dec, dv, dpre, dpre_bf, dY, dec_in, dec_da, dout, ldv0, lh1, lda1, lz,
        partials, T, Z, total;
    int maxd;
    size_t P0, Pl;
};

static TrainLayout train_layout(const FnoDev& d, int B) {
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    TrainLayout t;
    t.maxd = std::max(d.CP, d.DSP) <= 32 ? 32 : 64;
    t.Pl = (size_t)B * d.Hp * d.Wpad;
    t.P0 = (size_t)B * d.H * d.W;
    const size_t lat = t.Pl * d.CP;
    t.v = al(lat * 2);
    t.pre = al(lat * 4);
    t.X = al((size_t)B * d.m2 * d.R2 * d.CP * 4);
    t.a1 = al(t.P0 * 32 * 4);
    t.dec = al((size_t)std::max(d.dec_layers, 1) * t.P0 * std::max(d.DSP, 1) * 4);
    t.dv = al(lat * 4);
    t.dpre = al(lat * 4);
    t.dpre_bf = al(lat * 2);
    t.dY = t.X;
    t.dec_in = al((size_t)(d.dec_layers + 1) * t.P0 * t.maxd * 4);
    t.dec_da = al((size_t)std::max(d.dec_layers, 1) * t.P0 * std::max(d.DSP, 1) * 4);
    t.dout = al(t.P0 * 8 * 4);
    t.ldv0 = al(t.P0 * 64 * 4);
    t.lh1 = al(t.P0 * 32 * 4);
    t.lda1 = al(t.P0 * 32 * 4);
    t.lz = al(t.P0 * 8 * 4);
    t.partials = al((size_t)OUT_MAX_BLOCKS * 64 * 65 * 4 + 4096 * 8);
    t.T = al((size_t)B * d.m2 * d.CP * 2 * d.Hpad * 2);
    t.Z = al((size_t)B * 2 * d.m2 * d.Hp * d.CP * 2);
    t.total = (d.L + 1) * t.v + d.L * t.pre + d.L * t.X + t.a1 + t.dec + t.dv + t.dpre + t.dpre_bf +
              t.dY + t.dec_in + t.dec_da + t.dout + t.ldv0 + t.lh1 + t.lda1 + t.lz + t.partials +
              t.T + t.Z;
    return t;
}

struct TrainPtrs {
    __bf16* v[33];
    float* pre[32];
    float* X[32];
    float *a1, *dec;
    FnoBwd g;
    __bf16 *T, *Z;
};

static TrainPtrs train_ptrs(const FnoDev& d, const TrainLayout& t, void* ws) {
    unsigned char* p = static_cast<unsigned char*>(ws);
    TrainPtrs r{};
    for (int l = 0; l <= d.L; ++l) { r.v[l] = reinterpret_cast<__bf16*>(p); p += t.v; }
    for (int l = 0; l < d.L; ++l) { r.pre[l] = reinterpret_cast<float*>(p); p += t.pre; }
    for (int l = 0; l < d.L; ++l) { r.X[l] = reinterpret_cast<float*>(p); p += t.X; }
    r.a1 = reinterpret_cast<float*>(p); p += t.a1;
    r.dec = reinterpret_cast<float*>(p); p += t.dec;
    r.g.dv = reinterpret_cast<float*>(p); p += t.dv;
    r.g.dpre = reinterpret_cast<float*>(p); p += t.dpre;
    r.g.dpre_bf = reinterpret_cast<__bf16*>(p); p += t.dpre_bf;
    r.g.dY = reinterpret_cast<float*>(p); p += t.dY;
    r.g.dec_in = reinterpret_cast<float*>(p); p += t.dec_in;
    r.g.dec_da = reinterpret_cast<float*>(p); p += t.dec_da;
    r.g.d_out_cl = reinterpret_cast<float*>(p); p += t.dout;
    r.g.l_dv0 = reinterpret_cast<float*>(p); p += t.ldv0;
    r.g.l_h1 = reinterpret_cast<float*>(p); p += t.lh1;
    r.g.l_da1 = reinterpret_cast<float*>(p); p += t.lda1;
    r.g.l_z = reinterpret_cast<float*>(p); p += t.lz;
    r.g.partials = reinterpret_cast<float*>(p); p += t.partials;
    r.T = reinterpret_cast<__bf16*>(p); p += t.T;
    r.Z = reinterpret_cast<__bf16*>(p); p += t.Z;
    return r;
}

extern "C" int fno_train_workspace_size(const fno_model* m, int32_t B, size_t* bytes) {
    if (!m || !bytes) return fail(LBM_EINVAL, "NULL argument");
    if (B < 1) return fail(LBM_EINVAL, "B = %d", B);
    if (m->d.L > 32) return fail(LBM_EUNSUPPORTED, "training supports up to 32 layers");
    *bytes = train_layout(m->d, B).total;
    return LBM_OK;
}

static int check_train_args(const fno_model* m, int32_t B, void* ws, size_t ws_bytes) {
    if (!m) return fail(LBM_EINVAL, "model is NULL");
    if (!ws) return fail(LBM_EINVAL, "workspace is NULL");
    if (B < 1 || (int64_t)B * m->d.Hp * m->d.Wpad > ((int64_t)1 << 31) / 64) return fail(LBM_EINVAL, "B = %d", B);
    if ((uintptr_t)ws % 256) return fail(LBM_EINVAL, "workspace not 256-byte aligned");
    if (m->d.L > 32) return fail(LBM_EUNSUPPORTED, "training supports up to 32 layers");
    const size_t need = train_layout(m->d, B).total;
    if (ws_bytes < need) return fail(LBM_EINVAL, "training workspace %zu < %zu bytes", ws_bytes, need);
    return LBM_OK;
}

extern "C" int fno_forward_train(const fno_model* m, const float* d_in, float* d_out, int32_t B,
                                 void* d_ws, size_t ws_bytes, void* stream) {
    int rc = check_train_args(m, B, d_ws, ws_bytes);
    if (rc) return rc;
    if (!d_in || !d_out) return fail(LBM_EINVAL, "NULL buffer");
    FnoDev d = m->d;
    d.B = B;
    const TrainLayout t = train_layout(d, B);
    TrainPtrs P = train_ptrs(d, t, d_ws);
    hipStream_t st = (hipStream_t)stream;
    d.T = P.T;
    d.Z = P.Z;
    d.v0 = P.v[0];
    d.sv_a1 = P.a1;
    launch_lift(d, t.Pl, d_in, st);
    d.sv_a1 = nullptr;
    const size_t lds_row = (size_t)d.CP * vt_stride(d) * 2;
    const bool fused = fuse_row_dft(d);  // later layers' row DFT in the row inverse
    for (int l = 0; l < d.L; ++l) {
        if (l == 0 || !fused) k_fno_rowfwd<<<B * d.Hpad, 256, lds_row, st>>>(d, P.v[l]);
        d.sv_X = P.X[l];
        k_fno_col<<<B * d.m2, COL_THREADS, col_lds(d), st>>>(d, l);
        d.sv_X = nullptr;
        d.sv_pre = P.pre[l];
        launch_rowinv(d, P.v[l], P.v[l + 1], l, st);
        d.sv_pre = nullptr;
    }
    d.sv_dec = P.dec;
    launch_dec(d, P.v[d.L], d_out, st);
    LBM_HIP(hipGetLastError());
    return LBM_OK;
}

// Latent v[l] (bf16 [B][Hp][Wpad][CP], channels last) -> float32 [B][width][Hp][Wp].
__global__ __launch_bounds__(256) void k_fno_export_latent(FnoDev d, const __bf16* __restrict__ v,
                                                           float* __restrict__ out) {
    const size_t n = (size_t)d.B * d.width * d.Hp * d.Wp;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
        const int w = (int)(i % d.Wp);
        size_t r = i / d.Wp;
        const int h = (int)(r % d.Hp);
        r /= d.Hp;
        const int c = (int)(r % d.width);
        const size_t b = r / d.width;
        out[i] = (float)v[((b * d.Hp + h) * d.Wpad + w) * d.CP + c];
    }
}

extern "C" int fno_train_latent(const fno_model* m, const void* d_ws, size_t ws_bytes, int32_t B,
                                int32_t layer, float* d_out, void* stream) {
    int rc = check_train_args(m, B, const_cast<void*>(d_ws), ws_bytes);
    if (rc) return rc;
    if (!d_out) return fail(LBM_EINVAL, "NULL buffer");
    if (layer < 0 || layer > m->d.L) return fail(LBM_EINVAL, "layer = %d (0..%d)", layer, m->d.L);
    FnoDev d = m->d;
    d.B = B;
    const TrainPtrs P = train_ptrs(d, train_layout(d, B), const_cast<void*>(d_ws));
    const size_t n = (size_t)B * d.width * d.Hp * d.Wp;
    const unsigned grid = (unsigned)std::min<size_t>((n + 255) / 256, 65536);
    k_fno_export_latent<<<grid, 256, 0, (hipStream_t)stream>>>(d, P.v[layer], d_out);
    LBM_HIP(hipGetLastError());
    return LBM_OK;
}

static void outer_reduce(hipStream_t st, float* partials, const float* A, int lda, const void* X,
                         bool xbf, int ldx, size_t P, int N, int M, float* gw, float* gb) {
    const unsigned chunks = (unsigned)std::min<size_t>((P + OUT_TP - 1) / OUT_TP, OUT_MAX_BLOCKS);
    if (xbf)
        k_outer_partial<__bf16><<<chunks, 256, 0, st>>>(A, lda, static_cast<const __bf16*>(X), ldx, P, N, M, partials);
    else
        k_outer_partial<float><<<chunks, 256, 0, st>>>(A, lda, static_cast<const float*>(X), ldx, P, N, M, partials);
    const int n = N * (M + 1);
    k_outer_final<<<(n + 63) / 64, 256, 0, st>>>(partials, (int)chunks, N, M, gw, gb);
}

extern "C" int fno_backward(const fno_model* m, const float* d_in, const float* d_dout, int32_t B,
                            void* d_ws, size_t ws_bytes, float* d_grad, void* stream) {
    int rc = check_train_args(m, B, d_ws, ws_bytes);
    if (rc) return rc;
    if (!d_in || !d_dout || !d_grad) return fail(LBM_EINVAL, "NULL buffer");
    FnoDev d = m->d;
    d.B = B;
    const TrainLayout t = train_layout(d, B);
    TrainPtrs P = train_ptrs(d, t, d_ws);
    FnoBwd g = P.g;
    g.grad = d_grad;
    d.T = P.T;
    d.Z = P.Z;
    d.sv_dec = P.dec;
    d.sv_a1 = P.a1;
    hipStream_t st = (hipStream_t)stream;
    const fno_spec& s = m->spec;
    // packed offsets
    const int wd = s.width, half = d.half, cl = d.cl;
    const size_t o_l1w = 0, o_l1b = o_l1w + (size_t)half * cl, o_l2w = o_l1b + half,
                 o_l2b = o_l2w + (size_t)wd * half, o_layers = o_l2b + wd;
    const size_t blk = (size_t)wd * wd * s.m1 * s.m2 * 2, per_layer = 2 * blk + (size_t)wd * wd + wd;
    size_t o_dec = o_layers + (size_t)s.layers * per_layer;
    // decoder
    const size_t lat = t.Pl * d.CP;
    k_fill_f32<<<(unsigned)((lat + 255) / 256), 256, 0, st>>>(g.dv, lat);
    k_fno_dec_bwd<<<(unsigned)((t.P0 + 4 * DEC_PTS - 1) / (4 * DEC_PTS)), 256, dec_bwd_lds(d), st>>>(
        d, g, P.v[d.L], d_dout, t.maxd);
    {
        size_t off = o_dec;
        int din = wd;
        std::vector<size_t> wofs, bofs;
        std::vector<int> dins;
        for (int l = 0; l < s.dec_layers; ++l) {
            wofs.push_back(off); off += (size_t)s.dec_size * din;
            bofs.push_back(off); off += s.dec_size;
            dins.push_back(din);
            din = s.dec_size;
        }
        const size_t ow = off, ob = off + (size_t)s.cout * din;
        outer_reduce(st, g.partials, g.d_out_cl, 8, g.dec_in + (size_t)s.dec_layers * t.P0 * t.maxd, false,
                     t.maxd, t.P0, s.cout, din, d_grad + ow, d_grad + ob);
        for (int l = 0; l < s.dec_layers; ++l)
            outer_reduce(st, g.partials, g.dec_da + (size_t)l * t.P0 * d.DSP, d.DSP,
                         g.dec_in + (size_t)l * t.P0 * t.maxd, false, t.maxd, t.P0, s.dec_size, dins[l],
                         d_grad + wofs[l], d_grad + bofs[l]);
    }
    // Fourier layers, last first
    const size_t lds_row = (size_t)d.CP * vt_stride(d) * 2;
    const size_t lds_col = (size_t)d.CP * ts_stride(d) * 2 + (size_t)d.R2 * d.CP * 4 + (size_t)d.CP * d.R2 * 2;
    for (int l = d.L - 1; l >= 0; --l) {
        const size_t lo = o_layers + (size_t)l * per_layer;
        k_fno_act_bwd<<<(unsigned)((lat + 255) / 256), 256, 0, st>>>(d, g, P.pre[l], l == d.L - 1);
        outer_reduce(st, g.partials, g.dpre, d.CP, P.v[l], true, d.CP, t.Pl, wd, wd,
                     d_grad + lo + 2 * blk, d_grad + lo + 2 * blk + (size_t)wd * wd);
        k_fno_rowfwd<<<B * d.Hpad, 256, lds_row, st>>>(d, g.dpre_bf);
        k_fno_col_bwd<<<B * d.m2, 256, lds_col, st>>>(d, g, l);
        const size_t nR = (size_t)s.m2 * d.K1 * wd * wd;
        k_fno_dR<<<(unsigned)((nR + 255) / 256), 256, 0, st>>>(d, g, P.X[l], d_grad + lo, d_grad + lo + blk);
        k_fno_rowinv_bwd<<<B * d.Hp, 256, zs_lds(d), st>>>(d, g, l);  // dv = dLoss / d v_l
    }
    // lift
    k_fno_lift_bwd<<<(unsigned)((t.P0 + 255) / 256), 256, 0, st>>>(d, g, d_in);
    outer_reduce(st, g.partials, g.l_dv0, wd, g.l_h1, false, half, t.P0, wd, half, d_grad + o_l2w, d_grad + o_l2b);
    outer_reduce(st, g.partials, g.l_da1, half, g.l_z, false, cl, t.P0, half, cl, d_grad + o_l1w, d_grad + o_l1b);
    LBM_HIP(hipGetLastError());
    return LBM_OK;
}

extern "C" int fno_mse(const float* d_out, const float* d_tgt, size_t n, float* d_dout, void* d_ws,
                       size_t ws_bytes, double* h_loss, void* stream) {
    if (!d_out || !d_tgt || !d_dout || !d_ws || !h_loss) return fail(LBM_EINVAL, "NULL argument");
    if (n == 0) return fail(LBM_EINVAL, "n = 0");
    const unsigned nb = (unsigned)((n + 255) / 256);
    if (ws_bytes < ((size_t)nb + 1) * sizeof(double)) return fail(LBM_EINVAL, "workspace too small");
    hipStream_t st = (hipStream_t)stream;
    double* part = static_cast<double*>(d_ws);
    k_fno_mse<<<nb, 256, 0, st>>>(d_out, d_tgt, n, d_dout, part);
    k_sum_partials<<<1, 256, 0, st>>>(part, (int)nb, part + nb);
    LBM_HIP(hipGetLastError());
    LBM_HIP(hipMemcpyAsync(h_loss, part + nb, sizeof(double), hipMemcpyDeviceToHost, st));
    LBM_HIP(hipStreamSynchronize(st));
    *h_loss /= (double)n;
    return LBM_OK;
}

extern "C" int fno_set_params(fno_model* m, const float* d_params, void* stream) {
    if (!m || !d_params) return fail(LBM_EINVAL, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    for (const fno_model::Map& mp : m->maps)
        if (mp.n > 0)
            k_param_map<<<(unsigned)((mp.n + 255) / 256), 256, 0, st>>>(d_params, mp.map, mp.n, mp.dst, mp.bf16 ? 1 : 0);
    LBM_HIP(hipGetLastError());
    return LBM_OK;
}

extern "C" int fno_adamw(float* d_p, const float* d_g, float* d_m, float* d_v, int64_t n, double lr,
                         double beta1, double beta2, double eps, double weight_decay, int64_t step,
                         void* stream) {
    if (!d_p || !d_g || !d_m || !d_v) return fail(LBM_EINVAL, "NULL buffer");
    if (n < 0 || step < 1 || !(lr >= 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1))
        return fail(LBM_EINVAL, "AdamW arguments");
    const float c1 = (float)(1.0 - std::pow(beta1, (double)step));
    const float c2 = (float)(1.0 - std::pow(beta2, (double)step));
    k_adamw<<<(unsigned)((n + 255) / 256), 256, 0, (hipStream_t)stream>>>(
        d_p, d_g, d_m, d_v, n, (float)lr, (float)beta1, (float)beta2, (float)eps, (float)weight_decay, c1, c2);
    LBM_HIP(hipGetLastError());
    return LBM_OK;
}
