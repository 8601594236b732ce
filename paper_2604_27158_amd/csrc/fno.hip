// fno.hip -- Fourier Neural Operator forward pass (paper Sec. 2.2, Eq. 6) for
// gfx950: bfloat16 operands on MFMA (v_mfma_f32_32x32x16_bf16), float32
// accumulation.
//
// Data layout (device workspace, per sample b):
//   v  [Hp][Wpad][CP]   bf16  activations, channels last (CP = width rounded up to
//                             32, Wpad = W' rounded up to 32; w >= W' is zero)
//   T  [m2][CP][2][Hpad] bf16 row-DFT coefficients (re, im) with h fastest
//   Z  [Hp][CP][KKp]    bf16  column-inverse coefficients, (k2, re/im) fastest
// Every contraction is arranged so that both MFMA operands are contiguous along
// the summed index, i.e. each lane fetches its eight bf16 as one 16-byte load:
//   row forward   T[kk][c]   = sum_w  EwT[kk][w]   * vt[c][w]     (vt staged in LDS)
//   column        X[r][c]    = sum_hk EcolA[r][hk] * T[c][hk]     (per sample, k2)
//   mixing        Y[k][o]    = sum_i  X[k][i] R[i][o]              (complex, per mode)
//   column inv    Zc[q][o]   = sum_r  EcolB[q][r]  * Y[o][r]
//   row inverse   s[w][o]    = sum_kk BinvT[w][kk] * Z[o][kk] + sum_i v[w][i] * Wc[o][i]
// followed by bias and the activation, rounded to bf16 in the epilogue.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "common.hpp"

namespace lbmfno {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
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
    for (int k0 = 0; k0 < K; k0 += 16) {
        const bf16x8 av = *reinterpret_cast<const bf16x8*>(a + k0);
        const bf16x8 bv = *reinterpret_cast<const bf16x8*>(b + k0);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
    }
    return acc;
}

// Accumulator element r of this lane holds C[acc_row(r)][acc_col()].
__device__ __forceinline__ int acc_row(int r) {
    return 8 * (r >> 2) + 4 * ((threadIdx.x & 63) >> 5) + (r & 3);
}
__device__ __forceinline__ int acc_col() { return threadIdx.x & 31; }

__device__ __forceinline__ float act_f(int kind, float x) {
    switch (kind) {
        case FNO_ACT_GELU: return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f));
        case FNO_ACT_RELU: return x > 0.0f ? x : 0.0f;
        case FNO_ACT_SILU: return x / (1.0f + expf(-x));
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
    const __bf16* Rmix;     // [L][m2][K1][CP][CP][2]
    const __bf16* Wc;       // [L][CP][CP]
    const float* bc;        // [L][CP]
    const __bf16* decw;     // per decoder layer [DSP][in_p], then out [CoutP][DSP]
    const float* decb;      // per decoder layer [DSP], then out [cout]
    const __bf16 *EwT, *BinvT, *EcolA, *EcolB;
    // workspace
    __bf16 *v0, *v1, *T, *Z;
};

// ---------------------------------------------------------------- kernels

// Lift: x (cin channels, float32) + coordinates -> width/2 (act) -> width, rounded
// to bf16, written channels-last; the zero-padded region and w >= W' hold zeros.
__global__ __launch_bounds__(256) void k_fno_lift(FnoDev d, const float* __restrict__ x) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t total = (size_t)d.B * d.Hp * d.Wpad;
    if (idx >= total) return;
    const int w = (int)(idx % d.Wpad);
    const int h = (int)((idx / d.Wpad) % d.Hp);
    const int b = (int)(idx / ((size_t)d.Wpad * d.Hp));
    __bf16* out = d.v0 + idx * d.CP;
    float z[8];
    float hid[32];
    float o[64];
    const bool inside = h < d.H && w < d.W;
    if (inside) {
        for (int c = 0; c < d.cin; ++c) z[c] = x[(((size_t)b * d.cin + c) * d.H + h) * d.W + w];
        if (d.coords) {
            z[d.cin] = d.W > 1 ? (float)w / (float)(d.W - 1) : 0.0f;
            z[d.cin + 1] = d.H > 1 ? (float)h / (float)(d.H - 1) : 0.0f;
        }
        for (int k = 0; k < d.half; ++k) {
            float s = d.lift1b[k];
            for (int c = 0; c < d.cl; ++c) s = fmaf(d.lift1w[k * d.cl + c], z[c], s);
            hid[k] = act_f(d.act, s);
        }
        for (int c = 0; c < d.width; ++c) {
            float s = d.lift2b[c];
            for (int k = 0; k < d.half; ++k) s = fmaf(d.lift2w[c * d.half + k], hid[k], s);
            o[c] = s;
        }
    }
    for (int c0 = 0; c0 < d.CP; c0 += 8) {
        bf16x8 t;
        for (int e = 0; e < 8; ++e) {
            const int c = c0 + e;
            t[e] = to_bf16(inside && c < d.width ? o[c] : 0.0f);
        }
        *reinterpret_cast<bf16x8*>(out + c0) = t;
    }
}

// Row forward DFT: one workgroup per (b, h), h < Hpad (rows h >= H' write zeros so
// the column transform's padded K range is exactly zero).
__global__ __launch_bounds__(256) void k_fno_rowfwd(FnoDev d, const __bf16* __restrict__ v) {
    extern __shared__ __align__(16) unsigned char smem[];
    __bf16* vt = reinterpret_cast<__bf16*>(smem);  // [CP][Wpad]
    const int b = blockIdx.x / d.Hpad, h = blockIdx.x % d.Hpad;
    const int tid = threadIdx.x;
    const size_t tstride = (size_t)2 * d.Hpad;
    __bf16* Tb = d.T + (size_t)b * d.m2 * d.CP * tstride;
    if (h >= d.Hp) {
        for (int i = tid; i < d.m2 * d.CP * 2; i += blockDim.x) {
            const int ri = i & 1, kc = i >> 1;  // kc = k2 * CP + c
            Tb[(size_t)kc * tstride + ri * d.Hpad + h] = to_bf16(0.0f);
        }
        return;
    }
    const __bf16* row = v + ((size_t)b * d.Hp + h) * d.Wpad * d.CP;
    // stage the row transposed: vt[c][w] = row[w][c]
    const int nvec = d.Wpad * d.CP / 8;
    for (int i = tid; i < nvec; i += blockDim.x) {
        const bf16x8 t = *reinterpret_cast<const bf16x8*>(row + 8 * i);
        const int w = (8 * i) / d.CP, c0 = (8 * i) % d.CP;
        for (int e = 0; e < 8; ++e) vt[(c0 + e) * d.Wpad + w] = t[e];
    }
    __syncthreads();
    const int wave = tid >> 6;
    const int Mt = d.KKp / 32, Nt = d.CP / 32;
    for (int t = wave; t < Mt * Nt; t += blockDim.x >> 6) {
        const int mi = t / Nt, ni = t % Nt;
        f32x16 acc = {};
        acc = mma_tile(d.EwT + (size_t)mi * 32 * d.Wpad, d.Wpad, vt + ni * 32 * d.Wpad, d.Wpad,
                       d.Wpad, acc);
        const int c = ni * 32 + acc_col();
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int kk = mi * 32 + acc_row(r);
            if (kk < 2 * d.m2) {
                const int k2 = kk >> 1, ri = kk & 1;
                Tb[((size_t)k2 * d.CP + c) * tstride + ri * d.Hpad + h] = to_bf16(acc[r]);
            }
        }
    }
}

// Column forward DFT, per-mode complex mixing and column inverse DFT for one
// (sample, k2).  Also zeroes Z's padded coefficient columns (k2 == 0 group).
__global__ __launch_bounds__(256) void k_fno_col(FnoDev d, int layer) {
    extern __shared__ __align__(16) unsigned char smem[];
    float* xs = reinterpret_cast<float*>(smem);                                  // [R2][CP]
    __bf16* ys = reinterpret_cast<__bf16*>(smem + sizeof(float) * d.R2 * d.CP);  // [CP][R2]
    const int b = blockIdx.x / d.m2, k2 = blockIdx.x % d.m2;
    const int tid = threadIdx.x, wave = tid >> 6, nw = blockDim.x >> 6;
    const int H2 = 2 * d.Hpad;
    const int Nt = d.CP / 32;
    const __bf16* Ts = d.T + ((size_t)b * d.m2 + k2) * d.CP * H2;  // [CP][2 Hpad]
    // X[r][c] = sum_{ri,h} EcolA[r][ri,h] T[c][ri,h]
    const int Mt1 = d.R2 / 32;
    for (int t = wave; t < Mt1 * Nt; t += nw) {
        const int mi = t / Nt, ni = t % Nt;
        f32x16 acc = {};
        acc = mma_tile(d.EcolA + (size_t)mi * 32 * H2, H2, Ts + (size_t)ni * 32 * H2, H2, H2, acc);
        const int c = ni * 32 + acc_col();
#pragma unroll
        for (int r = 0; r < 16; ++r)
            xs[(mi * 32 + acc_row(r)) * d.CP + c] = from_bf16(to_bf16(acc[r]));
    }
    for (int i = tid; i < d.CP * d.R2; i += blockDim.x) ys[i] = to_bf16(0.0f);
    __syncthreads();
    // Y[k][o] = sum_i X[k][i] R[i][o][k][k2] (complex), k over the 2 m1 kept rows
    const __bf16* R = d.Rmix + ((size_t)layer * d.m2 + k2) * d.K1 * d.CP * d.CP * 2;
    for (int idx = tid; idx < d.K1 * d.CP; idx += blockDim.x) {
        const int k = idx / d.CP, o = idx % d.CP;
        const float* xr = xs + k * d.CP;
        const float* xi = xs + (d.K1 + k) * d.CP;
        const __bf16* Rk = R + ((size_t)k * d.CP + o) * d.CP * 2;
        float sr = 0.0f, si = 0.0f;
        for (int i = 0; i < d.CP; ++i) {
            const float rr = from_bf16(Rk[2 * i]), rim = from_bf16(Rk[2 * i + 1]);
            sr = fmaf(xr[i], rr, sr);
            sr = fmaf(-xi[i], rim, sr);
            si = fmaf(xr[i], rim, si);
            si = fmaf(xi[i], rr, si);
        }
        ys[o * d.R2 + k] = to_bf16(sr);
        ys[o * d.R2 + d.K1 + k] = to_bf16(si);
    }
    __syncthreads();
    // Zc[q][o] = sum_r EcolB[q][r] Y[o][r], q = ri * Hpad + h
    const int Mt2 = H2 / 32;
    for (int t = wave; t < Mt2 * Nt; t += nw) {
        const int mi = t / Nt, ni = t % Nt;
        f32x16 acc = {};
        acc = mma_tile(d.EcolB + (size_t)mi * 32 * d.R2, d.R2, ys + ni * 32 * d.R2, d.R2, d.R2, acc);
        const int o = ni * 32 + acc_col();
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int q = mi * 32 + acc_row(r);
            const int ri = q >= d.Hpad ? 1 : 0, h = q - ri * d.Hpad;
            if (h < d.Hp)
                d.Z[(((size_t)b * d.Hp + h) * d.CP + o) * d.KKp + 2 * k2 + ri] = to_bf16(acc[r]);
        }
    }
    if (k2 == 0) {
        const int padw = d.KKp - 2 * d.m2;
        for (int i = tid; i < d.Hp * d.CP * padw; i += blockDim.x) {
            const int p = i % padw, ho = i / padw;
            d.Z[((size_t)b * d.Hp * d.CP + ho) * d.KKp + 2 * d.m2 + p] = to_bf16(0.0f);
        }
    }
}

// Row inverse DFT + 1x1 convolution + bias (+ activation) for one (b, h).
__global__ __launch_bounds__(256) void k_fno_rowinv(FnoDev d, const __bf16* __restrict__ v,
                                                    __bf16* __restrict__ vout, int layer, int last) {
    const int b = blockIdx.x / d.Hp, h = blockIdx.x % d.Hp;
    const int tid = threadIdx.x, wave = tid >> 6, nw = blockDim.x >> 6;
    const size_t rowoff = ((size_t)b * d.Hp + h) * d.Wpad * d.CP;
    const __bf16* vrow = v + rowoff;
    const __bf16* Zrow = d.Z + ((size_t)b * d.Hp + h) * d.CP * d.KKp;
    const __bf16* Wc = d.Wc + (size_t)layer * d.CP * d.CP;
    const float* bias = d.bc + (size_t)layer * d.CP;
    const int Mt = d.Wpad / 32, Nt = d.CP / 32;
    for (int t = wave; t < Mt * Nt; t += nw) {
        const int mi = t / Nt, ni = t % Nt;
        f32x16 acc = {};
        acc = mma_tile(d.BinvT + (size_t)mi * 32 * d.KKp, d.KKp, Zrow + (size_t)ni * 32 * d.KKp,
                       d.KKp, d.KKp, acc);
        acc = mma_tile(vrow + (size_t)mi * 32 * d.CP, d.CP, Wc + (size_t)ni * 32 * d.CP, d.CP,
                       d.CP, acc);
        const int o = ni * 32 + acc_col();
        const float bo = bias[o];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int w = mi * 32 + acc_row(r);
            float val = acc[r] + bo;
            if (!last) val = act_f(d.act, val);
            if (w >= d.Wp) val = 0.0f;
            vout[rowoff + (size_t)w * d.CP + o] = to_bf16(val);
        }
    }
}

// Decoder: per output point, dec_layers hidden layers (bf16 operands, float32
// sums, decoder activation, rounded to bf16) and the output layer (float32 out).
template <int MAXD>
__global__ __launch_bounds__(256) void k_fno_dec(FnoDev d, const __bf16* __restrict__ v,
                                                 float* __restrict__ out) {
    const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t total = (size_t)d.B * d.H * d.W;
    if (idx >= total) return;
    const int w = (int)(idx % d.W);
    const int h = (int)((idx / d.W) % d.H);
    const int b = (int)(idx / ((size_t)d.W * d.H));
    const __bf16* vin = v + (((size_t)b * d.Hp + h) * d.Wpad + w) * d.CP;
    float a[MAXD], c[MAXD];
#pragma unroll
    for (int i = 0; i < MAXD; ++i) a[i] = i < d.CP ? from_bf16(vin[i]) : 0.0f;
    int din = d.CP;
    const __bf16* wp = d.decw;
    const float* bp = d.decb;
    for (int l = 0; l < d.dec_layers; ++l) {
#pragma unroll
        for (int s = 0; s < MAXD; ++s) {
            float acc = 0.0f;
            if (s < d.DSP) {
                acc = bp[s];
#pragma unroll
                for (int i = 0; i < MAXD; ++i)
                    if (i < din) acc = fmaf(from_bf16(wp[s * din + i]), a[i], acc);
                acc = from_bf16(to_bf16(act_f(d.dec_act, acc)));
                if (s >= d.dec_size) acc = 0.0f;
            }
            c[s] = acc;
        }
#pragma unroll
        for (int i = 0; i < MAXD; ++i) a[i] = c[i];
        wp += (size_t)d.DSP * din;
        bp += d.DSP;
        din = d.DSP;
    }
    for (int o = 0; o < d.cout; ++o) {
        float acc = bp[o];
#pragma unroll
        for (int i = 0; i < MAXD; ++i)
            if (i < din) acc = fmaf(from_bf16(wp[o * din + i]), a[i], acc);
        out[(((size_t)b * d.cout + o) * d.H + h) * d.W + w] = acc;
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
};

static int rup(int x, int m) { return (x + m - 1) / m * m; }

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
    d.cout = s.cout;
    d.act = s.act; d.dec_act = s.dec_act;
    if ((size_t)d.CP * d.Wpad * 2 > 64 * 1024) return fail(LBM_EUNSUPPORTED, "row of %d x %d too large for LDS", d.Wpad, d.CP);
    if (((size_t)d.R2 * d.CP * 4 + (size_t)d.CP * d.R2 * 2) > 64 * 1024)
        return fail(LBM_EUNSUPPORTED, "mode block too large for LDS");
    fno_model* m = new (std::nothrow) fno_model();
    if (!m) return fail(LBM_ENOMEM, "model allocation");
    m->spec = s;
    (void)hipGetDevice(&m->device);
    auto bail = [&](int code) { fno_model_destroy(m); return code; };

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
    // ---- DFT bases (angles reduced exactly in integers, values in double, RNE to bf16)
    const double two_pi = 6.283185307179586476925286766559;
    std::vector<uint16_t> EwT((size_t)d.KKp * d.Wpad, 0), BinvT((size_t)d.Wpad * d.KKp, 0);
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
    const uint16_t *u1, *u2, *u3, *u4, *u5, *u6, *u7;
    if ((rc = upload(m, l1w, &f1)) || (rc = upload(m, l1b, &f2)) || (rc = upload(m, l2w, &f3)) ||
        (rc = upload(m, l2b, &f4)) || (rc = upload(m, bc, &f5)) || (rc = upload(m, decb, &f6)) ||
        (rc = upload(m, Rmix, &u1)) || (rc = upload(m, Wc, &u2)) || (rc = upload(m, decw, &u3)) ||
        (rc = upload(m, EwT, &u4)) || (rc = upload(m, BinvT, &u5)) || (rc = upload(m, EcolA, &u6)) ||
        (rc = upload(m, EcolB, &u7)))
        return bail(rc);
    d.lift1w = f1; d.lift1b = f2; d.lift2w = f3; d.lift2b = f4; d.bc = f5; d.decb = f6;
    d.Rmix = reinterpret_cast<const __bf16*>(u1);
    d.Wc = reinterpret_cast<const __bf16*>(u2);
    d.decw = reinterpret_cast<const __bf16*>(u3);
    d.EwT = reinterpret_cast<const __bf16*>(u4);
    d.BinvT = reinterpret_cast<const __bf16*>(u5);
    d.EcolA = reinterpret_cast<const __bf16*>(u6);
    d.EcolB = reinterpret_cast<const __bf16*>(u7);
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
    L.Z = al((size_t)B * d.Hp * d.CP * d.KKp * 2);
    L.total = 2 * L.v + L.T + L.Z;
    return L;
}

extern "C" int fno_workspace_size(const fno_model* m, int32_t B, size_t* bytes) {
    if (!m || !bytes) return fail(LBM_EINVAL, "NULL argument");
    if (B < 1) return fail(LBM_EINVAL, "B = %d", B);
    *bytes = ws_layout(m->d, B).total;
    return LBM_OK;
}

extern "C" int fno_forward(const fno_model* m, const float* d_in, float* d_out, int32_t B,
                           void* d_ws, size_t ws_bytes, void* stream) {
    if (!m) return fail(LBM_EINVAL, "model is NULL");
    if (!d_in || !d_out || !d_ws) return fail(LBM_EINVAL, "NULL device buffer");
    if (B < 1 || (int64_t)B * m->d.Hp * m->d.Wpad > ((int64_t)1 << 31) / 64)
        return fail(LBM_EINVAL, "B = %d", B);
    if ((uintptr_t)d_ws % 256) return fail(LBM_EINVAL, "workspace not 256-byte aligned");
    FnoDev d = m->d;
    d.B = B;
    const WsLayout L = ws_layout(d, B);
    if (ws_bytes < L.total) return fail(LBM_EINVAL, "workspace %zu < %zu bytes", ws_bytes, L.total);
    unsigned char* ws = static_cast<unsigned char*>(d_ws);
    d.v0 = reinterpret_cast<__bf16*>(ws);
    d.v1 = reinterpret_cast<__bf16*>(ws + L.v);
    d.T = reinterpret_cast<__bf16*>(ws + 2 * L.v);
    d.Z = reinterpret_cast<__bf16*>(ws + 2 * L.v + L.T);
    hipStream_t st = (hipStream_t)stream;
    const size_t npts = (size_t)B * d.Hp * d.Wpad;
    k_fno_lift<<<(unsigned)((npts + 255) / 256), 256, 0, st>>>(d, d_in);
    const size_t lds_row = (size_t)d.CP * d.Wpad * 2;
    const size_t lds_col = (size_t)d.R2 * d.CP * 4 + (size_t)d.CP * d.R2 * 2;
    __bf16* cur = d.v0;
    __bf16* nxt = d.v1;
    for (int l = 0; l < d.L; ++l) {
        k_fno_rowfwd<<<B * d.Hpad, 256, lds_row, st>>>(d, cur);
        k_fno_col<<<B * d.m2, 256, lds_col, st>>>(d, l);
        k_fno_rowinv<<<B * d.Hp, 256, 0, st>>>(d, cur, nxt, l, l == d.L - 1);
        __bf16* t = cur; cur = nxt; nxt = t;
    }
    const size_t nout = (size_t)B * d.H * d.W;
    const int maxd = std::max(d.CP, d.DSP);
    if (maxd <= 32) k_fno_dec<32><<<(unsigned)((nout + 255) / 256), 256, 0, st>>>(d, cur, d_out);
    else k_fno_dec<64><<<(unsigned)((nout + 255) / 256), 256, 0, st>>>(d, cur, d_out);
    LBM_HIP(hipGetLastError());
    return LBM_OK;
}
