// lbm.hip -- D2Q9 BGK lattice Boltzmann hot path for gfx950 behind the C ABI of
// include/lbmfno.h: obstacle raster, link bits, equilibrium (re)initialisation,
// the fused pull-scheme collide+stream step, macroscopic fields and FP64 sums.
//
// Storage.  Populations live in two caller-owned float32 stores of 9 planes
// [ny][nx] (structure of arrays).  The store for time t holds, for every node y
// and direction p, the value that will be pulled into f_p(y + c_p, t) -- or, when
// y + c_p is solid or beyond a wall / open boundary, the value that bounces back
// into f_{opp p}(y, t) -- minus the weight w_p.  A step therefore reads one store
// with a pure gather (periodic wrap, halfway bounce-back from per-node link bits,
// Zou-He on the two open columns), computes the moments and the BGK + Guo
// collision in registers, and writes the other store in place order: 9 loads, 9
// stores and one link byte per fluid node, fully coalesced along x.
//
// Deviation storage (f - w) keeps FP32 rounding relative to the small
// non-equilibrium part of f, which the 1e-5 field tolerance against FP64 needs.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "common.hpp"

// No multiply-add contraction in the lattice kernels: every step kernel (one node
// or four nodes per lane, single or batched) then evaluates the same sequence of
// IEEE operations and gives bit-identical results, whichever the tuner picks.
#pragma clang fp contract(off)

namespace lbmfno {

static thread_local std::string g_err;

void set_error(const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
}

int fail(int code, const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

// --------------------------------------------------------------- kernels

constexpr int TX = 64;  // one wavefront along x
constexpr int TY = 4;   // four rows per workgroup

__global__ __launch_bounds__(256) void k_mask_raster(int nx, int ny, int wrap_x, int wrap_y,
                                                     const int64_t* __restrict__ shapes, int ns,
                                                     uint8_t* __restrict__ mask) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= nx) return;
    uint8_t solid = 0;
    for (int s = 0; s < ns && !solid; ++s) {
        const int64_t* p = shapes + 7 * s;
        int dx = i - (int)p[0], dy = j - (int)p[1];
        if (wrap_x) {
            dx %= nx;
            if (dx < 0) dx += nx;
            if (dx > nx / 2) dx -= nx;
        }
        if (wrap_y) {
            dy %= ny;
            if (dy < 0) dy += ny;
            if (dy > ny / 2) dy -= ny;
        }
        const int R = (int)p[6];
        if (dx > R || -dx > R || dy > R || -dy > R) continue;
        const int64_t X = dx, Y = dy;
        if (p[2] * X * X + p[3] * X * Y + p[4] * Y * Y <= p[5]) solid = 1;
    }
    mask[(size_t)j * nx + i] = solid;
}

// Link bits: bit q-1 (q = 1..8) is set when the pull source x - c_q is solid or
// lies beyond a non-periodic boundary (halfway bounce-back, or the unknown
// populations of a Zou-He column, which the closure overwrites).  Solid nodes
// store 0xFF; a fluid node can also have all eight links bounced (an isolated
// pocket), so 0xFF is disambiguated by the mask byte, which is read only then.
__global__ __launch_bounds__(256) void k_links(int nx, int ny, int bc_x, int bc_y,
                                               const uint8_t* __restrict__ mask,
                                               uint8_t* __restrict__ link) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= nx) return;
    const int n = j * nx + i;
    unsigned bits = 0;
#pragma unroll
    for (int q = 1; q < 9; ++q) {
        int si = i - cx_of(q), sj = j - cy_of(q);
        bool out = false;
        if (si < 0 || si >= nx) {
            if (bc_x == LBM_BC_PERIODIC) si = (si + nx) % nx; else out = true;
        }
        if (sj < 0 || sj >= ny) {
            if (bc_y == LBM_BC_PERIODIC) sj = (sj + ny) % ny; else out = true;
        }
        if (out || mask[sj * nx + si]) bits |= 1u << (q - 1);
    }
    link[n] = mask[n] ? (uint8_t)0xFF : (uint8_t)bits;
}

__device__ __forceinline__ bool is_solid(unsigned lk, const uint8_t* __restrict__ mask, int n) {
    return lk == 0xFFu && mask[n] != 0;
}

struct LatticeGeom {
    int nx, ny, N, gridx, bc_x, bc_y;
};

// Node y + c_p if it is a fluid node inside the domain, else -1.
__device__ __forceinline__ int push_target(const LatticeGeom& g, const uint8_t* __restrict__ mask,
                                           int i, int j, int p) {
    int ti = i + cx_of(p), tj = j + cy_of(p);
    if (ti < 0 || ti >= g.nx) {
        if (g.bc_x != LBM_BC_PERIODIC) return -1;
        ti = (ti + g.nx) % g.nx;
    }
    if (tj < 0 || tj >= g.ny) {
        if (g.bc_y != LBM_BC_PERIODIC) return -1;
        tj = (tj + g.ny) % g.ny;
    }
    const int t = tj * g.nx + ti;
    return mask[t] ? -1 : t;
}

// c_q . (x, y) for the integer velocity c_q, as additions only: with contraction
// off, a product by a literal 0 or 1 would otherwise be evaluated.
template <int Q, typename R>
__device__ __forceinline__ R cdot(R x, R y) {
    constexpr int cx = cx_of(Q), cy = cy_of(Q);
    R a = R(0);
    if constexpr (cx == 1) a = x;
    if constexpr (cx == -1) a = -x;
    if constexpr (cy == 1) a = (cx == 0) ? y : a + y;
    if constexpr (cy == -1) a = (cx == 0) ? -y : a - y;
    return a;
}

// Deviation equilibrium f_eq_p - w_p = w_p [(rho - 1) + rho (3 c.u + 4.5 (c.u)^2 - 1.5 u.u)],
// with every multiply-add written as an explicit fma (one fixed operation order).
// usq15 = 1.5 u.u.
template <int P, typename R>
__device__ __forceinline__ R feq_dev(R drho, R rho, R ux, R uy, R usq15) {
    const R cu = cdot<P, R>(ux, uy);
    const R t = fma(cu, fma(R(4.5), cu, R(3)), -usq15);
    return (R)w_of_d(P) * fma(rho, t, drho);
}

template <int P, typename R>
__device__ __forceinline__ R feq_dev(R drho, R rho, R ux, R uy) {
    return feq_dev<P, R>(drho, rho, ux, uy, R(1.5) * fma(ux, ux, uy * uy));
}

__device__ __forceinline__ double feq_dev_rt(int p, double drho, double rho, double ux, double uy) {
    switch (p) {
        case 0: return feq_dev<0>(drho, rho, ux, uy);
        case 1: return feq_dev<1>(drho, rho, ux, uy);
        case 2: return feq_dev<2>(drho, rho, ux, uy);
        case 3: return feq_dev<3>(drho, rho, ux, uy);
        case 4: return feq_dev<4>(drho, rho, ux, uy);
        case 5: return feq_dev<5>(drho, rho, ux, uy);
        case 6: return feq_dev<6>(drho, rho, ux, uy);
        case 7: return feq_dev<7>(drho, rho, ux, uy);
        default: return feq_dev<8>(drho, rho, ux, uy);
    }
}

// Derivative of the field u along x (axis 0) or y (axis 1) at fluid node (i, j):
// central difference when both neighbours are fluid nodes inside the domain
// (periodic axes wrap), one-sided when one is, zero when neither is.
__device__ __forceinline__ double vel_deriv(const LatticeGeom& g, const uint8_t* __restrict__ mask,
                                            const float* __restrict__ u, int i, int j, int axis) {
    bool ok[2];
    int nb[2];
#pragma unroll
    for (int s = 0; s < 2; ++s) {
        const int d = s == 0 ? 1 : -1;
        int a = i + (axis == 0 ? d : 0), b = j + (axis == 1 ? d : 0);
        bool inside = true;
        if (a < 0 || a >= g.nx) {
            if (g.bc_x == LBM_BC_PERIODIC) a = (a + g.nx) % g.nx; else inside = false;
        }
        if (b < 0 || b >= g.ny) {
            if (g.bc_y == LBM_BC_PERIODIC) b = (b + g.ny) % g.ny; else inside = false;
        }
        nb[s] = inside ? b * g.nx + a : 0;
        ok[s] = inside && mask[nb[s]] == 0;
    }
    const double u0 = u[j * g.nx + i];
    if (ok[0] && ok[1]) return 0.5 * ((double)u[nb[0]] - (double)u[nb[1]]);
    if (ok[0]) return (double)u[nb[0]] - u0;
    if (ok[1]) return u0 - (double)u[nb[1]];
    return 0.0;
}

// Scatter f(0) into a store: slot (p, y) receives what y + c_p pulls, or, when that
// node is solid/outside, what bounces back into y as opp(p).
//   FROM_FIELDS: f_q(x) = f_eq_q(rho(x), u(x))        (re-initialisation)
//   else:        f_q(x) = given populations (absolute) (state restore)
// NEQ (with FROM_FIELDS): add the first-order non-equilibrium part of the
// pre-collision populations, -tau w_q rho / c_s^2 (c_q c_q - c_s^2 I) : grad u.
// MASS: rho is shifted by (*m_cur - *m_in) * inv_fluid on every node (the current
// state's fluid mass minus the handed-over fields' fluid sum, both reduced on the
// device, over the fluid node count).
template <bool FROM_FIELDS, bool NEQ, bool MASS = false>
__global__ __launch_bounds__(256) void k_scatter(LatticeGeom g, const uint8_t* __restrict__ mask,
                                                 const float* __restrict__ rho,
                                                 const float* __restrict__ ux,
                                                 const float* __restrict__ uy,
                                                 const float* __restrict__ fin,
                                                 float* __restrict__ dst, double tau,
                                                 const double* __restrict__ m_cur = nullptr,
                                                 const double* __restrict__ m_in = nullptr,
                                                 double inv_fluid = 0.0) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int j = blockIdx.y;
    if (i >= g.nx) return;
    const int n = j * g.nx + i;
    const size_t N = (size_t)g.N;
    if (mask[n]) {
#pragma unroll
        for (int p = 0; p < 9; ++p) dst[p * N + n] = 0.0f;
        return;
    }
#pragma unroll
    for (int p = 0; p < 9; ++p) {
        const int t = p == 0 ? n : push_target(g, mask, i, j, p);
        const int src = t >= 0 ? t : n;
        const int dir = t >= 0 ? p : opp_of(p);
        float v;
        if (FROM_FIELDS) {
            const double r = MASS ? (double)rho[src] + (*m_cur - *m_in) * inv_fluid : (double)rho[src];
            double e = feq_dev_rt(dir, r - 1.0, r, ux[src], uy[src]);
            if (NEQ) {
                const int si = src % g.nx, sj = src / g.nx;
                const double dxux = vel_deriv(g, mask, ux, si, sj, 0);
                const double dyux = vel_deriv(g, mask, ux, si, sj, 1);
                const double dxuy = vel_deriv(g, mask, uy, si, sj, 0);
                const double dyuy = vel_deriv(g, mask, uy, si, sj, 1);
                const double cx = cx_of(dir), cy = cy_of(dir);
                const double contr = (cx * cx - 1.0 / 3.0) * dxux + cx * cy * (dyux + dxuy) +
                                     (cy * cy - 1.0 / 3.0) * dyuy;
                e -= 3.0 * tau * w_of_d(dir) * r * contr;
            }
            v = (float)e;
        } else {
            v = (float)((double)fin[dir * N + src] - w_of_d(dir));
        }
        dst[p * N + n] = v;
    }
}

struct StepArgs {
    const float* __restrict__ src;
    float* __restrict__ dst;
    const uint8_t* __restrict__ link;
    const uint8_t* __restrict__ mask;
    float* __restrict__ drho_out;
    LatticeGeom g;
    double omega, guo, gx, gy, u_in, rho_out;
    double omega_m, guo_m;  // TRT: odd-part relaxation rate and Guo factor
};

// Pull gather of f(t) at node (i, j) from the deviation store: direction q reads
// plane q at x - c_q, or, when link bit q-1 is set, plane opp(q) at x itself.
// The nine streaming loads are issued unconditionally (every address is valid), so
// they overlap the link-byte load instead of waiting for it; the few bounced
// directions are re-read afterwards.  Offsets are formed per direction (an
// indexed local array would be placed in scratch memory).
template <typename R>
__device__ __forceinline__ void gather_stream(const float* __restrict__ src, const LatticeGeom& g,
                                              int i, int j, int n, R f[9]) {
    const int im = i == 0 ? g.nx - 1 : i - 1, ip = i == g.nx - 1 ? 0 : i + 1;
    const int jm = j == 0 ? g.ny - 1 : j - 1, jp = j == g.ny - 1 ? 0 : j + 1;
    const int r0 = j * g.nx, rm = jm * g.nx, rp = jp * g.nx;
    const int N = g.N;
    f[0] = (R)src[n];
    f[1] = (R)src[1 * N + r0 + im];
    f[2] = (R)src[2 * N + rm + i];
    f[3] = (R)src[3 * N + r0 + ip];
    f[4] = (R)src[4 * N + rp + i];
    f[5] = (R)src[5 * N + rm + im];
    f[6] = (R)src[6 * N + rm + ip];
    f[7] = (R)src[7 * N + rp + ip];
    f[8] = (R)src[8 * N + rp + im];
}

template <typename R>
__device__ __forceinline__ void gather_bounce(const float* __restrict__ src, const LatticeGeom& g,
                                              unsigned lk, int n, R f[9]) {
    if (lk == 0u) return;
    const int N = g.N;
#define LBM_BOUNCE(Q) \
    if ((lk >> (Q - 1)) & 1u) f[Q] = (R)src[opp_of(Q) * N + n];
    LBM_BOUNCE(1) LBM_BOUNCE(2) LBM_BOUNCE(3) LBM_BOUNCE(4)
    LBM_BOUNCE(5) LBM_BOUNCE(6) LBM_BOUNCE(7) LBM_BOUNCE(8)
#undef LBM_BOUNCE
}

template <typename R>
__device__ __forceinline__ void gather(const float* __restrict__ src, const LatticeGeom& g,
                                       unsigned lk, int i, int j, int n, R f[9]) {
    gather_stream<R>(src, g, i, j, n, f);
    gather_bounce<R>(src, g, lk, n, f);
}

// Zou-He closures in deviation variables (w_1 = w_3, w_5 = w_7, w_6 = w_8 and
// sum of the known weights = 1 make the shifted formulas identical in form).
// Written branch-free (both closures evaluated, results selected) so the
// population array stays in registers.
template <typename R>
__device__ __forceinline__ void zouhe(R f[9], int i, int nx, R u_in, R rho_out) {
    const bool inl = i == 0, outl = i == nx - 1;
    const R h = R(0.5) * (f[2] - f[4]);
    // inlet x = 0: unknown f1, f5, f8 from u = (u_in, 0)
    const R s_in = f[0] + f[2] + f[4] + R(2) * (f[3] + f[6] + f[7]);
    const R ru_in = (R(1) + (s_in + u_in) / (R(1) - u_in)) * u_in;
    const R f1 = f[3] + (R(2) / R(3)) * ru_in;
    const R f5 = f[7] - h + (R(1) / R(6)) * ru_in;
    const R f8 = f[6] + h + (R(1) / R(6)) * ru_in;
    // outlet x = nx - 1: unknown f3, f6, f7 from rho = rho_out, u_y = 0
    const R s_out = f[0] + f[2] + f[4] + R(2) * (f[1] + f[5] + f[8]);
    const R ru_out = ((R(1) - rho_out) + s_out);  // rho_out * u_x
    const R f3 = f[1] - (R(2) / R(3)) * ru_out;
    const R f6 = f[8] - h - (R(1) / R(6)) * ru_out;
    const R f7 = f[5] + h - (R(1) / R(6)) * ru_out;
    f[1] = inl ? f1 : f[1];
    f[5] = inl ? f5 : f[5];
    f[8] = inl ? f8 : f[8];
    f[3] = outl ? f3 : f[3];
    f[6] = outl ? f6 : f[6];
    f[7] = outl ? f7 : f[7];
}

template <typename R>
struct Moments {
    R drho, rho, ux, uy;
};

template <bool FORCE, typename R>
__device__ __forceinline__ Moments<R> moments(const R f[9], R gx, R gy) {
    Moments<R> m;
    m.drho = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
    m.rho = R(1) + m.drho;
    const R jx = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
    const R jy = (f[2] - f[4]) + (f[5] - f[8]) + (f[6] - f[7]);
    const R inv = R(1) / m.rho;
    if (FORCE) {
        m.ux = fma(jx, inv, R(0.5) * gx);
        m.uy = fma(jy, inv, R(0.5) * gy);
    } else {
        m.ux = jx * inv;
        m.uy = jy * inv;
    }
    return m;
}

// Post-collision deviation of direction Q: f - omega (f - f_eq) (+ Guo term
// guo w rho [3 (c - u).g + 9 (c.u)(c.g)]), usq15 = 1.5 u.u of the node.
template <int Q, bool FORCE, typename R>
__device__ __forceinline__ float collide_q(R fq, const Moments<R>& m, R omega, R guo, R gx, R gy,
                                           R usq15) {
    const R fe = feq_dev<Q, R>(m.drho, m.rho, m.ux, m.uy, usq15);
    R out = fma(-omega, fq - fe, fq);
    if (FORCE) {
        const R cu = cdot<Q, R>(m.ux, m.uy);
        const R cg = cdot<Q, R>(gx, gy);
        const R ug = fma(m.ux, gx, m.uy * gy);
        const R t = fma(R(9) * cu, cg, R(3) * (cg - ug));
        out = fma(guo * (R)w_of_d(Q) * m.rho, t, out);
    }
    return (float)out;
}

template <int Q, bool FORCE, typename R>
__device__ __forceinline__ float collide_q(R fq, const Moments<R>& m, R omega, R guo, R gx, R gy) {
    return collide_q<Q, FORCE, R>(fq, m, omega, guo, gx, gy, R(1.5) * fma(m.ux, m.ux, m.uy * m.uy));
}

// Register arithmetic "lean" (LBM_ARITH_LEAN): FP32 everywhere except where the
// rounding would act as a force.  Rounding the velocity to FP32 before the linear
// equilibrium term w (drho + 3 rho c.u) gives every node a momentum bias that is
// nearly constant in time for slowly varying flow, i.e. a spurious body force.  So
// the moment sums stay FP32, u is formed in FP64 (reciprocal of rho from the FP32
// v_rcp refined by one FP64 Newton step: relative error ~1e-14), and the linear term
// is evaluated in FP64 and rounded once; the quadratic terms, the forcing and the
// relaxation are FP32.
struct Lean {};

template <int Q, bool FORCE>
__device__ __forceinline__ float collide_q_lean(float fq, double dr64, double rho3, double ux, double uy,
                                                float rho, float ux32, float uy32, float usq15,
                                                float omega, float guo, float gx, float gy) {
    const float lin = (float)(w_of_d(Q) * fma(rho3, cdot<Q, double>(ux, uy), dr64));
    const float cu = cdot<Q, float>(ux32, uy32);
    const float quad = w_of(Q) * rho * fmaf(4.5f * cu, cu, -usq15);
    const float fe = lin + quad;
    float out = fmaf(-omega, fq - fe, fq);
    if (FORCE) {
        const float cg = cdot<Q, float>(gx, gy);
        const float ug = fmaf(ux32, gx, uy32 * gy);
        const float t = fmaf(9.0f * cu, cg, 3.0f * (cg - ug));
        out = fmaf(guo * w_of(Q) * rho, t, out);
    }
    return out;
}

// Two-relaxation-time collision in the lean arithmetic (an extension; the paper
// uses BGK).  The pair (q, opp q) splits into the parts even and odd under
// c -> -c: f_e = (f_q + f_qb)/2 relaxes to w (drho + rho (4.5 (c.u)^2 - 1.5 u^2))
// at rate omega+ = 1/tau, f_o = (f_q - f_qb)/2 to 3 w rho c.u at rate omega-; the
// Guo source's even part w rho (9 (c.u)(c.g) - 3 u.g) gets 1 - omega+/2, its odd
// part 3 w rho c.g gets 1 - omega-/2.  The linear equilibrium terms are formed in
// FP64 as in Lean.
struct LeanTRT {};

template <int Q, int QB, bool FORCE>
__device__ __forceinline__ void collide_pair_trt(float v[9], double dr64, double rho3, double ux,
                                                 double uy, float rho, float ux32, float uy32,
                                                 float usq15, float omp, float omm, float guop,
                                                 float guom, float gx, float gy) {
    const float even_lin = (float)(w_of_d(Q) * dr64);
    const float odd_lin = (float)(w_of_d(Q) * rho3 * cdot<Q, double>(ux, uy));
    const float cu = cdot<Q, float>(ux32, uy32);
    const float quad = w_of(Q) * rho * fmaf(4.5f * cu, cu, -usq15);
    const float ne = 0.5f * (v[Q] + v[QB]) - (even_lin + quad);
    const float no = 0.5f * (v[Q] - v[QB]) - odd_lin;
    float a = fmaf(-omp, ne, fmaf(-omm, no, v[Q]));
    float b = fmaf(-omp, ne, fmaf(omm, no, v[QB]));
    if (FORCE) {
        const float cg = cdot<Q, float>(gx, gy);
        const float ug = fmaf(ux32, gx, uy32 * gy);
        const float se = w_of(Q) * rho * fmaf(9.0f * cu, cg, -3.0f * ug);
        const float so = 3.0f * w_of(Q) * rho * cg;
        a = fmaf(guop, se, fmaf(guom, so, a));
        b = fmaf(guop, se, fmaf(-guom, so, b));
    }
    v[Q] = a;
    v[QB] = b;
}

// Boundary closure, moments and collision of one fluid node in arithmetic R
// (float, double, Lean or LeanTRT) on its gathered float populations v (replaced
// by the post-collision deviations); returns drho.  Every step kernel calls this,
// so all of them evaluate one operation sequence.  ZB: evaluate the Zou-He
// closures only on the two boundary columns (a branch) instead of on every node
// with a select; the same values either way.  The branch pays on the 512-lane
// fused tiles (8192x4096 lattice 141 -> 147 GLUPS, batched flows 141 -> 144) and
// costs on the 1024-lane ones (1024x512: 18.5 -> 18.8 us per launch).
template <bool ZH, bool FORCE, typename R, bool ZB = false>
__device__ __forceinline__ float collide_node(float v[9], int x, int nx, const StepArgs& a) {
    if constexpr (std::is_same<R, Lean>::value || std::is_same<R, LeanTRT>::value) {
        if (ZH && (!ZB || x == 0 || x == nx - 1)) zouhe<float>(v, x, nx, (float)a.u_in, (float)a.rho_out);
        const float dr = ((v[0] + v[1]) + (v[2] + v[3])) + ((v[4] + v[5]) + (v[6] + v[7])) + v[8];
        const float jx = (v[1] - v[3]) + (v[5] - v[6]) + (v[8] - v[7]);
        const float jy = (v[2] - v[4]) + (v[5] - v[8]) + (v[6] - v[7]);
        const double dr64 = (double)dr, rho64 = 1.0 + dr64;
        const double r0 = (double)__builtin_amdgcn_rcpf((float)rho64);
        const double inv = fma(r0, fma(-rho64, r0, 1.0), r0);
        double ux, uy;
        if (FORCE) {
            ux = fma((double)jx, inv, 0.5 * a.gx);
            uy = fma((double)jy, inv, 0.5 * a.gy);
        } else {
            ux = (double)jx * inv;
            uy = (double)jy * inv;
        }
        const double rho3 = 3.0 * rho64;
        const float rho = (float)rho64, ux32 = (float)ux, uy32 = (float)uy;
        const float usq15 = 1.5f * fmaf(ux32, ux32, uy32 * uy32);
        const float om = (float)a.omega, guo = (float)a.guo, gx = (float)a.gx, gy = (float)a.gy;
        if constexpr (std::is_same<R, LeanTRT>::value) {
            const float omm = (float)a.omega_m, guom = (float)a.guo_m;
            v[0] = collide_q_lean<0, FORCE>(v[0], dr64, rho3, ux, uy, rho, ux32, uy32, usq15, om, guo, gx, gy);
#define LBM_TRT(Q, QB) \
    collide_pair_trt<Q, QB, FORCE>(v, dr64, rho3, ux, uy, rho, ux32, uy32, usq15, om, omm, guo, guom, gx, gy);
            LBM_TRT(1, 3) LBM_TRT(2, 4) LBM_TRT(5, 7) LBM_TRT(6, 8)
#undef LBM_TRT
        } else {
#define LBM_LEAN(Q) v[Q] = collide_q_lean<Q, FORCE>(v[Q], dr64, rho3, ux, uy, rho, ux32, uy32, usq15, om, guo, gx, gy);
            LBM_LEAN(0) LBM_LEAN(1) LBM_LEAN(2) LBM_LEAN(3) LBM_LEAN(4)
            LBM_LEAN(5) LBM_LEAN(6) LBM_LEAN(7) LBM_LEAN(8)
#undef LBM_LEAN
        }
        return dr;
    } else {
        R f[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) f[q] = (R)v[q];
        if (ZH) zouhe<R>(f, x, nx, (R)a.u_in, (R)a.rho_out);
        const R gx = (R)a.gx, gy = (R)a.gy, om = (R)a.omega, guo = (R)a.guo;
        const Moments<R> m = moments<FORCE, R>(f, gx, gy);
        v[0] = collide_q<0, FORCE, R>(f[0], m, om, guo, gx, gy);
        v[1] = collide_q<1, FORCE, R>(f[1], m, om, guo, gx, gy);
        v[2] = collide_q<2, FORCE, R>(f[2], m, om, guo, gx, gy);
        v[3] = collide_q<3, FORCE, R>(f[3], m, om, guo, gx, gy);
        v[4] = collide_q<4, FORCE, R>(f[4], m, om, guo, gx, gy);
        v[5] = collide_q<5, FORCE, R>(f[5], m, om, guo, gx, gy);
        v[6] = collide_q<6, FORCE, R>(f[6], m, om, guo, gx, gy);
        v[7] = collide_q<7, FORCE, R>(f[7], m, om, guo, gx, gy);
        v[8] = collide_q<8, FORCE, R>(f[8], m, om, guo, gx, gy);
        return (float)m.drho;
    }
}

// One fused step t -> t+1 for one node per thread.  R selects the collision
// arithmetic (Lean by default, double or float); the stores are float either way.
template <bool ZH, bool FORCE, bool WDRHO, bool NT, typename R>
__device__ __forceinline__ void step_node(const StepArgs& a, int bx, int by) {
    const int i = bx * TX + threadIdx.x, j = by * TY + threadIdx.y;
    if (i >= a.g.nx || j >= a.g.ny) return;
    const int n = j * a.g.nx + i;
    const unsigned lk = a.link[n];
    float f[9];
    gather_stream<float>(a.src, a.g, i, j, n, f);
    if (is_solid(lk, a.mask, n)) return;
    gather_bounce<float>(a.src, a.g, lk, n, f);
    const float drho = collide_node<ZH, FORCE, R>(f, i, a.g.nx, a);
    if (WDRHO) a.drho_out[n] = drho;
    float* __restrict__ d = a.dst + n;
    const size_t N = (size_t)a.g.N;
    // Stores that overflow the last-level cache stream past it (non-temporal);
    // a lattice whose two stores fit keeps them cached for the next step.
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        if (NT) __builtin_nontemporal_store(f[q], d + q * N); else d[q * N] = f[q];
    }
}

template <bool ZH, bool FORCE, bool WDRHO, bool NT, typename R>
__global__ __launch_bounds__(256) void k_bgk_step(StepArgs a) {
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int by = b / a.g.gridx;
    step_node<ZH, FORCE, WDRHO, NT, R>(a, b - by * a.g.gridx, by);
}

// S fused steps per launch (temporal blocking).  A workgroup of TX x RY lanes
// owns a TX x RY tile.  Level 0 advances the tile and the (S-1)-node ring around
// it by one step, gathering from the store in global memory as the one-step
// kernel does, and keeps the post-collision values in LDS.  Each further level
// advances a ring one node narrower from the level before in LDS (k_bgk_multi:
// in place, in the two-phase layout described at aa_read; the batched kernel: in
// the pull layout, the new values waiting in registers across a barrier before
// they overwrite the LDS copy); the last level advances the tile alone and only
// its result is stored.  Every
// level calls collide_node on the same float inputs as a one-step launch, so the
// result is bit-identical to S one-step launches, while one load and one store of
// the populations serve S steps.  Ring nodes outside a non-periodic axis, and
// solid ring nodes, are never pulled (their links bounce) and are skipped; on a
// periodic axis the ring wraps.
//
// Shapes in use (lattice update rates measured on 1024x512, 512x256, 128x128 and
// 8192x4096 porous flows):
//   S = 2, 64 x 8   cache-resident lattices, LBM_KERNEL_PAIR
//   S = 2, 64 x 4   lattices streamed from HBM, LBM_KERNEL_PAIR, and the batch
//   S = 5, 64 x 16  cache-resident lattices whose grid gives every CU two
//                   workgroups (1024x512: 119.7 against 116.0 GLUPS for S = 4 and
//                   117.5 for S = 6 with the levels updated in place; 66 KB of LDS)
//   S = 4, 64 x 8   smaller cache-resident lattices (512x256: 52.0 against 49.4 for
//                   S = 3 and 49.8 for S = 5 with the levels updated in place)
//   S = 4, 64 x 8   lattices streamed from HBM (8192x4096: 127 against 97; S = 3
//                   reaches 119, 64 x 16 tiles 113)
// Deeper blocking trades redundant ring collisions (29 % at S = 2, 64 x 8; 45 %
// at S = 4, 64 x 8; 34 % at S = 5, 64 x 16) for fewer global-memory round trips;
// on 1024x512 the vector ALUs are 60 % busy, the rest is memory latency and the
// barriers between levels.
template <int S, int RY>
struct Ring {
    static constexpr int W(int lvl) { return TX + 2 * (S - 1 - lvl); }
    static constexpr int H(int lvl) { return RY + 2 * (S - 1 - lvl); }
    static constexpr int LN(int lvl) { return W(lvl) * H(lvl); }
};

// Pull f at LDS position c of a level with row width W and plane stride LN: the
// streaming neighbours, or the node's own opposite population on a bounced link.
__device__ __forceinline__ void pull_lds(const float* __restrict__ P, int W, int LN, int c, unsigned lk,
                                         float f[9]) {
    f[0] = P[0 * LN + c];
    f[1] = P[1 * LN + c - 1];
    f[2] = P[2 * LN + c - W];
    f[3] = P[3 * LN + c + 1];
    f[4] = P[4 * LN + c + W];
    f[5] = P[5 * LN + c - W - 1];
    f[6] = P[6 * LN + c - W + 1];
    f[7] = P[7 * LN + c + W + 1];
    f[8] = P[8 * LN + c + W - 1];
    if (lk != 0u) {
#define LBM_BBL(Q) if ((lk >> (Q - 1)) & 1u) f[Q] = P[opp_of(Q) * LN + c];
        LBM_BBL(1) LBM_BBL(2) LBM_BBL(3) LBM_BBL(4) LBM_BBL(5) LBM_BBL(6) LBM_BBL(7) LBM_BBL(8)
#undef LBM_BBL
    }
}

// In-place two-phase layout of a fused tile's levels in LDS (the "AA" access
// pattern of Bailey, Myre, Walsh, Lilja & Saar, 2009).  A level of type A reads a
// node's incoming populations from the node's own slots and writes the outgoing
// ones back into its own slots, each into the opposite direction's slot; a level of
// type B reads each incoming population from the slot of the neighbour it comes from
// and writes each outgoing one into the slot of the neighbour it goes to.  Either
// way the slots a lane writes are slots only it reads, so a level updates in place,
// with no barrier between its reads and its writes and no copy held in registers.
// A blocked link (solid or outside neighbour) bounces: B reads the node's own slot
// of that direction, A the neighbour's slot of the opposite one, which is where the
// node itself wrote it one level earlier.  Level 0 (gathered from global memory)
// writes like A; a level L >= 1 reads and writes like B for odd L, like A for even
// L.  Every level uses level 0's layout: row width W0, plane size LN0, and c is a
// node's position in it.  The values are the pull scheme's, bit for bit.
template <int W0>
__device__ __forceinline__ constexpr int aa_off(int q) { return cx_of(q) + cy_of(q) * W0; }

template <bool B, int W0, int LN0>
__device__ __forceinline__ void aa_read(const float* __restrict__ P, int c, unsigned lk, float f[9]) {
#pragma unroll
    for (int q = 0; q < 9; ++q) f[q] = B ? P[opp_of(q) * LN0 + c - aa_off<W0>(q)] : P[q * LN0 + c];
    if (lk != 0u) {
#pragma unroll
        for (int q = 1; q < 9; ++q)
            if ((lk >> (q - 1)) & 1u) f[q] = B ? P[q * LN0 + c] : P[opp_of(q) * LN0 + c - aa_off<W0>(q)];
    }
}

template <bool B, int W0, int LN0>
__device__ __forceinline__ void aa_write(float* __restrict__ P, int c, const float f[9]) {
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        if (B) P[q * LN0 + c + aa_off<W0>(q)] = f[q];
        else P[opp_of(q) * LN0 + c] = f[q];
    }
}

// Lattice node of ring position (i, j), wrapped on a periodic axis; false when the
// position lies outside a non-periodic axis.
__device__ __forceinline__ bool ring_node(const LatticeGeom& g, int& i, int& j) {
    if (i < 0 || i >= g.nx) {
        if (g.bc_x != LBM_BC_PERIODIC) return false;
        i = ((i % g.nx) + g.nx) % g.nx;
    }
    if (j < 0 || j >= g.ny) {
        if (g.bc_y != LBM_BC_PERIODIC) return false;
        j = ((j % g.ny) + g.ny) % g.ny;
    }
    return true;
}

// Link codes of the level-0 region of a fused tile, kept in LDS for every level:
// the node's link bits, or LK_SKIP for a solid node or a position outside a
// non-periodic axis.
constexpr unsigned short LK_SKIP = 0x100;

// A level of LN nodes takes IT passes of nth lanes, the last one partial: the
// waves that have a node in it do one collision more than the rest, and the
// barrier at the end of the level waits for them.  On the 1024-lane tiles their
// instructions are issued first (a wave priority above the others' until the
// level's barrier; on level 0 from the link-code reads on), so that the others
// fill the issue slots they leave: 1024x512 porous flow 19.35 -> 18.25 us per
// four-step launch.  The 512-lane 64x8 tiles run
// in many rounds of workgroups and got slower with it (8192x4096 lattice 141 ->
// 132 GLUPS, batched flows 141 -> 134), so they keep one priority.
template <int NTH>
__device__ __forceinline__ void long_waves_first(int tid, int IT, int LN) {
    if constexpr (NTH == 1024)
        if ((tid & ~63) + (IT - 1) * NTH < LN) __builtin_amdgcn_s_setprio(2);
}
template <int NTH>
__device__ __forceinline__ void same_priority() {
    if constexpr (NTH == 1024) __builtin_amdgcn_s_setprio(0);
}

// Levels 1 .. S-2: the ring S-1-LVL nodes wide, from level LVL-1 in LDS.  AA:
// updated in place in the two-phase layout (type B for odd LVL, A for even);
// otherwise the pull layout, each level in its own compact layout, the new values
// held in registers across a barrier before they overwrite the old (the batched
// kernel, whose four boundary and forcing variants share one launch, runs 4 %
// faster this way).
template <int S, int RY, int LVL, bool ZH, bool FORCE, typename R, bool AA>
__device__ __forceinline__ void ring_levels(const StepArgs& a, int x0, int y0, int tid, float* __restrict__ P,
                                            const unsigned short* __restrict__ LKS) {
    if constexpr (LVL < S - 1) {
        using G = Ring<S, RY>;
        constexpr int W = G::W(LVL), LN = G::LN(LVL), W0 = G::W(0), LN0 = G::LN(0);
        constexpr int WP = G::W(LVL - 1), LNP = G::LN(LVL - 1);
        constexpr int IT = (LN + TX * RY - 1) / (TX * RY);
        constexpr int RING = S - 1 - LVL;
        constexpr bool B = (LVL & 1) != 0;
        float v[AA ? 1 : IT][9];
        bool ok[AA ? 1 : IT];
        long_waves_first<TX * RY>(tid, IT, LN);
#pragma unroll
        for (int t = 0; t < IT; ++t) {
            if constexpr (!AA) ok[t] = false;
            const int e = tid + t * TX * RY;
            if (e >= LN) continue;
            const int ly = e / W, lx = e - ly * W;
            const int c = (ly + LVL) * W0 + lx + LVL;
            const unsigned lk = LKS[c];
            if (lk == LK_SKIP) continue;
            int i = x0 - RING + lx, j = y0 - RING + ly;
            (void)ring_node(a.g, i, j);  // wraps i on a periodic axis (the node is inside)
            float f[9];
            if constexpr (AA) {
                aa_read<B, W0, LN0>(P, c, lk, f);
            } else {
                pull_lds(P, WP, LNP, (ly + 1) * WP + lx + 1, lk, f);
            }
            (void)collide_node<ZH, FORCE, R, TX * RY != 1024>(f, i, a.g.nx, a);
            if constexpr (AA) {
                aa_write<B, W0, LN0>(P, c, f);
            } else {
#pragma unroll
                for (int q = 0; q < 9; ++q) v[t][q] = f[q];
                ok[t] = true;
            }
        }
        same_priority<TX * RY>();
        __syncthreads();
        if constexpr (!AA) {
#pragma unroll
            for (int t = 0; t < IT; ++t) {
                if (!ok[t]) continue;
#pragma unroll
                for (int q = 0; q < 9; ++q) P[q * LN + tid + t * TX * RY] = v[t][q];
            }
            __syncthreads();
        }
        ring_levels<S, RY, LVL + 1, ZH, FORCE, R, AA>(a, x0, y0, tid, P, LKS);
    }
}

template <int S, int RY, bool ZH, bool FORCE, bool NT, typename R, bool AA>
__device__ __forceinline__ void step_multi(const StepArgs& a, int bx, int by, float* __restrict__ P,
                                           unsigned short* __restrict__ LKS) {
    using G = Ring<S, RY>;
    constexpr int W0 = G::W(0), LN0 = G::LN(0);
    constexpr int NTH = TX * RY, IT0 = (LN0 + NTH - 1) / NTH;
    const int x0 = bx * TX, y0 = by * RY;
    const int nx = a.g.nx, ny = a.g.ny;
    const int tid = threadIdx.y * TX + threadIdx.x;
    // level 0: a lane's IT0 nodes in three passes (link codes, then every
    // population load, then the collisions), so that their memory latencies overlap;
    // the link codes go to LDS for the later levels
    unsigned code[IT0];
    int ii[IT0], jj[IT0];
    long_waves_first<NTH>(tid, IT0, LN0);
#pragma unroll
    for (int t = 0; t < IT0; ++t) {
        code[t] = LK_SKIP;
        const int e = tid + t * NTH;
        if (e >= LN0) continue;
        const int ly = e / W0, lx = e - ly * W0;
        int i = x0 - (S - 1) + lx, j = y0 - (S - 1) + ly;
        if (ring_node(a.g, i, j)) {
            const int n = j * nx + i;
            const unsigned lk = a.link[n];
            if (!is_solid(lk, a.mask, n)) code[t] = lk;
        }
        ii[t] = i;
        jj[t] = j;
        LKS[e] = (unsigned short)code[t];
    }
    float f[IT0][9];
#pragma unroll
    for (int t = 0; t < IT0; ++t)
        if (code[t] != LK_SKIP) gather_stream<float>(a.src, a.g, ii[t], jj[t], jj[t] * nx + ii[t], f[t]);
#pragma unroll
    for (int t = 0; t < IT0; ++t) {
        if (code[t] == LK_SKIP) continue;
        gather_bounce<float>(a.src, a.g, code[t], jj[t] * nx + ii[t], f[t]);
        (void)collide_node<ZH, FORCE, R, NTH != 1024>(f[t], ii[t], nx, a);
        if constexpr (AA) {
            aa_write<false, W0, LN0>(P, tid + t * NTH, f[t]);
        } else {
#pragma unroll
            for (int q = 0; q < 9; ++q) P[q * LN0 + tid + t * NTH] = f[t][q];
        }
    }
    same_priority<NTH>();
    __syncthreads();
    ring_levels<S, RY, 1, ZH, FORCE, R, AA>(a, x0, y0, tid, P, LKS);
    const int i = x0 + threadIdx.x, j = y0 + threadIdx.y;
    if (i >= nx || j >= ny) return;
    const int n = j * nx + i;
    const unsigned lk = LKS[(threadIdx.y + S - 1) * W0 + threadIdx.x + S - 1];
    if (lk == LK_SKIP) return;
    float fl[9];
    if constexpr (AA) {
        aa_read<((S - 1) & 1) != 0, W0, LN0>(P, (threadIdx.y + S - 1) * W0 + threadIdx.x + S - 1, lk, fl);
    } else {
        constexpr int WL = G::W(S - 2), LNL = G::LN(S - 2);
        pull_lds(P, WL, LNL, (threadIdx.y + 1) * WL + threadIdx.x + 1, lk, fl);
    }
    (void)collide_node<ZH, FORCE, R, NTH != 1024>(fl, i, nx, a);
    const size_t N = (size_t)a.g.N;
    float* __restrict__ d = a.dst + n;
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        if (NT) __builtin_nontemporal_store(fl[q], d + q * N); else d[q * N] = fl[q];
    }
}

template <int S, int RY, bool ZH, bool FORCE, bool NT, typename R>
__global__ __launch_bounds__(TX * RY) void k_bgk_multi(StepArgs a) {
    __shared__ float P[9 * Ring<S, RY>::LN(0)];
    __shared__ unsigned short LKS[Ring<S, RY>::LN(0)];
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int by = b / a.g.gridx;
    step_multi<S, RY, ZH, FORCE, NT, R, true>(a, b - by * a.g.gridx, by, P, LKS);
}

// Four-wide step (nx % 4 == 0): each lane owns four consecutive x nodes of one
// row and a wavefront covers 256 nodes, so every plane is read and written with
// aligned 16-byte accesses.  The +-x shifted populations come from the
// neighbouring lane by a wavefront shuffle; the two values beyond the segment
// ends are loaded explicitly.  Lanes past the row end are clamped onto the last
// quad (every address stays valid) and store nothing.  Link bits arrive as one
// 32-bit word per quad; the mask byte is read only for 0xFF links.  Solid nodes
// store zeros (their slots are never read back).
typedef float f4 __attribute__((ext_vector_type(4)));

template <bool ZH, bool FORCE, bool WDRHO, bool NT, typename R>
__device__ __forceinline__ void step_quad(const StepArgs& a, int bx, int by) {
    const int lane = threadIdx.x;
    const int j = by * TY + threadIdx.y;
    if (j >= a.g.ny) return;  // uniform over the wavefront
    const int nx = a.g.nx, ny = a.g.ny, N = a.g.N;
    const int xw = bx * (4 * TX);
    const int x0r = xw + 4 * lane;
    const bool active = x0r < nx;
    const int x0 = active ? x0r : nx - 4;
    const int jm = j == 0 ? ny - 1 : j - 1, jp = j == ny - 1 ? 0 : j + 1;
    const int r0 = j * nx, rm = jm * nx, rp = jp * nx;
    const int xl = xw == 0 ? nx - 1 : xw - 1;
    const int xr = x0 + 4 >= nx ? x0 + 4 - nx : x0 + 4;
    const bool redge = lane == TX - 1 || x0 + 4 >= nx;
    const int n0 = r0 + x0;
    const unsigned lk4 = *reinterpret_cast<const unsigned*>(a.link + n0);
    float v[9][4];
#define LBM_LOAD0(Q, ROW)                                                              \
    {                                                                                  \
        const f4 t = *reinterpret_cast<const f4*>(a.src + (size_t)Q * N + (ROW) + x0); \
        v[Q][0] = t.x; v[Q][1] = t.y; v[Q][2] = t.z; v[Q][3] = t.w;                   \
    }
#define LBM_LOADP(Q, ROW) /* c_x = +1: pull from x - 1 */                             \
    {                                                                                  \
        const float* p_ = a.src + (size_t)Q * N + (ROW);                               \
        const f4 t = *reinterpret_cast<const f4*>(p_ + x0);                            \
        float left = __shfl_up(t.w, 1, 64);                                            \
        if (lane == 0) left = p_[xl];                                                  \
        v[Q][0] = left; v[Q][1] = t.x; v[Q][2] = t.y; v[Q][3] = t.z;                  \
    }
#define LBM_LOADM(Q, ROW) /* c_x = -1: pull from x + 1 */                             \
    {                                                                                  \
        const float* p_ = a.src + (size_t)Q * N + (ROW);                               \
        const f4 t = *reinterpret_cast<const f4*>(p_ + x0);                            \
        float right = __shfl_down(t.x, 1, 64);                                         \
        if (redge) right = p_[xr];                                                     \
        v[Q][0] = t.y; v[Q][1] = t.z; v[Q][2] = t.w; v[Q][3] = right;                 \
    }
    LBM_LOAD0(0, r0)
    LBM_LOADP(1, r0)
    LBM_LOAD0(2, rm)
    LBM_LOADM(3, r0)
    LBM_LOAD0(4, rp)
    LBM_LOADP(5, rm)
    LBM_LOADM(6, rm)
    LBM_LOADM(7, rp)
    LBM_LOADP(8, rp)
#undef LBM_LOAD0
#undef LBM_LOADP
#undef LBM_LOADM
    // solids (0xFF link and mask set) and bounced directions
    unsigned solid4 = 0;
    if (lk4 != 0u) {
        unsigned m4 = 0;
        const bool any_ff = ((lk4 & 0xFFu) == 0xFFu) | (((lk4 >> 8) & 0xFFu) == 0xFFu) |
                            (((lk4 >> 16) & 0xFFu) == 0xFFu) | ((lk4 >> 24) == 0xFFu);
        if (any_ff) m4 = *reinterpret_cast<const unsigned*>(a.mask + n0);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const unsigned lk = (lk4 >> (8 * k)) & 0xFFu;
            const bool sol = lk == 0xFFu && ((m4 >> (8 * k)) & 0xFFu) != 0u;
            solid4 |= (sol ? 1u : 0u) << k;
            if (lk != 0u && !sol) {
                const float* own = a.src + n0 + k;
#define LBM_BB(Q) if ((lk >> (Q - 1)) & 1u) v[Q][k] = own[(size_t)opp_of(Q) * N];
                LBM_BB(1) LBM_BB(2) LBM_BB(3) LBM_BB(4) LBM_BB(5) LBM_BB(6) LBM_BB(7) LBM_BB(8)
#undef LBM_BB
            }
        }
    }
    float drho4[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        float f[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) f[q] = v[q][k];
        drho4[k] = collide_node<ZH, FORCE, R>(f, x0 + k, nx, a);
        const bool sol = (solid4 >> k) & 1u;
#pragma unroll
        for (int q = 0; q < 9; ++q) v[q][k] = sol ? 0.0f : f[q];
        if (sol) drho4[k] = 0.0f;
    }
    // a quad of four solid nodes stores nothing (its slots are never read); its
    // loads above stay, since the neighbouring lanes' shuffles use them
    if (!active || solid4 == 0xFu) {
        if (WDRHO && active) {
            const f4 z = {0.0f, 0.0f, 0.0f, 0.0f};
            *reinterpret_cast<f4*>(a.drho_out + n0) = z;
        }
        return;
    }
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const f4 t = {v[q][0], v[q][1], v[q][2], v[q][3]};
        f4* d = reinterpret_cast<f4*>(a.dst + (size_t)q * N + n0);
        if (NT) __builtin_nontemporal_store(t, d); else *d = t;
    }
    if (WDRHO) {
        const f4 t = {drho4[0], drho4[1], drho4[2], drho4[3]};
        *reinterpret_cast<f4*>(a.drho_out + n0) = t;
    }
}

template <bool ZH, bool FORCE, bool WDRHO, bool NT, typename R>
__global__ __launch_bounds__(256) void k_bgk_step_v4(StepArgs a) {
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const int by = b / a.g.gridx;
    step_quad<ZH, FORCE, WDRHO, NT, R>(a, b - by * a.g.gridx, by);
}

// Batched step: one launch advances every trajectory of a batch by one step.  The
// flattened tile table lists (trajectory, tile x, tile y) for all trajectories;
// each workgroup reads its tile and that trajectory's step arguments (uniform
// over the workgroup, so the boundary / forcing branches do not diverge).
// Trajectories of one launch share the kernel shape (QUAD) and store policy (NT).
struct BatchTile {
    int traj, bx, by, pad;
};

template <bool QUAD, bool NT, typename R>
__global__ __launch_bounds__(256) void k_bgk_batch(const StepArgs* __restrict__ args,
                                                   const BatchTile* __restrict__ tiles) {
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const BatchTile t = tiles[b];
    const StepArgs a = args[t.traj];
    const bool zh = a.g.bc_x == LBM_BC_ZOUHE;
    const bool force = a.gx != 0.0 || a.gy != 0.0;
    if (QUAD) {
        if (zh) {
            if (force) step_quad<true, true, false, NT, R>(a, t.bx, t.by);
            else step_quad<true, false, false, NT, R>(a, t.bx, t.by);
        } else {
            if (force) step_quad<false, true, false, NT, R>(a, t.bx, t.by);
            else step_quad<false, false, false, NT, R>(a, t.bx, t.by);
        }
    } else {
        if (zh) {
            if (force) step_node<true, true, false, NT, R>(a, t.bx, t.by);
            else step_node<true, false, false, NT, R>(a, t.bx, t.by);
        } else {
            if (force) step_node<false, true, false, NT, R>(a, t.bx, t.by);
            else step_node<false, false, false, NT, R>(a, t.bx, t.by);
        }
    }
}

// Batched fused launch: the S-step tile routine over a trajectory-major table of
// 64 x RY tiles (for S = 2 the one-node kernel's 64 x TY table).
template <int S, int RY, bool NT, typename R>
__global__ __launch_bounds__(TX * RY) void k_bgk_batchm(const StepArgs* __restrict__ args,
                                                        const BatchTile* __restrict__ tiles) {
    __shared__ float P[9 * Ring<S, RY>::LN(0)];
    __shared__ unsigned short LKS[Ring<S, RY>::LN(0)];
    const int b = xcd_remap(blockIdx.x, gridDim.x);
    const BatchTile t = tiles[b];
    const StepArgs a = args[t.traj];
    const bool zh = a.g.bc_x == LBM_BC_ZOUHE;
    const bool force = a.gx != 0.0 || a.gy != 0.0;
    if (zh) {
        if (force) step_multi<S, RY, true, true, NT, R, false>(a, t.bx, t.by, P, LKS);
        else step_multi<S, RY, true, false, NT, R, false>(a, t.bx, t.by, P, LKS);
    } else {
        if (force) step_multi<S, RY, false, true, NT, R, false>(a, t.bx, t.by, P, LKS);
        else step_multi<S, RY, false, false, NT, R, false>(a, t.bx, t.by, P, LKS);
    }
}

struct MacroArgs {
    const float* __restrict__ src;
    const uint8_t* __restrict__ link;
    const uint8_t* __restrict__ mask;
    LatticeGeom g;
    double gx, gy, u_in, rho_out;
    float* __restrict__ rho;  // optional outputs
    float* __restrict__ ux;
    float* __restrict__ uy;
    int rho_minus_one;
    float* __restrict__ fpop;                 // optional absolute populations out
    const float* __restrict__ drho_prev;      // residual reference (SUMS)
    double* __restrict__ partials;            // [gridDim.x][4] (SUMS)
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// Gather-only pass over the current store: macroscopic fields, populations and,
// with SUMS, per-workgroup FP64 partial sums (|drho - drho_prev|, rho, rho ux, rho uy).
template <bool ZH, bool FORCE, bool SUMS>
__global__ __launch_bounds__(256) void k_macro(MacroArgs a) {
    const int b = blockIdx.x;
    const int by = b / a.g.gridx, bx = b - by * a.g.gridx;
    const int i = bx * TX + threadIdx.x, j = by * TY + threadIdx.y;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (i < a.g.nx && j < a.g.ny) {
        const int n = j * a.g.nx + i;
        const unsigned lk = a.link[n];
        const size_t N = (size_t)a.g.N;
        if (is_solid(lk, a.mask, n)) {
            if (a.rho) a.rho[n] = a.rho_minus_one ? 0.0f : 1.0f;
            if (a.ux) a.ux[n] = 0.0f;
            if (a.uy) a.uy[n] = 0.0f;
            if (a.fpop) {
#pragma unroll
                for (int q = 0; q < 9; ++q) a.fpop[q * N + n] = w_of(q);
            }
        } else {
            double f[9];
            gather<double>(a.src, a.g, lk, i, j, n, f);
            if (ZH) zouhe<double>(f, i, a.g.nx, a.u_in, a.rho_out);
            const Moments<double> m = moments<FORCE, double>(f, a.gx, a.gy);
            if (a.rho) a.rho[n] = (float)(a.rho_minus_one ? m.drho : m.rho);
            if (a.ux) a.ux[n] = (float)m.ux;
            if (a.uy) a.uy[n] = (float)m.uy;
            if (a.fpop) {
#pragma unroll
                for (int q = 0; q < 9; ++q) a.fpop[q * N + n] = (float)(f[q] + w_of_d(q));
            }
            if (SUMS) {
                // the residual compares FP32-stored density deviations of
                // consecutive steps (both sides rounded the same way)
                s0 = fabs((double)(float)m.drho - (double)a.drho_prev[n]);
                s1 = m.rho;
                s2 = m.rho * m.ux;
                s3 = m.rho * m.uy;
            }
        }
    }
    if (SUMS) {
        __shared__ double red[4][4];
        const int lane = threadIdx.x;  // blockDim.x == 64: one wavefront per row
        const int wave = threadIdx.y;
        s0 = wave_sum(s0); s1 = wave_sum(s1); s2 = wave_sum(s2); s3 = wave_sum(s3);
        if (lane == 0) { red[wave][0] = s0; red[wave][1] = s1; red[wave][2] = s2; red[wave][3] = s3; }
        __syncthreads();
        if (wave == 0 && lane < 4) {
            const double t = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
            a.partials[(size_t)b * 4 + lane] = t;
        }
    }
}

// Second, fixed-order pass over the per-workgroup partials (deterministic).
__global__ __launch_bounds__(256) void k_reduce_final(const double* __restrict__ partials, int nb,
                                                      double* __restrict__ out) {
    __shared__ double red[4][4];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = t; b < nb; b += 256)
        for (int k = 0; k < 4; ++k) s[k] += partials[(size_t)b * 4 + k];
    for (int k = 0; k < 4; ++k) {
        const double v = wave_sum(s[k]);
        if (lane == 0) red[wave][k] = v;
    }
    __syncthreads();
    if (t < 4) out[t] = ((red[0][t] + red[1][t]) + red[2][t]) + red[3][t];
}

// Field guard: per-workgroup (sum rho, max |u|, non-finite count), then a
// fixed-order second pass.  Partials reuse the [nblocks][4] double scratch.
__global__ __launch_bounds__(256) void k_field_stats(const uint8_t* __restrict__ mask, int N,
                                                     const float* __restrict__ rho,
                                                     const float* __restrict__ ux,
                                                     const float* __restrict__ uy,
                                                     double* __restrict__ partials) {
    __shared__ double red[4][3];
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0.0, mx = 0.0, bad = 0.0;
    if (n < N && !mask[n]) {
        const float r = rho[n], u = ux[n], v = uy[n];
        const bool fin = isfinite(r) && isfinite(u) && isfinite(v);
        if (fin) {
            s = (double)r;
            mx = sqrt((double)u * u + (double)v * v);
        } else {
            bad = 1.0;
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    s = wave_sum(s);
    bad = wave_sum(bad);
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_down(mx, o, 64));
    if (lane == 0) { red[wave][0] = s; red[wave][1] = mx; red[wave][2] = bad; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, m = 0.0, c = 0.0;
        for (int w = 0; w < 4; ++w) { a += red[w][0]; m = fmax(m, red[w][1]); c += red[w][2]; }
        partials[(size_t)blockIdx.x * 4 + 0] = a;
        partials[(size_t)blockIdx.x * 4 + 1] = m;
        partials[(size_t)blockIdx.x * 4 + 2] = c;
        partials[(size_t)blockIdx.x * 4 + 3] = 0.0;
    }
}

__global__ __launch_bounds__(256) void k_field_stats_final(const double* __restrict__ partials,
                                                           int nb, double* __restrict__ out) {
    __shared__ double red[4][3];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    double s = 0.0, m = 0.0, c = 0.0;
    for (int b = t; b < nb; b += 256) {
        s += partials[(size_t)b * 4];
        m = fmax(m, partials[(size_t)b * 4 + 1]);
        c += partials[(size_t)b * 4 + 2];
    }
    s = wave_sum(s);
    c = wave_sum(c);
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_down(m, o, 64));
    if (lane == 0) { red[wave][0] = s; red[wave][1] = m; red[wave][2] = c; }
    __syncthreads();
    if (t == 0) {
        double a = 0.0, mm = 0.0, cc = 0.0;
        for (int w = 0; w < 4; ++w) { a += red[w][0]; mm = fmax(mm, red[w][1]); cc += red[w][2]; }
        out[0] = a; out[1] = mm; out[2] = cc; out[3] = 0.0;
    }
}

// Plain float copy / zero fill, grid-stride.  Used instead of hipMemcpyAsync /
// hipMemsetAsync wherever a captured graph may be the next work on the stream:
// a graph launched right behind an asynchronous fill has been seen to start
// before the fill completed; kernels are ordered with graph launches.
__global__ __launch_bounds__(256) void k_copy_f32(const float* __restrict__ src, float* __restrict__ dst,
                                                  size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        dst[i] = src ? src[i] : 0.0f;
}

static unsigned copy_grid(size_t n) {
    const size_t b = (n + 255) / 256;
    return (unsigned)(b < 8192 ? (b ? b : 1) : 8192);
}

// Field comparison: per-workgroup FP64 partial sums over fluid nodes of
// |a - ref| and |ref| for rho (= 1 + drho), ux, uy, and of drho, drho_ref and the
// fluid-node count on the first and last columns (pressure drop); grid-stride,
// then a fixed-order second pass (deterministic).
constexpr int CMP_VALUES = 12;
constexpr int CMP_BLOCKS = 512;

__global__ __launch_bounds__(256) void k_compare(const uint8_t* __restrict__ mask, int nx, int N,
                                                 const float* __restrict__ drho,
                                                 const float* __restrict__ ux,
                                                 const float* __restrict__ uy,
                                                 const float* __restrict__ drho_ref,
                                                 const float* __restrict__ ux_ref,
                                                 const float* __restrict__ uy_ref,
                                                 double* __restrict__ partials) {
    __shared__ double red[4][CMP_VALUES];
    double s[CMP_VALUES];
#pragma unroll
    for (int k = 0; k < CMP_VALUES; ++k) s[k] = 0.0;
    for (int n = blockIdx.x * blockDim.x + threadIdx.x; n < N; n += gridDim.x * blockDim.x) {
        if (mask[n]) continue;
        const double r = drho[n], rr = drho_ref[n];
        const double u = ux[n], ur = ux_ref[n], v = uy[n], vr = uy_ref[n];
        s[0] += fabs(r - rr);
        s[1] += fabs(1.0 + rr);
        s[2] += fabs(u - ur);
        s[3] += fabs(ur);
        s[4] += fabs(v - vr);
        s[5] += fabs(vr);
        const int i = n % nx;
        if (i == 0) { s[6] += r; s[7] += rr; s[8] += 1.0; }
        if (i == nx - 1) { s[9] += r; s[10] += rr; s[11] += 1.0; }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < CMP_VALUES; ++k) {
        const double t = wave_sum(s[k]);
        if (lane == 0) red[wave][k] = t;
    }
    __syncthreads();
    if (threadIdx.x < CMP_VALUES) {
        const int k = threadIdx.x;
        partials[(size_t)blockIdx.x * CMP_VALUES + k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
    }
}

__global__ __launch_bounds__(64) void k_compare_final(const double* __restrict__ partials, int nb,
                                                      double* __restrict__ out) {
    const int k = threadIdx.x;
    if (k >= CMP_VALUES) return;
    double t = 0.0;
    for (int b = 0; b < nb; ++b) t += partials[(size_t)b * CMP_VALUES + k];
    out[k] = t;
}

}  // namespace lbmfno

// ------------------------------------------------------------ host side

using namespace lbmfno;

// Fused multi-step kernel shapes: steps per launch, tile height, store kind.
enum FusedShape { SHAPE_NONE, SHAPE_PAIR8, SHAPE_PAIR4_NT, SHAPE_DEEP4_8, SHAPE_DEEP5_16, SHAPE_DEEP4_8_NT };

struct lbm_ctx {
    lbm_config cfg;
    LatticeGeom g;
    float* f[2];
    int cur;
    hipStream_t stream;
    uint8_t* d_link;
    uint8_t* d_mask;
    float* d_drho;
    double* d_partials;
    double* d_cmp;      // [CMP_BLOCKS][CMP_VALUES] field-comparison partials
    double* d_out;      // [16] reduction results
    double* h_out;      // [16] pinned copy
    int nblocks;
    int64_t fluid;
    int64_t steps;
    hipGraphExec_t graph[2];
    int graph_chunk;
    int device;
    bool nontemporal;
    bool vec4;       // four-wide step kernel (nx % 4 == 0)
    int spl;         // steps per launch of the fused kernel (1: a one-step kernel)
    int shape;       // FusedShape of the fused kernel
    int gridx4;      // workgroups along x for the four-wide kernel
    int nblocks4;
};

static bool finite_d(double x) { return std::isfinite(x); }

static int validate_config(const lbm_config* c) {
    if (!c) return fail(LBM_EINVAL, "config is NULL");
    if (c->nx < 1 || c->ny < 1) return fail(LBM_EINVAL, "lattice size %d x %d", c->nx, c->ny);
    if ((int64_t)c->nx * c->ny * 9 >= (int64_t)1 << 31)
        return fail(LBM_EINVAL, "lattice %d x %d too large for 32-bit plane offsets", c->nx, c->ny);
    if (!(c->tau > 0.5) || !finite_d(c->tau))
        return fail(LBM_EINVAL, "tau = %g must be finite and > 1/2", c->tau);
    if (!finite_d(c->gx) || !finite_d(c->gy)) return fail(LBM_EINVAL, "non-finite body force");
    if (c->arith != LBM_ARITH_MIXED && c->arith != LBM_ARITH_FP32 && c->arith != LBM_ARITH_LEAN)
        return fail(LBM_EINVAL, "arith = %d", c->arith);
    if (!(c->trt_lambda >= 0.0) || !std::isfinite(c->trt_lambda))
        return fail(LBM_EINVAL, "trt_lambda = %g (0 for BGK, > 0 for TRT)", c->trt_lambda);
    if (c->trt_lambda > 0.0 && c->arith != LBM_ARITH_LEAN)
        return fail(LBM_EUNSUPPORTED, "the TRT collision runs in LBM_ARITH_LEAN");
    if (c->kernel < LBM_KERNEL_AUTO || c->kernel > LBM_KERNEL_DEEP)
        return fail(LBM_EINVAL, "kernel = %d", c->kernel);
    if (c->bc_x < 0 || c->bc_x > 2 || c->bc_y < 0 || c->bc_y > 1)
        return fail(LBM_EINVAL, "boundary codes bc_x=%d bc_y=%d", c->bc_x, c->bc_y);
    if (c->bc_x == LBM_BC_ZOUHE) {
        if (c->nx < 3) return fail(LBM_EINVAL, "Zou-He needs nx >= 3");
        if (!(c->u_in > -1.0 && c->u_in < 1.0) || !finite_d(c->u_in))
            return fail(LBM_EINVAL, "u_in = %g out of (-1, 1)", c->u_in);
        if (!(c->rho_out > 0.0) || !finite_d(c->rho_out))
            return fail(LBM_EINVAL, "rho_out = %g must be > 0", c->rho_out);
        if (c->gx != 0.0 || c->gy != 0.0)
            return fail(LBM_EUNSUPPORTED, "body force with Zou-He boundaries");
        if (c->bc_y == LBM_BC_WALL)
            return fail(LBM_EUNSUPPORTED, "Zou-He columns meeting wall rows (corners)");
    }
    return LBM_OK;
}

extern "C" const char* lbm_status_str(int code) {
    switch (code) {
        case LBM_OK: return "ok";
        case LBM_EINVAL: return "invalid argument";
        case LBM_ENOMEM: return "out of memory";
        case LBM_EHIP: return "HIP runtime error";
        case LBM_EUNSUPPORTED: return "unsupported";
        case LBM_ENOTCONVERGED: return "not converged";
        case LBM_EDIVERGED: return "diverged";
        default: return "unknown status";
    }
}

extern "C" const char* lbm_last_error(void) { return g_err.c_str(); }

extern "C" int lbm_mask_raster(int32_t nx, int32_t ny, int32_t wrap_x, int32_t wrap_y,
                               const int64_t* h_shapes, int32_t nshapes, uint8_t* d_mask,
                               void* stream) {
    if (nx < 1 || ny < 1 || (int64_t)nx * ny >= ((int64_t)1 << 31))
        return fail(LBM_EINVAL, "raster size %d x %d", nx, ny);
    if (nshapes < 0 || (nshapes > 0 && !h_shapes)) return fail(LBM_EINVAL, "shape list");
    if (!d_mask) return fail(LBM_EINVAL, "d_mask is NULL");
    for (int s = 0; s < nshapes; ++s) {
        const int64_t* p = h_shapes + 7 * (size_t)s;
        const __int128 R = p[6];
        if (p[6] < 0 || p[6] >= (1 << 15)) return fail(LBM_EINVAL, "shape %d: R = %lld", s, (long long)p[6]);
        if (p[0] < -(1 << 30) || p[0] > (1 << 30) || p[1] < -(1 << 30) || p[1] > (1 << 30))
            return fail(LBM_EINVAL, "shape %d: centre out of range", s);
        const __int128 mag = ((__int128)llabs(p[2]) + llabs(p[3]) + llabs(p[4])) * R * R;
        if (mag >= ((__int128)1 << 62) || llabs(p[5]) >= ((int64_t)1 << 62))
            return fail(LBM_EINVAL, "shape %d: coefficients overflow int64 on |dx|,|dy| <= R", s);
    }
    hipStream_t st = (hipStream_t)stream;
    int64_t* d_shapes = nullptr;
    if (nshapes > 0) {
        LBM_HIP(hipMalloc(&d_shapes, sizeof(int64_t) * 7 * (size_t)nshapes));
        hipError_t e = hipMemcpyAsync(d_shapes, h_shapes, sizeof(int64_t) * 7 * (size_t)nshapes,
                                      hipMemcpyHostToDevice, st);
        if (e != hipSuccess) {
            (void)hipFree(d_shapes);
            return fail(LBM_EHIP, "shape upload: %s", hipGetErrorString(e));
        }
    }
    dim3 blk(256), grd((nx + 255) / 256, ny);
    k_mask_raster<<<grd, blk, 0, st>>>(nx, ny, wrap_x, wrap_y, d_shapes, nshapes, d_mask);
    hipError_t e = hipGetLastError();
    hipError_t e2 = hipStreamSynchronize(st);
    if (d_shapes) (void)hipFree(d_shapes);
    if (e != hipSuccess) return fail(LBM_EHIP, "raster launch: %s", hipGetErrorString(e));
    if (e2 != hipSuccess) return fail(LBM_EHIP, "raster sync: %s", hipGetErrorString(e2));
    return LBM_OK;
}

static void release(lbm_ctx* c) {
    if (!c) return;
    for (int k = 0; k < 2; ++k)
        if (c->graph[k]) (void)hipGraphExecDestroy(c->graph[k]);
    if (c->d_link) (void)hipFree(c->d_link);
    if (c->d_mask) (void)hipFree(c->d_mask);
    if (c->d_drho) (void)hipFree(c->d_drho);
    if (c->d_partials) (void)hipFree(c->d_partials);
    if (c->d_cmp) (void)hipFree(c->d_cmp);
    if (c->d_out) (void)hipFree(c->d_out);
    if (c->h_out) (void)hipHostFree(c->h_out);
    delete c;
}

extern "C" void lbm_destroy(lbm_ctx* ctx) { release(ctx); }

// BGK rate and Guo factor from tau; with TRT (trt_lambda > 0) also the odd-part
// rate from the magic parameter lambda = (tau+ - 1/2)(tau- - 1/2).
static void set_relaxation(StepArgs& a, const lbm_config& cfg) {
    a.omega = 1.0 / cfg.tau;
    a.guo = 1.0 - 0.5 / cfg.tau;
    const double tau_m = cfg.trt_lambda > 0.0 ? 0.5 + cfg.trt_lambda / (cfg.tau - 0.5) : cfg.tau;
    a.omega_m = 1.0 / tau_m;
    a.guo_m = 1.0 - 0.5 / tau_m;
}

static int launch_step(lbm_ctx* c, bool write_drho) {
    StepArgs a;
    a.src = c->f[c->cur];
    a.dst = c->f[c->cur ^ 1];
    a.link = c->d_link;
    a.mask = c->d_mask;
    a.drho_out = c->d_drho;
    a.g = c->g;
    set_relaxation(a, c->cfg);
    a.gx = c->cfg.gx;
    a.gy = c->cfg.gy;
    a.u_in = c->cfg.u_in;
    a.rho_out = c->cfg.rho_out;
    const bool zh = c->cfg.bc_x == LBM_BC_ZOUHE;
    const bool force = c->cfg.gx != 0.0 || c->cfg.gy != 0.0;
    const int ar = c->cfg.arith;
    const bool trt = c->cfg.trt_lambda > 0.0;
    const bool nt = c->nontemporal;
    hipStream_t s = c->stream;
    if (c->vec4) {
        a.g.gridx = c->gridx4;
        dim3 blk(TX, TY), grd(c->nblocks4);
#define LBM_STEP_ARITH(R)                                                              \
    {                                                                                 \
        if (nt) k_bgk_step_v4<Z, F, W, true, R><<<grd, blk, 0, s>>>(a);               \
        else k_bgk_step_v4<Z, F, W, false, R><<<grd, blk, 0, s>>>(a);                 \
    }
#define LBM_STEP_CASE(Z_, F_, W_)                                                      \
    if (zh == Z_ && force == F_ && write_drho == W_) {                                \
        constexpr bool Z = Z_, F = F_, W = W_;                                        \
        if (ar == LBM_ARITH_FP32) LBM_STEP_ARITH(float)                               \
        else if (ar == LBM_ARITH_MIXED) LBM_STEP_ARITH(double)                        \
        else if (trt) LBM_STEP_ARITH(LeanTRT)                                         \
        else LBM_STEP_ARITH(Lean)                                                     \
    }
        LBM_STEP_CASE(false, false, false)
        LBM_STEP_CASE(false, false, true)
        LBM_STEP_CASE(false, true, false)
        LBM_STEP_CASE(false, true, true)
        LBM_STEP_CASE(true, false, false)
        LBM_STEP_CASE(true, false, true)
        LBM_STEP_CASE(true, true, false)
        LBM_STEP_CASE(true, true, true)
#undef LBM_STEP_CASE
#undef LBM_STEP_ARITH
        c->cur ^= 1;
        ++c->steps;
        return LBM_OK;
    }
    dim3 blk(TX, TY), grd(c->nblocks);
#define LBM_STEP_ARITH(R)                                                              \
    {                                                                                 \
        if (nt) k_bgk_step<Z, F, W, true, R><<<grd, blk, 0, s>>>(a);                  \
        else k_bgk_step<Z, F, W, false, R><<<grd, blk, 0, s>>>(a);                    \
    }
#define LBM_STEP_CASE(Z_, F_, W_)                                                      \
    if (zh == Z_ && force == F_ && write_drho == W_) {                                \
        constexpr bool Z = Z_, F = F_, W = W_;                                        \
        if (ar == LBM_ARITH_FP32) LBM_STEP_ARITH(float)                               \
        else if (ar == LBM_ARITH_MIXED) LBM_STEP_ARITH(double)                        \
        else if (trt) LBM_STEP_ARITH(LeanTRT)                                         \
        else LBM_STEP_ARITH(Lean)                                                     \
    }
    LBM_STEP_CASE(false, false, false)
    LBM_STEP_CASE(false, false, true)
    LBM_STEP_CASE(false, true, false)
    LBM_STEP_CASE(false, true, true)
    LBM_STEP_CASE(true, false, false)
    LBM_STEP_CASE(true, false, true)
    LBM_STEP_CASE(true, true, false)
    LBM_STEP_CASE(true, true, true)
#undef LBM_STEP_CASE
#undef LBM_STEP_ARITH
    c->cur ^= 1;
    ++c->steps;
    return LBM_OK;
}

// One shape of the fused multi-step kernel, dispatched over the boundary,
// forcing and arithmetic variants.
template <int S, int RY, bool NT>
static void launch_multi_shape(const lbm_ctx* c, const StepArgs& a) {
    const bool zh = c->cfg.bc_x == LBM_BC_ZOUHE;
    const bool force = c->cfg.gx != 0.0 || c->cfg.gy != 0.0;
    const int ar = c->cfg.arith;
    const bool trt = c->cfg.trt_lambda > 0.0;
    hipStream_t s = c->stream;
    dim3 blk(TX, RY), grd(c->g.gridx * ((c->g.ny + RY - 1) / RY));
#define LBM_MULTI_ARITH(Z, F)                                                           \
    {                                                                                 \
        if (ar == LBM_ARITH_FP32) k_bgk_multi<S, RY, Z, F, NT, float><<<grd, blk, 0, s>>>(a); \
        else if (ar == LBM_ARITH_MIXED) k_bgk_multi<S, RY, Z, F, NT, double><<<grd, blk, 0, s>>>(a); \
        else if (trt) k_bgk_multi<S, RY, Z, F, NT, LeanTRT><<<grd, blk, 0, s>>>(a);  \
        else k_bgk_multi<S, RY, Z, F, NT, Lean><<<grd, blk, 0, s>>>(a);              \
    }
    if (zh) {
        if (force) LBM_MULTI_ARITH(true, true) else LBM_MULTI_ARITH(true, false)
    } else {
        if (force) LBM_MULTI_ARITH(false, true) else LBM_MULTI_ARITH(false, false)
    }
#undef LBM_MULTI_ARITH
}

// c->spl steps in one launch (k_bgk_multi): the store parity flips once.
static int launch_multi(lbm_ctx* c) {
    StepArgs a;
    a.src = c->f[c->cur];
    a.dst = c->f[c->cur ^ 1];
    a.link = c->d_link;
    a.mask = c->d_mask;
    a.drho_out = c->d_drho;
    a.g = c->g;
    set_relaxation(a, c->cfg);
    a.gx = c->cfg.gx;
    a.gy = c->cfg.gy;
    a.u_in = c->cfg.u_in;
    a.rho_out = c->cfg.rho_out;
    switch (c->shape) {
        case SHAPE_PAIR8: launch_multi_shape<2, 8, false>(c, a); break;
        case SHAPE_PAIR4_NT: launch_multi_shape<2, 4, true>(c, a); break;
        case SHAPE_DEEP4_8: launch_multi_shape<4, 8, false>(c, a); break;
        case SHAPE_DEEP5_16: launch_multi_shape<5, 16, false>(c, a); break;
        case SHAPE_DEEP4_8_NT: launch_multi_shape<4, 8, true>(c, a); break;
        default: return fail(LBM_EINVAL, "no fused shape selected");
    }
    c->cur ^= 1;
    c->steps += c->spl;
    return LBM_OK;
}

static int launch_macro(lbm_ctx* c, float* rho, float* ux, float* uy, int rm1, float* fpop,
                        bool sums) {
    MacroArgs a;
    a.src = c->f[c->cur];
    a.link = c->d_link;
    a.mask = c->d_mask;
    a.g = c->g;
    a.gx = c->cfg.gx;
    a.gy = c->cfg.gy;
    a.u_in = c->cfg.u_in;
    a.rho_out = c->cfg.rho_out;
    a.rho = rho;
    a.ux = ux;
    a.uy = uy;
    a.rho_minus_one = rm1;
    a.fpop = fpop;
    a.drho_prev = c->d_drho;
    a.partials = c->d_partials;
    const bool zh = c->cfg.bc_x == LBM_BC_ZOUHE;
    const bool force = c->cfg.gx != 0.0 || c->cfg.gy != 0.0;
    dim3 blk(TX, TY), grd(c->nblocks);
    hipStream_t s = c->stream;
#define LBM_MACRO_CASE(Z, F, S) \
    if (zh == Z && force == F && sums == S) k_macro<Z, F, S><<<grd, blk, 0, s>>>(a);
    LBM_MACRO_CASE(false, false, false)
    LBM_MACRO_CASE(false, false, true)
    LBM_MACRO_CASE(false, true, false)
    LBM_MACRO_CASE(false, true, true)
    LBM_MACRO_CASE(true, false, false)
    LBM_MACRO_CASE(true, false, true)
    LBM_MACRO_CASE(true, true, false)
    LBM_MACRO_CASE(true, true, true)
#undef LBM_MACRO_CASE
    LBM_HIP(hipGetLastError());
    return LBM_OK;
}

extern "C" int lbm_init(lbm_ctx** out, const lbm_config* cfg, const uint8_t* d_mask, float* d_fA,
                        float* d_fB, void* stream) {
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate_config(cfg);
    if (rc) return rc;
    if (!d_mask || !d_fA || !d_fB) return fail(LBM_EINVAL, "NULL device buffer");
    if (d_fA == d_fB) return fail(LBM_EINVAL, "the two population stores must differ");
    lbm_ctx* c = new (std::nothrow) lbm_ctx();
    if (!c) return fail(LBM_ENOMEM, "context allocation");
    c->cfg = *cfg;
    c->g.nx = cfg->nx;
    c->g.ny = cfg->ny;
    c->g.N = cfg->nx * cfg->ny;
    c->g.gridx = (cfg->nx + TX - 1) / TX;
    c->g.bc_x = cfg->bc_x;
    c->g.bc_y = cfg->bc_y;
    c->nblocks = c->g.gridx * ((cfg->ny + TY - 1) / TY);
    // The four-wide kernel issues a quarter of the wavefronts; below ~4M nodes that
    // leaves too few in flight to hide latency and the one-node kernel is faster.
    const bool quad_ok = cfg->nx % 4 == 0 && cfg->nx >= 4 && ((uintptr_t)d_fA % 16 == 0) &&
                         ((uintptr_t)d_fB % 16 == 0);
    if (cfg->kernel == LBM_KERNEL_QUAD && !quad_ok) {
        delete c;
        return fail(LBM_EUNSUPPORTED, "four-wide kernel needs nx %% 4 == 0 and 16-byte aligned stores");
    }
    const size_t N = (size_t)c->g.N;
    // two stores above 128 MB cannot stay in the 256 MB last-level cache across a step
    c->nontemporal = 2 * 9 * N * sizeof(float) > ((size_t)128 << 20);
    // Fused multi-step launches beat every one-step kernel at every size measured
    // (128x128 to 8192x4096): on large lattices by cutting the population traffic
    // per step, on small, latency-bound ones by cutting the launches.  The deep
    // kernel (the default) runs five steps per launch on 64 x 16 tiles on
    // cache-resident lattices whose grid still gives every CU two such workgroups,
    // four steps on 64 x 8 tiles on smaller ones, and four steps on 64 x 8 tiles
    // with streaming stores on lattices streamed from HBM.
    const int64_t tiles16 = (int64_t)c->g.gridx * ((cfg->ny + 15) / 16);
    c->shape = SHAPE_NONE;
    c->spl = 1;
    if (cfg->kernel == LBM_KERNEL_PAIR) {
        c->shape = c->nontemporal ? SHAPE_PAIR4_NT : SHAPE_PAIR8;
        c->spl = 2;
    } else if (cfg->kernel == LBM_KERNEL_DEEP || cfg->kernel == LBM_KERNEL_AUTO) {
        c->shape = c->nontemporal ? SHAPE_DEEP4_8_NT : tiles16 >= 512 ? SHAPE_DEEP5_16 : SHAPE_DEEP4_8;
        c->spl = c->shape == SHAPE_DEEP5_16 ? 5 : 4;
    }
    c->vec4 = cfg->kernel == LBM_KERNEL_QUAD;
    c->gridx4 = (cfg->nx + 4 * TX - 1) / (4 * TX);
    c->nblocks4 = c->gridx4 * ((cfg->ny + TY - 1) / TY);
    c->f[0] = d_fA;
    c->f[1] = d_fB;
    c->cur = 0;
    c->stream = (hipStream_t)stream;
    // a graph chunk is an even number of launches (the store parity returns)
    c->graph_chunk = c->spl == 3 || c->spl == 5 ? 30 : 32;   // an even number of launches
#define LBM_TRY(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess) {                                                         \
            int r_ = fail(e_ == hipErrorOutOfMemory ? LBM_ENOMEM : LBM_EHIP, "%s: %s",   \
                          #call, hipGetErrorString(e_));                                \
            release(c);                                                                 \
            return r_;                                                                  \
        }                                                                               \
    } while (0)
    LBM_TRY(hipGetDevice(&c->device));
    LBM_TRY(hipMalloc(&c->d_link, N));
    LBM_TRY(hipMalloc(&c->d_mask, N));
    LBM_TRY(hipMemcpyAsync(c->d_mask, d_mask, N, hipMemcpyDeviceToDevice, c->stream));
    LBM_TRY(hipMalloc(&c->d_drho, N * sizeof(float)));
    LBM_TRY(hipMalloc(&c->d_partials, (size_t)c->nblocks * 4 * sizeof(double)));
    LBM_TRY(hipMalloc(&c->d_cmp, (size_t)CMP_BLOCKS * CMP_VALUES * sizeof(double)));
    LBM_TRY(hipMalloc(&c->d_out, 16 * sizeof(double)));
    LBM_TRY(hipHostMalloc(&c->h_out, 16 * sizeof(double), hipHostMallocDefault));
    dim3 blk(256), grd((cfg->nx + 255) / 256, cfg->ny);
    k_links<<<grd, blk, 0, c->stream>>>(cfg->nx, cfg->ny, cfg->bc_x, cfg->bc_y, c->d_mask, c->d_link);
    LBM_TRY(hipGetLastError());
    // rest state: f = w everywhere, i.e. zero deviations
    LBM_TRY(hipMemsetAsync(d_fA, 0, 9 * N * sizeof(float), c->stream));
    LBM_TRY(hipMemsetAsync(c->d_drho, 0, N * sizeof(float), c->stream));
    std::vector<uint8_t> h(N);
    LBM_TRY(hipMemcpyAsync(h.data(), d_mask, N, hipMemcpyDeviceToHost, c->stream));
    LBM_TRY(hipStreamSynchronize(c->stream));
#undef LBM_TRY
    int64_t fl = 0;
    for (size_t k = 0; k < N; ++k) fl += h[k] == 0;
    c->fluid = fl;
    c->steps = 0;
    *out = c;
    return LBM_OK;
}

static int reinit(lbm_ctx* c, const float* d_rho, const float* d_ux, const float* d_uy, bool neq) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (!d_rho || !d_ux || !d_uy) return fail(LBM_EINVAL, "NULL field");
    dim3 blk(256), grd((c->g.nx + 255) / 256, c->g.ny);
    if (neq)
        k_scatter<true, true><<<grd, blk, 0, c->stream>>>(c->g, c->d_mask, d_rho, d_ux, d_uy, nullptr,
                                                          c->f[c->cur], c->cfg.tau);
    else
        k_scatter<true, false><<<grd, blk, 0, c->stream>>>(c->g, c->d_mask, d_rho, d_ux, d_uy, nullptr,
                                                           c->f[c->cur], c->cfg.tau);
    LBM_HIP(hipGetLastError());
    c->steps = 0;
    return LBM_OK;
}

extern "C" int lbm_reinit_from_macro(lbm_ctx* c, const float* d_rho, const float* d_ux,
                                     const float* d_uy) {
    return reinit(c, d_rho, d_ux, d_uy, false);
}

extern "C" int lbm_reinit_from_macro_neq(lbm_ctx* c, const float* d_rho, const float* d_ux,
                                         const float* d_uy) {
    return reinit(c, d_rho, d_ux, d_uy, true);
}

static int launch_field_stats(lbm_ctx* c, const float* d_rho, const float* d_ux, const float* d_uy,
                              double* d_out);

extern "C" int lbm_reinit_from_macro_mass(lbm_ctx* c, const float* d_rho, const float* d_ux,
                                          const float* d_uy) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (!d_rho || !d_ux || !d_uy) return fail(LBM_EINVAL, "NULL field");
    // current mass: the report's FP64 reduction of the state's moments -> d_out[4 + 1]
    int rc = launch_macro(c, nullptr, nullptr, nullptr, 0, nullptr, true);
    if (rc) return rc;
    k_reduce_final<<<1, 256, 0, c->stream>>>(c->d_partials, c->nblocks, c->d_out + 4);
    // fluid sum of the handed-over density -> d_out[8]
    rc = launch_field_stats(c, d_rho, d_ux, d_uy, c->d_out + 8);
    if (rc) return rc;
    const double inv_fluid = c->fluid > 0 ? 1.0 / (double)c->fluid : 0.0;
    dim3 blk(256), grd((c->g.nx + 255) / 256, c->g.ny);
    k_scatter<true, false, true><<<grd, blk, 0, c->stream>>>(c->g, c->d_mask, d_rho, d_ux, d_uy, nullptr,
                                                             c->f[c->cur], c->cfg.tau, c->d_out + 5,
                                                             c->d_out + 8, inv_fluid);
    LBM_HIP(hipGetLastError());
    c->steps = 0;
    return LBM_OK;
}

extern "C" int lbm_set_populations(lbm_ctx* c, const float* d_f) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (!d_f) return fail(LBM_EINVAL, "d_f is NULL");
    dim3 blk(256), grd((c->g.nx + 255) / 256, c->g.ny);
    k_scatter<false, false><<<grd, blk, 0, c->stream>>>(c->g, c->d_mask, nullptr, nullptr, nullptr,
                                                        d_f, c->f[c->cur], c->cfg.tau);
    LBM_HIP(hipGetLastError());
    return LBM_OK;
}

static int build_graph(lbm_ctx* c) {
    const int start = c->cur;
    const int64_t steps0 = c->steps;
    hipGraph_t graph = nullptr;
    LBM_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    if (c->spl > 1) {
        for (int k = 0; k < c->graph_chunk; k += c->spl) launch_multi(c);
    } else {
        for (int k = 0; k < c->graph_chunk; ++k) launch_step(c, false);
    }
    hipError_t e = hipStreamEndCapture(c->stream, &graph);
    c->cur = start;
    c->steps = steps0;
    if (e != hipSuccess) return fail(LBM_EHIP, "graph capture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&c->graph[start], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
        c->graph[start] = nullptr;
        return fail(LBM_EHIP, "graph instantiate: %s", hipGetErrorString(e));
    }
    return LBM_OK;
}

extern "C" int lbm_step(lbm_ctx* c, int32_t n, lbm_report* rep) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (n < 0) return fail(LBM_EINVAL, "n = %d < 0", n);
    if (rep && n < 1) return fail(LBM_EINVAL, "a report needs n >= 1");
    int plain = rep ? n - 1 : n;
    // Replay graph-captured chunks of plain steps on a non-default stream; a
    // chunk flips the store parity an even number of times.
    if (c->stream != nullptr) {
        while (plain >= c->graph_chunk) {
            if (!c->graph[c->cur]) {
                int rc = build_graph(c);
                if (rc) return rc;
            }
            LBM_HIP(hipGraphLaunch(c->graph[c->cur], c->stream));
            c->steps += c->graph_chunk;
            plain -= c->graph_chunk;
        }
    }
    if (c->spl > 1)
        for (; plain >= c->spl; plain -= c->spl) launch_multi(c);
    for (int k = 0; k < plain; ++k) launch_step(c, false);
    LBM_HIP(hipGetLastError());
    if (!rep) return LBM_OK;
    launch_step(c, true);  // writes drho(n-1)
    LBM_HIP(hipGetLastError());
    int rc = launch_macro(c, nullptr, nullptr, nullptr, 0, nullptr, true);
    if (rc) return rc;
    k_reduce_final<<<1, 256, 0, c->stream>>>(c->d_partials, c->nblocks, c->d_out);
    LBM_HIP(hipGetLastError());
    LBM_HIP(hipMemcpyAsync(c->h_out, c->d_out, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    LBM_HIP(hipStreamSynchronize(c->stream));
    rep->mass = c->h_out[1];
    rep->residual = c->h_out[1] > 0.0 ? c->h_out[0] / c->h_out[1] : 0.0;  // no fluid: nothing changes
    rep->mom_x = c->h_out[2];
    rep->mom_y = c->h_out[3];
    rep->steps_done = c->steps;
    rep->fluid_nodes = c->fluid;
    if (!std::isfinite(rep->mass) || !std::isfinite(rep->residual))
        return fail(LBM_EDIVERGED, "non-finite mass %g or residual %g after %lld steps", rep->mass,
                    rep->residual, (long long)c->steps);
    return LBM_OK;
}

extern "C" int lbm_get_macro(lbm_ctx* c, float* d_rho, float* d_ux, float* d_uy,
                             int32_t rho_minus_one) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (!d_rho && !d_ux && !d_uy) return fail(LBM_EINVAL, "no output field");
    return launch_macro(c, d_rho, d_ux, d_uy, rho_minus_one, nullptr, false);
}

extern "C" int lbm_get_populations(lbm_ctx* c, float* d_f) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (!d_f) return fail(LBM_EINVAL, "d_f is NULL");
    return launch_macro(c, nullptr, nullptr, nullptr, 0, d_f, false);
}

// Field statistics [mass, max |u|, non-finite count, 0] into d_out (device, 4
// doubles), asynchronously on ctx's stream.
static int launch_field_stats(lbm_ctx* c, const float* d_rho, const float* d_ux, const float* d_uy,
                              double* d_out) {
    const int N = c->g.N;
    const int nb = (N + 255) / 256;
    if (nb > c->nblocks) {
        // the partials scratch holds nblocks rows; nblocks >= ceil(N / 256) always
        return fail(LBM_EINVAL, "internal: partial buffer too small");
    }
    k_field_stats<<<nb, 256, 0, c->stream>>>(c->d_mask, N, d_rho, d_ux, d_uy, c->d_partials);
    k_field_stats_final<<<1, 256, 0, c->stream>>>(c->d_partials, nb, d_out);
    LBM_HIP(hipGetLastError());
    return LBM_OK;
}

extern "C" int lbm_check_fields_async(lbm_ctx* c, const float* d_rho, const float* d_ux,
                                      const float* d_uy, double* d_stats) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (!d_rho || !d_ux || !d_uy || !d_stats) return fail(LBM_EINVAL, "NULL argument");
    return launch_field_stats(c, d_rho, d_ux, d_uy, d_stats);
}

extern "C" int lbm_check_fields(lbm_ctx* c, const float* d_rho, const float* d_ux,
                                const float* d_uy, lbm_field_stats* out) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (!d_rho || !d_ux || !d_uy || !out) return fail(LBM_EINVAL, "NULL argument");
    int rc = launch_field_stats(c, d_rho, d_ux, d_uy, c->d_out);
    if (rc) return rc;
    LBM_HIP(hipMemcpyAsync(c->h_out, c->d_out, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    LBM_HIP(hipStreamSynchronize(c->stream));
    out->mass = c->h_out[0];
    out->max_speed = c->h_out[1];
    out->nonfinite = (int64_t)c->h_out[2];
    out->fluid_nodes = c->fluid;
    return LBM_OK;
}

extern "C" int lbm_compare_fields(lbm_ctx* c, const float* d_drho, const float* d_ux,
                                  const float* d_uy, const float* d_drho_ref, const float* d_ux_ref,
                                  const float* d_uy_ref, lbm_field_error* out) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (!d_drho || !d_ux || !d_uy || !d_drho_ref || !d_ux_ref || !d_uy_ref || !out)
        return fail(LBM_EINVAL, "NULL argument");
    const int N = c->g.N;
    const int nb = std::min(CMP_BLOCKS, (N + 255) / 256);
    k_compare<<<nb, 256, 0, c->stream>>>(c->d_mask, c->cfg.nx, N, d_drho, d_ux, d_uy, d_drho_ref,
                                         d_ux_ref, d_uy_ref, c->d_cmp);
    k_compare_final<<<1, 64, 0, c->stream>>>(c->d_cmp, nb, c->d_out);
    LBM_HIP(hipGetLastError());
    LBM_HIP(hipMemcpyAsync(c->h_out, c->d_out, CMP_VALUES * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
    LBM_HIP(hipStreamSynchronize(c->stream));
    const double* h = c->h_out;
    auto ratio = [](double a, double b) { return b > 0.0 ? a / b : (a > 0.0 ? INFINITY : 0.0); };
    out->rel_l1_rho = ratio(h[0], h[1]);
    out->rel_l1_ux = ratio(h[2], h[3]);
    out->rel_l1_uy = ratio(h[4], h[5]);
    const double cs2 = 1.0 / 3.0;
    out->dp = (h[8] > 0 && h[11] > 0) ? cs2 * (h[6] / h[8] - h[9] / h[11]) : 0.0;
    out->dp_ref = (h[8] > 0 && h[11] > 0) ? cs2 * (h[7] / h[8] - h[10] / h[11]) : 0.0;
    out->rel_dp = ratio(fabs(out->dp - out->dp_ref), fabs(out->dp_ref));
    return LBM_OK;
}

extern "C" const char* lbm_step_kernel(const lbm_ctx* c) {
    if (!c) return "";
    const bool lean = c->cfg.arith == LBM_ARITH_LEAN, f32 = c->cfg.arith == LBM_ARITH_FP32;
    static const char* const fused[6][3] = {
        {"", "", ""},
        {"pair-64x8/lean", "pair-64x8/fp32", "pair-64x8/mixed"},
        {"pair-64x4/lean", "pair-64x4/fp32", "pair-64x4/mixed"},
        {"deep4-64x8/lean", "deep4-64x8/fp32", "deep4-64x8/mixed"},
        {"deep5-64x16/lean", "deep5-64x16/fp32", "deep5-64x16/mixed"},
        {"deep4-64x8/lean", "deep4-64x8/fp32", "deep4-64x8/mixed"}};
    if (c->spl > 1) return fused[c->shape][lean ? 0 : f32 ? 1 : 2];
    if (c->vec4) return lean ? "quad/lean" : f32 ? "quad/fp32" : "quad/mixed";
    return lean ? "node/lean" : f32 ? "node/fp32" : "node/mixed";
}

extern "C" int lbm_info(const lbm_ctx* c, int64_t* fluid_nodes, int64_t* steps_done) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (fluid_nodes) *fluid_nodes = c->fluid;
    if (steps_done) *steps_done = c->steps;
    return LBM_OK;
}

// ================================================================== batches

struct lbm_batch {
    int n = 0;
    std::vector<lbm_ctx*> ctx;
    hipStream_t stream = nullptr;
    StepArgs* d_args[2] = {nullptr, nullptr};
    BatchTile* d_tiles = nullptr;
    int ntiles = 0;
    bool quad = false, nt = false;
    int spl = 1;            // steps per launch: 2 pair (one-node tiles), 3 or 4 deep (64 x 8 tiles)
    BatchTile* d_mtiles = nullptr;   // 64 x 8 tile table of the deep shapes
    int nmtiles = 0;
    bool trt = false;       // every trajectory uses the TRT collision
    int parity = 0;
    int64_t steps = 0;
    int chunk = 32;         // graph chunk: an even number of launches
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    std::string choice;
};

static void batch_release(lbm_batch* b) {
    if (!b) return;
    for (int k = 0; k < 2; ++k) {
        if (b->graph[k]) (void)hipGraphExecDestroy(b->graph[k]);
        if (b->d_args[k]) (void)hipFree(b->d_args[k]);
    }
    if (b->d_tiles) (void)hipFree(b->d_tiles);
    if (b->d_mtiles) (void)hipFree(b->d_mtiles);
    for (lbm_ctx* c : b->ctx) release(c);
    delete b;
}

extern "C" void lbm_batch_destroy(lbm_batch* b) { batch_release(b); }

static StepArgs step_args_for(const lbm_ctx* c, int parity) {
    StepArgs a;
    a.src = c->f[parity];
    a.dst = c->f[parity ^ 1];
    a.link = c->d_link;
    a.mask = c->d_mask;
    a.drho_out = c->d_drho;
    a.g = c->g;
    set_relaxation(a, c->cfg);
    a.gx = c->cfg.gx;
    a.gy = c->cfg.gy;
    a.u_in = c->cfg.u_in;
    a.rho_out = c->cfg.rho_out;
    return a;
}

// Tile table for one kernel shape: trajectory-major, rows of tiles in order, so
// that the XCD remap keeps each trajectory's tiles (which share halo rows) together.
// Trajectory-major tile table of 64 x rows tiles (four-wide: 256 x rows).
static int make_tiles(lbm_batch* b, bool quad, int rows, BatchTile** d, int* count) {
    std::vector<BatchTile> t;
    for (int i = 0; i < b->n; ++i) {
        const lbm_ctx* c = b->ctx[i];
        const int gx = quad ? c->gridx4 : c->g.gridx;
        const int gy = (c->g.ny + rows - 1) / rows;
        for (int y = 0; y < gy; ++y)
            for (int x = 0; x < gx; ++x) t.push_back(BatchTile{i, x, y, 0});
    }
    if (*d) (void)hipFree(*d);
    *d = nullptr;
    LBM_HIP(hipMalloc(d, t.size() * sizeof(BatchTile)));
    LBM_HIP(hipMemcpy(*d, t.data(), t.size() * sizeof(BatchTile), hipMemcpyHostToDevice));
    *count = (int)t.size();
    return LBM_OK;
}

static int build_tiles(lbm_batch* b, bool quad) {
    b->quad = quad;
    int rc = make_tiles(b, quad, TY, &b->d_tiles, &b->ntiles);
    if (rc || b->spl < 3) return rc;
    return make_tiles(b, false, 8, &b->d_mtiles, &b->nmtiles);
}

template <int S, int RY, typename R>
static void launch_batchm_s(lbm_batch* b, int parity, const BatchTile* tiles, int ntiles) {
    dim3 blk(TX, RY), grd(ntiles);
    if (b->nt) k_bgk_batchm<S, RY, true, R><<<grd, blk, 0, b->stream>>>(b->d_args[parity], tiles);
    else k_bgk_batchm<S, RY, false, R><<<grd, blk, 0, b->stream>>>(b->d_args[parity], tiles);
}
template <typename R>
static void launch_batch2_r(lbm_batch* b, int parity) {
    if (b->spl == 2) launch_batchm_s<2, TY, R>(b, parity, b->d_tiles, b->ntiles);
    else if (b->spl == 3) launch_batchm_s<3, 8, R>(b, parity, b->d_mtiles, b->nmtiles);
    else launch_batchm_s<4, 8, R>(b, parity, b->d_mtiles, b->nmtiles);
}
// One fused launch of b->spl steps.
static void launch_batch2(lbm_batch* b, int parity) {
    if (b->trt) launch_batch2_r<LeanTRT>(b, parity);
    else launch_batch2_r<Lean>(b, parity);
}

template <typename R>
static void launch_batch_r(lbm_batch* b, int parity) {
    dim3 blk(TX, TY), grd(b->ntiles);
    if (b->quad) {
        if (b->nt) k_bgk_batch<true, true, R><<<grd, blk, 0, b->stream>>>(b->d_args[parity], b->d_tiles);
        else k_bgk_batch<true, false, R><<<grd, blk, 0, b->stream>>>(b->d_args[parity], b->d_tiles);
    } else {
        if (b->nt) k_bgk_batch<false, true, R><<<grd, blk, 0, b->stream>>>(b->d_args[parity], b->d_tiles);
        else k_bgk_batch<false, false, R><<<grd, blk, 0, b->stream>>>(b->d_args[parity], b->d_tiles);
    }
}

static void launch_batch(lbm_batch* b, int parity) {
    if (b->trt) launch_batch_r<LeanTRT>(b, parity);
    else launch_batch_r<Lean>(b, parity);
}

static int reset_rest(lbm_batch* b) {
    for (lbm_ctx* c : b->ctx) {
        const size_t n = 9 * (size_t)c->g.N;
        k_copy_f32<<<copy_grid(n), 256, 0, b->stream>>>(nullptr, c->f[0], n);
        c->cur = 0;
        c->steps = 0;
    }
    LBM_HIP(hipGetLastError());
    LBM_HIP(hipStreamSynchronize(b->stream));
    b->parity = 0;
    b->steps = 0;
    return LBM_OK;
}

// Autotuner: time every admissible (kernel shape, store policy) pair on the batch
// itself and keep the fastest.  Results are cached in a text file of
// "<key> <quad> <nt>" lines keyed by device and batch geometry.
static std::string batch_key(const lbm_batch* b) {
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        arch = prop.gcnArchName;
    for (char& ch : arch)
        if (ch == ' ' || ch == ':') ch = '_';
    uint64_t h = 1469598103934665603ull;
    for (const lbm_ctx* c : b->ctx) {
        const uint64_t v[3] = {(uint64_t)c->g.nx, (uint64_t)c->g.ny, (uint64_t)c->cfg.bc_x};
        for (uint64_t x : v) { h ^= x; h *= 1099511628211ull; }
    }
    char buf[256];
    snprintf(buf, sizeof buf, "%s:n%d:%016llx", arch.c_str(), b->n, (unsigned long long)h);
    return buf;
}

static bool cache_lookup(const char* path, const std::string& key, int* shape, bool* nt) {
    if (!path) return false;
    FILE* f = fopen(path, "r");
    if (!f) return false;
    char k[256];
    int q = 0, t = 0;
    bool found = false;
    while (fscanf(f, "%255s %d %d", k, &q, &t) == 3)
        if (key == k) { *shape = q; *nt = t != 0; found = true; }
    fclose(f);
    return found;
}

static void cache_store(const char* path, const std::string& key, int shape, bool nt) {
    if (!path) return;
    FILE* f = fopen(path, "a");
    if (!f) return;
    fprintf(f, "%s %d %d\n", key.c_str(), shape, nt ? 1 : 0);
    fclose(f);
}

// Kernel shapes of a batch: 0 one node per lane, 1 four nodes per lane, 2 two steps
// per launch (on the one-node tiles), 3 and 4 three and four steps per launch (on
// 64 x 8 tiles).
static const int kBatchShapes = 5;
static const char* shape_name(int shape) {
    static const char* const names[kBatchShapes] = {"node", "quad", "pair", "deep3", "deep4"};
    return names[shape];
}

static int set_shape(lbm_batch* b, int shape) {
    b->spl = shape >= 2 ? shape : 1;
    b->chunk = b->spl == 3 ? 30 : 32;
    return build_tiles(b, shape == 1);
}

static int autotune(lbm_batch* b, bool quad_ok, const char* cache) {
    const std::string key = batch_key(b);
    int q = 0;
    bool t = false;
    if (cache_lookup(cache, key, &q, &t) && q >= 0 && q < kBatchShapes && (quad_ok || q != 1)) {
        b->nt = t;
        int rc = set_shape(b, q);
        if (rc) return rc;
        b->choice = std::string("cached ") + shape_name(q) + (t ? "+nt" : "");
        return LBM_OK;
    }
    // three rounds over all candidates (the order reversed every round), each
    // candidate keeping its fastest round: one noisy timing does not decide
    float tmin[kBatchShapes][2];
    for (auto& r : tmin) r[0] = r[1] = 1e30f;
    hipEvent_t e0, e1;
    LBM_HIP(hipEventCreate(&e0));
    LBM_HIP(hipEventCreate(&e1));
    for (int round = 0; round < 3; ++round) {
        for (int c = 0; c < kBatchShapes; ++c) {
            const int qi = round % 2 ? c : kBatchShapes - 1 - c;
            if (qi == 1 && !quad_ok) continue;
            int rc = set_shape(b, qi);
            if (rc) return rc;
            for (int ti = 0; ti < 2; ++ti) {
                b->nt = ti != 0;
                // 16 timed launches (16 x spl steps), after an even warm-up
                for (int k = 0; k < 4; ++k) {
                    if (b->spl > 1) launch_batch2(b, k & 1); else launch_batch(b, k & 1);
                }
                LBM_HIP(hipEventRecord(e0, b->stream));
                for (int k = 0; k < 16; ++k) {
                    if (b->spl > 1) launch_batch2(b, k & 1); else launch_batch(b, k & 1);
                }
                LBM_HIP(hipEventRecord(e1, b->stream));
                LBM_HIP(hipEventSynchronize(e1));
                float ms = 0.0f;
                LBM_HIP(hipEventElapsedTime(&ms, e0, e1));
                ms /= 16.0f * b->spl;   // per lattice step
                tmin[qi][ti] = std::min(tmin[qi][ti], ms);
            }
        }
    }
    float best = 1e30f;
    int bq = 0;
    bool bt = false;
    for (int qi = kBatchShapes - 1; qi >= 0; --qi)
        for (int ti = 0; ti < 2; ++ti)
            if (tmin[qi][ti] < best) { best = tmin[qi][ti]; bq = qi; bt = ti != 0; }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->nt = bt;
    int rc = set_shape(b, bq);
    if (rc) return rc;
    char msg[96];
    snprintf(msg, sizeof msg, "tuned %s%s %.4f ms/step", shape_name(bq), bt ? "+nt" : "", best);
    b->choice = msg;
    cache_store(cache, key, bq, bt);
    return reset_rest(b);
}

extern "C" int lbm_batch_create(lbm_batch** out, const lbm_traj_desc* h_desc, int32_t ntraj,
                                const char* tune_cache, void* stream) {
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (!h_desc || ntraj < 1) return fail(LBM_EINVAL, "ntraj = %d", ntraj);
    for (int i = 0; i < ntraj; ++i) {
        int rc = validate_config(&h_desc[i].cfg);
        if (rc) return fail(rc, "trajectory %d: %s", i, lbm_last_error());
        if (h_desc[i].cfg.arith != LBM_ARITH_LEAN)
            return fail(LBM_EUNSUPPORTED, "trajectory %d: batches run the LBM_ARITH_LEAN step", i);
        if ((h_desc[i].cfg.trt_lambda > 0.0) != (h_desc[0].cfg.trt_lambda > 0.0))
            return fail(LBM_EINVAL, "trajectory %d: a batch is all BGK or all TRT", i);
        if (!h_desc[i].d_mask || !h_desc[i].d_fA || !h_desc[i].d_fB)
            return fail(LBM_EINVAL, "trajectory %d: NULL device buffer", i);
    }
    lbm_batch* b = new (std::nothrow) lbm_batch();
    if (!b) return fail(LBM_ENOMEM, "batch allocation");
    b->n = ntraj;
    b->trt = h_desc[0].cfg.trt_lambda > 0.0;
    b->stream = (hipStream_t)stream;
    bool quad_ok = true;
    for (int i = 0; i < ntraj; ++i) {
        lbm_ctx* c = nullptr;
        lbm_config cfg = h_desc[i].cfg;
        cfg.kernel = LBM_KERNEL_NODE;
        int rc = lbm_init(&c, &cfg, h_desc[i].d_mask, h_desc[i].d_fA, h_desc[i].d_fB, stream);
        if (rc) { batch_release(b); return rc; }
        b->ctx.push_back(c);
        quad_ok = quad_ok && cfg.nx % 4 == 0 && cfg.nx >= 4 &&
                  (uintptr_t)h_desc[i].d_fA % 16 == 0 && (uintptr_t)h_desc[i].d_fB % 16 == 0;
    }
    std::vector<StepArgs> a0, a1;
    for (lbm_ctx* c : b->ctx) {
        a0.push_back(step_args_for(c, 0));
        a1.push_back(step_args_for(c, 1));
    }
    for (int k = 0; k < 2; ++k) {
        hipError_t e = hipMalloc(&b->d_args[k], ntraj * sizeof(StepArgs));
        if (e == hipSuccess)
            e = hipMemcpy(b->d_args[k], k ? a1.data() : a0.data(), ntraj * sizeof(StepArgs),
                          hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            batch_release(b);
            return fail(LBM_EHIP, "batch arguments: %s", hipGetErrorString(e));
        }
    }
    int rc = autotune(b, quad_ok, tune_cache);
    if (rc) { batch_release(b); return rc; }
    *out = b;
    return LBM_OK;
}

static int batch_build_graph(lbm_batch* b) {
    const int start = b->parity;
    hipGraph_t g = nullptr;
    LBM_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    if (b->spl > 1) {
        for (int k = 0; k < b->chunk / b->spl; ++k) launch_batch2(b, start ^ (k & 1));
    } else {
        for (int k = 0; k < b->chunk; ++k) launch_batch(b, start ^ (k & 1));
    }
    hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (e != hipSuccess) return fail(LBM_EHIP, "batch graph capture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&b->graph[start], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        b->graph[start] = nullptr;
        return fail(LBM_EHIP, "batch graph instantiate: %s", hipGetErrorString(e));
    }
    return LBM_OK;
}

extern "C" int lbm_batch_step(lbm_batch* b, int32_t n) {
    if (!b) return fail(LBM_EINVAL, "batch is NULL");
    if (n < 0) return fail(LBM_EINVAL, "n = %d < 0", n);
    for (const lbm_ctx* c : b->ctx)
        if (c->cur != b->parity)
            return fail(LBM_EINVAL, "a trajectory was stepped outside the batch");
    int left = n;
    if (b->stream != nullptr) {
        while (left >= b->chunk) {
            if (!b->graph[b->parity]) {
                int rc = batch_build_graph(b);
                if (rc) return rc;
            }
            LBM_HIP(hipGraphLaunch(b->graph[b->parity], b->stream));
            left -= b->chunk;  // an even number of parity flips
        }
    }
    if (b->spl > 1) {
        for (; left >= b->spl; left -= b->spl) {
            launch_batch2(b, b->parity);
            b->parity ^= 1;
        }
    }
    for (int k = 0; k < left; ++k) {
        launch_batch(b, b->parity);
        b->parity ^= 1;
    }
    LBM_HIP(hipGetLastError());
    b->steps += n;
    for (lbm_ctx* c : b->ctx) {
        c->cur = b->parity;
        c->steps += n;
    }
    return LBM_OK;
}

extern "C" int lbm_batch_context(lbm_batch* b, int32_t i, lbm_ctx** out) {
    if (!b || !out) return fail(LBM_EINVAL, "NULL argument");
    if (i < 0 || i >= b->n) return fail(LBM_EINVAL, "trajectory %d of %d", i, b->n);
    *out = b->ctx[i];
    return LBM_OK;
}

extern "C" const char* lbm_batch_choice(const lbm_batch* b) { return b ? b->choice.c_str() : ""; }

namespace lbmfno {

// ================================================================= adjoint
//
// Vector-Jacobian product of one step f(n+1) = Z(P C(f(n))):
// lam_n = C'(f(n))^T P^T Z'^T lam_{n+1}.  Z is the Zou-He closure of the boundary
// columns (identity for periodic and wall boundaries); Z'^T, the transpose of its
// Jacobian, is applied on the fly where lam_{n+1} is read at a Zou-He column node
// (zh_nu).  P^T is the inverse of the pull permutation: slot (q, y) was pulled by
// y + c_q when that node is fluid and inside the domain (link bit opp(q)-1 of y
// clear), otherwise it bounced back into y as opp(q).  C' is the per-node collision
// Jacobian with d rho / d f_j = 1 and d u / d f_j = (c_j - u + g/2) / rho.  FP64
// registers, float32 in and out.
struct AdjArgs {
    const float* __restrict__ f;      // pre-collision populations f(n), absolute
    const float* __restrict__ lam1;   // lam_{n+1}
    float* __restrict__ lam0;         // lam_n
    const uint8_t* __restrict__ link;
    const uint8_t* __restrict__ mask;
    LatticeGeom g;
    double omega, guo, gx, gy, u_in, rho_out;
    double omega_m, guo_m;            // TRT: 1 / tau-, 1 - 1 / (2 tau-)
};

// (Z'^T lam)_q at a fluid node t of a Zou-He column.  The closures (zouhe()) set the
// three unknown populations from the known ones after streaming; in the transpose
// the unknowns' adjoints move onto the known populations they were formed from, and
// the unknown slots themselves get zero.  Inlet (x = 0, velocity u_in): unknowns
// 1, 5, 8, rho = (f0 + f2 + f4 + 2 (f3 + f6 + f7)) / (1 - u_in); outlet
// (x = nx - 1, density rho_out): unknowns 3, 6, 7, u_x = -1 + (f0 + f2 + f4 +
// 2 (f1 + f5 + f8)) / rho_out.
__device__ __forceinline__ double zh_nu(const float* __restrict__ lam, size_t N, int t, int q,
                                        bool inlet, double u_in) {
    if (inlet) {
        if (q == 1 || q == 5 || q == 8) return 0.0;
        const double l1 = lam[1 * N + t], l5 = lam[5 * N + t], l8 = lam[8 * N + t];
        const double drho = (q == 3 || q == 6 || q == 7) ? 2.0 : 1.0;   // q in {0, 2, 4}: 1
        double v = (double)lam[q * N + t] +
                   u_in / (1.0 - u_in) * drho * ((2.0 / 3.0) * l1 + (1.0 / 6.0) * (l5 + l8));
        if (q == 3) v += l1;
        if (q == 7) v += l5;
        if (q == 6) v += l8;
        if (q == 2) v += 0.5 * (l8 - l5);
        if (q == 4) v += 0.5 * (l5 - l8);
        return v;
    }
    if (q == 3 || q == 6 || q == 7) return 0.0;
    const double l3 = lam[3 * N + t], l6 = lam[6 * N + t], l7 = lam[7 * N + t];
    const double dux = (q == 1 || q == 5 || q == 8) ? 2.0 : 1.0;         // q in {0, 2, 4}: 1
    double v = (double)lam[q * N + t] - dux * ((2.0 / 3.0) * l3 + (1.0 / 6.0) * (l6 + l7));
    if (q == 1) v += l3;
    if (q == 8) v += l6;
    if (q == 5) v += l7;
    if (q == 2) v += 0.5 * (l7 - l6);
    if (q == 4) v += 0.5 * (l6 - l7);
    return v;
}

// TRT: the collision relaxes the pair-even part of f - f_eq at omega and the
// pair-odd part at omega_m, with the Guo source split the same way, so
// C^T mu = mu - nu + J^T nu + S'^T sg with nu = omega mu+ + omega_m mu- and
// sg = guo mu+ + guo_m mu- (mu+- the even and odd parts of mu, J = d f_eq / d f,
// S' the source's derivative without its prefactor).
template <bool FORCE, bool ZH, bool TRT>
__global__ __launch_bounds__(256) void k_adjoint_step(AdjArgs a) {
    const int b = blockIdx.x;
    const int by = b / a.g.gridx, bx = b - by * a.g.gridx;
    const int i = bx * TX + threadIdx.x, j = by * TY + threadIdx.y;
    if (i >= a.g.nx || j >= a.g.ny) return;
    const int n = j * a.g.nx + i;
    const size_t N = (size_t)a.g.N;
    const unsigned lk = a.link[n];
    if (is_solid(lk, a.mask, n)) {
#pragma unroll
        for (int q = 0; q < 9; ++q) a.lam0[q * N + n] = 0.0f;
        return;
    }
    const int im = i == 0 ? a.g.nx - 1 : i - 1, ip = i == a.g.nx - 1 ? 0 : i + 1;
    const int jm = j == 0 ? a.g.ny - 1 : j - 1, jp = j == a.g.ny - 1 ? 0 : j + 1;
    const int r0 = j * a.g.nx, rm = jm * a.g.nx, rp = jp * a.g.nx;
    // push target y + c_q for q = 1..8; (Z'^T lam_{n+1}) read at node t of column col
    const int nx = a.g.nx;
    auto nu = [&](int q, int t, int col) -> double {
        if (ZH && (col == 0 || col == nx - 1)) return zh_nu(a.lam1, N, t, q, col == 0, a.u_in);
        return (double)a.lam1[q * N + t];
    };
    double mu[9];
    mu[0] = nu(0, n, i);
#define LBM_PUSH(Q, TGT, COL)                                                             \
    mu[Q] = ((lk >> (opp_of(Q) - 1)) & 1u) ? nu(opp_of(Q), n, i) : nu(Q, (TGT), (COL));
    LBM_PUSH(1, r0 + ip, ip)
    LBM_PUSH(2, rp + i, i)
    LBM_PUSH(3, r0 + im, im)
    LBM_PUSH(4, rm + i, i)
    LBM_PUSH(5, rp + ip, ip)
    LBM_PUSH(6, rp + im, im)
    LBM_PUSH(7, rm + im, im)
    LBM_PUSH(8, rm + ip, ip)
#undef LBM_PUSH
    double nu_[9], sg[9];
    if (TRT) {
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            const int qb = opp_of(q);
            const double even = 0.5 * (mu[q] + mu[qb]), odd = 0.5 * (mu[q] - mu[qb]);
            nu_[q] = fma(a.omega, even, a.omega_m * odd);
            sg[q] = fma(a.guo, even, a.guo_m * odd);
        }
    }
    double f[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) f[q] = (double)a.f[q * N + n] - w_of_d(q);
    const Moments<double> m = moments<FORCE, double>(f, a.gx, a.gy);
    const double usq = fma(m.ux, m.ux, m.uy * m.uy);
    const double gu = fma(a.gx, m.ux, a.gy * m.uy);
    double A = 0.0, Bx = 0.0, By = 0.0;
#define LBM_ADJ_ACC(Q)                                                                        \
    {                                                                                         \
        const double cu = cdot<Q, double>(m.ux, m.uy);                                        \
        const double wq = w_of_d(Q);                                                          \
        /* d f_eq / d rho and d f_eq / d u */                                                 \
        const double dfr = wq * (1.0 + fma(cu, fma(4.5, cu, 3.0), -1.5 * usq));              \
        const double k = wq * m.rho * fma(9.0, cu, 3.0);                                      \
        double dfx = (double)cx_of(Q) * k - wq * m.rho * 3.0 * m.ux;                          \
        double dfy = (double)cy_of(Q) * k - wq * m.rho * 3.0 * m.uy;                          \
        if (TRT) {                                                                            \
            double t = nu_[Q] * dfr, tx = nu_[Q] * dfx, ty = nu_[Q] * dfy;                    \
            if (FORCE) {                                                                      \
                const double cg = cdot<Q, double>(a.gx, a.gy);                                \
                t = fma(sg[Q], wq * (3.0 * (cg - gu) + 9.0 * cu * cg), t);                    \
                tx = fma(sg[Q], wq * m.rho * (-3.0 * a.gx + 9.0 * (double)cx_of(Q) * cg), tx); \
                ty = fma(sg[Q], wq * m.rho * (-3.0 * a.gy + 9.0 * (double)cy_of(Q) * cg), ty); \
            }                                                                                 \
            A += t;                                                                           \
            Bx += tx;                                                                         \
            By += ty;                                                                         \
        } else {                                                                              \
            double t = a.omega * dfr, tx = a.omega * dfx, ty = a.omega * dfy;                \
            if (FORCE) {                                                                      \
                const double cg = cdot<Q, double>(a.gx, a.gy);                                \
                t += a.guo * wq * (3.0 * (cg - gu) + 9.0 * cu * cg);                          \
                tx += a.guo * wq * m.rho * (-3.0 * a.gx + 9.0 * (double)cx_of(Q) * cg);       \
                ty += a.guo * wq * m.rho * (-3.0 * a.gy + 9.0 * (double)cy_of(Q) * cg);       \
            }                                                                                 \
            A = fma(mu[Q], t, A);                                                             \
            Bx = fma(mu[Q], tx, Bx);                                                          \
            By = fma(mu[Q], ty, By);                                                          \
        }                                                                                     \
    }
    LBM_ADJ_ACC(0) LBM_ADJ_ACC(1) LBM_ADJ_ACC(2) LBM_ADJ_ACC(3) LBM_ADJ_ACC(4)
    LBM_ADJ_ACC(5) LBM_ADJ_ACC(6) LBM_ADJ_ACC(7) LBM_ADJ_ACC(8)
#undef LBM_ADJ_ACC
    const double inv = 1.0 / m.rho;
    const double vx = m.ux - 0.5 * a.gx, vy = m.uy - 0.5 * a.gy;  // (sum c f) / rho
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const double dux = ((double)cx_of(q) - vx) * inv, duy = ((double)cy_of(q) - vy) * inv;
        const double diag = TRT ? mu[q] - nu_[q] : (1.0 - a.omega) * mu[q];
        a.lam0[q * N + n] = (float)(diag + A + Bx * dux + By * duy);
    }
}

// lam = d L / d f(n) from upstream gradients of the macroscopic fields of f(n):
// lam_j = g_rho + g_u . (c_j - u + g/2) / rho (solids: 0).
__global__ __launch_bounds__(256) void k_macro_vjp(const float* __restrict__ fpop,
                                                   const uint8_t* __restrict__ mask, int N,
                                                   double gx, double gy,
                                                   const float* __restrict__ grho,
                                                   const float* __restrict__ gux,
                                                   const float* __restrict__ guy,
                                                   float* __restrict__ lam) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    const size_t NN = (size_t)N;
    if (mask[n]) {
        for (int q = 0; q < 9; ++q) lam[q * NN + n] = 0.0f;
        return;
    }
    double rho = 0.0, jx = 0.0, jy = 0.0;
    for (int q = 0; q < 9; ++q) {
        const double v = fpop[q * NN + n];
        rho += v;
        jx += cx_of(q) * v;
        jy += cy_of(q) * v;
    }
    const double vx = jx / rho, vy = jy / rho;
    const double ar = grho[n], ax = gux[n], ay = guy[n];
    (void)gx; (void)gy;  // u - g/2 = (sum c f)/rho: the half force cancels
    for (int q = 0; q < 9; ++q)
        lam[q * NN + n] = (float)(ar + (ax * (cx_of(q) - vx) + ay * (cy_of(q) - vy)) / rho);
}

// Pull-back through f(0) = Z(f_eq(rho, u)): g_rho = sum_q nu_q d f_eq_q / d rho,
// g_u = sum_q nu_q d f_eq_q / d u with nu = Z'^T lam (the Zou-He closures, zh != 0,
// at the boundary columns; lam itself elsewhere).  Solids: 0.
__global__ __launch_bounds__(256) void k_feq_vjp(const uint8_t* __restrict__ mask, int N, int nx,
                                                 int zh, double u_in,
                                                 const float* __restrict__ rho,
                                                 const float* __restrict__ ux,
                                                 const float* __restrict__ uy,
                                                 const float* __restrict__ lam,
                                                 float* __restrict__ grho, float* __restrict__ gux,
                                                 float* __restrict__ guy) {
    const int n = blockIdx.x * blockDim.x + threadIdx.x;
    if (n >= N) return;
    if (mask[n]) { grho[n] = 0.0f; gux[n] = 0.0f; guy[n] = 0.0f; return; }
    const size_t NN = (size_t)N;
    const int col = n % nx;
    const bool closed = zh && (col == 0 || col == nx - 1);
    const double r = rho[n], u = ux[n], v = uy[n];
    const double usq = fma(u, u, v * v);
    double a = 0.0, bx = 0.0, by = 0.0;
    for (int q = 0; q < 9; ++q) {
        const double l = closed ? zh_nu(lam, NN, n, q, col == 0, u_in) : (double)lam[q * NN + n];
        const double cu = cx_of(q) * u + cy_of(q) * v;
        const double wq = w_of_d(q);
        a = fma(l, wq * (1.0 + fma(cu, fma(4.5, cu, 3.0), -1.5 * usq)), a);
        const double k = wq * r * fma(9.0, cu, 3.0);
        bx = fma(l, cx_of(q) * k - 3.0 * wq * r * u, bx);
        by = fma(l, cy_of(q) * k - 3.0 * wq * r * v, by);
    }
    grho[n] = (float)a;
    gux[n] = (float)bx;
    guy[n] = (float)by;
}

}  // namespace lbmfno

using namespace lbmfno;

extern "C" int lbm_adjoint_step(lbm_ctx* c, const float* d_f_n, const float* d_lam_np1,
                                float* d_lam_n) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (!d_f_n || !d_lam_np1 || !d_lam_n) return fail(LBM_EINVAL, "NULL buffer");
    if (d_lam_np1 == d_lam_n) return fail(LBM_EINVAL, "lam_{n+1} and lam_n must differ");
    AdjArgs a;
    a.f = d_f_n;
    a.lam1 = d_lam_np1;
    a.lam0 = d_lam_n;
    a.link = c->d_link;
    a.mask = c->d_mask;
    a.g = c->g;
    a.omega = 1.0 / c->cfg.tau;
    a.guo = 1.0 - 0.5 / c->cfg.tau;
    const bool trt = c->cfg.trt_lambda > 0.0;
    const double tau_m = trt ? 0.5 + c->cfg.trt_lambda / (c->cfg.tau - 0.5) : c->cfg.tau;
    a.omega_m = 1.0 / tau_m;
    a.guo_m = 1.0 - 0.5 / tau_m;
    a.gx = c->cfg.gx;
    a.gy = c->cfg.gy;
    a.u_in = c->cfg.u_in;
    a.rho_out = c->cfg.rho_out;
    dim3 blk(TX, TY), grd(c->nblocks);
    const bool force = a.gx != 0.0 || a.gy != 0.0, zh = c->cfg.bc_x == LBM_BC_ZOUHE;
#define LBM_ADJ_LAUNCH(T)                                                                \
    if (zh) {                                                                            \
        if (force) k_adjoint_step<true, true, T><<<grd, blk, 0, c->stream>>>(a);         \
        else k_adjoint_step<false, true, T><<<grd, blk, 0, c->stream>>>(a);              \
    } else {                                                                             \
        if (force) k_adjoint_step<true, false, T><<<grd, blk, 0, c->stream>>>(a);        \
        else k_adjoint_step<false, false, T><<<grd, blk, 0, c->stream>>>(a);             \
    }
    if (trt) { LBM_ADJ_LAUNCH(true) } else { LBM_ADJ_LAUNCH(false) }
#undef LBM_ADJ_LAUNCH
    LBM_HIP(hipGetLastError());
    return LBM_OK;
}

extern "C" int lbm_macro_vjp(lbm_ctx* c, const float* d_f_n, const float* d_g_rho,
                             const float* d_g_ux, const float* d_g_uy, float* d_lam) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (!d_f_n || !d_g_rho || !d_g_ux || !d_g_uy || !d_lam) return fail(LBM_EINVAL, "NULL buffer");
    const int N = c->g.N;
    k_macro_vjp<<<(N + 255) / 256, 256, 0, c->stream>>>(d_f_n, c->d_mask, N, c->cfg.gx, c->cfg.gy,
                                                        d_g_rho, d_g_ux, d_g_uy, d_lam);
    LBM_HIP(hipGetLastError());
    return LBM_OK;
}

extern "C" int lbm_feq_vjp(lbm_ctx* c, const float* d_rho, const float* d_ux, const float* d_uy,
                           const float* d_lam, float* d_g_rho, float* d_g_ux, float* d_g_uy) {
    if (!c) return fail(LBM_EINVAL, "ctx is NULL");
    if (!d_rho || !d_ux || !d_uy || !d_lam || !d_g_rho || !d_g_ux || !d_g_uy)
        return fail(LBM_EINVAL, "NULL buffer");
    const int N = c->g.N;
    k_feq_vjp<<<(N + 255) / 256, 256, 0, c->stream>>>(c->d_mask, N, c->g.nx,
                                                      c->cfg.bc_x == LBM_BC_ZOUHE, c->cfg.u_in,
                                                      d_rho, d_ux, d_uy, d_lam, d_g_rho, d_g_ux, d_g_uy);
    LBM_HIP(hipGetLastError());
    return LBM_OK;
}

extern "C" size_t lbm_state_elems(const lbm_ctx* c) { return c ? 9 * (size_t)c->g.N : 0; }

extern "C" int lbm_save_state(lbm_ctx* c, float* d_out) {
    if (!c || !d_out) return fail(LBM_EINVAL, "NULL argument");
    const size_t n = 9 * (size_t)c->g.N;
    k_copy_f32<<<copy_grid(n), 256, 0, c->stream>>>(c->f[c->cur], d_out, n);
    LBM_HIP(hipGetLastError());
    return LBM_OK;
}

extern "C" int lbm_load_state(lbm_ctx* c, const float* d_in) {
    if (!c || !d_in) return fail(LBM_EINVAL, "NULL argument");
    const size_t n = 9 * (size_t)c->g.N;
    k_copy_f32<<<copy_grid(n), 256, 0, c->stream>>>(d_in, c->f[c->cur], n);
    LBM_HIP(hipGetLastError());
    return LBM_OK;
}
