/*
 * lbmfno.h -- C ABI of the MI355X (gfx950) hybrid FNO-LBM hot path.
 *
 * The library liblbmfno.so implements, in HIP kernels for gfx950:
 *   - the D2Q9 single-relaxation-time lattice Boltzmann step of the paper's
 *     Sec. 2.1 (equilibrium Eq. 1, BGK collision Eq. 2 read as
 *     f* = f - (f - f_eq)/tau, streaming Eq. 3, moments Eqs. 4-5) with halfway
 *     bounce-back on obstacle masks, periodic sides, Zou-He velocity inlet /
 *     pressure outlet (the porous-media setup of Sec. 3.1.1) and Guo body forcing;
 *   - the equilibrium re-initialisation f <- f_eq(rho, u) that hands macroscopic
 *     fields (e.g. an FNO prediction) back to the lattice (Sec. 2.3);
 *   - the Fourier Neural Operator forward pass of Sec. 2.2 (Eq. 6);
 *   - the adjoint (vector-Jacobian product) of one lattice step.
 *
 * Conventions (all entry points):
 *   - Return LBM_OK (0) on success or a negative LBM_E* code; no exception or
 *     signal crosses the ABI.  lbm_last_error() returns a message for the calling
 *     thread's most recent failure.
 *   - Pointers prefixed d_ are device pointers (HIP device memory of the current
 *     device), h_ host pointers.  All device buffers are owned by the caller and
 *     must outlive every call (and every context) that uses them.  A context owns
 *     only small internal buffers (link mask, reduction scratch, graphs).
 *   - `stream` is a hipStream_t passed as void*; NULL means the default stream.
 *     Work is enqueued asynchronously on it unless a call says it synchronises.
 *   - Arguments are validated on the host before any HIP call; invalid ones return
 *     LBM_EINVAL without touching the device.
 *   - Lattice planes are [ny][nx] with x fastest.  Populations are structure-of-
 *     arrays [9][ny][nx] float32 in the order
 *       q : 0     1     2     3      4      5      6       7       8
 *       c : (0,0) (1,0) (0,1) (-1,0) (0,-1) (1,1)  (-1,1)  (-1,-1) (1,-1)
 *     with weights w = 4/9, 1/9 (q=1..4), 1/36 (q=5..8) and c_s^2 = 1/3.
 *   - Obstacle masks are uint8 [ny][nx], 1 = solid, 0 = fluid.
 *   - One context must not be used from two threads at once.
 */
#ifndef LBMFNO_H
#define LBMFNO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
#define LBM_OK 0
#define LBM_EINVAL (-1)         /* invalid argument (checked before any HIP call) */
#define LBM_ENOMEM (-2)         /* device or host allocation failed */
#define LBM_EHIP (-3)           /* a HIP runtime call failed */
#define LBM_EUNSUPPORTED (-4)   /* valid but not implemented combination */
#define LBM_ENOTCONVERGED (-5)  /* step budget exhausted before the residual target */
#define LBM_EDIVERGED (-6)      /* non-finite mass or residual */

/* Boundary handling per axis. */
#define LBM_BC_PERIODIC 0  /* periodic wrap */
#define LBM_BC_WALL 1      /* no-slip wall half a cell beyond the first/last node
                              (halfway bounce-back, link-wise) */
#define LBM_BC_ZOUHE 2     /* x axis only: Zou-He velocity inlet (u_in, 0) at x = 0
                              and pressure outlet rho_out at x = nx-1 */

/* Register arithmetic of the collision.  Populations are stored and moved as
 * float32 in every mode; all modes meet 1e-5 relative field error against FP64
 * after 2000 steps except LBM_ARITH_FP32 under a body force. */
#define LBM_ARITH_MIXED 0  /* moments, equilibrium and relaxation in FP64 registers,
                              rounded once to FP32 at the store */
#define LBM_ARITH_FP32 1   /* everything in FP32 registers */
#define LBM_ARITH_LEAN 2   /* FP32 except the velocity and the linear equilibrium
                              term w (drho + 3 rho c.u), formed in FP64 (default):
                              an FP32-rounded velocity there acts as a spurious
                              force in slowly varying flow */

/* Step-kernel choice; every choice computes the same values. */
#define LBM_KERNEL_AUTO 0  /* LBM_KERNEL_DEEP (batches: the autotuner's cached pick) */
#define LBM_KERNEL_NODE 1  /* one node per lane, 4-byte accesses (any nx) */
#define LBM_KERNEL_QUAD 2  /* four x nodes per lane, 16-byte accesses (nx % 4 == 0,
                              16-byte aligned stores) */
#define LBM_KERNEL_PAIR 3  /* two steps per launch: a tile and its one-node ring
                              advance one step into LDS, then the tile advances
                              again from LDS (temporal blocking; half the store
                              traffic per step).  64 x 8 tiles when both population
                              copies fit 128 MiB, else 64 x 4 tiles with streaming
                              stores.  Any nx. */
#define LBM_KERNEL_DEEP 4  /* deeper temporal blocking: five steps per launch (a
                              four-node ring) on 64 x 16 tiles when both population
                              copies fit 128 MiB and the lattice has at least 512
                              such tiles, four steps (a three-node ring) on 64 x 8
                              tiles on smaller ones, four steps on 64 x 8 tiles with
                              streaming stores above 128 MiB.  Any nx. */

/* Lattice description.  tau > 1/2 is the BGK relaxation time (nu = (tau-1/2)/3 in
 * lattice units), (gx, gy) a uniform body force per unit mass (Guo forcing; use 0
 * with LBM_BC_ZOUHE), arith one of LBM_ARITH_*, kernel one of LBM_KERNEL_*. */
typedef struct lbm_config {
    int32_t nx, ny;
    int32_t bc_x, bc_y;
    double tau;
    double gx, gy;
    double u_in, rho_out;
    int32_t arith;
    int32_t kernel;
    double trt_lambda;  /* 0: BGK (Eq. 2).  > 0: two-relaxation-time collision (an
                           extension for stability at low tau): the parts of f, f_eq and
                           the Guo source even under c -> -c relax with tau, the odd parts
                           with tau- from lambda = (tau - 1/2)(tau- - 1/2) (1/4: the
                           stability-optimal choice, 3/16: walls exactly halfway for
                           Poiseuille flow).  LBM_ARITH_LEAN only; a batch is all BGK or
                           all TRT; lbm_adjoint_step differentiates either collision. */
} lbm_config;

/* Diagnostics of the state at time n (FP64 accumulation over fluid nodes). */
typedef struct lbm_report {
    double residual;     /* sum |rho(n) - rho(n-1)| / sum rho(n) (0 without fluid nodes) */
    double mass;         /* sum rho(n) */
    double mom_x, mom_y; /* sum rho(n) u(n) */
    int64_t steps_done;  /* n: steps since the last (re)initialisation */
    int64_t fluid_nodes;
} lbm_report;

typedef struct lbm_ctx lbm_ctx;

const char* lbm_status_str(int code);
/* Message of the calling thread's last failed call ("" if none). */
const char* lbm_last_error(void);

/* Obstacle raster (paper Sec. 3.1.1: random circular obstacles as a binary mask;
 * porosity Eq. 8 is 1 - solid fraction).  h_shapes holds nshapes descriptors of
 * 7 int64 each, (cx, cy, A, B, C, F, R): cell (i, j) is solid iff for some shape
 * A dx^2 + B dx dy + C dy^2 <= F with |dx|, |dy| <= R, dx = i - cx and dy = j - cy
 * taken as the periodic image in (-n/2, n/2] when wrap_x / wrap_y is set.  Exact
 * int64 arithmetic: 0 <= R < 2^15, |cx|, |cy| <= 2^30, (|A|+|B|+|C|) R^2 < 2^62
 * and |F| < 2^62 are required (else LBM_EINVAL).  Writes d_mask (uint8 [ny][nx]).  Copies the shapes to the device and synchronises
 * `stream` before returning. */
int lbm_mask_raster(int32_t nx, int32_t ny, int32_t wrap_x, int32_t wrap_y,
                    const int64_t* h_shapes, int32_t nshapes, uint8_t* d_mask, void* stream);

/* Create a lattice context on the current device.  d_mask: uint8 [ny][nx]
 * (copied into per-node link bits; the caller may free it afterwards).  d_fA and
 * d_fB: caller-owned float32 buffers of 9*nx*ny elements each, used as ping-pong
 * population stores.  The state is set to rest (rho = 1, u = 0; the paper's
 * default initialisation, Sec. 2.1, Fig. 1's caption).  nx*ny must be below 2^31
 * / 9.  Storage detail: a store holds, for every node, the populations its
 * neighbours pull in the next step, minus the lattice weight w_q (deviation
 * storage keeps FP32 rounding relative to the small non-equilibrium part). */
int lbm_init(lbm_ctx** out, const lbm_config* cfg, const uint8_t* d_mask, float* d_fA,
             float* d_fB, void* stream);

void lbm_destroy(lbm_ctx* ctx);

/* Equilibrium re-initialisation (Sec. 2.1 initialisation block; Sec. 2.3 hand-off
 * of FNO fields to the lattice): f_q(x, 0) = f_eq_q(rho(x), u(x)) (Eq. 1) on every
 * fluid node, then the boundary closures; the step counter restarts at 0.
 * d_rho, d_ux, d_uy: float32 [ny][nx]; values on solid nodes are ignored. */
int lbm_reinit_from_macro(lbm_ctx* ctx, const float* d_rho, const float* d_ux, const float* d_uy);

/* lbm_reinit_from_macro plus the first-order (Chapman-Enskog) non-equilibrium part
 * of the pre-collision populations, f_q = f_eq_q - tau w_q rho / c_s^2
 * (c_q c_q - c_s^2 I) : grad u, so that the hand-off also carries the viscous stress
 * -rho c_s^2 tau (grad u + grad u^T) that f_eq alone drops (Sec. 2.3 hand-off; the
 * stress-free start otherwise relaxes through a transient of a few tau).  grad u by
 * central differences between fluid nodes (one-sided next to solids and open
 * boundaries, zero with no fluid neighbour on an axis); body-force terms are not
 * included.  Same arguments and errors as lbm_reinit_from_macro. */
int lbm_reinit_from_macro_neq(lbm_ctx* ctx, const float* d_rho, const float* d_ux,
                              const float* d_uy);

/* lbm_reinit_from_macro with a mass-conserving hand-off (an extension; the paper
 * re-initialises from f_eq of the predicted fields, Sec. 2.3): rho is shifted by one
 * constant over the fluid nodes so that the new state's fluid mass equals the
 * current state's (the mass the lattice itself conserves with periodic and wall
 * boundaries).  Both sums are FP64 reductions on the device (the current mass as
 * lbm_step reports it), so the call stays asynchronous.  Same arguments and errors
 * as lbm_reinit_from_macro. */
int lbm_reinit_from_macro_mass(lbm_ctx* ctx, const float* d_rho, const float* d_ux,
                               const float* d_uy);

/* Advance n >= 0 steps: each gathers f(t) (streaming Eq. 3 with bounce-back and
 * Zou-He), takes moments (Eqs. 4-5, u = (sum c f + rho g/2)/rho), collides (Eq. 2
 * with the Guo term) and stores the result for the next pull.  With rep == NULL
 * the call is fully asynchronous.  With rep != NULL (then n >= 1) the residual,
 * mass and momentum of the final state are reduced in FP64 on the device, copied
 * back, and the stream is synchronised. */
int lbm_step(lbm_ctx* ctx, int32_t n, lbm_report* rep);

/* Macroscopic fields of the current state f(n) (Eqs. 4-5 with the half-force
 * velocity); solid nodes get (1, 0, 0).  If rho_minus_one != 0, d_rho receives
 * rho - 1 instead of rho (full FP32 resolution of small density deviations). */
int lbm_get_macro(lbm_ctx* ctx, float* d_rho, float* d_ux, float* d_uy, int32_t rho_minus_one);

/* Current pre-collision populations f(n) (after streaming and boundary closures),
 * float32 [9][ny][nx]; solid nodes get the rest weights w_q. */
int lbm_get_populations(lbm_ctx* ctx, float* d_f);

/* Replace the state by the given pre-collision populations f(n) (float32
 * [9][ny][nx], solid entries ignored); the step counter is kept. */
int lbm_set_populations(lbm_ctx* ctx, const float* d_f);

/* Statistics of macroscopic fields over the fluid nodes of ctx's mask. */
typedef struct lbm_field_stats {
    double mass;          /* sum rho (FP64) */
    double max_speed;     /* max |u| */
    int64_t nonfinite;    /* nodes with a NaN or Inf in rho, ux or uy */
    int64_t fluid_nodes;
} lbm_field_stats;

/* Guard for fields about to be handed to the lattice (e.g. an FNO prediction,
 * Sec. 2.3): mass, peak speed and non-finite count of float32 [ny][nx] fields
 * over fluid nodes, reduced on the device in a fixed order (deterministic).
 * Synchronises ctx's stream. */
int lbm_check_fields(lbm_ctx* ctx, const float* d_rho, const float* d_ux, const float* d_uy,
                     lbm_field_stats* out);

/* lbm_check_fields without the wait, for a guard resolved later (the hybrid's
 * speculative cycle, Sec. 2.3): writes mass (sum rho), max |u| and the non-finite
 * node count, as doubles, then 0, to d_stats[0..3] (device memory owned by the
 * caller, 4 doubles), asynchronously on ctx's stream.  Calls on one ctx share its
 * reduction scratch and are ordered by the stream. */
int lbm_check_fields_async(lbm_ctx* ctx, const float* d_rho, const float* d_ux, const float* d_uy,
                           double* d_stats);

/* Distance of macroscopic fields from a reference over the fluid nodes of ctx's
 * mask (the convergence measures of the porous steady-state study, Sec. 3.1):
 * relative L1 norms sum|a - ref| / sum|ref| of rho, ux and uy, and the pressure
 * drop dp = c_s^2 (mean rho on column x = 0 - mean rho on column x = nx - 1) of
 * both sets with its relative error.  A ratio with a zero denominator is 0 when
 * the numerator is 0 and +Inf otherwise; dp is 0 when an end column has no fluid. */
typedef struct lbm_field_error {
    double rel_l1_rho, rel_l1_ux, rel_l1_uy;
    double dp, dp_ref, rel_dp;
} lbm_field_error;

/* Compare float32 [ny][nx] device fields (d_drho = rho - 1, as lbm_get_macro
 * writes with rho_minus_one = 1; velocities in lattice units) with reference
 * fields of the same form.  FP64 sums in a fixed order (deterministic);
 * synchronises ctx's stream. */
int lbm_compare_fields(lbm_ctx* ctx, const float* d_drho, const float* d_ux, const float* d_uy,
                       const float* d_drho_ref, const float* d_ux_ref, const float* d_uy_ref,
                       lbm_field_error* out);

/* Plain device-to-device copy of n float32 values (n a multiple of 4, 16-byte
 * aligned buffers) with 16-byte loads and stores: the achievable-bandwidth
 * reference against which the lattice kernels' traffic and counters are read.
 * Asynchronous on `stream`. */
int lbm_stream_copy(const float* d_src, float* d_dst, size_t n, void* stream);

/* Exact checkpoints: copy the current population store (9*nx*ny float32 in the
 * library's internal pull/deviation layout) out to, or back from, a caller buffer.
 * Restoring a saved store reproduces every later step bit for bit.  The step
 * counter is not touched.  Asynchronous on ctx's stream. */
size_t lbm_state_elems(const lbm_ctx* ctx);
int lbm_save_state(lbm_ctx* ctx, float* d_out);
int lbm_load_state(lbm_ctx* ctx, const float* d_in);

/* The step kernel and arithmetic this context runs: "<shape>/<arith>" with shape
 * node (one node per lane), quad (four nodes per lane), pair-64xR (two steps per
 * launch on 64 x R tiles) or deepS-64xR (S steps per launch on 64 x R tiles) and
 * arith lean, mixed or fp32.  Static string; "" for a NULL ctx. */
const char* lbm_step_kernel(const lbm_ctx* ctx);

/* Number of fluid nodes and the current step counter (host values). */
int lbm_info(const lbm_ctx* ctx, int64_t* fluid_nodes, int64_t* steps_done);

/* ================================================================ adjoint
 *
 * Reverse-mode derivatives of the lattice (the paper's solver is differentiable,
 * Sec. 2.1): a rollout f(0) = Z(f_eq(rho0, u0)), f(n+1) = Z(P C(f(n))), loss
 * L(macros(f(N))), where Z is the Zou-He closure of the boundary columns (identity
 * for periodic and wall boundaries), is differentiated by
 *   lam_N = lbm_macro_vjp(f(N), dL/d macros),
 *   lam_n = lbm_adjoint_step(f(n), lam_{n+1})  for n = N-1 .. 0,
 *   dL/d(rho0, u0) = lbm_feq_vjp(rho0, u0, lam_0),
 * with f(n) recomputed from checkpoints.  All arrays float32 device, populations
 * [9][ny][nx] absolute (as from lbm_get_populations), fields [ny][nx]; solid
 * nodes get zeros.  Every boundary kind of lbm_init is covered. */

/* lam_n = C'(f(n))^T P^T Z'^T lam_{n+1}: Z'^T is the transposed Jacobian of the
 * Zou-He closures (the unknown populations' adjoints move onto the known populations
 * they are formed from), P^T the inverse of the streaming / bounce-back permutation,
 * C' the per-node collision Jacobian (with the Guo term): for BGK
 * (1 - 1/tau) I + (1/tau) J + (1 - 1/(2 tau)) S', for TRT (trt_lambda > 0)
 * I - (P+/tau + P-/tau-)(I - J) + ((1 - 1/(2 tau)) P+ + (1 - 1/(2 tau-)) P-) S', with
 * J = d f_eq / d f, S' the Guo source's derivative without its prefactor and P+-
 * the projections on the parts of a population pair even and odd under c -> -c.
 * d_lam_np1 and d_lam_n must differ.  Asynchronous on ctx's stream. */
int lbm_adjoint_step(lbm_ctx* ctx, const float* d_f_n, const float* d_lam_np1, float* d_lam_n);

/* lam_j = g_rho + g_u . d u / d f_j, d u / d f_j = (c_j - u + g/2) / rho, for
 * upstream gradients (g_rho, g_ux, g_uy) of the macroscopic fields of f. */
int lbm_macro_vjp(lbm_ctx* ctx, const float* d_f_n, const float* d_g_rho, const float* d_g_ux,
                  const float* d_g_uy, float* d_lam);

/* Gradient of the initial fields through f(0) = Z(f_eq(rho, u)) (Eq. 1 and the
 * boundary closures that lbm_init / lbm_reinit_from_macro apply). */
int lbm_feq_vjp(lbm_ctx* ctx, const float* d_rho, const float* d_ux, const float* d_uy,
                const float* d_lam, float* d_g_rho, float* d_g_ux, float* d_g_uy);

/* ================================================================ batches
 *
 * Many independent trajectories of possibly different sizes advanced together:
 * one launch per step covers every trajectory through a flattened tile table
 * (trajectory, tile), and chunks of steps are replayed as a captured hipGraph, so
 * 100 small lattices cost one launch per step instead of 100. */
typedef struct lbm_traj_desc {
    lbm_config cfg;        /* arith must be LBM_ARITH_LEAN; kernel is ignored */
    const uint8_t* d_mask; /* uint8 [ny][nx], copied */
    float* d_fA;           /* caller-owned stores of 9*nx*ny float32 each */
    float* d_fB;
} lbm_traj_desc;

typedef struct lbm_batch lbm_batch;

/* Create contexts for ntraj trajectories (h_desc: host array) on `stream`, then
 * pick the step kernel by measurement: every admissible (one-node / four-wide,
 * cached / non-temporal stores) variant is timed on the batch itself and the
 * fastest kept (autotuner).  With tune_cache != NULL the choice is read from, or
 * appended to, that text file (key: device architecture and batch geometry).
 * Every trajectory is left at rest (rho = 1, u = 0).  Synchronous. */
int lbm_batch_create(lbm_batch** out, const lbm_traj_desc* h_desc, int32_t ntraj,
                     const char* tune_cache, void* stream);

/* Advance every trajectory n steps (asynchronous).  Fails with LBM_EINVAL if a
 * trajectory's context was stepped on its own since the last batch step. */
int lbm_batch_step(lbm_batch* b, int32_t n);

/* Context of trajectory i (owned by the batch; use it for lbm_reinit_from_macro,
 * lbm_get_macro, lbm_get_populations, lbm_check_fields -- not for lbm_step). */
int lbm_batch_context(lbm_batch* b, int32_t i, lbm_ctx** out);

/* Human-readable autotuner decision ("tuned quad+nt 0.1 ms/step", "cached ..."). */
const char* lbm_batch_choice(const lbm_batch* b);

void lbm_batch_destroy(lbm_batch* b);

/* ================================================== Fourier Neural Operator
 *
 * FNO of the paper's Sec. 2.2 (Eq. 6): lift P (pointwise, input channels + two
 * coordinate channels x = w/(W-1), y = h/(H-1) -> width/2 -> width with the layer
 * activation between), L Fourier layers v <- act(W v + b + F^-1(R . F(v))) with
 * no activation after the last one, and a pointwise decoder Q (dec_layers hidden
 * layers of dec_size with the decoder activation, then a linear map to cout).
 * F is the 2-D DFT over the (zero-padded) H' x W' grid truncated to rows
 * k1 in {0..m1-1} U {H'-m1..H'-1} and columns k2 in {0..m2-1}; F^-1 the real
 * inverse (the k2 = 0 column contributes its real part once, the others twice,
 * 1/(H'W') normalisation).  H' = H + padding, W' = W + padding (zeros on the high
 * side, cropped before the decoder).
 *
 * Precision: activations between layers, spectral coefficients, DFT bases,
 * spectral/1x1/decoder weights are bfloat16 (round-to-nearest-even); every
 * contraction accumulates in float32 on MFMA (matrix cores); lift weights,
 * biases and activations functions are float32.
 *
 * Packed parameters (float32, in this order; weights [out][in]):
 *   lift1.w [width/2][cin+2*coords], lift1.b [width/2],
 *   lift2.w [width][width/2], lift2.b [width],
 *   per layer n: r_top [width][width][m1][m2][2], r_bot [width][width][m1][m2][2]
 *                (complex (re, im); r_top applies to k1 = 0..m1-1, r_bot to
 *                k1 = H'-m1..H'-1), conv.w [width][width], conv.b [width],
 *   per decoder layer: w [dec_size][in], b [dec_size], then out.w [cout][in],
 *   out.b [cout]. */
#define FNO_ACT_GELU 0
#define FNO_ACT_RELU 1
#define FNO_ACT_SILU 2
#define FNO_ACT_IDENTITY 3

typedef struct fno_spec {
    int32_t cin, width, layers, m1, m2;
    int32_t dec_layers, dec_size, cout;
    int32_t padding, coords;
    int32_t act, dec_act;
} fno_spec;

typedef struct fno_model fno_model;

/* Number of float32 values in the packed parameter vector of `spec`. */
int fno_param_count(const fno_spec* spec, int64_t* count);

/* Build a model for inputs of H x W points: validates the spec (width <= 64,
 * 1 <= m1 <= H'/2, 1 <= m2 <= W'/2, layers >= 1, ...), converts the host parameter
 * vector h_params (nparams float32, layout above) to the device layouts and
 * builds the DFT bases.  Synchronous. */
int fno_model_create(fno_model** out, const fno_spec* spec, const float* h_params,
                     int64_t nparams, int32_t H, int32_t W);
void fno_model_destroy(fno_model* m);

/* Device workspace bytes fno_forward needs for a batch of B. */
int fno_workspace_size(const fno_model* m, int32_t B, size_t* bytes);

/* out[B][cout][H][W] = FNO(in[B][cin][H][W]) (float32, device).  d_ws: caller-owned
 * device workspace of at least fno_workspace_size bytes (256-byte aligned).
 * Asynchronous on `stream`. */
int fno_forward(const fno_model* m, const float* d_in, float* d_out, int32_t B, void* d_ws,
                size_t ws_bytes, void* stream);

/* fno_forward replayed from a HIP graph: the first call for an (d_in, d_out, B,
 * d_ws) tuple captures the forward's launches on a stream private to the model
 * and instantiates them; later calls with the same tuple only launch that graph
 * on `stream` (one launch instead of 3 L + 2), which is what a batch-1 surrogate
 * step inside a hybrid loop needs.  A call with another tuple re-captures.  The
 * captured graph reads the model's weights through their device pointers, so
 * fno_set_params refreshes also reach it.  Same arguments, results and errors as
 * fno_forward (bitwise equal outputs); the model is not reentrant: calls on one
 * model from several threads must be serialised by the caller. */
int fno_forward_graph(fno_model* m, const float* d_in, float* d_out, int32_t B, void* d_ws,
                      size_t ws_bytes, void* stream);

/* fno_forward for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the workspace is
 * a library-owned static device array of FNO_NOALLOC_SCRATCH_BYTES bytes, one per
 * GPU, held until the process ends, so the call itself allocates nothing (no
 * hipMalloc, hipFree or allocating library routine).  Its device address is looked
 * up once per GPU by the first fno_model_create there.  The caller passes the
 * input and output buffers as for fno_forward; results are bitwise equal to
 * fno_forward's.  LBM_EINVAL when the batch needs more workspace than the array
 * holds (fno_workspace_size(m, B) > FNO_NOALLOC_SCRATCH_BYTES), with the sizes in
 * lbm_last_error().  Every call on one GPU shares that GPU's array and leaves its
 * contents behind: calls that overlap on one GPU (on different streams, or from
 * several threads) race and corrupt each other's results; serialise them, e.g. on
 * one stream.  Asynchronous on `stream`. */
#define FNO_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int fno_forward_noalloc(const fno_model* m, const float* d_in, float* d_out, int32_t B,
                        void* stream);

/* ---------------------------------------------------------------- FNO training
 * Training of the surrogate on lattice-generated samples (Sec. 2.2: FNO models
 * trained by minimising the mean squared error of the predicted fields, AdamW).
 * The gradient is the exact backward pass of the forward composition above with
 * every bfloat16 rounding treated as the identity (straight-through); backward
 * contractions use the same BF16-operand / FP32-accumulation policy, weight
 * gradients are reduced in FP32 partials summed in FP64 in a fixed order
 * (deterministic run to run). */

/* Device workspace bytes fno_forward_train / fno_backward need for a batch of B
 * (activations saved by the forward for the backward, plus backward scratch).
 * LBM_EUNSUPPORTED for more than 32 Fourier layers. */
int fno_train_workspace_size(const fno_model* m, int32_t B, size_t* bytes);

/* fno_forward that also saves, in d_ws, what fno_backward reads.  d_ws (256-byte
 * aligned, >= fno_train_workspace_size bytes) must then be passed unchanged to
 * fno_backward with the same d_in and B.  Asynchronous on `stream`. */
int fno_forward_train(const fno_model* m, const float* d_in, float* d_out, int32_t B,
                      void* d_ws, size_t ws_bytes, void* stream);

/* The latent state v_l that the last fno_forward_train saved in d_ws (same B):
 * layer 0 is the lift's output (after the zero padding), layer l = 1..L the output
 * of Fourier layer l - 1 (after its activation; none after the last), each as the
 * bfloat16 values the forward carried, converted to float32 into d_out
 * [B][width][H'][W'] (H' = H + padding, W' = W + padding).  For inspecting the
 * forward stage by stage (Sec. 2.2, Eq. 6: lift, Fourier layers, decoder).
 * Asynchronous on `stream`. */
int fno_train_latent(const fno_model* m, const void* d_ws, size_t ws_bytes, int32_t B,
                     int32_t layer, float* d_out, void* stream);

/* Gradient of a scalar loss w.r.t. the packed parameters (layout above):
 * d_dout[B][cout][H][W] = dLoss/d out (float32, device); writes every element of
 * d_grad[fno_param_count] (float32, device; overwritten, not accumulated).
 * Uses the activations the last fno_forward_train saved in d_ws (and overwrites
 * its backward scratch).  Asynchronous on `stream`. */
int fno_backward(const fno_model* m, const float* d_in, const float* d_dout, int32_t B,
                 void* d_ws, size_t ws_bytes, float* d_grad, void* stream);

/* Mean squared error of n float32 values: *h_loss = sum e^2 / n with
 * e = out - tgt taken in float32, squares and sum in FP64 (fixed order);
 * d_dout = 2 e / n (float32).  d_ws: device scratch of
 * at least (ceil(n / 256) + 1) * 8 bytes.  Synchronises `stream` (returns the
 * loss on the host). */
int fno_mse(const float* d_out, const float* d_tgt, size_t n, float* d_dout, void* d_ws,
            size_t ws_bytes, double* h_loss, void* stream);

/* Refresh the model's device weights from packed float32 parameters on the device
 * (d_params[fno_param_count]; converted exactly as fno_model_create converts host
 * parameters: bf16 round-to-nearest-even for contraction weights, float32 for lift
 * and biases).  Asynchronous on `stream`; forwards queued later on the same
 * stream see the new weights. */
int fno_set_params(fno_model* m, const float* d_params, void* stream);

/* One AdamW step (decoupled weight decay) over n float32 device values:
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 *   p = p (1 - lr wd) - lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps).
 * step >= 1 counts calls so far including this one.  Asynchronous on `stream`. */
int fno_adamw(float* d_p, const float* d_g, float* d_m, float* d_v, int64_t n, double lr,
              double beta1, double beta2, double eps, double weight_decay, int64_t step,
              void* stream);

#ifdef __cplusplus
}
#endif

#endif /* LBMFNO_H */
