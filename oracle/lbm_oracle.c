/*
 * lbm_oracle.c -- plain FP64 CPU oracle of the D2Q9 BGK lattice Boltzmann step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and the
 * benchmark's CPU-baseline leg load this library; the GPU product path never does.
 * It shares no code, header or table with the HIP implementation.
 *
 * What it computes (the paper's Sec. 2.1, "The Lattice Boltzmann Method"):
 *   - equilibrium f_eq (Eq. 1) on the D2Q9 lattice with c_s^2 = 1/3,
 *   - single-relaxation-time (BGK) collision (Eq. 2; printed with a sign slip,
 *     read here as f* = f - (f - f_eq)/tau so that mass is conserved),
 *   - streaming (Eq. 3) with periodic wrap, halfway bounce-back at obstacle and
 *     wall links, and Zou-He velocity inlet / pressure outlet columns,
 *   - moments rho = sum f, rho*u = sum c f (Eqs. 4-5), with the Guo half-force
 *     velocity u = (sum c f + rho g / 2) / rho when a body force g is present,
 *   - Guo forcing term S_q = (1 - 1/(2 tau)) w_q [3 (c_q - u) + 9 (c_q.u) c_q] . rho g,
 *   - obstacle raster (Sec. 3.1.1, Eq. 8), FP64 residual and mass sums,
 *   - the exact vector-Jacobian product of one step (adjoint), Zou-He closures included.
 *
 * State convention: f(n) is the pre-collision population at integer time n, i.e.
 * after streaming and boundary conditions.  One step maps f(n) -> f(n+1) =
 * BC(Stream(Collide(f(n)))).  Arrays are [q][ny][nx], x fastest, FP64.
 * Solid nodes (mask != 0) are never updated and their populations never read.
 *
 * Everything is written as the plain definition: one node at a time, no blocking,
 * no fusion.  OpenMP parallelises the loop over rows only.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q 9
enum { BC_PERIODIC = 0, BC_WALL = 1, BC_ZOUHE = 2 };

/* D2Q9 velocity set and weights (textbook values; Kruger et al. 2017, ch. 3). */
static const int CX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[Q] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double WQ[Q] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

typedef struct {
    int nx, ny;
    double tau, gx, gy;
    int bc_x, bc_y;
    double u_in, rho_out;
    double lambda;  /* > 0: two-relaxation-time collision with this magic parameter */
} cfg_t;

static size_t at(const cfg_t* c, int q, int j, int i) {
    return ((size_t)q * c->ny + (size_t)j) * c->nx + (size_t)i;
}

int oracle_q(void) { return Q; }

#ifdef _OPENMP
#include <omp.h>
int oracle_threads(void) { return omp_get_max_threads(); }
/* Rows run in parallel only on lattices large enough to pay for a parallel region:
 * on a tiny lattice run for tens of thousands of steps, the per-step fork and join
 * (worse, spinning threads when several such processes share the cores) costs
 * far more than the step.  Each row is independent, so the result is the same. */
#define PAR(nx, ny) ((size_t)(nx) * (size_t)(ny) >= 4096)
#else
int oracle_threads(void) { return 1; }
#endif
void oracle_lattice(int* cx, int* cy, int* opp, double* w) {
    for (int q = 0; q < Q; ++q) { cx[q] = CX[q]; cy[q] = CY[q]; opp[q] = OPP[q]; w[q] = WQ[q]; }
}

/* ---------------------------------------------------------------- obstacles */

/* Offset d reduced to the periodic image in (-n/2, n/2]. */
static int64_t periodic_offset(int64_t d, int64_t n) {
    d %= n;
    if (d < 0) d += n;
    if (d > n / 2) d -= n;
    return d;
}

/* Obstacle mask (Sec. 3.1.1): cell (i,j) is solid iff it lies inside any obstacle,
 * an obstacle being {A dx^2 + B dx dy + C dy^2 <= F, |dx|,|dy| <= R} around (cx,cy),
 * evaluated in exact int64 arithmetic.  shapes: nshapes x 7 int64. */
void oracle_raster(int nx, int ny, int wrap_x, int wrap_y, const int64_t* shapes,
                   int nshapes, uint8_t* mask) {
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            uint8_t solid = 0;
            for (int s = 0; s < nshapes && !solid; ++s) {
                const int64_t* p = shapes + 7 * (size_t)s;
                int64_t dx = (int64_t)i - p[0], dy = (int64_t)j - p[1];
                if (wrap_x) dx = periodic_offset(dx, nx);
                if (wrap_y) dy = periodic_offset(dy, ny);
                if (dx > p[6] || -dx > p[6] || dy > p[6] || -dy > p[6]) continue;
                if (p[2] * dx * dx + p[3] * dx * dy + p[4] * dy * dy <= p[5]) solid = 1;
            }
            mask[(size_t)j * nx + i] = solid;
        }
}

/* --------------------------------------------------------------- local maps */

/* Eq. 1 with c_s^2 = 1/3. */
static void equilibrium(double rho, double ux, double uy, double* feq) {
    const double usq = ux * ux + uy * uy;
    for (int q = 0; q < Q; ++q) {
        const double cu = CX[q] * ux + CY[q] * uy;
        feq[q] = WQ[q] * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
    }
}

void oracle_feq(double rho, double ux, double uy, double* feq) { equilibrium(rho, ux, uy, feq); }

/* Eqs. 4-5 with the Guo half-force velocity. */
static void moments(const double* f, double gx, double gy, double* rho, double* ux, double* uy) {
    double r = 0.0, jx = 0.0, jy = 0.0;
    for (int q = 0; q < Q; ++q) { r += f[q]; jx += CX[q] * f[q]; jy += CY[q] * f[q]; }
    *rho = r;
    *ux = (jx + 0.5 * r * gx) / r;
    *uy = (jy + 0.5 * r * gy) / r;
}

/* BGK collision (Eq. 2, sign-corrected) plus the Guo forcing term.  With
 * c->lambda > 0 the two-relaxation-time (TRT) collision instead (Ginzburg 2005; an
 * extension, the paper uses BGK): the parts of f, f_eq and the Guo source that are
 * even and odd under c -> -c relax with tau+ = tau and with tau- from the magic
 * parameter lambda = (tau+ - 1/2)(tau- - 1/2); the source's parts get the factors
 * (1 - 1/(2 tau+)) and (1 - 1/(2 tau-)).  tau- = tau+ gives back BGK. */
static void collide_node(const double* f, const cfg_t* c, double* fstar) {
    double rho, ux, uy, feq[Q], src[Q];
    moments(f, c->gx, c->gy, &rho, &ux, &uy);
    equilibrium(rho, ux, uy, feq);
    for (int q = 0; q < Q; ++q) {   /* Guo source without its relaxation factor */
        const double cu = CX[q] * ux + CY[q] * uy;
        const double sx = 3.0 * (CX[q] - ux) + 9.0 * cu * CX[q];
        const double sy = 3.0 * (CY[q] - uy) + 9.0 * cu * CY[q];
        src[q] = WQ[q] * (sx * rho * c->gx + sy * rho * c->gy);
    }
    if (c->lambda <= 0.0) {
        const double pref = 1.0 - 1.0 / (2.0 * c->tau);
        for (int q = 0; q < Q; ++q) fstar[q] = f[q] - (f[q] - feq[q]) / c->tau + pref * src[q];
        return;
    }
    const double tau_p = c->tau, tau_m = 0.5 + c->lambda / (c->tau - 0.5);
    for (int q = 0; q < Q; ++q) {
        const int b = OPP[q];
        const double fp = 0.5 * (f[q] + f[b]), fm = 0.5 * (f[q] - f[b]);
        const double ep = 0.5 * (feq[q] + feq[b]), em = 0.5 * (feq[q] - feq[b]);
        const double sp = 0.5 * (src[q] + src[b]), sm = 0.5 * (src[q] - src[b]);
        fstar[q] = f[q] - (fp - ep) / tau_p - (fm - em) / tau_m + (1.0 - 0.5 / tau_p) * sp +
                   (1.0 - 0.5 / tau_m) * sm;
    }
}

/* Zou & He (1997) closures for the three unknown populations of a boundary node. */
static void zouhe_inlet(double* f, double u_in) {
    const double rho = (f[0] + f[2] + f[4] + 2.0 * (f[3] + f[6] + f[7])) / (1.0 - u_in);
    f[1] = f[3] + (2.0 / 3.0) * rho * u_in;
    f[5] = f[7] - 0.5 * (f[2] - f[4]) + (1.0 / 6.0) * rho * u_in;
    f[8] = f[6] + 0.5 * (f[2] - f[4]) + (1.0 / 6.0) * rho * u_in;
}

static void zouhe_outlet(double* f, double rho_out) {
    const double ux = -1.0 + (f[0] + f[2] + f[4] + 2.0 * (f[1] + f[5] + f[8])) / rho_out;
    f[3] = f[1] - (2.0 / 3.0) * rho_out * ux;
    f[6] = f[8] - 0.5 * (f[2] - f[4]) - (1.0 / 6.0) * rho_out * ux;
    f[7] = f[5] + 0.5 * (f[2] - f[4]) - (1.0 / 6.0) * rho_out * ux;
}

/* Source node of the pull x - c_q; returns 0 if it leaves a non-periodic domain. */
static int source(const cfg_t* c, int i, int j, int q, int* si, int* sj) {
    int a = i - CX[q], b = j - CY[q];
    if (a < 0 || a >= c->nx) {
        if (c->bc_x != BC_PERIODIC) return 0;
        a = (a + c->nx) % c->nx;
    }
    if (b < 0 || b >= c->ny) {
        if (c->bc_y != BC_PERIODIC) return 0;
        b = (b + c->ny) % c->ny;
    }
    *si = a; *sj = b;
    return 1;
}

/* Target node of the push y + c_q; returns 0 if it leaves a non-periodic domain. */
static int target(const cfg_t* c, int i, int j, int q, int* ti, int* tj) {
    int a = i + CX[q], b = j + CY[q];
    if (a < 0 || a >= c->nx) {
        if (c->bc_x != BC_PERIODIC) return 0;
        a = (a + c->nx) % c->nx;
    }
    if (b < 0 || b >= c->ny) {
        if (c->bc_y != BC_PERIODIC) return 0;
        b = (b + c->ny) % c->ny;
    }
    *ti = a; *tj = b;
    return 1;
}

static void apply_bc(const cfg_t* c, const uint8_t* mask, double* f) {
    if (c->bc_x != BC_ZOUHE) return;
    for (int j = 0; j < c->ny; ++j) {
        double g[Q];
        if (!mask[(size_t)j * c->nx]) {
            for (int q = 0; q < Q; ++q) g[q] = f[at(c, q, j, 0)];
            zouhe_inlet(g, c->u_in);
            for (int q = 0; q < Q; ++q) f[at(c, q, j, 0)] = g[q];
        }
        const int i = c->nx - 1;
        if (!mask[(size_t)j * c->nx + i]) {
            for (int q = 0; q < Q; ++q) g[q] = f[at(c, q, j, i)];
            zouhe_outlet(g, c->rho_out);
            for (int q = 0; q < Q; ++q) f[at(c, q, j, i)] = g[q];
        }
    }
}

static cfg_t make_cfg(int nx, int ny, double tau, double gx, double gy, int bc_x, int bc_y,
                      double u_in, double rho_out) {
    cfg_t c = {nx, ny, tau, gx, gy, bc_x, bc_y, u_in, rho_out, 0.0};
    return c;
}

/* ------------------------------------------------------------ public steps */

/* f(0) = f_eq(rho0, u0) on fluid nodes, then the boundary closures (so that f(0) is
 * a valid post-boundary state); solids hold the rest weights. */
void oracle_init(int nx, int ny, double tau, double gx, double gy, int bc_x, int bc_y,
                 double u_in, double rho_out, const uint8_t* mask, const double* rho0,
                 const double* ux0, const double* uy0, double* f) {
    cfg_t c = make_cfg(nx, ny, tau, gx, gy, bc_x, bc_y, u_in, rho_out);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const size_t n = (size_t)j * nx + i;
            double feq[Q];
            if (mask[n]) {
                for (int q = 0; q < Q; ++q) f[at(&c, q, j, i)] = WQ[q];
                continue;
            }
            equilibrium(rho0[n], ux0[n], uy0[n], feq);
            for (int q = 0; q < Q; ++q) f[at(&c, q, j, i)] = feq[q];
        }
    apply_bc(&c, mask, f);
}

/* Velocity derivative along one axis at fluid node (i, j): central difference when
 * both neighbours are fluid nodes inside the domain (periodic axes wrap), one-sided
 * when only one is, zero when neither is. */
static double velocity_derivative(const cfg_t* c, const uint8_t* mask, const double* u, int i, int j,
                                  int axis) {
    int ok[2], nb[2];
    for (int s = 0; s < 2; ++s) {
        const int d = s == 0 ? 1 : -1;
        int a = i + (axis == 0 ? d : 0), b = j + (axis == 1 ? d : 0);
        int inside = 1;
        if (a < 0 || a >= c->nx) {
            if (c->bc_x == BC_PERIODIC) a = (a + c->nx) % c->nx; else inside = 0;
        }
        if (b < 0 || b >= c->ny) {
            if (c->bc_y == BC_PERIODIC) b = (b + c->ny) % c->ny; else inside = 0;
        }
        ok[s] = inside && !mask[(size_t)b * c->nx + a];
        nb[s] = inside ? b * c->nx + a : 0;
    }
    const double u0 = u[(size_t)j * c->nx + i];
    if (ok[0] && ok[1]) return 0.5 * (u[nb[0]] - u[nb[1]]);
    if (ok[0]) return u[nb[0]] - u0;
    if (ok[1]) return u0 - u[nb[1]];
    return 0.0;
}

/* f(0) = f_eq(rho0, u0) + f_neq on fluid nodes, then the boundary closures, where
 * f_neq is the first-order (Chapman-Enskog) non-equilibrium part of the
 * pre-collision populations, f_neq_q = -tau w_q rho / c_s^2 (c_q c_q - c_s^2 I) : grad u,
 * with the velocity gradient from velocity_derivative.  Its zeroth and first moments
 * vanish and its second moment is the viscous stress -rho c_s^2 tau (grad u + grad u^T).
 * Body-force contributions to f_neq are not included. */
void oracle_init_neq(int nx, int ny, double tau, double gx, double gy, int bc_x, int bc_y,
                     double u_in, double rho_out, const uint8_t* mask, const double* rho0,
                     const double* ux0, const double* uy0, double* f) {
    cfg_t c = make_cfg(nx, ny, tau, gx, gy, bc_x, bc_y, u_in, rho_out);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const size_t n = (size_t)j * nx + i;
            double feq[Q];
            if (mask[n]) {
                for (int q = 0; q < Q; ++q) f[at(&c, q, j, i)] = WQ[q];
                continue;
            }
            equilibrium(rho0[n], ux0[n], uy0[n], feq);
            const double dxux = velocity_derivative(&c, mask, ux0, i, j, 0);
            const double dyux = velocity_derivative(&c, mask, ux0, i, j, 1);
            const double dxuy = velocity_derivative(&c, mask, uy0, i, j, 0);
            const double dyuy = velocity_derivative(&c, mask, uy0, i, j, 1);
            const double cs2 = 1.0 / 3.0;
            for (int q = 0; q < Q; ++q) {
                const double qxx = CX[q] * CX[q] - cs2, qyy = CY[q] * CY[q] - cs2, qxy = CX[q] * CY[q];
                const double contr = qxx * dxux + qxy * (dyux + dxuy) + qyy * dyuy;
                f[at(&c, q, j, i)] = feq[q] - tau * WQ[q] * rho0[n] / cs2 * contr;
            }
        }
    apply_bc(&c, mask, f);
}

/* Collision on every fluid node: fstar = C(f). */
static void collide_all(const cfg_t* cp, const uint8_t* mask, const double* f, double* fstar) {
    const cfg_t c = *cp;
    const int nx = c.nx, ny = c.ny;
#pragma omp parallel for schedule(static) if (PAR(nx, ny))
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double g[Q], h[Q];
            if (mask[(size_t)j * nx + i]) {
                for (int q = 0; q < Q; ++q) fstar[at(&c, q, j, i)] = f[at(&c, q, j, i)];
                continue;
            }
            for (int q = 0; q < Q; ++q) g[q] = f[at(&c, q, j, i)];
            collide_node(g, &c, h);
            for (int q = 0; q < Q; ++q) fstar[at(&c, q, j, i)] = h[q];
        }
}

void oracle_collide(int nx, int ny, double tau, double gx, double gy, const uint8_t* mask,
                    const double* f, double* fstar) {
    cfg_t c = make_cfg(nx, ny, tau, gx, gy, 0, 0, 0.0, 1.0);
    collide_all(&c, mask, f, fstar);
}

/* TRT collision (collide_node with lambda > 0). */
void oracle_collide_trt(int nx, int ny, double tau, double lambda, double gx, double gy,
                        const uint8_t* mask, const double* f, double* fstar) {
    cfg_t c = make_cfg(nx, ny, tau, gx, gy, 0, 0, 0.0, 1.0);
    c.lambda = lambda;
    collide_all(&c, mask, f, fstar);
}

/* Streaming (Eq. 3) with halfway bounce-back, then the boundary closures. */
void oracle_stream(int nx, int ny, int bc_x, int bc_y, double u_in, double rho_out,
                   const uint8_t* mask, const double* fstar, double* fnew) {
    cfg_t c = make_cfg(nx, ny, 1.0, 0.0, 0.0, bc_x, bc_y, u_in, rho_out);
#pragma omp parallel for schedule(static) if (PAR(nx, ny))
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            if (mask[(size_t)j * nx + i]) {
                for (int q = 0; q < Q; ++q) fnew[at(&c, q, j, i)] = fstar[at(&c, q, j, i)];
                continue;
            }
            for (int q = 0; q < Q; ++q) {
                int si, sj;
                if (source(&c, i, j, q, &si, &sj) && !mask[(size_t)sj * nx + si])
                    fnew[at(&c, q, j, i)] = fstar[at(&c, q, sj, si)];
                else
                    fnew[at(&c, q, j, i)] = fstar[at(&c, OPP[q], j, i)];
            }
        }
    apply_bc(&c, mask, fnew);
}

/* nsteps full steps f(n) -> f(n+nsteps), in place on f. */
int oracle_run(int nx, int ny, double tau, double gx, double gy, int bc_x, int bc_y,
               double u_in, double rho_out, const uint8_t* mask, double* f, int nsteps) {
    const size_t n = (size_t)Q * nx * ny;
    double* tmp = (double*)malloc(n * sizeof(double));
    if (!tmp) return -1;
    for (int s = 0; s < nsteps; ++s) {
        oracle_collide(nx, ny, tau, gx, gy, mask, f, tmp);
        oracle_stream(nx, ny, bc_x, bc_y, u_in, rho_out, mask, tmp, f);
    }
    free(tmp);
    return 0;
}

/* oracle_run with the TRT collision (magic parameter lambda > 0). */
int oracle_run_trt(int nx, int ny, double tau, double lambda, double gx, double gy, int bc_x,
                   int bc_y, double u_in, double rho_out, const uint8_t* mask, double* f, int nsteps) {
    const size_t n = (size_t)Q * nx * ny;
    double* tmp = (double*)malloc(n * sizeof(double));
    if (!tmp) return -1;
    for (int s = 0; s < nsteps; ++s) {
        oracle_collide_trt(nx, ny, tau, lambda, gx, gy, mask, f, tmp);
        oracle_stream(nx, ny, bc_x, bc_y, u_in, rho_out, mask, tmp, f);
    }
    free(tmp);
    return 0;
}

/* Macroscopic fields of f (Eqs. 4-5 with the Guo half-force velocity); solids 1,0,0. */
void oracle_macros(int nx, int ny, double gx, double gy, const uint8_t* mask, const double* f,
                   double* rho, double* ux, double* uy) {
    cfg_t c = make_cfg(nx, ny, 1.0, gx, gy, 0, 0, 0.0, 1.0);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const size_t n = (size_t)j * nx + i;
            if (mask[n]) { rho[n] = 1.0; ux[n] = 0.0; uy[n] = 0.0; continue; }
            double g[Q];
            for (int q = 0; q < Q; ++q) g[q] = f[at(&c, q, j, i)];
            moments(g, gx, gy, rho + n, ux + n, uy + n);
        }
}

/* Neumaier compensated sum over fluid nodes. */
static double fluid_sum(int n, const uint8_t* mask, const double* a, const double* b, int absdiff) {
    double s = 0.0, comp = 0.0;
    for (int k = 0; k < n; ++k) {
        if (mask[k]) continue;
        const double x = absdiff ? fabs(a[k] - b[k]) : a[k];
        const double t = s + x;
        if (fabs(s) >= fabs(x)) comp += (s - t) + x; else comp += (x - t) + s;
        s = t;
    }
    return s + comp;
}

/* Residual r = sum_fluid |rho - rho_prev| / sum_fluid rho, mass = sum_fluid rho,
 * momentum = sum_fluid rho*u (out[0..3] = r, mass, mom_x, mom_y). */
void oracle_sums(int nx, int ny, const uint8_t* mask, const double* rho, const double* rho_prev,
                 const double* ux, const double* uy, double* out) {
    const int n = nx * ny;
    double* t = (double*)malloc(2 * (size_t)n * sizeof(double));
    for (int k = 0; k < n; ++k) { t[k] = rho[k] * ux[k]; t[n + k] = rho[k] * uy[k]; }
    const double mass = fluid_sum(n, mask, rho, NULL, 0);
    out[0] = rho_prev ? fluid_sum(n, mask, rho, rho_prev, 1) / mass : 0.0;
    out[1] = mass;
    out[2] = fluid_sum(n, mask, t, NULL, 0);
    out[3] = fluid_sum(n, mask, t + n, NULL, 0);
    free(t);
}

/* ---------------------------------------------------------------- adjoint */

/* Jacobians of the Zou-He closures (zouhe_inlet / zouhe_outlet above) with respect
 * to the node's populations after streaming: identity rows for the known
 * populations, the closure's derivative for the three unknown ones. */
static void zouhe_inlet_jacobian(double u_in, double J[Q][Q]) {
    double drho[Q] = {1.0, 0.0, 1.0, 2.0, 1.0, 0.0, 2.0, 2.0, 0.0};  /* d rho / d f_q */
    for (int q = 0; q < Q; ++q) drho[q] /= 1.0 - u_in;
    for (int a = 0; a < Q; ++a)
        for (int b = 0; b < Q; ++b) J[a][b] = a == b ? 1.0 : 0.0;
    for (int b = 0; b < Q; ++b) {
        J[1][b] = (2.0 / 3.0) * u_in * drho[b];
        J[5][b] = (1.0 / 6.0) * u_in * drho[b];
        J[8][b] = (1.0 / 6.0) * u_in * drho[b];
    }
    J[1][3] += 1.0;                                   /* f1 = f3 + 2/3 rho u_in */
    J[5][7] += 1.0; J[5][2] -= 0.5; J[5][4] += 0.5;   /* f5 = f7 - (f2 - f4)/2 + rho u_in/6 */
    J[8][6] += 1.0; J[8][2] += 0.5; J[8][4] -= 0.5;   /* f8 = f6 + (f2 - f4)/2 + rho u_in/6 */
}

static void zouhe_outlet_jacobian(double rho_out, double J[Q][Q]) {
    double dux[Q] = {1.0, 2.0, 1.0, 0.0, 1.0, 2.0, 0.0, 0.0, 2.0};  /* d u_x / d f_q */
    for (int q = 0; q < Q; ++q) dux[q] /= rho_out;
    for (int a = 0; a < Q; ++a)
        for (int b = 0; b < Q; ++b) J[a][b] = a == b ? 1.0 : 0.0;
    for (int b = 0; b < Q; ++b) {
        J[3][b] = -(2.0 / 3.0) * rho_out * dux[b];
        J[6][b] = -(1.0 / 6.0) * rho_out * dux[b];
        J[7][b] = -(1.0 / 6.0) * rho_out * dux[b];
    }
    J[3][1] += 1.0;                                   /* f3 = f1 - 2/3 rho_out u_x */
    J[6][8] += 1.0; J[6][2] -= 0.5; J[6][4] += 0.5;   /* f6 = f8 - (f2 - f4)/2 - rho_out u_x/6 */
    J[7][5] += 1.0; J[7][2] += 0.5; J[7][4] -= 0.5;   /* f7 = f5 + (f2 - f4)/2 - rho_out u_x/6 */
}

/* lam <- Z'^T lam in place: the transpose of the boundary closures' Jacobian at the
 * fluid nodes of the Zou-He columns (identity elsewhere and for other boundaries). */
void oracle_bc_vjp(int nx, int ny, int bc_x, double u_in, double rho_out, const uint8_t* mask,
                   double* lam) {
    if (bc_x != BC_ZOUHE) return;
    cfg_t c = make_cfg(nx, ny, 1.0, 0.0, 0.0, bc_x, 0, u_in, rho_out);
    double Jin[Q][Q], Jout[Q][Q];
    zouhe_inlet_jacobian(u_in, Jin);
    zouhe_outlet_jacobian(rho_out, Jout);
    for (int j = 0; j < ny; ++j)
        for (int side = 0; side < 2; ++side) {
            const int i = side == 0 ? 0 : nx - 1;
            if (mask[(size_t)j * nx + i]) continue;
            double (*J)[Q] = side == 0 ? Jin : Jout;
            double l[Q], nu[Q];
            for (int q = 0; q < Q; ++q) l[q] = lam[at(&c, q, j, i)];
            for (int b = 0; b < Q; ++b) {
                nu[b] = 0.0;
                for (int a = 0; a < Q; ++a) nu[b] += J[a][b] * l[a];
            }
            for (int q = 0; q < Q; ++q) lam[at(&c, q, j, i)] = nu[q];
        }
}

/* Vector-Jacobian product of one step f(n+1) = Z(P C(f(n))): given the pre-collision
 * state f(n) and lam_np1 = dL/df(n+1), returns lam_n = dL/df(n) =
 * C'(f(n))^T P^T Z'^T lam_np1, where Z is the Zou-He closure of the boundary columns
 * (identity for periodic and wall boundaries), P the streaming / bounce-back
 * permutation and C' the per-node collision Jacobian. */
static int adjoint_step(int nx, int ny, double tau, double lambda, double gx, double gy, int bc_x,
                        int bc_y, double u_in, double rho_out, const uint8_t* mask, const double* f,
                        const double* lam_in, double* lam_n) {
    if (bc_y == BC_ZOUHE) return -1;
    cfg_t c = make_cfg(nx, ny, tau, gx, gy, bc_x, bc_y, u_in, rho_out);
    const size_t total = (size_t)Q * nx * ny;
    double* lam_np1 = (double*)malloc(total * sizeof(double));
    if (!lam_np1) return -2;
    memcpy(lam_np1, lam_in, total * sizeof(double));
    oracle_bc_vjp(nx, ny, bc_x, u_in, rho_out, mask, lam_np1);
    const double om = 1.0 / tau;
    const double pref = 1.0 - 0.5 * om;
#pragma omp parallel for schedule(static) if (PAR(nx, ny))
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            if (mask[(size_t)j * nx + i]) {
                for (int q = 0; q < Q; ++q) lam_n[at(&c, q, j, i)] = 0.0;
                continue;
            }
            /* mu = P^T lam: the slot fstar_q(y) is read by y + c_q when that node is
             * fluid and inside the domain, otherwise it bounced back into y as q-bar. */
            double mu[Q], g[Q];
            for (int q = 0; q < Q; ++q) {
                int ti, tj;
                if (target(&c, i, j, q, &ti, &tj) && !mask[(size_t)tj * nx + ti])
                    mu[q] = lam_np1[at(&c, q, tj, ti)];
                else
                    mu[q] = lam_np1[at(&c, OPP[q], j, i)];
            }
            for (int q = 0; q < Q; ++q) g[q] = f[at(&c, q, j, i)];
            double rho, ux, uy;
            moments(g, gx, gy, &rho, &ux, &uy);
            const double usq = ux * ux + uy * uy;
            const double gdotu = gx * ux + gy * uy;
            double a = 0.0, bx = 0.0, by = 0.0;
            for (int q = 0; q < Q; ++q) {
                const double cu = CX[q] * ux + CY[q] * uy;
                const double cg = CX[q] * gx + CY[q] * gy;
                /* d f_eq_q / d rho and d f_eq_q / d u */
                const double dfe_dr = WQ[q] * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
                const double dfe_dux = WQ[q] * rho * (3.0 * CX[q] + 9.0 * cu * CX[q] - 3.0 * ux);
                const double dfe_duy = WQ[q] * rho * (3.0 * CY[q] + 9.0 * cu * CY[q] - 3.0 * uy);
                /* d S_q / d rho and d S_q / d u for S_q = pref w_q rho [3 (c.g - u.g) + 9 (c.u)(c.g)] */
                const double dS_dr = pref * WQ[q] * (3.0 * (cg - gdotu) + 9.0 * cu * cg);
                const double dS_dux = pref * WQ[q] * rho * (-3.0 * gx + 9.0 * CX[q] * cg);
                const double dS_duy = pref * WQ[q] * rho * (-3.0 * gy + 9.0 * CY[q] * cg);
                a += mu[q] * (om * dfe_dr + dS_dr);
                bx += mu[q] * (om * dfe_dux + dS_dux);
                by += mu[q] * (om * dfe_duy + dS_duy);
            }
            double diag[Q];
            for (int q = 0; q < Q; ++q) diag[q] = (1.0 - om) * mu[q];
            if (lambda > 0.0) {
                /* TRT: C = I - (w+ P+ + w- P-)(I - J) + (p+ P+ + p- P-) S', with P+- the
                 * projections on the parts of a population pair even and odd under
                 * c -> -c (symmetric), J = d f_eq / d f, S' = d S / d f without the
                 * relaxation prefactor and p+- = 1 - w+-/2.  So C^T mu = mu - nu +
                 * J^T nu + S'^T sg with nu = w+ mu+ + w- mu- and sg = p+ mu+ + p- mu-. */
                const double tau_m = 0.5 + lambda / (tau - 0.5);
                const double om_m = 1.0 / tau_m, pref_m = 1.0 - 0.5 * om_m;
                a = bx = by = 0.0;
                for (int q = 0; q < Q; ++q) {
                    const double even = 0.5 * (mu[q] + mu[OPP[q]]), odd = 0.5 * (mu[q] - mu[OPP[q]]);
                    const double nu = om * even + om_m * odd, sg = pref * even + pref_m * odd;
                    const double cu = CX[q] * ux + CY[q] * uy;
                    const double cg = CX[q] * gx + CY[q] * gy;
                    const double dfe_dr = WQ[q] * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
                    const double dfe_dux = WQ[q] * rho * (3.0 * CX[q] + 9.0 * cu * CX[q] - 3.0 * ux);
                    const double dfe_duy = WQ[q] * rho * (3.0 * CY[q] + 9.0 * cu * CY[q] - 3.0 * uy);
                    const double ds_dr = WQ[q] * (3.0 * (cg - gdotu) + 9.0 * cu * cg);
                    const double ds_dux = WQ[q] * rho * (-3.0 * gx + 9.0 * CX[q] * cg);
                    const double ds_duy = WQ[q] * rho * (-3.0 * gy + 9.0 * CY[q] * cg);
                    a += nu * dfe_dr + sg * ds_dr;
                    bx += nu * dfe_dux + sg * ds_dux;
                    by += nu * dfe_duy + sg * ds_duy;
                    diag[q] = mu[q] - nu;
                }
            }
            /* u = (sum c f)/rho + g/2, so du/df_j = (c_j - u + g/2)/rho. */
            for (int q = 0; q < Q; ++q) {
                const double dux = (CX[q] - ux + 0.5 * gx) / rho;
                const double duy = (CY[q] - uy + 0.5 * gy) / rho;
                lam_n[at(&c, q, j, i)] = diag[q] + a + bx * dux + by * duy;
            }
        }
    free(lam_np1);
    return 0;
}

int oracle_adjoint_step(int nx, int ny, double tau, double gx, double gy, int bc_x, int bc_y,
                        double u_in, double rho_out, const uint8_t* mask, const double* f,
                        const double* lam_in, double* lam_n) {
    return adjoint_step(nx, ny, tau, 0.0, gx, gy, bc_x, bc_y, u_in, rho_out, mask, f, lam_in, lam_n);
}

/* oracle_adjoint_step of the TRT step (magic parameter lambda > 0). */
int oracle_adjoint_step_trt(int nx, int ny, double tau, double lambda, double gx, double gy, int bc_x,
                            int bc_y, double u_in, double rho_out, const uint8_t* mask, const double* f,
                            const double* lam_in, double* lam_n) {
    if (!(lambda > 0.0)) return -1;
    return adjoint_step(nx, ny, tau, lambda, gx, gy, bc_x, bc_y, u_in, rho_out, mask, f, lam_in, lam_n);
}

/* Pull back dL/df(0) through f(0) = f_eq(rho0, u0): per node
 * dL/drho0 = sum_q lam_q d f_eq_q/d rho, dL/du0 = sum_q lam_q d f_eq_q/d u. */
void oracle_feq_vjp(int nx, int ny, const uint8_t* mask, const double* rho0, const double* ux0,
                    const double* uy0, const double* lam, double* g_rho, double* g_ux, double* g_uy) {
    cfg_t c = make_cfg(nx, ny, 1.0, 0.0, 0.0, 0, 0, 0.0, 1.0);
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const size_t n = (size_t)j * nx + i;
            if (mask[n]) { g_rho[n] = 0.0; g_ux[n] = 0.0; g_uy[n] = 0.0; continue; }
            const double rho = rho0[n], ux = ux0[n], uy = uy0[n];
            const double usq = ux * ux + uy * uy;
            double gr = 0.0, gx = 0.0, gy = 0.0;
            for (int q = 0; q < Q; ++q) {
                const double cu = CX[q] * ux + CY[q] * uy;
                const double l = lam[at(&c, q, j, i)];
                gr += l * WQ[q] * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
                gx += l * WQ[q] * rho * (3.0 * CX[q] + 9.0 * cu * CX[q] - 3.0 * ux);
                gy += l * WQ[q] * rho * (3.0 * CY[q] + 9.0 * cu * CY[q] - 3.0 * uy);
            }
            g_rho[n] = gr; g_ux[n] = gx; g_uy[n] = gy;
        }
}
