"""Python face of the FP64 lattice Boltzmann oracle (test infrastructure only).

Thin ctypes calls into oracle/liboracle.so (lbm_oracle.c) plus the loss and the
checkpoint-free adjoint driver used by the gradient tests.  Only tests/, the
package smoke check and the benchmark's CPU-baseline leg import this module.
Arrays are float64 [q][ny][nx] (populations) or [ny][nx] (fields); the mask is
uint8 [ny][nx] with 1 = solid.
"""
from __future__ import annotations

import ctypes
import os

import math

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_d = ctypes.c_double
_i = ctypes.c_int
_p = ctypes.c_void_p


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from oracle import build as _b
            _b.build()
        L = ctypes.CDLL(path)
        L.oracle_raster.argtypes = [_i, _i, _i, _i, _p, _i, _p]
        L.oracle_feq.argtypes = [_d, _d, _d, _p]
        L.oracle_init.argtypes = [_i, _i, _d, _d, _d, _i, _i, _d, _d, _p, _p, _p, _p, _p]
        L.oracle_init_neq.argtypes = [_i, _i, _d, _d, _d, _i, _i, _d, _d, _p, _p, _p, _p, _p]
        L.oracle_collide.argtypes = [_i, _i, _d, _d, _d, _p, _p, _p]
        L.oracle_stream.argtypes = [_i, _i, _i, _i, _d, _d, _p, _p, _p]
        L.oracle_run.argtypes = [_i, _i, _d, _d, _d, _i, _i, _d, _d, _p, _p, _i]
        L.oracle_run.restype = _i
        L.oracle_collide_trt.argtypes = [_i, _i, _d, _d, _d, _d, _p, _p, _p]
        L.oracle_run_trt.argtypes = [_i, _i, _d, _d, _d, _d, _i, _i, _d, _d, _p, _p, _i]
        L.oracle_run_trt.restype = _i
        L.oracle_macros.argtypes = [_i, _i, _d, _d, _p, _p, _p, _p, _p]
        L.oracle_sums.argtypes = [_i, _i, _p, _p, _p, _p, _p, _p]
        L.oracle_adjoint_step.argtypes = [_i, _i, _d, _d, _d, _i, _i, _d, _d, _p, _p, _p, _p]
        L.oracle_adjoint_step.restype = _i
        L.oracle_adjoint_step_trt.argtypes = [_i, _i, _d, _d, _d, _d, _i, _i, _d, _d, _p, _p, _p, _p]
        L.oracle_adjoint_step_trt.restype = _i
        L.oracle_bc_vjp.argtypes = [_i, _i, _i, _d, _d, _p, _p]
        L.oracle_bc_vjp.restype = None
        L.oracle_feq_vjp.argtypes = [_i, _i, _p, _p, _p, _p, _p, _p, _p, _p]
        L.oracle_lattice.argtypes = [_p, _p, _p, _p]
        L.oracle_threads.restype = _i
        _LIB = L
    return _LIB


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().oracle_threads())


def lattice():
    """(cx, cy, opp, w) of the oracle's D2Q9 set."""
    cx = np.zeros(9, np.int32); cy = np.zeros(9, np.int32); op = np.zeros(9, np.int32)
    w = np.zeros(9, np.float64)
    lib().oracle_lattice(_ptr(cx), _ptr(cy), _ptr(op), _ptr(w))
    return cx, cy, op, w


def raster(nx: int, ny: int, shapes: np.ndarray, wrap_x: bool, wrap_y: bool) -> np.ndarray:
    shapes = np.ascontiguousarray(shapes, dtype=np.int64).reshape(-1, 7)
    mask = np.zeros((ny, nx), dtype=np.uint8)
    lib().oracle_raster(nx, ny, int(wrap_x), int(wrap_y), _ptr(shapes), shapes.shape[0], _ptr(mask))
    return mask


def feq(rho: float, ux: float, uy: float) -> np.ndarray:
    out = np.zeros(9)
    lib().oracle_feq(rho, ux, uy, _ptr(out))
    return out


class Sim:
    """FP64 lattice state f(n) (pre-collision, after boundary closures)."""

    def __init__(self, lat, mask: np.ndarray | None = None):
        self.lat = lat
        self.nx, self.ny = lat.nx, lat.ny
        if mask is None:
            mask = raster(lat.nx, lat.ny, lat.shapes_array(), lat.wrap_x, lat.wrap_y)
        self.mask = np.ascontiguousarray(mask, dtype=np.uint8)
        self.f = np.zeros((9, self.ny, self.nx))
        self.steps = 0

    def _args(self):
        L = self.lat
        return (self.nx, self.ny, L.tau, L.gx, L.gy, L.bc_x, L.bc_y, L.u_in, L.rho_out)

    def init(self, rho=None, ux=None, uy=None, neq: bool = False, mass=None):
        """f(0) = f_eq(rho, u) (+ the first-order non-equilibrium part with neq), then
        the boundary closures.  With `mass`, rho is first shifted by one constant over
        the fluid nodes so that its fluid sum equals `mass` (a mass-conserving hand-off:
        pass the current state's mass())."""
        shp = (self.ny, self.nx)
        rho = _f64(np.ones(shp) if rho is None else rho)
        if mass is not None:
            fl = self.mask == 0
            nfl = int(fl.sum())
            if nfl:
                rho = rho + (float(mass) - math.fsum(rho[fl].tolist())) / nfl
        ux = _f64(np.zeros(shp) if ux is None else ux)
        uy = _f64(np.zeros(shp) if uy is None else uy)
        self.f = np.zeros((9, self.ny, self.nx))
        fn = lib().oracle_init_neq if neq else lib().oracle_init
        fn(*self._args(), _ptr(self.mask), _ptr(rho), _ptr(ux), _ptr(uy), _ptr(self.f))
        self.steps = 0
        return self

    def mass(self) -> float:
        """Sum of rho = sum_q f_q over the fluid nodes of the current state (fsum)."""
        rho = self.f.sum(axis=0)
        return math.fsum(rho[self.mask == 0].tolist())

    def run(self, n: int):
        lam = getattr(self.lat, "trt_lambda", 0.0)
        if lam > 0.0:
            L = self.lat
            rc = lib().oracle_run_trt(self.nx, self.ny, L.tau, lam, L.gx, L.gy, L.bc_x, L.bc_y, L.u_in,
                                      L.rho_out, _ptr(self.mask), _ptr(self.f), int(n))
        else:
            rc = lib().oracle_run(*self._args(), _ptr(self.mask), _ptr(self.f), int(n))
        if rc != 0:
            raise MemoryError("oracle_run")
        self.steps += n
        return self

    def macros(self):
        rho = np.zeros((self.ny, self.nx)); ux = np.zeros_like(rho); uy = np.zeros_like(rho)
        lib().oracle_macros(self.nx, self.ny, self.lat.gx, self.lat.gy, _ptr(self.mask),
                            _ptr(self.f), _ptr(rho), _ptr(ux), _ptr(uy))
        return rho, ux, uy


def collide(lat, mask, f):
    """BGK collision, or TRT when lat.trt_lambda > 0."""
    f = _f64(f); out = np.zeros_like(f)
    lam = getattr(lat, "trt_lambda", 0.0)
    if lam > 0.0:
        lib().oracle_collide_trt(lat.nx, lat.ny, lat.tau, lam, lat.gx, lat.gy, _ptr(mask), _ptr(f),
                                 _ptr(out))
    else:
        lib().oracle_collide(lat.nx, lat.ny, lat.tau, lat.gx, lat.gy, _ptr(mask), _ptr(f), _ptr(out))
    return out


def stream(lat, mask, fstar):
    fstar = _f64(fstar); out = np.zeros_like(fstar)
    lib().oracle_stream(lat.nx, lat.ny, lat.bc_x, lat.bc_y, lat.u_in, lat.rho_out, _ptr(mask),
                        _ptr(fstar), _ptr(out))
    return out


def macros(lat, mask, f):
    ny, nx = mask.shape
    f = _f64(f)
    rho = np.zeros((ny, nx)); ux = np.zeros_like(rho); uy = np.zeros_like(rho)
    lib().oracle_macros(nx, ny, lat.gx, lat.gy, _ptr(mask), _ptr(f), _ptr(rho), _ptr(ux), _ptr(uy))
    return rho, ux, uy


def sums(mask, rho, rho_prev, ux, uy):
    """(residual, mass, mom_x, mom_y) over fluid nodes (compensated FP64 sums)."""
    ny, nx = mask.shape
    out = np.zeros(4)
    rp = _f64(rho_prev) if rho_prev is not None else None
    lib().oracle_sums(nx, ny, _ptr(mask), _ptr(_f64(rho)), _ptr(rp) if rp is not None else None,
                      _ptr(_f64(ux)), _ptr(_f64(uy)), _ptr(out))
    return tuple(out)


def adjoint_step(lat, mask, f_n, lam_np1):
    """lam_n = C'(f(n))^T P^T Z'^T lam_{n+1} (Z: Zou-He closures, identity otherwise);
    C is the TRT collision when lat.trt_lambda > 0, else BGK."""
    f_n = _f64(f_n); lam_np1 = _f64(lam_np1); out = np.zeros_like(f_n)
    lam = float(getattr(lat, "trt_lambda", 0.0))
    if lam > 0.0:
        rc = lib().oracle_adjoint_step_trt(lat.nx, lat.ny, lat.tau, lam, lat.gx, lat.gy, lat.bc_x,
                                           lat.bc_y, lat.u_in, lat.rho_out, _ptr(mask), _ptr(f_n),
                                           _ptr(lam_np1), _ptr(out))
    else:
        rc = lib().oracle_adjoint_step(lat.nx, lat.ny, lat.tau, lat.gx, lat.gy, lat.bc_x, lat.bc_y,
                                       lat.u_in, lat.rho_out, _ptr(mask), _ptr(f_n), _ptr(lam_np1),
                                       _ptr(out))
    if rc != 0:
        raise ValueError("adjoint not defined for this boundary configuration")
    return out


def bc_vjp(lat, mask, lam):
    """Z'^T lam: the transposed Jacobian of the boundary closures (Zou-He columns)."""
    out = _f64(lam).copy()
    lib().oracle_bc_vjp(lat.nx, lat.ny, lat.bc_x, lat.u_in, lat.rho_out, _ptr(mask), _ptr(out))
    return out


def feq_vjp(mask, rho0, ux0, uy0, lam):
    ny, nx = mask.shape
    g = [np.zeros((ny, nx)) for _ in range(3)]
    lib().oracle_feq_vjp(nx, ny, _ptr(mask), _ptr(_f64(rho0)), _ptr(_f64(ux0)), _ptr(_f64(uy0)),
                         _ptr(_f64(lam)), _ptr(g[0]), _ptr(g[1]), _ptr(g[2]))
    return tuple(g)


# ----------------------------------------------------------- loss and adjoint

def macro_mse(mask, rho, ux, uy, target):
    """Mean squared error of (rho, ux, uy) against target fields over fluid nodes."""
    fl = mask == 0
    n = 3.0 * fl.sum()
    return float((((rho - target[0]) ** 2 + (ux - target[1]) ** 2 + (uy - target[2]) ** 2)[fl]).sum() / n)


def macro_mse_grad_f(lat, mask, f, target):
    """dL/df for L = macro_mse(macros(f)): through rho = sum f and
    u = (sum c f)/rho + g/2, i.e. du/df_j = (c_j - u + g/2)/rho."""
    cx, cy, _, _ = lattice()
    rho, ux, uy = macros(lat, mask, f)
    fl = (mask == 0)
    n = 3.0 * fl.sum()
    dr = 2.0 * (rho - target[0]) / n
    dx = 2.0 * (ux - target[1]) / n
    dy = 2.0 * (uy - target[2]) / n
    out = np.zeros_like(f)
    for q in range(9):
        out[q] = dr + dx * (cx[q] - ux + 0.5 * lat.gx) / rho + dy * (cy[q] - uy + 0.5 * lat.gy) / rho
    out[:, ~fl] = 0.0
    return out


def rollout_loss(lat, mask, rho0, ux0, uy0, nsteps, target):
    """L(rho0, u0) = MSE(macros(f(n)), target) with f(0) = f_eq(rho0, u0)."""
    s = Sim(lat, mask).init(rho0, ux0, uy0).run(nsteps)
    return macro_mse(mask, *s.macros(), target)


def rollout_grad(lat, mask, rho0, ux0, uy0, nsteps, target):
    """Gradient of rollout_loss w.r.t. (rho0, ux0, uy0) by the step adjoint, storing
    every state (the plain form; no checkpointing)."""
    s = Sim(lat, mask).init(rho0, ux0, uy0)
    states = [s.f.copy()]
    for _ in range(nsteps):
        s.run(1)
        states.append(s.f.copy())
    lam = macro_mse_grad_f(lat, mask, states[-1], target)
    for n in range(nsteps - 1, -1, -1):
        lam = adjoint_step(lat, mask, states[n], lam)
    # f(0) = Z(f_eq(rho0, u0)): through the closures, then the equilibrium
    return feq_vjp(mask, rho0, ux0, uy0, bc_vjp(lat, mask, lam))
