"""Hybrid FNO-LBM orchestration (the paper's Sec. 2.3).

Steady problems: the FNO predicts macroscopic fields once, the lattice is
re-initialised from them (f = f_eq(rho, u)) and plain lattice steps run until the
density residual falls below a tolerance.

Unsteady problems ("super-time-stepping"): cycles of K FNO calls, each advancing
the model time by dt_fno lattice steps with its output fed back as the next input,
then an equilibrium re-initialisation and n_lbm lattice steps.  A fixed temporal
switch, as in the paper (the paper's 1:k hybrids are K = 1, n_lbm = k * dt_fno).

Every FNO prediction passes a guard before it reaches the lattice -- finite values,
peak speed below a Mach limit, mass within a tolerance of the lattice's -- and a
rejected prediction is replaced by the equivalent K * dt_fno plain lattice steps
(plain LBM as fallback and judge).  All device work runs in liblbmfno kernels on
the lattice's stream.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import List, Optional


def step_reduction(k_fno: int, dt_fno: int, n_lbm: int) -> float:
    """Share of the horizon's lattice steps that the FNO replaces:
    eps_N = K dt_fno / (K dt_fno + n_lbm) (the paper's Table 'hybrid speedup',
    eps_N = (N_LBM - N_hybrid) / N_LBM)."""
    return k_fno * dt_fno / float(k_fno * dt_fno + n_lbm)


def runtime_reduction(t_lbm: float, t_hybrid: float) -> float:
    """eps_T = (T_LBM - T_hybrid) / T_LBM."""
    return (t_lbm - t_hybrid) / t_lbm


def error_reduction(e_fno: float, e_hybrid: float) -> float:
    """(e_FNO - e_hybrid) / e_FNO (the paper's error-reduction table)."""
    return (e_fno - e_hybrid) / e_fno


def convergence_speedup(n_lbm: float, n_init: float) -> float:
    """(N_LBM - N_FNO-init) / N_LBM (the paper's steady convergence table)."""
    return (n_lbm - n_init) / n_lbm


@dataclass
class Guard:
    max_speed: float = 0.3          # lattice Mach-number guard (|u| / c_s ~ 0.52)
    mass_rel_tol: float = 0.05      # |mass(pred) - mass(lattice)| / mass(lattice)

    def accept(self, stats: dict, ref_mass: float) -> tuple:
        if stats["nonfinite"] > 0:
            return False, f"{stats['nonfinite']} non-finite nodes"
        if stats["max_speed"] > self.max_speed:
            return False, f"peak speed {stats['max_speed']:.3g} > {self.max_speed}"
        if abs(stats["mass"] - ref_mass) > self.mass_rel_tol * abs(ref_mass):
            return False, f"mass {stats['mass']:.6g} vs lattice {ref_mass:.6g}"
        return True, ""


@dataclass
class CycleLog:
    fno_calls: int = 0
    lbm_steps: int = 0
    fallbacks: List[str] = field(default_factory=list)


class HybridRunner:
    """Unsteady super-time-stepping on one lattice with one FNO bound to its grid.

    lattice: lbmfno.Lattice (nx = W, ny = H of the FNO); fno: fno.Fno with cin = 4
    inputs (rho, ux, uy, mask) and cout = 3 outputs (rho, ux, uy).

    speculative=True takes the guard off the host's critical path: a cycle hands the
    prediction to the lattice at once, after saving the lattice state and queueing
    the guard's statistics into pinned host memory behind the FNO calls; the guard is
    resolved at the start of the next cycle (or by finish()), when those statistics
    have long been ready, and a rejected cycle is undone (state restored) and redone
    with lattice steps.  The states and the log equal those of the synchronous guard;
    the host no longer waits for the GPU twice per cycle."""

    def __init__(self, lattice, fno, dt_fno: int = 100, k_fno: int = 5, n_lbm: int = 200,
                 guard: Optional[Guard] = None, speculative: bool = False, graph: bool = False):
        import torch
        if fno.spec.cin != 4 or fno.spec.cout != 3:
            raise ValueError("the hybrid FNO maps (rho, ux, uy, mask) -> (rho, ux, uy)")
        if (fno.H, fno.W) != (lattice.ny, lattice.nx):
            raise ValueError("FNO grid must match the lattice")
        self.lat, self.fno = lattice, fno
        self.dt_fno, self.k_fno, self.n_lbm = int(dt_fno), int(k_fno), int(n_lbm)
        self.guard = guard or Guard()
        # graph=True replays the FNO's launches from a captured HIP graph; on MI355X
        # that is no faster than launching them (a few microseconds slower)
        self.graph = bool(graph)
        with torch.cuda.stream(lattice.stream):
            self.x = torch.empty((1, 4, lattice.ny, lattice.nx), dtype=torch.float32, device="cuda")
            self.y = torch.empty((1, 3, lattice.ny, lattice.nx), dtype=torch.float32, device="cuda")
            self.maskf = lattice.mask.to(torch.float32)
            self.x[0, 3].copy_(self.maskf)   # the mask channel never changes
        self.model_time = 0          # lattice-step units advanced so far
        self.log = CycleLog()
        self.speculative = bool(speculative)
        self._pending = None         # model time of a cycle whose guard is unresolved
        if self.speculative:
            with torch.cuda.stream(lattice.stream):
                self._saved = torch.empty(int(lattice.lib.lbm_state_elems(lattice.ctx)),
                                          dtype=torch.float32, device="cuda")
                self._dstats = torch.empty(8, dtype=torch.float64, device="cuda")
            self._hstats = torch.empty(8, dtype=torch.float64, pin_memory=True)
            self._ready = torch.cuda.Event()

    def _fno_rollout(self, macros):
        """K chained FNO calls from the lattice's current macroscopic fields."""
        import torch
        with torch.cuda.stream(self.lat.stream):
            if macros.data_ptr() != self.x.data_ptr():
                self.x[0, :3].copy_(macros)
            for k in range(self.k_fno):
                self.fno.forward(self.x, out=self.y, stream=self.lat.stream, graph=self.graph)
                if k + 1 < self.k_fno:
                    self.x[0, :3].copy_(self.y[0])
        return self.y[0]

    def cycle(self):
        """One cycle: K FNO calls (guarded), re-initialisation, n_lbm lattice steps,
        all issued on the lattice's stream (no cross-stream waits inside a cycle)."""
        import torch
        with torch.cuda.stream(self.lat.stream):
            self._cycle()

    def _cycle(self):
        if self.speculative:
            self._cycle_speculative()
            return
        macros = self.lat.macros()
        ref = self.lat.check_fields(macros[0], macros[1], macros[2])
        pred = self._fno_rollout(macros)
        stats = self.lat.check_fields(pred[0], pred[1], pred[2])
        ok, why = self.guard.accept(stats, ref["mass"])
        if ok:
            self.lat.reinit(pred[0], pred[1], pred[2])
            self.log.fno_calls += self.k_fno
        else:
            self.lat.step(self.k_fno * self.dt_fno)
            self.log.lbm_steps += self.k_fno * self.dt_fno
            self.log.fallbacks.append(f"t={self.model_time}: {why}")
        self.lat.step(self.n_lbm)
        self.log.lbm_steps += self.n_lbm
        self.model_time += self.k_fno * self.dt_fno + self.n_lbm

    def _cycle_speculative(self):
        import torch
        self._resolve()
        lat = self.lat
        lat.save_state(out=self._saved)
        macros = lat.macros(out=self.x[0, :3])   # straight into the FNO input
        lat.check_fields_async(macros[0], macros[1], macros[2], self._dstats[0:4])
        pred = self._fno_rollout(macros)
        lat.check_fields_async(pred[0], pred[1], pred[2], self._dstats[4:8])
        with torch.cuda.stream(lat.stream):
            self._hstats.copy_(self._dstats, non_blocking=True)
            self._ready.record(lat.stream)
        lat.reinit(pred[0], pred[1], pred[2])
        lat.step(self.n_lbm)
        self._pending = self.model_time
        self.log.fno_calls += self.k_fno
        self.log.lbm_steps += self.n_lbm
        self.model_time += self.k_fno * self.dt_fno + self.n_lbm

    def _resolve(self):
        """Apply the guard to the last speculative cycle; undo and redo it with
        lattice steps when the prediction is rejected."""
        if self._pending is None:
            return
        self._ready.synchronize()
        h = self._hstats.tolist()
        stats = {"mass": h[4], "max_speed": h[5], "nonfinite": int(h[6])}
        ok, why = self.guard.accept(stats, h[0])
        if not ok:
            self.lat.load_state(self._saved)
            self.lat.step(self.k_fno * self.dt_fno + self.n_lbm)
            self.log.fno_calls -= self.k_fno
            self.log.lbm_steps += self.k_fno * self.dt_fno
            self.log.fallbacks.append(f"t={self._pending}: {why}")
        self._pending = None

    def finish(self):
        """Resolve the last speculative cycle (a no-op for the synchronous guard)."""
        import torch
        with torch.cuda.stream(self.lat.stream):
            self._resolve()
        return self.log

    def run(self, cycles: int, on_cycle=None):
        for c in range(cycles):
            self.cycle()
            if on_cycle is not None:
                self.finish()     # the callback sees the guarded state
                on_cycle(c, self)
        return self.finish()


def time_call(fn, stream, reps: int = 1):
    """Milliseconds per call of fn() on `stream`, by HIP events."""
    import torch
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def steady_solve(lattice, tol: float = 1e-8, check_every: int = 500, max_steps: int = 2_000_000,
                 init_fields=None):
    """Run to steady state: optional re-initialisation from predicted fields, then
    lattice steps until the density residual (checked every `check_every` steps)
    is below tol.  Returns (steps, seconds, last report, residual history)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if init_fields is not None:
        lattice.reinit(*init_fields)
    steps, hist, rep = 0, [], None
    while steps < max_steps:
        rep = lattice.step(check_every, report=True)
        steps += check_every
        hist.append((steps, rep["residual"]))
        if rep["residual"] < tol:
            break
    lattice.synchronize()
    return steps, time.perf_counter() - t0, rep, hist
