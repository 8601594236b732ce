"""ctypes binding of liblbmfno.so (include/lbmfno.h): argument marshalling only.

Every step of the hot path runs in the library's HIP kernels; torch supplies
device memory and the stream.  There is no fallback: if the library or a GPU is
missing, load() raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbmfno.so")
_LIB = None

LBM_OK = 0
BC_PERIODIC, BC_WALL, BC_ZOUHE = 0, 1, 2

_p = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64


class LbmConfig(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32),
                ("tau", ctypes.c_double), ("gx", ctypes.c_double), ("gy", ctypes.c_double),
                ("u_in", ctypes.c_double), ("rho_out", ctypes.c_double),
                ("arith", ctypes.c_int32), ("kernel", ctypes.c_int32),
                ("trt_lambda", ctypes.c_double)]


ARITH_MIXED, ARITH_FP32, ARITH_LEAN = 0, 1, 2
KERNEL_AUTO, KERNEL_NODE, KERNEL_QUAD, KERNEL_PAIR, KERNEL_DEEP = 0, 1, 2, 3, 4


class LbmReport(ctypes.Structure):
    _fields_ = [("residual", ctypes.c_double), ("mass", ctypes.c_double),
                ("mom_x", ctypes.c_double), ("mom_y", ctypes.c_double),
                ("steps_done", ctypes.c_int64), ("fluid_nodes", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class LbmError(RuntimeError):
    def __init__(self, code, where):
        lib = _LIB
        msg = lib.lbm_last_error().decode() if lib else ""
        name = lib.lbm_status_str(code).decode() if lib else str(code)
        super().__init__(f"{where}: {name} ({code}): {msg}")
        self.code = code


class FieldStats(ctypes.Structure):
    _fields_ = [("mass", ctypes.c_double), ("max_speed", ctypes.c_double),
                ("nonfinite", ctypes.c_int64), ("fluid_nodes", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class FieldError(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("rel_l1_rho", "rel_l1_ux", "rel_l1_uy", "dp", "dp_ref",
                                                 "rel_dp")]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TrajDesc(ctypes.Structure):
    _fields_ = [("cfg", LbmConfig), ("d_mask", _p), ("d_fA", _p), ("d_fB", _p)]


class FnoSpecC(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("cin", "width", "layers", "m1", "m2", "dec_layers",
                                                "dec_size", "cout", "padding", "coords", "act",
                                                "dec_act")]


# (name, restype, argtypes) of every exported entry point declared in include/*.h
SIGNATURES = [
    ("lbm_status_str", ctypes.c_char_p, [ctypes.c_int]),
    ("lbm_last_error", ctypes.c_char_p, []),
    ("lbm_mask_raster", ctypes.c_int, [_i32, _i32, _i32, _i32, _p, _i32, _p, _p]),
    ("lbm_init", ctypes.c_int, [ctypes.POINTER(_p), ctypes.POINTER(LbmConfig), _p, _p, _p, _p]),
    ("lbm_destroy", None, [_p]),
    ("lbm_reinit_from_macro", ctypes.c_int, [_p, _p, _p, _p]),
    ("lbm_reinit_from_macro_neq", ctypes.c_int, [_p, _p, _p, _p]),
    ("lbm_reinit_from_macro_mass", ctypes.c_int, [_p, _p, _p, _p]),
    ("lbm_step", ctypes.c_int, [_p, _i32, ctypes.POINTER(LbmReport)]),
    ("lbm_get_macro", ctypes.c_int, [_p, _p, _p, _p, _i32]),
    ("lbm_get_populations", ctypes.c_int, [_p, _p]),
    ("lbm_set_populations", ctypes.c_int, [_p, _p]),
    ("lbm_info", ctypes.c_int, [_p, ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
    ("lbm_stream_copy", ctypes.c_int, [_p, _p, ctypes.c_size_t, _p]),
    ("lbm_step_kernel", ctypes.c_char_p, [_p]),
    ("lbm_check_fields", ctypes.c_int, [_p, _p, _p, _p, ctypes.POINTER(FieldStats)]),
    ("lbm_check_fields_async", ctypes.c_int, [_p, _p, _p, _p, _p]),
    ("lbm_compare_fields", ctypes.c_int, [_p, _p, _p, _p, _p, _p, _p, ctypes.POINTER(FieldError)]),
    ("lbm_adjoint_step", ctypes.c_int, [_p, _p, _p, _p]),
    ("lbm_state_elems", ctypes.c_size_t, [_p]),
    ("lbm_save_state", ctypes.c_int, [_p, _p]),
    ("lbm_load_state", ctypes.c_int, [_p, _p]),
    ("lbm_macro_vjp", ctypes.c_int, [_p, _p, _p, _p, _p, _p]),
    ("lbm_feq_vjp", ctypes.c_int, [_p, _p, _p, _p, _p, _p, _p, _p]),
    ("lbm_batch_create", ctypes.c_int, [ctypes.POINTER(_p), ctypes.POINTER(TrajDesc), _i32,
                                        ctypes.c_char_p, _p]),
    ("lbm_batch_step", ctypes.c_int, [_p, _i32]),
    ("lbm_batch_context", ctypes.c_int, [_p, _i32, ctypes.POINTER(_p)]),
    ("lbm_batch_choice", ctypes.c_char_p, [_p]),
    ("lbm_batch_destroy", None, [_p]),
    ("fno_param_count", ctypes.c_int, [ctypes.POINTER(FnoSpecC), ctypes.POINTER(_i64)]),
    ("fno_model_create", ctypes.c_int, [ctypes.POINTER(_p), ctypes.POINTER(FnoSpecC), _p, _i64,
                                        _i32, _i32]),
    ("fno_model_destroy", None, [_p]),
    ("fno_workspace_size", ctypes.c_int, [_p, _i32, ctypes.POINTER(ctypes.c_size_t)]),
    ("fno_forward", ctypes.c_int, [_p, _p, _p, _i32, _p, ctypes.c_size_t, _p]),
    ("fno_forward_graph", ctypes.c_int, [_p, _p, _p, _i32, _p, ctypes.c_size_t, _p]),
    ("fno_forward_noalloc", ctypes.c_int, [_p, _p, _p, _i32, _p]),
    ("fno_train_workspace_size", ctypes.c_int, [_p, _i32, ctypes.POINTER(ctypes.c_size_t)]),
    ("fno_forward_train", ctypes.c_int, [_p, _p, _p, _i32, _p, ctypes.c_size_t, _p]),
    ("fno_backward", ctypes.c_int, [_p, _p, _p, _i32, _p, ctypes.c_size_t, _p, _p]),
    ("fno_train_latent", ctypes.c_int, [_p, _p, ctypes.c_size_t, _i32, _i32, _p, _p]),
    ("fno_mse", ctypes.c_int, [_p, _p, ctypes.c_size_t, _p, _p, ctypes.c_size_t,
                               ctypes.POINTER(ctypes.c_double), _p]),
    ("fno_set_params", ctypes.c_int, [_p, _p, _p]),
    ("fno_adamw", ctypes.c_int, [_p, _p, _p, _p, _i64, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_double, _i64, _p]),
]


def load_library(path: str = LIB_PATH):
    """Load liblbmfno.so (no GPU needed to load) and bind every entry point."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build() "
                           "(or python paper_2604_27158_amd/build.py)")
    lib = ctypes.CDLL(path)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


def load():
    """Load the library and require a visible GPU (no CPU fallback exists)."""
    import torch
    lib = load_library()
    if not torch.cuda.is_available():
        raise RuntimeError("liblbmfno needs a ROCm GPU; none is visible")
    return lib


def check(rc: int, where: str):
    if rc != LBM_OK:
        raise LbmError(rc, where)


def _ptr(t) -> int:
    return t.data_ptr() if t is not None else None


def stream_handle(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def mask_raster(nx: int, ny: int, shapes: np.ndarray, wrap_x: bool, wrap_y: bool, stream=None):
    """Obstacle mask (uint8 [ny][nx] torch tensor on the GPU) from int64 descriptors."""
    import torch
    lib = load()
    shapes = np.ascontiguousarray(np.asarray(shapes, dtype=np.int64).reshape(-1, 7))
    mask = torch.empty((ny, nx), dtype=torch.uint8, device="cuda")
    check(lib.lbm_mask_raster(nx, ny, int(wrap_x), int(wrap_y),
                              shapes.ctypes.data_as(_p) if shapes.size else None,
                              shapes.shape[0], mask.data_ptr(), stream_handle(stream)),
          "lbm_mask_raster")
    return mask


def stream_copy(src, dst, stream=None):
    """dst[:] = src[:] (float32 device tensors) with the library's copy kernel."""
    lib = load()
    check(lib.lbm_stream_copy(src.data_ptr(), dst.data_ptr(), src.numel(), stream_handle(stream)),
          "lbm_stream_copy")


class Lattice:
    """A device lattice: two population stores (torch float32 [9][ny][nx]) and the
    library context, all on one dedicated non-default stream (graph replay needs a
    capturable stream)."""

    def __init__(self, nx, ny, tau, gx=0.0, gy=0.0, bc_x=BC_PERIODIC, bc_y=BC_PERIODIC,
                 u_in=0.0, rho_out=1.0, mask=None, stream=None, arith=ARITH_LEAN,
                 kernel=KERNEL_AUTO, trt_lambda=0.0):
        import torch
        self.lib = load()
        self.nx, self.ny = int(nx), int(ny)
        self.cfg = LbmConfig(self.nx, self.ny, bc_x, bc_y, float(tau), float(gx), float(gy),
                             float(u_in), float(rho_out), int(arith), int(kernel), float(trt_lambda))
        self.stream = stream if stream is not None else torch.cuda.Stream()
        with torch.cuda.stream(self.stream):
            self.fA = torch.empty((9, ny, nx), dtype=torch.float32, device="cuda")
            self.fB = torch.empty((9, ny, nx), dtype=torch.float32, device="cuda")
            if mask is None:
                mask = torch.zeros((ny, nx), dtype=torch.uint8, device="cuda")
            self.mask = mask
        self.ctx = _p()
        check(self.lib.lbm_init(ctypes.byref(self.ctx), ctypes.byref(self.cfg), mask.data_ptr(),
                                self.fA.data_ptr(), self.fB.data_ptr(), self.stream.cuda_stream),
              "lbm_init")

    @classmethod
    def from_workload(cls, lat, stream=None, arith=ARITH_LEAN, kernel=KERNEL_AUTO):
        """Build from a workloads.Lattice (its mask rasterised on the GPU)."""
        import torch
        stream = stream if stream is not None else torch.cuda.Stream()
        with torch.cuda.stream(stream):
            mask = mask_raster(lat.nx, lat.ny, lat.shapes_array(), lat.wrap_x, lat.wrap_y, stream)
        return cls(lat.nx, lat.ny, lat.tau, lat.gx, lat.gy, lat.bc_x, lat.bc_y, lat.u_in,
                   lat.rho_out, mask=mask, stream=stream, arith=arith, kernel=kernel,
                   trt_lambda=getattr(lat, "trt_lambda", 0.0))

    @classmethod
    def _view(cls, lib, ctx, nx, ny, mask, stream, owner):
        """Non-owning view of a context that belongs to a batch."""
        obj = cls.__new__(cls)
        obj.lib, obj.ctx, obj.nx, obj.ny = lib, ctx, nx, ny
        obj.mask, obj.stream, obj._owner = mask, stream, owner
        return obj

    def close(self):
        if getattr(self, "_owner", None) is not None:
            return
        if self.ctx:
            self.lib.lbm_destroy(self.ctx)
            self.ctx = _p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int, report: bool = False):
        rep = LbmReport() if report else None
        check(self.lib.lbm_step(self.ctx, int(n), ctypes.byref(rep) if rep is not None else None),
              "lbm_step")
        return rep.as_dict() if rep is not None else None

    def _after_caller(self):
        import torch
        cur = torch.cuda.current_stream()
        if cur != self.stream:   # a caller already on the lattice stream is ordered
            self.stream.wait_stream(cur)

    def _before_caller(self):
        import torch
        cur = torch.cuda.current_stream()
        if cur != self.stream:
            cur.wait_stream(self.stream)

    def _hand_over(self, *outs):
        """Outputs written on the lattice stream and returned to the caller: the
        caller's stream waits for them, and the allocator is told that the caller's
        stream uses them (else a block freed by the caller could be handed to the
        next lattice-stream allocation while the caller still reads it)."""
        import torch
        self._before_caller()
        cur = torch.cuda.current_stream()
        for t in outs:
            t.record_stream(cur)

    def _take_inputs(self, *ins):
        """Inputs from the caller's stream that lattice kernels read: the lattice
        stream waits for the caller, and the inputs are marked as used on it."""
        self._after_caller()
        for t in ins:
            t.record_stream(self.stream)

    def reinit(self, rho, ux, uy, neq: bool = False, mass: bool = False):
        """f = f_eq(rho, u) (with neq, plus the first-order non-equilibrium part from the
        velocity gradient; with mass, rho shifted by a constant so that the fluid mass
        stays the current state's), then the boundary closures; the step count restarts."""
        import torch
        self._after_caller()
        with torch.cuda.stream(self.stream):
            rho, ux, uy = (t.to(device="cuda", dtype=torch.float32).contiguous() for t in (rho, ux, uy))
        self._take_inputs(rho, ux, uy)
        self._keep = (rho, ux, uy)
        if neq and mass:
            raise ValueError("choose one of neq and mass")
        fn = (self.lib.lbm_reinit_from_macro_neq if neq else
              self.lib.lbm_reinit_from_macro_mass if mass else self.lib.lbm_reinit_from_macro)
        check(fn(self.ctx, rho.data_ptr(), ux.data_ptr(), uy.data_ptr()), "lbm_reinit_from_macro")

    def macros(self, rho_minus_one: bool = False, out=None):
        """(rho, ux, uy) [3][ny][nx] float32; written into `out` (a contiguous device
        tensor of that shape) when given, else into a new tensor."""
        import torch
        if out is None:
            with torch.cuda.stream(self.stream):
                out = torch.empty((3, self.ny, self.nx), dtype=torch.float32, device="cuda")
        else:
            if (tuple(out.shape) != (3, self.ny, self.nx) or out.dtype != torch.float32
                    or not out.is_cuda or not out.is_contiguous()):
                raise ValueError("out must be a contiguous float32 device tensor [3][ny][nx]")
            self._after_caller()   # the caller's pending use of `out` comes first
            out.record_stream(self.stream)
        check(self.lib.lbm_get_macro(self.ctx, out[0].data_ptr(), out[1].data_ptr(),
                                     out[2].data_ptr(), int(rho_minus_one)), "lbm_get_macro")
        self._hand_over(out)
        return out

    def populations(self, out=None):
        """Pre-collision populations f(n), absolute, [9][ny][nx] float32; written into
        `out` (a contiguous device tensor of that shape) when given."""
        import torch
        if out is None:
            with torch.cuda.stream(self.stream):
                out = torch.empty((9, self.ny, self.nx), dtype=torch.float32, device="cuda")
        else:
            if (tuple(out.shape) != (9, self.ny, self.nx) or out.dtype != torch.float32
                    or not out.is_cuda or not out.is_contiguous()):
                raise ValueError("out must be a contiguous float32 device tensor [9][ny][nx]")
            self._after_caller()
            out.record_stream(self.stream)
        check(self.lib.lbm_get_populations(self.ctx, out.data_ptr()), "lbm_get_populations")
        self._hand_over(out)
        return out

    def set_populations(self, f):
        import torch
        self._after_caller()
        with torch.cuda.stream(self.stream):
            f = f.to(device="cuda", dtype=torch.float32).contiguous()
        self._take_inputs(f)
        self._keep_f = f
        check(self.lib.lbm_set_populations(self.ctx, f.data_ptr()), "lbm_set_populations")

    def check_fields(self, rho, ux, uy):
        """Mass, peak speed and non-finite count of fields over fluid nodes."""
        self._take_inputs(rho, ux, uy)
        st = FieldStats()
        check(self.lib.lbm_check_fields(self.ctx, rho.data_ptr(), ux.data_ptr(), uy.data_ptr(),
                                        ctypes.byref(st)), "lbm_check_fields")
        return st.as_dict()

    def check_fields_async(self, rho, ux, uy, out):
        """lbm_check_fields without the wait: [mass, max |u|, non-finite count, 0] as
        float64 into the device tensor `out` (4 elements), on the lattice stream."""
        import torch
        if out.dtype != torch.float64 or out.numel() < 4 or not out.is_cuda or not out.is_contiguous():
            raise ValueError("out must be a contiguous float64 device tensor of 4 elements")
        self._take_inputs(rho, ux, uy, out)
        check(self.lib.lbm_check_fields_async(self.ctx, rho.data_ptr(), ux.data_ptr(), uy.data_ptr(),
                                              out.data_ptr()), "lbm_check_fields_async")

    def compare(self, fields, ref):
        """lbm_compare_fields of [3][ny][nx] (rho - 1, ux, uy) device tensors."""
        fields, ref = fields.contiguous(), ref.contiguous()
        self._take_inputs(fields, ref)
        e = FieldError()
        check(self.lib.lbm_compare_fields(self.ctx, fields[0].data_ptr(), fields[1].data_ptr(),
                                          fields[2].data_ptr(), ref[0].data_ptr(), ref[1].data_ptr(),
                                          ref[2].data_ptr(), ctypes.byref(e)), "lbm_compare_fields")
        return e.as_dict()

    def save_state(self, out=None):
        """Exact copy of the current store (a device tensor; into `out` when given)."""
        import torch
        n = int(self.lib.lbm_state_elems(self.ctx))
        if out is None:
            with torch.cuda.stream(self.stream):
                out = torch.empty(n, dtype=torch.float32, device="cuda")
        elif out.dtype != torch.float32 or out.numel() != n or not out.is_cuda or not out.is_contiguous():
            raise ValueError(f"out must be a contiguous float32 device tensor of {n} elements")
        else:
            self._take_inputs(out)
        check(self.lib.lbm_save_state(self.ctx, out.data_ptr()), "lbm_save_state")
        self._hand_over(out)
        return out

    def load_state(self, saved):
        self._take_inputs(saved)
        self._keep_state = saved
        check(self.lib.lbm_load_state(self.ctx, saved.data_ptr()), "lbm_load_state")

    def adjoint_step(self, f_n, lam_np1, out=None):
        """lam_n = C'(f(n))^T P^T lam_{n+1} (float32 [9][ny][nx] device tensors)."""
        import torch
        self._take_inputs(f_n, lam_np1)
        if out is None:
            with torch.cuda.stream(self.stream):
                out = torch.empty_like(lam_np1)
        else:
            self._take_inputs(out)
        check(self.lib.lbm_adjoint_step(self.ctx, f_n.data_ptr(), lam_np1.data_ptr(), out.data_ptr()),
              "lbm_adjoint_step")
        self._hand_over(out)
        return out

    def macro_vjp(self, f_n, g_rho, g_ux, g_uy):
        import torch
        with torch.cuda.stream(self.stream):
            lam = torch.empty_like(f_n)
            g = [t.to(device="cuda", dtype=torch.float32).contiguous() for t in (g_rho, g_ux, g_uy)]
        self._take_inputs(f_n, *g)
        check(self.lib.lbm_macro_vjp(self.ctx, f_n.data_ptr(), g[0].data_ptr(), g[1].data_ptr(),
                                     g[2].data_ptr(), lam.data_ptr()), "lbm_macro_vjp")
        self._hand_over(lam)
        return lam

    def feq_vjp(self, rho, ux, uy, lam):
        import torch
        with torch.cuda.stream(self.stream):
            fields = [t.to(device="cuda", dtype=torch.float32).contiguous() for t in (rho, ux, uy)]
            out = torch.empty((3, self.ny, self.nx), dtype=torch.float32, device="cuda")
        self._take_inputs(*fields, lam)
        check(self.lib.lbm_feq_vjp(self.ctx, fields[0].data_ptr(), fields[1].data_ptr(),
                                   fields[2].data_ptr(), lam.data_ptr(), out[0].data_ptr(),
                                   out[1].data_ptr(), out[2].data_ptr()), "lbm_feq_vjp")
        self._hand_over(out)
        return out

    def step_kernel(self) -> str:
        """"<shape>/<arith>" of the step kernel this lattice runs (lbm_step_kernel)."""
        return self.lib.lbm_step_kernel(self.ctx).decode()

    def info(self):
        fl, st = _i64(), _i64()
        check(self.lib.lbm_info(self.ctx, ctypes.byref(fl), ctypes.byref(st)), "lbm_info")
        return fl.value, st.value

    def synchronize(self):
        self.stream.synchronize()


class Batch:
    """Many trajectories (workloads.Lattice list) stepped by one launch per step;
    trajectory(i) returns a Lattice view for reinit / macros / field checks."""

    def __init__(self, lats, tune_cache=None, stream=None):
        import torch
        self.lib = load()
        self.stream = stream if stream is not None else torch.cuda.Stream()
        self.lats = list(lats)
        descs = (TrajDesc * len(self.lats))()
        self._bufs = []
        with torch.cuda.stream(self.stream):
            for k, lat in enumerate(self.lats):
                mask = mask_raster(lat.nx, lat.ny, lat.shapes_array(), lat.wrap_x, lat.wrap_y,
                                   self.stream)
                fA = torch.empty((9, lat.ny, lat.nx), dtype=torch.float32, device="cuda")
                fB = torch.empty_like(fA)
                self._bufs.append((mask, fA, fB))
                descs[k].cfg = LbmConfig(lat.nx, lat.ny, lat.bc_x, lat.bc_y, float(lat.tau),
                                         float(lat.gx), float(lat.gy), float(lat.u_in),
                                         float(lat.rho_out), ARITH_LEAN, KERNEL_AUTO,
                                         float(getattr(lat, "trt_lambda", 0.0)))
                descs[k].d_mask, descs[k].d_fA, descs[k].d_fB = mask.data_ptr(), fA.data_ptr(), fB.data_ptr()
        self.handle = _p()
        cache = tune_cache.encode() if tune_cache else None
        check(self.lib.lbm_batch_create(ctypes.byref(self.handle), descs, len(self.lats), cache,
                                        self.stream.cuda_stream), "lbm_batch_create")
        self.choice = self.lib.lbm_batch_choice(self.handle).decode()
        self.nodes = sum(l.nx * l.ny for l in self.lats)

    def step(self, n: int):
        check(self.lib.lbm_batch_step(self.handle, int(n)), "lbm_batch_step")

    def trajectory(self, i: int) -> "Lattice":
        ctx = _p()
        check(self.lib.lbm_batch_context(self.handle, int(i), ctypes.byref(ctx)), "lbm_batch_context")
        lat = self.lats[i]
        return Lattice._view(self.lib, ctx, lat.nx, lat.ny, self._bufs[i][0], self.stream, self)

    def synchronize(self):
        self.stream.synchronize()

    def close(self):
        if self.handle:
            self.lib.lbm_batch_destroy(self.handle)
            self.handle = _p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
