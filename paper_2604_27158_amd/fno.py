"""ctypes binding of the FNO entry points of liblbmfno.so (include/lbmfno.h):
argument marshalling only; the forward pass runs in the library's HIP kernels."""
from __future__ import annotations

import ctypes

import numpy as np

from . import lbmfno as _L

ACT = {"gelu": 0, "relu": 1, "silu": 2, "identity": 3}


FnoSpecC = _L.FnoSpecC


def to_c(spec) -> FnoSpecC:
    """C spec from any object with the FnoSpec fields (workloads.FnoSpec)."""
    return FnoSpecC(spec.cin, spec.width, spec.layers, spec.m1, spec.m2, spec.dec_layers,
                    spec.dec_size, spec.cout, spec.padding, int(bool(spec.coords)),
                    ACT[spec.act], ACT[spec.dec_act])


def param_count(spec) -> int:
    lib = _L.load_library()
    n = ctypes.c_int64()
    _L.check(lib.fno_param_count(ctypes.byref(to_c(spec)), ctypes.byref(n)), "fno_param_count")
    return n.value


def param_layout(spec):
    """(name, shape) of the packed parameter tensors in the order the C ABI reads
    them (lift, per-layer spectral/conv, decoder)."""
    cl = spec.cin + (2 if spec.coords else 0)
    h, wd = spec.width // 2, spec.width
    out = [("lift1.w", (h, cl)), ("lift1.b", (h,)), ("lift2.w", (wd, h)), ("lift2.b", (wd,))]
    for n in range(spec.layers):
        out += [(f"spec{n}.r_top", (wd, wd, spec.m1, spec.m2, 2)),
                (f"spec{n}.r_bot", (wd, wd, spec.m1, spec.m2, 2)),
                (f"conv{n}.w", (wd, wd)), (f"conv{n}.b", (wd,))]
    din = wd
    for n in range(spec.dec_layers):
        out += [(f"dec{n}.w", (spec.dec_size, din)), (f"dec{n}.b", (spec.dec_size,))]
        din = spec.dec_size
    out += [("dec_out.w", (spec.cout, din)), ("dec_out.b", (spec.cout,))]
    return out


class Fno:
    """Device FNO bound to an H x W grid; forward() takes float32 [B][cin][H][W]."""

    def __init__(self, spec, params, H: int, W: int):
        self.lib = _L.load()
        self.spec, self.H, self.W = spec, int(H), int(W)
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32).ravel())
        self.model = ctypes.c_void_p()
        _L.check(self.lib.fno_model_create(ctypes.byref(self.model), ctypes.byref(to_c(spec)),
                                           p.ctypes.data_as(ctypes.c_void_p), p.size, self.H, self.W),
                 "fno_model_create")
        self._ws = {}

    def workspace(self, B: int):
        import torch
        if B not in self._ws:
            n = ctypes.c_size_t()
            _L.check(self.lib.fno_workspace_size(self.model, int(B), ctypes.byref(n)), "fno_workspace_size")
            self._ws[B] = torch.empty(int(n.value), dtype=torch.uint8, device="cuda")
        return self._ws[B]

    def forward(self, x, out=None, stream=None, graph=False):
        """out = FNO(x) on `stream` (the current stream by default).  graph=True
        replays the launches from a HIP graph captured for this (x, out, B)
        tuple; keep x and out the same tensors from call to call to reuse it."""
        import torch
        x = x.to(device="cuda", dtype=torch.float32).contiguous()
        B = x.shape[0]
        if tuple(x.shape[1:]) != (self.spec.cin, self.H, self.W):
            raise ValueError(f"input shape {tuple(x.shape)} != [B][{self.spec.cin}][{self.H}][{self.W}]")
        if out is None:
            out = torch.empty((B, self.spec.cout, self.H, self.W), dtype=torch.float32, device="cuda")
        ws = self.workspace(B)
        cur = torch.cuda.current_stream()
        if stream is not None and stream != cur:
            # run on `stream` after the caller's pending work; mark the tensors as
            # used there so that the allocator does not recycle them early
            stream.wait_stream(cur)
            for t in (x, out):
                t.record_stream(stream)
        fn = self.lib.fno_forward_graph if graph else self.lib.fno_forward
        _L.check(fn(self.model, x.data_ptr(), out.data_ptr(), int(B), ws.data_ptr(), ws.numel(),
                    _L.stream_handle(stream)), "fno_forward")
        return out

    __call__ = forward

    def close(self):
        if self.model:
            self.lib.fno_model_destroy(self.model)
            self.model = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Trainer:
    """AdamW training of an Fno on device-resident samples: forward (saving
    activations), MSE loss, backward, AdamW and the weight refresh all run in the
    library's kernels on `stream` (argument marshalling only here)."""

    def __init__(self, fno: Fno, params, lr: float = 1e-3, betas=(0.9, 0.999), eps: float = 1e-8,
                 weight_decay: float = 1e-4, stream=None):
        import torch
        self.fno, self.lib = fno, fno.lib
        self.stream = stream
        self.p = torch.as_tensor(np.asarray(params, dtype=np.float32).ravel()).to("cuda")
        n = param_count(fno.spec)
        if self.p.numel() != n:
            raise ValueError(f"expected {n} parameters, got {self.p.numel()}")
        self.g = torch.zeros_like(self.p)
        self.m = torch.zeros_like(self.p)
        self.v = torch.zeros_like(self.p)
        self.lr, self.betas, self.eps, self.wd = float(lr), betas, float(eps), float(weight_decay)
        self.t = 0
        self._ws = {}
        self._mse_ws = None
        self._dout = {}
        _L.check(self.lib.fno_set_params(fno.model, self.p.data_ptr(), _L.stream_handle(stream)),
                 "fno_set_params")

    def workspace(self, B: int):
        import torch
        if B not in self._ws:
            n = ctypes.c_size_t()
            _L.check(self.lib.fno_train_workspace_size(self.fno.model, int(B), ctypes.byref(n)),
                     "fno_train_workspace_size")
            self._ws[B] = torch.empty(int(n.value), dtype=torch.uint8, device="cuda")
        return self._ws[B]

    def _check_x(self, x):
        import torch
        s = self.fno.spec
        if x.dtype != torch.float32 or not x.is_cuda or not x.is_contiguous():
            raise ValueError("x must be a contiguous float32 CUDA tensor")
        if tuple(x.shape[1:]) != (s.cin, self.fno.H, self.fno.W):
            raise ValueError(f"input shape {tuple(x.shape)}")

    def forward(self, x, out=None):
        import torch
        self._check_x(x)
        B = x.shape[0]
        if out is None:
            out = torch.empty((B, self.fno.spec.cout, self.fno.H, self.fno.W), dtype=torch.float32,
                              device="cuda")
        ws = self.workspace(B)
        _L.check(self.lib.fno_forward_train(self.fno.model, x.data_ptr(), out.data_ptr(), int(B),
                                            ws.data_ptr(), ws.numel(), _L.stream_handle(self.stream)),
                 "fno_forward_train")
        return out

    def latent(self, B: int, layer: int):
        """Latent v_layer [B][width][H'][W'] float32 that the last forward() saved
        (0: the lift's output, l: the output of Fourier layer l - 1)."""
        import torch
        s = self.fno.spec
        out = torch.empty((B, s.width, self.fno.H + s.padding, self.fno.W + s.padding),
                          dtype=torch.float32, device="cuda")
        ws = self.workspace(B)
        _L.check(self.lib.fno_train_latent(self.fno.model, ws.data_ptr(), ws.numel(), int(B), int(layer),
                                           out.data_ptr(), _L.stream_handle(self.stream)), "fno_train_latent")
        return out

    def backward(self, x, dout):
        """Gradient (into self.g) for the activations the last forward() saved."""
        self._check_x(x)
        B = x.shape[0]
        ws = self.workspace(B)
        _L.check(self.lib.fno_backward(self.fno.model, x.data_ptr(), dout.contiguous().data_ptr(),
                                       int(B), ws.data_ptr(), ws.numel(), self.g.data_ptr(),
                                       _L.stream_handle(self.stream)), "fno_backward")
        return self.g

    def mse(self, out, target):
        """(loss, dLoss/dout) of the mean squared error."""
        import torch
        n = out.numel()
        if target.shape != out.shape or target.dtype != torch.float32:
            raise ValueError("target must match out (float32)")
        nb = (n + 255) // 256 + 1
        if self._mse_ws is None or self._mse_ws.numel() < nb:
            self._mse_ws = torch.empty(nb, dtype=torch.float64, device="cuda")
        key = tuple(out.shape)
        if key not in self._dout:
            self._dout[key] = torch.empty_like(out)
        loss = ctypes.c_double()
        _L.check(self.lib.fno_mse(out.data_ptr(), target.contiguous().data_ptr(), n,
                                  self._dout[key].data_ptr(), self._mse_ws.data_ptr(),
                                  self._mse_ws.numel() * 8, ctypes.byref(loss),
                                  _L.stream_handle(self.stream)), "fno_mse")
        return loss.value, self._dout[key]

    def adamw(self):
        self.t += 1
        _L.check(self.lib.fno_adamw(self.p.data_ptr(), self.g.data_ptr(), self.m.data_ptr(),
                                    self.v.data_ptr(), self.p.numel(), self.lr, self.betas[0],
                                    self.betas[1], self.eps, self.wd, self.t,
                                    _L.stream_handle(self.stream)), "fno_adamw")
        _L.check(self.lib.fno_set_params(self.fno.model, self.p.data_ptr(),
                                         _L.stream_handle(self.stream)), "fno_set_params")

    def step(self, x, target):
        """One optimisation step on a batch; returns the batch loss before the update."""
        out = self.forward(x)
        loss, dout = self.mse(out, target)
        self.backward(x, dout)
        self.adamw()
        return loss

    def params(self):
        return self.p.detach().cpu().numpy().astype(np.float64)


def fold_affine(spec, params, in_scale, in_shift, out_scale, out_shift):
    """Packed parameters of the network on raw channels, given one trained on
    normalised ones: inputs z' = (z - in_shift) / in_scale (per input channel; the
    coordinate channels pass unchanged) folded into the lift's first layer, outputs
    y = out_scale * o + out_shift folded into the decoder's last layer."""
    p = np.array(params, dtype=np.float64, copy=True)
    off, o = {}, 0
    for name, shp in param_layout(spec):
        off[name] = (o, shp)
        o += int(np.prod(shp))
    o1, (h, cl) = off["lift1.w"]
    w1 = p[o1:o1 + h * cl].reshape(h, cl)
    ob1, _ = off["lift1.b"]
    b1 = p[ob1:ob1 + h]
    sc = np.ones(cl)
    sh = np.zeros(cl)
    sc[:spec.cin] = in_scale
    sh[:spec.cin] = in_shift
    b1 -= (w1 * (sh / sc)[None, :]).sum(axis=1)
    w1 /= sc[None, :]
    ow, (co, din) = off["dec_out.w"]
    ob, _ = off["dec_out.b"]
    wo = p[ow:ow + co * din].reshape(co, din)
    bo = p[ob:ob + co]
    wo *= np.asarray(out_scale, dtype=np.float64)[:, None]
    bo *= np.asarray(out_scale, dtype=np.float64)
    bo += np.asarray(out_shift, dtype=np.float64)
    return p
