"""FP64 gradient oracle of the FNO training loss -- TEST INFRASTRUCTURE ONLY.

Only tests/ import this module.  It shares no code with the GPU path.

What it computes: the gradient, with respect to the packed parameters, of the
mean squared error between the FNO output and a target (the training objective of
the paper's Sec. 2.2), for the forward pass that oracle/fno.py defines (lift,
Fourier layers with truncated DFTs and per-mode complex mixing, 1x1 convolution,
decoder).  The forward is written here a second time with torch float64 tensors,
the same explicit truncated DFTs and the same rounding points, so that reverse-mode
automatic differentiation (torch.autograd, a library step) yields the gradient.

Precision:
  "fp64"  everything in float64;
  "bf16"  the product path's policy: every value oracle/fno.py rounds in its "bf16"
          mode is rounded here too, with the rounding treated as the identity in the
          backward pass (straight-through: x + (round(x) - x) detached).  This is
          the exact derivative the GPU backward approximates; the GPU additionally
          rounds its own backward contraction operands to bfloat16.

Pins (tests/test_oracle_fno_grad.py): the forward equals oracle/fno.forward in
both modes; central differences of oracle/fno.forward's loss (explicit numpy
DFTs, float64) along random directions and for single elements of every parameter
group equal the gradient; the output-bias gradient equals its closed form.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import fno as ofno


def _st(precision):
    """Rounding maps for a precision: (bf16 round, float32 round), straight-through."""
    if precision == "fp64":
        ident = lambda a: a
        return ident, ident

    def rb(a):
        r = torch.from_numpy(ofno.round_bf16(a.detach().numpy()))
        return a + (r - a).detach()

    def r32(a):
        r = a.detach().to(torch.float32).to(torch.float64)
        return a + (r - a).detach()

    return rb, r32


def _act(name):
    if name == "gelu":
        return lambda x: 0.5 * x * (1.0 + torch.erf(x / math.sqrt(2.0)))
    if name == "silu":
        return lambda x: x * torch.sigmoid(x)
    if name == "relu":
        return torch.relu
    return lambda x: x


def _pointwise(w, b, x, rb):
    y = torch.einsum("oc,bc...->bo...", rb(w), rb(x))
    return y + b.reshape((1, -1) + (1,) * (x.dim() - 2))


def _spectral(v, r_top, r_bot, m1, m2, rb):
    """F^-1(R . F(v)) on [B][C][H'][W'] with the kept modes of oracle/fno.py."""
    B, C, hp, wp = v.shape
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a))
    k1 = ofno.kept_k1(hp, m1)
    k2 = np.arange(m2)
    aw = ofno.angle(k2, np.arange(wp), wp)
    cw, sw = rb(T(np.cos(aw))), rb(T(np.sin(aw)))
    vr = rb(v)
    t_re = torch.einsum("bchw,kw->bchk", vr, cw)
    t_im = -torch.einsum("bchw,kw->bchk", vr, sw)
    ah = ofno.angle(k1, np.arange(hp), hp)
    ch, sh = rb(T(np.cos(ah))), rb(T(np.sin(ah)))
    t_re, t_im = rb(t_re), rb(t_im)
    x_re = torch.einsum("bchk,lh->bclk", t_re, ch) + torch.einsum("bchk,lh->bclk", t_im, sh)
    x_im = torch.einsum("bchk,lh->bclk", t_im, ch) - torch.einsum("bchk,lh->bclk", t_re, sh)
    R = torch.cat([r_top, r_bot], dim=2)
    r_re, r_im = rb(R[..., 0]), rb(R[..., 1])
    x_re, x_im = rb(x_re), rb(x_im)
    y_re = torch.einsum("bilk,iolk->bolk", x_re, r_re) - torch.einsum("bilk,iolk->bolk", x_im, r_im)
    y_im = torch.einsum("bilk,iolk->bolk", x_re, r_im) + torch.einsum("bilk,iolk->bolk", x_im, r_re)
    y_re, y_im = rb(y_re), rb(y_im)
    z_re = torch.einsum("bolk,lh->bohk", y_re, ch) - torch.einsum("bolk,lh->bohk", y_im, sh)
    z_im = torch.einsum("bolk,lh->bohk", y_re, sh) + torch.einsum("bolk,lh->bohk", y_im, ch)
    ck = np.where(k2 == 0, 1.0, 2.0)[:, None] / (hp * wp)
    ciw, siw = rb(T(ck * np.cos(aw))), rb(T(-ck * np.sin(aw)))
    z_re, z_im = rb(z_re), rb(z_im)
    return torch.einsum("bohk,kw->bohw", z_re, ciw) + torch.einsum("bohk,kw->bohw", z_im, siw)


def forward(spec: ofno.Spec, flat: torch.Tensor, x: torch.Tensor, precision: str = "fp64"):
    """Differentiable FNO forward (float64 torch), x [B][Cin][H][W]."""
    if precision not in ("fp64", "bf16"):
        raise ValueError(precision)
    rb, r32 = _st(precision)
    P, off = {}, 0
    for name, shp in ofno.layout(spec):
        n = int(np.prod(shp))
        P[name] = flat[off:off + n].reshape(shp)
        off += n
    if precision == "bf16":
        x = x.to(torch.float32).to(torch.float64)
    B, _, H, W = x.shape
    act, dact = _act(spec.act), _act(spec.dec_act)
    if spec.coords:
        xs, ys = ofno.coords(B, H, W)
        x = torch.cat([x, torch.from_numpy(np.ascontiguousarray(xs)),
                       torch.from_numpy(np.ascontiguousarray(ys))], dim=1)
    h = act(_pointwise(r32(P["lift1.w"]), r32(P["lift1.b"]), x, lambda a: a))
    v = _pointwise(r32(P["lift2.w"]), r32(P["lift2.b"]), h, lambda a: a)
    p = spec.padding
    if p:
        v = torch.nn.functional.pad(v, (0, p, 0, p))
    v = rb(v)
    for n in range(spec.layers):
        s = _spectral(v, P[f"spec{n}.r_top"], P[f"spec{n}.r_bot"], spec.m1, spec.m2, rb)
        s = s + _pointwise(P[f"conv{n}.w"], r32(P[f"conv{n}.b"]), v, rb)
        v = act(s) if n < spec.layers - 1 else s
        v = rb(v)
    if p:
        v = v[:, :, :H, :W]
    for n in range(spec.dec_layers):
        v = rb(dact(_pointwise(P[f"dec{n}.w"], r32(P[f"dec{n}.b"]), v, rb)))
    return _pointwise(P["dec_out.w"], r32(P["dec_out.b"]), v, rb)


def loss_and_grad(spec: ofno.Spec, flat_params, x, target, precision: str = "fp64"):
    """(mean squared error, its gradient w.r.t. the packed parameters, output), all
    float64 numpy."""
    flat = torch.tensor(np.asarray(flat_params, dtype=np.float64).ravel(), requires_grad=True)
    xt = torch.from_numpy(np.asarray(x, dtype=np.float64))
    tt = torch.from_numpy(np.asarray(target, dtype=np.float64))
    out = forward(spec, flat, xt, precision)
    loss = ((out - tt) ** 2).mean()
    loss.backward()
    return float(loss.detach()), flat.grad.numpy().copy(), out.detach().numpy()


def vjp(spec: ofno.Spec, flat_params, x, g_out, precision: str = "fp64"):
    """(output, sum over outputs of g_out * d output / d params): the parameter
    gradient of any loss whose gradient with respect to the FNO output is g_out
    (float64 numpy)."""
    flat = torch.tensor(np.asarray(flat_params, dtype=np.float64).ravel(), requires_grad=True)
    xt = torch.from_numpy(np.asarray(x, dtype=np.float64))
    out = forward(spec, flat, xt, precision)
    (g,) = torch.autograd.grad(out, flat, grad_outputs=torch.from_numpy(np.asarray(g_out, np.float64)))
    return out.detach().numpy(), g.numpy().copy()


def group_slices(spec: ofno.Spec):
    """name -> slice of every parameter tensor in the packed vector."""
    out, off = {}, 0
    for name, shp in ofno.layout(spec):
        n = int(np.prod(shp))
        out[name] = slice(off, off + n)
        off += n
    return out
