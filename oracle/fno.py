"""Plain FP64 oracle of the Fourier Neural Operator forward pass -- TEST INFRASTRUCTURE ONLY.

Only tests/, the package smoke check and the benchmark's CPU-baseline leg import
this module.  It shares no code with the GPU path.

What it computes (the paper's Sec. 2.2, Eq. 6 and Fig. 2's caption):
  lift P: pointwise two-layer network (input channels + 2 coordinate channels
          -> width/2 -> width) with the layer activation in between;
  N Fourier layers: theta_{n+1} = sigma(W theta_n + F^-1(R(k) . F(theta_n)(k))),
          F a 2-D DFT truncated to the kept modes k1 in {0..m1-1} U {H'-m1..H'-1}
          (two-sided along H) and k2 in {0..m2-1} (one-sided along W), R a learned
          complex per-mode channel-mixing matrix (one block for the non-negative
          k1, one for the negative k1), F^-1 the real inverse transform (Hermitian
          completion along W: the k2 = 0 column contributes its real part once, the
          others twice; 1/(H'W') normalisation), W a 1x1 convolution with bias;
          no activation after the last layer;
  projection Q: pointwise decoder (dec_layers hidden layers of dec_size with the
          decoder activation, then a linear map to the output channels).
H' = H + padding, W' = W + padding: zero padding on the high side of both spatial
axes before the Fourier layers, cropped afterwards.  The structure (coordinate
channels, width/2 hidden lift, two complex blocks per layer, decoder) is the one
that reproduces all six parameter counts printed in the paper's tables.

Precision: "fp64" evaluates everything in float64.  "bf16" evaluates in float64 but
rounds to bfloat16 (round-to-nearest-even) every operand the GPU feeds to a BF16
matrix contraction -- activations, DFT bases (with the inverse normalisation folded
into the W-direction inverse basis), spectral and 1x1 weights, decoder weights and
the decoder hidden activation -- and rounds lift weights and biases to float32;
this is the precision policy of the product path (BF16 operands, wide
accumulation), so it is compared against the GPU with a tolerance derived from
accumulation order alone, while the fp64 mode gives the "error vs FP64" report.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


@dataclass
class Spec:
    cin: int = 4
    width: int = 32
    layers: int = 4
    m1: int = 12
    m2: int = 12
    dec_layers: int = 1
    dec_size: int = 32
    cout: int = 3
    padding: int = 0
    coords: bool = True
    act: str = "gelu"
    dec_act: str = "silu"


def layout(spec: Spec):
    """(name, shape) of every parameter tensor in packing order."""
    cl = spec.cin + (2 if spec.coords else 0)
    half = spec.width // 2
    out = [("lift1.w", (half, cl)), ("lift1.b", (half,)),
           ("lift2.w", (spec.width, half)), ("lift2.b", (spec.width,))]
    for n in range(spec.layers):
        out.append((f"spec{n}.r_top", (spec.width, spec.width, spec.m1, spec.m2, 2)))
        out.append((f"spec{n}.r_bot", (spec.width, spec.width, spec.m1, spec.m2, 2)))
        out.append((f"conv{n}.w", (spec.width, spec.width)))
        out.append((f"conv{n}.b", (spec.width,)))
    din = spec.width
    for n in range(spec.dec_layers):
        out.append((f"dec{n}.w", (spec.dec_size, din)))
        out.append((f"dec{n}.b", (spec.dec_size,)))
        din = spec.dec_size
    out.append(("dec_out.w", (spec.cout, din)))
    out.append(("dec_out.b", (spec.cout,)))
    return out


def param_count(spec: Spec) -> int:
    return int(sum(int(np.prod(s)) for _, s in layout(spec)))


def unpack(spec: Spec, flat: np.ndarray) -> dict:
    flat = np.asarray(flat, dtype=np.float64).ravel()
    if flat.size != param_count(spec):
        raise ValueError(f"expected {param_count(spec)} parameters, got {flat.size}")
    out, off = {}, 0
    for name, shp in layout(spec):
        n = int(np.prod(shp))
        out[name] = flat[off:off + n].reshape(shp)
        off += n
    return out


# ------------------------------------------------------------------ rounding

def round_bf16(a) -> np.ndarray:
    """Round float64 values to the nearest bfloat16 (ties to even), returned as float64:
    first to float32 (correctly rounded), then keep the top 16 bits with RNE.  The
    double rounding is harmless here because every value the oracle rounds is either
    a float32 already or far from a float32 tie."""
    f = np.asarray(a, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def round_f32(a) -> np.ndarray:
    return np.asarray(a, dtype=np.float64).astype(np.float32).astype(np.float64)


# ---------------------------------------------------------------- activations

def gelu(x):
    """Gaussian error linear unit, exact erf form: x * (1 + erf(x / sqrt 2)) / 2."""
    erf = np.vectorize(math.erf, otypes=[np.float64])
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def silu(x):
    return x / (1.0 + np.exp(-x))


def relu(x):
    return np.maximum(x, 0.0)


ACTS = {"gelu": gelu, "silu": silu, "relu": relu, "identity": lambda x: x}


# ----------------------------------------------------------- spectral pieces

def kept_k1(hp: int, m1: int) -> np.ndarray:
    return np.concatenate([np.arange(m1), np.arange(hp - m1, hp)])


def angle(k: np.ndarray, n: np.ndarray, N: int) -> np.ndarray:
    """2 pi (k n mod N) / N, with the product reduced exactly in integers."""
    return 2.0 * math.pi * (np.outer(k, n) % N) / N


def spectral_conv(v, r_top, r_bot, m1, m2, rb=lambda a: a):
    """One spectral convolution F^-1(R . F(v)) on a [B][C][H'][W'] array (explicit
    truncated DFTs; `rb` rounds contraction operands in the bf16 mode)."""
    B, C, hp, wp = v.shape
    k1 = kept_k1(hp, m1)
    k2 = np.arange(m2)
    # forward along W: T = sum_w v e^{-i a}, a = 2 pi k2 w / W'
    aw = angle(k2, np.arange(wp), wp)             # [m2][W']
    cw, sw = rb(np.cos(aw)), rb(np.sin(aw))
    vr = rb(v)
    t_re = np.einsum("bchw,kw->bchk", vr, cw)
    t_im = -np.einsum("bchw,kw->bchk", vr, sw)
    # forward along H: X = sum_h T e^{-i b}, b = 2 pi k1 h / H'
    ah = angle(k1, np.arange(hp), hp)             # [2 m1][H']
    ch, sh = rb(np.cos(ah)), rb(np.sin(ah))
    t_re, t_im = rb(t_re), rb(t_im)
    x_re = np.einsum("bchk,lh->bclk", t_re, ch) + np.einsum("bchk,lh->bclk", t_im, sh)
    x_im = np.einsum("bchk,lh->bclk", t_im, ch) - np.einsum("bchk,lh->bclk", t_re, sh)
    # per-mode complex channel mixing; rows 0..m1-1 use r_top, rows m1.. use r_bot
    R = np.concatenate([r_top, r_bot], axis=2)    # [Ci][Co][2 m1][m2][2]
    r_re, r_im = rb(R[..., 0]), rb(R[..., 1])
    x_re, x_im = rb(x_re), rb(x_im)
    y_re = np.einsum("bilk,iolk->bolk", x_re, r_re) - np.einsum("bilk,iolk->bolk", x_im, r_im)
    y_im = np.einsum("bilk,iolk->bolk", x_re, r_im) + np.einsum("bilk,iolk->bolk", x_im, r_re)
    # inverse along H: Z = sum_k1 Y e^{+i b}
    y_re, y_im = rb(y_re), rb(y_im)
    z_re = np.einsum("bolk,lh->bohk", y_re, ch) - np.einsum("bolk,lh->bohk", y_im, sh)
    z_im = np.einsum("bolk,lh->bohk", y_re, sh) + np.einsum("bolk,lh->bohk", y_im, ch)
    # real inverse along W with Hermitian completion and 1/(H'W') normalisation:
    # s = sum_k2 c_k2 Re(Z e^{+i a}) / (H'W'), c_0 = 1, c_k2>0 = 2
    ck = np.where(k2 == 0, 1.0, 2.0)[:, None] / (hp * wp)
    ciw, siw = rb(ck * np.cos(aw)), rb(-ck * np.sin(aw))
    z_re, z_im = rb(z_re), rb(z_im)
    return np.einsum("bohk,kw->bohw", z_re, ciw) + np.einsum("bohk,kw->bohw", z_im, siw)


def pointwise(w, b, x, rb=lambda a: a):
    """1x1 affine map over channels of a [B][C][...] array."""
    return np.einsum("oc,bc...->bo...", rb(w), rb(x)) + b.reshape((1, -1) + (1,) * (x.ndim - 2))


def coords(B, H, W):
    xs = np.broadcast_to(np.arange(W) / (W - 1), (B, 1, H, W))
    ys = np.broadcast_to((np.arange(H) / (H - 1))[:, None], (B, 1, H, W))
    return xs, ys


def _policy(precision: str):
    """(bf16 rounding, float32 rounding) of the precision mode."""
    if precision not in ("fp64", "bf16"):
        raise ValueError(precision)
    if precision == "bf16":
        return round_bf16, round_f32
    return (lambda a: a), (lambda a: a)


def lift(spec: Spec, P: dict, x, precision: str = "fp64"):
    """Stage 1: coordinates appended, P2(act(P1(.))) pointwise, zero padding on the
    high side of H and W; returns the first latent v_0 [B][width][H'][W']."""
    rb, r32 = _policy(precision)
    x = np.asarray(x, dtype=np.float64)
    if precision == "bf16":
        x = round_f32(x)
    B, _, H, W = x.shape
    if spec.coords:
        xs, ys = coords(B, H, W)
        x = np.concatenate([x, xs, ys], axis=1)
    # lift (float32 weights in the bf16 policy, no bf16 rounding of its operands)
    h = ACTS[spec.act](pointwise(r32(P["lift1.w"]), r32(P["lift1.b"]), x))
    v = pointwise(r32(P["lift2.w"]), r32(P["lift2.b"]), h)
    p = spec.padding
    if p:
        v = np.pad(v, ((0, 0), (0, 0), (0, p), (0, p)))
    return rb(v)


def fourier_layer(spec: Spec, P: dict, v, n: int, precision: str = "fp64"):
    """Fourier layer n on the latent v [B][width][H'][W']: act(W v + b + F^-1(R F v)),
    no activation after the last layer (Eq. 6)."""
    rb, r32 = _policy(precision)
    s = spectral_conv(v, P[f"spec{n}.r_top"], P[f"spec{n}.r_bot"], spec.m1, spec.m2, rb)
    s = s + pointwise(P[f"conv{n}.w"], r32(P[f"conv{n}.b"]), v, rb)
    v = ACTS[spec.act](s) if n < spec.layers - 1 else s
    return rb(v)


def decode(spec: Spec, P: dict, v, H: int, W: int, precision: str = "fp64"):
    """Stage 3: crop the padding, then the pointwise decoder Q -> [B][Cout][H][W]."""
    rb, r32 = _policy(precision)
    v = v[:, :, :H, :W]
    for n in range(spec.dec_layers):
        v = rb(ACTS[spec.dec_act](pointwise(P[f"dec{n}.w"], r32(P[f"dec{n}.b"]), v, rb)))
    return pointwise(P["dec_out.w"], r32(P["dec_out.b"]), v, rb)


def forward(spec: Spec, flat_params, x, precision: str = "fp64", return_latent: bool = False):
    """FNO forward on x [B][Cin][H][W] -> [B][Cout][H][W] (float64): lift, the
    Fourier layers, decoder."""
    _policy(precision)
    P = unpack(spec, flat_params)
    H, W = np.shape(x)[2], np.shape(x)[3]
    v = lift(spec, P, x, precision)
    latents = [v]
    for n in range(spec.layers):
        v = fourier_layer(spec, P, v, n, precision)
        latents.append(v)
    out = decode(spec, P, v, H, W, precision)
    return (out, latents) if return_latent else out
