"""Pins of the FP64 FNO oracle: the paper's printed parameter counts, numpy.fft's
real 2-D transforms, special cases with known outputs, symmetry, and torch's
bfloat16 conversion for the rounding helper."""
import math

import numpy as np
import pytest
import torch

from oracle import fno
from paper_2604_27158_amd import workloads as W


# (cin, width, layers, modes, dec_layers, dec_size, cout) -> count printed in the paper
PRINTED = [
    ((1, 16, 3, 6, 3, 32, 1), 114273),     # porous density model table
    ((1, 16, 6, 12, 3, 64, 2), 896082),    # porous velocity model table
    ((1, 14, 3, 8, 1, 32, 1), 151811),     # shear density model, 3 layers / 8 modes
    ((1, 14, 7, 32, 1, 32, 1), 5621835),   # shear density model, 7 layers / 32 modes
    ((2, 14, 3, 32, 1, 32, 2), 2409771),   # shear velocity model, 3 layers
    ((2, 14, 7, 32, 1, 32, 2), 5621875),   # shear velocity model, 7 layers
]


@pytest.mark.parametrize("args,count", PRINTED)
def test_param_count_matches_paper_tables(args, count):
    cin, wd, L, m, dl, ds, co = args
    spec = fno.Spec(cin=cin, width=wd, layers=L, m1=m, m2=m, dec_layers=dl, dec_size=ds, cout=co)
    assert fno.param_count(spec) == count


def test_shear_group_totals():
    """The two model groups sum to the printed 11 243 710 and 2 561 582."""
    assert 5621835 + 5621875 == 11243710 and 151811 + 2409771 == 2561582


def test_flagship_count():
    assert fno.param_count(fno.Spec()) == 2365331


def _rand(shape, seed):
    return W.random_array(seed, shape)


@pytest.mark.parametrize("H,Wd,m1,m2", [(16, 16, 4, 5), (12, 20, 3, 6), (32, 64, 12, 12)])
def test_spectral_conv_equals_numpy_rfft2(H, Wd, m1, m2):
    """F^-1(R . F(v)) equals numpy's rfft2 -> keep modes -> multiply -> irfft2."""
    B, C = 2, 3
    v = _rand((B, C, H, Wd), 1)
    rt = _rand((C, C, m1, m2, 2), 2)
    rbt = _rand((C, C, m1, m2, 2), 3)
    got = fno.spectral_conv(v, rt, rbt, m1, m2)
    X = np.fft.rfft2(v)                          # [B][C][H][W/2+1]
    Y = np.zeros((B, C, H, Wd // 2 + 1), complex)
    top = rt[..., 0] + 1j * rt[..., 1]
    bot = rbt[..., 0] + 1j * rbt[..., 1]
    Y[:, :, :m1, :m2] = np.einsum("bixy,ioxy->boxy", X[:, :, :m1, :m2], top)
    Y[:, :, H - m1:, :m2] = np.einsum("bixy,ioxy->boxy", X[:, :, H - m1:, :m2], bot)
    ref = np.fft.irfft2(Y, s=(H, Wd))
    assert np.max(np.abs(got - ref)) < 1e-12 * np.max(np.abs(ref))


def test_spectral_identity_on_band_limited_input():
    """R = identity on every kept mode reproduces a band-limited real input exactly.
    (In the k2 = 0 column a real input pairs k1 with -k1, so the lowest negative row
    H - m1, whose partner m1 is not kept, stays empty.)"""
    H, Wd, m1, m2, C = 16, 24, 4, 5, 3
    X = np.zeros((1, C, H, Wd // 2 + 1), complex)
    rng = np.random.default_rng(0)
    for k1 in list(range(m1)) + list(range(H - m1, H)):
        for k2 in range(m2):
            if k2 == 0 and k1 == H - m1:
                continue
            X[0, :, k1, k2] = rng.standard_normal(C) + 1j * rng.standard_normal(C)
    v = np.fft.irfft2(X, s=(H, Wd))
    eye = np.zeros((C, C, m1, m2, 2))
    for i in range(C):
        eye[i, i, :, :, 0] = 1.0
    got = fno.spectral_conv(v, eye, eye, m1, m2)
    assert np.max(np.abs(got - v)) < 1e-13


def test_translation_equivariance_without_coordinates():
    """Without coordinate channels and padding every piece is shift-equivariant:
    FNO(roll(x)) = roll(FNO(x)) for circular shifts."""
    spec = fno.Spec(cin=2, width=8, layers=2, m1=3, m2=4, cout=2, coords=False)
    p = W.fno_random_params(5, fno.layout(spec), spec.width)
    x = _rand((1, 2, 16, 20), 6)
    y = fno.forward(spec, p, x)
    ys = fno.forward(spec, p, np.roll(x, (3, -5), axis=(2, 3)))
    assert np.max(np.abs(ys - np.roll(y, (3, -5), axis=(2, 3)))) < 1e-12 * np.max(np.abs(y))


def test_inverse_drops_imaginary_part_of_k2_zero_column():
    """Real inverse semantics: an imaginary value placed only in the k2 = 0 column
    contributes nothing (numpy.fft.irfft2 does the same)."""
    H, Wd, C = 8, 8, 1
    rng = np.random.default_rng(3)
    # a spectral weight that maps X to i X only on mode (k1=1, k2=0)
    rt = np.zeros((C, C, 2, 2, 2)); rt[0, 0, 1, 0, 1] = 1.0
    rbt = np.zeros_like(rt)
    v = rng.standard_normal((1, C, H, Wd))
    got = fno.spectral_conv(v, rt, rbt, 2, 2)
    X = np.fft.rfft2(v)
    Y = np.zeros_like(X); Y[0, 0, 1, 0] = 1j * X[0, 0, 1, 0]
    ref = np.fft.irfft2(Y, s=(H, Wd))
    assert np.max(np.abs(got - ref)) < 1e-14


def test_gelu_erf_values():
    """GELU(x) = x Phi(x): Phi(1) = 0.8413447460685429, Phi(-1) = 0.15865525393145707."""
    x = np.array([1.0, -1.0, 0.0, 3.0])
    g = fno.gelu(x)
    assert abs(g[0] - 0.8413447460685429) < 1e-15
    assert abs(g[1] + 0.15865525393145707) < 1e-15
    assert g[2] == 0.0 and abs(g[3] - 3.0 * 0.9986501019683699) < 1e-14


def test_round_bf16_matches_torch():
    rng = np.random.default_rng(7)
    x = np.concatenate([rng.standard_normal(4000) * 10 ** rng.uniform(-6, 6, 4000),
                        [0.0, 1.0, -2.5, 1.00390625, 1.01171875]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(fno.round_bf16(x.astype(np.float64)), ref)


def test_bf16_mode_close_to_fp64():
    """The bf16 operand-rounding mode stays within bf16 accuracy of the fp64 mode
    (relative L2 ~ 1e-2 for four layers)."""
    spec = fno.Spec(cin=4, width=16, layers=2, m1=4, m2=4, dec_size=16)
    p = W.fno_random_params(9, fno.layout(spec), spec.width)
    x = _rand((1, 4, 16, 32), 10)
    a = fno.forward(spec, p, x, "fp64")
    b = fno.forward(spec, p, x, "bf16")
    rel = np.linalg.norm(a - b) / np.linalg.norm(a)
    assert 1e-5 < rel < 3e-2


def _torch_fno(spec, flat, x):
    """The same network assembled from torch library routines in float64:
    conv2d 1x1 for every pointwise map (weights [out][in]), F.pad for the zero
    padding on the high side of H and W after the lift (cropped before the
    decoder), torch.fft.rfft2/irfft2 for the spectral part, F.gelu (erf form) /
    F.silu for the activations."""
    import torch.nn.functional as F
    P = {k: torch.from_numpy(np.ascontiguousarray(v)) for k, v in fno.unpack(spec, flat).items()}
    t = torch.from_numpy(x)
    B, _, H, Wd = t.shape
    xs = torch.linspace(0, 1, Wd, dtype=torch.float64).expand(B, 1, H, Wd)
    ys = torch.linspace(0, 1, H, dtype=torch.float64)[:, None].expand(B, 1, H, Wd)
    t = torch.cat([t, xs, ys], 1)
    conv = lambda w, b, a: F.conv2d(a, w[:, :, None, None], b)
    t = conv(P["lift2.w"], P["lift2.b"], F.gelu(conv(P["lift1.w"], P["lift1.b"], t)))
    pad = spec.padding
    t = F.pad(t, (0, pad, 0, pad))
    H, Wd = H + pad, Wd + pad
    for n in range(spec.layers):
        X = torch.fft.rfft2(t)
        Y = torch.zeros_like(X)
        top = torch.view_as_complex(P[f"spec{n}.r_top"].contiguous())
        bot = torch.view_as_complex(P[f"spec{n}.r_bot"].contiguous())
        m1, m2 = spec.m1, spec.m2
        Y[:, :, :m1, :m2] = torch.einsum("bixy,ioxy->boxy", X[:, :, :m1, :m2], top)
        Y[:, :, H - m1:, :m2] = torch.einsum("bixy,ioxy->boxy", X[:, :, H - m1:, :m2], bot)
        t = torch.fft.irfft2(Y, s=(H, Wd)) + conv(P[f"conv{n}.w"], P[f"conv{n}.b"], t)
        if n < spec.layers - 1:
            t = F.gelu(t)
    t = t[:, :, :H - pad, :Wd - pad]
    for n in range(spec.dec_layers):
        t = F.silu(conv(P[f"dec{n}.w"], P[f"dec{n}.b"], t))
    return conv(P["dec_out.w"], P["dec_out.b"], t).numpy()


@pytest.mark.parametrize("padding", [0, 9, 4])
def test_forward_equals_torch_library_composition(padding):
    """Also pins the padding (9 in every model of the paper's tables): zeros on the
    high side of both axes after the lift, cropped before the decoder."""
    spec = fno.Spec(cin=4, width=8, layers=3, m1=3, m2=4, dec_layers=2, dec_size=6, cout=3,
                    padding=padding)
    p = W.fno_random_params(21, fno.layout(spec), spec.width)
    x = _rand((2, 4, 12, 20), 22)
    a = fno.forward(spec, p, x)
    b = _torch_fno(spec, p, x)
    assert np.max(np.abs(a - b)) < 1e-12 * np.max(np.abs(b))
