"""Pins of the FNO gradient oracle: its forward against oracle/fno.forward (explicit
numpy DFTs), central differences of that numpy forward's loss along random
directions and for one element of every parameter group, and the closed form of
the output-bias gradient."""
import numpy as np
import pytest

from oracle import fno as ofno
from oracle import fno_grad
from paper_2604_27158_amd import workloads as W

SPECS = [
    ("gelu-silu-pad", ofno.Spec(cin=3, width=6, layers=2, m1=3, m2=4, dec_layers=1, dec_size=5,
                                cout=2, padding=3), 14, 18),
    ("relu-gelu-dec2", ofno.Spec(cin=1, width=4, layers=3, m1=2, m2=3, dec_layers=2, dec_size=6,
                                 cout=3, padding=0, act="relu", dec_act="gelu"), 12, 10),
    ("no-coords-dec0", ofno.Spec(cin=2, width=4, layers=1, m1=2, m2=2, dec_layers=0, dec_size=0,
                                 cout=1, padding=2, coords=False), 9, 11),
]


def problem(spec, H, Wd, seed):
    n = ofno.param_count(spec)
    params = W.random_array(seed, (n,)) * 0.3
    x = W.random_array(seed + 1, (2, spec.cin, H, Wd))
    tgt = W.random_array(seed + 2, (2, spec.cout, H, Wd))
    return params, x, tgt


def np_loss(spec, params, x, tgt):
    out = ofno.forward(spec, params, x, "fp64")
    return float(np.mean((out - tgt) ** 2))


@pytest.mark.parametrize("name,spec,H,Wd", SPECS)
@pytest.mark.parametrize("precision", ["fp64", "bf16"])
def test_forward_equals_numpy_oracle(name, spec, H, Wd, precision):
    params, x, tgt = problem(spec, H, Wd, 11)
    _, _, out = fno_grad.loss_and_grad(spec, params, x, tgt, precision)
    ref = ofno.forward(spec, params, x, precision)
    tol = 1e-12 if precision == "fp64" else 1e-6   # bf16: rare one-ulp flips from sum order
    assert np.linalg.norm(out - ref) <= tol * np.linalg.norm(ref)


@pytest.mark.parametrize("name,spec,H,Wd", SPECS)
def test_directional_derivative_matches_central_difference(name, spec, H, Wd):
    params, x, tgt = problem(spec, H, Wd, 21)
    _, g, _ = fno_grad.loss_and_grad(spec, params, x, tgt)
    rng = np.random.default_rng(5)
    for _ in range(3):
        d = rng.standard_normal(params.size)
        d /= np.linalg.norm(d)
        h = 1e-5
        fd = (np_loss(spec, params + h * d, x, tgt) - np_loss(spec, params - h * d, x, tgt)) / (2 * h)
        assert abs(fd - g @ d) <= 1e-6 * (abs(fd) + 1e-3 * np.linalg.norm(g))


@pytest.mark.parametrize("name,spec,H,Wd", SPECS)
def test_every_group_matches_single_element_differences(name, spec, H, Wd):
    """One element of every parameter tensor (a wrong index, sign or dropped term in
    any single group shows here)."""
    params, x, tgt = problem(spec, H, Wd, 31)
    _, g, _ = fno_grad.loss_and_grad(spec, params, x, tgt)
    rng = np.random.default_rng(7)
    gn = np.linalg.norm(g)
    for name_, sl in fno_grad.group_slices(spec).items():
        j = sl.start + int(rng.integers(sl.stop - sl.start))
        h = 1e-5
        e = np.zeros_like(params)
        e[j] = h
        fd = (np_loss(spec, params + e, x, tgt) - np_loss(spec, params - e, x, tgt)) / (2 * h)
        assert abs(fd - g[j]) <= 1e-6 * abs(fd) + 1e-9 * gn, name_


def test_output_bias_gradient_closed_form():
    """dL/db_o = 2 sum_{b,h,w} (out - target)_o / n for L = mean squared error."""
    name, spec, H, Wd = SPECS[0]
    params, x, tgt = problem(spec, H, Wd, 41)
    loss, g, out = fno_grad.loss_and_grad(spec, params, x, tgt)
    sl = fno_grad.group_slices(spec)["dec_out.b"]
    want = 2.0 * (out - tgt).sum(axis=(0, 2, 3)) / out.size
    assert np.allclose(g[sl], want, rtol=1e-12, atol=0)
    assert loss == pytest.approx(np.mean((out - tgt) ** 2), rel=1e-14)


def test_straight_through_gradient_close_to_fp64():
    name, spec, H, Wd = SPECS[0]
    params, x, tgt = problem(spec, H, Wd, 51)
    _, g64, _ = fno_grad.loss_and_grad(spec, params, x, tgt, "fp64")
    _, gbf, _ = fno_grad.loss_and_grad(spec, params, x, tgt, "bf16")
    assert np.linalg.norm(gbf - g64) <= 3e-2 * np.linalg.norm(g64)


@pytest.mark.parametrize("name,spec,H,Wd", SPECS[:2])
def test_vjp_with_an_arbitrary_output_gradient_matches_central_differences(name, spec, H, Wd):
    """vjp(g_out) is the gradient of <g_out, FNO(x)>: central differences of the numpy
    oracle's forward along random parameter directions."""
    params, x, _ = problem(spec, H, Wd, 31)
    g_out = W.random_array(32, (2, spec.cout, H, Wd))
    _, g = fno_grad.vjp(spec, params, x, g_out)
    rng = np.random.default_rng(8)
    for _ in range(3):
        d = rng.standard_normal(params.size)
        d /= np.linalg.norm(d)
        h = 1e-5
        fp = float(np.sum(g_out * ofno.forward(spec, params + h * d, x, "fp64")))
        fm = float(np.sum(g_out * ofno.forward(spec, params - h * d, x, "fp64")))
        fd = (fp - fm) / (2 * h)
        assert abs(fd - g @ d) <= 1e-6 * (abs(fd) + 1e-3 * np.linalg.norm(g))
