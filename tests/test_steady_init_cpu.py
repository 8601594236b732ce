"""Host logic of the steady-initialisation study: tolerance crossing, geometric
means, the exact folding of a power-of-two output scale into the decoder, and the
workload parameters (the paper's porous Reynolds number)."""
import math

import numpy as np
import pytest
import torch

from oracle import fno as ofno
from paper_2604_27158_amd import steady_init as S
from paper_2604_27158_amd import workloads as W


def errs(seq, key="rel_l1_rho"):
    return [{key: v} for v in seq]


@pytest.mark.parametrize("seq,eps,want", [
    ([1e-3, 1e-4, 1e-5, 1e-6], 1e-4, 2),        # first output at or below and staying there
    ([1e-3, 5e-5, 2e-4, 5e-5, 1e-5], 1e-4, 4),  # a dip that comes back up does not count
    ([1e-3, 1e-3, 1e-3], 1e-4, None),           # never reached
    ([1e-5, 1e-5], 1e-4, 1),                    # reached from the first output
    ([1e-5, float("nan")], 1e-4, None),         # a non-finite last value is not converged
])
def test_outputs_to_tolerance(seq, eps, want):
    assert S.outputs_to_tolerance(errs(seq), "rel_l1_rho", eps) == want


def test_geo_mean_skips_unreached():
    assert S.geo_mean([2.0, 8.0, None]) == pytest.approx(4.0)
    assert S.geo_mean([None, None]) is None


def test_pow2_scale():
    t = torch.full((10,), 0.03)
    s = S.pow2_scale(t)
    assert s == 2.0 ** round(math.log2(0.03))
    assert math.log2(s) == int(math.log2(s))


@pytest.mark.parametrize("precision", ["fp64", "bf16"])
def test_fold_output_scale_is_exact(precision):
    """scale * f(x) == f_folded(x) bit for bit for a power-of-two scale (every
    product and sum in the output layer scales exactly)."""
    spec = ofno.Spec(cin=1, width=4, layers=1, m1=2, m2=2, dec_layers=2, dec_size=5, cout=2, padding=2)
    wspec = W.FnoSpec(cin=1, width=4, layers=1, m1=2, m2=2, dec_layers=2, dec_size=5, cout=2, padding=2)
    p = W.random_array(3, (ofno.param_count(spec),))
    x = W.random_array(4, (1, 1, 10, 12))
    for scale in (2.0 ** -6, 4.0):
        a = ofno.forward(spec, S.fold_output_scale(wspec, p, scale), x, precision)
        b = scale * ofno.forward(spec, p, x, precision)
        assert np.array_equal(a, b)


def test_geometry_matches_the_paper_setup():
    lat = S.geometry(S.TEST_SEEDS[0])
    nu = (lat.tau - 0.5) / 3.0
    assert (lat.nx, lat.ny) == (512, 256)
    assert lat.u_in * lat.ny / nu == pytest.approx(50.0)          # Re on the domain height
    assert lat.bc_x == W.BC_ZOUHE and lat.bc_y == W.BC_PERIODIC
    phi = float(lat.name.split("phi")[1].split("-")[0])
    assert 0.75 <= phi <= 0.9
    assert all(s[6] >= 8 and s[6] <= 20 for s in (np.asarray(x) for x in lat.shapes))


def test_seed_sets_are_disjoint():
    tr, va, te = set(S.TRAIN_SEEDS), set(S.VAL_SEEDS), set(S.TEST_SEEDS)
    assert not (tr & va) and not (tr & te) and not (va & te)
    assert len(tr) == 1700 and len(va) == 200 and len(te) == 20
