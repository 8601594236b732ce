"""Host logic of the unsteady hybrid study: folding the input and output
normalisation into the network's weights (checked with the FP64 oracle forward)."""
import numpy as np

from oracle import fno as ofno
from paper_2604_27158_amd import unsteady as U
from paper_2604_27158_amd import workloads as W


def test_folded_network_equals_normalised_network():
    spec = ofno.Spec()                       # the flagship 4 -> 3 model
    from paper_2604_27158_amd import fno as gfno
    p = W.fno_random_params(5, gfno.param_layout(U.SPEC), U.SPEC.width)
    s_r, s_u = 2.0 ** -6, 2.0 ** -5
    H, Wd = 24, 32
    x = np.stack([1.0 + 0.01 * W.random_array(1, (H, Wd)), 0.03 * W.random_array(2, (H, Wd)),
                  0.02 * W.random_array(3, (H, Wd)), (W.random_array(4, (H, Wd)) > 1.0).astype(float)])[None]
    xn = x.copy()
    xn[0, 0] = (x[0, 0] - 1.0) / s_r
    xn[0, 1:3] = x[0, 1:3] / s_u
    yn = ofno.forward(spec, p, xn, "fp64")
    want = yn.copy()
    want[0, 0] = 1.0 + s_r * yn[0, 0]
    want[0, 1:3] = s_u * yn[0, 1:3]
    got = ofno.forward(spec, U.fold(p, s_r, s_u), x, "fp64")
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_cadence_matches_the_configuration():
    from paper_2604_27158_amd.hybrid import step_reduction
    assert (U.NX, U.NY, U.DT_FNO, U.K_FNO, U.N_LBM, U.CYCLES) == (256, 128, 100, 5, 200, 20)
    assert abs(step_reduction(U.K_FNO, U.DT_FNO, U.N_LBM) - 500 / 700) < 1e-15
