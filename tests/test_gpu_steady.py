"""GPU checks of the steady-initialisation path: the field-comparison kernel
against its definition, the committed surrogates' predictions, and a short
study run end to end."""
import os

import numpy as np
import pytest

from paper_2604_27158_amd import steady_init as S
from paper_2604_27158_amd import workloads as W

pytestmark = pytest.mark.gpu


def compare_reference(mask, a, ref):
    """rel-L1 of (rho = 1 + drho, ux, uy) over fluid nodes and the pressure drop
    c_s^2 (mean rho on the first column - on the last), in float64."""
    fl = ~mask.astype(bool)
    out = {}
    for k, key in enumerate(("rel_l1_rho", "rel_l1_ux", "rel_l1_uy")):
        den = np.abs((1.0 + ref[0]) if k == 0 else ref[k])[fl].sum()
        out[key] = np.abs(a[k] - ref[k])[fl].sum() / den
    def dp(f):
        c0, c1 = fl[:, 0], fl[:, -1]
        return (f[0][:, 0][c0].mean() - f[0][:, -1][c1].mean()) / 3.0
    out["dp"], out["dp_ref"] = dp(a), dp(ref)
    out["rel_dp"] = abs(out["dp"] - out["dp_ref"]) / abs(out["dp_ref"])
    return out


def test_compare_fields_matches_definition(gpu):
    import torch
    lat = S.geometry(S.TEST_SEEDS[1])
    G = gpu.Lattice.from_workload(lat)
    G.step(500)
    a = G.macros(rho_minus_one=True)
    G.step(300)
    ref = G.macros(rho_minus_one=True)
    got = G.compare(a, ref)
    mask = G.mask.cpu().numpy()
    want = compare_reference(mask, a.cpu().numpy().astype(np.float64), ref.cpu().numpy().astype(np.float64))
    for k, v in want.items():
        assert got[k] == pytest.approx(v, rel=1e-11, abs=1e-300), k
    same = G.compare(ref, ref)
    assert same["rel_l1_rho"] == 0.0 and same["rel_l1_ux"] == 0.0 and same["rel_dp"] == 0.0


@pytest.mark.skipif(not os.path.exists(S.DEFAULT_WEIGHTS), reason="trained surrogate weights not present")
def test_committed_surrogates_predict_plausible_fields(gpu):
    import torch
    init = S.SteadyInit()
    for seed in list(S.TEST_SEEDS)[:3]:
        lat = S.geometry(seed)
        G = gpu.Lattice.from_workload(lat)
        rho, ux, uy = init.predict(G)
        st = G.check_fields(rho, ux, uy)
        assert st["nonfinite"] == 0
        assert st["max_speed"] < 0.3
        # mass of the prediction within a few percent of the fluid volume at rho = 1
        assert abs(st["mass"] / st["fluid_nodes"] - 1.0) < 0.1
        # mean inflow-direction speed over the fluid has the right sign and size
        fl = (G.mask == 0)
        mean_u = float(ux[fl].mean())
        assert 0.2 * lat.u_in < mean_u < 5.0 * lat.u_in
        G.reinit(rho, ux, uy)
        G.step(223)
        assert bool(torch.isfinite(G.macros()).all())


@pytest.mark.skipif(not os.path.exists(S.DEFAULT_WEIGHTS), reason="trained surrogate weights not present")
def test_study_runs_end_to_end(gpu):
    res = S.time_to_steady_study(S.SteadyInit(), list(S.TEST_SEEDS)[:2], outputs=40)
    assert len(res["per_seed"]) == 2 and len(res["table"]) == 16
    for rec in res["per_seed"]:
        # the converged start begins far closer to its steady state than rest does
        assert rec["first_output_steady"]["rho"] < rec["first_output_lbm"]["rho"]
        assert rec["first_output_steady"]["u"] < rec["first_output_lbm"]["u"]
    assert res["seconds_per_step"] > 0 and res["seconds_fno_init"] > 0
