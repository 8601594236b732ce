"""Hybrid FNO-LBM cycles on the GPU: accounting, guard and fallback, field check."""
import numpy as np
import pytest

from paper_2604_27158_amd import workloads as W

pytestmark = pytest.mark.gpu


def make(gpu, seed=1, scale=1.0):
    from paper_2604_27158_amd import fno as gfno, hybrid as H
    lat = W.ellipse_flow(seed, size=(256, 128))
    G = gpu.Lattice.from_workload(lat)
    import torch
    G.reinit(*(torch.from_numpy(a) for a in W.plug_flow(lat)))
    spec = W.FnoSpec()
    layout = gfno.param_layout(spec)
    p = W.fno_random_params(seed, layout, spec.width) * scale
    # output bias of the density channel = 1: predictions stay near rest density
    off = sum(int(np.prod(s)) for _, s in layout[:-1])
    p[off] = 1.0
    f = gfno.Fno(spec, p, lat.ny, lat.nx)
    return lat, G, f


def test_check_fields_matches_host(gpu):
    import math
    import torch
    lat, G, _ = make(gpu)
    G.step(50)
    m = G.macros()
    st = G.check_fields(m[0], m[1], m[2])
    h = m.cpu().numpy().astype(np.float64)
    mask = G.mask.cpu().numpy()
    fl = mask == 0
    assert st["nonfinite"] == 0 and st["fluid_nodes"] == int(fl.sum())
    assert abs(st["mass"] - math.fsum(h[0][fl])) < 1e-9 * st["mass"]
    assert abs(st["max_speed"] - np.sqrt(h[1] ** 2 + h[2] ** 2)[fl].max()) < 1e-7
    bad = m.clone()
    bad[1, 5, 7] = float("nan")
    bad[2, 9, 9] = float("inf")
    st2 = G.check_fields(bad[0], bad[1], bad[2])
    expect = int(fl[5, 7]) + int(fl[9, 9])
    assert st2["nonfinite"] == expect


def test_hybrid_cycles_accounting(gpu):
    from paper_2604_27158_amd import hybrid as H
    lat, G, f = make(gpu, scale=0.05)
    R = H.HybridRunner(G, f, dt_fno=100, k_fno=5, n_lbm=200,
                       guard=H.Guard(max_speed=1e30, mass_rel_tol=1e30))
    log = R.run(2)
    print(log)
    assert R.model_time == 1400
    assert log.fno_calls == 10 and log.lbm_steps == 400 and not log.fallbacks


def test_guard_falls_back_to_plain_lattice(gpu):
    """A model whose outputs overflow is rejected; the cycle then runs the
    replaced steps on the lattice, so the state equals a plain run bit for bit."""
    import torch
    from paper_2604_27158_amd import hybrid as H
    lat, G, f = make(gpu, scale=1e30)
    R = H.HybridRunner(G, f, dt_fno=100, k_fno=2, n_lbm=50)
    R.run(1)
    assert len(R.log.fallbacks) == 1 and R.log.fno_calls == 0 and R.log.lbm_steps == 250
    P = gpu.Lattice.from_workload(lat)
    P.reinit(*(torch.from_numpy(a) for a in W.plug_flow(lat)))
    P.step(250)
    assert np.array_equal(G.populations().cpu().numpy(), P.populations().cpu().numpy())


@pytest.mark.parametrize("scale,fallbacks", [(0.05, 0), (1e30, 3)])
def test_speculative_guard_equals_synchronous(gpu, scale, fallbacks):
    """The speculative runner (guard resolved one cycle later from pinned memory,
    rejected cycles undone and redone with lattice steps) leaves the same lattice
    bits and the same log as the synchronous guard: predictions accepted (a damped
    random model) and every one rejected (outputs overflow), 3 cycles each."""
    from paper_2604_27158_amd import hybrid as H
    lat, A, f = make(gpu, scale=scale)
    _, B, _ = make(gpu, scale=scale)
    guard = H.Guard(max_speed=0.35, mass_rel_tol=0.05)
    ra = H.HybridRunner(A, f, dt_fno=100, k_fno=2, n_lbm=60, guard=guard)
    rb = H.HybridRunner(B, f, dt_fno=100, k_fno=2, n_lbm=60, guard=guard, speculative=True)
    la, lb = ra.run(3), rb.run(3)
    assert len(la.fallbacks) == fallbacks
    assert (la.fno_calls, la.lbm_steps, la.fallbacks) == (lb.fno_calls, lb.lbm_steps, lb.fallbacks)
    assert ra.model_time == rb.model_time
    assert np.array_equal(A.populations().cpu().numpy(), B.populations().cpu().numpy())


def test_check_fields_async_matches_synchronous(gpu):
    import torch
    lat, G, _ = make(gpu)
    G.step(30)
    m = G.macros()
    st = G.check_fields(m[0], m[1], m[2])
    out = torch.full((4,), -1.0, dtype=torch.float64, device="cuda")
    G.check_fields_async(m[0], m[1], m[2], out)
    G.synchronize()
    h = out.cpu().tolist()
    assert h[0] == st["mass"] and h[1] == st["max_speed"] and int(h[2]) == st["nonfinite"] and h[3] == 0.0
