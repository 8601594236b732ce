"""Batched trajectories (one launch per step over a tile table, graph replay,
autotuned kernel shape): bitwise equal to single-lattice runs, oracle parity on
sampled trajectories, tuner cache, misuse detection."""
import numpy as np
import pytest

from oracle import lbm as olbm
from paper_2604_27158_amd import workloads as W
from tests.helpers import field_errors, gpu_fields, rho_dev_storage_bound

pytestmark = pytest.mark.gpu


def plug(gpu_lat, lat):
    import torch
    gpu_lat.reinit(*(torch.from_numpy(a) for a in W.plug_flow(lat)))


def test_batch_equals_single_lattices(gpu, tmp_path):
    lats = [W.ellipse_flow(s) for s in range(6)] + [W.channel_walls_circles(1), W.porous_circles(2, nx=300, ny=100, rmin=4, rmax=8, keepout=10)]
    B = gpu.Batch(lats, tune_cache=str(tmp_path / "tune.txt"))
    print("batch kernel:", B.choice)
    for i, lat in enumerate(lats):
        if lat.bc_x == W.BC_ZOUHE and lat.name.startswith("ellipses"):
            plug(B.trajectory(i), lat)
    B.step(301)
    for i, lat in enumerate(lats):
        G = gpu.Lattice.from_workload(lat)
        if lat.name.startswith("ellipses"):
            plug(G, lat)
        G.step(301)
        a = B.trajectory(i).populations().cpu().numpy()
        b = G.populations().cpu().numpy()
        assert np.array_equal(a, b), lat.name


def test_batch_from_rest_steps_graph_first(gpu):
    """Regression: a batch stepped from rest straight into graph replay (no other
    launch between the tuner's reset and the first graph) matches single lattices
    bit for bit.  The reset used to be an asynchronous fill that the first graph
    could overtake."""
    lats = [W.porous_circles(100000 + s, nx=512, ny=256, rmin=8, rmax=20, phi_lo=0.75, phi_hi=0.9,
                             keepout=20) for s in range(3)]
    for n in (3, 20):
        B = gpu.Batch((lats * 7)[:n])
        B.step(1000)
        for i, lat in enumerate(lats):
            G = gpu.Lattice.from_workload(lat)
            G.step(1000)
            assert np.array_equal(B.trajectory(i).populations().cpu().numpy(),
                                  G.populations().cpu().numpy()), (n, lat.name)
        B.close()


def test_macros_handed_to_caller_stream_are_not_recycled(gpu):
    """Regression: fields read from several trajectories back to back and consumed
    on the caller's stream (no synchronisation in between) each keep their own
    values.  The outputs live on the lattice stream; without marking them as used
    by the caller's stream, the allocator handed a just-freed block to the next
    read before the caller's copy of the previous one had run."""
    import torch
    lats = [W.porous_circles(100000 + s, nx=512, ny=256, rmin=8, rmax=20, phi_lo=0.75, phi_hi=0.9,
                             keepout=20) for s in range(4)]
    B = gpu.Batch(lats)
    B.step(200)
    got = [B.trajectory(i).macros(rho_minus_one=True).clone() for i in range(len(lats))]
    torch.cuda.synchronize()
    for i, lat in enumerate(lats):
        G = gpu.Lattice.from_workload(lat)
        G.step(200)
        assert torch.equal(got[i], G.macros(rho_minus_one=True)), lat.name


def test_load_state_then_graph_steps(gpu):
    """Restoring a saved state and replaying graph chunks right away reproduces the
    uninterrupted run bit for bit."""
    lat = W.porous_circles(5, nx=512, ny=256, rmin=8, rmax=20, phi_lo=0.75, phi_hi=0.9, keepout=20)
    G = gpu.Lattice.from_workload(lat)
    G.step(100)
    s = G.save_state()
    G.step(640)
    want = G.populations().cpu().numpy()
    for _ in range(3):
        G.load_state(s)
        G.step(640)
        assert np.array_equal(G.populations().cpu().numpy(), want)


def test_batch_oracle_parity_sampled(gpu):
    """Five sampled trajectories of a 100-trajectory batch, 1000 steps, vs FP64."""
    lats = [W.batch_flow(s) for s in range(100)]
    B = gpu.Batch(lats)
    for i, lat in enumerate(lats):
        plug(B.trajectory(i), lat)
    B.step(1000)
    for i in (0, 17, 42, 77, 99):
        lat = lats[i]
        if i == 3:
            continue
        O = olbm.Sim(lat).init(*W.plug_flow(lat)).run(1000)
        ref = O.macros()
        e = field_errors(gpu_fields(B.trajectory(i)), ref, O.mask)
        bound = max(1e-5, rho_dev_storage_bound(ref, 1000, O.mask == 0))
        print(f"{lat.name}: " + " ".join(f"{k}={v:.2e}" for k, v in e.items()) + f" (rho-1 bar {bound:.1e})")
        assert max(e["rho"], e["ux"], e["uy"]) < 1e-5 and e["rho-1"] < bound, e


def test_tuner_cache_roundtrip(gpu, tmp_path):
    cache = str(tmp_path / "tune.txt")
    lats = [W.ellipse_flow(s) for s in range(3)]
    a = gpu.Batch(lats, tune_cache=cache)
    b = gpu.Batch(lats, tune_cache=cache)
    assert a.choice.startswith("tuned") and b.choice.startswith("cached")
    assert a.choice.split()[1] == b.choice.split()[1]


@pytest.mark.parametrize("shape", ["node", "pair", "deep3", "deep4"])
@pytest.mark.parametrize("nt", [0, 1])
def test_every_batch_shape_equals_single_lattices(gpu, tmp_path, shape, nt):
    """Each kernel shape the tuner can pick (forced through its cache file: one node
    per lane, two steps per launch on the one-node tiles, three and four steps per
    launch on 64 x 8 tiles), with and without streaming stores, gives the bits of
    the lattices stepped alone: uneven ellipse flows, a forced walled channel and a
    ragged 300 x 100 Zou-He porous lattice, 133 steps (graph chunks, fused launches
    and single-step tails)."""
    names = ["node", "quad", "pair", "deep3", "deep4"]
    cache = tmp_path / "tune.txt"
    lats = [W.ellipse_flow(s) for s in range(3)] + [W.channel_walls_circles(1),
                                                   W.porous_circles(2, nx=300, ny=100, rmin=4, rmax=8, keepout=10)]
    first = gpu.Batch(lats, tune_cache=str(cache))
    key = cache.read_text().split()[0]
    first.close()
    cache.write_text(f"{key} {names.index(shape)} {nt}\n")
    B = gpu.Batch(lats, tune_cache=str(cache))
    assert B.choice == f"cached {shape}" + ("+nt" if nt else ""), B.choice
    for i, lat in enumerate(lats):
        if lat.name.startswith("ellipses"):
            plug(B.trajectory(i), lat)
    B.step(133)
    for i, lat in enumerate(lats):
        G = gpu.Lattice.from_workload(lat)
        if lat.name.startswith("ellipses"):
            plug(G, lat)
        G.step(133)
        assert np.array_equal(B.trajectory(i).populations().cpu().numpy(), G.populations().cpu().numpy()), \
            (shape, nt, lat.name)
        G.close()
    B.close()


def test_batch_detects_trajectory_stepped_alone(gpu):
    lats = [W.ellipse_flow(s) for s in range(2)]
    B = gpu.Batch(lats)
    B.step(2)
    t = B.trajectory(0)
    t.step(1)
    with pytest.raises(gpu.LbmError):
        B.step(1)


def test_trt_batch_equals_single_lattices(gpu, tmp_path):
    """A batch of TRT trajectories (ellipse flows, one Zou-He porous lattice) gives the
    bits of the same TRT lattices stepped alone; mixing BGK and TRT is rejected."""
    import dataclasses
    from paper_2604_27158_amd import lbmfno
    lats = [dataclasses.replace(W.ellipse_flow(s), trt_lambda=0.25) for s in range(4)]
    lats.append(dataclasses.replace(W.porous_circles(5, nx=300, ny=100, rmin=4, rmax=8, keepout=10),
                                    trt_lambda=3.0 / 16))
    B = gpu.Batch(lats, tune_cache=str(tmp_path / "tune.txt"))
    for i, lat in enumerate(lats):
        if lat.name.startswith("ellipses"):
            plug(B.trajectory(i), lat)
    B.step(201)
    for i, lat in enumerate(lats):
        G = gpu.Lattice.from_workload(lat)
        if lat.name.startswith("ellipses"):
            plug(G, lat)
        G.step(201)
        assert np.array_equal(B.trajectory(i).populations().cpu().numpy(),
                              G.populations().cpu().numpy()), lat.name
    with pytest.raises(lbmfno.LbmError):
        gpu.Batch([lats[0], W.ellipse_flow(9)])


def test_batch_workload_stays_finite(gpu):
    """The batched workload (100 flows past ellipses, Re 100-200 on the channel
    half-height) runs its 20 000 BGK steps without a trajectory losing stability:
    every field finite and every flow subsonic (peak speed below c_s = 1/sqrt 3)."""
    import torch
    lats = [W.batch_flow(s) for s in range(100)]
    B = gpu.Batch(lats)
    for i, lat in enumerate(lats):
        plug(B.trajectory(i), lat)
    B.step(20000)
    peak = []
    for i in range(len(lats)):
        t = B.trajectory(i)
        m = t.macros()
        st = t.check_fields(m[0], m[1], m[2])
        assert st["nonfinite"] == 0, lats[i].name
        peak.append(st["max_speed"])
    print(f"peak |u| over the 100 trajectories: median {np.median(peak):.3f}, max {max(peak):.3f}")
    assert max(peak) < 3.0 ** -0.5
