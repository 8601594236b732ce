"""GPU adjoint of the lattice step and the checkpointed differentiable rollout,
against the FP64 oracle's adjoint (itself pinned by central finite differences)."""
import numpy as np
import pytest

from oracle import lbm as olbm
from paper_2604_27158_amd import workloads as W
from tests.helpers import rel_l2

pytestmark = pytest.mark.gpu


def small_lattice(nx=64, ny=48, g=2e-5):
    return W.Lattice(nx=nx, ny=ny, tau=0.75, gx=g, gy=-g / 3, bc_x=W.BC_PERIODIC, bc_y=W.BC_WALL,
                     shapes=[W.circle(nx // 3, ny // 2, 5), W.circle(2 * nx // 3, ny // 4, 3)],
                     wrap_x=True, wrap_y=False)


def test_adjoint_step_matches_oracle(gpu):
    import torch
    lat = small_lattice()
    O = olbm.Sim(lat).init(*W.random_macro_fields(1, lat.nx, lat.ny)).run(20)
    f = O.f.astype(np.float32)
    lam = W.random_array(2, f.shape).astype(np.float32) * (O.mask == 0)
    ref = olbm.adjoint_step(lat, O.mask, f.astype(np.float64), lam.astype(np.float64))
    G = gpu.Lattice.from_workload(lat)
    out = G.adjoint_step(torch.from_numpy(f).cuda(), torch.from_numpy(lam).cuda()).cpu().numpy()
    fl = np.repeat((O.mask == 0)[None], 9, 0)
    e = rel_l2(out[fl], ref[fl])
    print(f"adjoint step rel-L2 vs FP64 oracle: {e:.2e}")
    assert e < 1e-6
    assert np.all(out[~fl] == 0)


def rollout_case(gpu, lat, nsteps, ckpt, seed=3):
    import torch
    from paper_2604_27158_amd.adjoint import rollout
    rho0, ux0, uy0 = W.random_macro_fields(seed, lat.nx, lat.ny)
    tgt = W.random_macro_fields(seed + 1, lat.nx, lat.ny)
    G = gpu.Lattice.from_workload(lat)
    mask = olbm.raster(lat.nx, lat.ny, lat.shapes_array(), lat.wrap_x, lat.wrap_y)
    fl = torch.from_numpy(mask == 0).cuda()
    x = [torch.tensor(a, dtype=torch.float32, device="cuda", requires_grad=True) for a in (rho0, ux0, uy0)]
    r, u, v = rollout(G, *x, nsteps=nsteps, ckpt_every=ckpt)
    t = [torch.tensor(a, dtype=torch.float32, device="cuda") for a in tgt]
    n = 3.0 * fl.sum()
    loss = (((r - t[0]) ** 2 + (u - t[1]) ** 2 + (v - t[2]) ** 2) * fl).sum() / n
    loss.backward()
    grads = [xx.grad.detach().cpu().numpy().astype(np.float64) for xx in x]
    return (rho0, ux0, uy0), tgt, mask, float(loss), grads


def test_rollout_gradient_matches_oracle(gpu):
    """32x32 with walls, obstacles and a body force, 120 steps, checkpoints every 50
    (a ragged last segment): gradient w.r.t. the initial fields vs the FP64 oracle."""
    lat = small_lattice(32, 32, 3e-6)
    init, tgt, mask, loss, g = rollout_case(gpu, lat, 120, 50)
    ref = olbm.rollout_grad(lat, mask, *init, 120, tgt)
    lref = olbm.rollout_loss(lat, mask, *init, 120, tgt)
    fl = mask == 0
    errs = [rel_l2(a[fl], b[fl]) for a, b in zip(g, ref)]
    print(f"loss gpu {loss:.8e} oracle {lref:.8e}; grad rel-L2 rho {errs[0]:.2e} ux {errs[1]:.2e} uy {errs[2]:.2e}")
    assert abs(loss - lref) <= 1e-5 * lref
    assert max(errs) < 1e-5


def test_checkpoint_interval_does_not_change_gradient(gpu):
    lat = small_lattice(40, 24)
    _, _, _, _, g1 = rollout_case(gpu, lat, 90, 50)
    _, _, _, _, g2 = rollout_case(gpu, lat, 90, 7)
    for a, b in zip(g1, g2):
        assert np.array_equal(a, b)


def test_full_size_rollout_directional_derivative(gpu):
    """512x256 channel with 40 obstacles, 200 steps, checkpoints every 50: <grad, d>
    from the GPU adjoint vs FP64 central differences (h = 1e-6) of the oracle loss."""
    lat = W.channel_walls_circles(4, nx=512, ny=256, n_circles=40, rmin=6, rmax=14, tau=0.8, g=1e-6)
    init, tgt, mask, loss, g = rollout_case(gpu, lat, 200, 50, seed=8)
    rng = np.random.default_rng(0)
    d = [rng.standard_normal(mask.shape) * (mask == 0) for _ in range(3)]
    h = 1e-6
    lp = olbm.rollout_loss(lat, mask, *[a + h * b for a, b in zip(init, d)], 200, tgt)
    lm = olbm.rollout_loss(lat, mask, *[a - h * b for a, b in zip(init, d)], 200, tgt)
    fd = (lp - lm) / (2 * h)
    an = sum(float(np.sum(a * b)) for a, b in zip(g, d))
    print(f"directional derivative: GPU adjoint {an:.8e}, FP64 central difference {fd:.8e}")
    assert abs(an - fd) <= 1e-4 * abs(fd)


def zouhe_lattice(nx=48, ny=24):
    return W.Lattice(nx=nx, ny=ny, tau=0.7, bc_x=W.BC_ZOUHE, bc_y=W.BC_PERIODIC, u_in=0.03,
                     rho_out=1.01, shapes=[W.circle(nx // 2, ny // 2, 4), W.circle(nx // 5, ny // 4, 2)],
                     wrap_x=False, wrap_y=True)


def test_adjoint_step_through_zouhe_columns_matches_oracle(gpu):
    """One step's adjoint on a lattice with Zou-He inlet and outlet columns (the
    closures' transposed Jacobian applied where lam_{n+1} is read), vs the FP64 oracle."""
    import torch
    lat = zouhe_lattice()
    O = olbm.Sim(lat).init(*W.random_macro_fields(5, lat.nx, lat.ny, amp_u=0.03)).run(15)
    f = O.f.astype(np.float32)
    lam = W.random_array(6, f.shape).astype(np.float32) * (O.mask == 0)
    ref = olbm.adjoint_step(lat, O.mask, f.astype(np.float64), lam.astype(np.float64))
    G = gpu.Lattice.from_workload(lat)
    out = G.adjoint_step(torch.from_numpy(f).cuda(), torch.from_numpy(lam).cuda()).cpu().numpy()
    fl = np.repeat((O.mask == 0)[None], 9, 0)
    e = rel_l2(out[fl], ref[fl])
    edge = np.zeros_like(fl)
    edge[:, :, :2] = edge[:, :, -2:] = True
    e_edge = rel_l2(out[fl & edge], ref[fl & edge])
    print(f"Zou-He adjoint step rel-L2 vs FP64 oracle: {e:.2e} (boundary columns {e_edge:.2e})")
    assert e < 1e-6 and e_edge < 1e-6
    assert np.all(out[~fl] == 0)


def test_rollout_gradient_through_zouhe_columns_matches_oracle(gpu):
    """Checkpointed rollout (80 steps, checkpoints every 30) on a Zou-He lattice:
    gradient w.r.t. the initial fields, through the closures of every step and of
    the initial equilibrium, vs the FP64 oracle."""
    lat = zouhe_lattice(40, 20)
    init, tgt, mask, loss, g = rollout_case(gpu, lat, 80, 30, seed=9)
    ref = olbm.rollout_grad(lat, mask, *init, 80, tgt)
    lref = olbm.rollout_loss(lat, mask, *init, 80, tgt)
    fl = mask == 0
    errs = [rel_l2(a[fl], b[fl]) for a, b in zip(g, ref)]
    print(f"Zou-He rollout: loss gpu {loss:.8e} oracle {lref:.8e}; grad rel-L2 " +
          " ".join(f"{x:.2e}" for x in errs))
    assert abs(loss - lref) <= 1e-5 * lref
    assert max(errs) < 1e-5


def test_fno_gradient_through_the_lattice_matches_oracle_chain(gpu):
    """FNO -> equilibrium hand-off -> 60 lattice steps (checkpoints every 25) -> MSE
    against a lattice target: the FNO parameter gradient from the GPU chain (lattice
    adjoint, then the FNO backward kernels) against the FP64 oracle chain (oracle
    rollout adjoint, then the straight-through bf16 oracle's vector-Jacobian product)."""
    import torch
    from oracle import fno as ofno, fno_grad
    from paper_2604_27158_amd import fno as gfno
    from paper_2604_27158_amd.adjoint import fno_through_lattice
    H = Wd = 32
    lat = W.Lattice(nx=Wd, ny=H, tau=0.8, bc_x=W.BC_PERIODIC, bc_y=W.BC_WALL,
                    shapes=[W.circle(12, 14, 4)], wrap_x=True, wrap_y=False)
    spec = W.FnoSpec(cin=4, width=8, layers=1, m1=4, m2=4, dec_layers=1, dec_size=8, cout=3, padding=2)
    ospec = ofno.Spec(cin=4, width=8, layers=1, m1=4, m2=4, dec_layers=1, dec_size=8, cout=3, padding=2)
    params = 0.2 * W.fno_random_params(5, gfno.param_layout(spec), spec.width)
    mask = olbm.raster(lat.nx, lat.ny, lat.shapes_array(), lat.wrap_x, lat.wrap_y)
    r0, u0, v0 = W.random_macro_fields(6, Wd, H)
    x = np.stack([r0 - 1.0, u0, v0, mask.astype(np.float64)])[None]
    tgt = np.stack(olbm.Sim(lat, mask).init(r0, u0, v0).run(60).macros())
    n = 60
    # GPU chain
    model = gfno.Fno(spec, params, H, Wd)
    tr = gfno.Trainer(model, params)
    G = gpu.Lattice.from_workload(lat)
    loss, g = fno_through_lattice(tr, torch.from_numpy(x).float().cuda(), G, n,
                                  torch.from_numpy(tgt).float().cuda(), ckpt_every=25)
    g = g.cpu().numpy().astype(np.float64)
    # oracle chain; the oracle's loss is the mean over fluid nodes, the library's over
    # all nodes (solids agree exactly), so both are scaled to the latter
    y = ofno.forward(ospec, params, x, "bf16")[0]
    scale = float((mask == 0).sum()) / mask.size
    g_fields = [scale * a for a in olbm.rollout_grad(lat, mask, 1.0 + y[0], y[1], y[2], n, tgt)]
    lref = scale * olbm.rollout_loss(lat, mask, 1.0 + y[0], y[1], y[2], n, tgt)
    _, gref = fno_grad.vjp(ospec, params, x, np.stack(g_fields)[None], "bf16")
    e = np.linalg.norm(g - gref) / np.linalg.norm(gref)
    print(f"loss gpu {loss:.6e} oracle {lref:.6e}; parameter-gradient rel-L2 {e:.2e}")
    assert abs(loss - lref) <= 1e-2 * lref
    assert e < 2e-2


def test_training_through_the_lattice_reduces_the_loss(gpu):
    """AdamW on an FNO whose fields hand off to 40 lattice steps, against the plain
    lattice's own states from the true initial fields (4 LBM-generated samples)."""
    import torch
    from paper_2604_27158_amd import fno as gfno
    from paper_2604_27158_amd.adjoint import train_through_lattice
    H = Wd = 32
    lat = W.Lattice(nx=Wd, ny=H, tau=0.8, bc_x=W.BC_PERIODIC, bc_y=W.BC_WALL,
                    shapes=[W.circle(12, 14, 4)], wrap_x=True, wrap_y=False)
    spec = W.FnoSpec(cin=4, width=8, layers=1, m1=4, m2=4, dec_layers=1, dec_size=8, cout=3, padding=2)
    params = 0.2 * W.fno_random_params(9, gfno.param_layout(spec), spec.width)
    tr = gfno.Trainer(gfno.Fno(spec, params, H, Wd), params, lr=3e-3, weight_decay=0.0)
    G = gpu.Lattice.from_workload(lat)
    mask = olbm.raster(lat.nx, lat.ny, lat.shapes_array(), lat.wrap_x, lat.wrap_y)
    samples = []
    for s in range(4):
        r0, u0, v0 = W.random_macro_fields(60 + s, Wd, H)
        G.reinit(*(torch.from_numpy(a).float() for a in (r0, u0, v0)))
        G.step(40)
        tgt = G.macros().clone()
        x = torch.from_numpy(np.stack([r0 - 1.0, u0, v0, mask.astype(np.float64)])[None]).float().cuda()
        samples.append((x, tgt))
    hist = train_through_lattice(tr, samples, G, 40, epochs=30)
    print("through-lattice losses:", " ".join(f"{h:.3e}" for h in hist[::5]), f"{hist[-1]:.3e}")
    assert np.isfinite(hist).all() and hist[-1] < 0.25 * hist[0]


@pytest.mark.parametrize("lam", [0.25, 3.0 / 16])
def test_trt_adjoint_step_matches_oracle(gpu, lam):
    """The adjoint of the TRT step (forced walled lattice with obstacles, and a Zou-He
    lattice) vs the FP64 oracle's TRT adjoint, which is pinned by central differences."""
    import dataclasses
    import torch
    for lat, seed in ((small_lattice(), 11), (zouhe_lattice(), 13)):
        lat = dataclasses.replace(lat, trt_lambda=lam)
        O = olbm.Sim(lat).init(*W.random_macro_fields(seed, lat.nx, lat.ny, amp_u=0.03)).run(15)
        f = O.f.astype(np.float32)
        lamv = W.random_array(seed + 1, f.shape).astype(np.float32) * (O.mask == 0)
        ref = olbm.adjoint_step(lat, O.mask, f.astype(np.float64), lamv.astype(np.float64))
        bgk = olbm.adjoint_step(dataclasses.replace(lat, trt_lambda=0.0), O.mask, f.astype(np.float64),
                                lamv.astype(np.float64))
        G = gpu.Lattice.from_workload(lat)
        out = G.adjoint_step(torch.from_numpy(f).cuda(), torch.from_numpy(lamv).cuda()).cpu().numpy()
        fl = np.repeat((O.mask == 0)[None], 9, 0)
        e = rel_l2(out[fl], ref[fl])
        print(f"TRT {lam:g} {lat.name}: adjoint step rel-L2 vs FP64 oracle {e:.2e} "
              f"(BGK adjoint differs by {rel_l2(bgk[fl], ref[fl]):.2e})")
        assert e < 1e-6 and rel_l2(bgk[fl], ref[fl]) > 1e-4
        assert np.all(out[~fl] == 0)


def test_trt_rollout_gradient_matches_oracle(gpu):
    """Checkpointed TRT rollout (lambda = 1/4; 80 steps, checkpoints every 30) on a
    Zou-He lattice: gradient w.r.t. the initial fields vs the FP64 oracle."""
    import dataclasses
    lat = dataclasses.replace(zouhe_lattice(40, 20), trt_lambda=0.25)
    init, tgt, mask, loss, g = rollout_case(gpu, lat, 80, 30, seed=17)
    ref = olbm.rollout_grad(lat, mask, *init, 80, tgt)
    lref = olbm.rollout_loss(lat, mask, *init, 80, tgt)
    fl = mask == 0
    errs = [rel_l2(a[fl], b[fl]) for a, b in zip(g, ref)]
    print(f"TRT rollout: loss gpu {loss:.8e} oracle {lref:.8e}; grad rel-L2 " + " ".join(f"{x:.2e}" for x in errs))
    assert abs(loss - lref) <= 1e-5 * lref
    assert max(errs) < 1e-5


def test_lattice_holds_final_state_after_backward(gpu):
    """The backward pass recomputes segments from checkpoints; afterwards the lattice
    holds f(N) again, so stepping on continues the forward trajectory."""
    import torch
    from paper_2604_27158_amd.adjoint import rollout
    lat = small_lattice(32, 32, 3e-6)
    rho0, ux0, uy0 = W.random_macro_fields(8, lat.nx, lat.ny)
    G = gpu.Lattice.from_workload(lat)
    x = [torch.tensor(a, dtype=torch.float32, device="cuda", requires_grad=True) for a in (rho0, ux0, uy0)]
    r, u, v = rollout(G, *x, nsteps=70, ckpt_every=30)
    want = G.populations().clone()
    (r.sum() + u.sum() + v.sum()).backward()
    assert torch.equal(G.populations(), want)
    G.step(10)
    P = gpu.Lattice.from_workload(lat)
    P.reinit(*(torch.from_numpy(a).float() for a in (rho0, ux0, uy0)))
    P.step(80)
    assert torch.equal(G.populations(), P.populations())
