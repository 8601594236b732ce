"""GPU parity of FNO training: the backward pass (fno_backward), the loss
(fno_mse), AdamW (fno_adamw) and the device weight refresh (fno_set_params).

Gradient references, both float64 autograd of the oracle's forward:
  "bf16"  straight-through: the GPU forward's bfloat16 rounding points, rounding
          treated as the identity in the backward.  What is left is the GPU
          backward's own bfloat16 operands (per Fourier layer: the pre-activation
          gradient, its row transform, the conjugate-mixed coefficients and the
          column-inverse coefficients, four roundings of relative RMS
          2^-9 / sqrt(3) ~ 1.1e-3 each) plus the forward's accumulation-order flips.
          Over up to 6 layers in quadrature that is at most ~6e-3 relative L2 for
          the whole gradient (measured 1e-4 to 1e-3 on these shapes); bar 5e-3,
          and 5e-2 for any single parameter tensor (the smaller groups average
          fewer independent roundings; measured up to 1.3e-2);
  "fp64"  the exact gradient; reported, bound 8e-2."""
import zlib

import numpy as np
import pytest

from oracle import fno as ofno
from oracle import fno_grad
from paper_2604_27158_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_ALL = 5e-3
TOL_GROUP = 5e-2
TOL_FP64 = 8e-2


def ospec(s):
    return ofno.Spec(cin=s.cin, width=s.width, layers=s.layers, m1=s.m1, m2=s.m2,
                     dec_layers=s.dec_layers, dec_size=s.dec_size, cout=s.cout, padding=s.padding,
                     coords=s.coords, act=s.act, dec_act=s.dec_act)


def rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


CASES = [
    # (name, spec, H, W, B)
    ("flagship-w32-L4-m12", W.FnoSpec(), 64, 64, 2),
    # the flagship at its own 256 x 128 grid
    ("flagship-128x256", W.FnoSpec(), 128, 256, 1),
    ("porous-rho-paper", W.FnoSpec(cin=1, width=16, layers=3, m1=6, m2=6, dec_layers=3, dec_size=32,
                                   cout=1, padding=9), 64, 128, 1),
    ("ragged-50x70-w64", W.FnoSpec(cin=3, width=64, layers=2, m1=5, m2=7, dec_layers=2, dec_size=48,
                                   cout=3, padding=3, act="relu", dec_act="gelu"), 50, 70, 2),
    ("no-coords-dec0-w14", W.FnoSpec(cin=2, width=14, layers=2, m1=5, m2=4, dec_layers=0, dec_size=0,
                                     cout=2, padding=2, coords=False), 30, 40, 3),
]


def problem(name, spec, H, Wd, B):
    from paper_2604_27158_amd import fno as gfno
    seed = zlib.crc32(name.encode()) & 0xFFFF
    params = W.fno_random_params(seed, gfno.param_layout(spec), spec.width)
    x = np.stack([np.stack([W.random_array(seed + 10 * b + c, (H, Wd)) * 0.5 for c in range(spec.cin)])
                  for b in range(B)])
    tgt = np.stack([np.stack([W.random_array(seed + 1000 + 10 * b + c, (H, Wd)) * 0.2
                              for c in range(spec.cout)]) for b in range(B)])
    return params, x, tgt


def gpu_loss_grad(spec, params, x, tgt, H, Wd):
    import torch
    from paper_2604_27158_amd import fno as gfno
    model = gfno.Fno(spec, params, H, Wd)
    tr = gfno.Trainer(model, params)
    xt = torch.from_numpy(x.astype(np.float32)).cuda()
    tt = torch.from_numpy(tgt.astype(np.float32)).cuda()
    out = tr.forward(xt)
    loss, dout = tr.mse(out, tt)
    g = tr.backward(xt, dout).cpu().numpy().astype(np.float64)
    return loss, g, out.cpu().numpy().astype(np.float64), tr, xt, tt


@pytest.mark.parametrize("name,spec,H,Wd,B", CASES, ids=[c[0] for c in CASES])
def test_fno_gradient_parity(gpu, name, spec, H, Wd, B):
    params, x, tgt = problem(name, spec, H, Wd, B)
    loss, g, out, *_ = gpu_loss_grad(spec, params, x, tgt, H, Wd)
    os_ = ospec(spec)
    loss_bf, g_bf, out_bf = fno_grad.loss_and_grad(os_, params, x.astype(np.float32), tgt.astype(np.float32), "bf16")
    loss_64, g_64, _ = fno_grad.loss_and_grad(os_, params, x, tgt, "fp64")
    e_all, e_64 = rel(g, g_bf), rel(g, g_64)
    worst = max(((rel(g[sl], g_bf[sl]), n) for n, sl in fno_grad.group_slices(os_).items()))
    print(f"{name}: loss {loss:.6e} (oracle bf16 {loss_bf:.6e}); grad rel-L2 vs straight-through "
          f"{e_all:.2e}, worst group {worst[1]} {worst[0]:.2e}; vs FP64 {e_64:.2e} "
          f"(oracle bf16 vs fp64 {rel(g_bf, g_64):.2e})")
    assert np.isfinite(g).all()
    assert abs(loss - loss_bf) <= 1e-2 * loss_bf
    assert e_all < TOL_ALL and worst[0] < TOL_GROUP and e_64 < TOL_FP64


def test_fno_backward_is_deterministic(gpu):
    name, spec, H, Wd, B = CASES[0]
    params, x, tgt = problem(name, spec, H, Wd, B)
    _, g1, _, tr, xt, tt = gpu_loss_grad(spec, params, x, tgt, H, Wd)
    out = tr.forward(xt)
    _, dout = tr.mse(out, tt)
    g2 = tr.backward(xt, dout).cpu().numpy().astype(np.float64)
    assert np.array_equal(g1, g2)


def test_fno_forward_train_equals_forward(gpu):
    import torch
    from paper_2604_27158_amd import fno as gfno
    name, spec, H, Wd, B = CASES[2]
    params, x, _ = problem(name, spec, H, Wd, B)
    m = gfno.Fno(spec, params, H, Wd)
    xt = torch.from_numpy(x.astype(np.float32)).cuda()
    y = m(xt).cpu().numpy()
    tr = gfno.Trainer(m, params)
    assert np.array_equal(tr.forward(xt).cpu().numpy(), y)


def test_fno_set_params_matches_fresh_model(gpu):
    """Weights refreshed on the device from packed parameters give bit-identical
    outputs to a model created from those parameters on the host."""
    import torch
    from paper_2604_27158_amd import fno as gfno
    name, spec, H, Wd, B = CASES[1]
    params, x, _ = problem(name, spec, H, Wd, B)
    params2 = params + 0.01 * W.random_array(77, params.shape)
    xt = torch.from_numpy(x.astype(np.float32)).cuda()
    m = gfno.Fno(spec, params, H, Wd)
    y0 = m(xt).cpu().numpy()
    tr = gfno.Trainer(m, params2)    # uploads params2 through fno_set_params
    y2 = m(xt).cpu().numpy()
    assert np.array_equal(y2, gfno.Fno(spec, params2, H, Wd)(xt).cpu().numpy())
    assert not np.array_equal(y0, y2)
    tr.p.copy_(torch.from_numpy(params.astype(np.float32)))
    m.lib.fno_set_params(m.model, tr.p.data_ptr(), None)
    assert np.array_equal(m(xt).cpu().numpy(), y0)


def test_fno_mse(gpu):
    import torch
    from paper_2604_27158_amd import fno as gfno
    name, spec, H, Wd, B = CASES[3]
    params, x, tgt = problem(name, spec, H, Wd, B)
    m = gfno.Fno(spec, params, H, Wd)
    tr = gfno.Trainer(m, params)
    out = torch.from_numpy(W.random_array(5, tgt.shape).astype(np.float32)).cuda()
    tt = torch.from_numpy(tgt.astype(np.float32)).cuda()
    loss, dout = tr.mse(out, tt)
    e32 = out.cpu().numpy() - tt.cpu().numpy()          # the difference is taken in float32
    assert loss == pytest.approx(np.mean(e32.astype(np.float64) ** 2), rel=1e-12)
    assert np.array_equal(dout.cpu().numpy(), (np.float32(2.0) * e32) / np.float32(e32.size))


def test_fno_adamw_matches_torch(gpu):
    import torch
    from paper_2604_27158_amd import lbmfno
    lib = lbmfno.load()
    n = 10007
    p0 = W.random_array(1, (n,)).astype(np.float32)
    pt = torch.from_numpy(p0.copy()).cuda()
    m = torch.zeros_like(pt)
    v = torch.zeros_like(pt)
    ref = torch.nn.Parameter(torch.from_numpy(p0.astype(np.float64)))
    opt = torch.optim.AdamW([ref], lr=3e-3, betas=(0.9, 0.99), eps=1e-8, weight_decay=0.05)
    for t in range(1, 6):
        g = W.random_array(10 + t, (n,)).astype(np.float32)
        gt = torch.from_numpy(g).cuda()
        rc = lib.fno_adamw(pt.data_ptr(), gt.data_ptr(), m.data_ptr(), v.data_ptr(), n, 3e-3, 0.9,
                           0.99, 1e-8, 0.05, t, None)
        assert rc == 0
        ref.grad = torch.from_numpy(g.astype(np.float64))
        opt.step()
    got = pt.cpu().numpy().astype(np.float64)
    want = ref.detach().numpy()
    assert np.max(np.abs(got - want)) <= 1e-5 * np.max(np.abs(want))


def test_fno_training_reduces_loss(gpu):
    import torch
    from paper_2604_27158_amd import fno as gfno
    name, spec, H, Wd, B = CASES[3]
    params, x, tgt = problem(name, spec, H, Wd, B)
    m = gfno.Fno(spec, params, H, Wd)
    tr = gfno.Trainer(m, params, lr=3e-3, weight_decay=0.0)
    xt = torch.from_numpy(x.astype(np.float32)).cuda()
    # a learnable target: a smooth function of the inputs
    tt = torch.tanh(xt[:, :spec.cout] * 1.5).contiguous()
    losses = [tr.step(xt, tt) for _ in range(60)]
    print(f"training loss {losses[0]:.4e} -> {losses[-1]:.4e}")
    assert np.isfinite(losses).all()
    assert losses[-1] < 0.2 * losses[0]


def test_fno_train_rejects_bad_arguments(gpu):
    import torch
    from paper_2604_27158_amd import fno as gfno
    name, spec, H, Wd, B = CASES[3]
    params, x, _ = problem(name, spec, H, Wd, B)
    m = gfno.Fno(spec, params, H, Wd)
    tr = gfno.Trainer(m, params)
    xt = torch.from_numpy(x.astype(np.float32)).cuda()
    out = torch.empty((B, spec.cout, H, Wd), device="cuda")
    ws = tr.workspace(B)
    assert m.lib.fno_forward_train(m.model, xt.data_ptr(), out.data_ptr(), B, ws.data_ptr(), 64, None) == -1
    assert m.lib.fno_backward(m.model, xt.data_ptr(), out.data_ptr(), B, ws.data_ptr(), ws.numel(),
                              None, None) == -1
    assert m.lib.fno_adamw(tr.p.data_ptr(), tr.g.data_ptr(), tr.m.data_ptr(), tr.v.data_ptr(), 4,
                           1e-3, 0.9, 0.999, 1e-8, 0.0, 0, None) == -1
