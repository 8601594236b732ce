"""fno_forward_noalloc (the FNO forward on the library's static device scratch, for
callers that cannot allocate) against fno_forward with a caller workspace, called
through the C ABI: two calls in a row, the second with a smaller input, bitwise
equal outputs; a batch beyond the scratch is rejected with LBM_EINVAL."""
import ctypes

import numpy as np
import pytest

from paper_2604_27158_amd import workloads as W

pytestmark = pytest.mark.gpu


def _model(gpu, spec, H, Wd, seed):
    from paper_2604_27158_amd import fno as gfno
    params = W.fno_random_params(seed, gfno.param_layout(spec), spec.width)
    return gfno.Fno(spec, params, H, Wd)


def _noalloc(gpu, lib, model, x, B):
    import torch
    out = torch.full((B, model.spec.cout, model.H, model.W), float("nan"), device="cuda")
    s = torch.cuda.current_stream()
    rc = lib.fno_forward_noalloc(model.model, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                 ctypes.c_int32(B), ctypes.c_void_p(s.cuda_stream))
    assert rc == 0, lib.lbm_last_error().decode()
    return out


def test_noalloc_forward_equals_forward_twice_then_smaller(gpu):
    import torch
    lib = gpu.load_library()
    lib.fno_forward_noalloc.restype = ctypes.c_int
    lib.fno_forward_noalloc.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int32, ctypes.c_void_p]
    big = _model(gpu, W.FnoSpec(), 128, 256, 11)                    # flagship 4 -> 3 on 128 x 256
    small = _model(gpu, W.FnoSpec(cin=2, width=16, layers=2, m1=6, m2=6, dec_size=16, cout=2,
                                  padding=9), 40, 72, 12)          # padded, ragged grid
    cases = [(big, 3, 1), (small, 1, 2)]                            # second call: smaller input
    for model, B, seed in cases:
        g = torch.Generator().manual_seed(seed)
        x = torch.randn((B, model.spec.cin, model.H, model.W), generator=g).cuda()
        ref = model.forward(x)
        got = _noalloc(gpu, lib, model, x, B)
        torch.cuda.synchronize()
        n_bad = int((got != ref).sum())
        print(f"noalloc B={B} grid {model.H}x{model.W}: {n_bad} of {ref.numel()} outputs differ")
        assert torch.isfinite(ref).all() and n_bad == 0


def test_noalloc_rejects_batch_beyond_scratch(gpu):
    import torch
    lib = gpu.load_library()
    lib.fno_forward_noalloc.restype = ctypes.c_int
    lib.fno_forward_noalloc.argtypes = [ctypes.c_void_p] * 3 + [ctypes.c_int32, ctypes.c_void_p]
    model = _model(gpu, W.FnoSpec(), 128, 256, 13)
    n = ctypes.c_size_t()
    limit = 64 << 20
    B = 1
    while True:
        assert lib.fno_workspace_size(model.model, B, ctypes.byref(n)) == 0
        if n.value > limit:
            break
        B += 1
    x = torch.zeros((1, 4, 128, 256), device="cuda")   # never read: the size check comes first
    y = torch.zeros((1, 3, 128, 256), device="cuda")
    rc = lib.fno_forward_noalloc(model.model, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                 ctypes.c_int32(B), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    msg = lib.lbm_last_error().decode()
    print(f"B={B} needs {n.value} bytes: rc={rc} ({msg})")
    assert rc == -1 and "static scratch" in msg
    assert int(y.abs().sum()) == 0
