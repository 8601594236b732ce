"""The C ABI library loads without a GPU, exports every entry point include/*.h
declares, and rejects invalid arguments on the host before any HIP call."""
import ctypes
import glob
import os
import re

import pytest

from paper_2604_27158_amd import lbmfno

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*\**\s*([a-z_][a-z0-9_]*)\s*\(",
                             txt, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    return lbmfno.load_library()


def test_header_declares_the_core_calls():
    names = declared_functions()
    for n in ("lbm_init", "lbm_step", "lbm_reinit_from_macro", "lbm_get_macro", "lbm_mask_raster"):
        assert n in names


def test_every_declared_symbol_is_exported_and_bound(lib):
    bound = {n for n, _, _ in lbmfno.SIGNATURES}
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert name in bound, f"{name} has no binding"


def _cfg(**kw):
    c = dict(nx=16, ny=8, bc_x=0, bc_y=0, tau=0.8, gx=0.0, gy=0.0, u_in=0.0, rho_out=1.0, arith=0, kernel=0,
             trt_lambda=0.0)
    c.update(kw)
    return lbmfno.LbmConfig(**c)


@pytest.mark.parametrize("kw", [dict(tau=0.5), dict(tau=float("nan")), dict(nx=0), dict(ny=-3),
                                dict(bc_x=7), dict(bc_y=2), dict(nx=30000, ny=30000),
                                dict(bc_x=2, u_in=1.5), dict(bc_x=2, rho_out=0.0),
                                dict(gx=float("inf")), dict(arith=5), dict(kernel=5),
                                dict(trt_lambda=-0.25), dict(trt_lambda=float("nan"))])
def test_lbm_init_rejects_invalid_config(lib, kw):
    ctx = ctypes.c_void_p()
    rc = lib.lbm_init(ctypes.byref(ctx), ctypes.byref(_cfg(**kw)), 1, 2, 3, None)
    assert rc == -1 and not ctx.value
    assert lib.lbm_last_error()


def test_unsupported_combinations(lib):
    ctx = ctypes.c_void_p()
    assert lib.lbm_init(ctypes.byref(ctx), ctypes.byref(_cfg(bc_x=2, gx=1e-6)), 1, 2, 3, None) == -4
    assert lib.lbm_init(ctypes.byref(ctx), ctypes.byref(_cfg(bc_x=2, bc_y=1)), 1, 2, 3, None) == -4
    # the TRT collision runs in the lean arithmetic only
    assert lib.lbm_init(ctypes.byref(ctx), ctypes.byref(_cfg(trt_lambda=0.25, arith=0)), 1, 2, 3, None) == -4


def test_null_arguments(lib):
    ctx = ctypes.c_void_p()
    assert lib.lbm_init(None, ctypes.byref(_cfg()), 1, 2, 3, None) == -1
    assert lib.lbm_init(ctypes.byref(ctx), None, 1, 2, 3, None) == -1
    assert lib.lbm_init(ctypes.byref(ctx), ctypes.byref(_cfg()), None, 2, 3, None) == -1
    assert lib.lbm_init(ctypes.byref(ctx), ctypes.byref(_cfg()), 1, 2, 2, None) == -1
    assert lib.lbm_step(None, 1, None) == -1
    assert lib.lbm_get_macro(None, 1, 2, 3, 0) == -1
    assert lib.lbm_reinit_from_macro(None, 1, 2, 3) == -1
    assert lib.lbm_reinit_from_macro_neq(None, 1, 2, 3) == -1
    assert lib.lbm_check_fields_async(None, 1, 2, 3, 4) == -1
    assert lib.lbm_reinit_from_macro_mass(None, 1, 2, 3) == -1


def test_raster_validation(lib):
    import numpy as np
    bad = np.array([[0, 0, 1 << 40, 0, 1 << 40, 5, 1 << 14]], dtype=np.int64)
    assert lib.lbm_mask_raster(8, 8, 0, 0, bad.ctypes.data_as(ctypes.c_void_p), 1, 1, None) == -1
    assert lib.lbm_mask_raster(0, 8, 0, 0, None, 0, 1, None) == -1
    assert lib.lbm_mask_raster(8, 8, 0, 0, None, 0, None, None) == -1


def test_status_strings(lib):
    for code in range(0, -7, -1):
        assert lib.lbm_status_str(code) not in (None, b"unknown status")


@pytest.mark.parametrize("args,count", [
    ((1, 16, 3, 6, 3, 32, 1), 114273), ((1, 16, 6, 12, 3, 64, 2), 896082),
    ((1, 14, 3, 8, 1, 32, 1), 151811), ((1, 14, 7, 32, 1, 32, 1), 5621835),
    ((2, 14, 3, 32, 1, 32, 2), 2409771), ((2, 14, 7, 32, 1, 32, 2), 5621875),
    ((4, 32, 4, 12, 1, 32, 3), 2365331)])
def test_fno_param_count_abi_matches_paper(lib, args, count):
    """fno_param_count (library) reproduces the paper's printed model sizes."""
    from paper_2604_27158_amd import fno as gfno, workloads as W
    cin, wd, L, m, dl, ds, co = args
    s = W.FnoSpec(cin=cin, width=wd, layers=L, m1=m, m2=m, dec_layers=dl, dec_size=ds, cout=co)
    assert gfno.param_count(s) == count
    assert sum(int(__import__("numpy").prod(sh)) for _, sh in gfno.param_layout(s)) == count


def test_fno_model_create_validates_on_host(lib):
    from paper_2604_27158_amd import fno as gfno, workloads as W
    import numpy as np
    m = ctypes.c_void_p()
    bad = W.FnoSpec(width=65)
    p = np.zeros(10, np.float32)
    assert lib.fno_model_create(ctypes.byref(m), ctypes.byref(gfno.to_c(bad)),
                                p.ctypes.data_as(ctypes.c_void_p), 10, 64, 64) == -1
    good = W.FnoSpec()
    assert lib.fno_model_create(ctypes.byref(m), ctypes.byref(gfno.to_c(good)),
                                p.ctypes.data_as(ctypes.c_void_p), 10, 64, 64) == -1
    assert lib.fno_forward(None, 1, 2, 1, 3, 100, None) == -1
    assert lib.fno_forward_graph(None, 1, 2, 1, 3, 100, None) == -1


@pytest.mark.parametrize("name,spl", [("node/lean", 1), ("quad/fp32", 1), ("pair-64x8/lean", 2),
                                      ("pair-64x4/mixed", 2), ("deep3-64x8/lean", 3),
                                      ("deep5-64x16/lean", 5), ("deep4-64x8/fp32", 4),
                                      ("tuned deep3+nt 0.0616 ms/step".split()[1].split("+")[0], 3)])
def test_bench_steps_per_launch_parses_every_kernel_name(name, spl):
    """bench.py divides the algorithmic bytes of one launch by its duration; the
    steps per launch come from the kernel name lbm_step_kernel (or the batch
    tuner) reports, so every shape the library can name must parse."""
    import sys
    sys.path.insert(0, ROOT)
    import bench
    assert bench.steps_per_launch(name) == spl


def test_every_fused_shape_name_is_reported_by_the_library(lib):
    """The library's kernel-name table and the bench parser agree: every name in
    the table parses to the steps its shape runs."""
    import sys
    sys.path.insert(0, ROOT)
    import bench
    src = open(os.path.join(ROOT, "paper_2604_27158_amd", "csrc", "lbm.hip")).read()
    names = set(re.findall(r'"((?:pair|deep\d)-64x\d+)/(?:lean|fp32|mixed)"', src))
    assert names == {"pair-64x8", "pair-64x4", "deep5-64x16", "deep4-64x8"}
    for n in names:
        assert bench.steps_per_launch(n + "/lean") == (2 if n.startswith("pair") else int(n[4]))
