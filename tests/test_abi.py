"""The C-ABI library: it loads, exports every symbol include/ffmm.h declares, its host-only
parameter choice matches the oracle, and its argument checks fail cleanly (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_0911_4114_amd as ff
from oracle.quadrature import level_quadrature, UNIT_ROUNDOFF

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "ffmm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ffmm_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_declared_symbols():
    lib = ff.load_library()
    syms = declared_symbols()
    assert len(syms) >= 15
    for s in syms:
        assert hasattr(lib, s), s


def test_options_default_and_status_strings():
    lib = ff.load_library()
    o = ff.Options()
    assert lib.ffmm_options_default(ctypes.byref(o)) == 0
    assert o.struct_size == ctypes.sizeof(ff.Options)
    assert o.precision == 0 and o.max_leaf_points == 64 and o.depth == 0
    assert abs(o.alpha - 0.8) < 1e-15 and abs(o.eps_safety - 0.1) < 1e-15
    assert o.max_rhs == 1 and o.reduce_depth == 1 and o.method == 0
    assert o.best_effort == 0 and o.fast_near_phase == 0
    assert lib.ffmm_options_default(None) == -1
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert lib.ffmm_status_string(code)


def test_tuning_default_and_null_plan():
    lib = ff.load_library()
    t = ff.Tuning()
    assert lib.ffmm_tuning_default(ctypes.byref(t)) == 0
    assert t.struct_size == ctypes.sizeof(ff.Tuning)
    assert (t.near_stream, t.p2p_blocks_per_cu, t.m2l_rhs_block) == (2, 0, 0)
    assert list(t.rs_slab) == [16, 32, 32, 16] and t.m2l_by_parent == 2 and t.m2l_chunk == 64
    assert lib.ffmm_tuning_default(None) == -1
    assert lib.ffmm_plan_set_tuning(None, ctypes.byref(t)) == -1
    assert lib.ffmm_plan_get_tuning(None, ctypes.byref(t)) == -1
    assert lib.ffmm_plan_autotune(None, None, None, 1, None, None) == -1


@pytest.mark.parametrize("ka", [1.95, 2.77, 3.14, 5.54, 11.1, 22.1, 44.3])
@pytest.mark.parametrize("eps,prec", [(1e-3, 1), (1e-4, 1), (1e-6, 0), (1e-8, 0)])
def test_host_parameter_choice_matches_oracle(ka, eps, prec):
    ell, nth, nphi, pred = ff.select_level_params(ka, 0.8, eps, prec)
    q, info = level_quadrature(ka, 0.8, eps, u=UNIT_ROUNDOFF["fp32" if prec else "fp64"])
    assert (ell, nth) == (q.ell, q.ntheta)
    assert nphi == list(q.nphi)
    assert abs(pred - info["predicted"]) <= 1e-3 * info["predicted"] + 1e-14


@pytest.mark.parametrize("ka,eps,prec", [(110.0, 1e-4, 1)])
def test_host_parameter_choice_matches_oracle_wide(ka, eps, prec):
    """Above ka = 100 the design radius becomes the box diagonal where eps is reachable there."""
    ell, nth, nphi, pred = ff.select_level_params(ka, 0.8, eps, prec)
    u = UNIT_ROUNDOFF["fp32" if prec else "fp64"]
    q, info = level_quadrature(ka, 0.8, eps, u=u)
    assert (ell, nth) == (q.ell, q.ntheta) and nphi == list(q.nphi)
    assert abs(pred - info["predicted"]) <= 1e-3 * info["predicted"] + 1e-14
    assert info["alpha"] in (0.8, 1.0)


def _create(points_ptr, n, kappa, eps, opts=None, alloc=None):
    lib = ff.load_library()
    h = ctypes.c_void_p()
    st = lib.ffmm_plan_create(points_ptr, n, kappa, eps, opts, alloc, None, ctypes.byref(h))
    return st, lib.ffmm_last_error_message().decode()


def test_plan_create_rejects_bad_arguments():
    dummy = ctypes.c_void_p(0x1000)   # never dereferenced: every case fails its checks first
    assert _create(None, 10, 1.0, 1e-4)[0] == -1
    assert _create(dummy, 0, 1.0, 1e-4)[0] == -1
    assert _create(dummy, 10, 0.0, 1e-4)[0] == -1
    assert _create(dummy, 10, float("nan"), 1e-4)[0] == -1
    assert _create(dummy, 10, 1.0, 0.9)[0] == -1
    assert _create(dummy, 10, 1.0, 1e-13)[0] == -1
    o = ff.Options()
    ff.load_library().ffmm_options_default(ctypes.byref(o))
    o.precision = 1
    st, msg = _create(dummy, 10, 1.0, 1e-9, ctypes.byref(o))
    assert st == -4 and "FP32" in msg
    o.precision = 0
    o.depth = 1
    assert _create(dummy, 10, 1.0, 1e-4, ctypes.byref(o))[0] == -1
    o.depth = 0
    o.alpha = 1.5
    assert _create(dummy, 10, 1.0, 1e-4, ctypes.byref(o))[0] == -1
    o.alpha = 0.8
    o.max_rhs = 0
    assert _create(dummy, 10, 1.0, 1e-4, ctypes.byref(o))[0] == -1
    o.max_rhs = 1
    o.method = 3
    st, msg = _create(dummy, 10, 1.0, 1e-4, ctypes.byref(o))
    assert st == -1 and "method" in msg
    o.method = 2
    o.depth = 4
    st, msg = _create(dummy, 10, 1.0, 1e-4, ctypes.byref(o))
    assert st == -1 and "AUTO" in msg
    o.method = 0
    o.depth = 0
    o.best_effort = 2
    st, msg = _create(dummy, 10, 1.0, 1e-4, ctypes.byref(o))
    assert st == -1 and "best_effort" in msg
    o.best_effort = 0
    o.fast_near_phase = -1
    st, msg = _create(dummy, 10, 1.0, 1e-4, ctypes.byref(o))
    assert st == -1 and "fast_near_phase" in msg
    o.fast_near_phase = 0
    # an allocator needs both hooks (checked before any device work)
    half = ff.Allocator(None, ff._TORCH_ALLOC, ctypes.cast(None, ff._FREE_FN))
    st, msg = _create(dummy, 10, 1.0, 1e-4, ctypes.byref(o), ctypes.byref(half))
    assert st == -1 and "allocator" in msg
    o.struct_size = 4
    assert _create(dummy, 10, 1.0, 1e-4, ctypes.byref(o))[0] == -1


def test_calls_on_null_plan_fail_cleanly():
    lib = ff.load_library()
    buf = ctypes.c_void_p(0x1000)
    assert lib.ffmm_matvec(None, buf, buf, 1, None) == -1
    assert lib.ffmm_adjoint(None, buf, buf, 1, None) == -1
    assert lib.ffmm_field_gradient(None, buf, buf, 1, None) == -1
    assert lib.ffmm_position_gradient(None, buf, buf, buf, 1, None) == -1
    assert lib.ffmm_plan_info_get(None, None) == -1
    assert lib.ffmm_profile_enable(None, 1) == -1
    assert lib.ffmm_plan_destroy(None) == 0
    assert lib.ffmm_select_level_params(-1.0, 0.8, 1e-4, 0, 0, None, None, None, 0, None) == -1
