"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/libgabor.h declares, and rejects bad arguments before
any device work (a rejected call must not touch the GPU)."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_1704_05231_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "libgabor.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gabor_\w+|lsdft_\w+|sdft_\w+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = binding.load()
    declared = header_functions()
    assert declared, "no functions parsed from the header"
    for name in declared:
        assert hasattr(lib, name), f"libgabor.so does not export {name}"
    assert sorted(binding.EXPORTS) == declared


def test_status_strings():
    for code, name in binding.STATUS.items():
        assert binding.gabor_status_string(code) == name
    assert binding.gabor_status_string(99) == "GABOR_ERR_UNKNOWN"


def _plan_raw(H=8, W=8, om=(1.0,), sg=(2.0,), N=4, th=None, rs=3.0, bnd=0, prec=0, out=True):
    lib = binding.load()
    om = np.asarray(om, np.float64)
    sg = np.asarray(sg, np.float64)
    th = None if th is None else np.asarray(th, np.float64)
    plan = ctypes.c_void_p(1234)
    ptr = ctypes.byref(plan) if out else None
    st = lib.gabor_bank_plan(ptr, H, W, len(om), om.ctypes.data_as(ctypes.c_void_p),
                             sg.ctypes.data_as(ctypes.c_void_p), N,
                             None if th is None else th.ctypes.data_as(ctypes.c_void_p),
                             rs, bnd, prec, None)
    return st, plan


@pytest.mark.parametrize("kw", [
    dict(H=0), dict(W=-3), dict(N=0), dict(om=()), dict(sg=(0.0,)), dict(sg=(-1.0,)),
    dict(sg=(float("inf"),)), dict(om=(float("nan"),)), dict(th=(0.0, float("inf"), 1.0, 2.0)),
    dict(rs=-1.0), dict(rs=float("nan")), dict(bnd=7), dict(prec=9), dict(out=False),
])
def test_plan_rejects_bad_arguments(kw):
    st, plan = _plan_raw(**kw)
    assert st == 1
    if kw.get("out", True):
        assert plan.value is None     # the handle is cleared on failure


def test_plan_rejects_null_parameter_arrays():
    lib = binding.load()
    plan = ctypes.c_void_p()
    sg = np.array([1.0])
    assert lib.gabor_bank_plan(ctypes.byref(plan), 4, 4, 1, None, sg.ctypes.data_as(ctypes.c_void_p),
                               2, None, 3.0, 0, 0, None) == 1


def test_apply_and_info_reject_null_plan():
    lib = binding.load()
    assert lib.gabor_bank_apply(None, ctypes.c_void_p(16), 8, ctypes.c_void_p(16), None) == 1
    info = binding.PlanInfo()
    assert lib.gabor_bank_plan_info(None, ctypes.byref(info)) == 1
    assert lib.gabor_bank_destroy(None) == 0


def test_forced_allocation_failure(monkeypatch):
    monkeypatch.setenv("LIBGABOR_FAIL_ALLOC", "1")
    st, plan = _plan_raw(om=(math.pi / 4, math.pi / 8), sg=(4.0, 4.0))
    assert st == 2 and plan.value is None


def test_oversized_radius_is_unsupported():
    st, _ = _plan_raw(sg=(5000.0,))
    assert st == 4


def _lsdft_raw(img=16, H=8, W=8, stride=8, my=4, mx=4, sigma=1.0, bnd=0, prec=0, out=16):
    lib = binding.load()
    return lib.lsdft_apply(None if img is None else ctypes.c_void_p(img), H, W, stride, my, mx,
                           sigma, bnd, prec, None if out is None else ctypes.c_void_p(out), None)


@pytest.mark.parametrize("kw", [
    dict(img=None), dict(out=None), dict(H=0), dict(W=-1), dict(stride=7), dict(my=0),
    dict(mx=-2), dict(sigma=0.0), dict(sigma=float("nan")), dict(sigma=-1.0), dict(bnd=2),
    dict(prec=5),
])
def test_lsdft_rejects_bad_arguments(kw):
    # rejected on the host: the fake device pointers are never touched
    assert _lsdft_raw(**kw) == 1


@pytest.mark.parametrize("kw", [dict(my=65), dict(mx=100), dict(H=1 << 15, W=1 << 14, stride=1 << 14),
                                dict(H=40000, W=2, stride=1 << 15)])
def test_lsdft_limits_are_unsupported(kw):
    assert _lsdft_raw(**kw) == 4


def test_lsdft_work_counts():
    """Bins u <= Mx/2, v <= My/2 (Eq. (19)-(20)); a pass over a complex
    operand costs two real products per tap, a real one one."""
    def count(my, mx):
        macs = 0
        for u in range(mx // 2 + 1):
            ju = 1 if (2 * u) % mx == 0 else 2
            macs += ju * mx
            for v in range(my // 2 + 1):
                cv = 1 if (2 * v) % my == 0 else 2
                macs += ju * cv * my
        return macs
    for (H, W, my, mx) in [(512, 512, 16, 16), (7, 9, 5, 12), (3, 4, 1, 1), (10, 10, 2, 7)]:
        macs, nbytes = binding.lsdft_work(H, W, my, mx)
        assert macs == count(my, mx) * H * W
        assert nbytes == 4 * H * W + 8 * my * mx * H * W
    assert binding.load().lsdft_work(0, 4, 4, 4, None, None) == 1


def test_adjoint_rejects_null_arguments():
    lib = binding.load()
    assert lib.gabor_bank_apply_adjoint(None, ctypes.c_void_p(16), ctypes.c_void_p(16), 8, None) == 1
    assert lib.gabor_bank_apply_adjoint_noalloc(None, ctypes.c_void_p(16), ctypes.c_void_p(16), 8, None) == 1
    assert lib.gabor_bank_apply_adjoint_batched(None, ctypes.c_void_p(16), 2, ctypes.c_void_p(16), 64, 8,
                                                None) == 1


def test_batched_apply_rejects_null_arguments():
    lib = binding.load()
    assert lib.gabor_bank_apply_batched(None, ctypes.c_void_p(16), 2, 64, 8, ctypes.c_void_p(16), None) == 1
    assert lib.gabor_bank_apply_batched(None, ctypes.c_void_p(16), -1, 64, 8, ctypes.c_void_p(16), None) == 1


def test_batch_rejects_null_arguments():
    lib = binding.load()
    P = ctypes.c_void_p
    batch = ctypes.c_void_p(99)
    assert lib.gabor_batch_create(None, None, 1, None, None, None, None, None, None) == 1
    assert lib.gabor_batch_create(ctypes.byref(batch), None, 1, None, None, None, None, None, None) == 1
    assert batch.value is None
    assert lib.gabor_batch_apply(None, None) == 1
    assert lib.gabor_batch_info(None, None, None) == 1
    assert lib.gabor_batch_destroy(None) == 0


def test_tuning_rejects_null_arguments():
    lib = binding.load()
    n = ctypes.c_int32()
    assert lib.gabor_bank_autotune(None, ctypes.c_void_p(16), 8, ctypes.c_void_p(16), 3, None) == 1
    assert lib.gabor_bank_get_tuning(None, None, 0, ctypes.byref(n)) == 1
    assert lib.gabor_bank_set_tuning(None, None, 0) == 1
    g = ctypes.c_int32()
    assert lib.gabor_bank_get_grouping(None, ctypes.byref(g)) == 1
    assert lib.gabor_bank_set_grouping(None, 1) == 1


def test_iir_plan_rejects_bad_arguments():
    lib = binding.load()
    om, sg = np.array([1.0]), np.array([2.0])
    P = lambda a: a.ctypes.data_as(ctypes.c_void_p)
    plan = ctypes.c_void_p(7)
    assert lib.gabor_bank_plan_iir(None, 8, 8, 1, P(om), P(sg), 4, None, 0, None) == 1
    assert lib.gabor_bank_plan_iir(ctypes.byref(plan), 0, 8, 1, P(om), P(sg), 4, None, 0, None) == 1
    assert plan.value is None
    assert lib.gabor_bank_plan_iir(ctypes.byref(plan), 8, 8, 1, P(om), P(np.array([-1.0])), 4, None, 0, None) == 1
    assert lib.gabor_bank_plan_iir(ctypes.byref(plan), 8, 8, 1, P(om), P(sg), 4, None, 3, None) == 1
    # sigma below the recursive design's range: valid but unsupported, before any allocation
    assert lib.gabor_bank_plan_iir(ctypes.byref(plan), 8, 8, 1, P(om), P(np.array([0.3])), 4, None, 0, None) == 4


def _sdft_raw(img=16, H=8, W=8, stride=8, my=4, mx=4, bnd=0, out=16):
    lib = binding.load()
    return lib.sdft_box_apply(None if img is None else ctypes.c_void_p(img), H, W, stride, my, mx, bnd,
                              None if out is None else ctypes.c_void_p(out), None)


@pytest.mark.parametrize("kw", [
    dict(img=None), dict(out=None), dict(H=0), dict(W=-1), dict(stride=7), dict(my=0), dict(mx=-2),
    dict(bnd=2), dict(bnd=-1),
])
def test_sdft_box_rejects_bad_arguments(kw):
    # rejected on the host: the fake device pointers are never touched
    assert _sdft_raw(**kw) == 1


@pytest.mark.parametrize("kw", [dict(my=65), dict(mx=100), dict(W=8193, stride=8193),
                                dict(H=65536, W=2, stride=2)])
def test_sdft_box_limits_are_unsupported(kw):
    assert _sdft_raw(**kw) == 4
