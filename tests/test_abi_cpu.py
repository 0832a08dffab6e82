"""C ABI checks that need no GPU: the library loads, exports every declared entry point,
and rejects bad arguments on the host before any device call."""
import math
import os
import re

import numpy as np
import pytest

import gen
from paper_2112_10059_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "ph.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ph_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = binding.load()
    names = declared_functions()
    assert len(names) >= 12
    for name in names:
        assert hasattr(lib, name), f"{name} declared in ph.h but not exported"
    assert sorted(binding.EXPORTED) == names


def test_status_strings():
    lib = binding.load()
    for s in range(7):
        assert lib.ph_status_string(s)
    assert lib.ph_status_string(99) == b"unknown status"


def _plan(**over):
    wl = gen.config1()
    kw = dict(h=wl.h)
    thr = dict(wl.thresholds)
    gas = dict(wl.gas)
    xyz = wl.xyz
    for k, v in over.items():
        if k in ("src_rel", "e_abs", "e_rel", "e_applied", "r_s"):
            thr[k] = v
        elif k in gas:
            gas[k] = v
        elif k == "xyz":
            xyz = v
        else:
            kw[k] = v
    return binding.Plan(xyz, gas, thr, **kw)


@pytest.mark.parametrize("over,needle", [
    (dict(src_rel=1.5), "src_rel"),
    (dict(src_rel=float("nan")), "src_rel"),
    (dict(chi_min=3.0), "chi_min"),
    (dict(p_torr=0.0), "p_torr"),
    (dict(o2_fraction=1.5), "o2_fraction"),
    (dict(h=0.0), "h must be > 0"),
    (dict(order_q=11), "order_q"),
    (dict(leaf_capacity=-1), "leaf_capacity"),
    (dict(max_depth=40), "max_depth"),
    (dict(cube_lo=(0.05, 0.0, 0.0), cube_size=0.1), "outside the root cube"),
    (dict(selector="learned"), "selector_weights"),
])
def test_validation_rejects_before_device(over, needle):
    with pytest.raises(binding.PhError) as ei:
        _plan(**over)
    assert ei.value.status == binding.PH_EINVAL
    assert needle in str(ei.value)


def test_nonfinite_coordinates_rejected():
    xyz = gen.config1().xyz.copy()
    xyz[5, 1] = np.inf
    with pytest.raises(binding.PhError) as ei:
        _plan(xyz=xyz)
    assert ei.value.status == binding.PH_EINVAL


@pytest.mark.parametrize("r_s", [-1e-4, float("nan"), float("inf")])
def test_third_strategy_ratio_validated(r_s):
    with pytest.raises(binding.PhError) as ei:
        _plan(r_s=r_s)
    assert ei.value.status == binding.PH_EINVAL
    assert "r_s" in str(ei.value)


def test_null_arguments():
    lib = binding.load()
    import ctypes
    h = ctypes.c_void_p()
    assert lib.ph_plan_create(None, None, None, None, ctypes.byref(h)) == binding.PH_EINVAL
    assert lib.ph_evaluate(None, None, None, None, None, None) == binding.PH_EINVAL
    assert lib.ph_plan_size(None) == -1
    lib.ph_plan_destroy(None)
    assert lib.ph_mlp_forward(None, None, 4, None, 0, None) == binding.PH_EINVAL
    assert lib.ph_adam_step(None, None, None, None, 4, 1e-3, 0.9, 0.999, 1e-8, 1, None) == binding.PH_EINVAL
