"""Caller-owned workspaces (ph_evaluate_ws): results equal the plan's own calls bit for bit,
and calls with distinct workspaces enqueued on different streams without synchronisation in
between give the same results as serial calls."""
import numpy as np
import pytest

import gen
from tests.helpers import plan_kwargs

pytestmark = pytest.mark.gpu


def _t(a, dtype=None):
    import torch
    return torch.tensor(np.asarray(a), dtype=dtype or torch.float32, device="cuda")


def _bits(x):
    return x.cpu().numpy().view(np.uint32 if x.element_size() == 4 else np.uint64)


@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_workspace_calls_equal_own_calls_and_overlap_safely(gpu_lib, precision):
    import torch
    dt = torch.float64 if precision == "fp64" else torch.float32
    print(f"workspace calls {precision}", flush=True)
    wl = gen.config2(seed=1031, n_axis=48)
    plan = gpu_lib.Plan(wl.xyz, wl.gas, dict(src_rel=1e-5, e_abs=3e6), precision=precision, leaf_capacity=32,
                        **plan_kwargs(wl))
    assert plan.workspace_bytes() > 0
    inputs = []
    for k in range(3):
        I = np.roll(wl.I, 7 * k) * (1.0 + 0.3 * k)
        inputs.append((_t(I, dt), _t(np.roll(wl.E, -3 * k))))
    ref = [plan.evaluate(I, E).clone() for I, E in inputs]
    torch.cuda.synchronize()
    ws = [plan.new_workspace() for _ in range(3)]
    streams = [torch.cuda.Stream() for _ in range(3)]
    outs = [torch.empty(wl.n, dtype=dt, device="cuda") for _ in range(3)]
    torch.cuda.synchronize()
    for rep in range(2):  # the second round reuses workspaces that hold earlier calls' state
        for k in range(3):
            with torch.cuda.stream(streams[k]):
                plan.evaluate(inputs[k][0], inputs[k][1], out=outs[k], workspace=ws[k], stream=streams[k])
        torch.cuda.synchronize()
        for k in range(3):
            assert np.array_equal(_bits(outs[k]), _bits(ref[k])), (rep, k)
    # a workspace call with statistics, and the plan's own workspace still intact afterwards
    S, st = plan.evaluate(inputs[1][0], inputs[1][1], workspace=ws[0], stats=True)
    assert st["n_src"] > 0 and np.array_equal(_bits(S), _bits(ref[1]))
    again = plan.evaluate(inputs[2][0], inputs[2][1])
    torch.cuda.synchronize()
    assert np.array_equal(_bits(again), _bits(ref[2]))
    plan.close()


def test_workspace_is_checked(gpu_lib):
    import torch
    wl = gen.config1()
    plan = gpu_lib.Plan(wl.xyz, wl.gas, wl.thresholds, leaf_capacity=27, **plan_kwargs(wl))
    I = _t(wl.I.astype(np.float32))
    ws = plan.new_workspace()
    with pytest.raises(gpu_lib.PhError) as e:
        plan.evaluate(I, workspace=ws[1:])  # misaligned
    assert e.value.status == gpu_lib.PH_EINVAL
    plan.close()
