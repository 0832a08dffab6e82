"""Graph replay of ph_evaluate is switched off in this library: ph_plan_set_graph refuses to
turn it on and keeps eager launches.

A benchmark run that replayed evaluations as one HIP graph ended with a host heap-corruption
abort after the graph timing.  Reading the code found two real faults in the graph path (an
executable graph destroyed while its last replay could still run, and a plan teardown that
destroyed the streams and events a graph was captured across before the graph), but neither
was on the path that run took, so the abort's cause is not shown; the replay path was removed
rather than run again."""
import numpy as np
import pytest

import gen
from tests.helpers import plan_kwargs

pytestmark = pytest.mark.gpu


def test_graph_replay_is_refused_and_eager_calls_still_work(gpu_lib):
    import torch
    wl = gen.config2(seed=1021, n_axis=32)
    print("graph replay refused", flush=True)
    plan = gpu_lib.Plan(wl.xyz, wl.gas, dict(src_rel=1e-4, e_abs=3e6), **plan_kwargs(wl))
    with pytest.raises(gpu_lib.PhError) as e:
        plan.set_graph(True)
    assert e.value.status == gpu_lib.PH_EUNSUPPORTED
    plan.set_graph(False)
    I = torch.tensor(wl.I.astype(np.float32), device="cuda")
    E = torch.tensor(wl.E.astype(np.float32), device="cuda")
    a = plan.evaluate(I, E).cpu().numpy()
    b = plan.evaluate(I, E).cpu().numpy()
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32)) and np.all(np.isfinite(a))
    plan.close()
