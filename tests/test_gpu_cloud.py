"""GPU parity on nonuniform point clouds (adaptive trees with U, V, W and X lists) against the FP64
oracle: small clouds in full, the 4-million-point cloud on sampled targets."""
import numpy as np
import pytest

import gen
from oracle import photoionization, rel_l2
from tests.helpers import plan_kwargs

pytestmark = pytest.mark.gpu


def _t(a, dtype):
    import torch
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda")


def _say(msg):
    print(msg, flush=True)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-6), ("fp32", 1e-3)])
def test_cloud_all_sources_small(gpu_lib, precision, tol):
    """200k-point cloud, every point a source and a target: W and X lists are in use."""
    import torch
    wl = gen.config3(seed=2001, n=200_000, src_rel=0.0)
    _say(f"cloud 200k {precision} all sources")
    plan = gpu_lib.Plan(wl.xyz, wl.gas, dict(src_rel=0.0), precision=precision, **plan_kwargs(wl))
    dt = torch.float64 if precision == "fp64" else torch.float32
    Iin = wl.I if precision == "fp64" else wl.I.astype(np.float32).astype(np.float64)
    S, st = plan.evaluate(_t(Iin, dt), stats=True)
    w = st["work"]
    _say(f"  levels {st['levels']} boxes {st['n_boxes']} work {w}")
    assert w["m2p_evals"] > 0 and w["p2l_evals"] > 0, "the cloud must exercise the W and X lists"
    tg = gen.sample_targets(np.arange(wl.n), wl.xyz, wl.head, k=1500, seed=3, head_radius=0.2, head_cap=500)
    ref = photoionization(wl.xyz, Iin, wl.gas, w=wl.w, targets=tg)
    err = rel_l2(S.double().cpu().numpy()[tg], ref.S_t)
    _say(f"  rel-L2 = {err:.3e} on {tg.size} targets")
    assert err <= tol
    plan.close()


@pytest.mark.parametrize("gas_name", ["760", "40"])
@pytest.mark.parametrize("src_rel", [1e-3, 1e-4, 1e-5])
def test_cloud_4m_thresholds(gpu_lib, gas_name, src_rel):
    """The 4M-point cloud at two pressures and three source thresholds (FP32), sampled targets."""
    import torch
    gas = gen.GAS_760 if gas_name == "760" else gen.GAS_40
    wl = gen.config3(seed=2000, gas=gas, src_rel=src_rel)
    _say(f"cloud 4M {gas_name} Torr src_rel {src_rel:g}")
    plan = gpu_lib.Plan(wl.xyz, wl.gas, wl.thresholds, **plan_kwargs(wl))
    I32 = wl.I.astype(np.float32)
    E32 = wl.E.astype(np.float32)
    S, st = plan.evaluate(_t(I32, torch.float32), _t(E32, torch.float32), stats=True)
    _say(f"  n_src {st['n_src']} levels {st['levels']} boxes {st['n_boxes']}")
    tg = gen.sample_targets(np.arange(wl.n), wl.xyz, wl.head, k=400, seed=5, head_radius=0.2, head_cap=200)
    ref = photoionization(wl.xyz, I32.astype(np.float64), wl.gas, w=wl.w, src_rel=src_rel,
                          E=E32.astype(np.float64), e_abs=3e6, targets=tg)
    assert int(ref.smask.sum()) == st["n_src"]
    err = rel_l2(S.double().cpu().numpy()[tg], ref.S_t)
    _say(f"  rel-L2 = {err:.3e} on {tg.size} targets")
    assert err <= 1e-3
    plan.close()
