"""Graph replay of ph_evaluate: every replay equals an eager evaluation of the same inputs bit for
bit, while the buffers' contents (and with them the selected sources, the tree and the lists)
change between replays, eager work runs in between, and a new set of buffers is captured anew."""
import numpy as np
import pytest

import gen
from tests.helpers import plan_kwargs

pytestmark = pytest.mark.gpu


def _t(a, dtype=None):
    import torch
    return torch.tensor(np.asarray(a), dtype=dtype or torch.float32, device="cuda")


def _say(msg):
    print(msg, flush=True)


def _variants(wl, k):
    """Input k: the field and the intensities moved and rescaled, so the source set changes."""
    rng = np.random.default_rng(100 + k)
    I = np.roll(wl.I, 3 * k, axis=0) * (1.0 + 0.25 * k)
    I = I * (1.0 + 0.05 * rng.random(I.shape))
    E = np.roll(wl.E, -5 * k, axis=0)
    return I.astype(np.float32), E.astype(np.float32)


@pytest.mark.parametrize("selector", ["threshold", "learned"])
def test_graph_replays_equal_eager(gpu_lib, selector):
    import torch
    # leaves of 4^3 cells, as in the configuration the committed selector was trained on
    wl = gen.config2(seed=1021, n_axis=64)
    thr = dict(src_rel=1e-5, e_abs=3e6)
    kw = dict(leaf_capacity=64, **plan_kwargs(wl))
    if selector == "learned":
        from paper_2112_10059_amd.train_selector import load_selector
        w, meta = load_selector()
        thr = dict(src_rel=meta["base_src_rel"], e_abs=3e6)
        kw.update(selector="learned", selector_weights=w, selector_logit_threshold=meta["threshold"],
                  selector_fallback_rel=1e-4)
    _say(f"graph replay, {selector} selector")
    pe = gpu_lib.Plan(wl.xyz, wl.gas, thr, **kw)
    pg = gpu_lib.Plan(wl.xyz, wl.gas, thr, **kw)
    pg.set_graph(True)
    bI = torch.empty(wl.n, dtype=torch.float32, device="cuda")
    bE = torch.empty(wl.n, dtype=torch.float32, device="cuda")
    out = torch.empty(wl.n, dtype=torch.float32, device="cuda")
    n_src = set()
    for k in range(4):
        I, E = _variants(wl, k)
        bI.copy_(_t(I))
        bE.copy_(_t(E))
        pg.evaluate(bI, bE, out=out)
        # eager work between the replays
        ref, st = pe.evaluate(_t(I), _t(E), stats=True)
        scratch = torch.randn(1 << 16, device="cuda").sum()
        torch.cuda.synchronize()
        assert np.isfinite(scratch.item())
        n_src.add(st["n_src"])
        got = out.cpu().numpy()
        _say(f"  input {k}: n_src {st['n_src']}")
        assert np.array_equal(got.view(np.uint32), ref.cpu().numpy().view(np.uint32)), k
    assert len(n_src) > 1  # the replays saw different source sets
    # the same inputs replayed twice in a row
    pg.evaluate(bI, bE, out=out)
    pg.evaluate(bI, bE, out=out)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy().view(np.uint32), ref.cpu().numpy().view(np.uint32))
    # new buffers: captured again
    I, E = _variants(wl, 5)
    cI, cE = _t(I), _t(E)
    out2 = pg.evaluate(cI, cE)
    ref2 = pe.evaluate(cI, cE)
    torch.cuda.synchronize()
    assert np.array_equal(out2.cpu().numpy().view(np.uint32), ref2.cpu().numpy().view(np.uint32))
    # graph off again: eager launches on the same plan
    pg.set_graph(False)
    out3 = pg.evaluate(cI, cE)
    torch.cuda.synchronize()
    assert np.array_equal(out3.cpu().numpy().view(np.uint32), ref2.cpu().numpy().view(np.uint32))
    pe.close()
    pg.close()
