"""Batched stepping of uneven meshes: the graph-captured batch, in either
form (one launch per stage over all meshes through the library batch, or
every mesh's own launches over four streams), replayed step after step with
the cameras of each step copied in, then Adam over every mesh's positions and
maps (the maps' mip chains adjoined and rebuilt in the same kernel), gives
the same losses and parameters as stepping the meshes one at a time: bit for
bit in deterministic mode, at every replay, and within float tolerance with
atomics.  The autotuner picks and caches a work split per shape bucket."""
import sys

import numpy as np
import pytest
import torch

from paper_2104_03989_amd import synth

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _workloads(n=5):
    return synth.workload_batched(n_meshes=n, tris=(200, 2000), views=(2, 4), res_choices=(32, 48),
                                  map_sizes=(16, 32))


def _state(b):
    out = []
    for m in b.meshes:
        out.append([p.detach().cpu().numpy().copy() for p, _, _, _ in m.params] +
                   [tex.data.detach().cpu().numpy().copy() for tex, _, _, _ in m.maps])
    return out


@pytest.mark.parametrize("form", ["launch", "streams"])
@pytest.mark.parametrize("det", [True, False])
def test_graph_batch_equals_plain(det, form):
    from paper_2104_03989_amd.batch import Batch
    _say(f"batched ({form}) vs plain, " + ("deterministic" if det else "atomic"))
    ws = _workloads()
    steps = 4
    plain = Batch(ws, steps, det=det, tune=False, form="streams")
    batched = Batch(ws, steps, det=det, tune=False, form=form)
    batched.step_eager(0)                 # warm-up sizes the scratch
    plain.step_plain(0)
    torch.cuda.synchronize()
    batched.capture()
    for t in range(1, steps):
        plain.step_plain(t)
        batched.step(t)                   # graph replay, then eager Adam
        torch.cuda.synchronize()
        lp, lb = plain.losses(), batched.losses()
        sp, sb = _state(plain), _state(batched)
        for k in range(len(ws)):
            if det:
                assert lp[k] == lb[k], (t, k)
                for a, b in zip(sp[k], sb[k]):
                    assert np.array_equal(a, b), (t, k)
            else:
                assert abs(lp[k] - lb[k]) <= 1e-5 * abs(lp[k]) + 1e-9, (t, k)
                for a, b in zip(sp[k], sb[k]):
                    assert np.abs(a - b).max() <= 1e-5 * max(1.0, np.abs(a).max()), (t, k)
        _say(f"  step {t}: losses {np.round(lb, 6).tolist()}")
    plain.close()
    batched.close()


def test_autotune_cache(tmp_path):
    from paper_2104_03989_amd.autotune import CANDIDATES, Tuner
    from paper_2104_03989_amd.batch import Batch
    _say("autotune")
    ws = _workloads(2)
    path = str(tmp_path / "autotune.json")
    b = Batch(ws, 2, tune=True, tuner=Tuner(path))
    for m in b.meshes:
        assert m.split_ref in CANDIDATES and m.split_lat in CANDIDATES
    t2 = Tuner(path)
    assert len(t2.cache) >= 2
    m = b.meshes[0]
    w = m.w
    picked = t2.pick(b.ctxs[0], "latent", w.latent.mesh.tri.shape[0], w.dirs.shape[0], w.width,
                     run=lambda: (_ for _ in ()).throw(AssertionError("cached bucket re-timed")))
    assert picked == m.split_lat
    b.close()
