"""Visibility of large triangle batches: keys and coverage bit-exact
against the oracle's rasterizer on the paper-scale reference (297,680
triangles), a dense leaf cloud (320,000 triangles, heavy overdraw) and
depth-peeled layers of it."""
import sys

import numpy as np
import pytest
import torch

from oracle import loop as OL
from oracle import oit as O
from oracle import render as R
from paper_2104_03989_amd import synth
from tests import oracle_scenes as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2104_03989_amd import adr
    c = adr.Context(0)
    yield c
    c.close()


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _views(w, mvp32, eye):
    from paper_2104_03989_amd import adr
    return adr.DeviceViews(mvp32, eye, w.light_dir, w.light_rgb, w.width, w.height)


@pytest.mark.parametrize("case", ["paper", "leaves"])
def test_large_batch_visibility_and_coverage(ctx, case):
    from paper_2104_03989_amd import adr
    _say("large-batch raster", case)
    if case == "paper":
        w = synth.scaled(synth.workload_paper_loop(map_size=64), views=1, res=512)
        mesh = w.ref.mesh
        scene = w.ref
    else:
        w = synth.scaled(synth.workload_aggregate(map_size=64, n_leaves=40000, n_quads=16), views=1, res=256)
        mesh = w.ref.mesh
        scene = w.ref
    mvp32, eye = OL.cameras(w)
    out = adr.render_fwd(ctx, adr.DeviceMesh(mesh), adr.DeviceMaterial(scene, ctx=ctx), _views(w, mvp32, eye),
                         want_coverage=True)
    torch.cuda.synchronize()
    sv = R.snap(mesh.pos, mvp32[0], w.width, w.height)
    keys, cov, _ = R.raster(mesh.tri, sv, w.width, w.height)
    assert np.array_equal(out["vis"][0].cpu().numpy().view(np.uint64), keys)
    assert np.array_equal(out["coverage"][0].cpu().numpy().astype(np.uint32), cov)
    _say(f"  max coverage {int(cov.max())}")


def test_large_batch_depth_peeling(ctx):
    # three peeled layers of a 320k-triangle leaf cloud
    from paper_2104_03989_amd import adr
    _say("large-batch peeling")
    w = synth.scaled(synth.workload_aggregate(map_size=64, n_leaves=40000, n_quads=16), views=1, res=256)
    ref = w.ref
    mvp32, eye = OL.cameras(w)
    lat = synth.Scene(ref.mesh, "blinn_phong", S.const_tex((0.5, 0.5, 0.5)), S.flat_normals(), None)
    out = adr.render_oit_fwd(ctx, adr.DeviceMesh(ref.mesh), adr.DeviceMaterial(lat, ctx=ctx), _views(w, mvp32, eye), 3)
    torch.cuda.synchronize()
    vis = out["vis"].cpu().numpy().view(np.uint64)
    sv = R.snap(ref.mesh.pos, mvp32[0], w.width, w.height)
    layers = O.peel(ref.mesh.tri, sv, w.width, w.height, 3)
    for k in range(3):
        assert np.array_equal(vis[k, 0], layers[k]), k
