"""Multisampled visibility (Sec. 5.2) on the HIP path against the oracle:
per-sample visibility bit-exact, resolved images within the forward
tolerance, loss within 1e-5, gradients within 1e-4 relative L2."""
import sys

import numpy as np
import pytest
import torch

from oracle import loop as OL
from oracle import render as R
from paper_2104_03989_amd import synth
from tests import oracle_scenes as S
from tests.gpu_common import GpuScene, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2104_03989_amd import adr
    c = adr.Context(0)
    yield c
    c.close()


def _case(ctx, w, names, extra=0):
    from paper_2104_03989_amd import adr
    m = w.msaa
    flags = (adr.MSAA_4X4 if m == 4 else adr.MSAA_2X2) | extra
    mvp32, eye = OL.cameras(w)
    gs = GpuScene(w, ctx, mvp32, eye)
    ref = OL.reference_image(w, mvp32, eye)
    B, H, W = w.dirs.shape[0], w.height, w.width
    out = gs.render("latent", ref=ref.reshape(B, H, W, 3).to(torch.float32).cuda().contiguous(), flags=flags,
                    want_coverage=True)
    assert tuple(out["vis"].shape) == (B, m * H, m * W) and tuple(out["image"].shape) == (B, H, W, 3)
    pos32 = np.asarray(w.latent.mesh.pos, np.float32)
    for b in range(B):
        sv = R.snap(pos32, mvp32[b], m * W, m * H)
        k, c, _ = R.raster(w.latent.mesh.tri, sv, m * W, m * H)
        assert np.array_equal(out["vis"][b].cpu().numpy().view(np.uint64), k), b
    loss_o, grads_o, o = OL.loss_and_grads(w, ref, mvp32, eye)
    got = out["image"].cpu().numpy().reshape(B, H * W, 3).astype(np.float64)
    exp = o["image"].detach().numpy()
    tm = lambda x: R.tonemap(torch.from_numpy(x)).numpy()
    assert np.abs(tm(got) - tm(exp)).max() < 1e-5
    assert abs(float(out["loss"][0]) - float(loss_o)) <= 1e-5 * float(loss_o)
    runs = [gs.grads(out, names, flags=flags) for _ in range(2 if extra else 1)]
    for n in names:
        e = rel_l2(runs[0][n], grads_o[n].numpy())
        print(f"  msaa {m} grad {n}: rel-L2 {e:.3g}", flush=True)
        assert e < 1e-4, (n, e)
        if extra:
            assert np.array_equal(runs[0][n].view(np.uint32), runs[1][n].view(np.uint32))


@pytest.mark.parametrize("m", [2, 4])
def test_msaa_ggx(ctx, m):
    print("msaa ggx", m, flush=True)
    w = S.tiny_sphere_workload("ggx", nu=3, res=32, views=2, tex=16, loss="l1_tonemap", seed=3)
    w.msaa = m
    _case(ctx, w, ("pos", "kd", "normal", "orm"))


def test_msaa_plain_step(ctx):
    print("msaa plain", flush=True)
    w = synth.scaled(synth.workload_plain_step(map_size=64), views=2, res=48)
    w.msaa = 2
    _case(ctx, w, ("pos", "normal"))


def test_msaa_deterministic(ctx):
    from paper_2104_03989_amd import adr
    print("msaa deterministic", flush=True)
    w = S.tiny_sphere_workload("blinn_phong", nu=3, res=32, views=2, tex=16, loss="l2", seed=5)
    w.msaa = 2
    _case(ctx, w, ("pos", "kd", "normal"), extra=adr.DETERMINISTIC)
