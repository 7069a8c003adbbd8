"""Prefiltering (Sec. 4.2) on the HIP path: the supersampled reference
(render at k times the resolution, box filter) and a step of a
multisampled latent with independent mip levels, against the oracle."""
import numpy as np
import pytest
import torch

from oracle import loop as OL
from oracle import render as R
from paper_2104_03989_amd import synth
from tests.gpu_common import GpuScene, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2104_03989_amd import adr
    c = adr.Context(0)
    yield c
    c.close()


def _small():
    return synth.workload_prefilter(views=2, res=32, ssaa=4, msaa=4, map_size=64, ref_nu=24, lat_nu=6)


def _gpu_reference(ctx, gs, w):
    from paper_2104_03989_amd import adr
    k = w.ref_ssaa
    big = adr.DeviceViews(gs.mvp32, gs.eye, w.light_dir, w.light_rgb, w.width * k, w.height * k)
    out = adr.render_fwd(ctx, gs.ref_mesh, gs.ref_mat, big)
    return adr.image_downsample(ctx, out["image"], k)


def test_supersampled_reference(ctx):
    print("prefilter reference", flush=True)
    w = _small()
    mvp32, eye = OL.cameras(w)
    gs = GpuScene(w, ctx, mvp32, eye)
    got = _gpu_reference(ctx, gs, w)
    torch.cuda.synchronize()
    exp = OL.reference_image(w, mvp32, eye).numpy()
    B = w.dirs.shape[0]
    g = got.cpu().numpy().reshape(B, -1, 3).astype(np.float64)
    tm = lambda x: R.tonemap(torch.from_numpy(x)).numpy()
    assert np.abs(tm(g) - tm(exp)).max() < 1e-5


def test_prefilter_step(ctx):
    from paper_2104_03989_amd import adr
    print("prefilter step", flush=True)
    w = _small()
    mvp32, eye = OL.cameras(w)
    gs = GpuScene(w, ctx, mvp32, eye)
    ref = _gpu_reference(ctx, gs, w)
    flags = adr.MSAA_4X4 | adr.INDEPENDENT_MIPS
    out = gs.render("latent", ref=ref, flags=flags)
    ref_o = OL.reference_image(w, mvp32, eye)
    loss_o, grads_o, _ = OL.loss_and_grads(w, ref_o, mvp32, eye)
    assert abs(float(out["loss"][0]) - float(loss_o)) <= 1e-5 * float(loss_o)
    g = {"pos": torch.zeros_like(gs.lat_mesh.pos)}
    for n in ("kd", "normal", "orm"):
        g[n] = getattr(gs.lat_mat, n).grad_buffer()
    adr.render_bwd(ctx, gs.lat_mesh, gs.lat_mat, gs.views, out, g, flags=flags)
    torch.cuda.synchronize()
    for n in ("pos", "kd", "normal", "orm"):
        e = rel_l2(g[n].cpu().numpy(), grads_o[n].numpy())
        print(f"  grad {n}: rel-L2 {e:.3g}", flush=True)
        assert e < 1e-4, (n, e)
