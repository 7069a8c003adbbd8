"""Independent mip levels (Sec. 4.2) on the HIP path: every level of the
kd, normal and ORM chains is its own variable; the chain gradients (all
levels) match the oracle's within 1e-4 relative L2."""
import numpy as np
import pytest
import torch

from oracle import loop as OL
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


def _chain(size, seed, lo, hi, normal=False):
    t = synth.independent_chain(size, 3, seed, lo, hi)
    if normal:
        t.chain[:, 2] = 1.0
        t.data[..., 2] = 1.0
    return t


@pytest.mark.parametrize("model", ["ggx", "blinn_phong"])
def test_independent_chain_gradients(ctx, model):
    from paper_2104_03989_amd import adr
    print("independent mips", model, flush=True)
    w = S.tiny_sphere_workload(model, nu=3, res=48, views=2, tex=16, loss="l1_tonemap", seed=8)
    w.latent.kd = _chain(16, 11, 0.1, 0.9)
    # a strong normal chain: near the sphere's UV poles the tangent frame is
    # ill-conditioned, which the float64 vertex accumulators must absorb
    w.latent.normal = _chain(16, 12, -0.2, 0.2, normal=True)
    names = ("kd", "normal")
    if model == "ggx":
        w.latent.orm = _chain(16, 13, 0.1, 0.6)
        names = ("kd", "normal", "orm")
    w.optimize = ("pos",) + names
    mvp32, eye = OL.cameras(w)
    gs = GpuScene(w, ctx, mvp32, eye)
    ref = OL.reference_image(w, mvp32, eye)
    B, H, W = w.dirs.shape[0], w.height, w.width
    out = gs.render("latent", ref=ref.reshape(B, H, W, 3).to(torch.float32).cuda().contiguous())
    loss_o, grads_o, _ = OL.loss_and_grads(w, ref, mvp32, eye)
    assert abs(float(out["loss"][0]) - float(loss_o)) <= 1e-5 * float(loss_o)
    g = {"pos": torch.zeros_like(gs.lat_mesh.pos)}
    for n in names:
        g[n] = getattr(gs.lat_mat, n).grad_buffer()
    adr.render_bwd(ctx, gs.lat_mesh, gs.lat_mat, gs.views, out, g, flags=adr.INDEPENDENT_MIPS)
    torch.cuda.synchronize()
    e = rel_l2(g["pos"].cpu().numpy(), grads_o["pos"].numpy())
    assert e < 1e-4, ("pos", e)
    for n in names:
        got = g[n].cpu().numpy()
        exp = grads_o[n].numpy()
        e = rel_l2(got, exp)
        print(f"  chain {n}: rel-L2 {e:.3g}", flush=True)
        assert e < 1e-4, (n, e)
        assert np.abs(got[256:]).max() > 0                 # coarse levels get their own gradient
    with pytest.raises(adr.AdrError):
        gs.render("latent", flags=adr.INDEPENDENT_MIPS | adr.FWD_BUILD_MIPS)
