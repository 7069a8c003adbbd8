"""Stage timing: the all-stage switch and the per-stage mask bracket exactly
the stages they name, and a mask naming no stage is rejected."""
import pytest
import torch

from oracle import loop as OL
from paper_2104_03989_amd import synth
from tests.gpu_common import GpuScene

pytestmark = pytest.mark.gpu


def test_profile_stage_mask():
    from paper_2104_03989_amd import adr
    ctx = adr.Context(0)
    try:
        w = synth.scaled(synth.workload_plain_step(map_size=64, ref_nu=16, lat_nu=4), views=2, res=64)
        gs = GpuScene(w, ctx)
        ref = gs.render("reference")["image"]
        ctx.profile(True)
        ctx.profile_read()
        out = gs.render("latent", ref=ref)
        every = ctx.profile_read()
        assert every["raster"][1] > 0 and every["shade"][1] > 0 and every["aa_loss"][1] > 0
        ctx.profile_stages(["shade", "raster"])
        gs.render("latent", ref=ref)
        gs.grads(out, names=("pos", "kd", "normal"))
        some = ctx.profile_read()
        assert some["shade"][1] == every["shade"][1] and some["raster"][1] == every["raster"][1]
        assert all(cnt == 0 for k, (_, cnt) in some.items() if k not in ("shade", "raster")), some
        assert some["shade"][0] > 0.0
        ctx.profile(False)
        gs.render("latent", ref=ref)
        assert all(cnt == 0 for _, cnt in ctx.profile_read().values())
        with pytest.raises(adr.AdrError):
            adr._check(adr._lib.adr_ctx_profile_stages(ctx.h, 1 << adr.N_STAGES))
        torch.cuda.synchronize()
    finally:
        ctx.close()


def test_profile_map_adam_stages():
    """The map Adam is timed as two stages: the level-0 tiles and the levels
    above them; each names its own launch."""
    import numpy as np
    from paper_2104_03989_amd import adr
    ctx = adr.Context(0)
    try:
        S, C, levels = 128, 3, 8          # levels 6 and 7 lie above the 32x32 tiles
        g = np.random.default_rng(11)
        tex = adr.DeviceTexture(g.normal(size=(S, S, C)).astype(np.float32), "f32", levels=levels, ctx=ctx)
        gd = torch.from_numpy(g.normal(size=tex.data.shape).astype(np.float32)).cuda()
        md = torch.zeros(S * S, C, device="cuda")
        vd = torch.zeros(S * S, C, device="cuda")
        ctx.profile_stages(["adam_maps", "adam_maps_top"])
        ctx.profile_read()
        adr.adam_step_maps(ctx, [(tex, gd, md, vd)], 1, 1e-3)
        got = ctx.profile_read()
        assert got["adam_maps"][1] == 1 and got["adam_maps_top"][1] == 1, got
        assert got["adam_maps"][0] > 0.0 and got["adam_maps_top"][0] > 0.0, got
        assert all(cnt == 0 for k, (_, cnt) in got.items() if k not in ("adam_maps", "adam_maps_top")), got
        assert float(gd.abs().max()) == 0.0      # the whole gradient chain is cleared
        ctx.profile(False)
        torch.cuda.synchronize()
    finally:
        ctx.close()
