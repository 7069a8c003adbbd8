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
