"""Parity of tessellation + displacement (Sec. 5.1, Eq. 3) on the HIP path
with the FP64 oracle: displaced positions equal to the float32 rounding of
the oracle's, the tessellated visibility bit-exact, the whole step's loss and
the gradients w.r.t. base positions, displacement texels and normal-map
texels within 1e-4 relative L2, on the 64-triangle crop (also against
central differences), a reduced displacement loop and the full-size one
(visibility, positions and forward on sampled views)."""
import sys

import numpy as np
import pytest
import torch

from oracle import loop as OL
from oracle import render as R
from oracle import tess as T
from paper_2104_03989_amd import synth
from tests import oracle_scenes as S
from tests.gpu_common import TessGpuScene, oracle_tess_keys, rel_l2

pytestmark = pytest.mark.gpu

FWD_TOL = 1e-5
GRAD_TOL = 1e-4


@pytest.fixture(scope="module")
def ctx():
    from paper_2104_03989_amd import adr
    c = adr.Context(0)
    yield c
    c.close()


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _random_disp(w, size, sigma, seed):
    g = np.random.default_rng(seed)
    w.disp = synth.Texture(g.normal(0.0, sigma, size=(size, size, 1)).astype(np.float32), "f32")
    return w


def _base_case(nu=7, levels=3, size=64, seed=0):
    w = synth.scaled(synth.workload_displacement(map_size=size, ref_nu=8, base_nu=nu, levels=levels),
                     views=1, res=32)
    return _random_disp(w, size, 0.03, seed)


def _positions_match(got, vd64):
    exp = vd64.astype(np.float32)
    ne = int((got != exp).sum())
    # the float64 expressions agree to ~1e-16; a differing rounding is ~1e-9 likely
    assert ne <= max(1, got.size // 100000), ne
    assert np.abs(got.astype(np.float64) - vd64).max() <= 2.5e-7


@pytest.mark.parametrize("levels", [0, 1, 3])
def test_displaced_positions(ctx, levels):
    from paper_2104_03989_amd import adr
    _say("tess fwd levels", levels)
    w = _base_case(levels=levels)
    ts = adr.DeviceTess(w.latent.mesh, levels)
    disp = adr.DeviceTexture(w.disp.data, "f32", levels=1)
    got = adr.tess_fwd(ctx, ts, disp)
    torch.cuda.synchronize()
    table = T.build(w.latent.mesh.tri, w.latent.mesh.uv_tri, w.latent.mesh.uv, w.latent.mesh.pos.shape[0], levels)
    with torch.no_grad():
        vd = T.displaced_positions(torch.as_tensor(w.latent.mesh.pos, dtype=R.F64), w.latent.mesh, table,
                                   torch.as_tensor(w.disp.data, dtype=R.F64)).numpy()
    _positions_match(got.cpu().numpy(), vd)


def test_tess_adjoint_matches_autograd(ctx):
    from paper_2104_03989_amd import adr
    _say("tess bwd")
    w = _base_case()
    m = w.latent.mesh
    ts = adr.DeviceTess(m, w.tess_levels)
    disp = adr.DeviceTexture(w.disp.data, "f32", levels=1)
    g = np.random.default_rng(5).normal(size=(ts.n_vert, 3))
    g[::7] = 0.0                                   # some vertices without gradient
    g_base = torch.zeros_like(ts.base.pos)
    g_disp = torch.zeros_like(disp.data)
    g_dev = torch.from_numpy(g.astype(np.float32)).cuda()
    adr.tess_bwd(ctx, ts, disp, g_dev, g_base, g_disp)
    torch.cuda.synchronize()
    assert float(g_dev.abs().max()) == 0.0         # the input gradient is consumed
    table = OL.tess_table(w)
    pos = torch.tensor(m.pos, dtype=R.F64, requires_grad=True)
    d = torch.tensor(w.disp.data, dtype=R.F64, requires_grad=True)
    vd = T.displaced_positions(pos, m, table, d)
    gp, gd = torch.autograd.grad((vd * torch.from_numpy(np.float32(g).astype(np.float64))).sum(), [pos, d])
    e_p = rel_l2(g_base.cpu().numpy(), gp.numpy())
    e_d = rel_l2(g_disp.cpu().numpy().reshape(gd.shape), gd.numpy())
    _say(f"  base pos {e_p:.3g}  disp {e_d:.3g}")
    assert e_p < 1e-5 and e_d < 1e-5


def test_tess_rejects_bad_arguments(ctx):
    from paper_2104_03989_amd import adr
    w = _base_case(levels=1)
    ts = adr.DeviceTess(w.latent.mesh, 1)
    rgb = adr.DeviceTexture(np.zeros((8, 8, 3), np.float32), "f32", levels=1)
    with pytest.raises(adr.AdrError):
        adr.tess_fwd(ctx, ts, rgb)                 # displacement must have one channel


def _step_case(ctx, w, names=("pos", "disp", "normal")):
    mvp32, eye = OL.cameras(w)
    gs = TessGpuScene(w, ctx, mvp32, eye)
    ref = OL.reference_image(w, mvp32, eye)
    B, H, W = w.dirs.shape[0], w.height, w.width
    ref_dev = ref.reshape(B, H, W, 3).to(torch.float32).cuda().contiguous()
    out = gs.render("latent", ref=ref_dev, want_coverage=True)
    keys, cov, vd = oracle_tess_keys(w, mvp32)
    _positions_match(gs.ts.mesh.pos.cpu().numpy(), vd)
    assert np.array_equal(out["vis"].cpu().numpy().view(np.uint64), keys)
    assert np.array_equal(out["coverage"].cpu().numpy().astype(np.uint32), cov)
    loss_o, grads_o, o = OL.loss_and_grads(w, ref, mvp32, eye)
    got = out["image"].cpu().numpy().reshape(B, H * W, 3).astype(np.float64)
    assert np.abs(got - o["image"].detach().numpy()).max() < FWD_TOL
    loss_g = float(out["loss"][0])
    assert abs(loss_g - float(loss_o)) <= 1e-5 * abs(float(loss_o)) + 1e-9
    g = gs.grads(out, names)
    for n in names:
        e = rel_l2(g[n], grads_o[n].numpy())
        _say(f"  grad {n}: rel-L2 {e:.3g}")
        assert e < GRAD_TOL, (n, e)
        if n in ("kd", "normal", "orm"):
            assert g[n + "_coarse_max"] == 0.0
    return gs, g, grads_o, (ref, mvp32, eye)


def test_crop_step_matches_oracle_and_central_differences(ctx):
    _say("tess crop step")
    w = S.tess_crop_workload(res=32, views=2, seed=1)
    gs, g, grads_o, (ref, mvp32, eye) = _step_case(ctx, w)
    # the GPU gradient of displacement texels against central differences
    # of the oracle's loss (h = 1e-4, renders with unchanged visibility)
    base = {k: v.detach().clone() for k, v in OL.latent_params(w).items()}

    def loss_at(p):
        out = OL.render_latent(w, mvp32, eye, p, round32=False)
        return float(R.image_loss(out["image"], ref, w.loss)), R.key_tri(out["keys"])

    _, ids0 = loss_at(base)
    flat = g["disp"].reshape(-1)
    scale = float(np.abs(flat).max())
    checked = 0
    for idx in np.argsort(-np.abs(flat))[:8]:
        vals, same = [], True
        for sgn in (1, -1):
            p = {k: v.clone() for k, v in base.items()}
            p["disp"].reshape(-1)[idx] += sgn * 1e-4
            L, ids = loss_at(p)
            same &= np.array_equal(ids, ids0)
            vals.append(L)
        if not same:
            continue
        fd = (vals[0] - vals[1]) / 2e-4
        assert abs(fd - flat[idx]) <= 1e-4 * scale + 1e-3 * abs(fd), (idx, fd, flat[idx])
        checked += 1
    assert checked >= 4


def test_displacement_loop_reduced(ctx):
    _say("tess reduced loop")
    w = synth.scaled(synth.workload_displacement(map_size=128, ref_nu=40), views=2, res=128)
    _random_disp(w, 128, 0.02, 11)
    _step_case(ctx, w)


def test_displacement_loop_full_size_sampled(ctx):
    # Full shapes (62,720 tessellated triangles, 1024^2 maps, 512^2 views):
    # visibility of all 8 views bit-exact; forward images of two views.
    _say("tess full size")
    w = synth.workload_displacement()
    _random_disp(w, 1024, 0.01, 12)
    mvp32, eye = OL.cameras(w)
    gs = TessGpuScene(w, ctx, mvp32, eye)
    out = gs.render("latent", want_coverage=True)
    keys, cov, vd = oracle_tess_keys(w, mvp32)
    _positions_match(gs.ts.mesh.pos.cpu().numpy(), vd)
    assert np.array_equal(out["vis"].cpu().numpy().view(np.uint64), keys)
    assert np.array_equal(out["coverage"].cpu().numpy().astype(np.uint32), cov)
    w2 = synth.scaled(w, views=2)
    o = OL.render_latent(w2, mvp32[:2], eye[:2])
    got = out["image"][:2].cpu().numpy().reshape(2, -1, 3).astype(np.float64)
    assert np.abs(got - o["image"].detach().numpy()).max() < FWD_TOL
