"""Parity of dense linear blend skinning (Sec. 5.1, Eq. 2) on the HIP path
with the FP64 oracle: skinned positions equal to the float32 rounding of the
oracle's (float64 matrix-core contraction), the adjoint w.r.t. bind-pose
positions and every dense weight within 1e-6 relative L2, at ragged sizes,
bone counts off the 4- and 16-lane grain, the full-size animation rig, and a
whole rigged step (visibility bit-exact, loss, image and gradients of bind
pose, weights and maps within 1e-4 relative L2)."""
import sys

import numpy as np
import pytest
import torch

from oracle import loop as OL
from oracle import skin as K
from paper_2104_03989_amd import synth
from tests import oracle_scenes as S
from tests.gpu_common import SkinGpuScene, oracle_skinned_keys, rel_l2

pytestmark = pytest.mark.gpu

F64 = torch.float64
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


def _inputs(V, nb, seed):
    g = np.random.default_rng(seed)
    pos = g.normal(size=(V, 3)).astype(np.float32)
    w = g.normal(0.3, 0.5, size=(V, nb)).astype(np.float32)       # unnormalised, some negative
    bones = g.normal(size=(nb, 3, 4)).astype(np.float32)
    return pos, w, bones


def _positions_match(got, exp64):
    exp = exp64.astype(np.float32)
    ne = int((got != exp).sum())
    # float64 sums agree to ~1e-16: a different float32 rounding is ~1e-8 likely
    assert ne <= max(1, got.size // 100000), ne
    scale = np.abs(exp64).max()
    assert np.abs(got.astype(np.float64) - exp64).max() <= 1.2e-7 * max(scale, 1.0)


@pytest.mark.parametrize("V,nb", [(1000, 32), (37, 31), (16, 1), (5003, 64), (129, 18), (1, 4)])
def test_skin_forward(ctx, V, nb):
    from paper_2104_03989_amd import adr
    _say("skin fwd", V, nb)
    pos, w, bones = _inputs(V, nb, V + nb)
    out, blend = adr.skin_fwd(ctx, torch.from_numpy(pos).cuda(), torch.from_numpy(w).cuda(),
                              torch.from_numpy(bones).cuda())
    torch.cuda.synchronize()
    P, Wt, M = (torch.as_tensor(x, dtype=F64) for x in (pos, w, bones))
    _positions_match(out.cpu().numpy(), K.skin(P, Wt, M).numpy())
    A = torch.einsum("ib,bjk->ijk", Wt, M).reshape(V, 12).numpy()
    assert np.abs(blend.cpu().numpy() - A).max() <= 1.2e-7 * max(np.abs(A).max(), 1.0)


def test_skin_forward_unaligned_weights(ctx):
    # a weight matrix that starts 4 bytes into its allocation takes the scalar load path
    from paper_2104_03989_amd import adr
    V, nb = 300, 32
    pos, w, bones = _inputs(V, nb, 9)
    flat = torch.zeros(V * nb + 1, dtype=torch.float32, device="cuda")
    flat[1:] = torch.from_numpy(w.reshape(-1)).cuda()
    out, _ = adr.skin_fwd(ctx, torch.from_numpy(pos).cuda(), flat[1:].view(V, nb), torch.from_numpy(bones).cuda())
    torch.cuda.synchronize()
    _positions_match(out.cpu().numpy(), K.skin(*(torch.as_tensor(x, dtype=F64) for x in (pos, w, bones))).numpy())


@pytest.mark.parametrize("V,nb", [(1000, 32), (37, 31), (5003, 64), (16, 1)])
def test_skin_adjoint(ctx, V, nb):
    from paper_2104_03989_amd import adr
    _say("skin bwd", V, nb)
    pos, w, bones = _inputs(V, nb, 100 + V + nb)
    g = np.random.default_rng(V).normal(size=(V, 3)).astype(np.float32)
    g[::5] = 0.0
    pd, wd, bd = (torch.from_numpy(x).cuda() for x in (pos, w, bones))
    _, blend = adr.skin_fwd(ctx, pd, wd, bd)
    g0p = np.random.default_rng(1).normal(size=(V, 3)).astype(np.float32)     # accumulation onto existing values
    g0w = np.random.default_rng(2).normal(size=(V, nb)).astype(np.float32)
    gp, gw, gd = torch.from_numpy(g0p).cuda(), torch.from_numpy(g0w).cuda(), torch.from_numpy(g).cuda()
    adr.skin_bwd(ctx, pd, bd, blend, gd, g_pos=gp, g_weights=gw)
    torch.cuda.synchronize()
    assert float(gd.abs().max()) == 0.0                      # consumed
    P = torch.tensor(pos, dtype=F64, requires_grad=True)
    Wt = torch.tensor(w, dtype=F64, requires_grad=True)
    ep, ew = torch.autograd.grad((K.skin(P, Wt, torch.as_tensor(bones, dtype=F64)) * torch.as_tensor(g, dtype=F64)).sum(),
                                 [P, Wt])
    e_p = rel_l2(gp.cpu().numpy() - g0p, ep.numpy())
    e_w = rel_l2(gw.cpu().numpy() - g0w, ew.numpy())
    _say(f"  pos {e_p:.3g}  weights {e_w:.3g}")
    assert e_p < 1e-6 and e_w < 1e-6


def test_skin_adjoint_optional_outputs(ctx):
    from paper_2104_03989_amd import adr
    V, nb = 200, 20
    pos, w, bones = _inputs(V, nb, 3)
    pd, wd, bd = (torch.from_numpy(x).cuda() for x in (pos, w, bones))
    _, blend = adr.skin_fwd(ctx, pd, wd, bd)
    g = torch.ones(V, 3, device="cuda")
    gw = torch.zeros(V, nb, device="cuda")
    adr.skin_bwd(ctx, pd, bd, blend, g, g_pos=None, g_weights=gw)
    g2 = torch.ones(V, 3, device="cuda")
    gp = torch.zeros(V, 3, device="cuda")
    adr.skin_bwd(ctx, pd, bd, blend, g2, g_pos=gp, g_weights=None)
    torch.cuda.synchronize()
    assert float(g.abs().max()) == 0.0 and float(g2.abs().max()) == 0.0
    assert float(gw.abs().max()) > 0.0 and float(gp.abs().max()) > 0.0


def test_skin_rejects_bad_arguments(ctx):
    from paper_2104_03989_amd import adr
    pos, w, bones = _inputs(8, 4, 4)
    pd, wd, bd = (torch.from_numpy(x).cuda() for x in (pos, w, bones))
    with pytest.raises(adr.AdrError):
        adr.skin_fwd(ctx, pd, wd[:, :0], bd[:0])                  # no bones
    _, blend = adr.skin_fwd(ctx, pd, wd, bd)
    g = torch.zeros(8, 3, device="cuda")
    with pytest.raises(adr.AdrError):
        adr.skin_bwd(ctx, pd, bd, blend, g, g_pos=g)             # aliasing adjoint buffers
    e = torch.zeros(0, 3, device="cuda")
    out, _ = adr.skin_fwd(ctx, e, torch.zeros(0, 4, device="cuda"), bd)   # empty mesh: no work
    assert out.shape == (0, 3)


def test_full_size_rig(ctx):
    # the 9,612-vertex reference and 2,562-vertex latent of the animation loop, 32 bones, several frames
    from paper_2104_03989_amd import adr
    w = synth.workload_animation()
    _say("full-size rig")
    rig = w.rig
    for which, mesh, wts in (("ref", w.ref.mesh, rig.ref_weights), ("latent", w.latent.mesh, w.weights)):
        pd, wd = torch.from_numpy(mesh.pos).cuda(), torch.from_numpy(np.ascontiguousarray(wts)).cuda()
        for f in (0, 17, 39):
            out, _ = adr.skin_fwd(ctx, pd, wd, torch.from_numpy(np.ascontiguousarray(rig.bones[f])).cuda())
            torch.cuda.synchronize()
            exp = K.skin(torch.as_tensor(mesh.pos, dtype=F64), torch.as_tensor(wts, dtype=F64),
                         torch.as_tensor(rig.bones[f], dtype=F64)).numpy()
            _positions_match(out.cpu().numpy(), exp)


def _step_case(ctx, w, names=("pos", "weights", "kd", "normal")):
    mvp32, eye = OL.cameras(w)
    gs = SkinGpuScene(w, ctx, mvp32, eye)
    B, H, W = w.dirs.shape[0], w.height, w.width
    ref = OL.reference_image(w, mvp32, eye)
    ref_out = gs.render("ref")
    keys_r, _, vs_r = oracle_skinned_keys(w, mvp32, "ref")
    _positions_match(gs.ref_mesh.pos.cpu().numpy(), vs_r)
    assert np.array_equal(ref_out["vis"].cpu().numpy().view(np.uint64), keys_r)
    assert np.abs(ref_out["image"].cpu().numpy().reshape(B, H * W, 3) - ref.numpy()).max() < FWD_TOL
    ref_dev = ref.reshape(B, H, W, 3).to(torch.float32).cuda().contiguous()
    out = gs.render("latent", ref=ref_dev, want_coverage=True)
    keys, cov, vs = oracle_skinned_keys(w, mvp32)
    _positions_match(gs.lat_mesh.pos.cpu().numpy(), vs)
    assert np.array_equal(out["vis"].cpu().numpy().view(np.uint64), keys)
    assert np.array_equal(out["coverage"].cpu().numpy().astype(np.uint32), cov)
    loss_o, grads_o, o = OL.loss_and_grads(w, ref, mvp32, eye)
    got = out["image"].cpu().numpy().reshape(B, H * W, 3).astype(np.float64)
    assert np.abs(got - o["image"].detach().numpy()).max() < FWD_TOL
    assert abs(float(out["loss"][0]) - float(loss_o)) <= 1e-5 * abs(float(loss_o)) + 1e-9
    g = gs.grads(out, names)
    assert g["g_skinned_max"] == 0.0
    for n in names:
        e = rel_l2(g[n], grads_o[n].numpy())
        _say(f"  grad {n}: rel-L2 {e:.3g}")
        assert e < GRAD_TOL, (n, e)


def test_rigged_step_small(ctx):
    _say("rigged step small")
    w = S.rig_workload(S.tiny_sphere_workload(nu=3, res=32, views=2, tex=16), n_bones=6, n_frames=8, frame=3)
    _step_case(ctx, w)


def test_rigged_step_animation_scene(ctx):
    # the animation loop's scene at reduced size: 32 bones, random dense weights
    _say("rigged step animation scene")
    w = synth.scaled(synth.workload_animation(map_size=64, ref_nu=10, lat_nu=5), views=2, res=48)
    g = np.random.default_rng(11)
    wt = g.uniform(0.0, 1.0, size=w.weights.shape)
    w.weights = (wt / wt.sum(1, keepdims=True)).astype(np.float32)
    w.frame = 21
    _step_case(ctx, w, names=("pos", "weights", "kd", "normal", "orm"))
