"""Adam on mip-mapped maps fused with the chain's adjoint and rebuild
(adr_adam_step_maps): against the oracle (the chain's adjoint taken by
autograd through its box-filter pyramid, Adam, the rebuilt chain) on chains
of several shapes, and bit for bit against the unfused sequence (mip
adjoint in the backward, adr_adam_step, mip build in the next forward) over
a few steps of a deterministic-mode loop."""
import sys

import numpy as np
import pytest
import torch

from oracle import loop as OL
from oracle import render as R
from paper_2104_03989_amd import synth
from tests.gpu_common import GpuScene

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


def _oracle(p0, gchain, m, v, levels, t, lr, b1=0.9, b2=0.999, eps=1e-8, fold_only=False):
    """Folded level-0 gradient d/dp0 sum_l <g_l, chain_l(p0)> and one Adam
    step, in float64 (with fold_only: (None, folded gradient, None))."""
    S, C = p0.shape[0], p0.shape[2]
    x = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    chain = R.mip_chain_f32(x, levels)
    obj = sum((lv * torch.tensor(gl, dtype=torch.float64)).sum() for lv, gl in zip(chain, gchain))
    (g0,) = torch.autograd.grad(obj, [x])
    if fold_only:
        return None, g0.numpy(), None
    pn, mn, vn = R.adam(p0, g0.numpy(), m, v, t, lr, b1, b2, eps)
    return pn, mn, vn


def _split(flat, S, C, levels):
    out, o = [], 0
    for l in range(levels):
        s = S >> l
        out.append(flat[o:o + s * s].reshape(s, s, C))
        o += s * s
    return out


# (size, channels, levels): full chains with levels above the 32^2 tiles, a
# chain inside one tile, a truncated chain, one level, a 1x1 map, and tiles
# whose rows are not float4 multiples (the scalar path)
CASES = [(2048, 3, 12), (4096, 1, 13), (64, 1, 7), (16, 3, 5), (256, 3, 4), (128, 3, 1), (1, 3, 1), (2, 3, 2),
         (4, 1, 3)]


@pytest.mark.parametrize("case", CASES, ids=[f"{s}x{c}x{l}" for s, c, l in CASES])
def test_adam_maps_matches_oracle(ctx, case):
    from paper_2104_03989_amd import adr
    S, C, levels = case
    _say("adam maps", case)
    g = np.random.default_rng(S * 7 + C * 3 + levels)
    p0 = g.normal(size=(S, S, C)).astype(np.float32)
    tex = adr.DeviceTexture(p0, "f32", levels=levels, ctx=ctx)
    n = tex.data.shape[0]
    # per-level gradients as a deferred backward leaves them, scaled per level
    gflat = np.concatenate([g.normal(size=((S >> l) ** 2, C)) * (0.5 ** l) for l in range(levels)]).astype(np.float32)
    m = (g.normal(size=(S * S, C)) * 0.1).astype(np.float32)
    v = (np.abs(g.normal(size=(S * S, C))) * 0.01).astype(np.float32)
    gd = torch.from_numpy(gflat).cuda()
    md, vd = torch.from_numpy(m).cuda(), torch.from_numpy(v).cuda()
    t, lr = 5, 1e-2
    adr.adam_step_maps(ctx, [(tex, gd, md, vd)], t, lr)
    torch.cuda.synchronize()
    # The oracle takes the hyper-parameters as they cross the ABI (float32:
    # beta2 = 0.999 arrives as 0.99900001, which moves the bias correction by
    # 1e-5 relative), so the remaining difference is the kernel's float32
    # arithmetic.  Forward error bound per texel, in units u = 2^-24 of the
    # magnitudes involved: the new texel and the step (a few roundings
    # each), and the first moment's rounding (the folded gradient is a sum
    # of up to `levels` terms, each rounded) carried through the step's
    # division by sqrt(v_hat) + eps.
    b1, b2, lr32, eps32 = (float(np.float32(x)) for x in (0.9, 0.999, lr, 1e-8))
    m64 = m.reshape(S, S, C).astype(np.float64)
    v64 = v.reshape(S, S, C).astype(np.float64)
    gch = _split(gflat.astype(np.float64), S, C, levels)
    pn, mn, vn = _oracle(p0.astype(np.float64), gch, m64, v64, levels, t, lr32, b1, b2, eps32)
    _, g_abs, _ = _oracle(p0.astype(np.float64), [np.abs(x) for x in gch], np.zeros_like(m64),
                          np.zeros_like(v64), levels, t, lr32, b1, b2, eps32, fold_only=True)
    got = _split(tex.data.cpu().numpy().astype(np.float64), S, C, levels)
    mg = md.cpu().numpy().reshape(S, S, C).astype(np.float64)
    vg = vd.cpu().numpy().reshape(S, S, C).astype(np.float64)
    u = 2.0 ** -24
    step_o = p0.astype(np.float64) - pn
    vhat = vn / (1 - b2 ** t)
    m_mag = b1 * np.abs(m64) + (1 - b1) * (levels + 1) * g_abs
    g_fold = (mn - b1 * m64) / (1 - b1)
    v_err = 8 * u * (b2 * v64 + (1 - b2) * (g_fold ** 2 + 2 * np.abs(g_fold) * (levels + 1) * g_abs))
    tol0 = 8 * u * (np.abs(p0) + np.abs(step_o)) + 8 * u * lr32 * m_mag / (1 - b1 ** t) / (np.sqrt(vhat) + eps32)
    tol0 += 0.5 * np.abs(step_o) * v_err / np.maximum(vn, 1e-300)
    tol0 += np.spacing(np.abs(pn).astype(np.float32)).astype(np.float64)
    err0 = np.abs(got[0] - pn)
    em = np.abs(mg - mn) / (8 * u * m_mag + 1e-30)
    ev = np.abs(vg - vn) / (v_err + 1e-30)
    _say(f"  level 0 vs oracle: max {err0.max():.3g} ({(err0 / tol0).max():.2f} of the bound); "
         f"m {em.max():.2f}, v {ev.max():.2f} of theirs")
    if not np.all(err0 <= tol0):
        i = np.unravel_index(np.argmax(err0 / tol0), err0.shape)
        _say("  worst", i, "p0", repr(p0[i]), "m0", repr(m64[i]), "v0", repr(v64[i]), "got", repr(np.float32(got[0][i])),
             "oracle", pn[i], "bound", tol0[i])
    assert np.all(err0 <= tol0)
    assert np.all(em <= 1.0) and np.all(ev <= 1.0)
    # the rebuilt levels: box averages of the kernel's new level 0 (float32
    # rounding of the pairwise sums, at most a few units of the largest
    # level-0 magnitude per level)
    chain = [c.numpy() for c in R.mip_chain_f32(torch.tensor(got[0]), levels)]
    u0 = float(np.spacing(np.float32(2 * np.abs(got[0]).max())))
    for l in range(1, levels):
        el = np.abs(got[l] - chain[l]).max()
        assert el <= 2 * l * u0, (l, el)
    assert float(gd.abs().max()) == 0.0
    assert n == sum((S >> l) ** 2 for l in range(levels))


def test_adam_maps_rejects_bad_arguments(ctx):
    from paper_2104_03989_amd import adr
    tex = adr.DeviceTexture(np.zeros((8, 8, 4), np.uint8), "rgba8")
    z = torch.zeros(64 * 4, device="cuda")
    with pytest.raises(adr.AdrError):
        adr._check(adr._lib.adr_adam_step_maps(ctx.h, (adr.MapParam_ * 1)(adr.MapParam_(tex.struct(), z.data_ptr(),
                                                                                        z.data_ptr(), z.data_ptr())),
                                               1, 1, 1e-3, 0.9, 0.999, 1e-8, None))
    f = adr.DeviceTexture(np.zeros((8, 8, 3), np.float32), "f32")
    with pytest.raises(adr.AdrError):
        adr._check(adr._lib.adr_adam_step_maps(ctx.h, (adr.MapParam_ * 1)(adr.MapParam_(f.struct(), None, None, None)),
                                               1, 1, 1e-3, 0.9, 0.999, 1e-8, None))
    with pytest.raises(adr.AdrError):
        adr._check(adr._lib.adr_adam_step_maps(ctx.h, None, 1, 1, 1e-3, 0.9, 0.999, 1e-8, None))
    adr._check(adr._lib.adr_adam_step_maps(ctx.h, None, 0, 1, 1e-3, 0.9, 0.999, 1e-8, None))


def _loop(ctx, w, fused, steps):
    """Deterministic-mode steps of the render loop; returns the final maps
    (whole chains), positions and Adam moments."""
    from paper_2104_03989_amd import adr
    gs = GpuScene(w, ctx)
    ref = gs.render("reference", flags=adr.DETERMINISTIC)["image"]
    mat, mesh = gs.lat_mat, gs.lat_mesh
    grads = {"pos": torch.zeros_like(mesh.pos), "orm": None}
    maps = []
    for name in ("kd", "normal"):
        tex = getattr(mat, name)
        grads[name] = tex.grad_buffer()
        n0 = tex.size * tex.size
        maps.append((tex, grads[name], torch.zeros_like(tex.data[:n0]), torch.zeros_like(tex.data[:n0])))
    pos_state = (mesh.pos, grads["pos"], torch.zeros_like(mesh.pos), torch.zeros_like(mesh.pos))
    det = adr.DETERMINISTIC
    out = None
    for t in range(steps):
        fflags = det | (0 if fused else adr.FWD_BUILD_MIPS)
        out = adr.render_fwd(ctx, mesh, mat, gs.views, ref=ref, loss=w.loss, flags=fflags, want_image=False,
                             outputs=out)
        adr.render_bwd(ctx, mesh, mat, gs.views, out, grads, flags=det | (adr.BWD_DEFER_MIP_ADJOINT if fused else 0))
        lr = w.lr * 10.0 ** (-0.0002 * t)
        if fused:
            adr.adam_step(ctx, [pos_state], t + 1, lr)
            adr.adam_step_maps(ctx, maps, t + 1, lr)
        else:
            adr.adam_step(ctx, [pos_state] + [(tex.data[:m.shape[0]], g[:m.shape[0]], m, v) for tex, g, m, v in maps],
                          t + 1, lr)
    if not fused:
        for tex, _, _, _ in maps:
            adr.mip_build(ctx, tex)
    torch.cuda.synchronize()
    res = {"pos": mesh.pos.cpu().numpy(), "loss": out["loss"].cpu().numpy()}
    for (tex, g, m, v), name in zip(maps, ("kd", "normal")):
        res[name] = tex.data.cpu().numpy()
        res[name + "_m"], res[name + "_v"] = m.cpu().numpy(), v.cpu().numpy()
        res[name + "_g"] = float(g.abs().max())
    return res


def test_fused_loop_is_bit_identical_to_unfused(ctx):
    _say("fused vs unfused loop")
    w = synth.scaled(synth.workload_paper_loop(map_size=256, ref_nu=40, lat_nu=10), views=2, res=128)
    a = _loop(ctx, w, False, 4)
    b = _loop(ctx, w, True, 4)
    for k in a:
        if k.endswith("_g"):
            assert a[k] == 0.0 and b[k] == 0.0, k
        else:
            assert np.array_equal(np.asarray(a[k]).view(np.uint32), np.asarray(b[k]).view(np.uint32)), k


def _oit_step(ctx, w, mvp32, eye, ref, deferred):
    """One depth-peeled step: backward, then Adam on positions and the maps,
    with the mip adjoint in the backward (and the chains rebuilt after) or
    deferred to the map Adam.  The Adam moments start from the same seeded
    non-zero values on both sides, so that the step depends smoothly on the
    gradients (whose float atomics sum in no fixed order)."""
    from paper_2104_03989_amd import adr
    views = adr.DeviceViews(mvp32, eye, w.light_dir, w.light_rgb, w.width, w.height)
    mesh, mat = adr.DeviceMesh(w.latent.mesh), adr.DeviceMaterial(w.latent, ctx=ctx)
    out = adr.render_oit_fwd(ctx, mesh, mat, views, w.oit_layers, ref=ref, loss=w.loss)
    g = {"pos": torch.zeros_like(mesh.pos)}
    for n in ("kd", "normal", "alpha"):
        g[n] = getattr(mat, n).grad_buffer()
    adr.render_oit_bwd(ctx, mesh, mat, views, out, g, flags=adr.BWD_DEFER_MIP_ADJOINT if deferred else 0)
    rng = np.random.default_rng(7)
    mom = lambda x: (torch.from_numpy((rng.normal(size=tuple(x.shape)) * 0.01).astype(np.float32)).cuda(),
                     torch.from_numpy((np.abs(rng.normal(size=tuple(x.shape))) * 0.01 + 1e-3).astype(np.float32)).cuda())
    pos_state = (mesh.pos, g["pos"], *mom(mesh.pos))
    maps = []
    for n in ("kd", "normal", "alpha"):
        tex = getattr(mat, n)
        n0 = tex.size * tex.size
        maps.append((tex, g[n], *mom(tex.data[:n0])))
    if deferred:
        adr.adam_step(ctx, [pos_state], 3, 1e-2)
        adr.adam_step_maps(ctx, maps, 3, 1e-2)
    else:
        n0s = [tex.size * tex.size for tex, _, _, _ in maps]
        adr.adam_step(ctx, [pos_state] + [(tex.data[:k], gr[:k], m, v) for (tex, gr, m, v), k in zip(maps, n0s)],
                      3, 1e-2)
        for tex, _, _, _ in maps:
            adr.mip_build(ctx, tex)
    torch.cuda.synchronize()
    res = {"pos": mesh.pos.cpu().numpy()}
    for (tex, gr, m, v), n in zip(maps, ("kd", "normal", "alpha")):
        res[n] = tex.data.cpu().numpy()
        res[n + "_m"] = m.cpu().numpy()
        res[n + "_g"] = float(gr.abs().max())
    return res


def test_deferred_adjoint_on_peeled_layers(ctx):
    from tests import oracle_scenes as S
    _say("deferred mip adjoint, depth-peeled")
    w = S.aggregate_case(res=32, views=2, n_leaves=80, n_quads=8, tex=16, layers=4)
    mvp32, eye = OL.cameras(w)
    ref = OL.reference_image(w, mvp32, eye)
    ref_dev = ref.reshape(w.dirs.shape[0], w.height, w.width, 3).to(torch.float32).cuda().contiguous()
    a = _oit_step(ctx, w, mvp32, eye, ref_dev, False)
    b = _oit_step(ctx, w, mvp32, eye, ref_dev, True)
    for k in a:
        if k.endswith("_g"):
            assert a[k] == 0.0 and b[k] == 0.0, k
            continue
        err = np.abs(a[k] - b[k]).max()
        _say(f"  {k}: max diff {err:.3g}")
        assert err < 1e-6, (k, err)
