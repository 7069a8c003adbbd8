"""Pins of the oracle's interpolation, textures, shading, antialiasing, tone
map, loss and Adam against closed forms, invariants and special cases."""
import json
import math
import os

import numpy as np
import pytest
import torch

from oracle import loop
from oracle import render as R
from paper_2104_03989_amd import synth
from tests import oracle_scenes as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _pixel_rays(w, mvp32, eye, b):
    """Ray origin and directions through every pixel centre, obtained by
    inverting the float32 camera matrix the renderer uses (the matrix itself
    is pinned against the camera definition in test_look_at_closed_form)."""
    W, H = w.width, w.height
    Minv = np.linalg.inv(mvp32[b].astype(np.float64))
    j, i = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    px = (2 * (i + 0.5) / W - 1).reshape(-1)
    py = (2 * (j + 0.5) / H - 1).reshape(-1)
    one = np.ones_like(px)
    a = (Minv @ np.stack([px, py, -one, one])).T
    c = (Minv @ np.stack([px, py, one, one])).T
    a = a[:, :3] / a[:, 3:]
    c = c[:, :3] / c[:, 3:]
    o = Minv @ np.array([0.0, 0.0, -1.0, 0.0])   # camera centre: the w = 0 point
    e = np.asarray(eye[b], dtype=np.float64)
    return e, c - a


def _blinn_phong(n, l, v, kd):
    h = l + v
    h = h / np.linalg.norm(h, axis=-1, keepdims=True)
    nl = np.clip((n * l).sum(-1, keepdims=True), 0, None)
    nh = np.clip((n * h).sum(-1, keepdims=True), 0, None)
    return nl * (kd + 0.04 * nh ** 32)


def test_flat_quad_matches_ray_plane_closed_form():
    kd = (0.5, 0.3, 0.2)
    scene = synth.Scene(S.quad_mesh(), "blinn_phong", S.const_tex(kd), S.flat_normals(), None)
    w = S.workload(scene, scene, [(0.0, 0.0, 1.0)], [(0.3, 0.2, 1.0)], 40, 32)
    mvp32, eye = loop.cameras(w)
    out = R.render(scene.mesh, "blinn_phong", loop._levels(scene.kd), loop._levels(scene.normal),
                   None, torch.as_tensor(scene.mesh.pos, dtype=R.F64), mvp32,
                   eye.astype(np.float64), w.light_dir, w.light_rgb, w.width, w.height,
                   keep_gbuf=True)
    g = out["gbuf"][0]
    e, d = _pixel_rays(w, mvp32, eye, 0)
    d = d[g["pix"]]
    t = -e[2] / d[:, 2]
    hit = e[None] + t[:, None] * d
    # perspective-correct interpolation puts the pixel exactly on the ray
    assert np.abs(g["x"].numpy() - hit).max() < 1e-9
    assert np.abs(g["lam"].sum(1).numpy() - 1).max() < 1e-12
    v = e[None] - hit
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    n = np.tile([0.0, 0.0, 1.0], (hit.shape[0], 1))
    expect = _blinn_phong(n, w.light_dir[0][None], v, np.array(kd)[None])
    got = out["color"][0][torch.from_numpy(g["pix"])].numpy()
    assert g["pix"].size > 300
    assert np.abs(got - expect).max() < 2e-7  # kd is stored in float32


def test_tilted_triangle_interpolation_is_ray_plane_hit():
    pos = np.array([(-0.9, -0.7, 0.3), (1.1, -0.5, -0.6), (-0.2, 0.9, 0.1)], dtype=np.float32)
    tri = np.array([(0, 1, 2)], dtype=np.int32)
    mesh = synth.Mesh(pos, tri, np.array([(0, 0), (1, 0), (0, 1)], dtype=np.float32), tri.copy())
    scene = synth.Scene(mesh, "blinn_phong", S.const_tex((1, 1, 1)), S.flat_normals(), None)
    w = S.workload(scene, scene, [(0.2, 0.3, 1.0)], [(0.0, 0.0, 1.0)], 48, 48)
    mvp32, eye = loop.cameras(w)
    out = R.render(mesh, "blinn_phong", loop._levels(scene.kd), loop._levels(scene.normal), None,
                   torch.as_tensor(pos, dtype=R.F64), mvp32, eye.astype(np.float64), w.light_dir,
                   w.light_rgb, 48, 48, keep_gbuf=True)
    g = out["gbuf"][0]
    # the camera actually used is the float32 MVP: invert it for the rays
    M = mvp32[0].astype(np.float64)
    Minv = np.linalg.inv(M)
    pix = g["pix"]
    i, j = pix % 48, pix // 48
    px, py = 2 * (i + 0.5) / 48 - 1, 2 * (j + 0.5) / 48 - 1
    a = (Minv @ np.stack([px, py, -np.ones_like(px), np.ones_like(px)])).T
    b = (Minv @ np.stack([px, py, np.ones_like(px), np.ones_like(px)])).T
    a = a[:, :3] / a[:, 3:]
    b = b[:, :3] / b[:, 3:]
    p64 = pos.astype(np.float64)
    nrm = np.cross(p64[1] - p64[0], p64[2] - p64[0])
    t = ((p64[0] - a) @ nrm) / ((b - a) @ nrm)
    hit = a + t[:, None] * (b - a)
    assert pix.size > 100
    assert np.abs(g["x"].numpy() - hit).max() < 1e-9
    lam = g["lam"].numpy()
    assert np.abs(lam @ p64 - hit).max() < 1e-9


@pytest.mark.parametrize("nu", [8, 16])
def test_sphere_converges_to_closed_form(nu):
    errs = {}
    for n in (nu, 2 * nu):
        mesh = synth.sphere_mesh(n)
        scene = synth.Scene(mesh, "blinn_phong", S.const_tex((0.6, 0.5, 0.4)), S.flat_normals(), None)
        w = S.workload(scene, scene, [(0.3, 0.4, 0.8)], [(0.5, 0.6, 0.6)], 64, 64)
        mvp32, eye = loop.cameras(w)
        out = loop.render_scene(scene, mvp32, eye, w, aa=False)
        e, d = _pixel_rays(w, mvp32, eye, 0)
        d = d / np.linalg.norm(d, axis=1, keepdims=True)
        bq = (e[None] * d).sum(1)
        disc = bq ** 2 - (e @ e - 1.0)
        ok = disc > 0
        t = -bq - np.sqrt(np.where(ok, disc, 0))
        hit = e[None] + t[:, None] * d
        v = -d
        nv = (hit * v).sum(1)
        sel = ok & (nv > 0.4) & (R.key_tri(out["keys"][0]).reshape(-1) > 0)
        expect = _blinn_phong(hit[sel], w.light_dir[0][None], v[sel], np.array([0.6, 0.5, 0.4])[None])
        got = out["color"][0].numpy()[sel]
        errs[n] = (np.abs(got - expect).max(), np.abs(got - expect).mean())
    # mean error falls as O(h^2) (x4 per halving of the edge length); the
    # maximum sits next to the twelve valence-5 vertices and falls slower
    assert errs[2 * nu][0] < 0.002
    assert errs[nu][1] / errs[2 * nu][1] > 3.0, errs


def test_sphere_normals_and_tangents_are_radial_and_azimuthal():
    mesh = synth.sphere_mesh(16)
    pos = torch.as_tensor(mesh.pos, dtype=R.F64)
    tri = torch.as_tensor(mesh.tri, dtype=torch.long)
    n = R.vertex_normals(pos, tri).numpy()
    p = pos.numpy()
    assert np.abs(n - p / np.linalg.norm(p, axis=1, keepdims=True)).max() < 5e-3
    t = R.vertex_tangents(pos, tri, torch.as_tensor(mesh.uv, dtype=R.F64),
                          torch.as_tensor(mesh.uv_tri, dtype=torch.long)).numpy()
    sel = np.abs(p[:, 1]) < 0.9
    az = np.stack([-p[:, 2], np.zeros(len(p)), p[:, 0]], 1)
    az /= np.linalg.norm(az, axis=1, keepdims=True)
    assert np.abs(t[sel] - az[sel]).max() < 2e-2


# --------------------------------------------------------------- textures

def test_constant_texture_and_constant_mips():
    lv = R.mip_chain_f32(torch.full((16, 16, 3), 0.37, dtype=R.F64))
    for l in lv:
        assert torch.allclose(l, torch.full_like(l, 0.37), atol=1e-15)
    g = np.random.default_rng(0)
    uv = torch.as_tensor(g.uniform(-2, 3, size=(200, 2)))
    dd = torch.as_tensor(g.uniform(-0.5, 0.5, size=(200, 2)))
    s = R.sample_trilinear(lv, uv, dd, dd * 0.3)
    assert (s - 0.37).abs().max() < 1e-15


def test_checker_level1_is_mean_and_rgba8_rounding():
    x = torch.zeros(2, 2, 1, dtype=R.F64)
    x[0, 0] = x[1, 1] = 1.0
    assert float(R.mip_chain_f32(x)[1][0, 0, 0]) == 0.5
    q = np.zeros((2, 2, 4), dtype=np.uint8)
    q[..., 0] = [[1, 2], [3, 5]]   # sum 11 -> (11+2)//4 = 3
    q[..., 1] = [[1, 1], [1, 0]]   # sum 3 -> 5//4 = 1
    lv = R.mip_chain_rgba8(q)
    assert abs(float(lv[1][0, 0, 0]) - 3 / 255) < 1e-15
    assert abs(float(lv[1][0, 0, 1]) - 1 / 255) < 1e-15


def test_linear_ramp_reproduced_at_lod0():
    S_ = 64
    cols = (torch.arange(S_, dtype=R.F64) + 0.5) / S_
    rows = (torch.arange(S_, dtype=R.F64) + 0.5) / S_
    tex = torch.stack([cols[None, :].expand(S_, S_), rows[:, None].expand(S_, S_)], -1)
    lv = R.mip_chain_f32(tex)
    g = np.random.default_rng(1)
    uv = torch.as_tensor(g.uniform(0.05, 0.95, size=(300, 2)))
    tiny = torch.full((300, 2), 1e-4, dtype=R.F64)
    s = R.sample_trilinear(lv, uv, tiny, tiny)
    assert (s - uv).abs().max() < 1e-13


def test_trilinear_at_integer_lod_is_that_level():
    g = np.random.default_rng(2)
    lv = R.mip_chain_f32(torch.as_tensor(g.uniform(size=(32, 32, 3))))
    uv = torch.as_tensor(g.uniform(0, 1, size=(100, 2)))
    # |duv/dx| * 32 = 4 -> lod = 2 exactly
    ddx = torch.tensor([[4.0 / 32, 0.0]], dtype=R.F64).expand(100, 2)
    ddy = torch.zeros(100, 2, dtype=R.F64)
    s = R.sample_trilinear(lv, uv, ddx, ddy)
    s2 = R._bilinear(lv[2], uv[:, 0], uv[:, 1])
    assert (s - s2).abs().max() < 1e-14
    # beyond the coarsest level: clamped to it
    s = R.sample_trilinear(lv, uv, ddx * 1000, ddy)
    assert (s - lv[-1][0, 0]).abs().max() < 1e-14


def test_texture_gradients_partition_of_unity():
    g = np.random.default_rng(3)
    t0 = torch.as_tensor(g.uniform(size=(16, 16, 3)), dtype=R.F64).requires_grad_(True)
    lv = R.mip_chain_f32(t0)
    n = 500
    uv = torch.as_tensor(g.uniform(-1, 2, size=(n, 2)))
    d = torch.as_tensor(g.uniform(-0.3, 0.3, size=(n, 2)))
    w = torch.as_tensor(g.normal(size=(n, 3)))
    (R.sample_trilinear(lv, uv, d, d.flip(1)) * w).sum().backward()
    assert torch.allclose(t0.grad.sum(dim=(0, 1)), w.sum(0), atol=1e-11)


# --------------------------------------------------------------- antialias

@pytest.mark.parametrize("xe", [0.1234, -0.5, 0.0371])
def test_aa_of_straight_silhouette_is_box_filter(xe):
    W, H = 32, 8
    pos = np.array([(xe, -6.0, 0.5), (7.0, 0.0, 0.5), (xe, 6.0, 0.5)], dtype=np.float32)
    tri = np.array([(0, 1, 2)], dtype=np.int32)
    sv = R.snap(pos, np.eye(4, dtype=np.float32), W, H)
    keys, cov, orient = R.raster(tri, sv, W, H)
    color = torch.as_tensor((R.key_tri(keys).reshape(-1) > 0).astype(np.float64))[:, None].repeat(1, 3)
    clip = torch.as_tensor(np.concatenate([pos, np.ones((3, 1))], 1), dtype=R.F64)
    pairs = R.aa_pairs(keys, tri, sv, orient, R.adjacency(tri))
    out = R.antialias(color, clip, pairs, W, H).reshape(H, W, 3)[..., 0].numpy()
    Xe = (float(np.float32(xe)) + 1) * W / 2
    expect = np.clip(np.arange(W) + 1 - Xe, 0, 1)[None].repeat(H, 0)
    assert np.abs(out - expect).max() < 1e-12


def test_aa_skips_interior_edges():
    W = H = 24
    quad = S.quad_mesh(half=0.6)
    sv = R.snap(quad.pos, np.eye(4, dtype=np.float32), W, H)
    keys, cov, orient = R.raster(quad.tri, sv, W, H)
    P, Q, va, vb = R.aa_pairs(keys, quad.tri, sv, orient, R.adjacency(quad.tri))
    ids = R.key_tri(keys).reshape(-1)
    assert P.size > 0
    assert (ids[Q] == 0).all() and (ids[P] > 0).all()
    # the diagonal separates different ids but is never a crossing edge
    d = {(0, 3), (3, 0)}
    assert not any((a, b) in d for a, b in zip(va.tolist(), vb.tolist()))


# --------------------------------------------------------------- tone map, loss, Adam

def test_tonemap_paper_constants():
    with open(os.path.join(GOLDEN, "paper_constants.json")) as f:
        c = json.load(f)
    th = c["srgb_threshold"]
    x = torch.tensor([0.0, th, 1.0, 0.5], dtype=R.F64)
    y = R.srgb(x).numpy()
    assert y[0] == 0.0
    assert abs(y[1] - c["srgb_linear_slope"] * th) < 1e-18
    assert abs(y[2] - 1.0) < 1e-15  # (1 + a) * 1 - a
    assert abs(y[3] - ((1 + c["srgb_a"]) * 0.5 ** (1 / c["srgb_exponent"]) - c["srgb_a"])) < 1e-15
    # the two printed branches meet within 3e-8 at the printed threshold
    hi = (1 + c["srgb_a"]) * th ** (1 / c["srgb_exponent"]) - c["srgb_a"]
    assert abs(hi - c["srgb_linear_slope"] * th) < 3e-8
    # tonemap(e - 1) = Gamma(1) = 1
    assert abs(float(R.tonemap(torch.tensor(math.e - 1, dtype=R.F64))) - 1.0) < 1e-15
    xs = torch.linspace(0, 50, 2001, dtype=R.F64)
    assert (R.tonemap(xs).diff() > 0).all()


def test_lr_schedule_paper_constant():
    with open(os.path.join(GOLDEN, "paper_constants.json")) as f:
        c = json.load(f)
    k = c["lr_decay_k"]
    assert R.lr_schedule(0.01, 1, k) == 0.01
    assert abs(R.lr_schedule(0.01, 5001, k) - 0.001) < 1e-15  # one decade per 5000 steps


def test_adam_first_step_closed_form():
    g = np.random.default_rng(4).normal(size=100)
    p = np.zeros(100)
    pn, m, v = R.adam(p, g, np.zeros(100), np.zeros(100), 1, 1e-3)
    assert np.abs(pn - (-1e-3 * g / (np.abs(g) + 1e-8))).max() < 1e-15
    # second step with the same gradient: same step length
    pn2, _, _ = R.adam(pn, g, m, v, 2, 1e-3)
    assert np.abs((pn2 - pn) - (-1e-3 * g / (np.abs(g) + 1e-8))).max() < 1e-12


def test_identical_latent_and_reference_give_zero_loss_and_gradient():
    w = S.tiny_sphere_workload("ggx", loss="l1_tonemap")
    w.latent = w.ref
    w.optimize = ("pos", "kd", "normal", "orm")
    mvp32, eye = loop.cameras(w)
    ref = loop.reference_image(w, mvp32, eye)
    loss, grads, _ = loop.loss_and_grads(w, ref, mvp32, eye)
    assert float(loss) == 0.0
    for g in grads.values():
        assert float(g.abs().max()) == 0.0


def test_tonemap_odd_extension_to_negative_radiance():
    x = torch.linspace(0, 20, 401, dtype=R.F64)
    assert torch.equal(R.tonemap(-x), -R.tonemap(x))
    # smooth through zero: slope 12.92 on both sides
    h = torch.tensor([1e-9, -1e-9], dtype=R.F64)
    assert torch.allclose(R.tonemap(h) / h, torch.full_like(h, 12.92), rtol=1e-6)


def test_aa_of_subpixel_triangle_stays_convex():
    # a triangle much smaller than a pixel that still covers one pixel centre:
    # edges cross all four segments next to that pixel, whose received
    # weights then sum past 1 and are normalised; every output stays in the
    # range of the colours and the tiny triangle's pixel tends to background
    W = H = 9
    cx, cy = 2 * (4 + 0.5) / W - 1, 2 * (4 + 0.5) / H - 1
    e = 0.25 * 2 / W
    pos = np.array([(cx - e, cy - e, 0.5), (cx + e, cy - e, 0.5), (cx, cy + e, 0.5)], dtype=np.float32)
    tri = np.array([(0, 1, 2)], dtype=np.int32)
    sv = R.snap(pos, np.eye(4, dtype=np.float32), W, H)
    keys, cov, orient = R.raster(tri, sv, W, H)
    assert cov.sum() == 1
    color = torch.as_tensor((R.key_tri(keys).reshape(-1) > 0).astype(np.float64))[:, None].repeat(1, 3)
    clip = torch.as_tensor(np.concatenate([pos, np.ones((3, 1))], 1), dtype=R.F64)
    pairs = R.aa_pairs(keys, tri, sv, orient, R.adjacency(tri))
    assert pairs[0].size >= 3
    out = R.antialias(color, clip, pairs, W, H)[:, 0].numpy()
    assert out.min() >= 0.0 and out.max() <= 1.0
    assert out[4 * W + 4] < 0.5
