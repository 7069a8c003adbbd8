"""Pins of the oracle's GGX shading (Sec. 5.2), its screen-space texture
derivatives and level of detail (the mip-mapped texture representation of
Sec. 4.2), and its loss normalisation (Sec. 5.3), each against a closed form,
a textbook result or a limit that a plausible mistake breaks.  Every pin is
written as a check function; the ``*_catches_*`` tests plant that mistake in
a copy of the oracle function (on the CPU) and show that the check fails."""
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


def _golden():
    with open(os.path.join(GOLDEN, "paper_constants.json")) as f:
        return json.load(f)


def _t(x):
    return torch.as_tensor(np.asarray(x, dtype=np.float64))


# --------------------------------------------------------------- GGX terms

def check_ndf(ndf):
    """The GGX distribution is a normalised distribution of microfacet
    normals: the projected area of the microfacets equals the macro surface,
    integral over the hemisphere of D(h) (n.h) d omega_h = 1 for every
    roughness; at n.h = 1 the GGX lobe peaks at 1 / (pi alpha^2)."""
    for r in (0.08, 0.2, 0.5, 0.8, 1.0):
        alpha = r * r
        # mu = n.h = 1 - s^2 spreads the samples where the lobe is sharp
        s = np.linspace(0.0, 1.0, 400001)
        mu = 1.0 - s * s
        f = ndf(_t(mu), alpha).numpy() * mu * 2.0 * s
        integral = 2.0 * math.pi * np.trapezoid(f, s)
        assert abs(integral - 1.0) < 2e-4, (r, integral)
        peak = float(ndf(_t([1.0]), alpha)[0])
        assert abs(peak * math.pi * alpha * alpha - 1.0) < 1e-11, (r, peak)


def test_ggx_ndf_is_normalised():
    check_ndf(R.ggx_ndf)


def test_ndf_pin_catches_missing_pi_and_wrong_power():
    with pytest.raises(AssertionError):
        check_ndf(lambda nh, a: R.ggx_ndf(nh, a) * math.pi)
    with pytest.raises(AssertionError):  # alpha = r in place of r^2 inside D
        check_ndf(lambda nh, a: R.ggx_ndf(nh, math.sqrt(a)))


def _smith_g1_exact(x, alpha):
    """Smith's masking term of the GGX distribution (Walter et al. 2007):
    G1(x) = 2 x / (x + sqrt(alpha^2 + (1 - alpha^2) x^2))."""
    return 2.0 * x / (x + np.sqrt(alpha * alpha + (1.0 - alpha * alpha) * x * x))


def check_g1(g1):
    """Schlick's form x / (x (1-k) + k) is exact at x = 1 (G1 = 1) and matches
    Smith's GGX masking term in its slope at grazing angles, 2 / alpha, only
    with k = alpha / 2; at alpha = 1 the two functions coincide."""
    for r in (0.08, 0.3, 0.5, 0.7, 1.0):
        alpha = r * r
        assert abs(float(g1(_t([1.0]), alpha)[0]) - 1.0) < 1e-15
        x = 1e-9
        slope = float(g1(_t([x]), alpha)[0]) / x
        assert abs(slope * alpha / 2.0 - 1.0) < 1e-6, (r, slope)
    xs = np.linspace(0.0, 1.0, 101)
    assert np.abs(g1(_t(xs), 1.0).numpy() - _smith_g1_exact(xs, 1.0)).max() < 1e-15


def test_smith_g1_matches_smith_ggx_limits():
    check_g1(R.smith_g1_schlick)


def test_g1_pin_catches_the_analytic_light_remap():
    # k = (r + 1)^2 / 8, the remap meant for analytic lights in Karis 2013
    def g1_bad(x, alpha):
        k = (math.sqrt(alpha) + 1.0) ** 2 / 8.0
        return x / (x * (1.0 - k) + k)
    with pytest.raises(AssertionError):
        check_g1(g1_bad)


def _fresnel_exact_dielectric(cos_i, eta):
    """Unpolarised Fresnel reflectance of a dielectric interface (air to
    relative index eta) from the Fresnel equations."""
    sin_t2 = (1.0 - cos_i * cos_i) / (eta * eta)
    cos_t = np.sqrt(1.0 - sin_t2)
    rs = (cos_i - eta * cos_t) / (cos_i + eta * cos_t)
    rp = (eta * cos_i - cos_t) / (eta * cos_i + cos_t)
    return 0.5 * (rs * rs + rp * rp)


def check_fresnel(fres):
    """Schlick's Fresnel: F0 at normal incidence, 1 at grazing incidence, and
    within 0.025 of the exact Fresnel reflectance of glass (eta 1.5, whose
    normal reflectance ((eta-1)/(eta+1))^2 is the 0.04 the paper prints) for
    every angle up to 80 degrees (powers 4 and 6 miss it by 0.10 and 0.055)."""
    f0 = _t([[0.04], [0.5], [1.0]])
    assert torch.allclose(fres(f0, _t([[1.0]])), f0, atol=1e-15)
    assert torch.allclose(fres(f0, _t([[0.0]])), torch.ones_like(f0), atol=1e-15)
    cos_i = np.cos(np.radians(np.linspace(0.0, 80.0, 81)))
    exact = _fresnel_exact_dielectric(cos_i, 1.5)
    assert abs(exact[0] - _golden()["dielectric_specular"]) < 1e-15
    approx = fres(_t(np.full_like(cos_i, 0.04)), _t(cos_i)).numpy()
    assert np.abs(approx - exact).max() < 0.025, np.abs(approx - exact).max()


def test_fresnel_schlick_limits_and_glass():
    check_fresnel(R.fresnel_schlick)


def test_fresnel_pin_catches_wrong_power():
    with pytest.raises(AssertionError):
        check_fresnel(lambda f0, vh: f0 + (1.0 - f0) * (1.0 - vh) ** 4)
    with pytest.raises(AssertionError):
        check_fresnel(lambda f0, vh: f0 + (1.0 - f0) * vh ** 5)


def check_specular_colour(spec):
    """Sec. 5.2: k_s = (1-m) 0.04 + m k_d and k_s' = (1-gamma) k_s: a
    dielectric (m = 0) reflects the printed 0.04, a metal (m = 1) its base
    colour, full specular occlusion (gamma = 1) nothing."""
    c = _golden()["dielectric_specular"]
    kd = _t([[0.9, 0.5, 0.1]])
    z, o = _t([[0.0]]), _t([[1.0]])
    assert torch.allclose(spec(kd, z, z), torch.full_like(kd, c), atol=1e-15)
    assert torch.allclose(spec(kd, z, o), kd, atol=1e-15)
    assert torch.allclose(spec(kd, o, _t([[0.3]])), torch.zeros_like(kd), atol=1e-15)
    m = _t([[0.25]])
    g = _t([[0.4]])
    # linear in the metalness between the two ends, scaled by 1 - gamma
    expect = (1 - 0.4) * (0.75 * c + 0.25 * kd)
    assert torch.allclose(spec(kd, g, m), expect, atol=1e-15)


def test_specular_colour_paper_formula():
    check_specular_colour(R.specular_colour)


def test_specular_colour_pin_catches_mistakes():
    with pytest.raises(AssertionError):
        check_specular_colour(lambda kd, g, m: (1.0 - m) * 0.04 + m * kd)       # gamma dropped
    with pytest.raises(AssertionError):
        check_specular_colour(lambda kd, g, m: (1.0 - g) * (m * 0.04 + (1.0 - m) * kd))  # m swapped


# --------------------------------------------------------------- whole GGX shading

def _albedo(shade, rough, metal, gamma, kd=1.0):
    """Directional albedo at normal view incidence, v = n: the integral over
    light directions of c(l) (radiance 1), which by symmetry is
    2 pi * integral_0^1 c(mu) d mu with mu = n.l."""
    s = np.linspace(0.0, 1.0, 200001)
    mu = 1.0 - s * s
    N = mu.size
    n = torch.zeros(N, 3, dtype=R.F64)
    n[:, 2] = 1.0
    l = torch.zeros(N, 3, dtype=R.F64)
    l[:, 0] = _t(np.sqrt(np.clip(1.0 - mu * mu, 0, None)))
    l[:, 2] = _t(mu)
    v = n.clone()
    kd_t = torch.full((N, 3), kd, dtype=R.F64)
    orm = torch.zeros(N, 3, dtype=R.F64)
    orm[:, 0], orm[:, 1], orm[:, 2] = gamma, rough, metal
    c = shade(n, l, v, kd_t, orm, torch.ones(1, 3, dtype=R.F64))[:, 0].numpy()
    return 2.0 * math.pi * np.trapezoid(c * 2.0 * s, s)


def check_shading(shade):
    """Energy: a Lambertian base colour of 1 reflects exactly what it
    receives (albedo 1), so a dielectric seen head-on has an albedo of 1 plus
    a small specular part; a white metal (F = 1) is a pure microfacet lobe
    whose albedo stays below 1 and tends to 1 as the surface gets smoother.
    A wrong factor in D F G / (4 n.l n.v) or in k_d (1-m) / pi moves these by
    2x or pi.  Head-on light and view (n = v = l, so h = n): D = 1 / (pi
    alpha^2), G = 1 and F = F0, c = k_d (1-m) / pi + F0 / (4 pi alpha^2)."""
    a = _albedo(shade, 0.5, 0.0, 1.0)
    assert 1.0 <= a < 1.001, a
    prev = 0.0
    for r in (0.5, 0.4, 0.3, 0.2, 0.1):
        a = _albedo(shade, r, 1.0, 0.0)
        assert 0.85 < a <= 1.0 + 1e-6, (r, a)
        assert a > prev
        prev = a
    assert prev > 0.999
    one = torch.tensor([[0.0, 0.0, 1.0]], dtype=R.F64)
    kd = _t([[0.6, 0.4, 0.2]])
    for (g, r, m) in ((0.0, 0.5, 0.0), (0.3, 0.8, 0.6)):
        orm = _t([[g, r, m]])
        got = shade(one, one, one, kd, orm, torch.ones(1, 3, dtype=R.F64))
        alpha = r * r
        f0 = (1 - g) * ((1 - m) * 0.04 + m * kd)
        expect = kd * (1 - m) / math.pi + f0 / (4 * math.pi * alpha * alpha)
        assert torch.allclose(got, expect, rtol=1e-12, atol=0), (got, expect)


def test_ggx_shading_energy_and_head_on_closed_form():
    check_shading(R.shade_ggx)


def _shade_variant(denom=4.0, diffuse_pi=True):
    def shade(n, l, v, kd, orm, light_rgb):
        gamma, rough, metal = orm[:, 0:1], orm[:, 1:2], orm[:, 2:3]
        alpha = torch.clamp(rough, 0.08, 1.0) ** 2
        h = R.safe_normalize(l + v)
        nl = torch.clamp(R._dot(n, l), min=0.0)
        nv = torch.clamp(R._dot(n, v), min=1e-4)
        nh = torch.clamp(R._dot(n, h), min=0.0)
        vh = torch.clamp(R._dot(v, h), min=0.0)
        G = R.smith_g1_schlick(nl, alpha) * R.smith_g1_schlick(nv, alpha)
        F = R.fresnel_schlick(R.specular_colour(kd, gamma, metal), vh)
        spec = R.ggx_ndf(nh, alpha) * F * G / (denom * torch.clamp(nl, min=1e-4) * nv)
        diffuse = kd * (1.0 - metal) / (math.pi if diffuse_pi else 1.0)
        return light_rgb * (diffuse + spec) * nl
    return shade


def test_shading_pin_catches_wrong_denominator_and_diffuse():
    check_shading(_shade_variant())          # the variant itself is the oracle's formula
    with pytest.raises(AssertionError):
        check_shading(_shade_variant(denom=2.0))
    with pytest.raises(AssertionError):
        check_shading(_shade_variant(diffuse_pi=False))


@pytest.mark.parametrize("orm", [(0.0, 0.5, 0.0), (0.3, 0.8, 0.6), (1.0, 0.3, 1.0), (0.0, 0.02, 0.0)])
def test_ggx_render_of_facing_quad_with_constant_maps(orm):
    """Through the whole render: a screen-filling quad under an orthographic
    camera with the eye far along its normal and the light along it too, so
    n = v = l at every pixel; constant k_d and (gamma, r, m) maps give the
    head-on closed form everywhere, with k_s' from the printed 0.04 (the
    roughness clamped to 0.08 below it)."""
    c = _golden()["dielectric_specular"]
    kd_v = np.array([0.6, 0.4, 0.2])
    scene = synth.Scene(S.quad_mesh(), "ggx", S.const_tex(kd_v), S.flat_normals(), S.const_tex(orm))
    W = 12
    out = R.render(scene.mesh, "ggx", loop._levels(scene.kd), loop._levels(scene.normal),
                   loop._levels(scene.orm), torch.as_tensor(scene.mesh.pos, dtype=R.F64),
                   np.eye(4, dtype=np.float32)[None], np.array([[0.0, 0.0, 1e9]]),
                   np.array([[0.0, 0.0, 1.0]]), np.ones((1, 3)), W, W, aa=False)
    g, r, m = (float(np.float32(x)) for x in orm)
    kd = kd_v.astype(np.float32).astype(np.float64)
    alpha = max(r, 0.08) ** 2
    f0 = (1 - g) * ((1 - m) * c + m * kd)
    expect = kd * (1 - m) / math.pi + f0 / (4 * math.pi * alpha * alpha)
    got = out["image"][0].numpy()
    assert got.shape == (W * W, 3)
    assert np.abs(got - expect[None]).max() <= 1e-9 * expect.max()


# --------------------------------------------------------------- screen derivatives and LOD

def _tilted_render(W=40, H=36):
    pos = np.array([(-0.9, -0.7, 0.3), (1.1, -0.5, -0.6), (-0.2, 0.9, 0.1)], dtype=np.float32)
    tri = np.array([(0, 1, 2)], dtype=np.int32)
    uvs = np.array([(0.1, 0.2), (0.8, 0.05), (0.3, 0.9)], dtype=np.float32)
    mesh = synth.Mesh(pos, tri, uvs, tri.copy())
    scene = synth.Scene(mesh, "blinn_phong", S.const_tex((1, 1, 1)), S.flat_normals(), None)
    w = S.workload(scene, scene, [(0.2, 0.3, 1.0)], [(0.0, 0.0, 1.0)], W, H)
    mvp32, eye = loop.cameras(w)
    out = R.render(mesh, "blinn_phong", loop._levels(scene.kd), loop._levels(scene.normal), None,
                   torch.as_tensor(pos, dtype=R.F64), mvp32, eye.astype(np.float64), w.light_dir,
                   w.light_rgb, W, H, keep_gbuf=True)
    return out["gbuf"][0], pos.astype(np.float64), uvs.astype(np.float64), mvp32[0].astype(np.float64)


def _uv_on_ray(px, py, p, uvs, Minv):
    """Texture coordinates where the ray through NDC point (px, py) meets the
    triangle's plane: the ray-plane hit, then its barycentric coordinates in
    the triangle (3-D areas), then the UVs blended with them."""
    one = np.ones_like(px)
    a = (Minv @ np.stack([px, py, -one, one])).T
    b = (Minv @ np.stack([px, py, one, one])).T
    a = a[:, :3] / a[:, 3:]
    b = b[:, :3] / b[:, 3:]
    nrm = np.cross(p[1] - p[0], p[2] - p[0])
    t = ((p[0] - a) @ nrm) / ((b - a) @ nrm)
    x = a + t[:, None] * (b - a)
    area = nrm @ nrm
    l0 = (np.cross(p[1] - x, p[2] - x) @ nrm) / area
    l1 = (np.cross(p[2] - x, p[0] - x) @ nrm) / area
    l2 = 1.0 - l0 - l1
    return l0[:, None] * uvs[0] + l1[:, None] * uvs[1] + l2[:, None] * uvs[2]


def check_uv_derivatives(gbuf, p, uvs, M, W, H):
    """duv/dx and duv/dy (per pixel) equal central differences, over a
    hundredth of a pixel, of the UV at which the pixel ray meets the
    triangle."""
    Minv = np.linalg.inv(M)
    pix = gbuf["pix"]
    i, j = (pix % W).astype(np.float64), (pix // W).astype(np.float64)
    h = 1e-2
    def uv_at(di, dj):
        return _uv_on_ray(2 * (i + 0.5 + di) / W - 1, 2 * (j + 0.5 + dj) / H - 1, p, uvs, Minv)
    assert np.abs(gbuf["uv"].numpy() - uv_at(0, 0)).max() < 1e-9
    fd_x = (uv_at(h, 0) - uv_at(-h, 0)) / (2 * h)
    fd_y = (uv_at(0, h) - uv_at(0, -h)) / (2 * h)
    scale = np.abs(fd_x).max() + np.abs(fd_y).max()
    assert pix.size > 100
    assert np.abs(gbuf["duv_dx"].numpy() - fd_x).max() < 1e-6 * scale
    assert np.abs(gbuf["duv_dy"].numpy() - fd_y).max() < 1e-6 * scale


def test_uv_derivatives_are_central_differences_of_ray_plane_uv():
    W, H = 40, 36
    check_uv_derivatives(*_tilted_render(W, H), W, H)


def _facing_quad_lookup(W, tex_size, H=None, seed=0):
    """A quad filling the screen under an orthographic camera (identity
    matrix, w = 1), its UV square spread over the W x H image: a pixel step
    moves u by 1/W (tex_size / W level-0 texels) and v by 1/H.  Returns the
    sampled base colour per pixel, the pixel UVs and the map's chain."""
    H = W if H is None else H
    g = np.random.default_rng(seed)
    kd = synth.Texture(g.uniform(0, 1, size=(tex_size, tex_size, 3)).astype(np.float32), "f32")
    scene = synth.Scene(S.quad_mesh(), "blinn_phong", kd, S.flat_normals(), None)
    mvp32 = np.eye(4, dtype=np.float32)[None]
    levels = loop._levels(scene.kd)
    out = R.render(scene.mesh, "blinn_phong", levels, loop._levels(scene.normal), None,
                   torch.as_tensor(scene.mesh.pos, dtype=R.F64), mvp32, np.array([[0.0, 0.0, 50.0]]),
                   np.array([[0.0, 0.0, 1.0]]), np.ones((1, 3)), W, H, keep_gbuf=True)
    gb = out["gbuf"][0]
    assert gb["pix"].size == W * H
    return gb["kd"], gb["uv"], levels


def check_lod(render_lookup):
    """With tex_size / W = 2^k level-0 texels per pixel the LOD is exactly k
    and the lookup is the bilinear sample of level k; with 64 / 24 texels per
    pixel it blends levels 1 and 2 with weight log2(64/24) - 1.  On a
    stretched footprint the longer screen axis decides."""
    for W, S_, H, k in ((16, 64, 16, 2), (8, 64, 8, 3), (32, 32, 32, 0), (16, 64, 64, 2), (64, 64, 8, 3)):
        kd, uv, levels = render_lookup(W, S_, H)
        expect = R._bilinear(levels[k], uv[:, 0], uv[:, 1])
        assert (kd - expect).abs().max() < 1e-12, (W, S_, k)
    kd, uv, levels = render_lookup(24, 64)
    f = math.log2(64 / 24) - 1.0
    a = R._bilinear(levels[1], uv[:, 0], uv[:, 1])
    b = R._bilinear(levels[2], uv[:, 0], uv[:, 1])
    assert (kd - (a + f * (b - a))).abs().max() < 1e-12


def test_lod_on_facing_quad_is_log2_of_texels_per_pixel():
    check_lod(_facing_quad_lookup)


def test_derivative_and_lod_pins_catch_one_over_w(monkeypatch):
    def half_scale(k, lam, S_, W, H):
        Ka = k[:, :, 0].sum(1, keepdim=True)
        Kb = k[:, :, 1].sum(1, keepdim=True)
        return (k[:, :, 0] - lam * Ka) / S_ * (1.0 / W), (k[:, :, 1] - lam * Kb) / S_ * (1.0 / H)
    monkeypatch.setattr(R, "screen_derivatives", half_scale)
    W, H = 40, 36
    with pytest.raises(AssertionError):
        check_uv_derivatives(*_tilted_render(W, H), W, H)
    with pytest.raises(AssertionError):
        check_lod(_facing_quad_lookup)


# --------------------------------------------------------------- loss normalisation

def check_loss(loss_fn):
    """The loss is a mean over B x H x W x 3 colour channels: a latent image
    offset by a constant c from the reference scores |c| (L1) and c^2 (L2);
    tone-mapped against a black reference, a constant e - 1 scores
    Gamma(log e) = Gamma(1) = 1, and a constant 0.001 (below the sRGB knee
    after the log) 12.92 log(1.001)."""
    g = np.random.default_rng(5)
    ref = _t(g.uniform(0.0, 2.0, size=(3, 20, 3)))
    for c in (0.25, -0.7):
        assert abs(float(loss_fn(ref + c, ref, "l1")) - abs(c)) < 1e-14
        assert abs(float(loss_fn(ref + c, ref, "l2")) - c * c) < 1e-14
    zero = torch.zeros(2, 30, 3, dtype=R.F64)
    assert abs(float(loss_fn(zero + (math.e - 1.0), zero, "l1_tonemap")) - 1.0) < 1e-14
    assert abs(float(loss_fn(zero + 1e-3, zero, "l1_tonemap")) - 12.92 * math.log(1.001)) < 1e-15
    assert abs(float(loss_fn(zero + (math.e - 1.0), zero, "l2_tonemap")) - 1.0) < 1e-14
    # only one channel of one pixel differs: the mean divides by B H W 3
    one = zero.clone()
    one[1, 7, 2] = 0.6
    assert abs(float(loss_fn(one, zero, "l1")) - 0.6 / (2 * 30 * 3)) < 1e-16


def test_loss_normalisation_closed_forms():
    check_loss(R.image_loss)


def test_loss_pin_catches_per_pixel_normalisation():
    def per_pixel(img, ref, kind):
        a, b = (R.tonemap(img), R.tonemap(ref)) if kind.endswith("tonemap") else (img, ref)
        d = a - b
        e = d.abs() if kind.startswith("l1") else d * d
        return e.sum() / (img.shape[0] * img.shape[1])
    with pytest.raises(AssertionError):
        check_loss(per_pixel)
