"""Pins of the oracle's multisampled visibility (Sec. 5.2, "Antialiasing"):
samples of one pixel on one triangle share the pixel-centre shading, and a
vertical silhouette edge resolves to the exact covered area of the pixel
times that shading."""
import math

import numpy as np
import pytest
import torch

from oracle import loop as OL
from oracle import render as R
from paper_2104_03989_amd import synth
from tests import oracle_scenes as S


def _edge_scene(W, edge_px, m):
    # one camera-facing triangle whose only visible edge is vertical at
    # pixel coordinate edge_px (the camera looks down -z from (0, 0, 3))
    half = 3.0 * math.tan(math.radians(22.5))
    xe = (2.0 * edge_px / W - 1.0) * half
    pos = np.array([[-5.0, -5.0, 0.0], [xe, -5.0, 0.0], [xe, 5.0, 0.0]], np.float32)
    tri = np.array([[0, 1, 2]], np.int32)
    uv = np.array([[0.1, 0.1], [0.9, 0.1], [0.9, 0.9]], np.float32)
    mesh = synth.Mesh(pos, tri, uv, tri.copy())
    scene = synth.Scene(mesh, "blinn_phong", S.const_tex((0.8, 0.5, 0.3)), S.flat_normals(), None)
    w = S.workload(scene, scene, [(0, 0, 1)], [(0.2, 0.3, 1.0)], W, W)
    w.msaa = m
    return w


@pytest.mark.parametrize("m", [2, 4])
def test_vertical_edge_resolves_to_exact_coverage(m):
    # The edge crosses pixel x0 at 0.6 of its width, between two sample
    # columns of that pixel: each sample row box-filters to exactly the
    # covered width, so the pixel is 0.6 times its centre shading, and a
    # fully covered pixel equals the one-sample shading at its centre.
    W, x0, frac = 16, 9, 0.6
    w = _edge_scene(W, x0 + frac, m)
    mvp32, eye = OL.cameras(w)
    c1 = OL.render_latent(_edge_scene(W, x0 + frac, 1), mvp32, eye)["color"][0].reshape(W, W, 3)
    out = OL.render_latent(w, mvp32, eye)
    img = out["image"][0].reshape(W, W, 3).detach()
    rows = slice(2, W - 2)
    assert torch.allclose(img[rows, :x0], c1[rows, :x0], rtol=1e-12, atol=0)
    assert float(img[rows, x0 + 1:].abs().max()) == 0.0
    col = out["color"][0].detach().reshape(W, m, W, m, 3)
    inside = int(frac * m)          # sample columns of pixel x0 left of the edge
    for r in range(rows.start, rows.stop):
        c = col[r, :, x0, :inside].reshape(-1, 3)
        assert torch.equal(c, c[:1].expand_as(c))          # one shading per pixel
        assert float(col[r, :, x0, inside:].abs().max()) == 0.0
        # the edge vertex is stored in float32: its position holds to ~1e-7 pixel
        np.testing.assert_allclose(img[r, x0].numpy(), frac * c[0].numpy(), rtol=1e-6)


def test_samples_of_a_pixel_share_the_pixel_shading():
    w = S.tiny_sphere_workload("ggx", nu=3, res=20, views=1, tex=16, seed=4)
    w.msaa = 4
    mvp32, eye = OL.cameras(w)
    out = OL.render_latent(w, mvp32, eye)
    ids = R.key_tri(out["keys"][0]).reshape(20, 4, 20, 4).transpose(0, 2, 1, 3).reshape(400, 16)
    col = out["color"][0].detach().reshape(20, 4, 20, 4, 3).permute(0, 2, 1, 3, 4).reshape(400, 16, 3)
    checked = 0
    for p in range(400):
        for t in set(ids[p].tolist()) - {0}:
            sel = torch.from_numpy(ids[p] == t)
            cs = col[p][sel]
            assert torch.equal(cs, cs[:1].expand_as(cs))
            checked += 1
    assert checked > 100
