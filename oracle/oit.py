"""ORACLE -- test infrastructure only.

Order-independent transparency by depth peeling (Sec. 5.2, "Order-independent
transparency"), which the aggregate-geometry application (Sec. 4.4) uses to
optimise transparency: L rasterization passes, each keeping per pixel the
nearest fragment behind the previous pass's (a two-sided depth test), then
back-to-front blending starting from the background, with the silhouette
antialiasing applied to each layer.

Readings:
  * the two-sided test compares the 64-bit visibility keys (depth, then
    triangle id): layer k holds the k-th smallest fragment key of the pixel,
    so fragments of equal depth are peeled one after the other instead of
    being lost;
  * alpha comes from a one-channel map of the material, sampled with the
    same trilinear lookup as the other maps and clamped to [0, 1];
  * blending is the over operator on straight (not premultiplied) colour:
    B_k = alpha_k c_k + (1 - alpha_k) C_{k+1} where layer k covers the pixel,
    B_k = C_{k+1} where it does not; C_L = 0 (black background);
  * each layer is antialiased as the opaque render is, with its own
    visibility keys and B_k as the colours: C_k = AA_k(B_k); the image is C_0.
"""
from __future__ import annotations

import numpy as np
import torch

from . import render as R

F64 = torch.float64


def peel(tri: np.ndarray, snapv: np.ndarray, W: int, H: int, n_layers: int) -> list:
    """Keys [H,W] of layers 0..n_layers-1 of one view."""
    layers = []
    floor = None
    for _ in range(n_layers):
        keys = R.raster_peel(tri, snapv, W, H, floor)
        layers.append(keys)
        floor = keys
    return layers


def composite(colors, alphas, keys, clip, pairs, W: int, H: int, aa: bool = True):
    """Back-to-front blending of one view's layers (front first in the
    lists); returns the image [H*W,3] and the per-layer blends B_k and
    composites C_k."""
    C = torch.zeros(H * W, 3, dtype=F64)
    blends, comps = [None] * len(keys), [None] * len(keys)
    for k in reversed(range(len(keys))):
        cov = torch.from_numpy(R.key_tri(keys[k]).reshape(-1) > 0)[:, None]
        a = alphas[k][:, None]
        Bk = torch.where(cov, a * colors[k] + (1.0 - a) * C, C)
        C = R.antialias(Bk, clip, pairs[k], W, H) if aa else Bk
        blends[k], comps[k] = Bk, C
    return C, blends, comps


def render_oit(mesh, model: str, kd_levels, nrm_levels, orm_levels, alpha_levels, pos: torch.Tensor,
               mvp32: np.ndarray, eye: np.ndarray, light_dir: np.ndarray, light_rgb: np.ndarray,
               W: int, H: int, n_layers: int, adj: np.ndarray | None = None, aa: bool = True,
               frozen: dict | None = None):
    """Render B views with n_layers peeled layers.  alpha_levels: mip levels
    of the alpha map, or None (opaque).  ``frozen``: an earlier output whose
    layer keys and antialiasing pairs are reused (smooth in the parameters,
    for finite differences)."""
    tri_np = np.asarray(mesh.tri, dtype=np.int64)
    tri = torch.from_numpy(tri_np)
    uv = R._t(mesh.uv)
    uv_tri = torch.from_numpy(np.asarray(mesh.uv_tri, dtype=np.int64))
    if adj is None:
        adj = R.adjacency(tri_np)
    nrm = R.vertex_normals(pos, tri)
    tan = R.vertex_tangents(pos, tri, uv, uv_tri)
    pos32 = pos.detach().numpy().astype(np.float32)
    images, keys_all, pairs_all, colors_all, alphas_all, blends_all, comps_all = [], [], [], [], [], [], []
    for b in range(mvp32.shape[0]):
        M = R._t(mvp32[b].astype(np.float64))
        clip = torch.cat([pos, torch.ones(pos.shape[0], 1, dtype=F64)], dim=1) @ M.T
        sv = R.snap(pos32, mvp32[b], W, H)
        if frozen is None:
            keys = peel(tri_np, sv, W, H, n_layers)
            _, _, orient = R.raster(tri_np, sv, W, H)
            pairs = [R.aa_pairs(k, tri_np, sv, orient, adj) for k in keys]
        else:
            keys, pairs = frozen["keys"][b], frozen["pairs"][b]
        colors, alphas = [], []
        for k in keys:
            c, a, _ = R.shade_view(k, tri, uv, uv_tri, pos, nrm, tan, clip, model, kd_levels, nrm_levels,
                                   orm_levels, eye[b], light_dir[b], light_rgb[b], W, H, 1,
                                   alpha_levels=alpha_levels)
            if a is None:
                a = torch.from_numpy((R.key_tri(k).reshape(-1) > 0).astype(np.float64))
            colors.append(c)
            alphas.append(a)
        img, blends, comps = composite(colors, alphas, keys, clip, pairs, W, H, aa)
        images.append(img)
        keys_all.append(keys)
        pairs_all.append(pairs)
        colors_all.append(colors)
        alphas_all.append(alphas)
        blends_all.append(blends)
        comps_all.append(comps)
    return dict(image=torch.stack(images), keys=keys_all, pairs=pairs_all, colors=colors_all, alphas=alphas_all,
                blends=blends_all, comps=comps_all)
