"""Central finite differences of the oracle's FP64 loss pin its gradients
(autograd of the forward pass) w.r.t. vertex positions and texels."""
import numpy as np
import pytest
import torch

from oracle import loop
from oracle import render as R
from tests import oracle_scenes as S


def _loss_at(w, ref, mvp32, eye, params):
    out = loop.render_scene(w.latent, mvp32, eye, w, pos=params.get("pos"), params=params)
    loss = R.image_loss(out["image"], ref, w.loss)
    sig = (R.key_tri(out["keys"]), [tuple(map(np.ndarray.tobytes, p)) for p in out["pairs"]])
    return float(loss), sig


def _same(a, b):
    return np.array_equal(a[0], b[0]) and a[1] == b[1]


@pytest.mark.parametrize("model,loss", [("blinn_phong", "l1"), ("ggx", "l1_tonemap"), ("ggx", "l2")])
def test_central_differences_match_autograd(model, loss):
    w = S.tiny_sphere_workload(model, nu=2, res=24, views=2, tex=8, loss=loss, seed=1)
    mvp32, eye = loop.cameras(w)
    ref = loop.reference_image(w, mvp32, eye)
    params = loop.latent_params(w)
    L0, grads, out0 = loop.loss_and_grads(w, ref, mvp32, eye, params)
    base = {k: v.detach().clone() for k, v in params.items()}
    _, sig0 = _loss_at(w, ref, mvp32, eye, base)
    g = np.random.default_rng(7)
    h = 1e-4
    checked = 0
    for name in params:
        flat = grads[name].reshape(-1)
        scale = float(flat.abs().max())
        assert scale > 0, name
        # probe the largest entries and some random ones
        order = torch.argsort(flat.abs(), descending=True)[:6].tolist()
        order += g.integers(0, flat.numel(), size=4).tolist()
        for idx in order:
            ad = float(flat[idx])
            fds = []
            # h = 1e-4 first; a kink of the piecewise-smooth loss (a bilinear
            # texel crossing, |d| at 0) within +-h is retried at h = 1e-6
            for hh in (h, 1e-6):
                vals = []
                ok = True
                for sgn in (1, -1):
                    p = {k: v.clone() for k, v in base.items()}
                    p[name].reshape(-1)[idx] += sgn * hh
                    Lh, sig = _loss_at(w, ref, mvp32, eye, p)
                    ok &= _same(sig, sig0)
                    vals.append(Lh)
                if not ok:
                    break  # visibility or AA decisions changed: FD not valid
                fds.append((vals[0] - vals[1]) / (2 * hh))
                if abs(fds[-1] - ad) <= 1e-6 * scale + 1e-4 * abs(ad):
                    break
            if not fds or len(fds) < 2 and abs(fds[-1] - ad) > 1e-6 * scale + 1e-4 * abs(ad):
                continue
            assert abs(fds[-1] - ad) <= 1e-6 * scale + 1e-4 * abs(ad), (name, idx, fds, ad, scale)
            checked += 1
    assert checked >= 25


def _tess_loss_at(w, ref, mvp32, eye, params, frozen=None):
    out = loop.render_latent(w, mvp32, eye, params, frozen=frozen, round32=False)
    loss = R.image_loss(out["image"], ref, w.loss)
    sig = (R.key_tri(out["keys"]), [tuple(map(np.ndarray.tobytes, p)) for p in out["pairs"]])
    return float(loss), sig


def test_tessellated_crop_central_differences():
    # Eq. 3 end to end on one base triangle split into 64: d loss / d base
    # positions (through the displaced positions and the base normals) and
    # d loss / d displacement texels, at h = 1e-4.  A shift of a base vertex
    # moves all 45 tessellated vertices, so its +-h renders rarely keep every
    # snapped coordinate; those are differenced with the base render's
    # visibility and antialiasing pairs held fixed, which is the function
    # the adjoint differentiates.
    w = S.tess_crop_workload(res=32, views=2, seed=1)
    mvp32, eye = loop.cameras(w)
    ref = loop.reference_image(w, mvp32, eye)
    params = loop.latent_params(w)
    _, grads, out = loop.loss_and_grads(w, ref, mvp32, eye, params)
    assert int((R.key_tri(out["keys"]) > 0).sum()) > 200          # the crop covers the views
    base = {k: v.detach().clone() for k, v in params.items()}
    _, sig0 = _tess_loss_at(w, ref, mvp32, eye, base)
    g = np.random.default_rng(3)
    checked = {}
    for name in ("pos", "disp"):
        flat = grads[name].reshape(-1)
        scale = float(flat.abs().max())
        assert scale > 0, name
        idxs = list(range(flat.numel())) if name == "pos" else \
            torch.argsort(flat.abs(), descending=True)[:10].tolist() + g.integers(0, flat.numel(), 4).tolist()
        for idx in idxs:
            ad = float(flat[idx])
            vals, ok = [], True
            for sgn in (1, -1):
                p = {k: v.clone() for k, v in base.items()}
                p[name].reshape(-1)[idx] += sgn * 1e-4
                Lh, sig = _tess_loss_at(w, ref, mvp32, eye, p, frozen=out if name == "pos" else None)
                ok &= name == "pos" or _same(sig, sig0)
                vals.append(Lh)
            if not ok:
                continue
            fd = (vals[0] - vals[1]) / 2e-4
            assert abs(fd - ad) <= 1e-5 * scale + 1e-3 * abs(ad), (name, idx, fd, ad, scale)
            checked[name] = checked.get(name, 0) + 1
    assert checked.get("pos", 0) == 9 and checked.get("disp", 0) >= 8, checked
