"""ORACLE -- test infrastructure only.

One optimisation step of Eq. 1 (Sec. 3) for a synthetic workload: render the
reference under the sampled cameras and lights, render the latent model,
score the image loss (Sec. 5.3), differentiate it w.r.t. the latent
parameters (vertex positions and level-0 texels) and apply Adam (Sec. 5.3).
"""
from __future__ import annotations

import types

import numpy as np
import torch

from . import oit as O
from . import render as R
from . import skin as K
from . import tess as T


def cameras(w):
    """float32 MVPs and eyes of a workload's views (Sec. 3 camera sampling)."""
    mvp, eye = R.look_at_mvp(w.dirs, w.dist, w.fov_deg, w.width, w.height)
    return mvp.astype(np.float32), eye.astype(np.float32)


def _levels(tex, param=None):
    return R.texture_levels(tex.data, tex.fmt, param, getattr(tex, "chain", None))


def render_scene(scene, mvp32, eye, w, pos=None, params=None, aa=True, frozen=None, msaa=1):
    params = params or {}
    if pos is None:
        pos = torch.as_tensor(scene.mesh.pos, dtype=R.F64)
    kd = _levels(scene.kd, params.get("kd"))
    nm = _levels(scene.normal, params.get("normal"))
    orm = _levels(scene.orm, params.get("orm")) if scene.orm is not None else None
    return R.render(scene.mesh, scene.model, kd, nm, orm, pos, mvp32,
                    np.asarray(eye, dtype=np.float64), np.asarray(w.light_dir, dtype=np.float64),
                    np.asarray(w.light_rgb, dtype=np.float64), w.width, w.height, aa=aa, frozen=frozen,
                    msaa=msaa)


def tess_table(w):
    """The oracle's own tessellation of the latent base mesh (Sec. 5.1)."""
    m = w.latent.mesh
    key = (id(m), w.tess_levels)
    if getattr(w, "_oracle_tess", (None,))[0] != key:
        w._oracle_tess = (key, T.build(m.tri, m.uv_tri, m.uv, m.pos.shape[0], w.tess_levels))
    return w._oracle_tess[1]


def _round32(x, on=True):
    """The renderer's vertex format is float32: positions computed by a mesh
    operation are rounded to it, and the adjoint passes through unchanged."""
    return x + (x.detach().to(torch.float32).to(R.F64) - x.detach()) if on else x


def skinned_positions(w, pos, weights, frame=None):
    """Eq. 2 with the bone transforms of the workload's animation frame."""
    f = w.frame if frame is None else frame
    return K.skin(pos, weights, torch.as_tensor(w.rig.bones[f], dtype=R.F64))


def render_latent(w, mvp32, eye, params=None, aa=True, frozen=None, round32=True):
    """Latent render; with tessellation the base positions and the
    displacement map are mapped to displaced positions first (Eq. 3); with a
    rig the bind-pose positions are skinned with the latent weights (Eq. 2).
    Positions a mesh operation computes are rounded to float32 (``round32``)."""
    params = params or {}
    msaa = getattr(w, "msaa", 1)
    if getattr(w, "oit_layers", 0):
        s = w.latent
        pos = params.get("pos", torch.as_tensor(s.mesh.pos, dtype=R.F64))
        al = _levels(s.alpha, params.get("alpha")) if s.alpha is not None else None
        orm = _levels(s.orm, params.get("orm")) if s.orm is not None else None
        return O.render_oit(s.mesh, s.model, _levels(s.kd, params.get("kd")), _levels(s.normal, params.get("normal")),
                            orm, al, pos, mvp32, np.asarray(eye, dtype=np.float64),
                            np.asarray(w.light_dir, dtype=np.float64), np.asarray(w.light_rgb, dtype=np.float64),
                            w.width, w.height, w.oit_layers, aa=aa, frozen=frozen)
    if getattr(w, "rig", None) is not None:
        pos0 = params.get("pos", torch.as_tensor(w.latent.mesh.pos, dtype=R.F64))
        wts = params.get("weights", torch.as_tensor(w.weights, dtype=R.F64))
        vs = _round32(skinned_positions(w, pos0, wts), round32)
        out = render_scene(w.latent, mvp32, eye, w, pos=vs, params=params, aa=aa, frozen=frozen, msaa=msaa)
        out["pos"] = vs
        return out
    if not w.tess_levels:
        return render_scene(w.latent, mvp32, eye, w, pos=params.get("pos"), params=params, aa=aa,
                            frozen=frozen, msaa=msaa)
    table = tess_table(w)
    base = w.latent.mesh
    pos0 = params.get("pos", torch.as_tensor(base.pos, dtype=R.F64))
    disp = params.get("disp", torch.as_tensor(w.disp.data, dtype=R.F64))
    vd = _round32(T.displaced_positions(pos0, base, table, disp), round32)
    mesh = types.SimpleNamespace(pos=None, tri=table["tri"], uv=table["uv"], uv_tri=table["uv_tri"])
    scene = types.SimpleNamespace(mesh=mesh, model=w.latent.model, kd=w.latent.kd,
                                  normal=w.latent.normal, orm=w.latent.orm)
    out = render_scene(scene, mvp32, eye, w, pos=vd, params=params, aa=aa, frozen=frozen, msaa=msaa)
    out["pos"] = vd
    return out


def reference_image(w, mvp32=None, eye=None):
    """Reference render; with ``ref_ssaa`` = k it is rendered at k times the
    resolution (the cameras' aspect is unchanged) and box-filtered (Sec. 4.2)."""
    if mvp32 is None:
        mvp32, eye = cameras(w)
    k = getattr(w, "ref_ssaa", 1)
    with torch.no_grad():
        pos = None
        if getattr(w, "rig", None) is not None:
            pos = _round32(skinned_positions(w, torch.as_tensor(w.ref.mesh.pos, dtype=R.F64),
                                             torch.as_tensor(w.rig.ref_weights, dtype=R.F64)))
        if k == 1:
            return render_scene(w.ref, mvp32, eye, w, pos=pos)["image"]
        big = types.SimpleNamespace(width=w.width * k, height=w.height * k, light_dir=w.light_dir,
                                    light_rgb=w.light_rgb)
        img = render_scene(w.ref, mvp32, eye, big, pos=pos)["image"]
        B, H, W = img.shape[0], w.height, w.width
        return img.reshape(B, H, k, W, k, 3).mean(dim=(2, 4)).reshape(B, H * W, 3)


def latent_params(w):
    """float64 leaf tensors of the optimised latent parameters."""
    out = {}
    s = w.latent
    for name in w.optimize:
        if name == "pos":
            out["pos"] = torch.tensor(s.mesh.pos, dtype=R.F64, requires_grad=True)
        elif name == "disp":
            out["disp"] = torch.tensor(w.disp.data, dtype=R.F64, requires_grad=True)
        elif name == "weights":
            out["weights"] = torch.tensor(w.weights, dtype=R.F64, requires_grad=True)
        else:
            tex = getattr(s, name)
            assert tex.fmt == "f32", "only float32 maps are optimised"
            src = tex.chain if getattr(tex, "chain", None) is not None else tex.data
            out[name] = torch.tensor(src, dtype=R.F64, requires_grad=True)
    return out


def loss_and_grads(w, ref_img, mvp32=None, eye=None, params=None, aa=True):
    """Forward + backward of the latent render: (loss, grads, render dict)."""
    if mvp32 is None:
        mvp32, eye = cameras(w)
    params = params if params is not None else latent_params(w)
    out = render_latent(w, mvp32, eye, params, aa=aa)
    loss = R.image_loss(out["image"], ref_img, w.loss)
    leaves = [params[k] for k in params]
    gl = torch.autograd.grad(loss, leaves, allow_unused=True)
    grads = {k: (g if g is not None else torch.zeros_like(params[k])) for k, g in zip(params, gl)}
    return loss.detach(), grads, out


def adam_update(params, grads, state, t, lr):
    """Adam on every parameter (Sec. 5.3); state maps name -> (m, v)."""
    new = {}
    for k, p in params.items():
        m, v = state.get(k, (np.zeros(p.shape), np.zeros(p.shape)))
        pn, m, v = R.adam(p.detach().numpy(), grads[k].numpy(), m, v, t, lr)
        state[k] = (m, v)
        new[k] = pn
    return new, state
