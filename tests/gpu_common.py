"""Shared set-up of GPU parity tests: the same seeded inputs go to the HIP
path (through the C ABI) and to the oracle.  Cameras come from the oracle
so that no oracle input is produced by the code under test."""
from __future__ import annotations

import numpy as np
import torch

from oracle import loop as OL
from oracle import render as R


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).reshape(-1)
    b = np.asarray(b, dtype=np.float64).reshape(-1)
    n = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (n if n > 0 else 1.0))


class GpuScene:
    """A workload uploaded for the HIP path."""

    def __init__(self, w, ctx, mvp32=None, eye=None):
        from paper_2104_03989_amd import adr
        self.adr = adr
        self.w = w
        self.ctx = ctx
        if mvp32 is None:
            mvp32, eye = OL.cameras(w)
        self.mvp32, self.eye = mvp32, eye
        self.views = adr.DeviceViews(mvp32, eye, w.light_dir, w.light_rgb, w.width, w.height)
        self.ref_mesh = adr.DeviceMesh(w.ref.mesh)
        self.ref_mat = adr.DeviceMaterial(w.ref, ctx=ctx)
        self.lat_mesh = adr.DeviceMesh(w.latent.mesh)
        self.lat_mat = adr.DeviceMaterial(w.latent, ctx=ctx)

    def render(self, which="latent", ref=None, flags=0, **kw):
        adr = self.adr
        mesh = self.lat_mesh if which == "latent" else self.ref_mesh
        mat = self.lat_mat if which == "latent" else self.ref_mat
        out = adr.render_fwd(self.ctx, mesh, mat, self.views, ref=ref, loss=self.w.loss, flags=flags, **kw)
        torch.cuda.synchronize()
        return out

    def grads(self, out, names=("pos", "kd", "normal", "orm"), flags=0):
        adr = self.adr
        g = {"pos": torch.zeros_like(self.lat_mesh.pos) if "pos" in names else None}
        for n in ("kd", "normal", "orm"):
            tex = getattr(self.lat_mat, n)
            g[n] = tex.grad_buffer() if (n in names and tex is not None and tex.fmt == adr.TEX_F32) else None
        adr.render_bwd(self.ctx, self.lat_mesh, self.lat_mat, self.views, out, g, flags=flags)
        torch.cuda.synchronize()
        res = {}
        for n, t in g.items():
            if t is None:
                continue
            if n == "pos":
                res[n] = t.cpu().numpy()
            else:
                tex = getattr(self.lat_mat, n)
                res[n] = t[:tex.size * tex.size].cpu().numpy().reshape(tex.size, tex.size, -1)
                res[n + "_coarse_max"] = float(t[tex.size * tex.size:].abs().max()) if t.shape[0] > tex.size ** 2 else 0.0
        return res


def oracle_keys(w, scene, mvp32):
    """Oracle visibility of every view: keys [B,H,W] uint64, coverage."""
    keys, cov = [], []
    for b in range(mvp32.shape[0]):
        sv = R.snap(scene.mesh.pos, mvp32[b], w.width, w.height)
        k, c, _ = R.raster(scene.mesh.tri, sv, w.width, w.height)
        keys.append(k)
        cov.append(c)
    return np.stack(keys), np.stack(cov)


class TessGpuScene(GpuScene):
    """A workload whose latent is a tessellated, displaced base mesh: the
    latent render runs tess_fwd first, the gradients end in tess_bwd."""

    def __init__(self, w, ctx, mvp32=None, eye=None):
        super().__init__(w, ctx, mvp32, eye)
        adr = self.adr
        self.ts = adr.DeviceTess(w.latent.mesh, w.tess_levels)
        self.disp = adr.DeviceTexture(w.disp.data, "f32", levels=1)
        self.lat_mesh = self.ts.mesh

    def render(self, which="latent", ref=None, flags=0, **kw):
        if which == "latent":
            self.adr.tess_fwd(self.ctx, self.ts, self.disp)
        return super().render(which, ref, flags, **kw)

    def grads(self, out, names=("pos", "disp", "normal")):
        adr = self.adr
        g = {"pos": torch.zeros_like(self.ts.mesh.pos)}
        for n in ("kd", "normal", "orm"):
            tex = getattr(self.lat_mat, n)
            g[n] = tex.grad_buffer() if (n in names and tex is not None and tex.fmt == adr.TEX_F32) else None
        adr.render_bwd(self.ctx, self.ts.mesh, self.lat_mat, self.views, out, g)
        g_base = torch.zeros_like(self.ts.base.pos)
        g_disp = torch.zeros_like(self.disp.data)
        adr.tess_bwd(self.ctx, self.ts, self.disp, g["pos"], g_base, g_disp)
        torch.cuda.synchronize()
        S = self.disp.size
        res = {"pos": g_base.cpu().numpy(), "disp": g_disp.cpu().numpy().reshape(S, S, 1)}
        for n in ("kd", "normal", "orm"):
            t = g[n]
            if t is None:
                continue
            tex = getattr(self.lat_mat, n)
            res[n] = t[:tex.size * tex.size].cpu().numpy().reshape(tex.size, tex.size, -1)
            res[n + "_coarse_max"] = float(t[tex.size * tex.size:].abs().max()) if t.shape[0] > tex.size ** 2 else 0.0
        return res


def oracle_tess_keys(w, mvp32):
    """Oracle visibility of the tessellated, displaced latent of every view."""
    from oracle import tess as T
    table = OL.tess_table(w)
    base = w.latent.mesh
    with torch.no_grad():
        vd = T.displaced_positions(torch.as_tensor(base.pos, dtype=R.F64), base, table,
                                   torch.as_tensor(w.disp.data, dtype=R.F64))
    pos32 = vd.numpy().astype(np.float32)
    keys, cov = [], []
    for b in range(mvp32.shape[0]):
        sv = R.snap(pos32, mvp32[b], w.width, w.height)
        k, c, _ = R.raster(table["tri"], sv, w.width, w.height)
        keys.append(k)
        cov.append(c)
    return np.stack(keys), np.stack(cov), vd.numpy()


class SkinGpuScene(GpuScene):
    """A workload with a rig: both meshes are skinned (Eq. 2) with the bone
    transforms of ``w.frame`` before they are rendered; the latent's
    gradients end in skin_bwd (bind-pose positions and weights)."""

    def __init__(self, w, ctx, mvp32=None, eye=None):
        super().__init__(w, ctx, mvp32, eye)
        self.bones = torch.from_numpy(np.ascontiguousarray(w.rig.bones[w.frame])).cuda()
        self.ref_bind = torch.from_numpy(w.ref.mesh.pos).cuda()
        self.ref_w = torch.from_numpy(np.ascontiguousarray(w.rig.ref_weights)).cuda()
        self.lat_bind = torch.from_numpy(w.latent.mesh.pos).cuda()
        self.lat_w = torch.from_numpy(np.ascontiguousarray(w.weights)).cuda()
        self.blend = torch.empty(self.lat_bind.shape[0], 12, dtype=torch.float32, device="cuda")

    def render(self, which="latent", ref=None, flags=0, **kw):
        if which == "latent":
            self.adr.skin_fwd(self.ctx, self.lat_bind, self.lat_w, self.bones, out=self.lat_mesh.pos, blend=self.blend)
        else:
            self.adr.skin_fwd(self.ctx, self.ref_bind, self.ref_w, self.bones, out=self.ref_mesh.pos)
        return super().render(which, ref, flags, **kw)

    def grads(self, out, names=("pos", "weights", "kd", "normal"), flags=0):
        adr = self.adr
        g = {"pos": torch.zeros_like(self.lat_mesh.pos)}
        for n in ("kd", "normal", "orm"):
            tex = getattr(self.lat_mat, n)
            g[n] = tex.grad_buffer() if (n in names and tex is not None and tex.fmt == adr.TEX_F32) else None
        adr.render_bwd(self.ctx, self.lat_mesh, self.lat_mat, self.views, out, g, flags=flags)
        g_bind = torch.zeros_like(self.lat_bind)
        g_w = torch.zeros_like(self.lat_w)
        adr.skin_bwd(self.ctx, self.lat_bind, self.bones, self.blend, g["pos"], g_pos=g_bind, g_weights=g_w)
        torch.cuda.synchronize()
        res = {"pos": g_bind.cpu().numpy(), "weights": g_w.cpu().numpy(), "g_skinned_max": float(g["pos"].abs().max())}
        for n in ("kd", "normal", "orm"):
            t = g[n]
            if t is None:
                continue
            tex = getattr(self.lat_mat, n)
            res[n] = t[:tex.size * tex.size].cpu().numpy().reshape(tex.size, tex.size, -1)
        return res


def oracle_skinned_keys(w, mvp32, which="latent"):
    """Oracle visibility of a skinned mesh in every view, and its float64
    skinned positions."""
    from oracle import skin as K
    scene = w.latent if which == "latent" else w.ref
    wts = w.weights if which == "latent" else w.rig.ref_weights
    with torch.no_grad():
        vs = K.skin(torch.as_tensor(scene.mesh.pos, dtype=R.F64), torch.as_tensor(wts, dtype=R.F64),
                    torch.as_tensor(w.rig.bones[w.frame], dtype=R.F64)).numpy()
    pos32 = vs.astype(np.float32)
    keys, cov = [], []
    for b in range(mvp32.shape[0]):
        sv = R.snap(pos32, mvp32[b], w.width, w.height)
        k, c, _ = R.raster(scene.mesh.tri, sv, w.width, w.height)
        keys.append(k)
        cov.append(c)
    return np.stack(keys), np.stack(cov), vs


def oracle_grads_and_reach(w, ref, mvp32, eye, tau=1e-5, seed=0):
    """The oracle's loss and gradients of the latent (as OL.loss_and_grads)
    and, from the same forward pass, the entries of each optimised parameter
    that receive gradient from a pixel channel whose L1 residual
    |T(x) - T(ref)| lies within tau (the forward tolerance) of zero.  There
    float32 and float64 may disagree on the sign of the residual, and so on
    the sign of that channel's whole contribution to the gradient (L1 is not
    differentiable at 0); a per-entry bound cannot hold for them.  They are
    found by a second backward pass, of the sum over those channels of T(x)
    times a random weight in [1, 2): an entry is reached iff its gradient is
    non-zero.  Squared losses have no such entries.
    Returns (loss, grads, render dict, reach, number of such channels)."""
    params = OL.latent_params(w)
    out = OL.render_latent(w, mvp32, eye, params)
    img = out["image"]
    loss = R.image_loss(img, ref, w.loss)
    leaves = [params[k] for k in params]
    gl = torch.autograd.grad(loss, leaves, allow_unused=True, retain_graph=True)
    grads = {k: (g if g is not None else torch.zeros_like(params[k])) for k, g in zip(params, gl)}
    reach = {k: np.zeros(tuple(p.shape), dtype=bool) for k, p in params.items()}
    n_amb = 0
    if w.loss.startswith("l1"):
        tm = w.loss.endswith("tonemap")
        a = R.tonemap(img) if tm else img
        b = R.tonemap(ref) if tm else ref
        amb = (a - b).detach().abs() < tau
        n_amb = int(amb.sum())
        if n_amb:
            r = 1.0 + torch.from_numpy(np.random.default_rng(seed).random(tuple(a.shape)))
            obj = (a * (amb.to(a.dtype) * r)).sum()
            gl = torch.autograd.grad(obj, leaves, allow_unused=True)
            for k, g in zip(params, gl):
                if g is not None:
                    reach[k] = (g.detach().abs() > 0).numpy()
    return loss.detach(), grads, out, reach, n_amb


def check_adam_first_step(name, p0, p_new, g_o, lr, delta, exempt=None, eps=1e-8, say=print):
    """A first Adam step from zero moments, p1 = p0 - lr g / (|g| + eps)
    (the bias corrections cancel), against the oracle's gradient g_o, entry
    by entry.  If the gradient behind p_new is within delta of g_o, the two
    steps differ by at most lr min(2, 4 delta / (|g_o| + eps)): the step is
    smooth in g except at 0, where its sign may flip, so entries whose
    oracle gradient is within a few delta of zero get a loose bound (at
    most 2 lr, any valid step).  ``exempt`` entries (see
    oracle_grads_and_reach) get 2 lr.  float32 rounding adds a few units in the
    last place of p and of the step."""
    p0 = np.asarray(p0, dtype=np.float64).reshape(-1)
    p_new = np.asarray(p_new, dtype=np.float64).reshape(-1)
    g_o = np.asarray(g_o, dtype=np.float64).reshape(-1)
    p_o = p0 - lr * g_o / (np.abs(g_o) + eps)
    bound = lr * np.minimum(2.0, 4.0 * delta / (np.abs(g_o) + eps))
    if exempt is not None:
        bound = np.where(np.asarray(exempt).reshape(-1), 2.0 * lr, bound)
    bound = bound + 4 * np.spacing(np.abs(p0).astype(np.float32)).astype(np.float64) + 1e-6 * lr
    err = np.abs(p_new - p_o)
    loose = bound > 1e-2 * lr
    n_ex = 0 if exempt is None else int(np.asarray(exempt).sum())
    say(f"  adam {name}: max error {err.max() / lr:.3g} lr; {int(loose.sum())} of {err.size} entries with a "
        f"loose bound ({n_ex} reached by ambiguous L1 residuals)")
    bad = err > bound
    assert not bad.any(), (name, int(bad.sum()), float((err / bound).max()))


def check_grad_entries(name, got, exp, rel_tol, sup_tol, exempt=None, say=print):
    """Relative L2 error within rel_tol, and every entry outside ``exempt``
    within sup_tol times the largest oracle entry."""
    got = np.asarray(got, dtype=np.float64).reshape(-1)
    exp = np.asarray(exp, dtype=np.float64).reshape(-1)
    e = rel_l2(got, exp)
    diff = np.abs(got - exp)
    if exempt is not None:
        diff = np.where(np.asarray(exempt).reshape(-1), 0.0, diff)
    sup = float(diff.max() / max(np.abs(exp).max(), 1e-300)) if diff.size else 0.0
    n_ex = 0 if exempt is None else int(np.asarray(exempt).sum())
    say(f"  grad {name}: rel-L2 {e:.3g}, max entry error {sup:.3g} of the largest entry ({n_ex} exempt)")
    assert e < rel_tol, (name, e)
    assert sup < sup_tol, (name, sup)
