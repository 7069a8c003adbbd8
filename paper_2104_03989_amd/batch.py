"""Batched stepping of many meshes of uneven size.

Every mesh keeps its own device state (meshes, maps, gradients, Adam state,
the cameras and lights of every step).  One step renders each mesh's
reference and latent views, scores the image loss and back-propagates
(Sec. 3, Eq. 1), then Adam updates the parameters of all meshes (Sec. 5.3):
one launch over every mesh's positions, and the maps four per launch with
their mip chains' adjoint and rebuild fused in.

Three forms of the same step:
- ``launch`` (the batched form): two library batches (adr_batch_*), one of
  every mesh's reference render and one of every latent render with its
  backward, so that each stage of the render runs as one launch over the
  work of all meshes; the three calls are captured once as a HIP graph
  (through torch.cuda.CUDAGraph) and a step is a copy of that step's cameras
  into the buffers the graph reads, one graph launch and the Adam launches.
- ``streams``: the per-mesh launches of every mesh captured as one graph,
  spread over several streams, each with its own library context.
- plain (``step_plain``): one mesh at a time, each with its own launches.
The rasterizer's work split of each mesh's renders comes from the autotuner.
"""
from __future__ import annotations

import numpy as np
import torch

from . import adr
from .autotune import DEFAULT, Tuner


class MeshState:
    """Device state of one mesh of a batch."""

    def __init__(self, w, ctx: adr.Context, n_steps: int, seed: int, det: bool = False):
        self.w = w
        B, H, W = w.dirs.shape[0], w.height, w.width
        g = np.random.Generator(np.random.PCG64(seed))
        dirs = g.normal(size=(n_steps, B, 3))
        lights = g.normal(size=(n_steps, B, 3))
        lights /= np.linalg.norm(lights, axis=2, keepdims=True)
        mvps, eyes = zip(*[adr.views_build(dirs[t], w.dist, w.fov_deg, W, H) for t in range(n_steps)])
        dev = lambda x: torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()
        self.mvp_all, self.eye_all, self.light_all = dev(np.stack(mvps)), dev(np.stack(eyes)), dev(lights)
        # the buffers every render of a step reads (a captured graph reads them too)
        self.mvp, self.eye, self.light = self.mvp_all[0].clone(), self.eye_all[0].clone(), self.light_all[0].clone()
        self.views = adr.DeviceViews(self.mvp, self.eye, self.light, dev(np.ones((B, 3))), W, H)
        self.ref_mesh = adr.DeviceMesh(w.ref.mesh)
        self.ref_mesh.precompute_frame(ctx)
        self.ref_mat = adr.DeviceMaterial(w.ref, ctx=ctx)
        self.lat_mesh = adr.DeviceMesh(w.latent.mesh)
        self.lat_mat = adr.DeviceMaterial(w.latent, ctx=ctx)
        self.det = adr.DETERMINISTIC if det else 0
        self.grads = {"pos": torch.zeros_like(self.lat_mesh.pos) if "pos" in w.optimize else None}
        params = [(self.lat_mesh.pos, self.grads["pos"])] if self.grads["pos"] is not None else []
        # mip-mapped maps: Adam fused with the chain's adjoint and rebuild
        # (the backward defers the adjoint; the forward needs no rebuild)
        self.maps = []
        for name in ("kd", "normal", "orm"):
            tex = getattr(self.lat_mat, name)
            if name in w.optimize and tex is not None and tex.fmt == adr.TEX_F32:
                self.grads[name] = tex.grad_buffer()
                n0 = tex.size * tex.size
                self.maps.append((tex, self.grads[name], torch.zeros_like(tex.data[:n0]),
                                  torch.zeros_like(tex.data[:n0])))
            else:
                self.grads[name] = None
        self.params = [(p, gr, torch.zeros_like(p), torch.zeros_like(p)) for p, gr in params]
        self.ref_out = self.lat_out = None
        self.split_ref = self.split_lat = DEFAULT

    def load_views(self, t: int):
        self.mvp.copy_(self.mvp_all[t])
        self.eye.copy_(self.eye_all[t])
        self.light.copy_(self.light_all[t])

    def render_ref(self, ctx, stream=None):
        ctx.set_raster(*self.split_ref)
        self.ref_out = adr.render_fwd(ctx, self.ref_mesh, self.ref_mat, self.views, flags=self.det,
                                      outputs=self.ref_out, stream=stream)

    def render_latent(self, ctx, stream=None):
        ctx.set_raster(*self.split_lat)
        self.lat_out = adr.render_fwd(ctx, self.lat_mesh, self.lat_mat, self.views, ref=self.ref_out["image"],
                                      loss=self.w.loss, flags=self.det, want_image=False,
                                      outputs=self.lat_out, stream=stream)

    def fwd_bwd(self, ctx, stream=None):
        self.render_ref(ctx, stream)
        self.render_latent(ctx, stream)
        adr.render_bwd(ctx, self.lat_mesh, self.lat_mat, self.views, self.lat_out, self.grads,
                       flags=self.det | adr.BWD_DEFER_MIP_ADJOINT, stream=stream)

    def loss(self) -> float:
        return float(self.lat_out["loss"][0])

    def alloc_outputs(self):
        dev = self.lat_mesh.pos.device
        if self.ref_out is None:
            self.ref_out = adr.fwd_outputs(self.views, dev, False, want_image=True)
        if self.lat_out is None:
            self.lat_out = adr.fwd_outputs(self.views, dev, True, want_image=False)

    def batch_items(self):
        """This mesh's reference render and its latent render (with
        gradients) as batch items."""
        self.alloc_outputs()
        ref = dict(mesh=self.ref_mesh, mat=self.ref_mat, views=self.views, out=self.ref_out, flags=self.det,
                   split=self.split_ref)
        grads = {k: g for k, g in self.grads.items() if g is not None}
        lat = dict(mesh=self.lat_mesh, mat=self.lat_mat, views=self.views, out=self.lat_out,
                   ref=self.ref_out["image"], loss=self.w.loss, grads=grads,
                   flags=self.det | adr.BWD_DEFER_MIP_ADJOINT, split=self.split_lat)
        return ref, lat

    def tune(self, ctx, tuner: Tuner):
        w = self.w
        B, res = w.dirs.shape[0], w.width
        self.render_ref(ctx)                        # allocates the outputs the tuner's runs reuse
        self.split_ref = tuner.pick(ctx, "ref", w.ref.mesh.tri.shape[0], B, res, lambda: self.render_ref(ctx))
        self.render_latent(ctx)
        self.split_lat = tuner.pick(ctx, "latent", w.latent.mesh.tri.shape[0], B, res, lambda: self.render_latent(ctx))


def lr_at(lr0: float, t: int) -> float:
    """lr_t = lr_0 10^(-k t), k = 2e-4, iterations counted from 0 (Sec. 5.3)."""
    return lr0 * 10.0 ** (-0.0002 * t)


class Batch:
    """Meshes stepped either one at a time (``step_plain``) or as one
    graph-captured batch (``capture`` then ``step``) of the given form
    ("launch": one launch per stage over all meshes; "streams": per-mesh
    launches over several streams)."""

    def __init__(self, workloads, n_steps: int, n_streams: int = 4, det: bool = False, tune: bool = True,
                 seed: int = 0, tuner: Tuner | None = None, progress=None, form: str = "launch"):
        assert form in ("launch", "streams")
        self.form = form
        if form == "launch":
            n_streams = 1
        self.ctxs = [adr.Context(0) for _ in range(n_streams)]
        self.streams = [torch.cuda.Stream() for _ in range(n_streams)]   # default priority
        self.meshes = []
        for k, w in enumerate(workloads):
            self.meshes.append(MeshState(w, self.ctxs[k % n_streams], n_steps, seed + k, det))
            if progress is not None:
                progress(k)
        if tune:
            tuner = tuner or Tuner()
            for m in self.meshes:
                m.tune(self.ctxs[0], tuner)
            tuner.save()
        self.all_params = [p for m in self.meshes for p in m.params]
        self.all_maps = [mp for m in self.meshes for mp in m.maps]
        self.graph = None
        self.lr = workloads[0].lr
        self.ref_batch = self.lat_batch = None
        if form == "launch":
            items = [m.batch_items() for m in self.meshes]
            self.ref_batch = adr.RenderBatch(self.ctxs[0], [r for r, _ in items])
            self.lat_batch = adr.RenderBatch(self.ctxs[0], [lt for _, lt in items])

    def _adam(self, t: int):
        adr.adam_step(self.ctxs[0], self.all_params, t + 1, lr_at(self.lr, t))
        adr.adam_step_maps(self.ctxs[0], self.all_maps, t + 1, lr_at(self.lr, t))

    def _launch_all(self):
        if self.form == "launch":
            self.ref_batch.fwd()
            self.lat_batch.fwd()
            self.lat_batch.bwd()
            return
        cur = torch.cuda.current_stream()
        for s in self.streams:
            s.wait_stream(cur)
        for k, m in enumerate(self.meshes):
            i = k % len(self.streams)
            with torch.cuda.stream(self.streams[i]):
                m.fwd_bwd(self.ctxs[i], self.streams[i])
        for s in self.streams:
            cur.wait_stream(s)

    def step_eager(self, t: int):
        """The batched step without the graph (also the warm-up that sizes
        every context's scratch before capture)."""
        for m in self.meshes:
            m.load_views(t)
        self._launch_all()
        self._adam(t)

    def capture(self):
        """Capture all meshes' forward and backward launches as one graph
        (after at least one eager step: no allocation may happen inside)."""
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._launch_all()
        torch.cuda.synchronize()

    def step(self, t: int):
        for m in self.meshes:
            m.load_views(t)
        self.graph.replay()
        self._adam(t)

    def step_plain(self, t: int):
        """One mesh at a time: its renders, backward and Adam."""
        ctx = self.ctxs[0]
        lr = lr_at(self.lr, t)
        for m in self.meshes:
            m.load_views(t)
            m.fwd_bwd(ctx)
            adr.adam_step(ctx, m.params, t + 1, lr)
            adr.adam_step_maps(ctx, m.maps, t + 1, lr)

    def losses(self):
        return [m.loss() for m in self.meshes]

    def snapshot(self):
        """Copies of every mesh's optimised state (positions, maps with their
        chains, gradients and Adam moments), for ``restore``."""
        return [[t.clone() for t in self._state(m)] for m in self.meshes]

    def restore(self, snap):
        for m, saved in zip(self.meshes, snap):
            for t, x in zip(self._state(m), saved):
                t.copy_(x)

    @staticmethod
    def _state(m):
        out = [m.lat_mesh.pos]
        for p, g, mm, vv in m.params:
            out += [g, mm, vv]
        for tex, g, mm, vv in m.maps:
            out += [tex.data, g, mm, vv]
        return out

    def scratch_bytes(self) -> int:
        """Device bytes of the two library batches (launch form)."""
        return sum(b.info()["bytes"] for b in (self.ref_batch, self.lat_batch) if b is not None)

    def close(self):
        self.graph = None
        for b in (self.ref_batch, self.lat_batch):
            if b is not None:
                b.close()
        self.ref_batch = self.lat_batch = None
        for c in self.ctxs:
            c.close()
