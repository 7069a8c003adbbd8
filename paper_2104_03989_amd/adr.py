"""Python binding of the C ABI in include/adr.h (argument marshalling only).

Device memory comes from PyTorch; every step of the render loop runs in the
HIP kernels of libadr.so.  Importing this module fails loudly if the library
has not been built (``python -m paper_2104_03989_amd.csrc.build`` or
``__graft_entry__.build()``): there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libadr.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                      "(python paper_2104_03989_amd/csrc/build.py)")
_lib = C.CDLL(LIB_PATH)

OK, PENDING = 0, 1
E_INVALID, E_NOMEM, E_HIP, E_OVER_BUDGET, E_NOTFOUND, E_NONFINITE, E_UNIMPL = -1, -2, -3, -4, -5, -6, -7
TEX_F32, TEX_RGBA8 = 0, 1
SHADE_BLINN_PHONG, SHADE_GGX = 0, 1
LOSS = {"l1": 0, "l1_tonemap": 1, "l2": 2, "l2_tonemap": 3}
FWD_BUILD_MIPS, FWD_NO_AA, DETERMINISTIC, INDEPENDENT_MIPS, MSAA_2X2, MSAA_4X4 = 1, 2, 4, 8, 16, 32
BWD_DEFER_MIP_ADJOINT = 64
NOALLOC_SCRATCH_BYTES = 64 << 20


def msaa_factor(flags: int) -> int:
    return 4 if flags & MSAA_4X4 else (2 if flags & MSAA_2X2 else 1)
JOB_QUEUED, JOB_RUNNING, JOB_DONE, JOB_FAILED = 0, 1, 2, 3

EXPORTS = ("adr_last_error", "adr_ctx_create", "adr_ctx_destroy", "adr_render_fwd", "adr_render_bwd",
           "adr_adam_step", "adr_mip_build", "adr_mesh_adjacency", "adr_views_build",
           "adr_job_submit", "adr_job_poll", "adr_ctx_profile", "adr_ctx_profile_read", "adr_job_views",
           "adr_tess_counts", "adr_tess_build", "adr_tess_fwd", "adr_tess_bwd", "adr_mesh_frame", "adr_mesh_one_ring", "adr_laplacian", "adr_image_downsample",
           "adr_skin_fwd", "adr_skin_bwd", "adr_render_oit_fwd", "adr_render_oit_bwd", "adr_ctx_set_raster",
           "adr_adam_step_maps", "adr_ctx_profile_stages", "adr_render_fwd_noalloc", "adr_batch_create",
           "adr_batch_fwd", "adr_batch_bwd", "adr_batch_info", "adr_batch_destroy")
N_STAGES = 19
STAGES = ("vertex_frame", "transform", "raster", "shade", "aa_loss", "aa_bwd", "shade_bwd",
          "mip_adjoint", "mesh_bwd", "adam", "mip_build", "tex_bwd", "clear", "skin", "skin_bwd", "blend",
          "adam_maps", "adam_maps_top", "loss_reduce")


class AdrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"adr error {code}: {msg}")
        self.code = code


P = C.c_void_p
I32 = C.c_int32


class Texture_(C.Structure):
    _fields_ = [("data", P), ("size", I32), ("levels", I32), ("channels", I32), ("format", I32)]


class Mesh_(C.Structure):
    _fields_ = [("pos", P), ("tri", P), ("uv", P), ("uv_tri", P), ("adj", P),
                ("n_pos", I32), ("n_tri", I32), ("n_uv", I32), ("nrm", P), ("tan", P)]


class Material_(C.Structure):
    _fields_ = [("model", I32), ("kd", Texture_), ("normal", Texture_), ("orm", Texture_), ("alpha", Texture_)]


class Views_(C.Structure):
    _fields_ = [("mvp", P), ("eye", P), ("light_dir", P), ("light_rgb", P),
                ("n_views", I32), ("width", I32), ("height", I32)]


class FwdOut_(C.Structure):
    _fields_ = [("vis", P), ("color", P), ("image", P), ("dimage", P), ("loss", P),
                ("tri_id", P), ("coverage", P), ("aa", P)]


class Grads_(C.Structure):
    _fields_ = [("pos", P), ("vnormal", P), ("kd", P), ("normal", P), ("orm", P), ("alpha", P)]


class OitOut_(C.Structure):
    _fields_ = [("n_layers", I32), ("vis", P), ("color", P), ("alpha", P), ("blend", P), ("comp", P),
                ("dimage", P), ("loss", P), ("aa", P)]


class Param_(C.Structure):
    _fields_ = [("param", P), ("grad", P), ("m", P), ("v", P), ("n", C.c_int64)]


class MapParam_(C.Structure):
    _fields_ = [("tex", Texture_), ("grad", P), ("m", P), ("v", P)]


class Tess_(C.Structure):
    _fields_ = [("vidx", P), ("w", P), ("duv", P), ("n_vert", I32)]


class OneRing_(C.Structure):
    _fields_ = [("offs", P), ("nbr", P), ("n_pos", I32)]


class JobDesc_(C.Structure):
    _fields_ = [("ref_pos", P), ("ref_tri", P), ("ref_uv", P), ("ref_uv_tri", P),
                ("ref_n_pos", I32), ("ref_n_tri", I32), ("ref_n_uv", I32), ("model", I32),
                ("ref_kd", P), ("ref_kd_size", I32), ("ref_kd_format", I32),
                ("ref_normal", P), ("ref_normal_size", I32),
                ("ref_orm", P), ("ref_orm_size", I32),
                ("lat_pos", P), ("lat_tri", P), ("lat_uv", P), ("lat_uv_tri", P),
                ("lat_n_pos", I32), ("lat_n_tri", I32), ("lat_n_uv", I32),
                ("lat_kd", P), ("lat_kd_size", I32), ("lat_kd_format", I32),
                ("lat_normal", P), ("lat_normal_size", I32),
                ("lat_orm", P), ("lat_orm_size", I32),
                ("opt_mask", I32),
                ("seed", C.c_uint64),
                ("n_views", I32), ("width", I32), ("height", I32), ("light_per_view", I32),
                ("dist", C.c_float), ("fov_deg", C.c_float),
                ("n_steps", I32), ("loss_kind", I32),
                ("lr0", C.c_float), ("lr_decay_k", C.c_float)]


class JobStatus_(C.Structure):
    _fields_ = [("state", I32), ("step", I32), ("last_loss", C.c_float), ("p50_ms", C.c_float),
                ("p99_ms", C.c_float), ("device_bytes", C.c_uint64)]


class JobResult_(C.Structure):
    _fields_ = [("pos", P), ("kd", P), ("normal", P), ("orm", P)]


class BatchItem_(C.Structure):
    _fields_ = [("mesh", C.POINTER(Mesh_)), ("mat", C.POINTER(Material_)), ("views", C.POINTER(Views_)),
                ("ref_image", P), ("loss_kind", I32), ("out", C.POINTER(FwdOut_)), ("grads", C.POINTER(Grads_)),
                ("dloss", P), ("flags", I32), ("tiny_bbox", I32), ("med_bbox", I32)]


_lib.adr_last_error.restype = C.c_char_p
_lib.adr_ctx_create.argtypes = [I32, C.c_uint64, C.POINTER(P)]
_lib.adr_ctx_destroy.argtypes = [P]
_lib.adr_render_fwd.argtypes = [P, C.POINTER(Mesh_), C.POINTER(Material_), C.POINTER(Views_), P, I32,
                                C.POINTER(FwdOut_), I32, P]
_lib.adr_render_fwd_noalloc.argtypes = _lib.adr_render_fwd.argtypes
_lib.adr_render_bwd.argtypes = [P, C.POINTER(Mesh_), C.POINTER(Material_), C.POINTER(Views_),
                                C.POINTER(FwdOut_), P, C.POINTER(Grads_), I32, P]
_lib.adr_adam_step.argtypes = [P, C.POINTER(Param_), I32, I32, C.c_float, C.c_float, C.c_float,
                               C.c_float, P]
_lib.adr_adam_step_maps.argtypes = [P, C.POINTER(MapParam_), I32, I32, C.c_float, C.c_float, C.c_float,
                                    C.c_float, P]
_lib.adr_mip_build.argtypes = [P, C.POINTER(Texture_), P]
_lib.adr_mesh_adjacency.argtypes = [P, I32, P]
_lib.adr_views_build.argtypes = [P, I32, C.c_float, C.c_float, I32, I32, P, P]
_lib.adr_job_submit.argtypes = [P, C.POINTER(JobDesc_), C.POINTER(C.c_uint64)]
_lib.adr_job_poll.argtypes = [P, C.c_uint64, C.POINTER(JobStatus_), C.POINTER(JobResult_)]
_lib.adr_ctx_profile.argtypes = [P, I32]
_lib.adr_ctx_profile_stages.argtypes = [P, C.c_uint32]
_lib.adr_ctx_set_raster.argtypes = [P, I32, I32]
_lib.adr_ctx_profile_read.argtypes = [P, P, P]
_lib.adr_mesh_one_ring.argtypes = [P, I32, I32, P, P, P]
_lib.adr_image_downsample.argtypes = [P, P, I32, I32, I32, I32, P, P]
_lib.adr_laplacian.argtypes = [P, C.POINTER(OneRing_), P, P, C.c_float, P, P, P, P]
_lib.adr_mesh_frame.argtypes = [P, C.POINTER(Mesh_), P, P, P]
_lib.adr_tess_counts.argtypes = [P, I32, I32, I32, P, P, P]
_lib.adr_tess_build.argtypes = [P, P, P, I32, I32, I32, I32, P, P, P, P, P, P]
_lib.adr_tess_fwd.argtypes = [P, C.POINTER(Mesh_), C.POINTER(Tess_), C.POINTER(Texture_), P, P]
_lib.adr_tess_bwd.argtypes = [P, C.POINTER(Mesh_), C.POINTER(Tess_), C.POINTER(Texture_), P, P, P, P]
_lib.adr_skin_fwd.argtypes = [P, P, P, P, I32, I32, P, P, P]
_lib.adr_render_oit_fwd.argtypes = [P, C.POINTER(Mesh_), C.POINTER(Material_), C.POINTER(Views_), P, I32,
                                    C.POINTER(OitOut_), I32, P]
_lib.adr_render_oit_bwd.argtypes = [P, C.POINTER(Mesh_), C.POINTER(Material_), C.POINTER(Views_),
                                    C.POINTER(OitOut_), P, C.POINTER(Grads_), I32, P]
_lib.adr_skin_bwd.argtypes = [P, P, P, P, I32, I32, P, P, P, P]
_lib.adr_batch_create.argtypes = [P, I32, C.POINTER(BatchItem_), C.POINTER(P)]
_lib.adr_batch_fwd.argtypes = [P, P]
_lib.adr_batch_bwd.argtypes = [P, P]
_lib.adr_batch_info.argtypes = [P, C.POINTER(I32), C.POINTER(C.c_uint64)]
_lib.adr_batch_destroy.argtypes = [P]
for _n in EXPORTS[1:]:
    getattr(_lib, _n).restype = I32


def _check(code):
    if code < 0:
        raise AdrError(code, _lib.adr_last_error().decode())
    return code


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


# ---------------------------------------------------------------- host helpers

def mesh_adjacency(tri: np.ndarray) -> np.ndarray:
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    adj = np.zeros_like(tri)
    _check(_lib.adr_mesh_adjacency(_ptr(tri), tri.shape[0], _ptr(adj)))
    return adj


def views_build(dirs: np.ndarray, dist: float, fov_deg: float, width: int, height: int):
    dirs = np.ascontiguousarray(dirs, dtype=np.float32)
    n = dirs.shape[0]
    mvp = np.zeros((n, 16), dtype=np.float32)
    eye = np.zeros((n, 3), dtype=np.float32)
    _check(_lib.adr_views_build(_ptr(dirs), n, dist, fov_deg, width, height, _ptr(mvp), _ptr(eye)))
    return mvp, eye


# ---------------------------------------------------------------- context

class Context:
    def __init__(self, device: int = 0, hbm_budget: int = 0):
        h = P()
        _check(_lib.adr_ctx_create(device, hbm_budget, C.byref(h)))
        self.h = h
        self.device = device

    def set_raster(self, tiny_bbox: int = 64, med_bbox: int = 4096):
        """Raster work split of this context (see adr_ctx_set_raster)."""
        _check(_lib.adr_ctx_set_raster(self.h, int(tiny_bbox), int(med_bbox)))

    def profile(self, enable: bool = True):
        _check(_lib.adr_ctx_profile(self.h, 1 if enable else 0))

    def profile_stages(self, names):
        """Time only the named stages (see adr_ctx_profile_stages)."""
        mask = 0
        for n in names:
            mask |= 1 << STAGES.index(n)
        _check(_lib.adr_ctx_profile_stages(self.h, mask))

    def profile_read(self) -> dict:
        """{stage: (total ms, launches)} since the last read."""
        ms = np.zeros(N_STAGES, dtype=np.float64)
        cnt = np.zeros(N_STAGES, dtype=np.int64)
        _check(_lib.adr_ctx_profile_read(self.h, ms.ctypes.data, cnt.ctypes.data))
        return {STAGES[k]: (float(ms[k]), int(cnt[k])) for k in range(N_STAGES)}

    def close(self):
        if self.h:
            _lib.adr_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- device data

def chain_texels(size: int, levels: int) -> int:
    return sum((size >> l) ** 2 for l in range(levels))


class DeviceTexture:
    """A square texture with its mip chain in one device tensor."""

    def __init__(self, level0: np.ndarray, fmt: str, device="cuda", levels: int | None = None,
                 ctx: Context | None = None, chain: np.ndarray | None = None):
        S = level0.shape[0]
        assert level0.shape[1] == S and S & (S - 1) == 0, "square power-of-two texture"
        self.size = S
        self.levels = int(math.log2(S)) + 1 if levels is None else levels
        n = chain_texels(S, self.levels)
        if fmt == "rgba8":
            self.fmt, self.channels = TEX_RGBA8, 4
            self.data = torch.zeros(n, 4, dtype=torch.uint8, device=device)
            self.data[:S * S] = torch.from_numpy(np.ascontiguousarray(level0, dtype=np.uint8).reshape(-1, 4))
        else:
            self.fmt = TEX_F32
            self.channels = level0.shape[2]
            self.data = torch.zeros(n, self.channels, dtype=torch.float32, device=device)
            self.data[:S * S] = torch.from_numpy(np.ascontiguousarray(level0, dtype=np.float32).reshape(-1, self.channels))
        if chain is not None:
            # independent mip levels (Sec. 4.2): every level given
            assert self.fmt == TEX_F32 and chain.shape == (n, self.channels)
            self.data.copy_(torch.from_numpy(np.ascontiguousarray(chain, dtype=np.float32)))
        elif ctx is not None and self.levels > 1:
            mip_build(ctx, self)

    @property
    def level0(self):
        return self.data[:self.size * self.size]

    def struct(self):
        return Texture_(self.data.data_ptr(), self.size, self.levels, self.channels, self.fmt)

    def grad_buffer(self):
        assert self.fmt == TEX_F32
        return torch.zeros_like(self.data)


class DeviceMesh:
    def __init__(self, mesh, device="cuda"):
        self.pos = torch.from_numpy(np.ascontiguousarray(mesh.pos, dtype=np.float32)).to(device)
        self.tri = torch.from_numpy(np.ascontiguousarray(mesh.tri, dtype=np.int32)).to(device)
        self.uv = torch.from_numpy(np.ascontiguousarray(mesh.uv, dtype=np.float32)).to(device)
        self.uv_tri = torch.from_numpy(np.ascontiguousarray(mesh.uv_tri, dtype=np.int32)).to(device)
        self.adj = torch.from_numpy(mesh_adjacency(mesh.tri)).to(device)
        self.nrm = self.tan = None

    def precompute_frame(self, ctx: "Context", stream=None):
        """Compute the vertex frame once; later forward renders of these
        positions reuse it (for a mesh that does not move)."""
        nrm = torch.empty_like(self.pos)
        tan = torch.empty_like(self.pos)
        m = self.struct()
        _check(_lib.adr_mesh_frame(ctx.h, C.byref(m), _ptr(nrm), _ptr(tan), _stream(stream)))
        self.nrm, self.tan = nrm, tan
        return nrm, tan

    def struct(self, pos=None):
        p = self.pos if pos is None else pos
        fr = (self.nrm, self.tan) if (pos is None and self.nrm is not None) else (None, None)
        return Mesh_(p.data_ptr(), self.tri.data_ptr(), self.uv.data_ptr(), self.uv_tri.data_ptr(),
                     self.adj.data_ptr(), p.shape[0], self.tri.shape[0], self.uv.shape[0],
                     _ptr(fr[0]), _ptr(fr[1]))


class DeviceMaterial:
    def __init__(self, scene, device="cuda", ctx: Context | None = None):
        self.model = SHADE_GGX if scene.model == "ggx" else SHADE_BLINN_PHONG
        tex = lambda t: DeviceTexture(t.data, t.fmt, device, ctx=ctx, chain=getattr(t, "chain", None))
        self.kd = tex(scene.kd)
        self.normal = tex(scene.normal)
        self.orm = tex(scene.orm) if scene.orm is not None else None
        al = getattr(scene, "alpha", None)
        self.alpha = tex(al) if al is not None else None

    def struct(self):
        orm = self.orm.struct() if self.orm is not None else Texture_()
        al = self.alpha.struct() if self.alpha is not None else Texture_()
        return Material_(self.model, self.kd.struct(), self.normal.struct(), orm, al)


class DeviceViews:
    def __init__(self, mvp, eye, light_dir, light_rgb, width, height, device="cuda"):
        f = lambda x: x if torch.is_tensor(x) else torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(device)
        self.mvp = f(mvp).reshape(-1, 16)
        self.eye = f(eye).reshape(-1, 3)
        self.light_dir = f(light_dir).reshape(-1, 3)
        self.light_rgb = f(light_rgb).reshape(-1, 3)
        self.n = self.mvp.shape[0]
        self.width, self.height = width, height

    def struct(self):
        return Views_(self.mvp.data_ptr(), self.eye.data_ptr(), self.light_dir.data_ptr(),
                      self.light_rgb.data_ptr(), self.n, self.width, self.height)


# ---------------------------------------------------------------- calls

def mip_build(ctx: Context, tex: DeviceTexture, stream=None):
    t = tex.struct()
    _check(_lib.adr_mip_build(ctx.h, C.byref(t), _stream(stream)))


def fwd_outputs(views: DeviceViews, dev, with_ref: bool, want_image=True, want_tri_id=False, want_coverage=False,
                flags: int = 0) -> dict:
    """Output buffers of a forward render: vis, color, image, dimage, loss,
    tri_id, coverage and aa (the received antialiasing the backward reads)."""
    B, H, W = views.n, views.height, views.width
    ms = msaa_factor(flags)
    Hs, Ws = H * ms, W * ms          # visibility samples (multisampling: per sample)
    out = dict(vis=torch.empty(B, Hs, Ws, dtype=torch.int64, device=dev),
               color=torch.empty(B, Hs, Ws, 3, dtype=torch.float32, device=dev))
    out["image"] = torch.empty(B, H, W, 3, dtype=torch.float32, device=dev) if want_image else None
    out["tri_id"] = torch.empty(B, Hs, Ws, dtype=torch.int32, device=dev) if want_tri_id else None
    out["coverage"] = torch.empty(B, Hs, Ws, dtype=torch.int32, device=dev) if want_coverage else None
    if with_ref:
        out["dimage"] = torch.empty(B, H, W, 3, dtype=torch.float32, device=dev)
        out["loss"] = torch.empty(1, dtype=torch.float32, device=dev)
        # received antialiasing per sample, kept for the backward pass
        out["aa"] = torch.empty(B, Hs, Ws, 8, dtype=torch.float32, device=dev)
    else:
        out["dimage"] = out["loss"] = out["aa"] = None
    return out


def _fwd_out(out: dict):
    return FwdOut_(*[_ptr(out.get(k)) for k in ("vis", "color", "image", "dimage", "loss", "tri_id", "coverage",
                                                "aa")])


def _grads(grads: dict):
    return Grads_(*[_ptr(grads.get(k)) for k in ("pos", "vnormal", "kd", "normal", "orm", "alpha")])


def render_fwd(ctx: Context, mesh: DeviceMesh, mat: DeviceMaterial, views: DeviceViews, ref=None,
               loss: str = "l1", flags: int = 0, pos=None, want_image=True, want_tri_id=False,
               want_coverage=False, stream=None, outputs: dict | None = None, noalloc: bool = False):
    """Returns a dict with vis, color, image, dimage, loss, tri_id, coverage
    (``outputs``: a dict returned by an earlier call, reused in place).
    ``noalloc``: call adr_render_fwd_noalloc, whose scratch is the library's
    static per-device array (no device allocation by the library)."""
    out = outputs if outputs is not None else fwd_outputs(views, mesh.tri.device, ref is not None, want_image,
                                                          want_tri_id, want_coverage, flags)
    fo = _fwd_out(out)
    ms, mt, vs = mesh.struct(pos), mat.struct(), views.struct()
    fn = _lib.adr_render_fwd_noalloc if noalloc else _lib.adr_render_fwd
    _check(fn(ctx.h, C.byref(ms), C.byref(mt), C.byref(vs), _ptr(ref), LOSS[loss], C.byref(fo), flags,
              _stream(stream)))
    return out


def render_bwd(ctx: Context, mesh: DeviceMesh, mat: DeviceMaterial, views: DeviceViews, saved: dict,
               grads: dict, dloss=None, flags: int = 0, pos=None, stream=None):
    """Accumulates into grads['pos'|'vnormal'|'kd'|'normal'|'orm'] (tensors or None)."""
    fo, g = _fwd_out(saved), _grads(grads)
    ms, mt, vs = mesh.struct(pos), mat.struct(), views.struct()
    _check(_lib.adr_render_bwd(ctx.h, C.byref(ms), C.byref(mt), C.byref(vs), C.byref(fo),
                               _ptr(dloss), C.byref(g), flags, _stream(stream)))


class RenderBatch:
    """adr_batch_*: the forward (and backward) of many renders, one launch
    per stage over all of them.  ``items``: dicts with mesh, mat, views
    (DeviceMesh / DeviceMaterial / DeviceViews), out (a fwd_outputs dict) and
    optionally ref (reference image tensor), loss ('l1'...), grads (dict as
    render_bwd's; needs ref), dloss, flags, split ((tiny, med) raster work
    split).  The tensors are read at every call and must stay alive."""

    def __init__(self, ctx: Context, items: list):
        self.ctx = ctx
        arr = (BatchItem_ * len(items))()
        for k, it in enumerate(items):
            split = it.get("split") or (0, 0)
            grads = it.get("grads")
            arr[k] = BatchItem_(C.pointer(it["mesh"].struct()), C.pointer(it["mat"].struct()),
                                C.pointer(it["views"].struct()), _ptr(it.get("ref")), LOSS[it.get("loss", "l1")],
                                C.pointer(_fwd_out(it["out"])), C.pointer(_grads(grads)) if grads else None,
                                _ptr(it.get("dloss")), it.get("flags", 0), split[0], split[1])
        self.h = P()
        _check(_lib.adr_batch_create(ctx.h, len(items), arr, C.byref(self.h)))

    def fwd(self, stream=None):
        _check(_lib.adr_batch_fwd(self.h, _stream(stream)))

    def bwd(self, stream=None):
        _check(_lib.adr_batch_bwd(self.h, _stream(stream)))

    def info(self) -> dict:
        n, b = I32(), C.c_uint64()
        _check(_lib.adr_batch_info(self.h, C.byref(n), C.byref(b)))
        return {"items": n.value, "bytes": b.value}

    def close(self):
        if self.h:
            _check(_lib.adr_batch_destroy(self.h))
            self.h = P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def adam_step(ctx: Context, params: list, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8,
              stream=None):
    """params: list of (param, grad, m, v) float32 device tensors of equal size."""
    arr = (Param_ * max(len(params), 1))()
    for k, (p, g, m, v) in enumerate(params):
        arr[k] = Param_(p.data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr(), p.numel())
    _check(_lib.adr_adam_step(ctx.h, arr, len(params), t, lr, beta1, beta2, eps, _stream(stream)))


def adam_step_maps(ctx: Context, maps: list, t: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8,
                   stream=None):
    """maps: list of (DeviceTexture, grad chain, m, v): Adam on each F32
    map's level 0 with the chain's adjoint before it and its rebuild after
    it (grad as left by a backward with BWD_DEFER_MIP_ADJOINT; zeroed)."""
    arr = (MapParam_ * max(len(maps), 1))()
    for k, (tex, g, m, v) in enumerate(maps):
        n0 = tex.size * tex.size * tex.channels
        assert g.numel() == tex.data.numel() and m.numel() == n0 and v.numel() == n0
        arr[k] = MapParam_(tex.struct(), g.data_ptr(), m.data_ptr(), v.data_ptr())
    _check(_lib.adr_adam_step_maps(ctx.h, arr, len(maps), t, lr, beta1, beta2, eps, _stream(stream)))


class RenderLoss(torch.autograd.Function):
    """Image loss of a latent render against a reference image; the backward
    is adr_render_bwd.  Differentiable inputs: pos [V,3], and the level-0
    slices of the F32 maps ``kd``, ``normal``, ``orm`` (``tex.level0`` of the
    material's textures, so that the render reads the tensors autograd
    tracks; pass FWD_BUILD_MIPS when level 0 changed since the chain was
    built).  The gradient of a map is w.r.t. its level-0 texels with the
    coarser levels derived from them, so the flags that keep per-level
    gradients (INDEPENDENT_MIPS, BWD_DEFER_MIP_ADJOINT) are rejected.
    forward(pos, kd0, normal0, orm0, ctx, mesh, mat, views, ref, loss, flags)."""

    @staticmethod
    def forward(fctx, pos, kd0, normal0, orm0, ctx, mesh, mat, views, ref, loss, flags):
        if flags & (INDEPENDENT_MIPS | BWD_DEFER_MIP_ADJOINT):
            raise ValueError("RenderLoss differentiates level 0 of derived mip chains: "
                             "INDEPENDENT_MIPS and BWD_DEFER_MIP_ADJOINT are not supported")
        for name, t in (("kd", kd0), ("normal", normal0), ("orm", orm0)):
            if t is None:
                continue
            tex = getattr(mat, name)
            if tex is None:
                raise ValueError(f"RenderLoss: the material has no {name} map")
            if tex.fmt != TEX_F32:
                raise ValueError(f"RenderLoss: {name} is not an F32 map and cannot be differentiated")
            lv0 = tex.level0
            if t.data_ptr() != lv0.data_ptr() or t.shape != lv0.shape:
                raise ValueError(f"RenderLoss: {name}0 must be mat.{name}.level0 (the tensor the render reads)")
        out = render_fwd(ctx, mesh, mat, views, ref=ref, loss=loss, flags=flags, pos=pos, want_image=False)
        fctx.state = (ctx, mesh, mat, views, flags & ~FWD_BUILD_MIPS, out)
        fctx.save_for_backward(pos)
        return out["loss"][0].clone()

    @staticmethod
    def backward(fctx, gout):
        ctx, mesh, mat, views, flags, out = fctx.state
        (pos,) = fctx.saved_tensors
        grads = {"pos": torch.zeros_like(pos) if fctx.needs_input_grad[0] else None}
        for k, name in ((1, "kd"), (2, "normal"), (3, "orm")):
            tex = getattr(mat, name)
            grads[name] = tex.grad_buffer() if fctx.needs_input_grad[k] and tex is not None else None
        dl = gout.reshape(1).to(torch.float32).contiguous()
        render_bwd(ctx, mesh, mat, views, out, grads, dloss=dl, flags=flags, pos=pos)
        res = [grads["pos"]]
        for name in ("kd", "normal", "orm"):
            g = grads[name]
            tex = getattr(mat, name)
            res.append(None if g is None else g[:tex.size * tex.size])
        return (*res, None, None, None, None, None, None, None)


# ---------------------------------------------------------------- job server

_lib.adr_job_views.argtypes = [C.c_uint64, I32, I32, I32, P, P]
_lib.adr_job_views.restype = I32


def job_views(seed: int, step: int, n_views: int, light_per_view: bool = True):
    dirs = np.zeros((n_views, 3), dtype=np.float32)
    lights = np.zeros((n_views, 3), dtype=np.float32)
    _check(_lib.adr_job_views(seed, step, n_views, 1 if light_per_view else 0, _ptr(dirs), _ptr(lights)))
    return dirs, lights


def _tex_arg(tex):
    if tex is None:
        return None, 0, TEX_F32
    if tex.fmt == "rgba8":
        a = np.ascontiguousarray(tex.data, dtype=np.uint8)
        return a, a.shape[0], TEX_RGBA8
    a = np.ascontiguousarray(tex.data, dtype=np.float32)
    return a, a.shape[0], TEX_F32


def job_submit(ctx: Context, w, n_steps: int, seed: int, lr_decay_k: float = 0.0002,
               light_per_view: bool = True) -> int:
    """Queue a whole optimisation of workload ``w`` (host arrays are copied)."""
    keep = []
    def arr(x, dt):
        a = np.ascontiguousarray(x, dtype=dt)
        keep.append(a)
        return a.ctypes.data
    ref, lat = w.ref, w.latent
    rkd, rkd_s, rkd_f = _tex_arg(ref.kd)
    lkd, lkd_s, lkd_f = _tex_arg(lat.kd)
    rn, rn_s, _ = _tex_arg(ref.normal)
    ln, ln_s, _ = _tex_arg(lat.normal)
    ro, ro_s, _ = _tex_arg(ref.orm)
    lo, lo_s, _ = _tex_arg(lat.orm)
    keep += [x for x in (rkd, lkd, rn, ln, ro, lo) if x is not None]
    mask = sum(1 << k for k, n in enumerate(("pos", "kd", "normal", "orm")) if n in w.optimize)
    d = JobDesc_()
    d.ref_pos, d.ref_tri = arr(ref.mesh.pos, np.float32), arr(ref.mesh.tri, np.int32)
    d.ref_uv, d.ref_uv_tri = arr(ref.mesh.uv, np.float32), arr(ref.mesh.uv_tri, np.int32)
    d.ref_n_pos, d.ref_n_tri, d.ref_n_uv = ref.mesh.pos.shape[0], ref.mesh.tri.shape[0], ref.mesh.uv.shape[0]
    d.model = SHADE_GGX if ref.model == "ggx" else SHADE_BLINN_PHONG
    d.ref_kd, d.ref_kd_size, d.ref_kd_format = _ptr(rkd), rkd_s, rkd_f
    d.ref_normal, d.ref_normal_size = _ptr(rn), rn_s
    d.ref_orm, d.ref_orm_size = (_ptr(ro), ro_s) if ro is not None else (None, 0)
    d.lat_pos, d.lat_tri = arr(lat.mesh.pos, np.float32), arr(lat.mesh.tri, np.int32)
    d.lat_uv, d.lat_uv_tri = arr(lat.mesh.uv, np.float32), arr(lat.mesh.uv_tri, np.int32)
    d.lat_n_pos, d.lat_n_tri, d.lat_n_uv = lat.mesh.pos.shape[0], lat.mesh.tri.shape[0], lat.mesh.uv.shape[0]
    d.lat_kd, d.lat_kd_size, d.lat_kd_format = _ptr(lkd), lkd_s, lkd_f
    d.lat_normal, d.lat_normal_size = _ptr(ln), ln_s
    d.lat_orm, d.lat_orm_size = (_ptr(lo), lo_s) if lo is not None else (None, 0)
    d.opt_mask = mask
    d.seed = seed
    d.n_views, d.width, d.height = w.dirs.shape[0], w.width, w.height
    d.light_per_view = 1 if light_per_view else 0
    d.dist, d.fov_deg = w.dist, w.fov_deg
    d.n_steps, d.loss_kind = n_steps, LOSS[w.loss]
    d.lr0, d.lr_decay_k = w.lr, lr_decay_k
    jid = C.c_uint64(0)
    _check(_lib.adr_job_submit(ctx.h, C.byref(d), C.byref(jid)))
    return int(jid.value)


def job_poll(ctx: Context, job_id: int, w=None):
    """(status dict, result dict or None).  With ``w`` (the submitted
    workload, for the result shapes) a finished job's latent model is
    returned and the job is released."""
    st = JobStatus_()
    res = None
    out = None
    if w is not None:
        lat = w.latent
        res = {"pos": np.zeros_like(lat.mesh.pos, dtype=np.float32),
               "kd": np.zeros_like(lat.kd.data),
               "normal": np.zeros_like(lat.normal.data, dtype=np.float32),
               "orm": np.zeros_like(lat.orm.data, dtype=np.float32) if lat.orm is not None else None}
        out = JobResult_(_ptr(res["pos"]), _ptr(res["kd"]), _ptr(res["normal"]), _ptr(res["orm"]))
    code = _lib.adr_job_poll(ctx.h, job_id, C.byref(st), C.byref(out) if out is not None else None)
    if code < 0 and code not in (E_NONFINITE, E_HIP):
        _check(code)
    status = {"code": code, "state": st.state, "step": st.step, "loss": st.last_loss,
              "p50_ms": st.p50_ms, "p99_ms": st.p99_ms, "device_bytes": st.device_bytes}
    if code < 0:   # the job failed and has been released
        status["state"] = JOB_FAILED
        status["error"] = _lib.adr_last_error().decode()
    return status, (res if (code == OK and st.state == JOB_DONE and w is not None) else None)


# ---------------------------------------------------------------- displacement mapping

def tess_build(tri: np.ndarray, uv_tri: np.ndarray, uv: np.ndarray, n_pos: int, levels: int) -> dict:
    """Host tables of the fixed edge-midpoint tessellation (Sec. 5.1)."""
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    uv_tri = np.ascontiguousarray(uv_tri, dtype=np.int32)
    uv = np.ascontiguousarray(uv, dtype=np.float32)
    nv, nt, nu = C.c_int64(), C.c_int64(), C.c_int64()
    _check(_lib.adr_tess_counts(_ptr(tri), tri.shape[0], n_pos, levels, C.byref(nv), C.byref(nt),
                                C.byref(nu)))
    out = dict(vidx=np.zeros((nv.value, 3), np.int32), w=np.zeros((nv.value, 3), np.float32),
               duv=np.zeros((nv.value, 2), np.float32), tri=np.zeros((nt.value, 3), np.int32),
               uv=np.zeros((nu.value, 2), np.float32), uv_tri=np.zeros((nt.value, 3), np.int32))
    _check(_lib.adr_tess_build(_ptr(tri), _ptr(uv_tri), _ptr(uv), tri.shape[0], n_pos, uv.shape[0], levels,
                               _ptr(out["vidx"]), _ptr(out["w"]), _ptr(out["duv"]), _ptr(out["tri"]),
                               _ptr(out["uv"]), _ptr(out["uv_tri"])))
    return out


class DeviceTess:
    """A base mesh, its tessellation tables and the tessellated mesh (whose
    positions ``tess_fwd`` rewrites)."""

    def __init__(self, base, levels: int, device="cuda"):
        self.base = DeviceMesh(base, device)
        t = tess_build(base.tri, base.uv_tri, base.uv, base.pos.shape[0], levels)
        self.levels = levels
        f = lambda a: torch.from_numpy(a).to(device)
        self.vidx, self.w, self.duv = f(t["vidx"]), f(t["w"]), f(t["duv"])
        self.n_vert = t["vidx"].shape[0]
        self.mesh = DeviceMesh.__new__(DeviceMesh)
        self.mesh.nrm = self.mesh.tan = None
        self.mesh.pos = torch.zeros(self.n_vert, 3, dtype=torch.float32, device=device)
        self.mesh.tri, self.mesh.uv, self.mesh.uv_tri = f(t["tri"]), f(t["uv"]), f(t["uv_tri"])
        self.mesh.adj = f(mesh_adjacency(t["tri"]))
        self.tables = t

    def struct(self):
        return Tess_(self.vidx.data_ptr(), self.w.data_ptr(), self.duv.data_ptr(), self.n_vert)


def tess_fwd(ctx: Context, ts: DeviceTess, disp: DeviceTexture, base_pos=None, out=None, stream=None):
    """Displaced tessellated positions v + disp(uv) n (Eq. 3)."""
    b = ts.base.struct(base_pos)
    t = ts.struct()
    d = disp.struct()
    out = ts.mesh.pos if out is None else out
    _check(_lib.adr_tess_fwd(ctx.h, C.byref(b), C.byref(t), C.byref(d), _ptr(out), _stream(stream)))
    return out


def tess_bwd(ctx: Context, ts: DeviceTess, disp: DeviceTexture, g_pos, g_base_pos, g_disp,
             base_pos=None, stream=None):
    """Accumulates dL/d(base positions) and dL/d(displacement level 0) from
    dL/d(tessellated positions) ``g_pos``, which is zeroed (consumed)."""
    b = ts.base.struct(base_pos)
    t = ts.struct()
    d = disp.struct()
    _check(_lib.adr_tess_bwd(ctx.h, C.byref(b), C.byref(t), C.byref(d), _ptr(g_pos), _ptr(g_base_pos),
                             _ptr(g_disp), _stream(stream)))


# ---------------------------------------------------------------- Laplacian regularizer

def mesh_one_ring(tri: np.ndarray, n_pos: int):
    """Host CSR (offs [n_pos+1], nbr) of the sorted one-rings."""
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    offs = np.zeros(n_pos + 1, np.int32)
    n = C.c_int64()
    _check(_lib.adr_mesh_one_ring(_ptr(tri), tri.shape[0], n_pos, _ptr(offs), None, C.byref(n)))
    nbr = np.zeros(max(n.value, 1), np.int32)
    _check(_lib.adr_mesh_one_ring(_ptr(tri), tri.shape[0], n_pos, _ptr(offs), _ptr(nbr), C.byref(n)))
    return offs, nbr[:n.value]


class DeviceOneRing:
    def __init__(self, tri: np.ndarray, n_pos: int, device="cuda"):
        offs, nbr = mesh_one_ring(tri, n_pos)
        self.offs = torch.from_numpy(offs).to(device)
        self.nbr = torch.from_numpy(nbr if nbr.size else np.zeros(1, np.int32)).to(device)
        self.n_pos = n_pos

    def struct(self):
        return OneRing_(self.offs.data_ptr(), self.nbr.data_ptr(), self.n_pos)


def laplacian(ctx: Context, ring: DeviceOneRing, pos, delta_ref=None, lam: float = 1.0, delta_out=None,
              loss=None, g_pos=None, stream=None):
    """Uniform Laplacian regularizer (Sec. 5.3): optional delta, loss and
    g_pos += lam dL/dpos outputs (device tensors)."""
    r = ring.struct()
    _check(_lib.adr_laplacian(ctx.h, C.byref(r), _ptr(pos), _ptr(delta_ref), float(lam), _ptr(delta_out),
                              _ptr(loss), _ptr(g_pos), _stream(stream)))


def image_downsample(ctx: Context, img, k: int, out=None, stream=None):
    """[B, kH, kW, 3] -> [B, H, W, 3] box filter (supersampled reference)."""
    B, Hs, Ws, _ = img.shape
    H, W = Hs // k, Ws // k
    out = torch.empty(B, H, W, 3, dtype=torch.float32, device=img.device) if out is None else out
    _check(_lib.adr_image_downsample(ctx.h, _ptr(img), B, H, W, k, _ptr(out), _stream(stream)))
    return out


def skin_fwd(ctx: Context, pos, weights, bones, out=None, blend=None, stream=None):
    """Dense linear blend skinning (Sec. 5.1, Eq. 2): pos [V,3], weights
    [V,nb], bones [nb,3,4] device float32 -> (skinned [V,3], blend [V,12])."""
    V, nb = weights.shape
    out = torch.empty(V, 3, dtype=torch.float32, device=pos.device) if out is None else out
    blend = torch.empty(V, 12, dtype=torch.float32, device=pos.device) if blend is None else blend
    _check(_lib.adr_skin_fwd(ctx.h, _ptr(pos), _ptr(weights), _ptr(bones), V, nb, _ptr(out), _ptr(blend),
                             _stream(stream)))
    return out, blend


def skin_bwd(ctx: Context, pos, bones, blend, g_out, g_pos=None, g_weights=None, stream=None):
    """Adjoint of skin_fwd: g_pos += dL/dpos, g_weights += dL/dweights (either
    may be None); g_out (dL/d skinned positions) is consumed (zeroed)."""
    V = pos.shape[0]
    nb = bones.shape[0]
    _check(_lib.adr_skin_bwd(ctx.h, _ptr(pos), _ptr(bones), _ptr(blend), V, nb, _ptr(g_out), _ptr(g_pos),
                             _ptr(g_weights), _stream(stream)))


def render_oit_fwd(ctx: Context, mesh: DeviceMesh, mat: DeviceMaterial, views: DeviceViews, layers: int, ref=None,
                   loss: str = "l2", flags: int = 0, stream=None, outputs: dict | None = None):
    """Depth-peeled render (Sec. 5.2, order-independent transparency):
    returns vis [L,B,H,W], color [L,B,H,W,3], alpha [L,B,H,W], blend and
    comp [L,B,H,W,3] (comp[0] is the image), dimage, loss."""
    B, H, W = views.n, views.height, views.width
    dev = mesh.tri.device
    if outputs is not None:
        out = outputs
    else:
        out = dict(vis=torch.empty(layers, B, H, W, dtype=torch.int64, device=dev),
                   color=torch.empty(layers, B, H, W, 3, dtype=torch.float32, device=dev),
                   alpha=torch.empty(layers, B, H, W, dtype=torch.float32, device=dev),
                   blend=torch.empty(layers, B, H, W, 3, dtype=torch.float32, device=dev),
                   comp=torch.empty(layers, B, H, W, 3, dtype=torch.float32, device=dev))
        out["dimage"] = torch.empty(B, H, W, 3, dtype=torch.float32, device=dev) if ref is not None else None
        out["loss"] = torch.empty(1, dtype=torch.float32, device=dev) if ref is not None else None
        out["aa"] = torch.empty(layers, B, H, W, 8, dtype=torch.float32, device=dev) if ref is not None else None
    out["layers"] = layers
    oo = OitOut_(layers, *[_ptr(out.get(k)) for k in ("vis", "color", "alpha", "blend", "comp", "dimage", "loss",
                                                      "aa")])
    ms, mt, vs = mesh.struct(), mat.struct(), views.struct()
    _check(_lib.adr_render_oit_fwd(ctx.h, C.byref(ms), C.byref(mt), C.byref(vs), _ptr(ref), LOSS[loss],
                                   C.byref(oo), flags, _stream(stream)))
    return out


def render_oit_bwd(ctx: Context, mesh: DeviceMesh, mat: DeviceMaterial, views: DeviceViews, saved: dict,
                   grads: dict, dloss=None, flags: int = 0, stream=None):
    """Adjoint of render_oit_fwd; accumulates into grads['pos'|'vnormal'|'kd'|'normal'|'orm'|'alpha']."""
    oo = OitOut_(saved["layers"], *[_ptr(saved.get(k)) for k in ("vis", "color", "alpha", "blend", "comp", "dimage",
                                                                  "loss", "aa")])
    g = Grads_(*[_ptr(grads.get(k)) for k in ("pos", "vnormal", "kd", "normal", "orm", "alpha")])
    ms, mt, vs = mesh.struct(), mat.struct(), views.struct()
    _check(_lib.adr_render_oit_bwd(ctx.h, C.byref(ms), C.byref(mt), C.byref(vs), C.byref(oo), _ptr(dloss), C.byref(g),
                                   flags, _stream(stream)))
