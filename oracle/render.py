"""ORACLE -- test infrastructure only.

A plain, slow FP64 CPU implementation of one step of the appearance-driven
simplification loop (Hasselgren et al., "Appearance-Driven Automatic 3D Model
Simplification"): render the latent mesh from a batch of cameras (Sec. 3,
Eq. 1), with smooth vertex normals and UV tangent frames (Sec. 5.1, "Tangent
space"), perspective-correct interpolation into a deferred G-buffer of
position, normal, tangent, bitangent and texture coordinates (Sec. 5.2),
mip-mapped texture lookups (Sec. 4.2 treats the mip chain as the texture
representation), Lambert/Blinn-Phong or diffuse + GGX shading with
k_s = (1-m) 0.04 + m k_d and k_s' = (1-gamma) k_s (Sec. 5.2), silhouette
antialiasing (Sec. 5.2, "Antialiasing"), an L1 (or squared L2) loss on colours
tone mapped with Gamma(log(x+1)) (Sec. 5.3, "Objective function"), gradients
w.r.t. vertex positions and texels, and an Adam update with default
parameters and lr_t = lr_0 10^(-k t) (Sec. 5.3, "Learning rate and runtime").

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this module.  It shares no code with the GPU path.  The forward pass is
written out in float64 torch CPU ops; the backward pass is torch autograd of
that forward pass, i.e. the exact derivative of the function defined here.

Readings taken where the paper is silent:
  * visibility: the integer rules R1-R6 in raster.c;
  * camera: look-at from dist * dir to the origin, up +y (or +z when the view
    direction is within 0.999 of +-y), OpenGL perspective with near 0.1 and
    far 10, pixel centres at +0.5, row 0 at the bottom;
  * interpolation: perspective-correct barycentrics of the pixel centre from
    the unsnapped clip coordinates, lambda_i = D_i / sum D with
    D_i = (h_j x h_k) . (px, py, 1), h = (x, y, w);
  * normals: area-weighted smooth vertex normals; tangents: per-face UV
    tangent summed per vertex and normalised, Gram-Schmidt against the
    interpolated normal, bitangent N x T (handedness ignored);
  * textures: mip levels are 2x2 box averages of level 0 (RGBA8 maps round
    (a+b+c+d+2)//4), isotropic LOD = 0.5 log2 max(|duv/dx|^2, |duv/dy|^2) in
    level-0 texels clamped to [0, L-1], trilinear between floor(LOD) and the
    next level, texel centres at +0.5, wrap in u, clamp in v, gradients flow
    through the LOD where it is not clamped;
  * Blinn-Phong: c = E max(0, n.l) (k_d + 0.04 max(0, n.h)^32);
  * GGX: roughness clamped to [0.08, 1], alpha = r^2,
    D = alpha^2 / (pi ((n.h)^2 (alpha^2-1) + 1)^2), Schlick-GGX G with
    k = alpha/2, Schlick Fresnel with F0 = (1-gamma)((1-m) 0.04 + m k_d),
    c = E (k_d (1-m)/pi + D F G / (4 max(n.l,1e-4) max(n.v,1e-4))) max(0, n.l);
  * antialiasing: see ``antialias``;
  * loss: mean over B*H*W*3 of |T(x) - T(ref)|, sign(0) = 0.
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np
import torch

F64 = torch.float64
KEY_EMPTY = np.uint64(0xFFFFFFFF00000000)

# ---------------------------------------------------------------------------
# C part (integer visibility)
# ---------------------------------------------------------------------------

_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        from . import build as _build
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        lib = ctypes.CDLL(path)
        P = ctypes.c_void_p
        I = ctypes.c_int32
        lib.oracle_snap.argtypes = [P, I, P, I, I, P]
        lib.oracle_clip32.argtypes = [P, I, P, P]
        lib.oracle_raster.argtypes = [P, I, P, I, I, P, P, P, I]
        lib.oracle_raster_peel.argtypes = [P, I, P, I, I, P, P, I]
        lib.oracle_edge_inside_batch.argtypes = [P, P, I, P, P, P, P, P]
        _LIB = lib
    return _LIB


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def snap(pos32: np.ndarray, mvp32: np.ndarray, W: int, H: int) -> np.ndarray:
    """R1/R2: snapped (X, Y, Z, usable) per vertex, int32 [V,4]."""
    pos32 = np.ascontiguousarray(pos32, dtype=np.float32)
    mvp32 = np.ascontiguousarray(mvp32, dtype=np.float32).reshape(16)
    out = np.zeros((pos32.shape[0], 4), dtype=np.int32)
    _lib().oracle_snap(_ptr(pos32), pos32.shape[0], _ptr(mvp32), W, H, _ptr(out))
    return out


def clip32(pos32: np.ndarray, mvp32: np.ndarray) -> np.ndarray:
    pos32 = np.ascontiguousarray(pos32, dtype=np.float32)
    mvp32 = np.ascontiguousarray(mvp32, dtype=np.float32).reshape(16)
    out = np.zeros((pos32.shape[0], 4), dtype=np.float32)
    _lib().oracle_clip32(_ptr(pos32), pos32.shape[0], _ptr(mvp32), _ptr(out))
    return out


def raster(tri: np.ndarray, snapv: np.ndarray, W: int, H: int, brute: bool = False):
    """R3-R6 for one view: (keys uint64 [H,W], coverage uint32 [H,W], orient int8 [T])."""
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    snapv = np.ascontiguousarray(snapv, dtype=np.int32)
    keys = np.zeros((H, W), dtype=np.uint64)
    cov = np.zeros((H, W), dtype=np.uint32)
    orient = np.zeros(tri.shape[0], dtype=np.int8)
    _lib().oracle_raster(_ptr(tri), tri.shape[0], _ptr(snapv), W, H, _ptr(keys), _ptr(cov),
                         _ptr(orient), 1 if brute else 0)
    return keys, cov, orient


def raster_peel(tri: np.ndarray, snapv: np.ndarray, W: int, H: int, floor_keys: np.ndarray | None,
                brute: bool = False) -> np.ndarray:
    """One depth-peeling pass: per pixel the smallest fragment key above
    ``floor_keys`` (None: the front layer), uint64 [H,W]."""
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    snapv = np.ascontiguousarray(snapv, dtype=np.int32)
    keys = np.zeros((H, W), dtype=np.uint64)
    fl = None if floor_keys is None else np.ascontiguousarray(floor_keys, dtype=np.uint64)
    _lib().oracle_raster_peel(_ptr(tri), tri.shape[0], _ptr(snapv), W, H, None if fl is None else _ptr(fl),
                              _ptr(keys), 1 if brute else 0)
    return keys


def edge_inside(tri, snapv, t, i, j):
    """Inside bits of oriented edges of triangles t at pixels (i, j), and the
    original corner index of each oriented corner."""
    tri = np.ascontiguousarray(tri, dtype=np.int32)
    snapv = np.ascontiguousarray(snapv, dtype=np.int32)
    t = np.ascontiguousarray(t, dtype=np.int32)
    i = np.ascontiguousarray(i, dtype=np.int32)
    j = np.ascontiguousarray(j, dtype=np.int32)
    n = t.shape[0]
    bits = np.zeros(n, dtype=np.int32)
    vid = np.zeros((n, 3), dtype=np.int32)
    if n:
        _lib().oracle_edge_inside_batch(_ptr(tri), _ptr(snapv), n, _ptr(t), _ptr(i), _ptr(j),
                                        _ptr(bits), _ptr(vid))
    return bits, vid


def key_tri(keys: np.ndarray) -> np.ndarray:
    """Triangle id (0 = empty, else triangle + 1) of visibility keys."""
    return (keys & np.uint64(0xFFFFFFFF)).astype(np.int64)


# ---------------------------------------------------------------------------
# Cameras (Sec. 3: random camera and light per iteration)
# ---------------------------------------------------------------------------

def look_at_mvp(dirs: np.ndarray, dist: float, fov_deg: float, W: int, H: int,
                near: float = 0.1, far: float = 10.0):
    """Projection * view for eye = dist * dir looking at the origin.
    Returns (mvp [B,4,4] float64, eye [B,3] float64)."""
    dirs = np.asarray(dirs, dtype=np.float64)
    B = dirs.shape[0]
    mvp = np.zeros((B, 4, 4))
    eyes = np.zeros((B, 3))
    fy = 1.0 / math.tan(math.radians(fov_deg) / 2.0)
    aspect = W / H
    P = np.array([[fy / aspect, 0, 0, 0], [0, fy, 0, 0],
                  [0, 0, (far + near) / (near - far), 2 * far * near / (near - far)],
                  [0, 0, -1, 0]], dtype=np.float64)
    for b in range(B):
        e = dist * dirs[b] / np.linalg.norm(dirs[b])
        f = -e / np.linalg.norm(e)
        up = np.array([0.0, 1.0, 0.0])
        if abs(f @ up) > 0.999:
            up = np.array([0.0, 0.0, 1.0])
        s = np.cross(f, up)
        s /= np.linalg.norm(s)
        u = np.cross(s, f)
        V = np.eye(4)
        V[0, :3], V[1, :3], V[2, :3] = s, u, -f
        V[0, 3], V[1, 3], V[2, 3] = -s @ e, -u @ e, f @ e
        mvp[b] = P @ V
        eyes[b] = e
    return mvp, eyes


# ---------------------------------------------------------------------------
# Mesh operations (Sec. 5.1, "Tangent space")
# ---------------------------------------------------------------------------

def safe_normalize(x: torch.Tensor) -> torch.Tensor:
    """x / |x| along the last axis; vectors with |x|^2 <= 1e-20 pass unchanged."""
    n2 = (x * x).sum(-1, keepdim=True)
    ok = n2 > 1e-20
    return torch.where(ok, x / torch.sqrt(torch.where(ok, n2, torch.ones_like(n2))), x)


def vertex_normals(pos: torch.Tensor, tri: torch.Tensor) -> torch.Tensor:
    """n_v = normalize(sum over faces at v of (p1-p0) x (p2-p0))."""
    p0, p1, p2 = pos[tri[:, 0]], pos[tri[:, 1]], pos[tri[:, 2]]
    fn = torch.cross(p1 - p0, p2 - p0, dim=1)
    acc = torch.zeros_like(pos)
    for k in range(3):
        acc = acc.index_add(0, tri[:, k], fn)
    return safe_normalize(acc)


def vertex_tangents(pos, tri, uv, uv_tri) -> torch.Tensor:
    """Per-face t_f = (e1 dv2 - e2 dv1) / (du1 dv2 - du2 dv1) (faces with
    |r| < 1e-12 skipped), summed per position vertex and normalised."""
    p0, p1, p2 = pos[tri[:, 0]], pos[tri[:, 1]], pos[tri[:, 2]]
    t0, t1, t2 = uv[uv_tri[:, 0]], uv[uv_tri[:, 1]], uv[uv_tri[:, 2]]
    e1, e2 = p1 - p0, p2 - p0
    d1, d2 = t1 - t0, t2 - t0
    r = d1[:, 0] * d2[:, 1] - d2[:, 0] * d1[:, 1]
    ok = (r.abs() >= 1e-12)
    rs = torch.where(ok, r, torch.ones_like(r))
    tf = (e1 * d2[:, 1:2] - e2 * d1[:, 1:2]) / rs[:, None]
    tf = torch.where(ok[:, None], tf, torch.zeros_like(tf))
    acc = torch.zeros_like(pos)
    for k in range(3):
        acc = acc.index_add(0, tri[:, k], tf)
    return safe_normalize(acc)


def adjacency(tri: np.ndarray) -> np.ndarray:
    """adj[t, k] = the triangle sharing the edge opposite corner k of t, or -1
    when that edge is a boundary (or shared by more than two triangles)."""
    tri = np.asarray(tri, dtype=np.int64)
    T = tri.shape[0]
    edges = {}
    for t in range(T):
        for k in range(3):
            a, b = int(tri[t, (k + 1) % 3]), int(tri[t, (k + 2) % 3])
            edges.setdefault((min(a, b), max(a, b)), []).append((t, k))
    adj = -np.ones((T, 3), dtype=np.int32)
    for lst in edges.values():
        if len(lst) == 2:
            (t0, k0), (t1, k1) = lst
            adj[t0, k0] = t1
            adj[t1, k1] = t0
    return adj


# ---------------------------------------------------------------------------
# Textures (mip chain, trilinear lookup)
# ---------------------------------------------------------------------------

def mip_chain_f32(level0: torch.Tensor, levels: int | None = None):
    """[S,S,C] -> list of levels, L_{l+1}[i,j] = mean of the 2x2 block."""
    S = level0.shape[0]
    L = int(math.log2(S)) + 1 if levels is None else levels
    out = [level0]
    for _ in range(1, L):
        x = out[-1]
        s = x.shape[0] // 2
        out.append(x.reshape(s, 2, s, 2, x.shape[2]).mean(dim=(1, 3)))
    return out


def mip_chain_rgba8(level0: np.ndarray, levels: int | None = None):
    """uint8 [S,S,4] -> list of float64 rgb levels decoded x/255; coarser levels
    round the 2x2 sum as (a+b+c+d+2)//4 in integers."""
    S = level0.shape[0]
    L = int(math.log2(S)) + 1 if levels is None else levels
    ints = [level0.astype(np.int64)]
    for _ in range(1, L):
        x = ints[-1]
        s = x.shape[0] // 2
        ints.append((x.reshape(s, 2, s, 2, 4).sum(axis=(1, 3)) + 2) // 4)
    return [torch.from_numpy(x[..., :3].astype(np.float64) / 255.0) for x in ints]


def _bilinear(level: torch.Tensor, u, v):
    S = level.shape[0]
    x = u * S - 0.5
    y = v * S - 0.5
    x0 = torch.floor(x.detach())
    y0 = torch.floor(y.detach())
    fx = (x - x0)[:, None]
    fy = (y - y0)[:, None]
    x0 = x0.long()
    y0 = y0.long()
    c0 = torch.remainder(x0, S)
    c1 = torch.remainder(x0 + 1, S)
    r0 = torch.clamp(y0, 0, S - 1)
    r1 = torch.clamp(y0 + 1, 0, S - 1)
    t00 = level[r0, c0]
    t10 = level[r0, c1]
    t01 = level[r1, c0]
    t11 = level[r1, c1]
    return (1 - fx) * (1 - fy) * t00 + fx * (1 - fy) * t10 + (1 - fx) * fy * t01 + fx * fy * t11


def sample_trilinear(levels, uv, duv_dx, duv_dy):
    """Trilinear lookup of N points: uv [N,2], pixel-unit derivatives [N,2]."""
    S = levels[0].shape[0]
    L = len(levels)
    sx2 = (duv_dx[:, 0] * S) ** 2 + (duv_dx[:, 1] * S) ** 2
    sy2 = (duv_dy[:, 0] * S) ** 2 + (duv_dy[:, 1] * S) ** 2
    m = torch.where(sx2 >= sy2, sx2, sy2)
    pos_m = m > 0
    lod_raw = 0.5 * torch.log2(torch.where(pos_m, m, torch.ones_like(m)))
    lod_raw = torch.where(pos_m, lod_raw, torch.zeros_like(lod_raw))
    lod = torch.clamp(lod_raw, 0.0, float(L - 1))
    l0 = torch.floor(lod.detach()).long().clamp(max=L - 1)
    f = (lod - l0.to(lod.dtype))[:, None]
    u, v = uv[:, 0], uv[:, 1]
    C = levels[0].shape[2]
    out = torch.zeros(uv.shape[0], C, dtype=F64)
    for l in range(L):
        sel = l0 == l
        if bool(sel.any()):
            a = _bilinear(levels[l], u[sel], v[sel])
            if l + 1 < L:
                b = _bilinear(levels[l + 1], u[sel], v[sel])
                val = a + f[sel] * (b - a)
            else:
                val = a
            out = out.index_put((sel.nonzero()[:, 0],), val)
    return out


# ---------------------------------------------------------------------------
# Shading (Sec. 5.2)
# ---------------------------------------------------------------------------

def _dot(a, b):
    return (a * b).sum(-1, keepdim=True)


def shade_blinn_phong(n, l, v, kd, light_rgb):
    h = safe_normalize(l + v)
    diff = torch.clamp(_dot(n, l), min=0.0)
    spec = 0.04 * torch.clamp(_dot(n, h), min=0.0) ** 32
    return light_rgb * diff * (kd + spec)


def specular_colour(kd, gamma, metal):
    """Sec. 5.2: k_s = (1 - m) 0.04 + m k_d, and k_s' = (1 - gamma) k_s, the
    specular colour scaled down by the specular-occlusion map gamma."""
    ks = (1.0 - metal) * 0.04 + metal * kd
    return (1.0 - gamma) * ks


def ggx_ndf(nh, alpha):
    """GGX / Trowbridge-Reitz normal distribution of half vectors at cosine
    nh = n.h (reading: the Karis 2013 form the paper cites for its shading
    model), D = alpha^2 / (pi ((n.h)^2 (alpha^2 - 1) + 1)^2)."""
    a2 = alpha * alpha
    return a2 / (math.pi * (nh * nh * (a2 - 1.0) + 1.0) ** 2)


def smith_g1_schlick(x, alpha):
    """Schlick's approximation of Smith's masking term for one direction at
    cosine x, G1(x) = x / (x (1 - k) + k), with k = alpha / 2 (reading: the
    Karis 2013 remap, chosen to match the Smith GGX term)."""
    k = alpha * 0.5
    return x / (x * (1.0 - k) + k)


def fresnel_schlick(f0, vh):
    """Schlick's Fresnel: F = F0 + (1 - F0) (1 - v.h)^5."""
    return f0 + (1.0 - f0) * (1.0 - vh) ** 5


def shade_ggx(n, l, v, kd, orm, light_rgb):
    """Diffuse + GGX specular under one directional light (Sec. 5.2 gives the
    specular colour; the microfacet terms are the readings above):
    c = E (k_d (1 - m) / pi + D F G / (4 max(n.l,1e-4) max(n.v,1e-4))) max(0, n.l),
    roughness clamped to [0.08, 1] and alpha = r^2."""
    gamma, rough, metal = orm[:, 0:1], orm[:, 1:2], orm[:, 2:3]
    r = torch.clamp(rough, 0.08, 1.0)
    alpha = r * r
    h = safe_normalize(l + v)
    nl = torch.clamp(_dot(n, l), min=0.0)
    nv = torch.clamp(_dot(n, v), min=1e-4)
    nh = torch.clamp(_dot(n, h), min=0.0)
    vh = torch.clamp(_dot(v, h), min=0.0)
    D = ggx_ndf(nh, alpha)
    G = smith_g1_schlick(nl, alpha) * smith_g1_schlick(nv, alpha)
    F = fresnel_schlick(specular_colour(kd, gamma, metal), vh)
    spec = D * F * G / (4.0 * torch.clamp(nl, min=1e-4) * nv)
    diffuse = kd * (1.0 - metal) / math.pi
    return light_rgb * (diffuse + spec) * nl


# ---------------------------------------------------------------------------
# Loss (Sec. 5.3)
# ---------------------------------------------------------------------------

def srgb(x):
    """Gamma(x) = 12.92 x for x <= 0.0031308, else 1.055 x^(1/2.4) - 0.055."""
    hi = 1.055 * torch.clamp(x, min=0.0031308) ** (1.0 / 2.4) - 0.055
    return torch.where(x <= 0.0031308, 12.92 * x, hi)


def tonemap(x):
    """x' = Gamma(log(x + 1)) for x >= 0, extended as an odd function,
    T(x) = sign(x) T(|x|), to the negative radiance that freely optimised
    texels can produce (smooth through 0, where T(x) = 12.92 x)."""
    a = torch.abs(x)
    return torch.sign(x) * srgb(torch.log(a + 1.0))


def image_loss(img, ref, kind: str):
    if kind.endswith("tonemap"):
        a, b = tonemap(img), tonemap(ref)
    else:
        a, b = img, ref
    d = a - b
    if kind.startswith("l1"):
        return torch.abs(d).mean()
    return (d * d).mean()


# ---------------------------------------------------------------------------
# Antialiasing (Sec. 5.2; operator of Laine et al. 2020, read as below)
# ---------------------------------------------------------------------------

def aa_pairs(keys: np.ndarray, tri: np.ndarray, snapv: np.ndarray, orient: np.ndarray,
             adj: np.ndarray):
    """Integer decisions of the silhouette antialiasing of one view.

    For each pair of horizontally or vertically adjacent pixels whose
    triangle ids differ, the front triangle F is the one with the smaller key
    (the empty key is largest).  P is the pixel F is visible at, Q the other.
    Among F's oriented edges 0, 1, 2, the first one that Q lies outside of
    (integer edge test, top-left rule) and that is a silhouette edge (a
    boundary edge, or one whose neighbouring triangle has the other screen
    orientation in this view) is the crossing edge.  Returns arrays
    (P flat index, Q flat index, vertex a, vertex b) of the pairs that have a
    crossing edge; the edge runs from a to b with F on its left.
    """
    H, W = keys.shape
    ids = key_tri(keys)
    P_l, Q_l, T_l = [], [], []
    for (dj, di) in ((0, 1), (1, 0)):
        ja, ia = np.meshgrid(np.arange(H - dj), np.arange(W - di), indexing="ij")
        jb, ib = ja + dj, ia + di
        ka, kb = keys[ja, ia], keys[jb, ib]
        diff = ids[ja, ia] != ids[jb, ib]
        a_front = ka < kb
        Pj = np.where(a_front, ja, jb)[diff]
        Pi = np.where(a_front, ia, ib)[diff]
        Qj = np.where(a_front, jb, ja)[diff]
        Qi = np.where(a_front, ib, ia)[diff]
        F = (np.minimum(ka, kb)[diff] & np.uint64(0xFFFFFFFF)).astype(np.int64) - 1
        P_l.append(Pj * W + Pi)
        Q_l.append(np.stack([Qj, Qi], axis=1))
        T_l.append(F)
    P = np.concatenate(P_l)
    Qji = np.concatenate(Q_l)
    F = np.concatenate(T_l)
    bits, vid = edge_inside(tri, snapv, F, Qji[:, 1], Qji[:, 0])
    keep = np.zeros(F.shape[0], dtype=bool)
    va = np.zeros(F.shape[0], dtype=np.int64)
    vb = np.zeros(F.shape[0], dtype=np.int64)
    for k in (2, 1, 0):  # last assignment wins: edge 0 has priority
        ca = vid[:, (k + 1) % 3]
        cb = vid[:, (k + 2) % 3]
        opp = vid[:, k]  # original corner opposite the edge
        nb = adj[F, opp]
        sil = (nb < 0) | (orient[np.maximum(nb, 0)] != orient[F])
        outside = (bits & (1 << k)) == 0
        hit = outside & sil & (bits >= 0)
        va = np.where(hit, tri[F, ca], va)
        vb = np.where(hit, tri[F, cb], vb)
        keep |= hit
    Q = Qji[:, 0] * W + Qji[:, 1]
    return P[keep], Q[keep], va[keep], vb[keep]


def antialias(color: torch.Tensor, clip: torch.Tensor, pairs, W: int, H: int):
    """One view: color [H*W,3] (un-antialiased), clip [V,4] float64.

    For each pair (P, Q, a, b): e(X) is the edge function of the projected
    edge a->b at the NDC centre of pixel X, s = e(P) / (e(P) - e(Q)) clamped
    to [0,1] is where the edge crosses the segment from P to Q.  A box filter
    one pixel wide gives: if s > 1/2, out(Q) += (s - 1/2)(c(P) - c(Q)); if
    s < 1/2, out(P) += (1/2 - s)(c(Q) - c(P)).  All contributions are formed
    from the un-antialiased colours, so their order does not matter.  A pixel
    whose received weights sum to W > 1 has its contributions scaled by 1/W.
    """
    P, Q, va, vb = pairs
    if P.size == 0:
        return color
    P_t = torch.from_numpy(P)
    Q_t = torch.from_numpy(Q)
    def ndc_center(idx):
        i = (idx % W).astype(np.float64)
        j = (idx // W).astype(np.float64)
        return (torch.from_numpy(2.0 * (i + 0.5) / W - 1.0), torch.from_numpy(2.0 * (j + 0.5) / H - 1.0))
    pa = clip[torch.from_numpy(va)]
    pb = clip[torch.from_numpy(vb)]
    ax, ay = pa[:, 0] / pa[:, 3], pa[:, 1] / pa[:, 3]
    bx, by = pb[:, 0] / pb[:, 3], pb[:, 1] / pb[:, 3]
    def efun(c):
        x, y = c
        return (bx - ax) * (y - ay) - (by - ay) * (x - ax)
    eP = efun(ndc_center(P))
    eQ = efun(ndc_center(Q))
    den = eP - eQ
    ok = den != 0
    s = torch.where(ok, eP / torch.where(ok, den, torch.ones_like(den)), torch.full_like(den, 0.5))
    s = torch.clamp(s, 0.0, 1.0)
    cP, cQ = color[P_t], color[Q_t]
    wq = torch.clamp(s - 0.5, min=0.0)[:, None]
    wp = torch.clamp(0.5 - s, min=0.0)[:, None]
    # Weights a pixel receives from several pairs can sum past 1 (several
    # edges of sub-pixel triangles cross near it); they are then scaled by
    # 1 / sum so that every output stays a convex blend of colours.
    wsum = torch.zeros(color.shape[0], 1, dtype=color.dtype)
    wsum = wsum.index_add(0, Q_t, wq).index_add(0, P_t, wp)
    acc = torch.zeros_like(color).index_add(0, Q_t, wq * (cP - cQ)).index_add(0, P_t, wp * (cQ - cP))
    scale = 1.0 / torch.clamp(wsum, min=1.0)
    return color + acc * scale


# ---------------------------------------------------------------------------
# Full render of one batch of views
# ---------------------------------------------------------------------------

def _t(x, dtype=F64):
    return torch.as_tensor(np.asarray(x), dtype=dtype)


def texture_levels(tex_data: np.ndarray, fmt: str, param: torch.Tensor | None = None, chain=None):
    """Mip chain of a map; ``param`` (float64 level 0) replaces the data when
    the map is being differentiated.  With ``chain`` (all levels,
    level-major [N,C]) the levels are independent variables (Sec. 4.2) and
    ``param``, if given, is that whole chain."""
    if fmt == "rgba8":
        return mip_chain_rgba8(tex_data)
    if chain is not None:
        flat = param if param is not None else _t(chain)
        S = tex_data.shape[0]
        out, off = [], 0
        for l in range(int(math.log2(S)) + 1):
            s = S >> l
            out.append(flat[off:off + s * s].reshape(s, s, flat.shape[1]))
            off += s * s
        return out
    base = param if param is not None else _t(tex_data)
    return mip_chain_f32(base)


def screen_derivatives(k, lam, S, W, H):
    """Derivatives of the perspective-correct barycentrics w.r.t. the pixel
    coordinates.  With D_i = k_i . (px, py, 1) and lambda_i = D_i / sum D,
    d lambda_i / d px = (k_ix - lambda_i sum_j k_jx) / sum D, and one pixel
    step moves the NDC coordinate by 2/W in x (2/H in y)."""
    Ka = k[:, :, 0].sum(1, keepdim=True)
    Kb = k[:, :, 1].sum(1, keepdim=True)
    dlam_dx = (k[:, :, 0] - lam * Ka) / S * (2.0 / W)
    dlam_dy = (k[:, :, 1] - lam * Kb) / S * (2.0 / H)
    return dlam_dx, dlam_dy


def shade_view(keys, tri, uv, uv_tri, pos, nrm, tan, clip, model, kd_levels, nrm_levels, orm_levels,
               eye_b, light_dir_b, light_rgb_b, W, H, m=1, alpha_levels=None, keep_gbuf=False):
    """Deferred shading of one view's visibility samples (Sec. 5.2): the
    colour [Hs*Ws,3] of each sample's triangle evaluated at its pixel centre
    (zero where empty), with ``alpha_levels`` the clamped alpha [Hs*Ws] of
    the same lookup (Sec. 4.4, transparency; zero where empty), and the
    G-buffer if asked for."""
    Hs, Ws = keys.shape
    gbuf = None
    alpha = torch.zeros(Hs * Ws, dtype=F64) if alpha_levels is not None else None
    ids = key_tri(keys).reshape(-1)
    pix = np.nonzero(ids)[0]
    color = torch.zeros(Hs * Ws, 3, dtype=F64)
    if pix.size:
        t_idx = torch.from_numpy(ids[pix] - 1)
        # the pixel of each sample; shading is evaluated at its centre
        i = torch.from_numpy(((pix % Ws) // m).astype(np.float64))
        j = torch.from_numpy(((pix // Ws) // m).astype(np.float64))
        px = 2.0 * (i + 0.5) / W - 1.0
        py = 2.0 * (j + 0.5) / H - 1.0
        corners = tri[t_idx]                      # [N,3]
        hh = clip[corners][:, :, [0, 1, 3]]       # [N,3,3] (x, y, w)
        k = torch.stack([torch.cross(hh[:, 1], hh[:, 2], dim=1),
                         torch.cross(hh[:, 2], hh[:, 0], dim=1),
                         torch.cross(hh[:, 0], hh[:, 1], dim=1)], dim=1)  # [N,3,3]
        D = k[:, :, 0] * px[:, None] + k[:, :, 1] * py[:, None] + k[:, :, 2]
        S = D.sum(1, keepdim=True)
        lam = D / S
        dlam_dx, dlam_dy = screen_derivatives(k, lam, S, W, H)
        def interp(attr, idx):
            return (lam[:, :, None] * attr[idx]).sum(1)
        x = interp(pos, corners)
        N = safe_normalize(interp(nrm, corners))
        T = interp(tan, corners)
        tcorn = uv_tri[t_idx]
        uvc = uv[tcorn]                           # [N,3,2]
        uvp = (lam[:, :, None] * uvc).sum(1)
        duv_dx = (dlam_dx[:, :, None] * uvc).sum(1)
        duv_dy = (dlam_dy[:, :, None] * uvc).sum(1)
        Tp = safe_normalize(T - _dot(N, T) * N)
        Bt = torch.cross(N, Tp, dim=1)
        kd = sample_trilinear(kd_levels, uvp, duv_dx, duv_dy)
        nt = sample_trilinear(nrm_levels, uvp, duv_dx, duv_dy)
        n = safe_normalize(nt[:, 0:1] * Tp + nt[:, 1:2] * Bt + nt[:, 2:3] * N)
        e = _t(eye_b)[None, :]
        v = safe_normalize(e - x)
        l = _t(light_dir_b)[None, :].expand_as(n)
        E = _t(light_rgb_b)[None, :]
        if model == "blinn_phong":
            c = shade_blinn_phong(n, l, v, kd, E)
        else:
            orm = sample_trilinear(orm_levels, uvp, duv_dx, duv_dy)
            c = shade_ggx(n, l, v, kd, orm, E)
        color = color.index_put((torch.from_numpy(pix),), c)
        if alpha_levels is not None:
            a = torch.clamp(sample_trilinear(alpha_levels, uvp, duv_dx, duv_dy)[:, 0], 0.0, 1.0)
            alpha = alpha.index_put((torch.from_numpy(pix),), a)
        if keep_gbuf:
            gbuf = dict(pix=pix, lam=lam.detach(), x=x.detach(), N=N.detach(), uv=uvp.detach(),
                        duv_dx=duv_dx.detach(), duv_dy=duv_dy.detach(), n=n.detach(), kd=kd.detach())
    return color, alpha, gbuf


def render(mesh, model: str, kd_levels, nrm_levels, orm_levels, pos: torch.Tensor,
           mvp32: np.ndarray, eye: np.ndarray, light_dir: np.ndarray, light_rgb: np.ndarray,
           W: int, H: int, adj: np.ndarray | None = None, aa: bool = True,
           keep_gbuf: bool = False, frozen: dict | None = None, msaa: int = 1):
    """Render B views.  ``pos`` is float64 [V,3] (may require grad); the
    visibility uses its float32 rounding (R1).  Returns a dict with
    image [B,H*W,3] (antialiased), color [B,Hs*Ws,3], keys [B,Hs,Ws] uint64,
    coverage [B,Hs,Ws] and per-view AA pair lists.  ``frozen``: the output of
    an earlier call whose visibility and antialiasing pairs are reused (the
    loss is then a smooth function of the positions, for finite
    differences).

    Multisampling (Sec. 5.2, "Antialiasing"; ``msaa`` = m > 1): visibility is
    sampled on an m x m grid per pixel (the rasterizer at Ws = m W,
    Hs = m H), each sample's triangle is shaded once per pixel at the pixel
    centre, the silhouette antialiasing runs between adjacent samples, and
    the image is the mean of each pixel's m^2 samples."""
    tri_np = np.asarray(mesh.tri, dtype=np.int64)
    tri = torch.from_numpy(tri_np)
    uv = _t(mesh.uv)
    uv_tri = torch.from_numpy(np.asarray(mesh.uv_tri, dtype=np.int64))
    if adj is None:
        adj = adjacency(tri_np)
    nrm = vertex_normals(pos, tri)
    tan = vertex_tangents(pos, tri, uv, uv_tri)
    B = mvp32.shape[0]
    m = int(msaa)
    Ws, Hs = W * m, H * m
    pos32 = pos.detach().numpy().astype(np.float32)
    images, colors, keys_all, cov_all, pairs_all, gbufs = [], [], [], [], [], []
    for b in range(B):
        M = _t(mvp32[b].astype(np.float64))
        clip = torch.cat([pos, torch.ones(pos.shape[0], 1, dtype=F64)], dim=1) @ M.T
        sv = snap(pos32, mvp32[b], Ws, Hs)
        if frozen is None:
            keys, cov, orient = raster(tri_np, sv, Ws, Hs)
        else:
            keys, cov = frozen["keys"][b], frozen["coverage"][b]
        color, _, gb = shade_view(keys, tri, uv, uv_tri, pos, nrm, tan, clip, model, kd_levels, nrm_levels,
                                  orm_levels, eye[b], light_dir[b], light_rgb[b], W, H, m, keep_gbuf=keep_gbuf)
        if gb is not None:
            gbufs.append(gb)
        pairs = aa_pairs(keys, tri_np, sv, orient, adj) if frozen is None else frozen["pairs"][b]
        img = antialias(color, clip, pairs, Ws, Hs) if aa else color
        if m > 1:
            img = img.reshape(H, m, W, m, 3).mean(dim=(1, 3)).reshape(H * W, 3)
        images.append(img)
        colors.append(color)
        keys_all.append(keys)
        cov_all.append(cov)
        pairs_all.append(pairs)
    return dict(image=torch.stack(images), color=torch.stack(colors), keys=np.stack(keys_all),
                coverage=np.stack(cov_all), pairs=pairs_all, normals=nrm, tangents=tan, gbuf=gbufs)


# ---------------------------------------------------------------------------
# Optimiser (Sec. 5.3: Adam with default parameters)
# ---------------------------------------------------------------------------

def lr_schedule(lr0: float, t: int, k: float = 0.0002) -> float:
    """lr at 1-based step t: lr0 * 10^(-k (t-1)) (iterations counted from 0)."""
    return lr0 * 10.0 ** (-k * (t - 1))


def adam(p, g, m, v, t: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam step (t 1-based); returns (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
