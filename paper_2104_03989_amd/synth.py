"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws and lays out inputs: geodesic spheres, their UV
parameterisation, radial displacement fields, value-noise texture maps and
random view/light directions.  It holds none of the render loop's arithmetic
(no projection, rasterization, shading, loss or optimiser step), so that the
GPU path and the FP64 oracle can both consume the same inputs while sharing no
computation.

The paper's assets (Smithsonian scans, the Paragon character, Moana) are not
available; the shapes below stand in for them with the triangle counts,
texture sizes and view counts of the experiments in Sec. 4.1 (normal-map
baking, complex materials, displacement baking).

Every random draw goes through ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

BASE_SEED = 2104_03989


def seed_for(config: int, item: int) -> int:
    """Seed of input ``item`` of workload ``config``."""
    return BASE_SEED + config * 1000 + item


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# ---------------------------------------------------------------------------
# Geodesic sphere of frequency nu: 20 nu^2 triangles, 10 nu^2 + 2 vertices.
# ---------------------------------------------------------------------------

_T = (1.0 + 5.0 ** 0.5) / 2.0
_ICO_V = np.array(
    [(-1, _T, 0), (1, _T, 0), (-1, -_T, 0), (1, -_T, 0),
     (0, -1, _T), (0, 1, _T), (0, -1, -_T), (0, 1, -_T),
     (_T, 0, -1), (_T, 0, 1), (-_T, 0, -1), (-_T, 0, 1)], dtype=np.float64)
_ICO_F = np.array(
    [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
     (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
     (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
     (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)], dtype=np.int64)


def _pole_rotation() -> np.ndarray:
    # rotate about z so that corner 0 lies on +y (and corner 3 on -y): every
    # frequency then has a vertex exactly at each pole of the UV mapping
    a = _ICO_V[0] / np.linalg.norm(_ICO_V[0])
    ang = math.atan2(a[0], a[1])
    c, s = math.cos(ang), math.sin(ang)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


_ICO_V = _ICO_V @ _pole_rotation().T


def geodesic_sphere(nu: int):
    """Unit geodesic sphere: each icosahedron face split into nu^2 triangles.

    Returns (dirs [V,3] float64 unit vectors, tri [T,3] int32), triangles
    wound counter-clockwise seen from outside.  nu = 2^k gives the same
    counts as an icosphere subdivided k times.
    """
    nu = int(nu)
    if nu < 1:
        raise ValueError("nu must be >= 1")
    ii, jj = [], []
    for i in range(nu + 1):
        for j in range(nu + 1 - i):
            ii.append(i)
            jj.append(j)
    ii = np.array(ii, dtype=np.int64)
    jj = np.array(jj, dtype=np.int64)
    npf = ii.size
    local = -np.ones((nu + 1, nu + 1), dtype=np.int64)
    local[ii, jj] = np.arange(npf)
    # integer barycentric weights on the 12 icosahedron corners
    keys = np.zeros((20 * npf, 12), dtype=np.int32)
    for f, (a, b, c) in enumerate(_ICO_F):
        rows = slice(f * npf, (f + 1) * npf)
        keys[rows, a] += (nu - ii - jj).astype(np.int32)
        keys[rows, b] += ii.astype(np.int32)
        keys[rows, c] += jj.astype(np.int32)
    uniq, inverse = np.unique(keys, axis=0, return_inverse=True)
    inverse = inverse.reshape(-1)
    pts = uniq.astype(np.float64) @ _ICO_V
    dirs = pts / np.linalg.norm(pts, axis=1, keepdims=True)
    # local triangles of one face
    up = [(local[i, j], local[i + 1, j], local[i, j + 1])
          for i in range(nu) for j in range(nu - i)]
    down = [(local[i + 1, j], local[i + 1, j + 1], local[i, j + 1])
            for i in range(nu - 1) for j in range(nu - 1 - i)]
    loc = np.array(up + down, dtype=np.int64)
    tris = np.concatenate([inverse[f * npf + loc] for f in range(20)], axis=0)
    assert dirs.shape[0] == 10 * nu * nu + 2
    assert tris.shape[0] == 20 * nu * nu
    return dirs, tris.astype(np.int32)


def sphere_uv(dirs: np.ndarray, tri: np.ndarray):
    """Equirectangular UVs with a separate UV index buffer.

    u = 0.5 + atan2(z, x) / 2pi, v = acos(y) / pi.  Triangles straddling the
    u seam get u + 1 on their low side (texture lookups wrap in u); a pole
    corner takes the mean u of its triangle's two other corners.  Returns
    (uv [Vt,2] float32, uv_tri [T,3] int32).
    """
    y = np.clip(dirs[:, 1], -1.0, 1.0)
    u = 0.5 + np.arctan2(dirs[:, 2], dirs[:, 0]) / (2.0 * math.pi)
    v = np.arccos(y) / math.pi
    pole = np.abs(np.abs(y) - 1.0) < 1e-12
    cu = u[tri].copy()
    cv = v[tri].copy()
    cpole = pole[tri]
    big = 1e9
    lo = np.where(cpole, big, cu).min(axis=1)
    hi = np.where(cpole, -big, cu).max(axis=1)
    seam = (hi - lo) > 0.5
    fix = seam[:, None] & (cu < 0.5) & ~cpole
    cu = np.where(fix, cu + 1.0, cu)
    n_np = (~cpole).sum(axis=1)
    mean_u = np.where(cpole, 0.0, cu).sum(axis=1) / np.maximum(n_np, 1)
    cu = np.where(cpole, mean_u[:, None], cu)
    corners = np.stack([cu.reshape(-1), cv.reshape(-1)], axis=1)
    uniq, inv = np.unique(corners, axis=0, return_inverse=True)
    return uniq.astype(np.float32), inv.reshape(-1, 3).astype(np.int32)


# ---------------------------------------------------------------------------
# Radial displacement fields
# ---------------------------------------------------------------------------

def _real_sh(lmax: int, dirs: np.ndarray) -> np.ndarray:
    from scipy.special import sph_harm_y
    theta = np.arccos(np.clip(dirs[:, 2], -1.0, 1.0))
    phi = np.arctan2(dirs[:, 1], dirs[:, 0])
    cols = []
    for l in range(lmax + 1):
        for m in range(-l, l + 1):
            y = sph_harm_y(l, abs(m), theta, phi)
            if m > 0:
                cols.append(math.sqrt(2.0) * (-1) ** m * y.real)
            elif m < 0:
                cols.append(math.sqrt(2.0) * (-1) ** m * y.imag)
            else:
                cols.append(y.real)
    return np.stack(cols, axis=1)


def sh_radius(dirs: np.ndarray, seed: int, lmax: int = 6, sigma: float = 0.05):
    """r = 1 + sum_{l<=lmax,m} c_lm Y_lm(d), c_lm ~ N(0, sigma^2)."""
    basis = _real_sh(lmax, dirs)
    c = _rng(seed).normal(0.0, sigma, size=basis.shape[1])
    return 1.0 + basis @ c


class _Noise3:
    """Seeded 3-D value noise in [-1, 1] on the integer lattice."""

    def __init__(self, seed: int):
        g = _rng(seed)
        self.perm = g.permutation(256).astype(np.int64)
        self.vals = g.uniform(-1.0, 1.0, size=256)

    def _lat(self, ix, iy, iz):
        p = self.perm
        h = p[(p[(p[ix & 255] + iy) & 255] + iz) & 255]
        return self.vals[h]

    def __call__(self, pts: np.ndarray) -> np.ndarray:
        f = np.floor(pts)
        i = f.astype(np.int64)
        t = pts - f
        s = t * t * (3.0 - 2.0 * t)
        out = np.zeros(pts.shape[0])
        for dx in (0, 1):
            wx = s[:, 0] if dx else 1.0 - s[:, 0]
            for dy in (0, 1):
                wy = s[:, 1] if dy else 1.0 - s[:, 1]
                for dz in (0, 1):
                    wz = s[:, 2] if dz else 1.0 - s[:, 2]
                    out += wx * wy * wz * self._lat(i[:, 0] + dx, i[:, 1] + dy, i[:, 2] + dz)
        return out


def fbm_radius(dirs: np.ndarray, seed: int, octaves: int = 6, amp: float = 0.1):
    """r = 1 + amp * sum_{o<octaves} 0.5^o * vnoise(2^(o+1) d)."""
    n = _Noise3(seed)
    acc = np.zeros(dirs.shape[0])
    for o in range(octaves):
        acc += 0.5 ** o * n(dirs * 2.0 ** (o + 1))
    return 1.0 + amp * acc


# ---------------------------------------------------------------------------
# Texture maps (value noise on an 8x8 lattice, periodic in u)
# ---------------------------------------------------------------------------

def _interp_matrix(size: int, cells: int, periodic: bool) -> np.ndarray:
    x = (np.arange(size) + 0.5) / size * cells - 0.5
    x0 = np.floor(x).astype(np.int64)
    t = x - x0
    s = t * t * (3.0 - 2.0 * t)
    n = cells if periodic else cells + 1
    m = np.zeros((size, n))
    for off, w in ((0, 1.0 - s), (1, s)):
        idx = x0 + off
        idx = np.mod(idx, cells) if periodic else np.clip(idx + 0, 0, cells)
        np.add.at(m, (np.arange(size), idx), w)
    return m


def value_noise_map(size: int, channels: int, seed: int, cells: int = 8) -> np.ndarray:
    """[size, size, channels] float64 in [0, 1); row index is v, column is u."""
    g = _rng(seed)
    lat = g.uniform(0.0, 1.0, size=(channels, cells + 1, cells))
    wu = _interp_matrix(size, cells, periodic=True)
    wv = _interp_matrix(size, cells, periodic=False)
    out = np.einsum("vi,cij,uj->vuc", wv, lat, wu)
    return np.clip(out, 0.0, np.nextafter(1.0, 0.0))


def to_rgba8(rgb: np.ndarray) -> np.ndarray:
    """Quantise [0,1) colours to RGBA8 (alpha 255)."""
    q = np.clip(np.floor(rgb * 256.0), 0, 255).astype(np.uint8)
    a = np.full(rgb.shape[:2] + (1,), 255, dtype=np.uint8)
    return np.concatenate([q[..., :3], a], axis=-1)


def detail_normal_map(size: int, seed: int, tilt: float = 0.2) -> np.ndarray:
    """Tangent-space normals (tilt*(2n-1), tilt*(2n-1), sqrt(1-x^2-y^2))."""
    n = value_noise_map(size, 2, seed)
    xy = tilt * (2.0 * n - 1.0)
    z = np.sqrt(1.0 - (xy ** 2).sum(-1, keepdims=True))
    return np.concatenate([xy, z], axis=-1)


def flat_normal_map(size: int) -> np.ndarray:
    out = np.zeros((size, size, 3))
    out[..., 2] = 1.0
    return out


def orm_map(size: int, seed: int, r_lo: float = 0.2, r_hi: float = 0.8) -> np.ndarray:
    """(gamma=0, roughness in [r_lo, r_hi], metalness in [0,1))."""
    n = value_noise_map(size, 2, seed)
    g = np.zeros((size, size, 1))
    r = r_lo + (r_hi - r_lo) * n[..., :1]
    m = n[..., 1:2]
    return np.concatenate([g, r, m], axis=-1)


# ---------------------------------------------------------------------------
# Views and lights
# ---------------------------------------------------------------------------

def random_unit(n: int, seed: int) -> np.ndarray:
    """n directions uniform on the unit sphere (normalised N(0, I3))."""
    g = _rng(seed).normal(size=(n, 3))
    return g / np.linalg.norm(g, axis=1, keepdims=True)


# ---------------------------------------------------------------------------
# Scenes
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Mesh:
    pos: np.ndarray      # [V,3] float32
    tri: np.ndarray      # [T,3] int32
    uv: np.ndarray       # [Vt,2] float32
    uv_tri: np.ndarray   # [T,3] int32


@dataclasses.dataclass
class Texture:
    """Level-0 texel data; rows are v, columns are u.  ``chain``: for a map
    whose mip levels are independent latent variables, all levels
    (level-major, [sum_l (S>>l)^2, C] float32); None: levels derived."""
    data: np.ndarray     # [S,S,C] float32, or [S,S,4] uint8 for RGBA8
    fmt: str             # "f32" or "rgba8"
    chain: np.ndarray | None = None


@dataclasses.dataclass
class Scene:
    mesh: Mesh
    model: str           # "blinn_phong" or "ggx"
    kd: Texture
    normal: Texture
    orm: Texture | None
    alpha: Texture | None = None   # [S,S,1] f32 transparency map (depth-peeled rendering only)


@dataclasses.dataclass
class Workload:
    name: str
    ref: Scene
    latent: Scene
    dirs: np.ndarray        # [B,3] camera directions (eye = dist * dir)
    light_dir: np.ndarray   # [B,3] unit, towards the light
    light_rgb: np.ndarray   # [B,3]
    width: int
    height: int
    dist: float
    fov_deg: float
    loss: str               # "l1", "l1_tonemap", "l2", "l2_tonemap"
    lr: float
    optimize: tuple         # names among "pos", "kd", "normal", "orm", "disp"
    disp: Texture | None = None   # [S,S,1] f32 displacement map of a tessellated latent
    tess_levels: int = 0          # midpoint subdivisions of the latent (base) mesh
    msaa: int = 1                 # latent visibility samples per pixel axis
    ref_ssaa: int = 1             # reference rendered at this many times the resolution, box-filtered
    rig: "Rig | None" = None      # skeletal animation shared by reference and latent
    weights: np.ndarray | None = None   # [V_latent, n_bones] float32 initial latent skinning weights
    frame: int = 0                # animation frame a single step renders
    oit_layers: int = 0           # latent rendered with this many depth-peeled layers (0: opaque)


@dataclasses.dataclass
class Rig:
    """A skeleton with known per-frame bone transforms (constants of the
    optimisation) and the reference's skinning weights."""
    joints: np.ndarray       # [B,3] float32 bind-pose pivot of each bone
    parent: np.ndarray       # [B] int32, -1 for the root
    bones: np.ndarray        # [F,B,3,4] float32: top rows of each bone's bind-to-frame affine transform
    ref_weights: np.ndarray  # [V_ref,B] float32, at most four non-zero weights per row, rows sum to 1


def _axis_angle(axis: np.ndarray, theta: float) -> np.ndarray:
    x, y, z = axis
    c, s, t = math.cos(theta), math.sin(theta), 1.0 - math.cos(theta)
    return np.array([[t * x * x + c, t * x * y - s * z, t * x * z + s * y],
                     [t * x * y + s * z, t * y * y + c, t * y * z - s * x],
                     [t * x * z - s * y, t * y * z + s * x, t * z * z + c]])


def synthetic_rig(ref_pos: np.ndarray, n_bones: int, n_frames: int, seed: int, chains: int = 5,
                  reach: float = 0.8, amplitude: float = 0.25, sigma: float = 0.2) -> Rig:
    """A root bone and ``chains`` chains of bones radiating from the centre
    to ``reach``; each non-root bone swings about its own pivot by
    amplitude * sin(2 pi f / F + phase) around a random axis, composed down
    its chain (forward kinematics of the input animation), and the root
    sways about y.  Reference weights: Gaussian falloff (``sigma``) from each
    bone's segment midpoint, the four largest kept and normalised."""
    rng = _rng(seed)
    n_chain = n_bones - 1
    lengths = [n_chain // chains + (1 if c < n_chain % chains else 0) for c in range(chains)]
    dirs = random_unit(chains, seed + 1)
    joints = [np.zeros(3)]
    parent = [-1]
    centre = [np.zeros(3)]
    for c, ln in enumerate(lengths):
        seg = reach / max(ln, 1)
        p, d, par = np.zeros(3), dirs[c], 0
        for k in range(ln):
            d = d + rng.normal(0.0, 0.15, 3)
            d = d / np.linalg.norm(d)
            q = p + seg * d if k > 0 else p + 0.15 * d
            joints.append(q)
            parent.append(par)
            centre.append(q + 0.5 * seg * d)
            par = len(joints) - 1
            p = q
    joints = np.array(joints)
    centre = np.array(centre)
    B = joints.shape[0]
    axes = random_unit(B, seed + 2)
    phase = rng.uniform(0.0, 2.0 * math.pi, B)
    bones = np.zeros((n_frames, B, 3, 4))
    for f in range(n_frames):
        world = [None] * B
        for b in range(B):
            th = amplitude * math.sin(2.0 * math.pi * f / n_frames + phase[b])
            if parent[b] < 0:
                local = np.eye(4)
                local[:3, :3] = _axis_angle(np.array([0.0, 1.0, 0.0]), 0.5 * th)
                local[:3, 3] = [0.05 * math.sin(2.0 * math.pi * f / n_frames), 0.0, 0.0]
            else:
                r = _axis_angle(axes[b], th)
                local = np.eye(4)
                local[:3, :3] = r
                local[:3, 3] = joints[b] - r @ joints[b]       # rotate about the bone's pivot
            world[b] = local if parent[b] < 0 else world[parent[b]] @ local
            bones[f, b] = world[b][:3]
    d2 = ((ref_pos[:, None, :].astype(np.float64) - centre[None]) ** 2).sum(-1)
    w = np.exp(-d2 / (2.0 * sigma * sigma))
    keep = np.argsort(-w, axis=1)[:, :4]
    dense = np.zeros_like(w)
    rows = np.arange(w.shape[0])[:, None]
    dense[rows, keep] = w[rows, keep]
    dense /= dense.sum(1, keepdims=True)
    return Rig(joints.astype(np.float32), np.array(parent, dtype=np.int32), bones.astype(np.float32),
               dense.astype(np.float32))


def sphere_mesh(nu: int, radius_fn=None, jitter: float = 0.0, seed: int = 0) -> Mesh:
    dirs, tri = geodesic_sphere(nu)
    uv, uv_tri = sphere_uv(dirs, tri)
    r = np.ones(dirs.shape[0]) if radius_fn is None else radius_fn(dirs)
    pos = dirs * r[:, None]
    if jitter > 0.0:
        pos = pos + _rng(seed).normal(0.0, jitter, size=pos.shape)
    return Mesh(pos.astype(np.float32), tri, uv, uv_tri)


def _f32(x):
    return Texture(np.ascontiguousarray(x, dtype=np.float32), "f32")


def independent_chain(size: int, channels: int, seed: int, lo: float = 0.0, hi: float = 1.0) -> Texture:
    """A map whose every mip level is its own seeded value-noise map in
    [lo, hi) (4x4 lattice cells; a different seed per level)."""
    levels = []
    for l in range(int(np.log2(size)) + 1):
        s = size >> l
        levels.append((lo + (hi - lo) * value_noise_map(s, channels, seed * 64 + l, cells=4)).reshape(-1, channels))
    chain = np.concatenate(levels).astype(np.float32)
    return Texture(chain[:size * size].reshape(size, size, channels).copy(), "f32", chain)


def workload_plain_step(views: int = 4, res: int = 256, map_size: int = 256,
                        ref_nu: int = 32, lat_nu: int = 8) -> Workload:
    """Plain single step: icosphere(3x) vs SH-displaced icosphere(5x), Lambert
    + Blinn-Phong, RGBA8 base colour shared and fixed, FP32 normal map
    optimised from flat, 4 views at 256^2, one directional light, L1 loss."""
    c = 1
    kd = Texture(to_rgba8(value_noise_map(map_size, 3, seed_for(c, 1))), "rgba8")
    ref_mesh = sphere_mesh(ref_nu, lambda d: sh_radius(d, seed_for(c, 2)))
    lat_mesh = sphere_mesh(lat_nu, None, jitter=0.01, seed=seed_for(c, 3))
    ref = Scene(ref_mesh, "blinn_phong", kd, _f32(detail_normal_map(map_size, seed_for(c, 4))), None)
    lat = Scene(lat_mesh, "blinn_phong", kd, _f32(flat_normal_map(map_size)), None)
    dirs = random_unit(views, seed_for(c, 5))
    light = np.repeat(random_unit(1, seed_for(c, 6)), views, axis=0)
    return Workload("plain_step", ref, lat, dirs, light, np.ones((views, 3)), res, res,
                    3.0, 45.0, "l1", 1e-3, ("pos", "normal"))


def workload_paper_loop(views: int = 8, res: int = 512, map_size: int = 2048,
                        ref_nu: int = 122, lat_nu: int = 19) -> Workload:
    """Paper-scale loop: ~300k-tri fbm sphere with 2048^2 base colour
    (RGBA8), normal and ORM maps under GGX; ~7k-tri latent resampled on the
    same fbm surface with 2048^2 FP32 normal and base-colour maps; 8 views
    at 512^2, one random directional light per view, tonemapped L1."""
    c = 2
    rad = lambda d: fbm_radius(d, seed_for(c, 1))
    ref_mesh = sphere_mesh(ref_nu, rad)
    lat_mesh = sphere_mesh(lat_nu, rad)
    kd_ref = Texture(to_rgba8(value_noise_map(map_size, 3, seed_for(c, 2))), "rgba8")
    ref = Scene(ref_mesh, "ggx", kd_ref, _f32(detail_normal_map(map_size, seed_for(c, 3))),
                _f32(orm_map(map_size, seed_for(c, 4))))
    kd_lat = _rng(seed_for(c, 5)).uniform(0.0, 1.0, size=(map_size, map_size, 3))
    orm_lat = np.array([0.0, 0.5, 0.0]).reshape(1, 1, 3)
    lat = Scene(lat_mesh, "ggx", _f32(kd_lat), _f32(flat_normal_map(map_size)), _f32(orm_lat))
    dirs = random_unit(views, seed_for(c, 6))
    light = random_unit(views, seed_for(c, 7))
    return Workload("paper_loop", ref, lat, dirs, light, np.ones((views, 3)), res, res,
                    3.0, 45.0, "l1_tonemap", 2e-3, ("pos", "kd", "normal"))


def workload_displacement(views: int = 8, res: int = 512, map_size: int = 1024,
                          ref_nu: int = 136, base_nu: int = 7, levels: int = 3) -> Workload:
    """Differentiation-heavy loop: a 980-tri base mesh resampled on an fbm
    sphere, tessellated three times (62,720 tris) and displaced along its
    interpolated normals by a 1024^2 FP32 map (initialised to 0), with a
    1024^2 FP32 normal map; the reference is a 369,920-tri fbm sphere; 8 views
    at 512^2 with a light per view, Lambert + Blinn-Phong, L1 loss."""
    c = 3
    rad = lambda d: fbm_radius(d, seed_for(c, 1))
    kd = _f32(np.full((1, 1, 3), 0.7))
    ref = Scene(sphere_mesh(ref_nu, rad), "blinn_phong", kd, _f32(flat_normal_map(1)), None)
    lat = Scene(sphere_mesh(base_nu, rad), "blinn_phong", kd, _f32(flat_normal_map(map_size)), None)
    disp = _f32(np.zeros((map_size, map_size, 1)))
    dirs = random_unit(views, seed_for(c, 2))
    light = random_unit(views, seed_for(c, 3))
    return Workload("displacement", ref, lat, dirs, light, np.ones((views, 3)), res, res,
                    3.0, 45.0, "l1", 1e-3, ("pos", "disp", "normal"), disp, levels)


def workload_prefilter(views: int = 8, res: int = 128, ssaa: int = 8, msaa: int = 4, map_size: int = 512,
                       ref_nu: int = 122, lat_nu: int = 19) -> Workload:
    """Joint shape and appearance prefiltering (Sec. 4.2): the paper-scale
    GGX reference rendered with ssaa^2 samples per pixel at a low target
    resolution; a ~7k-triangle latent with multisampled visibility and base
    colour and normal maps whose mip levels are independent variables."""
    c = 6
    rad = lambda d: fbm_radius(d, seed_for(2, 1))
    ref_mesh = sphere_mesh(ref_nu, rad)
    kd_ref = Texture(to_rgba8(value_noise_map(2048, 3, seed_for(2, 2))), "rgba8")
    ref = Scene(ref_mesh, "ggx", kd_ref, _f32(detail_normal_map(2048, seed_for(2, 3))),
                _f32(orm_map(2048, seed_for(2, 4))))
    kd = independent_chain(map_size, 3, seed_for(c, 1), 0.0, 1.0)
    nm = independent_chain(map_size, 3, seed_for(c, 2), -0.05, 0.05)
    nm.chain[:, 2] = 1.0
    nm.data[..., 2] = 1.0
    orm = independent_chain(map_size, 3, seed_for(c, 3), 0.2, 0.6)
    lat = Scene(sphere_mesh(lat_nu, rad), "ggx", kd, nm, orm)
    dirs = random_unit(views, seed_for(c, 4))
    light = random_unit(views, seed_for(c, 5))
    return Workload("prefilter", ref, lat, dirs, light, np.ones((views, 3)), res, res, 3.0, 45.0, "l1_tonemap",
                    2e-3, ("pos", "kd", "normal", "orm"), msaa=msaa, ref_ssaa=ssaa)


def workload_animation(views: int = 8, res: int = 512, map_size: int = 1024, ref_nu: int = 31,
                       lat_nu: int = 16, n_bones: int = 32, n_frames: int = 40) -> Workload:
    """Animated character (Sec. 4.3): a 19,220-tri SH blob skinned to a
    32-bone skeleton (a root and five chains) with 40 frames of known bone
    transforms; a 5,120-tri reduced latent with dense skinning weights
    initialised to 1/32 per bone, optimised with its bind-pose positions and
    1024^2 base colour, normal and ORM maps under GGX; 8 views at 512^2 of one
    frame per step, a light per view, tonemapped L1."""
    c = 7
    rad = lambda d: sh_radius(d, seed_for(c, 1), lmax=4, sigma=0.08)
    ref_mesh = sphere_mesh(ref_nu, rad)
    rig = synthetic_rig(ref_mesh.pos, n_bones, n_frames, seed_for(c, 2))
    kd_ref = Texture(to_rgba8(value_noise_map(map_size, 3, seed_for(c, 3))), "rgba8")
    ref = Scene(ref_mesh, "ggx", kd_ref, _f32(detail_normal_map(map_size, seed_for(c, 4))),
                _f32(orm_map(map_size, seed_for(c, 5))))
    lat_mesh = sphere_mesh(lat_nu, rad)
    kd_lat = _rng(seed_for(c, 6)).uniform(0.0, 1.0, size=(map_size, map_size, 3))
    orm_lat = np.broadcast_to(np.array([0.0, 0.5, 0.0]), (map_size, map_size, 3))
    lat = Scene(lat_mesh, "ggx", _f32(kd_lat), _f32(flat_normal_map(map_size)), _f32(orm_lat))
    weights = np.full((lat_mesh.pos.shape[0], n_bones), 1.0 / n_bones, dtype=np.float32)
    dirs = random_unit(views, seed_for(c, 7))
    light = random_unit(views, seed_for(c, 8))
    return Workload("animation", ref, lat, dirs, light, np.ones((views, 3)), res, res, 3.0, 45.0, "l1_tonemap",
                    2e-3, ("pos", "weights", "kd", "normal", "orm"), rig=rig, weights=weights)


def leaf_cloud(n_leaves: int, seed: int, radius: float = 1.0, size: float = 0.06, rim: int = 8,
               uv_extent: float = 0.02) -> Mesh:
    """Aggregate geometry: n_leaves flat elliptic leaves (a fan of ``rim``
    triangles each) at uniform positions in a ball, random orientations,
    each mapping to a small random region of the texture."""
    g = _rng(seed)
    c = g.normal(size=(n_leaves, 3))
    c *= (radius * g.uniform(0.0, 1.0, n_leaves) ** (1.0 / 3.0) / np.linalg.norm(c, axis=1))[:, None]
    nrm = random_unit(n_leaves, seed + 1)
    helper = np.where(np.abs(nrm[:, :1]) < 0.9, np.array([[1.0, 0.0, 0.0]]), np.array([[0.0, 1.0, 0.0]]))
    t1 = np.cross(nrm, helper)
    t1 /= np.linalg.norm(t1, axis=1, keepdims=True)
    t2 = np.cross(nrm, t1)
    a = size * g.uniform(0.7, 1.3, n_leaves)
    bb = 0.5 * a
    ang = 2.0 * np.pi * np.arange(rim) / rim
    ring = (a[:, None, None] * np.cos(ang)[None, :, None] * t1[:, None, :]
            + bb[:, None, None] * np.sin(ang)[None, :, None] * t2[:, None, :])
    pos = np.concatenate([c[:, None, :], c[:, None, :] + ring], axis=1).reshape(-1, 3)
    uc = g.uniform(uv_extent, 1.0 - uv_extent, size=(n_leaves, 2))
    uv_ring = np.stack([np.cos(ang), 0.5 * np.sin(ang)], axis=1) * uv_extent
    uv = np.concatenate([uc[:, None, :], uc[:, None, :] + uv_ring[None]], axis=1).reshape(-1, 2)
    base = (np.arange(n_leaves) * (rim + 1))[:, None]
    k = np.arange(rim)
    tri = np.stack([np.zeros(rim, np.int64), 1 + k, 1 + (k + 1) % rim], axis=1)[None] + base[:, :, None]
    tri = tri.reshape(-1, 3).astype(np.int32)
    return Mesh(pos.astype(np.float32), tri, uv.astype(np.float32), tri.copy())


def quad_cloud(n_quads: int, seed: int, radius: float = 1.0, size: float = 0.15) -> Mesh:
    """Billboard quads (two triangles each) at uniform positions in a ball
    with random orientations, each mapped to its own cell of a square
    texture atlas (ceil(sqrt(n)) cells per side, half a cell-texel margin)."""
    g = _rng(seed)
    c = g.normal(size=(n_quads, 3))
    c *= (radius * g.uniform(0.0, 1.0, n_quads) ** (1.0 / 3.0) / np.linalg.norm(c, axis=1))[:, None]
    nrm = random_unit(n_quads, seed + 1)
    helper = np.where(np.abs(nrm[:, :1]) < 0.9, np.array([[1.0, 0.0, 0.0]]), np.array([[0.0, 1.0, 0.0]]))
    t1 = np.cross(nrm, helper)
    t1 /= np.linalg.norm(t1, axis=1, keepdims=True)
    t2 = np.cross(nrm, t1)
    h = 0.5 * size
    corners = np.array([(-1, -1), (1, -1), (-1, 1), (1, 1)], dtype=np.float64)
    pos = (c[:, None, :] + h * corners[None, :, 0:1] * t1[:, None, :]
           + h * corners[None, :, 1:2] * t2[:, None, :]).reshape(-1, 3)
    n = int(math.ceil(math.sqrt(n_quads)))
    cell = 1.0 / n
    q = np.arange(n_quads)
    cu, cv = (q % n) * cell, (q // n) * cell
    m = 0.02 * cell
    uvc = (np.array([(0, 0), (1, 0), (0, 1), (1, 1)], dtype=np.float64) * (cell - 2 * m) + m)
    uv = (np.stack([cu, cv], 1)[:, None, :] + uvc[None]).reshape(-1, 2)
    base = (4 * q)[:, None, None]
    tri = (np.array([[0, 1, 3], [0, 3, 2]])[None] + base).reshape(-1, 3).astype(np.int32)
    return Mesh(pos.astype(np.float32), tri, uv.astype(np.float32), tri.copy())


def workload_aggregate(views: int = 8, res: int = 512, map_size: int = 2048, n_leaves: int = 150_000,
                       n_quads: int = 4800, layers: int = 8) -> Workload:
    """Aggregate geometry (Sec. 4.4): a foliage stand-in of 150,000 leaves
    (1.2M triangles) against 4,800 textured quads (9,600 triangles, 0.8%)
    whose base colour, normal and transparency maps (2048^2 atlases) and
    positions are optimised; the latent is rendered with 8 depth-peeled
    layers; 8 views at 512^2, a light per view, Blinn-Phong, squared L2."""
    c = 8
    leaves = leaf_cloud(n_leaves, seed_for(c, 1))
    kd_ref = Texture(to_rgba8(0.15 + 0.6 * value_noise_map(1024, 3, seed_for(c, 2)) * np.array([0.5, 1.0, 0.3])),
                     "rgba8")
    ref = Scene(leaves, "blinn_phong", kd_ref, _f32(flat_normal_map(1)), None)
    quads = quad_cloud(n_quads, seed_for(c, 3))
    kd_lat = 0.3 + 0.1 * _rng(seed_for(c, 4)).uniform(-1.0, 1.0, size=(map_size, map_size, 3))
    lat = Scene(quads, "blinn_phong", _f32(kd_lat), _f32(flat_normal_map(map_size)), None,
                _f32(np.full((map_size, map_size, 1), 0.5)))
    dirs = random_unit(views, seed_for(c, 5))
    light = random_unit(views, seed_for(c, 6))
    return Workload("aggregate", ref, lat, dirs, light, np.ones((views, 3)), res, res, 3.0, 45.0, "l2", 1e-3,
                    ("pos", "kd", "normal", "alpha"), oit_layers=layers)


def workload_batched(n_meshes: int = 64, tris=(1000, 50000), views=(4, 16), res_choices=(256, 512, 1024),
                     map_sizes=(512, 1024, 2048), max_ref_nu: int = 192, progress=None) -> list:
    """Batched meshes of uneven size: per mesh a latent of T triangles
    (log-uniform in ``tris``, a geodesic sphere of frequency round(sqrt(T/20))
    resampled on its own fbm surface), a reference at four times the
    frequency (at most ``max_ref_nu``), 4-16 views at one resolution out of
    ``res_choices``, and maps of one size out of ``map_sizes``: a fixed RGBA8
    base colour shared with the reference, FP32 normal (flat) and ORM
    (constant) maps optimised with the positions under GGX; L1 loss.  Maps of
    one size are shared between meshes."""
    c = 9
    g = _rng(seed_for(c, 0))
    shared = {}

    def ref_maps(S):
        if S not in shared:
            shared[S] = (Texture(to_rgba8(value_noise_map(S, 3, seed_for(c, 10 + S))), "rgba8"),
                         _f32(detail_normal_map(S, seed_for(c, 20 + S))), _f32(orm_map(S, seed_for(c, 30 + S))))
        return shared[S]

    out = []
    for k in range(n_meshes):
        T = math.exp(g.uniform(math.log(tris[0]), math.log(tris[1])))
        nu = max(3, int(round(math.sqrt(T / 20.0))))
        nu_ref = min(4 * nu, max_ref_nu)
        B = int(g.integers(views[0], views[1] + 1))
        res = int(res_choices[int(g.integers(0, len(res_choices)))])
        S = int(map_sizes[int(g.integers(0, len(map_sizes)))])
        rad = lambda d, k=k: fbm_radius(d, seed_for(c, 100 + k))
        kd, nm, orm = ref_maps(S)
        ref = Scene(sphere_mesh(nu_ref, rad), "ggx", kd, nm, orm)
        lat = Scene(sphere_mesh(nu, rad), "ggx", kd, _f32(flat_normal_map(S)),
                    _f32(np.broadcast_to(np.array([0.0, 0.5, 0.0]), (S, S, 3))))
        dirs = random_unit(B, seed_for(c, 200 + k))
        light = random_unit(B, seed_for(c, 300 + k))
        out.append(Workload(f"batched_{k}", ref, lat, dirs, light, np.ones((B, 3)), res, res, 3.0, 45.0, "l1", 1e-3,
                            ("pos", "normal", "orm")))
        if progress is not None:
            progress(k, out[-1])
    return out


def scaled(w: Workload, views: int | None = None, res: int | None = None) -> Workload:
    """Same scene with fewer views and/or another resolution (test sizes)."""
    out = dataclasses.replace(w)
    if views is not None:
        out.dirs = w.dirs[:views]
        out.light_dir = w.light_dir[:views]
        out.light_rgb = w.light_rgb[:views]
    if res is not None:
        out.width = out.height = res
    return out
