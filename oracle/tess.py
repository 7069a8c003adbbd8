"""ORACLE -- test infrastructure only.

Displacement mapping on a tessellated base mesh (Sec. 5.1, "Displacement
mapping", Eq. 3): edge-midpoint subdivision (each triangle into four,
applied `levels` times, topology fixed), tessellated positions recomputed
from the base mesh every step and displaced along the interpolated smooth
normal by a scalar texture lookup: v_d = v + tex2d(t) n.

Readings: the tessellated vertex is the flat barycentric combination of its
base triangle's corners (midpoint subdivision without smoothing); n is the
normalised barycentric combination of the base mesh's smooth vertex
normals; tex2d is a bilinear level-0 lookup (wrap u, clamp v) at the vertex's
UV in the lowest-index base triangle containing it.  Numbering: base
vertices; then per base edge (a < b, lexicographic) its n-1 interior points
from a to b; then per base triangle its interior lattice points
c0 + (i/n)(c1-c0) + (j/n)(c2-c0), i, j >= 1, i + j <= n-1, i then j (n =
2^levels).  Triangles per base triangle: "up" (i,j),(i+1,j),(i,j+1) for
i+j < n, then "down" (i+1,j),(i+1,j+1),(i,j+1) for i+j < n-1, i then j.
UVs: per base triangle its lattice points (i then j).  UVs are stored as
float32 like every mesh UV: the float64 combination of float32 corner UVs
with dyadic weights is exact and is rounded once.  Displaced positions are
computed in float64 here; the render loop rounds them to float32, the
renderer's vertex format.
"""
from __future__ import annotations

import numpy as np
import torch

from . import render as R


def build(tri: np.ndarray, uv_tri: np.ndarray, uv: np.ndarray, n_pos: int, levels: int):
    """Returns dict(vidx [Vt,3], w [Vt,3], duv [Vt,2], tri [Tt,3], uv [Ut,2], uv_tri [Tt,3])."""
    tri = np.asarray(tri, dtype=np.int64)
    uv_tri = np.asarray(uv_tri, dtype=np.int64)
    uv = np.asarray(uv, dtype=np.float64)
    n = 2 ** levels
    edges = sorted({(min(a, b), max(a, b)) for t in tri for a, b in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0]))})
    eid = {e: k for k, e in enumerate(edges)}
    E = len(edges)
    per_face = (n - 1) * (n - 2) // 2
    npf = (n + 1) * (n + 2) // 2
    V = n_pos + E * (n - 1) + len(tri) * per_face
    vidx = -np.ones((V, 3), dtype=np.int64)
    w = np.zeros((V, 3))
    duv = np.zeros((V, 2))
    seen = np.zeros(V, dtype=bool)
    out_tri, out_uvt = [], []
    out_uv = np.zeros((len(tri) * npf, 2))
    lattice = [(i, j) for i in range(n + 1) for j in range(n + 1 - i)]
    local = {ij: k for k, ij in enumerate(lattice)}
    interior = [(i, j) for i in range(1, n - 1) for j in range(1, n - i)]
    interior_idx = {ij: k for k, ij in enumerate(interior)}
    for t, (c0, c1, c2) in enumerate(tri):
        u0, u1, u2 = uv[uv_tri[t]]
        lat = {}
        for (i, j) in lattice:
            a, b = i / n, j / n
            corners = {(0, 0): c0, (n, 0): c1, (0, n): c2}
            if (i, j) in corners:
                c = corners[(i, j)]
                vid, vi, vw = c, (c, c, c), (1.0, 0.0, 0.0)
            elif j == 0 or i == 0 or i + j == n:
                if j == 0:
                    p, q, k = c0, c1, i
                elif i == 0:
                    p, q, k = c0, c2, j
                else:
                    p, q, k = c1, c2, j
                lo, hi = min(p, q), max(p, q)
                k = k if p == lo else n - k
                vid = n_pos + eid[(lo, hi)] * (n - 1) + (k - 1)
                vi, vw = (lo, hi, hi), (1.0 - k / n, k / n, 0.0)
            else:
                vid = n_pos + E * (n - 1) + t * per_face + interior_idx[(i, j)]
                vi, vw = (c0, c1, c2), (1.0 - a - b, a, b)
            lat[(i, j)] = vid
            uvp = (1.0 - a - b) * u0 + a * u1 + b * u2
            out_uv[t * npf + local[(i, j)]] = uvp
            if not seen[vid]:
                seen[vid] = True
                vidx[vid], w[vid], duv[vid] = vi, vw, uvp
        ups = [((i, j), (i + 1, j), (i, j + 1)) for i in range(n) for j in range(n - i)]
        downs = [((i + 1, j), (i + 1, j + 1), (i, j + 1)) for i in range(n - 1) for j in range(n - 1 - i)]
        for tr in ups + downs:
            out_tri.append([lat[p] for p in tr])
            out_uvt.append([t * npf + local[p] for p in tr])
    return dict(vidx=vidx, w=w, duv=duv.astype(np.float32), tri=np.array(out_tri, dtype=np.int64),
                uv=out_uv.astype(np.float32), uv_tri=np.array(out_uvt, dtype=np.int64))


def displaced_positions(base_pos: torch.Tensor, base_mesh, table: dict, disp0: torch.Tensor):
    """v_d = sum w P + tex2d(duv) normalize(sum w N) (float64, differentiable in
    base_pos and disp0 [S,S,1])."""
    tri = torch.as_tensor(np.asarray(base_mesh.tri, dtype=np.int64))
    N = R.vertex_normals(base_pos, tri)
    vidx = torch.as_tensor(table["vidx"])
    w = torch.as_tensor(table["w"], dtype=R.F64)
    p = (w[:, :, None] * base_pos[vidx]).sum(1)
    m = (w[:, :, None] * N[vidx]).sum(1)
    n = R.safe_normalize(m)
    duv = torch.as_tensor(table["duv"], dtype=R.F64)
    d = R._bilinear(disp0, duv[:, 0], duv[:, 1])
    return p + d * n
