"""Pins of the oracle's tessellation and displacement (Sec. 5.1, Eq. 3)."""
import numpy as np
import pytest
import torch

from oracle import render as R
from oracle import tess as T
from paper_2104_03989_amd import synth


def _edges(tri):
    return [tuple(sorted((int(t[a]), int(t[b])))) for t in tri for a, b in ((0, 1), (1, 2), (2, 0))]


@pytest.mark.parametrize("nu,levels", [(1, 1), (2, 2), (3, 3)])
def test_counts_and_closed_manifold(nu, levels):
    # A flat midpoint subdivision of a nu-geodesic sphere has the combinatorics
    # of the (nu 2^levels)-geodesic sphere: 10 k^2 + 2 vertices, 20 k^2 faces.
    m = synth.sphere_mesh(nu)
    t = T.build(m.tri, m.uv_tri, m.uv, m.pos.shape[0], levels)
    k = nu * 2 ** levels
    assert t["vidx"].shape[0] == 10 * k * k + 2
    assert t["tri"].shape[0] == 20 * k * k
    # closed, consistently oriented 2-manifold: each directed edge once, each
    # undirected edge twice
    directed = [(int(a[i]), int(a[(i + 1) % 3])) for a in t["tri"] for i in range(3)]
    assert len(set(directed)) == len(directed)
    und, cnt = np.unique(np.array(_edges(t["tri"])), axis=0, return_counts=True)
    assert (cnt == 2).all()
    assert len(und) == 30 * k * k
    # every tessellated vertex is used, with weights on the simplex
    assert set(np.unique(t["tri"])) == set(range(t["vidx"].shape[0]))
    assert (t["w"] >= 0).all() and np.allclose(t["w"].sum(1), 1.0, atol=0)


def _flat_positions(m, t):
    pos = torch.as_tensor(m.pos, dtype=torch.float64)
    zero = torch.zeros(4, 4, 1, dtype=torch.float64)
    return T.displaced_positions(pos, m, t, zero).numpy()


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_subtriangles_tile_their_base_triangle(levels):
    # Without displacement every base triangle is split into 4^levels
    # triangles of equal area and the same orientation.
    m = synth.sphere_mesh(2, lambda d: 1.0 + 0.2 * d[:, 0] * d[:, 1], jitter=0.01, seed=3)
    t = T.build(m.tri, m.uv_tri, m.uv, m.pos.shape[0], levels)
    p = _flat_positions(m, t)
    P = m.pos.astype(np.float64)
    base_n = np.cross(P[m.tri[:, 1]] - P[m.tri[:, 0]], P[m.tri[:, 2]] - P[m.tri[:, 0]])
    sub_n = np.cross(p[t["tri"][:, 1]] - p[t["tri"][:, 0]], p[t["tri"][:, 2]] - p[t["tri"][:, 0]])
    per = 4 ** levels
    owner = np.repeat(np.arange(len(m.tri)), per)
    np.testing.assert_allclose(sub_n * per, base_n[owner], rtol=1e-12, atol=1e-14)


def _as_sets(m, t):
    p = _flat_positions(m, t)
    key = lambda x: tuple(np.round(x, 9))
    verts = {key(v) for v in p}
    tris = set()
    for a in t["tri"]:
        c = [key(p[i]) for i in a]
        r = min(range(3), key=lambda i: c[i])    # rotation-invariant, winding kept
        tris.add(tuple(c[r:] + c[:r]))
    return verts, tris


def test_two_levels_equal_one_level_applied_twice():
    m = synth.sphere_mesh(2, lambda d: 1.0 + 0.1 * d[:, 2], jitter=0.02, seed=5)
    t2 = T.build(m.tri, m.uv_tri, m.uv, m.pos.shape[0], 2)
    t1 = T.build(m.tri, m.uv_tri, m.uv, m.pos.shape[0], 1)
    p1 = _flat_positions(m, t1)
    m1 = synth.Mesh(p1, t1["tri"], t1["uv"], t1["uv_tri"])
    t11 = T.build(m1.tri, m1.uv_tri, m1.uv, p1.shape[0], 1)
    assert _as_sets(m, t2) == _as_sets(m1, t11)
    # the UVs of the lattice points agree too
    uv2 = {tuple(np.round(u, 6)) for u in t2["uv"]}
    uv11 = {tuple(np.round(u, 6)) for u in t11["uv"]}
    assert uv2 == uv11


def _plane(lo=0.2, hi=0.8):
    # a square in z = 0, counter-clockwise seen from +z, uv = (x, y)
    pos = np.array([[lo, lo, 0], [hi, lo, 0], [hi, hi, 0], [lo, hi, 0]], np.float32)
    tri = np.array([[0, 1, 2], [0, 2, 3]], np.int32)
    uv = pos[:, :2].copy()
    return synth.Mesh(pos, tri, uv, tri.copy())


@pytest.mark.parametrize("axis", [0, 1])
def test_linear_displacement_of_a_plane_is_exact(axis):
    # Smooth normals of a flat counter-clockwise mesh are +z; bilinear lookup
    # reproduces a map linear in u (or v) exactly inside the texel-centre
    # range, so v_d = (x, y, a * uv[axis] + c).
    S, a, c = 16, 0.3, -0.05
    centres = (np.arange(S) + 0.5) / S
    ramp = a * centres + c
    tex = np.zeros((S, S, 1))
    if axis == 0:
        tex[:, :, 0] = ramp[None, :]      # rows are v, columns are u
    else:
        tex[:, :, 0] = ramp[:, None]
    m = _plane()
    t = T.build(m.tri, m.uv_tri, m.uv, 4, 3)
    vd = T.displaced_positions(torch.as_tensor(m.pos, dtype=torch.float64), m, t,
                               torch.as_tensor(tex)).numpy()
    flat = _flat_positions(m, t)
    np.testing.assert_allclose(vd[:, :2], flat[:, :2], atol=1e-15)
    np.testing.assert_allclose(vd[:, 2], a * t["duv"][:, axis].astype(np.float64) + c, atol=1e-12)
    # duv is the point's own (u, v) = (x, y) to float32 rounding
    np.testing.assert_allclose(t["duv"], flat[:, :2], atol=1e-7)


def test_constant_displacement_moves_each_vertex_by_that_distance_outwards():
    m = synth.sphere_mesh(3, lambda d: 1.0 + 0.15 * d[:, 0] ** 2, seed=2)
    t = T.build(m.tri, m.uv_tri, m.uv, m.pos.shape[0], 2)
    c = 0.07
    pos = torch.as_tensor(m.pos, dtype=torch.float64)
    vd = T.displaced_positions(pos, m, t, torch.full((8, 8, 1), c, dtype=torch.float64)).numpy()
    flat = _flat_positions(m, t)
    dv = vd - flat
    np.testing.assert_allclose(np.linalg.norm(dv, axis=1), c, rtol=1e-12)
    assert (np.einsum("ij,ij->i", dv, flat) > 0).all()   # along the outward normals
    # at base vertices the direction is the smooth vertex normal itself
    n = R.vertex_normals(pos, torch.as_tensor(m.tri.astype(np.int64))).numpy()
    np.testing.assert_allclose(dv[:m.pos.shape[0]], c * n, atol=1e-13)
