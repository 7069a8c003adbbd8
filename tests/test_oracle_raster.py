"""Pins of the oracle's visibility (integer rules R1-R6 of oracle/raster.c)
against brute force, watertightness and closed-form camera geometry."""
import math

import numpy as np
import pytest

from oracle import render as R


def _clip_mesh(xy, z=0.5):
    """Vertices given directly in NDC (identity MVP, w = 1)."""
    xy = np.asarray(xy, dtype=np.float64)
    pos = np.concatenate([xy, np.full((xy.shape[0], 1), z)], axis=1).astype(np.float32)
    return pos, np.eye(4, dtype=np.float32)


def _pix_center(i, n):
    return 2.0 * (i + 0.5) / n - 1.0


@pytest.mark.parametrize("seed", range(6))
def test_bbox_walk_equals_brute_force(seed):
    g = np.random.default_rng(seed)
    W, H = [(8, 8), (16, 12), (32, 32), (13, 7), (32, 16), (20, 20)][seed]
    V, T = 24, 30
    xy = g.uniform(-1.3, 1.3, size=(V, 2))
    # some vertices exactly on pixel centres
    for v in range(0, V, 3):
        xy[v, 0] = _pix_center(g.integers(0, W), W)
        xy[v, 1] = _pix_center(g.integers(0, H), H)
    pos = np.concatenate([xy, g.uniform(-0.9, 0.9, size=(V, 1))], axis=1).astype(np.float32)
    tri = g.integers(0, V, size=(T, 3)).astype(np.int32)
    sv = R.snap(pos, np.eye(4, dtype=np.float32), W, H)
    k1, c1, o1 = R.raster(tri, sv, W, H, brute=False)
    k2, c2, o2 = R.raster(tri, sv, W, H, brute=True)
    assert np.array_equal(k1, k2)
    assert np.array_equal(c1, c2)
    assert np.array_equal(o1, o2)
    assert c1.sum() > 0


def _grid_mesh(n, W, H, on_centers):
    # (n+1)^2 vertices covering [-1.5,1.5]^2 (beyond the screen), 2 n^2 tris
    if on_centers:
        xs = np.array([_pix_center(int(round(i * (W - 1) / n)), W) for i in range(n + 1)])
        ys = np.array([_pix_center(int(round(i * (H - 1) / n)), H) for i in range(n + 1)])
        xs[0], xs[-1], ys[0], ys[-1] = -1.5, 1.5, -1.5, 1.5
    else:
        xs = np.linspace(-1.5, 1.5, n + 1)
        ys = np.linspace(-1.5, 1.5, n + 1) + 0.013
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    xy = np.stack([X.reshape(-1), Y.reshape(-1)], axis=1)
    tri = []
    for j in range(n):
        for i in range(n):
            a = j * (n + 1) + i
            b, c, d = a + 1, a + n + 1, a + n + 2
            tri += [(a, b, d), (a, d, c)] if (i + j) % 2 == 0 else [(a, b, c), (b, d, c)]
    return xy, np.array(tri, dtype=np.int32)


@pytest.mark.parametrize("n,on_centers", [(1, False), (5, False), (7, True), (16, True)])
def test_watertight_every_pixel_covered_once(n, on_centers):
    W, H = 32, 24
    xy, tri = _grid_mesh(n, W, H, on_centers)
    pos, mvp = _clip_mesh(xy)
    sv = R.snap(pos, mvp, W, H)
    keys, cov, _ = R.raster(tri, sv, W, H)
    assert (cov == 1).all()
    assert (R.key_tri(keys) > 0).all()


def test_fan_around_pixel_center_is_watertight():
    W = H = 16
    c = (_pix_center(7, W), _pix_center(9, H))
    ring = [(c[0] + 2.5 * math.cos(a), c[1] + 2.5 * math.sin(a)) for a in np.linspace(0, 2 * math.pi, 13)[:-1]]
    xy = np.array([c] + ring)
    tri = np.array([(0, 1 + k, 1 + (k + 1) % 12) for k in range(12)], dtype=np.int32)
    pos, mvp = _clip_mesh(xy)
    keys, cov, _ = R.raster(tri, R.snap(pos, mvp, W, H), W, H)
    assert (cov == 1).all()


def test_equal_depth_goes_to_lower_index_and_nearer_wins():
    W = H = 16
    xy = np.array([(-1.2, -1.2), (1.3, -1.1), (-1.1, 1.4)])
    pos, mvp = _clip_mesh(np.concatenate([xy, xy]))
    tri = np.array([(0, 1, 2), (3, 4, 5)], dtype=np.int32)
    keys, cov, _ = R.raster(tri, R.snap(pos, mvp, W, H), W, H)
    ids = R.key_tri(keys)
    assert set(np.unique(ids[cov > 0])) == {1}
    assert (cov[cov > 0] == 2).all()
    # second copy nearer (smaller z): it wins wherever both cover
    pos2 = pos.copy()
    pos2[3:, 2] = 0.1
    keys, cov, _ = R.raster(tri, R.snap(pos2, mvp, W, H), W, H)
    assert set(np.unique(R.key_tri(keys)[cov > 0])) == {2}


def test_depth_plane_is_the_snapped_depth_interpolant():
    # a tilted plane z = 0.3 x + 0.2 y: stored depth within 1 unit of
    # (z/w 0.5 + 0.5) 2^24 at every covered pixel centre
    W = H = 32
    xy = np.array([(-1.5, -1.5), (1.5, -1.5), (-1.5, 1.5), (1.5, 1.5)])
    z = 0.3 * xy[:, 0] + 0.2 * xy[:, 1]
    pos = np.concatenate([xy, z[:, None]], axis=1).astype(np.float32)
    tri = np.array([(0, 1, 3), (0, 3, 2)], dtype=np.int32)
    keys, cov, _ = R.raster(tri, R.snap(pos, np.eye(4, dtype=np.float32), W, H), W, H)
    d = (keys >> np.uint64(32)).astype(np.float64)
    jj, ii = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    px, py = _pix_center(ii, W), _pix_center(jj, H)
    expect = ((0.3 * px + 0.2 * py) * 0.5 + 0.5) * 2 ** 24
    assert np.abs(d - expect).max() <= 2.0


def test_snap_of_pixel_centres_and_screen_centre():
    W, H = 64, 32
    pts = np.array([(_pix_center(5, W), _pix_center(7, H)), (0.0, 0.0), (-1.0, -1.0), (1.0, 1.0)])
    pos, mvp = _clip_mesh(pts, z=0.0)
    sv = R.snap(pos, mvp, W, H)
    assert tuple(sv[0, :2]) == (256 * 5 + 128, 256 * 7 + 128)
    assert tuple(sv[1, :2]) == (W * 128, H * 128)
    assert tuple(sv[2, :2]) == (0, 0)
    assert tuple(sv[3, :2]) == (W * 256, H * 256)
    assert sv[1, 2] == 2 ** 23
    assert (sv[:, 3] == 1).all()


def test_unusable_vertices_drop_triangles():
    W = H = 8
    pos = np.array([(-0.5, -0.5, 0.0), (0.5, -0.5, 0.0), (9.5, 0.5, 0.0)], dtype=np.float32)
    sv = R.snap(pos, np.eye(4, dtype=np.float32), W, H)
    assert sv[2, 3] == 0
    keys, cov, orient = R.raster(np.array([(0, 1, 2)], dtype=np.int32), sv, W, H)
    assert cov.sum() == 0 and orient[0] == 0


def test_orientation_and_no_culling():
    W = H = 8
    xy = np.array([(-0.9, -0.9), (0.9, -0.9), (-0.9, 0.9)])
    pos, mvp = _clip_mesh(xy)
    sv = R.snap(pos, mvp, W, H)
    k1, c1, o1 = R.raster(np.array([(0, 1, 2)], dtype=np.int32), sv, W, H)
    k2, c2, o2 = R.raster(np.array([(0, 2, 1)], dtype=np.int32), sv, W, H)
    assert o1[0] == 1 and o2[0] == -1
    assert np.array_equal(c1, c2) and c1.sum() > 0


def test_look_at_closed_form():
    d = np.array([[0.3, 0.5, -0.8]])
    W, H = 64, 48
    mvp, eye = R.look_at_mvp(d, 3.0, 45.0, W, H)
    M = mvp[0]
    o = M @ np.array([0, 0, 0, 1.0])
    assert abs(o[0] / o[3]) < 1e-12 and abs(o[1] / o[3]) < 1e-12
    assert abs(o[3] - 3.0) < 1e-12  # w = distance along the view axis
    assert np.allclose(eye[0], 3.0 * d[0] / np.linalg.norm(d[0]))
    # a point 22.5 degrees above the axis (in the camera's up plane) lands on y_ndc = 1
    f = -eye[0] / 3.0
    up = np.array([0, 1.0, 0])
    s = np.cross(f, up); s /= np.linalg.norm(s)
    u = np.cross(s, f)
    p = eye[0] + 2.0 * (f + math.tan(math.radians(22.5)) * u)
    c = M @ np.append(p, 1.0)
    assert abs(c[1] / c[3] - 1.0) < 1e-12
    # horizontal: aspect W/H
    p = eye[0] + 2.0 * (f + math.tan(math.radians(22.5)) * (W / H) * s)
    c = M @ np.append(p, 1.0)
    assert abs(c[0] / c[3] - 1.0) < 1e-12
    # near and far planes map to z_ndc = -1 and +1
    for dist, zn in ((0.1, -1.0), (10.0, 1.0)):
        c = M @ np.append(eye[0] + dist * f, 1.0)
        assert abs(c[2] / c[3] - zn) < 1e-9


def test_clip32_close_to_float64():
    g = np.random.default_rng(3)
    pos = g.normal(size=(50, 3)).astype(np.float32)
    mvp, _ = R.look_at_mvp(np.array([[0.2, 0.1, 0.9]]), 3.0, 45.0, 32, 32)
    m32 = mvp[0].astype(np.float32)
    c32 = R.clip32(pos, m32)
    c64 = np.concatenate([pos.astype(np.float64), np.ones((50, 1))], 1) @ m32.astype(np.float64).T
    assert np.abs(c32 - c64).max() < 1e-5


def test_adjacency_of_closed_sphere():
    from paper_2104_03989_amd import synth
    _, tri = synth.geodesic_sphere(3)
    adj = R.adjacency(tri)
    assert (adj >= 0).all()
    for t in range(tri.shape[0]):
        for k in range(3):
            n = adj[t, k]
            edge = {tri[t, (k + 1) % 3], tri[t, (k + 2) % 3]}
            assert edge <= set(tri[n].tolist())
            assert t in adj[n]
