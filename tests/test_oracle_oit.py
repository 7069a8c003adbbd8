"""Pins of the oracle's depth-peeled order-independent transparency
(Sec. 5.2, "Order-independent transparency"; Sec. 4.4)."""
import numpy as np
import pytest
import torch

from oracle import loop as OL
from oracle import oit as O
from oracle import render as R
from paper_2104_03989_amd import synth
from tests import oracle_scenes as S

F64 = torch.float64


def _random_triangles(n, seed):
    g = np.random.default_rng(seed)
    pos = g.uniform(-0.8, 0.8, size=(3 * n, 3)).astype(np.float32)
    tri = np.arange(3 * n, dtype=np.int32).reshape(n, 3)
    return pos, tri


def test_layers_are_the_sorted_fragments():
    # the k-th peeled layer of a pixel is its k-th smallest fragment key;
    # fragments come from rasterizing every triangle on its own
    pos, tri = _random_triangles(25, 0)
    W = H = 20
    mvp, _ = R.look_at_mvp(np.array([[0.1, 0.2, 1.0]]), 3.0, 45.0, W, H)
    sv = R.snap(pos, mvp[0].astype(np.float32), W, H)
    frags = [[] for _ in range(W * H)]
    for t in range(tri.shape[0]):
        k, _, _ = R.raster(tri[t:t + 1], sv, W, H)
        k = k.reshape(-1)
        for o in np.nonzero(R.key_tri(k.reshape(H, W)).reshape(-1))[0]:
            frags[o].append((int(k[o]) >> 32 << 32) | (t + 1))
    depth = max(len(f) for f in frags)
    assert depth >= 4
    layers = O.peel(tri, sv, W, H, depth + 1)
    for o in range(W * H):
        fs = sorted(frags[o])
        for k in range(depth + 1):
            got = int(layers[k].reshape(-1)[o])
            exp = fs[k] if k < len(fs) else 0xFFFFFFFF00000000
            assert got == exp, (o, k)
    # brute-force pixel loop agrees with the bounding-box walk
    brute = R.raster_peel(tri, sv, W, H, layers[1], brute=True)
    np.testing.assert_array_equal(brute, layers[2])


def _two_quads(alpha_front, alpha_back, kd_front=(0.8, 0.2, 0.1), kd_back=(0.1, 0.3, 0.9)):
    # two camera-facing quads at z = 0.3 (front, smaller) and z = -0.2 (back)
    front = S.quad_mesh(z=0.3, half=0.5)
    back = S.quad_mesh(z=-0.2, half=0.9)
    mesh = synth.Mesh(np.concatenate([front.pos, back.pos]), np.concatenate([front.tri, back.tri + 4]),
                      np.concatenate([front.uv, back.uv]), np.concatenate([front.uv_tri, back.uv_tri + 4]))
    return front, back, mesh


def _plain(mesh, kd, W, H, mvp, eye, light, aa=False):
    out = R.render(mesh, "blinn_phong", R.texture_levels(S.const_tex(kd).data, "f32"),
                   R.texture_levels(S.flat_normals().data, "f32"), None, torch.as_tensor(mesh.pos, dtype=F64),
                   mvp, eye, light, np.ones((1, 3)), W, H, aa=aa)
    return out["color"][0]


def test_two_quads_over_operator():
    # alpha-blended pair: where both cover, alpha_f c_f + (1 - alpha_f) alpha_b c_b
    # with c_f and c_b the opaque renders of each quad alone
    W = H = 24
    mvp, eye = R.look_at_mvp(np.array([[0.0, 0.0, 1.0]]), 3.0, 45.0, W, H)
    mvp32 = mvp.astype(np.float32)
    light = np.array([[0.2, 0.3, 1.0]]) / np.linalg.norm([0.2, 0.3, 1.0])
    front, back, mesh = _two_quads(0.3, 0.6)
    af, ab = 0.3, 0.6
    # per-quad colour and alpha through one map of 8 x 8 texels: the front
    # quad's UVs lie in u 0.1..0.4, whose bilinear footprints stay in the
    # left four columns, the back quad's in u 0.6..0.9 (right four)
    mesh.uv = mesh.uv.copy()
    mesh.uv[:4, 0] = 0.1 + 0.3 * mesh.uv[:4, 0]
    mesh.uv[4:, 0] = 0.6 + 0.3 * mesh.uv[4:, 0]
    kd = np.zeros((8, 8, 3), np.float32)
    kd[:, :4] = (0.8, 0.2, 0.1)
    kd[:, 4:] = (0.1, 0.3, 0.9)
    al = np.zeros((8, 8, 1), np.float32)
    al[:, :4] = af
    al[:, 4:] = ab
    out = O.render_oit(mesh, "blinn_phong", [torch.as_tensor(kd, dtype=F64)],
                       [torch.as_tensor(np.tile(np.float32([0, 0, 1]), (8, 8, 1)), dtype=F64)], None,
                       [torch.as_tensor(al, dtype=F64)], torch.as_tensor(mesh.pos, dtype=F64), mvp32, eye, light,
                       np.ones((1, 3)), W, H, 3, aa=False)
    img = out["image"][0].numpy()
    cf = _plain(front, (0.8, 0.2, 0.1), W, H, mvp32, eye, light).numpy()
    cb = _plain(back, (0.1, 0.3, 0.9), W, H, mvp32, eye, light).numpy()
    kf = R.raster(front.tri, R.snap(front.pos, mvp32[0], W, H), W, H)[0].reshape(-1)
    kb = R.raster(back.tri, R.snap(back.pos, mvp32[0], W, H), W, H)[0].reshape(-1)
    inf = R.key_tri(kf.reshape(H, W)).reshape(-1) > 0
    inb = R.key_tri(kb.reshape(H, W)).reshape(-1) > 0
    both = inf & inb
    assert both.sum() > 50 and (inb & ~inf).sum() > 50
    np.testing.assert_allclose(img[both], af * cf[both] + (1 - af) * ab * cb[both], atol=1e-12)
    np.testing.assert_allclose(img[inb & ~inf], ab * cb[inb & ~inf], atol=1e-12)
    assert np.abs(img[~inb]).max() == 0.0
    # the third layer is empty: two quads have depth complexity two
    assert np.all(R.key_tri(out["keys"][0][2]) == 0)


@pytest.mark.parametrize("aa", [False, True])
def test_opaque_and_clear_limits(aa):
    w = S.tiny_sphere_workload(nu=2, res=24, views=1, tex=8)
    mvp32, eye = OL.cameras(w)
    s = w.latent
    args = (s.mesh, s.model, R.texture_levels(s.kd.data, "f32"), R.texture_levels(s.normal.data, "f32"), None)
    rest = (torch.as_tensor(s.mesh.pos, dtype=F64), mvp32, eye, w.light_dir, w.light_rgb, w.width, w.height, 4)
    # alpha = 1: only the front layer is seen; without antialiasing that is the opaque colour
    opaque = O.render_oit(*args, R.texture_levels(np.ones((8, 8, 1), np.float32), "f32"), *rest, aa=aa)
    plain = R.render(s.mesh, s.model, args[2], args[3], None, rest[0], mvp32, eye, w.light_dir, w.light_rgb,
                     w.width, w.height, aa=aa)
    if not aa:
        np.testing.assert_allclose(opaque["image"].numpy(), plain["color"].numpy(), atol=1e-14)
    else:
        # pixels no pair of any layer touches equal the opaque render (the
        # back layer's antialiasing spreads into the background next to the
        # shared silhouette, and the front layer passes that through)
        touched = set()
        for P, Q, _, _ in opaque["pairs"][0]:
            touched |= set(P.tolist()) | set(Q.tolist())
        keep = np.array([o not in touched for o in range(w.width * w.height)])
        np.testing.assert_allclose(opaque["image"][0].numpy()[keep], plain["image"][0].numpy()[keep], atol=1e-14)
    # alpha = 0: nothing is seen, antialiasing included
    clear = O.render_oit(*args, R.texture_levels(np.zeros((8, 8, 1), np.float32), "f32"), *rest, aa=aa)
    assert float(clear["image"].abs().max()) == 0.0


def test_more_layers_than_depth_change_nothing():
    w = S.tiny_sphere_workload(nu=2, res=24, views=1, tex=8)
    mvp32, eye = OL.cameras(w)
    s = w.latent
    al = R.texture_levels(np.random.default_rng(0).uniform(0.2, 0.8, (8, 8, 1)).astype(np.float32), "f32")
    def run(L):
        return O.render_oit(s.mesh, s.model, R.texture_levels(s.kd.data, "f32"), R.texture_levels(s.normal.data, "f32"),
                            None, al, torch.as_tensor(s.mesh.pos, dtype=F64), mvp32, eye, w.light_dir, w.light_rgb,
                            w.width, w.height, L)
    a, b = run(2), run(3)
    # a closed sphere has depth complexity two: a third layer is empty
    assert np.all(R.key_tri(b["keys"][0][2]) == 0)
    np.testing.assert_array_equal(a["image"].numpy(), b["image"].numpy())
    # and one layer drops the back face: the images differ
    assert float((run(1)["image"] - a["image"]).abs().max()) > 1e-3


def test_aggregate_gradients_central_differences():
    # loss with the layers and antialiasing pairs held fixed: central
    # differences w.r.t. alpha and base-colour texels and vertex positions
    w = S.aggregate_case()
    ref = OL.reference_image(w)
    mvp32, eye = OL.cameras(w)
    params = OL.latent_params(w)
    out = OL.render_latent(w, mvp32, eye, params)
    loss = R.image_loss(out["image"], ref, w.loss)
    keys = list(params)
    grads = dict(zip(keys, torch.autograd.grad(loss, [params[k] for k in keys])))
    frozen = {"keys": out["keys"], "pairs": out["pairs"]}

    def f(name, idx, h):
        p = {k: v.detach().clone() for k, v in params.items()}
        p[name].view(-1)[idx] += h
        o = OL.render_latent(w, mvp32, eye, p, frozen=frozen)
        return float(R.image_loss(o["image"], ref, w.loss))

    checked = 0
    for name in ("alpha", "kd", "pos"):
        g = grads[name].reshape(-1)
        cand = torch.nonzero(g.abs() > 1e-3 * float(g.abs().max()))[:, 0].numpy()
        for idx in np.random.default_rng(1).choice(cand, size=min(4, cand.size), replace=False):
            h = 1e-6
            fd = (f(name, idx, h) - f(name, idx, -h)) / (2 * h)
            assert abs(fd - float(g[idx])) <= 1e-5 * max(1.0, abs(fd)) + 1e-6 * float(g.abs().max()), (name, idx)
            checked += 1
    assert checked >= 8
