"""Pins of the oracle's dense linear blend skinning (Sec. 5.1, Eq. 2)."""
import math

import numpy as np
import torch

from oracle import skin as S

F64 = torch.float64


def _rot_z(theta, t=(0.0, 0.0, 0.0)):
    c, s = math.cos(theta), math.sin(theta)
    return torch.tensor([[c, -s, 0.0, t[0]], [s, c, 0.0, t[1]], [0.0, 0.0, 1.0, t[2]]], dtype=F64)


def _rot_x(theta):
    c, s = math.cos(theta), math.sin(theta)
    return torch.tensor([[1.0, 0.0, 0.0, 0.0], [0.0, c, -s, 0.0], [0.0, s, c, 0.0]], dtype=F64)


def test_one_hot_weights_are_rigid_motions():
    # one-hot rows: each vertex follows exactly its bone, here a rotation about
    # z by theta_b followed by a translation, written out in closed form
    rng = np.random.default_rng(0)
    V, B = 40, 5
    pos = torch.as_tensor(rng.normal(size=(V, 3)))
    thetas = rng.uniform(-3, 3, B)
    trans = rng.normal(size=(B, 3))
    bones = torch.stack([_rot_z(thetas[b], trans[b]) for b in range(B)])
    owner = rng.integers(0, B, V)
    w = torch.zeros(V, B, dtype=F64)
    w[torch.arange(V), torch.as_tensor(owner)] = 1.0
    out = S.skin(pos, w, bones).numpy()
    p = pos.numpy()
    for i in range(V):
        th, t = thetas[owner[i]], trans[owner[i]]
        x, y, z = p[i]
        exp = (math.cos(th) * x - math.sin(th) * y + t[0], math.sin(th) * x + math.cos(th) * y + t[1], z + t[2])
        np.testing.assert_allclose(out[i], exp, atol=1e-12)
        # a rotation about z keeps the distance to the z axis
        assert abs(math.hypot(out[i][0] - t[0], out[i][1] - t[1]) - math.hypot(x, y)) < 1e-12


def test_partition_of_unity():
    # identity bones with weights summing to one leave the mesh in place;
    # translation-only bones move each vertex by the weighted mean offset
    rng = np.random.default_rng(1)
    V, B = 30, 7
    pos = torch.as_tensor(rng.normal(size=(V, 3)))
    w = torch.as_tensor(rng.uniform(0, 1, (V, B)))
    w = w / w.sum(1, keepdim=True)
    eye = torch.eye(3, 4, dtype=F64).expand(B, 3, 4)
    np.testing.assert_allclose(S.skin(pos, w, eye).numpy(), pos.numpy(), atol=1e-13)
    t = torch.as_tensor(rng.normal(size=(B, 3)))
    bones = eye.clone()
    bones[:, :, 3] = t
    np.testing.assert_allclose(S.skin(pos, w, bones).numpy(), (pos + w @ t).numpy(), atol=1e-13)


def test_equal_bones_give_that_bone():
    # all bones equal to one rotation: any weights summing to one reproduce it
    rng = np.random.default_rng(2)
    V, B = 25, 4
    pos = torch.as_tensor(rng.normal(size=(V, 3)))
    w = torch.as_tensor(rng.uniform(0, 1, (V, B)))
    w = w / w.sum(1, keepdim=True)
    R = _rot_x(0.7)
    out = S.skin(pos, w, R.expand(B, 3, 4)).numpy()
    p = pos.numpy()
    exp = np.stack([p[:, 0], math.cos(0.7) * p[:, 1] - math.sin(0.7) * p[:, 2],
                    math.sin(0.7) * p[:, 1] + math.cos(0.7) * p[:, 2]], 1)
    np.testing.assert_allclose(out, exp, atol=1e-12)


def test_blend_of_two_half_turns():
    # half weight each on the identity and on a half turn about z: x and y
    # cancel, z stays (the known collapse of linear blending)
    pos = torch.tensor([[1.0, 2.0, 3.0], [-4.0, 0.5, -1.0]], dtype=F64)
    bones = torch.stack([_rot_z(0.0), _rot_z(math.pi)])
    w = torch.full((2, 2), 0.5, dtype=F64)
    np.testing.assert_allclose(S.skin(pos, w, bones).numpy(), [[0.0, 0.0, 3.0], [0.0, 0.0, -1.0]], atol=1e-15)


def test_linear_in_the_weights():
    rng = np.random.default_rng(3)
    V, B = 20, 6
    pos = torch.as_tensor(rng.normal(size=(V, 3)))
    bones = torch.as_tensor(rng.normal(size=(B, 3, 4)))
    w1 = torch.as_tensor(rng.normal(size=(V, B)))
    w2 = torch.as_tensor(rng.normal(size=(V, B)))
    lhs = S.skin(pos, 2.5 * w1 - 0.75 * w2, bones)
    rhs = 2.5 * S.skin(pos, w1, bones) - 0.75 * S.skin(pos, w2, bones)
    np.testing.assert_allclose(lhs.numpy(), rhs.numpy(), atol=1e-12)
    # a weight column of zeros switches its bone off
    w1[:, 2] = 0
    bones2 = bones.clone()
    bones2[2] = torch.as_tensor(rng.normal(size=(3, 4)))
    np.testing.assert_allclose(S.skin(pos, w1, bones).numpy(), S.skin(pos, w1, bones2).numpy(), atol=1e-13)


def test_gradients_central_differences():
    rng = np.random.default_rng(4)
    V, B = 12, 5
    pos = torch.tensor(rng.normal(size=(V, 3)), requires_grad=True)
    w = torch.tensor(rng.uniform(0, 1, (V, B)), requires_grad=True)
    bones = torch.as_tensor(rng.normal(size=(B, 3, 4)))
    g_out = torch.as_tensor(rng.normal(size=(V, 3)))

    def f(p, ww):
        return float((S.skin(p, ww, bones) * g_out).sum())

    gp, gw = torch.autograd.grad((S.skin(pos, w, bones) * g_out).sum(), [pos, w])
    h = 1e-6
    for i, j in [(0, 0), (3, 2), (11, 1)]:
        e = torch.zeros(V, 3, dtype=F64)
        e[i, j] = h
        fd = (f(pos.detach() + e, w.detach()) - f(pos.detach() - e, w.detach())) / (2 * h)
        assert abs(fd - float(gp[i, j])) < 1e-7
    for i, b in [(0, 0), (5, 4), (11, 2)]:
        e = torch.zeros(V, B, dtype=F64)
        e[i, b] = h
        fd = (f(pos.detach(), w.detach() + e) - f(pos.detach(), w.detach() - e)) / (2 * h)
        assert abs(fd - float(gw[i, b])) < 1e-7


def test_identity_rig_reduces_to_the_static_step():
    # identity bones with weights summing to one: the skinned render is the
    # static render, the position adjoint is unchanged and every weight of a
    # vertex receives g_i . v_i
    import copy

    from oracle import loop
    from tests import oracle_scenes as OS

    static = OS.tiny_sphere_workload(nu=2, res=24, views=2)
    rigged = OS.rig_workload(copy.deepcopy(static), identity=True)
    ref = loop.reference_image(static)
    np.testing.assert_array_equal(loop.reference_image(rigged).numpy(), ref.numpy())
    l0, g0, o0 = loop.loss_and_grads(static, ref)
    l1, g1, o1 = loop.loss_and_grads(rigged, ref)
    np.testing.assert_array_equal(o1["image"].detach().numpy(), o0["image"].detach().numpy())
    assert float(l1) == float(l0)
    np.testing.assert_allclose(g1["pos"].numpy(), g0["pos"].numpy(), rtol=1e-12, atol=1e-15)
    gv = (g0["pos"] * torch.as_tensor(static.latent.mesh.pos, dtype=F64)).sum(1, keepdim=True)
    np.testing.assert_allclose(g1["weights"].numpy(), gv.expand(-1, rigged.weights.shape[1]).numpy(),
                               rtol=1e-12, atol=1e-15)
    for k in ("kd", "normal"):
        np.testing.assert_array_equal(g1[k].numpy(), g0[k].numpy())


def test_rigged_reference_moves_with_the_frame():
    from oracle import loop
    from tests import oracle_scenes as OS

    w = OS.rig_workload(OS.tiny_sphere_workload(nu=2, res=24, views=1), n_frames=8, frame=0)
    a = loop.reference_image(w)
    w.frame = 3
    b = loop.reference_image(w)
    assert float((a - b).abs().max()) > 0.05
