"""Pins of the oracle's uniform Laplacian regularizer and its weight
schedule (Sec. 5.3, "Objective function")."""
import math

import numpy as np
import pytest
import torch

from oracle import laplacian as L
from paper_2104_03989_amd import synth


def test_icosahedron_closed_form():
    # Each vertex of the unit icosahedron has five neighbours at polar angle
    # theta with cos(theta) = 1/sqrt(5); their mean is v/sqrt(5), so
    # delta = (1 - 1/sqrt(5)) v and the absolute regularizer is its square.
    dirs, tri = synth.geodesic_sphere(1)
    ring = L.one_ring(tri, dirs.shape[0])
    assert all(len(r) == 5 for r in ring)
    pos = torch.as_tensor(dirs, dtype=torch.float64)
    d = L.differentials(pos, ring).numpy()
    np.testing.assert_allclose(d, (1 - 1 / math.sqrt(5)) * dirs, atol=1e-12)
    assert abs(float(L.regularizer(pos, ring)) - (1 - 1 / math.sqrt(5)) ** 2) < 1e-12


@pytest.mark.parametrize("nu", [2, 5])
def test_one_ring_of_a_closed_sphere(nu):
    dirs, tri = synth.geodesic_sphere(nu)
    ring = L.one_ring(tri, dirs.shape[0])
    counts = np.array([len(r) for r in ring])
    assert (counts == 5).sum() == 12 and (counts == 6).sum() == dirs.shape[0] - 12
    assert counts.sum() == 3 * tri.shape[0]            # 2 E = 3 T on a closed mesh
    for i, r in enumerate(ring):
        assert i not in r and all(i in ring[j] for j in r)


def test_planar_grid_interior_is_flat():
    # a regular triangulated grid in a plane: every interior vertex is the
    # mean of its six neighbours
    n = 6
    xs, ys = np.meshgrid(np.arange(n, dtype=np.float64), np.arange(n, dtype=np.float64))
    pos = np.stack([xs.ravel() + 0.5 * ys.ravel(), ys.ravel() * math.sqrt(3) / 2, np.zeros(n * n)], 1)
    tri = []
    for j in range(n - 1):
        for i in range(n - 1):
            a, b, c, d = j * n + i, j * n + i + 1, (j + 1) * n + i, (j + 1) * n + i + 1
            tri += [(a, b, c), (b, d, c)]
    ring = L.one_ring(np.array(tri), n * n)
    d = L.differentials(torch.as_tensor(pos), ring).numpy()
    interior = [j * n + i for j in range(1, n - 1) for i in range(1, n - 1)]
    assert np.abs(d[interior]).max() < 1e-12
    assert np.abs(d[0]).max() > 0.1                      # a corner is not flat


def test_invariances_and_relative_mode():
    m = synth.sphere_mesh(4, lambda d: synth.sh_radius(d, 5), jitter=0.02, seed=1)
    ring = L.one_ring(m.tri, m.pos.shape[0])
    pos = torch.as_tensor(m.pos, dtype=torch.float64)
    base = float(L.regularizer(pos, ring))
    shifted = float(L.regularizer(pos + torch.tensor([0.3, -2.0, 5.0], dtype=torch.float64), ring))
    assert abs(shifted - base) < 1e-12 * max(1.0, base)
    q, _ = np.linalg.qr(np.random.default_rng(0).normal(size=(3, 3)))
    rotated = float(L.regularizer(pos @ torch.as_tensor(q), ring))
    assert abs(rotated - base) < 1e-12
    assert abs(float(L.regularizer(2 * pos, ring)) - 4 * base) < 1e-12
    ref = L.differentials(pos, ring)
    p = pos.clone().requires_grad_(True)
    r = L.regularizer(p, ring, ref)
    (g,) = torch.autograd.grad(r, [p])
    assert float(r.detach()) == 0.0 and float(g.abs().max()) == 0.0


def test_gradient_central_differences():
    m = synth.sphere_mesh(3, None, jitter=0.05, seed=2)
    ring = L.one_ring(m.tri, m.pos.shape[0])
    pos = torch.tensor(m.pos, dtype=torch.float64, requires_grad=True)
    ref = L.differentials(torch.as_tensor(synth.sphere_mesh(3).pos, dtype=torch.float64), ring)
    (g,) = torch.autograd.grad(L.regularizer(pos, ring, ref), [pos])
    base = pos.detach()
    h = 1e-6
    for idx in np.random.default_rng(1).integers(0, base.numel(), 20):
        e = torch.zeros_like(base).reshape(-1)
        e[idx] = h
        e = e.reshape(base.shape)
        fd = (float(L.regularizer(base + e, ring, ref)) - float(L.regularizer(base - e, ring, ref))) / (2 * h)
        assert abs(fd - float(g.reshape(-1)[idx])) < 1e-7


def test_lambda_schedule():
    lam = L.lambda_schedule(3.0, 4000)
    lmin = 0.02 * 3.0
    # closed form of the recursion: lambda_i = lmin + (lambda_0 - lmin) 10^(-k i (i+1)/2)
    for i in (0, 1, 10, 999, 2000, 3999):
        exact = lmin + (3.0 - lmin) * 10.0 ** (-1e-6 * i * (i + 1) / 2)
        assert abs(lam[i] - exact) < 1e-12
    assert lam[0] == 3.0 and all(a >= b for a, b in zip(lam, lam[1:]))
    assert abs(lam[3999] - lmin) < 1e-3 * lmin             # reaches lambda_min within ~3k steps
    assert L.heuristic_lambda0(0.2, 0.01) == pytest.approx(5.0)
