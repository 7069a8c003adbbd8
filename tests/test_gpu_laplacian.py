"""Parity of the HIP Laplacian regularizer (Sec. 5.3) with the oracle:
differentials, loss and lambda-scaled gradient, absolute and relative, and
the same bits on repeated runs (the adjoint is a gather)."""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import laplacian as L
from paper_2104_03989_amd import synth
from tests.gpu_common import rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2104_03989_amd import adr
    c = adr.Context(0)
    yield c
    c.close()


def _gpu(ctx, m, ref_pos=None, lam=0.7):
    from paper_2104_03989_amd import adr
    ring = adr.DeviceOneRing(m.tri, m.pos.shape[0])
    pos = torch.from_numpy(np.ascontiguousarray(m.pos, np.float32)).cuda()
    dref = None
    if ref_pos is not None:
        dref = torch.zeros_like(pos)
        adr.laplacian(ctx, ring, torch.from_numpy(np.ascontiguousarray(ref_pos, np.float32)).cuda(), delta_out=dref)
    delta = torch.zeros_like(pos)
    loss = torch.zeros(1, device="cuda")
    g = torch.zeros_like(pos)
    adr.laplacian(ctx, ring, pos, dref, lam, delta, loss, g)
    torch.cuda.synchronize()
    return delta.cpu().numpy(), float(loss[0]), g.cpu().numpy()


def _oracle(m, ref_pos=None, lam=0.7):
    ring = L.one_ring(m.tri, m.pos.shape[0])
    p = torch.tensor(m.pos, dtype=torch.float64, requires_grad=True)
    dref = None if ref_pos is None else L.differentials(torch.as_tensor(ref_pos, dtype=torch.float64), ring)
    loss = L.regularizer(p, ring, dref)
    (g,) = torch.autograd.grad(lam * loss, [p])
    return L.differentials(p.detach(), ring).numpy(), float(loss.detach()), g.numpy()


def test_icosahedron(ctx):
    print("laplacian icosahedron", flush=True)
    m = synth.sphere_mesh(1)
    d, loss, _ = _gpu(ctx, m)
    assert abs(loss - (1 - 1 / math.sqrt(5)) ** 2) < 1e-6
    np.testing.assert_allclose(d, (1 - 1 / math.sqrt(5)) * m.pos, atol=1e-6)


@pytest.mark.parametrize("mode", ["absolute", "relative"])
def test_matches_oracle(ctx, mode):
    print("laplacian", mode, flush=True)
    w = synth.workload_paper_loop(map_size=8, ref_nu=4)
    m = synth.sphere_mesh(19, None, jitter=0.01, seed=4)
    ref = w.latent.mesh.pos if mode == "relative" else None
    d, loss, g = _gpu(ctx, m, ref)
    od, oloss, og = _oracle(m, ref)
    assert np.abs(d - od).max() < 1e-6
    assert abs(loss - oloss) <= 1e-5 * oloss
    assert rel_l2(g, og) < 1e-5
    d2, loss2, g2 = _gpu(ctx, m, ref)
    assert np.array_equal(g2, g) and loss2 == loss
