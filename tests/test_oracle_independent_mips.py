"""Independent mip levels as latent variables (Sec. 4.2), oracle side:
a chain equal to the box pyramid of its level 0 renders exactly like the
derived chain, and the chain's per-level gradients, pushed down through the
box filter, sum to the derived level-0 gradient."""
import numpy as np
import torch

from oracle import loop as OL
from oracle import render as R
from paper_2104_03989_amd import synth
from tests import oracle_scenes as S


def _with_chain(w, name):
    tex = getattr(w.latent, name)
    lv = R.mip_chain_f32(torch.as_tensor(tex.data, dtype=torch.float64))
    chain = torch.cat([x.reshape(-1, x.shape[2]) for x in lv]).numpy()
    setattr(w.latent, name, synth.Texture(tex.data, "f32", chain))


def test_box_pyramid_chain_equals_derived_and_gradients_fold():
    w = S.tiny_sphere_workload("ggx", nu=3, res=32, views=2, tex=16, loss="l1_tonemap", seed=2)
    w.optimize = ("kd", "normal")
    mvp32, eye = OL.cameras(w)
    ref = OL.reference_image(w, mvp32, eye)
    l_der, g_der, o_der = OL.loss_and_grads(w, ref, mvp32, eye)
    for n in ("kd", "normal"):
        _with_chain(w, n)
    l_ind, g_ind, o_ind = OL.loss_and_grads(w, ref, mvp32, eye)
    assert float(l_ind) == float(l_der)
    assert torch.equal(o_ind["image"], o_der["image"])
    for n in ("kd", "normal"):
        S0 = getattr(w.latent, n).data.shape[0]
        g = g_ind[n]
        sizes = [(S0 >> l) ** 2 for l in range(int(np.log2(S0)) + 1)]
        levels = list(torch.split(g, sizes))
        acc = levels[-1].reshape(1, 1, -1)
        for l in range(len(levels) - 2, -1, -1):
            s = S0 >> l
            up = acc.repeat_interleave(2, 0).repeat_interleave(2, 1) * 0.25
            acc = levels[l].reshape(s, s, -1) + up
        np.testing.assert_allclose(acc.numpy(), g_der[n].numpy(), rtol=1e-10, atol=1e-15)
        assert float(levels[1].abs().max()) > 0          # coarse levels do receive gradient
