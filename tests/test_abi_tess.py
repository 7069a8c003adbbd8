"""The library's host tessellation builder (Sec. 5.1): tables identical to
the oracle's independent builder, and bad input rejected."""
import numpy as np
import pytest

from oracle import tess as T
from paper_2104_03989_amd import synth


@pytest.mark.parametrize("nu,levels", [(3, 0), (3, 1), (4, 2), (7, 3)])
def test_library_builder_matches_oracle(nu, levels):
    from paper_2104_03989_amd import adr
    m = synth.sphere_mesh(nu)
    o = T.build(m.tri, m.uv_tri, m.uv, m.pos.shape[0], levels)
    g = adr.tess_build(m.tri, m.uv_tri, m.uv, m.pos.shape[0], levels)
    for k in ("vidx", "w", "duv", "tri", "uv", "uv_tri"):
        assert o[k].shape == g[k].shape, k
        assert np.array_equal(o[k], g[k]), k


def test_library_builder_rejects_bad_input():
    from paper_2104_03989_amd import adr
    m = synth.sphere_mesh(2)
    with pytest.raises(adr.AdrError):
        adr.tess_build(m.tri, m.uv_tri, m.uv, m.pos.shape[0], 7)
    bad = m.uv_tri.copy()
    bad[3, 2] = m.uv.shape[0]
    with pytest.raises(adr.AdrError):
        adr.tess_build(m.tri, bad, m.uv, m.pos.shape[0], 1)
    bad = m.tri.copy()
    bad[0, 0] = -1
    with pytest.raises(adr.AdrError):
        adr.tess_build(bad, m.uv_tri, m.uv, m.pos.shape[0], 1)
