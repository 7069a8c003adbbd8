"""The library's host one-ring builder against the oracle's."""
import numpy as np
import pytest

from oracle import laplacian as L
from paper_2104_03989_amd import synth


@pytest.mark.parametrize("nu", [1, 3, 8])
def test_one_ring_matches_oracle(nu):
    from paper_2104_03989_amd import adr
    m = synth.sphere_mesh(nu)
    offs, nbr = adr.mesh_one_ring(m.tri, m.pos.shape[0])
    ring = L.one_ring(m.tri, m.pos.shape[0])
    assert offs[-1] == sum(len(r) for r in ring)
    for i, r in enumerate(ring):
        assert list(nbr[offs[i]:offs[i + 1]]) == r


def test_one_ring_open_mesh_and_isolated_vertex():
    from paper_2104_03989_amd import adr
    tri = np.array([[0, 1, 2], [2, 1, 3]], np.int32)
    offs, nbr = adr.mesh_one_ring(tri, 5)               # vertex 4 is isolated
    ring = L.one_ring(tri, 5)
    assert [list(nbr[offs[i]:offs[i + 1]]) for i in range(5)] == ring
    assert ring[4] == []


def test_one_ring_rejects_bad_index():
    from paper_2104_03989_amd import adr
    with pytest.raises(adr.AdrError):
        adr.mesh_one_ring(np.array([[0, 1, 7]], np.int32), 3)
