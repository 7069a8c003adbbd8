"""The C-ABI library loads, exports every symbol include/adr.h declares, and
its host-only helpers agree with the oracle (no device work here)."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import render as R
from paper_2104_03989_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "adr.h")).read()
    return sorted(set(re.findall(r"\b(adr_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2104_03989_amd import adr
    lib = ctypes.CDLL(adr.LIB_PATH)
    names = _declared()
    assert len(names) >= 11
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(adr.EXPORTS)


def _param_counts():
    src = open(os.path.join(ROOT, "include", "adr.h")).read()
    out = {}
    for m in re.finditer(r"\b(adr_[a-z_0-9]+)\s*\(([^)]*)\)\s*;", src):
        params = m.group(2).strip()
        out[m.group(1)] = 0 if params in ("", "void") else params.count(",") + 1
    return out


def test_binding_declares_every_signature():
    # ctypes passes an undeclared argument as a 32-bit int, which cuts a
    # 64-bit device pointer: every entry point needs its argtypes
    from paper_2104_03989_amd import adr
    counts = _param_counts()
    assert set(counts) == set(adr.EXPORTS)
    for n, k in counts.items():
        f = getattr(adr._lib, n)
        if k == 0:
            continue
        assert f.argtypes is not None, n
        assert len(f.argtypes) == k, (n, len(f.argtypes), k)


@pytest.mark.parametrize("nu", [1, 3, 8])
def test_adjacency_matches_oracle(nu):
    from paper_2104_03989_amd import adr
    _, tri = synth.geodesic_sphere(nu)
    assert np.array_equal(adr.mesh_adjacency(tri), R.adjacency(tri))


def test_adjacency_boundary_and_nonmanifold():
    from paper_2104_03989_amd import adr
    tri = np.array([(0, 1, 2), (2, 1, 3), (1, 2, 4), (5, 6, 7)], dtype=np.int32)
    assert np.array_equal(adr.mesh_adjacency(tri), R.adjacency(tri))
    assert adr.mesh_adjacency(np.zeros((0, 3), np.int32)).shape == (0, 3)


def test_views_build_matches_oracle_cameras():
    from paper_2104_03989_amd import adr
    dirs = synth.random_unit(16, 5)
    dirs[3] = (0.0, 1.0, 0.0)          # straight down the up axis
    dirs[4] = (0.0, -0.9999, 0.0141)
    for W, H in ((256, 256), (512, 384)):
        mvp, eye = adr.views_build(dirs, 3.0, 45.0, W, H)
        m2, e2 = R.look_at_mvp(dirs, 3.0, 45.0, W, H)
        assert np.abs(mvp.reshape(-1, 4, 4) - m2).max() < 1e-6
        assert np.abs(eye - e2).max() < 1e-6


def test_invalid_arguments_are_rejected():
    from paper_2104_03989_amd import adr
    with pytest.raises(adr.AdrError) as e:
        adr.views_build(np.zeros((1, 3)), 3.0, 45.0, 64, 64)
    assert e.value.code == adr.E_INVALID
    with pytest.raises(adr.AdrError):
        adr.views_build(np.ones((1, 3)), -1.0, 45.0, 64, 64)


def test_splitmix64_reference_values():
    # the first outputs of SplitMix64 seeded with 0, as published with the
    # generator (Vigna's splitmix64.c test vector)
    from oracle import sampling as Sm
    outs = [Sm.splitmix64_output((0 + (i + 1) * Sm.GAMMA) & Sm.M64) for i in range(3)]
    assert outs == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


@pytest.mark.parametrize("per_view", [True, False])
def test_job_views_match_oracle_sampler(per_view):
    from oracle import sampling as Sm
    from paper_2104_03989_amd import adr
    for seed, step, B in ((0, 0, 3), (12345, 7, 8), (2**63 + 5, 1999, 4)):
        d, l = adr.job_views(seed, step, B, per_view)
        d2, l2 = Sm.step_views(seed, step, B, per_view)
        assert np.abs(d - np.array(d2)).max() < 1e-6
        assert np.abs(l - np.array(l2)).max() < 1e-6
        assert np.abs(np.linalg.norm(d, axis=1) - 1).max() < 1e-6
