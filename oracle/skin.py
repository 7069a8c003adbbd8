"""ORACLE -- test infrastructure only.

Dense linear blend skinning (Sec. 5.1, "Animation & skinning", Eq. 2): the
skinned position of vertex i is v_i^s = sum_b w_ib M_b v_i, with M_b the
transform of bone b for the current frame and v_i in homogeneous form
(x, y, z, 1).  Every weight w_ib is a variable (the dense operator), and the
bone transforms are constants (Sec. 4.3, "Animation and Skinning").

Readings: M_b is affine, given by its top three rows (a 3x4 matrix); the
weights are used as they are, with no normalisation or clamping, since the
equation applies none; the smooth normals and tangents of the skinned mesh are
derived from the skinned positions, as for any other deforming mesh
(Sec. 5.1, "Tangent space").
"""
from __future__ import annotations

import torch

F64 = torch.float64


def homogeneous(pos: torch.Tensor) -> torch.Tensor:
    return torch.cat([pos, torch.ones(pos.shape[0], 1, dtype=pos.dtype)], 1)


def skin(pos: torch.Tensor, weights: torch.Tensor, bones: torch.Tensor) -> torch.Tensor:
    """Eq. 2.  pos [V,3], weights [V,B], bones [B,3,4] -> skinned positions [V,3].

    Each bone moves every vertex (M_b v_i), and the moved copies are summed
    with the vertex's weights."""
    moved = torch.einsum("bjk,ik->bij", bones, homogeneous(pos))     # [B,V,3]: M_b v_i
    return torch.einsum("ib,bij->ij", weights, moved)
