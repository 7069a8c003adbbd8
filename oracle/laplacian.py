"""ORACLE -- test infrastructure only.

Uniform Laplacian regularizer of the latent mesh (Sec. 5.3, "Objective
function"): the uniformly weighted differential of vertex i is
delta_i = v_i - mean of v_j over its one-ring N_i (vertices sharing an edge
with it); the regularizer is L_delta = (1/n) sum_i |delta_i - delta'_i|^2 with
delta' the differential of the initial mesh (relative) or 0 (absolute); the
objective is L_image + lambda_t L_delta.

Readings: iterations are counted from 0 (as for the learning rate): the
weight used at iteration i is lambda_i, with lambda_0 the initial weight and
lambda_i = (lambda_{i-1} - lambda_min) 10^(-k i) + lambda_min for i >= 1,
k = 1e-6, lambda_min = 0.02 lambda_0, taken literally as printed (a
recursion whose exponent grows with i); the heuristic initial weight is
lambda_0 = 0.25 L_image / L_delta at the start of optimisation.
"""
from __future__ import annotations

import numpy as np
import torch

F64 = torch.float64
K_DECAY = 1e-6
MIN_FRACTION = 0.02
HEURISTIC = 0.25


def one_ring(tri: np.ndarray, n_pos: int) -> list[list[int]]:
    """Sorted neighbour lists: vertices that share an edge with each vertex."""
    ring = [set() for _ in range(n_pos)]
    for a, b, c in np.asarray(tri, dtype=np.int64):
        for p, q in ((a, b), (b, c), (c, a)):
            ring[p].add(int(q))
            ring[q].add(int(p))
    return [sorted(r) for r in ring]


def differentials(pos: torch.Tensor, ring: list[list[int]]) -> torch.Tensor:
    """delta_i = v_i - (1/|N_i|) sum_{j in N_i} v_j (an isolated vertex: 0)."""
    rows = []
    for i, r in enumerate(ring):
        if r:
            rows.append(pos[i] - pos[torch.as_tensor(r)].mean(0))
        else:
            rows.append(torch.zeros(3, dtype=pos.dtype))
    return torch.stack(rows)


def regularizer(pos: torch.Tensor, ring, delta_ref: torch.Tensor | None = None) -> torch.Tensor:
    """L_delta = (1/n) sum_i |delta_i - delta'_i|^2 (delta' = 0 if None)."""
    d = differentials(pos, ring)
    if delta_ref is not None:
        d = d - delta_ref
    return (d * d).sum() / pos.shape[0]


def lambda_schedule(lambda0: float, iterations: int) -> list[float]:
    """Weights lambda_0 .. lambda_{iterations-1} by the recursion."""
    lmin = MIN_FRACTION * lambda0
    out = [lambda0]
    for i in range(1, iterations):
        out.append((out[-1] - lmin) * 10.0 ** (-K_DECAY * i) + lmin)
    return out


def heuristic_lambda0(l_image: float, l_delta: float) -> float:
    return HEURISTIC * l_image / l_delta
