"""ORACLE -- test infrastructure only.

The camera and light draws of a whole-job optimisation (Sec. 3: a random
camera and light per iteration), generated from a counter-based stream so
that any step can be drawn without the ones before it.  Uniforms come from
SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): the i-th output of a stream seeded with s is the
SplitMix64 output function applied to s + (i+1) * 0x9E3779B97F4A7C15 (mod
2^64), and the uniform is its top 53 bits times 2^-53.  Normal deviates come
from the Box-Muller transform (r = sqrt(-2 ln(1-u1)), angle 2 pi u2); a
direction is three of them normalised.
"""
from __future__ import annotations

import math

M64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def splitmix64_output(z: int) -> int:
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def uniform(seed: int, i: int) -> float:
    return (splitmix64_output((seed + (i + 1) * GAMMA) & M64) >> 11) * 2.0 ** -53


def unit_vector(seed: int, base: int):
    g = []
    for k in range(2):
        u1 = 1.0 - uniform(seed, base + 2 * k)
        u2 = uniform(seed, base + 2 * k + 1)
        r = math.sqrt(-2.0 * math.log(u1))
        g += [r * math.cos(2 * math.pi * u2), r * math.sin(2 * math.pi * u2)]
    n = math.sqrt(g[0] ** 2 + g[1] ** 2 + g[2] ** 2)
    return [g[0] / n, g[1] / n, g[2] / n]


def step_views(seed: int, step: int, n_views: int, light_per_view: bool = True):
    """Directions and lights of one step: 8 uniforms per view, indices
    (step n_views + b) 8 + k, k 0..3 direction, 4..7 light."""
    dirs, lights = [], []
    for b in range(n_views):
        base = (step * n_views + b) * 8
        dirs.append(unit_vector(seed, base))
        lb = base + 4 if light_per_view else step * n_views * 8 + 4
        lights.append(unit_vector(seed, lb))
    return dirs, lights
