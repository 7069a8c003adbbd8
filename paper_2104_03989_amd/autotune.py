"""Autotuner of the rasterizer's work split (adr_ctx_set_raster).

Per shape bucket (triangle count rounded to a power of two, views,
resolution) and role (reference render or latent render), the forward
render is timed with HIP events for a few candidate splits (largest pixel
bounding box walked by one thread, largest walked by one wave) and the
fastest is kept.  Results are cached in a JSON file keyed by the GPU's
architecture name, the role and the bucket: ADR_AUTOTUNE_CACHE, else
~/.cache/paper_2104_03989_amd/autotune.json.  The split changes only the
speed of the rasterizer, never its output.
"""
from __future__ import annotations

import json
import math
import os

import torch

from . import adr

CANDIDATES = ((16, 1024), (32, 2048), (64, 4096), (128, 4096), (64, 16384))
DEFAULT = (64, 4096)


def cache_path() -> str:
    return os.environ.get("ADR_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_2104_03989_amd", "autotune.json"))


def bucket(n_tri: int, views: int, res: int) -> str:
    return f"t{int(math.log2(max(n_tri, 1)))}_v{views}_r{res}"


class Tuner:
    def __init__(self, path: str | None = None):
        self.path = path or cache_path()
        self.arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
        try:
            with open(self.path) as fh:
                self.cache = json.load(fh)
        except (OSError, ValueError):
            self.cache = {}
        self.dirty = False

    def key(self, role: str, n_tri: int, views: int, res: int) -> str:
        return f"{self.arch}|{role}|{bucket(n_tri, views, res)}"

    def pick(self, ctx: adr.Context, role: str, n_tri: int, views: int, res: int, run, reps: int = 3):
        """The cached split of the bucket, else the fastest candidate for
        ``run()`` (one forward render on the current stream)."""
        k = self.key(role, n_tri, views, res)
        if k in self.cache:
            return tuple(self.cache[k])
        best, best_ms = DEFAULT, float("inf")
        for cand in CANDIDATES:
            ctx.set_raster(*cand)
            run()                                   # warm
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                run()
            b.record()
            b.synchronize()
            ms = a.elapsed_time(b) / reps
            if ms < best_ms:
                best, best_ms = cand, ms
        ctx.set_raster(*DEFAULT)
        self.cache[k] = list(best)
        self.dirty = True
        return best

    def save(self):
        if not self.dirty:
            return
        os.makedirs(os.path.dirname(self.path), exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(self.cache, fh, indent=1, sort_keys=True)
        os.replace(tmp, self.path)
        self.dirty = False
