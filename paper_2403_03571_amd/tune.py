"""Autotuning cache: the fastest exact kernel per problem class.

A problem class is (device architecture, dim, N bucket, pixel-count bucket,
tier); buckets are powers of two.  The first call for a class runs the
library's apd_autotune (which times every exact kernel of the tier, with its
tile shapes, on the given problem and keeps the fastest) and stores the
choice in a JSON file; later calls set the context from the file.
"""
from __future__ import annotations

import json
import math
import os

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "apd_tune.json")


def problem_class(prob, prec: str, arch: str) -> str:
    nb = 1 << max(0, math.ceil(math.log2(max(1, prob.n))))
    jb = 1 << max(0, math.ceil(math.log2(max(1, prob.J))))
    return f"{arch}:d{prob.dim}:n{nb}:j{jb}:{prec}"


def _arch() -> str:
    import torch
    try:
        return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:
        return "unknown"


def tuned(ctx, prob, prec: str = "fp32", cache: str | None = None, reps: int = 5) -> dict:
    """Set ctx to the fastest kernel for prob's class; returns the choice."""
    path = cache or DEFAULT_CACHE
    table = {}
    if os.path.exists(path):
        with open(path) as f:
            table = json.load(f)
    key = problem_class(prob, prec, _arch())
    if key in table:
        choice = table[key]
        ctx.apd_set_variant(choice["variant"])
        ctx.apd_set_culling(bool(choice["culling"]))
        ctx.apd_set_pixels_per_lane(int(choice.get("pixels_per_lane", 0)))
        return dict(choice, cached=True)
    choice = ctx.apd_autotune(prob, prec=prec, reps=reps)
    table[key] = choice
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return dict(choice, cached=False)
