"""Persistent cache of autotuned launch plans (JSON), keyed by device and workload.

The library's autotuner (``Context.autotune`` -> ``kohler_autotune``) times candidate plans on the
device; this module stores the winner so that later processes on the same kind of device skip the
search. Keys name the device architecture and compute-unit count, the family (dtype, M, nbhd) and
a coarse workload class, so a plan tuned for one 18 MP image is not reused for a batch of small
images.
"""
from __future__ import annotations

import json
import math
import os

DEFAULT_PATH = os.path.join(os.path.expanduser("~"), ".cache", "kohler_plans.json")


def workload_class(shapes: list[tuple[int, int]]) -> str:
    """'single:<log2 px>' for one image, 'batch:<log2 n>:<log2 px total>' for several."""
    px = sum(int(h) * int(w) for h, w in shapes)
    lp = int(round(math.log2(max(px, 1))))
    if len(shapes) == 1:
        return f"single:{lp}"
    return f"batch:{int(round(math.log2(len(shapes))))}:{lp}"


def plan_key(device_name: str, cus: int, dtype: int, M: int, nbhd: int, shapes) -> str:
    return f"{device_name}:{cus}:{dtype}:{M}:{nbhd}:{workload_class(list(shapes))}"


def load(path: str = DEFAULT_PATH) -> dict:
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def store(key: str, plan: dict, us: float, path: str = DEFAULT_PATH) -> None:
    data = load(path)
    data[key] = {"plan": {k: int(v) for k, v in plan.items()}, "us": float(us)}
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tuned_plan(ctx, imgs, M: int, nbhd: int, path: str | None = DEFAULT_PATH, reps: int = 5,
               retune: bool = False) -> tuple[dict, float, bool]:
    """Apply a cached plan for this device and workload to `ctx`, or autotune and cache it.
    Returns (plan, us, from_cache)."""
    import torch

    from . import _dtype_code
    imgs = list(imgs)
    props = torch.cuda.get_device_properties(ctx.device)
    name = getattr(props, "gcnArchName", props.name)
    code = _dtype_code(imgs[0].dtype)
    key = plan_key(name, props.multi_processor_count, code, M, nbhd, [tuple(im.shape) for im in imgs])
    if path and not retune:
        hit = load(path).get(key)
        if hit:
            p = hit["plan"]
            ctx.set_plan(code, M, nbhd, **p)
            return p, float(hit["us"]), True
    plan, us = ctx.autotune(imgs, M, nbhd, reps)
    if path:
        store(key, plan, us, path)
    return plan, us, False
