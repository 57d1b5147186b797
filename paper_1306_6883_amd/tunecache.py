"""A file cache of autotuned launch shapes.

ccmg_plan_autotune times every candidate tile shape of every level on the
device at hand.  The best shapes depend on the device (its architecture and
compute-unit count), the ROCm runtime, the library build and the problem's
signature (size, side types, precision, smoothing counts, bottom), not on the
right-hand side.  This module keeps them in a JSON file keyed by all of those,
so that a later plan of the same signature on the same device and build takes
the stored shapes (ccmg_plan_set_shape) instead of timing again.  Entries of
another device, runtime or build are never applied.

    shapes = tuned(plan, f, phi, path="~/.cache/ccmg_tune.json")
"""
from __future__ import annotations

import hashlib
import json
import os
import tempfile

import torch

from . import (LIB_PATH, Plan, ccmg_plan_autotune, ccmg_plan_fused_shape, ccmg_plan_set_shape, ccmg_plan_shape,
               ccmg_plan_shapes)

_lib_digest = None


def library_digest() -> str:
    """SHA-256 of the loaded library file: any rebuild makes a new key."""
    global _lib_digest
    if _lib_digest is None:
        h = hashlib.sha256()
        with open(LIB_PATH, "rb") as fh:
            for block in iter(lambda: fh.read(1 << 20), b""):
                h.update(block)
        _lib_digest = h.hexdigest()
    return _lib_digest


def device_key(device=None) -> dict:
    """The device and runtime part of a cache key."""
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    p = torch.cuda.get_device_properties(dev)
    return {"arch": getattr(p, "gcnArchName", p.name), "name": p.name, "cus": p.multi_processor_count,
            "hip": torch.version.hip or "", "library": library_digest()}


def problem_key(prob) -> dict:
    """The problem part of a cache key: what the launch shapes depend on."""
    return {"n": prob.n, "bc": "".join(str(b) for b in prob.bc_codes()), "prec": prob.prec, "nu1": prob.nu1,
            "nu2": prob.nu2, "singular": prob.alpha == 0.0 and 0 not in prob.bc_codes(),
            "helmholtz": prob.alpha != 0.0}


def cache_key(prob, device=None) -> str:
    return json.dumps({"device": device_key(device), "problem": problem_key(prob)}, sort_keys=True)


def _load(path: str) -> dict:
    try:
        with open(path) as fh:
            data = json.load(fh)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def _store(path: str, data: dict) -> None:
    d = os.path.dirname(os.path.abspath(path))
    os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=d, suffix=".tmp")
    with os.fdopen(fd, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _row_march_levels(plan: Plan) -> int:
    """Levels above the one-workgroup tail (those of more than 32 x 32 cells)."""
    return max(0, plan.n.bit_length() - 1 - 5)


def shapes_of(plan: Plan) -> dict:
    """The plan's launch shapes: per level (pre ty, pre wpb, post ty, post
    wpb), the fused finest launch in FP64 and FP32, per level below the
    finest its visit shapes (restricting ty, wpb, visit ty, wpb; visit ty 0:
    the level runs its two launches), and the first fused launch that
    recomputes the first pre-smoothing (ty 0: not used)."""
    return {"levels": [list(s) for s in ccmg_plan_shapes(plan)],
            "fused64": list(ccmg_plan_fused_shape(plan, 2)), "fused32": list(ccmg_plan_fused_shape(plan, 3)),
            "visits": [[*ccmg_plan_shape(plan, lv, 4), *ccmg_plan_shape(plan, lv, 5)]
                       for lv in range(1, _row_march_levels(plan))],
            "fused0": list(ccmg_plan_shape(plan, 0, 6))}


def apply_shapes(plan: Plan, shapes: dict) -> None:
    for level, (tp, wp, tq, wq) in enumerate(shapes["levels"]):
        ccmg_plan_set_shape(plan, level, 0, tp, wp)
        ccmg_plan_set_shape(plan, level, 1, tq, wq)
    ccmg_plan_set_shape(plan, 0, 2, *shapes["fused64"])
    ccmg_plan_set_shape(plan, 0, 3, *shapes["fused32"])
    for level, (tp, wp, tv, wv) in enumerate(shapes.get("visits", []), start=1):
        ccmg_plan_set_shape(plan, level, 4, tp, wp)
        ccmg_plan_set_shape(plan, level, 5, tv, wv)
    if "fused0" in shapes:
        ccmg_plan_set_shape(plan, 0, 6, *shapes["fused0"])


def tuned(plan: Plan, f: torch.Tensor, phi: torch.Tensor, path: str) -> tuple:
    """Launch shapes for `plan` from the cache at `path`, or by autotuning on
    (f, phi) and storing the result.  Returns (shapes, hit)."""
    path = os.path.expanduser(path)
    key = cache_key(plan.prob, plan.workspace.device)
    data = _load(path)
    if key in data:
        apply_shapes(plan, data[key])
        return data[key], True
    ccmg_plan_autotune(plan, f, phi)
    shapes = shapes_of(plan)
    data = _load(path)  # another process may have written meanwhile
    data[key] = shapes
    _store(path, data)
    return shapes, False
