"""Autotuner of the GEMM call sites of the MPDO update.

Each call site of the update's contractions (``mpdo_tune_set``: the one-,
two- and three-site updates, the transfer steps, the truncation sweep) can
run with a 32 or 64 tile, the four- or three-product complex form, and a
factor on its split-K count.  ``tune`` times candidates on a representative
step of the caller's workload: the step runs launch by launch with the
library's profiler on, and each site's summed HIP-event time decides.  The
sites are visited by decreasing time share; for each, the form, then the
tile, then (Gram sites) the split factor is varied with the others fixed at
their best so far (coordinate descent), and a candidate replaces the
incumbent only if it is faster by more than `margin`.  Results are kept in a
JSON cache keyed by device, precision, limits and workload name.
"""
from __future__ import annotations

import json
import os
from typing import Callable, Dict, Optional

from . import mpdo as M

SITE_INDEX = {name: i for i, name in enumerate(M.GEMM_SITES)}
GRAM_SITES = {"q1_gram", "q2_gram_E", "q2_gram_H", "q2_gram_C", "q3_gram_NE", "q3_gram_H", "q3_gram_C1",
              "q3_gram_C2", "sweep_gram"}


def _site_times(step: Callable[[], None]) -> Dict[str, float]:
    M.profile_enable(True)
    step()
    t = {k: v["ms"] for k, v in M.profile_sites().items() if k != "other"}
    M.profile_enable(False)
    return t


def tune(step: Callable[[], None], top: int = 8, margin: float = 0.03, log: Optional[Callable] = None) -> dict:
    """Tune the `top` most expensive call sites of `step` (a callable that
    runs one representative step, launch by launch).  Returns {site: {tile,
    form, split_scale, ms, default_ms}} of the tuned sites; the settings are
    left applied."""
    step()  # warm-up (allocations, caches)
    base = _site_times(step)
    order = sorted(base, key=lambda k: -base[k])[:top]
    out = {}
    for name in order:
        s = SITE_INDEX[name]
        best = {"tile": 0, "form": 0, "split_scale": 0.0}
        best_ms = _site_times(step)[name]
        default_ms = best_ms
        axes = [("form", (3, 4)), ("tile", (32, 64))]
        if name in GRAM_SITES:
            axes.append(("split_scale", (0.5, 2.0)))
        for key, values in axes:
            for v in values:
                cand = dict(best)
                cand[key] = v
                M.tune_set(s, cand["tile"], cand["form"], cand["split_scale"])
                ms = _site_times(step).get(name, float("inf"))
                if ms < best_ms * (1 - margin):
                    best, best_ms = cand, ms
            M.tune_set(s, best["tile"], best["form"], best["split_scale"])
        out[name] = {**best, "ms": best_ms, "default_ms": default_ms}
        if log:
            log(f"autotune {name}: {default_ms:.2f} -> {best_ms:.2f} ms with {best}")
    return out


def apply(settings: dict) -> None:
    for name, s in settings.items():
        M.tune_set(SITE_INDEX[name], int(s["tile"]), int(s["form"]), float(s["split_scale"]))


def reset() -> None:
    for i in range(1, len(M.GEMM_SITES)):
        M.tune_set(i, 0, 0, 0.0)


def snapshot() -> list:
    """The current settings of every call site (sites 1.., for restore)."""
    return [M.tune_get(i) for i in range(1, len(M.GEMM_SITES))]


def restore(snap: list) -> None:
    for i, (tile, form, split) in enumerate(snap, start=1):
        M.tune_set(i, tile, form, split)


class applied:
    """Context manager: the given settings (or the built-in choices for
    None) while the block runs, the previous ones afterwards."""

    def __init__(self, settings: Optional[dict]):
        self.settings = settings

    def __enter__(self):
        self.snap = snapshot()
        reset()
        if self.settings:
            apply(self.settings)
        return self

    def __exit__(self, *exc):
        restore(self.snap)
        return False


def device_name() -> str:
    import torch
    return torch.cuda.get_device_name(0)


def cache_key(prec: int, chi: int, kappa: int, mmax: int, workload: str) -> str:
    return f"{device_name()}|prec{prec}|chi{chi}|kappa{kappa}|m{mmax}|{workload}"


def load(path: str, key: str) -> Optional[dict]:
    try:
        with open(path) as f:
            return json.load(f).get(key)
    except (OSError, ValueError):
        return None


def save(path: str, key: str, settings: dict) -> None:
    data = {}
    try:
        with open(path) as f:
            data = json.load(f)
    except (OSError, ValueError):
        pass
    data[key] = settings
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    with open(path, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)


def tuned(step: Callable[[], None], path: str, key: str, log: Optional[Callable] = None, **kw) -> dict:
    """Apply the cached settings of `key`, or tune and cache them."""
    s = load(path, key)
    if s:
        apply(s)
        return {"source": "cache", "settings": s}
    s = tune(step, log=log, **kw)
    save(path, key, s)
    return {"source": "tuned", "settings": s}
