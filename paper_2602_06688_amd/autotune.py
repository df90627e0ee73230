"""Autotuner of a plan's execution: searches the launch mode (per-sensor
launches or one persistent launch for all sensors), frames per pass,
persistent workgroups per CU and the row-pass split, timing whole forward
passes with HIP events; the best setting is cached in a JSON file keyed by
(GPU architecture, sensors, frames per call).

Candidates only change how the same arithmetic is scheduled, so every
setting gives bit-identical results.
"""

from __future__ import annotations

import json
import os
from typing import Callable, Dict, Iterable, List, Optional

from . import pwfs as P


def plan_key(plan, n_frames: int, arch: str) -> str:
    parts = []
    for s in plan.sensors:
        parts.append(f"D{s.n_pupil}N{s.n_fft}m{s.n_mod}l{len(s.lambdas_nm)}f{getattr(s, 'flags', 1)}")
    return f"{arch}|{'+'.join(parts)}|F{n_frames}"


def candidates(plan) -> List[dict]:
    t = plan.get_tuning()
    mc = t["max_chunk"]
    chunks = sorted({mc, max(1, mc // 2), max(1, mc // 4)}, reverse=True)
    out = []
    for c in chunks:
        for rg in (1024, 2048, 4096):
            out.append({"mode": P.MODE_LAUNCHES, "chunk": c, "wg_per_cu": t["wg_per_cu"], "row_groups": rg})
    persistent_ok = True
    try:
        plan.set_tuning(mode=P.MODE_PERSISTENT)
    except P.PwfsError:
        persistent_ok = False
    plan.set_tuning(**t)
    if persistent_ok:
        for c in chunks:
            for w in (1, 2, 3):
                out.append({"mode": P.MODE_PERSISTENT, "chunk": c, "wg_per_cu": w, "row_groups": 2048})
    return out


def measure(plan, run: Callable[[], None], reps: int = 3) -> float:
    """Mean ms of ``run`` (after one warm-up call) with HIP events."""
    import torch
    run()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        run()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def load_cache(path: Optional[str]) -> Dict[str, dict]:
    if not path or not os.path.exists(path):
        return {}
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(path: Optional[str], cache: Dict[str, dict]) -> None:
    if not path:
        return
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def autotune(plan, run: Callable[[], None], n_frames: int, arch: str = "gfx950", cache_path: Optional[str] = None,
             cands: Optional[Iterable[dict]] = None, reps: int = 3, timer=None) -> dict:
    """Applies and returns the fastest tuning for ``run`` (one forward call
    on ``plan``).  A cached entry for the same key is applied without search."""
    key = plan_key(plan, n_frames, arch)
    cache = load_cache(cache_path)
    if key in cache:
        plan.set_tuning(**{k: cache[key][k] for k in ("mode", "chunk", "wg_per_cu", "row_groups")})
        return dict(cache[key], cached=True)
    timer = timer or (lambda: measure(plan, run, reps))
    results = []
    for c in (list(cands) if cands is not None else candidates(plan)):
        try:
            plan.set_tuning(**c)
        except P.PwfsError:
            continue
        results.append((timer(), c))
    results.sort(key=lambda r: r[0])
    best_ms, best = results[0]
    plan.set_tuning(**best)
    rec = dict(best, ms=best_ms, tried=[dict(c, ms=ms) for ms, c in results])
    cache[key] = rec
    save_cache(cache_path, cache)
    return dict(rec, cached=False)
