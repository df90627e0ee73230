"""Autotuner of a plan's execution, timing whole forward passes with HIP
events.  Two stages:

1. schedule: the launch mode (per-sensor launches or one persistent launch
   for all sensors), frames per pass, persistent workgroups per CU and the
   row-pass split, every sensor at its default tile;
2. tile shapes: for the best schedule of each mode, the row-pass tile (rows
   of the field per workgroup) of each group of sensors with the same FFT
   size, tried in turn and kept where it is faster (a greedy pass: the
   groups are few and nearly independent).

The winner is cached in a JSON file keyed by (GPU architecture, sensors,
frames per call).  Candidates only change how the same arithmetic is
scheduled and tiled, so every setting gives bit-identical results.
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


ROW_TILES = (8, 16, 32)   # tried per FFT size; the library accepts the ones compiled for it


def tile_groups(plan) -> Dict[int, List[int]]:
    """Sensors grouped by FFT size (the row tiles compiled depend on it)."""
    groups: Dict[int, List[int]] = {}
    for i, s in enumerate(plan.sensors):
        groups.setdefault(int(s.n_fft), []).append(i)
    return groups


def set_row_tiles(plan, tiles: List[int]) -> None:
    """Applies one selection per sensor (0 = the sensor's default tile)."""
    for i, r in enumerate(tiles):
        plan.set_row_tile(i, r)


def tile_options(plan, sensors: List[int], current: List[int]) -> List[int]:
    """Row tiles other than the default that the library accepts for every
    sensor of a group; the selection ``current`` is restored afterwards."""
    set_row_tiles(plan, [0] * len(current))
    default = plan.row_tile(sensors[0])
    ok = []
    for r in ROW_TILES:
        if r == default:
            continue
        try:
            for i in sensors:
                plan.set_row_tile(i, r)
            ok.append(r)
        except P.PwfsError:
            pass
        finally:
            set_row_tiles(plan, [0] * len(current))
    set_row_tiles(plan, current)
    return ok


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
        if "row_tiles" in cache[key]:
            set_row_tiles(plan, cache[key]["row_tiles"])
        return dict(cache[key], cached=True)
    timer = timer or (lambda: measure(plan, run, reps))
    defaults = [0] * len(plan.sensors)
    set_row_tiles(plan, defaults)
    # stage 1: schedules at the default tiles
    results = []
    for c in (list(cands) if cands is not None else candidates(plan)):
        try:
            plan.set_tuning(**c)
        except P.PwfsError:
            continue
        results.append((timer(), c, defaults))
    results.sort(key=lambda r: r[0])
    # stage 2: row tiles per FFT size, from the best schedule of each mode
    tried_tiles = []
    finals = []
    for mode in sorted({c["mode"] for _, c, _ in results}):
        ms, c, _ = next(r for r in results if r[1]["mode"] == mode)
        plan.set_tuning(**c)
        tiles = list(defaults)
        set_row_tiles(plan, tiles)
        for n_fft, group in sorted(tile_groups(plan).items()):
            for r in tile_options(plan, group, tiles):
                trial = list(tiles)
                for i in group:
                    trial[i] = r
                set_row_tiles(plan, trial)
                t = timer()
                tried_tiles.append(dict(c, row_tiles=trial, ms=t))
                if t < ms:
                    ms, tiles = t, trial
            set_row_tiles(plan, tiles)
        finals.append((ms, c, tiles))
    finals.sort(key=lambda r: r[0])
    best_ms, best, best_tiles = finals[0]
    plan.set_tuning(**best)
    set_row_tiles(plan, best_tiles)
    rec = dict(best, row_tiles=best_tiles, ms=best_ms,
               tried=[dict(c, row_tiles=tl, ms=ms) for ms, c, tl in results] + tried_tiles)
    cache[key] = rec
    save_cache(cache_path, cache)
    return dict(rec, cached=False)
