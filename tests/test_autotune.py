"""Autotuner search and cache logic with a fake plan and timer (no GPU)."""

import json

from paper_2602_06688_amd import autotune as A
from paper_2602_06688_amd import pwfs as P


def _sensor(d, n):
    return type("S", (), dict(n_pupil=d, n_fft=n, n_mod=48, lambdas_nm=(750.0,), flags=1))()


class FakePlan:
    """Stands in for a plan: tuning fields, and per-sensor row tiles with the
    library's rule (default 8, alternative 16; N = 384 the other way round;
    N = 128 one tile)."""
    TILES = {128: (16,), 256: (8, 16), 384: (16, 8), 512: (8, 16), 768: (8, 16)}

    def __init__(self, sensors=None):
        self.sensors = sensors or [_sensor(160, 512)]
        self.t = {"mode": 0, "chunk": 26, "wg_per_cu": 2, "row_groups": 2048, "max_chunk": 26}
        self.tiles = [0] * len(self.sensors)

    def row_tile(self, i):
        return self.tiles[i] or self.TILES[self.sensors[i].n_fft][0]

    def set_row_tile(self, i, r):
        if r and r not in self.TILES[self.sensors[i].n_fft]:
            raise P.PwfsError(-1, "tile not compiled")
        self.tiles[i] = r

    def get_tuning(self):
        return dict(self.t)

    def set_tuning(self, **kw):
        if kw.get("mode") == P.MODE_PERSISTENT and kw.get("wg_per_cu", 1) > 2:
            raise P.PwfsError(-2, "unsupported")
        self.t.update({k: v for k, v in kw.items() if v is not None})
        return self.get_tuning()


def test_autotune_picks_fastest_and_caches(tmp_path):
    plan = FakePlan()
    # persistent, chunk 13, 2 workgroups per CU is the fastest candidate
    def timer():
        t = plan.t
        return 1.0 + (0 if t["mode"] == 1 else 0.5) + abs(t["chunk"] - 13) * 0.01 + (0 if t["wg_per_cu"] == 2 else 0.1)
    path = str(tmp_path / "cache.json")
    rec = A.autotune(plan, lambda: None, 1000, cache_path=path, timer=timer)
    assert rec["mode"] == 1 and rec["chunk"] == 13 and rec["wg_per_cu"] == 2 and not rec["cached"]
    assert plan.t["mode"] == 1 and plan.t["chunk"] == 13
    data = json.load(open(path))
    assert len(data) == 1 and list(data.values())[0]["chunk"] == 13
    # a second call applies the cached choice without timing anything
    plan2 = FakePlan()
    rec2 = A.autotune(plan2, lambda: None, 1000, cache_path=path, timer=lambda: 1 / 0)
    assert rec2["cached"] and plan2.t["chunk"] == 13 and plan2.t["mode"] == 1
    # the key separates frame counts and architectures
    assert A.plan_key(plan, 1000, "gfx950") != A.plan_key(plan, 500, "gfx950")
    assert A.plan_key(plan, 1000, "gfx950") != A.plan_key(plan, 1000, "gfx942")


def test_autotune_searches_row_tiles_per_fft_size(tmp_path):
    sens = [_sensor(80, 256), _sensor(160, 512), _sensor(160, 512), _sensor(240, 768), _sensor(64, 128)]
    plan = FakePlan(sens)
    # launches beat persistent; 16-row tiles help the 768 sensor only
    def timer():
        eff = [plan.row_tile(i) for i in range(len(sens))]
        return (2.0 + (0.3 if plan.t["mode"] == 1 else 0) + abs(plan.t["chunk"] - 26) * 0.01
                - (0.2 if eff[3] == 16 else 0) + (0.1 if eff[1] == 16 or eff[0] == 16 else 0))
    rec = A.autotune(plan, lambda: None, 500, cache_path=str(tmp_path / "c.json"), timer=timer)
    assert rec["mode"] == 0 and rec["chunk"] == 26
    assert rec["row_tiles"] == [0, 0, 0, 16, 0]
    assert [plan.row_tile(i) for i in range(5)] == [8, 8, 8, 16, 16]
    # the tile stage tried 16 for each group that has it, as one change per group
    tile_trials = [t["row_tiles"] for t in rec["tried"] if any(t["row_tiles"])]
    assert [0, 0, 0, 16, 0] in tile_trials and [16, 0, 0, 0, 0] in tile_trials
    assert [0, 16, 16, 0, 0] in tile_trials and not any(t[4] for t in tile_trials)
    # the cached record restores the tiles as well
    plan2 = FakePlan(sens)
    rec2 = A.autotune(plan2, lambda: None, 500, cache_path=str(tmp_path / "c.json"), timer=lambda: 1 / 0)
    assert rec2["cached"] and plan2.tiles == [0, 0, 0, 16, 0]
