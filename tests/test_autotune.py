"""Autotuner search and cache logic with a fake plan and timer (no GPU)."""

import json

from paper_2602_06688_amd import autotune as A
from paper_2602_06688_amd import pwfs as P


class FakePlan:
    def __init__(self):
        self.sensors = [type("S", (), dict(n_pupil=160, n_fft=512, n_mod=48, lambdas_nm=(750.0,), flags=1))()]
        self.t = {"mode": 0, "chunk": 26, "wg_per_cu": 2, "row_groups": 2048, "max_chunk": 26}

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
