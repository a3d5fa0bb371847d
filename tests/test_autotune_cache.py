"""The launch-schedule cache (host logic only): keys bucket the plan shape,
a cached entry is applied without timing, a missing one is timed once and
stored."""
import json

from paper_1706_01420_amd import autotune


class FakeLib:
    def __init__(self):
        self.applied = []
        self.tuned = 0

    def ipx_plan_set_schedule(self, plan, workgroups=0, order=0, graph=1, variant=0):
        self.applied.append((workgroups, order, graph, variant))

    def ipx_plan_autotune(self, ctx, plan, theta, grad=True, reps=5):
        self.tuned += 1
        rows = [({"workgroups": 0, "order": 0, "graph": 1, "variant": 0}, 120.0),
                ({"workgroups": 4096, "order": 1, "graph": 0, "variant": 1}, 100.0)]
        return {"workgroups": 4096, "order": 1, "graph": 0, "variant": 1}, 100.0, rows


def test_bucket_and_key():
    assert autotune.bucket(0) == 1 and autotune.bucket(1) == 1
    assert autotune.bucket(3) == 4 and autotune.bucket(5) == 4 and autotune.bucket(6) == 8
    assert autotune.bucket(100000) == 131072
    k1 = autotune.key(3, True, 512, 3.4e7, "gfx950")
    k2 = autotune.key(3, True, 500, 3.3e7, "gfx950")
    assert k1 == k2                      # same shape bucket
    assert k1 != autotune.key(3, False, 512, 3.4e7, "gfx950")
    assert k1 != autotune.key(2, True, 512, 3.4e7, "gfx950")
    assert k1 != autotune.key(3, True, 512, 3.4e7, "gfx942")


def test_tune_then_cache(tmp_path):
    path = str(tmp_path / "sub" / "tune.json")
    lib = FakeLib()
    s, src = autotune.tune_plan(lib, None, None, 3, None, [1000, 2000], path=path, arch="gfx950")
    assert src == "tuned" and s == {"workgroups": 4096, "order": 1, "graph": 0, "variant": 1} and lib.tuned == 1
    data = json.load(open(path))
    assert len(data) == 1
    (entry,) = data.values()
    assert entry["workgroups"] == 4096 and entry["order"] == 1 and entry["graph"] == 0 and entry["variant"] == 1
    assert len(entry["candidates"]) == 2
    s, src = autotune.tune_plan(lib, None, None, 3, None, [1100, 1900], path=path, arch="gfx950")
    assert src == "cache" and s == {"workgroups": 4096, "order": 1, "graph": 0, "variant": 1}
    assert lib.tuned == 1 and lib.applied == [(4096, 1, 0, 1)]


def test_unreadable_cache_is_empty(tmp_path):
    p = tmp_path / "bad.json"
    p.write_text("{not json")
    assert autotune.load(str(p)) == {}
    assert autotune.load(str(tmp_path / "missing.json")) == {}
