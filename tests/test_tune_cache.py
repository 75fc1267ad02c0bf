"""CPU tests of the autotuner's shape buckets and JSON cache (with a stand-in
context and batch; the timing itself is native and runs on the GPU)."""
import json

from paper_1504_01883_amd import tune


class FakeBatch:
    def __init__(self):
        self.cfg = None

    def set_launch(self, **cfg):
        self.cfg = cfg


class FakeCtx:
    dim = 7552

    def __init__(self):
        self.calls = 0

    def tune(self, batch, hist, reps):
        self.calls += 1
        cfg = {"persistent": 1, "wg_per_cu": 2, "row_prefetch": 4, "sorted": 1}
        batch.set_launch(**cfg)
        return cfg, 123.5


def test_bucket_keys():
    assert tune.shape_key(4096, 16384, 7552) == tune.shape_key(3000, 10000, 7552)
    assert tune.shape_key(4096, 16384, 7552) != tune.shape_key(4097, 16384, 7552)
    assert tune.shape_key(1, 1, 7552) == "features|n=1|area=1|dim=7552"


def test_cache_miss_then_hit(tmp_path):
    path = tmp_path / "cache.json"
    ctx, b = FakeCtx(), FakeBatch()
    r = tune.tuned(ctx, b, None, 16384, 27000, path=path)
    assert not r["cached"] and ctx.calls == 1
    data = json.loads(path.read_text())
    assert list(data) == [tune.shape_key(16384, 27000, 7552)]
    b2 = FakeBatch()
    r2 = tune.tuned(ctx, b2, None, 16000, 26000, path=path)
    assert r2["cached"] and ctx.calls == 1 and b2.cfg == r["cfg"]
    r3 = tune.tuned(ctx, b2, None, 16000, 26000, path=path, retune=True)
    assert not r3["cached"] and ctx.calls == 2


def test_env_override(tmp_path, monkeypatch):
    monkeypatch.setenv("LBPF_TUNE_CACHE", str(tmp_path / "x.json"))
    assert tune.cache_path() == tmp_path / "x.json"
