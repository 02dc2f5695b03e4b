"""Host logic of the autotuner (CPU): the JSON cache round trip, workload keys, and that a cached
winner is applied without timing anything."""
import json

from paper_2207_12011_amd import autotune as AT


class FakeRp:
    """Records the calls the autotuner makes; times nothing."""

    def __init__(self):
        self.calls = []

    def set_launch_shape(self, ctx, s, t):
        self.calls.append(("set", s, t))

    def autotune_render(self, ctx, vid, cam, w, h, lod, step, repeats):
        self.calls.append(("tune", w, h))
        return (1, 3), [[1.2 + t, 1.0 + t, 1.1 + t, 1.3 + t] for t in (0.5, 0.4, 0.3, -0.1, 0.2)]


def test_cache_round_trip(tmp_path):
    path = str(tmp_path / "sub" / "autotune.json")
    assert AT.load_cache(path) == {}
    cache = {"render|gpu|n512|f16|1920x1080|lod0|step0.5": {"super_log2": 2, "tile_log2w": 2, "ms": [[1, 2, 3, 4]]}}
    AT.save_cache(cache, path)
    assert AT.load_cache(path) == cache
    with open(path) as f:
        assert json.load(f) == cache
    (tmp_path / "bad.json").write_text("[1, 2]")
    try:
        AT.load_cache(str(tmp_path / "bad.json"))
        raise AssertionError("a non-object cache must be rejected")
    except ValueError:
        pass


def test_keys_name_the_workload_class():
    a = AT.render_key("MI355X", 512, "f16", 1920, 1080, 0, 0.5)
    assert a == "render|MI355X|n512|f16|1920x1080|lod0|step0.5"
    assert a != AT.render_key("MI355X", 512, "f32", 1920, 1080, 0, 0.5)
    assert AT.server_key("MI355X", "trace") == "server|MI355X|trace"


def test_tune_render_uses_and_fills_the_cache():
    rp = FakeRp()
    cache = {}
    key = AT.render_key("dev", 64, "f16", 200, 136, 0, 0.5)
    r = AT.tune_render(rp, None, 1, None, 200, 136, cache=cache, key=key)
    assert not r["cached"] and (r["super_log2"], r["tile_log2w"]) == (1, 3)
    assert r["wave_tile_px"] == [8, 2] and r["super_tile_px"] == [32, 8] and rp.calls == [("tune", 200, 136)]
    assert (cache[key]["super_log2"], cache[key]["tile_log2w"]) == (1, 3)
    rp.calls.clear()
    r = AT.tune_render(rp, None, 1, None, 200, 136, cache=cache, key=key)
    assert r["cached"] and rp.calls == [("set", 1, 3)]
    rp.calls.clear()
    AT.tune_render(rp, None, 1, None, 200, 136, cache=cache, key=key, retune=True)
    assert rp.calls == [("tune", 200, 136)]


def test_tune_server_cache_hit_runs_nothing():
    cache = {"server|dev|mix": {"tiles_per_step": 8192, "steps_in_flight": 2, "requests": 4, "candidates": []}}
    r = AT.tune_server(None, None, [], cache=cache, key="server|dev|mix")
    assert r["cached"] and r["tiles_per_step"] == 8192
