"""Host logic of the synthetic input recipes (CPU): the serving trace is a deterministic function of
its seed, and every request stays within the recipe's ranges."""
import numpy as np

from paper_2207_12011_amd import workloads as W


def small_qtables():
    wl = W.make_workload(1, n=32, width=16, height=16)
    m = W.shell_mask(W.radius(32))
    return [W.quantile_table(wl.fields, m, np.random.default_rng(1), levels=101, sample=4096)]


def key(r):
    return (r.volume, tuple(np.round(r.camera.eye, 12)), r.width, r.height, r.active.tobytes(), r.lo.tobytes(),
            r.hi.tobytes(), r.gap)


def test_serving_trace_is_deterministic_given_the_seed():
    qt = small_qtables()
    a = W.serving_trace(qt, n=64, seed=5)
    b = W.serving_trace(qt, n=64, seed=5)
    c = W.serving_trace(qt, n=64, seed=6)
    assert [key(r) for r in a] == [key(r) for r in b]
    assert [key(r) for r in a] != [key(r) for r in c]


def test_serving_trace_ranges():
    qt = small_qtables()
    for r in W.serving_trace(qt, n=200, seed=7):
        assert (r.width, r.height) in W.SERVING_SIZES
        k = int(r.active.sum())
        assert 1 <= k <= 5
        assert np.all(r.lo[r.active == 1] <= r.hi[r.active == 1])
        assert abs(float(np.linalg.norm(r.camera.eye)) - 3.0) < 1e-9
        assert r.gap > 0
