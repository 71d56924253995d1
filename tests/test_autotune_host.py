"""Host logic of the autotuner: the search, the candidate spaces, the cache
keys and the JSON cache (no GPU: costs are synthetic functions)."""
import itertools
import json

import pytest

from paper_2506_11586_amd import autotune


def test_coordinate_descent_finds_separable_minimum():
    """With a cost that is a sum over knobs, one sweep reaches the exact
    minimum, whatever the start."""
    space = [("a", [{"a": v} for v in (1, 2, 3, 4)]), ("b", [{"b": v} for v in (10, 20, 30)])]
    pa = {1: 5.0, 2: 1.0, 3: 3.0, 4: 2.0}
    pb = {10: 7.0, 20: 9.0, 30: 0.5}
    for a0, b0 in itertools.product(pa, pb):
        best, c, trail = autotune.coordinate_descent(space, {"a": a0, "b": b0, "x": 7},
                                                     lambda t: pa[t["a"]] + pb[t["b"]])
        assert best == {"a": 2, "b": 30, "x": 7} and c == 1.5
        assert trail[0] == ({"a": a0, "b": b0, "x": 7}, pa[a0] + pb[b0])
        assert len({tuple(sorted(t.items())) for t, _ in trail}) == len(trail)  # each tuning timed once


def test_coordinate_descent_never_worse_and_skips_rejected():
    """An interacting cost: the result costs no more than the start and no
    more than anything it timed; an infinite (rejected) candidate is never
    chosen; equal costs keep the earlier value."""
    space = [("a", [{"a": v} for v in range(4)]), ("b", [{"b": v} for v in range(4)])]

    def cost(t):
        if t["a"] == 3:
            return float("inf")
        return (t["a"] - 1) * (t["b"] - 2) + 10

    best, c, trail = autotune.coordinate_descent(space, {"a": 0, "b": 0}, cost, sweeps=3)
    assert c == min(v for _, v in trail) and c <= cost({"a": 0, "b": 0})
    assert best["a"] != 3
    flat = [("a", [{"a": 0}, {"a": 1}])]
    best, c, _ = autotune.coordinate_descent(flat, {"a": 1}, lambda t: 1.0)
    assert best == {"a": 1}


def test_min_gain_keeps_the_start_on_small_differences():
    """A candidate within the margin does not replace the best; one beyond
    it does; the result is within 1/(1 - min_gain) of the cheapest timed."""
    space = [("a", [{"a": v} for v in range(3)])]
    costs = {0: 1.0, 1: 0.995, 2: 0.5}
    best, c, _ = autotune.coordinate_descent(space[:1], {"a": 0}, lambda t: costs[t["a"]] if t["a"] < 2 else 2.0,
                                             min_gain=0.01)
    assert best == {"a": 0} and c == 1.0
    best, c, trail = autotune.coordinate_descent(space, {"a": 0}, lambda t: costs[t["a"]], min_gain=0.01)
    assert best == {"a": 2} and c == 0.5
    best, c, trail = autotune.coordinate_descent(space, {"a": 0}, lambda t: costs[t["a"]] if t["a"] < 2 else 2.0,
                                                 min_gain=0.01)
    assert c * (1 - 0.01) <= min(v for _, v in trail)


def test_spaces_hold_only_supported_values():
    """MAC tiles are the library's supported pairs or (0, 0) (by shape); 8
    words per thread is offered only where N/8 threads fit a workgroup."""
    supported = {(4, 4), (4, 2), (2, 4), (8, 2), (2, 8), (8, 1), (1, 8), (2, 2), (0, 0), (6, 4)}
    for N in (4096, 8192, 16384):
        for space in (autotune.layer_space(N), autotune.batch_space(N)):
            for name, values in space:
                for v in values:
                    if "mac_mt" in v:
                        assert (v["mac_mt"], v["mac_rt"]) in supported
                    for k in ("ntt_loge_small", "ntt_loge_large"):
                        if k in v:
                            assert v[k] in ((3, 4) if N <= 8192 else (4,))
    names = [n for n, _ in autotune.layer_space(8192)]
    assert names == ["ntt_loge_small", "ntt_loge_large", "mac", "mac_lds", "layer_split", "ntt_split_below",
                     "ntt_inv_split_below", "layer_fused", "ntt_fp64"]
    assert [n for n, _ in autotune.batch_space(8192)] == ["mac", "mac_lds", "mac_grid", "mac_tiles",
                                                         "ntt_loge_small", "ntt_loge_large"]


class _Desc:
    def __init__(self, shape, pk):
        self._s, (self.Cw, self.Hw, self.Ww) = shape, pk

    def shape(self):
        return self._s


class _Ctx:
    def __init__(self, N, q):
        self.N, self.L, self.q = N, len(q), q


def test_cache_keys_separate_what_changes_timing():
    ctx = _Ctx(8192, [1, 2, 3])
    d = _Desc((64, 56, 56, 64, 3, 3, 1, 1), (4, 58, 35))
    k = autotune.layer_key("dev", ctx, d, 1)
    assert k != autotune.layer_key("dev", ctx, d, 2)
    assert k != autotune.layer_key("dev2", ctx, d, 1)
    assert k != autotune.layer_key("dev", _Ctx(8192, [1, 2, 4]), d, 1)
    assert k != autotune.layer_key("dev", ctx, _Desc(d.shape(), (2, 58, 35)), 1)
    assert k != autotune.layer_key("dev", ctx, _Desc((64, 56, 56, 32, 3, 3, 1, 1), (4, 58, 35)), 1)
    jobs = [(d, 1), (_Desc((16, 28, 28, 8, 1, 1, 1, 0), (16, 28, 9)), 2)]
    kb = autotune.batch_key("dev", ctx, jobs)
    assert kb != autotune.batch_key("dev", ctx, jobs[::-1])
    assert kb != autotune.batch_key("dev", ctx, [(jobs[0][0], 1), (jobs[1][0], 3)])
    assert kb == autotune.batch_key("dev", ctx, list(jobs))


def test_cache_json_round_trip(tmp_path):
    p = str(tmp_path / "tune.json")
    c = autotune.TuneCache(p)
    assert c.get("k") is None
    c.put("k", {"mac_mt": 4, "mac_rt": 2}, 0.1, 0.2)
    c2 = autotune.TuneCache(p)
    assert c2.get("k") == {"mac_mt": 4, "mac_rt": 2}
    assert json.load(open(p))["k"]["default_ms"] == 0.2
    got = c2.get("k")
    got["mac_mt"] = 99  # callers get copies
    assert c2.get("k")["mac_mt"] == 4
    (tmp_path / "bad.json").write_text("[1, 2]")
    with pytest.raises(ValueError):
        autotune.TuneCache(str(tmp_path / "bad.json"))
