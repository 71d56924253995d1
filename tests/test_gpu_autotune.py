"""GPU: the autotuner.  Every tuning it times gives the same output words,
equal to the oracle's; the chosen tuning is one it timed; the cache returns
it without a search; a tuned batch equals the per-layer calls and the
oracle."""
import numpy as np
import pytest

import oracle
import synth
from synth import Stream
from tests.gpu_util import empty_words, require_gpu, to_dev, to_host
from tests.libload import ensure_built
from tests.test_gpu_batch import SHAPES_4096, make_jobs

pytestmark = pytest.mark.gpu

# (N, L, bits, shape, B): config 1's layer, layers with M >= 8 so that the
# output-channel pipeline is a live knob at B = 1, and a batch of 2
LAYERS = [
    (4096, 2, 50, (4, 16, 16, 4, 3, 3, 1, 1), 1),
    (4096, 2, 50, (16, 14, 14, 16, 3, 3, 1, 1), 1),
    (8192, 3, 60, (32, 20, 20, 24, 3, 3, 1, 1), 1),
    (8192, 3, 60, (12, 9, 9, 10, 1, 1, 2, 0), 2),
]


def _ctx(N, L, bits):
    require_gpu()
    ensure_built()
    from paper_2506_11586_amd import heconv
    return heconv.Context(N, heconv.gen_primes(N, bits, L)), oracle.Params(N, L, bits, 2 ** 37)


@pytest.mark.parametrize("N,L,bits,shape,B", LAYERS)
def test_every_timed_tuning_gives_the_oracle_words(tmp_path, N, L, bits, shape, B):
    import torch
    from paper_2506_11586_amd import autotune
    ctx, prm = _ctx(N, L, bits)
    d = ctx.plan(shape, batch=B)
    s = ctx.sizes(d)
    cv = oracle.Conv(*shape)
    g = oracle.geometry(cv, d.Cw, d.Hw, d.Ww)
    K = Stream(N + B, synth.WEIGHT).ints(cv.M * cv.C * cv.kh * cv.kw, -2 ** 8, 2 ** 8)
    K = K.reshape(cv.M, cv.C, cv.kh, cv.kw)
    x = synth.uniform_mod(Stream(N + B, synth.UNIFORM), (B * s.in_cts * 2, prm.L, prm.N), prm.q)
    wntt = empty_words(s.w_words)
    ctx.encode_weights(d, to_dev(K), wntt)
    pristine = to_dev(x)
    work = pristine.clone()
    out = empty_words(B * s.out_cts * 2 * prm.L * prm.N)

    cache = autotune.TuneCache(str(tmp_path / "tune.json"))
    res = autotune.tune_layer(torch, ctx, d, B, work, wntt, out, cache=cache, reps=5, warm_s=0.02)
    assert not res.cached and len(res.evaluations) >= 5
    assert np.isfinite(res.ms) and res.ms * (1 - 0.01) <= min(ms for _, ms in res.evaluations)
    assert any(t == res.tuning for t, _ in res.evaluations)
    assert ctx.get_tuning().as_dict() == res.tuning

    want = oracle.conv_layer_ntt(x.reshape(B, g.CB, g.S, 2, prm.L, prm.N),
                                 oracle.encode_weights(K, cv, g, prm), B, g, cv.M, prm)
    for t, _ in res.evaluations:
        ctx.set_tuning(**t)
        work.copy_(pristine)
        out.fill_(-1)
        ctx.conv_layer(d, B, work, wntt, out)
        torch.cuda.synchronize()
        assert np.array_equal(to_host(out).reshape(want.shape), want), t

    again = autotune.tune_layer(torch, ctx, d, B, work, wntt, out, cache=autotune.TuneCache(cache.path),
                                reps=3, warm_s=0.01, apply=False)
    assert again.cached and again.tuning == res.tuning


def test_tuned_batch_equals_layers_and_oracle(tmp_path):
    import torch
    from paper_2506_11586_amd import autotune, heconv
    ctx, prm = _ctx(4096, 2, 50)
    jobs, host = make_jobs(ctx, prm, SHAPES_4096, 700)
    pristine = [j[2].clone() for j in jobs]
    res = autotune.tune_batch(torch, ctx, jobs, cache=autotune.TuneCache(str(tmp_path / "b.json")), reps=3,
                              warm_s=0.02)
    assert res.schedule in (heconv.SCHED_ONE_CHAIN, heconv.SCHED_TWO_CHAINS)
    assert np.isfinite(res.ms) and res.ms * (1 - 0.01) <= min(ms for _, ms in res.evaluations)
    wants = []
    for (d, B, *_), (cv, _, _, x, K) in zip(jobs, host):
        g = oracle.geometry(cv, d.Cw, d.Hw, d.Ww)
        wants.append(oracle.conv_layer_ntt(x.reshape(B, g.CB, g.S, 2, prm.L, prm.N),
                                           oracle.encode_weights(K, cv, g, prm), B, g, cv.M, prm))
    for t, _ in res.evaluations:
        t = dict(t)
        sched = t.pop("schedule")
        ctx.set_tuning(**t)
        for j, p in zip(jobs, pristine):
            j[2].copy_(p)
            j[4].fill_(-1)
        b = heconv.Batch(ctx, jobs, schedule=sched)
        b.launch(graph=True)
        b.status()
        for j, w in zip(jobs, wants):
            assert np.array_equal(to_host(j[4]).reshape(w.shape), w), (t, sched)
        b.close()
    hit = autotune.tune_batch(torch, ctx, jobs, cache=autotune.TuneCache(str(tmp_path / "b.json")))
    assert hit.cached and hit.schedule == res.schedule and hit.tuning == res.tuning
