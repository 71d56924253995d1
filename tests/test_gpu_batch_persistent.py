"""GPU tests of the persistent single-kernel batch executor -- SKIPPED.

That executor hung on the GPU twice and is disabled (he_batch_create
rejects its schedule value 0).  The tests are kept, skipped, as the record
of the case; they call the executor's diagnostics (item counters, spin
limit, workgroup count), which were removed with its kernel and would come
back with a restructured one.  The batch executor in use is tested in
test_gpu_batch.py."""
import numpy as np
import pytest

import oracle
import synth
from synth import Stream
from tests.gpu_util import empty_words, require_gpu, to_dev, to_host
from tests.libload import ensure_built

pytestmark = [
    pytest.mark.gpu,
    pytest.mark.skip(reason="persistent batch kernel disabled: it hung on MI355X twice. Its main loop was compiled "
                            "into a nested loop whose inner loop (barrier + read of the shared item index) can "
                            "repeat without the thread-0 atomic that fetches the next item, so lanes re-read a "
                            "stale index forever. Not to be run on the GPU again before the loop is restructured "
                            "and the cause is confirmed."),
]

# uneven shapes: (shape, B); N=4096, L=2
SHAPES_4096 = [
    ((4, 16, 16, 4, 3, 3, 1, 1), 1),
    ((8, 11, 9, 5, 3, 3, 2, 1), 2),
    ((20, 7, 7, 12, 1, 1, 1, 0), 1),
    ((6, 13, 13, 3, 1, 1, 2, 0), 3),
    ((3, 23, 23, 4, 7, 7, 2, 3), 1),
]


def make_jobs(ctx, prm, shapes, seed):
    jobs, host = [], []
    for i, (shape, B) in enumerate(shapes):
        d = ctx.plan(shape, batch=B)
        s = ctx.sizes(d)
        cv = oracle.Conv(*shape)
        K = Stream(seed + i, synth.WEIGHT).ints(cv.M * cv.C * cv.kh * cv.kw, -2 ** 12, 2 ** 12)
        K = K.reshape(cv.M, cv.C, cv.kh, cv.kw)
        x = synth.uniform_mod(Stream(seed + i, synth.UNIFORM), (B * s.in_cts * 2, prm.L, prm.N), prm.q)
        wntt = empty_words(s.w_words)
        ctx.encode_weights(d, to_dev(K), wntt)
        d_in = to_dev(x)
        d_out = empty_words(B * s.out_cts * 2 * prm.L * prm.N)
        d_out.fill_(-1)
        jobs.append((d, B, d_in, wntt, d_out))
        host.append((cv, d, B, x, K))
    return jobs, host


@pytest.fixture(scope="module")
def ctx4096():
    require_gpu()
    ensure_built()
    from paper_2506_11586_amd import heconv
    prm = oracle.Params(4096, 2, 50, 2 ** 37)
    return heconv.Context(4096, heconv.gen_primes(4096, 50, 2)), prm


@pytest.mark.parametrize("schedule", [0, 1])
@pytest.mark.parametrize("graph", [False, True])
def test_batch_equals_layer_and_oracle(ctx4096, schedule, graph):
    from paper_2506_11586_amd import heconv
    ctx, prm = ctx4096
    jobs, host = make_jobs(ctx, prm, SHAPES_4096, 100 + schedule)
    b = heconv.Batch(ctx, jobs, schedule=schedule)
    assert b.n_items > 0 and b.n_workgroups > 0
    b.launch(graph=graph)
    disp, err, seen, target, per_job = b.counters()
    print(f"items={b.n_items} wg={b.n_workgroups} dispensed={disp} err={err} seen={seen} target={target} "
          f"jobs={per_job}", flush=True)
    b.status()
    assert disp >= b.n_items
    for (d, B, d_in, wntt, d_out), (cv, _, _, x, K) in zip(jobs, host):
        g = oracle.geometry(cv, d.Cw, d.Hw, d.Ww)
        got = to_host(d_out).reshape(B, cv.M, g.S, 2, prm.L, prm.N)
        # standalone entry point on the same input
        ref_in = to_dev(x)
        ref_out = empty_words(got.size)
        ctx.conv_layer(d, B, ref_in, wntt, ref_out)
        assert np.array_equal(got, to_host(ref_out).reshape(got.shape))
        # oracle: the paper's flow on the same words
        w_ntt = oracle.encode_weights(K, cv, g, prm)
        want = oracle.conv_layer_ntt(x.reshape(B, g.CB, g.S, 2, prm.L, prm.N), w_ntt, B, g, cv.M, prm)
        assert np.array_equal(got, want)
    b.close()


def test_graph_replays_match_eager(ctx4096):
    """The captured graph replayed several times, with eager work (restoring
    the inputs) and synchronisation between replays: every replay equals the
    eager launch."""
    import torch
    from paper_2506_11586_amd import heconv
    ctx, prm = ctx4096
    jobs, host = make_jobs(ctx, prm, SHAPES_4096[:3], 300)
    pristine = [j[2].clone() for j in jobs]
    b = heconv.Batch(ctx, jobs)
    b.launch(graph=False)
    b.status()
    eager = [to_host(j[4]).copy() for j in jobs]
    for rep in range(4):
        for j, p in zip(jobs, pristine):
            j[2].copy_(p)
            j[4].fill_(rep)
        torch.cuda.synchronize()
        b.launch(graph=True)
        b.status()
        for j, e in zip(jobs, eager):
            assert np.array_equal(to_host(j[4]), e), rep
    b.close()


def test_dependency_timeout_reports_error(ctx4096):
    """A spin bound of 1 makes the dependent items give up waiting: the
    kernel still drains (every access stays in bounds) and the batch
    reports HE_EDEVICE."""
    from paper_2506_11586_amd import heconv
    ctx, prm = ctx4096
    jobs, _ = make_jobs(ctx, prm, SHAPES_4096[:2], 400)
    b = heconv.Batch(ctx, jobs, schedule=1)
    b.set_spin_limit(1)
    b.launch(graph=False)
    with pytest.raises(heconv.HeError) as e:
        b.status()
    assert e.value.status == heconv.HE_EDEVICE
    b.close()


def test_batch_cfg2_and_fire_layers():
    """N=8192, L=3: the 64->64 layer plus three fire-module layers in one
    batch equal their standalone layer calls."""
    require_gpu()
    ensure_built()
    from paper_2506_11586_amd import heconv
    prm = oracle.Params(8192, 3, 60, 2 ** 37)
    ctx = heconv.Context(8192, heconv.gen_primes(8192, 60, 3))
    fire = synth.fire_cnn_layers()
    shapes = [(synth.WORKLOADS["conv64_56x56"]["layers"][0], 1), (fire[1], 1), (fire[3], 1), (fire[-1], 1)]
    jobs, host = make_jobs(ctx, prm, shapes, 500)
    b = heconv.Batch(ctx, jobs)
    b.launch(graph=True)
    b.status()
    for (d, B, d_in, wntt, d_out), (cv, _, _, x, K) in zip(jobs, host):
        s = ctx.sizes(d)
        ref_out = empty_words(B * s.out_cts * 2 * prm.L * prm.N)
        ctx.conv_layer(d, B, to_dev(x), wntt, ref_out)
        assert np.array_equal(to_host(d_out), to_host(ref_out)), d
    b.close()
