"""GPU: the batch executor (three grids per chain over many layer solves,
eager or as one hipGraph) equals he_conv_layer job by job, and the oracle
word for word."""
import numpy as np
import pytest

import oracle
import synth
from synth import Stream
from tests.gpu_util import empty_words, require_gpu, to_dev, to_host
from tests.libload import ensure_built

pytestmark = pytest.mark.gpu

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


@pytest.mark.parametrize("schedule", [1, 2, 3, 4])
@pytest.mark.parametrize("graph", [False, True])
def test_batch_equals_layer_and_oracle(ctx4096, schedule, graph):
    from paper_2506_11586_amd import heconv
    ctx, prm = ctx4096
    jobs, host = make_jobs(ctx, prm, SHAPES_4096, 100 + schedule)
    b = heconv.Batch(ctx, jobs, schedule=schedule)
    assert b.n_items > 0 and b.n_chains == min(schedule, 2)
    b.launch(graph=graph)
    b.status()
    for (d, B, d_in, wntt, d_out), (cv, _, _, x, K) in zip(jobs, host):
        g = oracle.geometry(cv, d.Cw, d.Hw, d.Ww)
        got = to_host(d_out).reshape(B, cv.M, g.S, 2, prm.L, prm.N)
        ref_out = empty_words(got.size)
        ctx.conv_layer(d, B, to_dev(x), wntt, ref_out)
        assert np.array_equal(got, to_host(ref_out).reshape(got.shape))
        w_ntt = oracle.encode_weights(K, cv, g, prm)
        want = oracle.conv_layer_ntt(x.reshape(B, g.CB, g.S, 2, prm.L, prm.N), w_ntt, B, g, cv.M, prm)
        assert np.array_equal(got, want)
    b.close()


@pytest.mark.parametrize("lds", [0, 3])
@pytest.mark.parametrize("tile", [(4, 2), (2, 4), (2, 2), (4, 4), (6, 4), (8, 4), (4, 8)])
def test_batch_forced_tiles_and_timed_launch(ctx4096, tile, lds):
    """Every register tile the batch MAC is built for, forced through the
    context's tuning, gives the oracle's words; the timed eager launch gives
    the same words and one duration per grid.  (6,4), (8,4) and (4,8) exist
    for the streamed MAC only (lds 0 falls back to (4,4))."""
    from paper_2506_11586_amd import heconv
    ctx, prm = ctx4096
    before = ctx.get_tuning().as_dict()
    ctx.set_tuning(mac_mt=tile[0], mac_rt=tile[1], mac_lds=lds)
    jobs, host = make_jobs(ctx, prm, SHAPES_4096, 200 + tile[0] * 10 + tile[1])
    pristine = [j[2].clone() for j in jobs]
    b = heconv.Batch(ctx, jobs, schedule=2)
    ctx.set_tuning(**before)
    ms = b.launch_timed()
    assert len(ms) == b.n_chains and all(len(r) == 3 and min(r) >= 0 for r in ms)
    assert sum(ms[0]) > 0
    for (d, B, d_in, wntt, d_out), (cv, _, _, x, K) in zip(jobs, host):
        g = oracle.geometry(cv, d.Cw, d.Hw, d.Ww)
        got = to_host(d_out).reshape(B, cv.M, g.S, 2, prm.L, prm.N)
        w_ntt = oracle.encode_weights(K, cv, g, prm)
        want = oracle.conv_layer_ntt(x.reshape(B, g.CB, g.S, 2, prm.L, prm.N), w_ntt, B, g, cv.M, prm)
        assert np.array_equal(got, want), (tile, cv)
    timed_out = [to_host(j[4]).copy() for j in jobs]
    for j, p in zip(jobs, pristine):
        j[2].copy_(p)
        j[4].fill_(-1)
    b.launch(graph=True)
    b.status()
    for j, t in zip(jobs, timed_out):
        assert np.array_equal(to_host(j[4]), t)
    b.close()


def test_graph_replays_match_eager(ctx4096):
    """The captured graph replayed several times, with eager work (restoring
    the inputs, clearing the outputs) and synchronisation between replays:
    every replay equals the eager launch."""
    import torch
    from paper_2506_11586_amd import heconv
    ctx, prm = ctx4096
    jobs, host = make_jobs(ctx, prm, SHAPES_4096, 300)
    pristine = [j[2].clone() for j in jobs]
    b = heconv.Batch(ctx, jobs, schedule=2)
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


def test_batch_rejects_disabled_and_bad_input(ctx4096):
    from paper_2506_11586_amd import heconv
    ctx, prm = ctx4096
    jobs, _ = make_jobs(ctx, prm, SHAPES_4096[:1], 400)
    for sched in (0, 5):
        with pytest.raises(heconv.HeError) as e:
            heconv.Batch(ctx, jobs, schedule=sched)
        assert e.value.status == heconv.HE_EINVAL


def test_batch_rejects_grids_beyond_one_launch(ctx4096):
    """A batch whose MAC grid would exceed 2^32 - 1 work-items (here 300,000
    images of the small layer with 2x2 tiles: 19.2 million tiles of 256
    threads) is refused with HE_ESHAPE when it is created; nothing is
    launched, so the buffer addresses are never used."""
    import ctypes
    from paper_2506_11586_amd import heconv
    ctx, prm = ctx4096
    d = ctx.plan(SHAPES_4096[0][0])
    before = ctx.get_tuning().as_dict()
    ctx.set_tuning(mac_mt=2, mac_rt=2)
    arr = (heconv._Job * 1)()
    arr[0] = heconv._Job(d, 300000, 0x1000, 0x2000, 0x3000)
    h = ctypes.c_void_p()
    s = heconv.lib().he_batch_create(ctx.handle, arr, 1, 1, ctypes.byref(h))
    ctx.set_tuning(**before)
    assert s == heconv.HE_ESHAPE and not h.value


def test_batch_cfg2_and_fire_layers():
    """N=8192, L=3: the 64->64 layer plus three fire-module layers in one
    batch (two chains, graph) equal their standalone layer calls."""
    require_gpu()
    ensure_built()
    from paper_2506_11586_amd import heconv
    prm = oracle.Params(8192, 3, 60, 2 ** 37)
    ctx = heconv.Context(8192, heconv.gen_primes(8192, 60, 3))
    fire = synth.fire_cnn_layers()
    shapes = [(synth.WORKLOADS["conv64_56x56"]["layers"][0], 1), (fire[1], 1), (fire[3], 1), (fire[-1], 1)]
    jobs, host = make_jobs(ctx, prm, shapes, 500)
    b = heconv.Batch(ctx, jobs, schedule=2)
    b.launch(graph=True)
    b.status()
    for (d, B, d_in, wntt, d_out), (cv, _, _, x, K) in zip(jobs, host):
        s = ctx.sizes(d)
        ref_out = empty_words(B * s.out_cts * 2 * prm.L * prm.N)
        ctx.conv_layer(d, B, to_dev(x), wntt, ref_out)
        assert np.array_equal(to_host(d_out), to_host(ref_out)), d
    b.close()


def test_full_fire_cnn_batched_sampled_against_oracle():
    """The whole fire-module CNN (26 convs at 224 input, batch 1, N=8192,
    L=3, the weights 3.9 GiB resident) as one batch (two chains, hipGraph):
    three sampled output words of every layer equal the oracle's layer by
    definition (one coefficient of the negacyclic sum over channel blocks)."""
    require_gpu()
    ensure_built()
    from paper_2506_11586_amd import heconv
    cfg = synth.WORKLOADS["fire_cnn"]
    prm = oracle.Params(cfg["N"], cfg["L"], cfg["bits"], 2 ** 37)
    ctx = heconv.Context(cfg["N"], heconv.gen_primes(cfg["N"], cfg["bits"], cfg["L"]))
    jobs, host = make_jobs(ctx, prm, [(s, 1) for s in cfg["layers"]], 900)
    b = heconv.Batch(ctx, jobs, schedule=2)
    b.launch(graph=True)
    b.status()
    rng = Stream(901, synth.MIX)
    for (d, B, d_in, wntt, d_out), (cv, _, _, x, K) in zip(jobs, host):
        g = oracle.geometry(cv, d.Cw, d.Hw, d.Ww)
        got = to_host(d_out).reshape(1, cv.M, g.S, 2, prm.L, prm.N)
        xin = x.reshape(1, g.CB, g.S, 2, prm.L, prm.N)
        for _ in range(3):
            m, s, c, l, k = (int(rng.below(1, v)[0]) for v in (cv.M, g.S, 2, prm.L, prm.N))
            wc = oracle.pack_weights(K[m:m + 1], cv, g, prm)
            assert int(got[0, m, s, c, l, k]) == oracle.conv_layer_coeff(xin, wc, g, prm, 0, 0, s, c, l, k), \
                (cv, m, s, c, l, k)
    b.close()
    ctx.close()


# Shapes whose channel blocks span one chunk of the streamed MAC (CB <= 8),
# two (9-16) and three (17-24), so that carries between chunks and tile
# boundaries inside a workgroup's stream are exercised, and shapes with
# several spatial tiles (a tile's row pairs then span tiles and images);
# N=4096, L=2.
SHAPES_DEEP = [
    ((256, 12, 12, 8, 3, 3, 1, 1), 2),
    ((600, 5, 5, 6, 1, 1, 1, 0), 3),
    ((4000, 4, 4, 7, 1, 1, 1, 0), 2),
    ((6000, 4, 4, 3, 1, 1, 1, 0), 2),
    ((40, 9, 9, 10, 3, 3, 2, 1), 4),
    ((8, 64, 64, 5, 3, 3, 1, 1), 3),   # 3 spatial tiles: row pairs cross tiles and images
    ((3, 60, 60, 4, 7, 7, 2, 3), 5),   # 2 spatial tiles, 20 rows
]


@pytest.fixture(scope="module")
def deep_jobs(ctx4096):
    ctx, prm = ctx4096
    jobs, host = make_jobs(ctx, prm, SHAPES_DEEP, 500)
    cbs = sorted({ctx.sizes(j[0]).CB for j in jobs})
    assert cbs[0] <= 8 and any(8 < c <= 16 for c in cbs) and cbs[-1] > 16, cbs
    pristine = [j[2].clone() for j in jobs]
    want = []
    for (d, B, d_in, wntt, d_out), (cv, _, _, x, K) in zip(jobs, host):
        g = oracle.geometry(cv, d.Cw, d.Hw, d.Ww)
        w_ntt = oracle.encode_weights(K, cv, g, prm)
        want.append(oracle.conv_layer_ntt(x.reshape(B, g.CB, g.S, 2, prm.L, prm.N), w_ntt, B, g, cv.M, prm).reshape(-1))
    return jobs, pristine, want


@pytest.mark.parametrize("tile,lds,tiles", [
    ((4, 4), 3, 0), ((4, 4), 2, 1), ((4, 4), 4, 3), ((4, 4), 3, 16),
    ((6, 4), 3, 0), ((6, 4), 2, 2), ((6, 4), 4, 5),
    ((8, 4), 3, 0), ((4, 8), 3, 2), ((4, 2), 3, 0), ((2, 4), 2, 7), ((2, 2), 4, 1)])
def test_streamed_mac_chunks_and_tile_lists(ctx4096, deep_jobs, tile, lds, tiles):
    """The streamed MAC (tiles decoded on the host, several per workgroup,
    loads running ahead across tile boundaries, a fold every 8 channel blocks
    carried in registers) on layers of 4 to 24 channel blocks: every output
    word equals the oracle's, for each tile, LDS depth and tiles per
    workgroup."""
    from paper_2506_11586_amd import heconv
    ctx, prm = ctx4096
    jobs, pristine, want = deep_jobs
    before = ctx.get_tuning().as_dict()
    ctx.set_tuning(mac_mt=tile[0], mac_rt=tile[1], mac_lds=lds, mac_tiles=tiles)
    b = heconv.Batch(ctx, jobs, schedule=1)
    ctx.set_tuning(**before)
    for j, p in zip(jobs, pristine):
        j[2].copy_(p)
        j[4].fill_(-1)
    b.launch(graph=True)
    b.status()
    for j, w in zip(jobs, want):
        assert np.array_equal(to_host(j[4]), w), (tile, lds, tiles, j[0])
    b.close()


# Jobs that fill a 2x2 wave grid of the streamed MAC (at least 8 rows and
# 12 output channels each): one to three chunks of channel blocks, ragged
# rows and channels, several spatial tiles; N=4096, L=2.
SHAPES_GRID = [
    ((64, 12, 12, 16, 3, 3, 1, 1), 4),
    ((600, 5, 5, 13, 1, 1, 1, 0), 5),
    ((4000, 4, 4, 12, 1, 1, 1, 0), 4),
    ((6000, 4, 4, 14, 1, 1, 1, 0), 4),
    ((8, 64, 64, 12, 3, 3, 1, 1), 3),
    ((3, 60, 60, 16, 7, 7, 2, 3), 5),
]


@pytest.fixture(scope="module")
def grid_jobs(ctx4096):
    ctx, prm = ctx4096
    jobs, host = make_jobs(ctx, prm, SHAPES_GRID, 700)
    pristine = [j[2].clone() for j in jobs]
    want = []
    for (d, B, d_in, wntt, d_out), (cv, _, _, x, K) in zip(jobs, host):
        g = oracle.geometry(cv, d.Cw, d.Hw, d.Ww)
        w_ntt = oracle.encode_weights(K, cv, g, prm)
        want.append(oracle.conv_layer_ntt(x.reshape(B, g.CB, g.S, 2, prm.L, prm.N), w_ntt, B, g, cv.M, prm).reshape(-1))
    return jobs, pristine, want


@pytest.mark.parametrize("tile,lds,tiles", [
    ((6, 4), 3, 0), ((6, 4), 2, 3), ((6, 4), 4, 1), ((4, 4), 3, 0), ((4, 4), 2, 5), ((4, 2), 3, 2),
    ((2, 4), 4, 0), ((2, 2), 3, 1)])
def test_streamed_mac_wave_grid(ctx4096, grid_jobs, tile, lds, tiles):
    """The streamed MAC with its four waves as a 2x2 grid sharing the rows
    they load (one workgroup barrier per channel block): the batch picks the
    grid for these jobs, and every output word equals the oracle's."""
    from paper_2506_11586_amd import heconv
    ctx, prm = ctx4096
    jobs, pristine, want = grid_jobs
    before = ctx.get_tuning().as_dict()
    ctx.set_tuning(mac_mt=tile[0], mac_rt=tile[1], mac_lds=lds, mac_tiles=tiles, mac_grid=1)
    b = heconv.Batch(ctx, jobs, schedule=1)
    ctx.set_tuning(**before)
    assert b.mac_form["grid"] == 1 and (b.mac_form["mt"], b.mac_form["rt"]) == tile, b.mac_form
    for j, p in zip(jobs, pristine):
        j[2].copy_(p)
        j[4].fill_(-1)
    b.launch(graph=True)
    b.status()
    for j, w in zip(jobs, want):
        assert np.array_equal(to_host(j[4]), w), (tile, lds, tiles, j[0])
    b.close()


def test_wave_grid_falls_back_when_jobs_do_not_fill_it(ctx4096):
    """A job with fewer rows than the grid covers keeps the per-wave stream."""
    from paper_2506_11586_amd import heconv
    ctx, prm = ctx4096
    jobs, host = make_jobs(ctx, prm, [((8, 11, 9, 16, 3, 3, 2, 1), 1)], 800)  # 2 rows
    before = ctx.get_tuning().as_dict()
    ctx.set_tuning(mac_mt=4, mac_rt=4, mac_lds=3, mac_grid=1)
    b = heconv.Batch(ctx, jobs, schedule=1)
    ctx.set_tuning(**before)
    assert b.mac_form["grid"] == 0
    b.close()


def test_batch_default_tile_for_jobs_of_few_rows(ctx4096):
    """With the context's tile left to the shape (mac_mt = 0): a job of two
    ciphertext rows (one image, one spatial tile) gives the batch 4x2 tiles,
    a job of fewer than four output channels 2x2; every output word equals
    the oracle's."""
    from paper_2506_11586_amd import heconv
    ctx, prm = ctx4096
    cases = [([((8, 11, 9, 16, 3, 3, 2, 1), 1), ((16, 12, 12, 8, 3, 3, 1, 1), 2)], (4, 2)),
             ([((8, 11, 9, 3, 3, 3, 1, 1), 2), ((16, 12, 12, 8, 3, 3, 1, 1), 2)], (2, 2))]
    before = ctx.get_tuning().as_dict()
    for shapes, tile in cases:
        jobs, host = make_jobs(ctx, prm, shapes, 990)
        ctx.set_tuning(mac_mt=0, mac_rt=0)
        b = heconv.Batch(ctx, jobs, schedule=1)
        ctx.set_tuning(**before)
        assert (b.mac_form["mt"], b.mac_form["rt"]) == tile, (shapes, b.mac_form)
        b.launch(graph=False)
        b.status()
        for (d, B, d_in, wntt, d_out), (cv, _, _, x, K) in zip(jobs, host):
            g = oracle.geometry(cv, d.Cw, d.Hw, d.Ww)
            want = oracle.conv_layer_ntt(x.reshape(B, g.CB, g.S, 2, prm.L, prm.N), oracle.encode_weights(K, cv, g, prm),
                                         B, g, cv.M, prm)
            assert np.array_equal(to_host(d_out), want.reshape(-1)), (shapes, cv)
        b.close()
