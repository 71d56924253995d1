"""GPU: the request server -- every result is the same alone and in the mix
(bit-exact), queued requests of one layer merge into one launch, served
outputs equal the oracle's layer (and one real encryption decrypts to the
plaintext conv), and the HBM budget holds."""
import numpy as np
import pytest

import synth
from synth import Stream
from tests.gpu_util import empty_words, require_gpu, to_dev, to_host
from tests.libload import ensure_built

pytestmark = pytest.mark.gpu

SHAPES = [  # (N, L, bits, shape)
    (4096, 2, 50, (4, 16, 16, 4, 3, 3, 1, 1)),
    (4096, 2, 50, (8, 11, 9, 5, 3, 3, 2, 1)),
    (8192, 3, 60, (64, 56, 56, 64, 3, 3, 1, 1)),
    (8192, 3, 60, (16, 55, 55, 64, 1, 1, 1, 0)),
    (8192, 3, 60, (48, 13, 13, 192, 3, 3, 1, 1)),
]


def build_server(n_streams, budget):
    import torch
    from paper_2506_11586_amd import heconv, serving
    ctxs, layers = {}, []
    for i, (N, L, bits, shape) in enumerate(SHAPES):
        if (N, L) not in ctxs:
            ctxs[(N, L)] = heconv.Context(N, heconv.gen_primes(N, bits, L))
        ctx = ctxs[(N, L)]
        C, M, kh, kw = shape[0], shape[3], shape[4], shape[5]
        K = Stream(700 + i, synth.WEIGHT).ints(M * C * kh * kw, -2 ** 12, 2 ** 12)
        layers.append(serving.make_layer(ctx, shape, to_dev(K)))
    torch.cuda.synchronize()
    return serving.Server(layers, n_streams=n_streams, hbm_budget=budget), layers


def make_requests(layers, n, rate, seed):
    import torch
    from paper_2506_11586_amd import serving
    mix = Stream(seed, synth.MIX).below(n, len(layers)).astype(int)
    times = serving.poisson_arrivals(rate, n, Stream(seed, synth.ARRIVAL).uniform_f64(n))
    reqs = []
    for i in range(n):
        lay = layers[mix[i]]
        words = synth.uniform_mod(Stream(seed * 1000 + i, synth.UNIFORM),
                                  (lay.in_words // lay.ctx.N // lay.ctx.L, lay.ctx.L, lay.ctx.N), lay.ctx.q)
        host = torch.from_numpy(words.view(np.int64).ravel().copy()).pin_memory()
        reqs.append(serving.Request(i, int(mix[i]), float(times[i]), host))
    return reqs


def alone_outputs(layers, reqs):
    """Each request by itself: default stream, fresh buffers, one image."""
    out = []
    for r in reqs:
        lay = layers[r.layer]
        d_in = r.host_in.cuda()
        d_out = empty_words(lay.out_words)
        lay.ctx.conv_layer(lay.desc, 1, d_in, lay.wntt, d_out)
        out.append(to_host(d_out).copy())
    return out


def test_alone_equals_in_the_mix():
    require_gpu()
    ensure_built()
    server, layers = build_server(n_streams=4, budget=200e9)
    reqs = make_requests(layers, 40, rate=5000.0, seed=41)
    alone = alone_outputs(layers, reqs)
    # in the mix: open loop at 5000 req/s over 4 streams
    st = server.run(reqs, keep_outputs=True)
    assert st.n == len(reqs) and st.max_inflight > 1
    for r, a in zip(reqs, alone):
        assert np.array_equal(to_host(r.result), a), r.rid
    assert server.used <= 200e9
    # saturated (all at once): queued requests of a layer share launches
    st = server.run(reqs, closed_loop=True, keep_outputs=True)
    assert st.launches < len(reqs) and max(r.batch for r in reqs) > 1
    for r, a in zip(reqs, alone):
        assert np.array_equal(to_host(r.result), a), (r.rid, r.batch)


def test_served_outputs_match_oracle():
    """Merged launches against the oracle: one served request of each layer
    (each in a launch with others of its layer) equals oracle.conv_layer_ntt
    on its input word for word; and a real encryption of a packed input to
    the small layer, served in the mix, decrypts to the plaintext conv."""
    require_gpu()
    ensure_built()
    import torch
    import oracle
    from tests import workload as wl
    server, layers = build_server(n_streams=4, budget=200e9)
    reqs = make_requests(layers, 30, rate=1e6, seed=45)
    # the small 4->4 layer: a real encryption as one more request
    lay0 = layers[0]
    N, L = lay0.ctx.N, lay0.ctx.L
    prm = oracle.Params(N, L, 50, 2 ** synth.T_BITS)
    assert prm.q == lay0.ctx.q
    cv = oracle.Conv(*lay0.shape)
    g = oracle.geometry(cv, lay0.desc.Cw, lay0.desc.Hw, lay0.desc.Ww)
    x = Stream(46, synth.INPUT).ints(cv.C * cv.H * cv.W, 0, 2 ** 37).reshape(cv.C, cv.H, cv.W)
    sk = wl.secret_key(46, N)
    ct = wl.encrypt_input(x, cv, g, prm, 46, sk)
    from paper_2506_11586_amd import serving
    enc = serving.Request(len(reqs), 0, 0.0, torch.from_numpy(ct.view(np.int64).ravel().copy()).pin_memory())
    reqs.append(enc)
    st = server.run(reqs, closed_loop=True, keep_outputs=True)
    assert st.launches < len(reqs) and enc.batch > 1
    checked = set()
    for r in reqs:
        if r.layer in checked or r is enc or r.batch < 2:
            continue
        checked.add(r.layer)
        lay = layers[r.layer]
        p = oracle.Params(lay.ctx.N, lay.ctx.L, 60 if lay.ctx.N == 8192 else 50, 2 ** synth.T_BITS)
        assert p.q == lay.ctx.q
        c = oracle.Conv(*lay.shape)
        gg = oracle.geometry(c, lay.desc.Cw, lay.desc.Hw, lay.desc.Ww)
        K = Stream(700 + r.layer, synth.WEIGHT).ints(c.M * c.C * c.kh * c.kw, -2 ** 12, 2 ** 12)
        w_ntt = oracle.encode_weights(K.reshape(c.M, c.C, c.kh, c.kw), c, gg, p)
        xin = r.host_in.numpy().view(np.uint64).reshape(1, gg.CB, gg.S, 2, p.L, p.N)
        want = oracle.conv_layer_ntt(xin, w_ntt, 1, gg, c.M, p)
        assert np.array_equal(to_host(r.result).reshape(want.shape), want), (r.rid, r.layer, r.batch)
    assert len(checked) >= 3
    K0 = Stream(700, synth.WEIGHT).ints(cv.M * cv.C * cv.kh * cv.kw, -2 ** 12, 2 ** 12).reshape(
        cv.M, cv.C, cv.kh, cv.kw)
    got = to_host(enc.result).reshape(cv.M, g.S, 2, L, N)
    y = wl.decrypt_output(got, cv, g, prm, sk)
    assert np.array_equal(y, oracle.centre_mod(oracle.plain_conv(x, K0, cv.stride, cv.pad), prm.t))


def test_budget_limits_admission():
    """With a budget that fits the weights and one launch buffer of the
    largest layer only, requests queue for buffers, never exceed the budget,
    and still all complete with the same results."""
    require_gpu()
    ensure_built()
    server, layers = build_server(n_streams=4, budget=200e9)
    server.budget = server.resident + max(server._buf_bytes(i) for i in range(len(layers)))
    reqs = make_requests(layers, 12, rate=1e5, seed=43)
    alone = alone_outputs(layers, reqs)
    st = server.run(reqs, closed_loop=True, keep_outputs=True)
    assert st.n == 12 and server.used <= server.budget
    assert all(np.isfinite(r.t_done) for r in reqs)
    for r, a in zip(reqs, alone):
        assert np.array_equal(to_host(r.result), a), r.rid


def test_budget_too_small_for_weights():
    require_gpu()
    ensure_built()
    from paper_2506_11586_amd import serving
    _, layers = build_server(n_streams=1, budget=200e9)
    with pytest.raises(MemoryError):
        serving.Server(layers, hbm_budget=1e6)


def test_protocol_mode_equals_direct_calls():
    """Protocol mode (share folded in, layer, masked extraction; requests of
    one layer merged into one launch) gives the same extracted words as the
    three calls made directly for each request."""
    require_gpu()
    ensure_built()
    import torch
    from paper_2506_11586_amd import serving
    _, layers = build_server(n_streams=4, budget=200e9)
    server = serving.Server(layers, n_streams=4, hbm_budget=200e9, protocol=True)
    reqs = make_requests(layers, 24, rate=5000.0, seed=43)
    for r in reqs:
        lay = layers[r.layer]
        r.host_share = torch.from_numpy(Stream(4300 + r.rid, synth.SHARE).words(lay.share_words).view(np.int64)
                                        .copy()).pin_memory()
        r.host_mask = torch.from_numpy(Stream(4300 + r.rid, synth.MASK).words(lay.mask_words).view(np.int64)
                                       .copy()).pin_memory()
    direct = []
    for r in reqs:
        lay = layers[r.layer]
        d_in, d_out, y = r.host_in.cuda(), empty_words(lay.out_words), empty_words(lay.y_words)
        lay.ctx.add_share(lay.desc, 1, d_in, r.host_share.cuda())
        lay.ctx.conv_layer(lay.desc, 1, d_in, lay.wntt, d_out)
        lay.ctx.mask_extract(lay.desc, 1, d_out, r.host_mask.cuda(), None, y)
        direct.append(to_host(y).copy())
    st = server.run(reqs, closed_loop=True, keep_outputs=True)
    assert st.n == len(reqs) and max(r.batch for r in reqs) > 1
    for r, want in zip(reqs, direct):
        assert np.array_equal(to_host(r.result), want), r.rid
