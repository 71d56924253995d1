"""GPU parity of the polyphase form of strided convolutions (a fusion
variant of the layer): the weight and input rearrangements against the
oracle, and the fire-module CNN's first layer (3x3 stride 2 at 224) run as
its polyphase stride-1 layer on real encryptions decrypts to the strided
integer conv, as does the stride-1 + subsample form."""
import numpy as np
import pytest

import oracle
import synth
from synth import Stream
from tests import workload as wl
from tests.gpu_util import empty_words, require_gpu, to_dev, to_host
from tests.libload import ensure_built

pytestmark = pytest.mark.gpu

SHAPES = [(3, 16, 16, 4, 3, 3, 2, 1), (2, 15, 13, 3, 3, 3, 2, 1), (3, 23, 23, 2, 7, 7, 2, 3), (2, 9, 11, 3, 5, 5, 2, 2),
          (3, 17, 17, 2, 3, 3, 3, 1), (4, 12, 12, 2, 1, 1, 2, 0)]


@pytest.mark.parametrize("shape", SHAPES)
def test_polyphase_transforms_match_oracle(shape):
    require_gpu()
    ensure_built()
    from paper_2506_11586_amd import heconv
    cv = oracle.Conv(*shape)
    pc = oracle.polyphase_conv(cv)
    B = 2
    x = Stream(140, synth.INPUT).ints(B * cv.C * cv.H * cv.W, -2 ** 40, 2 ** 40).reshape(B, cv.C, cv.H, cv.W)
    K = Stream(141, synth.WEIGHT).ints(cv.M * cv.C * cv.kh * cv.kw, -99, 99).reshape(cv.M, cv.C, cv.kh, cv.kw)
    xp = empty_words(B * pc.C * pc.H * pc.W)
    xp.fill_(7)
    heconv.polyphase_input(shape, B, to_dev(x), xp)
    want = np.stack([oracle.polyphase_input(x[b], cv) for b in range(B)])
    assert np.array_equal(xp.cpu().numpy().reshape(want.shape), want)
    wp = empty_words(pc.M * pc.C * pc.kh * pc.kw)
    wp.fill_(7)
    heconv.polyphase_weights(shape, to_dev(K), wp)
    assert np.array_equal(wp.cpu().numpy().reshape(pc.M, pc.C, pc.kh, pc.kw), oracle.polyphase_weights(K, cv))


def test_fire_conv1_polyphase_decrypts_to_strided_conv():
    require_gpu()
    ensure_built()
    from paper_2506_11586_amd import heconv
    cfg = synth.WORKLOADS["fire_cnn"]
    N, L = cfg["N"], cfg["L"]
    prm = oracle.Params(N, L, cfg["bits"], 2 ** 37)
    ctx = heconv.Context(N, heconv.gen_primes(N, cfg["bits"], L))
    shape = cfg["layers"][0]
    assert shape == (3, 224, 224, 64, 3, 3, 2, 1)
    cv = oracle.Conv(*shape)
    x = Stream(142, synth.INPUT).ints(cv.C * cv.H * cv.W, -2 ** 12, 2 ** 12).reshape(cv.C, cv.H, cv.W)
    K = Stream(143, synth.WEIGHT).ints(cv.M * cv.C * 9, -2 ** 12, 2 ** 12).reshape(cv.M, cv.C, 3, 3)
    want = oracle.plain_conv(x, K, 2, 1)
    sk = wl.secret_key(144, N)
    skn = empty_words(L * N)
    ctx.key_encode(to_dev(np.asarray(sk, dtype=np.int64)), skn)
    results = {}
    for form in ("polyphase", "strided"):
        if form == "polyphase":
            pshape = heconv.polyphase_shape(shape)
            pcv = oracle.Conv(*pshape)
            d = ctx.plan(pshape)
            wdev = empty_words(pcv.M * pcv.C * pcv.kh * pcv.kw)
            heconv.polyphase_weights(shape, to_dev(K), wdev)
            xin, lcv = oracle.polyphase_input(x, cv), pcv
        else:
            d = ctx.plan(shape)
            wdev, xin, lcv = to_dev(K), x, cv
        s = ctx.sizes(d)
        g = oracle.geometry(lcv, d.Cw, d.Hw, d.Ww)
        wntt = empty_words(s.w_words)
        ctx.encode_weights(d, wdev, wntt)
        ct = wl.encrypt_input(xin, lcv, g, prm, 145, sk)
        out = empty_words(s.out_cts * 2 * L * N)
        ctx.conv_layer(d, 1, to_dev(ct), wntt, out)
        dec = empty_words(s.out_cts * N)
        ctx.decrypt(s.out_cts, out, skn, dec, empty_words(s.out_cts * L * N))
        vals = dec.cpu().numpy().reshape(lcv.M, g.S, N)[:, :, oracle.output_slots(g)]
        y = oracle.assemble_output(vals, lcv, g)
        results[form] = (s.out_cts, y[:, :want.shape[1], :want.shape[2]])
    assert results["polyphase"][0] < results["strided"][0]  # fewer output ciphertexts
    for form, (_, y) in results.items():
        assert np.array_equal(y, want), form
    ctx.close()
