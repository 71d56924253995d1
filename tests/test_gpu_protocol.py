"""GPU parity of the protocol steps either side of the layer (Sec. 7;
Sec. 6.2): he_add_share and he_mask_extract against the oracle word for
word, and the whole server flow (add share -> layer -> mask + extract) on
real encryptions, whose client decryption plus the server's mask gives the
plaintext convolution of the full input mod t."""
import numpy as np
import pytest

import oracle
import synth
from synth import Stream
from tests import workload as wl
from tests.gpu_util import empty_words, require_gpu, to_dev, to_host
from tests.libload import ensure_built

pytestmark = pytest.mark.gpu
_cache = {}


def ctx_and_prm(N, L, bits, t=2 ** 37):
    key = (N, L, bits, t)
    if key not in _cache:
        require_gpu()
        ensure_built()
        from paper_2506_11586_amd import heconv
        _cache[key] = (heconv.Context(N, heconv.gen_primes(N, bits, L), t), oracle.Params(N, L, bits, t))
    return _cache[key]


def int64s(seed, purpose, n):
    """Full-range signed 64-bit values (negative and >= t included)."""
    return Stream(seed, purpose).words(n).view(np.int64)


# (N, L, bits, shape (C, H, W, M, k, stride, pad), B)
CASES = [(4096, 2, 50, (4, 16, 16, 4, 3, 1, 1), 2), (4096, 2, 50, (3, 15, 13, 5, 3, 2, 1), 2),
         (4096, 2, 50, (6, 14, 14, 3, 1, 2, 0), 3), (4096, 2, 50, (2, 12, 12, 2, 5, 1, 2), 1),
         (1024, 2, 50, (9, 20, 7, 3, 3, 1, 1), 2), (8192, 3, 60, (64, 56, 56, 64, 3, 1, 1), 1)]


def _desc(ctx, shape):
    C, H, W, M, k, stride, pad = shape
    return ctx.plan((C, H, W, M, k, k, stride, pad)), oracle.Conv(C, H, W, M, k, k, stride, pad)


@pytest.mark.parametrize("N,L,bits,shape,B", CASES)
def test_add_share_matches_oracle(N, L, bits, shape, B):
    ctx, prm = ctx_and_prm(N, L, bits)
    d, cv = _desc(ctx, shape)
    g = oracle.geometry(cv, d.Cw, d.Hw, d.Ww)
    ct = synth.uniform_mod(Stream(51, synth.UNIFORM), (B, g.CB, g.S, 2, prm.L, prm.N), prm.q)
    xs = int64s(51, synth.SHARE, B * cv.C * cv.H * cv.W).reshape(B, cv.C, cv.H, cv.W)
    dev = to_dev(ct)
    ctx.add_share(d, B, dev, to_dev(xs))
    got = to_host(dev).reshape(ct.shape)
    for b in range(B):
        assert np.array_equal(got[b], oracle.add_share(ct[b], xs[b], cv, g, prm)), b


@pytest.mark.parametrize("with_noise", [False, True])
@pytest.mark.parametrize("N,L,bits,shape,B", CASES)
def test_mask_extract_matches_oracle(N, L, bits, shape, B, with_noise):
    ctx, prm = ctx_and_prm(N, L, bits)
    d, cv = _desc(ctx, shape)
    g = oracle.geometry(cv, d.Cw, d.Hw, d.Ww)
    Ho, Wo = ctx.out_hw(d)
    assert (Ho, Wo) == (g.Ho, g.Wo)
    out = synth.uniform_mod(Stream(52, synth.UNIFORM), (B, cv.M, g.S, 2, prm.L, prm.N), prm.q)
    R = int64s(52, synth.MASK, B * cv.M * Ho * Wo).reshape(B, cv.M, Ho, Wo)
    e = int64s(52, synth.FLOOD, B * cv.M * Ho * Wo).reshape(B, cv.M, Ho, Wo) if with_noise else None
    y = empty_words(B * cv.M * prm.L * Ho * Wo)
    y.fill_(-1)
    ctx.mask_extract(d, B, to_dev(out), to_dev(R), to_dev(e) if with_noise else None, y)
    got = to_host(y).reshape(B, cv.M, prm.L, Ho, Wo)
    for b in range(B):
        want = oracle.mask_extract(out[b], R[b], None if e is None else e[b], cv, g, prm)
        assert np.array_equal(got[b], want), b


@pytest.mark.parametrize("cfg_id", ["conv4_16x16", "conv64_56x56"])
def test_server_flow_reconstructs_convolution(cfg_id):
    """Client encrypts its share; the GPU adds the server's share, runs the
    layer, masks and extracts; client decryption + mask = conv(x) mod t."""
    cfg = synth.WORKLOADS[cfg_id]
    shape = cfg["layers"][0]
    ctx, prm = ctx_and_prm(cfg["N"], cfg["L"], cfg["bits"])
    cv = wl.conv_of(shape)
    d = ctx.plan(shape)
    g = oracle.geometry(cv, d.Cw, d.Hw, d.Ww)
    n_x = cv.C * cv.H * cv.W
    xc = Stream(53, synth.INPUT).below(n_x, prm.t).astype(np.int64).reshape(cv.C, cv.H, cv.W)
    xs = Stream(53, synth.SHARE).below(n_x, prm.t).astype(np.int64).reshape(cv.C, cv.H, cv.W)
    K = Stream(53, synth.WEIGHT).ints(cv.M * cv.C * 9, *cfg["w_range"]).reshape(cv.M, cv.C, 3, 3)
    sk = wl.secret_key(53, prm.N)
    ct = wl.encrypt_input(xc, cv, g, prm, 53, sk)
    s = ctx.sizes(d)
    wntt = empty_words(s.w_words)
    ctx.encode_weights(d, to_dev(K), wntt)
    d_in = to_dev(ct)
    ctx.add_share(d, 1, d_in, to_dev(xs))
    out = empty_words(s.out_cts * 2 * prm.L * prm.N)
    ctx.conv_layer(d, 1, d_in, wntt, out)
    R = Stream(53, synth.MASK).below(cv.M * g.Ho * g.Wo, prm.t).astype(np.int64).reshape(cv.M, g.Ho, g.Wo)
    y = empty_words(cv.M * prm.L * g.Ho * g.Wo)
    ctx.mask_extract(d, 1, out, to_dev(R), None, y)
    out_h = to_host(out).reshape(cv.M, g.S, 2, prm.L, prm.N)
    client = oracle.decrypt_extracted(out_h[:, :, 0], to_host(y).reshape(cv.M, prm.L, g.Ho, g.Wo), sk, cv, g, prm)
    want = np.mod(oracle.plain_conv(xc + xs, K, cv.stride, cv.pad), prm.t)
    assert np.array_equal(np.mod(client.astype(object) + R, prm.t), want.astype(object))


def test_protocol_errors():
    from paper_2506_11586_amd import heconv
    ctx, prm = ctx_and_prm(4096, 2, 50)
    d, cv = _desc(ctx, (4, 16, 16, 4, 3, 1, 1))
    L = heconv.lib()
    assert L.he_add_share(ctx.handle, heconv.ctypes.byref(d), 1, None, None, None) == heconv.HE_EINVAL
    assert L.he_mask_extract(ctx.handle, heconv.ctypes.byref(d), 1, None, None, None, None, None) == heconv.HE_EINVAL
    assert L.he_add_share(ctx.handle, heconv.ctypes.byref(d), 0, None, None, None) == heconv.HE_OK  # B = 0
    bad = heconv.ConvDesc(*d.shape(), 5, d.Hw, d.Ww)  # Cw > C
    assert L.he_add_share(ctx.handle, heconv.ctypes.byref(bad), 1, None, None, None) == heconv.HE_ESHAPE
    ctx_t0, _ = ctx_and_prm(4096, 2, 50, t=1)  # no usable plaintext modulus: the layer path still works
    d0 = ctx_t0.plan((4, 16, 16, 4, 3, 3, 1, 1))
    assert L.he_add_share(ctx_t0.handle, heconv.ctypes.byref(d0), 1, None, None, None) == heconv.HE_EPARAM
    assert L.he_mask_extract(ctx_t0.handle, heconv.ctypes.byref(d0), 1, None, None, None, None,
                             None) == heconv.HE_EPARAM
