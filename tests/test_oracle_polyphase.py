"""Pins for the polyphase form of strided convolutions (a fusion variant of
the layer): the stride-1 conv on the phase channels with the rearranged
kernel equals the strided conv, by the plain integer convolution, over
strides 2 and 3, kernels 1-7, paddings 0-3 and odd and even sizes; the
equivalent descriptor's sizes are written out for the two CNN stems."""
import numpy as np
import pytest

import oracle
import synth
from synth import Stream

SHAPES = [(3, 16, 16, 4, 3, 3, 2, 1), (2, 15, 13, 3, 3, 3, 2, 1), (3, 23, 23, 2, 7, 7, 2, 3), (2, 9, 11, 3, 5, 5, 2, 2),
          (4, 12, 12, 2, 1, 1, 2, 0), (2, 14, 10, 2, 4, 2, 2, 0), (3, 17, 17, 2, 3, 3, 3, 1), (1, 20, 20, 2, 5, 3, 3, 2)]


@pytest.mark.parametrize("shape", SHAPES)
def test_polyphase_equals_strided_conv(shape):
    cv = oracle.Conv(*shape)
    x = Stream(130, synth.INPUT).ints(cv.C * cv.H * cv.W, -50, 50).reshape(cv.C, cv.H, cv.W)
    K = Stream(131, synth.WEIGHT).ints(cv.M * cv.C * cv.kh * cv.kw, -9, 9).reshape(cv.M, cv.C, cv.kh, cv.kw)
    want = oracle.plain_conv(x, K, cv.stride, cv.pad)
    pc = oracle.polyphase_conv(cv)
    got = oracle.plain_conv(oracle.polyphase_input(x, cv), oracle.polyphase_weights(K, cv), 1, 0)
    assert got.shape[1] >= want.shape[1] and got.shape[2] >= want.shape[2]
    assert np.array_equal(got[:, :want.shape[1], :want.shape[2]], want)
    assert pc.stride == 1 and pc.pad == 0 and pc.C == cv.stride ** 2 * cv.C


def test_polyphase_descriptors_of_the_stems():
    assert oracle.polyphase_conv(oracle.Conv(3, 224, 224, 64, 3, 3, 2, 1)) == oracle.Conv(12, 113, 113, 64, 2, 2, 1, 0)
    assert oracle.polyphase_conv(oracle.Conv(3, 224, 224, 64, 7, 7, 2, 3)) == oracle.Conv(12, 115, 115, 64, 4, 4, 1, 0)


def test_polyphase_layer_through_the_encrypted_flow(prm4096):
    """A 3x3 stride-2 layer in polyphase form through packing, the NTT-domain
    layer and decryption (N=4096, L=2) gives the strided conv."""
    from tests import workload as wl
    cv = oracle.Conv(3, 20, 20, 4, 3, 3, 2, 1)
    pc = oracle.polyphase_conv(cv)
    x = Stream(132, synth.INPUT).ints(cv.C * cv.H * cv.W, -2 ** 7, 2 ** 7).reshape(cv.C, cv.H, cv.W)
    K = Stream(133, synth.WEIGHT).ints(cv.M * cv.C * 9, -2 ** 7, 2 ** 7).reshape(cv.M, cv.C, 3, 3)
    g = oracle.plan_conv(pc, prm4096.N, prm4096.L)
    sk = wl.secret_key(134, prm4096.N)
    ct = wl.encrypt_input(oracle.polyphase_input(x, cv), pc, g, prm4096, 134, sk)
    w_ntt = oracle.encode_weights(oracle.polyphase_weights(K, cv), pc, g, prm4096)
    out = oracle.conv_layer_ntt(ct[None], w_ntt, 1, g, pc.M, prm4096)[0]
    dec = oracle.bfv_decrypt(out.reshape(-1, 2, prm4096.L, prm4096.N), sk, prm4096)
    y = oracle.assemble_output(dec.reshape(pc.M, g.S, prm4096.N)[:, :, oracle.output_slots(g)], pc, g)
    want = oracle.plain_conv(x, K, 2, 1)
    assert np.array_equal(y[:, :want.shape[1], :want.shape[2]], want)
