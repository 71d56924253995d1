"""GPU: the two CNN workloads through the batch executor, every output word
against the oracle's layer (Sec. 6.2 flow: forward NTT, MAC over channel
blocks against NTT-preprocessed weights, inverse NTT), and the outputs
decrypted against the plaintext integer convolution mod t.

  - the fire-module CNN: all 26 convolutions at 224 input, one image, in one
    batch (two chains, one hipGraph launch);
  - the bottleneck residual CNN at 16 images: the 7x7/2 stem and the first
    block of every stage (1x1, 3x3 -- strided in stages 2-4 -- 1x1 and the
    projection shortcut, strided 1x1 in stages 2-4), 17 layers in one batch.

Inputs are real encryptions (oracle, seeded key, a-polynomials and errors)
of additive shares uniform in [0, 2^37), the worst case for noise; weights
are uniform in [-2^12, 2^12) (12-bit scale).  The batch runs once per
module; each layer is then its own test: its output words equal the
oracle's, and image 0 decrypts to conv(x, K) mod t."""
import numpy as np
import pytest

import oracle
import synth
from synth import Stream
from tests import workload as wl
from tests.gpu_util import empty_words, require_gpu, to_dev, to_host
from tests.libload import ensure_built

pytestmark = pytest.mark.gpu

FIRE = synth.WORKLOADS["fire_cnn"]
BOTTLENECK = synth.WORKLOADS["bottleneck_cnn_b16"]
# stem, then the first block of each stage: 1x1, 3x3, 1x1, projection
BOTTLENECK_SUBSET = [0, 1, 2, 3, 4, 11, 12, 13, 14, 24, 25, 26, 27, 43, 44, 45, 46]


def _params(cfg):
    return oracle.Params(cfg["N"], cfg["L"], cfg["bits"], 2 ** synth.T_BITS)


def draw_layer(cfg, idx, B, sk, prm, g, cv):
    """Seeded shares x [B][C][H][W] in [0, 2^37), kernel K, and the
    encrypted packed inputs [B][CB][S][2][L][N]."""
    seed = cfg["seed"] * 1000 + idx
    x = Stream(seed, synth.INPUT).ints(B * cv.C * cv.H * cv.W, *cfg["x_range"]).reshape(B, cv.C, cv.H, cv.W)
    K = Stream(seed, synth.WEIGHT).ints(cv.M * cv.C * cv.kh * cv.kw, *cfg["w_range"]).reshape(
        cv.M, cv.C, cv.kh, cv.kw)
    polys = np.stack([oracle.pack_input(x[b], cv, g, prm.t, prm.N) for b in range(B)])  # [B][CB][S][N]
    ct = wl.encrypt_polys(polys.reshape(-1, prm.N), prm, seed, sk)
    return x, K, ct.reshape(B, g.CB, g.S, 2, prm.L, prm.N)


class BatchRun:
    """One batch over the chosen layers of a workload, run once on the GPU;
    the host keeps what the oracle needs."""

    def __init__(self, cfg, layer_ids, B, schedule=2):
        require_gpu()
        ensure_built()
        from paper_2506_11586_amd import heconv
        self.prm = prm = _params(cfg)
        self.ctx = heconv.Context(cfg["N"], heconv.gen_primes(cfg["N"], cfg["bits"], cfg["L"]))
        assert self.ctx.q == prm.q
        self.sk = wl.secret_key(cfg["seed"], prm.N)
        self.B = B
        self.layers = {}
        jobs = []
        for idx in layer_ids:
            shape = cfg["layers"][idx]
            cv = oracle.Conv(*shape)
            d = self.ctx.plan(shape, batch=B)
            g = oracle.geometry(cv, d.Cw, d.Hw, d.Ww)
            assert g == oracle.plan_conv(cv, prm.N, prm.L, B)
            x, K, ct = draw_layer(cfg, idx, B, self.sk, prm, g, cv)
            s = self.ctx.sizes(d)
            wntt = empty_words(s.w_words)
            self.ctx.encode_weights(d, to_dev(K), wntt)
            d_in = to_dev(ct)
            d_out = empty_words(B * s.out_cts * 2 * prm.L * prm.N)
            d_out.fill_(-1)
            jobs.append((d, B, d_in, wntt, d_out))
            self.layers[idx] = dict(cv=cv, g=g, x0=x[0], K=K, ct=ct, d_out=d_out)
        self.batch = heconv.Batch(self.ctx, jobs, schedule=schedule)
        self.batch.launch(graph=True)
        self.batch.status()
        self.jobs = jobs  # keep the device buffers alive

    def check(self, idx):
        lay, prm, B = self.layers[idx], self.prm, self.B
        cv, g = lay["cv"], lay["g"]
        got = to_host(lay["d_out"]).reshape(B, cv.M, g.S, 2, prm.L, prm.N)
        w_ntt = oracle.encode_weights(lay["K"], cv, g, prm)
        want = oracle.conv_layer_ntt(lay["ct"], w_ntt, B, g, cv.M, prm)
        del w_ntt
        assert np.array_equal(got, want), (idx, cv)
        del want
        y = wl.decrypt_output(got[0], cv, g, prm, self.sk)
        ref = oracle.centre_mod(oracle.plain_conv(lay["x0"], lay["K"], cv.stride, cv.pad), prm.t)
        assert np.array_equal(y, ref), (idx, cv)


@pytest.fixture(scope="module")
def fire_run():
    run = BatchRun(FIRE, list(range(len(FIRE["layers"]))), 1, schedule=2)
    yield run
    run.batch.close()
    run.ctx.close()


@pytest.fixture(scope="module")
def bottleneck_run():
    run = BatchRun(BOTTLENECK, BOTTLENECK_SUBSET, BOTTLENECK["batch"], schedule=2)
    yield run
    run.batch.close()
    run.ctx.close()


@pytest.mark.parametrize("idx", range(len(FIRE["layers"])))
def test_fire_cnn_batched_layer(fire_run, idx):
    fire_run.check(idx)


def test_fire_cnn_other_schedules_equal(fire_run):
    """The same 26 jobs as one chain and pipelined in 4 and 8 groups (inverse
    NTTs of a group beside the next group's MAC, hipGraph and eager): every
    output word equals the two-chain batch's, which the tests above compare
    with the oracle."""
    import torch
    from paper_2506_11586_amd import heconv
    run = fire_run
    want = [run.layers[i]["d_out"].clone() for i in sorted(run.layers)]
    for sched in (1, 3, 4):
        b = heconv.Batch(run.ctx, run.jobs, schedule=sched)
        for graph in (True, False):
            for i, (d, B, d_in, wntt, d_out) in zip(sorted(run.layers), run.jobs):
                d_in.copy_(to_dev(run.layers[i]["ct"]))
                d_out.fill_(-1)
            torch.cuda.synchronize()
            b.launch(graph=graph)
            b.status()
            for (d, B, d_in, wntt, d_out), w in zip(run.jobs, want):
                assert torch.equal(d_out, w), (sched, graph)
        b.close()


@pytest.mark.parametrize("idx", BOTTLENECK_SUBSET)
def test_bottleneck_b16_batched_layer(bottleneck_run, idx):
    bottleneck_run.check(idx)
