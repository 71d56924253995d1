"""Test-side wiring: seeded draws from `synth` fed into the oracle's client
side (key, encryption, decryption) and the layer shapes of the workloads."""
from __future__ import annotations

import numpy as np

import oracle
import synth
from synth import Stream

ETA = 21  # centred binomial error, sigma = sqrt(21/2) ~ 3.24


def conv_of(shape) -> oracle.Conv:
    return oracle.Conv(*shape)


def params_of(cfg: dict) -> oracle.Params:
    return oracle.Params(cfg["N"], cfg["L"], cfg["bits"], 2 ** synth.T_BITS)


def secret_key(seed: int, N: int) -> np.ndarray:
    return Stream(seed, synth.KEY).ternary(N)


def encrypt_polys(msgs: np.ndarray, prm: oracle.Params, seed: int, sk: np.ndarray, mode=oracle.MODE_FAST):
    """Encrypt msgs [n][N] (values in [0, t)) -> ct [n][2][L][N]."""
    n = msgs.shape[0]
    a = synth.uniform_mod(Stream(seed, synth.UNIFORM), (n, prm.L, prm.N), prm.q)
    e = Stream(seed, synth.ERROR).cbd(n * prm.N, ETA).reshape(n, prm.N)
    return oracle.bfv_encrypt(msgs, sk, a, e, prm, mode)


def encrypt_input(x: np.ndarray, cv, g, prm, seed, sk) -> np.ndarray:
    """Pack x [C][H][W] and encrypt: ct [CB][S][2][L][N]."""
    polys = oracle.pack_input(x, cv, g, prm.t, prm.N)
    ct = encrypt_polys(polys.reshape(-1, prm.N), prm, seed, sk)
    return ct.reshape(g.CB, g.S, 2, prm.L, prm.N)


def decrypt_output(out_ct: np.ndarray, cv, g, prm, sk, with_noise=False):
    """Decrypt the output slots of out_ct [M][S][2][L][N] -> [M][Ho][Wo]."""
    slots = oracle.output_slots(g)
    M = out_ct.shape[0]
    r = oracle.bfv_decrypt(out_ct.reshape(-1, 2, prm.L, prm.N), sk, prm, coeffs=slots, with_noise=with_noise)
    dec, bits = (r if with_noise else (r, None))
    y = oracle.assemble_output(dec.reshape(M, g.S, -1), cv, g)
    return (y, bits) if with_noise else y


def draw_layer(cfg: dict, shape, seed_offset: int = 0):
    """Seeded input tensor and kernel for one layer of a workload."""
    C, H, W, M, kh, kw, _, _ = shape
    seed = cfg["seed"] * 1000 + seed_offset
    x = Stream(seed, synth.INPUT).ints(C * H * W, *cfg["x_range"]).reshape(C, H, W)
    K = Stream(seed, synth.WEIGHT).ints(M * C * kh * kw, *cfg["w_range"]).reshape(M, C, kh, kw)
    return x, K
