"""Oracle: parameters, packing, planner, BFV client side and layer references.

TEST INFRASTRUCTURE ONLY -- see oracle/__init__.py.

Paper passages (SecONNds, arXiv 2506.11586):
  ring and notation ................ Sec. 2.1
  BFV encryption b = a*sk+d*m+e .... App. C (encryption equation)
  product as coefficient convolution App. C (its printed sum lacks the
                                     negacyclic wrap term; included here)
  NTT multiplication ............... App. C.1
  NTT preprocessing flow ........... Sec. 6.2 (NTT preprocessing)
  coefficient encoding, sparse
  results, extraction .............. Sec. 6.1 (HE kernels) and Sec. 2.3
                                     (Cheetah paragraph)
  server share, mask, extraction ... Sec. 7 (online protocol, linear
                                     layers) and Sec. 6.2
  rotation (automorphism and key
  switching) for the Z_P variant .... Sec. 2 (HE operations: rotations need
                                     key switching with evaluation keys),
                                     Sec. 6.1 (iterative MAC + rotation);
                                     the key-switching method is a reading
  Z_P slots and the multiply-
  accumulate-rotate kernel .......... Sec. 6.1 (HE kernels); the slot order
                                     and diagonal layout are readings
  polyphase form of strided convs ... a restatement of the layer (the same
                                     outputs, Sec. 9.1 on composite-op
                                     overheads); pinned by the plain conv
The paper gives no formula for the packing, no HE parameters and no tiling
rule; the readings used (packing layout, largest primes, smallest root,
bytes-objective planner, round-half-up decode) are listed with the design
notes and pinned by the CPU tests.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np

from . import build as _build

# --------------------------------------------------------------------------
# C core binding
# --------------------------------------------------------------------------
_lib = None
_u64p = ctypes.POINTER(ctypes.c_uint64)
_i64p = ctypes.POINTER(ctypes.c_int64)


def lib():
    """Load oracle/liboracle.so, compiling it with gcc first if it is absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        u32, u64, i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
        L.or_is_prime.argtypes = [u64]
        L.or_is_prime.restype = i32
        L.or_find_primes.argtypes = [u32, u32, u32, _u64p]
        L.or_find_primes.restype = i32
        L.or_find_psi.argtypes = [u64, u32]
        L.or_find_psi.restype = u64
        L.or_negacyclic_mul.argtypes = [_u64p, _u64p, _u64p, u32, u64]
        L.or_negacyclic_coeff.argtypes = [_u64p, _u64p, u32, u32, u64]
        L.or_negacyclic_coeff.restype = u64
        L.or_ntt_def.argtypes = [_u64p, _u64p, u32, u64, u64]
        L.or_intt_def.argtypes = [_u64p, _u64p, u32, u64, u64]
        L.or_ntt_fast.argtypes = [_u64p, u32, u64, u64]
        L.or_intt_fast.argtypes = [_u64p, u32, u64, u64]
        L.or_ntt_batch.argtypes = [_u64p, u64, u32, u32, _u64p, _u64p, i32, i32]
        L.or_conv_mac.argtypes = [_u64p, _u64p, _u64p, u32, u32, u32, u32, u32, u32, _u64p]
        L.or_conv_layer_def.argtypes = [_u64p, _u64p, _u64p, u32, u32, u32, u32, u32, u32, _u64p]
        L.or_conv_layer_coeff.argtypes = [_u64p, _u64p, u32, u32, u32, u32, _u64p, u32, u32, u32, u32, u32, u32]
        L.or_conv_layer_coeff.restype = u64
        L.or_bfv_encrypt.argtypes = [u64, u32, u32, _u64p, _u64p, _i64p, _u64p, _i64p, _u64p, _u64p, _u64p, i32]
        L.or_bfv_phase.argtypes = [u64, u32, u32, _u64p, _u64p, _i64p, _u64p, _u64p, i32]
        L.or_num_threads.restype = i32
        L.or_set_threads.argtypes = [i32]
        L.or_set_threads.restype = None
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"], "oracle arrays must be C-contiguous"
    if a.dtype == np.uint64:
        return a.ctypes.data_as(_u64p)
    if a.dtype == np.int64:
        return a.ctypes.data_as(_i64p)
    raise TypeError(a.dtype)


def _u64(x) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(x, dtype=np.uint64))


def num_threads() -> int:
    """Threads the oracle's OpenMP loops use."""
    return int(lib().or_num_threads())


def set_threads(n: int) -> None:
    """Threads for the oracle's OpenMP loops from now on."""
    lib().or_set_threads(int(n))


# --------------------------------------------------------------------------
# Parameters
# --------------------------------------------------------------------------
def is_prime(n: int) -> bool:
    return bool(lib().or_is_prime(int(n)))


def find_primes(N: int, bits: int, L: int) -> list[int]:
    """The L largest primes below 2^bits with q = 1 mod 2N, descending."""
    out = np.zeros(L, dtype=np.uint64)
    got = lib().or_find_primes(N, bits, L, _p(out))
    if got != L:
        raise ValueError(f"only {got} primes below 2^{bits} are 1 mod {2 * N}")
    return [int(v) for v in out]


def find_psi(q: int, N: int) -> int:
    """Smallest primitive 2N-th root of unity mod q."""
    return int(lib().or_find_psi(int(q), int(N)))


@dataclass
class Params:
    """RNS BFV parameters: N, L primes of `bits` bits, plaintext modulus t."""

    N: int
    L: int
    bits: int
    t: int
    q: list = field(default_factory=list)
    psi: list = field(default_factory=list)

    def __post_init__(self):
        if not self.q:
            self.q = find_primes(self.N, self.bits, self.L)
        if not self.psi:
            self.psi = [find_psi(q, self.N) for q in self.q]
        self.Q = math.prod(self.q)
        self.delta = self.Q // self.t  # BFV scale floor(Q/t) (App. C: delta)
        self.delta_l = [self.delta % q for q in self.q]
        self.q_arr = _u64(self.q)
        self.psi_arr = _u64(self.psi)
        self.logN = self.N.bit_length() - 1


# --------------------------------------------------------------------------
# Ring products and transforms
# --------------------------------------------------------------------------
def negacyclic_mul(a, b, q: int) -> np.ndarray:
    a, b = _u64(a), _u64(b)
    c = np.zeros_like(a)
    lib().or_negacyclic_mul(_p(a), _p(b), _p(c), a.size, int(q))
    return c


def negacyclic_coeff(a, b, k: int, q: int) -> int:
    a, b = _u64(a), _u64(b)
    return int(lib().or_negacyclic_coeff(_p(a), _p(b), int(k), a.size, int(q)))


def ntt_def(a, q: int, psi: int) -> np.ndarray:
    a = _u64(a)
    out = np.zeros_like(a)
    lib().or_ntt_def(_p(a), _p(out), a.size, int(q), int(psi))
    return out


def intt_def(a, q: int, psi: int) -> np.ndarray:
    a = _u64(a)
    out = np.zeros_like(a)
    lib().or_intt_def(_p(a), _p(out), a.size, int(q), int(psi))
    return out


def ntt_fast(a, q: int, psi: int) -> np.ndarray:
    a = _u64(a).copy()
    lib().or_ntt_fast(_p(a), a.size, int(q), int(psi))
    return a


def intt_fast(a, q: int, psi: int) -> np.ndarray:
    a = _u64(a).copy()
    lib().or_intt_fast(_p(a), a.size, int(q), int(psi))
    return a


MODE_DEF, MODE_FAST = 0, 1


def ntt(polys, prm: Params, mode: int = MODE_FAST, inverse: bool = False) -> np.ndarray:
    """Forward (or inverse) NTT of every limb of polys [..., L, N] (copy)."""
    a = _u64(polys).copy()
    assert a.shape[-1] == prm.N and a.shape[-2] == prm.L
    n = a.size // (prm.L * prm.N)
    lib().or_ntt_batch(_p(a), n, prm.L, prm.N, _p(prm.q_arr), _p(prm.psi_arr), int(mode), int(inverse))
    return a


def intt(polys, prm: Params, mode: int = MODE_FAST) -> np.ndarray:
    return ntt(polys, prm, mode, inverse=True)


# --------------------------------------------------------------------------
# Convolution geometry, planner and packing
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class Conv:
    """A conv layer: input C x H x W, M output channels, kh x kw kernel."""

    C: int
    H: int
    W: int
    M: int
    kh: int
    kw: int
    stride: int = 1
    pad: int = 0


@dataclass(frozen=True)
class Geometry:
    Cw: int
    Hw: int
    Ww: int
    Hp: int  # padded input height (before any subsampling)
    Wp: int
    Ho: int  # output height at the layer's stride
    Wo: int
    sub: bool  # 1x1 strided conv: the padded input is subsampled first
    He: int  # height of the tensor the tiles read (subsampled if sub)
    We: int
    R1: int  # stride-1 output rows that must be produced
    C1: int
    bh: int  # stride-1 output rows per tile
    bw: int
    nsi: int
    nsj: int
    S: int
    CB: int
    O: int  # coefficient index of output (0, 0) in a product


def geometry(cv: Conv, Cw: int, Hw: int, Ww: int) -> Geometry:
    """Tiling of a conv for the packing descriptor (Cw, Hw, Ww).

    Stride s > 1 with a kernel larger than 1x1 is computed at stride 1 and
    every s-th output kept; a strided 1x1 conv subsamples the padded input
    first and then runs at stride 1."""
    s = cv.stride
    Hp, Wp = cv.H + 2 * cv.pad, cv.W + 2 * cv.pad
    Ho, Wo = (Hp - cv.kh) // s + 1, (Wp - cv.kw) // s + 1
    sub = cv.kh == 1 and cv.kw == 1 and s > 1
    if sub:
        He, We, R1, C1 = Ho, Wo, Ho, Wo
    else:
        He, We, R1, C1 = Hp, Wp, (Ho - 1) * s + 1, (Wo - 1) * s + 1
    bh, bw = Hw - cv.kh + 1, Ww - cv.kw + 1
    nsi, nsj = -(-R1 // bh), -(-C1 // bw)
    CB = -(-cv.C // Cw)
    O = (Cw - 1) * Hw * Ww + (cv.kh - 1) * Ww + (cv.kw - 1)
    return Geometry(Cw, Hw, Ww, Hp, Wp, Ho, Wo, sub, He, We, R1, C1, bh, bw, nsi, nsj, nsi * nsj, CB, O)


def layer_cost(cv: Conv, g: Geometry, N: int, L: int, B: int) -> tuple[int, int]:
    """(HBM bytes, modmuls) of one unfused layer solve for B images: weights
    read once, every ciphertext word read and written in each of the three
    steps; NTTs at (N/2) log2 N modmuls per limb-polynomial, MACs at one
    modmul per word."""
    in_cts, out_cts = g.CB * g.S, cv.M * g.S
    ct_bytes = 2 * L * N * 8
    byts = cv.M * g.CB * L * N * 8 + B * 3 * (in_cts + out_cts) * ct_bytes
    logN = N.bit_length() - 1
    mm = B * (in_cts + out_cts) * 2 * L * (N // 2) * logN + B * cv.M * g.CB * g.S * 2 * L * N
    return byts, mm


def plan_conv(cv: Conv, N: int, L: int, B: int = 1) -> Geometry:
    """Packing descriptor by exhaustive search: every Hw in [kh, He], Ww in
    [kw, We] with Hw*Ww <= N, Cw = min(C, floor(N/(Hw*Ww))); minimise HBM
    bytes, then modmuls, then prefer larger Hw, then larger Ww."""
    g0 = geometry(cv, 1, cv.kh, cv.kw)
    best, best_key = None, None
    for Hw in range(cv.kh, g0.He + 1):
        for Ww in range(cv.kw, g0.We + 1):
            if Hw * Ww > N:
                break
            Cw = min(cv.C, N // (Hw * Ww))
            g = geometry(cv, Cw, Hw, Ww)
            byts, mm = layer_cost(cv, g, N, L, B)
            key = (byts, mm, -Hw, -Ww)
            if best_key is None or key < best_key:
                best, best_key = g, key
    if best is None:
        raise ValueError("no packing fits N")
    return best


def padded_input(x: np.ndarray, cv: Conv, g: Geometry) -> np.ndarray:
    """Zero-padded input, subsampled for a strided 1x1 conv: [C][He][We]."""
    C, H, W = x.shape
    xp = np.zeros((C, g.Hp, g.Wp), dtype=np.int64)
    xp[:, cv.pad:cv.pad + H, cv.pad:cv.pad + W] = x
    if g.sub:
        xp = np.ascontiguousarray(xp[:, ::cv.stride, ::cv.stride])
    return xp


def pack_input(x: np.ndarray, cv: Conv, g: Geometry, t: int, N: int) -> np.ndarray:
    """Client-side coefficient encoding of one input tensor x[C][H][W]:
    polys [CB][S][N] with coefficient cc*Hw*Ww + i*Ww + j of block cb, tile
    (si, sj) equal to the padded input at channel cb*Cw+cc, row si*bh+i,
    column sj*bw+j, reduced mod t into [0, t); zero outside the tensor."""
    xp = padded_input(x, cv, g)
    HW = g.Hw * g.Ww
    out = np.zeros((g.CB, g.S, N), dtype=np.uint64)
    for cb in range(g.CB):
        for si in range(g.nsi):
            for sj in range(g.nsj):
                s = si * g.nsj + sj
                for cc in range(g.Cw):
                    c = cb * g.Cw + cc
                    if c >= cv.C:
                        break
                    r0, c0 = si * g.bh, sj * g.bw
                    blk = xp[c, r0:r0 + g.Hw, c0:c0 + g.Ww]  # clipped at the tensor edge
                    for i in range(blk.shape[0]):
                        base = cc * HW + i * g.Ww
                        out[cb, s, base:base + blk.shape[1]] = np.mod(blk[i], t).astype(np.uint64)
    return out


def pack_weights(K: np.ndarray, cv: Conv, g: Geometry, prm: Params) -> np.ndarray:
    """Server-side kernel encoding, coefficient form: wc [M][CB][L][N] with
    coefficient O - cc*Hw*Ww - l*Ww - l' of (m, cb) equal to K[m][cb*Cw+cc][l][l'],
    a signed integer lifted into [0, q_l)."""
    M, C, kh, kw = K.shape
    HW = g.Hw * g.Ww
    out = np.zeros((M, g.CB, prm.L, prm.N), dtype=np.uint64)
    K = np.asarray(K, dtype=np.int64)
    for c in range(C):
        cb, cc = divmod(c, g.Cw)
        for i in range(kh):
            for j in range(kw):
                idx = g.O - cc * HW - i * g.Ww - j
                v = K[:, c, i, j]  # every output channel at once
                for l, q in enumerate(prm.q):
                    # signed lift into [0, q): integer floor-mod by q < 2^63
                    out[:, cb, l, idx] = np.mod(v, np.int64(q)).astype(np.uint64)
    return out


def encode_weights(K: np.ndarray, cv: Conv, g: Geometry, prm: Params, mode: int = MODE_FAST) -> np.ndarray:
    """NTT preprocessing of the weights (Sec. 6.2): pack, then forward NTT of
    every limb.  W [M][CB][L][N] in NTT form."""
    return ntt(pack_weights(K, cv, g, prm), prm, mode)


def conv_mac(in_ntt, w_ntt, B: int, g: Geometry, M: int, prm: Params) -> np.ndarray:
    """out[b][m][s][c][l][k] = sum_cb in[b][cb][s][c][l][k] * w[m][cb][l][k] mod q_l."""
    in_ntt, w_ntt = _u64(in_ntt), _u64(w_ntt)
    assert in_ntt.size == B * g.CB * g.S * 2 * prm.L * prm.N
    assert w_ntt.size == M * g.CB * prm.L * prm.N
    out = np.zeros((B, M, g.S, 2, prm.L, prm.N), dtype=np.uint64)
    lib().or_conv_mac(_p(in_ntt), _p(w_ntt), _p(out), B, g.CB, g.S, M, prm.L, prm.N, _p(prm.q_arr))
    return out


def conv_layer_ntt(in_ct, w_ntt, B: int, g: Geometry, M: int, prm: Params, mode: int = MODE_FAST) -> np.ndarray:
    """The paper's online flow (Sec. 6.2): NTT every input ciphertext, MAC in
    the NTT domain, inverse NTT of the results.  Coefficient form in and out."""
    x = ntt(in_ct, prm, mode)
    y = conv_mac(x, w_ntt, B, g, M, prm)
    return intt(y, prm, mode)


def conv_layer_def(in_ct, wc, B: int, g: Geometry, M: int, prm: Params) -> np.ndarray:
    """The same layer by its plain definition: schoolbook negacyclic products
    of every input ciphertext with the coefficient-form kernel polynomials,
    summed over channel blocks.  O(N^2) per product."""
    in_ct, wc = _u64(in_ct), _u64(wc)
    out = np.zeros((B, M, g.S, 2, prm.L, prm.N), dtype=np.uint64)
    lib().or_conv_layer_def(_p(in_ct), _p(wc), _p(out), B, g.CB, g.S, M, prm.L, prm.N, _p(prm.q_arr))
    return out


def conv_layer_coeff(in_ct, wc, g: Geometry, prm: Params, b, m, s, c, l, k) -> int:
    """One output word of the layer by definition, O(CB*N)."""
    in_ct, wc = _u64(in_ct), _u64(wc)
    return int(lib().or_conv_layer_coeff(_p(in_ct), _p(wc), g.CB, g.S, prm.L, prm.N, _p(prm.q_arr),
                                         b, m, s, c, l, k))


# --------------------------------------------------------------------------
# BFV client side (App. C); the server path never sees the key
# --------------------------------------------------------------------------
def bfv_encrypt(msgs, sk, a, e, prm: Params, mode: int = MODE_FAST) -> np.ndarray:
    """Symmetric-key encryption of n messages (msgs [n][N] in [0, t)) with
    secret key sk [N] (ternary), uniform a [n][L][N] and error e [n][N]:
    ct[i][0] = a_i, ct[i][1] = a_i*sk + delta*m_i + e_i per limb.
    Returns ct [n][2][L][N]."""
    msgs = _u64(msgs)
    n = msgs.shape[0]
    a = _u64(a).reshape(n, prm.L, prm.N)
    e = np.ascontiguousarray(np.asarray(e, dtype=np.int64).reshape(n, prm.N))
    sk = np.ascontiguousarray(np.asarray(sk, dtype=np.int64))
    ct = np.zeros((n, 2, prm.L, prm.N), dtype=np.uint64)
    dl = _u64(prm.delta_l)
    lib().or_bfv_encrypt(n, prm.L, prm.N, _p(prm.q_arr), _p(prm.psi_arr), _p(sk), _p(a), _p(e), _p(msgs),
                         _p(dl), _p(ct), int(mode))
    return ct


def bfv_phase(ct, sk, prm: Params, mode: int = MODE_FAST) -> np.ndarray:
    """v_l = b_l - a_l*sk mod q_l for ct [n][2][L][N] -> [n][L][N]."""
    ct = _u64(ct)
    n = ct.size // (2 * prm.L * prm.N)
    sk = np.ascontiguousarray(np.asarray(sk, dtype=np.int64))
    v = np.zeros((n, prm.L, prm.N), dtype=np.uint64)
    lib().or_bfv_phase(n, prm.L, prm.N, _p(prm.q_arr), _p(prm.psi_arr), _p(sk), _p(ct), _p(v), int(mode))
    return v


def crt(v: np.ndarray, prm: Params) -> np.ndarray:
    """Chinese remaindering of residues v[..., L] into [0, Q) (object array of
    Python ints)."""
    acc = np.zeros(v.shape[:-1], dtype=object)
    for l, q in enumerate(prm.q):
        Ql = prm.Q // q
        c = Ql * pow(Ql % q, -1, q)
        acc = acc + v[..., l].astype(object) * c
    return acc % prm.Q


def bfv_decode(v: np.ndarray, prm: Params, with_noise: bool = False):
    """Phase residues v[..., L] -> messages centred in [-t/2, t/2):
    m = floor((t*V + floor(Q/2)) / Q) mod t (round half up).  With
    with_noise, also the largest |V - delta*m mod Q| (centred) in bits."""
    V = crt(v, prm)
    t, Q = prm.t, prm.Q
    m = ((t * V + Q // 2) // Q) % t
    mc = np.where(2 * m >= t, m - t, m).astype(np.int64)
    if not with_noise:
        return mc
    noise = (V - prm.delta * (m % t)) % Q
    noise = np.where(noise > Q // 2, Q - noise, noise)
    mx = max([int(z) for z in noise.ravel()] + [0])
    return mc, (mx.bit_length() if mx else 0)


def bfv_decrypt(ct, sk, prm: Params, coeffs=None, mode: int = MODE_FAST, with_noise: bool = False):
    """Decrypt ct [n][2][L][N]; decode only the coefficient indexes in
    `coeffs` if given.  Returns centred messages [n][len(coeffs) or N]."""
    v = bfv_phase(ct, sk, prm, mode)  # [n][L][N]
    v = np.moveaxis(v, -2, -1)  # [n][N][L]
    if coeffs is not None:
        v = v[:, np.asarray(coeffs), :]
    return bfv_decode(v, prm, with_noise)


# --------------------------------------------------------------------------
# Output decoding and the plaintext reference
# --------------------------------------------------------------------------
def output_slots(g: Geometry) -> np.ndarray:
    """Coefficient indexes O + i*Ww + j (i < bh, j < bw) that hold results."""
    i = np.arange(g.bh)[:, None]
    j = np.arange(g.bw)[None, :]
    return (g.O + i * g.Ww + j).ravel()


def assemble_output(slot_vals: np.ndarray, cv: Conv, g: Geometry) -> np.ndarray:
    """slot_vals [M][S][bh*bw] (decoded output slots of every tile) ->
    output tensor [M][Ho][Wo] at the layer's stride."""
    M = slot_vals.shape[0]
    full = np.zeros((M, g.nsi * g.bh, g.nsj * g.bw), dtype=np.int64)
    for si in range(g.nsi):
        for sj in range(g.nsj):
            s = si * g.nsj + sj
            full[:, si * g.bh:(si + 1) * g.bh, sj * g.bw:(sj + 1) * g.bw] = slot_vals[:, s].reshape(M, g.bh, g.bw)
    if g.sub:
        return full[:, :g.Ho, :g.Wo]
    return full[:, :g.R1:cv.stride, :g.C1:cv.stride][:, :g.Ho, :g.Wo]


def plain_conv(x: np.ndarray, K: np.ndarray, stride: int, pad: int) -> np.ndarray:
    """Plaintext integer convolution (cross-correlation, as CNNs use):
    y[m][i][j] = sum_{c,u,v} K[m][c][u][v] * xpad[c][i*stride+u][j*stride+v],
    in wrapping int64 (exact whenever the true sum fits, and always exact
    mod 2^k for k <= 64)."""
    C, H, W = x.shape
    M, C2, kh, kw = K.shape
    assert C == C2
    xp = np.zeros((C, H + 2 * pad, W + 2 * pad), dtype=np.int64)
    xp[:, pad:pad + H, pad:pad + W] = x
    Ho = (H + 2 * pad - kh) // stride + 1
    Wo = (W + 2 * pad - kw) // stride + 1
    y = np.zeros((M, Ho, Wo), dtype=np.int64)
    with np.errstate(over="ignore"):
        for u in range(kh):
            for v in range(kw):
                patch = xp[:, u:u + stride * (Ho - 1) + 1:stride, v:v + stride * (Wo - 1) + 1:stride]
                y += np.tensordot(K[:, :, u, v].astype(np.int64), patch, axes=([1], [0]))
    return y


def centre_mod(y: np.ndarray, t: int) -> np.ndarray:
    """y mod t, centred into [-t/2, t/2)."""
    r = np.mod(y, t)
    return np.where(2 * r >= t, r - t, r).astype(np.int64)


# --------------------------------------------------------------------------
# Protocol steps either side of the layer (Sec. 7, online protocol for
# linear layers; Sec. 6.2, extraction of the sparse results)
# --------------------------------------------------------------------------
def add_share(ct, xs: np.ndarray, cv: Conv, g: Geometry, prm: Params) -> np.ndarray:
    """The server folds its additive share of the layer input into the
    client's input ciphertexts of one image: with m = pack_input(xs) (values
    taken mod t), b_l <- b_l + delta_l * m mod q_l; the a components are
    untouched.  ct [CB][S][2][L][N] in coefficient form -> a new array that
    decrypts to the packing of (x_client + xs) mod t."""
    m = pack_input(np.asarray(xs, dtype=np.int64), cv, g, prm.t, prm.N).astype(object)  # [CB][S][N]
    out = _u64(ct).reshape(g.CB, g.S, 2, prm.L, prm.N).copy()
    for l, q in enumerate(prm.q):
        b = out[:, :, 1, l, :].astype(object)
        out[:, :, 1, l, :] = ((b + prm.delta_l[l] * m) % q).astype(np.uint64)
    return out


def output_coeffs(cv: Conv, g: Geometry):
    """For every output position (oy, ox) at the layer's stride: the tile s
    and the coefficient index that hold it (as assemble_output reads them),
    two int arrays [Ho][Wo]."""
    step = 1 if g.sub else cv.stride
    si, i = np.divmod(np.arange(g.Ho) * step, g.bh)
    sj, j = np.divmod(np.arange(g.Wo) * step, g.bw)
    s = si[:, None] * g.nsj + sj[None, :]
    k = g.O + i[:, None] * g.Ww + j[None, :]
    return s, k


def mask_extract(out_ct, R: np.ndarray, e, cv: Conv, g: Geometry, prm: Params) -> np.ndarray:
    """After the inverse NTT the server keeps only the b coefficients that
    hold outputs, masked with its output share R (values taken mod t) and an
    optional signed smudging term e (None = 0):
    y[m][l][oy][ox] = b_l[slot(oy, ox)] - delta_l * R[m][oy][ox] + e[m][oy][ox] mod q_l.
    out_ct [M][S][2][L][N] (coefficient form, one image) -> y [M][L][Ho][Wo].
    The a components go to the client unchanged."""
    s, k = output_coeffs(cv, g)
    ct = _u64(out_ct).reshape(cv.M, g.S, 2, prm.L, prm.N)
    Rm = np.mod(np.asarray(R, dtype=np.int64), prm.t).astype(object)
    ev = 0 if e is None else np.asarray(e, dtype=np.int64).astype(object)
    y = np.zeros((cv.M, prm.L, g.Ho, g.Wo), dtype=np.uint64)
    for l, q in enumerate(prm.q):
        b = ct[:, s, 1, l, k].astype(object)  # [M][Ho][Wo]
        y[:, l] = ((b - prm.delta_l[l] * Rm + ev) % q).astype(np.uint64)
    return y


def decrypt_extracted(a_polys, y, sk, cv: Conv, g: Geometry, prm: Params, with_noise: bool = False):
    """Client side: decode the extracted outputs y [M][L][Ho][Wo] with the a
    components a_polys [M][S][L][N] of the output ciphertexts: the phase of
    output (m, oy, ox) is y - (a*sk)[slot] mod q_l.  -> [M][Ho][Wo] centred."""
    a = _u64(a_polys).reshape(cv.M * g.S, prm.L, prm.N)
    ct0 = np.zeros((cv.M * g.S, 2, prm.L, prm.N), dtype=np.uint64)
    ct0[:, 0] = a
    v0 = bfv_phase(ct0, sk, prm).reshape(cv.M, g.S, prm.L, prm.N)  # -(a*sk) mod q_l
    s, k = output_coeffs(cv, g)
    v = np.zeros((cv.M, g.Ho, g.Wo, prm.L), dtype=np.uint64)
    for l, q in enumerate(prm.q):
        v[..., l] = ((_u64(y)[:, l].astype(object) + v0[:, s, l, k].astype(object)) % q).astype(np.uint64)
    return bfv_decode(v, prm, with_noise)


# --------------------------------------------------------------------------
# Ciphertext rotation for the Z_P variant (Sec. 6.1: its linear kernels
# combine multiply-accumulates with rotations; App. C, rotation): the Galois
# automorphism X -> X^g and hybrid key switching with one special prime P.
# --------------------------------------------------------------------------
def automorphism(polys, g: int, q_list) -> np.ndarray:
    """a(X) -> a(X^g) in Z_q[X]/(X^N+1) for odd g: coefficient i moves to
    i*g mod 2N, negated (mod q_l) when that index is N or more.
    polys [..., L, N] with q_list the L moduli."""
    a = _u64(polys)
    N = a.shape[-1]
    assert g % 2 == 1
    out = np.zeros_like(a)
    idx = (np.arange(N, dtype=np.int64) * g) % (2 * N)
    neg = idx >= N
    dst = np.where(neg, idx - N, idx)
    for l, q in enumerate(q_list):
        src = a[..., l, :]
        vals = np.where(neg, np.where(src == 0, np.uint64(0), np.uint64(q) - src), src)
        o = out[..., l, :]
        o[..., dst] = vals
    return out


def ext_params(prm: Params, P: int) -> Params:
    """The extended basis q_0..q_{L-1}, P (P last) of the same ring."""
    return Params(prm.N, prm.L + 1, prm.bits, prm.t, q=list(prm.q) + [int(P)])


def galois_key(sk, g: int, a, e, prm: Params, P: int) -> np.ndarray:
    """Key switching key from s(X^g) to s over Z_{QP}: for every digit l < L
    a pair (k_a, k_b) with k_a = a[l] (uniform, [L+1][N] residues) and
    k_b = k_a*s + e[l] + G_l*s(X^g), where G_l = P*Qhat_l*(Qhat_l^-1 mod q_l)
    and Qhat_l = Q/q_l, all mod QP (per modulus).  Returns [L][2][L+1][N]
    in coefficient form (k_a first, as a ciphertext's a component)."""
    ext = ext_params(prm, P)
    N, L = prm.N, prm.L
    sk = np.asarray(sk, dtype=np.int64)
    s_lift = np.array([[int(v) % q for v in sk.tolist()] for q in ext.q], dtype=np.uint64)  # [L+1][N]
    sg = automorphism(s_lift, g, ext.q)
    QP = prm.Q * P
    out = np.zeros((L, 2, L + 1, N), dtype=np.uint64)
    e = np.asarray(e, dtype=np.int64).reshape(L, N)
    for l in range(L):
        Qh = prm.Q // prm.q[l]
        G = (P * Qh * pow(Qh % prm.q[l], -1, prm.q[l])) % QP
        ka = _u64(a).reshape(L, L + 1, N)[l]
        out[l, 0] = ka
        for j, q in enumerate(ext.q):
            prod = negacyclic_mul(ka[j], s_lift[j], q)
            el = np.array([int(v) % q for v in e[l].tolist()], dtype=object)
            gj = G % q
            v = (prod.astype(object) + el + (gj * sg[j].astype(object))) % q
            out[l, 1, j] = v.astype(np.uint64)
    return out


def key_switch(ct, ksk, prm: Params, P: int) -> np.ndarray:
    """Key switching of ct [n][2][L][N] (coefficient form, phase b - a*s')
    with a key from s' to s (galois_key): digits d_l = the limb-l residues
    of a, as integers in [0, q_l); over Z_{QP}, A = sum_l d_l*k_a[l] and
    B = sum_l d_l*k_b[l] (ring products per modulus); then division by P
    with rounding, y = (x - [x]_P)/P with [x]_P the residue mod P centred
    into (-P/2, P/2], computed on the integer x from the CRT of all L+1
    residues; result (-A', b - B') mod Q, of phase b - a*s' up to a small
    error."""
    ext = ext_params(prm, P)
    N, L = prm.N, prm.L
    ct = _u64(ct).reshape(-1, 2, L, N)
    n = ct.shape[0]
    ksk = _u64(ksk).reshape(L, 2, L + 1, N)
    QP = prm.Q * P
    out = np.zeros_like(ct)
    for i in range(n):
        acc = np.zeros((2, L + 1, N), dtype=object)
        for l in range(L):
            d = ct[i, 0, l]  # digit l: integers below q_l
            for j, q in enumerate(ext.q):
                dj = (d % np.uint64(q)).astype(np.uint64)
                for c in range(2):
                    acc[c, j] = (acc[c, j] + negacyclic_mul(dj, ksk[l, c, j], q).astype(object)) % q
        # exact division by P with rounding, coefficient by coefficient
        crt_c = []
        for j, q in enumerate(ext.q):
            Mj = QP // q
            crt_c.append(Mj * pow(Mj % q, -1, q))
        for c in range(2):
            X = sum(acc[c, j] * crt_c[j] for j in range(L + 1)) % QP  # [N] Python ints
            xp = X % P
            xp = np.where(xp > P // 2, xp - P, xp)
            Y = (X - xp) // P
            for j, q in enumerate(prm.q):
                y = (Y % q).astype(np.uint64)
                if c == 0:
                    out[i, 0, j] = ((q - y.astype(object)) % q).astype(np.uint64)
                else:
                    out[i, 1, j] = ((ct[i, 1, j].astype(object) - y.astype(object)) % q).astype(np.uint64)
    return out


def rotate(ct, g: int, ksk, prm: Params, P: int) -> np.ndarray:
    """Automorphism of both components, then key switching back to s."""
    return key_switch(automorphism(_u64(ct), g, prm.q), ksk, prm, P)


# --------------------------------------------------------------------------
# Z_P variant: batched (SIMD) plaintext slots and the iterative
# multiply-accumulate-rotate linear kernel (Sec. 6.1: the Z_P kernels
# multiply the input by NTT-preprocessed weights, accumulate, and rotate the
# accumulated result once per iteration; Sec. 2, HE operations).
# --------------------------------------------------------------------------
def _brv(i: int, logn: int) -> int:
    return int(format(i, f"0{logn}b")[::-1], 2) if logn else 0


def simd_exponents(N: int) -> np.ndarray:
    """Odd exponent e_s of slot s: a plaintext m in Z_t[X]/(X^N+1), t prime
    with t = 1 mod 2N, holds in slot s the value m(zeta^e_s), zeta a
    primitive 2N-th root of unity mod t.  Slot r*N/2 + j (row r < 2, column
    j < N/2) takes e = 5^j mod 2N in row 0 and -5^j mod 2N in row 1: 5
    generates a cyclic group of order N/2 in the odd residues mod 2N and -1
    lies outside it, so every odd residue occurs once."""
    h = N // 2
    e = np.zeros(N, dtype=np.int64)
    p = 1
    for j in range(h):
        e[j] = p
        e[h + j] = (2 * N - p) % (2 * N)
        p = p * 5 % (2 * N)
    return e


def _t_params(N: int, t: int) -> Params:
    return Params(N, 1, max(int(t).bit_length(), 2), t, q=[int(t)])


def simd_decode(m, t: int) -> np.ndarray:
    """Slots of the plaintexts m [..., N] (coefficients mod t): the forward
    NTT over the single prime t evaluates at psi^(2 brv(i) + 1) at index i,
    psi the transforms' root of t; slot s reads the index i with
    2 brv(i) + 1 = e_s."""
    a = np.mod(np.asarray(m, dtype=object), t).astype(np.uint64)
    N = a.shape[-1]
    logn = N.bit_length() - 1
    tp = _t_params(N, t)
    ev = ntt(a.reshape(-1, 1, N), tp).reshape(a.shape)
    idx = np.array([_brv(int((e - 1) // 2), logn) for e in simd_exponents(N)], dtype=np.int64)
    return ev[..., idx]


def simd_encode(v, t: int) -> np.ndarray:
    """Plaintexts [..., N] (coefficients in [0, t)) whose slots are v [..., N]
    (values mod t): the inverse of simd_decode."""
    a = np.mod(np.asarray(v, dtype=object), t).astype(np.uint64)
    N = a.shape[-1]
    logn = N.bit_length() - 1
    idx = np.array([_brv(int((e - 1) // 2), logn) for e in simd_exponents(N)], dtype=np.int64)
    ev = np.zeros_like(a)
    ev[..., idx] = a
    return intt(ev.reshape(-1, 1, N), _t_params(N, t)).reshape(a.shape)


def zp_diagonals(W: np.ndarray, n: int, N: int, t: int) -> np.ndarray:
    """Slot vectors [n][N] of the weight matrix W [rows][cols] (rows, cols
    <= n, n a power of two dividing N/2; zero padding to n x n): diagonal i
    holds W[(k - i) mod n][k mod n] in slot k of each row (period n), the
    factor that meets input x[k] in u_i = d_i * x before u_i is rotated
    left by i."""
    rows, cols = W.shape
    Wp = np.zeros((n, n), dtype=object)
    Wp[:rows, :cols] = np.mod(W.astype(object), t)
    h = N // 2
    k = np.arange(h) % n
    out = np.zeros((n, N), dtype=object)
    for i in range(n):
        row = Wp[(k - i) % n, k]
        out[i, :h] = row
        out[i, h:] = row
    return out


def zp_input_slots(x: np.ndarray, n: int, N: int, t: int) -> np.ndarray:
    """Slot vector [N] of the input x (length <= n): x repeated with period n
    in both rows, so that a left rotation of a row by one slot is a cyclic
    shift of x mod n."""
    xp = np.zeros(n, dtype=object)
    xp[:len(x)] = np.mod(np.asarray(x, dtype=object), t)
    return np.tile(xp, N // n)


def centred_lift(m, t: int) -> np.ndarray:
    """Coefficients mod t as integers in [-t/2, t/2) (int64)."""
    return centre_mod(np.asarray(m, dtype=object), t)


def ct_mul_plain(ct, w, prm: Params) -> np.ndarray:
    """ct [n][2][L][N] times the plaintext with integer coefficients w [N]
    (lifted mod every q_l): both components multiplied in Z_q[X]/(X^N+1)."""
    ct = _u64(ct).reshape(-1, 2, prm.L, prm.N)
    out = np.zeros_like(ct)
    w = np.asarray(w, dtype=object)
    for l, q in enumerate(prm.q):
        wl = np.mod(w, q).astype(np.uint64)
        for i in range(ct.shape[0]):
            for c in range(2):
                out[i, c, l] = negacyclic_mul(ct[i, c, l], wl, q)
    return out


def ct_add(x, y, prm: Params) -> np.ndarray:
    x = _u64(x)
    y = _u64(y)
    out = np.zeros_like(x)
    for l, q in enumerate(prm.q):
        out[..., l, :] = ((x[..., l, :].astype(object) + y[..., l, :].astype(object)) % q).astype(np.uint64)
    return out


def zp_matvec_ct(ct_x, diag_polys, g: int, ksk, prm: Params, P: int) -> np.ndarray:
    """The iterative kernel on ciphertexts: acc = ct_x * d_{n-1}; then for
    i = n-2 down to 0, acc = rotate(acc, g) + ct_x * d_i, with diag_polys
    [n][N] the plaintexts of the diagonals (integer coefficients).  With
    g = 5 (one slot left per rotation) the slots of the result hold
    sum_i rot^i(d_i * x), i.e. W x."""
    n = len(diag_polys)
    acc = ct_mul_plain(ct_x, diag_polys[n - 1], prm)
    for i in range(n - 2, -1, -1):
        acc = ct_add(rotate(acc, g, ksk, prm, P), ct_mul_plain(ct_x, diag_polys[i], prm), prm)
    return acc


# --------------------------------------------------------------------------
# Polyphase form of a strided convolution (a fusion variant: the same layer,
# fewer output ciphertexts when the packing keeps a full window per
# channel).  A stride-s conv equals a stride-1, pad-0 conv on s*s*C phase
# channels with a ceil(k/s) kernel: with u = s*i + a, v = s*j + b,
# xpad[c][s*y + u][s*x + v] = X_(c,a,b)[y + i][x + j].
# --------------------------------------------------------------------------
def polyphase_conv(cv: Conv) -> Conv:
    """The stride-1, pad-0 conv on the phases of cv's padded input; its
    first Ho x Wo outputs are cv's outputs (its output is never smaller)."""
    s = cv.stride
    assert s >= 2
    return Conv(s * s * cv.C, -(-(cv.H + 2 * cv.pad) // s), -(-(cv.W + 2 * cv.pad) // s), cv.M,
                -(-cv.kh // s), -(-cv.kw // s), 1, 0)


def polyphase_input(x: np.ndarray, cv: Conv) -> np.ndarray:
    """X[c*s*s + a*s + b][y][x'] = xpad[c][s*y + a][s*x' + b] (zero outside
    the padded input); x [C][H][W] -> [s*s*C][H'][W']."""
    s, pc = cv.stride, polyphase_conv(cv)
    C, H, W = x.shape
    xp = np.zeros((C, pc.H * s, pc.W * s), dtype=np.int64)
    xp[:, cv.pad:cv.pad + H, cv.pad:cv.pad + W] = x
    out = np.zeros((pc.C, pc.H, pc.W), dtype=np.int64)
    for c in range(C):
        for a in range(s):
            for b in range(s):
                out[c * s * s + a * s + b] = xp[c, a::s, b::s]
    return out


def polyphase_weights(K: np.ndarray, cv: Conv) -> np.ndarray:
    """K'[m][c*s*s + a*s + b][i][j] = K[m][c][s*i + a][s*j + b] (zero where
    s*i + a >= kh or s*j + b >= kw)."""
    s, pc = cv.stride, polyphase_conv(cv)
    M, C = K.shape[0], K.shape[1]
    Kp = np.zeros((M, pc.C, pc.kh, pc.kw), dtype=K.dtype)
    for c in range(C):
        for a in range(s):
            for b in range(s):
                sub = K[:, c, a::s, b::s]
                Kp[:, c * s * s + a * s + b, :sub.shape[1], :sub.shape[2]] = sub
    return Kp


def zp_matvec_grouped_ct(ct_x, diag_polys, G: int, g: int, ksk, g2: int, ksk2, prm: Params, P: int) -> np.ndarray:
    """The same kernel as G independent chains: chain c runs the iteration
    over diagonals c*n/G .. (c+1)*n/G - 1 (acc = x*d_last, then
    acc = rotate(acc, g) + x*d_i), and the chains are combined by
    acc = chain_{G-1}, then acc = rotate(acc, g2) + chain_c for c = G-2 .. 0,
    g2 the Galois element of a rotation by n/G slots (5^(n/G) mod 2N).
    The slots hold sum_c rot^(c n/G)(sum_i rot^i(d_(c n/G + i) * x)) = W x."""
    n = len(diag_polys)
    assert n % G == 0
    h = n // G
    chains = [zp_matvec_ct(ct_x, diag_polys[c * h:(c + 1) * h], g, ksk, prm, P) for c in range(G)]
    acc = chains[G - 1]
    for c in range(G - 2, -1, -1):
        acc = ct_add(rotate(acc, g2, ksk2, prm, P), chains[c], prm)
    return acc


def zp_diagonals_rect(W: np.ndarray, n_out: int, n_in: int, N: int, t: int) -> np.ndarray:
    """The n_out generalized diagonals of W [rows][cols] (rows <= n_out,
    cols <= n_in, n_out | n_in | N/2, powers of two): diagonal i holds
    W[(k - i) mod n_out][k mod n_in] in slot k of each row.  With x repeated
    with period n_in, z = sum_i rot^i(d_i * x) has
    z[r + j*n_out] = sum over columns r + j*n_out .. r + (j+1)*n_out - 1 of
    row r, so y = sum_j z[r + j*n_out], log2(n_in/n_out) rotate-and-add
    steps (rotations by n_out, 2*n_out, ...); n_out = n_in is zp_diagonals."""
    rows, cols = W.shape
    Wp = np.zeros((n_out, n_in), dtype=object)
    Wp[:rows, :cols] = np.mod(W.astype(object), t)
    h = N // 2
    k = np.arange(h) % n_in
    out = np.zeros((n_out, N), dtype=object)
    for i in range(n_out):
        row = Wp[(k - i) % n_out, k]
        out[i, :h] = row
        out[i, h:] = row
    return out


def zp_fold_ct(ct, g2: int, ksk2, prm: Params, P: int) -> np.ndarray:
    """One rotate-and-add step: ct + rotate(ct, g2)."""
    return ct_add(ct, rotate(ct, g2, ksk2, prm, P), prm)
