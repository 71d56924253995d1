"""ctypes binding of libheconv.so (include/heconv.h), argument marshalling only.

Every step of the path runs in the library's HIP kernels; torch is used for
device buffers and streams.  Device tensors are int64 (or uint64) torch
tensors whose words are the residues; they are passed as raw pointers.
The module fails loudly if the built library is missing: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libheconv.so")

HE_OK, HE_EINVAL, HE_ESHAPE, HE_EPARAM, HE_ENOMEM, HE_EDEVICE, HE_EBUSY = 0, -1, -2, -3, -4, -5, -6


class HeError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {_lib_handle().he_status_str(status).decode()} ({status})")


class Tuning(ctypes.Structure):
    """he_tuning: launch-shape choices (speed only, never results)."""

    _fields_ = [(n, ctypes.c_uint32) for n in ("ntt_loge_small", "ntt_loge_large", "ntt_small_below",
                                               "mac_mt", "mac_rt", "layer_fused", "layer_split",
                                               "ntt_split_below", "ntt_fp64", "ks_fused",
                                               "ntt_inv_split_below", "mac_lds", "mac_tiles", "mac_grid")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class _Params(ctypes.Structure):
    _fields_ = [("N", ctypes.c_uint32), ("L", ctypes.c_uint32), ("q", ctypes.POINTER(ctypes.c_uint64)),
                ("t", ctypes.c_uint64)]


class ConvDesc(ctypes.Structure):
    """he_conv_desc: C, H, W, M, kh, kw, stride, pad, Cw, Hw, Ww."""

    _fields_ = [(n, ctypes.c_uint32) for n in ("C", "H", "W", "M", "kh", "kw", "stride", "pad", "Cw", "Hw", "Ww")]

    def shape(self):
        return (self.C, self.H, self.W, self.M, self.kh, self.kw, self.stride, self.pad)

    def packing(self):
        return (self.Cw, self.Hw, self.Ww)

    def __repr__(self):
        return "ConvDesc(" + ", ".join(f"{n}={getattr(self, n)}" for n, _ in self._fields_) + ")"


class _Job(ctypes.Structure):
    _fields_ = [("desc", ConvDesc), ("B", ctypes.c_uint32), ("d_in", ctypes.c_void_p), ("d_wntt", ctypes.c_void_p),
                ("d_out", ctypes.c_void_p)]


SCHED_ONE_CHAIN, SCHED_TWO_CHAINS, SCHED_PIPELINED_4, SCHED_PIPELINED_8 = 1, 2, 3, 4
# he_probe_valu probes (include/heconv_probe.h)
PROBE_MAD_U64_U32, PROBE_MUL_HI_U32, PROBE_MUL_LO_U32, PROBE_ADD_U32, PROBE_MAC_MIX, PROBE_INTT_MIX, PROBE_NTT_MIX = range(7)

_LIB = None


def _lib_handle():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"HIP library not built: {LIB_PATH} is missing (run paper_2506_11586_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        P, u32, u64, vp = ctypes.POINTER, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p
        i32 = ctypes.c_int
        L.he_status_str.argtypes = [i32]
        L.he_status_str.restype = ctypes.c_char_p
        L.he_gen_primes.argtypes = [u32, u32, u32, P(u64)]
        L.he_ctx_create.argtypes = [P(_Params), P(vp)]
        L.he_ctx_destroy.argtypes = [vp]
        L.he_ctx_destroy.restype = None
        L.he_ctx_psi.argtypes = [vp, P(u64)]
        L.he_ctx_get_tuning.argtypes = [vp, P(Tuning)]
        L.he_ctx_set_tuning.argtypes = [vp, P(Tuning)]
        L.he_plan_conv.argtypes = [vp, P(ConvDesc), u32]
        L.he_plan_conv_host.argtypes = [u32, u32, P(ConvDesc), u32]
        L.he_min_root.argtypes = [u64, u32, P(u64)]
        L.he_conv_sizes.argtypes = [vp, P(ConvDesc), P(u32), P(u32), P(u64), P(u64), P(u64)]
        L.he_encode_weights.argtypes = [vp, P(ConvDesc), vp, vp, vp]
        L.he_ntt_fwd.argtypes = [vp, vp, u64, vp]
        L.he_ntt_inv.argtypes = [vp, vp, u64, vp]
        L.he_conv_ntt_mac.argtypes = [vp, P(ConvDesc), u32, vp, vp, vp, vp]
        L.he_conv_layer.argtypes = [vp, P(ConvDesc), u32, vp, vp, vp, vp]
        L.he_conv_mac_intt.argtypes = [vp, P(ConvDesc), u32, vp, vp, vp, vp]
        L.he_delta_host.argtypes = [P(u64), u32, u64, P(u64)]
        L.he_key_encode.argtypes = [vp, vp, vp, vp]
        L.he_encrypt.argtypes = [vp, u64, vp, vp, vp, vp, vp, vp, vp]
        L.he_decrypt.argtypes = [vp, u64, vp, vp, vp, vp, vp]
        L.he_add_share.argtypes = [vp, P(ConvDesc), u32, vp, vp, vp]
        L.he_mask_extract.argtypes = [vp, P(ConvDesc), u32, vp, vp, vp, vp, vp]
        L.he_keyswitch_work_words.argtypes = [vp, u64, P(u64)]
        L.he_automorph.argtypes = [vp, u64, u64, vp, vp, vp]
        L.he_galois_key.argtypes = [vp, u64, vp, vp, vp, vp, vp, vp]
        L.he_keyswitch.argtypes = [vp, u64, vp, vp, vp, vp, vp]
        L.he_rotate.argtypes = [vp, u64, u64, vp, vp, vp, vp, vp]
        L.he_simd_encode.argtypes = [vp, u64, vp, vp, vp]
        L.he_simd_decode.argtypes = [vp, u64, vp, vp, vp, vp]
        L.he_zp_diagonals.argtypes = [vp, vp, u32, u32, u32, vp, vp]
        L.he_zp_encode_plain.argtypes = [vp, u64, vp, vp, vp]
        L.he_zp_work_words.argtypes = [vp, u64, P(u64)]
        L.he_zp_matvec.argtypes = [vp, u64, u64, vp, vp, u32, vp, vp, vp, vp]
        L.he_zp_grouped_work_words.argtypes = [vp, u64, u32, P(u64)]
        L.he_zp_matvec_grouped.argtypes = [vp, u64, u64, vp, vp, u32, u32, vp, u64, vp, vp, vp, vp]
        L.he_zp_diagonals_rect.argtypes = [vp, vp, u32, u32, u32, u32, vp, vp]
        L.he_zp_fold.argtypes = [vp, u64, u64, vp, vp, vp, vp, vp]
        L.he_rotate_noalloc.argtypes = [vp, u64, u64, vp, vp, vp, vp]
        L.he_probe_valu.argtypes = [vp, u32, u32, u32, vp, P(ctypes.c_double), vp]
        L.he_polyphase_desc.argtypes = [P(ConvDesc), P(ConvDesc)]
        L.he_polyphase_advised.argtypes = [u32, u32, P(ConvDesc), u32, P(i32)]
        L.he_polyphase_weights.argtypes = [P(ConvDesc), vp, vp, vp]
        L.he_polyphase_input.argtypes = [P(ConvDesc), u32, vp, vp, vp]
        L.he_batch_create.argtypes = [vp, P(_Job), u32, u32, P(vp)]
        L.he_batch_launch.argtypes = [vp, vp, i32]
        L.he_batch_launch_timed.argtypes = [vp, vp, P(ctypes.c_float)]
        L.he_batch_status.argtypes = [vp, vp]
        L.he_batch_info.argtypes = [vp, P(u64), P(u32)]
        L.he_batch_mac_form.argtypes = [vp, P(u32), P(u32), P(u32), P(u32), P(u32)]
        L.he_batch_destroy.argtypes = [vp]
        L.he_batch_destroy.restype = None
        for name in ("he_batch_create", "he_batch_launch", "he_batch_launch_timed", "he_batch_status", "he_batch_info",
                     "he_batch_mac_form"):
            getattr(L, name).restype = i32
        for name in ("he_gen_primes", "he_ctx_create", "he_ctx_psi", "he_ctx_get_tuning", "he_ctx_set_tuning", "he_plan_conv", "he_plan_conv_host", "he_min_root", "he_conv_sizes",
                     "he_encode_weights", "he_ntt_fwd", "he_ntt_inv", "he_conv_ntt_mac", "he_conv_layer",
                     "he_conv_mac_intt", "he_add_share", "he_mask_extract", "he_delta_host",
                     "he_key_encode", "he_encrypt", "he_decrypt", "he_keyswitch_work_words", "he_automorph", "he_galois_key",
                     "he_keyswitch", "he_rotate", "he_simd_encode", "he_simd_decode", "he_zp_diagonals",
                     "he_zp_encode_plain", "he_zp_work_words", "he_zp_matvec", "he_zp_grouped_work_words",
                     "he_zp_matvec_grouped", "he_zp_diagonals_rect", "he_zp_fold", "he_rotate_noalloc", "he_probe_valu", "he_polyphase_desc",
                     "he_polyphase_advised",
                     "he_polyphase_weights", "he_polyphase_input"):
            getattr(L, name).restype = i32
        _LIB = L
    return _LIB


def lib():
    """The loaded ctypes library (raises ImportError if it is not built)."""
    return _lib_handle()


def _check(status: int, what: str):
    if status != HE_OK:
        raise HeError(status, what)


def gen_primes(N: int, bits: int, L: int) -> list[int]:
    out = (ctypes.c_uint64 * L)()
    _check(lib().he_gen_primes(N, bits, L, out), "he_gen_primes")
    return [int(v) for v in out]


def plan_host(N: int, L: int, shape, batch: int = 1) -> ConvDesc:
    """The library's planner without a context (host only)."""
    d = ConvDesc(*[int(v) for v in shape], 0, 0, 0)
    _check(lib().he_plan_conv_host(int(N), int(L), ctypes.byref(d), int(batch)), "he_plan_conv_host")
    return d


def delta_host(q: list[int], t: int) -> list[int]:
    """The library's delta_l = floor(Q/t) mod q_l (host only)."""
    qa = (ctypes.c_uint64 * len(q))(*[int(v) for v in q])
    out = (ctypes.c_uint64 * len(q))()
    _check(lib().he_delta_host(qa, len(q), int(t), out), "he_delta_host")
    return [int(v) for v in out]


def min_root(q: int, N: int) -> int:
    """The library's choice of psi for (q, N) (host only)."""
    out = ctypes.c_uint64()
    _check(lib().he_min_root(int(q), int(N), ctypes.byref(out)), "he_min_root")
    return int(out.value)


def _ptr(t, words: int | None = None, what: str = "buffer") -> int:
    """Raw device pointer of a contiguous 64-bit-word CUDA tensor."""
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what}: expected a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{what}: must be a device tensor")
    if t.dtype not in (torch.int64, torch.uint64):
        raise TypeError(f"{what}: dtype must be int64/uint64, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what}: must be contiguous")
    if words is not None and t.numel() < words:
        raise ValueError(f"{what}: needs {words} words, has {t.numel()}")
    return t.data_ptr()


def _stream(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


@dataclass
class Sizes:
    CB: int
    S: int
    in_cts: int
    out_cts: int
    w_words: int


def polyphase_shape(shape) -> tuple:
    """he_polyphase_desc: the stride-1, pad-0 conv shape on the phase
    channels equal to the strided conv `shape` (C, H, W, M, kh, kw, stride, pad)."""
    d_in = ConvDesc(*[int(v) for v in shape], 0, 0, 0)
    d_out = ConvDesc()
    _check(lib().he_polyphase_desc(ctypes.byref(d_in), ctypes.byref(d_out)), "he_polyphase_desc")
    return d_out.shape()


def polyphase_advised(N: int, L: int, shape, batch: int = 1) -> bool:
    """he_polyphase_advised: whether the planner's objective prefers the
    polyphase form of the strided conv `shape` at this batch (host only)."""
    d = ConvDesc(*[int(v) for v in shape], 0, 0, 0)
    use = ctypes.c_int()
    _check(lib().he_polyphase_advised(int(N), int(L), ctypes.byref(d), int(batch), ctypes.byref(use)),
           "he_polyphase_advised")
    return bool(use.value)


def polyphase_weights(shape, w_dev, wp_dev, stream=None):
    """he_polyphase_weights: int64 [M][C][kh][kw] -> the polyphase conv's weights."""
    C, H, W, M, kh, kw, s, pad = shape
    pc = polyphase_shape(shape)
    d = ConvDesc(*[int(v) for v in shape], 0, 0, 0)
    _check(lib().he_polyphase_weights(ctypes.byref(d), _ptr(w_dev, M * C * kh * kw, "w"),
                                      _ptr(wp_dev, pc[3] * pc[0] * pc[4] * pc[5], "wp"), _stream(stream)),
           "he_polyphase_weights")


def polyphase_input(shape, B: int, x_dev, xp_dev, stream=None):
    """he_polyphase_input: int64 [B][C][H][W] -> the phase channels [B][s*s*C][H'][W']."""
    C, H, W = shape[:3]
    pc = polyphase_shape(shape)
    d = ConvDesc(*[int(v) for v in shape], 0, 0, 0)
    _check(lib().he_polyphase_input(ctypes.byref(d), int(B), _ptr(x_dev, B * C * H * W, "x"),
                                    _ptr(xp_dev, B * pc[0] * pc[1] * pc[2], "xp"), _stream(stream)),
           "he_polyphase_input")


class Context:
    """he_ctx on the current device: parameters, roots and twiddle tables."""

    def __init__(self, N: int, q: list[int], t: int = 2 ** 37):
        self.N, self.L, self.q, self.t = int(N), len(q), [int(v) for v in q], int(t)
        self._qarr = (ctypes.c_uint64 * self.L)(*self.q)
        prm = _Params(self.N, self.L, self._qarr, self.t)
        h = ctypes.c_void_p()
        _check(lib().he_ctx_create(ctypes.byref(prm), ctypes.byref(h)), "he_ctx_create")
        self._h = h
        psi = (ctypes.c_uint64 * self.L)()
        _check(lib().he_ctx_psi(self._h, psi), "he_ctx_psi")
        self.psi = [int(v) for v in psi]

    @classmethod
    def from_bits(cls, N: int, L: int, bits: int, t: int = 2 ** 37) -> "Context":
        return cls(N, gen_primes(N, bits, L), t)

    def close(self):
        if getattr(self, "_h", None):
            lib().he_ctx_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h

    # -- launch-shape tuning ----------------------------------------------
    def get_tuning(self) -> Tuning:
        t = Tuning()
        _check(lib().he_ctx_get_tuning(self._h, ctypes.byref(t)), "he_ctx_get_tuning")
        return t

    def set_tuning(self, **kw) -> Tuning:
        """Change named fields of the tuning (others keep their value)."""
        t = self.get_tuning()
        for k, v in kw.items():
            setattr(t, k, int(v))
        _check(lib().he_ctx_set_tuning(self._h, ctypes.byref(t)), "he_ctx_set_tuning")
        return t

    # -- planning ----------------------------------------------------------
    def plan(self, shape, batch: int = 1, packing=None) -> ConvDesc:
        """Descriptor for a layer shape (C, H, W, M, kh, kw, stride, pad);
        the planner fills the packing unless `packing` = (Cw, Hw, Ww)."""
        d = ConvDesc(*[int(v) for v in shape], 0, 0, 0)
        if packing is None:
            _check(lib().he_plan_conv(self._h, ctypes.byref(d), int(batch)), "he_plan_conv")
        else:
            d.Cw, d.Hw, d.Ww = (int(v) for v in packing)
        self.sizes(d)  # validates
        return d

    def sizes(self, d: ConvDesc) -> Sizes:
        CB, S = ctypes.c_uint32(), ctypes.c_uint32()
        i, o, w = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        _check(lib().he_conv_sizes(self._h, ctypes.byref(d), ctypes.byref(CB), ctypes.byref(S), ctypes.byref(i),
                                   ctypes.byref(o), ctypes.byref(w)), "he_conv_sizes")
        return Sizes(CB.value, S.value, i.value, o.value, w.value)

    # -- the hot path ------------------------------------------------------
    def encode_weights(self, d: ConvDesc, w_dev, wntt_dev, stream=None):
        s = self.sizes(d)
        nw = d.M * d.C * d.kh * d.kw
        _check(lib().he_encode_weights(self._h, ctypes.byref(d), _ptr(w_dev, nw, "weights"),
                                       _ptr(wntt_dev, s.w_words, "wntt"), _stream(stream)), "he_encode_weights")

    def ntt_fwd(self, polys_dev, n: int | None = None, stream=None):
        n = polys_dev.numel() // (self.L * self.N) if n is None else int(n)
        _check(lib().he_ntt_fwd(self._h, _ptr(polys_dev, n * self.L * self.N, "polys"), n, _stream(stream)),
               "he_ntt_fwd")

    def ntt_inv(self, polys_dev, n: int | None = None, stream=None):
        n = polys_dev.numel() // (self.L * self.N) if n is None else int(n)
        _check(lib().he_ntt_inv(self._h, _ptr(polys_dev, n * self.L * self.N, "polys"), n, _stream(stream)),
               "he_ntt_inv")

    def conv_ntt_mac(self, d: ConvDesc, B: int, in_dev, wntt_dev, out_dev, stream=None):
        s = self.sizes(d)
        ct = 2 * self.L * self.N
        _check(lib().he_conv_ntt_mac(self._h, ctypes.byref(d), int(B), _ptr(in_dev, B * s.in_cts * ct, "in"),
                                     _ptr(wntt_dev, s.w_words, "wntt"), _ptr(out_dev, B * s.out_cts * ct, "out"),
                                     _stream(stream)), "he_conv_ntt_mac")

    def conv_mac_intt(self, d: ConvDesc, B: int, in_dev, wntt_dev, out_dev, stream=None):
        s = self.sizes(d)
        ct = 2 * self.L * self.N
        _check(lib().he_conv_mac_intt(self._h, ctypes.byref(d), int(B), _ptr(in_dev, B * s.in_cts * ct, "in"),
                                      _ptr(wntt_dev, s.w_words, "wntt"), _ptr(out_dev, B * s.out_cts * ct, "out"),
                                      _stream(stream)), "he_conv_mac_intt")

    def conv_layer(self, d: ConvDesc, B: int, in_dev, wntt_dev, out_dev, stream=None):
        s = self.sizes(d)
        ct = 2 * self.L * self.N
        _check(lib().he_conv_layer(self._h, ctypes.byref(d), int(B), _ptr(in_dev, B * s.in_cts * ct, "in"),
                                   _ptr(wntt_dev, s.w_words, "wntt"), _ptr(out_dev, B * s.out_cts * ct, "out"),
                                   _stream(stream)), "he_conv_layer")

    @staticmethod
    def out_hw(d: ConvDesc) -> tuple[int, int]:
        """(Ho, Wo): output size at the layer's stride."""
        return ((d.H + 2 * d.pad - d.kh) // d.stride + 1, (d.W + 2 * d.pad - d.kw) // d.stride + 1)

    def add_share(self, d: ConvDesc, B: int, in_dev, share_dev, stream=None):
        """he_add_share: b_l += delta_l * pack(share) on the input cts (in place)."""
        s = self.sizes(d)
        _check(lib().he_add_share(self._h, ctypes.byref(d), int(B),
                                  _ptr(in_dev, B * s.in_cts * 2 * self.L * self.N, "in"),
                                  _ptr(share_dev, B * d.C * d.H * d.W, "share"), _stream(stream)), "he_add_share")

    def mask_extract(self, d: ConvDesc, B: int, out_dev, mask_dev, noise_dev, y_dev, stream=None):
        """he_mask_extract: y[b][m][l][oy][ox] = masked output coefficients."""
        s = self.sizes(d)
        Ho, Wo = self.out_hw(d)
        n = B * d.M * Ho * Wo
        _check(lib().he_mask_extract(self._h, ctypes.byref(d), int(B),
                                     _ptr(out_dev, B * s.out_cts * 2 * self.L * self.N, "out"),
                                     _ptr(mask_dev, n, "mask"), _ptr(noise_dev, n, "noise"),
                                     _ptr(y_dev, n * self.L, "y"), _stream(stream)), "he_mask_extract")

    # -- client side (holds the secret key) ----------------------------------
    def key_encode(self, sk_dev, sk_ntt_dev, stream=None):
        """he_key_encode: sk (int64 [N]) -> NTT form [L][N]."""
        _check(lib().he_key_encode(self._h, _ptr(sk_dev, self.N, "sk"), _ptr(sk_ntt_dev, self.L * self.N, "sk_ntt"),
                                   _stream(stream)), "he_key_encode")

    def encrypt(self, n: int, msgs_dev, a_dev, err_dev, sk_ntt_dev, ct_dev, work_dev, stream=None):
        """he_encrypt: n coefficient-encoded messages -> ct [n][2][L][N]."""
        LN = self.L * self.N
        _check(lib().he_encrypt(self._h, int(n), _ptr(msgs_dev, n * self.N, "msgs"), _ptr(a_dev, n * LN, "a"),
                                _ptr(err_dev, n * self.N, "err"), _ptr(sk_ntt_dev, LN, "sk_ntt"),
                                _ptr(ct_dev, n * 2 * LN, "ct"), _ptr(work_dev, n * LN, "work"), _stream(stream)),
               "he_encrypt")

    def decrypt(self, n: int, ct_dev, sk_ntt_dev, msgs_dev, work_dev, stream=None):
        """he_decrypt: ct [n][2][L][N] -> centred messages int64 [n][N]."""
        LN = self.L * self.N
        _check(lib().he_decrypt(self._h, int(n), _ptr(ct_dev, n * 2 * LN, "ct"), _ptr(sk_ntt_dev, LN, "sk_ntt"),
                                _ptr(msgs_dev, n * self.N, "msgs"), _ptr(work_dev, n * LN, "work"),
                                _stream(stream)), "he_decrypt")

    # ---- rotation (this context is the extended one: L-1 ciphertext primes, then P) ----

    def keyswitch_work_words(self, n: int) -> int:
        """he_keyswitch_work_words: scratch words for n ciphertexts."""
        w = ctypes.c_uint64()
        _check(lib().he_keyswitch_work_words(self._h, int(n), ctypes.byref(w)), "he_keyswitch_work_words")
        return int(w.value)

    def galois_key_work_words(self) -> int:
        """Scratch words of galois_key: (2L+2)*(L+1)*N for L = self.L - 1."""
        return 2 * self.L * self.L * self.N

    def galois_key(self, g: int, sk_dev, a_dev, err_dev, ksk_ntt_dev, work_dev, stream=None):
        """he_galois_key (client side): the key for g in NTT form [L][2][L+1][N]."""
        Lc, N = self.L - 1, self.N
        _check(lib().he_galois_key(self._h, int(g), _ptr(sk_dev, N, "sk"), _ptr(a_dev, Lc * self.L * N, "a"),
                                   _ptr(err_dev, Lc * N, "err"), _ptr(ksk_ntt_dev, Lc * 2 * self.L * N, "ksk"),
                                   _ptr(work_dev, self.galois_key_work_words(), "work"), _stream(stream)),
               "he_galois_key")

    def automorph(self, g: int, n: int, in_dev, out_dev, stream=None):
        """he_automorph: a(X) -> a(X^g) of n RNS polynomials [n][L][N]."""
        LN = self.L * self.N
        _check(lib().he_automorph(self._h, int(g), int(n), _ptr(in_dev, n * LN, "in"), _ptr(out_dev, n * LN, "out"),
                                  _stream(stream)), "he_automorph")

    def keyswitch(self, n: int, ct_dev, ksk_ntt_dev, out_dev, work_dev, stream=None):
        """he_keyswitch on the extended context: ct [n][2][L-1][N] -> out."""
        Lc = self.L - 1
        ct = n * 2 * Lc * self.N
        _check(lib().he_keyswitch(self._h, int(n), _ptr(ct_dev, ct, "ct"),
                                  _ptr(ksk_ntt_dev, Lc * 2 * self.L * self.N, "ksk"), _ptr(out_dev, ct, "out"),
                                  _ptr(work_dev, self.keyswitch_work_words(n), "work"), _stream(stream)),
               "he_keyswitch")

    def rotate(self, g: int, n: int, ct_dev, ksk_ntt_dev, out_dev, work_dev, stream=None):
        """he_rotate on the extended context: automorphism by g, then key switching."""
        Lc = self.L - 1
        ct = n * 2 * Lc * self.N
        _check(lib().he_rotate(self._h, int(g), int(n), _ptr(ct_dev, ct, "ct"),
                               _ptr(ksk_ntt_dev, Lc * 2 * self.L * self.N, "ksk"), _ptr(out_dev, ct, "out"),
                               _ptr(work_dev, self.keyswitch_work_words(n), "work"), _stream(stream)),
               "he_rotate")

    def rotate_noalloc(self, g: int, n: int, ct_dev, ksk_ntt_dev, out_dev, stream=None):
        """he_rotate_noalloc: he_rotate with the library's fixed device scratch
        (no work buffer, no allocation; calls on one GPU must not overlap)."""
        Lc = self.L - 1
        ct = n * 2 * Lc * self.N
        _check(lib().he_rotate_noalloc(self._h, int(g), int(n), _ptr(ct_dev, ct, "ct"),
                                       _ptr(ksk_ntt_dev, Lc * 2 * self.L * self.N, "ksk"), _ptr(out_dev, ct, "out"),
                                       _stream(stream)),
               "he_rotate_noalloc")

    def probe_valu(self, which: int, iters: int, blocks: int = 2048) -> float:
        """he_probe_valu (include/heconv_probe.h): the measured rate of one
        integer instruction or of one kernel's arithmetic mix, in that
        probe's unit per second (synchronises the current stream)."""
        import torch
        work = torch.randint(1, 2 ** 62, (64 + 256 * blocks,), dtype=torch.int64, device="cuda")
        rate = ctypes.c_double(0.0)
        _check(lib().he_probe_valu(self._h, int(which), int(iters), int(blocks), _ptr(work, 64 + 256 * blocks, "work"),
                                   ctypes.byref(rate), _stream(None)), "he_probe_valu")
        return rate.value

    # ---- Z_P variant (slot calls on a one-prime context over t) ----

    def simd_encode(self, n: int, slots_dev, coeffs_dev, stream=None):
        """he_simd_encode: slots [n][N] -> centred plaintext coefficients [n][N]."""
        _check(lib().he_simd_encode(self._h, int(n), _ptr(slots_dev, n * self.N, "slots"),
                                    _ptr(coeffs_dev, n * self.N, "coeffs"), _stream(stream)), "he_simd_encode")

    def simd_decode(self, n: int, coeffs_dev, slots_dev, work_dev, stream=None):
        """he_simd_decode: plaintext coefficients [n][N] -> slots [n][N]."""
        _check(lib().he_simd_decode(self._h, int(n), _ptr(coeffs_dev, n * self.N, "coeffs"),
                                    _ptr(slots_dev, n * self.N, "slots"), _ptr(work_dev, n * self.N, "work"),
                                    _stream(stream)), "he_simd_decode")

    def zp_diagonals(self, w_dev, rows: int, cols: int, n: int, slots_dev, stream=None):
        """he_zp_diagonals: W [rows][cols] -> n diagonal slot vectors [n][N]."""
        _check(lib().he_zp_diagonals(self._h, _ptr(w_dev, rows * cols, "W"), int(rows), int(cols), int(n),
                                     _ptr(slots_dev, n * self.N, "slots"), _stream(stream)), "he_zp_diagonals")

    def zp_diagonals_rect(self, w_dev, rows: int, cols: int, n_out: int, n_in: int, slots_dev, stream=None):
        """he_zp_diagonals_rect: W [rows][cols] -> n_out generalized diagonals [n_out][N]."""
        _check(lib().he_zp_diagonals_rect(self._h, _ptr(w_dev, rows * cols, "W"), int(rows), int(cols), int(n_out),
                                          int(n_in), _ptr(slots_dev, n_out * self.N, "slots"), _stream(stream)),
               "he_zp_diagonals_rect")

    def zp_fold(self, g: int, n: int, ct_dev, ksk_ntt_dev, out_dev, work_dev, stream=None):
        """he_zp_fold (extended context): out = ct + rotate(ct, g)."""
        Lc, N = self.L - 1, self.N
        ct = n * 2 * Lc * N
        _check(lib().he_zp_fold(self._h, int(g), int(n), _ptr(ct_dev, ct, "ct"),
                                _ptr(ksk_ntt_dev, Lc * 2 * self.L * N, "ksk"), _ptr(out_dev, ct, "out"),
                                _ptr(work_dev, self.keyswitch_work_words(n), "work"), _stream(stream)), "he_zp_fold")

    def zp_encode_plain(self, n: int, coeffs_dev, w_dev, stream=None):
        """he_zp_encode_plain (extended context): coefficients [n][N] -> [n][L-1][N]."""
        _check(lib().he_zp_encode_plain(self._h, int(n), _ptr(coeffs_dev, n * self.N, "coeffs"),
                                        _ptr(w_dev, n * (self.L - 1) * self.N, "w"), _stream(stream)),
               "he_zp_encode_plain")

    def zp_work_words(self, n: int) -> int:
        w = ctypes.c_uint64()
        _check(lib().he_zp_work_words(self._h, int(n), ctypes.byref(w)), "he_zp_work_words")
        return int(w.value)

    def zp_matvec(self, g: int, n: int, x_ntt_dev, w_dev, n_diag: int, ksk_ntt_dev, out_dev, work_dev,
                  stream=None):
        """he_zp_matvec (extended context): the multiply-accumulate-rotate kernel."""
        Lc, N = self.L - 1, self.N
        ct = n * 2 * Lc * N
        _check(lib().he_zp_matvec(self._h, int(g), int(n), _ptr(x_ntt_dev, ct, "x_ntt"),
                                  _ptr(w_dev, n_diag * Lc * N, "w"), int(n_diag),
                                  _ptr(ksk_ntt_dev, Lc * 2 * self.L * N, "ksk"), _ptr(out_dev, ct, "out"),
                                  _ptr(work_dev, self.zp_work_words(n), "work"), _stream(stream)), "he_zp_matvec")

    def zp_grouped_work_words(self, n: int, groups: int) -> int:
        w = ctypes.c_uint64()
        _check(lib().he_zp_grouped_work_words(self._h, int(n), int(groups), ctypes.byref(w)),
               "he_zp_grouped_work_words")
        return int(w.value)

    def zp_matvec_grouped(self, g: int, n: int, x_ntt_dev, w_dev, n_diag: int, groups: int, ksk_ntt_dev, g2: int,
                          ksk2_ntt_dev, out_dev, work_dev, stream=None):
        """he_zp_matvec_grouped (extended context): the kernel as `groups` chains."""
        Lc, N = self.L - 1, self.N
        ct = n * 2 * Lc * N
        kw = Lc * 2 * self.L * N
        _check(lib().he_zp_matvec_grouped(self._h, int(g), int(n), _ptr(x_ntt_dev, ct, "x_ntt"),
                                          _ptr(w_dev, n_diag * Lc * N, "w"), int(n_diag), int(groups),
                                          _ptr(ksk_ntt_dev, kw, "ksk"), int(g2),
                                          _ptr(ksk2_ntt_dev, kw, "ksk2") if ksk2_ntt_dev is not None else None,
                                          _ptr(out_dev, ct, "out"),
                                          _ptr(work_dev, self.zp_grouped_work_words(n, groups), "work"),
                                          _stream(stream)), "he_zp_matvec_grouped")


class Batch:
    """he_batch: many layer solves in one launch (three grids per chain,
    optionally one hipGraph).

    jobs: list of (desc, B, d_in, d_wntt, d_out) with device tensors; the
    tensors are kept referenced for the batch's lifetime."""

    def __init__(self, ctx: Context, jobs, schedule: int = SCHED_ONE_CHAIN):
        self.ctx = ctx
        self.n_jobs = len(jobs)
        self._keep = []
        arr = (_Job * len(jobs))()
        ct = 2 * ctx.L * ctx.N
        for i, (d, B, din, dw, dout) in enumerate(jobs):
            s = ctx.sizes(d)
            arr[i] = _Job(d, int(B), _ptr(din, B * s.in_cts * ct, "in"), _ptr(dw, s.w_words, "wntt"),
                          _ptr(dout, B * s.out_cts * ct, "out"))
            self._keep += [din, dw, dout]
        h = ctypes.c_void_p()
        _check(lib().he_batch_create(ctx.handle, arr, len(jobs), int(schedule), ctypes.byref(h)), "he_batch_create")
        self._h = h
        n, c = ctypes.c_uint64(), ctypes.c_uint32()
        _check(lib().he_batch_info(self._h, ctypes.byref(n), ctypes.byref(c)), "he_batch_info")
        self.n_items, self.n_chains = n.value, c.value
        f = [ctypes.c_uint32() for _ in range(5)]
        _check(lib().he_batch_mac_form(self._h, *[ctypes.byref(v) for v in f]), "he_batch_mac_form")
        # the MAC form the batch picked: register tile, LDS stages, tiles per
        # workgroup of the streamed MAC, 2x2 wave grid
        self.mac_form = dict(zip(("mt", "rt", "lds", "tiles", "grid"), (v.value for v in f)))

    def launch(self, stream=None, graph: bool = True):
        _check(lib().he_batch_launch(self._h, _stream(stream), int(bool(graph))), "he_batch_launch")

    def launch_timed(self, stream=None):
        """he_batch_launch_timed: one eager execution with events around every
        grid; returns [[fwd, mac, inv] ms per chain] (synchronises)."""
        ms = (ctypes.c_float * 6)()
        _check(lib().he_batch_launch_timed(self._h, _stream(stream), ms), "he_batch_launch_timed")
        return [[ms[3 * c + p] for p in range(3)] for c in range(self.n_chains)]

    def status(self, stream=None):
        _check(lib().he_batch_status(self._h, _stream(stream)), "he_batch_status")

    def close(self):
        if getattr(self, "_h", None):
            lib().he_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
