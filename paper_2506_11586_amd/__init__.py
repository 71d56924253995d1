"""MI355X-native homomorphic-convolution hot path (SecONNds, arXiv 2506.11586,
Sec. 6.2): forward NTT of RNS BFV ciphertexts, channel-block MAC against
NTT-preprocessed weights, inverse NTT -- hand-written HIP for gfx950 behind
the C ABI in include/heconv.h.  `heconv` is the ctypes binding."""
from . import heconv  # noqa: F401
from .heconv import ConvDesc, Context, HeError, gen_primes  # noqa: F401
