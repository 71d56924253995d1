"""Host-side checks of the C ABI that need no GPU: the library loads and
exports every function include/heconv.h declares, and its host logic (prime
search, root choice, planner) agrees with the oracle's independent code."""
import ctypes
import os
import re

import pytest

import oracle
import synth
from tests.libload import ensure_built

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "heconv.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(he_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    path = ensure_built()
    lib = ctypes.CDLL(path)
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings():
    ensure_built()
    from paper_2506_11586_amd import heconv
    for s in range(-6, 1):
        assert heconv.lib().he_status_str(s).decode()


@pytest.mark.parametrize("N,bits,L", [(4096, 50, 2), (8192, 60, 3), (1024, 40, 4), (16384, 60, 2)])
def test_primes_and_roots_match_oracle(N, bits, L):
    ensure_built()
    from paper_2506_11586_amd import heconv
    qs = heconv.gen_primes(N, bits, L)
    assert qs == oracle.find_primes(N, bits, L)
    for q in qs:
        assert heconv.min_root(q, N) == oracle.find_psi(q, N)


def test_bad_parameters_rejected():
    ensure_built()
    from paper_2506_11586_amd import heconv
    with pytest.raises(heconv.HeError):
        heconv.gen_primes(1000, 50, 2)  # N not a power of two
    with pytest.raises(heconv.HeError):
        heconv.min_root(1125899906826241 + 2, 4096)  # not 1 mod 2N
    with pytest.raises(heconv.HeError):
        heconv.plan_host(4096, 2, (4, 16, 16, 4, 0, 3, 1, 1))  # zero kernel height


def all_shapes():
    shapes = set()
    for cfg in synth.WORKLOADS.values():
        for s in cfg["layers"]:
            shapes.add((cfg["N"], cfg["L"], s))
    return sorted(shapes)


def test_planner_matches_oracle_on_every_workload_shape():
    """Same descriptor from the library's planner and the oracle's, for every
    layer of every workload, at batch 1 and 16."""
    ensure_built()
    from paper_2506_11586_amd import heconv
    for N, L, s in all_shapes():
        for B in (1, 16):
            d = heconv.plan_host(N, L, s, B)
            g = oracle.plan_conv(oracle.Conv(*s), N, L, B)
            assert (d.Cw, d.Hw, d.Ww) == (g.Cw, g.Hw, g.Ww), (s, B)


@pytest.mark.parametrize("N,bits,L,t", [(4096, 50, 2, 2 ** 37), (8192, 60, 3, 2 ** 37), (1024, 40, 4, 3),
                                        (2048, 31, 1, 2 ** 30 + 3), (8192, 60, 8, 2 ** 62)])
def test_delta_matches_oracle(N, bits, L, t):
    """delta_l = floor(Q/t) mod q_l from the library's multi-word arithmetic
    equals the oracle's Python big integers."""
    ensure_built()
    from paper_2506_11586_amd import heconv
    prm = oracle.Params(N, L, bits, t)
    assert heconv.delta_host(prm.q, t) == prm.delta_l


def test_delta_rejects_unusable_t():
    ensure_built()
    from paper_2506_11586_amd import heconv
    q = oracle.find_primes(1024, 31, 1)
    for t in (0, 1, 2 ** 62 + 1, q[0] + 1):
        with pytest.raises(heconv.HeError) as e:
            heconv.delta_host(q, t)
        assert e.value.status == heconv.HE_EPARAM


def test_polyphase_descriptor_matches_oracle():
    """he_polyphase_desc (host only) equals the oracle's polyphase conv for
    strides 2 and 3 and several kernels; stride 1 is HE_ESHAPE."""
    import oracle
    from paper_2506_11586_amd import heconv
    for shape in [(3, 224, 224, 64, 3, 3, 2, 1), (3, 224, 224, 64, 7, 7, 2, 3), (128, 56, 56, 128, 3, 3, 2, 1),
                  (2, 9, 11, 3, 5, 5, 2, 2), (3, 17, 17, 2, 3, 3, 3, 1), (4, 12, 12, 2, 1, 1, 2, 0)]:
        pc = oracle.polyphase_conv(oracle.Conv(*shape))
        assert heconv.polyphase_shape(shape) == (pc.C, pc.H, pc.W, pc.M, pc.kh, pc.kw, pc.stride, pc.pad)
    with pytest.raises(heconv.HeError) as e:
        heconv.polyphase_shape((3, 16, 16, 4, 3, 3, 1, 1))
    assert e.value.status == heconv.HE_ESHAPE


def test_polyphase_advice_matches_oracle_costs():
    """he_polyphase_advised equals the decision taken from the oracle
    planner's costs of both forms (bytes, then modmuls) for the strided
    layers of the two CNNs at their batches; stride 1 is never advised."""
    import oracle
    import synth
    from paper_2506_11586_amd import heconv
    seen = 0
    for wl in ("fire_cnn", "bottleneck_cnn_b16"):
        cfg = synth.WORKLOADS[wl]
        B = cfg.get("batch", 1)
        for shape in cfg["layers"]:
            if shape[6] == 1:
                assert not heconv.polyphase_advised(cfg["N"], cfg["L"], shape, B)
                continue
            cv = oracle.Conv(*shape)
            pc = oracle.polyphase_conv(cv)
            bs, ms = oracle.layer_cost(cv, oracle.plan_conv(cv, cfg["N"], cfg["L"], B), cfg["N"], cfg["L"], B)
            bp, mp = oracle.layer_cost(pc, oracle.plan_conv(pc, cfg["N"], cfg["L"], B), cfg["N"], cfg["L"], B)
            want = bp < bs or (bp == bs and mp < ms)
            assert heconv.polyphase_advised(cfg["N"], cfg["L"], shape, B) == want, shape
            seen += 1
    assert seen >= 5
    assert heconv.polyphase_advised(8192, 3, (3, 224, 224, 64, 3, 3, 2, 1), 1)
