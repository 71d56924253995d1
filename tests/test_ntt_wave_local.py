"""Host check of the NTT kernels' thread/element mappings: a transpose
between two mappings whose low split is at bit 6 or below stays inside each
wave (the kernels run it without workgroup barriers), wave blocks are
disjoint, the transpose before a wave-local one ends with every wave
reading its own block, and the full transforms' first transpose is
cross-wave unless the workgroup is a single wave (a kernel may use LDS just
before the transform: the rotation kernel stages the row there; the
two-grid forward's second grid reads its input from global memory, so its
first transpose may be wave-local).  The mapping of a pass at bit offset LO:
register k of thread t holds element (t mod 2^LO) | k << LO | (t >> LO) <<
(LO + loge); the transform sequences are those of the forward (bits from
the top down, then back to the top mapping for the store), the inverse
(from the top mapping to bit 0, then up) and the two-grid forward's second
grid (128 threads over a 1024-element block)."""
import pytest


def elem(loge, lo, t, k):
    return (t & ((1 << lo) - 1)) | (k << lo) | ((t >> lo) << (lo + loge))


def wave_local(frm, to):
    return frm <= 6 and to <= 6


def fwd_seq(logn, loge):
    nfull, rem = logn // loge, logn % loge
    seq = [(logn - loge * p, logn - loge * (p + 1)) for p in range(1, nfull)]
    if rem:
        seq.append((logn - loge * nfull, 0))
    return seq + [(0, logn - loge)]


def inv_seq(logn, loge):
    nfull, rem = logn // loge, logn % loge
    seq = [(logn - loge, 0)]
    for p in range(nfull):
        if p > 0 or rem > 0:
            seq.append((0 if p == 0 else rem + loge * (p - 1), rem + loge * p))
    return seq


def split_b_seq(logn):
    nb = logn - 6
    nfull, rem = nb // 3, nb % 3
    seq = [(nb - 3 * p, nb - 3 * (p + 1)) for p in range(1, nfull)]
    if rem:
        seq.append((nb - 3 * nfull, 0))
    return seq + [(0, 7)]


def check(loge, seq, threads, lds_before=True):
    e = 1 << loge
    waves = (threads + 63) // 64
    frm0, to0 = seq[0]
    assert not (lds_before and wave_local(frm0, to0)) or waves == 1
    for s, (frm, to) in enumerate(seq):
        if not wave_local(frm, to):
            continue
        blocks = []
        for w in range(waves):
            ts = range(64 * w, min(64 * w + 64, threads))
            a = {elem(loge, frm, t, k) for t in ts for k in range(e)}
            assert a == {elem(loge, to, t, k) for t in ts for k in range(e)}
            assert a == set(range(w * (e << 6), (w + 1) * (e << 6)))  # aligned block
            blocks.append(a)
        assert sum(len(b) for b in blocks) == len(set().union(*blocks))
        if s > 0:
            assert seq[s - 1][1] <= 6 or waves == 1


@pytest.mark.parametrize("logn", range(10, 16))
@pytest.mark.parametrize("loge", [3, 4])
def test_full_transforms(logn, loge):
    threads = (1 << logn) >> loge
    if threads > 1024:
        pytest.skip("more threads than a workgroup holds: not instantiated")
    check(loge, fwd_seq(logn, loge), threads)
    check(loge, inv_seq(logn, loge), threads)


@pytest.mark.parametrize("logn", [12, 13, 14])
def test_two_grid_forward_second_grid(logn):
    check(3, split_b_seq(logn), 128, lds_before=False)


def test_the_8192_point_sequences():
    """The 64->64 layer's transforms: two of five transposes wave-local in
    each direction."""
    assert fwd_seq(13, 3) == [(10, 7), (7, 4), (4, 1), (1, 0), (0, 10)]
    assert inv_seq(13, 3) == [(10, 0), (0, 1), (1, 4), (4, 7), (7, 10)]
    assert [wave_local(*p) for p in fwd_seq(13, 3)] == [False, False, True, True, False]
    assert [wave_local(*p) for p in inv_seq(13, 3)] == [False, True, True, False, False]
