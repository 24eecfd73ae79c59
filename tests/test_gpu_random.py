"""Random access (Section IV) through the C ABI (needs an MI355X).

Block-start probes equal the oracle's search (Section VI-A, Appendix A) at
every offset.  Decoding from block 2 with an undetermined context gives,
byte for byte, the oracle's symbolic decode with every placeholder shown as
the marker, and the per-window undetermined counts equal the oracle's.  The
measurements of Section IV-C and Fig. 2 are pinned where the paper prints
them: random DNA at level 6 has a mean match distance near o_a = 3602 and
its undetermined share vanishes after about 150 windows of o_a; levels 1 to
3 emit (almost) no literals after block 2, so it never vanishes; at level 9
it does not vanish within 1 Mbp; in the 150 DNA + 300 'x' string at level 1
the DNA becomes fully determined, after more than 7000 windows.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

O_A = 3602  # average match offset at level 6 on random DNA (Section IV-C)
NONE = (1 << 64) - 1


def _say(*a):
    print("[case]", *a, flush=True)


def _dev(b):
    return torch.frombuffer(bytearray(b), dtype=torch.uint8).to("cuda:0")


def _oracle_profile(orc, comp, bit, window):
    sr = orc.symbolic(comp, bit, 1 << 62, first=False)
    assert sr.status == orc.OK
    und = sr.sym >= 0x8000
    counts = np.add.reduceat(und.astype(np.int64), np.arange(0, und.size, window))
    return sr.sym, und, counts


def _random_access(comp, bit, window, marker=0, segment_bytes=0, **opts):
    import paper_1905_07224_amd as gz

    s = gz.Stream(_dev(comp), segment_bytes, at_bit=bit, marker=marker, **opts)
    parts = [p.cpu().numpy().copy() for p in s]
    assert s.last["done"] == 1
    s.close()
    out = np.concatenate(parts) if parts else np.zeros(0, np.uint8)
    start, total, counts = gz.undetermined_profile(_dev(comp), bit, window, marker=marker,
                                                   segment_bytes=segment_bytes, **opts)
    assert start == bit and total == out.size
    return out, counts


def test_probes_match_oracle(orc):
    import paper_1905_07224_amd as gz

    raw = synth.fastq_like(8 << 20, 901)
    comp = synth.gzip_member(raw, 6)
    g = orc.gunzip(comp)
    lo, hi = 8 * g.payload_start, 8 * (len(comp) - 8)
    rng = np.random.default_rng(5)
    bits = sorted(set([lo, int(g.block_bit[3]), int(g.block_bit[3]) + 1, hi - 8 * 100]
                      + [int(x) for x in rng.integers(lo, hi - 8 * 100, 40)]))
    _say("probes", len(bits))
    starts, rej = gz.find_blocks(_dev(comp), bits, 256 << 10)
    for b, s in zip(bits, starts):
        ref = orc.find_start(comp, b, min(hi, b + 8 * (256 << 10)))
        assert (s if s is not None else -1) == ref, b
        if s is not None:
            assert s in set(g.block_bit.tolist())
    assert starts[-1] is None


def test_probes_full_size(orc):
    """64 probes across the 1 GiB FASTQ-like member in one launch."""
    import paper_1905_07224_amd as gz

    raw, comp = synth.workload("fastq_1GiB_L6")
    lo, hi = 8 * 10, 8 * (len(comp) - 8)
    bits = [int(x) for x in np.random.default_rng(6).integers(lo, hi - 8 * (1 << 20), 64)]
    _say("probes across fastq_1GiB_L6", len(bits))
    starts, rej = gz.find_blocks(_dev(comp), bits, 1 << 20)
    for b, s in zip(bits, starts[:12]):
        ref = orc.find_start(comp, b, b + 8 * (1 << 20))
        assert (s if s is not None else -1) == ref, b
    assert all(s is not None and s >= b for b, s in zip(bits, starts))


@pytest.mark.parametrize("level", [1, 2, 3, 4, 6, 9])
def test_fig2_random_dna(orc, level):
    raw = synth.random_dna(1_000_000, 2019)
    comp = synth.gzip_member(raw, level)
    g = orc.gunzip(comp, parent=True)
    b = int(g.block_bit[1])  # decoding starts at block 2
    _say("random DNA 1 Mbp, level", level)
    out, counts = _random_access(comp, b, O_A, marker=0, segment_bytes=64 << 10, chunk_bytes=8192)
    sym, und, ref_counts = _oracle_profile(orc, comp, b, O_A)
    assert np.array_equal(out, np.where(und, 0, sym).astype(np.uint8))
    assert np.array_equal(counts, ref_counts)
    nz = np.nonzero(counts)[0]
    last = int(nz[-1]) if nz.size else -1
    par = g.parent
    lits_after = int((par[int(g.block_out_off[1]):] < 0).sum())
    if level <= 3:
        # (almost) no literal after block 2: undetermined to the end
        assert lits_after <= 8 and last == counts.size - 1
    elif level in (4, 6):
        assert 60 <= last <= 250, last
        assert not counts[last + 1:].any()
    else:
        assert last == counts.size - 1
    if level == 6:
        d = np.arange(par.size)[par >= 0] - par[par >= 0]
        assert abs(d.mean() - O_A) < 0.1 * O_A


@pytest.mark.parametrize("level", range(1, 10))
def test_fig2_dna_x_string(orc, level):
    """The 150 DNA + 300 'x' string (150 MB) decoded from block 2: the
    undetermined count per o_a window equals the oracle's, and so does the
    count over the DNA positions alone, which the device output gives byte
    for byte.  The 'x' runs stay undetermined (they are copies); the DNA
    becomes fully determined after more than 7000 windows at levels 1 and 2
    (Section IV-D reports this for the lowest level), never within the
    string at level 3, and within 1000 windows at levels 4 to 9."""
    raw = synth.dna_x_string(150_000_000, 2020)
    comp = synth.gzip_member(raw, level)
    g = orc.gunzip(comp)
    b = int(g.block_bit[1])
    _say("150 DNA + 300 x, 150 MB, level", level)
    out, counts_all = _random_access(comp, b, O_A, marker=0, segment_bytes=16 << 20)
    sym, und, ref_all = _oracle_profile(orc, comp, b, O_A)
    assert out.size == und.size and np.array_equal(counts_all, ref_all)
    # the DNA bases only: positions whose offset in the 450-byte period is below 150
    o = int(g.block_out_off[1])
    dna = ((np.arange(und.size) + o) % 450) < 150
    edges = np.arange(0, und.size, O_A)
    c = np.add.reduceat((und & dna).astype(np.int64), edges)
    c_dev = np.add.reduceat(((out == 0) & dna).astype(np.int64), edges)
    assert np.array_equal(c_dev, c)
    nz = np.nonzero(c)[0]
    assert ref_all[-1] > 0
    if level <= 2:
        assert nz.size and 7000 < nz[-1] < c.size - 100
    elif level == 3:
        assert nz[-1] == c.size - 1
    else:
        assert nz[-1] < 1000


@pytest.mark.parametrize("level,window", [(6, O_A), (9, 12755)])
def test_fig2_model_line(orc, level, window):
    """Fig. 2's model line (Section V-C, 1 - L_i with L_1 = E_l / W) against
    the device's undetermined share per window on random DNA from block 2:
    level 6 with windows of o_a, level 9 with windows of o'_a = 12755; the
    counts equal the oracle's, and the model stays within 0.1 of the
    measured share and within 0.04 in RMS over 150 windows."""
    import paper_1905_07224_amd as gz
    from paper_1905_07224_amd import analytics as A

    raw = synth.random_dna(1_000_000, 2019)
    comp = synth.gzip_member(raw, level)
    g = orc.gunzip(comp)
    b = int(g.block_bit[1])
    _say("model line, level", level, "window", window)
    start, total, counts = gz.undetermined_profile(_dev(comp), b, window, marker=0, segment_bytes=64 << 10,
                                                   chunk_bytes=8192)
    _, und, ref = _oracle_profile(orc, comp, b, window)
    assert np.array_equal(counts, ref)
    n = min(150, total // window)
    frac = counts[:n] / window
    model = np.array(A.undetermined_model(n, A.lazy_literals() / A.WINDOW))
    assert np.abs(frac - model).max() < 0.1 and np.sqrt(((frac - model) ** 2).mean()) < 0.04


def test_random_access_c2_half(orc):
    """From the block after half of the 1 GiB member to its end: the bytes
    equal the oracle's symbolic decode with placeholders as markers."""
    import paper_1905_07224_amd as gz

    raw, comp = synth.workload("fastq_1GiB_L6")
    bit = 8 * (len(comp) // 2)
    starts, _ = gz.find_blocks(_dev(comp), [bit], 1 << 20)
    b = starts[0]
    assert b is not None and b == orc.find_start(comp, bit, bit + 8 * (1 << 20))
    _say("random access at half of fastq_1GiB_L6, block", b)
    out, counts = _random_access(comp, b, 1 << 20, marker=255, segment_bytes=64 << 20)
    sr = orc.symbolic(comp, b, 1 << 62, first=False)
    und = sr.sym >= 0x8000
    assert np.array_equal(out, np.where(und, 255, sr.sym).astype(np.uint8))
    assert int(counts.sum()) == int(und.sum())
    assert not (np.frombuffer(raw, np.uint8) == 255).any()
