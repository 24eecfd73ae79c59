"""The device path's HIP source executed on the CPU (tests/emu), checked against the oracle.

The executor runs every GPU thread of every kernel as a fiber with lockstep
wave intrinsics, so the kernels' logic (block-start search, symbolic inflate,
stitching, window propagation, translation) is exercised here without a GPU.
The executor also reports divergence bugs (lanes of one wave at different
intrinsics) and deadlocks by aborting the run.
"""
import numpy as np
import pytest

import synth
from bitwriter import gzip_wrap

E = pytest.importorskip("emu_harness")

NONE = (1 << 64) - 1


def _starts(tab):
    return np.array([-1 if int(s) == NONE else int(s) for s in tab["start"]], dtype=np.int64)


def _check(orc, comp, n, raw):
    st, out, r, tab = E.run(comp, n, out_cap=len(raw) + 64, sync_limit=3_000_000_000)
    ref = orc.pugz(comp, n)
    assert ref.status == orc.OK, ref.reason
    assert st == 0
    assert out == raw == ref.out.tobytes()
    assert np.array_equal(_starts(tab), ref.start), (list(_starts(tab)), list(ref.start))
    ne = ref.start >= 0
    assert np.array_equal(tab["end"][ne].astype(np.int64), ref.end[ne])
    assert np.array_equal(tab["len"][ne].astype(np.int64), ref.len[ne])
    assert np.array_equal(tab["out_off"][ne].astype(np.int64), ref.off[ne])
    assert r.n_placeholders == int(ref.placeholders.sum())
    return r, tab


def test_emu_handbuilt(orc):
    from test_oracle import HAND, wrap_tokens

    for name, blocks in HAND.items():
        deflate, data = wrap_tokens(blocks)
        st, out, r, tab = E.run(gzip_wrap(deflate, data), 1, out_cap=len(data) + 16)
        assert st == 0 and out == data, name


@pytest.mark.parametrize("kind,level,n", [("fastq", 6, 3), ("words", 6, 4), ("fastq", 1, 3), ("fastq", 9, 2)])
def test_emu_multichunk(orc, kind, level, n):
    raw = (synth.fastq_like(160 << 10, 301) if kind == "fastq" else synth.word_stream(160 << 10, 302))
    comp = synth.gzip_member(raw, level)
    _check(orc, comp, n, raw)


def test_emu_more_chunks_than_blocks(orc):
    raw = synth.fastq_like(120 << 10, 303)
    comp = synth.gzip_member(raw, 6)
    r, tab = _check(orc, comp, 40, raw)
    assert (tab["start"] == NONE).sum() > 20


def test_emu_segmented_and_stored(orc):
    raw = synth.fastq_like(200 << 10, 304)
    comp = synth.gzip_member(raw, 6, segment_bytes=48 << 10)
    _check(orc, comp, 4, raw)
    comp0 = synth.gzip_member(raw[:70000], 0)
    st, out, r, tab = E.run(comp0, 3, out_cap=70064)
    assert st == 0 and out == raw[:70000]


def test_emu_window_sizes(orc):
    raw = synth.fastq_like(100 << 10, 305)
    comp = synth.gzip_member(raw, 6)
    for win in (4096, 8192, 16384, 32768):
        st, out, r, tab = E.run(comp, 3, out_cap=len(raw) + 64, window_syms=win)
        assert st == 0 and out == raw


def test_emu_errors(orc):
    raw = synth.word_stream(60 << 10, 306)
    comp = bytearray(synth.gzip_member(raw, 6))
    bad = bytearray(comp)
    bad[-4] ^= 1
    st, out, r, tab = E.run(bytes(bad), 2, out_cap=len(raw) + 64)
    assert st == -7
    st, out, r, tab = E.run(bytes(comp) + synth.gzip_member(b"zz", 6), 2, out_cap=len(raw) + 64)
    assert st == -3
    st, out, r, tab = E.run(bytes(comp[: len(comp) // 2]) + bytes(comp[-8:]), 2, out_cap=len(raw) + 64)
    assert st == -4
    st, out, r, tab = E.run(bytes(comp), 2, out_cap=100)
    assert st == -5 and r.out_needed == len(raw)


def test_emu_short_distances(orc):
    # matches whose source lies in the same 64-symbol batch (distances 1..63,
    # lengths up to 258): runs, short periods, and periods just under and over 64
    rng = np.random.default_rng(307)
    parts = [b"A" * 5000, b"ab" * 3000, b"xyz" * 2000]
    for period in (5, 17, 63, 64, 65, 130):
        unit = bytes(rng.integers(97, 123, period, dtype=np.uint8))
        parts.append(unit * (4000 // period))
        parts.append(bytes(rng.integers(32, 127, 300, dtype=np.uint8)))
    raw = b"".join(parts)
    for level in (1, 6, 9):
        comp = synth.gzip_member(raw, level)
        # far more symbols per compressed byte than the default capacity factor
        st, out, r, tab = E.run(comp, 1, out_cap=len(raw) + 64, sym_factor=4096)
        assert st == 0 and out == raw, level
