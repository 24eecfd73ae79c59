"""Device path against the CPU oracle, through the C ABI (needs an MI355X).

Bytes, chunk starts, chunk ends, symbol counts, the 16-bit symbolic output of
pass 1, the resolved windows and the statuses are compared with the oracle on
the same seeded inputs.  All of it is integer work, so the bar is equality.
"""
import numpy as np
import pytest

import synth
from bitwriter import gzip_wrap

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _gz():
    import paper_1905_07224_amd as gz
    return gz


def _dev(b):
    return torch.frombuffer(bytearray(b), dtype=torch.uint8).to("cuda:0")


def _say(*a):
    print("[case]", *a, flush=True)


def _run(comp, n_chunks, **opts):
    gz = _gz()
    plan = gz.Plan(_dev(comp), n_chunks, **opts)
    out = plan.run()
    torch.cuda.synchronize()
    return out.cpu().numpy().tobytes(), plan


def _starts(tab):
    gz = _gz()
    return np.array([-1 if int(s) == gz.NONE else int(s) for s in tab["start"]], dtype=np.int64)


def _check_against_oracle(orc, comp, n_chunks, raw=None, **opts):
    got, plan = _run(comp, n_chunks, **opts)
    ref = orc.pugz(comp, n_chunks)
    assert ref.status == orc.OK, ref.reason
    assert got == ref.out.tobytes()
    if raw is not None:
        assert got == raw
    tab = plan.chunk_table()
    assert np.array_equal(_starts(tab), ref.start), (list(_starts(tab)), list(ref.start))
    ne = ref.start >= 0
    assert np.array_equal(tab["end"][ne].astype(np.int64), ref.end[ne])
    assert np.array_equal(tab["len"][ne].astype(np.int64), ref.len[ne])
    assert np.array_equal(tab["out_off"][ne].astype(np.int64), ref.off[ne])
    r = plan.result()
    assert r.out_len == len(got)
    assert r.n_placeholders == int(ref.placeholders.sum())
    return plan, ref


@pytest.fixture(scope="module")
def c1():
    raw = synth.fastq_like(4 << 20, 1)
    return raw, synth.gzip_member(raw, 6)


def test_c1_fastq_8_chunks(orc, c1):
    raw, comp = c1
    _say("fastq 4 MiB L6, 8 chunks")
    _check_against_oracle(orc, comp, 8, raw)


def test_c1_pass1_symbols_and_windows(orc, c1):
    """Pass 1 symbols of every chunk equal decompress(C_i, w_hat_i) at the same start,
    and pass 2 windows equal the true preceding 32 KiB."""
    raw, comp = c1
    _say("fastq 4 MiB L6, per-chunk symbols and windows")
    plan, ref = _check_against_oracle(orc, comp, 8, raw)
    N = ref.n_chunks
    nz = [i for i in range(N) if ref.start[i] >= 0]
    for k, i in enumerate(nz):
        stop = ref.start[nz[k + 1]] if k + 1 < len(nz) else (1 << 62)
        sr = orc.symbolic(comp, int(ref.start[i]), int(stop), first=(i == 0))
        assert sr.status == orc.OK
        L = int(ref.len[i])
        dev = plan.symbols(i, L).cpu().numpy().view(np.uint16)
        assert np.array_equal(dev, sr.sym[:L]), f"chunk {i}"
        if k > 0:
            w = plan.window(i).cpu().numpy()
            v = int(ref.valid[i])
            assert np.array_equal(w[32768 - v:], ref.windows[i][32768 - v:]), f"window {i}"


@pytest.mark.parametrize("n", [1, 2, 3, 64, 500])
def test_chunk_count_invariance(orc, c1, n):
    raw, comp = c1
    _say("fastq 4 MiB L6 chunks", n)
    got, plan = _run(comp, n)
    assert got == raw
    if n <= 64:
        ref = orc.pugz(comp, n)
        assert np.array_equal(_starts(plan.chunk_table()), ref.start)


@pytest.mark.parametrize("kind,level", [("words", 6), ("fastq", 1), ("fastq", 9), ("words", 1), ("dna", 6)])
def test_other_inputs(orc, kind, level):
    gen = {"words": lambda: synth.word_stream(3 << 20, 61), "fastq": lambda: synth.fastq_like(3 << 20, 62),
           "dna": lambda: synth.random_dna(2 << 20, 63)}[kind]
    raw = gen()
    comp = synth.gzip_member(raw, level)
    _say(kind, "level", level)
    _check_against_oracle(orc, comp, 6, raw)


@pytest.mark.parametrize("level", [0, 1, 6])
def test_small_and_special(orc, level):
    for name, raw in [("empty", b""), ("one", b"x"), ("tiny", b"hello gzip\n" * 3),
                      ("20k", synth.fastq_like(20000, 5)),
                      ("binary", np.random.default_rng(3).integers(0, 256, 300000, dtype=np.uint8).tobytes())]:
        comp = synth.gzip_member(raw, level)
        for n in (1, 3):
            _say("special", name, "level", level, "chunks", n)
            got, plan = _run(comp, n)
            assert got == raw, (name, n)


def test_segmented_member(orc):
    raw = synth.fastq_like(3 << 20, 71)
    comp = synth.gzip_member(raw, 6, segment_bytes=512 << 10)
    _say("segmented member")
    _check_against_oracle(orc, comp, 12, raw)


def test_handbuilt_streams(orc):
    from test_oracle import HAND, wrap_tokens

    for name, blocks in HAND.items():
        deflate, data = wrap_tokens(blocks)
        _say("handbuilt", name)
        got, _ = _run(gzip_wrap(deflate, data), 1)
        assert got == data, name


def test_long_codes_across_chunks(orc):
    """Literal/length and distance codes of up to 15 bits (decoded alone,
    past the lookup tables) in chunk starts, trial and confirmation blocks."""
    from test_oracle import _LONG_DIST, _LONG_LIT, _LONG_TOKENS, wrap_tokens

    kw = {"lit_lengths": _LONG_LIT, "dist_lengths": _LONG_DIST}
    deflate, data = wrap_tokens([("dynamic", _LONG_TOKENS * 4, kw)] * 30)
    _say("long codes across chunks")
    _check_against_oracle(orc, gzip_wrap(deflate, data), 8, data)


def test_negative_statuses(orc):
    gz = _gz()
    raw = synth.fastq_like(600 << 10, 81)
    comp = bytearray(synth.gzip_member(raw, 6))
    cases = {}
    bad = bytearray(comp)
    bad[-8] ^= 1
    cases["crc"] = (bytes(bad), gz.GZ_E_CRC)
    bad = bytearray(comp)
    bad[-4] ^= 1
    cases["isize"] = (bytes(bad), gz.GZ_E_SIZE)
    truncated = bytes(comp[: len(comp) // 2]) + bytes(comp[-8:])
    ref = orc.pugz(truncated, 4)
    assert ref.status == orc.E_DATA and ref.reason == "TRUNC"
    cases["truncated"] = (truncated, gz.GZ_E_DATA)
    cases["trailing_member"] = (bytes(comp) + synth.gzip_member(b"abc", 6), gz.GZ_E_UNSUPPORTED)
    for name, (data, want) in cases.items():
        _say("negative", name)
        plan = gz.Plan(_dev(data), 4)
        out = torch.empty(len(raw) + 1000, dtype=torch.uint8, device="cuda:0")
        plan.launch(out)
        r = plan.result()
        assert r.status == want, (name, r.status)
    with pytest.raises(gz.GzError):
        gz.Plan(_dev(b"\x1f\x8c" + bytes(30)), 1)


def test_corrupt_bits_match_oracle_status(orc):
    """Flipped bits: the device reports the oracle's status (a data error, a
    CRC-32 or a length mismatch), and otherwise produces the oracle's bytes."""
    gz = _gz()
    raw = synth.word_stream(300 << 10, 91)
    comp = synth.gzip_member(raw, 6)
    rng = np.random.default_rng(5)
    classes = set()
    for k in range(48):
        b = bytearray(comp)
        pos = int(rng.integers(20, len(b) - 20))
        b[pos] ^= 1 << int(rng.integers(0, 8))
        ref = orc.pugz(bytes(b), 3)
        _say("flip", k, pos, "oracle", ref.reason)
        plan = gz.Plan(_dev(bytes(b)), 3)
        out = torch.empty(2 * len(raw) + 4096, dtype=torch.uint8, device="cuda:0")
        plan.launch(out)
        r = plan.result()
        # the two status enumerations agree value for value
        assert r.status == ref.status, (k, pos, r.status, ref.reason)
        if ref.status == orc.OK:
            assert out[: r.out_len].cpu().numpy().tobytes() == ref.out.tobytes()
        classes.add(ref.status)
    assert {orc.E_DATA, orc.E_CRC} <= classes


def test_batch_equals_single(orc):
    gz = _gz()
    files = [synth.gzip_member(synth.fastq_like((1 + i) * (300 << 10), 200 + i), [1, 6, 9][i % 3]) for i in range(5)]
    files.append(synth.gzip_member(synth.word_stream(700 << 10, 299), 6))
    _say("batch of", len(files))
    outs = gz.decompress_batch([_dev(f) for f in files], n_chunks=4)
    for f, o in zip(files, outs):
        ref = orc.gunzip(f)
        assert o.cpu().numpy().tobytes() == ref.out.tobytes()


def test_repeat_determinism(orc, c1):
    raw, comp = c1
    _say("repeat determinism")
    gz = _gz()
    plan = gz.Plan(_dev(comp), 8)
    outs = []
    stats = []
    for _ in range(3):
        o = plan.run()
        torch.cuda.synchronize()
        outs.append(o.cpu().numpy().tobytes())
        stats.append(plan.result().as_dict())
    assert outs[0] == outs[1] == outs[2] == raw
    assert stats[0] == stats[1] == stats[2]


@pytest.mark.parametrize("win", [512, 1024, 2048, 4096, 8192, 16384, 32768])
def test_window_sizes(orc, c1, win):
    raw, comp = c1
    _say("LDS window", win)
    _check_against_oracle(orc, comp, 8, raw, window_syms=win)


@pytest.mark.parametrize("n", [64, 200])
def test_deferred_confirmation_decoded_alone(orc, c1, n):
    """Confirmation blocks owed past a chunk's stop, decoded on their own
    instead of taken from the next chunks: same starts and bytes."""
    raw, comp = c1
    _say("deferred confirmation decoded alone,", n, "chunks")
    _check_against_oracle(orc, comp, n, raw, confirm_decode=1)


@pytest.mark.parametrize("size", [0, 1, 3, 16383, 16384, 16385, 200_003, 1 << 20])
def test_device_crc32(size):
    """The CRC-32 computed on the device equals zlib's, for outputs within one
    16 KiB unit, on unit edges, and over many units; the second run writes to
    an output at an odd address (byte-wise loads)."""
    import zlib

    gz = _gz()
    raw = synth.fastq_like(size, 500 + size % 97)[:size]
    comp = synth.gzip_member(raw, 6)
    _say("device crc", size)
    for shift in (0, 1):
        plan = gz.Plan(_dev(comp), 3 if size > 100000 else 1)
        buf = torch.zeros(len(raw) + 64, dtype=torch.uint8, device="cuda:0")
        out = buf[shift:]
        plan.launch(out)
        r = plan.result()
        assert r.status == 0 and r.out_len == len(raw)
        assert r.crc32 == zlib.crc32(raw), (size, shift)
        assert out[: r.out_len].cpu().numpy().tobytes() == raw


def test_device_crc32_batch_and_mismatch(orc):
    """Every file of a batch gets its own CRC; a corrupted trailer CRC is
    reported as a CRC error, a corrupted ISIZE (CRC intact) as a size error."""
    import zlib

    gz = _gz()
    raws = [synth.word_stream(n, 600 + n % 11) for n in (5000, 70000, 300000)]
    comps = [synth.gzip_member(x, 6) for x in raws]
    outs = gz.decompress_batch([_dev(c) for c in comps], n_chunks=2)
    for x, o in zip(raws, outs):
        assert o.cpu().numpy().tobytes() == x
    bp = gz.BatchPlan([_dev(c) for c in comps], 2, outs=[torch.empty(len(x) + 8, dtype=torch.uint8, device="cuda:0")
                                                         for x in raws])
    bp.launch()
    for i, x in enumerate(raws):
        assert bp.result(i).crc32 == zlib.crc32(x)
    bad_crc = bytearray(comps[1])
    bad_crc[-8] ^= 0x40
    bad_len = bytearray(comps[1])
    bad_len[-4] ^= 0x01
    for b, want in ((bytes(bad_crc), gz.GZ_E_CRC), (bytes(bad_len), gz.GZ_E_SIZE)):
        ref = orc.pugz(b, 2)
        assert ref.status == want
        plan = gz.Plan(_dev(b), 2)
        plan.launch(torch.empty(2 * len(raws[1]) + 64, dtype=torch.uint8, device="cuda:0"))
        assert plan.result().status == want


# ---------------------------------------------------------------- false block starts (tests/decoy.py)

@pytest.mark.parametrize("final_last", [True, False], ids=["inner-final", "inner-nonfinal"])
def test_false_starts_repaired(orc, final_last):
    """Starts that pass Appendix A's checks inside a stored block are caught
    by the stitch check and the chunk is decoded again from where its
    predecessor stopped: device starts before and after the repair, ends,
    lengths, offsets, repair counts and bytes equal the oracle's at every
    chunk count from 2 to 15, with the default and the direct confirmation."""
    import decoy

    gz, raw, real_bits, decoy_bits = decoy.decoy_member(final_last=final_last)
    total = 0
    for n in range(2, 16):
        ref = orc.pugz(gz, n)
        assert ref.status == orc.OK and ref.out.tobytes() == raw
        for cd in (0, 1):
            _say("decoy final_last", final_last, "chunks", n, "confirm_decode", cd)
            got, plan = _run(gz, n, confirm_decode=cd)
            assert got == raw
            tab = plan.chunk_table()
            found = np.array([-1 if int(s) == _gz().NONE else int(s) for s in tab["cand"]], dtype=np.int64)
            assert np.array_equal(found, ref.cand), (n, list(found), list(ref.cand))
            assert np.array_equal(_starts(tab), ref.start), (n, list(_starts(tab)), list(ref.start))
            ne = ref.start >= 0
            assert np.array_equal(tab["end"][ne].astype(np.int64), ref.end[ne])
            assert np.array_equal(tab["len"][ne].astype(np.int64), ref.len[ne])
            assert np.array_equal(tab["out_off"][ne].astype(np.int64), ref.off[ne])
            r = plan.result()
            assert r.n_repairs == ref.n_repairs >= 1
            assert r.n_placeholders == int(ref.placeholders.sum())
            total += r.n_repairs
    assert total >= 50


def test_too_far_across_chunks(orc):
    """A match reaching before the data start inside chunk 0 (empty context)
    or a later chunk (found by the translation): GZ_E_DATA, as the oracle."""
    import decoy

    gz, bad_bit, bits = decoy.too_far_member()
    for n in range(1, 9):
        _say("too-far member, chunks", n)
        ref = orc.pugz(gz, n)
        assert ref.status == orc.E_DATA
        plan = _gz().Plan(_dev(gz), n)
        with pytest.raises(_gz().GzError) as ei:
            plan.run()
        assert ei.value.code == -4


@pytest.mark.parametrize("case", ["trial-fail-3", "trial-fail-10", "dense"])
def test_room_of_empty_chunks(orc, case):
    """Candidates rejected after the symbol regions were sized (tests/decoy.py):
    the chunk before decodes on through the empty chunk's range, within its
    region and the empty chunks' regions, stopping early in pass 1 when even
    its first blocks do not fit.  Every chunk count where the oracle succeeds
    gives the oracle's starts, ends, lengths and bytes without a capacity
    error (a plain launch, no re-plan)."""
    import decoy

    if case == "trial-fail-3":
        gz, raw, _ = decoy.trial_fail_member(real_before=3)
    elif case == "trial-fail-10":
        gz, raw, _ = decoy.trial_fail_member(real_before=10, stored_bytes=65000)
    else:
        gz, raw, _, _ = decoy.dense_block_member(dense_bytes=40000, mutate=0.02)
    cuts = 0
    for n in range(2, 40):
        ref = orc.pugz(gz, n)
        assert ref.status == orc.OK
        _say(case, "chunks", n)
        plan = _gz().Plan(_dev(gz), n)
        out = torch.empty(len(raw) + 64, dtype=torch.uint8, device="cuda:0")
        plan.launch(out)
        r = plan.result()
        if case == "dense" and r.status == _gz().GZ_E_CAPACITY:
            # the dense block can outgrow even the empty chunks' room: the
            # plan is made again with a larger symbol factor
            got = plan.run().cpu().numpy().tobytes()
            assert got == raw
            r = plan.result()
            out = None
        assert r.status == 0, (n, r.status)
        if out is not None:
            assert out[: r.out_len].cpu().numpy().tobytes() == raw
        tab = plan.chunk_table()
        assert np.array_equal(_starts(tab), ref.start), n
        ne = ref.start >= 0
        assert np.array_equal(tab["end"][ne].astype(np.int64), ref.end[ne])
        assert np.array_equal(tab["len"][ne].astype(np.int64), ref.len[ne])
        # pass 1 cut short (64), or continued into empty chunks' room (4)
        cuts += int(((tab["flags"] & (64 if case != "trial-fail-10" else 4)) != 0).sum())
    assert cuts >= 1


@pytest.mark.parametrize("level", [1, 6, 9])
def test_binary_mode(orc, level):
    """Binary inputs (Section VIII), 8 MiB with stored stretches: with the
    binary option, 24 chunks have the oracle's binary-mode starts, ends,
    lengths and output offsets and the source's bytes; with the default
    chunking every accepted start lies on gunzip's block map; in text mode no
    chunk after the first finds a start and the bytes are still the source."""
    gz = _gz()
    raw = synth.binary_records(8 << 20, 30 + level)
    comp = synth.gzip_member(raw, level)
    _say("binary 8 MiB level", level)
    ref = orc.pugz(comp, 24, binary=True)
    assert ref.status == orc.OK and ref.out.tobytes() == raw
    got, plan = _run(comp, 24, binary=1)
    assert got == raw
    tab = plan.chunk_table()
    assert np.array_equal(_starts(tab), ref.start)
    ne = ref.start >= 0
    for k, v in (("end", ref.end), ("len", ref.len), ("out_off", ref.off)):
        assert np.array_equal(tab[k][ne].astype(np.int64), v[ne]), k
    g = orc.gunzip(comp)
    blocks = set(g.block_bit.tolist())
    got, plan = _run(comp, 0, binary=1)
    assert got == raw
    s = _starts(plan.chunk_table())
    assert set(s[s >= 0].tolist()) <= blocks and (s >= 0).sum() > len(blocks) // 2
    got, plan = _run(comp, 24)
    assert got == raw and (_starts(plan.chunk_table())[1:] < 0).all()


@pytest.mark.parametrize("case", ["level0-text", "binary-stored"])
def test_stored_starts(orc, case):
    """Stored blocks as chunk starts (opts.start_types = GZ_START_STORED): at
    24 chunks the starts, ends, lengths and offsets equal the oracle's method
    with stored starts, with no repair; with the default chunking every start
    is a block of gunzip's map and the bytes are the source's."""
    gz = _gz()
    if case == "level0-text":
        raw = synth.fastq_like(8 << 20, 75)
        comp, binary = synth.gzip_member(raw, 0), 0
    else:
        raw = synth.binary_records(8 << 20, 76, noise_every=2, noise_bytes=256 << 10)
        comp, binary = synth.gzip_member(raw, 6), 1
    _say("stored starts", case)
    ref = orc.pugz(comp, 24, binary=bool(binary), types=orc.START_DYNAMIC | orc.START_STORED)
    assert ref.status == orc.OK and ref.out.tobytes() == raw and ref.n_repairs == 0
    got, plan = _run(comp, 24, start_types=gz.GZ_START_STORED, binary=binary)
    assert got == raw and plan.result().n_repairs == 0
    tab = plan.chunk_table()
    assert np.array_equal(_starts(tab), ref.start)
    ne = ref.start >= 0
    for k, v in (("end", ref.end), ("len", ref.len), ("out_off", ref.off)):
        assert np.array_equal(tab[k][ne].astype(np.int64), v[ne]), k
    g = orc.gunzip(comp)
    got, plan = _run(comp, 0, start_types=gz.GZ_START_STORED, binary=binary)
    assert got == raw
    s = _starts(plan.chunk_table())
    assert set(s[s >= 0].tolist()) <= set(g.block_bit.tolist())
    with pytest.raises(gz.GzError):
        gz.Plan(_dev(comp), 4, start_types=4)
