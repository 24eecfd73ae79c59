"""The device path's HIP source executed on the CPU (tests/emu), checked against the oracle.

The executor runs every GPU thread of every kernel as a fiber with lockstep
wave intrinsics, so the kernels' logic (block-start search, symbolic inflate,
stitching, window propagation, translation) is exercised here without a GPU.
The executor also reports divergence bugs (lanes of one wave at different
intrinsics) and deadlocks by aborting the run.
"""
import zlib

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
    assert r.crc32 == ref.crc_trailer == zlib.crc32(raw)
    return r, tab


def test_emu_handbuilt(orc):
    from test_oracle import HAND, wrap_tokens

    for name, blocks in HAND.items():
        deflate, data = wrap_tokens(blocks)
        st, out, r, tab = E.run(gzip_wrap(deflate, data), 1, out_cap=len(data) + 16)
        assert st == 0 and out == data, name


def test_emu_long_codes_across_chunks(orc):
    """Blocks whose literal/length and distance codes reach 15 bits (longer
    than the lookup tables: decoded alone) as chunk starts found by the scan,
    trial and confirmation blocks included: same starts, ends and bytes as
    the oracle."""
    from test_oracle import _LONG_DIST, _LONG_LIT, _LONG_TOKENS, wrap_tokens

    kw = {"lit_lengths": _LONG_LIT, "dist_lengths": _LONG_DIST}
    deflate, data = wrap_tokens([("dynamic", _LONG_TOKENS * 4, kw)] * 30)
    r, tab = _check(orc, gzip_wrap(deflate, data), 8, data)
    assert (tab["start"] != NONE).sum() == 8


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
    raw = synth.fastq_like(48 << 10, 305)
    comp = synth.gzip_member(raw, 6)
    for win in (512, 1024, 2048, 4096, 8192, 16384, 32768):
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


def test_emu_serving_loop_budget_and_order():
    """The serving loop on the CPU executor: jobs queue while the workspace
    arena is full, are admitted FIFO as batches finish, and every output equals
    its source text; the arena never holds more than its budget."""
    import ctypes as C

    L = E.server_lib()
    raws = [synth.fastq_like(20 << 10, 310 + k) if k % 2 == 0 else synth.word_stream(24 << 10, 310 + k)
            for k in range(6)]
    comps = [E.padded(synth.gzip_member(r, 6)) for r in raws]
    outs = [np.zeros(len(r) + 64, dtype=np.uint8) for r in raws]
    # budget: room for about two of these jobs' workspaces at a time
    o = E.ServerOpts()
    o.opts.chunk_bytes = 4096
    probe = C.c_void_p()
    L.gz_plan(C.byref(probe), C.c_void_p(comps[0].ctypes.data), len(synth.gzip_member(raws[0], 6)), 0,
              C.byref(o.opts))
    info = E.Info()
    L.gz_plan_info(probe, C.byref(info))
    L.gz_plan_destroy(probe)
    # the arena is the caller's (the library allocates no device memory)
    arena_bytes = int(info.ws_bytes * 2.6)
    raw_arena = np.zeros(arena_bytes + 512, dtype=np.uint8)
    arena = raw_arena[(-raw_arena.ctypes.data) % 256:][:arena_bytes]
    h = C.c_void_p()
    assert L.gz_server_create(C.byref(h), C.byref(o)) == -1  # GZ_E_ARG: no arena
    o.arena = C.c_void_p(arena.ctypes.data)
    o.arena_bytes = arena_bytes
    o.budget_bytes = 0  # the arena's size
    o.max_inflight = 2
    o.max_batch = 2
    assert L.gz_server_create(C.byref(h), C.byref(o)) == 0
    for k, (r, c) in enumerate(zip(raws, comps)):
        n = len(synth.gzip_member(r, 6))
        assert L.gz_server_submit(h, C.c_void_p(c.ctypes.data), n, C.c_void_p(outs[k].ctypes.data),
                                  outs[k].size, 100 + k) == 0
    st = E.ServerInfo()
    L.gz_server_stats(h, C.byref(st))
    assert st.queued == 6
    buf = (E.Done * 16)()
    done = []
    for _ in range(50):
        n = L.gz_server_poll(h, buf, 16)
        assert n >= 0
        done += [(buf[i].tag, buf[i].status, buf[i].out_len, buf[i].t_start) for i in range(n)]
        if len(done) == 6:
            break
    L.gz_server_stats(h, C.byref(st))
    L.gz_server_destroy(h)
    assert sorted(t for t, *_ in done) == list(range(100, 106))
    for tag, status, out_len, _ in done:
        k = tag - 100
        assert status == 0 and out_len == len(raws[k])
        assert outs[k][:out_len].tobytes() == raws[k]
    # admitted in submission order, never more workspace than the budget
    starts = [t for _, _, _, t in sorted(done)]
    assert starts == sorted(starts)
    assert st.arena_peak <= arena_bytes and st.batches >= 3
    # the budget counts inputs, outputs and workspaces of the jobs in flight
    assert 0 < st.resident_peak <= st.budget_bytes == arena_bytes


@pytest.mark.parametrize("decode", [0, 1])
def test_emu_deferred_confirmation_paths(orc, decode):
    """Chunks much smaller than a block owe most of their confirmation blocks
    past their stop; they are settled from the next chunks' checked blocks, or
    (decode=1) by decoding them on their own.  Starts and bytes equal the
    oracle's either way, also with a bit flipped in the middle of the stream."""
    raw = synth.word_stream(90 << 10, 308)
    comp = synth.gzip_member(raw, 6)
    for flip in (None, len(comp) // 2, len(comp) // 3):
        c = bytearray(comp)
        if flip is not None:
            c[flip] ^= 0x10
        c = bytes(c)
        ref = orc.pugz(c, 24)
        st, out, r, tab = E.run(c, 24, out_cap=len(raw) + 64, confirm_decode=decode)
        if ref.status == orc.OK or ref.reason in ("CRC", "ISIZE"):
            # the device checks the CRC-32, then the length, as the oracle does
            assert st == ref.status, (flip, st, ref.reason)
            if st == 0:
                assert out == ref.out.tobytes()
            assert np.array_equal(_starts(tab), ref.start)
        else:
            assert st != 0, (flip, ref.reason)


def _stream_expect(g, start_bit, seg):
    """From the oracle's block map: the block where a segment starting at
    start_bit stops (the first block at or past start_bit + 8 * seg), as
    (bit, output offset), or None for the end of the member."""
    stop = start_bit + 8 * seg
    later = np.nonzero(g.block_bit >= stop)[0]
    if len(later) == 0:
        return None
    i = int(later[0])
    return int(g.block_bit[i]), int(g.block_out_off[i])


@pytest.mark.parametrize("seg", [9000, 23456])
def test_emu_stream_segments(orc, seg):
    raw = synth.fastq_like(200 << 10, 311)
    comp = synth.gzip_member(raw, 6, segment_bytes=20 << 10)
    g = orc.gunzip(comp)
    assert g.status == orc.OK
    segs = E.stream_run(comp, seg, chunk_bytes=4096)
    assert len(segs) >= 2
    got = b""
    bit = 8 * g.payload_start
    for i, (d, data, cp) in enumerate(segs):
        assert d["status"] == 0, d
        assert d["start_bit"] == bit
        got += data
        exp = _stream_expect(g, bit, seg)
        if exp is None:
            assert d["done"] == 1 and i == len(segs) - 1
            assert d["end_bit"] == g.end_bit
        else:
            assert d["done"] == 0
            assert (d["end_bit"], d["out_total"]) == exp
        assert d["out_total"] == len(got)
        assert d["crc32"] == zlib.crc32(raw[: len(got)])
        # the checkpoint: position, running CRC, and the window before it
        assert cp.bit == d["end_bit"] and cp.out_total == len(got) and cp.crc32 == d["crc32"]
        v = min(len(got), 32768)
        assert cp.valid == v
        w = bytes(cp.window)
        assert w[32768 - v:] == raw[len(got) - v: len(got)] and w[: 32768 - v] == bytes(32768 - v)
        bit = d["end_bit"]
    assert got == raw


def test_emu_stream_resume_and_checks(orc):
    raw = synth.word_stream(240 << 10, 312)
    comp = synth.gzip_member(raw, 6)
    full = E.stream_run(comp, 6000, chunk_bytes=2048)
    assert len(full) >= 3
    assert all(d["status"] == 0 for d, _, _ in full) and b"".join(x for _, x, _ in full) == raw
    # resume from the checkpoint after the second segment in a new stream
    cp = full[1][2]
    assert not cp.done
    rest = E.stream_run(comp, 6000, resume=cp, chunk_bytes=2048)
    assert b"".join(x for _, x, _ in rest) == b"".join(x for _, x, _ in full[2:])
    assert rest[-1][0]["crc32"] == zlib.crc32(raw) and rest[-1][0]["done"] == 1
    # one segment covering the whole member equals the plain path
    one = E.stream_run(comp, 1 << 30, chunk_bytes=4096)
    assert len(one) == 1 and one[0][1] == raw and one[0][0]["done"] == 1
    # a wrong trailer CRC fails only the last segment, as the oracle fails the member
    bad = bytearray(comp)
    bad[-8] ^= 1
    assert orc.gunzip(bytes(bad)).status != orc.OK
    segs = E.stream_run(bytes(bad), 6000, chunk_bytes=2048)
    assert [d["status"] for d, _, _ in segs[:-1]] == [0] * (len(segs) - 1)
    assert segs[-1][0]["status"] == -6


def test_emu_block_probes(orc):
    # flush points every 20 KiB give many short blocks
    raw = synth.fastq_like(400 << 10, 321)
    comp = synth.gzip_member(raw, 6, segment_bytes=20 << 10)
    g = orc.gunzip(comp)
    assert g.block_bit.size >= 20
    P = 8 * g.payload_start
    end = 8 * (len(comp) - 8)
    # at a block start, just after one, mid-stream, and too close to the end
    bits = [P, int(g.block_bit[1]), int(g.block_bit[1]) + 1, P + 8 * 30000 + 5, end - 8 * 200]
    rng = 64 << 10
    starts, rej = E.probe_run(comp, bits, rng, chunk_bytes=8192)
    for b, s in zip(bits, starts):
        ref = orc.find_start(comp, b, min(end, b + 8 * rng))
        assert int(s) == (ref if ref >= 0 else NONE), (b, int(s), ref)
    dyn = g.block_bit[g.block_type == 2]
    assert int(starts[1]) == int(dyn[dyn >= bits[1]][0])
    assert int(starts[2]) == int(dyn[dyn > bits[1]][0]) and int(starts[-1]) == NONE
    # a bit outside the payload is an argument error
    st, _ = E.probe_run(comp, [end + 8], rng)
    assert st == -1


@pytest.mark.parametrize("level", [1, 6])
def test_emu_random_access_undetermined(orc, level):
    raw = synth.random_dna(300000, 322 + level)
    comp = synth.gzip_member(raw, level)
    g = orc.gunzip(comp)
    b = int(g.block_bit[1])  # from block 2, as Section IV-C
    segs, data, counts = E.stream_at(comp, b, 0, 9000, 3602, chunk_bytes=4096)
    assert all(d["status"] == 0 for d in segs) and segs[-1]["done"] == 1
    sr = orc.symbolic(comp, b, 1 << 62, first=False)
    assert sr.status == orc.OK
    sym = sr.sym
    und = sym >= 0x8000
    exp = np.where(und, 0, sym).astype(np.uint8)
    assert data == exp.tobytes()
    # determined bytes are the true bytes at the block's output offset
    o = int(g.block_out_off[1])
    assert np.array_equal(exp[~und], np.frombuffer(raw, np.uint8)[o:][~und])
    n_win = (und.size + 3601) // 3602
    ref_counts = np.add.reduceat(und.astype(np.int64), np.arange(0, und.size, 3602)) if und.size else []
    assert n_win == counts.size and np.array_equal(counts, ref_counts)


def _stage1_survivors(comp: bytes, limit_bits: int):
    """Bits passing the cheap block-start checks (header pattern, HLIT and
    HDIST ranges, complete code-length code), computed with numpy."""
    bits = np.unpackbits(np.frombuffer(comp, np.uint8), bitorder="little").astype(np.int64)
    n = min(bits.size - 17 - 57, limit_bits)
    b = np.arange(n)
    b = b[(bits[b] == 0) & (bits[b + 1] == 0) & (bits[b + 2] == 1)]

    def field(off, width):
        v = np.zeros(b.size, np.int64)
        for k in range(width):
            v |= bits[b + off + k] << k
        return v

    ok = (field(3, 5) <= 29) & (field(8, 5) <= 29)
    b = b[ok]
    hclen = field(13, 4) + 4
    left = np.full(b.size, 128, np.int64)
    for i in range(19):
        L = field(17 + 3 * i, 3)
        left -= np.where((i < hclen) & (L > 0), 128 >> L, 0)
    return b[left == 0]


@pytest.mark.parametrize("kind", ["fastq6", "words1", "dna9", "binary6"])
def test_emu_scan_table_check_equals_decoder(orc, kind):
    """The scan's table checks (whole wave, and one candidate per lane) accept
    exactly the candidates the decoder's table reader accepts, and all agree
    with the oracle's static block-start check (Appendix A)."""
    import ctypes as C

    raw = {"fastq6": lambda: synth.fastq_like(3 << 20, 331), "words1": lambda: synth.word_stream(3 << 20, 332),
           "dna9": lambda: synth.random_dna(3 << 20, 333),
           "binary6": lambda: np.random.default_rng(334).integers(0, 256, 2 << 20, dtype=np.uint8).tobytes()}[kind]()
    level = int(kind[-1])
    comp = synth.gzip_member(raw, level)
    # the stage-1 survivors of the first MiB; the true (non-final, dynamic)
    # block starts there are among them
    cand = _stage1_survivors(comp, 8 * min(len(comp), 1 << 20)).astype(np.uint64)
    g = orc.gunzip(comp)
    true_starts = set(int(x) for x, t, f in zip(g.block_bit, g.block_type, g.block_final)
                      if t == 2 and not f and x < 8 * (1 << 20))
    assert true_starts <= set(int(x) for x in cand) and cand.size > 50
    # the true starts and a seeded sample of the other survivors
    others = np.array(sorted(set(int(x) for x in cand) - true_starts), np.uint64)
    pick = np.random.default_rng(335).choice(others.size, min(others.size, 600), replace=False)
    cand = np.array(sorted(true_starts | set(int(x) for x in others[pick])), np.uint64)
    L = E.lib()
    L.emu_stage2_diff.argtypes = [C.c_void_p, C.c_uint64, C.c_void_p, C.c_int, C.c_void_p, C.c_void_p, C.c_void_p]
    store = E.padded(comp)
    r_read = np.zeros(cand.size, np.int32)
    r_check = np.zeros(cand.size, np.int32)
    r_lane = np.zeros(cand.size, np.int32)
    L.emu_set_sync_limit(0)
    L.emu_stage2_diff(store.ctypes.data, len(comp), cand.ctypes.data, cand.size, r_read.ctypes.data,
                      r_check.ctypes.data, r_lane.ctypes.data)
    assert np.array_equal(r_read, r_check), np.nonzero(r_read != r_check)[0][:10]
    assert np.array_equal(r_read, r_lane), np.nonzero(r_read != r_lane)[0][:10]
    ref = np.array([orc.block_static(comp, int(x))[0] for x in cand], np.int32)
    assert np.array_equal(r_check, ref)
    assert all(r_check[np.searchsorted(cand, t)] for t in true_starts)


def test_emu_window_propagation_many_segments(orc):
    """More than 4 * 64 accepted chunks: the windows of the propagation
    segments come from prefix compositions of their maps (several rounds)."""
    raw = synth.fastq_like(640 << 10, 341)
    comp = synth.gzip_member(raw, 6, segment_bytes=2048)
    g = orc.gunzip(comp)
    assert (g.block_type == 2).sum() > 280
    r, tab = _check(orc, comp, 300, raw)
    assert (tab["start"] != NONE).sum() > 4 * 64


def _members():

    parts = [synth.fastq_like(120 << 10, 351), synth.word_stream(60 << 10, 352), b"", synth.fastq_like(40 << 10, 353),
             synth.word_stream(30 << 10, 354)]
    comps = [synth.gzip_member(parts[0], 6), synth.gzip_member(parts[1], 1), synth.gzip_member(parts[2], 6),
             synth.bgzf_member(parts[3], 9), synth.bgzf_member(parts[4], 6)]
    return parts, comps


def test_emu_stream_multiple_members(orc):
    """Concatenated members (one empty, two BGZF-style): the stream's output
    is the oracle's gunzip of the whole input; each member ends with its own
    CRC-32; bytes after the last member that are not a member fail with the
    oracle's status (header)."""
    parts, comps = _members()
    comp = b"".join(comps)
    g = orc.gunzip(comp)
    assert g.status == orc.OK and g.n_members == len(parts)
    segs = E.stream_run(comp, 15000, chunk_bytes=4096)
    assert all(d["status"] == 0 for d, _, _ in segs) and segs[-1][0]["done"] == 1
    got = b"".join(x for _, x, _ in segs)
    assert got == g.out.tobytes() == b"".join(parts)
    ends = [d for d, _, _ in segs if d["member_done"]]
    assert [d["member"] for d in ends] == list(range(len(parts)))
    assert [d["crc32"] for d in ends] == [zlib.crc32(p) for p in parts]
    # a checkpoint inside a member resumes to the same bytes
    k = next(i for i, (d, _, _) in enumerate(segs) if not d["member_done"])
    rest = E.stream_run(comp, 15000, resume=segs[k][2], chunk_bytes=4096)
    assert b"".join(x for _, x, _ in rest) == b"".join(x for _, x, _ in segs[k + 1:])
    # trailing bytes that are not a gzip member
    bad = comp + b"\x00garbage"
    gb = orc.gunzip(bad)
    assert gb.status == orc.E_HEADER
    sb = E.stream_run(bad, 15000, chunk_bytes=4096)
    head = b"".join(x for _, x, _ in sb[:-1])
    assert sb[-1][0]["status"] == -2 and sb[-1][0]["member_done"] == 1
    assert head + g.out.tobytes()[len(head):] == g.out.tobytes()
    assert len(head) + sb[-1][0]["out_len"] == g.out.size
    # a wrong CRC in the second member
    crc_at = len(comps[0]) + len(comps[1]) - 8
    bc = bytearray(comp)
    bc[crc_at] ^= 1
    assert orc.gunzip(bytes(bc)).reason == "CRC"
    sc = E.stream_run(bytes(bc), 15000, chunk_bytes=4096)
    assert sc[-1][0]["status"] == -6 and sc[-1][0]["member"] == 1


def test_emu_decompress_members(orc):
    """gz_decompress_members: concatenated members (one empty, two
    BGZF-style) decoded member after member by the whole path give the
    oracle's gunzip of the whole input; a wrong CRC in the second member
    gives the oracle's CRC status; a full output gives CAPACITY; a
    non-member tail gives the oracle's header status."""
    parts, comps = _members()
    comp = b"".join(comps)
    g = orc.gunzip(comp)
    st, out, n = E.members_run(comp, g.out.size + 16, chunk_bytes=4096)
    assert st == 0 and out == g.out.tobytes() and n == len(parts)
    # the failure cases on three small members
    parts = [synth.fastq_like(16 << 10, 355), synth.word_stream(12 << 10, 356), synth.fastq_like(8 << 10, 357)]
    comps = [synth.gzip_member(parts[0], 6), synth.gzip_member(parts[1], 1), synth.bgzf_member(parts[2], 9)]
    comp = b"".join(comps)
    g = orc.gunzip(comp)
    crc_at = len(comps[0]) + len(comps[1]) - 8
    bc = bytearray(comp)
    bc[crc_at] ^= 1
    st, out, n = E.members_run(bytes(bc), g.out.size + 16, chunk_bytes=4096)
    assert st == -6 and n == 1 and out == b"".join(parts[:1])
    st, out, n = E.members_run(comp, len(parts[0]) + 10, chunk_bytes=4096)
    assert st == -5 and out == parts[0]
    bad = comp + b"\x00garbage"
    assert orc.gunzip(bad).status == orc.E_HEADER
    st, out, n = E.members_run(bad, g.out.size + 16, chunk_bytes=4096)
    assert st == -2 and out == g.out.tobytes() and n == len(parts)


def test_emu_bgzf_batch(orc):
    """A BGZF-style file (64 KiB members and the empty end member) decoded
    as one batch of members equals the oracle's gunzip; a member without the
    size subfield is refused; a bad CRC fails that member only."""

    raw = synth.fastq_like(300 << 10, 361)
    parts = [raw[i:i + (64 << 10)] for i in range(0, len(raw), 64 << 10)] + [b""]
    comps = [synth.bgzf_member(p, 6) for p in parts]
    comp = b"".join(comps)
    g = orc.gunzip(comp)
    assert g.status == orc.OK and g.n_members == len(parts)
    st, out, sts = E.bgzf_run(comp, chunk_bytes=8192)
    assert st == 0 and out == g.out.tobytes() == raw and sts == [0] * len(parts)
    st, _, _ = E.bgzf_run(comp + synth.gzip_member(b"abc", 6))
    assert st == -2
    bad = bytearray(comp)
    bad[len(comps[0]) + len(comps[1]) - 8] ^= 1
    st, out, sts = E.bgzf_run(bytes(bad), chunk_bytes=8192)
    assert st == 0 and sts[1] == -6 and sts[0] == 0 and all(x == 0 for x in sts[2:])


@pytest.mark.parametrize("final_last,n", [(True, 2), (True, 4), (True, 9), (False, 4), (False, 12)])
def test_emu_false_starts_repaired(orc, final_last, n):
    """Chunk starts that pass Appendix A's checks inside a stored block
    (tests/decoy.py) are replaced by where the previous chunk stopped, as the
    oracle does: same starts before and after the repair, ends, lengths,
    offsets, repair count and bytes."""
    import decoy

    gz, raw, real_bits, decoy_bits = decoy.decoy_member(final_last=final_last)
    ref = orc.pugz(gz, n)
    assert ref.status == orc.OK and ref.n_repairs >= 1
    st, out, r, tab = E.run(gz, n, out_cap=len(raw) + 64, sync_limit=3_000_000_000)
    assert st == 0 and out == raw == ref.out.tobytes()
    found = np.array([-1 if int(s) == NONE else int(s) for s in tab["cand"]], dtype=np.int64)
    assert np.array_equal(found, ref.cand), (list(found), list(ref.cand))
    assert np.array_equal(_starts(tab), ref.start)
    ne = ref.start >= 0
    for k in ("end", "len", "out_off"):
        assert np.array_equal(tab[k][ne].astype(np.int64), getattr(ref, "off" if k == "out_off" else k)[ne]), k
    assert r.n_repairs == ref.n_repairs
    assert r.n_placeholders == int(ref.placeholders.sum())
    # per-chunk statistics: placeholders of the accepted decodes, and every
    # rejected candidate counted at the stage that rejected it
    assert np.array_equal(tab["n_placeholders"][ne].astype(np.int64), ref.placeholders[ne])
    assert int(tab["trial_rej"].sum()) + int(tab["confirm_rej"].sum()) == r.n_retries
    assert (tab["stage2"][1:][ne[1:]] >= 1).all() and (tab["stage1"] >= tab["stage2"]).all()
    repaired = (tab["flags"] & 8) != 0
    assert np.array_equal(np.nonzero(repaired)[0], np.nonzero((ref.cand != ref.start) & ne)[0])
    assert set(found[repaired].tolist()) <= set(decoy_bits)


def test_emu_too_far_across_chunks(orc):
    """A match reaching before the data start: a data error whether the chunk
    holding it has an empty context (one chunk) or a placeholder context
    (found by the translation, as in the oracle)."""
    import decoy

    gz, bad_bit, bits = decoy.too_far_member()
    for n in (1, 3, 6):
        ref = orc.pugz(gz, n)
        assert ref.status == orc.E_DATA
        st, out, r, tab = E.run(gz, n, out_cap=64 << 10, sync_limit=3_000_000_000)
        assert st == -4, (n, st)


def _same_as_oracle(orc, gz, raw, n):
    ref = orc.pugz(gz, n)
    assert ref.status == orc.OK and ref.out.tobytes() == raw
    st, out, r, tab = E.run(gz, n, out_cap=len(raw) + 64, sync_limit=3_000_000_000)
    assert st == 0 and out == raw
    assert np.array_equal(_starts(tab), ref.start)
    ne = ref.start >= 0
    assert np.array_equal(tab["end"][ne].astype(np.int64), ref.end[ne])
    assert np.array_equal(tab["len"][ne].astype(np.int64), ref.len[ne])
    assert r.n_placeholders == int(ref.placeholders.sum())
    return tab


@pytest.mark.parametrize("case", ["first-cut", "extend-over-empty", "dense-cut-a", "dense-cut-b"])
def test_emu_room_of_empty_chunks(orc, case):
    """A candidate rejected after the symbol regions were sized leaves its
    chunk empty, and the chunk before it decodes through that chunk's range:
    it continues into the empty chunk's region (the stitch pass), and when
    even its own first blocks outgrow its region, pass 1 stops at the last
    block boundary that fits and the stitch pass continues from there.  Same
    starts, ends, lengths and bytes as the oracle, with no capacity error."""
    import decoy

    if case == "first-cut":
        gz, raw, _ = decoy.trial_fail_member(real_before=3)
        tab = _same_as_oracle(orc, gz, raw, 12)
        assert tab["flags"][0] & 64 and tab["trial_rej"][1] == 1  # chunk 0 cut, chunk 1's candidate rejected
    elif case == "extend-over-empty":
        gz, raw, _ = decoy.trial_fail_member(real_before=10, stored_bytes=65000)
        tab = _same_as_oracle(orc, gz, raw, 16)
        assert tab["flags"][1] & 4 and tab["len"][1] == 89000 and (tab["flags"][2] & 2)
    else:
        gz, raw, dbit, bits = decoy.dense_block_member(dense_bytes=40000, mutate=0.02)
        n = 8 if case == "dense-cut-a" else 12
        tab = _same_as_oracle(orc, gz, raw, n)
        k = int(np.nonzero(_starts(tab) == dbit)[0][0])
        assert k >= 1 and tab["flags"][k] & 64 and tab["flags"][k + 1] & 2


def test_emu_serving_budget_counts_footprints():
    """With an arena far larger than the budget, admission is bounded by the
    budget over the jobs' inputs, outputs and workspaces: one job at a time."""
    import ctypes as C

    L = E.server_lib()
    raws = [synth.fastq_like(12 << 10, 330 + k) for k in range(3)]
    gzs = [synth.gzip_member(r, 6) for r in raws]
    comps = [E.padded(g) for g in gzs]
    outs = [np.zeros(len(r) + 64, dtype=np.uint8) for r in raws]
    o = E.ServerOpts()
    o.opts.chunk_bytes = 4096
    probe = C.c_void_p()
    L.gz_plan(C.byref(probe), C.c_void_p(comps[0].ctypes.data), len(gzs[0]), 0, C.byref(o.opts))
    info = E.Info()
    L.gz_plan_info(probe, C.byref(info))
    L.gz_plan_destroy(probe)
    foot = len(gzs[0]) + outs[0].size + info.ws_bytes
    arena_bytes = 8 * info.ws_bytes
    raw_arena = np.zeros(arena_bytes + 512, dtype=np.uint8)
    arena = raw_arena[(-raw_arena.ctypes.data) % 256:][:arena_bytes]
    o.arena = C.c_void_p(arena.ctypes.data)
    o.arena_bytes = arena_bytes
    o.budget_bytes = int(foot * 1.5)
    o.max_inflight = 3
    o.max_batch = 3
    h = C.c_void_p()
    assert L.gz_server_create(C.byref(h), C.byref(o)) == 0
    for k in range(3):
        assert L.gz_server_submit(h, C.c_void_p(comps[k].ctypes.data), len(gzs[k]), C.c_void_p(outs[k].ctypes.data),
                                  outs[k].size, k) == 0
    buf = (E.Done * 8)()
    done = []
    for _ in range(50):
        n = L.gz_server_poll(h, buf, 8)
        assert n >= 0
        done += [(buf[i].tag, buf[i].status) for i in range(n)]
        if len(done) == 3:
            break
    st = E.ServerInfo()
    L.gz_server_stats(h, C.byref(st))
    L.gz_server_destroy(h)
    assert sorted(done) == [(0, 0), (1, 0), (2, 0)]
    assert all(outs[k][: len(raws[k])].tobytes() == raws[k] for k in range(3))
    assert st.batches == 3 and st.resident_peak <= o.budget_bytes and st.arena_peak < arena_bytes // 2
    # the second and third jobs each waited for the budget
    assert st.mem_waited == 2


def test_emu_static_workspace_entry_point():
    """gz_decompress_static (the entry point that allocates nothing) on the
    CPU executor: the same bytes and chunk starts as gz_decompress, twice in a
    row, the second input smaller."""
    import ctypes as C

    L = E.lib()
    L.gz_decompress_static.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]
    for k, raw in enumerate([synth.fastq_like(96 << 10, 340), synth.word_stream(40 << 10, 341)]):
        comp = synth.gzip_member(raw, 6)
        st, want, r, tab = E.run(comp, 3, out_cap=len(raw) + 64)
        assert st == 0 and want == raw
        store = E.padded(comp)
        h = C.c_void_p()
        assert L.gz_plan(C.byref(h), C.c_void_p(store.ctypes.data), len(comp), 3, C.byref(E.Opts())) == 0
        out = np.full(len(raw) + 64, 0xAB, dtype=np.uint8)
        assert L.gz_decompress_static(h, C.c_void_p(out.ctypes.data), out.size, None) == 0
        res = E.Result()
        assert L.gz_result_get(h, 0, C.byref(res)) == 0
        starts = np.zeros(3, dtype=np.uint64)
        assert L.gz_chunk_table(h, 0, C.c_void_p(starts.ctypes.data), None, None, None, None, None, None) == 0
        L.gz_plan_destroy(h)
        assert res.status == 0 and out[: res.out_len].tobytes() == raw
        assert (out[res.out_len:] == 0xAB).all()
        assert np.array_equal(starts, tab["start"]), k


def _cls_bytes(s):
    cb = {"D": ord("A"), "U": 0, "L": 10, "O": ord("x")}
    return np.array([cb[c] for c in s], np.uint8)


def test_emu_extract_dna_random_class_strings():
    """The device extractor (Appendix B) on random class strings spanning many
    tiles and groups of runs equals the oracle, as bytes with a marker and as
    16-bit symbols; also a chain of newline-shared runs across groups, an
    empty buffer, a buffer without runs, and the sequence cap."""
    from oracle import dna

    rng = np.random.default_rng(1)
    for n, alpha in ((5000, "DDDDULLO"), (40000, "DDDDULLO"), (30000, "DDUUL")):
        a = _cls_bytes("".join(rng.choice(list(alpha), n)))
        want = dna.extract(a, 0, 1)
        got, tot, _ = E.dna_run(a, 0, 1)
        assert got == want and tot == len(want)
        sym = np.where(a == 0, 0x8000 + rng.integers(0, 32768, n), a).astype(np.uint16)
        got, tot, _ = E.dna_run(sym, 0, 3)
        assert got == dna.extract(sym, min_len=3)
    a = _cls_bytes("L" + "DL" * 70000)
    got, tot, _ = E.dna_run(a, 0, 1)
    assert got == dna.extract(a, 0, 1) and tot == 35000
    assert E.dna_run(np.zeros(0, np.uint8), 0, 1)[:2] == ([], 0)
    assert E.dna_run(_cls_bytes("OLOLLO" * 100), 0, 1)[:2] == ([], 0)
    got, tot, _ = E.dna_run(a, 0, 1, max_seqs=10)
    assert tot == 35000 and got == dna.extract(a, 0, 1)[:10]


def test_emu_extract_dna_fastq_ranges():
    """FASTQ-like text with undetermined headers, qualities and bases: the
    sequences and the per-range (sequence-resolved) statistics equal the
    oracle's."""
    from oracle import dna

    raw = np.frombuffer(synth.fastq_like(300 << 10, 17), np.uint8)
    rng = np.random.default_rng(2)
    und = rng.random(raw.size) < np.where(np.arange(raw.size) < raw.size * 6 // 10, 0.2, 0.0)
    sym = np.where(und, 0x8000 + rng.integers(0, 32768, raw.size), raw).astype(np.uint16)
    bounds = np.linspace(0, raw.size, 9).astype(np.int64)
    want = dna.extract(sym, min_len=50)
    got, tot, st = E.dna_run(sym, 0, 50, bounds=bounds, threshold=20)
    assert got == want and tot == len(want)
    assert np.array_equal(st, dna.range_stats(want, bounds, 20))
    assert st[:, 2].any() and not st[:, 2].all()
    b8 = np.where(und, 0, raw).astype(np.uint8)
    got, _, st8 = E.dna_run(b8, 0, 50, bounds=bounds, threshold=20)
    assert got == want and np.array_equal(st8, st)


def test_emu_binary_mode(orc):
    """Binary inputs (Section VIII): with the binary option the chunk starts,
    ends, lengths and bytes equal the oracle's binary-mode method; without it
    no chunk after the first finds a start (non-ASCII literals), as in the
    oracle's text mode, and the output is still the source."""
    raw = synth.binary_records(300 << 10, 8, noise_every=1, noise_bytes=24 << 10)
    comp = synth.gzip_member(raw, 6)
    n = 5
    ref = orc.pugz(comp, n, binary=True)
    assert (ref.start >= 0).sum() >= 3
    assert ref.status == orc.OK and ref.out.tobytes() == raw
    st, out, r, tab = E.run(comp, n, out_cap=len(raw) + 64, sync_limit=3_000_000_000, binary=1)
    assert st == 0 and out == raw
    assert np.array_equal(_starts(tab), ref.start)
    ne = ref.start >= 0
    assert np.array_equal(tab["end"][ne].astype(np.int64), ref.end[ne])
    assert np.array_equal(tab["len"][ne].astype(np.int64), ref.len[ne])
    assert np.array_equal(tab["out_off"][ne].astype(np.int64), ref.off[ne])
    assert r.n_placeholders == int(ref.placeholders.sum())
    txt = orc.pugz(comp, n)
    st, out, r, tab = E.run(comp, n, out_cap=len(raw) + 64, sync_limit=3_000_000_000)
    assert st == 0 and out == raw
    assert np.array_equal(_starts(tab), txt.start) and (txt.start[1:] < 0).all()


def test_emu_stored_starts(orc):
    """Stored blocks as chunk starts (opts.start_types): on a level-0 member
    and on binary data with stored stretches (binary mode too), starts, ends,
    lengths and repair counts equal the oracle's, starts found in the zero run
    before a stored block's LEN/NLEN are taken as the previous chunk's end."""
    T = orc.START_DYNAMIC | orc.START_STORED
    cases = [(synth.fastq_like(400 << 10, 72), 0, 7, False)]
    rawb = synth.binary_records(300 << 10, 8, noise_every=1, noise_bytes=80 << 10)
    cases.append((rawb, 6, 6, True))
    for raw, level, n, binary in cases:
        comp = synth.gzip_member(raw, level)
        ref = orc.pugz(comp, n, binary=binary, types=T)
        assert ref.status == orc.OK and ref.out.tobytes() == raw and ref.n_equivalent >= 1
        st, out, r, tab = E.run(comp, n, out_cap=len(raw) + 64, sync_limit=3_000_000_000, start_types=2,
                                binary=int(binary))
        assert st == 0 and out == raw
        assert np.array_equal(_starts(tab), ref.start)
        ne = ref.start >= 0
        assert np.array_equal(tab["end"][ne].astype(np.int64), ref.end[ne])
        assert np.array_equal(tab["len"][ne].astype(np.int64), ref.len[ne])
        assert r.n_repairs == ref.n_repairs == 0
    # fixed blocks are not offered as starts
    st, out, r, tab = E.run(comp, 2, out_cap=len(rawb) + 64, start_types=4)
    assert st == -1
