"""Full-size cases through the C ABI (needs an MI355X).

The 1 GiB FASTQ-like member at level 6 (read lengths 100 and 150), decoded in
the launch configuration the benchmark times (library defaults: 40 KiB
chunks, 512-symbol LDS ring, about 12 000 chunks), is compared with the
oracle's sequential gunzip byte for byte.  Chunk starts and ends must be
block boundaries of the oracle's block map with the oracle's output offsets,
and a seeded sample of chunks must have exactly the oracle's pass-1 symbols
(decompress(C_i, w_hat_i), Section VI-C) and resolved windows, which the
oracle computes one chunk at a time.  The bounded-memory stream is checked on
the same member: every segment's bytes, where each segment stops (predicted
from the block map), the running CRC-32 and a checkpoint's window.
"""
import zlib

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def c2(orc):
    _say("generating fastq_1GiB_L6")
    raw, comp = synth.workload("fastq_1GiB_L6")
    _say("oracle gunzip of", len(comp), "compressed bytes")
    g = orc.gunzip(comp)
    assert g.status == orc.OK and g.n_members == 1
    assert g.out.size == len(raw)
    return raw, comp, g


def test_c2_full_size_against_oracle(orc, c2):
    import paper_1905_07224_amd as gz

    raw, comp, g = c2
    _say("fastq_1GiB_L6, default launch configuration")
    d_comp = torch.frombuffer(bytearray(comp), dtype=torch.uint8).to("cuda:0")
    plan = gz.Plan(d_comp, 0)
    assert plan.n_chunks > 5000
    out = torch.empty(len(raw), dtype=torch.uint8, device="cuda:0")
    plan.launch(out)
    r = plan.result()
    assert r.status == 0 and r.out_len == g.out.size
    assert np.array_equal(out.cpu().numpy(), g.out)
    assert r.crc32 == g.crc_computed == g.crc_trailer
    tab = plan.chunk_table()
    start = tab["start"].astype(np.uint64)
    ne = np.nonzero(start != np.uint64(gz.NONE))[0]
    # a chunk has a start exactly when its nominal range holds a true
    # (non-final, dynamic) block start, chunk 0 always
    N = plan.n_chunks
    h, P = plan.info.payload_start, plan.info.payload_end - plan.info.payload_start
    lo = np.array([8 * (h + (j * P) // N) for j in range(N + 1)], dtype=np.int64)
    dyn = np.sort(g.block_bit[(g.block_type == 2) & (g.block_final == 0)])
    has = np.searchsorted(dyn, lo[1:]) > np.searchsorted(dyn, lo[:-1])
    has[0] = True
    assert np.array_equal(ne, np.nonzero(has)[0])
    bits = g.block_bit
    pos = np.searchsorted(bits, start[ne].astype(np.int64))
    assert np.all(pos < bits.size) and np.array_equal(bits[pos], start[ne].astype(np.int64))
    assert np.array_equal(tab["out_off"][ne].astype(np.int64), g.block_out_off[pos])
    ends = tab["end"][ne].astype(np.int64)
    assert np.array_equal(ends[:-1], start[ne][1:].astype(np.int64))
    assert ends[-1] == g.end_bit
    # a seeded sample of chunks: symbols and windows, one chunk at a time
    rng = np.random.default_rng(7)
    sample = sorted(set([int(ne[0]), int(ne[-1])] + [int(x) for x in rng.choice(ne, 6, replace=False)]))
    for j in sample:
        k = int(np.nonzero(ne == j)[0][0])
        s, e = int(start[j]), int(ends[k])
        _say("chunk", j, "bits", s, e)
        sr = orc.symbolic(comp, s, e, first=(k == 0))
        assert sr.status == orc.OK and sr.end_bit == e
        L = int(tab["len"][j])
        assert sr.sym.size == L
        dev = plan.symbols(j, L).cpu().numpy().view(np.uint16)
        assert np.array_equal(dev, sr.sym), f"symbols of chunk {j}"
        if k > 0:
            off = int(tab["out_off"][j])
            v = min(off, 32768)
            w = plan.window(j).cpu().numpy()
            assert np.array_equal(w[32768 - v:], g.out[off - v:off]), f"window of chunk {j}"


def _stop_after(g, start_bit, seg):
    later = np.nonzero(g.block_bit >= start_bit + 8 * seg)[0]
    return None if later.size == 0 else (int(g.block_bit[later[0]]), int(g.block_out_off[later[0]]))


def test_c2_stream_full_size(orc, c2):
    import paper_1905_07224_amd as gz

    raw, comp, g = c2
    seg = 96 << 20
    _say("fastq_1GiB_L6 streamed in", seg, "byte segments")
    d_comp = torch.frombuffer(bytearray(comp), dtype=torch.uint8).to("cuda:0")
    s = gz.Stream(d_comp, seg)
    info = s.info()
    bit, tot, crc = 8 * g.payload_start, 0, 0
    n = 0
    for part in s:
        d = s.last
        _say("segment", n, d["start_bit"], d["end_bit"], d["out_len"])
        assert d["start_bit"] == bit
        a = part.cpu().numpy()
        assert np.array_equal(a, g.out[tot:tot + a.size]), f"segment {n}"
        tot += a.size
        crc = zlib.crc32(a, crc)
        assert d["out_total"] == tot and d["crc32"] == crc
        exp = _stop_after(g, bit, seg)
        if exp is None:
            assert d["done"] == 1 and d["end_bit"] == g.end_bit
        else:
            assert (d["end_bit"], d["out_total"]) == exp
        if n == 2:
            cp = s.checkpoint()
            assert cp.bit == d["end_bit"] and cp.valid == 32768
            assert bytes(cp.window) == g.out[tot - 32768:tot].tobytes()
        bit = d["end_bit"]
        n += 1
    assert tot == g.out.size and crc == g.crc_trailer and n >= 5
    # the workspace of one segment is a fraction of the whole-member plan's
    whole = gz.Plan(d_comp, 0)
    assert info["ws_bytes"] * 3 < whole.info.ws_bytes
    s.close()


def test_stream_small_members(orc):
    """Stream parity on small inputs: segment boundaries, CRC, checkpoints,
    resume, and the same statuses as the oracle for a bad trailer."""
    import paper_1905_07224_amd as gz

    raw = synth.fastq_like(6 << 20, 811)
    comp = synth.gzip_member(raw, 6)
    g = orc.gunzip(comp)
    d_comp = torch.frombuffer(bytearray(comp), dtype=torch.uint8).to("cuda:0")
    for seg in (40000, 300000, 1 << 30):
        _say("stream 6 MiB, segment", seg)
        s = gz.Stream(d_comp, seg, chunk_bytes=8192)
        got, bit, cps = [], 8 * g.payload_start, []
        for part in s:
            d = s.last
            got.append(part.cpu().numpy().tobytes())
            exp = _stop_after(g, bit, seg)
            assert d["done"] == (exp is None)
            if exp is not None:
                assert (d["end_bit"], d["out_total"]) == exp
            cps.append(s.checkpoint())
            bit = d["end_bit"]
        assert b"".join(got) == raw and s.last["crc32"] == zlib.crc32(raw)
        s.close()
        if len(cps) >= 3:
            # a new stream resumed from the second checkpoint gives the rest
            s2 = gz.Stream(d_comp, seg, chunk_bytes=8192)
            s2.resume(cps[1])
            rest = [p.cpu().numpy().tobytes() for p in s2]
            assert b"".join(rest) == b"".join(got[2:])
            s2.close()
    # the trailer is CRC-32 (bytes -8..-5) then ISIZE (-4..-1)
    for at, reason, code in ((-6, "CRC", gz.GZ_E_CRC), (-3, "ISIZE", gz.GZ_E_SIZE)):
        bad = bytearray(comp)
        bad[at] ^= 0x10
        assert orc.gunzip(bytes(bad)).reason == reason
        _say("stream with a bad", reason)
        s = gz.Stream(torch.frombuffer(bad, dtype=torch.uint8).to("cuda:0"), 300000, chunk_bytes=8192)
        n_ok = 0
        with pytest.raises(gz.GzError) as ei:
            for _ in s:
                n_ok += 1
        assert ei.value.code == code and n_ok >= 2
        s.close()


def test_stream_multiple_members(orc):
    """Concatenated members (an empty one, BGZF-style ones) streamed: the
    output is the oracle's gunzip of the whole input, each member ends with
    its own CRC-32, and a non-member tail fails with the oracle's status."""
    import paper_1905_07224_amd as gz

    parts = [synth.fastq_like(5 << 20, 821), synth.word_stream(3 << 20, 822), b"", synth.fastq_like(60 << 10, 823),
             synth.word_stream(50 << 10, 824), synth.fastq_like(2 << 20, 825)]
    comps = [synth.gzip_member(parts[0], 6), synth.gzip_member(parts[1], 1), synth.gzip_member(b"", 6),
             synth.bgzf_member(parts[3], 6), synth.bgzf_member(parts[4], 9), synth.gzip_member(parts[5], 9)]
    comp = b"".join(comps)
    g = orc.gunzip(comp)
    assert g.status == orc.OK and g.n_members == len(parts)
    for seg in (1 << 20, 1 << 30):
        _say("members streamed, segment", seg)
        s = gz.Stream(torch.frombuffer(bytearray(comp), dtype=torch.uint8).to("cuda:0"), seg)
        got, ends = [], []
        for part in s:
            got.append(part.cpu().numpy().tobytes())
            if s.last["member_done"]:
                ends.append((s.last["member"], s.last["crc32"]))
        s.close()
        assert b"".join(got) == g.out.tobytes()
        assert ends == [(i, zlib.crc32(p)) for i, p in enumerate(parts)]
    bad = bytearray(comp + b"\x1f\x8b\x08")
    assert orc.gunzip(bytes(bad)).status == orc.E_HEADER
    s = gz.Stream(torch.frombuffer(bad, dtype=torch.uint8).to("cuda:0"), 1 << 20)
    with pytest.raises(gz.GzError) as ei:
        for _ in s:
            pass
    assert ei.value.code == gz.GZ_E_HEADER
    s.close()


def test_decompress_members(orc):
    """gz_decompress_members on concatenated members (an empty one,
    BGZF-style ones, levels 1/6/9): the oracle's gunzip of the whole input,
    members counted; a wrong CRC in the second member gives the oracle's
    status with the first member's bytes; a non-member tail gives the
    oracle's header status after all members."""
    import paper_1905_07224_amd as gz

    parts = [synth.fastq_like(5 << 20, 821), synth.word_stream(3 << 20, 822), b"", synth.fastq_like(60 << 10, 823),
             synth.word_stream(50 << 10, 824), synth.fastq_like(2 << 20, 825)]
    comps = [synth.gzip_member(parts[0], 6), synth.gzip_member(parts[1], 1), synth.gzip_member(b"", 6),
             synth.bgzf_member(parts[3], 6), synth.bgzf_member(parts[4], 9), synth.gzip_member(parts[5], 9)]
    comp = b"".join(comps)
    g = orc.gunzip(comp)
    assert g.status == orc.OK and g.n_members == len(parts)
    _say("members through gz_decompress_members")
    out = torch.empty(g.out.size + 64, dtype=torch.uint8, device="cuda:0")
    n, m = gz.decompress_members(comp, out)
    assert n == g.out.size and m == len(parts)
    assert np.array_equal(out[:n].cpu().numpy(), g.out)
    bad = bytearray(comp)
    bad[len(comps[0]) + len(comps[1]) - 8] ^= 1
    assert orc.gunzip(bytes(bad)).reason == "CRC"
    with pytest.raises(gz.GzError) as ei:
        gz.decompress_members(bytes(bad), out)
    assert ei.value.code == gz.GZ_E_CRC
    assert out[:len(parts[0])].cpu().numpy().tobytes() == parts[0]
    tail = comp + b"\x1f\x8b\x08"
    assert orc.gunzip(tail).status == orc.E_HEADER
    with pytest.raises(gz.GzError) as ei:
        gz.decompress_members(tail, out)
    assert ei.value.code == gz.GZ_E_HEADER


def test_bgzf_batch(orc):
    """A BGZF-style file of 64 KiB members (about 64 MiB) decoded as one
    batch: byte for byte the oracle's gunzip of all members."""
    import paper_1905_07224_amd as gz

    raw = synth.fastq_like(64 << 20, 831)
    comp = b"".join(synth.bgzf_member(raw[i:i + (64 << 10)], 6) for i in range(0, len(raw), 64 << 10)) + synth.bgzf_member(b"")
    g = orc.gunzip(comp)
    assert g.status == orc.OK
    _say("bgzf", len(comp), "bytes,", g.n_members, "members")
    out = gz.decompress_bgzf(comp)
    assert np.array_equal(out.cpu().numpy(), g.out)
    bad = bytearray(comp)
    bad[100] ^= 0x40
    with pytest.raises(gz.GzError):
        gz.decompress_bgzf(bytes(bad))
