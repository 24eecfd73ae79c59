"""Pins for the CPU oracle (no GPU).

Each check ties the oracle to something other than itself: the seeded source
text of a round trip through an independent encoder (zlib, GNU gzip), the
CRC-32 check value, hand-derived fixtures, streams whose output is known by
construction (tests/bitwriter.py), and invariants the paper states for the
two-pass method (Section VI-C): w_1 is fully determined, resolved windows
equal the true preceding 32 KiB, and replacing every U_j gives the file.
"""
import os
import shutil
import subprocess
import zlib

import numpy as np
import pytest

import synth
from bitwriter import (BitWriter, dynamic_block, expand, fixed_block, gzip_wrap, rle_lengths,
                       stored_block)

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _gold_lines(name):
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                yield [x.strip() for x in line.split("|")]


def wrap_tokens(blocks):
    """blocks: list of (kind, tokens or data, kwargs); last one is final."""
    bw = BitWriter()
    data = b""
    for i, (kind, payload, kw) in enumerate(blocks):
        final = i == len(blocks) - 1
        if kind == "stored":
            stored_block(bw, payload, final, **kw)
            data += payload
        elif kind == "fixed":
            fixed_block(bw, payload, final, **kw)
            data += expand(payload, data)
        else:
            dynamic_block(bw, payload, final, **kw)
            data += expand(payload, data)
    return bw.getvalue(), data


# ---------------------------------------------------------------- CRC-32

def test_crc32_check_value(orc):
    for inp, val, _ in _gold_lines("crc32_check.txt"):
        assert orc.crc32(inp.encode()) == int(val, 16)


@pytest.mark.parametrize("n", [0, 1, 7, 1000, 100003])
def test_crc32_matches_zlib(orc, n):
    b = np.random.default_rng(n).integers(0, 256, n, dtype=np.uint8).tobytes()
    assert orc.crc32(b) == zlib.crc32(b) & 0xFFFFFFFF


# ---------------------------------------------------------------- fixtures

def test_tiny_streams_golden(orc):
    for name, d, e, _ in _gold_lines("tiny_streams.txt"):
        data = bytes.fromhex(e)
        gz = gzip_wrap(bytes.fromhex(d), data)
        r = orc.gunzip(gz)
        assert r.status == orc.OK, (name, r.reason)
        assert r.out.tobytes() == data, name


# ---------------------------------------------------------------- round trips

def _texts():
    return {
        "fastq": synth.fastq_like(96 << 10, 7),
        "words": synth.word_stream(96 << 10, 8),
        "binary": np.random.default_rng(9).integers(0, 256, 20000, dtype=np.uint8).tobytes(),
        "dna": synth.random_dna(50000, 10),
        "empty": b"",
        "one": b"x",
    }


TEXTS = _texts()
STRATS = {"default": zlib.Z_DEFAULT_STRATEGY, "filtered": zlib.Z_FILTERED,
          "huffman": zlib.Z_HUFFMAN_ONLY, "rle": zlib.Z_RLE, "fixed": zlib.Z_FIXED}


@pytest.mark.parametrize("level", list(range(10)))
@pytest.mark.parametrize("strat", list(STRATS))
def test_roundtrip_zlib(orc, level, strat):
    for name, raw in TEXTS.items():
        gz = synth.gzip_member(raw, level, strategy=STRATS[strat])
        r = orc.gunzip(gz)
        assert r.status == orc.OK, (name, r.reason)
        assert r.out.tobytes() == raw, name
        assert r.crc_computed == r.crc_trailer == (zlib.crc32(raw) & 0xFFFFFFFF)
        assert r.isize_trailer == len(raw)
        if level == 0:
            assert set(r.block_type.tolist()) <= {0}
        if strat == "fixed" and level > 0 and raw:
            assert set(r.block_type.tolist()) <= ({0, 1} if name == "binary" else {1})


def test_roundtrip_segmented_member(orc):
    """One member made of sync-flushed segments with preset dictionaries."""
    raw = synth.fastq_like(600 << 10, 11)
    gz = synth.gzip_member(raw, 6, segment_bytes=128 << 10)
    r = orc.gunzip(gz)
    assert r.status == orc.OK and r.out.tobytes() == raw
    assert r.n_members == 1
    assert (r.block_type == 0).sum() >= 4  # the sync-flush markers


@pytest.mark.skipif(shutil.which("gzip") is None, reason="no gzip binary")
@pytest.mark.parametrize("level", [1, 6, 9])
def test_roundtrip_gzip_cli(orc, level):
    raw = TEXTS["fastq"] + TEXTS["words"]
    gz = subprocess.run(["gzip", "-n", "-%d" % level, "-c"], input=raw, capture_output=True, check=True).stdout
    r = orc.gunzip(gz)
    assert r.status == orc.OK and r.out.tobytes() == raw


# ---------------------------------------------------------------- hand-built streams

HIST32K = bytes((i * 7 + 3) & 0xFF for i in range(32768))

def _chain_lengths(order, n):
    """Code lengths 1, 2, ..., k - 1, k - 1 for the symbols in `order` (a
    complete code whose last two codes are the longest, k - 1 bits)."""
    lengths = [0] * n
    for i, sym in enumerate(order):
        lengths[sym] = min(i + 1, len(order) - 1)
    return lengths


# Literal/length and distance codes of 13 to 15 bits, longer than any lookup
# table of the decoder, including end-of-block, a length code and two
# distance codes at 15 bits (distances 129..256 of codes 14 and 15).
_LONG_LIT = _chain_lengths(list(range(97, 110)) + [257, 256, 110], 286)
_LONG_DIST = _chain_lengths(list(range(16)), 30)
_LONG_TOKENS = list(b"abcdefghijklmn") * 25 + [(3, 200), (3, 150), (3, 1), 110, (3, 130), 97, (3, 256), (3, 2)]

HAND = {
    "stored_len0": [("stored", b"", {})],
    "stored_len65535": [("stored", bytes(range(256)) * 255 + bytes(range(255)), {}), ("stored", b"", {})],
    "fixed_all_literals": [("fixed", list(range(256)), {})],
    "fixed_len3_len258": [("fixed", [65, 66, 67, (3, 3), (258, 2)], {})],
    "fixed_258_via_284": [("fixed", [65, 66, (258, 2, "284")], {})],
    "dynamic_258_via_284": [("dynamic", [65, 66, (258, 2, "284"), (258, 1)], {})],
    "fixed_dist1_rle": [("fixed", [120, (258, 1), (17, 1)], {})],
    "overlap_d_lt_len": [("fixed", [1, 2, 3, (10, 3), (7, 2)], {})],
    "dist_32768": [("stored", HIST32K[:16384], {}), ("stored", HIST32K[16384:], {}),
                   ("fixed", [(258, 32768), (3, 32768), (5, 32767)], {})],
    "dynamic_dist_32768": [("stored", HIST32K[:16384], {}), ("stored", HIST32K[16384:], {}),
                           ("dynamic", [(258, 32768), 65, (4, 32768)], {})],
    "dynamic_single_1bit_dist": [("dynamic", [97, 98, 99, (6, 3), 100, (9, 4)], {})],
    "dynamic_literal_only": [("dynamic", list(b"hello, literal-only block"), {})],
    "mixed_blocks": [("dynamic", list(b"abcabcabcabc") + [(20, 3)], {}), ("stored", b"raw bytes", {}),
                     ("fixed", [(9, 12), 33], {}), ("dynamic", [(30, 30), 10], {})],
    "dynamic_15bit_codes": [("dynamic", _LONG_TOKENS, {"lit_lengths": _LONG_LIT, "dist_lengths": _LONG_DIST}),
                            ("dynamic", _LONG_TOKENS, {"lit_lengths": _LONG_LIT, "dist_lengths": _LONG_DIST})],
}


@pytest.mark.parametrize("name", list(HAND))
def test_handbuilt(orc, name):
    deflate, data = wrap_tokens(HAND[name])
    r = orc.gunzip(gzip_wrap(deflate, data))
    assert r.status == orc.OK, r.reason
    assert r.out.tobytes() == data


def test_single_1bit_distance_code_shape(orc):
    """The lone distance code must be sent as one bit (RFC 1951 section 3.2.7)."""
    bw = BitWriter()
    toks = [97, 98, 99, (6, 3)]
    lit = [0] * 286
    for s in (97, 98, 99, 256, 260):
        lit[s] = 2 if s in (97, 98, 99) else 3
    # lengths 2,2,2,3,3 -> Kraft 3/4 + 2/8 = 1
    dist = [0] * 30
    dist[2] = 1  # distance 3 is code 2
    dynamic_block(bw, toks, True, lit_lengths=lit, dist_lengths=dist)
    data = expand(toks)
    r = orc.gunzip(gzip_wrap(bw.getvalue(), data))
    assert r.status == orc.OK and r.out.tobytes() == data


def _crossing(syms, boundary):
    pos = 0
    for s, e, _ in syms:
        n = 1 if s < 16 else (3 + e if s in (16, 17) else 11 + e)
        if s >= 16 and pos < boundary < pos + n:
            return s
        pos += n
    return None


def test_repeat_codes_cross_lit_dist_boundary(orc):
    """16 and 18 runs that span the literal/length and distance length lists
    (RFC 1951 section 3.2.7: the two lists form one sequence)."""
    # (a) a run of 5s: literal/length 256..285 and distance 0..23 are all 5 bits
    lit = [0] * 286
    lit[97] = lit[98] = 5
    for s in range(256, 286):
        lit[s] = 5            # 32 codes of 5 bits: complete
    dist = [5] * 24 + [4] * 4  # 24/32 + 4/16 = 1
    toks = [97, 98] * 20 + [(3, 1), (10, 2), (258, 1), (100, 300), (7, 3)]
    syms = rle_lengths(lit + dist)
    assert _crossing(syms, 286) == 16
    bw = BitWriter()
    dynamic_block(bw, toks, True, lit_lengths=lit, dist_lengths=dist, hlit=286, hdist=28, cl_syms=syms)
    data = expand(toks)
    r = orc.gunzip(gzip_wrap(bw.getvalue(), data))
    assert r.status == orc.OK, r.reason
    assert r.out.tobytes() == data
    # (b) a run of zeros: literal/length 262..285 and distance 0..9 are unused
    lit = [0] * 286
    for s in (97, 98, 256, 257, 258, 259, 260, 261):
        lit[s] = 3            # 8 codes of 3 bits: complete
    dist = [0] * 10 + [2] * 4  # distances 33..128 only
    toks = [97, 98] * 70 + [(5, 33), (7, 40), (6, 100), (3, 128)]
    syms = rle_lengths(lit + dist)
    assert _crossing(syms, 286) == 18
    bw = BitWriter()
    dynamic_block(bw, toks, True, lit_lengths=lit, dist_lengths=dist, hlit=286, hdist=14, cl_syms=syms)
    data = expand(toks)
    r = orc.gunzip(gzip_wrap(bw.getvalue(), data))
    assert r.status == orc.OK, r.reason
    assert r.out.tobytes() == data


# ---------------------------------------------------------------- negative cases

def _dyn_raw(bits_fn):
    bw = BitWriter()
    bits_fn(bw)
    return bw.getvalue()


def _neg(orc, deflate, reason, data=b"", status=None):
    r = orc.gunzip(gzip_wrap(deflate, data))
    assert r.status == (orc.E_DATA if status is None else status), r.reason
    assert r.reason == reason, r.reason


def test_neg_btype3(orc):
    _neg(orc, _dyn_raw(lambda b: (b.put(1, 1), b.put(3, 2), b.put(0, 16))), "BTYPE3")


def test_neg_nlen(orc):
    bw = BitWriter()
    stored_block(bw, b"abc", True, nlen_override=0x1234)
    _neg(orc, bw.getvalue(), "NLEN", b"abc")


def _dyn_header(bw, hlit, hdist, cl_lengths, final=1):
    from bitwriter import CL_ORDER
    bw.put(final, 1)
    bw.put(2, 2)
    bw.put(hlit - 257, 5)
    bw.put(hdist - 1, 5)
    hclen = 19
    bw.put(hclen - 4, 4)
    for i in range(hclen):
        bw.put(cl_lengths[CL_ORDER[i]], 3)


def test_neg_hlit_hdist(orc):
    _neg(orc, _dyn_raw(lambda b: _dyn_header(b, 287, 1, [2] * 4 + [0] * 15)), "HLIT")
    _neg(orc, _dyn_raw(lambda b: _dyn_header(b, 257, 31, [2] * 4 + [0] * 15)), "HDIST")


def test_neg_cl_codes(orc):
    _neg(orc, _dyn_raw(lambda b: _dyn_header(b, 257, 1, [1, 1, 1] + [0] * 16) or b.put(0, 64)), "CL_OVERSUB")
    _neg(orc, _dyn_raw(lambda b: _dyn_header(b, 257, 1, [2, 2, 2] + [0] * 16) or b.put(0, 64)), "CL_INCOMPLETE")


def _cl_complete_header(bw, hlit, hdist):
    """Code-length code: symbols 0..15,16,17,18 get lengths making a complete code.
    Symbols 0-12 length 5? simpler: 16 symbols of length 4 -> symbols 0..15."""
    cl = [4] * 16 + [0, 0, 0]
    _dyn_header(bw, hlit, hdist, cl)
    return cl


def _emit_lengths(bw, lengths, cl):
    from bitwriter import canonical
    c = canonical(cl)
    for L in lengths:
        bw.put_code(*c[L])


def test_neg_repeat_rules(orc):
    def no_prev(b):
        cl = [0] * 16 + [1, 1, 0]  # symbols 16 and 17, one bit each
        _dyn_header(b, 257, 1, cl)
        from bitwriter import canonical
        c = canonical(cl)
        b.put_code(*c[16])
        b.put(0, 2)
        b.put(0, 64)
    _neg(orc, _dyn_raw(no_prev), "REPEAT_NO_PREV")

    def overrun(b):
        cl = [0] * 16 + [0, 1, 1]  # 17 and 18
        _dyn_header(b, 257, 1, cl)
        from bitwriter import canonical
        c = canonical(cl)
        b.put_code(*c[18])
        b.put(127, 7)  # 138 zeros
        b.put_code(*c[18])
        b.put(127, 7)  # 276 zeros
        b.put_code(*c[17])
        b.put(0, 3)  # +3 = 279 > 258
        b.put(0, 64)
    _neg(orc, _dyn_raw(overrun), "REPEAT_OVERRUN")


def _lit_dist_block(lit, dist, hlit, hdist, body=None, pad=True):
    def f(b):
        cl = _cl_complete_header(b, hlit, hdist)
        _emit_lengths(b, list(lit) + list(dist), cl)
        if body:
            body(b)
        if pad:
            b.put(0, 64)
    return _dyn_raw(f)


def test_neg_table_validity(orc):
    lit = [0] * 257
    lit[65] = 1
    lit[66] = 1
    _neg(orc, _lit_dist_block(lit, [1], 257, 1), "NO_EOB")
    lit = [0] * 257
    lit[65] = lit[66] = lit[256] = 1
    _neg(orc, _lit_dist_block(lit, [1], 257, 1), "LIT_OVERSUB")
    lit = [0] * 257
    lit[65] = 1
    lit[256] = 2
    _neg(orc, _lit_dist_block(lit, [1], 257, 1), "LIT_INCOMPLETE")
    lit = [0] * 257
    lit[65] = lit[256] = 1
    _neg(orc, _lit_dist_block(lit, [1, 1, 1], 257, 3), "DIST_OVERSUB")
    _neg(orc, _lit_dist_block(lit, [2, 2], 257, 2), "DIST_INCOMPLETE")


def test_lone_litlen_code_is_accepted_by_decoder(orc):
    """A literal/length code made of the end-of-block symbol alone (one 1-bit code)."""
    lit = [0] * 257
    lit[256] = 1
    deflate = _lit_dist_block(lit, [0], 257, 1, body=lambda b: b.put_code(0, 1), pad=False)
    r = orc.gunzip(gzip_wrap(deflate, b""))
    assert r.status == orc.OK, r.reason


def test_neg_symbols(orc):
    bw = BitWriter()
    fixed_block(bw, [], True, raw_symbols=[65, 286])
    _neg(orc, bw.getvalue(), "BAD_LITLEN")
    bw = BitWriter()
    fixed_block(bw, [], True, raw_symbols=[65, 287])
    _neg(orc, bw.getvalue(), "BAD_LITLEN")

    def bad_dist(code):
        def f(b):
            from bitwriter import canonical, fixed_lengths
            b.put(1, 1)
            b.put(1, 2)
            lc = canonical(fixed_lengths())
            b.put_code(*lc[65])
            b.put_code(*lc[257])  # length 3
            b.put_code(code, 5)
            b.put(0, 32)
        return _dyn_raw(f)
    _neg(orc, bad_dist(30), "BAD_DIST")
    _neg(orc, bad_dist(31), "BAD_DIST")


def test_neg_no_dist_codes(orc):
    lit = [0] * 258
    lit[65] = lit[256] = 2
    lit[257] = 1
    # literal-only distance code (all zero) but a length symbol appears
    def body(b):
        from bitwriter import canonical
        c = canonical(lit)
        b.put_code(*c[65])
        b.put_code(*c[257])
    _neg(orc, _lit_dist_block(lit, [0], 258, 1, body=body), "NO_DIST")


def test_neg_too_far(orc):
    deflate, _ = wrap_tokens([("fixed", [65, 66, (3, 2)], {})])
    # a distance one more than the output so far
    bw = BitWriter()
    fixed_block(bw, [65, 66], False)
    bw2 = BitWriter()
    from bitwriter import canonical, fixed_lengths
    bw.put(1, 1)
    bw.put(1, 2)
    lc = canonical(fixed_lengths())
    bw.put_code(*lc[257])
    bw.put_code(2, 5)  # distance 3 > 2 bytes of history
    bw.put_code(*lc[256])
    _neg(orc, bw.getvalue(), "TOO_FAR", b"AB")


def test_neg_truncation(orc):
    raw = TEXTS["fastq"][:20000]
    gz = synth.gzip_member(raw, 6)
    for cut in (12, len(gz) // 2, len(gz) - 9, len(gz) - 1):
        r = orc.gunzip(gz[:cut])
        assert r.status != orc.OK
    r = orc.gunzip(gz[:len(gz) // 2])
    assert r.reason == "TRUNC"


def test_neg_header_and_trailer(orc):
    raw = b"header and trailer checks\n" * 50
    gz = bytearray(synth.gzip_member(raw, 6))
    bad = bytearray(gz); bad[0] = 0x1e
    assert orc.gunzip(bytes(bad)).reason == "MAGIC"
    bad = bytearray(gz); bad[2] = 7
    assert orc.gunzip(bytes(bad)).reason == "CM"
    bad = bytearray(gz); bad[3] |= 0x20
    assert orc.gunzip(bytes(bad)).reason == "FLG"
    bad = bytearray(gz); bad[-8] ^= 1
    r = orc.gunzip(bytes(bad)); assert r.status == orc.E_CRC and r.reason == "CRC"
    bad = bytearray(gz); bad[-4] ^= 1
    r = orc.gunzip(bytes(bad)); assert r.status == orc.E_SIZE and r.reason == "ISIZE"
    deflate = zlib.compress(raw, 6)[2:-4]
    g = bytearray(gzip_wrap(deflate, raw, hcrc=True))
    assert orc.gunzip(bytes(g)).status == orc.OK
    g[10] ^= 1
    assert orc.gunzip(bytes(g)).reason == "HCRC"


def test_header_optional_fields(orc):
    raw = b"optional fields " * 100
    deflate = zlib.compress(raw, 6)[2:-4]
    gz = gzip_wrap(deflate, raw, extra=b"\x01\x02ab", name=b"file.txt", comment=b"a comment", hcrc=True)
    r = orc.gunzip(gz)
    assert r.status == orc.OK and r.out.tobytes() == raw
    st, h, _ = orc.parse_header(gz)
    assert st == orc.OK and h == len(gz) - len(deflate) - 8


def test_multi_member(orc):
    a, b = b"first member\n" * 100, b"second member\n" * 77
    gz = synth.gzip_member(a, 6) + synth.gzip_member(b, 1)
    r = orc.gunzip(gz)
    assert r.status == orc.OK and r.out.tobytes() == a + b and r.n_members == 2
    r = orc.gunzip(gz + b"\x00")
    assert r.status == orc.E_HEADER and r.reason == "GARBAGE"


# ---------------------------------------------------------------- provenance and pass 1

@pytest.fixture(scope="module")
def fq():
    raw = synth.fastq_like(1 << 20, 21)
    gz = synth.gzip_member(raw, 6)
    return raw, gz


def test_provenance(orc, fq):
    raw, gz = fq
    r = orc.gunzip(gz, parent=True)
    out = r.out
    par = r.parent
    assert out.tobytes() == raw
    m = par >= 0
    x = np.nonzero(m)[0]
    assert np.all(par[m] < x) and np.all(x - par[m] <= 32768)
    # rebuild the text from literal bytes and parent links alone
    rebuilt = np.zeros_like(out)
    lit = ~m
    rebuilt[lit] = np.frombuffer(raw, np.uint8)[lit]
    for i in x:  # parents come first, so one forward pass suffices
        rebuilt[i] = rebuilt[par[i]]
    assert rebuilt.tobytes() == raw


def _sym_from_parent(out, parent, o, n):
    """sym(x) for x in [o, o+n): a byte for literal provenance, else U_(x - o + 32768) for x < o."""
    sym = np.zeros(n, dtype=np.int64)
    for k in range(n):
        x = o + k
        p = parent[x]
        if p < 0:
            sym[k] = out[x]
        elif p < o:
            sym[k] = 0x8000 | (p - o + 32768)
        else:
            sym[k] = sym[p - o]
    return sym.astype(np.uint16)


def test_symbolic_pass_matches_provenance(orc, fq):
    """decompress(C_i, w_hat_i) from a true block start equals the symbols derived
    from the plain decoder's provenance; U_j marks exactly the bytes whose
    copy chain leaves the chunk."""
    raw, gz = fq
    r = orc.gunzip(gz, parent=True)
    nb = len(r.block_bit)
    assert nb >= 6
    for k in (1, nb // 2, nb - 3):
        s = int(r.block_bit[k])
        stop = int(r.block_bit[k + 2])
        sr = orc.symbolic(gz, s, stop, first=False)
        assert sr.status == orc.OK
        o = int(r.block_out_off[k])
        n = int(r.block_out_off[k + 2] - o)
        assert len(sr.sym) == n and sr.end_bit == stop and sr.n_blocks == 2
        exp = _sym_from_parent(r.out, r.parent, o, n)
        assert np.array_equal(sr.sym, exp)
        assert sr.n_placeholders == int((exp >= 0x8000).sum())
        assert sr.n_syms == int(r.block_nsym[k] + r.block_nsym[k + 1])
        # replacing U_j by the true window gives the bytes (Section VI-C)
        win = r.out[o - 32768:o] if o >= 32768 else None
        if win is not None:
            t = sr.sym
            res = np.where(t < 256, t, win[t & 0x7FFF].astype(np.uint16))
            assert res.astype(np.uint8).tobytes() == raw[o:o + n]
    # the first chunk has an empty context and no placeholders
    s0 = orc.symbolic(gz, r.payload_start * 8, 1 << 60, first=True)
    assert s0.status == orc.OK and s0.final_reached and s0.n_placeholders == 0
    assert s0.sym.astype(np.uint8).tobytes() == raw


# ---------------------------------------------------------------- two-pass method

@pytest.mark.parametrize("n_chunks", [1, 2, 3, 8, 40])
def test_pugz_equals_gunzip(orc, fq, n_chunks):
    raw, gz = fq
    p = orc.pugz(gz, n_chunks)
    assert p.status == orc.OK, p.reason
    assert p.out.tobytes() == raw
    assert p.crc_computed == p.crc_trailer
    r = orc.gunzip(gz)
    bits = set(r.block_bit.tolist())
    nonempty = p.start >= 0
    assert all(int(s) in bits for s in p.start[nonempty])
    # lengths add up, offsets are the exclusive prefix sum
    assert int(p.len.sum()) == len(raw)
    assert np.array_equal(p.off[1:], np.cumsum(p.len)[:-1])
    # resolved windows are the true preceding 32 KiB (invariants of Section VI-C)
    out = np.frombuffer(raw, np.uint8)
    for i in np.nonzero(nonempty)[0]:
        o, v = int(p.off[i]), int(p.valid[i])
        assert v == min(o, 32768)
        if v:
            assert np.array_equal(p.windows[i][32768 - v:], out[o - v:o])
    # chunk 0 decodes without placeholders
    assert p.placeholders[0] == 0


@pytest.mark.parametrize("kind,level", [("words", 6), ("fastq", 1), ("fastq", 9), ("dna", 6), ("dna", 1)])
def test_pugz_other_inputs(orc, kind, level):
    raw = {"words": lambda: synth.word_stream(700 << 10, 31), "fastq": lambda: synth.fastq_like(700 << 10, 32),
           "dna": lambda: synth.random_dna(700 << 10, 33)}[kind]()
    gz = synth.gzip_member(raw, level)
    for n in (2, 7):
        p = orc.pugz(gz, n)
        assert p.status == orc.OK, p.reason
        assert p.out.tobytes() == raw


def test_pugz_more_chunks_than_blocks(orc):
    raw = synth.fastq_like(300 << 10, 41)
    gz = synth.gzip_member(raw, 6)
    p = orc.pugz(gz, 200)
    assert p.status == orc.OK and p.out.tobytes() == raw
    assert (p.start < 0).sum() > 100  # most chunks hold no block start


def test_pugz_level0_no_dynamic_blocks(orc):
    raw = synth.fastq_like(200 << 10, 42)
    gz = synth.gzip_member(raw, 0)
    p = orc.pugz(gz, 4)
    assert p.status == orc.OK and p.out.tobytes() == raw
    assert (p.start[1:] < 0).all()


def test_pugz_rejects_second_member(orc):
    gz = synth.gzip_member(b"a" * 5000, 6) + synth.gzip_member(b"b" * 5000, 6)
    p = orc.pugz(gz, 2)
    assert p.status == orc.E_UNSUPPORTED


# ---------------------------------------------------------------- block-start checks

def test_predicate_accepts_true_starts(orc, fq):
    raw, gz = fq
    r = orc.gunzip(gz)
    nb = len(r.block_bit)
    for k in range(nb):
        ok, why = orc.block_predicate(gz, int(r.block_bit[k]))
        eligible = (r.block_type[k] == 2 and not r.block_final[k] and 1024 < r.block_out_len[k] < (4 << 20))
        assert ok == eligible, (k, why)


def test_find_start_lands_on_true_blocks(orc):
    raw = synth.word_stream(900 << 10, 51)
    gz = synth.gzip_member(raw, 6)
    r = orc.gunzip(gz)
    bits = r.block_bit
    n = len(gz)
    lo = 8 * (n // 3)
    s = orc.find_start(gz, lo, 8 * n)
    assert s in set(bits.tolist())
    assert s == int(bits[bits >= lo].min())  # no false positive before the true one
    s_static = orc.find_start(gz, lo, 8 * n, static_only=True)
    assert s_static <= s


def test_predicate_rules_on_handbuilt(orc):
    text = (b"The quick brown fox jumps over the lazy dog. " * 40)[:1500]
    toks = list(text)

    def stream(first_tokens, final_first=False, btype="dynamic", more=5):
        bw = BitWriter()
        if btype == "dynamic":
            dynamic_block(bw, first_tokens, final_first)
        else:
            fixed_block(bw, first_tokens, final_first)
        for i in range(more):
            dynamic_block(bw, toks[:200], i == more - 1)
        return bw.getvalue()

    ok, why = orc.block_predicate(stream(toks), 0)
    assert ok, why
    ok, why = orc.block_predicate(stream(toks, final_first=True, more=0), 0)
    assert not ok and why == "FINAL"
    ok, why = orc.block_predicate(stream(toks, btype="fixed"), 0)
    assert not ok and why == "NOT_DYNAMIC"
    ok, why = orc.block_predicate(stream(toks[:1024]), 0)
    assert not ok and why == "SIZE"
    ok, why = orc.block_predicate(stream(toks[:1025]), 0)
    assert ok, why
    ok, why = orc.block_predicate(stream(toks[:600] + [1] + toks[600:]), 0)
    assert not ok and why == "NOT_ASCII"
    # matches into the unknown context before the candidate are allowed
    ok, why = orc.block_predicate(stream([(200, 30000)] + toks), 0)
    assert ok, why
    # a bad block among the five that follow rejects the candidate
    bw = BitWriter()
    dynamic_block(bw, toks, False)
    dynamic_block(bw, toks[:100], False)
    bw.put(0, 1)
    bw.put(3, 2)
    bw.put(0, 64)
    ok, why = orc.block_predicate(bw.getvalue(), 0)
    assert not ok and why == "BTYPE3"
    # a final block among the five ends the check successfully
    bw = BitWriter()
    dynamic_block(bw, toks, False)
    dynamic_block(bw, toks[:100], True)
    ok, why = orc.block_predicate(bw.getvalue(), 0)
    assert ok, why


# ---------------------------------------------------------------- false block starts and repair

@pytest.fixture(scope="module", params=[True, False], ids=["inner-final", "inner-nonfinal"])
def decoy_case(request):
    import decoy

    return decoy.decoy_member(final_last=request.param)


def test_decoy_is_a_false_positive(orc, decoy_case):
    """The inner stream's block starts pass Appendix A's checks although they
    lie inside a stored block of the real chain (Section VI-A's false
    positives); the real chain is the encoder's."""
    gz, raw, real_bits, decoy_bits = decoy_case
    g = orc.gunzip(gz)
    assert g.status == orc.OK and g.out.tobytes() == raw
    assert g.block_bit.tolist() == real_bits  # the sequential decoder follows the encoder's chain
    assert not set(decoy_bits) & set(real_bits)
    # each stored block holds 40 inner blocks; all but the last six have a
    # non-final trial block and five more blocks inside the stored payload
    for g0 in range(0, len(decoy_bits), 40):
        for b in decoy_bits[g0:g0 + 34]:
            ok, why = orc.block_predicate(gz, b)
            assert ok, (b, why)


@pytest.mark.parametrize("n_chunks", [2, 3, 4, 6, 9, 13])
def test_pugz_repairs_false_starts(orc, decoy_case, n_chunks):
    """Every false start the search accepts is replaced by the bit where the
    previous chunk stopped; the output stays the encoder's text (the
    exactness argument of the stitch check: by induction from the first
    chunk, every start that is kept is on the real chain)."""
    gz, raw, real_bits, decoy_bits = decoy_case
    p = orc.pugz(gz, n_chunks)
    assert p.status == orc.OK, p.reason
    assert p.out.tobytes() == raw
    assert p.n_repairs >= 1
    repaired = [i for i in range(n_chunks) if p.cand[i] >= 0 and p.cand[i] != p.start[i] and p.start[i] >= 0]
    assert len(repaired) == p.n_repairs
    real, dec = set(real_bits), set(decoy_bits)
    for i in repaired:
        assert int(p.cand[i]) in dec and int(p.start[i]) in real
        assert p.start[i] == p.end[i - 1 - int(np.argmax(p.start[:i][::-1] >= 0))]
    assert all(int(s) in real for s in p.start[p.start >= 0])
    assert int(p.len.sum()) == len(raw)


def test_pugz_too_far_found_by_translation(orc):
    """A match reaching before the data start, inside a chunk other than the
    first: pass 1 decodes it as a placeholder (the chunk's context is
    unknown), and the translation finds the placeholder outside the real
    history.  The sequential decoder reports the same error."""
    import decoy

    gz, bad_bit, bits = decoy.too_far_member()
    g = orc.gunzip(gz)
    assert g.status == orc.E_DATA and g.reason == "TOO_FAR"
    seen = 0
    for n in range(2, 9):
        p = orc.pugz(gz, n)
        assert p.status == orc.E_DATA and p.reason == "TOO_FAR", (n, p.reason)
        ne = np.nonzero(p.start >= 0)[0]
        i = int(ne[np.searchsorted(p.start[ne], bad_bit, side="right") - 1])
        if i == 0:
            continue
        seen += 1
        # pass 1 of that chunk alone succeeds; the bad reference is a placeholder
        nxt = [int(p.start[j]) for j in ne if j > i]
        s = orc.symbolic(gz, int(p.start[i]), nxt[0] if nxt else 1 << 62, first=False)
        assert s.status == orc.OK
        ph = s.sym[s.sym >= 0x8000] & 0x7FFF
        # the windows and offsets were resolved before the translation failed
        assert int(p.valid[i]) == min(int(p.off[i]), 32768) < 20000
        assert ph.size and int(ph.min()) < 32768 - int(p.valid[i])
    assert seen >= 4
    # the whole member as one chunk: the first chunk has an empty context
    p = orc.pugz(gz, 1)
    assert p.status == orc.E_DATA and p.reason == "TOO_FAR"


def test_symbolic_block_bits(orc, decoy_case):
    """The symbolic pass records where each block it decodes begins: from the
    payload, the encoder's own block chain (and the sequential decoder's
    block map); from an encoder segment boundary of a pigz-style member, the
    rest of the sequential decoder's block map up to the stop."""
    gz, raw, real_bits, decoy_bits = decoy_case
    s = orc.symbolic(gz, real_bits[0], 1 << 62, first=True)
    assert s.status == orc.OK and s.final_reached
    assert s.block_bits.tolist() == real_bits
    data = synth.fastq_like(3 << 20, 77)
    comp, seg = synth.gzip_member_indexed(data, 6, segment_bytes=1 << 20)
    g = orc.gunzip(comp)
    assert g.status == orc.OK
    for k in range(len(seg)):
        stop = seg[k + 1] if k + 1 < len(seg) else 1 << 62
        s = orc.symbolic(comp, seg[k], stop, first=(k == 0))
        assert s.status == orc.OK
        want = g.block_bit[(g.block_bit >= seg[k]) & (g.block_bit < stop)]
        assert np.array_equal(s.block_bits, want), k
        assert s.sym.size == (min((k + 1) << 20, len(data)) - (k << 20))


@pytest.mark.parametrize("level", [1, 6, 9])
def test_binary_mode_predicate_on_block_map(orc, level):
    """Binary inputs (Section VIII): every non-final dynamic block of a binary
    member (gunzip's block map) passes Appendix A's checks without the ASCII
    test, and fails the text checks on a non-ASCII literal; stored blocks
    (from the random stretches) and the final block fail both."""
    raw = synth.binary_records(3 << 20, 5)
    comp = synth.gzip_member(raw, level)
    g = orc.gunzip(comp)
    assert g.status == orc.OK and g.out.tobytes() == raw
    assert (g.block_type == 0).sum() >= 2 and (g.block_type == 2).sum() >= 20
    for b, t, f, size in zip(g.block_bit, g.block_type, g.block_final, g.block_out_len):
        ok_bin, why_bin = orc.block_predicate(comp, int(b), binary=True)
        ok_txt, why_txt = orc.block_predicate(comp, int(b))
        assert not ok_txt
        if t == 2 and not f and 1024 < size < (4 << 20):
            assert ok_bin, (int(b), why_bin)
            assert why_txt == "NOT_ASCII"
        else:
            assert not ok_bin and why_bin in ("FINAL", "NOT_DYNAMIC", "SIZE")


@pytest.mark.parametrize("n", [2, 3, 5, 8, 13])
def test_binary_mode_pugz(orc, n):
    """The two-pass method on a binary member: in binary mode every chunk
    start is a block of the map and the output is the source; in text mode
    no chunk after the first finds a start, and the first chunk's decode
    still gives the source."""
    raw = synth.binary_records(2 << 20, 6)
    comp = synth.gzip_member(raw, 6)
    g = orc.gunzip(comp)
    blocks = set(g.block_bit.tolist())
    r = orc.pugz(comp, n, binary=True)
    assert r.status == orc.OK and r.out.tobytes() == raw and r.n_repairs == 0
    starts = r.start[r.start >= 0]
    assert set(starts.tolist()) <= blocks and starts.size >= min(n, 10)
    t = orc.pugz(comp, n)
    assert t.status == orc.OK and t.out.tobytes() == raw
    assert (t.start[1:] < 0).all()


def test_stored_start_predicate(orc):
    """Stored blocks as chunk starts: on a level-0 member (stored blocks only)
    every non-final stored block of more than 1 KiB passes the static check
    with the stored type and not without it; a bit just after its LEN/NLEN
    bytes does not; the first passing bit of a range holding a stored header
    lies in the zero run just before that header's LEN/NLEN."""
    raw = synth.fastq_like(1 << 20, 73)
    comp = synth.gzip_member(raw, 0)
    g = orc.gunzip(comp)
    assert (g.block_type == 0).all() and len(g.block_bit) > 10
    T = orc.START_DYNAMIC | orc.START_STORED
    for b, f, size in zip(g.block_bit, g.block_final, g.block_out_len):
        b = int(b)
        ok, why = orc.block_static(comp, b, T)
        assert ok == (not f and size > 1024), (b, why)
        assert not orc.block_static(comp, b)[0]
        p = (b + 10) >> 3  # byte holding LEN
        assert not orc.block_static(comp, 8 * p + 33, T)[0]
        if not f:
            s = orc.find_start(comp, b - 12, b + 64, static_only=True, types=T)
            assert b - 10 <= s <= b and ((s + 10) >> 3) == p


@pytest.mark.parametrize("n", [2, 5, 11])
def test_stored_starts_pugz(orc, n):
    """The two-pass method with stored starts on a level-0 member: byte exact,
    every chunk start after the stitch check is a block of the map, and the
    starts found a bit or two early (in the zero run before the same LEN)
    are taken as the previous chunk's end without a repair."""
    raw = synth.fastq_like(1 << 20, 74)
    comp = synth.gzip_member(raw, 0)
    g = orc.gunzip(comp)
    blocks = set(g.block_bit.tolist())
    r = orc.pugz(comp, n, types=orc.START_DYNAMIC | orc.START_STORED)
    assert r.status == orc.OK and r.out.tobytes() == raw and r.n_repairs == 0
    s = r.start[r.start >= 0]
    assert s.size == n and set(s.tolist()) <= blocks
    assert r.n_equivalent == int((r.cand[1:] != r.start[1:]).sum()) and r.n_equivalent >= 1
    d = orc.pugz(comp, n)
    assert d.out.tobytes() == raw and (d.start[1:] < 0).all()


def test_fixed_starts_resynchronise(orc):
    """Why fixed blocks are not offered as chunk starts: on a member of fixed
    blocks only (zlib's Z_FIXED strategy), searching fixed starts with
    Appendix A's checks finds positions inside blocks whose decode has
    resynchronised with the true code stream; the stitch check repairs them,
    so the output stays exact, but most starts are repairs."""
    import struct

    raw = synth.fastq_like(2 << 20, 71)
    co = zlib.compressobj(6, zlib.DEFLATED, -15, 9, zlib.Z_FIXED)
    deflate = co.compress(raw) + co.flush()
    comp = (b"\x1f\x8b\x08\x00\x00\x00\x00\x00\x00\x03" + deflate
            + struct.pack("<II", zlib.crc32(raw) & 0xFFFFFFFF, len(raw) & 0xFFFFFFFF))
    g = orc.gunzip(comp)
    assert g.status == orc.OK and (g.block_type == 1).all()
    r = orc.pugz(comp, 8, types=orc.START_DYNAMIC | orc.START_FIXED)
    assert r.status == orc.OK and r.out.tobytes() == raw
    found = r.cand[1:][r.cand[1:] >= 0]
    assert found.size >= 4 and r.n_repairs * 2 > found.size
    # the repaired starts were not blocks of the map
    assert len(set(found.tolist()) - set(g.block_bit.tolist())) >= r.n_repairs
