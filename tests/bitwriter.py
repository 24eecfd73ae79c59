"""Test-side DEFLATE bit writer for hand-built streams (RFC 1951).

Streams are built from an explicit token list (literal bytes and
(length, distance) matches) with chosen block types and code lengths, so the
expected output is known by construction: ``expand(tokens)`` applies the
tokens with plain LZ77 semantics.  This is an encoder used only to make test
inputs; it shares nothing with either decoder under test.
"""
from __future__ import annotations

import heapq
import struct
import zlib

# RFC 1951 section 3.2.5, restated for the encoder side
LEN_BASE = [3, 4, 5, 6, 7, 8, 9, 10, 11, 13, 15, 17, 19, 23, 27, 31, 35, 43, 51, 59, 67, 83, 99,
            115, 131, 163, 195, 227, 258]
LEN_EXTRA = [0] * 8 + [1] * 4 + [2] * 4 + [3] * 4 + [4] * 4 + [5] * 4 + [0]
DIST_BASE = [1, 2, 3, 4, 5, 7, 9, 13, 17, 25, 33, 49, 65, 97, 129, 193, 257, 385, 513, 769, 1025,
             1537, 2049, 3073, 4097, 6145, 8193, 12289, 16385, 24577]
DIST_EXTRA = [0, 0, 0, 0] + [k for k in range(1, 14) for _ in (0, 1)]
CL_ORDER = [16, 17, 18, 0, 8, 7, 9, 6, 10, 5, 11, 4, 12, 3, 13, 2, 14, 1, 15]


class BitWriter:
    def __init__(self):
        self.bits: list[int] = []

    def put(self, value: int, n: int):
        """A field of n bits, least significant bit first."""
        for i in range(n):
            self.bits.append((value >> i) & 1)

    def put_code(self, code: int, length: int):
        """A Huffman code, most significant bit first."""
        for i in range(length - 1, -1, -1):
            self.bits.append((code >> i) & 1)

    def align(self):
        while len(self.bits) % 8:
            self.bits.append(0)

    @property
    def nbits(self) -> int:
        return len(self.bits)

    def getvalue(self) -> bytes:
        bits = self.bits + [0] * (-len(self.bits) % 8)
        out = bytearray(len(bits) // 8)
        for i, b in enumerate(bits):
            out[i >> 3] |= b << (i & 7)
        return bytes(out)


def canonical(lengths):
    """{symbol: (code, length)} for the canonical code of RFC 1951 section 3.2.2."""
    maxl = max(lengths) if lengths else 0
    bl = [0] * (maxl + 2)
    for L in lengths:
        if L:
            bl[L] += 1
    code = 0
    nxt = [0] * (maxl + 2)
    for L in range(1, maxl + 1):
        code = (code + bl[L - 1]) << 1
        nxt[L] = code
    out = {}
    for s, L in enumerate(lengths):
        if L:
            out[s] = (nxt[L], L)
            nxt[L] += 1
    return out


def huffman_lengths(freqs: dict, n: int, maxlen: int = 15):
    """Code lengths (complete code) for the symbols with nonzero frequency."""
    syms = [s for s in range(n) if freqs.get(s, 0) > 0]
    lengths = [0] * n
    if len(syms) == 1:
        lengths[syms[0]] = 1
        return lengths
    if not syms:
        return lengths
    heap = [(freqs[s], i, [s]) for i, s in enumerate(syms)]
    heapq.heapify(heap)
    depth = {s: 0 for s in syms}
    k = len(syms)
    while len(heap) > 1:
        f1, _, a = heapq.heappop(heap)
        f2, _, b = heapq.heappop(heap)
        for s in a + b:
            depth[s] += 1
        k += 1
        heapq.heappush(heap, (f1 + f2, k, a + b))
    if max(depth.values()) > maxlen:
        # flat fallback: smallest complete code with enough leaves
        m = len(syms)
        L = 1
        while (1 << L) < m:
            L += 1
        # (1<<L) - m leaves at L-1 make it complete
        short = (1 << L) - m
        for i, s in enumerate(syms):
            depth[s] = L - 1 if i < short else L
    for s in syms:
        lengths[s] = depth[s]
    return lengths


def len_code(length: int, use_284_for_258: bool = False):
    if length == 258 and use_284_for_258:
        return 284, 31, 5
    for i in range(28, -1, -1):
        if length >= LEN_BASE[i]:
            if i == 28 and length != 258:
                continue
            return 257 + i, length - LEN_BASE[i], LEN_EXTRA[i]
    raise ValueError(length)


def dist_code(d: int):
    for i in range(29, -1, -1):
        if d >= DIST_BASE[i]:
            return i, d - DIST_BASE[i], DIST_EXTRA[i]
    raise ValueError(d)


def expand(tokens, history: bytes = b"") -> bytes:
    """Plain LZ77 semantics: literal appends a byte, (L, d) copies byte by byte."""
    out = bytearray(history)
    for t in tokens:
        if isinstance(t, int):
            out.append(t)
        else:
            L, d = t[0], t[1]
            if d > len(out):
                raise ValueError("distance too far back")
            for _ in range(L):
                out.append(out[-d])
    return bytes(out[len(history):])


def _tok_syms(tokens, t284=False):
    for t in tokens:
        if isinstance(t, int):
            yield ("lit", t)
        else:
            L, d = t[0], t[1]
            use284 = t284 or (len(t) > 2 and t[2] == "284")
            yield ("len", len_code(L, use284))
            yield ("dist", dist_code(d))


def stored_block(bw: BitWriter, data: bytes, final: bool, nlen_override=None):
    assert len(data) <= 65535
    bw.put(1 if final else 0, 1)
    bw.put(0, 2)
    bw.align()
    bw.put(len(data), 16)
    bw.put((len(data) ^ 0xFFFF) if nlen_override is None else nlen_override, 16)
    for c in data:
        bw.put(c, 8)


def fixed_lengths():
    return [8] * 144 + [9] * 112 + [7] * 24 + [8] * 8


def _emit_tokens(bw, tokens, lit_codes, dist_codes, t284=False, fixed_dist=False):
    for kind, v in _tok_syms(tokens, t284):
        if kind == "lit":
            bw.put_code(*lit_codes[v])
        elif kind == "len":
            sym, extra, nb = v
            bw.put_code(*lit_codes[sym])
            bw.put(extra, nb)
        else:
            sym, extra, nb = v
            if fixed_dist:
                bw.put_code(sym, 5)
            else:
                bw.put_code(*dist_codes[sym])
            bw.put(extra, nb)
    bw.put_code(*lit_codes[256])


def fixed_block(bw: BitWriter, tokens, final: bool, raw_symbols=None):
    """raw_symbols: optional list of extra literal/length symbols (e.g. 286) to emit before EOB."""
    bw.put(1 if final else 0, 1)
    bw.put(1, 2)
    lit = canonical(fixed_lengths())
    if raw_symbols is None:
        _emit_tokens(bw, tokens, lit, None, fixed_dist=True)
    else:
        for s in raw_symbols:
            bw.put_code(*lit[s])


def rle_lengths(seq, allow16=True):
    """Code-length symbols (sym, extra, nbits) for a length sequence (RFC 1951 section 3.2.7)."""
    out = []
    i = 0
    n = len(seq)
    while i < n:
        v = seq[i]
        run = 1
        while i + run < n and seq[i + run] == v:
            run += 1
        if v == 0 and run >= 3:
            r = run
            while r >= 11:
                k = min(r, 138)
                out.append((18, k - 11, 7))
                r -= k
            if r >= 3:
                out.append((17, r - 3, 3))
                r = 0
            for _ in range(r):
                out.append((0, 0, 0))
            i += run
        elif v != 0 and run >= 4 and allow16:
            out.append((v, 0, 0))
            r = run - 1
            while r >= 3:
                k = min(r, 6)
                out.append((16, k - 3, 2))
                r -= k
            for _ in range(r):
                out.append((v, 0, 0))
            i += run
        else:
            out.append((v, 0, 0))
            i += 1
    return out


def dynamic_block(bw: BitWriter, tokens, final: bool, lit_lengths=None, dist_lengths=None,
                  cl_syms=None, cl_lengths=None, hlit=None, hdist=None, t284=False):
    """A dynamic-Huffman block.  By default code lengths come from token frequencies."""
    syms = list(_tok_syms(tokens, t284))
    if lit_lengths is None:
        f = {256: 1}
        for kind, v in syms:
            if kind == "lit":
                f[v] = f.get(v, 0) + 1
            elif kind == "len":
                f[v[0]] = f.get(v[0], 0) + 1
        lit_lengths = huffman_lengths(f, 286)
    if dist_lengths is None:
        f = {}
        for kind, v in syms:
            if kind == "dist":
                f[v[0]] = f.get(v[0], 0) + 1
        dist_lengths = huffman_lengths(f, 30) if f else [0]
    if hlit is None:
        hlit = max(257, max(i for i, L in enumerate(lit_lengths) if L) + 1)
    if hdist is None:
        used = [i for i, L in enumerate(dist_lengths) if L]
        hdist = max(1, (max(used) + 1) if used else 1)
    seq = list(lit_lengths[:hlit]) + [0] * max(0, hlit - len(lit_lengths))
    seq += list(dist_lengths[:hdist]) + [0] * max(0, hdist - len(dist_lengths))
    if cl_syms is None:
        cl_syms = rle_lengths(seq)
    if cl_lengths is None:
        f = {}
        for s, _, _ in cl_syms:
            f[s] = f.get(s, 0) + 1
        cl_lengths = huffman_lengths(f, 19, maxlen=7)
        if sum(1 for L in cl_lengths if L) == 1:
            # a lone code-length symbol: add a dummy so the code is complete
            other = 0 if cl_lengths[0] == 0 else 1
            cl_lengths[other] = 1
    hclen = 19
    while hclen > 4 and cl_lengths[CL_ORDER[hclen - 1]] == 0:
        hclen -= 1
    bw.put(1 if final else 0, 1)
    bw.put(2, 2)
    bw.put(hlit - 257, 5)
    bw.put(hdist - 1, 5)
    bw.put(hclen - 4, 4)
    for i in range(hclen):
        bw.put(cl_lengths[CL_ORDER[i]], 3)
    clc = canonical(cl_lengths)
    for s, extra, nb in cl_syms:
        bw.put_code(*clc[s])
        bw.put(extra, nb)
    litc = canonical(list(lit_lengths[:hlit]))
    distc = canonical(list(dist_lengths[:hdist])) if any(dist_lengths[:hdist]) else {}
    _emit_tokens(bw, tokens, litc, distc, t284)


def gzip_wrap(deflate: bytes, data: bytes, flags: int = 0, extra: bytes = b"", name: bytes = b"",
              comment: bytes = b"", hcrc: bool = False, crc=None, isize=None) -> bytes:
    flg = flags
    hdr = bytearray(b"\x1f\x8b\x08")
    if extra:
        flg |= 4
    if name:
        flg |= 8
    if comment:
        flg |= 16
    if hcrc:
        flg |= 2
    hdr.append(flg)
    hdr += b"\x00\x00\x00\x00\x00\xff"
    if extra:
        hdr += struct.pack("<H", len(extra)) + extra
    if name:
        hdr += name + b"\x00"
    if comment:
        hdr += comment + b"\x00"
    if hcrc:
        hdr += struct.pack("<H", zlib.crc32(bytes(hdr)) & 0xFFFF)
    c = (zlib.crc32(data) & 0xFFFFFFFF) if crc is None else crc
    s = (len(data) & 0xFFFFFFFF) if isize is None else isize
    return bytes(hdr) + deflate + struct.pack("<II", c, s)

