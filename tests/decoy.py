"""Hand-built gzip members whose block-start search meets false starts.

Appendix A's checks (a dynamic non-final header with valid code tables, a
trial block of ASCII literals between 1 KiB and 4 MiB, five more decodable
ASCII blocks) are a heuristic: a bit offset that is not on the member's block
chain can pass them (Section VI-A names such false positives).  The cheapest
way to make one is a stored block whose raw payload is itself the bit stream
of several dynamic ASCII blocks: every block start of that inner stream passes
the checks, yet it lies inside a stored block of the real chain.

The two-pass method stays exact only if such a start is caught: the chunk
before it stops at the first real block header at or past the false start,
which is not the false start, and the chunk is decoded again from where its
predecessor stopped.  These members make that happen at many chunk counts.

Also here: a member whose second part references bytes before the data start
(the "distance too far back" error, found by the translation step when the
reference crosses a chunk boundary).

Everything is built with the test-side encoder (``bitwriter``), so the
expected output is known by construction.
"""
from __future__ import annotations

import numpy as np

from bitwriter import BitWriter, dynamic_block, gzip_wrap, stored_block

MAX_DIST = 32768
HEADER_BITS = 80  # gzip_wrap's 10-byte member header with no optional fields


class Tokenizer:
    """Greedy LZ77 over one output sequence (matches of 3..258 bytes, at most
    32768 back), fed range by range in output order; stored ranges only enter
    the history."""

    def __init__(self, out: bytes, min_dist: int = 1):
        self.out = out
        self.head: dict[bytes, int] = {}
        self.pos = 0
        self.min_dist = min_dist

    def _insert(self, p):
        if p + 3 <= len(self.out):
            self.head[self.out[p:p + 3]] = p

    def skip(self, hi):
        for p in range(self.pos, hi):
            self._insert(p)
        self.pos = hi

    def tokens(self, hi):
        out = self.out
        toks = []
        p = self.pos
        while p < hi:
            cand = self.head.get(out[p:p + 3]) if p + 3 <= hi else None
            L = 0
            if cand is not None and self.min_dist <= p - cand <= MAX_DIST:
                lim = min(258, hi - p)
                while L < lim and out[cand + L] == out[p + L]:
                    L += 1
            if L >= 3:
                toks.append((L, p - cand))
                for q in range(p, p + L):
                    self._insert(q)
                p += L
            else:
                toks.append(out[p])
                self._insert(p)
                p += 1
        self.pos = hi
        return toks


def ascii_text(n: int, seed: int) -> bytes:
    """Seeded lowercase words, spaces and newlines (all in the checks' ASCII set)."""
    rng = np.random.default_rng(seed)
    vocab = [bytes(rng.integers(97, 123, int(rng.integers(2, 9)), dtype=np.uint8)) for _ in range(300)]
    out = bytearray()
    col = 0
    while len(out) < n:
        w = vocab[int(rng.zipf(1.3)) % len(vocab)]
        out += w
        col += len(w) + 1
        if col >= 70:
            out += b"\n"
            col = 0
        else:
            out += b" "
    return bytes(out[:n])


def inner_stream(n_blocks: int, block_bytes: int, seed: int, final_last: bool):
    """The raw DEFLATE bits of n_blocks dynamic ASCII blocks (the decoy), and
    the bit offset of each block header in them."""
    text = ascii_text(n_blocks * block_bytes, seed)
    tk = Tokenizer(text)
    bw = BitWriter()
    bits = []
    for k in range(n_blocks):
        toks = tk.tokens((k + 1) * block_bytes)
        bits.append(bw.nbits)
        dynamic_block(bw, toks, final=final_last and k == n_blocks - 1)
    return bw.getvalue(), bits


def decoy_member(seed: int = 1, layout=("R3", "S", "R6", "S", "R8"), real_bytes: int = 4000,
                 inner_blocks: int = 40, inner_bytes: int = 1400, final_last: bool = True):
    """A gzip member built from `layout`: "Rk" is k real dynamic blocks of
    real_bytes of text each (the last one of the member is final), "S" one
    stored block whose payload is an inner stream of inner_blocks dynamic
    ASCII blocks (its last one final when final_last).  Returns (member
    bytes, output bytes, bit offsets in the member of the real block headers,
    bit offsets of the inner streams' block headers); the bit offsets come
    from the encoder, not from any decoder."""
    parts = []  # ("R", text) or ("S", payload, inner block bits)
    s = seed * 1000
    for item in layout:
        if item == "S":
            s += 1
            pay, ibits = inner_stream(inner_blocks, inner_bytes, s, final_last)
            assert len(pay) <= 65535, len(pay)
            parts.append(("S", pay, ibits))
        else:
            for _ in range(int(item[1:])):
                s += 1
                parts.append(("R", ascii_text(real_bytes, s), None))
    out = b"".join(p[1] for p in parts)
    tk = Tokenizer(out)
    bw = BitWriter()
    real_bits, decoy_bits = [], []
    pos = 0
    for i, (kind, data, ibits) in enumerate(parts):
        last = i == len(parts) - 1
        real_bits.append(HEADER_BITS + bw.nbits)
        if kind == "S":
            tk.skip(pos + len(data))
            # payload after the 3 header bits, the alignment and LEN/NLEN
            pay0 = ((bw.nbits + 3 + 7) // 8) * 8 + 32
            decoy_bits += [HEADER_BITS + pay0 + b for b in ibits]
            stored_block(bw, data, final=last)
        else:
            dynamic_block(bw, tk.tokens(pos + len(data)), final=last)
        pos += len(data)
    return gzip_wrap(bw.getvalue(), out), out, real_bits, decoy_bits


def too_far_member(seed: int = 7, head_bytes: int = 3000, tail_blocks: int = 8, tail_bytes: int = 3000,
                   far: int = 20000):
    """A member whose first block gives head_bytes of text and whose later
    blocks (each one a valid block start) hold one match `far` bytes back,
    more than the output before it: the sequential decoder reports a distance
    too far back.  Returns (member bytes, bit offset of the block holding the
    bad match, bit offsets of all block headers), bits from the encoder."""
    assert far > head_bytes
    head = ascii_text(head_bytes, seed)
    tails = [ascii_text(tail_bytes, seed + 1 + k) for k in range(tail_blocks)]
    out = head + b"".join(tails)
    tk = Tokenizer(out)
    bw = BitWriter()
    bits = [HEADER_BITS]
    dynamic_block(bw, tk.tokens(head_bytes), final=False)
    bad_block = tail_blocks // 2
    p = head_bytes
    for k, t in enumerate(tails):
        toks = tk.tokens(p + len(t))
        if k == bad_block:
            # a 5-byte match reaching before the first byte of the member
            i = len(toks) // 2
            if not isinstance(toks[i], int):
                toks.insert(i, 32)
            toks.insert(i, (5, far))
            assert far > p + len(expand_len(toks[:i]))
        bits.append(HEADER_BITS + bw.nbits)
        dynamic_block(bw, toks, final=k == tail_blocks - 1)
        p += len(t)
    # the output is not defined; the trailer holds the text's CRC and size
    return gzip_wrap(bw.getvalue(), out), bits[1 + bad_block], bits


def expand_len(tokens):
    """Bytes that a token list produces (only their count matters here)."""
    return b"".join(bytes([t]) if isinstance(t, int) else bytes(t[0]) for t in tokens)


def trial_fail_member(seed: int = 3, real_before: int = 3, real_after: int = 6, real_bytes: int = 4000,
                      stored_bytes: int = 40000):
    """A member with one stored block of ASCII text whose payload starts with
    a small dynamic block (about 300 bytes of output): its header and code
    tables pass the static checks, its trial block is too small (not more
    than 1 KiB), and the rest of the payload holds no block start.  A chunk
    whose range starts inside that payload ends up empty after the rejection,
    and the chunk before it decodes through the whole stored block, far more
    than the span to the rejected candidate.  Returns (member bytes, output
    bytes, bit offset of the rejected candidate)."""
    small = BitWriter()
    small_text = ascii_text(300, seed * 7919)
    dynamic_block(small, Tokenizer(small_text).tokens(len(small_text)), final=False)
    head = small.getvalue()
    pad = ascii_text(stored_bytes - len(head), seed * 7919 + 1)
    payload = head + pad
    texts = [ascii_text(real_bytes, seed * 100 + k) for k in range(real_before + real_after)]
    out = b"".join(texts[:real_before]) + payload + b"".join(texts[real_before:])
    tk = Tokenizer(out)
    bw = BitWriter()
    pos = 0
    cand = None
    for k in range(real_before + real_after + 1):
        if k == real_before:
            tk.skip(pos + len(payload))
            cand = HEADER_BITS + ((bw.nbits + 3 + 7) // 8) * 8 + 32
            stored_block(bw, payload, final=False)
            pos += len(payload)
            continue
        t = texts[k if k < real_before else k - 1]
        dynamic_block(bw, tk.tokens(pos + len(t)), final=k == real_before + real_after)
        pos += len(t)
    return gzip_wrap(bw.getvalue(), out), out, cand


def dense_block_member(seed: int = 5, dense_bytes: int = 36000, mutate: float = 0.02, good_after: int = 5,
                       tail_blocks: int = 8, real_bytes: int = 4000):
    """A member whose dynamic block D compresses far better than the rest
    (repeated 100-byte lines with a few changed characters), followed by
    good_after ordinary text blocks, a block with one non-ASCII literal (B),
    and tail_blocks ordinary blocks.  Every block between D and B fails the
    block-start confirmation (B lies within their five confirmation blocks)
    and B fails its trial block, so a chunk whose range holds only those
    blocks ends up empty, and the chunk that starts at D decodes through it.
    Returns (member bytes, output bytes, bit offsets of D and of all block
    headers)."""
    rng = np.random.default_rng(seed)
    line = bytearray(ascii_text(100, seed * 31)[:99] + b"\n")
    dense = bytearray()
    while len(dense) < dense_bytes:
        for i in np.nonzero(rng.random(99) < mutate)[0]:
            line[int(i)] = 97 + int(rng.integers(0, 26))
        dense += line
    dense = bytes(dense[:dense_bytes])
    head = [ascii_text(real_bytes, seed * 100 + k) for k in range(6)]
    mid = [ascii_text(real_bytes, seed * 100 + 10 + k) for k in range(good_after)]
    bad = bytearray(ascii_text(real_bytes, seed * 100 + 30))
    bad[len(bad) // 2] = 0xFF
    tail = [ascii_text(real_bytes, seed * 100 + 40 + k) for k in range(tail_blocks)]
    parts = head + [dense] + mid + [bytes(bad)] + tail
    out = b"".join(parts)
    tk = Tokenizer(out)
    bw = BitWriter()
    bits = []
    pos = 0
    for i, t in enumerate(parts):
        bits.append(HEADER_BITS + bw.nbits)
        dynamic_block(bw, tk.tokens(pos + len(t)), final=i == len(parts) - 1)
        pos += len(t)
    return gzip_wrap(bw.getvalue(), out), out, bits[len(head)], bits
