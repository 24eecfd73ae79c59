"""Seeded synthetic inputs for the gzip workloads (test and benchmark plumbing).

This module only *makes* inputs: text generators and a gzip encoder wrapper
around the system zlib.  It holds none of the decompression arithmetic, and
both the CPU oracle and the device path consume what it produces.

Generators
----------
* ``fastq_like``  -- 4-line FASTQ-style records with uniform random DNA.  The
  paper's speed test and random-access study use real ENA FASTQ files
  (Section VII); those are not available, so this generator stands in for
  them.  Record layout:

    ``@SIM:1:<lane>:<tile>:<x>:<y>``  lane = 1 + (k // 10**6) % 8,
                                      tile = 1101 + (k // 10**4) % 100,
                                      x ~ U[1000, 30000], y ~ U[1000, 100000]
    read      each base is N with probability 0.001, else uniform over ACGT
    ``+``
    quality   one char per base: 33 + clip(rint(N(35, 5)), 2, 40)

* ``word_stream`` -- generic ASCII text: Zipf(s=1.1) draws over a seeded
  vocabulary of 50 000 random lowercase words (length 2..12), punctuation
  from ``.,;:!?`` after a word with probability 0.05, a space between words
  and a newline once a line reaches 80 characters.

* ``gzip_member`` -- one RFC 1952 member around one raw DEFLATE stream made by
  zlib (a black-box encoder).  Large inputs are compressed as independent
  segments that each get the previous 32 KiB as a preset dictionary and end
  in a sync flush, so the result is still ONE member whose matches may reach
  across segment boundaries (the technique pigz uses).  Segment boundaries
  show up as an empty stored block.
"""
from __future__ import annotations

import os
import struct
import zlib
from concurrent.futures import ThreadPoolExecutor

import numpy as np

__all__ = [
    "fastq_like",
    "word_stream",
    "random_dna",
    "gzip_member",
    "gzip_member_indexed",
    "make",
    "cache_dir",
]

_ACGT = np.frombuffer(b"ACGT", dtype=np.uint8)


def _digits(out, pos, vals, nd):
    """Write the nd decimal digits of vals at out[pos .. pos + nd - 1]."""
    for d in range(nd):
        out[pos + d] = (vals // (10 ** (nd - 1 - d))) % 10 + 48


def _fastq_batch(rng, k0, n, read_lens):
    """n records, numbered from k0, laid out with array operations."""
    lens = rng.choice(np.asarray(read_lens, dtype=np.int64), size=n)
    tot = int(lens.sum())
    bases = _ACGT[rng.integers(0, 4, size=tot, dtype=np.uint8)]
    nmask = rng.random(tot, dtype=np.float32) < 0.001
    bases[nmask] = ord("N")
    q = rng.standard_normal(tot, dtype=np.float32) * 5.0 + 35.0
    qual = (np.clip(np.rint(q), 2, 40) + 33).astype(np.uint8)
    xs = rng.integers(1000, 30001, size=n)
    ys = rng.integers(1000, 100001, size=n)
    k = k0 + np.arange(n, dtype=np.int64)
    lane = 1 + (k // 1000000) % 8
    tile = 1101 + (k // 10000) % 100
    xd = np.where(xs >= 10000, 5, 4)
    yd = np.where(ys >= 100000, 6, np.where(ys >= 10000, 5, 4))
    # "@SIM:1:" lane ":" tile ":" x ":" y "\n", read "\n+\n", quality "\n"
    hdr = 7 + 1 + 1 + 4 + 1 + xd + 1 + yd + 1
    rec = hdr + lens + 3 + lens + 1
    start = np.concatenate(([0], np.cumsum(rec)[:-1]))
    out = np.empty(int(rec.sum()), dtype=np.uint8)
    out[start[:, None] + np.arange(7)] = np.frombuffer(b"@SIM:1:", dtype=np.uint8)
    out[start + 7] = lane + 48
    out[start + 8] = ord(":")
    _digits(out, start + 9, tile, 4)
    out[start + 13] = ord(":")
    p = start + 14
    for nd in (4, 5):
        m = xd == nd
        _digits(out, p[m], xs[m], nd)
    p = p + xd
    out[p] = ord(":")
    p = p + 1
    for nd in (4, 5, 6):
        m = yd == nd
        _digits(out, p[m], ys[m], nd)
    p = p + yd
    out[p] = 10
    rs = p + 1  # first base of each read
    boff = np.concatenate(([0], np.cumsum(lens)[:-1]))
    for L in np.unique(lens):
        m = lens == L
        ar = np.arange(L)
        out[rs[m][:, None] + ar] = bases[boff[m][:, None] + ar]
        out[(rs[m] + L + 3)[:, None] + ar] = qual[boff[m][:, None] + ar]
    out[rs + lens] = 10
    out[rs + lens + 1] = ord("+")
    out[rs + lens + 2] = 10
    out[rs + 2 * lens + 3] = 10
    return out.tobytes()


# Records are generated in blocks of FASTQ_BLOCK records; block b draws from
# the generator seeded with (seed, b) and holds records b*FASTQ_BLOCK onward,
# so blocks are independent and large inputs are made by a pool of threads
# while the bytes do not depend on the pool's size.
FASTQ_BLOCK = 16384


def _fastq_block(job):
    seed, b, read_lens = job
    return _fastq_batch(np.random.default_rng([seed, b]), b * FASTQ_BLOCK, FASTQ_BLOCK, read_lens)


def _pool_map(fn, jobs):
    """fn over jobs in a pool of at most 16 threads (the block generators are
    array operations, which run outside the interpreter lock)."""
    if len(jobs) <= 2:
        return [fn(j) for j in jobs]
    nw = min(16, os.cpu_count() or 1, len(jobs))
    with ThreadPoolExecutor(max_workers=nw) as ex:
        return list(ex.map(fn, jobs))


def _blocks_until(make_jobs, fn, target_bytes: int, est_block_bytes: float):
    """Blocks 0, 1, ... (made in parallel) until their total reaches target_bytes."""
    out, size, b = [], 0, 0
    while size < target_bytes:
        n = max(1, int((target_bytes - size) / est_block_bytes) + 1)
        parts = _pool_map(fn, make_jobs(b, b + n))
        for part in parts:
            if size >= target_bytes:
                break
            out.append(part)
            size += len(part)
            b += 1
    return out, size


def fastq_like(target_bytes: int, seed: int, read_lens=(150,)) -> bytes:
    """Whole FASTQ-like records until the size reaches ``target_bytes``."""
    read_lens = tuple(int(x) for x in read_lens)
    est = FASTQ_BLOCK * (31 + 2 * float(np.mean(read_lens)))
    parts, size = _blocks_until(lambda b0, b1: [(seed, b, read_lens) for b in range(b0, b1)], _fastq_block,
                                max(1, target_bytes), est)
    last = parts[-1]
    need = target_bytes - (size - len(last))
    # keep whole records only: stop at the first record end at or past the target
    cut = last.find(b"\n@SIM", max(0, need - 1))
    if cut >= 0:
        parts[-1] = last[: cut + 1]
    return b"".join(parts)


def _vocabulary(rng, n_words=50000):
    lens = rng.integers(2, 13, size=n_words)
    letters = rng.integers(ord("a"), ord("z") + 1, size=(n_words, 12), dtype=np.uint8)
    return letters, lens


WORD_BLOCK = 1 << 20  # tokens per block; block b draws from the generator seeded with (seed, b + 1)


def _line_ends(tl):
    """Greedy line breaking of tokens of lengths tl (separator excluded): a
    line takes tokens while it is shorter than 80 characters, and the token
    that brings it to 80 or more ends it with a newline.  Returns a mask of
    the tokens followed by a newline.  With C the prefix sums of the token
    lengths plus separators, the line that starts at token j ends before
    token nxt[j], the first m with C[m] >= C[j] + 81; the line starts are the
    chain 0, nxt[0], nxt[nxt[0]], ..., found by doubling (log2 rounds)."""
    n = tl.size
    C = np.concatenate(([0], np.cumsum(tl.astype(np.int64) + 1)))
    nxt = np.searchsorted(C, C[:n] + 81, side="left")  # in [j + 1, n + 1]
    jump = np.append(np.minimum(nxt, n), n)  # n: past the end (absorbing)
    starts = np.zeros(1, dtype=np.int64)
    while True:
        new = jump[starts]
        new = new[new < n]
        if new.size == 0:
            break
        starts = np.concatenate((starts, new))
        jump = jump[jump]
    ends = nxt[starts] - 1
    mask = np.zeros(n, dtype=bool)
    mask[ends[ends < n]] = True
    return mask


def _word_block(job):
    seed, b, n_words, s = job
    letters, wlens = _vocabulary(np.random.default_rng(seed), n_words)
    ranks = np.arange(1, n_words + 1, dtype=np.float64)
    p = ranks ** (-s)
    cdf = np.cumsum(p / p.sum())
    punct = np.frombuffer(b".,;:!?", dtype=np.uint8)
    rng = np.random.default_rng([seed, b + 1])
    n = WORD_BLOCK
    tok = np.minimum(np.searchsorted(cdf, rng.random(n), side="right"), n_words - 1)
    has_p = rng.random(n) < 0.05
    pch = punct[rng.integers(0, len(punct), size=n)]
    wl = wlens[tok]
    tl = wl + has_p  # token length without separator
    sep = np.where(_line_ends(tl), ord("\n"), ord(" ")).astype(np.uint8)
    full = tl + 1
    starts = np.concatenate(([0], np.cumsum(full)[:-1]))
    buf = np.empty(int(full.sum()), dtype=np.uint8)
    for j in range(12):
        m = wl > j
        buf[starts[m] + j] = letters[tok[m], j]
    buf[starts[has_p] + wl[has_p]] = pch[has_p]
    buf[starts + tl] = sep
    return buf.tobytes()


def word_stream(target_bytes: int, seed: int, n_words: int = 50000, s: float = 1.1) -> bytes:
    """Zipf word stream with punctuation and ~80-column lines (each block of
    WORD_BLOCK tokens starts a new line)."""
    parts, size = _blocks_until(lambda b0, b1: [(seed, b, n_words, s) for b in range(b0, b1)], _word_block,
                                max(1, target_bytes), 7.0 * WORD_BLOCK)
    last = parts[-1]
    need = target_bytes - (size - len(last))
    cut = last.find(b"\n", max(0, need - 1))
    if cut >= 0:
        parts[-1] = last[: cut + 1]
    return b"".join(parts)


def random_dna(n: int, seed: int) -> bytes:
    rng = np.random.default_rng(seed)
    return _ACGT[rng.integers(0, 4, size=n, dtype=np.uint8)].tobytes()


def dna_x_string(n: int, seed: int, dna: int = 150, xs: int = 300) -> bytes:
    """Repeats of `dna` random bases then `xs` 'x' characters, cut to n bytes
    (the FASTQ-like string of Section IV-D)."""
    rng = np.random.default_rng(seed)
    period = dna + xs
    reps = (n + period - 1) // period
    a = np.empty((reps, period), dtype=np.uint8)
    a[:, :dna] = _ACGT[rng.integers(0, 4, size=(reps, dna), dtype=np.uint8)]
    a[:, dna:] = ord("x")
    return a.reshape(-1)[:n].tobytes()


def binary_records(n: int, seed: int, noise_every: int = 8, noise_bytes: int = 96 << 10) -> bytes:
    """Binary data, cut to n bytes: 32-byte records (a little-endian uint32
    counter, four int16 random walks, a float32 ramp with noise, eight bytes
    of small flags), with a stretch of uniformly random bytes (compressed as
    stored blocks) after every `noise_every` stretches of 8192 records."""
    rng = np.random.default_rng(seed)
    rec_n = 8192
    parts, size, k = [], 0, 0
    while size < n:
        base = k * rec_n
        a = np.zeros((rec_n, 32), dtype=np.uint8)
        a[:, 0:4] = np.arange(base, base + rec_n, dtype="<u4").view(np.uint8).reshape(rec_n, 4)
        walk = np.cumsum(rng.integers(-3, 4, size=(rec_n, 4)), axis=0).astype("<i2")
        a[:, 4:12] = walk.view(np.uint8).reshape(rec_n, 8)
        ramp = (np.arange(base, base + rec_n) * 0.25 + rng.normal(0, 0.01, rec_n)).astype("<f4")
        a[:, 12:16] = ramp.view(np.uint8).reshape(rec_n, 4)
        a[:, 16:24] = rng.integers(0, 4, size=(rec_n, 8), dtype=np.uint8)
        parts.append(a.tobytes())
        size += a.size
        k += 1
        if k % noise_every == 0:
            parts.append(rng.integers(0, 256, size=noise_bytes, dtype=np.uint8).tobytes())
            size += noise_bytes
    return b"".join(parts)[:n]


def _deflate_segment(data: bytes, level: int, zdict: bytes | None, last: bool, strategy: int) -> bytes:
    if zdict:
        c = zlib.compressobj(level, zlib.DEFLATED, -15, 9, strategy, zdict=zdict)
    else:
        c = zlib.compressobj(level, zlib.DEFLATED, -15, 9, strategy)
    body = c.compress(data)
    body += c.flush(zlib.Z_FINISH if last else zlib.Z_SYNC_FLUSH)
    return body


def gzip_member(
    data: bytes,
    level: int = 6,
    segment_bytes: int = 64 << 20,
    threads: int | None = None,
    strategy: int = zlib.Z_DEFAULT_STRATEGY,
    mtime: int = 0,
) -> bytes:
    """One gzip member (RFC 1952) of ``data`` compressed by zlib."""
    return gzip_member_indexed(data, level, segment_bytes, threads, strategy, mtime)[0]


def gzip_member_indexed(
    data: bytes,
    level: int = 6,
    segment_bytes: int = 64 << 20,
    threads: int | None = None,
    strategy: int = zlib.Z_DEFAULT_STRATEGY,
    mtime: int = 0,
):
    """gzip_member, and the bit offset in the member where the first block of
    each compression segment begins (the encoder's own record: segment k > 0
    starts right after the sync flush that ends segment k - 1, so each offset
    is a block boundary of the member, and segment k's first output byte is
    data[k * segment_bytes])."""
    xfl = 2 if level == 9 else (4 if level == 1 else 0)
    header = b"\x1f\x8b\x08\x00" + struct.pack("<I", mtime) + bytes([xfl, 255])
    n = len(data)
    if n <= segment_bytes:
        parts = [_deflate_segment(data, level, None, True, strategy)]
    else:
        mv = memoryview(data)
        cuts = list(range(0, n, segment_bytes)) + [n]
        jobs = []
        for a, b in zip(cuts[:-1], cuts[1:]):
            zd = bytes(mv[max(0, a - 32768):a]) if a > 0 else None
            jobs.append((bytes(mv[a:b]), zd, b == n))
        nt = threads or min(16, os.cpu_count() or 1)
        with ThreadPoolExecutor(max_workers=nt) as ex:
            parts = list(ex.map(lambda j: _deflate_segment(j[0], level, j[1], j[2], strategy), jobs))
    seg_bits = []
    off = len(header)
    for p in parts:
        seg_bits.append(8 * off)
        off += len(p)
    trailer = struct.pack("<II", zlib.crc32(data) & 0xFFFFFFFF, n & 0xFFFFFFFF)
    return header + b"".join(parts) + trailer, seg_bits


def cache_dir() -> str:
    d = os.environ.get("GZGPU_CACHE", "/tmp/gzgpu_cache")
    os.makedirs(d, exist_ok=True)
    return d


# Named workloads: (generator, target bytes, seed, level, generator kwargs)
WORKLOADS = {
    "fastq_4MiB_L6": ("fastq", 4 << 20, 1, 6, {"read_lens": (150,)}),
    "fastq_1GiB_L6": ("fastq", 1 << 30, 2, 6, {"read_lens": (100, 150)}),
    "fastq_4GiB_L1": ("fastq", 4 << 30, 3, 1, {"read_lens": (100, 150)}),
    "fastq_4GiB_L9": ("fastq", 4 << 30, 3, 9, {"read_lens": (100, 150)}),
    "words_2GiB_L6": ("words", 2 << 30, 4, 6, {}),
}


def _gen(kind, size, seed, kw):
    if kind == "fastq":
        return fastq_like(size, seed, **kw)
    if kind == "words":
        return word_stream(size, seed, **kw)
    if kind == "dna":
        return random_dna(size, seed)
    if kind == "binary":
        return binary_records(size, seed)
    raise ValueError(kind)


SEGMENT_BYTES = 64 << 20  # input bytes per compression segment of large members
CACHE_MAX_BYTES = int(os.environ.get("GZGPU_CACHE_MAX", str(3 << 29)))
_RAW_MEMO: dict = {}  # the last generated text, kept for the next level of the same text


def make(kind: str, size: int, seed: int, level: int, use_cache: bool = True, index: bool = False, **kw):
    """Return (raw_text, gzip_bytes) for a generated workload, cached on disk;
    with index=True also the encoder's segment start bits (gzip_member_indexed)."""
    tag = f"{kind}_{size}_{seed}_{level}_" + "_".join(f"{k}{v}" for k, v in sorted(kw.items()))
    tag = tag.replace(" ", "").replace("(", "").replace(")", "").replace(",", "-")
    if use_cache:
        d = cache_dir()
        pr, pg, pi = (os.path.join(d, tag + e) for e in (".raw", ".gz", ".idx"))
        if os.path.exists(pr) and os.path.exists(pg) and os.path.exists(pi):
            with open(pr, "rb") as f:
                raw = f.read()
            with open(pg, "rb") as f:
                gz = f.read()
            with open(pi) as f:
                seg = [int(x) for x in f.read().split()]
            return (raw, gz, seg) if index else (raw, gz)
    key = (kind, size, seed, tuple(sorted(kw.items())))
    if _RAW_MEMO.get("key") == key:
        raw = _RAW_MEMO["raw"]  # the same text at another level (the level sweep)
    else:
        _RAW_MEMO.clear()
        raw = _gen(kind, size, seed, kw)
        _RAW_MEMO.update(key=key, raw=raw)
    gz, seg = gzip_member_indexed(raw, level, SEGMENT_BYTES)
    # inputs above the cache limit are made again rather than written out
    if use_cache and size <= CACHE_MAX_BYTES:
        for p, b in ((pr, raw), (pg, gz), (pi, " ".join(map(str, seg)).encode())):
            tmp = p + ".tmp%d" % os.getpid()
            with open(tmp, "wb") as f:
                f.write(b)
            os.replace(tmp, p)
    return (raw, gz, seg) if index else (raw, gz)


def workload(name: str, use_cache: bool = True, index: bool = False):
    kind, size, seed, level, kw = WORKLOADS[name]
    return make(kind, size, seed, level, use_cache=use_cache, index=index, **kw)


def bgzf_member(data: bytes, level: int = 6) -> bytes:
    """One BGZF-style gzip member (RFC 1952 with an FEXTRA field holding the
    'BC' subfield: the member's total size minus one)."""
    c = zlib.compressobj(level, zlib.DEFLATED, -15, 8)
    body = c.compress(data) + c.flush()
    total = 10 + 2 + 6 + len(body) + 8  # header, XLEN, the subfield, payload, trailer
    extra = b"BC" + struct.pack("<H", 2) + struct.pack("<H", total - 1)
    header = b"\x1f\x8b\x08\x04" + b"\x00\x00\x00\x00" + b"\x00\xff" + struct.pack("<H", len(extra)) + extra
    trailer = struct.pack("<II", zlib.crc32(data) & 0xFFFFFFFF, len(data) & 0xFFFFFFFF)
    return header + body + trailer


def bgzf(data: bytes, level: int = 6, block: int = 64 << 10, threads: int | None = None) -> bytes:
    """A BGZF-style file: members of `block` input bytes, then the empty member."""
    pieces = [data[i:i + block] for i in range(0, len(data), block)]
    nt = threads or min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=nt) as ex:
        members = list(ex.map(lambda x: bgzf_member(x, level), pieces))
    return b"".join(members) + bgzf_member(b"", level)
