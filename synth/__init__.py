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
    "make",
    "cache_dir",
]

_ACGT = np.frombuffer(b"ACGT", dtype=np.uint8)


def _fastq_batch(rng, k0, n, read_lens):
    lens = rng.choice(np.asarray(read_lens, dtype=np.int64), size=n)
    tot = int(lens.sum())
    bases = _ACGT[rng.integers(0, 4, size=tot, dtype=np.uint8)]
    nmask = rng.random(tot, dtype=np.float32) < 0.001
    bases[nmask] = ord("N")
    q = rng.standard_normal(tot, dtype=np.float32) * 5.0 + 35.0
    qual = (np.clip(np.rint(q), 2, 40) + 33).astype(np.uint8)
    xs = rng.integers(1000, 30001, size=n)
    ys = rng.integers(1000, 100001, size=n)
    bb = bases.tobytes()
    qb = qual.tobytes()
    parts = []
    pos = 0
    for j in range(n):
        k = k0 + j
        L = int(lens[j])
        lane = 1 + (k // 1000000) % 8
        tile = 1101 + (k // 10000) % 100
        parts.append(
            b"@SIM:1:%d:%d:%d:%d\n%s\n+\n%s\n"
            % (lane, tile, xs[j], ys[j], bb[pos:pos + L], qb[pos:pos + L])
        )
        pos += L
    return b"".join(parts)


def fastq_like(target_bytes: int, seed: int, read_lens=(150,)) -> bytes:
    """Whole FASTQ-like records until the size reaches ``target_bytes``."""
    rng = np.random.default_rng(seed)
    out = []
    size = 0
    k = 0
    mean_rec = 40 + 2 * float(np.mean(read_lens)) + 3
    while size < target_bytes:
        n = int(max(16, min(200000, (target_bytes - size) / mean_rec + 16)))
        b = _fastq_batch(rng, k, n, read_lens)
        k += n
        if size + len(b) >= target_bytes:
            # keep whole records only, stop at the first record end >= target
            need = target_bytes - size
            cut = b.find(b"\n@SIM", max(0, need - 1))
            if cut >= 0:
                b = b[: cut + 1]
        out.append(b)
        size += len(b)
    return b"".join(out)


def _vocabulary(rng, n_words=50000):
    lens = rng.integers(2, 13, size=n_words)
    letters = rng.integers(ord("a"), ord("z") + 1, size=(n_words, 12), dtype=np.uint8)
    return letters, lens


def word_stream(target_bytes: int, seed: int, n_words: int = 50000, s: float = 1.1) -> bytes:
    """Zipf word stream with punctuation and ~80-column lines."""
    rng = np.random.default_rng(seed)
    letters, wlens = _vocabulary(rng, n_words)
    ranks = np.arange(1, n_words + 1, dtype=np.float64)
    p = ranks ** (-s)
    cdf = np.cumsum(p / p.sum())
    punct = np.frombuffer(b".,;:!?", dtype=np.uint8)
    out = []
    size = 0
    line = 0
    while size < target_bytes:
        n = int(min(4_000_000, max(1024, (target_bytes - size) / 6 + 1024)))
        tok = np.searchsorted(cdf, rng.random(n), side="right")
        tok = np.minimum(tok, n_words - 1)
        has_p = rng.random(n) < 0.05
        pch = punct[rng.integers(0, len(punct), size=n)]
        tl = wlens[tok] + has_p  # token length without separator
        # greedy line breaking: newline after the token that brings the line to >= 80
        tl_list = tl.tolist()
        sep_nl = bytearray(n)
        for j, L in enumerate(tl_list):
            line += L
            if line >= 80:
                sep_nl[j] = 1
                line = 0
            else:
                line += 1
        sep = np.where(np.frombuffer(bytes(sep_nl), dtype=np.uint8) == 1, ord("\n"), ord(" ")).astype(np.uint8)
        full = tl + 1
        starts = np.concatenate(([0], np.cumsum(full)[:-1]))
        total = int(full.sum())
        buf = np.empty(total, dtype=np.uint8)
        wl = wlens[tok]
        for j in range(12):
            m = wl > j
            buf[starts[m] + j] = letters[tok[m], j]
        pm = has_p
        buf[starts[pm] + wl[pm]] = pch[pm]
        buf[starts + tl] = sep
        b = buf.tobytes()
        if size + len(b) >= target_bytes:
            need = target_bytes - size
            cut = b.find(b"\n", max(0, need - 1))
            if cut >= 0:
                b = b[: cut + 1]
        out.append(b)
        size += len(b)
    return b"".join(out)


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
    xfl = 2 if level == 9 else (4 if level == 1 else 0)
    header = b"\x1f\x8b\x08\x00" + struct.pack("<I", mtime) + bytes([xfl, 255])
    n = len(data)
    if n <= segment_bytes:
        body = _deflate_segment(data, level, None, True, strategy)
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
        body = b"".join(parts)
    trailer = struct.pack("<II", zlib.crc32(data) & 0xFFFFFFFF, n & 0xFFFFFFFF)
    return header + body + trailer


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
    raise ValueError(kind)


def make(kind: str, size: int, seed: int, level: int, use_cache: bool = True, **kw):
    """Return (raw_text, gzip_bytes) for a generated workload, cached on disk."""
    tag = f"{kind}_{size}_{seed}_{level}_" + "_".join(f"{k}{v}" for k, v in sorted(kw.items()))
    tag = tag.replace(" ", "").replace("(", "").replace(")", "").replace(",", "-")
    if use_cache:
        d = cache_dir()
        pr, pg = os.path.join(d, tag + ".raw"), os.path.join(d, tag + ".gz")
        if os.path.exists(pr) and os.path.exists(pg):
            with open(pr, "rb") as f:
                raw = f.read()
            with open(pg, "rb") as f:
                gz = f.read()
            return raw, gz
    raw = _gen(kind, size, seed, kw)
    gz = gzip_member(raw, level)
    if use_cache:
        for p, b in ((pr, raw), (pg, gz)):
            tmp = p + ".tmp%d" % os.getpid()
            with open(tmp, "wb") as f:
                f.write(b)
            os.replace(tmp, p)
    return raw, gz


def workload(name: str, use_cache: bool = True):
    kind, size, seed, level, kw = WORKLOADS[name]
    return make(kind, size, seed, level, use_cache=use_cache, **kw)


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
