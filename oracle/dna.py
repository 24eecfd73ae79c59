"""Oracle of the DNA-sequence extractor over partly undetermined text.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Appendix B of the paper: a decompressed block in which some characters are
still undetermined is searched for every maximal, non-overlapping substring
of the grammar  T D+ (U+ D+)* T,  where D is a nucleotide letter (A, C, G, T,
N), U an undetermined character and T a newline or an undetermined
character.  The two T's are dropped from each result; results shorter than a
minimum read length are discarded.  Section VI-B calls a block
sequence-resolved when the parser returns at least a threshold number of
sequences and none of them holds an undetermined character.

Readings (where the paper leaves the details open):
  - nucleotides are the upper-case letters A, C, G, T, N only;
  - the search is leftmost-first and, from a given start, as long as
    possible; the next search resumes after the closing T, so a newline that
    closes one sequence cannot open the next;
  - the minimum length filters the sequences found, it does not change the
    search;
  - a sequence belongs to the block (range of positions) holding its first
    nucleotide.

The input is either 16-bit symbols, where every value of 256 and above is
undetermined (the placeholders of Section VI-C), or bytes with one marker
value standing for undetermined (the random-access output of Section IV-B).
The grammar is matched by Python's regular-expression engine over a string
of character classes; nothing else is done.
"""
from __future__ import annotations

import re

import numpy as np

_GRAMMAR = re.compile(r"[LU]D+(?:U+D+)*[LU]")
NUCLEOTIDES = b"ACGTN"


def classes(buf, marker=None) -> str:
    """One class letter per element: D nucleotide, U undetermined, L newline,
    O anything else."""
    a = np.asarray(buf)
    if a.dtype == np.uint16:
        und = a >= 256
        byte = np.where(und, 0, a).astype(np.uint8)
    else:
        if marker is None:
            raise ValueError("a byte buffer needs the marker value")
        byte = a.astype(np.uint8)
        und = byte == marker
    cls = np.full(byte.size, ord("O"), np.uint8)
    cls[np.isin(byte, np.frombuffer(NUCLEOTIDES, np.uint8))] = ord("D")
    cls[byte == 0x0A] = ord("L")
    cls[und] = ord("U")
    return cls.tobytes().decode("ascii")


def extract(buf, marker=None, min_len: int = 1):
    """List of (start, length, undetermined count) of the sequences, in order;
    start is the position of the first nucleotide."""
    s = classes(buf, marker)
    out = []
    for m in _GRAMMAR.finditer(s):
        a, b = m.start() + 1, m.end() - 1
        if b - a >= min_len:
            out.append((a, b - a, s.count("U", a, b)))
    return out


def range_stats(seqs, bounds, threshold: int):
    """Per range [bounds[r], bounds[r+1]): (sequences, sequences holding an
    undetermined character, sequence-resolved flag)."""
    n = len(bounds) - 1
    cnt = np.zeros(n, np.int64)
    bad = np.zeros(n, np.int64)
    for a, _, u in seqs:
        r = int(np.searchsorted(bounds, a, side="right")) - 1
        if 0 <= r < n:
            cnt[r] += 1
            bad[r] += u > 0
    res = (cnt >= threshold) & (bad == 0)
    return np.stack([cnt, bad, res.astype(np.int64)], axis=1)
