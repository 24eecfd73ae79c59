"""Pins of the DNA-sequence extractor's oracle (Appendix B, Section VI-B).

The oracle matches the grammar T D+ (U+ D+)* T with a regular expression.
It is checked against (1) a brute-force search written from the definition
(every substring tested by hand-written rules, leftmost start first, longest
from there, resumed after the match) on every short class string and on
random longer ones, and (2) FASTQ text built record by record, whose
sequence lines are known by construction, with undetermined characters put
into headers, quality lines and sequences at known places.
"""
import itertools

import numpy as np
import pytest

import synth
from oracle import dna

pytestmark = pytest.mark.filterwarnings("ignore")

CLS_BYTE = {"D": ord("A"), "U": 0, "L": 0x0A, "O": ord("x")}


def _brute(s: str):
    """Leftmost-longest non-overlapping substrings T D+ (U+ D+)* T of a class
    string, by testing every substring."""

    def is_seq(t):
        if len(t) < 3 or t[0] not in "LU" or t[-1] not in "LU":
            return False
        mid = t[1:-1]
        return mid[0] == "D" and mid[-1] == "D" and set(mid) <= {"D", "U"}

    out, pos, n = [], 0, len(s)
    while pos < n:
        hit = None
        for i in range(pos, n):
            ends = [j for j in range(i + 2, n) if is_seq(s[i:j + 1])]
            if ends:
                hit = (i, max(ends))
                break
        if hit is None:
            break
        i, j = hit
        out.append((i + 1, j - i - 1, s.count("U", i + 1, j)))
        pos = j + 1
    return out


def _bytes_of(s: str) -> np.ndarray:
    return np.array([CLS_BYTE[c] for c in s], np.uint8)


def test_classes_of_bytes_and_symbols():
    b = np.frombuffer(b"ACGTNacgtn\nx@", np.uint8)
    assert dna.classes(b, marker=ord("@")) == "DDDDDOOOOOLOU"
    s = np.array([65, 67, 256, 0x8000, 10, 120], np.uint16)
    assert dna.classes(s) == "DDUULO"


def test_every_short_string_equals_brute_force():
    for n in range(1, 8):
        for t in itertools.product("DULO", repeat=n):
            s = "".join(t)
            assert dna.extract(_bytes_of(s), marker=0) == _brute(s), s


def test_random_strings_equal_brute_force():
    rng = np.random.default_rng(11)
    for _ in range(1500):
        n = int(rng.integers(8, 22))
        s = "".join(rng.choice(list("DDDULO"), n))
        assert dna.extract(_bytes_of(s), marker=0) == _brute(s), s


def test_closing_newline_does_not_open_the_next():
    s = "LDLDLDL"  # \nA\nA\nA\n : the second line's newline closed the first
    assert _brute(s) == [(1, 1, 0), (5, 1, 0)]
    assert dna.extract(_bytes_of(s), marker=0) == _brute(s)


def _records(n, seed, read_len=150):
    """FASTQ records and the offsets of their sequence lines."""
    rng = np.random.default_rng(seed)
    parts, seqs, off = [], [], 0
    for k in range(n):
        head = b"@SIM:1:1:1101:%d:%d\n" % (rng.integers(1000, 30000), rng.integers(1000, 100000))
        seq = bytes(rng.choice(np.frombuffer(b"ACGT", np.uint8), read_len))
        if k % 7 == 3:
            seq = seq[:40] + b"N" + seq[41:]
        qual = bytes(np.clip(rng.normal(35, 5, read_len), 2, 41).astype(np.uint8) + 33)
        rec = head + seq + b"\n+\n" + qual + b"\n"
        seqs.append((off + len(head), read_len))
        parts.append(rec)
        off += len(rec)
    return b"".join(parts), seqs


def test_fastq_sequences_by_construction():
    text, seqs = _records(300, 3)
    got = dna.extract(np.frombuffer(text, np.uint8), marker=0)
    assert got == [(a, n, 0) for a, n in seqs]
    # the generator's records too: every second line of four
    raw = synth.fastq_like(200 << 10, 7)
    lines = raw.split(b"\n")
    starts = np.cumsum([0] + [len(x) + 1 for x in lines[:-1]])
    want = [(int(starts[i]), len(lines[i]), 0) for i in range(1, len(lines) - 1, 4)]
    assert dna.extract(np.frombuffer(raw, np.uint8), marker=0, min_len=30) == want


def test_fastq_with_undetermined_characters():
    """Undetermined headers and quality characters leave the sequences
    (min length 30) as they were; undetermined bases inside a sequence are
    counted; a sequence whose opening newline is undetermined is still
    found; as 16-bit symbols (placeholders 0x8000 + j) the result is the same."""
    text, seqs = _records(200, 5)
    a = np.frombuffer(text, np.uint8).astype(np.uint16)
    rng = np.random.default_rng(9)
    is_seq = np.zeros(a.size, bool)
    for s0, n in seqs:
        is_seq[s0:s0 + n] = True
    newline = a == 0x0A
    other = np.nonzero(~is_seq & ~newline)[0]
    und = np.zeros(a.size, bool)
    und[rng.choice(other, other.size // 3, replace=False)] = True
    inside = {}
    for k in (4, 50, 51, 120):
        s0, n = seqs[k]
        pos = s0 + 5 + rng.choice(n - 10, 3 + k % 3, replace=False)
        und[pos] = True
        inside[k] = pos.size
    s0, _ = seqs[77]
    und[s0 - 1] = True  # the newline before sequence 77
    sym = np.where(und, 0x8000 + rng.integers(0, 32768, a.size), a).astype(np.uint16)
    want = [(s0, n, inside.get(k, 0)) for k, (s0, n) in enumerate(seqs)]
    assert dna.extract(sym, min_len=30) == want
    as_bytes = np.where(und, 0, a).astype(np.uint8)
    assert dna.extract(as_bytes, marker=0, min_len=30) == want
    # without the length filter, quality fragments between undetermined
    # characters come out too, never overlapping a sequence
    loose = dna.extract(sym, min_len=1)
    assert set(want) <= set(loose) and len(loose) > len(want)


def test_range_stats():
    text, seqs = _records(40, 8)
    a = np.frombuffer(text, np.uint8).copy()
    s0, n = seqs[25]
    a[s0 + 10] = 0  # one undetermined base in sequence 25
    got = dna.extract(a, marker=0, min_len=30)
    bounds = np.array([0, seqs[10][0], seqs[20][0] + 3, seqs[30][0], a.size])
    st = dna.range_stats(got, bounds, threshold=5)
    # sequence 20 starts before its range's bound + 3, so it counts in range 1
    assert st.tolist() == [[10, 0, 1], [11, 0, 1], [9, 1, 0], [10, 0, 1]]
    assert dna.range_stats(got, bounds, threshold=11)[:, 2].tolist() == [0, 1, 0, 0]


def test_lazy_parsing_model_values():
    """Section V-C: E_l for W = 2^15 and l_a = 7.6 is printed as about 1283,
    i.e. about 4 % of W; the closed form 1 - L_i = (1 - L_1)^i holds for the
    recurrence; p_k agrees with the Poisson approximation of Section V-A and
    is one (to double precision) at k = 3."""
    from paper_1905_07224_amd import analytics as A

    e = A.lazy_literals()
    assert abs(e - 1283) < 0.03 * 1283          # 1257 here: the printed value rounds l_a + 2 to about 9.4
    assert abs(e / A.WINDOW - 0.04) < 0.003
    # p_k, and its Poisson approximation 1 - exp(-4^-k (W - k + 1)) of Section V-A
    import math
    for k in range(3, 24):
        approx = 1 - math.exp(-(4.0 ** -k) * (A.WINDOW - k + 1))
        assert abs(A.match_probability(k) - approx) <= 1e-4 * approx
    assert A.match_probability(3) == 1.0  # 1 - 10^-224, one to double precision
    m = A.undetermined_model(300, 0.04)
    assert np.allclose(m, [(1 - 0.04) ** i for i in range(1, 301)], rtol=1e-12)
    # a literal rate of zero (levels 1 to 3 after block 2) leaves everything undetermined
    assert A.undetermined_model(5, 0.0) == [1.0] * 5


@pytest.mark.parametrize("level,window", [(6, 3602), (9, 12755)])
def test_lazy_parsing_model_fits_oracle_profile(orc, level, window):
    """Fig. 2's model line against the oracle's undetermined share per
    window when random DNA (1 Mbp) is decoded from block 2: at level 6 with
    windows of o_a = 3602, and at level 9 with windows of o'_a = 12755
    (Section V-D), the model with L_1 = E_l / W stays within 0.1 of the
    measured share everywhere and within 0.04 in RMS over 150 windows."""
    from paper_1905_07224_amd import analytics as A

    raw = synth.random_dna(1_000_000, 2019)
    comp = synth.gzip_member(raw, level)
    g = orc.gunzip(comp)
    sr = orc.symbolic(comp, int(g.block_bit[1]), 1 << 62, first=False)
    und = sr.sym >= 0x8000
    n = min(150, und.size // window)
    frac = und[: n * window].reshape(n, window).mean(axis=1)
    model = np.array(A.undetermined_model(n, A.lazy_literals() / A.WINDOW))
    dev = frac - model
    assert np.abs(dev).max() < 0.1 and np.sqrt((dev ** 2).mean()) < 0.04
