"""Closed forms of the paper's compression model of random DNA (Section V),
for comparison with the undetermined share measured by random access.

Section V-A: with W positions of random DNA before it, a match of length k
exists at a position with probability p_k = 1 - (1 - 4^-k)^(W - k + 1).
Section V-C: under lazy (non-greedy) parsing a literal is emitted where the
longest match at a position is followed by a longer one at the next
position, p_l = sum over k >= 3 of p_k (1 - p_{k+1}) p_{k+1}; one position
in l_a + 1 is open for matching and lazy parsing adds one literal, so a
window of W characters holds E_l = p_l W / (l_a + 2) literals.  With L_1 =
E_l / W and every later window made of E_l new literals plus copies drawn
from the window before it, L_{i+1} = L_1 + (1 - L_1) L_i, so the share of
characters that are neither literals nor copies of literals after i windows
is 1 - L_i = (1 - L_1)^i (the "model" line of Fig. 2).
"""
from __future__ import annotations

WINDOW = 1 << 15  # DEFLATE's history, the W of the model


def match_probability(k: int, w: int = WINDOW) -> float:
    """p_k: a match of length k at a given position (Section V-A)."""
    return 1.0 - (1.0 - 4.0 ** -k) ** (w - k + 1)


def lazy_literal_probability(w: int = WINDOW, k_max: int = 64) -> float:
    """p_l: a literal emitted by lazy parsing at a given position (Section V-C);
    the terms past k_max are below double precision."""
    return sum(match_probability(k, w) * (1.0 - match_probability(k + 1, w)) * match_probability(k + 1, w)
               for k in range(3, k_max))


def lazy_literals(w: int = WINDOW, mean_match_len: float = 7.6) -> float:
    """E_l: literals per window of w characters (Section V-C)."""
    return lazy_literal_probability(w) * w / (mean_match_len + 2.0)


def undetermined_model(n_windows: int, l1: float) -> list:
    """1 - L_i for i = 1 .. n_windows, by the recurrence L_{i+1} = L_1 + (1 - L_1) L_i."""
    out, li = [], l1
    for _ in range(n_windows):
        out.append(1.0 - li)
        li = l1 + (1.0 - l1) * li
    return out
