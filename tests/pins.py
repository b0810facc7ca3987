"""Independent checks that pin the oracle: GF(2) elimination and exhaustive enumeration.

Footnote to Section "The model and its energy landscape": with s_i = (-1)^{x_i}, satisfying every
triplet is the linear system x_a + x_b + x_c = j_t (mod 2), j_t = 1 iff J_t = -1. Its solutions
are exactly the configurations with E = -N, so their number is 2^(N - rank) when the system is
consistent. Neither function here shares code with the oracle.
"""
from __future__ import annotations

import numpy as np


def gf2_rank_and_consistent(n: int, tri: np.ndarray, J: np.ndarray) -> tuple[int, bool]:
    """Rank of the triplet incidence matrix over GF(2) and whether the system is consistent.

    Rows are Python integers used as bitsets: bits 0..n-1 hold the coefficients, bit n the
    right-hand side."""
    rows = []
    for t in range(tri.shape[0]):
        r = 0
        for v in tri[t]:
            r ^= 1 << int(v)
        if J[t] < 0:
            r |= 1 << n
        rows.append(r)
    rank = 0
    for col in range(n):
        bit = 1 << col
        piv = next((k for k in range(rank, len(rows)) if rows[k] & bit), None)
        if piv is None:
            continue
        rows[rank], rows[piv] = rows[piv], rows[rank]
        for k in range(len(rows)):
            if k != rank and rows[k] & bit:
                rows[k] ^= rows[rank]
        rank += 1
    consistent = all(r != (1 << n) for r in rows[rank:])
    return rank, consistent


def all_energies(n: int, tri: np.ndarray, J: np.ndarray) -> np.ndarray:
    """E = 2U - N for all 2^n configurations; configuration index bit i = x_i (x = 1 <=> s = -1).

    U counts triplets with x_a xor x_b xor x_c xor j_t = 1."""
    assert n <= 22
    x = np.arange(1 << n, dtype=np.int64)
    U = np.zeros(1 << n, dtype=np.int32)
    for t in range(tri.shape[0]):
        a, b, c = (int(v) for v in tri[t])
        j = 1 if J[t] < 0 else 0
        U += (((x >> a) ^ (x >> b) ^ (x >> c) ^ j) & 1).astype(np.int32)
    return 2 * U - n


def spins_of(n: int, idx: int) -> np.ndarray:
    """+1/-1 spins of configuration index idx (bit i set <=> s_i = -1)."""
    return np.array([-1 if (idx >> i) & 1 else 1 for i in range(n)], dtype=np.int8)
