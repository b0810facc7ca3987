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



def ground_law(n: int, tri: np.ndarray, J: np.ndarray, order, w1: float, w0: float,
               n_sweeps: int) -> np.ndarray:
    """Exact P(the configuration after t sweeps has E = -n), t = 0..n_sweeps, for one clone
    started uniformly at random.

    The clone's state is a Markov chain over the 2^n configurations: a sweep visits the spins in
    `order`; a spin with k unsatisfied triplets among its own flips with probability w0 (k = 0),
    w1 (k = 1) or 1 (k >= 2) (Section "The quasi-greedy algorithm"; w0 = 0 there, w0 > 0 the
    Metropolis-like variant). The law of the state is propagated over all configurations, one
    single-spin update at a time. With w0 = 0 a ground state has k = 0 at every spin and is never
    left, so the result is then also P(first hit <= t)."""
    assert n <= 14
    x = np.arange(1 << n, dtype=np.int64)
    ground = all_energies(n, tri, J) == -n
    # unsat[t] is 1 where triplet t is unsatisfied (x_a ^ x_b ^ x_c ^ j_t = 1).
    unsat = []
    for t in range(tri.shape[0]):
        a, b, c = (int(v) for v in tri[t])
        j = 1 if J[t] < 0 else 0
        unsat.append(((x >> a) ^ (x >> b) ^ (x >> c) ^ j) & 1)
    p_flip = []
    for i in range(n):
        k = np.zeros(1 << n, dtype=np.int64)
        for t in range(tri.shape[0]):
            k += unsat[t] * sum(1 for v in tri[t] if int(v) == i)
        p_flip.append(np.where(k == 0, w0, np.where(k == 1, w1, 1.0)))
    p = np.full(1 << n, 1.0 / (1 << n))
    out = np.zeros(n_sweeps + 1)
    out[0] = p[ground].sum()
    for t in range(1, n_sweeps + 1):
        for i in order:
            moved = p * p_flip[int(i)]
            p = p - moved + moved[x ^ (1 << int(i))]
        out[t] = p[ground].sum()
    return out


def group_tolerance(F, groups: int, z: float):
    """z standard deviations of a mean over `groups` independent 32-clone groups. A group's hit
    fraction lies in [0, 1] with mean F, so its variance is at most F (1 - F), whatever the
    correlation of the clones that share its draws."""
    F = np.asarray(F, dtype=np.float64)
    return z * np.sqrt(np.maximum(F * (1 - F), 1e-12) / groups)
