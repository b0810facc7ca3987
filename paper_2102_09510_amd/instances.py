"""Seeded synthetic inputs: planted 3-XORSAT instances on a random 3-regular 3-uniform hypergraph.

This module only draws inputs. It holds none of the solver's arithmetic (no energy, no update
rule, no random stream of the dynamics) and it is shared by the oracle tests, the GPU tests and
the benchmark, so that both sides see the same instances.

Family (Section "The model and its energy landscape"): N spins, N triplets, the three indices of
a triplet distinct, every index in exactly three triplets. The challenge instances the paper runs
on are not available; planted instances of the same family stand in for them. A hidden solution
tau in {+1,-1}^N is drawn and J_t = tau_a tau_b tau_c, which is the gauge image of the paper's
ferromagnet (J = +1) under s -> tau * s, so the energy landscape is the same.

Generator: configuration model. The 3N stubs (each spin three times) are shuffled with a seeded
PCG64 stream and cut into N consecutive triplets; the whole draw is rejected if a triplet repeats
a spin or two triplets hold the same three spins. tau is drawn from the same stream after the
graph is accepted.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

# Default acceptance threshold for a spin in exactly one unsatisfied triplet: the paper fixes
# w1 = 0.055 (Section "Numerical results"); the dynamics compares a 16-bit draw d with thr and
# flips iff d < thr, so thr = floor(0.055 * 2^16) = 3604 (w1 = 0.054993).
W1_PAPER = 0.055
THR_PAPER = int(W1_PAPER * 65536)


@dataclass(frozen=True)
class Instance:
    n: int
    tri: np.ndarray  # int32 [n, 3], 0-based spin indices
    J: np.ndarray  # int8 [n], +1 / -1
    tau: np.ndarray  # int8 [n], the planted solution (+1 / -1)
    seed: int


def planted_instance(n: int, seed: int, max_tries: int = 100000) -> Instance:
    """Draw one planted instance with n spins from the seeded configuration model."""
    if n < 4:
        raise ValueError("a 3-regular 3-uniform hypergraph with distinct triplets needs n >= 4")
    rng = np.random.Generator(np.random.PCG64(seed))
    stubs = np.repeat(np.arange(n, dtype=np.int64), 3)
    for _ in range(max_tries):
        tri = rng.permutation(stubs).reshape(n, 3)
        s = np.sort(tri, axis=1)
        if np.any(s[:, 0] == s[:, 1]) or np.any(s[:, 1] == s[:, 2]):
            continue
        key = (s[:, 0] * n + s[:, 1]) * n + s[:, 2]
        if np.unique(key).size != n:
            continue
        break
    else:  # pragma: no cover - astronomically unlikely for n >= 4
        raise RuntimeError(f"no valid hypergraph after {max_tries} draws (n={n})")
    tau = (1 - 2 * rng.integers(0, 2, size=n)).astype(np.int8)
    J = (tau[tri[:, 0]] * tau[tri[:, 1]] * tau[tri[:, 2]]).astype(np.int8)
    return Instance(n=n, tri=np.ascontiguousarray(tri, dtype=np.int32), J=J, tau=tau, seed=seed)


def gen_seed(config: int, idx: int) -> int:
    """Instance seed for workload `config` (1-based) and instance index idx."""
    return 1_000_000 * config + idx


def run_seed(config: int, idx: int) -> int:
    """Seed of the dynamics' random stream for the same instance."""
    return gen_seed(config, idx) ^ 0xA5A5A5A5A5A5A5A5


# Workload recipes. Sizes follow the paper's setting (3-regular 3-uniform, M = N) at the
# sizes of the five measured workloads.
WORKLOADS = {
    1: dict(desc="1 planted instance, N=64, 1024 clones, to first ground state or 1e5 sweeps",
            count=1, n=64, clones=1024, max_sweeps=100000),
    2: dict(desc="64 planted instances, N=256, 65536 clones each, to first ground state",
            count=64, n=256, clones=65536, max_sweeps=None),
    3: dict(desc="16 planted instances, N=1024, 2^20 clones each, fixed 1e4 sweeps",
            count=16, n=1024, clones=1 << 20, max_sweeps=10000),
    4: dict(desc="512 planted instances, N in {32,...,1024}, 4096..65536 clones each",
            count=512, n=None, clones=None, max_sweeps=10000),
    5: dict(desc="Poisson stream at 200/s for 60 s, N log-uniform in [64,2048], 16384 clones",
            count=None, n=None, clones=16384, max_sweeps=10000),
}


def uneven_sizes(count: int = 512, seed: int = 4_000_000) -> list[tuple[int, int]]:
    """(N, clones) pairs of the uneven batch: N uniform on {32, 64, ..., 1024}, clones uniform on
    {4096, 8192, 16384, 32768, 65536}."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ns = 32 * rng.integers(1, 33, size=count)
    cl = 4096 << rng.integers(0, 5, size=count)
    return [(int(a), int(b)) for a, b in zip(ns, cl)]


def poisson_stream(rate: float = 200.0, duration: float = 60.0, seed: int = 5_000_000,
                   n_lo: int = 64, n_hi: int = 2048) -> list[tuple[float, int]]:
    """(arrival time in s, N) of the served stream: Poisson arrivals, N log-uniform."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        n = int(round(float(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi))))))
        out.append((t, max(n, 4)))
    return out
