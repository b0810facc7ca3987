"""Pins of the CPU oracle against facts fixed by the paper, the mathematics, published test
vectors and hand-worked examples. None of these tests uses a GPU or the HIP library."""
from __future__ import annotations

import math
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_2102_09510_amd.instances import THR_PAPER, planted_instance
from tests.pins import (all_energies, gf2_rank_and_consistent, ground_law, group_tolerance,
                        spins_of)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def n10(golden):
    g = golden("n10_instance.txt")
    tri = np.array([[int(v) for v in r[1:4]] for r in g["tri"]], dtype=np.int32)
    J = np.array([int(r[4]) for r in g["tri"]], dtype=np.int8)
    vec = {k: np.array([int(v) for v in g[k][0]]) for k in g if k not in ("tri", "n")}
    return tri, J, vec


# ------------------------------------------------------------------------- Philox4x32-10

def test_philox_known_answers():
    rows = []
    with open(os.path.join(ROOT, "tests", "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].split()
            if line:
                rows.append(line)
    assert len(rows) == 3
    for row in rows:
        vals = [int(v, 16) for v in row]
        ctr, key, want = vals[0:4], vals[4:6], vals[6:10]
        assert list(oracle.philox4x32_10(ctr, key)) == want


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_philox_matches_rocrand_host(tmp_path):
    """The oracle's bijection equals rocRAND's own Philox4x32-10 rounds (host build of the
    library header) on 200 seeded random (counter, key) pairs."""
    rng = np.random.default_rng(12345)
    cases = rng.integers(0, 2**32, size=(200, 6), dtype=np.uint64)
    src = tmp_path / "rr.cpp"
    src.write_text(
        "#include <rocrand/rocrand_philox4x32_10.h>\n#include <cstdio>\n"
        "struct P : rocrand_device::philox4x32_10_engine {\n"
        "  uint4 f(uint4 c, uint2 k) { return ten_rounds(c, k); } };\n"
        "int main() { P p; unsigned v[6];\n"
        "  while (scanf(\"%u %u %u %u %u %u\", v, v+1, v+2, v+3, v+4, v+5) == 6) {\n"
        "    uint4 c; c.x = v[0]; c.y = v[1]; c.z = v[2]; c.w = v[3];\n"
        "    uint2 k; k.x = v[4]; k.y = v[5]; uint4 r = p.f(c, k);\n"
        "    printf(\"%u %u %u %u\\n\", r.x, r.y, r.z, r.w); } }\n")
    exe = tmp_path / "rr"
    subprocess.run(["hipcc", "-O1", "-o", str(exe), str(src)], check=True,
                   capture_output=True)
    inp = "\n".join(" ".join(str(int(v)) for v in r) for r in cases)
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True)
    got = [list(map(int, line.split())) for line in out.stdout.strip().splitlines()]
    assert len(got) == len(cases)
    for r, g in zip(cases, got):
        assert list(oracle.philox4x32_10(r[:4], r[4:6])) == g


def test_draw16_layout_uses_all_halves():
    """Eight consecutive 32-clone groups of one site and sweep take the eight 16-bit halves of
    one Philox output, low half first."""
    seed, inst, i, t = 77, 5, 3, 9
    out = oracle.philox4x32_10([i, t, 2, inst], [seed & 0xFFFFFFFF, seed >> 32])
    halves = [(int(out[k // 2]) >> (16 * (k % 2))) & 0xFFFF for k in range(8)]
    got = [oracle.draw16(seed, inst, i, t, 32 * (16 + k) + 7) for k in range(8)]
    assert got == halves


# ------------------------------------------------------------------------- instances, Eq. (1)

@pytest.mark.parametrize("n,seed", [(4, 1), (10, 11), (64, 1000001), (256, 2000000),
                                    (1024, 3000000), (2048, 5)])
def test_generator_family(n, seed):
    """Section "The model and its energy landscape": N triplets, three distinct indices each,
    every index in exactly three triplets; no repeated triplet; the planted tau has E = -N."""
    inst = planted_instance(n, seed)
    tri = inst.tri
    assert tri.shape == (n, 3)
    assert np.all(np.bincount(tri.ravel(), minlength=n) == 3)
    s = np.sort(tri, axis=1)
    assert np.all(s[:, 0] < s[:, 1]) and np.all(s[:, 1] < s[:, 2])
    assert len({tuple(r) for r in s}) == n
    assert np.all(np.abs(inst.J) == 1)
    assert oracle.energy(tri, inst.J, inst.tau) == -n


@pytest.mark.parametrize("n,seed", [(8, 7), (10, 11), (12, 3), (14, 21), (16, 5)])
def test_energy_brute_force_and_gf2(n, seed):
    """Exhaustive enumeration: the minimum energy is -N and the number of ground states is
    2^(N - rank) from GF(2) elimination (footnote on linear equations mod 2). The oracle's
    product form agrees with the XOR count E = 2U - N on sampled configurations."""
    inst = planted_instance(n, seed)
    E = all_energies(n, inst.tri, inst.J)
    rank, consistent = gf2_rank_and_consistent(n, inst.tri, inst.J)
    assert consistent
    assert E.min() == -n
    assert int((E == -n).sum()) == 2 ** (n - rank)
    rng = np.random.default_rng(seed)
    for idx in rng.integers(0, 1 << n, size=64):
        assert oracle.energy(inst.tri, inst.J, spins_of(n, int(idx))) == E[idx]


def test_gf2_detects_unsatisfiable():
    """A full-rank system stays solvable after one coupling is flipped (its solution moves);
    a rank-deficient one can become inconsistent, and then exhaustive enumeration finds no
    configuration with E = -N, as GF(2) elimination predicts."""
    for seed in range(40):
        inst = planted_instance(12, seed)
        rank, _ = gf2_rank_and_consistent(12, inst.tri, inst.J)
        if rank == 12:
            break
    J = inst.J.copy()
    J[0] = -J[0]
    rank, consistent = gf2_rank_and_consistent(12, inst.tri, J)
    E = all_energies(12, inst.tri, J)
    assert rank == 12 and consistent  # full rank: still consistent, one unique solution moved
    assert E.min() == -12
    # A dependent system can be made inconsistent: find one.
    for seed in range(200):
        inst = planted_instance(12, seed)
        rank, _ = gf2_rank_and_consistent(12, inst.tri, inst.J)
        if rank < 12:
            break
    else:
        pytest.skip("no rank-deficient 12-spin instance among the seeds tried")
    for t in range(12):
        J = inst.J.copy()
        J[t] = -J[t]
        rank2, consistent = gf2_rank_and_consistent(12, inst.tri, J)
        if not consistent:
            assert all_energies(12, inst.tri, J).min() > -12
            return
    pytest.fail("no single coupling flip made the dependent system inconsistent")


# ------------------------------------------------------------------------- colouring

def test_colour_hand_worked(golden):
    tri, _, vec = n10(golden)
    perm, off = oracle.colour(tri, 32)
    assert perm.tolist() == vec["perm32"].tolist() and off.tolist() == vec["off32"].tolist()
    perm, off = oracle.colour(tri, 2)
    assert perm.tolist() == vec["perm2"].tolist() and off.tolist() == vec["off2"].tolist()


def _neighbours(n, tri):
    nb = [set() for _ in range(n)]
    for a, b, c in tri:
        for u, v in ((a, b), (a, c), (b, c)):
            nb[u].add(int(v))
            nb[v].add(int(u))
    return nb


@pytest.mark.parametrize("n,cap", [(64, 32), (256, 32), (1024, 32), (200, 7), (100, 64)])
def test_colour_is_the_greedy_partition(n, cap):
    """Every class is an independent set of at most `cap` sites, the classes partition the
    sites, and the partition is exactly what the repeated ascending scan produces: a site is
    missing from an earlier class only because that class was already full when the scan
    reached it or because it shares a triplet with a member added before it."""
    inst = planted_instance(n, n + cap)
    perm, off = oracle.colour(inst.tri, cap)
    nb = _neighbours(n, inst.tri)
    assert sorted(perm.tolist()) == list(range(n))
    cls = np.empty(n, dtype=np.int64)
    for k in range(len(off) - 1):
        members = perm[off[k]:off[k + 1]].tolist()
        assert 1 <= len(members) <= cap
        assert members == sorted(members)
        for q, u in enumerate(members):
            assert not (nb[u] & set(members[q + 1:]))
            cls[u] = k
    for v in range(n):
        for k in range(int(cls[v])):
            before = [u for u in perm[off[k]:off[k + 1]].tolist() if u < v]
            assert len(before) == cap or (nb[v] & set(before)), (v, k)


# ------------------------------------------------------------------------- the dynamics

def test_hand_worked_sweeps(golden):
    """One sweep at w1 = 0 and one at w1 = 1 from s = +1 match the hand derivation."""
    tri, J, vec = n10(golden)
    perm = vec["perm32"]
    for thr, tag in ((0, "greedy"), (65536, "all")):
        s, k, flip, en = oracle.trace(tri, J, perm, np.ones(10), seed=1, instance_id=0,
                                      thr=thr, clone=0, n_sweeps=1)
        assert k[0].tolist() == vec[f"{tag}_k"].tolist()
        assert flip[0].tolist() == vec[f"{tag}_flip"].tolist()
        assert s.tolist() == vec[f"{tag}_spins"].tolist()
        assert en.tolist() == [-2, int(vec[f"{tag}_energy"][0])]


@pytest.mark.parametrize("thr", [0, THR_PAPER, 20000, 65536])
def test_trace_invariants(thr):
    """Per update: w0 = 0 (k = 0 never flips), w2 = w3 = 1 (k >= 2 always flips), k = 1 flips
    iff the shared 16-bit draw is below thr. Per sweep: the energy computed from scratch moves
    by the sum of 6 - 4k over the flips (flipping a spin toggles its three triplets), which
    pins the k the rule sees."""
    inst = planted_instance(64, 99)
    perm, _ = oracle.colour(inst.tri, 32)
    clone, seed, iid, T = 517, 0xDEADBEEF12345, 3, 40
    s0 = np.array([oracle.initial_spin(seed, iid, i, clone) for i in range(64)])
    s, k, flip, en = oracle.trace(inst.tri, inst.J, perm, s0, seed=seed, instance_id=iid,
                                  thr=thr, clone=clone, n_sweeps=T)
    for t in range(T):
        assert np.all(flip[t][k[t] == 0] == 0)
        assert np.all(flip[t][k[t] >= 2] == 1)
        for pos in np.flatnonzero(k[t] == 1):
            d = oracle.draw16(seed, iid, int(perm[pos]), t, clone)
            assert flip[t][pos] == int(d < thr)
        dE = int(((6 - 4 * k[t].astype(int)) * flip[t]).sum())
        assert en[t + 1] - en[t] == dE
    if thr == 0:
        assert np.all(np.diff(en) <= 0)


def test_acceptance_frequency():
    """k = 1 updates flip with frequency thr / 2^16 (binomial, 5 sigma)."""
    inst = planted_instance(128, 4)
    perm, _ = oracle.colour(inst.tri, 32)
    seed, iid = 2024, 1
    n1 = f1 = 0
    for clone in range(0, 2048, 97):
        s0 = np.array([oracle.initial_spin(seed, iid, i, clone) for i in range(128)])
        _, k, flip, _ = oracle.trace(inst.tri, inst.J, perm, s0, seed=seed, instance_id=iid,
                                     thr=THR_PAPER, clone=clone, n_sweeps=60)
        n1 += int((k == 1).sum())
        f1 += int(flip[k == 1].sum())
    p = THR_PAPER / 65536
    assert n1 > 20000
    assert abs(f1 / n1 - p) < 5 * np.sqrt(p * (1 - p) / n1)


def test_initial_spins_uniform_and_grouped():
    """Initial bits: balanced, and one 32-bit Philox word per (site, 32-clone group)."""
    seed, iid = 31337, 2
    s = oracle.initial_spins(16, seed=seed, instance_id=iid, clone_begin=0, clone_count=512)
    assert abs(float((s == -1).mean()) - 0.5) < 0.03
    out = oracle.philox4x32_10([5, 0xFFFFFFFF, 1, iid], [seed & 0xFFFFFFFF, seed >> 32])
    for c in range(128, 256):
        bit = (int(out[(c >> 5) & 3]) >> (c & 31)) & 1
        assert s[c, 5] == (-1 if bit else 1)


def test_first_hit_and_absorbing():
    """first_hit is the first t whose configuration has E = -N; with w0 = 0 the ground state
    is never left (Section "The quasi-greedy algorithm", property (iii))."""
    inst = planted_instance(64, 1000001)
    perm, _ = oracle.colour(inst.tri, 32)
    seed, iid = 7, 0
    r = oracle.run(inst.tri, inst.J, perm, seed=seed, instance_id=iid, thr=THR_PAPER,
                   n_sweeps=400, clone_count=1024, want_final=True)
    fh = r["first_hit"]
    hits = np.flatnonzero(fh >= 0)
    assert hits.size > 0
    assert np.all(r["energy"][hits] == -64)
    for c in hits[:6]:
        s0 = np.array([oracle.initial_spin(seed, iid, i, int(c)) for i in range(64)])
        _, _, _, en = oracle.trace(inst.tri, inst.J, perm, s0, seed=seed, instance_id=iid,
                                   thr=THR_PAPER, clone=int(c), n_sweeps=400)
        assert en[fh[c]] == -64
        assert np.all(en[:fh[c]] > -64)
        assert np.all(en[fh[c]:] == -64)
    for c in np.flatnonzero(fh < 0)[:50]:
        assert r["energy"][c] > -64


def test_start_in_ground_state():
    """A clone that starts in a ground state has first_hit = start_sweep and never moves."""
    inst = planted_instance(64, 5)
    perm, _ = oracle.colour(inst.tri, 32)
    init = np.tile(inst.tau, (4, 1))
    r = oracle.run(inst.tri, inst.J, perm, seed=1, instance_id=0, thr=65536, n_sweeps=5,
                   clone_count=4, start_sweep=123, init_spins=init, want_final=True)
    assert r["first_hit"].tolist() == [123] * 4
    assert np.array_equal(r["final_spins"], init)
    r = oracle.run(inst.tri, inst.J, perm, seed=1, instance_id=0, thr=65536, n_sweeps=0,
                   clone_count=4, init_spins=init)
    assert r["first_hit"].tolist() == [0] * 4


def test_shuffle_within_classes_is_neutral():
    """Members of one class share no triplet, so their order inside the class does not change
    any trajectory (Supplementary Material: a set's nodes are updated in parallel)."""
    inst = planted_instance(96, 8)
    perm, off = oracle.colour(inst.tri, 32)
    rng = np.random.default_rng(0)
    perm2 = perm.copy()
    for k in range(len(off) - 1):
        rng.shuffle(perm2[off[k]:off[k + 1]])
    assert not np.array_equal(perm, perm2)
    kw = dict(seed=55, instance_id=4, thr=THR_PAPER, n_sweeps=150, clone_begin=256,
              clone_count=128, want_final=True)
    a = oracle.run(inst.tri, inst.J, perm, **kw)
    b = oracle.run(inst.tri, inst.J, perm2, **kw)
    for key in ("first_hit", "energy", "final_spins"):
        assert np.array_equal(a[key], b[key])


def test_gauge_invariance():
    """The planted instance is the image of the ferromagnet (J = +1, Eq. (1)) under
    s -> tau * s; the dynamics commutes with that map sweep by sweep, because k and the draws
    do not change."""
    inst = planted_instance(80, 12)
    perm, _ = oracle.colour(inst.tri, 32)
    ones = np.ones(80, dtype=np.int8)
    kw = dict(seed=9, instance_id=2, thr=THR_PAPER, n_sweeps=60, clone_count=64,
              want_final=True)
    init = oracle.initial_spins(80, seed=321, instance_id=0, clone_begin=0, clone_count=64)
    a = oracle.run(inst.tri, inst.J, perm, init_spins=init, **kw)
    b = oracle.run(inst.tri, ones, perm, init_spins=init * inst.tau[None, :], **kw)
    assert np.array_equal(a["final_spins"], b["final_spins"] * inst.tau[None, :])
    assert np.array_equal(a["energy"], b["energy"])
    assert np.array_equal(a["first_hit"], b["first_hit"])


def test_greedy_ignores_update_stream():
    """With w1 = 0 no random number is ever used after the start, so the update seed is
    irrelevant; with w1 > 0 it matters."""
    inst = planted_instance(64, 3)
    perm, _ = oracle.colour(inst.tri, 32)
    init = oracle.initial_spins(64, seed=5, instance_id=0, clone_begin=0, clone_count=32)
    kw = dict(instance_id=0, n_sweeps=30, clone_count=32, init_spins=init, want_final=True)
    a = oracle.run(inst.tri, inst.J, perm, seed=1, thr=0, **kw)
    b = oracle.run(inst.tri, inst.J, perm, seed=2, thr=0, **kw)
    assert np.array_equal(a["final_spins"], b["final_spins"])
    a = oracle.run(inst.tri, inst.J, perm, seed=1, thr=THR_PAPER, **kw)
    b = oracle.run(inst.tri, inst.J, perm, seed=2, thr=THR_PAPER, **kw)
    assert not np.array_equal(a["final_spins"], b["final_spins"])


def test_clone_ranges_compose():
    """Clones are independent: running a range equals the same clones inside a larger run."""
    inst = planted_instance(64, 21)
    perm, _ = oracle.colour(inst.tri, 32)
    kw = dict(seed=3, instance_id=7, thr=THR_PAPER, n_sweeps=50, want_final=True)
    full = oracle.run(inst.tri, inst.J, perm, clone_count=512, **kw)
    part = oracle.run(inst.tri, inst.J, perm, clone_begin=300, clone_count=70, **kw)
    assert np.array_equal(full["final_spins"][300:370], part["final_spins"])
    assert np.array_equal(full["first_hit"][300:370], part["first_hit"])


def test_resume_equals_uninterrupted():
    """Stopping after t sweeps and continuing from the exported spins at start_sweep = t gives
    the same final configuration as one run (the draws are keyed by the absolute sweep)."""
    inst = planted_instance(64, 22)
    perm, _ = oracle.colour(inst.tri, 32)
    kw = dict(seed=11, instance_id=1, thr=THR_PAPER, clone_count=64, want_final=True)
    full = oracle.run(inst.tri, inst.J, perm, n_sweeps=70, **kw)
    a = oracle.run(inst.tri, inst.J, perm, n_sweeps=30, **kw)
    b = oracle.run(inst.tri, inst.J, perm, n_sweeps=40, start_sweep=30,
                   init_spins=a["final_spins"], **kw)
    assert np.array_equal(full["final_spins"], b["final_spins"])


# ------------------------------------------------------------------------- Metropolis variant

def test_metropolis_rule_per_update():
    """With a second threshold thr0, a spin with k = 0 flips iff the same 16-bit draw is below
    thr0; the other rules are unchanged (Section "The quasi-greedy algorithm": w0 = w1^3 gives
    the Metropolis rule)."""
    inst = planted_instance(64, 199)
    perm, _ = oracle.colour(inst.tri, 32)
    clone, seed, iid, T = 77, 4321, 5, 30
    thr, thr0 = 8869, 4000
    s0 = np.array([oracle.initial_spin(seed, iid, i, clone) for i in range(64)])
    _, k, flip, en = oracle.trace(inst.tri, inst.J, perm, s0, seed=seed, instance_id=iid,
                                  thr=thr, thr0=thr0, clone=clone, n_sweeps=T)
    seen0 = 0
    for t in range(T):
        assert np.all(flip[t][k[t] >= 2] == 1)
        for pos in np.flatnonzero(k[t] <= 1):
            d = oracle.draw16(seed, iid, int(perm[pos]), t, clone)
            want = d < (thr if k[t][pos] == 1 else thr0)
            assert flip[t][pos] == int(want)
            seen0 += int(k[t][pos] == 0 and want)
        dE = int(((6 - 4 * k[t].astype(int)) * flip[t]).sum())
        assert en[t + 1] - en[t] == dE
    assert seen0 > 0


@pytest.mark.parametrize("T", [1.0, 0.8])
def test_metropolis_paramagnetic_energy(T):
    """w1 = exp(-2/T), w0 = w1^3 satisfies detailed balance for flips costing 6 - 4k; above the
    dynamical temperature the chain equilibrates in the paramagnet, whose energy per spin on a
    locally tree-like 3-regular hypergraph is -tanh(1/T) (cavity equations with u = h = 0,
    Section "Analytic prediction"). Thresholds are 16-bit roundings of w1 and w0."""
    beta = 1.0 / T
    thr = round(math.exp(-2 * beta) * 65536)
    thr0 = round(math.exp(-6 * beta) * 65536)
    inst = planted_instance(2048, 91)
    perm, _ = oracle.colour(inst.tri, 32)
    r = oracle.run(inst.tri, inst.J, perm, seed=17, instance_id=0, thr=thr, thr0=thr0,
                   n_sweeps=300, clone_count=256)
    e = r["energy"].mean() / 2048
    assert abs(e + math.tanh(beta)) < 0.006
    # the quasi-greedy rule at the same w1 never pays for a k = 0 flip and sits lower
    q = oracle.run(inst.tri, inst.J, perm, seed=17, instance_id=0, thr=thr, n_sweeps=300,
                   clone_count=64)
    assert q["energy"].mean() / 2048 < e - 0.003


def test_metropolis_first_hit_only_at_end():
    """With w0 > 0 only the final configuration is tested for E = -N."""
    inst = planted_instance(64, 5)
    perm, _ = oracle.colour(inst.tri, 32)
    init = np.tile(inst.tau, (4, 1))
    r = oracle.run(inst.tri, inst.J, perm, seed=1, instance_id=0, thr=3604, thr0=1,
                   n_sweeps=0, clone_count=4, start_sweep=9, init_spins=init)
    assert r["first_hit"].tolist() == [9] * 4
    r = oracle.run(inst.tri, inst.J, perm, seed=1, instance_id=0, thr=3604, thr0=30000,
                   n_sweeps=3, clone_count=4, init_spins=init)
    assert np.all((r["first_hit"] == 3) == (r["energy"] == -64))
    assert np.all(r["first_hit"][r["energy"] > -64] == -1)


@pytest.mark.parametrize("n,seed", [(8, 3), (10, 3), (12, 3)])
def test_first_hit_law_of_the_exact_chain(n, seed):
    """The distribution of first_hit over 131,072 clones equals the exact law of the sweep as a
    Markov chain over all 2^N configurations (Section "The quasi-greedy algorithm": k = 0 never
    flips, k = 1 with probability w1, k >= 2 always), computed without the oracle by propagating
    the law of the state. This pins the whole dynamics independently of the random stream:
    doubling or halving w1 or inverting the k = 1 test moves the exact law by 11 to 45 times the
    tolerance, and an off-by-one sweep in first_hit by 1.6 to 4.9 times (N = 12 to 10)."""
    inst = planted_instance(n, seed)
    perm, _ = oracle.colour(inst.tri, 32)
    T, clones = 300, 131072
    exact = ground_law(n, inst.tri, inst.J, perm, THR_PAPER / 65536, 0.0, T)
    fh = oracle.run(inst.tri, inst.J, perm, seed=11, instance_id=0, thr=THR_PAPER, n_sweeps=T,
                    clone_count=clones)["first_hit"]
    emp = np.cumsum(np.bincount(fh[fh >= 0], minlength=T + 1)) / clones
    assert np.all(np.abs(emp - exact) <= group_tolerance(exact, clones // 32, 5.5) + 1e-9)
    # Tighter than the worst case in practice: the clones of a group start independently.
    assert np.abs(emp - exact).max() < 0.015


@pytest.mark.parametrize("thr0", [3277, 13107])
def test_metropolis_end_state_law_of_the_exact_chain(thr0):
    """With w0 > 0 the share of clones whose configuration after T sweeps is a ground state
    (the only first_hit the rule records) equals the exact chain's P(E = -N after T sweeps).
    Halving w0 moves the exact values by 2.6 to 3.8 times the tolerance at some T, dropping it
    (the quasi-greedy rule) by up to 49 times."""
    n = 10
    inst = planted_instance(n, 3)
    perm, _ = oracle.colour(inst.tri, 32)
    clones = 1 << 20
    exact = ground_law(n, inst.tri, inst.J, perm, THR_PAPER / 65536, thr0 / 65536, 30)
    for T in (1, 3, 10, 30):
        r = oracle.run(inst.tri, inst.J, perm, seed=5, instance_id=0, thr=THR_PAPER, thr0=thr0,
                       n_sweeps=T, clone_count=clones)
        share = float(np.mean(r["first_hit"] == T))
        assert abs(share - exact[T]) <= group_tolerance(exact[T], clones // 32, 5.0), (T, share)



# ------------------------------------------------------------------ run-level results (TTS, winner)

@pytest.mark.parametrize("first_hit,expect", [
    # a run's time is its fastest clone (Section "Numerical results"); equal times resolve to
    # the lowest clone index
    ([5, 3, 7, 3, 3], (3, 1)),
    ([9, 9, 9, 9], (9, 0)),
    ([-1, -1, 4, -1, 4], (4, 2)),
    # no clone reached a ground state
    ([-1, -1, -1], (-1, -1)),
    ([-1], (-1, -1)),
    # a start configuration that is already a ground state is a hit at sweep 0
    ([-1, 0, 4, 0], (0, 1)),
    ([0], (0, 0)),
    # a resumed run starting at sweep 17: hits only at its first sweep
    ([-1, 17, -1, 17, 30], (17, 1)),
    # the last clone alone
    ([-1] * 1023 + [250], (250, 1023)),
])
def test_solve_results_hand_built(first_hit, expect):
    assert oracle.solve_results(np.array(first_hit, dtype=np.int32)) == expect


def test_solve_results_large_sweep_indices():
    """Sweep indices near the top of the int32 range and a winner far into the array."""
    fh = np.full(1 << 16, -1, dtype=np.int32)
    fh[40000] = 2_000_000_000
    fh[50000] = 1_999_999_999
    fh[60000] = 1_999_999_999
    assert oracle.solve_results(fh) == (1_999_999_999, 50000)
