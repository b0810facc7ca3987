"""The execution schedule the kernels use (the greedy update order regrouped into steps) is a
valid reordering of the sequential sweep: checked structurally on the library's schedule, and
dynamically by running the oracle in both orders (no GPU)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2102_09510_amd import xorsat
from paper_2102_09510_amd.instances import THR_PAPER, planted_instance


def _partners(tri, n):
    out = [set() for _ in range(n)]
    for t in np.asarray(tri).tolist():
        for v in t:
            out[v].update(u for u in t if u != v)
    return out


@pytest.mark.parametrize("n,cap", [(64, 32), (256, 32), (1024, 32), (2048, 32), (200, 7),
                                   (512, 64)])
@pytest.mark.parametrize("step_cap", [0, 16, 32, 64, 256])
def test_schedule_structure(n, cap, step_cap):
    """A permutation; every step an independent set of at most step_cap spins; every pair of
    spins sharing a triplet keeps its update-order precedence."""
    inst = planted_instance(n, 4100 + n)
    h = xorsat.Instance(inst.tri, inst.J, colour_cap=cap)
    perm, _ = h.partition()
    order, off = h.schedule(step_cap)
    assert sorted(order.tolist()) == list(range(n))
    assert off[0] == 0 and off[-1] == n and np.all(np.diff(off) > 0)
    if step_cap:
        assert np.diff(off).max() <= step_cap
    step = np.empty(n, dtype=np.int64)
    for s in range(len(off) - 1):
        step[order[off[s]:off[s + 1]]] = s
    pos = np.empty(n, dtype=np.int64)
    pos[perm] = np.arange(n)
    partners = _partners(inst.tri, n)
    for v in range(n):
        for u in partners[v]:
            assert step[u] != step[v]
            if pos[u] < pos[v]:
                assert step[u] < step[v]
    # inside a step the update order is kept
    for s in range(len(off) - 1):
        assert np.all(np.diff(pos[order[off[s]:off[s + 1]]]) > 0)
    if step_cap == 0:
        assert len(off) - 1 == h.n_levels <= h.n_classes
    h.close()


@pytest.mark.parametrize("n,cap,step_cap,sweeps", [(64, 32, 0, 300), (100, 5, 0, 200),
                                                   (200, 7, 16, 60), (256, 32, 64, 40),
                                                   (96, 64, 8, 100)])
def test_schedule_order_gives_the_same_trajectories(n, cap, step_cap, sweeps):
    """The oracle swept in the schedule's order reproduces the sweep in the greedy order bit for
    bit: final spins, energies and first hits of every clone."""
    inst = planted_instance(n, 5100 + n)
    h = xorsat.Instance(inst.tri, inst.J, colour_cap=cap)
    perm, _ = h.partition()
    order, _ = h.schedule(step_cap)
    assert not np.array_equal(order, perm) or n <= 64
    kw = dict(seed=77 + n, instance_id=3, thr=THR_PAPER, n_sweeps=sweeps, clone_count=512,
              want_final=True)
    a = oracle.run(inst.tri, inst.J, perm, **kw)
    b = oracle.run(inst.tri, inst.J, order, **kw)
    for k in ("first_hit", "energy", "final_spins"):
        assert np.array_equal(a[k], b[k]), k
    h.close()


def test_shuffled_order_changes_trajectories():
    """Control: an order that breaks the precedence of triplet-sharing spins gives different
    trajectories, so the equality above is not vacuous."""
    n = 100
    inst = planted_instance(n, 5200)
    h = xorsat.Instance(inst.tri, inst.J, colour_cap=5)
    perm, _ = h.partition()
    rev = perm[::-1].copy()
    kw = dict(seed=5, instance_id=0, thr=THR_PAPER, n_sweeps=50, clone_count=256,
              want_final=True)
    a = oracle.run(inst.tri, inst.J, perm, **kw)
    b = oracle.run(inst.tri, inst.J, rev, **kw)
    assert not np.array_equal(a["final_spins"], b["final_spins"])
    h.close()


@pytest.mark.parametrize("n,cap,step_cap,must", [(256, 32, 32, True), (512, 32, 64, True),
                                                 (1024, 32, 64, True), (2048, 32, 64, False),
                                                 (1024, 32, 96, False), (1024, 32, 128, False),
                                                 (2048, 32, 128, False), (544, 32, 64, False),
                                                 (640, 32, 64, False), (900, 32, 64, False),
                                                 (300, 7, 40, False),
                                                 (96, 32, 16, False)])
def test_body_replays_the_sequential_sweeps(n, cap, step_cap, must):
    """Symbolic replay of the cross-sweep body over a chunk of sweeps [3, 10): iterations 3 .. 10,
    each running its steps in order, a step's updates reading before any of them writes. Every
    update must read the version of each spin that the sequential sweeps give it (its own and
    its later partners' from the previous sweep, its earlier partners' from the current one),
    no two updates of a step may touch each other's spin, and every update runs exactly once.
    The body is also shorter than the plain schedule and within the step cap."""
    inst = planted_instance(n, 4300 + n)
    h = xorsat.Instance(inst.tri, inst.J, colour_cap=cap)
    body = h.body(step_cap)
    if body is None:
        assert not must, "the headline shapes have a body"
        h.close()
        return
    order, off, late = body
    ii = len(off) - 1
    perm, _ = h.partition()
    _, plain_off = h.schedule(step_cap)
    assert ii < len(plain_off) - 1
    assert sorted(order.tolist()) == list(range(n))
    assert np.diff(off).max() <= step_cap and set(np.unique(late)) <= {0, 1}
    pos = np.empty(n, dtype=np.int64)
    pos[perm] = np.arange(n)
    partners = _partners(inst.tri, n)
    t0, t1 = 3, 10
    ver = np.full(n, t0 - 1)
    runs = np.zeros(n, dtype=np.int64)
    for k in range(t0, t1 + 1):
        for s in range(ii):
            tasks = [(int(j), k - int(late[j])) for j in order[off[s]:off[s + 1]]
                     if t0 <= k - int(late[j]) < t1]
            spins = {j for j, _ in tasks}
            for j, t in tasks:
                assert ver[j] == t - 1, (j, t)
                for u in partners[j]:
                    assert u not in spins, (j, u)
                    assert ver[u] == (t if pos[u] < pos[j] else t - 1), (j, u, t)
            for j, t in tasks:
                ver[j] = t
                runs[j] += 1
    assert np.all(ver == t1 - 1) and np.all(runs == t1 - t0)
    h.close()
