"""Host checks of the LDS row placement (csrc/place.h), compiled with g++ into a small driver:
the row map and the re-ordered steps are permutations, slot orders keep every triplet's two
partners together, the search lowers the modelled conflict cycles, and it is deterministic."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2102_09510_amd import xorsat
from paper_2102_09510_amd.instances import planted_instance

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PLACE_H = os.path.join(ROOT, "paper_2102_09510_amd", "csrc", "place.h")

DRIVER = r"""
#include <cstdio>
#include "place.h"
using namespace xsh;
int main(int argc, char **argv) {
    int n, nst, B, CW, effort;
    if (scanf("%d %d %d %d %d", &n, &nst, &B, &CW, &effort) != 5) return 1;
    std::vector<int32_t> order(n), off(nst + 1), roles(7 * n);
    for (auto &v : order) if (scanf("%d", &v) != 1) return 1;
    for (auto &v : off) if (scanf("%d", &v) != 1) return 1;
    for (auto &v : roles) if (scanf("%d", &v) != 1) return 1;
    const RowModel m = row_model(B, CW);
    const Placement pl = place_rows(order, off, roles, n, m, effort);
    printf("%ld\n", placement_cost(pl, off, roles, m));
    for (int i = 0; i < n; ++i) printf("%d ", pl.row[i]);
    printf("\n");
    for (int i = 0; i < n; ++i) printf("%d ", pl.order[i]);
    printf("\n");
    for (int i = 0; i < n; ++i) printf("%d ", pl.slots[i]);
    printf("\n");
    for (int s = 0; s < kSlotOrders; ++s)
        for (int k = 0; k < 7; ++k) printf("%d ", slot_source(s, k));
    printf("\n");
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("place")
    src = d / "driver.cpp"
    src.write_text(DRIVER)
    exe = d / "driver"
    subprocess.run([gxx, "-O2", "-std=c++17", "-I", os.path.dirname(PLACE_H), str(src), "-o",
                    str(exe)], check=True)
    return str(exe)


def _roles(tri, n):
    """Own index, then the two other spins of each triplet (ascending triplet index)."""
    roles = np.zeros((n, 7), dtype=np.int64)
    roles[:, 0] = np.arange(n)
    fill = np.ones(n, dtype=np.int64)
    for t in range(len(tri)):
        a, b, c = (int(x) for x in tri[t])
        for v, (p, q) in ((a, (b, c)), (b, (a, c)), (c, (a, b))):
            roles[v, fill[v]] = p
            roles[v, fill[v] + 1] = q
            fill[v] += 2
    assert np.all(fill == 7)
    return roles


def _place(driver, order, off, roles, B, CW, effort):
    n = len(order)
    text = f"{n} {len(off) - 1} {B} {CW} {effort}\n" + " ".join(map(str, order)) + "\n" + \
        " ".join(map(str, off)) + "\n" + " ".join(map(str, roles.reshape(-1))) + "\n"
    out = subprocess.run([driver], input=text, capture_output=True, text=True, check=True)
    lines = out.stdout.split("\n")
    cost = int(lines[0])
    row, ordr, slots = (np.array(lines[i].split(), dtype=np.int64) for i in (1, 2, 3))
    src = np.array(lines[4].split(), dtype=np.int64).reshape(48, 7)
    return cost, row, ordr, slots, src


@pytest.mark.parametrize("n,cap,B,CW", [(1024, 64, 1, 8), (256, 64, 4, 16), (512, 64, 2, 16),
                                        (300, 64, 1, 8)])
def test_placement_is_a_valid_relabelling(driver, n, cap, B, CW):
    inst = planted_instance(n, 6100 + n)
    h = xorsat.Instance(inst.tri, inst.J)
    body = h.body(cap)
    order, off = (body[0], body[1]) if body is not None else h.schedule(cap)
    h.close()
    roles = _roles(np.asarray(inst.tri), n)
    base, row0, ord0, _, _ = _place(driver, order, off, roles, B, CW, 0)
    cost, row, ordr, slots, src = _place(driver, order, off, roles, B, CW, 200)
    # the row map and the steps are permutations; every step keeps its spins
    assert sorted(row.tolist()) == list(range(n)) and sorted(row0.tolist()) == list(range(n))
    for s in range(len(off) - 1):
        assert sorted(ordr[off[s]:off[s + 1]].tolist()) == sorted(order[off[s]:off[s + 1]].tolist())
    assert np.array_equal(ord0, order)  # effort 0 leaves the order
    # slot orders: role 0 stays the own row; the six partner slots are a permutation that
    # keeps each triplet's two spins in one slot pair
    assert src.shape == (48, 7) and len({tuple(r) for r in src}) == 48
    for r in src:
        assert r[0] == 0 and sorted(r[1:].tolist()) == [1, 2, 3, 4, 5, 6]
        for q in range(3):
            assert (r[1 + 2 * q] - 1) // 2 == (r[2 + 2 * q] - 1) // 2
    assert slots.min() >= 0 and slots.max() < 48
    # the search lowers the modelled conflict cycles, deterministically
    assert cost < base
    again = _place(driver, order, off, roles, B, CW, 200)
    assert again[0] == cost and np.array_equal(again[1], row) and np.array_equal(again[2], ordr)
    assert np.array_equal(again[3], slots)


def test_eight_block_rows_need_no_placement(driver):
    """256-byte rows span all banks: no groups, identity rows, order and slots unchanged."""
    n = 128
    inst = planted_instance(n, 6200)
    h = xorsat.Instance(inst.tri, inst.J)
    order, off = h.schedule(64)
    h.close()
    roles = _roles(np.asarray(inst.tri), n)
    cost, row, ordr, slots, _ = _place(driver, order, off, roles, 8, 16, 200)
    assert cost == 0 and np.array_equal(row, np.arange(n)) and np.array_equal(ordr, order)
    assert not slots.any()
