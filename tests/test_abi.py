"""CPU-side checks of the C ABI: the library loads, exports every declared function, validates
instances, and its host-side partition is the same greedy partition the oracle computes."""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import pytest
from hypothesis import given, settings
from hypothesis import strategies as st

import oracle
from paper_2102_09510_amd import xorsat
from paper_2102_09510_amd.instances import planted_instance

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(xorsat.LIB_PATH):
        from paper_2102_09510_amd import build
        build.build()
    return xorsat.load()


def declared_functions():
    text = open(os.path.join(ROOT, "include", "xorsat.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(xs_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 20
    assert sorted(xorsat.EXPORTS) == names
    for name in names:
        assert hasattr(lib, name), name
    assert lib.xs_abi_version() == 2
    assert lib.xs_status_str(1) == b"XS_EINVAL"


def test_header_constants_match_the_binding():
    text = open(os.path.join(ROOT, "include", "xorsat.h")).read()
    defs = {m.group(1): int(m.group(2), 0)
            for m in re.finditer(r"#define\s+(XS_[A-Z_]+)\s+(0x[0-9a-fA-F]+|\d+)u?\b", text)}
    for name in ("XS_STOP_ON_FIRST", "XS_RESUME", "XS_PLACE_ROWS", "XS_PER_CHUNK",
                 "XS_ONE_SWEEP_STEPS", "XS_MAX_N",
                 "XS_CLONE_QUANTUM", "XS_MAX_CLONES", "XS_TUNE_MAX_TRIALS",
                 "XS_NOALLOC_SCRATCH_BYTES"):
        assert defs[name] == getattr(xorsat, name), name
    for code, name in xorsat.XS_STATUS.items():
        assert defs[name] == code, name
    # The largest clone count is a whole number of quanta whose last index is below INT32_MAX.
    assert defs["XS_MAX_CLONES"] % defs["XS_CLONE_QUANTUM"] == 0
    assert defs["XS_MAX_CLONES"] - 1 < 2**31 - 1 < defs["XS_MAX_CLONES"] + defs["XS_CLONE_QUANTUM"]
    flags = [defs[k] for k in ("XS_STOP_ON_FIRST", "XS_RESUME", "XS_PLACE_ROWS", "XS_PER_CHUNK",
                               "XS_ONE_SWEEP_STEPS")]
    assert len(set(flags)) == 5 and all(f & (f - 1) == 0 for f in flags)
    cfg = xorsat.make_config(n_clones=256, seed=1, stop_on_first=False, place_rows=True)
    assert cfg.flags == xorsat.XS_PLACE_ROWS
    cfg = xorsat.make_config(n_clones=256, seed=1, stop_on_first=False, one_sweep_steps=True)
    assert cfg.flags == xorsat.XS_ONE_SWEEP_STEPS


def test_body_query_validation():
    """xs_instance_get_body: step caps outside [1, 65535] are XS_EINVAL; an instance whose
    schedule has no cross-sweep body for a cap gives XS_ENOTFOUND (None from the binding)."""
    import numpy as np
    from paper_2102_09510_amd.instances import planted_instance
    inst = planted_instance(20, 5120)
    h = xorsat.Instance(inst.tri, inst.J)
    lib = xorsat.load()
    buf = np.zeros(h.n + 1, dtype=np.int32)
    late = np.zeros(h.n, dtype=np.uint8)
    steps = ctypes.c_int32()
    for cap in (0, 65536):
        st = lib.xs_instance_get_body(h.handle, cap, buf.ctypes.data, buf.ctypes.data,
                                      late.ctypes.data, ctypes.byref(steps))
        assert st == xorsat.XS_STATUS_CODES["XS_EINVAL"], cap
    assert h.body(64) is None  # five colour classes: no shorter overlapped schedule
    big = planted_instance(1024, 5121)
    hb = xorsat.Instance(big.tri, big.J)
    order, off, lt = hb.body(64)
    assert sorted(order.tolist()) == list(range(1024)) and off[-1] == 1024
    assert len(off) - 1 < len(hb.schedule(64)[1]) - 1 and lt.max() == 1


def test_struct_layouts():
    assert ctypes.sizeof(xorsat.RunConfig) == 64  # 64 bytes of fields
    assert ctypes.sizeof(xorsat.RunBuffers) == 32
    assert ctypes.sizeof(xorsat.RunResult) == 56
    assert ctypes.sizeof(xorsat.InstanceInfo) == 24
    assert ctypes.sizeof(xorsat.ServerConfig) == 24
    assert ctypes.sizeof(xorsat.ServerOutputs) == 32
    assert ctypes.sizeof(xorsat.ServerCompletion) == 80
    assert ctypes.sizeof(xorsat.ServerStats) == 64
    assert ctypes.sizeof(xorsat.TuneResult) == 32 + 64 * 24  # trials: 4 x u32, double


@pytest.mark.parametrize("n,cap", [(10, 32), (10, 2), (64, 32), (256, 32), (1024, 32),
                                   (2048, 32), (200, 7), (100, 64)])
def test_partition_matches_oracle(lib, n, cap):
    inst = planted_instance(n, 77 + n) if n != 10 else planted_instance(10, 11)
    h = xorsat.Instance(inst.tri, inst.J, colour_cap=cap)
    perm, off = h.partition()
    operm, ooff = oracle.colour(inst.tri, cap)
    assert np.array_equal(perm, operm)
    assert np.array_equal(off, ooff)
    assert h.n_classes == len(ooff) - 1
    assert h.max_class == int(np.diff(ooff).max())
    # dependency levels of the update order: one level after the latest earlier spin that
    # shares a triplet
    pos = np.empty(n, dtype=np.int64)
    pos[operm] = np.arange(n)
    partners = [[] for _ in range(n)]
    for t in inst.tri.tolist():
        for v in t:
            partners[v] += [u for u in t if u != v]
    level = np.zeros(n, dtype=np.int64)
    for v in operm:
        level[v] = max((level[u] + 1 for u in partners[v] if pos[u] < pos[v]), default=0)
    sizes = np.bincount(level)
    assert h.n_levels == len(sizes) <= h.n_classes
    assert h.max_level == int(sizes.max())
    h.close()


def test_instance_validation(lib):
    inst = planted_instance(16, 3)
    tri, J = inst.tri.copy(), inst.J.copy()
    bad = []
    t = tri.copy(); t[0, 1] = t[0, 0]; bad.append((t, J, "repeats"))
    t = tri.copy(); t[0, 0] = 16; bad.append((t, J, "outside"))
    t = tri.copy(); t[0, 0] = (t[0, 0] + 1) % 16
    if len(set(t[0])) == 3:
        bad.append((t, J, "triplets, not 3"))
    j = J.copy(); j[3] = 0; bad.append((tri, j, "+1/-1"))
    for t, j, msg in bad:
        with pytest.raises(xorsat.XsError) as e:
            xorsat.Instance(t, j)
        assert e.value.status == 1 and msg in str(e.value)
    with pytest.raises(xorsat.XsError):
        xorsat.Instance(tri[:3], J[:3])
    big = planted_instance(2049, 1)
    with pytest.raises(xorsat.XsError):
        xorsat.Instance(big.tri, big.J)


def test_last_error_is_thread_local_message(lib):
    with pytest.raises(xorsat.XsError):
        xorsat.Instance(np.zeros((4, 3), dtype=np.int32), np.ones(4, dtype=np.int8))
    assert lib.xs_last_error().decode()


def test_tune_table_roundtrip(lib, tmp_path):
    """The tuned-knob table loads, rejects invalid rows and saves what it holds (no GPU)."""
    src = tmp_path / "tune.txt"
    src.write_text("# comment\n256 65536 64 4 256 16 2 40000.0\n1024 1048576 16 1 256 8 1 19000.5\n"
                   "64 1024 1 3 256 16 2 1.0\n64 1024 1 2 32 16 2 1.0\n64 1024 1 2 256 12 2 1.0\n"
                   "64 1024 1 2 256 16 3 1.0\nnot a row\n")
    xorsat.tune_clear()
    xorsat.tune_load(str(src))
    out = tmp_path / "out.txt"
    xorsat.tune_save(str(out))
    rows = [r.split() for r in out.read_text().splitlines() if not r.startswith("#")]
    assert rows == [["256", "65536", "64", "4", "256", "16", "2", "40000.0"],
                    ["1024", "1048576", "16", "1", "256", "8", "1", "19000.5"]]
    xorsat.tune_clear()
    xorsat.tune_save(str(out))
    assert [r for r in out.read_text().splitlines() if not r.startswith("#")] == []
    with pytest.raises(xorsat.XsError) as e:
        xorsat.tune_load(str(tmp_path / "missing.txt"))
    assert e.value.status == 5


@settings(max_examples=150, deadline=None)
@given(st.data())
def test_instance_create_fuzz(lib, data):
    """Random triplet lists (valid or not): creation either succeeds, and then the partition is
    the oracle's and the schedule covers every spin, or fails with XS_EINVAL; never anything
    else."""
    n = data.draw(st.integers(4, 40))
    m = data.draw(st.sampled_from([n, n, n, n - 1, n + 1]))
    tri = np.array(data.draw(st.lists(st.lists(st.integers(-1, n), min_size=3, max_size=3),
                                      min_size=max(m, 1), max_size=max(m, 1))),
                   dtype=np.int32).reshape(-1, 3)[:m]
    J = np.array(data.draw(st.lists(st.sampled_from([1, -1, 1, -1, 0]), min_size=m,
                                    max_size=m)), dtype=np.int8)
    cap = data.draw(st.integers(0, 40))
    try:
        h = xorsat.Instance(tri, J, colour_cap=cap)
    except xorsat.XsError as e:
        assert e.status == 1
        return
    # accepted: it must be a valid 3-regular instance
    assert m == n and set(np.unique(J)) <= {1, -1}
    assert np.all(np.bincount(tri.ravel(), minlength=n) == 3)
    perm, off = h.partition()
    operm, ooff = oracle.colour(tri, cap or 32)
    assert np.array_equal(perm, operm) and np.array_equal(off, ooff)
    order, soff = h.schedule(0)
    assert sorted(order.tolist()) == list(range(n)) and soff[-1] == n
    h.close()


@settings(max_examples=100, deadline=None)
@given(n=st.integers(4, 300), seed=st.integers(0, 10**6), cap=st.integers(0, 64),
       mutate=st.sampled_from(["none", "none", "index", "spin", "coupling"]),
       where=st.integers(0, 10**6))
def test_instance_create_mutations(lib, n, seed, cap, mutate, where):
    """Planted instances with at most one corrupted entry: valid ones are accepted with the
    oracle's partition, corrupted ones (a spin out of range or repeated, a coupling not +-1)
    are rejected with XS_EINVAL."""
    inst = planted_instance(n, seed)
    tri, J = inst.tri.copy(), inst.J.copy()
    t, q = where % n, (where // n) % 3
    if mutate == "index":
        tri[t, q] = n + where % 3
    elif mutate == "spin":
        tri[t, q] = tri[t, (q + 1) % 3]
    elif mutate == "coupling":
        J[t] = 0
    if mutate != "none":
        with pytest.raises(xorsat.XsError) as e:
            xorsat.Instance(tri, J, colour_cap=cap)
        assert e.value.status == 1
        return
    h = xorsat.Instance(tri, J, colour_cap=cap)
    perm, off = h.partition()
    operm, ooff = oracle.colour(tri, cap or 32)
    assert np.array_equal(perm, operm) and np.array_equal(off, ooff)
    h.close()


def test_batch_binding_rejects_empty_and_mismatched_lists():
    """The binding checks list lengths before any marshalling or device work."""
    with pytest.raises(ValueError):
        xorsat.run_batch([], [])
    with pytest.raises(ValueError):
        xorsat.run_batch([object()], [])
    with pytest.raises(ValueError):
        xorsat.run_batch_async([], [])
