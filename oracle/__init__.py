"""CPU oracle of the quasi-greedy many-clone dynamics -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
this package. The product path (the HIP library and its binding) never imports or calls it, and
this package imports nothing from the product package.

The arithmetic lives in ``qg_oracle.c`` (plain C, scalar, one int8 spin per site and clone);
this module compiles it with gcc and exposes it through ctypes with numpy arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle library in place (gcc, OpenMP over clones)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wextra",
               "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i32, u32, i64, u64 = ctypes.c_int32, ctypes.c_uint32, ctypes.c_int64, ctypes.c_uint64
    lib.or_philox4x32_10.argtypes = [P, P, P]
    lib.or_philox4x32_10.restype = None
    lib.or_initial_spin.argtypes = [u64, u32, i32, i64]
    lib.or_initial_spin.restype = ctypes.c_int8
    lib.or_draw16.argtypes = [u64, u32, i32, u32, i64]
    lib.or_draw16.restype = u32
    lib.or_energy.argtypes = [i32, P, P, P]
    lib.or_energy.restype = i32
    lib.or_colour.argtypes = [i32, P, i32, P, P]
    lib.or_colour.restype = i32
    lib.or_run.argtypes = [i32, P, P, P, u64, u32, u32, u32, i64, i64, u32, u32, P, P, P, P, i32]
    lib.or_run.restype = i32
    lib.or_trace.argtypes = [i32, P, P, P, u64, u32, u32, u32, i64, u32, u32, P, P, P, P]
    lib.or_trace.restype = i32
    _lib = lib
    return lib


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _tri(tri) -> np.ndarray:
    return np.ascontiguousarray(tri, dtype=np.int32).reshape(-1, 3)


def philox4x32_10(ctr, key) -> np.ndarray:
    """Philox4x32-10 bijection on one 128-bit counter and 64-bit key."""
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    _load().or_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def initial_spin(seed: int, instance_id: int, i: int, clone: int) -> int:
    return int(_load().or_initial_spin(seed, instance_id, i, clone))


def draw16(seed: int, instance_id: int, i: int, t: int, clone: int) -> int:
    return int(_load().or_draw16(seed, instance_id, i, t, clone))


def energy(tri, J, s) -> int:
    """E = -sum_t J_t s_a s_b s_c for one configuration s (+1/-1)."""
    tri = _tri(tri)
    J = np.ascontiguousarray(J, dtype=np.int8)
    s = np.ascontiguousarray(s, dtype=np.int8)
    return int(_load().or_energy(tri.shape[0], _ptr(tri), _ptr(J), _ptr(s)))


def colour(tri, cap: int = 32):
    """Greedy independent-set partition: (perm, class_off)."""
    tri = _tri(tri)
    n = tri.shape[0]
    perm = np.zeros(n, dtype=np.int32)
    off = np.zeros(n + 1, dtype=np.int32)
    k = _load().or_colour(n, _ptr(tri), cap, _ptr(perm), _ptr(off))
    if k < 0:
        raise ValueError("invalid instance")
    return perm, off[: k + 1].copy()


def run(tri, J, perm, *, seed: int, instance_id: int, thr: int, n_sweeps: int,
        clone_begin: int = 0, clone_count: int, start_sweep: int = 0, init_spins=None,
        want_final: bool = False, threads: int = 0, thr0: int = 0):
    """Run clones [clone_begin, clone_begin+clone_count) for n_sweeps sweeps (thr0 > 0: k = 0
    spins flip iff the draw is below thr0; then only the final configuration is tested).

    Returns dict(first_hit, energy[, final_spins]) as numpy arrays."""
    tri = _tri(tri)
    n = tri.shape[0]
    J = np.ascontiguousarray(J, dtype=np.int8)
    perm = np.ascontiguousarray(perm, dtype=np.int32)
    init = None
    if init_spins is not None:
        init = np.ascontiguousarray(init_spins, dtype=np.int8).reshape(clone_count, n)
    fh = np.zeros(clone_count, dtype=np.int32)
    en = np.zeros(clone_count, dtype=np.int32)
    fin = np.zeros((clone_count, n), dtype=np.int8) if want_final else None
    rc = _load().or_run(n, _ptr(tri), _ptr(J), _ptr(perm), seed & (2**64 - 1), instance_id,
                        thr, thr0, clone_begin, clone_count, start_sweep, n_sweeps, _ptr(init),
                        _ptr(fh), _ptr(en), _ptr(fin), threads)
    if rc != 0:
        raise ValueError("invalid instance")
    out = dict(first_hit=fh, energy=en)
    if want_final:
        out["final_spins"] = fin
    return out


def trace(tri, J, perm, spins, *, seed: int, instance_id: int, thr: int, clone: int,
          n_sweeps: int, start_sweep: int = 0, thr0: int = 0):
    """Single-clone trajectory: (final spins, k[n_sweeps][n], flip[n_sweeps][n], energies)."""
    tri = _tri(tri)
    n = tri.shape[0]
    J = np.ascontiguousarray(J, dtype=np.int8)
    perm = np.ascontiguousarray(perm, dtype=np.int32)
    s = np.array(spins, dtype=np.int8).copy()
    tk = np.zeros((n_sweeps, n), dtype=np.int8)
    tf = np.zeros((n_sweeps, n), dtype=np.int8)
    en = np.zeros(n_sweeps + 1, dtype=np.int32)
    rc = _load().or_trace(n, _ptr(tri), _ptr(J), _ptr(perm), seed & (2**64 - 1), instance_id,
                          thr, thr0, clone, start_sweep, n_sweeps, _ptr(s), _ptr(tk), _ptr(tf),
                          _ptr(en))
    if rc != 0:
        raise ValueError("invalid instance")
    return s, tk, tf, en


def initial_spins(n: int, *, seed: int, instance_id: int, clone_begin: int, clone_count: int):
    """[clone_count][n] initial spins drawn from the stream (slow, per element)."""
    lib = _load()
    out = np.zeros((clone_count, n), dtype=np.int8)
    for q in range(clone_count):
        for i in range(n):
            out[q, i] = lib.or_initial_spin(seed & (2**64 - 1), instance_id, i, clone_begin + q)
    return out


def solve_results(first_hit: np.ndarray):
    """Instance-level results from per-clone first hits: (tts, winner) with tts = min over
    clones (Section "Numerical results": the run's time is the shortest clone time) and the
    winner the lowest clone index attaining it; (-1, -1) if no clone hit."""
    fh = np.asarray(first_hit)
    hit = fh >= 0
    if not hit.any():
        return -1, -1
    tts = int(fh[hit].min())
    return tts, int(np.flatnonzero(fh == tts)[0])
