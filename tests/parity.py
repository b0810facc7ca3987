"""Helpers of the GPU <-> oracle parity tests: read clones out of the device state, replay
clones in the oracle from the same start, and compare per clone (first hit, end energy, end
spins). All integer, so the bar is exact equality."""
from __future__ import annotations

import numpy as np

import oracle


def spins_of_clones(state, clones) -> np.ndarray:
    """[len(clones)][n] spins (+1/-1) from a device tensor or host array of the state (bit
    c & 63 of word c >> 6)."""
    st = state.cpu().numpy() if hasattr(state, "cpu") else np.asarray(state)
    st = st.view(np.uint64)
    clones = np.asarray(clones, dtype=np.int64)
    bits = (st[:, clones >> 6] >> (clones & 63).astype(np.uint64)) & np.uint64(1)
    return (1 - 2 * bits.T.astype(np.int16)).astype(np.int8)


def pack_spins(spins: np.ndarray) -> np.ndarray:
    """[n_clones][n] spins (+1/-1) -> uint64 state [n][n_clones / 64] (bit 1 <=> s = -1)."""
    bits = np.ascontiguousarray((np.asarray(spins).T < 0).astype(np.uint8))
    assert bits.shape[1] % 64 == 0
    return np.ascontiguousarray(np.packbits(bits, axis=1, bitorder="little")).view(np.uint64)


def group_sample(n_clones: int, groups) -> np.ndarray:
    """All clones of the given 32-clone groups, ascending."""
    g = np.unique(np.asarray(groups, dtype=np.int64))
    assert g.min() >= 0 and g.max() < n_clones // 32
    return np.sort(np.concatenate([32 * x + np.arange(32) for x in g]))


def oracle_replay(tri, J, perm, *, seed, instance_id, thr, thr0, start_sweep, sweeps, clones,
                  init_spins=None):
    """The oracle run of the given clones (ascending) from the same start for `sweeps` sweeps."""
    res = {"first_hit": [], "energy": [], "final_spins": []}
    clones = np.asarray(clones)
    # contiguous runs of clones keep the oracle call count small
    starts = np.flatnonzero(np.diff(np.r_[-2, clones]) != 1)
    ends = np.r_[starts[1:], clones.size]
    for a, b in zip(starts, ends):
        init = None if init_spins is None else init_spins[a:b]
        r = oracle.run(tri, J, perm, seed=seed, instance_id=instance_id, thr=thr, thr0=thr0,
                       n_sweeps=sweeps, start_sweep=start_sweep, clone_begin=int(clones[a]),
                       clone_count=int(b - a), init_spins=init, want_final=True)
        for k in res:
            res[k].append(r[k])
    return {k: np.concatenate(v) for k, v in res.items()}


def check_clones(tri, J, perm, cfg, sweeps_done, clones, first_hit, energy, state,
                 init_spins=None, what=""):
    """Oracle replay of `clones` compared with the GPU's first_hit and energy arrays (indexed by
    clone) and its end state, element by element. Returns the oracle's results."""
    clones = np.asarray(clones)
    ref = oracle_replay(tri, J, perm, seed=cfg.seed, instance_id=cfg.instance_id,
                        thr=cfg.accept_thr, thr0=cfg.accept_thr0, start_sweep=cfg.start_sweep,
                        sweeps=sweeps_done, clones=clones, init_spins=init_spins)
    fh = np.asarray(first_hit)[clones]
    bad = np.flatnonzero(fh != ref["first_hit"])
    assert bad.size == 0, (f"{what}: first_hit differs at clones {clones[bad[:8]]}: "
                           f"gpu {fh[bad[:8]]} oracle {ref['first_hit'][bad[:8]]}")
    en = np.asarray(energy)[clones]
    bad = np.flatnonzero(en != ref["energy"])
    assert bad.size == 0, f"{what}: energy differs at clones {clones[bad[:8]]}"
    sp = spins_of_clones(state, clones)
    bad = np.flatnonzero((sp != ref["final_spins"]).any(axis=1))
    assert bad.size == 0, f"{what}: end spins differ at clones {clones[bad[:8]]}"
    return ref


def check_run_reduction(first_hit, tts, winner):
    """The run's TTS and winner are the reduction of its per-clone first hits (minimum, lowest
    clone index attaining it), as the oracle defines them."""
    assert (tts, winner) == oracle.solve_results(np.asarray(first_hit))
