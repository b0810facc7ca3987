"""GPU <-> oracle parity through the C ABI: bit-exact per clone (first hit, energy at the end
sweep, final spins) and per run (TTS, winner, solved configuration). All integer, so the bar is
exact equality."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2102_09510_amd import xorsat
from paper_2102_09510_amd.instances import THR_PAPER, planted_instance
from tests.parity import check_clones
from tests.pins import ground_law, group_tolerance

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def assert_parity(inst, h, cfg, out, clones=None, init_spins=None):
    """Every given clone (default: all) against the oracle from the same start to the GPU's end
    sweep, after checking that the library's partition is the oracle's."""
    perm, _ = h.partition()
    operm, _ = oracle.colour(inst.tri, h.colour_cap)
    assert np.array_equal(perm, operm)
    if clones is None:
        clones = np.arange(cfg.n_clones)
    return check_clones(inst.tri, inst.J, operm, cfg, out.sweeps_done, clones,
                        out.first_hit.cpu().numpy(), out.energy.cpu().numpy(), out.state,
                        init_spins)


def run_and_check_full(n, seed, n_clones, *, max_sweeps, stop=True, chunk=0, tile_blocks=0,
                       thr=THR_PAPER, cap=32, iid=3, place=False):
    _torch()
    inst = planted_instance(n, seed)
    h = xorsat.Instance(inst.tri, inst.J, colour_cap=cap)
    cfg = xorsat.make_config(n_clones=n_clones, seed=seed * 7 + 1, instance_id=iid,
                             accept_thr=thr, max_sweeps=max_sweeps, stop_on_first=stop,
                             chunk_sweeps=chunk, tile_blocks=tile_blocks, place_rows=place)
    out = xorsat.run(h, cfg)
    ref = assert_parity(inst, h, cfg, out)
    tts, winner = oracle.solve_results(ref["first_hit"])
    assert out.tts_sweeps == tts and out.winner_clone == winner
    if winner >= 0:
        assert np.array_equal(out.solved, ref["final_spins"][winner])
        assert oracle.energy(inst.tri, inst.J, out.solved) == -n
    return inst, h, cfg, out


def test_small_instance_full_parity_to_first_ground_state():
    """N = 64, 1024 clones, stop at the first ground state (the single-instance workload):
    every clone, every output, TTS and winner."""
    inst, h, cfg, out = run_and_check_full(64, 1000001, 1024, max_sweeps=100000)
    assert out.tts_sweeps >= 0
    assert out.end_sweep % 100 == 0 or out.end_sweep == 100000


def test_first_ground_state_with_placed_rows():
    """The same run with the LDS rows placed (one-block tiles: eight rows per LDS cycle),
    through the end-of-chunk check and the replay."""
    inst, h, cfg, out = run_and_check_full(64, 1000001, 1024, max_sweeps=100000, place=True)
    assert out.tile_blocks < 8 and out.tts_sweeps >= 0


@pytest.mark.parametrize("n,clones,B,chunk,sweeps,place", [
    (100, 4096, 2, 7, 40, False),  # ragged classes, 8 tiles, chunk does not divide the budget
    (100, 4096, 2, 7, 40, True),   # the same with LDS rows placed
    (37, 2048, 0, 0, 33, True),    # odd N, auto tiling, single chunk
    (257, 1024, 1, 5, 23, False),  # N just above 256, one-block tiles
    (257, 1024, 1, 5, 23, True),
    (4, 256, 1, 1, 9, True),       # smallest instance and clone count (too small to place)
    (64, 8192, 32, 10, 30, False),  # largest tile: 32 blocks, n * B = 2048 (1,024-byte rows)
    (50, 768, 0, 9, 20, True),      # three 256-clone blocks: one-block tiles, ragged batch
])
def test_budget_runs_every_clone(n, clones, B, chunk, sweeps, place):
    run_and_check_full(n, 500 + n, clones, max_sweeps=sweeps, stop=False, chunk=chunk,
                       tile_blocks=B, place=place)


def test_ferromagnet_instance():
    """The paper's own model, J = +1 on every triplet (its ground state is all spins up): every
    clone matches the oracle, and the solved configuration is a ground state."""
    import types

    _torch()
    base = planted_instance(120, 31)
    inst = types.SimpleNamespace(tri=base.tri, J=np.ones(120, np.int8))
    h = xorsat.Instance(inst.tri, inst.J)
    cfg = xorsat.make_config(n_clones=4096, seed=123, instance_id=4, max_sweeps=20000,
                             chunk_sweeps=50)
    out = xorsat.run(h, cfg)
    assert_parity(inst, h, cfg, out)
    if out.winner_clone >= 0:
        assert oracle.energy(inst.tri, inst.J, out.solved) == -120


@pytest.mark.parametrize("jdup", [1, -1])
def test_repeated_triplet_instance(jdup):
    """An instance with a repeated triplet (each copy counted, as in the energy) and triplets
    sharing two spins: every clone matches the oracle. With opposite couplings on the two copies
    one of them is always unsatisfied, so no clone can reach E = -N and the run ends at its
    budget unsolved."""
    import types

    tri = np.array([[0, 1, 2], [0, 1, 2], [0, 3, 4], [1, 3, 5], [2, 4, 5], [3, 4, 5]], np.int32)
    J = np.array([1, jdup, -1, 1, -1, 1], np.int8)
    inst = types.SimpleNamespace(tri=tri, J=J)
    _torch()
    h = xorsat.Instance(tri, J)
    cfg = xorsat.make_config(n_clones=2048, seed=77, instance_id=9, accept_thr=THR_PAPER,
                             max_sweeps=60, stop_on_first=False, chunk_sweeps=7)
    out = xorsat.run(h, cfg)
    ref = assert_parity(inst, h, cfg, out)
    if jdup == -1:
        assert np.all(ref["first_hit"] == -1) and out.tts_sweeps == -1
        assert out.energy.min().item() > -6


@pytest.mark.parametrize("thr", [0, 65536])
def test_deterministic_rules(thr):
    """w1 = 0 (greedy) and w1 = 1 (every spin with k >= 1 flips)."""
    run_and_check_full(128, 61, 2048, max_sweeps=30, stop=False, thr=thr)


def test_colour_cap_variants():
    run_and_check_full(96, 62, 1024, max_sweeps=25, stop=False, cap=5)
    run_and_check_full(96, 62, 1024, max_sweeps=25, stop=False, cap=64)


def test_tiling_is_result_neutral():
    """tile_blocks only moves work between workgroups; every output is identical."""
    torch = _torch()
    inst = planted_instance(128, 9)
    h = xorsat.Instance(inst.tri, inst.J)
    outs = []
    shapes = ((1, 0, 0, 0), (2, 0, 0, 0), (4, 0, 0, 0), (8, 0, 0, 0), (16, 0, 0, 0),
              (1, 64, 16, 2), (2, 128, 16, 1), (4, 1024, 16, 2), (8, 256, 16, 1),
              (16, 256, 16, 2), (1, 256, 4, 1), (1, 64, 8, 2), (2, 256, 4, 1),
              (4, 256, 8, 1), (16, 128, 4, 1), (8, 512, 8, 2))
    # tiles under eight blocks again with their LDS rows placed
    for (B, T, C, G), place in [(s, False) for s in shapes] + [(s, True) for s in shapes
                                                               if s[0] < 8]:
        cfg = xorsat.make_config(n_clones=8192, seed=99, instance_id=1, max_sweeps=300,
                                 stop_on_first=False, tile_blocks=B, chunk_sweeps=64,
                                 wg_threads=T, col_bytes=C, rec_global=G, place_rows=place)
        out = xorsat.run(h, cfg)
        if G:
            assert out.rec_global == (G == 1)
        assert out.tile_blocks == B and out.wg_threads == (T or out.wg_threads)
        assert out.col_bytes == (C or out.col_bytes)
        outs.append(out)
    for o in outs[1:]:
        assert torch.equal(o.state, outs[0].state)
        assert torch.equal(o.first_hit, outs[0].first_hit)
        assert torch.equal(o.energy, outs[0].energy)
        assert o.tts_sweeps == outs[0].tts_sweeps and o.winner_clone == outs[0].winner_clone


def test_chunk_length_changes_only_end_sweep():
    """TTS, winner, solved configuration and each clone's hit up to the TTS do not depend on
    the chunk length; the end sweep (and so later state) may."""
    _torch()
    inst = planted_instance(64, 1000001)
    h = xorsat.Instance(inst.tri, inst.J)
    res = []
    for K in (1, 13, 100, 1000):
        cfg = xorsat.make_config(n_clones=1024, seed=5, instance_id=0, chunk_sweeps=K,
                                 max_sweeps=100000)
        res.append(xorsat.run(h, cfg))
    for o in res[1:]:
        assert o.tts_sweeps == res[0].tts_sweeps and o.winner_clone == res[0].winner_clone
        assert np.array_equal(o.solved, res[0].solved)
        assert o.end_sweep >= o.tts_sweeps
    assert res[0].end_sweep == res[0].tts_sweeps + 1 or res[0].end_sweep == res[0].tts_sweeps


def test_graph_replay_equals_eager_launches():
    """The launch-per-chunk loop (XS_PER_CHUNK): untimed runs replay it from a captured hipGraph
    (groups of up to 64 chunks, replayed many times with host synchronisations between
    replays); timed runs launch every chunk eagerly. Both give the same outputs, in a budget run
    and in a stop-on-first batch."""
    torch = _torch()
    inst = planted_instance(64, 4242)
    h = xorsat.Instance(inst.tri, inst.J)
    insts = [planted_instance(n, 4300 + n) for n in (40, 72, 96)]
    hs = [xorsat.Instance(i.tri, i.J) for i in insts]
    budget = xorsat.make_config(n_clones=4096, seed=5, instance_id=2, max_sweeps=12000,
                                stop_on_first=False, chunk_sweeps=25, per_chunk=True)
    batch = [xorsat.make_config(n_clones=2048, seed=11 + k, instance_id=k, max_sweeps=60000,
                                chunk_sweeps=10, per_chunk=True) for k in range(3)]
    outs = {}
    for timed in (False, True):
        xorsat.profile_enable(timed)
        try:
            outs[timed] = [xorsat.run(h, budget)] + xorsat.run_batch(hs, batch)
        finally:
            xorsat.profile_enable(False)
    xorsat.profile_read(reset=True)  # leave no timing totals to later tests
    for a, b in zip(outs[False], outs[True]):
        assert (a.persistent, b.persistent) == (0, 0)
        assert torch.equal(a.state, b.state)
        assert torch.equal(a.first_hit, b.first_hit)
        assert torch.equal(a.energy, b.energy)
        assert (a.tts_sweeps, a.winner_clone, a.end_sweep) == (b.tts_sweeps, b.winner_clone,
                                                               b.end_sweep)
    assert outs[False][0].end_sweep == 12000
    assert_parity(inst, h, budget, outs[False][0], clones=np.r_[0:32, 4064:4096])


def test_batch_equals_single_runs():
    """Uneven instances in one batched run give bit-identical results to one run each."""
    torch = _torch()
    sizes = [(48, 512), (64, 1024), (200, 2048), (33, 256), (512, 1024)]
    insts, hs, cfgs = [], [], []
    for k, (n, nc) in enumerate(sizes):
        inst = planted_instance(n, 300 + k)
        insts.append(inst)
        hs.append(xorsat.Instance(inst.tri, inst.J))
        cfgs.append(xorsat.make_config(n_clones=nc, seed=1000 + k, instance_id=k,
                                       max_sweeps=400 if n < 100 else 60,
                                       stop_on_first=n < 100, chunk_sweeps=20))
    batch = xorsat.run_batch(hs, cfgs)
    for k in range(len(sizes)):
        single = xorsat.run(hs[k], cfgs[k])
        b = batch[k]
        assert torch.equal(b.state, single.state)
        assert torch.equal(b.first_hit, single.first_hit)
        assert torch.equal(b.energy, single.energy)
        assert (b.tts_sweeps, b.winner_clone, b.end_sweep) == \
            (single.tts_sweeps, single.winner_clone, single.end_sweep)
    # and the batch itself against the oracle on the small ones
    for k in (0, 3):
        assert_parity(insts[k], hs[k], cfgs[k], batch[k])


def test_resume_equals_uninterrupted():
    torch = _torch()
    inst = planted_instance(80, 44)
    h = xorsat.Instance(inst.tri, inst.J)
    kw = dict(n_clones=2048, seed=77, instance_id=2, stop_on_first=False, chunk_sweeps=16)
    full = xorsat.run(h, xorsat.make_config(max_sweeps=90, **kw))
    a = xorsat.run(h, xorsat.make_config(max_sweeps=40, **kw))
    b = xorsat.run(h, xorsat.make_config(max_sweeps=50, start_sweep=40, resume=True, **kw),
                   state=a.state.clone())
    assert torch.equal(full.state, b.state)
    assert torch.equal(full.energy, b.energy)
    assert b.end_sweep == 90


def test_zero_budget_and_ground_state_start():
    """max_sweeps = 0 only checks the start; a start in the planted solution is a hit at
    start_sweep and never moves (w0 = 0)."""
    torch = _torch()
    inst = planted_instance(64, 45)
    h = xorsat.Instance(inst.tri, inst.J)
    cfg = xorsat.make_config(n_clones=512, seed=3, max_sweeps=0)
    out = xorsat.run(h, cfg)
    assert out.sweeps_done == 0 and out.end_sweep == 0
    assert_parity(inst, h, cfg, out)
    # all clones start in the planted solution tau
    bits = (inst.tau < 0).astype(np.uint64)
    word = np.where(bits[:, None] == 1, np.uint64(2**64 - 1), np.uint64(0))
    state = torch.from_numpy(np.repeat(word, 512 // 64, axis=1).view(np.int64)).cuda()
    cfg = xorsat.make_config(n_clones=512, seed=3, max_sweeps=10, start_sweep=17, resume=True,
                             stop_on_first=False)
    out = xorsat.run(h, cfg, state=state.clone())
    assert torch.equal(out.state, state)
    assert (out.first_hit.cpu().numpy() == 17).all()
    assert (out.energy.cpu().numpy() == -64).all()
    assert out.tts_sweeps == 17 and out.winner_clone == 0


@pytest.mark.parametrize("n,clones,sweeps,place", [(256, 65536, 120, False),
                                                   (1024, 1 << 20, 12, True),
                                                   (2048, 16384, 20, True)])
def test_full_size_sampled_clones(n, clones, sweeps, place):
    """Full-size lone instances (N = 256 with 65,536 clones, N = 1024 with 2^20 clones and its
    LDS rows placed, the largest N) in the library's default shape for a lone instance: every
    clone's energy must be a valid E = 2U - N; sampled clones from different tiles match the
    oracle bit for bit. The batched and steady-state workloads' own launch shapes are checked
    over several chunks in test_gpu_shapes.py."""
    _torch()
    inst = planted_instance(n, 9000 + n)
    h = xorsat.Instance(inst.tri, inst.J)
    cfg = xorsat.make_config(n_clones=clones, seed=n, instance_id=n, max_sweeps=sweeps,
                             stop_on_first=False, place_rows=place)
    out = xorsat.run(h, cfg)
    en = out.energy.cpu().numpy()
    assert en.min() >= -n and en.max() <= n and np.all((en + n) % 2 == 0)
    rng = np.random.default_rng(n)
    groups = rng.choice(clones // 32, size=6, replace=False)
    sample = np.sort(np.concatenate([32 * g + np.arange(32) for g in groups]))
    sample = np.r_[sample, clones - 1]
    assert_parity(inst, h, cfg, out, clones=sample)


# --------------------------------------------------------------------------- w0 > 0 (Metropolis)

def _w_thresholds(T):
    """w1 = exp(-2/T) and w0 = w1^3 (the detailed-balance rule at temperature T) as 16-bit
    thresholds."""
    import math
    return round(math.exp(-2.0 / T) * 65536), round(math.exp(-6.0 / T) * 65536)


@pytest.mark.parametrize("n,clones,B,T,C,G,chunk,sweeps,thr,thr0", [
    (100, 4096, 2, 0, 0, 0, 7, 40, *_w_thresholds(1.0)),     # ragged classes, 8 tiles
    (37, 2048, 0, 0, 0, 0, 0, 33, THR_PAPER, 20000),          # odd N, large w0, one chunk
    (257, 1024, 1, 64, 8, 1, 5, 23, *_w_thresholds(0.69)),    # global records, narrow columns
    (128, 8192, 4, 256, 4, 2, 16, 50, 65536, 65536),          # every spin flips each visit
    (4, 256, 1, 0, 0, 0, 1, 9, 30000, 1),                     # smallest case
])
def test_metropolis_budget_runs(n, clones, B, T, C, G, chunk, sweeps, thr, thr0):
    """w0 > 0: every clone's end configuration, energy and end-only ground-state mark equal the
    oracle's."""
    _torch()
    inst = planted_instance(n, 800 + n)
    h = xorsat.Instance(inst.tri, inst.J)
    cfg = xorsat.make_config(n_clones=clones, seed=n * 3 + 1, instance_id=5, accept_thr=thr,
                             accept_thr0=thr0, max_sweeps=sweeps, stop_on_first=False,
                             chunk_sweeps=chunk, tile_blocks=B, wg_threads=T, col_bytes=C,
                             rec_global=G, place_rows=n % 2 == 1)
    out = xorsat.run(h, cfg)
    ref = assert_parity(inst, h, cfg, out)
    assert set(np.unique(ref["first_hit"])) <= {-1, sweeps}
    tts, winner = oracle.solve_results(ref["first_hit"])
    assert (out.tts_sweeps, out.winner_clone) == (tts, winner)


def test_metropolis_end_ground_states_marked():
    """A small instance at low w0: many clones end in a ground state; exactly those are marked
    with the end sweep, and the solved configuration is the lowest such clone's."""
    _torch()
    inst = planted_instance(12, 4242)
    h = xorsat.Instance(inst.tri, inst.J)
    cfg = xorsat.make_config(n_clones=4096, seed=11, instance_id=0, accept_thr=THR_PAPER,
                             accept_thr0=11, max_sweeps=200, stop_on_first=False,
                             chunk_sweeps=50)
    out = xorsat.run(h, cfg)
    ref = assert_parity(inst, h, cfg, out)
    fh = out.first_hit.cpu().numpy()
    en = out.energy.cpu().numpy()
    assert np.array_equal(fh == 200, en == -12)
    assert (fh == 200).sum() > 100
    winner = int(np.flatnonzero(fh == 200)[0])
    assert out.tts_sweeps == 200 and out.winner_clone == winner
    assert np.array_equal(out.solved, ref["final_spins"][winner])


def test_metropolis_rejects_stop_on_first():
    _torch()
    inst = planted_instance(16, 1)
    h = xorsat.Instance(inst.tri, inst.J)
    cfg = xorsat.make_config(n_clones=256, seed=1, accept_thr0=5, max_sweeps=10,
                             stop_on_first=True)
    with pytest.raises(xorsat.XsError):
        xorsat.run(h, cfg)


def test_metropolis_tiling_and_batch_neutral():
    """Launch knobs and batching with quasi-greedy instances change nothing for w0 > 0 runs."""
    torch = _torch()
    inst = planted_instance(128, 21)
    h = xorsat.Instance(inst.tri, inst.J)
    thr, thr0 = _w_thresholds(0.8)
    outs = []
    for B, T, C, G in ((1, 0, 0, 0), (4, 1024, 16, 2), (8, 256, 8, 1), (2, 128, 4, 2)):
        cfg = xorsat.make_config(n_clones=8192, seed=7, instance_id=2, accept_thr=thr,
                                 accept_thr0=thr0, max_sweeps=100, stop_on_first=False,
                                 chunk_sweeps=30, tile_blocks=B, wg_threads=T, col_bytes=C,
                                 rec_global=G)
        outs.append(xorsat.run(h, cfg))
    for o in outs[1:]:
        assert torch.equal(o.state, outs[0].state)
        assert torch.equal(o.first_hit, outs[0].first_hit)
        assert torch.equal(o.energy, outs[0].energy)
    # mixed batch: quasi-greedy and w0 > 0 runs of the same instance side by side
    base = dict(n_clones=8192, seed=7, instance_id=2, accept_thr=thr, max_sweeps=100,
                stop_on_first=False, chunk_sweeps=30)
    cfgs = [xorsat.make_config(accept_thr0=thr0, **base), xorsat.make_config(**base)]
    batch = xorsat.run_batch([h, h], cfgs)
    qg = xorsat.run(h, cfgs[1])
    assert torch.equal(batch[0].state, outs[0].state)
    assert torch.equal(batch[0].energy, outs[0].energy)
    assert torch.equal(batch[1].state, qg.state)
    assert torch.equal(batch[1].first_hit, qg.first_hit)
    # the two rules differ (w0 > 0 moves k = 0 spins)
    assert not torch.equal(batch[0].state, batch[1].state)


@pytest.mark.parametrize("T", [1.0, 0.8])
def test_metropolis_full_size_paramagnetic_energy(T):
    """N = 2048, 2^17 clones, w0 = w1^3 at temperature T: the mean energy per spin after 300
    sweeps is the paramagnet's -tanh(1/T) (a property at any size), and sampled clones from
    different tiles match the oracle bit for bit."""
    import math
    _torch()
    n, clones = 2048, 1 << 17
    inst = planted_instance(n, 31337)
    h = xorsat.Instance(inst.tri, inst.J)
    thr, thr0 = _w_thresholds(T)
    cfg = xorsat.make_config(n_clones=clones, seed=12345, instance_id=9, accept_thr=thr,
                             accept_thr0=thr0, max_sweeps=300, stop_on_first=False)
    out = xorsat.run(h, cfg)
    en = out.energy.cpu().numpy()
    e = en.mean() / n
    assert abs(e + math.tanh(1.0 / T)) < 0.004, e
    rng = np.random.default_rng(int(T * 10))
    groups = rng.choice(clones // 32, size=3, replace=False)
    sample = np.sort(np.concatenate([32 * g + np.arange(32) for g in groups]))
    assert_parity(inst, h, cfg, out, clones=sample)


def test_host_buffers_rejected_before_launch():
    """A state buffer in ordinary host memory is refused by the library (XS_EINVAL, nothing
    launched), and the binding refuses a CPU tensor before calling it."""
    import ctypes
    torch = _torch()
    inst = planted_instance(64, 3)
    h = xorsat.Instance(inst.tri, inst.J)
    cfg = xorsat.make_config(n_clones=256, seed=1, max_sweeps=5)
    host_state = np.zeros((64, 4), dtype=np.int64)
    fh = torch.empty(256, dtype=torch.int32, device="cuda")
    bufs = xorsat.RunBuffers(host_state.ctypes.data, fh.data_ptr(), None, None)
    res = xorsat.RunResult()
    lib = xorsat.load()
    st = lib.xs_run(h.handle, ctypes.byref(cfg), ctypes.byref(bufs), xorsat._stream(),
                    ctypes.byref(res))
    assert st == xorsat.XS_STATUS_CODES["XS_EINVAL"]
    assert "device memory" in lib.xs_last_error().decode()
    with pytest.raises(ValueError):
        xorsat.run(h, cfg, state=torch.zeros((64, 4), dtype=torch.int64))
    # the device is still fine
    out = xorsat.run(h, cfg)
    assert out.sweeps_done <= 5


def test_async_batches_equal_sync():
    """Two asynchronous batches on two streams, driven from library threads while the host
    keeps working, give the same results as the synchronous batch."""
    torch = _torch()
    sizes = [(48, 512), (100, 2048), (256, 4096)]
    hs, cfgs = [], []
    for k, (n, nc) in enumerate(sizes):
        inst = planted_instance(n, 7700 + k)
        hs.append(xorsat.Instance(inst.tri, inst.J))
        cfgs.append(xorsat.make_config(n_clones=nc, seed=31 + k, instance_id=k,
                                       max_sweeps=400 if n < 100 else 60, stop_on_first=n < 100,
                                       chunk_sweeps=20))
    sync = xorsat.run_batch(hs, cfgs)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    a = xorsat.run_batch_async(hs, cfgs, stream=s1)
    b = xorsat.run_batch_async(hs[::-1], cfgs[::-1], stream=s2)
    busy = sum(range(100000))  # host work meanwhile
    ra, rb = a.wait(), b.wait()[::-1]
    assert busy > 0
    for x, y, z in zip(sync, ra, rb):
        for o in (y, z):
            assert torch.equal(o.state, x.state)
            assert torch.equal(o.first_hit, x.first_hit)
            assert torch.equal(o.energy, x.energy)
            assert (o.tts_sweeps, o.winner_clone, o.end_sweep) == \
                (x.tts_sweeps, x.winner_clone, x.end_sweep)
    with pytest.raises(RuntimeError):
        a.wait()
    # argument errors come back from the call itself, before any thread starts
    bad = xorsat.make_config(n_clones=300, seed=1)
    with pytest.raises(xorsat.XsError):
        xorsat.run_batch_async([hs[0]], [bad])


@pytest.mark.parametrize("n", [8, 10, 12])
def test_first_hit_law_of_the_exact_chain(n):
    """Without the oracle: the GPU's first_hit distribution over 131,072 clones equals the exact
    law of the sweep's Markov chain over all 2^N configurations (quasi-greedy rule), computed by
    propagating the law of the state in the library's update order."""
    _torch()
    inst = planted_instance(n, 3)
    h = xorsat.Instance(inst.tri, inst.J)
    perm, _ = h.partition()
    T, clones = 300, 131072
    out = xorsat.run(h, xorsat.make_config(n_clones=clones, seed=23, max_sweeps=T,
                                           stop_on_first=False))
    assert out.sweeps_done == T
    exact = ground_law(n, inst.tri, inst.J, perm, THR_PAPER / 65536, 0.0, T)
    fh = out.first_hit.cpu().numpy()
    emp = np.cumsum(np.bincount(fh[fh >= 0], minlength=T + 1)) / clones
    assert np.all(np.abs(emp - exact) <= group_tolerance(exact, clones // 32, 5.5) + 1e-9)
    assert np.abs(emp - exact).max() < 0.015


@pytest.mark.parametrize("thr0", [3277, 13107])
def test_metropolis_end_state_law_of_the_exact_chain(thr0):
    """Without the oracle: with w0 > 0 the share of 2^20 clones in a ground state after T sweeps
    equals the exact chain's P(E = -N after T sweeps)."""
    _torch()
    n = 10
    inst = planted_instance(n, 3)
    h = xorsat.Instance(inst.tri, inst.J)
    perm, _ = h.partition()
    clones = 1 << 20
    exact = ground_law(n, inst.tri, inst.J, perm, THR_PAPER / 65536, thr0 / 65536, 30)
    for T in (1, 3, 10, 30):
        out = xorsat.run(h, xorsat.make_config(n_clones=clones, seed=29, max_sweeps=T,
                                               stop_on_first=False, accept_thr0=thr0))
        share = float((out.first_hit == T).float().mean())
        assert abs(share - exact[T]) <= group_tolerance(exact[T], clones // 32, 5.0), (T, share)


def test_clone_count_limit_rejected_before_any_work():
    """n_clones above XS_MAX_CLONES (clone indices would leave int32) is XS_EINVAL from the run
    and the autotuner, found before any buffer is looked at or any kernel is launched."""
    import ctypes
    _torch()
    inst = planted_instance(16, 1)
    h = xorsat.Instance(inst.tri, inst.J)
    lib = xorsat.load()
    cfg = xorsat.make_config(n_clones=xorsat.XS_MAX_CLONES + xorsat.XS_CLONE_QUANTUM, seed=1,
                             stop_on_first=False, max_sweeps=1)
    res = xorsat.RunResult()
    st = lib.xs_run(h.handle, ctypes.byref(cfg), ctypes.byref(xorsat.RunBuffers()), None,
                    ctypes.byref(res))
    assert xorsat.XS_STATUS[st] == "XS_EINVAL"
    assert b"n_clones" in lib.xs_last_error()
    tune = xorsat.TuneResult()
    st = lib.xs_autotune(h.handle, xorsat.XS_MAX_CLONES + xorsat.XS_CLONE_QUANTUM, 1, None,
                         ctypes.byref(tune))
    assert xorsat.XS_STATUS[st] == "XS_EINVAL"

