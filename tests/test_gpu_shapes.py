"""GPU <-> oracle parity at the launch shapes the throughput numbers come from.

* The batched N = 256 workload's kernel (tiles of four 256-clone blocks, 256 threads, 16-byte
  columns, records in global memory, coupling gauge; and eight-block tiles with records in LDS)
  inside a batch, over several chunks.
* The steady-state N = 1024 workload's kernel (the library's default shape for 2^20 clones, rows
  placed), over several chunks.
* An uneven batch of many instances (N from 32 to 1024, mixed clone counts, mixed stop rules),
  each instance against the oracle and against its run alone.

Starts are given (XS_RESUME): most groups random, some a few spin flips away from the planted
solution, so that clones reach a ground state at the start, inside the first chunk (the
end-of-chunk test and its replay) and in later chunks (per-sweep tracking). Sampled 32-clone
groups from different tiles are compared with the oracle clone by clone (first hit, energy at
the end sweep, end spins); the run's TTS and winner with the oracle's reduction of the GPU's
first hits, with the winner's group among the sampled ones."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2102_09510_amd import xorsat
from paper_2102_09510_amd.instances import THR_PAPER, planted_instance, uneven_sizes
from tests.parity import check_clones, check_run_reduction, group_sample, pack_spins, \
    spins_of_clones

pytestmark = pytest.mark.gpu

# The library's default launch shape of the steady-state workload (16 x N = 1024 x 2^20 clones,
# rows placed), which bench.py times: (tile_blocks, wg_threads, col_bytes, rec_global).
STEADY_SHAPE = (1, 256, 8, 1)


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def near_solution_state(inst, n_clones, rng, groups_flips):
    """A start state: random words, except the given groups, whose clones start from the planted
    solution tau with `flips` distinct spins flipped (each clone its own). Returns (state as
    int64 [n][W] numpy, {group: spins [32][n]})."""
    n = inst.n
    W = n_clones // 64
    state = np.frombuffer(rng.bytes(8 * n * W), dtype=np.uint64).reshape(n, W).copy()
    starts = {}
    for g, flips in groups_flips.items():
        sp = np.tile(inst.tau, (32, 1)).astype(np.int8)
        for c in range(32):
            sp[c, rng.choice(n, flips, replace=False)] *= -1
        starts[g] = sp
        # write the group's 32 bits (half a word) into the state
        bits = pack_spins(np.concatenate([sp, sp]))[:, 0]  # 64 clones -> one word; keep 32 bits
        w, half = divmod(g, 2)
        lo = np.uint64(0xFFFFFFFF)
        mask = lo << np.uint64(32 * half)
        state[:, w] = (state[:, w] & ~mask) | ((bits & lo) << np.uint64(32 * half))
    return state.view(np.int64), starts


def sample_init(state_i64, clones):
    """Start spins of the given clones, read from the start state."""
    return spins_of_clones(state_i64, clones)


def check_instance(inst, h, cfg, out, start_state, groups, what):
    """Oracle parity of the sampled groups (plus the winner's group) from the given start."""
    perm, _ = h.partition()
    operm, _ = oracle.colour(inst.tri, h.colour_cap)
    assert np.array_equal(perm, operm), what
    fh = out.first_hit.cpu().numpy()
    check_run_reduction(fh, out.tts_sweeps, out.winner_clone)
    groups = list(groups)
    if out.winner_clone >= 0:
        groups.append(out.winner_clone // 32)
    clones = group_sample(cfg.n_clones, groups)
    clones = np.unique(np.r_[clones, cfg.n_clones - 1])
    init = sample_init(start_state, clones)
    ref = check_clones(inst.tri, inst.J, operm, cfg, out.sweeps_done, clones, fh,
                       out.energy.cpu().numpy(), out.state, init_spins=init, what=what)
    if out.winner_clone >= 0:
        k = int(np.flatnonzero(clones == out.winner_clone)[0])
        assert np.array_equal(out.solved, ref["final_spins"][k]), what
        assert oracle.energy(inst.tri, inst.J, out.solved) == -inst.n, what
    return ref


@pytest.mark.parametrize("shape", [(4, 256, 16, 1), (8, 512, 16, 2)],
                         ids=["default-4blk-global-records-gauge", "8blk-lds-records"])
def test_batched_n256_timed_shape_resumed_near_solution(shape):
    """The batched N = 256 workload's kernel: three instances of 65,536 clones in one batch with
    the default shape (tile_blocks = 4, wg_threads = 256, col_bytes = 16, records in global
    memory, so the persistent launch runs them in their coupling gauge), and with eight-block
    tiles of 512 threads and records in LDS; 200 sweeps in chunks of 50 from sweep 1000 (budget
    runs, the resumed states flipped into the gauge and back) and a stop-on-first run that ends
    after its first chunk."""
    torch = _torch()
    B, T, C, G = shape
    n, nc = 256, 65536  # tiles of 2,048 clones: 64 groups per tile, 32 tiles per instance
    rng = np.random.default_rng(256)
    insts, hs, cfgs, starts, picks = [], [], [], [], []
    for k in range(3):
        inst = planted_instance(n, 2_000_000 + k)
        insts.append(inst)
        hs.append(xorsat.Instance(inst.tri, inst.J))
        # near-solution groups: one per flip level, each in its own tile (tiles 3, 7, ..., 27)
        levels = {0: 0, 1: 1, 4: 4, 16: 16, 32: 32, 40: 32, 48: 48}
        gf = {}
        for t, (lvl, flips) in enumerate(levels.items()):
            gf[64 * (3 + 4 * t) + 5 * t + 1] = flips
        # the zero-flip group only in the third instance, so the others' TTS comes from a
        # descent inside the first chunk rather than from the start check
        if k != 2:
            gf = {g: f for g, f in gf.items() if f > 0}
        st, sp = near_solution_state(inst, nc, rng, gf)
        starts.append(st)
        picks.append(sorted(gf)[:5] + [64 * 1 + 9, 64 * 30 + 63])  # + two random groups
        cfgs.append(xorsat.make_config(
            n_clones=nc, seed=0xC2 + k, instance_id=k, accept_thr=THR_PAPER, max_sweeps=200,
            start_sweep=1000, resume=True, stop_on_first=(k == 1), chunk_sweeps=50,
            tile_blocks=B, wg_threads=T, col_bytes=C, rec_global=G))
    outs = xorsat.run_batch(hs, cfgs, states=[torch.from_numpy(s.copy()).cuda() for s in starts])
    for k, out in enumerate(outs):
        assert (out.tile_blocks, out.wg_threads, out.col_bytes, out.rec_global) == \
            (B, T, C, 1 if G == 1 else 0)
        assert out.persistent == 1
        if k == 1:
            assert out.end_sweep == 1050 and out.tts_sweeps < 1050
        else:
            assert out.end_sweep == 1200
        fh = out.first_hit.cpu().numpy()
        # hits at the start (instance 2), inside the first chunk and in later chunks
        assert ((fh > 1000) & (fh < 1050)).any()
        if k != 1:
            assert (fh >= 1050).any(), "no hit after the first chunk: tracking not exercised"
        if k == 2:
            assert (fh == 1000).any()
        check_instance(insts[k], hs[k], cfgs[k], out, starts[k], picks[k], f"instance {k}")


def test_batched_n256_long_chunks_stop_on_first():
    """The batched N = 256 workload as the benchmark times it: its launch shape (four-block
    tiles of 256 threads, 16-byte columns, records in global memory, rows placed), runs to the
    first ground state in chunks of 500 sweeps, from near-solution starts. Each run ends at the
    end of the chunk that holds its first hit, with the same TTS and winner as in chunks of 50
    (the first hits up to that sweep agree clone for clone), and sampled clone groups equal the
    oracle."""
    torch = _torch()
    n, nc = 256, 65536
    rng = np.random.default_rng(2561)
    insts, hs, starts, picks = [], [], [], []
    for k in range(2):
        inst = planted_instance(n, 2_000_000 + k)
        insts.append(inst)
        hs.append(xorsat.Instance(inst.tri, inst.J))
        gf = {64 * (3 + 4 * t) + 5 * t + 1: f for t, f in enumerate((4, 16, 32, 48))}
        st, _ = near_solution_state(inst, nc, rng, gf)
        starts.append(st)
        picks.append(sorted(gf) + [64 * 30 + 63])

    def run(chunk):
        cfgs = [xorsat.make_config(n_clones=nc, seed=0xB5 + k, instance_id=k,
                                   accept_thr=THR_PAPER, max_sweeps=1000, resume=True,
                                   stop_on_first=True, chunk_sweeps=chunk, tile_blocks=4,
                                   wg_threads=256, col_bytes=16, rec_global=1, place_rows=True)
                for k in range(2)]
        return cfgs, xorsat.run_batch(hs, cfgs,
                                      states=[torch.from_numpy(s.copy()).cuda() for s in starts])

    cfgs, long_runs = run(500)
    _, short_runs = run(50)
    for k in range(2):
        a, b = long_runs[k], short_runs[k]
        assert (a.tile_blocks, a.wg_threads, a.col_bytes, a.rec_global) == (4, 256, 16, 1)
        assert 0 <= a.tts_sweeps < 500, "no hit in the first long chunk"
        assert a.end_sweep == 500 and b.end_sweep == 50 * (b.tts_sweeps // 50 + 1)
        assert (a.tts_sweeps, a.winner_clone) == (b.tts_sweeps, b.winner_clone)
        fa, fb = a.first_hit.cpu().numpy(), b.first_hit.cpu().numpy()
        upto = (fb >= 0) & (fb < b.end_sweep)
        assert np.array_equal(fa[upto], fb[upto]), f"instance {k}"
        early = (fa >= 0) & (fa < b.end_sweep)
        assert np.array_equal(fa[early], fb[early]), f"instance {k}"
        check_instance(insts[k], hs[k], cfgs[k], a, starts[k], picks[k], f"instance {k}")


def test_steady_n1024_shape_over_chunks():
    """The steady-state workload's kernel at its real size: two instances of N = 1024 with 2^20
    clones in one batch, the library's default shape with the LDS rows placed, 30 sweeps in
    chunks of 10 from given starts."""
    torch = _torch()
    n, nc = 1024, 1 << 20
    rng = np.random.default_rng(1024)
    insts, hs, cfgs, starts, picks = [], [], [], [], []
    for k in range(2):
        inst = planted_instance(n, 3_000_000 + k)
        insts.append(inst)
        hs.append(xorsat.Instance(inst.tri, inst.J))
        flips = (4, 32, 64, 96, 96, 128)
        gf = {8 * (100 + 611 * t) + t: f for t, f in enumerate(flips)}  # one tile each
        st, _ = near_solution_state(inst, nc, rng, gf)
        starts.append(st)
        picks.append(sorted(gf) + [8 * 7 + 3, 8 * 4000 + 5])
        cfgs.append(xorsat.make_config(
            n_clones=nc, seed=0xC3 + k, instance_id=k, accept_thr=THR_PAPER, max_sweeps=30,
            resume=True, stop_on_first=False, chunk_sweeps=10, place_rows=True))
    outs = xorsat.run_batch(hs, cfgs, states=[torch.from_numpy(s).cuda() for s in starts])
    for k, out in enumerate(outs):
        assert (out.tile_blocks, out.wg_threads, out.col_bytes, out.rec_global) == STEADY_SHAPE
        assert out.end_sweep == 30
        fh = out.first_hit.cpu().numpy()
        assert (fh[fh >= 0] < 10).any() and (fh >= 10).any()
        en = out.energy.cpu().numpy()
        assert en.min() >= -n and en.max() <= n and np.all((en + n) % 2 == 0)
        check_instance(insts[k], hs[k], cfgs[k], out, starts[k], picks[k], f"instance {k}")


def test_steady_n1024_long_chunks():
    """The steady-state workload as the benchmark times it: two instances of N = 1024 with 2^20
    clones in one batch, the library's default shape with the rows placed, 2,000 sweeps in
    chunks of 1,000 (each a cross-sweep body run over its 1,000 sweeps). The outputs equal those
    of chunks of 100 bit for bit, and sampled clone groups equal the oracle from the same
    starts."""
    torch = _torch()
    n, nc = 1024, 1 << 20
    rng = np.random.default_rng(2024)
    insts, hs, starts = [], [], []
    for k in range(2):
        inst = planted_instance(n, 3_000_000 + k)
        insts.append(inst)
        hs.append(xorsat.Instance(inst.tri, inst.J))
        starts.append(near_solution_state(inst, nc, rng, {})[0])

    def run(chunk):
        cfgs = [xorsat.make_config(n_clones=nc, seed=0x5C + k, instance_id=k,
                                   accept_thr=THR_PAPER, max_sweeps=2000, resume=True,
                                   stop_on_first=False, chunk_sweeps=chunk, place_rows=True)
                for k in range(2)]
        return cfgs, xorsat.run_batch(hs, cfgs,
                                      states=[torch.from_numpy(s).cuda() for s in starts])

    cfgs, long_runs = run(1000)
    _, short_runs = run(100)
    for k in range(2):
        a, b = long_runs[k], short_runs[k]
        assert (a.tile_blocks, a.wg_threads, a.col_bytes, a.rec_global) == STEADY_SHAPE
        assert a.end_sweep == b.end_sweep == 2000
        assert torch.equal(a.state, b.state), f"instance {k}"
        assert torch.equal(a.first_hit, b.first_hit) and torch.equal(a.energy, b.energy)
        check_instance(insts[k], hs[k], cfgs[k], a, starts[k], [3, 16001, nc // 32 - 1],
                       f"instance {k}")


def test_uneven_batch_against_oracle_and_alone():
    """Twenty instances of the uneven workload's family (N uniform on {32, ..., 1024}, clones
    from 4,096 to 65,536), half run to the first ground state and half to a budget, in one
    batch: each instance equals its run alone bit for bit, and sampled groups of each equal the
    oracle."""
    torch = _torch()
    sizes = uneven_sizes(20, seed=4_000_777)
    assert len({n for n, _ in sizes}) >= 10 and len({c for _, c in sizes}) >= 3
    insts, hs, cfgs = [], [], []
    for k, (n, nc) in enumerate(sizes):
        inst = planted_instance(n, 4_000_000 + k)
        insts.append(inst)
        hs.append(xorsat.Instance(inst.tri, inst.J))
        cfgs.append(xorsat.make_config(n_clones=nc, seed=0xC4 + k, instance_id=k,
                                       accept_thr=THR_PAPER, max_sweeps=300,
                                       stop_on_first=(k % 2 == 0), chunk_sweeps=50))
    batch = xorsat.run_batch(hs, cfgs)
    rng = np.random.default_rng(4)
    for k, (inst, h, cfg, out) in enumerate(zip(insts, hs, cfgs, batch)):
        alone = xorsat.run(h, cfg)
        assert torch.equal(out.state, alone.state), k
        assert torch.equal(out.first_hit, alone.first_hit), k
        assert torch.equal(out.energy, alone.energy), k
        assert (out.tts_sweeps, out.winner_clone, out.end_sweep) == \
            (alone.tts_sweeps, alone.winner_clone, alone.end_sweep), k
        groups = rng.choice(cfg.n_clones // 32, size=2, replace=False)
        perm, _ = h.partition()
        operm, _ = oracle.colour(inst.tri, h.colour_cap)
        assert np.array_equal(perm, operm)
        fh = out.first_hit.cpu().numpy()
        check_run_reduction(fh, out.tts_sweeps, out.winner_clone)
        gl = list(groups) + ([out.winner_clone // 32] if out.winner_clone >= 0 else [])
        clones = np.unique(np.r_[group_sample(cfg.n_clones, gl), cfg.n_clones - 1])
        ref = check_clones(inst.tri, inst.J, operm, cfg, out.sweeps_done, clones, fh,
                           out.energy.cpu().numpy(), out.state, what=f"instance {k} (N={inst.n})")
        if out.winner_clone >= 0:
            w = int(np.flatnonzero(clones == out.winner_clone)[0])
            assert np.array_equal(out.solved, ref["final_spins"][w])


def test_persistent_queue_launch_equals_launch_per_chunk():
    """The persistent work-queue launch (the default) and the launch-per-chunk loop
    (XS_PER_CHUNK) on the same uneven batch: 24 instances, N from 32 to 2048, clone counts
    from 4,096 to 65,536, mixed stop rules and chunk lengths, some instances solved in their
    first chunks, one with no sweep budget; every buffer and result is equal, and sampled groups
    equal the oracle."""
    torch = _torch()
    sizes = uneven_sizes(22, seed=4_000_999) + [(2048, 16384), (48, 4096)]
    insts, hs, cfgs_q, cfgs_c = [], [], [], []
    for k, (n, nc) in enumerate(sizes):
        inst = planted_instance(n, 4_100_000 + k)
        insts.append(inst)
        hs.append(xorsat.Instance(inst.tri, inst.J))
        kw = dict(n_clones=nc, seed=0x9E + k, instance_id=k, accept_thr=THR_PAPER,
                  max_sweeps=0 if k == 5 else 240, stop_on_first=(k % 3 != 0),
                  chunk_sweeps=(40, 60, 100)[k % 3])
        cfgs_q.append(xorsat.make_config(**kw))
        cfgs_c.append(xorsat.make_config(per_chunk=True, **kw))
    print("# queue launch vs launch per chunk: 24 instances", flush=True)
    q = xorsat.run_batch(hs, cfgs_q)
    c = xorsat.run_batch(hs, cfgs_c)
    assert len({o.wg_threads for o in q}) == 1  # one workgroup size for the persistent launch
    rng = np.random.default_rng(9)
    for k, (a, b) in enumerate(zip(q, c)):
        assert torch.equal(a.state, b.state), k
        assert torch.equal(a.first_hit, b.first_hit), k
        assert torch.equal(a.energy, b.energy), k
        assert (a.tts_sweeps, a.winner_clone, a.end_sweep, a.sweeps_done) == \
            (b.tts_sweeps, b.winner_clone, b.end_sweep, b.sweeps_done), k
        assert (a.persistent, b.persistent) == (1, 0), k
        if a.winner_clone >= 0:
            assert np.array_equal(a.solved, b.solved), k
    assert q[5].end_sweep == 0 and q[5].sweeps_done == 0
    assert any(o.tts_sweeps >= 0 for o in q) and any(o.tts_sweeps < 0 for o in q)
    for k in (0, 7, 22, 23):
        inst, h, cfg, out = insts[k], hs[k], cfgs_q[k], q[k]
        operm, _ = oracle.colour(inst.tri, h.colour_cap)
        fh = out.first_hit.cpu().numpy()
        check_run_reduction(fh, out.tts_sweeps, out.winner_clone)
        groups = list(rng.choice(cfg.n_clones // 32, size=2, replace=False))
        if out.winner_clone >= 0:
            groups.append(out.winner_clone // 32)
        clones = np.unique(group_sample(cfg.n_clones, groups))
        check_clones(inst.tri, inst.J, operm, cfg, out.sweeps_done, clones, fh,
                     out.energy.cpu().numpy(), out.state, what=f"queue instance {k}")


def test_persistent_queue_over_several_epochs_and_timed():
    """A run longer than one persistent launch (300 chunks of 10 sweeps: five epochs of 60
    chunks) and a stop-on-first batch, each with launch timing on and off, against the
    launch-per-chunk loop: all equal, and sampled clones equal the oracle."""
    torch = _torch()
    inst = planted_instance(96, 4_200_001)
    h = xorsat.Instance(inst.tri, inst.J)
    kw = dict(n_clones=4096, seed=0x51, instance_id=3, accept_thr=THR_PAPER, max_sweeps=3000,
              stop_on_first=False, chunk_sweeps=10)
    others = [planted_instance(n, 4_200_100 + n) for n in (40, 72, 200)]
    ho = [xorsat.Instance(i.tri, i.J) for i in others]
    kb = [dict(n_clones=8192, seed=0x61 + k, instance_id=k, max_sweeps=40000, chunk_sweeps=7)
          for k in range(3)]
    print("# queue over several epochs, timed and untimed", flush=True)
    runs = {}
    for name, per_chunk, timed in (("queue", False, False), ("queue-timed", False, True),
                                   ("per-chunk", True, False)):
        xorsat.profile_enable(timed)
        try:
            runs[name] = [xorsat.run(h, xorsat.make_config(per_chunk=per_chunk, **kw))] + \
                xorsat.run_batch(ho, [xorsat.make_config(per_chunk=per_chunk, **c) for c in kb])
        finally:
            xorsat.profile_enable(False)
    xorsat.profile_read(reset=True)
    assert all(o.persistent == 1 for o in runs["queue"] + runs["queue-timed"])
    assert all(o.persistent == 0 for o in runs["per-chunk"])
    for name in ("queue-timed", "per-chunk"):
        for a, b in zip(runs["queue"], runs[name]):
            assert torch.equal(a.state, b.state), name
            assert torch.equal(a.first_hit, b.first_hit), name
            assert torch.equal(a.energy, b.energy), name
            assert (a.tts_sweeps, a.winner_clone, a.end_sweep) == \
                (b.tts_sweeps, b.winner_clone, b.end_sweep), name
    out = runs["queue"][0]
    assert out.end_sweep == 3000
    operm, _ = oracle.colour(inst.tri, h.colour_cap)
    cfg = xorsat.make_config(**kw)
    clones = np.r_[0:32, 2048:2080, 4064:4096]
    check_clones(inst.tri, inst.J, operm, cfg, out.sweeps_done, clones,
                 out.first_hit.cpu().numpy(), out.energy.cpu().numpy(), out.state,
                 what="several epochs")
    assert all(o.tts_sweeps >= 0 for o in runs["queue"][1:3])  # N = 40, 72 solve


@pytest.mark.parametrize("n,nc,shape", [(1024, 1 << 18, STEADY_SHAPE), (256, 65536, (4, 256, 16, 1))])
def test_cross_sweep_body_equals_one_sweep_at_a_time(n, nc, shape):
    """Untracked chunks run the cross-sweep body (the end of a sweep overlapped with the start
    of the next); XS_ONE_SWEEP_STEPS runs the same chunks one sweep after another. From the same
    near-solution starts, over chunks of 25 sweeps (hits inside the first chunk, so its replay
    follows a body chunk, and in later chunks), both give bit-identical states, first hits and
    energies, and sampled groups match the oracle."""
    torch = _torch()
    rng = np.random.default_rng(n + 7)
    inst = planted_instance(n, 3_100_000 + n)
    h = xorsat.Instance(inst.tri, inst.J)
    B, T, C, G = shape
    assert h.body(T * C // (32 * B)) is not None, "this shape's steps have a cross-sweep body"
    gf = {16 * (3 + 5 * t) + t: f for t, f in enumerate((2, 8, 24, 48))}
    st, _ = near_solution_state(inst, nc, rng, gf)
    outs = []
    for one in (False, True):
        cfg = xorsat.make_config(n_clones=nc, seed=0xB0D + n, instance_id=3, accept_thr=THR_PAPER,
                                 max_sweeps=100, start_sweep=500, resume=True,
                                 stop_on_first=False, chunk_sweeps=25, one_sweep_steps=one,
                                 tile_blocks=B, wg_threads=T, col_bytes=C, rec_global=G)
        outs.append((cfg, xorsat.run(h, cfg, state=torch.from_numpy(st.copy()).cuda())))
    (cfg, a), (_, b) = outs
    for o in (a, b):
        assert (o.tile_blocks, o.wg_threads, o.col_bytes, o.rec_global) == shape
    assert a.end_sweep == b.end_sweep == 600
    fh = a.first_hit.cpu().numpy()
    assert ((fh > 500) & (fh < 525)).any() and (fh >= 525).any()
    assert np.array_equal(a.state.cpu().numpy(), b.state.cpu().numpy())
    assert np.array_equal(fh, b.first_hit.cpu().numpy())
    assert np.array_equal(a.energy.cpu().numpy(), b.energy.cpu().numpy())
    assert (a.tts_sweeps, a.winner_clone) == (b.tts_sweeps, b.winner_clone)
    check_instance(inst, h, cfg, a, st, sorted(gf) + [5, nc // 32 - 2], f"n={n}")


@pytest.mark.parametrize("n,shape,nc", [
    (48, (4, 64, 16, 1), 2048), (64, (1, 64, 8, 1), 1024), (64, (4, 64, 16, 1), 1024),
    (200, (1, 256, 8, 1), 2048), (300, (1, 256, 8, 1), 1024), (200, (4, 64, 16, 1), 1024)])
def test_cross_sweep_body_every_clone(n, shape, nc):
    """Small instances with records in global memory, in shapes whose step cap has a cross-sweep
    body (64-thread workgroups run the launch-per-chunk kernel, 256-thread ones the persistent
    launch): every clone against the oracle over 61 sweeps in chunks of 7 (many clones reach a
    ground state, so replays and tracked chunks follow body chunks), and bit-identical to one
    sweep at a time."""
    _torch()
    B, T, C, G = shape
    inst = planted_instance(n, 5100 + n)
    h = xorsat.Instance(inst.tri, inst.J)
    assert h.body(T * C // (32 * B)) is not None
    outs = []
    for one in (False, True):
        cfg = xorsat.make_config(n_clones=nc, seed=n + 17, instance_id=n, accept_thr=THR_PAPER,
                                 max_sweeps=61, stop_on_first=False, chunk_sweeps=7,
                                 one_sweep_steps=one, tile_blocks=B, wg_threads=T, col_bytes=C,
                                 rec_global=G)
        outs.append((cfg, xorsat.run(h, cfg)))
    (cfg, a), (_, b) = outs
    assert (a.tile_blocks, a.wg_threads, a.col_bytes, a.rec_global) == shape
    assert a.end_sweep == 61
    for x, y in ((a.state, b.state), (a.first_hit, b.first_hit), (a.energy, b.energy)):
        assert np.array_equal(x.cpu().numpy(), y.cpu().numpy())
    operm, _ = oracle.colour(inst.tri, h.colour_cap)
    fh = a.first_hit.cpu().numpy()
    check_run_reduction(fh, a.tts_sweeps, a.winner_clone)
    check_clones(inst.tri, inst.J, operm, cfg, a.sweeps_done, np.arange(nc), fh,
                 a.energy.cpu().numpy(), a.state, what=f"n={n} shape={shape}")
