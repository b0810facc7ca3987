"""GPU tests of the continuous-batching server and of the autotuner: every request's result is
bit-identical alone (xs_run) and in the mix; tuned launch knobs change speed only."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2102_09510_amd import xorsat
from paper_2102_09510_amd.instances import planted_instance
from tests.parity import check_clones, check_run_reduction, group_sample

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


REQS = [  # (n, clones, max_sweeps, stop_on_first, chunk)
    (64, 1024, 3000, True, 100),
    (200, 2048, 60, False, 25),
    (48, 512, 500, True, 7),
    (512, 1024, 30, False, 100),
    (33, 256, 400, True, 50),
    (1024, 512, 12, False, 5),
    (96, 4096, 80, False, 30),
    (2048, 16384, 20, False, 7),  # the largest N of the served stream, at its clone count
]


def _make(k, spec):
    n, nc, sweeps, stop, chunk = spec
    inst = planted_instance(n, 7000 + k)
    h = xorsat.Instance(inst.tri, inst.J)
    cfg = xorsat.make_config(n_clones=nc, seed=900 + k, instance_id=k, max_sweeps=sweeps,
                             stop_on_first=stop, chunk_sweeps=chunk)
    return inst, h, cfg


def _alone(h, cfg):
    out = xorsat.run(h, cfg)
    st = out.state.cpu().numpy().view(np.uint64)
    return out, st, out.first_hit.cpu().numpy(), out.energy.cpu().numpy()


def oracle_check_completion(k, c, inst, h, cfg):
    """Sampled groups of a completed request (two groups, the winner's group and the last
    clone) against the oracle, from the host outputs the server filled."""
    perm, _ = h.partition()
    operm, _ = oracle.colour(inst.tri, h.colour_cap)
    assert np.array_equal(perm, operm)
    fh = c.outputs["first_hit"]
    check_run_reduction(fh, c.tts_sweeps, c.winner_clone)
    rng = np.random.default_rng(k)
    groups = list(rng.choice(cfg.n_clones // 32, size=2, replace=False))
    if c.winner_clone >= 0:
        groups.append(c.winner_clone // 32)
    clones = np.unique(np.r_[group_sample(cfg.n_clones, groups), cfg.n_clones - 1])
    ref = check_clones(inst.tri, inst.J, operm, cfg, c.sweeps_done, clones, fh,
                       c.outputs["energy"], c.outputs["state"], what=f"request {k}")
    if c.winner_clone >= 0:
        w = int(np.flatnonzero(clones == c.winner_clone)[0])
        assert np.array_equal(c.outputs["solved"], ref["final_spins"][w])


def test_server_results_equal_alone():
    """Requests submitted in three waves while others are resident: every completion equals the
    oracle on sampled clones and its run alone (xs_run) bit for bit."""
    _torch()
    made = [_make(k, s) for k, s in enumerate(REQS)]
    srv = xorsat.Server(hbm_budget_bytes=1 << 30)
    tickets = {}
    # staggered arrivals: two waves submitted while others are already resident
    for k in (0, 1, 2):
        tickets[srv.submit(made[k][1], made[k][2], want_state=True)] = k
    srv.step()
    srv.step()
    for k in (3, 4):
        tickets[srv.submit(made[k][1], made[k][2], want_state=True)] = k
    srv.step()
    for k in (5, 6, 7):
        tickets[srv.submit(made[k][1], made[k][2], want_state=True)] = k
    done = []
    for _ in range(10000):
        active = srv.step()
        done += srv.poll()
        if active == 0:
            break
    done += srv.poll()
    assert sorted(c.ticket for c in done) == sorted(tickets)
    for c in done:
        k = tickets[c.ticket]
        inst, h, cfg = made[k]
        assert c.status == 0
        oracle_check_completion(k, c, inst, h, cfg)
        out, st, fh, en = _alone(h, cfg)
        assert (c.tts_sweeps, c.winner_clone, c.end_sweep, c.sweeps_done) == \
            (out.tts_sweeps, out.winner_clone, out.end_sweep, out.sweeps_done), k
        assert np.array_equal(c.outputs["state"], st), k
        assert np.array_equal(c.outputs["first_hit"], fh), k
        assert np.array_equal(c.outputs["energy"], en), k
        if out.winner_clone >= 0:
            assert np.array_equal(c.outputs["solved"], out.solved)
        assert c.latency_s >= c.queued_s >= 0
    stats = srv.stats()
    assert stats["completed"] == len(REQS) and stats["resident"] == 0
    assert stats["bytes_in_use"] == 0
    srv.close()


ENDING_TOGETHER = [  # (n, clones): mixed sizes, so the gathered final pass spans unlike grids
    (48, 256), (96, 1024), (200, 4096), (512, 512), (1024, 2048), (2048, 16384), (33, 768),
    (64, 1024), (300, 8192), (128, 256), (1500, 1024), (80, 2048),
]


def test_server_requests_ending_in_the_same_step():
    """Twelve requests of unlike N and clone count with the same budget and chunk, submitted
    together, end in the same step and share one final pass: each equals its run alone bit for
    bit and the oracle on sampled clones."""
    _torch()
    made = []
    for k, (n, nc) in enumerate(ENDING_TOGETHER):
        inst = planted_instance(n, 8100 + k)
        h = xorsat.Instance(inst.tri, inst.J)
        cfg = xorsat.make_config(n_clones=nc, seed=4400 + k, instance_id=k, max_sweeps=40,
                                 stop_on_first=False, chunk_sweeps=20)
        made.append((inst, h, cfg))
    srv = xorsat.Server(hbm_budget_bytes=1 << 30)
    tickets = {srv.submit(h, cfg, want_state=True): k for k, (_, h, cfg) in enumerate(made)}
    per_step = []
    for _ in range(10):
        active = srv.step()
        per_step.append(srv.poll())
        if active == 0:
            break
    assert [len(p) for p in per_step] == [0, len(made)]
    for c in per_step[-1]:
        k = tickets[c.ticket]
        inst, h, cfg = made[k]
        assert c.status == 0 and c.end_sweep == 40
        oracle_check_completion(k, c, inst, h, cfg)
        out, st, fh, en = _alone(h, cfg)
        assert (c.tts_sweeps, c.winner_clone) == (out.tts_sweeps, out.winner_clone), k
        assert np.array_equal(c.outputs["state"], st), k
        assert np.array_equal(c.outputs["first_hit"], fh), k
        assert np.array_equal(c.outputs["energy"], en), k
    srv.close()


def test_server_admission_by_footprint_and_cancel():
    _torch()
    made = [_make(k, s) for k, s in enumerate(REQS[:3])]
    # footprint of request 1 (n=200, 2048 clones): 51200 + 2*8192 + 256 bytes, rounded to 256
    srv = xorsat.Server(hbm_budget_bytes=80_000, max_resident=2)
    t = [srv.submit(h, cfg) for _, h, cfg in made]
    big = planted_instance(2048, 1)
    hb = xorsat.Instance(big.tri, big.J)
    t_big = srv.submit(hb, xorsat.make_config(n_clones=1024, seed=1, max_sweeps=5))
    t_cancel = srv.submit(made[0][1], made[0][2])
    srv.cancel(t_cancel)
    seen_resident = 0
    done = []
    for _ in range(10000):
        active = srv.step()
        seen_resident = max(seen_resident, srv.stats()["resident"])
        assert srv.stats()["bytes_in_use"] <= 80_000
        done += srv.poll()
        if active == 0:
            break
    by = {c.ticket: c for c in done}
    assert by[t_cancel].status == xorsat.XS_STATUS_CODES["XS_ECANCELED"]
    assert by[t_big].status == xorsat.XS_STATUS_CODES["XS_ENOMEM"]
    for k, tk in enumerate(t):
        out, _, fh, en = _alone(made[k][1], made[k][2])
        assert by[tk].status == 0
        assert np.array_equal(by[tk].outputs["first_hit"], fh)
        assert np.array_equal(by[tk].outputs["energy"], en)
    assert 1 <= seen_resident <= 2
    with pytest.raises(xorsat.XsError):
        srv.cancel(t[0])  # already completed
    srv.close()


def test_server_back_pressure():
    """With max_pending set, a submit beyond the queue limit is refused with XS_EAGAIN and
    accepted again once a step has admitted the waiting requests."""
    _torch()
    made = [_make(k, s) for k, s in enumerate(REQS[:3])]
    srv = xorsat.Server(hbm_budget_bytes=1 << 30, max_pending=2)
    t = [srv.submit(h, cfg) for _, h, cfg in made[:2]]
    with pytest.raises(xorsat.XsError) as e:
        srv.submit(made[2][1], made[2][2])
    assert e.value.status == xorsat.XS_STATUS_CODES["XS_EAGAIN"]
    srv.step()  # admits both
    t.append(srv.submit(made[2][1], made[2][2]))
    done = []
    for _ in range(10000):
        active = srv.step()
        done += srv.poll()
        if active == 0:
            break
    done += srv.poll()
    by = {c.ticket: c for c in done}
    for k, tk in enumerate(t):
        _, fh, en = _alone(made[k][1], made[k][2])[1:]
        assert by[tk].status == 0
        assert np.array_equal(by[tk].outputs["first_hit"], fh)
        assert np.array_equal(by[tk].outputs["energy"], en)
    srv.close()


def test_autotune_is_result_neutral():
    """A tuned batch runs the tuned launch knobs, equals the same batch at fixed knobs bit for
    bit, and every clone of two of its runs equals the oracle."""
    torch = _torch()
    inst = planted_instance(128, 17)
    h = xorsat.Instance(inst.tri, inst.J)
    try:
        res = xorsat.autotune(h, 8192, count=4)
        assert res["updates_per_ns"] > 0 and len(res["trials"]) >= 4
        assert (res["tile_blocks"], res["wg_threads"], res["col_bytes"], res["rec_global"]) in \
            [(b, t, c, g) for b, t, c, g, _ in res["trials"]]
        cfgs = [xorsat.make_config(n_clones=8192, seed=5 + k, instance_id=k, max_sweeps=120,
                                   stop_on_first=False, chunk_sweeps=40) for k in range(4)]
        tuned = xorsat.run_batch([h] * 4, cfgs)
        assert all((o.tile_blocks, o.wg_threads, o.col_bytes) ==
                   (res["tile_blocks"], res["wg_threads"], res["col_bytes"]) for o in tuned)
        assert all(o.rec_global == (res["rec_global"] == 1) for o in tuned)
        perm, _ = h.partition()
        operm, _ = oracle.colour(inst.tri, h.colour_cap)
        assert np.array_equal(perm, operm)
        for k in (0, 3):
            o = tuned[k]
            check_run_reduction(o.first_hit.cpu().numpy(), o.tts_sweeps, o.winner_clone)
            check_clones(inst.tri, inst.J, operm, cfgs[k], o.sweeps_done, np.arange(8192),
                         o.first_hit.cpu().numpy(), o.energy.cpu().numpy(), o.state,
                         what=f"tuned run {k}")
        for k, c in enumerate(cfgs):
            c.tile_blocks, c.wg_threads, c.col_bytes, c.rec_global = 1, 64, 16, 2
        plain = xorsat.run_batch([h] * 4, cfgs)
        for a, b in zip(tuned, plain):
            assert torch.equal(a.state, b.state)
            assert torch.equal(a.first_hit, b.first_hit)
            assert torch.equal(a.energy, b.energy)
    finally:
        xorsat.tune_clear()
