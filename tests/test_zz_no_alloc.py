"""xs_run_batch_noalloc (the entry point for callers that cannot allocate device memory)
against xs_run_batch, through the C ABI: two calls in a row, the second on a smaller batch,
each compared with the allocating entry point on the same instances, seeds and starts, buffer
by buffer (end state, first hits, energies) and result by result. All integer, so the bar is
exact equality. Also: a batch whose device scratch would exceed the fixed array is rejected
before any launch, and the smaller call still matches the oracle on sampled clones."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

import oracle
from paper_2102_09510_amd import xorsat
from paper_2102_09510_amd.instances import THR_PAPER, planted_instance
from tests.parity import check_clones, check_run_reduction

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _raw_batch(fn, handles, cfgs, want_energy=True):
    """Call a batch entry point of the C ABI directly on fresh torch buffers."""
    torch = _torch()
    count = len(handles)
    outs = []
    for h, c in zip(handles, cfgs):
        n, nc = h.n, c.n_clones
        st = torch.empty((n, nc // 64), dtype=torch.int64, device="cuda")
        fh = torch.empty(nc, dtype=torch.int32, device="cuda")
        en = torch.empty(nc, dtype=torch.int32, device="cuda") if want_energy else None
        solved = np.zeros(n, dtype=np.int8)
        outs.append((st, fh, en, solved))
    hs = (ctypes.c_void_p * count)(*[h.handle.value for h in handles])
    cfg_arr = (xorsat.RunConfig * count)(*cfgs)
    buf_arr = (xorsat.RunBuffers * count)(*[
        xorsat.RunBuffers(o[0].data_ptr(), o[1].data_ptr(),
                          o[2].data_ptr() if o[2] is not None else None, o[3].ctypes.data)
        for o in outs])
    res = (xorsat.RunResult * count)()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    status = fn(count, hs, cfg_arr, buf_arr, stream, res)
    return status, outs, [res[k] for k in range(count)]


RESULT_FIELDS = ("tts_sweeps", "winner_clone", "end_sweep", "sweeps_done", "tile_blocks",
                 "wg_threads", "col_bytes", "rec_global", "clone_spin_updates")


def _compare(lib, handles, cfgs, what):
    """The no-allocation call against xs_run_batch: equal results and buffers."""
    st_a, out_a, res_a = _raw_batch(lib.xs_run_batch, handles, cfgs)
    assert st_a == xorsat.XS_OK, lib.xs_last_error().decode()
    st_b, out_b, res_b = _raw_batch(lib.xs_run_batch_noalloc, handles, cfgs)
    assert st_b == xorsat.XS_OK, lib.xs_last_error().decode()
    for k in range(len(handles)):
        for f in RESULT_FIELDS:
            assert getattr(res_a[k], f) == getattr(res_b[k], f), (what, k, f)
        for a, b, name in zip(out_a[k][:3], out_b[k][:3], ("state", "first_hit", "energy")):
            assert torch_equal(a, b), (what, k, name)
        assert np.array_equal(out_a[k][3], out_b[k][3]), (what, k, "solved")
    return out_b, res_b


def torch_equal(a, b):
    import torch
    return bool(torch.equal(a, b))


def test_noalloc_matches_batch_on_two_calls_second_smaller():
    _torch()
    lib = xorsat.load()
    print("# no-alloc: first call, 3 instances N = 256/1024/512", flush=True)
    insts = [planted_instance(256, 8100), planted_instance(1024, 8101),
             planted_instance(512, 8102)]
    handles = [xorsat.Instance(i.tri, i.J) for i in insts]
    clones = [65536, 1 << 18, 16384]
    cfgs = [xorsat.make_config(n_clones=c, seed=0x5151 + k, instance_id=k,
                               accept_thr=THR_PAPER, max_sweeps=300, stop_on_first=False,
                               chunk_sweeps=100)
            for k, c in enumerate(clones)]
    _compare(lib, handles, cfgs, "first call")

    print("# no-alloc: second call, 1 instance N = 64, 1024 clones to first ground state",
          flush=True)
    small = planted_instance(64, 1000001)
    hs = xorsat.Instance(small.tri, small.J)
    cfg = xorsat.make_config(n_clones=1024, seed=1, instance_id=0, accept_thr=THR_PAPER,
                             max_sweeps=2000, stop_on_first=True, chunk_sweeps=50)
    out, res = _compare(lib, [hs], [cfg], "second call")
    st, fh, en, _ = out[0]
    fh_np = fh.cpu().numpy()
    check_run_reduction(fh_np, res[0].tts_sweeps, res[0].winner_clone)
    operm, _ = oracle.colour(small.tri, 32)
    check_clones(small.tri, small.J, operm, cfg, res[0].sweeps_done, np.arange(1024), fh_np,
                 en.cpu().numpy(), st, what="second call vs oracle")


def test_noalloc_rejects_a_batch_beyond_its_scratch():
    _torch()
    lib = xorsat.load()
    print("# no-alloc: oversized batch (scratch check before any launch)", flush=True)
    inst = planted_instance(2048, 8200)
    # Distinct instance handles each get their own tables in the scratch: per handle about
    # 80 KB (triplets 16 KB, records 32 KB, global-memory records 32 KB, step offsets), so 120
    # of them need more than the 8 MiB array.
    count = 120
    handles = [xorsat.Instance(inst.tri, inst.J) for _ in range(count)]
    cfgs = [xorsat.make_config(n_clones=256, seed=k, instance_id=k, max_sweeps=10,
                               stop_on_first=False, tile_blocks=1, rec_global=1)
            for k in range(count)]
    assert count * 80 * 1024 > xorsat.XS_NOALLOC_SCRATCH_BYTES
    status, _, _ = _raw_batch(lib.xs_run_batch_noalloc, handles, cfgs, want_energy=False)
    assert status == xorsat.XS_STATUS_CODES["XS_EINVAL"]
    msg = lib.xs_last_error().decode()
    assert "bytes of device scratch" in msg, msg
    # the same batch minus most handles fits and matches xs_run_batch
    _compare(lib, handles[:8], cfgs[:8], "after the rejection")
