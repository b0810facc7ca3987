"""Python binding of libxorsat.so (include/xorsat.h): argument marshalling only.

Every step of the dynamics runs in the HIP library. torch supplies device buffers and the
stream; nothing here computes spins, energies or random numbers. If the library is not built
this module raises instead of falling back to anything else.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libxorsat.so")

XS_OK = 0
XS_STATUS = {0: "XS_OK", 1: "XS_EINVAL", 2: "XS_ENOMEM", 3: "XS_EDEVICE", 4: "XS_EAGAIN",
             5: "XS_ENOTFOUND", 6: "XS_ECANCELED"}
XS_STATUS_CODES = {v: k for k, v in XS_STATUS.items()}
XS_ENOTFOUND = 5
XS_STOP_ON_FIRST = 0x1
XS_RESUME = 0x2
XS_PLACE_ROWS = 0x4
XS_PER_CHUNK = 0x8
XS_ONE_SWEEP_STEPS = 0x10
XS_MAX_N = 2048
XS_CLONE_QUANTUM = 256
XS_MAX_CLONES = 0x7FFFFF00
XS_NOALLOC_SCRATCH_BYTES = 8 << 20

# Every function the header declares, for the export check.
EXPORTS = ["xs_abi_version", "xs_status_str", "xs_last_error", "xs_instance_create",
           "xs_instance_destroy", "xs_instance_get_info", "xs_instance_get_partition",
           "xs_instance_get_schedule", "xs_instance_get_body",
           "xs_run", "xs_run_batch", "xs_run_batch_noalloc", "xs_run_batch_async", "xs_wait",
           "xs_profile_enable", "xs_profile_read",
           "xs_autotune", "xs_tune_save", "xs_tune_load", "xs_tune_clear",
           "xs_server_create", "xs_server_destroy", "xs_server_submit", "xs_server_step",
           "xs_server_poll", "xs_server_cancel", "xs_server_get_stats"]
XS_TUNE_MAX_TRIALS = 64


class XsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{XS_STATUS.get(status, status)}: {message}")
        self.status = status


class RunConfig(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("instance_id", ctypes.c_uint32),
                ("seed", ctypes.c_uint64), ("n_clones", ctypes.c_uint32),
                ("accept_thr", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("max_sweeps", ctypes.c_uint32), ("start_sweep", ctypes.c_uint32),
                ("chunk_sweeps", ctypes.c_uint32), ("tile_blocks", ctypes.c_uint32),
                ("wg_threads", ctypes.c_uint32), ("col_bytes", ctypes.c_uint32),
                ("rec_global", ctypes.c_uint32), ("accept_thr0", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class RunBuffers(ctypes.Structure):
    _fields_ = [("state", ctypes.c_void_p), ("first_hit", ctypes.c_void_p),
                ("energy", ctypes.c_void_p), ("solved", ctypes.c_void_p)]


class RunResult(ctypes.Structure):
    _fields_ = [("tts_sweeps", ctypes.c_int64), ("winner_clone", ctypes.c_int32),
                ("end_sweep", ctypes.c_uint32), ("sweeps_done", ctypes.c_uint32),
                ("tile_blocks", ctypes.c_uint32), ("wg_threads", ctypes.c_uint32),
                ("col_bytes", ctypes.c_uint32), ("rec_global", ctypes.c_uint32),
                ("persistent", ctypes.c_uint32),
                ("clone_spin_updates", ctypes.c_uint64), ("seconds", ctypes.c_double)]


class KernelStats(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_uint64), ("total_ms", ctypes.c_double),
                ("clone_spin_updates", ctypes.c_uint64)]


class TuneTrial(ctypes.Structure):
    _fields_ = [("tile_blocks", ctypes.c_uint32), ("wg_threads", ctypes.c_uint32),
                ("col_bytes", ctypes.c_uint32), ("rec_global", ctypes.c_uint32),
                ("updates_per_ns", ctypes.c_double)]


class TuneResult(ctypes.Structure):
    _fields_ = [("tile_blocks", ctypes.c_uint32), ("wg_threads", ctypes.c_uint32),
                ("col_bytes", ctypes.c_uint32), ("rec_global", ctypes.c_uint32),
                ("updates_per_ns", ctypes.c_double), ("n_trials", ctypes.c_int32),
                ("trials", TuneTrial * XS_TUNE_MAX_TRIALS)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("max_resident", ctypes.c_uint32),
                ("hbm_budget_bytes", ctypes.c_uint64), ("max_pending", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]


class ServerOutputs(ctypes.Structure):
    _fields_ = [("state", ctypes.c_void_p), ("first_hit", ctypes.c_void_p),
                ("energy", ctypes.c_void_p), ("solved", ctypes.c_void_p)]


class ServerCompletion(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("result", RunResult), ("queued_s", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_uint64), ("admitted", ctypes.c_uint64),
                ("completed", ctypes.c_uint64), ("pending", ctypes.c_uint64),
                ("resident", ctypes.c_uint64), ("clone_spin_updates", ctypes.c_uint64),
                ("bytes_in_use", ctypes.c_uint64), ("step_seconds", ctypes.c_double)]


class InstanceInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("n_classes", ctypes.c_int32),
                ("colour_cap", ctypes.c_int32), ("max_class", ctypes.c_int32),
                ("n_levels", ctypes.c_int32), ("max_level", ctypes.c_int32)]


_lib = None


def load():
    """Load libxorsat.so (built in place by paper_2102_09510_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2102_09510_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32 = ctypes.c_int32
    lib.xs_abi_version.restype = i32
    lib.xs_status_str.argtypes = [i32]
    lib.xs_status_str.restype = ctypes.c_char_p
    lib.xs_last_error.restype = ctypes.c_char_p
    lib.xs_instance_create.argtypes = [i32, i32, P, P, i32, ctypes.POINTER(P)]
    lib.xs_instance_create.restype = i32
    lib.xs_instance_destroy.argtypes = [P]
    lib.xs_instance_destroy.restype = None
    lib.xs_instance_get_info.argtypes = [P, ctypes.POINTER(InstanceInfo)]
    lib.xs_instance_get_info.restype = i32
    lib.xs_instance_get_partition.argtypes = [P, P, P]
    lib.xs_instance_get_partition.restype = i32
    lib.xs_instance_get_schedule.argtypes = [P, ctypes.c_uint32, P, P, P]
    lib.xs_instance_get_schedule.restype = i32
    lib.xs_instance_get_body.argtypes = [P, ctypes.c_uint32, P, P, P, P]
    lib.xs_instance_get_body.restype = i32
    lib.xs_run.argtypes = [P, ctypes.POINTER(RunConfig), ctypes.POINTER(RunBuffers), P,
                           ctypes.POINTER(RunResult)]
    lib.xs_run.restype = i32
    lib.xs_run_batch.argtypes = [i32, P, P, P, P, P]
    lib.xs_run_batch.restype = i32
    lib.xs_run_batch_noalloc.argtypes = [i32, P, P, P, P, P]
    lib.xs_run_batch_noalloc.restype = i32
    lib.xs_run_batch_async.argtypes = [i32, P, P, P, P, P, ctypes.POINTER(P)]
    lib.xs_run_batch_async.restype = i32
    lib.xs_wait.argtypes = [P]
    lib.xs_wait.restype = i32
    lib.xs_autotune.argtypes = [P, ctypes.c_uint32, i32, P, ctypes.POINTER(TuneResult)]
    lib.xs_autotune.restype = i32
    lib.xs_tune_save.argtypes = [ctypes.c_char_p]
    lib.xs_tune_save.restype = i32
    lib.xs_tune_load.argtypes = [ctypes.c_char_p]
    lib.xs_tune_load.restype = i32
    lib.xs_tune_clear.argtypes = []
    lib.xs_tune_clear.restype = i32
    lib.xs_server_create.argtypes = [ctypes.POINTER(ServerConfig), P, ctypes.POINTER(P)]
    lib.xs_server_create.restype = i32
    lib.xs_server_destroy.argtypes = [P]
    lib.xs_server_destroy.restype = None
    lib.xs_server_submit.argtypes = [P, P, ctypes.POINTER(RunConfig),
                                     ctypes.POINTER(ServerOutputs), ctypes.POINTER(ctypes.c_uint64)]
    lib.xs_server_submit.restype = i32
    lib.xs_server_step.argtypes = [P, ctypes.POINTER(i32)]
    lib.xs_server_step.restype = i32
    lib.xs_server_poll.argtypes = [P, ctypes.POINTER(ServerCompletion), i32, ctypes.POINTER(i32)]
    lib.xs_server_poll.restype = i32
    lib.xs_server_cancel.argtypes = [P, ctypes.c_uint64]
    lib.xs_server_cancel.restype = i32
    lib.xs_server_get_stats.argtypes = [P, ctypes.POINTER(ServerStats)]
    lib.xs_server_get_stats.restype = i32
    lib.xs_profile_enable.argtypes = [i32]
    lib.xs_profile_enable.restype = i32
    lib.xs_profile_read.argtypes = [ctypes.POINTER(KernelStats), i32]
    lib.xs_profile_read.restype = i32
    _lib = lib
    return lib


def _check(status: int):
    if status != XS_OK:
        raise XsError(status, load().xs_last_error().decode())


class Instance:
    """An instance loaded into the library (host tables; device tables on first use)."""

    def __init__(self, tri, J, colour_cap: int = 32):
        lib = load()
        tri = np.ascontiguousarray(tri, dtype=np.int32).reshape(-1, 3)
        J = np.ascontiguousarray(J, dtype=np.int8)
        h = ctypes.c_void_p()
        _check(lib.xs_instance_create(tri.shape[0], J.shape[0], tri.ctypes.data,
                                      J.ctypes.data, colour_cap, ctypes.byref(h)))
        self._h = h
        info = InstanceInfo()
        _check(lib.xs_instance_get_info(h, ctypes.byref(info)))
        self.n = info.n
        self.n_classes = info.n_classes
        self.colour_cap = info.colour_cap
        self.max_class = info.max_class
        self.n_levels = info.n_levels
        self.max_level = info.max_level

    @property
    def handle(self):
        return self._h

    def partition(self):
        perm = np.zeros(self.n, dtype=np.int32)
        off = np.zeros(self.n_classes + 1, dtype=np.int32)
        _check(load().xs_instance_get_partition(self._h, perm.ctypes.data, off.ctypes.data))
        return perm, off

    def schedule(self, step_cap: int = 0):
        """The kernels' execution order for steps of at most step_cap spins: (order, step_off)."""
        order = np.zeros(self.n, dtype=np.int32)
        off = np.zeros(self.n + 1, dtype=np.int32)
        steps = ctypes.c_int32()
        _check(load().xs_instance_get_schedule(self._h, step_cap, order.ctypes.data,
                                               off.ctypes.data, ctypes.byref(steps)))
        return order, off[: steps.value + 1].copy()

    def body(self, step_cap: int):
        """The cross-sweep body for steps of at most step_cap spins: (order, step_off, late), or
        None if the instance has none for that cap."""
        order = np.zeros(self.n, dtype=np.int32)
        off = np.zeros(self.n + 1, dtype=np.int32)
        late = np.zeros(self.n, dtype=np.uint8)
        steps = ctypes.c_int32()
        st = load().xs_instance_get_body(self._h, step_cap, order.ctypes.data, off.ctypes.data,
                                         late.ctypes.data, ctypes.byref(steps))
        if st == XS_ENOTFOUND:
            return None
        _check(st)
        return order, off[: steps.value + 1].copy(), late

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().xs_instance_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class RunOutput:
    tts_sweeps: int
    winner_clone: int
    end_sweep: int
    sweeps_done: int
    tile_blocks: int
    wg_threads: int
    col_bytes: int
    rec_global: int
    persistent: int
    clone_spin_updates: int
    seconds: float
    state: object        # torch int64 [n][n_clones/64] on the device
    first_hit: object    # torch int32 [n_clones]
    energy: object       # torch int32 [n_clones] or None
    solved: np.ndarray | None  # int8 [n] (+1/-1) of the winner, None if no clone hit


def make_config(*, n_clones: int, seed: int, instance_id: int = 0, accept_thr: int = 3604,
                max_sweeps: int = 100000, stop_on_first: bool = True, resume: bool = False,
                start_sweep: int = 0, chunk_sweeps: int = 0, tile_blocks: int = 0,
                wg_threads: int = 0, col_bytes: int = 0, rec_global: int = 0,
                accept_thr0: int = 0, place_rows: bool = False,
                per_chunk: bool = False, one_sweep_steps: bool = False) -> RunConfig:
    """accept_thr0 > 0 selects the rule with w0 = accept_thr0 / 65536 (no ground-state
    tracking: first_hit marks only clones whose end configuration is a ground state).
    place_rows builds the LDS row placement even for a short run (speed only)."""
    flags = ((XS_STOP_ON_FIRST if stop_on_first else 0) | (XS_RESUME if resume else 0) |
             (XS_PLACE_ROWS if place_rows else 0) | (XS_PER_CHUNK if per_chunk else 0) |
             (XS_ONE_SWEEP_STEPS if one_sweep_steps else 0))
    return RunConfig(ctypes.sizeof(RunConfig), instance_id, seed & (2**64 - 1), n_clones,
                     accept_thr, flags, max_sweeps, start_sweep, chunk_sweeps, tile_blocks,
                     wg_threads, col_bytes, rec_global, accept_thr0, 0)


def _buffers(inst: Instance, cfg: RunConfig, state, want_energy: bool, device):
    import torch
    n, nc = inst.n, cfg.n_clones
    if state is None:
        state = torch.empty((n, nc // 64), dtype=torch.int64, device=device)
    elif (state.dtype != torch.int64 or tuple(state.shape) != (n, nc // 64)
          or not state.is_contiguous() or state.device.type != "cuda"):
        raise ValueError(f"state must be a contiguous int64 device tensor of shape "
                         f"({n}, {nc // 64})")
    first_hit = torch.empty(nc, dtype=torch.int32, device=device)
    energy = torch.empty(nc, dtype=torch.int32, device=device) if want_energy else None
    solved = np.zeros(n, dtype=np.int8)
    bufs = RunBuffers(state.data_ptr(), first_hit.data_ptr(),
                      energy.data_ptr() if energy is not None else None, solved.ctypes.data)
    return bufs, state, first_hit, energy, solved


def _output(res: RunResult, state, first_hit, energy, solved) -> RunOutput:
    return RunOutput(int(res.tts_sweeps), int(res.winner_clone), int(res.end_sweep),
                     int(res.sweeps_done), int(res.tile_blocks), int(res.wg_threads),
                     int(res.col_bytes), int(res.rec_global), int(res.persistent),
                     int(res.clone_spin_updates),
                     float(res.seconds), state, first_hit, energy,
                     solved if res.winner_clone >= 0 else None)


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def run(inst: Instance, cfg: RunConfig, *, state=None, want_energy: bool = True,
        device="cuda") -> RunOutput:
    """xs_run on torch-owned device buffers (state is drawn unless cfg has XS_RESUME)."""
    bufs, state, fh, en, solved = _buffers(inst, cfg, state, want_energy, device)
    res = RunResult()
    _check(load().xs_run(inst.handle, ctypes.byref(cfg), ctypes.byref(bufs), _stream(),
                         ctypes.byref(res)))
    return _output(res, state, fh, en, solved)


def run_batch(insts: list[Instance], cfgs: list[RunConfig], *, states=None,
              want_energy: bool = True, device="cuda") -> list[RunOutput]:
    """xs_run_batch over several instances (one chunk launch covers all of them)."""
    count = len(insts)
    if count == 0 or count != len(cfgs):
        raise ValueError(f"need one config per instance and at least one instance "
                         f"({count} instances, {len(cfgs)} configs)")
    states = states or [None] * count
    made = [_buffers(i, c, s, want_energy, device) for i, c, s in zip(insts, cfgs, states)]
    handles = (ctypes.c_void_p * count)(*[i.handle.value for i in insts])
    cfg_arr = (RunConfig * count)(*cfgs)
    buf_arr = (RunBuffers * count)(*[m[0] for m in made])
    res_arr = (RunResult * count)()
    _check(load().xs_run_batch(count, handles, cfg_arr, buf_arr, _stream(), res_arr))
    return [_output(res_arr[k], *made[k][1:]) for k in range(count)]


def run_batch_noalloc(insts: list[Instance], cfgs: list[RunConfig], *, states=None,
                      want_energy: bool = True, device="cuda") -> list[RunOutput]:
    """xs_run_batch_noalloc: the batch with the library's fixed device scratch (no device
    allocation inside the call; torch allocates the caller's output buffers here)."""
    count = len(insts)
    if count == 0 or count != len(cfgs):
        raise ValueError(f"need one config per instance and at least one instance "
                         f"({count} instances, {len(cfgs)} configs)")
    states = states or [None] * count
    made = [_buffers(i, c, s, want_energy, device) for i, c, s in zip(insts, cfgs, states)]
    handles = (ctypes.c_void_p * count)(*[i.handle.value for i in insts])
    cfg_arr = (RunConfig * count)(*cfgs)
    buf_arr = (RunBuffers * count)(*[m[0] for m in made])
    res_arr = (RunResult * count)()
    _check(load().xs_run_batch_noalloc(count, handles, cfg_arr, buf_arr, _stream(), res_arr))
    return [_output(res_arr[k], *made[k][1:]) for k in range(count)]


class Pending:
    """An asynchronous batch (xs_run_batch_async): keeps the buffers alive until wait()."""

    def __init__(self, handle, made, res_arr):
        self._h, self._made, self._res = handle, made, res_arr

    def wait(self) -> list[RunOutput]:
        if self._h is None:
            raise RuntimeError("already waited")
        h, self._h = self._h, None
        _check(load().xs_wait(h))
        return [_output(self._res[k], *self._made[k][1:]) for k in range(len(self._made))]


def run_batch_async(insts: list[Instance], cfgs: list[RunConfig], *, want_energy: bool = True,
                    device="cuda", stream=None) -> Pending:
    """xs_run_batch_async: returns at once; Pending.wait() gives the outputs. `stream` (a torch
    stream) must not be used until then; default: the current stream."""
    count = len(insts)
    if count == 0 or count != len(cfgs):
        raise ValueError(f"need one config per instance and at least one instance "
                         f"({count} instances, {len(cfgs)} configs)")
    made = [_buffers(i, c, None, want_energy, device) for i, c in zip(insts, cfgs)]
    handles = (ctypes.c_void_p * count)(*[i.handle.value for i in insts])
    cfg_arr = (RunConfig * count)(*cfgs)
    buf_arr = (RunBuffers * count)(*[m[0] for m in made])
    res_arr = (RunResult * count)()
    s = _stream() if stream is None else ctypes.c_void_p(stream.cuda_stream)
    h = ctypes.c_void_p()
    _check(load().xs_run_batch_async(count, handles, cfg_arr, buf_arr, s, res_arr,
                                     ctypes.byref(h)))
    return Pending(h, made, res_arr)


def profile_enable(on: bool = True):
    """Time every sweep-chunk launch with HIP events on the run's stream."""
    _check(load().xs_profile_enable(1 if on else 0))


def profile_read(reset: bool = False) -> dict:
    st = KernelStats()
    _check(load().xs_profile_read(ctypes.byref(st), 1 if reset else 0))
    return dict(launches=int(st.launches), total_ms=float(st.total_ms),
                clone_spin_updates=int(st.clone_spin_updates))


def autotune(inst: Instance, n_clones: int, count: int = 1) -> dict:
    """Time every valid (tile_blocks, wg_threads) pair for `count` instances like `inst` and
    record the fastest for later runs that leave both knobs at 0."""
    res = TuneResult()
    _check(load().xs_autotune(inst.handle, n_clones, count, _stream(), ctypes.byref(res)))
    trials = [(res.trials[k].tile_blocks, res.trials[k].wg_threads, res.trials[k].col_bytes,
               res.trials[k].rec_global, res.trials[k].updates_per_ns)
              for k in range(res.n_trials)]
    return dict(tile_blocks=res.tile_blocks, wg_threads=res.wg_threads,
                col_bytes=res.col_bytes, rec_global=res.rec_global,
                updates_per_ns=res.updates_per_ns, trials=trials)


def tune_save(path: str):
    _check(load().xs_tune_save(path.encode()))


def tune_load(path: str):
    _check(load().xs_tune_load(path.encode()))


def tune_clear():
    _check(load().xs_tune_clear())


@dataclass
class Completion:
    ticket: int
    status: int
    tts_sweeps: int
    winner_clone: int
    end_sweep: int
    sweeps_done: int
    clone_spin_updates: int
    latency_s: float   # submission to completion
    queued_s: float    # submission to admission
    outputs: dict      # host numpy arrays given at submission (state, first_hit, energy, solved)


class Server:
    """Continuous-batching server (xs_server_*). Host numpy buffers receive each request's
    outputs when it completes."""

    def __init__(self, hbm_budget_bytes: int, max_resident: int = 0, max_pending: int = 0):
        cfg = ServerConfig(ctypes.sizeof(ServerConfig), max_resident, hbm_budget_bytes,
                           max_pending, 0)
        h = ctypes.c_void_p()
        _check(load().xs_server_create(ctypes.byref(cfg), _stream(), ctypes.byref(h)))
        self._h = h
        self._outs = {}  # ticket -> (instance, dict of numpy buffers) kept alive until done

    def submit(self, inst: Instance, cfg: RunConfig, *, want_state: bool = False,
               want_first_hit: bool = True, want_energy: bool = True) -> int:
        n, nc = inst.n, cfg.n_clones
        bufs = {"solved": np.zeros(n, dtype=np.int8)}
        if want_state:
            bufs["state"] = np.zeros((n, nc // 64), dtype=np.uint64)
        if want_first_hit:
            bufs["first_hit"] = np.zeros(nc, dtype=np.int32)
        if want_energy:
            bufs["energy"] = np.zeros(nc, dtype=np.int32)
        outs = ServerOutputs(*(bufs[k].ctypes.data if k in bufs else None
                               for k in ("state", "first_hit", "energy", "solved")))
        t = ctypes.c_uint64()
        _check(load().xs_server_submit(self._h, inst.handle, ctypes.byref(cfg),
                                       ctypes.byref(outs), ctypes.byref(t)))
        self._outs[t.value] = (inst, bufs)
        return t.value

    def step(self) -> int:
        n = ctypes.c_int32()
        _check(load().xs_server_step(self._h, ctypes.byref(n)))
        return n.value

    def poll(self, cap: int = 1024) -> list[Completion]:
        arr = (ServerCompletion * cap)()
        n = ctypes.c_int32()
        _check(load().xs_server_poll(self._h, arr, cap, ctypes.byref(n)))
        out = []
        for k in range(n.value):
            c = arr[k]
            _, bufs = self._outs.pop(c.ticket)
            if c.result.winner_clone < 0:
                bufs["solved"] = None
            out.append(Completion(int(c.ticket), int(c.status), int(c.result.tts_sweeps),
                                  int(c.result.winner_clone), int(c.result.end_sweep),
                                  int(c.result.sweeps_done), int(c.result.clone_spin_updates),
                                  float(c.result.seconds), float(c.queued_s), bufs))
        return out

    def cancel(self, ticket: int):
        _check(load().xs_server_cancel(self._h, ticket))

    def stats(self) -> dict:
        st = ServerStats()
        _check(load().xs_server_get_stats(self._h, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().xs_server_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
