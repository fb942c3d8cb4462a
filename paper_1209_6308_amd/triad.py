"""Python binding of ``libtriad.so`` (include/triad.h): argument marshalling only.

Every step of the census runs in the library's HIP kernels. There is no CPU
fallback: if the library is missing or no HIP device is present, the calls
raise. PyTorch is used for device memory and streams only.

Functions mirror the C entry points:

* :func:`triad_census`         host arrays in, census out (blocking)
* :func:`triad_census_device`  torch device tensors in, census out
* :func:`triad_validate_host`  contract check on the host (no device needed)
* batched plans, the autotuner and the learned-schedule entry points below
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import _build

TYPES = ["003", "012", "102", "021D", "021U", "021C", "111D", "111U",
         "030T", "030C", "201", "120D", "120U", "120C", "210", "300"]

OK, OK_003_WRAPPED = 0, 1
EINVAL, EUNSORTED, ESELFLOOP, EASYM, ERANGE, ENOMEM, EDEVICE = -1, -2, -3, -4, -5, -6, -7
STATUS_NAMES = {0: "TRIAD_OK", 1: "TRIAD_OK_003_WRAPPED", -1: "TRIAD_EINVAL", -2: "TRIAD_EUNSORTED",
                -3: "TRIAD_ESELFLOOP", -4: "TRIAD_EASYM", -5: "TRIAD_ERANGE", -6: "TRIAD_ENOMEM",
                -7: "TRIAD_EDEVICE"}
SCHED = {"plain": 0, "heuristic": 1, "learned": 2}
MLP_IN, MLP_HIDDEN = 6, 32
MLP_PARAMS = MLP_HIDDEN * MLP_IN + MLP_HIDDEN + MLP_HIDDEN * MLP_HIDDEN + MLP_HIDDEN + MLP_HIDDEN + 1

EXPORTS = [
    "triad_census", "triad_census_ex", "triad_census_device", "triad_census_device_noalloc",
    "triad_labelled_census_device", "triad_validate_host",
    "triad_batch_plan_create", "triad_batch_plan_launch", "triad_batch_plan_status",
    "triad_batch_plan_destroy", "triad_census_batch", "triad_batch_autotune",
    "triad_csr_from_arcs", "triad_census_update", "triad_significance_profile", "triad_task_features", "triad_mlp_forward", "triad_mlp_loss_grad", "triad_mlp_adam",
    "triad_mlp_train", "triad_last_error", "triad_version", "triad_set_memory_cap",
    "triad_test_inject_device_error", "triad_held_memory", "triad_release_memory",
]


class TriadError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Timing(ctypes.Structure):
    _fields_ = [("prep_ms", ctypes.c_float), ("tasks_ms", ctypes.c_float), ("census_ms", ctypes.c_float),
                ("finalize_ms", ctypes.c_float), ("tasks", ctypes.c_int64), ("hub_tasks", ctypes.c_int64),
                ("items", ctypes.c_int64), ("waves", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Opts(ctypes.Structure):
    _fields_ = [("schedule", ctypes.c_int32), ("validate", ctypes.c_int32), ("hub_threshold", ctypes.c_int64),
                ("chunk", ctypes.c_int64), ("model", ctypes.c_void_p), ("task_cycles", ctypes.c_void_p),
                ("timing", ctypes.POINTER(Timing)), ("waves_per_group", ctypes.c_int32),
                ("grid_groups", ctypes.c_int32), ("kernel_variant", ctypes.c_int32),
                ("wave_span", ctypes.c_void_p), ("tail_share", ctypes.c_int32), ("short_tasks", ctypes.c_int32)]


_LIB = None


def lib():
    """Load libtriad.so (built by __graft_entry__.build()); raises if absent."""
    global _LIB
    if _LIB is None:
        path = _build.triad_lib_path()
        if not os.path.exists(path):
            raise ImportError(f"{path} is not built; run __graft_entry__.build() first")
        L = ctypes.CDLL(path)
        i64, i32, vp, u64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_uint64
        po = ctypes.POINTER(Opts)
        sigs = {
            "triad_census": [i64, vp, vp, vp, vp],
            "triad_census_ex": [i64, vp, vp, vp, po, vp, vp],
            "triad_census_device": [i64, i64, vp, vp, vp, po, vp, vp, vp],
            "triad_census_device_noalloc": [i64, i64, vp, vp, vp, po, vp, vp, vp],
            "triad_labelled_census_device": [i64, i64, vp, vp, vp, po, vp, vp, vp],
            "triad_validate_host": [i64, vp, vp, vp, i32],
            "triad_batch_plan_create": [i32, i64, i64, vp, vp, vp, vp, vp, po, vp, ctypes.POINTER(vp)],
            "triad_batch_plan_launch": [vp, vp],
            "triad_batch_plan_status": [vp],
            "triad_batch_plan_destroy": [vp],
            "triad_census_batch": [i32, i64, i64, vp, vp, vp, vp, po, vp, vp],
            "triad_batch_autotune": [i32, i64, i64, vp, vp, vp, vp, vp, ctypes.c_char_p, po],
            "triad_csr_from_arcs": [i64, i64, vp, vp, vp, vp, vp, vp, ctypes.POINTER(i64),
                                    ctypes.POINTER(ctypes.c_float)],
            "triad_census_update": [i64, i64, vp, vp, vp, i64, vp, vp, vp, vp, vp, vp, vp, vp,
                                    ctypes.POINTER(i64), ctypes.POINTER(i64), vp],
            "triad_significance_profile": [i32, vp, vp, vp, vp, vp],
            "triad_task_features": [i64, i64, vp, vp, vp, vp, ctypes.POINTER(i64)],
            "triad_mlp_forward": [vp, vp, i64, vp, vp],
            "triad_mlp_loss_grad": [vp, vp, vp, i64, vp, vp, vp],
            "triad_mlp_adam": [vp, vp, vp, vp, i32, ctypes.c_float, vp],
            "triad_mlp_train": [vp, vp, vp, i64, i32, i32, ctypes.c_float, u64, vp, vp],
            "triad_last_error": [],
            "triad_version": [],
            "triad_set_memory_cap": [i64],
            "triad_test_inject_device_error": [i32],
            "triad_release_memory": [],
        }
        for name, args in sigs.items():
            if hasattr(L, name):
                fn = getattr(L, name)
                fn.argtypes = args
                fn.restype = ctypes.c_int
        L.triad_last_error.restype = ctypes.c_char_p
        if hasattr(L, "triad_held_memory"):
            L.triad_held_memory.argtypes = []
            L.triad_held_memory.restype = ctypes.c_int64
        if hasattr(L, "triad_batch_plan_destroy"):
            L.triad_batch_plan_destroy.restype = None
        _LIB = L
    return _LIB


def last_error():
    return lib().triad_last_error().decode()


def _check(st):
    if st < 0:
        raise TriadError(st, last_error())
    return st


def _p(a):
    return ctypes.c_void_p(a.ctypes.data) if a.size else ctypes.c_void_p(0)


def _tp(t):
    """Device pointer of a torch tensor (None -> NULL)."""
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() else ctypes.c_void_p(0)


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def make_opts(schedule="plain", validate=0, hub_threshold=0, chunk=0, model=None, task_cycles=None,
              waves_per_group=0, grid_groups=0, timing=None, wave_span=None, kernel_variant=0, tail_share=0,
              short_tasks=0):
    o = Opts()
    o.schedule = SCHED[schedule] if isinstance(schedule, str) else int(schedule)
    o.validate = validate
    o.hub_threshold = hub_threshold
    o.chunk = chunk
    o.model = model.data_ptr() if model is not None else None
    o.task_cycles = task_cycles.data_ptr() if task_cycles is not None else None
    o.waves_per_group = waves_per_group
    o.grid_groups = grid_groups
    o.kernel_variant = kernel_variant
    o.wave_span = wave_span.data_ptr() if wave_span is not None else None
    o.tail_share = tail_share
    o.short_tasks = short_tasks
    if timing is not None:
        o.timing = ctypes.pointer(timing)
    return o


def _result(out, hi):
    res = [int(x) for x in out[:16]]
    res[0] += int(hi) << 64
    return res


def set_memory_cap(nbytes):
    """Cap the device memory any one later call may allocate (0 = no cap)."""
    return _check(lib().triad_set_memory_cap(int(nbytes)))


def held_memory():
    """Bytes of device scratch the library holds between calls (all devices)."""
    return int(lib().triad_held_memory())


def release_memory():
    """Free every device block the library holds between calls."""
    return _check(lib().triad_release_memory())


def inject_device_error(count):
    """Test hook: the next `count` single-graph census calls report a device fault."""
    return _check(lib().triad_test_inject_device_error(int(count)))


def triad_validate_host(n, offsets, nbrs, flags, level=0):
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    nb = np.ascontiguousarray(nbrs, dtype=np.int32)
    fl = np.ascontiguousarray(flags, dtype=np.uint8)
    return lib().triad_validate_host(n, _p(off), _p(nb), _p(fl), level)


def triad_census(n, offsets, nbrs, flags, **kw):
    """Census from host arrays; returns 16 Python ints (003 including its high word)."""
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    nb = np.ascontiguousarray(nbrs, dtype=np.int32)
    fl = np.ascontiguousarray(flags, dtype=np.uint8)
    out = np.zeros(16, dtype=np.uint64)
    hi = np.zeros(1, dtype=np.uint64)
    o = make_opts(**kw)
    _check(lib().triad_census_ex(n, _p(off), _p(nb), _p(fl), ctypes.byref(o), _p(out), _p(hi)))
    return _result(out, hi[0])


def triad_census_device(n, nnz, d_off, d_nbr, d_flg, stream=None, d_out=None, **kw):
    """Census from torch device tensors (int64 offsets, int32 ids, uint8 flags).

    Returns (counts, status, timing dict). `d_out` (uint64/int64 tensor with 17
    elements on the device) may be given to receive the raw output."""
    import torch
    if d_out is None:
        d_out = torch.empty(17, dtype=torch.int64, device=d_off.device)
    h = np.zeros(17, dtype=np.uint64)
    tm = Timing()
    o = make_opts(timing=tm, **kw)
    st = _check(lib().triad_census_device(n, nnz, _tp(d_off), _tp(d_nbr), _tp(d_flg), ctypes.byref(o),
                                          _stream(stream), _tp(d_out), _p(h)))
    return _result(h, h[16]), st, tm.as_dict()


def triad_census_device_noalloc(n, nnz, d_off, d_nbr, d_flg, d_out, stream=None, **kw):
    """As triad_census_device, through the entry point that allocates nothing
    (its scratch is the library's static device array). `d_out` (17 x 64-bit
    on the device) is required: this path allocates no output either.
    Returns (counts, status)."""
    h = np.zeros(17, dtype=np.uint64)
    o = make_opts(**kw)
    st = _check(lib().triad_census_device_noalloc(n, nnz, _tp(d_off), _tp(d_nbr), _tp(d_flg), ctypes.byref(o),
                                                  _stream(stream), _tp(d_out), _p(h)))
    return _result(h, h[16]), st


def labelled_census_device(n, nnz, d_off, d_nbr, d_flg, stream=None, d_out=None, **kw):
    """64-state labelled census from torch device tensors: returns (64 Python
    ints, state 0 including its high word; status; timing dict)."""
    import torch
    if d_out is None:
        d_out = torch.empty(65, dtype=torch.int64, device=d_off.device)
    h = np.zeros(65, dtype=np.uint64)
    tm = Timing()
    o = make_opts(timing=tm, **kw)
    st = _check(lib().triad_labelled_census_device(n, nnz, _tp(d_off), _tp(d_nbr), _tp(d_flg), ctypes.byref(o),
                                                   _stream(stream), _tp(d_out), _p(h)))
    res = [int(x) for x in h[:64]]
    res[0] += int(h[64]) << 64
    return res, st, tm.as_dict()


def to_device(g, device="cuda"):
    """Copy a CSR (graphs.CSR) to device tensors: (off, nbrs, flags)."""
    import torch
    return (torch.from_numpy(g.offsets).to(device), torch.from_numpy(g.nbrs).to(device),
            torch.from_numpy(g.flags).to(device))


def csr_from_arcs(n, d_src, d_dst, stream=None, timed=False):
    """Symmetric CSR with direction flags built on the device from int32 arc
    tensors; returns (offsets, ids, flags) device tensors trimmed to nnz (and the
    device milliseconds if timed)."""
    import torch
    narcs = int(d_src.numel())
    if int(d_dst.numel()) != narcs:
        raise ValueError("src and dst differ in length")
    dev = d_src.device if narcs else torch.device("cuda")
    off = torch.empty(n + 1, dtype=torch.int64, device=dev)
    nbr = torch.empty(max(2 * narcs, 1), dtype=torch.int32, device=dev)
    flg = torch.empty(max((2 * narcs + 3) // 4, 1), dtype=torch.uint8, device=dev)
    nnz = ctypes.c_int64(0)
    ms = ctypes.c_float(0.0)
    _check(lib().triad_csr_from_arcs(n, narcs, _tp(d_src), _tp(d_dst), _stream(stream), _tp(off), _tp(nbr),
                                     _tp(flg), ctypes.byref(nnz), ctypes.byref(ms) if timed else None))
    k = int(nnz.value)
    out = (off, nbr[:k], flg[:(k + 3) // 4])
    return out + (float(ms.value),) if timed else out


def census_update(n, nnz, d_off, d_nbr, d_flg, census, d_src, d_dst, d_ins, new_csr=True, stream=None):
    """Census after a batch of arc updates (insert when d_ins[i] = 1, delete
    when 0, in order) from `census` (16 Python ints) of the graph before it.
    Returns (census after, (offsets, ids, flags) of the graph after or None,
    number of changed pairs)."""
    import torch
    k = int(d_src.numel())
    cin = np.zeros(17, dtype=np.uint64)
    c0 = int(census[0])
    cin[0] = c0 & ((1 << 64) - 1)
    cin[16] = c0 >> 64
    cin[1:16] = np.array([int(x) for x in census[1:16]], dtype=np.uint64)
    cout = np.zeros(17, dtype=np.uint64)
    nn = ctypes.c_int64(0)
    chg = ctypes.c_int64(0)
    out = None
    dev = d_off.device
    if new_csr:
        cap = nnz + 2 * k
        out = (torch.empty(n + 1, dtype=torch.int64, device=dev), torch.empty(max(cap, 1), dtype=torch.int32, device=dev),
               torch.empty(max((cap + 3) // 4, 1), dtype=torch.uint8, device=dev))
    _check(lib().triad_census_update(n, nnz, _tp(d_off), _tp(d_nbr), _tp(d_flg), k, _tp(d_src), _tp(d_dst),
                                     _tp(d_ins), _p(cin), _p(cout), _tp(out[0]) if out else None,
                                     _tp(out[1]) if out else None, _tp(out[2]) if out else None,
                                     ctypes.byref(nn), ctypes.byref(chg), _stream(stream)))
    if out:
        m = int(nn.value)
        out = (out[0], out[1][:m], out[2][:(m + 3) // 4])
    return _result(cout, cout[16]), out, int(chg.value)


def significance_profile(d_ensemble, real, stream=None):
    """z-scores and significance profile of the census `real` (16 ints) against
    the batched censuses `d_ensemble` (device tensor [G, 16] of 64-bit counts).
    Returns (z[16], sp[16]) as lists of floats."""
    G = int(d_ensemble.shape[0])
    r = np.array([int(x) & ((1 << 64) - 1) for x in real], dtype=np.uint64)
    z = np.zeros(16, dtype=np.float64)
    sp = np.zeros(16, dtype=np.float64)
    _check(lib().triad_significance_profile(G, _tp(d_ensemble), _p(r), _p(z), _p(sp), _stream(stream)))
    return z.tolist(), sp.tolist()


# ------------------------------------------------------------------ batches

def batch_to_device(B, device="cuda"):
    """Copy a graphs.BatchCSR to device tensors: (vbase, offsets, nbrs, flags)."""
    import torch
    return tuple(torch.from_numpy(a).to(device) for a in (B.vbase, B.offsets, B.nbrs, B.flags))


class BatchPlan:
    """A captured hipGraph of the batched census for one concatenated CSR."""

    def __init__(self, G, nv, nnz, d_vbase, d_off, d_nbr, d_flg, d_out=None, stream=None, **kw):
        import torch
        self.G = G
        self.d_out = d_out if d_out is not None else torch.empty((G, 16), dtype=torch.int64, device=d_off.device)
        self._keep = (d_vbase, d_off, d_nbr, d_flg)
        o = make_opts(**kw)
        h = ctypes.c_void_p()
        _check(lib().triad_batch_plan_create(G, nv, nnz, _tp(d_vbase), _tp(d_off), _tp(d_nbr), _tp(d_flg),
                                             _tp(self.d_out), ctypes.byref(o), _stream(stream), ctypes.byref(h)))
        self.h = h

    def launch(self, stream=None):
        _check(lib().triad_batch_plan_launch(self.h, _stream(stream)))

    def status(self):
        return _check(lib().triad_batch_plan_status(self.h))

    def result(self):
        """Per-graph censuses as a [G][16] list of Python ints (waits for the launch)."""
        self.status()
        return [[int(x) & ((1 << 64) - 1) for x in row] for row in self.d_out.cpu().tolist()]

    def close(self):
        if self.h:
            lib().triad_batch_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def triad_census_batch(G, nv, nnz, d_vbase, d_off, d_nbr, d_flg, stream=None, **kw):
    """One-shot batched census; returns a [G][16] list of Python ints."""
    import torch
    out = torch.empty((G, 16), dtype=torch.int64, device=d_off.device)
    o = make_opts(**kw)
    _check(lib().triad_census_batch(G, nv, nnz, _tp(d_vbase), _tp(d_off), _tp(d_nbr), _tp(d_flg), ctypes.byref(o),
                                    _stream(stream), _tp(out)))
    return [[int(x) & ((1 << 64) - 1) for x in row] for row in out.cpu().tolist()]


def batch_autotune(G, nv, nnz, d_vbase, d_off, d_nbr, d_flg, cache_path=None, stream=None):
    """Fastest launch shape for this batch (dict of triad_opts fields)."""
    o = Opts()
    cp = cache_path.encode() if cache_path else None
    _check(lib().triad_batch_autotune(G, nv, nnz, _tp(d_vbase), _tp(d_off), _tp(d_nbr), _tp(d_flg), _stream(stream),
                                      cp, ctypes.byref(o)))
    return {"kernel_variant": o.kernel_variant, "waves_per_group": o.waves_per_group, "grid_groups": o.grid_groups}
