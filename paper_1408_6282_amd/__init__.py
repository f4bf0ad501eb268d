"""Python binding of the gfx950 sketch-based influence library (C ABI in include/skim.h).

Argument marshalling only: every step runs in the HIP library.  Device
buffers are torch tensors on a HIP device; streams are torch streams.  There
is no CPU fallback: importing works without a GPU, but every call needs the
built ``libskim_hip.so`` and raises if it is missing or a call fails.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libskim_hip.so")

SKIM_OK, SKIM_EINVAL, SKIM_ENOMEM, SKIM_EDEVICE, SKIM_EBUSY, SKIM_EUNSUPPORTED = range(6)
_STATUS = {0: "SKIM_OK", 1: "SKIM_EINVAL", 2: "SKIM_ENOMEM", 3: "SKIM_EDEVICE", 4: "SKIM_EBUSY",
           5: "SKIM_EUNSUPPORTED"}

EXPORTS = ["skim_abi_version", "skim_last_error", "skim_build_sketches", "skim_estimates",
           "skim_query_batch", "skim_greedy", "skim_greedy_state_free",
           "skim_greedy_state_selected", "skim_timing_enable", "skim_timing_reset",
           "skim_timing_read", "skim_server_create", "skim_server_destroy", "skim_server_submit",
           "skim_server_poll", "skim_server_set_graph", "skim_server_submit_greedy",
           "skim_server_poll_greedy", "skim_server_replay", "skim_set_build_params",
           "skim_get_build_params", "skim_tune_build", "skim_query_plan_create",
           "skim_query_plan_launch", "skim_query_plan_free", "skim_greedy_records",
           "skim_discrepancy_tail", "skim_influence_batch", "skim_build_ic_sketches",
           "skim_greedy_exact", "skim_ic_query_batch", "skim_tune_build_cached",
           "skim_debug_inject", "skim_server_cancel", "skim_sketches_create",
           "skim_build_sketches_resident", "skim_sketches_data", "skim_sketches_query",
           "skim_sketches_free", "skim_discrepancy_tail_noalloc", "skim_build_sketches_perm",
           "skim_perm_query_batch", "skim_greedy_state_save", "skim_greedy_state_load"]

SKIM_FAULT_ALLOC, SKIM_FAULT_SERVE, SKIM_FAULT_IC_RECORDS = 1, 2, 3


class SkimError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn}: {_STATUS.get(status, status)}: {msg}")
        self.status = status


class skim_server_config(C.Structure):
    _fields_ = [("budget_bytes", C.c_uint64), ("max_batch", C.c_uint32), ("streams", C.c_uint32),
                ("estimator", C.c_uint32)]


class skim_build_params(C.Structure):
    _fields_ = [("small_frontier", C.c_uint32), ("small_batch", C.c_uint32),
                ("large_batch", C.c_uint32), ("thread_frontier", C.c_uint32),
                ("heavy_visits", C.c_uint32), ("sort_frontier", C.c_uint32),
                ("window_span", C.c_uint32), ("first_span", C.c_uint32),
                ("pull_frontier", C.c_uint32)]

    def as_dict(self):
        return {name: int(getattr(self, name)) for name, _ in self._fields_}


class skim_graph(C.Structure):
    _fields_ = [("n", C.c_uint32), ("m", C.c_uint64), ("row_ptr", C.c_void_p),
                ("col", C.c_void_p), ("thr", C.c_void_p)]


_lib = None


def load_library(path: str | None = None):
    """Load libskim_hip.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    # torch first: the library then binds to the HIP runtime torch already
    # loaded (one runtime per process) rather than loading its own copy.
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing "
                           "(run __graft_entry__.build() or python -m paper_1408_6282_amd.build)")
    lib = C.CDLL(path)
    vp = C.c_void_p
    lib.skim_abi_version.restype = C.c_uint32
    lib.skim_abi_version.argtypes = []
    lib.skim_last_error.restype = C.c_char_p
    lib.skim_last_error.argtypes = []
    lib.skim_build_sketches.restype = C.c_int
    lib.skim_build_sketches.argtypes = [C.POINTER(skim_graph), C.c_uint32, C.c_uint32, C.c_uint64,
                                        vp, vp, vp, C.POINTER(C.c_uint64), vp]
    lib.skim_estimates.restype = C.c_int
    lib.skim_estimates.argtypes = [vp, vp, C.c_uint32, C.c_uint32, C.c_uint32, vp, vp]
    lib.skim_query_batch.restype = C.c_int
    lib.skim_query_batch.argtypes = [vp, vp, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64, vp,
                                     vp, C.c_uint32, C.c_uint32, vp, vp, vp]
    lib.skim_greedy.restype = C.c_int
    lib.skim_greedy.argtypes = [C.POINTER(skim_graph), C.c_uint32, C.c_uint32, C.c_uint64,
                                C.c_uint32, vp, vp, vp, C.POINTER(vp), vp]
    lib.skim_greedy_state_free.restype = None
    lib.skim_greedy_state_free.argtypes = [vp]
    lib.skim_greedy_state_selected.restype = C.c_uint32
    lib.skim_greedy_state_selected.argtypes = [vp]
    lib.skim_greedy_state_save.restype = C.c_int
    lib.skim_greedy_state_save.argtypes = [vp, vp, C.POINTER(C.c_uint64), vp]
    lib.skim_greedy_state_load.restype = C.c_int
    lib.skim_greedy_state_load.argtypes = [vp, C.c_uint32, C.c_uint32, C.c_uint64, vp, C.c_uint64,
                                           C.POINTER(vp), vp]
    lib.skim_greedy_records.restype = C.c_int
    lib.skim_greedy_records.argtypes = [vp, C.c_uint32, C.c_uint32, vp, vp, vp]
    lib.skim_tune_build_cached.restype = C.c_int
    lib.skim_tune_build_cached.argtypes = [C.POINTER(skim_graph), C.c_uint32, C.c_uint32,
                                           C.c_uint64, vp, vp, C.c_uint32, C.c_char_p,
                                           C.POINTER(skim_build_params), C.POINTER(C.c_double),
                                           C.POINTER(C.c_double), C.POINTER(C.c_uint32), vp]
    lib.skim_ic_query_batch.restype = C.c_int
    lib.skim_ic_query_batch.argtypes = [vp, C.c_uint32, C.c_uint32, C.c_uint64, vp, vp,
                                        C.c_uint32, vp, vp, vp]
    lib.skim_greedy_exact.restype = C.c_int
    lib.skim_greedy_exact.argtypes = [C.POINTER(skim_graph), C.c_uint32, C.c_uint64, C.c_uint32,
                                      vp, vp, vp]
    lib.skim_build_ic_sketches.restype = C.c_int
    lib.skim_build_ic_sketches.argtypes = [C.POINTER(skim_graph), C.c_uint32, C.c_uint64, vp, vp,
                                           vp]
    lib.skim_influence_batch.restype = C.c_int
    lib.skim_influence_batch.argtypes = [C.POINTER(skim_graph), C.c_uint32, C.c_uint64,
                                         C.c_uint64, vp, vp, vp, vp, vp]
    lib.skim_discrepancy_tail.restype = C.c_int
    lib.skim_discrepancy_tail.argtypes = [C.c_uint32, vp, vp, vp, C.c_uint32, C.c_double, vp, vp]
    lib.skim_discrepancy_tail_noalloc.restype = C.c_int
    lib.skim_discrepancy_tail_noalloc.argtypes = [C.c_uint32, vp, vp, vp, C.c_uint32, C.c_double,
                                                  vp, vp]
    P64 = C.POINTER(C.c_uint64)
    PD = C.POINTER(C.c_double)
    lib.skim_server_create.restype = C.c_int
    lib.skim_server_create.argtypes = [vp, vp, C.c_uint32, C.c_uint32, C.c_uint32,
                                       C.POINTER(skim_server_config), C.POINTER(vp)]
    lib.skim_server_destroy.restype = None
    lib.skim_server_destroy.argtypes = [vp]
    lib.skim_server_submit.restype = C.c_int
    lib.skim_server_submit.argtypes = [vp, vp, C.c_uint32, P64]
    lib.skim_server_poll.restype = C.c_int
    lib.skim_server_poll.argtypes = [vp, C.c_uint64, PD, C.POINTER(C.c_int32), PD]
    lib.skim_server_set_graph.restype = C.c_int
    lib.skim_server_set_graph.argtypes = [vp, C.POINTER(skim_graph), C.c_uint32, C.c_uint32,
                                          C.c_uint64]
    lib.skim_server_submit_greedy.restype = C.c_int
    lib.skim_server_submit_greedy.argtypes = [vp, C.c_uint32, P64]
    lib.skim_build_sketches_perm.restype = C.c_int
    lib.skim_build_sketches_perm.argtypes = [C.POINTER(skim_graph), C.c_uint32, C.c_uint32,
                                             C.c_uint64, vp, vp, vp, vp, vp]
    lib.skim_perm_query_batch.restype = C.c_int
    lib.skim_perm_query_batch.argtypes = [vp, vp, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64,
                                          vp, vp, C.c_uint32, vp, vp, vp]
    lib.skim_sketches_create.restype = C.c_int
    lib.skim_sketches_create.argtypes = [vp, vp, C.c_uint32, C.c_uint32, C.c_uint32, vp,
                                         C.POINTER(vp)]
    lib.skim_build_sketches_resident.restype = C.c_int
    lib.skim_build_sketches_resident.argtypes = [C.POINTER(skim_graph), C.c_uint32, C.c_uint32,
                                                 C.c_uint64, vp, vp, C.POINTER(vp)]
    lib.skim_sketches_data.restype = C.c_int
    lib.skim_sketches_data.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp),
                                       C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                       C.POINTER(C.c_uint32)]
    lib.skim_sketches_query.restype = C.c_int
    lib.skim_sketches_query.argtypes = [vp, C.c_uint64, vp, vp, C.c_uint64, C.c_uint32, vp, vp,
                                        vp, vp]
    lib.skim_sketches_free.restype = None
    lib.skim_sketches_free.argtypes = [vp]
    lib.skim_server_cancel.restype = C.c_int
    lib.skim_server_cancel.argtypes = [vp, C.c_uint64]
    lib.skim_debug_inject.restype = C.c_int
    lib.skim_debug_inject.argtypes = [C.c_uint32, C.c_uint32]
    lib.skim_server_poll_greedy.restype = C.c_int
    lib.skim_server_poll_greedy.argtypes = [vp, C.c_uint64, vp, vp, PD]
    lib.skim_server_replay.restype = C.c_int
    lib.skim_server_replay.argtypes = [vp, C.c_uint64, vp, vp, vp, vp, vp, vp, P64]
    lib.skim_set_build_params.restype = C.c_int
    lib.skim_set_build_params.argtypes = [C.POINTER(skim_build_params)]
    lib.skim_get_build_params.restype = None
    lib.skim_get_build_params.argtypes = [C.POINTER(skim_build_params)]
    lib.skim_tune_build.restype = C.c_int
    lib.skim_tune_build.argtypes = [C.POINTER(skim_graph), C.c_uint32, C.c_uint32, C.c_uint64, vp,
                                    vp, C.c_uint32, C.POINTER(skim_build_params), PD, PD, vp]
    lib.skim_query_plan_create.restype = C.c_int
    lib.skim_query_plan_create.argtypes = [vp, vp, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint64,
                                           vp, vp, C.c_uint32, vp, vp, vp, C.POINTER(vp)]
    lib.skim_query_plan_launch.restype = C.c_int
    lib.skim_query_plan_launch.argtypes = [vp, vp]
    lib.skim_query_plan_free.restype = None
    lib.skim_query_plan_free.argtypes = [vp]
    lib.skim_timing_enable.restype = None
    lib.skim_timing_enable.argtypes = [C.c_char_p]
    lib.skim_timing_reset.restype = None
    lib.skim_timing_reset.argtypes = []
    lib.skim_timing_read.restype = C.c_int
    lib.skim_timing_read.argtypes = [C.c_char_p, C.POINTER(C.c_double), C.POINTER(C.c_uint64)]
    _lib = lib
    return lib


def _check(fn: str, status: int):
    if status != SKIM_OK:
        msg = _lib.skim_last_error().decode(errors="replace") if _lib else ""
        raise SkimError(fn, status, msg)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class DeviceGraph:
    """A forward-CSR graph resident in device memory (torch tensors) plus its ABI struct."""

    def __init__(self, n: int, row_ptr, col, thr):
        self.n = int(n)
        self.row_ptr, self.col, self.thr = row_ptr, col, thr
        self.m = int(col.numel())
        self.struct = skim_graph(self.n, self.m, row_ptr.data_ptr(),
                                 col.data_ptr() if self.m else None,
                                 thr.data_ptr() if self.m else None)

    @classmethod
    def from_host(cls, g, device="cuda"):
        """Upload a ``workloads.Graph`` (numpy arrays) to the device."""
        import torch
        rp = torch.from_numpy(np.ascontiguousarray(g.row_ptr).view(np.int64)).to(device)
        col = torch.from_numpy(np.ascontiguousarray(g.col).view(np.int32)).to(device)
        thr = torch.from_numpy(np.ascontiguousarray(g.thr).view(np.int32)).to(device)
        return cls(g.n, rp, col, thr)


def skim_abi_version() -> int:
    return int(load_library().skim_abi_version())


def skim_last_error() -> str:
    return load_library().skim_last_error().decode(errors="replace")


def skim_build_sketches(graph: DeviceGraph, ell: int, k: int, seed: int, ranks, size, est=None,
                        stream=None):
    """Fill ranks [n*k] (int64 view of uint64), size [n] (int32 view of uint32) and est [n].

    Returns the device work counters (items, live-edge scans, records, windows).
    """
    lib = load_library()
    work = (C.c_uint64 * 6)()
    st = lib.skim_build_sketches(C.byref(graph.struct), ell, k, seed & 0xFFFFFFFFFFFFFFFF,
                                 _ptr(ranks), _ptr(size), _ptr(est), work, _stream(stream))
    _check("skim_build_sketches", st)
    return {"visits": int(work[0]), "scans": int(work[1]), "records": int(work[2]),
            "windows": int(work[3]), "restarts": int(work[4]), "restart_flags": int(work[5])}


def skim_debug_inject(what: int, count: int = 1):
    """Make the next `count` device allocations (SKIM_FAULT_ALLOC) or serving
    batch copies/launches (SKIM_FAULT_SERVE) fail on the host side, or IC-model
    sketch builds take their counting path (SKIM_FAULT_IC_RECORDS); 0 disarms."""
    _check("skim_debug_inject", load_library().skim_debug_inject(what, count))


def skim_build_sketches_perm(graph: DeviceGraph, ell: int, k: int, seed: int, ranks, size,
                             est=None, stream=None):
    """Sketches of structured permutation positions (Section 3.1): as
    skim_build_sketches, with positions 1..n l as the ranks."""
    lib = load_library()
    work = (C.c_uint64 * 6)()
    st = lib.skim_build_sketches_perm(C.byref(graph.struct), ell, k, seed & 0xFFFFFFFFFFFFFFFF,
                                      _ptr(ranks), _ptr(size), _ptr(est), work, _stream(stream))
    _check("skim_build_sketches_perm", st)
    return {"visits": int(work[0]), "scans": int(work[1]), "records": int(work[2]),
            "windows": int(work[3]), "restarts": int(work[4]), "restart_flags": int(work[5])}


def skim_perm_query_batch(ranks, size, n: int, k: int, ell: int, qoff, qnodes, est, qstatus=None,
                          estimator: int = 0, stream=None):
    """Union estimates over sketches of permutation positions."""
    lib = load_library()
    q = int(qoff.numel()) - 1
    st = lib.skim_perm_query_batch(_ptr(ranks), _ptr(size), n, k, ell, max(q, 0), _ptr(qoff),
                                   _ptr(qnodes) if qnodes is not None and qnodes.numel() else None,
                                   estimator, _ptr(est), _ptr(qstatus), _stream(stream))
    _check("skim_perm_query_batch", st)


def skim_estimates(ranks, size, n: int, k: int, ell: int, est, stream=None):
    lib = load_library()
    st = lib.skim_estimates(_ptr(ranks), _ptr(size), n, k, ell, _ptr(est), _stream(stream))
    _check("skim_estimates", st)


def skim_query_batch(ranks, size, n: int, k: int, ell: int, qoff, qnodes, est, qstatus=None,
                     estimator: int = 0, mode: int = 0, stream=None):
    """Estimates for the seed sets qnodes[qoff[j]:qoff[j+1]] (device tensors)."""
    lib = load_library()
    q = int(qoff.numel()) - 1
    st = lib.skim_query_batch(_ptr(ranks), _ptr(size), n, k, ell, max(q, 0), _ptr(qoff),
                              _ptr(qnodes) if qnodes is not None and qnodes.numel() else None,
                              estimator, mode, _ptr(est), _ptr(qstatus), _stream(stream))
    _check("skim_query_batch", st)


class Sketches:
    """skim_sketches_*: a resident, library-owned sketch table; query() only
    enqueues its launch on the stream (capturable into a HIP graph)."""

    def __init__(self, handle):
        self.handle = handle
        lib = load_library()
        r, s, e = C.c_void_p(), C.c_void_p(), C.c_void_p()
        n, k, ell = C.c_uint32(), C.c_uint32(), C.c_uint32()
        _check("skim_sketches_data", lib.skim_sketches_data(self.handle, C.byref(r), C.byref(s),
                                                            C.byref(e), C.byref(n), C.byref(k),
                                                            C.byref(ell)))
        self.n, self.k, self.ell = int(n.value), int(k.value), int(ell.value)
        self.ranks_ptr, self.size_ptr, self.est_ptr = r.value, s.value, e.value

    @classmethod
    def from_tables(cls, ranks, size, n: int, k: int, ell: int, stream=None):
        h = C.c_void_p(None)
        _check("skim_sketches_create", load_library().skim_sketches_create(
            _ptr(ranks), _ptr(size), n, k, ell, _stream(stream), C.byref(h)))
        return cls(h)

    @classmethod
    def build(cls, graph: DeviceGraph, ell: int, k: int, seed: int, stream=None):
        h = C.c_void_p(None)
        work = (C.c_uint64 * 6)()
        _check("skim_build_sketches_resident", load_library().skim_build_sketches_resident(
            C.byref(graph.struct), ell, k, seed & 0xFFFFFFFFFFFFFFFF, work, _stream(stream),
            C.byref(h)))
        return cls(h)

    def query(self, qoff, qnodes, est, qstatus=None, estimator: int = 0, workspace=None,
              stream=None):
        q = int(qoff.numel()) - 1
        nn = int(qnodes.numel()) if qnodes is not None else 0
        _check("skim_sketches_query", load_library().skim_sketches_query(
            self.handle, max(q, 0), _ptr(qoff), _ptr(qnodes) if nn else None, nn, estimator,
            _ptr(est), _ptr(qstatus), _ptr(workspace), _stream(stream)))

    def tables(self, torch):
        """Host copies of the resident (ranks, size, est) as numpy arrays."""
        import numpy as _np
        n, k = self.n, self.k
        out = []
        for ptr, count, dt in ((self.ranks_ptr, n * k, _np.uint64), (self.size_ptr, n, _np.uint32),
                               (self.est_ptr, n, _np.float64)):
            a = _np.empty(count, dtype=dt)
            torch.cuda.synchronize()
            if not _copy_d2h(a, ptr):
                raise SkimError("hipMemcpy", SKIM_EDEVICE, "copy of the resident sketches failed")
            out.append(a)
        return out[0].reshape(n, k), out[1], out[2]

    def free(self):
        if self.handle:
            load_library().skim_sketches_free(self.handle)
            self.handle = C.c_void_p(None)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def _copy_d2h(dst, src_ptr) -> bool:
    """Blocking copy of dst.nbytes from device address src_ptr into the host
    numpy array dst (hipMemcpy of the HIP runtime torch has loaded)."""
    global _hip_rt
    if _hip_rt is None:
        _hip_rt = C.CDLL("libamdhip64.so")
        _hip_rt.hipMemcpy.restype = C.c_int
        _hip_rt.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    return _hip_rt.hipMemcpy(dst.ctypes.data_as(C.c_void_p), C.c_void_p(src_ptr), dst.nbytes,
                             2) == 0  # hipMemcpyDeviceToHost


_hip_rt = None


class QueryPlan:
    """skim_query_plan_*: a batched query launch captured once into a HIP graph;
    launch() replays it on a stream without waiting."""

    def __init__(self, ranks, size, n: int, k: int, ell: int, qoff, qnodes, est, qstatus=None,
                 estimator: int = 0, stream=None):
        lib = load_library()
        self.handle = C.c_void_p(None)
        q = int(qoff.numel()) - 1
        self._keep = (ranks, size, qoff, qnodes, est, qstatus)  # buffers outlive the plan
        st = lib.skim_query_plan_create(_ptr(ranks), _ptr(size), n, k, ell, max(q, 0), _ptr(qoff),
                                        _ptr(qnodes) if qnodes is not None and qnodes.numel()
                                        else None, estimator, _ptr(est), _ptr(qstatus),
                                        _stream(stream), C.byref(self.handle))
        _check("skim_query_plan_create", st)

    def launch(self, stream=None):
        _check("skim_query_plan_launch",
               load_library().skim_query_plan_launch(self.handle, _stream(stream)))

    def free(self):
        if self.handle:
            load_library().skim_query_plan_free(self.handle)
            self.handle = C.c_void_p(None)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def skim_set_build_params(params: dict | None):
    """Launch shapes of the build's search (None restores the defaults)."""
    lib = load_library()
    if params is None:
        _check("skim_set_build_params", lib.skim_set_build_params(None))
        return
    p = skim_get_build_params()
    p.update(params)
    _check("skim_set_build_params", lib.skim_set_build_params(C.byref(skim_build_params(**p))))


def skim_get_build_params() -> dict:
    p = skim_build_params()
    load_library().skim_get_build_params(C.byref(p))
    return p.as_dict()


def skim_tune_build(graph: DeviceGraph, ell: int, k: int, seed: int, ranks, size, reps: int = 2,
                    stream=None):
    """Autotune the build's launch shapes on this graph; returns (params, best_ms, start_ms)
    and leaves the best parameters in force."""
    lib = load_library()
    best = skim_build_params()
    best_ms = C.c_double(0)
    start_ms = C.c_double(0)
    st = lib.skim_tune_build(C.byref(graph.struct), ell, k, seed & 0xFFFFFFFFFFFFFFFF, _ptr(ranks),
                             _ptr(size), reps, C.byref(best), C.byref(best_ms),
                             C.byref(start_ms), _stream(stream))
    _check("skim_tune_build", st)
    return best.as_dict(), float(best_ms.value), float(start_ms.value)


def skim_tune_build_cached(graph: DeviceGraph, ell: int, k: int, seed: int, ranks, size,
                           cache_path: str, reps: int = 2, stream=None):
    """skim_tune_build behind a persistent cache keyed by device and configuration;
    returns (params, best_ms, start_ms, hit)."""
    lib = load_library()
    best = skim_build_params()
    best_ms = C.c_double(0)
    start_ms = C.c_double(0)
    hit = C.c_uint32(0)
    st = lib.skim_tune_build_cached(C.byref(graph.struct), ell, k, seed & 0xFFFFFFFFFFFFFFFF,
                                    _ptr(ranks), _ptr(size), reps, cache_path.encode(),
                                    C.byref(best), C.byref(best_ms), C.byref(start_ms),
                                    C.byref(hit), _stream(stream))
    _check("skim_tune_build_cached", st)
    return best.as_dict(), float(best_ms.value), float(start_ms.value), bool(hit.value)


class GreedyState:
    """Owner of a resumable SKIM state (freed with skim_greedy_state_free)."""

    def __init__(self):
        self.handle = C.c_void_p(None)

    @property
    def selected(self) -> int:
        return int(load_library().skim_greedy_state_selected(self.handle))

    def free(self):
        if self.handle:
            load_library().skim_greedy_state_free(self.handle)
            self.handle = C.c_void_p(None)

    def save(self, stream=None) -> bytes:
        """The run's progress as bytes (skim_greedy_state_save)."""
        lib = load_library()
        n = C.c_uint64(0)
        _check("skim_greedy_state_save",
               lib.skim_greedy_state_save(self.handle, None, C.byref(n), _stream(stream)))
        buf = C.create_string_buffer(max(int(n.value), 1))
        _check("skim_greedy_state_save",
               lib.skim_greedy_state_save(self.handle, buf, C.byref(n), _stream(stream)))
        return buf.raw[:int(n.value)]

    @classmethod
    def load(cls, graph: "DeviceGraph", ell: int, k: int, seed: int, data: bytes, stream=None):
        """A state resumed from saved bytes (skim_greedy_state_load)."""
        st = cls()
        buf = C.create_string_buffer(bytes(data), len(data))
        _check("skim_greedy_state_load",
               load_library().skim_greedy_state_load(C.byref(graph.struct), ell, k,
                                                     seed & 0xFFFFFFFFFFFFFFFF, buf, len(data),
                                                     C.byref(st.handle), _stream(stream)))
        return st

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def skim_greedy(graph: DeviceGraph, ell: int, k: int, seed: int, s: int, seeds, gain_pairs,
                gain=None, state: GreedyState | None = None, stream=None):
    """Select s seeds (resuming `state` when given) into device tensors."""
    lib = load_library()
    ref = C.byref(state.handle) if state is not None else None
    st = lib.skim_greedy(C.byref(graph.struct), ell, k, seed & 0xFFFFFFFFFFFFFFFF, s, _ptr(seeds),
                         _ptr(gain_pairs), _ptr(gain), ref, _stream(stream))
    _check("skim_greedy", st)


def skim_greedy_state_free(state: GreedyState):
    state.free()


def skim_ic_query_batch(positions, n: int, k: int, qoff, qnodes, est, qstatus=None,
                        estimator: int = 0, stream=None):
    """Union estimates over IC-model sketches into the float64 device tensor est."""
    q = int(qoff.numel()) - 1
    st = load_library().skim_ic_query_batch(
        _ptr(positions), n, k, q, _ptr(qoff),
        _ptr(qnodes) if qnodes is not None and qnodes.numel() else None, estimator, _ptr(est),
        _ptr(qstatus), _stream(stream))
    _check("skim_ic_query_batch", st)


def skim_greedy_exact(graph: DeviceGraph, ell: int, seed: int, s: int, seeds, gain_pairs,
                      stream=None):
    """Exact greedy (largest marginal gain, smallest id on ties) for s seeds."""
    st = load_library().skim_greedy_exact(C.byref(graph.struct), ell, seed & 0xFFFFFFFFFFFFFFFF,
                                          s, _ptr(seeds), _ptr(gain_pairs), _stream(stream))
    _check("skim_greedy_exact", st)


def skim_build_ic_sketches(graph: DeviceGraph, k: int, seed: int, positions, est=None,
                           stream=None):
    """IC-model sketches (structured permutation positions, uint32 [n, k]) and
    their influence estimates n (k - 1) / (T - 1) into device tensors."""
    st = load_library().skim_build_ic_sketches(C.byref(graph.struct), k,
                                               seed & 0xFFFFFFFFFFFFFFFF, _ptr(positions),
                                               _ptr(est), _stream(stream))
    _check("skim_build_ic_sketches", st)


def skim_influence_batch(graph: DeviceGraph, ell: int, seed: int, qoff, qnodes, reach_pairs,
                         qstatus=None, stream=None):
    """Exact sum_i |reach_i(S_j)| over the l instances of `seed` for every set
    S_j = qnodes[qoff[j]:qoff[j+1]], into the uint64 device tensor reach_pairs."""
    q = int(qoff.numel()) - 1
    st = load_library().skim_influence_batch(
        C.byref(graph.struct), ell, seed & 0xFFFFFFFFFFFFFFFF, q, _ptr(qoff),
        _ptr(qnodes) if qnodes is not None and qnodes.numel() else None, _ptr(reach_pairs),
        _ptr(qstatus), _stream(stream))
    _check("skim_influence_batch", st)


def skim_greedy_records(state: GreedyState, first: int, count: int, tau=None, second=None,
                        stream=None):
    """Per-seed tau (uint64) and second largest sketch (uint32) of seeds
    first .. first+count-1 of a SKIM run, into device tensors."""
    st = load_library().skim_greedy_records(state.handle, first, count, _ptr(tau), _ptr(second),
                                            _stream(stream))
    _check("skim_greedy_records", st)


def skim_discrepancy_tail(tau, second, gain_pairs, bins: int, max_rel_error: float, tail,
                          stream=None):
    """Upper bounds on P[total discrepancy >= t * max_rel_error * I / bins],
    t = 0..bins, into the float64 device tensor ``tail``; s = len(tau)."""
    s = 0 if tau is None else int(tau.numel())
    st = load_library().skim_discrepancy_tail(s, _ptr(tau), _ptr(second), _ptr(gain_pairs), bins,
                                              float(max_rel_error), _ptr(tail), _stream(stream))
    _check("skim_discrepancy_tail", st)


def skim_discrepancy_tail_noalloc(tau, second, gain_pairs, bins: int, max_rel_error: float,
                                  tail, stream=None):
    """skim_discrepancy_tail without allocation: only enqueued on the stream
    (the caller synchronises); s * (bins + 1) <= 2^20."""
    s = 0 if tau is None else int(tau.numel())
    st = load_library().skim_discrepancy_tail_noalloc(s, _ptr(tau), _ptr(second), _ptr(gain_pairs),
                                                      bins, float(max_rel_error), _ptr(tail),
                                                      _stream(stream))
    _check("skim_discrepancy_tail_noalloc", st)


def skim_timing_enable(kernel: str | None):
    load_library().skim_timing_enable(kernel.encode() if kernel else None)


def skim_timing_reset():
    load_library().skim_timing_reset()


def skim_timing_read(kernel: str):
    """(total milliseconds, launches) of the timed kernel so far."""
    ms = C.c_double(0)
    n = C.c_uint64(0)
    load_library().skim_timing_read(kernel.encode(), C.byref(ms), C.byref(n))
    return float(ms.value), int(n.value)


class Server:
    """A serving loop over resident sketches (see skim_server_* in include/skim.h)."""

    def __init__(self, ranks, size, n: int, k: int, ell: int, budget_bytes: int = 64 << 20,
                 max_batch: int = 4096, streams: int = 4, estimator: int = 0):
        lib = load_library()
        self._keep = (ranks, size)
        cfg = skim_server_config(budget_bytes, max_batch, streams, estimator)
        self.handle = C.c_void_p(None)
        _check("skim_server_create", lib.skim_server_create(_ptr(ranks), _ptr(size), n, k, ell,
                                                            C.byref(cfg), C.byref(self.handle)))

    def submit(self, nodes) -> int:
        """Submit one set (host array); returns a ticket.  Raises SkimError on EBUSY."""
        a = np.ascontiguousarray(nodes, dtype=np.uint32)
        t = C.c_uint64(0)
        _check("skim_server_submit", _lib.skim_server_submit(
            self.handle, a.ctypes.data_as(C.c_void_p) if a.size else None, a.size, C.byref(t)))
        return int(t.value)

    def poll(self, ticket: int):
        """(est, status, latency_us) when done, else None."""
        e, s, l = C.c_double(0), C.c_int32(0), C.c_double(0)
        st = _lib.skim_server_poll(self.handle, ticket, C.byref(e), C.byref(s), C.byref(l))
        if st == SKIM_EBUSY:
            return None
        _check("skim_server_poll", st)
        return float(e.value), int(s.value), float(l.value)

    def cancel(self, ticket: int):
        """Cancel a query request: it completes with status -6."""
        _check("skim_server_cancel", _lib.skim_server_cancel(self.handle, ticket))

    def set_graph(self, graph: DeviceGraph, ell: int, k: int, seed: int):
        self._graph = graph
        _check("skim_server_set_graph", _lib.skim_server_set_graph(
            self.handle, C.byref(graph.struct), ell, k, seed & 0xFFFFFFFFFFFFFFFF))

    def submit_greedy(self, s: int) -> int:
        t = C.c_uint64(0)
        _check("skim_server_submit_greedy", _lib.skim_server_submit_greedy(self.handle, s,
                                                                           C.byref(t)))
        return int(t.value)

    def poll_greedy(self, ticket: int, s: int):
        """(seeds, gain_pairs, latency_us) when done, else None."""
        seeds = np.zeros(max(s, 1), dtype=np.uint32)
        gains = np.zeros(max(s, 1), dtype=np.uint64)
        l = C.c_double(0)
        st = _lib.skim_server_poll_greedy(self.handle, ticket, seeds.ctypes.data_as(C.c_void_p),
                                          gains.ctypes.data_as(C.c_void_p), C.byref(l))
        if st == SKIM_EBUSY:
            return None
        _check("skim_server_poll_greedy", st)
        return seeds[:s], gains[:s], float(l.value)

    def replay(self, offsets, nodes, arrival_s):
        """Open-loop replay of host query sets; returns (est, status, latency_us, retries)."""
        off = np.ascontiguousarray(offsets, dtype=np.uint64)
        nd = np.ascontiguousarray(nodes, dtype=np.uint32)
        arr = np.ascontiguousarray(arrival_s, dtype=np.float64)
        q = off.size - 1
        est = np.zeros(max(q, 1))
        st = np.zeros(max(q, 1), dtype=np.int32)
        lat = np.zeros(max(q, 1))
        retries = C.c_uint64(0)
        vp = C.c_void_p
        _check("skim_server_replay", _lib.skim_server_replay(
            self.handle, q, off.ctypes.data_as(vp), nd.ctypes.data_as(vp) if nd.size else None,
            arr.ctypes.data_as(vp), est.ctypes.data_as(vp), st.ctypes.data_as(vp),
            lat.ctypes.data_as(vp), C.byref(retries)))
        return est[:q], st[:q], lat[:q], int(retries.value)

    def close(self):
        if self.handle:
            _lib.skim_server_destroy(self.handle)
            self.handle = C.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
