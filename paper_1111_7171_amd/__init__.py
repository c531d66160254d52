"""MI355X (gfx950) Pass-Join edit-distance similarity join.

Thin ctypes binding of libpassjoin (C ABI declared in include/passjoin.h).  It only marshals
arguments: every step of the join runs in the library's HIP kernels.  If the library has not
been built, every call raises :class:`PassJoinError` -- there is no CPU fallback.

String sets are given as any of:
  * an object with ``chars`` (uint8) and ``offsets`` (int32, n+1) numpy arrays (host memory);
  * a ``(chars, offsets)`` tuple of numpy arrays (host memory);
  * a ``(chars, offsets)`` tuple of torch tensors on a HIP device (device memory; the work is
    ordered on torch's current stream).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

__all__ = [
    "PassJoinError", "load", "pj_self_join", "pj_join", "pj_build_index", "pj_query",
    "pj_index_info", "pj_index_free", "pj_last_error", "pj_last_stats", "pj_version",
    "MODE_AUTO", "MODE_PLAIN", "MODE_BATCHED", "MODE_SHARE_PREFIX", "PJ_TAU_MAX", "PJ_LEN_MAX",
    "Server", "Index",
    "pj_tune", "pj_query_noalloc", "pj_self_join_host", "HostPairs", "Plan",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpassjoin.so")

PJ_OK, PJ_EINVAL, PJ_ERANGE, PJ_ENOMEM, PJ_EDEVICE = 0, -1, -2, -3, -4
PJ_TAU_MAX, PJ_LEN_MAX = 63, 2047
MODE_AUTO, MODE_PLAIN, MODE_BATCHED, MODE_SHARE_PREFIX = 0, 1, 2, 3
SELECT_MULTIMATCH, SELECT_POSITION, SELECT_SHIFT, SELECT_LENGTH = 0, 1, 2, 3
_CODES = {PJ_EINVAL: "EINVAL", PJ_ERANGE: "ERANGE", PJ_ENOMEM: "ENOMEM", PJ_EDEVICE: "EDEVICE"}


class PassJoinError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_CODES.get(code, code)}: {msg}")
        self.code = code


class PjStrings(C.Structure):
    _fields_ = [("n", C.c_int64), ("bytes", C.c_void_p), ("offsets", C.c_void_p)]


class PjPairs(C.Structure):
    _fields_ = [("count", C.c_int64), ("a", C.c_void_p), ("b", C.c_void_p),
                ("on_device", C.c_int32)]


class PjOptions(C.Structure):
    _fields_ = [("hip_stream", C.c_void_p), ("inputs_on_device", C.c_int32),
                ("outputs_on_device", C.c_int32), ("mode", C.c_int32), ("selection", C.c_int32),
                ("mem_budget_bytes", C.c_int64), ("tune_cache", C.c_char_p)]


class PjStats(C.Structure):
    _fields_ = [(k, C.c_int64) for k in ("strings", "index_entries", "selected", "hits",
                                         "candidates", "cells", "accepted", "side_pairs",
                                         "pairs")] + \
               [(k, C.c_double) for k in ("ms_upload", "ms_index", "ms_probe", "ms_verify",
                                          "ms_output", "ms_total", "ms_probe_kernel",
                                          "ms_verify_kernel")] + \
               [("verify_launches", C.c_int64), ("ms_list_kernel", C.c_double),
                ("list_cells", C.c_int64), ("list_launches", C.c_int64),
                ("key_collisions", C.c_int64), ("shared_rows", C.c_int64),
                ("shared_cells", C.c_int64), ("replayed", C.c_int64)]


class PjServerConfig(C.Structure):
    _fields_ = [("slots", C.c_int32), ("max_batch_queries", C.c_int32),
                ("mem_budget_bytes", C.c_int64), ("tune_cache", C.c_char_p),
                ("eager", C.c_int32)]


class PjTuneResult(C.Structure):
    _fields_ = [("verify_waves_per_cu", C.c_int32), ("seg_chunk", C.c_int32),
                ("big_list", C.c_int32), ("probe_blocks_per_cu", C.c_int32),
                ("lane_cands", C.c_int32), ("probe_map", C.c_int32),
                ("len_bucket", C.c_int32), ("trials", C.c_int32),
                ("ms_default", C.c_double), ("ms_best", C.c_double)]


class PjRequestInfo(C.Structure):
    _fields_ = [("t_submit_ms", C.c_double), ("t_admit_ms", C.c_double),
                ("t_done_ms", C.c_double), ("footprint_bytes", C.c_int64),
                ("batch_requests", C.c_int32), ("slot", C.c_int32),
                ("deferrals", C.c_int32), ("deferred_by_memory", C.c_int32)]


_lib = None


def load():
    """Loads libpassjoin.so (built in-tree by paper_1111_7171_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise PassJoinError(PJ_EDEVICE, f"{LIB_PATH} is not built; run "
                                "`python -m paper_1111_7171_amd.build`")
        # One HIP runtime per process: PyTorch ships its own copy of the runtime under the same
        # soname.  Loaded first, it is the one libpassjoin.so binds to; loaded after the
        # system's, PyTorch would bring in a second runtime that finds no device.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        lib = C.CDLL(LIB_PATH)
        sp, pp, op = C.POINTER(PjStrings), C.POINTER(PjPairs), C.POINTER(PjOptions)
        lib.pj_self_join.argtypes = [sp, C.c_int32, op, pp]
        lib.pj_self_join.restype = C.c_int
        lib.pj_join.argtypes = [sp, sp, C.c_int32, op, pp]
        lib.pj_self_join_streamed.argtypes = [sp, C.c_int32, C.c_int64, op, pp]
        lib.pj_self_join_streamed.restype = C.c_int
        lib.pj_join.restype = C.c_int
        lib.pj_build_index.argtypes = [sp, C.c_int32, C.c_int32, op, C.POINTER(C.c_void_p)]
        lib.pj_build_index.restype = C.c_int
        lib.pj_index_info.argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                                      C.POINTER(C.c_int32), C.POINTER(C.c_int64)]
        lib.pj_index_info.restype = C.c_int
        lib.pj_query.argtypes = [C.c_void_p, sp, C.c_void_p, op, pp]
        lib.pj_query.restype = C.c_int
        lib.pj_pairs_free.argtypes = [pp]
        lib.pj_pairs_free.restype = None
        lib.pj_index_free.argtypes = [C.c_void_p]
        lib.pj_index_free.restype = None
        lib.pj_last_error.argtypes = []
        lib.pj_last_error.restype = C.c_char_p
        lib.pj_last_stats.argtypes = [C.POINTER(PjStats)]
        lib.pj_last_stats.restype = C.c_int
        lib.pj_version.argtypes = []
        lib.pj_version.restype = C.c_char_p
        lib.pj_server_start.argtypes = [C.c_void_p, C.POINTER(PjServerConfig),
                                        C.POINTER(C.c_void_p)]
        lib.pj_server_start.restype = C.c_int
        lib.pj_server_submit.argtypes = [C.c_void_p, sp, C.c_void_p]
        lib.pj_server_submit.restype = C.c_int64
        lib.pj_server_wait.argtypes = [C.c_void_p, C.c_int64, pp, C.POINTER(PjRequestInfo)]
        lib.pj_server_wait.restype = C.c_int
        lib.pj_server_stop.argtypes = [C.c_void_p]
        lib.pj_server_stop.restype = C.c_int
        lib.pj_query_noalloc.argtypes = [C.c_void_p, sp, C.c_void_p, op, C.c_void_p,
                                         C.c_void_p, C.c_int64, C.POINTER(C.c_int64)]
        lib.pj_query_noalloc.restype = C.c_int
        lib.pj_tune.argtypes = [sp, C.c_int32, op, C.POINTER(PjTuneResult)]
        lib.pj_tune.restype = C.c_int
        lib.pj_self_join_plan.argtypes = [sp, C.c_int32, op, C.POINTER(C.c_void_p)]
        lib.pj_self_join_plan.restype = C.c_int
        lib.pj_plan_run.argtypes = [C.c_void_p, pp]
        lib.pj_plan_run.restype = C.c_int
        lib.pj_plan_free.argtypes = [C.c_void_p]
        lib.pj_plan_free.restype = None
        _lib = lib
    return _lib


def pj_last_error() -> str:
    return load().pj_last_error().decode()


def pj_version() -> str:
    return load().pj_version().decode()


def pj_last_stats() -> dict:
    st = PjStats()
    load().pj_last_stats(C.byref(st))
    return {k: getattr(st, k) for k, _ in PjStats._fields_}


def _check(rc: int):
    if rc != PJ_OK:
        raise PassJoinError(rc, pj_last_error())


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


class _Marshalled:
    """A PjStrings view of a string set plus whatever keeps its memory alive."""

    def __init__(self, strings):
        if hasattr(strings, "chars") and hasattr(strings, "offsets"):
            chars, offs = strings.chars, strings.offsets
        else:
            chars, offs = strings
        self.on_device = (_is_torch(offs) and offs.is_cuda) or \
            (_is_torch(chars) and chars.is_cuda)
        if self.on_device:
            import torch
            # both arrays on the same device (the library also checks the pointers and the
            # allocation sizes before any kernel reads them)
            if not (_is_torch(chars) and _is_torch(offs) and chars.is_cuda and offs.is_cuda):
                raise PassJoinError(PJ_EINVAL, "chars and offsets must both be device tensors")
            if chars.device != offs.device:
                raise PassJoinError(PJ_EINVAL, "chars and offsets are on different devices")
            if chars.dtype != torch.uint8 or offs.dtype != torch.int32:
                raise PassJoinError(PJ_EINVAL, "device strings must be uint8 chars, int32 offsets")
            if not (chars.is_contiguous() and offs.is_contiguous()):
                raise PassJoinError(PJ_EINVAL, "device strings must be contiguous")
            if offs.dim() != 1 or offs.numel() < 1:
                raise PassJoinError(PJ_EINVAL, "offsets must be a 1-D tensor of n+1 entries")
            self.keep = (chars, offs)
            self.s = PjStrings(offs.numel() - 1, chars.data_ptr() if chars.numel() else None,
                               offs.data_ptr())
        else:
            if _is_torch(chars):
                chars, offs = chars.numpy(), offs.numpy()
            chars = np.ascontiguousarray(chars, dtype=np.uint8)
            offs = np.ascontiguousarray(offs, dtype=np.int32)
            if offs.ndim != 1 or offs.size < 1:
                raise PassJoinError(PJ_EINVAL, "offsets must be a 1-D array of n+1 entries")
            self.keep = (chars, offs)
            self.s = PjStrings(offs.size - 1, chars.ctypes.data if chars.size else None,
                               offs.ctypes.data)


def _options(on_device: bool, outputs_on_device: bool, mode: int, mem_budget: int,
             stream, tune_cache: str | None, selection: int = 0) -> PjOptions:
    o = PjOptions()
    o.inputs_on_device = 1 if on_device else 0
    o.outputs_on_device = 1 if outputs_on_device else 0
    o.mode = mode
    o.selection = int(selection)
    o.mem_budget_bytes = int(mem_budget)
    o.tune_cache = tune_cache.encode() if tune_cache else None
    if stream is None and on_device:
        import torch
        stream = torch.cuda.current_stream()
    if stream is not None:
        o.hip_stream = C.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))
    return o


@dataclass
class DevicePairs:
    """Result pairs left in device memory (outputs_on_device=True).  Call free() when done."""
    raw: PjPairs

    @property
    def count(self) -> int:
        return int(self.raw.count)

    def to_numpy(self) -> np.ndarray:
        m = self.count
        out = np.empty((m, 2), dtype=np.int32)
        if m:
            for col, ptr in ((0, self.raw.a), (1, self.raw.b)):
                host = np.empty(m, dtype=np.int32)
                _hip_d2h(host, ptr)
                out[:, col] = host
        return out

    def free(self):
        load().pj_pairs_free(C.byref(self.raw))


_hip = None


def _hip_d2h(host: np.ndarray, dev_ptr: int):
    """Copies device memory into a host array with the HIP runtime's hipMemcpy."""
    global _hip
    if _hip is None:
        # the runtime libpassjoin.so is bound to (resolved through the library's own handle)
        _hip = load().hipMemcpy
        _hip.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        _hip.restype = C.c_int
    rc = _hip(host.ctypes.data, dev_ptr, host.nbytes, 2)   # hipMemcpyDeviceToHost
    if rc != 0:
        raise PassJoinError(PJ_EDEVICE, f"hipMemcpy failed ({rc})")


class HostPairs:
    """Result pairs left in the library's host memory (pj_self_join_host): a and b are numpy
    views of the C arrays (no copy); call free() when done."""

    def __init__(self, raw: PjPairs):
        self.raw = raw
        m = int(raw.count)
        self.count = m
        self.a = np.ctypeslib.as_array(C.cast(raw.a, C.POINTER(C.c_int32)), shape=(m,)) \
            if m else np.empty(0, np.int32)
        self.b = np.ctypeslib.as_array(C.cast(raw.b, C.POINTER(C.c_int32)), shape=(m,)) \
            if m else np.empty(0, np.int32)

    def free(self):
        self.a = self.b = None
        load().pj_pairs_free(C.byref(self.raw))


def _take_pairs(raw: PjPairs, outputs_on_device: bool):
    if outputs_on_device:
        return DevicePairs(raw)
    m = int(raw.count)
    out = np.empty((m, 2), dtype=np.int32)
    if m:
        out[:, 0] = np.ctypeslib.as_array(C.cast(raw.a, C.POINTER(C.c_int32)), shape=(m,))
        out[:, 1] = np.ctypeslib.as_array(C.cast(raw.b, C.POINTER(C.c_int32)), shape=(m,))
    load().pj_pairs_free(C.byref(raw))
    return out


def pj_self_join(strings, tau: int, *, mode: int = MODE_AUTO, outputs_on_device: bool = False,
                 mem_budget: int = 0, stream=None, tune_cache: str | None = None,
                 selection: int = 0):
    """All pairs (a, b), a < b, of one string set with ED <= tau, as an int32 [m, 2] array
    sorted by (a, b).  selection: SELECT_* substring selection (multi-match by default)."""
    lib = load()
    s = _Marshalled(strings)
    o = _options(s.on_device, outputs_on_device, mode, mem_budget, stream, tune_cache,
                 selection)
    raw = PjPairs()
    _check(lib.pj_self_join(C.byref(s.s), int(tau), C.byref(o), C.byref(raw)))
    return _take_pairs(raw, outputs_on_device)


class Plan:
    """pj_self_join_plan / pj_plan_run / pj_plan_free: the self-join of one device-resident
    string set captured once in a hipGraph and replayed by run() (which checks first that the
    strings are unchanged, else joins them anew).  The device tensors are kept alive here."""

    def __init__(self, strings, tau: int, *, mode: int = MODE_AUTO, mem_budget: int = 0,
                 stream=None, tune_cache: str | None = None, selection: int = 0):
        lib = load()
        self._s = _Marshalled(strings)
        if not self._s.on_device:
            raise PassJoinError(PJ_EINVAL, "a plan takes device strings")
        o = _options(True, True, mode, mem_budget, stream, tune_cache, selection)
        self._h = C.c_void_p()
        _check(lib.pj_self_join_plan(C.byref(self._s.s), int(tau), C.byref(o), C.byref(self._h)))

    def run(self) -> DevicePairs:
        raw = PjPairs()
        _check(load().pj_plan_run(self._h, C.byref(raw)))
        return DevicePairs(raw)

    def free(self):
        if self._h:
            load().pj_plan_free(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def pj_self_join_host(strings, tau: int, *, mode: int = MODE_AUTO, mem_budget: int = 0,
                      stream=None, tune_cache: str | None = None, selection: int = 0) -> HostPairs:
    """pj_self_join of a host string set returning the library's host result arrays as they
    are (HostPairs: numpy views of a and b, released by free()), without the copy into an
    interleaved [m, 2] array."""
    lib = load()
    s = _Marshalled(strings)
    if s.on_device:
        raise PassJoinError(PJ_EINVAL, "pj_self_join_host takes host strings")
    o = _options(False, False, mode, mem_budget, stream, tune_cache, selection)
    raw = PjPairs()
    _check(lib.pj_self_join(C.byref(s.s), int(tau), C.byref(o), C.byref(raw)))
    return HostPairs(raw)


def pj_self_join_streamed(strings, tau: int, window_bytes: int, *, mode: int = MODE_AUTO,
                          mem_budget: int = 0, stream=None, tune_cache: str | None = None,
                          selection: int = 0):
    """pj_self_join of a host string set in length windows whose strings hold at most
    window_bytes bytes each (for sets larger than device memory); same result."""
    lib = load()
    s = _Marshalled(strings)
    if s.on_device:
        raise PassJoinError(PJ_EINVAL, "pj_self_join_streamed takes host strings")
    o = _options(False, False, mode, mem_budget, stream, tune_cache, selection)
    raw = PjPairs()
    _check(lib.pj_self_join_streamed(C.byref(s.s), int(tau), C.c_int64(int(window_bytes)),
                                     C.byref(o), C.byref(raw)))
    return _take_pairs(raw, False)


def pj_join(R, S, tau: int, *, mode: int = MODE_AUTO, outputs_on_device: bool = False,
            mem_budget: int = 0, stream=None, tune_cache: str | None = None,
            selection: int = 0):
    """All (r, s) with ED(R[r], S[s]) <= tau, int32 [m, 2] sorted by (r, s)."""
    lib = load()
    r = _Marshalled(R)
    s = _Marshalled(S)
    if r.on_device != s.on_device:
        raise PassJoinError(PJ_EINVAL, "R and S must both be on the host or both on the device")
    o = _options(s.on_device, outputs_on_device, mode, mem_budget, stream, tune_cache,
                 selection)
    raw = PjPairs()
    _check(lib.pj_join(C.byref(r.s), C.byref(s.s), int(tau), C.byref(o), C.byref(raw)))
    return _take_pairs(raw, outputs_on_device)


def pj_tune(strings, tau: int, *, tune_cache: str | None = None, mem_budget: int = 0,
            stream=None) -> dict:
    """Autotunes the batched path's launch parameters on the self-join of `strings` (host
    memory) at tau; the setting is kept for this process and, with tune_cache, merged into that
    file.  Returns the chosen setting and its timing."""
    lib = load()
    s = _Marshalled(strings)
    if s.on_device:
        raise PassJoinError(PJ_EINVAL, "pj_tune takes host strings")
    o = _options(False, False, MODE_BATCHED, mem_budget, stream, tune_cache)
    r = PjTuneResult()
    _check(lib.pj_tune(C.byref(s.s), int(tau), C.byref(o), C.byref(r)))
    return {k: getattr(r, k) for k, _ in PjTuneResult._fields_}


class Index:
    """A device-resident index (pj_build_index); released by free() or garbage collection."""

    def __init__(self, handle: int):
        self.handle = C.c_void_p(handle)

    def info(self) -> dict:
        return pj_index_info(self)

    def free(self):
        if self.handle:
            load().pj_index_free(self.handle)
            self.handle = C.c_void_p(None)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def pj_build_index(strings, tau_min: int, tau_max: int, *, mem_budget: int = 0,
                   stream=None) -> Index:
    lib = load()
    s = _Marshalled(strings)
    o = _options(s.on_device, False, MODE_AUTO, mem_budget, stream, None)
    h = C.c_void_p()
    _check(lib.pj_build_index(C.byref(s.s), int(tau_min), int(tau_max), C.byref(o), C.byref(h)))
    return Index(h.value)


def pj_index_info(index: Index) -> dict:
    n, tmin, tmax, nb = C.c_int64(), C.c_int32(), C.c_int32(), C.c_int64()
    _check(load().pj_index_info(index.handle, C.byref(n), C.byref(tmin), C.byref(tmax),
                                C.byref(nb)))
    return {"n": n.value, "tau_min": tmin.value, "tau_max": tmax.value, "device_bytes": nb.value}


def pj_index_free(index: Index):
    index.free()


def pj_query(index: Index, queries, taus, *, outputs_on_device: bool = False,
             mem_budget: int = 0, stream=None):
    """(q, s) pairs with ED(Q[q], S[s]) <= taus[q], int32 [m, 2] sorted by (q, s)."""
    lib = load()
    q = _Marshalled(queries)
    t = np.ascontiguousarray(taus, dtype=np.int32)
    if t.size != q.s.n:
        raise PassJoinError(PJ_EINVAL, "one tau per query is required")
    o = _options(q.on_device, outputs_on_device, MODE_AUTO, mem_budget, stream, None)
    raw = PjPairs()
    _check(lib.pj_query(index.handle, C.byref(q.s), t.ctypes.data if t.size else None,
                        C.byref(o), C.byref(raw)))
    return _take_pairs(raw, outputs_on_device)


def pj_query_noalloc(index: Index, queries, taus, out_q: np.ndarray, out_s: np.ndarray, *,
                     stream=None) -> int:
    """pj_query into caller-owned int32 arrays, with no allocation in the library (static
    device scratch).  Returns the number of pairs written to out_q[:m], out_s[:m]."""
    lib = load()
    q = _Marshalled(queries)
    if q.on_device:
        raise PassJoinError(PJ_EINVAL, "pj_query_noalloc takes host queries")
    t = np.ascontiguousarray(taus, dtype=np.int32)
    if t.size != q.s.n:
        raise PassJoinError(PJ_EINVAL, "one tau per query is required")
    for a in (out_q, out_s):
        if not (isinstance(a, np.ndarray) and a.dtype == np.int32 and a.flags.c_contiguous
                and a.flags.writeable):
            raise PassJoinError(PJ_EINVAL, "outputs must be writable contiguous int32 arrays")
    cap = min(out_q.size, out_s.size)
    o = _options(False, False, MODE_AUTO, 0, stream, None)
    m = C.c_int64(0)
    _check(lib.pj_query_noalloc(index.handle, C.byref(q.s), t.ctypes.data if t.size else None,
                                C.byref(o), out_q.ctypes.data, out_s.ctypes.data, cap,
                                C.byref(m)))
    return int(m.value)


class Server:
    """Serving loop over a resident index (pj_server_*): submit() returns a request id at once;
    wait(id) returns the request's (q, s) pairs and its timing info."""

    def __init__(self, index: Index, slots: int = 2, max_batch_queries: int = 256,
                 mem_budget: int = 0, tune_cache: str | None = None, eager: bool = False):
        self.index = index          # keeps the index alive while the server runs
        cfg = PjServerConfig(slots, max_batch_queries, int(mem_budget),
                             tune_cache.encode() if tune_cache else None, 1 if eager else 0)
        h = C.c_void_p()
        _check(load().pj_server_start(index.handle, C.byref(cfg), C.byref(h)))
        self.handle = h

    def submit(self, queries, taus) -> int:
        q = _Marshalled(queries)
        if q.on_device:
            raise PassJoinError(PJ_EINVAL, "server requests are host memory")
        t = np.ascontiguousarray(taus, dtype=np.int32)
        if t.size != q.s.n:
            raise PassJoinError(PJ_EINVAL, "one tau per query is required")
        rid = load().pj_server_submit(self.handle, C.byref(q.s), t.ctypes.data if t.size else None)
        if rid < 0:
            raise PassJoinError(int(rid), pj_last_error())
        return int(rid)

    def wait(self, rid: int):
        raw = PjPairs()
        info = PjRequestInfo()
        _check(load().pj_server_wait(self.handle, int(rid), C.byref(raw), C.byref(info)))
        pairs = _take_pairs(raw, False)
        return pairs, {k: getattr(info, k) for k, _ in PjRequestInfo._fields_}

    def stop(self):
        if self.handle:
            _check(load().pj_server_stop(self.handle))
            self.handle = C.c_void_p(None)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.stop()
