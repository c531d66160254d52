"""CPU oracle for the Pass-Join similarity join -- TEST INFRASTRUCTURE.

Only the tests, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline`` leg may import
this package.  The GPU library never loads it, and it shares no code with the GPU library: the
arithmetic lives in ``pj_oracle.c`` (plain C, written out from the paper) and this module only
marshals arguments with ctypes.

Functions (paper sections in brackets):
  ed_full            textbook Levenshtein distance                         [Sec. 2, 5.1]
  ed_band            min(ED, t+1) by the 2t+1 band with prefix pruning     [Sec. 5.1]
  ed_band_rows       the same, with the last row computed                  [Sec. 5.1]
  partition          even partition (p_i, l_i)                             [Sec. 3.1]
  window             substring-selection window of one method              [Sec. 4, 4.1, 4.2]
  verify_pair        VerifyStringPair: length-aware band + early stop      [Sec. 5.1, Alg. 3]
  extension_verify   extension-based verification of one candidate         [Sec. 5.2, Alg. 3]
  self_join_bf       all pairs with ED <= tau (brute force)                [Definition 1]
  join_bf            all (r, s) with ED <= tau (brute force)               [Definition 1]
  partners_bf        partners of listed strings (brute force)              [Definition 1]
  self_join_pj       Pass-Join self-join with candidate/cell counts, any   [Alg. 1-3, Sec. 4]
                     of the four substring-selection methods
  join_pj            Pass-Join join of two sets                            [Sec. 3.2]
  *_parallel         the two runs split over processes by probe string (disjoint shares)
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pj_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

SEL_LENGTH, SEL_SHIFT, SEL_POSITION, SEL_MULTIMATCH = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compiles pj_oracle.c with gcc into liboracle.so next to it."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
                               "-pthread", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class _Result(C.Structure):
    _fields_ = [
        ("count", C.c_int64), ("a", C.POINTER(C.c_int32)), ("b", C.POINTER(C.c_int32)),
        ("candidates", C.c_int64), ("cells", C.c_int64), ("selected", C.c_int64),
        ("side_pairs", C.c_int64),
        ("ncand", C.c_int64), ("cy", C.POINTER(C.c_int32)), ("cx", C.POINTER(C.c_int32)),
        ("ci", C.POINTER(C.c_int32)), ("cp", C.POINTER(C.c_int32)),
        ("cpass", C.POINTER(C.c_int32)), ("ccells", C.POINTER(C.c_int64)),
        ("cap", C.c_int64), ("ccap", C.c_int64),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = C.CDLL(_LIB)
        u8p, i32p, i64p = C.c_void_p, C.c_void_p, C.c_void_p
        i32, i64 = C.c_int32, C.c_int64
        lib.orc_ed_full.argtypes = [u8p, i32, u8p, i32]
        lib.orc_ed_full.restype = i32
        lib.orc_ed_band.argtypes = [u8p, i32, u8p, i32, i32]
        lib.orc_ed_band.restype = i32
        lib.orc_ed_band_rows.argtypes = [u8p, i32, u8p, i32, i32, C.POINTER(i32)]
        lib.orc_ed_band_rows.restype = i32
        lib.orc_partition.argtypes = [i32, i32, i32p, i32p]
        lib.orc_partition.restype = None
        lib.orc_window.argtypes = [i32, i32, i32, i32, i32, C.POINTER(i32), C.POINTER(i32)]
        lib.orc_window.restype = i32
        lib.orc_verify_pair.argtypes = [u8p, i32, u8p, i32, i32, C.POINTER(i64), C.POINTER(i32)]
        lib.orc_verify_pair.restype = i32
        lib.orc_extension_verify.argtypes = [u8p, i32, u8p, i32, i32, i32, i32, C.POINTER(i64)]
        lib.orc_extension_verify.restype = i32
        rp = C.POINTER(_Result)
        lib.orc_self_join_bf.argtypes = [u8p, i32p, i64, i32, i32]
        lib.orc_self_join_bf.restype = rp
        lib.orc_join_bf.argtypes = [u8p, i32p, i64, u8p, i32p, i64, i32, i32]
        lib.orc_join_bf.restype = rp
        lib.orc_partners_bf.argtypes = [u8p, i32p, i64, i32p, i64, i32, i32]
        lib.orc_partners_bf.restype = rp
        lib.orc_self_join_pj.argtypes = [u8p, i32p, i64, i32, i32, i32, i32, i32, i32]
        lib.orc_self_join_pj.restype = rp
        lib.orc_join_pj.argtypes = [u8p, i32p, i64, u8p, i32p, i64, i32, i32, i32, i32, i32]
        lib.orc_join_pj.restype = rp
        lib.orc_result_free.argtypes = [rp]
        lib.orc_result_free.restype = None
        _lib = lib
    return _lib


def _buf(b: bytes):
    """A ctypes pointer to a copy of b (kept alive by the returned array)."""
    arr = np.frombuffer(b if b else b"\0", dtype=np.uint8).copy()
    return arr, arr.ctypes.data


def _arena(col):
    chars = np.ascontiguousarray(col.chars, dtype=np.uint8)
    if chars.size == 0:
        chars = np.zeros(1, dtype=np.uint8)
    offs = np.ascontiguousarray(col.offsets, dtype=np.int32)
    return chars, offs


@dataclass
class JoinResult:
    pairs: np.ndarray            # int32[m, 2], sorted by (a, b), unique
    candidates: int = 0
    cells: int = 0
    selected: int = 0
    side_pairs: int = 0
    cands: dict | None = None    # y, x, i, p, pass, cells arrays when requested


def _take(rp, keep_cands: bool = False) -> JoinResult:
    r = rp.contents
    m = int(r.count)
    pairs = np.empty((m, 2), dtype=np.int32)
    if m:
        pairs[:, 0] = np.ctypeslib.as_array(r.a, shape=(m,))
        pairs[:, 1] = np.ctypeslib.as_array(r.b, shape=(m,))
    cands = None
    if keep_cands:
        k = int(r.ncand)
        def arr(p, dt):
            return np.ctypeslib.as_array(p, shape=(k,)).astype(dt) if k else np.empty(0, dt)
        cands = {"y": arr(r.cy, np.int32), "x": arr(r.cx, np.int32), "i": arr(r.ci, np.int32),
                 "p": arr(r.cp, np.int32), "pass": arr(r.cpass, np.int32),
                 "cells": arr(r.ccells, np.int64)}
    out = JoinResult(pairs, int(r.candidates), int(r.cells), int(r.selected), int(r.side_pairs),
                     cands)
    _load().orc_result_free(rp)
    return out


def ed_full(r: bytes, s: bytes) -> int:
    ra, rp = _buf(r)
    sa, sp = _buf(s)
    return int(_load().orc_ed_full(rp, len(r), sp, len(s)))


def ed_band(r: bytes, s: bytes, t: int) -> int:
    ra, rp = _buf(r)
    sa, sp = _buf(s)
    return int(_load().orc_ed_band(rp, len(r), sp, len(s), t))


def ed_band_rows(r: bytes, s: bytes, t: int) -> tuple[int, int]:
    """(min(ED, t+1), last row computed) of the 2t+1 band with prefix pruning."""
    ra, rp = _buf(r)
    sa, sp = _buf(s)
    rows = C.c_int32()
    d = _load().orc_ed_band_rows(rp, len(r), sp, len(s), t, C.byref(rows))
    return int(d), int(rows.value)


def partition(l: int, tau: int) -> list[tuple[int, int]]:
    """[(p_1, l_1), ..., (p_{tau+1}, l_{tau+1})], 1-based starts."""
    st = np.zeros(tau + 1, dtype=np.int32)
    ln = np.zeros(tau + 1, dtype=np.int32)
    _load().orc_partition(l, tau, st.ctypes.data, ln.ctypes.data)
    return list(zip(st.tolist(), ln.tolist()))


def window(method: int, n: int, l: int, tau: int, i: int) -> tuple[int, int]:
    lo, hi = C.c_int32(), C.c_int32()
    _load().orc_window(method, n, l, tau, i, C.byref(lo), C.byref(hi))
    return int(lo.value), int(hi.value)


def verify_pair(r: bytes, s: bytes, t: int) -> tuple[int, int, int]:
    """(min(t+1, ED), cells, last row computed); r = indexed part, s = probe part."""
    ra, rp = _buf(r)
    sa, sp = _buf(s)
    cells, rows = C.c_int64(), C.c_int32()
    d = _load().orc_verify_pair(rp, len(r), sp, len(s), t, C.byref(cells), C.byref(rows))
    return int(d), int(cells.value), int(rows.value)


def extension_verify(x: bytes, y: bytes, tau: int, i: int, p: int) -> tuple[bool, int]:
    """(pass, cells) for candidate (y, x, i, p): x probe string, y indexed string."""
    xa, xp = _buf(x)
    ya, yp = _buf(y)
    cells = C.c_int64()
    ok = _load().orc_extension_verify(xp, len(x), yp, len(y), tau, i, p, C.byref(cells))
    return bool(ok), int(cells.value)


def self_join_bf(col, tau: int, nthreads: int = 0) -> np.ndarray:
    ch, of = _arena(col)
    nt = nthreads or os.cpu_count() or 1
    return _take(_load().orc_self_join_bf(ch.ctypes.data, of.ctypes.data, col.n, tau, nt)).pairs


def join_bf(R, S, tau: int, nthreads: int = 0) -> np.ndarray:
    rc, ro = _arena(R)
    sc, so = _arena(S)
    nt = nthreads or os.cpu_count() or 1
    return _take(_load().orc_join_bf(rc.ctypes.data, ro.ctypes.data, R.n, sc.ctypes.data,
                                     so.ctypes.data, S.n, tau, nt)).pairs


def partners_bf(col, xs, tau: int, nthreads: int = 0) -> np.ndarray:
    """(min, max) pairs of every listed x with each other string within distance tau."""
    ch, of = _arena(col)
    xs = np.ascontiguousarray(xs, dtype=np.int32)
    nt = nthreads or os.cpu_count() or 1
    return _take(_load().orc_partners_bf(ch.ctypes.data, of.ctypes.data, col.n, xs.ctypes.data,
                                         len(xs), tau, nt)).pairs


def self_join_pj(col, tau: int, tiebreak: int = 0, probe_stride: int = 1,
                 keep_cands: bool = False, method: int = SEL_MULTIMATCH,
                 probe_offset: int = 0) -> JoinResult:
    """Pass-Join self-join; tiebreak 0 visits equal lengths by id, 1 by bytes (the paper's
    alphabetical order).  With probe_stride k > 1 only the strings at visiting ranks
    r = probe_offset (mod k) probe; every string is still indexed.  method is the substring
    selection (SEL_*; multi-match, Sec. 4.2, by default)."""
    ch, of = _arena(col)
    rp = _load().orc_self_join_pj(ch.ctypes.data, of.ctypes.data, col.n, tau, tiebreak,
                                  probe_stride, probe_offset, int(keep_cands), int(method))
    return _take(rp, keep_cands)


def join_pj(R, S, tau: int, keep_cands: bool = False,
            method: int = SEL_MULTIMATCH, probe_stride: int = 1,
            probe_offset: int = 0) -> JoinResult:
    """Pass-Join join of two sets; with probe_stride k > 1 only the r = probe_offset (mod k)
    probe."""
    rc, ro = _arena(R)
    sc, so = _arena(S)
    rp = _load().orc_join_pj(rc.ctypes.data, ro.ctypes.data, R.n, sc.ctypes.data,
                             so.ctypes.data, S.n, tau, int(keep_cands), int(method),
                             probe_stride, probe_offset)
    return _take(rp, keep_cands)


# ---- the same runs split over processes --------------------------------------------------
#
# The probe strings are dealt round-robin to k worker processes (probe offset w of stride k).
# Each worker runs the unchanged sequential algorithm: it indexes every string in visiting order
# and probes only with its own share.  A pair is found only by its later-visited string (self-
# join) or by its r (join), so the shares' pair lists are disjoint and their counters add up to
# the single-process run's.

_SHARED: dict = {}


def _self_share(args):
    tau, k, w, method = args
    r = self_join_pj(_SHARED["col"], tau, probe_stride=k, probe_offset=w, method=method)
    return r.pairs, r.candidates, r.cells, r.selected, r.side_pairs


def _join_share(args):
    tau, k, w, method = args
    r = join_pj(_SHARED["R"], _SHARED["S"], tau, method=method, probe_stride=k, probe_offset=w)
    return r.pairs, r.candidates, r.cells, r.selected, r.side_pairs


def _run_shares(fn, shared: dict, tau: int, procs: int, method: int, shares: int | None = None,
                only: list | None = None) -> JoinResult:
    import multiprocessing as mp
    k = max(1, int(shares or procs))
    todo = list(range(k)) if only is None else list(only)
    _SHARED.clear()
    _SHARED.update(shared)
    _load()
    try:
        if procs <= 1 or len(todo) <= 1:
            parts = [fn((tau, k, w, method)) for w in todo]
        else:
            ctx = mp.get_context("fork")        # workers inherit the arena without copying it
            with ctx.Pool(min(procs, len(todo))) as pool:
                parts = pool.map(fn, [(tau, k, w, method) for w in todo], chunksize=1)
    finally:
        _SHARED.clear()
    pairs = np.concatenate([p[0] for p in parts]) if parts else np.empty((0, 2), np.int32)
    if len(pairs):
        key = pairs[:, 0].astype(np.int64) << 32 | pairs[:, 1].astype(np.int64)
        order = np.argsort(key, kind="stable")
        pairs = pairs[order]
    return JoinResult(np.ascontiguousarray(pairs, dtype=np.int32),
                      sum(int(p[1]) for p in parts), sum(int(p[2]) for p in parts),
                      sum(int(p[3]) for p in parts), sum(int(p[4]) for p in parts))


def self_join_pj_parallel(col, tau: int, procs: int = 0, method: int = SEL_MULTIMATCH,
                          shares: int | None = None, only: list | None = None) -> JoinResult:
    """self_join_pj split over `procs` processes (default: every CPU).  `shares` (default procs)
    is the number of probe offsets; `only` restricts the run to some of them (a sample)."""
    procs = procs or os.cpu_count() or 1
    return _run_shares(_self_share, {"col": col}, tau, procs, method, shares, only)


def join_pj_parallel(R, S, tau: int, procs: int = 0, method: int = SEL_MULTIMATCH,
                     shares: int | None = None, only: list | None = None) -> JoinResult:
    """join_pj split over `procs` processes (default: every CPU)."""
    procs = procs or os.cpu_count() or 1
    return _run_shares(_join_share, {"R": R, "S": S}, tau, procs, method, shares, only)
