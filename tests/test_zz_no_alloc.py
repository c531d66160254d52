"""pj_query_noalloc (the query entry point that allocates nothing: its device work buffers are a
static device array) against pj_query on the same index and queries, through the C ABI: two
calls in a row, the second with a smaller batch, then the capacity errors.  Collected last
(its static device array keeps the last call's contents; it must pass after any other test and
alone in a fresh process)."""
import ctypes as C

import numpy as np
import pytest

import paper_1111_7171_amd as P
import workloads as W

pytestmark = pytest.mark.gpu


def _noalloc(idx, Q, taus, cap):
    fn = P.load().pj_query_noalloc          # the C entry point itself
    chars = np.ascontiguousarray(Q.chars, dtype=np.uint8)
    offs = np.ascontiguousarray(Q.offsets, dtype=np.int32)
    s = P.PjStrings(Q.n, chars.ctypes.data if chars.size else None, offs.ctypes.data)
    t = np.ascontiguousarray(taus, dtype=np.int32)
    oq = np.full(max(cap, 1), -1, np.int32)
    os_ = np.full(max(cap, 1), -1, np.int32)
    cnt = C.c_int64(-1)
    rc = fn(idx.handle, C.byref(s), t.ctypes.data if t.size else None, None, oq.ctypes.data,
            os_.ctypes.data, cap, C.byref(cnt))
    m = cnt.value
    return rc, np.stack([oq[:max(m, 0)], os_[:max(m, 0)]], axis=1) if rc == 0 else None, m


def test_noalloc_query_matches_pj_query_twice():
    S = W.cfg5_index(200_000)
    idx = P.pj_build_index(S, 1, 8)
    try:
        rng = np.random.default_rng(4242)
        big = [W.cfg5_batch(rng, S, mean=64) for _ in range(6)]
        Qa = W.concat([q for q, _ in big])
        ta = np.concatenate([t for _, t in big])
        Qb, tb = W.cfg5_batch(rng, S, mean=24)
        assert Qa.n > Qb.n
        for Q, t in ((Qa, ta), (Qb, tb)):
            print("noalloc query:", Q.n, "queries", flush=True)
            exp = P.pj_query(idx, Q, t)
            st_exp = P.pj_last_stats()
            rc, got, m = _noalloc(idx, Q, t, 8192)
            assert rc == 0, P.pj_last_error()
            st = P.pj_last_stats()
            assert m == len(exp) and np.array_equal(got, exp)
            for k in ("candidates", "cells", "selected", "side_pairs", "pairs"):
                assert st[k] == st_exp[k], k
        # beyond the capacities: clear errors, and the next call is still right
        Qc = W.concat([q for q, _ in big] * 2)
        tc = np.concatenate([t for _, t in big] * 2)
        if Qc.n > 512:
            rc, _, _ = _noalloc(idx, Qc, tc, 8192)
            assert rc == P.PJ_ERANGE and "queries" in P.pj_last_error()
        exp = P.pj_query(idx, Qb, tb)
        if len(exp) > 0:
            rc, _, m = _noalloc(idx, Qb, tb, len(exp) - 1)
            assert rc == P.PJ_ERANGE and m == len(exp)
        rc, got, m = _noalloc(idx, Qb, tb, 8192)
        assert rc == 0 and np.array_equal(got, exp)
    finally:
        idx.free()


def test_noalloc_binding_and_empty_batch():
    S = W.cfg5_index(5_000)
    idx = P.pj_build_index(S, 1, 4)
    try:
        rng = np.random.default_rng(77)
        Q, t = W.cfg5_batch(rng, S, mean=16, tau_max=4)
        exp = P.pj_query(idx, Q, t)
        oq = np.empty(8192, np.int32)
        os_ = np.empty(8192, np.int32)
        m = P.pj_query_noalloc(idx, Q, t, oq, os_)
        assert m == len(exp) and np.array_equal(np.stack([oq[:m], os_[:m]], axis=1), exp)
        empty = W.from_list([])
        assert P.pj_query_noalloc(idx, empty, np.zeros(0, np.int32), oq, os_) == 0
        with pytest.raises(P.PassJoinError) as ei:                 # tau outside the index
            P.pj_query_noalloc(idx, Q, np.full(Q.n, 5, np.int32), oq, os_)
        assert ei.value.code == P.PJ_ERANGE
    finally:
        idx.free()
