"""Serving loop: each request's result is the same alone and in the mix (tolerance 0: the
method is exact), admission by footprint, oversize rejection, draining on stop."""
import threading

import numpy as np
import pytest

import oracle as O
import paper_1111_7171_amd as P
import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def served():
    import torch
    assert torch.cuda.is_available()
    S = W.cfg5_index(20_000)
    idx = P.pj_build_index(S, 1, 8)
    rng = np.random.default_rng(4242)
    batches = [W.cfg5_batch(rng, S, mean=24) for _ in range(24)]
    alone = [P.pj_query(idx, q, t) for q, t in batches]
    yield S, idx, batches, alone
    idx.free()


def test_alone_equals_oracle(served):
    S, idx, batches, alone = served
    for (q, t), got in list(zip(batches, alone))[:3]:
        exp = []
        for tau in range(1, 9):
            ids = np.nonzero(t == tau)[0]
            if len(ids):
                for a, b in O.join_pj(q.subset(ids), S, tau).pairs.tolist():
                    exp.append((int(ids[a]), b))
        exp = np.array(sorted(exp), dtype=np.int32).reshape(-1, 2)
        assert np.array_equal(got, exp)


def test_mix_equals_alone(served):
    S, idx, batches, alone = served
    with P.Server(idx, slots=3, max_batch_queries=80) as srv:
        ids = [srv.submit(q, t) for q, t in batches]       # all at once: they get merged
        res = [srv.wait(i) for i in ids]
    merged = 0
    for (pairs, info), exp in zip(res, alone):
        assert np.array_equal(pairs, exp)
        merged += info["batch_requests"] > 1
        assert info["t_submit_ms"] <= info["t_admit_ms"] <= info["t_done_ms"]
    _say("requests sharing a device batch:", merged)
    assert merged > 0


def test_concurrent_submitters(served):
    S, idx, batches, alone = served
    out = {}
    with P.Server(idx, slots=2, max_batch_queries=64) as srv:
        def client(k0):
            for k in range(k0, len(batches), 3):
                rid = srv.submit(*batches[k])
                out[k] = srv.wait(rid)[0]
        th = [threading.Thread(target=client, args=(k,)) for k in range(3)]
        for t in th:
            t.start()
        for t in th:
            t.join()
    for k, exp in enumerate(alone):
        assert np.array_equal(out[k], exp)


def test_tiny_budget_admits_one_at_a_time(served):
    S, idx, batches, alone = served
    lib = P.load()
    # footprints are reported per request; a budget just above the largest single one forces
    # batches to run (mostly) alone
    with P.Server(idx, slots=4, max_batch_queries=1000) as srv:
        probe = srv.submit(*batches[0])
        fp = srv.wait(probe)[1]["footprint_bytes"]
    budget = int(fp * 3)
    # a captured server keeps fixed buffers per slot, taken off the budget at start: a budget
    # below them is refused
    with pytest.raises(P.PassJoinError) as ei:
        P.Server(idx, slots=4, max_batch_queries=1000, mem_budget=budget)
    assert ei.value.code == P.PJ_ENOMEM and "fixed buffers" in str(ei.value)
    # uncaptured slots hold no fixed buffers: the whole budget goes to admission
    with P.Server(idx, slots=4, max_batch_queries=1000, mem_budget=budget, eager=True) as srv:
        ok_ids = []
        for q, t in batches:
            try:
                ok_ids.append((srv.submit(q, t), q, t))
            except P.PassJoinError as e:
                assert e.code == P.PJ_ENOMEM
                ok_ids.append((None, q, t))
        for (rid, q, t), exp in zip(ok_ids, alone):
            if rid is not None:
                pairs, info = srv.wait(rid)
                assert np.array_equal(pairs, exp)
                assert info["footprint_bytes"] <= budget
    assert lib is not None


def test_oversize_request_rejected(served):
    S, idx, batches, alone = served
    with P.Server(idx, slots=1, max_batch_queries=10, mem_budget=1024, eager=True) as srv:
        with pytest.raises(P.PassJoinError) as ei:
            srv.submit(*batches[0])
        assert ei.value.code == P.PJ_ENOMEM
        with pytest.raises(P.PassJoinError) as ei:
            srv.submit(batches[0][0], np.full(batches[0][0].n, 9, np.int32))
        assert ei.value.code in (P.PJ_ERANGE, P.PJ_ENOMEM)


def test_stop_drains_pending(served):
    S, idx, batches, alone = served
    srv = P.Server(idx, slots=1, max_batch_queries=8)
    ids = [srv.submit(q, t) for q, t in batches[:8]]
    got = [srv.wait(i)[0] for i in ids[:2]]
    srv.stop()
    for g, e in zip(got, alone[:2]):
        assert np.array_equal(g, e)


def test_captured_and_uncaptured_batches_agree(served):
    """Each slot replays one captured graph per batch; the uncaptured path (eager=True) gives
    the same pairs for the same merged batches."""
    S, idx, batches, alone = served
    for eager in (False, True):
        with P.Server(idx, slots=2, max_batch_queries=64, eager=eager) as srv:
            ids = [srv.submit(q, t) for q, t in batches]
            res = [srv.wait(i) for i in ids]
        for (pairs, _), exp in zip(res, alone):
            assert np.array_equal(pairs, exp), f"eager={eager}"


def test_captured_batch_falls_back_on_overflow():
    """A batch with more accepted pairs than the captured pipeline can sort, and a request
    with more queries than the plan holds, run uncaptured and still give the exact result."""
    rng = np.random.default_rng(77)
    hot = b"abcdefghij"
    strs = [hot] * 300 + [bytes(rng.integers(97, 123, size=int(rng.integers(5, 30))).astype(np.uint8))
                          for _ in range(2000)]
    S = W.from_list(strs)
    idx = P.pj_build_index(S, 1, 3)
    try:
        Q = W.from_list([hot] * 40)               # 40 x 300 pairs > the sort capacity
        T = np.ones(40, np.int32)
        exp = P.pj_query(idx, Q, T)
        assert len(exp) == 12000
        big = W.from_list([bytes(rng.integers(97, 123, size=12).astype(np.uint8))
                           for _ in range(50)] + [hot])
        TB = rng.integers(1, 4, size=big.n).astype(np.int32)
        exp_big = P.pj_query(idx, big, TB)
        with P.Server(idx, slots=1, max_batch_queries=40) as srv:
            got, _ = srv.wait(srv.submit(Q, T))
            got_big, _ = srv.wait(srv.submit(big, TB))   # 51 queries > 40
        assert np.array_equal(got, exp)
        assert np.array_equal(got_big, exp_big)
    finally:
        idx.free()


@pytest.mark.parametrize("seed", range(2))
def test_captured_batches_with_short_strings(seed):
    """Indexed and query strings shorter than tau + 1 (the side path inside the captured graph),
    per-query thresholds from 0 to 6: the server's pairs equal pj_query's and the oracle's."""
    rng = np.random.default_rng(5000 + seed)
    S = W.random_small(rng, 400, alphabet=b"abc", lmin=0, lmax=12, dup_frac=0.4)
    idx = P.pj_build_index(S, 0, 6)
    try:
        reqs = []
        for _ in range(6):
            Q = W.random_small(rng, 40, alphabet=b"abc", lmin=0, lmax=12, dup_frac=0.2)
            reqs.append((Q, rng.integers(0, 7, size=Q.n).astype(np.int32)))
        with P.Server(idx, slots=2, max_batch_queries=128) as srv:
            ids = [srv.submit(q, t) for q, t in reqs]
            got = [srv.wait(i)[0] for i in ids]
        for (Q, T), g in zip(reqs, got):
            exp = []
            for t in range(0, 7):
                ids_t = np.nonzero(T == t)[0]
                if len(ids_t):
                    for a, b in O.join_bf(Q.subset(ids_t), S, t, 4).tolist():
                        exp.append((int(ids_t[a]), b))
            exp = np.array(sorted(exp), dtype=np.int32).reshape(-1, 2)
            assert np.array_equal(g, exp)
            assert np.array_equal(g, P.pj_query(idx, Q, T))
    finally:
        idx.free()


def test_captured_batches_index_tau_range_above_zero():
    """An index over tau 2..5 served with thresholds in that range (captured path)."""
    S = W.cfg5_index(5_000)
    rng = np.random.default_rng(88)
    idx = P.pj_build_index(S, 2, 5)
    try:
        Q, _ = W.cfg5_batch(rng, S, mean=48)
        T = rng.integers(2, 6, size=Q.n).astype(np.int32)
        exp = P.pj_query(idx, Q, T)
        with P.Server(idx, slots=1) as srv:
            got, _ = srv.wait(srv.submit(Q, T))
        assert np.array_equal(got, exp)
        with pytest.raises(P.PassJoinError):
            with P.Server(idx, slots=1) as srv:
                srv.submit(Q, np.ones(Q.n, np.int32))       # tau 1 is outside the index
    finally:
        idx.free()
