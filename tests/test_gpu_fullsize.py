"""Parity at the full workload sizes, in the launch configuration the benchmark times
(batched mode, inputs and outputs in HBM).  The oracle cannot join 10^5-10^6 strings, so each
case checks: (1) for a seeded sample of strings, the partners the GPU reports equal the
brute-force partners by Definition 1; (2) a sample of reported pairs has ED <= tau (textbook
DP); (3) the list is sorted, unique and a < b."""
import numpy as np
import pytest

import oracle as O
import paper_1111_7171_amd as P
import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _device(col):
    import torch
    return (torch.from_numpy(col.chars.copy()).cuda(), torch.from_numpy(col.offsets.copy()).cuda())


def _check(col, pairs, tau, nsample, seed):
    assert pairs.ndim == 2 and pairs.shape[1] == 2
    a, b = pairs[:, 0].astype(np.int64), pairs[:, 1].astype(np.int64)
    assert np.all(a < b)
    key = a * col.n + b
    assert np.all(np.diff(key) > 0), "not sorted / not unique"
    rng = np.random.default_rng(seed)
    xs = np.sort(rng.choice(col.n, size=nsample, replace=False)).astype(np.int32)
    exp = O.partners_bf(col, xs, tau)
    sel = np.isin(a, xs) | np.isin(b, xs)
    got = pairs[sel]
    assert np.array_equal(got, exp), (len(got), len(exp))
    if len(pairs):
        pick = rng.choice(len(pairs), size=min(300, len(pairs)), replace=False)
        for k in pick:
            assert O.ed_full(col.get(int(pairs[k, 0])), col.get(int(pairs[k, 1]))) <= tau


@pytest.fixture(scope="module")
def cfg2():
    return W.cfg2()


@pytest.fixture(scope="module")
def cfg2_tuned(cfg2, tmp_path_factory):
    """The launch parameters bench.py times: tuned on this workload, per tau."""
    cache = str(tmp_path_factory.mktemp("tune") / "tune.txt")
    for tau in (1, 2, 3, 4):
        _say("tuning cfg2 tau", tau)
        P.pj_tune(cfg2, tau, tune_cache=cache)
    return cache


def _join_dev(col, tau, **kw):
    dp = P.pj_self_join(_device(col), tau, outputs_on_device=True, **kw)
    try:
        return dp.to_numpy(), P.pj_last_stats()
    finally:
        dp.free()


@pytest.mark.parametrize("tau", [1, 2, 3, 4])
def test_cfg2_full(cfg2, cfg2_tuned, tau):
    _say("cfg2 full tau", tau, "(tuned launch parameters)")
    pairs, st = _join_dev(cfg2, tau, tune_cache=cfg2_tuned)
    _say("  pairs", len(pairs), "candidates", st["candidates"])
    _check(cfg2, pairs, tau, 64, 100 + tau)
    # the built-in defaults give the same result and the same counts
    pairs0, st0 = _join_dev(cfg2, tau)
    assert np.array_equal(pairs0, pairs)
    for k in ("candidates", "cells", "accepted", "hits", "selected"):
        assert st0[k] == st[k], k


@pytest.mark.parametrize("tau", [2, 4, 6, 8])
def test_cfg3_full(tau):
    col = W.cfg3()
    _say("cfg3 full tau", tau)
    pairs = P.pj_self_join(_device(col), tau)
    _say("  pairs", len(pairs), "candidates", P.pj_last_stats()["candidates"])
    _check(col, pairs, tau, 48, 200 + tau)


@pytest.mark.parametrize("tau", [8, 16, 32])
def test_cfg4_full(tau):
    col = W.cfg4()
    _say("cfg4 full tau", tau)
    pairs = P.pj_self_join(_device(col), tau)
    _say("  pairs", len(pairs), "candidates", P.pj_last_stats()["candidates"])
    _check(col, pairs, tau, 24, 300 + tau)


def test_serving_index_full():
    S = W.cfg5_index()
    idx = P.pj_build_index(S, 1, 8)
    rng = np.random.default_rng(77)
    try:
        for _ in range(1):
            Q, taus = W.cfg5_batch(rng, S)
            got = P.pj_query(idx, Q, taus)
            exp = []
            for t in range(1, 9):
                ids = np.nonzero(taus == t)[0]
                if len(ids):
                    for a, b in O.join_bf(Q.subset(ids), S, t).tolist():
                        exp.append((int(ids[a]), b))
            exp = np.array(sorted(exp), dtype=np.int32).reshape(-1, 2)
            assert np.array_equal(got, exp)
    finally:
        idx.free()
