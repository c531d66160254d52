"""The four substring-selection methods (Sec. 4, 4.1, 4.2) on the GPU: each returns the
oracle's pairs, and its selected-substring, candidate and cell counts equal the oracle's
Pass-Join run with the same method.  Every call goes through the C ABI."""
import numpy as np
import pytest

import oracle as O
import paper_1111_7171_amd as P
import workloads as W

pytestmark = pytest.mark.gpu

# library method -> oracle method
METHODS = {
    P.SELECT_MULTIMATCH: O.SEL_MULTIMATCH,
    P.SELECT_POSITION: O.SEL_POSITION,
    P.SELECT_SHIFT: O.SEL_SHIFT,
    P.SELECT_LENGTH: O.SEL_LENGTH,
}


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    P.load()
    yield


def _check_counts(st, pj):
    assert st["selected"] == pj.selected
    assert st["candidates"] == pj.candidates
    assert st["cells"] == pj.cells


@pytest.mark.parametrize("mode", [P.MODE_PLAIN, P.MODE_BATCHED, "bucketed"])
@pytest.mark.parametrize("sel", list(METHODS))
def test_self_join_each_method(sel, mode, monkeypatch):
    if mode == "bucketed":
        monkeypatch.setenv("PJ_BUCKET_MIN_CANDIDATES", "0")
        mode = P.MODE_BATCHED
    col = W.cfg2(12_000, seed=41)
    for tau in (1, 2, 3):
        _say("selection", sel, "mode", mode, "tau", tau)
        got = P.pj_self_join(col, tau, mode=mode, selection=sel)
        st = P.pj_last_stats()
        pj = O.self_join_pj(col, tau, method=METHODS[sel])
        assert np.array_equal(got, pj.pairs), (sel, tau)
        _check_counts(st, pj)


@pytest.mark.parametrize("sel", list(METHODS))
def test_join_each_method(sel):
    rng = np.random.default_rng(51)
    R = W.random_small(rng, 400, alphabet=b"abcd", lmin=0, lmax=20, dup_frac=0.4, kmax=3)
    S = W.random_small(rng, 500, alphabet=b"abcd", lmin=0, lmax=20, dup_frac=0.4, kmax=3)
    for tau in (0, 1, 2, 3, 4):
        _say("join selection", sel, "tau", tau)
        got = P.pj_join(R, S, tau, selection=sel)
        st = P.pj_last_stats()
        pj = O.join_pj(R, S, tau, method=METHODS[sel])
        assert np.array_equal(got, O.join_bf(R, S, tau, 8)), (sel, tau)
        assert np.array_equal(got, pj.pairs)
        _check_counts(st, pj)


def test_methods_agree_and_nest():
    col = W.cfg1(3000)
    for tau in (1, 2, 3):
        res = {}
        for sel in METHODS:
            got = P.pj_self_join(col, tau, selection=sel)
            res[sel] = (got, P.pj_last_stats())
        base = res[P.SELECT_MULTIMATCH][0]
        for sel, (got, _) in res.items():
            assert np.array_equal(got, base), (sel, tau)
        order = [P.SELECT_MULTIMATCH, P.SELECT_POSITION, P.SELECT_SHIFT, P.SELECT_LENGTH]
        sel_counts = [res[s][1]["selected"] for s in order]
        cand_counts = [res[s][1]["candidates"] for s in order]
        assert sel_counts == sorted(sel_counts) and cand_counts == sorted(cand_counts)
