"""Verification of long strings by row blocks (indexed strings longer than 128 bytes, tau <= 32):
candidates in slot order, passes of at most 64 rows per task, unfinished tasks carried to the
next pass with their band row.  Pairs, candidates and cells equal the oracle's, with the path on
(the default for such strings) and off (PJ_LONG_VERIFY=0, the per-candidate kernel)."""
import numpy as np
import pytest

import oracle as O
import paper_1111_7171_amd as P
import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _long_set(seed, n, tau, lmin=150, lmax=300):
    rng = np.random.default_rng(seed)
    return W.random_small(rng, n, alphabet=b"abcd", lmin=lmin, lmax=lmax, dup_frac=0.6,
                          kmax=tau + 2)


@pytest.mark.parametrize("tau", [3, 8, 13, 20, 27, 32])
def test_long_self_join_matches_oracle(tau, monkeypatch):
    col = _long_set(500 + tau, 500, tau)
    _say(f"long strings tau={tau} n={col.n}")
    exp = O.self_join_pj(col, tau)
    for flag in ("1", "0"):
        monkeypatch.setenv("PJ_LONG_VERIFY", flag)
        got = P.pj_self_join(col, tau)
        st = P.pj_last_stats()
        assert np.array_equal(got, exp.pairs), flag
        assert st["candidates"] == exp.candidates and st["cells"] == exp.cells, flag
    _say(f"  pairs {len(got)} candidates {exp.candidates} cells {exp.cells}")


def test_long_join_and_row_passes(monkeypatch):
    """Two sets, and strings long enough (up to 1,500 bytes) for many passes of 64 rows."""
    R = _long_set(61, 120, 16, lmin=600, lmax=1500)
    S = _long_set(62, 200, 16, lmin=600, lmax=1500)
    S = W.concat([S, R.subset(np.arange(0, R.n, 3))])        # exact copies: full-length passes
    for tau in (8, 16, 32):
        exp = O.join_pj(R, S, tau)
        monkeypatch.setenv("PJ_LONG_VERIFY", "1")
        got = P.pj_join(R, S, tau)
        st = P.pj_last_stats()
        assert np.array_equal(got, exp.pairs), tau
        assert st["candidates"] == exp.candidates and st["cells"] == exp.cells, tau


# library method -> oracle method
_METHODS = {P.SELECT_MULTIMATCH: O.SEL_MULTIMATCH, P.SELECT_POSITION: O.SEL_POSITION,
            P.SELECT_SHIFT: O.SEL_SHIFT, P.SELECT_LENGTH: O.SEL_LENGTH}


@pytest.mark.parametrize("tau", [4, 16, 32])
def test_long_strings_all_selection_methods(tau):
    """Long strings, hashed and exact segment keys (4 symbols: segments of up to 13 bytes are
    keyed exactly): the oracle's selected-substring, candidate and cell counts and pairs under
    every selection method, for a self-join and a two-set join."""
    col = _long_set(900 + tau, 300, tau, lmin=200, lmax=420)
    for meth, ometh in _METHODS.items():
        exp = O.self_join_pj(col, tau, method=ometh)
        got = P.pj_self_join(col, tau, selection=meth)
        st = P.pj_last_stats()
        assert np.array_equal(got, exp.pairs), meth
        assert (st["selected"], st["candidates"], st["cells"]) == \
            (exp.selected, exp.candidates, exp.cells), meth
    R = _long_set(950 + tau, 80, tau, lmin=200, lmax=420)
    jexp = O.join_pj(R, col, tau)
    jgot = P.pj_join(R, col, tau)
    jst = P.pj_last_stats()
    assert np.array_equal(jgot, jexp.pairs)
    assert (jst["selected"], jst["candidates"]) == (jexp.selected, jexp.candidates)


@pytest.mark.parametrize("passes", ["8,4096", "1,2,3", "64", "16,16,32,64,128,4096"])
def test_pass_schedules(passes, monkeypatch):
    """Any schedule of pass lengths (PJ_LONG_PASSES: rows per pass, the last repeated) gives
    the oracle's pairs, candidates and cells: a pass only decides where a task's rows are cut."""
    monkeypatch.setenv("PJ_LONG_PASSES", passes)
    for tau in (5, 24):
        col = _long_set(900 + tau, 400, tau, lmin=140, lmax=700)
        _say(f"long strings passes={passes} tau={tau}")
        exp = O.self_join_pj(col, tau)
        got = P.pj_self_join(col, tau)
        st = P.pj_last_stats()
        assert np.array_equal(got, exp.pairs), (passes, tau)
        assert st["candidates"] == exp.candidates and st["cells"] == exp.cells, (passes, tau)
