"""Shared-prefix verification (PJ_MODE_SHARE_PREFIX, Sec. 5.3): list members in content order,
each lane verifying a chain of consecutive members and resuming every DP after the rows a
member shares with its predecessor.  The pairs, candidates and cells (the cells of the method's
band, whether computed or taken over) equal the oracle's; some rows are actually shared."""
import numpy as np
import pytest

import oracle as O
import paper_1111_7171_amd as P
import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(autouse=True)
def _bucket_always(monkeypatch):
    # bucket the hits at any size, so that lists with >= 32 candidates reach the chain kernel
    monkeypatch.setenv("PJ_BUCKET_MIN_CANDIDATES", "0")


def _clustered(seed, n, alphabet=b"abc", lmin=6, lmax=24, kmax=3):
    rng = np.random.default_rng(seed)
    return W.random_small(rng, n, alphabet=alphabet, lmin=lmin, lmax=lmax, dup_frac=0.6, kmax=kmax)


@pytest.mark.parametrize("seed,tau", [(0, 1), (1, 2), (2, 3), (3, 4), (4, 6), (5, 8)])
def test_share_prefix_self_join_matches_oracle(seed, tau):
    # two symbols and segments of 2-4 characters: lists of dozens of members at every tau
    col = _clustered(100 + seed, 6000, alphabet=b"ab", lmin=2 * (tau + 1), lmax=4 * (tau + 1))
    _say(f"share-prefix self-join seed={seed} tau={tau} n={col.n}")
    exp = O.self_join_pj(col, tau)
    got = P.pj_self_join(col, tau, mode=P.MODE_SHARE_PREFIX)
    st = P.pj_last_stats()
    assert np.array_equal(got, exp.pairs)
    assert st["candidates"] == exp.candidates and st["cells"] == exp.cells
    assert 0 <= st["shared_cells"] <= st["cells"]
    _say(f"  pairs {len(got)} cells {st['cells']} shared cells {st['shared_cells']} "
         f"shared rows {st['shared_rows']} list launches {st['list_launches']}")
    assert st["list_launches"] == 1 and st["shared_rows"] > 0


@pytest.mark.parametrize("tau", [2, 4])
def test_share_prefix_cfg2_sample_and_join(tau):
    col = W.cfg2(40_000, seed=7)
    exp = O.self_join_pj(col, tau)
    got = P.pj_self_join(col, tau, mode=P.MODE_SHARE_PREFIX)
    st = P.pj_last_stats()
    assert np.array_equal(got, exp.pairs)
    assert st["candidates"] == exp.candidates and st["cells"] == exp.cells
    _say(f"cfg2 40k tau={tau}: shared cells {st['shared_cells']} of {st['cells']}")
    # two sets (every list member is a candidate: no visiting-order filter)
    R = col.subset(np.arange(0, col.n, 7))
    S = col.subset(np.arange(3, col.n, 2))
    jexp = O.join_pj(R, S, tau)
    jgot = P.pj_join(R, S, tau, mode=P.MODE_SHARE_PREFIX)
    jst = P.pj_last_stats()
    assert np.array_equal(jgot, jexp.pairs)
    assert jst["candidates"] == jexp.candidates and jst["cells"] == jexp.cells


def test_share_prefix_long_identical_parts():
    """Many members with identical long left and right parts (the whole-part and inherited-
    stop shortcuts) and near-identical ones differing beyond the stored rows."""
    rng = np.random.default_rng(9)
    base = bytes(rng.choice(list(b"xyz"), size=90))
    strs = []
    for k in range(400):
        s = bytearray(base)
        for _ in range(int(rng.integers(0, 4))):
            pos = int(rng.integers(len(s)))
            s[pos] = int(rng.choice(list(b"xyz")))
        strs.append(bytes(s))
    col = W.from_list(strs)
    for tau in (2, 5, 8):
        exp = O.self_join_pj(col, tau)
        got = P.pj_self_join(col, tau, mode=P.MODE_SHARE_PREFIX)
        st = P.pj_last_stats()
        assert np.array_equal(got, exp.pairs), tau
        assert st["candidates"] == exp.candidates and st["cells"] == exp.cells, tau
        assert st["shared_rows"] > 0


def test_share_prefix_high_tau_falls_back():
    col = _clustered(77, 600, lmax=60)
    exp = O.self_join_pj(col, 10)
    got = P.pj_self_join(col, 10, mode=P.MODE_SHARE_PREFIX)
    st = P.pj_last_stats()
    assert np.array_equal(got, exp.pairs) and st["cells"] == exp.cells
    assert st["shared_rows"] == 0
