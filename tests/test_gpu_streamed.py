"""Self-join in length windows (pj_self_join_streamed): the same pairs as the whole-set join and
the brute-force oracle for window sizes down to a single length, and the same candidate, cell
and selected-substring counts as the whole-set join (every probe string still probes all of its
lengths, within its own window).  Every call goes through the C ABI."""
import numpy as np
import pytest

import oracle as O
import paper_1111_7171_amd as P
import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    P.load()
    yield


@pytest.mark.parametrize("seed", range(4))
def test_small_windows_match_bruteforce(seed):
    rng = np.random.default_rng(700 + seed)
    alph = [b"ab", b"abc", b"abcd", b"abcdefgh"][seed % 4]
    col = W.random_small(rng, 500, alphabet=alph, lmin=0, lmax=18, dup_frac=0.4, kmax=3)
    for tau in range(0, 6):
        bf = O.self_join_bf(col, tau, 8)
        for wb in (1, 60, 400, 1 << 30):   # one length per window ... one window
            _say("streamed seed", seed, "tau", tau, "window_bytes", wb)
            got = P.pj_self_join_streamed(col, tau, wb)
            assert np.array_equal(got, bf), (seed, tau, wb)


@pytest.mark.parametrize("mode", [P.MODE_PLAIN, P.MODE_BATCHED])
def test_cfg2_windows_same_pairs_and_counts(mode):
    col = W.cfg2(20_000, seed=61)
    arena = int(col.offsets[-1])
    for tau in (1, 2, 3, 4):
        whole = P.pj_self_join(col, tau, mode=mode)
        sw = P.pj_last_stats()
        for parts in (3, 8):
            _say("cfg2 streamed tau", tau, "parts", parts, "mode", mode)
            got = P.pj_self_join_streamed(col, tau, arena // parts, mode=mode)
            st = P.pj_last_stats()
            assert np.array_equal(got, whole), (tau, parts)
            for k in ("selected", "candidates", "cells", "pairs"):
                assert st[k] == sw[k], (tau, parts, k)


@pytest.mark.parametrize("cap", [1, 700, 20_000])
def test_key_batches_moved_to_host(cap, monkeypatch):
    """Windows' pairs held on the device in batches of at most `cap` keys (a batch that would
    pass it is sorted and moved to the host first, and the host merges the runs): the same
    pairs as the whole-set join, for one window per batch up to every window in one batch."""
    col = W.cfg2(20_000, seed=62)
    arena = int(col.offsets[-1])
    monkeypatch.setenv("PJ_STREAM_KEY_CAP", str(cap))
    for tau in (1, 3):
        whole = P.pj_self_join(col, tau)
        _say("streamed key cap", cap, "tau", tau)
        got = P.pj_self_join_streamed(col, tau, arena // 8)
        assert np.array_equal(got, whole), (cap, tau)
