"""Self-join plans (pj_self_join_plan / pj_plan_run): the join's launches captured once in a
hipGraph and replayed.  Every replay gives pj_self_join's pairs and counts; replays alternate
with ordinary joins (eager work between graph launches); a plan whose strings changed joins
them anew and replays again once they are restored.  Every call goes through the C ABI."""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle as O
import paper_1111_7171_amd as P
import workloads as W

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    P.load()
    yield


def _dev(col):
    import torch
    return (torch.from_numpy(col.chars.copy()).to("cuda:0"),
            torch.from_numpy(col.offsets.copy()).to("cuda:0"))


def _eager(ds, tau, **kw):
    got = P.pj_self_join(ds, tau, outputs_on_device=True, **kw)
    pairs = got.to_numpy()
    got.free()
    return pairs, P.pj_last_stats()


def _replay(plan):
    got = plan.run()
    pairs = got.to_numpy()
    got.free()
    return pairs, P.pj_last_stats()


KEYS = ("selected", "hits", "candidates", "cells", "pairs", "side_pairs", "key_collisions")


@pytest.mark.parametrize("cfg,n,taus", [(2, 20_000, (1, 2, 3, 4)), (3, 6_000, (4, 8)),
                                        (4, 800, (8, 32))])
def test_replays_equal_self_join(cfg, n, taus):
    col = W.CONFIGS[cfg](n)
    ds = _dev(col)
    for tau in taus:
        exp, est = _eager(ds, tau)
        plan = P.Plan(ds, tau)
        for rep in range(3):
            _say(f"cfg{cfg} n={n} tau={tau} replay {rep}")
            got, st = _replay(plan)
            assert st["replayed"] == 1
            assert np.array_equal(got, exp), (cfg, tau, rep)
            for k in KEYS:
                assert st[k] == est[k], (cfg, tau, rep, k)
            # ordinary work between the graph's launches
            again, _ = _eager(ds, tau)
            assert np.array_equal(again, exp)
        plan.free()


@pytest.mark.parametrize("mode,selection", [(P.MODE_PLAIN, 0), (P.MODE_BATCHED, 1),
                                            (P.MODE_SHARE_PREFIX, 0)])
def test_modes_and_selection(mode, selection):
    rng = np.random.default_rng(4242)
    col = W.random_small(rng, 3000, alphabet=b"abcd", lmin=0, lmax=24, dup_frac=0.5, kmax=3)
    ds = _dev(col)
    for tau in (0, 2, 3):
        exp = O.self_join_bf(col, tau, 8)
        plan = P.Plan(ds, tau, mode=mode, selection=selection)
        for rep in range(2):
            got, st = _replay(plan)
            assert st["replayed"] == 1
            assert np.array_equal(got, exp), (mode, selection, tau, rep)
        plan.free()


def test_changed_strings_join_anew_then_replay():
    import torch
    col = W.cfg2(8000, seed=77)
    chars, offs = _dev(col)
    plan = P.Plan((chars, offs), 2)
    exp, _ = _eager((chars, offs), 2)
    got, st = _replay(plan)
    assert st["replayed"] == 1 and np.array_equal(got, exp)
    # change a few bytes in place: same sizes, other strings
    saved = chars[100:140].clone()
    chars[100:140] = torch.flip(saved, [0])
    torch.cuda.synchronize()
    exp2, _ = _eager((chars, offs), 2)
    got, st = _replay(plan)
    assert st["replayed"] == 0 and np.array_equal(got, exp2)
    # change the offsets (one string one byte longer, its neighbour one shorter)
    offs2 = offs.clone()
    offs[1] = offs2[1] + 1
    torch.cuda.synchronize()
    exp3, _ = _eager((chars, offs), 2)
    got, st = _replay(plan)
    assert st["replayed"] == 0 and np.array_equal(got, exp3)
    # restored: the plan replays again
    offs.copy_(offs2)
    chars[100:140] = saved
    torch.cuda.synchronize()
    got, st = _replay(plan)
    assert st["replayed"] == 1 and np.array_equal(got, exp)
    plan.free()


def test_full_size_cfg2_tau4_matches_oracle():
    """The benchmark's configuration: the replayed cfg2 self-join at tau = 4 (10^6 strings)
    hashes to the oracle's pair list, with the oracle's counts."""
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "fullsize.json")))
    e = gold["cfg2"]["taus"]["4"]
    col = W.cfg2()
    ds = _dev(col)
    plan = P.Plan(ds, 4)
    for rep in range(2):
        got, st = _replay(plan)
        assert st["replayed"] == 1
        sha = hashlib.sha256(np.ascontiguousarray(got, dtype="<i4").tobytes()).hexdigest()
        assert len(got) == e["pairs"] and sha == e["pairs_sha256"], rep
        for k in ("selected", "candidates", "cells", "side_pairs"):
            assert st[k] == e[k], (k, st[k], e[k])
    plan.free()
