"""Autotuner: launch parameters never change a result.  pj_tune writes a cache line that later
joins read; settings written into the cache by hand (the extremes of every parameter) give the
oracle's pairs, candidate count and cell count.  Every call goes through the C ABI."""
import numpy as np
import pytest

import oracle as O
import paper_1111_7171_amd as P
import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _len_bucket(col):
    mean = (col.offsets[-1] - col.offsets[0]) / max(col.n, 1)
    return int(mean + 0.5).bit_length()


def _read_cache(path):
    # v3 lines: arch tau len_bucket and six parameters (the last the probe's thread mapping), ms
    rows = []
    for line in open(path):
        if line.startswith("#"):
            continue
        f = line.split()
        assert len(f) == 10, line
        rows.append((f[0], int(f[1]), int(f[2]), tuple(int(v) for v in f[3:9]), float(f[9])))
    return rows


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    P.load()
    yield


def test_pj_tune_writes_cache_and_keeps_results(tmp_path):
    col = W.cfg2(20_000, seed=21)
    cache = str(tmp_path / "tune.txt")
    _say("pj_tune cfg2 n=20000 tau=3")
    r = P.pj_tune(col, 3, tune_cache=cache)
    assert r["verify_waves_per_cu"] in (8, 16, 32, 64, 128, 256, 512, 1024)
    assert r["seg_chunk"] in (1, 2, 4, 8, 16, 32, 64, 128, 256, 512, 1024, 2048)
    assert r["big_list"] in (16, 32, 64, 128)
    assert r["probe_blocks_per_cu"] in (4, 8, 16)
    assert r["lane_cands"] in (1, 2)
    assert r["probe_map"] in (0, 1)
    assert r["len_bucket"] == _len_bucket(col)
    assert r["trials"] >= 10 and 0 < r["ms_best"] <= r["ms_default"]
    rows = _read_cache(cache)
    assert len(rows) == 1
    arch, tau, lb, params, ms = rows[0]
    assert arch.startswith("gfx") and tau == 3 and lb == r["len_bucket"]
    assert params == (r["verify_waves_per_cu"], r["seg_chunk"], r["big_list"],
                      r["probe_blocks_per_cu"], r["lane_cands"], r["probe_map"])
    plain = P.pj_self_join(col, 3)
    st0 = P.pj_last_stats()
    tuned = P.pj_self_join(col, 3, tune_cache=cache)
    st1 = P.pj_last_stats()
    assert np.array_equal(plain, tuned)
    for k in ("candidates", "cells", "accepted", "pairs"):
        assert st0[k] == st1[k], k
    # a second tau is merged into the same file
    P.pj_tune(col, 2, tune_cache=cache)
    assert sorted(t for _, t, _, _, _ in _read_cache(cache)) == [2, 3]


# six values: a v3 line (the last is the probe's thread mapping); five: a v2 line (mapping 0)
@pytest.mark.parametrize("params", [(8, 1, 16, 4, 1, 1), (512, 512, 128, 16, 2, 0),
                                    (16, 2, 64, 8, 2, 1), (32, 4, 32, 8, 1)])
def test_forced_settings_match_oracle(tmp_path, monkeypatch, params):
    # the list-segment kernel at these sizes needs the slot bucketing forced on
    monkeypatch.setenv("PJ_BUCKET_MIN_CANDIDATES", "0")
    col = W.cfg2(20_000, seed=22)
    cache = str(tmp_path / "tune.txt")
    probe = W.cfg2(2_000, seed=23)
    P.pj_tune(probe, 0, tune_cache=cache)          # learns this GPU's architecture name
    arch = _read_cache(cache)[0][0]
    lb = _len_bucket(col)
    with open(cache, "w") as f:
        f.write(f"# passjoin tune cache v{3 if len(params) == 6 else 2}\n")
        for tau in (1, 2, 3, 4):
            f.write(f"{arch} {tau} {lb} {' '.join(map(str, params))} 1.0\n")
    for tau in (1, 2, 3, 4):
        _say("forced", params, "tau", tau)
        pj = O.self_join_pj(col, tau)
        got = P.pj_self_join(col, tau, mode=P.MODE_BATCHED, tune_cache=cache)
        st = P.pj_last_stats()
        assert np.array_equal(got, pj.pairs), (params, tau)
        assert st["candidates"] == pj.candidates
        assert st["cells"] == pj.cells


def test_server_reads_tune_cache(tmp_path):
    S = W.cfg5_index(20_000)
    rng = np.random.default_rng(31)
    Q, taus = W.cfg5_batch(rng, S, mean=64)
    cache = str(tmp_path / "tune.txt")
    with open(cache, "w") as f:
        f.write("# passjoin tune cache v2\nnot-a-gpu 1 1 8 1 16 4 2 1.0\nbroken line\n")
    idx = P.pj_build_index(S, 1, 8)
    try:
        exp = P.pj_query(idx, Q, taus)
        with P.Server(idx, slots=2, tune_cache=cache) as srv:
            rid = srv.submit(Q, taus)
            got, _ = srv.wait(rid)
        assert np.array_equal(got, exp)
    finally:
        idx.free()
