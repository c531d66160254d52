"""GPU parity: the HIP join equals the oracle bit-exactly (sorted pair lists), and its candidate
and cell counts equal the oracle's Pass-Join counts.  Every call goes through the C ABI."""
import os

import numpy as np
import pytest

import oracle as O
import paper_1111_7171_amd as P
import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)


def _same(got, exp, what=""):
    assert got.dtype == np.int32 and got.ndim == 2 and got.shape[1] == 2
    if not np.array_equal(got, exp):
        g = {tuple(p) for p in got.tolist()}
        e = {tuple(p) for p in exp.tolist()}
        raise AssertionError(f"{what}: {len(got)} pairs vs {len(exp)} expected; "
                             f"missing {sorted(e - g)[:5]} extra {sorted(g - e)[:5]}")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    P.load()
    yield


def test_table1_all_tau(golden):
    col = W.from_list(golden["table1"]["strings"])
    for tau in range(0, 8):
        _say("table1 tau", tau)
        _same(P.pj_self_join(col, tau), O.self_join_bf(col, tau, 1), f"tau={tau}")


MODES = [P.MODE_PLAIN, P.MODE_BATCHED]


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("seed", range(8))
def test_random_small_self_join(seed, mode):
    rng = np.random.default_rng(1000 + seed)
    alph = [b"ab", b"abc", b"abcd", b"abcdefgh"][seed % 4]
    col = W.random_small(rng, 400, alphabet=alph, lmin=0, lmax=16, dup_frac=0.4, kmax=3)
    for tau in range(0, 6):
        _say("random self seed", seed, "tau", tau, "mode", mode)
        got = P.pj_self_join(col, tau, mode=mode)
        _same(got, O.self_join_bf(col, tau, 8), f"seed={seed} tau={tau}")


@pytest.mark.parametrize("seed", range(4))
def test_random_small_join(seed):
    rng = np.random.default_rng(2000 + seed)
    alph = [b"ab", b"abc", b"abcd", b"abcdefgh"][seed % 4]
    R = W.random_small(rng, 250, alphabet=alph, lmin=0, lmax=14, dup_frac=0.3)
    S = W.random_small(rng, 300, alphabet=alph, lmin=0, lmax=14, dup_frac=0.3)
    for tau in range(0, 6):
        _say("random join seed", seed, "tau", tau)
        _same(P.pj_join(R, S, tau), O.join_bf(R, S, tau, 8), f"seed={seed} tau={tau}")


def test_cfg1_full_exact_pairs_and_counts():
    col = W.cfg1()
    exp = O.self_join_bf(col, 2)
    got = P.pj_self_join(col, 2)
    st = P.pj_last_stats()
    _same(got, exp, "cfg1")
    pj = O.self_join_pj(col, 2)
    assert st["candidates"] == pj.candidates
    assert st["cells"] == pj.cells
    assert st["selected"] == pj.selected


@pytest.mark.parametrize("mode", MODES + ["bucketed"])
@pytest.mark.parametrize("cfg,n,taus", [
    (2, 20_000, (1, 2, 3, 4)),
    (3, 8_000, (2, 4, 6, 8)),
    (4, 1_500, (8, 16, 32)),
])
def test_scaled_configs_match_oracle(cfg, n, taus, mode, monkeypatch):
    if mode == "bucketed":
        # the batched path's slot bucketing and list-segment kernel at any candidate count
        monkeypatch.setenv("PJ_BUCKET_MIN_CANDIDATES", "0")
        mode = P.MODE_BATCHED
    col = W.CONFIGS[cfg](n)
    for tau in taus:
        _say("cfg", cfg, "n", n, "tau", tau, "mode", mode)
        pj = O.self_join_pj(col, tau)
        got = P.pj_self_join(col, tau, mode=mode)
        st = P.pj_last_stats()
        _same(got, pj.pairs, f"cfg{cfg} tau={tau}")
        assert st["candidates"] == pj.candidates, (st["candidates"], pj.candidates)
        assert st["cells"] == pj.cells, (st["cells"], pj.cells)


def test_join_two_sets_counts():
    R = W.cfg2(6000, seed=7)
    S = W.cfg2(9000, seed=8)
    for tau in (1, 2, 3):
        _say("join tau", tau)
        pj = O.join_pj(R, S, tau)
        got = P.pj_join(R, S, tau)
        st = P.pj_last_stats()
        _same(got, pj.pairs, f"join tau={tau}")
        assert st["candidates"] == pj.candidates


def test_edge_cases():
    # empty set, one string, all-empty strings, all shorter than tau+1, exact duplicates
    empty = W.from_list([])
    assert P.pj_self_join(empty, 2).shape == (0, 2)
    one = W.from_list([b"abc"])
    assert P.pj_self_join(one, 2).shape == (0, 2)
    blanks = W.from_list([b""] * 5)
    _same(P.pj_self_join(blanks, 0), O.self_join_bf(blanks, 0, 1), "blanks")
    shorts = W.from_list([b"a", b"b", b"ab", b"", b"ba", b"abc"])
    for tau in range(0, 5):
        _same(P.pj_self_join(shorts, tau), O.self_join_bf(shorts, tau, 1), f"shorts {tau}")
    dups = W.from_list([b"hello world"] * 7 + [b"hello warld"] * 3)
    for tau in (0, 1, 2):
        _same(P.pj_self_join(dups, tau), O.self_join_bf(dups, tau, 1), f"dups {tau}")
    # join with an empty side
    _same(P.pj_join(empty, dups, 1), np.empty((0, 2), np.int32), "empty R")
    _same(P.pj_join(dups, empty, 1), np.empty((0, 2), np.int32), "empty S")


def test_maximum_length_and_tau():
    rng = np.random.default_rng(5)
    base = bytes(rng.integers(97, 101, size=2047).astype(np.uint8))
    strs = [base]
    for k in range(5):
        b = bytearray(base)
        for _ in range(k * 12):
            b[int(rng.integers(len(b)))] = int(rng.integers(97, 101))
        strs.append(bytes(b[: 2047 - k]))
    col = W.from_list(strs)
    for tau in (0, 31, 63):
        _say("maxlen tau", tau)
        _same(P.pj_self_join(col, tau), O.self_join_bf(col, tau, 4), f"maxlen tau={tau}")


def test_device_inputs_and_outputs():
    import torch
    col = W.cfg1(4000)
    chars = torch.from_numpy(col.chars.copy()).cuda()
    offs = torch.from_numpy(col.offsets.copy()).cuda()
    host = P.pj_self_join(col, 2)
    dev_in = P.pj_self_join((chars, offs), 2)
    _same(dev_in, host, "device inputs")
    dp = P.pj_self_join((chars, offs), 2, outputs_on_device=True)
    try:
        _same(dp.to_numpy(), host, "device outputs")
    finally:
        dp.free()


def test_query_matches_oracle_per_tau():
    S = W.cfg5_index(20_000)
    rng = np.random.default_rng(9)
    Q, taus = W.cfg5_batch(rng, S, mean=64)
    idx = P.pj_build_index(S, 1, 8)
    try:
        got = P.pj_query(idx, Q, taus)
    finally:
        idx.free()
    exp = []
    for t in range(1, 9):
        ids = np.nonzero(taus == t)[0]
        if len(ids) == 0:
            continue
        sub = Q.subset(ids)
        for a, b in O.join_pj(sub, S, t).pairs.tolist():
            exp.append((int(ids[a]), b))
    exp = np.array(sorted(exp), dtype=np.int32).reshape(-1, 2)
    _same(got, exp, "query")


def test_repeatable_runs_identical():
    col = W.cfg2(30_000, seed=11)
    a = P.pj_self_join(col, 3)
    b = P.pj_self_join(col, 3)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("seed", range(3))
def test_query_mixed_tau_with_short_strings(seed):
    """Per-query thresholds in one device pass, including strings shorter than tau+1 on both
    sides (the direct path takes each query's own tau)."""
    rng = np.random.default_rng(3000 + seed)
    S = W.random_small(rng, 300, alphabet=b"abc", lmin=0, lmax=12, dup_frac=0.4)
    Q = W.random_small(rng, 120, alphabet=b"abc", lmin=0, lmax=12, dup_frac=0.2)
    taus = rng.integers(0, 7, size=Q.n).astype(np.int32)
    idx = P.pj_build_index(S, 0, 6)
    try:
        got = P.pj_query(idx, Q, taus)
    finally:
        idx.free()
    exp = []
    for t in range(0, 7):
        ids = np.nonzero(taus == t)[0]
        if len(ids):
            for a, b in O.join_bf(Q.subset(ids), S, t, 4).tolist():
                exp.append((int(ids[a]), b))
    exp = np.array(sorted(exp), dtype=np.int32).reshape(-1, 2)
    _same(got, exp, f"mixed tau seed={seed}")


def test_symbol_map_keys_small_alphabet_long_strings():
    """Two symbols pack into 2 bits, so segments of up to 20 characters have exact keys and
    longer ones are hashed; both kinds must give the oracle's candidates and pairs."""
    rng = np.random.default_rng(61)
    col = W.random_small(rng, 600, alphabet=b"ab", lmin=30, lmax=70, dup_frac=0.5, kmax=3)
    for tau in (1, 2, 3):
        _say("two-symbol alphabet tau", tau)
        pj = O.self_join_pj(col, tau)
        got = P.pj_self_join(col, tau)
        st = P.pj_last_stats()
        _same(got, pj.pairs, f"ab tau={tau}")
        assert st["candidates"] == pj.candidates and st["cells"] == pj.cells


def test_symbol_map_bytes_absent_from_indexed_side():
    """Probe strings with bytes the indexed set lacks (their code is 0): no false matches."""
    rng = np.random.default_rng(62)
    S = W.random_small(rng, 400, alphabet=b"abc", lmin=4, lmax=14, dup_frac=0.3)
    R0 = W.random_small(rng, 300, alphabet=b"abcxyz", lmin=4, lmax=14, dup_frac=0.3)
    R = W.from_list(R0.as_list() + S.as_list()[:100])
    for tau in (0, 1, 2, 3):
        _say("absent bytes tau", tau)
        pj = O.join_pj(R, S, tau)
        got = P.pj_join(R, S, tau)
        st = P.pj_last_stats()
        _same(got, pj.pairs, f"absent tau={tau}")
        assert st["candidates"] == pj.candidates


def test_symbol_map_all_byte_values():
    """All 256 byte values present: 9-bit codes, exact keys up to 4 bytes."""
    rng = np.random.default_rng(63)
    base = [bytes(rng.integers(0, 256, size=int(rng.integers(6, 24))).astype(np.uint8))
            for _ in range(300)]
    base.append(bytes(range(256))[:40])
    strs = []
    for b in base:
        strs.append(b)
        e = bytearray(b)
        if e:
            e[int(rng.integers(len(e)))] = int(rng.integers(0, 256))
        strs.append(bytes(e))
    col = W.from_list(strs)
    for tau in (1, 2, 3):
        _say("all bytes tau", tau)
        pj = O.self_join_pj(col, tau)
        got = P.pj_self_join(col, tau)
        st = P.pj_last_stats()
        _same(got, pj.pairs, f"bytes tau={tau}")
        assert st["candidates"] == pj.candidates


@pytest.mark.parametrize("rounds", ["1", "3", "16"])
def test_batched_chunk_sizes(rounds, monkeypatch):
    # the small-list kernel's wave chunks (64 x rounds candidates) change no result
    monkeypatch.setenv("PJ_BATCHED_ROUNDS", rounds)
    col = W.cfg3(6_000, seed=71)
    for tau in (2, 4, 6):
        _say("batched rounds", rounds, "tau", tau)
        got = P.pj_self_join(col, tau, mode=P.MODE_BATCHED)
        st = P.pj_last_stats()
        pj = O.self_join_pj(col, tau)
        _same(got, pj.pairs, f"rounds={rounds} tau={tau}")
        assert st["candidates"] == pj.candidates
        assert st["cells"] == pj.cells


@pytest.mark.parametrize("xmajor", ["0", "1"])
def test_probe_thread_mappings(xmajor, monkeypatch):
    # the probe's two thread mappings (string-major; pair-major over blocks of 64 probe strings,
    # with a partial last block, strings of several lengths per block and unstaged blocks of
    # long strings) and the window-size order of the pairs change no result, for self-joins
    # and joins of two sets
    monkeypatch.setenv("PJ_PROBE_XMAJOR", xmajor)
    col = W.cfg3(3_001, seed=72)
    for tau in (1, 3, 8):
        _say("probe mapping", xmajor, "tau", tau)
        got = P.pj_self_join(col, tau)
        st = P.pj_last_stats()
        pj = O.self_join_pj(col, tau)
        _same(got, pj.pairs, f"xmajor={xmajor} tau={tau}")
        assert st["candidates"] == pj.candidates and st["selected"] == pj.selected
    R = W.cfg2(1_500, seed=73)
    S = W.cfg2(1_250, seed=74)
    for tau in (2, 4):
        got = P.pj_join(R, S, tau)
        st = P.pj_last_stats()
        pj = O.join_pj(R, S, tau)
        _same(got, pj.pairs, f"join xmajor={xmajor} tau={tau}")
        assert st["candidates"] == pj.candidates and st["selected"] == pj.selected


def _clusters(seed, nbase, per, lmin, lmax, kmax):
    """nbase random base strings over a-z (lengths U{lmin..lmax}), each with per - 1 copies
    carrying U{0..kmax} random edits kept within [lmin, lmax]: the members of a cluster share
    most segments, so inverted lists are long."""
    rng = np.random.default_rng(seed)
    alpha = b"abcdefghijklmnopqrstuvwxyz"
    out = []
    for _ in range(nbase):
        size = int(rng.integers(lmin, lmax + 1))
        base = bytes(alpha[int(c)] for c in rng.integers(0, 26, size=size))
        out.append(base)
        for _ in range(per - 1):
            b = bytearray(base)
            for _ in range(int(rng.integers(0, kmax + 1))):
                op, pos = int(rng.integers(0, 3)), int(rng.integers(0, len(b)))
                if op == 0:
                    b[pos] = alpha[int(rng.integers(0, 26))]
                elif op == 1 and len(b) < lmax:
                    b.insert(pos, alpha[int(rng.integers(0, 26))])
                elif len(b) > lmin:
                    del b[pos]
            out.append(bytes(b))
    perm = rng.permutation(len(out))
    return W.from_list([out[k] for k in perm])


@pytest.mark.parametrize("lanes", [1, 2])
@pytest.mark.parametrize("lmin,lmax", [(20, 40), (44, 64), (10, 120)])
def test_list_kernel_wide_bands(lanes, lmin, lmax, tmp_path, monkeypatch):
    # the list-segment kernel on every band class up to 9 wide (tau 1..8, parts with t up to
    # 8, the final diagonal a constant for t <= 4 and a runtime value above), indexed strings
    # of up to 40, up to 64 and (10..120) of every length class in one set, each class with a
    # launch of its own, one or two candidates per lane
    monkeypatch.setenv("PJ_BUCKET_MIN_CANDIDATES", "0")
    col = _clusters(5 + lmin, 40, 60, lmin, lmax, 8)
    cache = str(tmp_path / "tune.txt")
    P.pj_tune(W.cfg2(2_000, seed=23), 0, tune_cache=cache)    # learns this GPU's architecture
    arch = [ln.split()[0] for ln in open(cache) if not ln.startswith("#")][0]
    mean = (col.offsets[-1] - col.offsets[0]) / col.n
    lb = int(mean + 0.5).bit_length()
    with open(cache, "w") as f:
        f.write("# passjoin tune cache v2\n")
        for tau in range(0, 9):
            f.write(f"{arch} {tau} {lb} 32 4 16 4 {lanes} 1.0\n")
    for tau in (1, 2, 4, 5, 6, 7, 8):
        _say("wide bands lanes", lanes, "lengths", lmin, lmax, "tau", tau)
        pj = O.self_join_pj(col, tau)
        got = P.pj_self_join(col, tau, mode=P.MODE_BATCHED, tune_cache=cache)
        st = P.pj_last_stats()
        _same(got, pj.pairs, f"lanes={lanes} len {lmin}-{lmax} tau={tau}")
        assert st["candidates"] == pj.candidates
        assert st["cells"] == pj.cells
        if lmax <= 64:
            assert st["ms_list_kernel"] > 0      # the list-segment kernel ran
        elif tau >= 4:
            # the mixed set's clusters spread over many lists: long lists from tau 4 on, of
            # several length classes
            assert st["ms_list_kernel"] > 0 and st["list_launches"] >= 2
