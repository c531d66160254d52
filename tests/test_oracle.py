"""Pins of the CPU oracle against what the paper and the mathematics fix.

Nothing here retypes the oracle's formulas: the checks are the paper's printed examples
(tests/golden/paper_examples.json), closed forms stated in the paper (Lemma 2), set relations it
proves (Lemma 1, Lemma 3, Theorem 6), edit distance found by breadth-first search over single
edit operations (the definition), metric invariants, and brute-force joins.
"""
import itertools
import random
from collections import deque

import numpy as np
import pytest

import oracle as O
import workloads as W


def b(s):
    return s.encode() if isinstance(s, str) else s


# --------------------------------------------------------------------------------------------
# Edit distance
# --------------------------------------------------------------------------------------------

def _all_strings(alphabet, maxlen):
    out = [b""]
    for n in range(1, maxlen + 1):
        out += [bytes(t) for t in itertools.product(alphabet, repeat=n)]
    return out


def _bfs_distances(src, alphabet, maxlen):
    """Edit distance from src to every string of length <= maxlen, by breadth-first search over
    single-character insertions, deletions and substitutions (the definition, Sec. 2)."""
    dist = {src: 0}
    q = deque([src])
    while q:
        u = q.popleft()
        d = dist[u]
        nbrs = []
        for k in range(len(u)):
            nbrs.append(u[:k] + u[k + 1:])
            for c in alphabet:
                if c != u[k]:
                    nbrs.append(u[:k] + bytes([c]) + u[k + 1:])
        if len(u) < maxlen:
            for k in range(len(u) + 1):
                for c in alphabet:
                    nbrs.append(u[:k] + bytes([c]) + u[k:])
        for v in nbrs:
            if v not in dist:
                dist[v] = d + 1
                q.append(v)
    return dist


@pytest.fixture(scope="module")
def bfs_table():
    alphabet = b"ab"
    strs = _all_strings(alphabet, 4)
    # intermediate strings up to one character longer than the longest endpoint
    return strs, {s: _bfs_distances(s, alphabet, 5) for s in strs}


def test_ed_full_matches_bfs_definition(bfs_table):
    strs, table = bfs_table
    for r in strs:
        for s in strs:
            assert O.ed_full(r, s) == table[r][s], (r, s)


def test_ed_full_matches_bfs_ternary():
    alphabet = b"abc"
    strs = _all_strings(alphabet, 3)
    for r in strs:
        d = _bfs_distances(r, alphabet, 4)
        for s in strs:
            assert O.ed_full(r, s) == d[s], (r, s)


def test_ed_paper_examples(golden):
    for e in golden["edit_distance"]:
        assert O.ed_full(b(e["r"]), b(e["s"])) == e["ed"], e["cite"]
    for e in golden["similar_at_tau"]:
        assert (O.ed_full(b(e["r"]), b(e["s"])) <= e["tau"]) == e["similar"], e["cite"]


def test_ed_metric_invariants():
    rng = random.Random(5)
    alph = b"abcd"
    for _ in range(400):
        x, y, z = (bytes(rng.choice(alph) for _ in range(rng.randint(0, 12))) for _ in range(3))
        dxy, dyx = O.ed_full(x, y), O.ed_full(y, x)
        assert dxy == dyx
        assert O.ed_full(x, z) <= dxy + O.ed_full(y, z)
        assert abs(len(x) - len(y)) <= dxy <= max(len(x), len(y))
        assert O.ed_full(x, x) == 0
        assert O.ed_full(x, b"") == len(x)
        # a common prefix and suffix do not change the distance
        assert O.ed_full(b"pq" + x + b"rs", b"pq" + y + b"rs") == dxy
        if len(x) == len(y):
            assert dxy <= sum(u != v for u, v in zip(x, y))   # Hamming bound


def test_ed_band_equals_thresholded_full():
    rng = random.Random(7)
    for _ in range(3000):
        alph = rng.choice([b"ab", b"abc", b"abcdefgh"])
        la, lb = rng.randint(0, 60), rng.randint(0, 60)
        x = bytes(rng.choice(alph) for _ in range(la))
        y = bytes(rng.choice(alph) for _ in range(lb))
        d = O.ed_full(x, y)
        for t in (0, 1, 2, 3, 5, 8, 13):
            assert O.ed_band(x, y, t) == min(d, t + 1), (x, y, t)


def test_ed_band_long_strings():
    rng = np.random.default_rng(3)
    for _ in range(20):
        x = bytes(rng.integers(97, 100, size=int(rng.integers(200, 400))).astype(np.uint8))
        y = bytearray(x)
        for _ in range(int(rng.integers(0, 30))):
            k = int(rng.integers(len(y)))
            y[k] = int(rng.integers(97, 100))
        y = bytes(y)
        d = O.ed_full(x, y)
        for t in (4, 16, 32, 64):
            assert O.ed_band(x, y, t) == min(d, t + 1)


# --------------------------------------------------------------------------------------------
# Partition and substring selection
# --------------------------------------------------------------------------------------------

def test_partition_paper_example(golden):
    for e in golden["partition"]:
        s = b(e["s"])
        segs = [s[p - 1:p - 1 + l] for p, l in O.partition(len(s), e["tau"])]
        assert segs == [b(t) for t in e["segments"]], e["cite"]
        q = len(s) // (e["tau"] + 1)
        assert len(s) - q * (e["tau"] + 1) == e["k"]


def test_partition_shape():
    for tau in range(0, 40):
        for l in range(tau + 1, 260):
            parts = O.partition(l, tau)
            assert len(parts) == tau + 1
            assert parts[0][0] == 1
            lens = [x[1] for x in parts]
            assert sum(lens) == l
            assert max(lens) - min(lens) <= 1 and min(lens) >= 1
            assert lens == sorted(lens)      # the longer segments come last
            for (p0, l0), (p1, _) in zip(parts, parts[1:]):
                assert p1 == p0 + l0


def test_pigeonhole_paper_example(golden):
    e = golden["pigeonhole"]
    r = b(e["r"])
    segs = [r[p - 1:p - 1 + l] for p, l in O.partition(len(r), e["tau"])]
    for s in e["no_segment_in"]:
        assert not any(g in b(s) for g in segs), e["cite"]


def _sel_sets(method, r, s, tau):
    out = []
    parts = O.partition(len(r), tau)
    for i, (p, l) in enumerate(parts, start=1):
        lo, hi = O.window(method, len(s), len(r), tau, i)
        out.append([s[q - 1:q - 1 + l] for q in range(lo, hi + 1)])
    return out


def test_position_aware_paper_example(golden):
    e = golden["position_aware"]
    r, s = b(e["r"]), b(e["s"])
    sets = _sel_sets(O.SEL_POSITION, r, s, e["tau"])
    assert sets == [[b(t) for t in g] for g in e["sets"]], e["cite"]
    assert sum(map(len, sets)) == e["total"]
    shift = sum(hi - lo + 1 for lo, hi in
                (O.window(O.SEL_SHIFT, len(s), len(r), e["tau"], i) for i in range(1, 5)))
    assert shift == e["shift_total"]


def test_multi_match_paper_example(golden):
    e = golden["multi_match"]
    r, s = b(e["r"]), b(e["s"])
    sets = _sel_sets(O.SEL_MULTIMATCH, r, s, e["tau"])
    assert sets == [[b(t) for t in g] for g in e["sets"]], e["cite"]
    assert sum(map(len, sets)) == e["total"]
    # the combined window is the intersection of the printed one-sided windows
    right = {3: e["right_windows_3_4"][0], 4: e["right_windows_3_4"][1]}
    for i in (3, 4):
        lo, hi = O.window(O.SEL_MULTIMATCH, len(s), len(r), e["tau"], i)
        ll, lh = e["left_windows"][i - 1]
        rl, rh = right[i]
        assert (lo, hi) == (max(ll, rl), min(lh, rh))


def test_selection_counts_paper(golden):
    e = golden["selection_counts"]
    n, l, tau = e["n"], e["l"], e["tau"]

    def total(method):
        return sum(max(0, hi - lo + 1) for lo, hi in
                   (O.window(method, n, l, tau, i) for i in range(1, tau + 2)))
    assert total(O.SEL_LENGTH) == e["length"], e["cite"]
    assert total(O.SEL_SHIFT) == e["shift"], e["cite"]
    assert total(O.SEL_MULTIMATCH) == e["multi_match"], e["cite"]
    # The printed position-aware count is the (tau+1)^2 size estimate; the window definition
    # of Sec. 4.1 holds floor((tau-D)/2) + floor((tau+D)/2) + 1 starts per slot, which is
    # tau+1 only when tau - D is even (here tau = 1, D = 0: one start per slot).
    assert e["position_printed"] == (tau + 1) ** 2
    assert total(O.SEL_POSITION) == tau + 1


def test_lemma2_multimatch_count():
    """|W_m(s, l)| = floor((tau^2 - D^2) / 2) + tau + 1 (Lemma 2), for the self-join windows
    (0 <= D <= tau) and for the signed D of a join of two sets."""
    for tau in range(0, 17):
        for l in range(tau + 1, 140, 3):
            for d in range(-tau, tau + 1):
                n = l + d
                if n < 1:
                    continue
                cnt = sum(max(0, hi - lo + 1) for lo, hi in
                          (O.window(O.SEL_MULTIMATCH, n, l, tau, i) for i in range(1, tau + 2)))
                assert cnt == (tau * tau - d * d) // 2 + tau + 1, (tau, l, d)


def test_position_count_even_parity():
    """|W_p(s, L_l^i)| = tau + 1 (Sec. 4.1) when tau - D is even and the bounds do not bind."""
    for tau in range(0, 12):
        for l in range(3 * (tau + 1), 120, 7):
            for d in range(0, tau + 1):
                if (tau - d) % 2:
                    continue
                for i in range(1, tau + 2):
                    lo, hi = O.window(O.SEL_POSITION, l + d, l, tau, i)
                    if lo > 1 and hi < l + d - O.partition(l, tau)[i - 1][1] + 1:
                        assert hi - lo + 1 == tau + 1


def test_lemma3_subset_chain():
    """W_m subset W_p subset W_f subset W_l as sets of valid start positions (Lemma 3)."""
    for tau in range(0, 10):
        for l in range(tau + 1, 70):
            for d in range(0, tau + 1):
                n = l + d
                for i in range(1, tau + 2):
                    li = O.partition(l, tau)[i - 1][1]
                    valid = set(range(1, n - li + 2))
                    sets = []
                    for m in (O.SEL_MULTIMATCH, O.SEL_POSITION, O.SEL_SHIFT, O.SEL_LENGTH):
                        lo, hi = O.window(m, n, l, tau, i)
                        sets.append(set(range(lo, hi + 1)) & valid)
                    for small, big in zip(sets, sets[1:]):
                        assert small <= big, (tau, l, d, i)


# --------------------------------------------------------------------------------------------
# Verification
# --------------------------------------------------------------------------------------------

def test_early_termination_paper_rows(golden):
    e0, e1 = golden["early_termination"]
    d, cells, rows = O.verify_pair(b(e0["r"]), b(e0["s"]), e0["tau"])
    assert d == e0["tau"] + 1 and rows == e0["length_aware_stop_row"], e0["cite"]
    d2, rows2 = O.ed_band_rows(b(e0["r"]), b(e0["s"]), e0["tau"])
    assert d2 == e0["tau"] + 1 and rows2 == e0["naive_band_stop_row"], e0["cite"]
    d, cells, rows = O.verify_pair(b(e1["r"]), b(e1["s"]), e1["tau"])
    assert d == e1["tau"] + 1 and rows == e1["stop_row"], e1["cite"]
    assert cells == e1["cells_per_row"] * e1["stop_row"]


def test_length_aware_cells_paper_example(golden):
    """The cells of the Sec. 5.1 example (a 3-wide band, Delta = 2), derived by hand from the
    printed band bounds: the band edges and the stopping row are counted as the paper states."""
    e0 = golden["early_termination"][0]
    r, s, t = b(e0["r"]), b(e0["s"]), e0["tau"]
    delta = len(s) - len(r)
    assert (t - delta) // 2 == e0["band_left"] and (t + delta) // 2 == e0["band_right"]
    d, cells, rows = O.verify_pair(r, s, t)
    assert rows == e0["length_aware_stop_row"] and cells == e0["length_aware_cells"]


def test_length_aware_cells_full_pass_closed_form():
    """No early stop when r is a prefix of s (every diagonal cell has E = Delta <= t), so every
    row of the band is computed.  The band j in [i - a, i + b], a = floor((t-D)/2),
    b = floor((t+D)/2), clipped to 1..|s| holds |r|(a+b+1) cells less the triangle cut off at
    column 0 (a(a+1)/2) and the one past column |s| (c(c+1)/2 with c = b - D): a count derived
    from the band's geometry, not by walking it as the oracle does.  A miscount at column 0, at
    the right edge or in a band wider than one cell fails here."""
    rng = random.Random(5)
    checked = 0
    for _ in range(600):
        t = rng.randint(0, 12)
        D = rng.randint(0, t)
        a, bb = (t - D) // 2, (t + D) // 2
        c = bb - D
        nr = rng.randint(max(a, c), max(a, c) + 30)
        r = bytes(rng.choice(b"abcd") for _ in range(nr))
        s = r + bytes(rng.choice(b"abcd") for _ in range(D))
        expect = nr * (a + bb + 1) - a * (a + 1) // 2 - c * (c + 1) // 2
        for x, y in ((r, s), (s, r)):          # the shorter part gives the rows either way
            d, cells, rows = O.verify_pair(x, y, t)
            assert d == D and rows == nr and cells == expect, (t, D, nr)
        checked += 1
    assert checked == 600


def test_extension_split_paper_example(golden):
    e = golden["extension"]
    r, s, w = b(e["r"]), b(e["s"]), b(e["shared"])
    tau = e["tau"]
    parts = O.partition(len(r), tau)
    i = next(k for k, (p, l) in enumerate(parts, start=1) if r[p - 1:p - 1 + l] == w)
    p_i, l_i = parts[i - 1]
    p = s.find(w) + 1
    assert r[:p_i - 1] == b(e["r_left"]) and s[:p - 1] == b(e["s_left"])
    assert r[p_i - 1 + l_i:] == b(e["r_right"]) and s[p - 1 + l_i:] == b(e["s_right"])
    ok, _ = O.extension_verify(s, r, tau, i, p)
    assert ok == (O.ed_full(r, s) <= tau)


def test_verify_pair_equals_thresholded_ed():
    """VerifyStringPair returns min(t+1, ED) (the function of Algorithm 3)."""
    rng = random.Random(11)
    for _ in range(4000):
        alph = rng.choice([b"ab", b"abc", b"abcdefghij"])
        x = bytes(rng.choice(alph) for _ in range(rng.randint(0, 40)))
        y = bytes(rng.choice(alph) for _ in range(rng.randint(0, 40)))
        d = O.ed_full(x, y)
        for t in (0, 1, 2, 3, 4, 6, 9):
            v, cells, rows = O.verify_pair(x, y, t)
            assert v == min(d, t + 1), (x, y, t)
            nr = min(len(x), len(y))
            assert 0 <= rows <= nr
            assert cells <= (t + 1) * rows


def test_extension_verification_correct_and_complete():
    """Every passing candidate is a similar pair, and every similar pair has a passing candidate
    among the multi-match selections (Theorem 5 with the windows of Sec. 4.2)."""
    rng = random.Random(13)
    checked = 0
    for _ in range(2500):
        tau = rng.randint(0, 5)
        alph = rng.choice([b"ab", b"abc", b"abcd"])
        l = rng.randint(tau + 1, tau + 14)
        y = bytes(rng.choice(alph) for _ in range(l))
        x = bytearray(y)
        for _ in range(rng.randint(0, tau + 2)):
            op = rng.randint(0, 2)
            if op == 0 and x:
                x[rng.randrange(len(x))] = rng.choice(alph)
            elif op == 1:
                x.insert(rng.randint(0, len(x)), rng.choice(alph))
            elif x:
                del x[rng.randrange(len(x))]
        x = bytes(x)
        n = len(x)
        if abs(n - l) > tau:
            continue
        d = O.ed_full(x, y)
        passed = False
        for i, (p_i, l_i) in enumerate(O.partition(l, tau), start=1):
            lo, hi = O.window(O.SEL_MULTIMATCH, n, l, tau, i)
            for p in range(lo, hi + 1):
                if x[p - 1:p - 1 + l_i] == y[p_i - 1:p_i - 1 + l_i]:
                    ok, _ = O.extension_verify(x, y, tau, i, p)
                    if ok:
                        assert d <= tau, (x, y, tau, i, p)
                        passed = True
        assert passed == (d <= tau), (x, y, tau)
        checked += 1
    assert checked > 1000


def test_lemma1_pigeonhole_random():
    """A string within distance tau of y contains one of y's tau+1 segments (Lemma 1)."""
    rng = random.Random(17)
    for _ in range(3000):
        tau = rng.randint(0, 6)
        l = rng.randint(tau + 1, 30)
        y = bytes(rng.choice(b"abc") for _ in range(l))
        x = bytes(rng.choice(b"abc") for _ in range(rng.randint(max(0, l - tau), l + tau)))
        if O.ed_full(x, y) <= tau:
            segs = [y[p - 1:p - 1 + li] for p, li in O.partition(l, tau)]
            assert any(g in x for g in segs)


# --------------------------------------------------------------------------------------------
# Joins
# --------------------------------------------------------------------------------------------

def _py_self_join(strings, tau, ed):
    out = []
    for a in range(len(strings)):
        for c in range(a + 1, len(strings)):
            if ed(strings[a], strings[c]) <= tau:
                out.append((a, c))
    return np.array(sorted(out), dtype=np.int32).reshape(-1, 2)


def test_self_join_bf_against_bfs_definition(bfs_table):
    strs, table = bfs_table
    rng = random.Random(19)
    for _ in range(30):
        sample = [rng.choice(strs) for _ in range(rng.randint(0, 25))]
        col = W.from_list(sample)
        for tau in (0, 1, 2, 3):
            exp = _py_self_join(sample, tau, lambda u, v: table[u][v])
            assert np.array_equal(O.self_join_bf(col, tau, 2), exp)


def test_table1_join(golden):
    strings = golden["table1"]["strings"]
    col = W.from_list(strings)
    idx = {s: k for k, s in enumerate(strings)}
    r3 = O.self_join_pj(col, 3).pairs
    pair = tuple(sorted((idx["kaushik chakrab"], idx["caushik chakrabar"])))
    assert pair in {tuple(p) for p in r3.tolist()}
    for tau in range(0, 8):
        assert np.array_equal(O.self_join_pj(col, tau).pairs, O.self_join_bf(col, tau, 1))
    # Sec. 3.2: with all substrings selected, "avataresha" finds the segments "va", "at" and
    # "esh" of "vankatesh" and the pair is a candidate but not an answer.  The multi-match
    # windows of Sec. 4.2 select {av}, {va, at, ta}, {ar, re, es}, {sha}, none of which equals
    # the segment of its own slot, so the pair is not even a candidate there.
    segs = [b"vankatesh"[p - 1:p - 1 + l] for p, l in O.partition(9, 3)]
    assert [g for g in segs if g in b"avataresha"] == [b"va", b"at", b"esh"]
    res = O.self_join_pj(col, 3, keep_cands=True)
    va = {idx["vankatesh"], idx["avataresha"]}
    cands = [(y, x) for y, x in zip(res.cands["y"], res.cands["x"]) if {int(y), int(x)} == va]
    assert not cands
    assert tuple(sorted(va)) not in {tuple(p) for p in r3.tolist()}


@pytest.mark.parametrize("seed", range(12))
def test_theorem6_passjoin_equals_bruteforce(seed):
    rng = np.random.default_rng(seed)
    alph = [b"ab", b"abc", b"abcd"][seed % 3]
    col = W.random_small(rng, 300, alphabet=alph, lmin=0, lmax=14, dup_frac=0.4, kmax=3)
    for tau in range(0, 6):
        bf = O.self_join_bf(col, tau, 4)
        pj = O.self_join_pj(col, tau, tiebreak=seed % 2)
        assert np.array_equal(pj.pairs, bf), tau


@pytest.mark.parametrize("seed", range(6))
def test_theorem6_join_two_sets(seed):
    rng = np.random.default_rng(100 + seed)
    alph = [b"ab", b"abc", b"abcd"][seed % 3]
    R = W.random_small(rng, 150, alphabet=alph, lmin=0, lmax=14, dup_frac=0.3, kmax=3)
    S = W.random_small(rng, 200, alphabet=alph, lmin=0, lmax=14, dup_frac=0.3, kmax=3)
    for tau in range(0, 6):
        assert np.array_equal(O.join_pj(R, S, tau).pairs, O.join_bf(R, S, tau, 4)), tau


SEL_METHODS = (O.SEL_MULTIMATCH, O.SEL_POSITION, O.SEL_SHIFT, O.SEL_LENGTH)


@pytest.mark.parametrize("seed", range(6))
def test_every_selection_method_is_complete(seed):
    # Sec. 4: the length, shift, position and multi-match selections all find every similar
    # pair (completeness), so each Pass-Join equals the brute-force join
    rng = np.random.default_rng(300 + seed)
    alph = [b"ab", b"abc", b"abcd"][seed % 3]
    col = W.random_small(rng, 250, alphabet=alph, lmin=0, lmax=14, dup_frac=0.4, kmax=3)
    S = W.random_small(rng, 150, alphabet=alph, lmin=0, lmax=14, dup_frac=0.3, kmax=3)
    for tau in range(0, 5):
        bf = O.self_join_bf(col, tau, 4)
        jbf = O.join_bf(col, S, tau, 4)
        for m in SEL_METHODS:
            assert np.array_equal(O.self_join_pj(col, tau, method=m).pairs, bf), (tau, m)
            assert np.array_equal(O.join_pj(col, S, tau, method=m).pairs, jbf), (tau, m)


def test_selection_methods_nest():
    # Lemma 3 and Sec. 4: multi-match selects a subset of position-aware, which selects a subset
    # of shift-based, which selects a subset of all substrings; so the candidate sets nest too
    col = W.cfg1(1500)
    for tau in (1, 2, 3):
        res = [O.self_join_pj(col, tau, method=m, keep_cands=True) for m in SEL_METHODS]
        sets = [set(zip(r.cands["y"].tolist(), r.cands["x"].tolist(), r.cands["i"].tolist(),
                        r.cands["p"].tolist())) for r in res]
        for a, b_ in zip(sets, sets[1:]):
            assert a <= b_
        sel = [r.selected for r in res]
        assert sel == sorted(sel) and sel[0] < sel[-1]
        # every pair a method finds comes from candidates it verified
        for r in res:
            assert np.array_equal(r.pairs, res[0].pairs)


def test_length_selection_count():
    # the length method selects every substring of length l_i: a probe string of length n has
    # n - l_i + 1 of them for each probed length l and slot i (closed form over the lengths)
    rng = np.random.default_rng(7)
    col = W.random_small(rng, 60, alphabet=b"abc", lmin=3, lmax=12, dup_frac=0.0, kmax=1)
    tau = 2
    lens = (col.offsets[1:] - col.offsets[:-1]).tolist()
    expect = 0
    order = sorted(range(col.n), key=lambda k: (lens[k], k))
    for x in order:
        n = lens[x]
        if n < tau + 1:
            continue
        for l in range(max(n - tau, tau + 1), n + 1):
            q, k = divmod(l, tau + 1)
            for i in range(1, tau + 2):
                li = q + (1 if i > tau + 1 - k else 0)
                expect += n - li + 1
    assert O.self_join_pj(col, tau, method=O.SEL_LENGTH).selected == expect


def test_tiebreak_order_gives_same_set():
    col = W.cfg1(2000)
    for tau in (1, 2, 3):
        a = O.self_join_pj(col, tau, tiebreak=0)
        c = O.self_join_pj(col, tau, tiebreak=1)
        assert np.array_equal(a.pairs, c.pairs)


def test_cfg1_passjoin_equals_bruteforce():
    col = W.cfg1()
    bf = O.self_join_bf(col, 2)
    pj = O.self_join_pj(col, 2)
    assert np.array_equal(pj.pairs, bf)
    assert pj.candidates > 0 and len(bf) > 1000


def test_join_symmetry_and_self():
    """join(S, S) = self-join pairs in both orientations plus the diagonal."""
    rng = np.random.default_rng(23)
    S = W.random_small(rng, 200, alphabet=b"abc", lmin=0, lmax=10, dup_frac=0.4)
    for tau in range(0, 4):
        sj = {tuple(p) for p in O.self_join_pj(S, tau).pairs.tolist()}
        jj = {tuple(p) for p in O.join_pj(S, S, tau).pairs.tolist()}
        exp = sj | {(b_, a) for a, b_ in sj} | {(k, k) for k in range(S.n)}
        assert jj == exp


def test_monotone_and_permutation_invariant():
    rng = np.random.default_rng(29)
    S = W.random_small(rng, 250, alphabet=b"abcd", lmin=1, lmax=12, dup_frac=0.4)
    prev = set()
    for tau in range(0, 5):
        cur = {tuple(p) for p in O.self_join_pj(S, tau).pairs.tolist()}
        assert prev <= cur
        prev = cur
    perm = rng.permutation(S.n)
    P = S.subset(perm)                       # P[k] = S[perm[k]]
    base = {tuple(p) for p in O.self_join_pj(S, 3).pairs.tolist()}
    got = {tuple(sorted((int(perm[a]), int(perm[c]))))
           for a, c in O.self_join_pj(P, 3).pairs.tolist()}
    assert got == base


def test_candidates_pass_implies_similar_and_cells_consistent():
    col = W.cfg1(3000)
    res = O.self_join_pj(col, 2, keep_cands=True)
    c = res.cands
    assert len(c["y"]) == res.candidates
    assert int(c["cells"].sum()) == res.cells
    strs = col.as_list()
    pairs = {tuple(p) for p in res.pairs.tolist()}
    for k in range(0, len(c["y"]), 7):
        y, x = int(c["y"][k]), int(c["x"][k])
        # visiting order: shorter first, then lower id
        assert (len(strs[y]), y) < (len(strs[x]), x)
        if c["pass"][k]:
            assert O.ed_full(strs[x], strs[y]) <= 2
            assert (min(x, y), max(x, y)) in pairs


def test_partners_bf_matches_self_join():
    col = W.cfg1(2000)
    allp = O.self_join_bf(col, 2)
    xs = np.arange(0, col.n, 13, dtype=np.int32)
    got = O.partners_bf(col, xs, 2)
    sel = set(xs.tolist())
    exp = np.array([p for p in allp.tolist() if p[0] in sel or p[1] in sel],
                   dtype=np.int32).reshape(-1, 2)
    assert np.array_equal(got, exp)


def test_probe_stride_samples_subset():
    col = W.cfg1(3000)
    full = {tuple(p) for p in O.self_join_pj(col, 2).pairs.tolist()}
    samp = O.self_join_pj(col, 2, probe_stride=5)
    assert {tuple(p) for p in samp.pairs.tolist()} <= full
    assert 0 < samp.candidates < O.self_join_pj(col, 2).candidates


def test_probe_shares_partition_the_run():
    """The runs for probe offsets 0..k-1 of stride k (how the full-size golden values are made
    over several processes) have disjoint pairs whose union is the single run's, and their
    counters add up to the single run's."""
    col = W.cfg1()
    full = O.self_join_pj(col, 2)
    k = 7
    parts = [O.self_join_pj(col, 2, probe_stride=k, probe_offset=w) for w in range(k)]
    allp = np.concatenate([p.pairs for p in parts])
    assert len({tuple(p) for p in allp.tolist()}) == len(allp)          # disjoint
    key = allp[:, 0].astype(np.int64) << 32 | allp[:, 1]
    assert np.array_equal(allp[np.argsort(key)], full.pairs)
    for f in ("candidates", "cells", "selected", "side_pairs"):
        assert sum(getattr(p, f) for p in parts) == getattr(full, f), f
    par = O.self_join_pj_parallel(col, 2, procs=3, shares=k)
    assert np.array_equal(par.pairs, full.pairs) and par.cells == full.cells
    # the join of two sets, with strings shorter than tau+1 on both sides
    rng = np.random.default_rng(21)
    R = W.random_small(rng, 400, alphabet=b"abc", lmin=0, lmax=12, dup_frac=0.4)
    S = W.random_small(rng, 500, alphabet=b"abc", lmin=0, lmax=12, dup_frac=0.4)
    jf = O.join_pj(R, S, 3)
    jp = O.join_pj_parallel(R, S, 3, procs=2, shares=5)
    assert np.array_equal(jp.pairs, jf.pairs) and np.array_equal(jf.pairs, O.join_bf(R, S, 3, 2))
    for f in ("candidates", "cells", "selected", "side_pairs"):
        assert getattr(jp, f) == getattr(jf, f), f
