"""Seeded synthetic string collections shaped like the paper's workloads.

The paper evaluates on DBLP Author (short strings, avg 14.8 chars), AOL Query Log (avg 44.75) and
DBLP Author+Title (avg 105.8) (Sec. 6, Table 2).  Those datasets are not available here, so these
generators draw collections of the same shape: length distribution, alphabet skew and a share of
near-duplicates made by random edits.  Every collection is a deterministic function of its seed.

This module holds none of the similarity-join arithmetic: it only draws strings.  The GPU library's
tests and benchmark and the CPU oracle consume the same arenas made here.

An arena is a pair ``(chars, offsets)``: ``chars`` is a ``uint8`` array of all strings
concatenated, ``offsets`` an ``int32`` array of length ``n + 1`` with ``offsets[0] == 0``; string
``k`` is ``chars[offsets[k]:offsets[k + 1]]`` and its id is ``k``.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np

BASE_SEED = 71710

# 27-symbol alphabet: a-z plus space.
ALPHA27 = np.frombuffer(b"abcdefghijklmnopqrstuvwxyz ", dtype=np.uint8)

# English letter frequencies (a standard table, renormalised below), used with space = 0.18.
_ENGLISH = {
    "e": .127, "t": .091, "a": .082, "o": .075, "i": .070, "n": .067, "s": .063, "h": .061,
    "r": .060, "d": .043, "l": .040, "c": .028, "u": .028, "m": .024, "w": .024, "f": .022,
    "g": .020, "y": .020, "p": .019, "b": .015, "v": .0098, "k": .0077, "j": .0015, "x": .0015,
    "q": .00095, "z": .00074,
}


def english27_probs() -> np.ndarray:
    """Probabilities over ALPHA27: letters share 0.82 by the English table, space has 0.18."""
    letters = np.array([_ENGLISH[chr(c)] for c in ALPHA27[:26]], dtype=np.float64)
    letters = 0.82 * letters / letters.sum()
    return np.concatenate([letters, [0.18]])


# 40-symbol alphabet for the medium-length collection, in rank order (rank 1 = 'a').
ALPHA40 = np.frombuffer(b"abcdefghijklmnopqrstuvwxyz0123456789 .-_", dtype=np.uint8)


def zipf_probs(m: int, s: float) -> np.ndarray:
    p = np.arange(1, m + 1, dtype=np.float64) ** (-s)
    return p / p.sum()


@dataclass
class Collection:
    chars: np.ndarray            # uint8[total]
    offsets: np.ndarray          # int32[n + 1]
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.offsets.shape[0] - 1)

    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets.astype(np.int64)).astype(np.int32)

    def get(self, k: int) -> bytes:
        return self.chars[self.offsets[k]:self.offsets[k + 1]].tobytes()

    def as_list(self) -> list[bytes]:
        b = self.chars.tobytes()
        o = self.offsets
        return [b[o[k]:o[k + 1]] for k in range(self.n)]

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(self.offsets.astype("<i4").tobytes())
        h.update(self.chars.tobytes())
        return h.hexdigest()

    def subset(self, ids) -> "Collection":
        return from_list([self.get(int(k)) for k in ids], name=self.name + "[subset]")


def from_list(strings, name: str = "") -> Collection:
    strings = [s.encode() if isinstance(s, str) else bytes(s) for s in strings]
    lens = np.fromiter((len(s) for s in strings), dtype=np.int64, count=len(strings))
    offs = np.zeros(len(strings) + 1, dtype=np.int64)
    np.cumsum(lens, out=offs[1:])
    if offs[-1] >= 2**31:
        raise ValueError("arena larger than int32 offsets allow")
    chars = np.frombuffer(b"".join(strings), dtype=np.uint8).copy()
    return Collection(chars, offs.astype(np.int32), name)


def _from_chunks(chars: np.ndarray, lens: np.ndarray) -> list[bytes]:
    offs = np.zeros(len(lens) + 1, dtype=np.int64)
    np.cumsum(lens, out=offs[1:])
    b = chars.tobytes()
    return [b[offs[k]:offs[k + 1]] for k in range(len(lens))]


def _iid_strings(rng, lens, symbols, probs) -> list[bytes]:
    total = int(np.sum(lens))
    idx = rng.choice(len(symbols), size=total, p=probs)
    return _from_chunks(symbols[idx], np.asarray(lens, dtype=np.int64))


class _Editor:
    """Applies k random single-character edits: each op is uniform over {substitute, insert,
    delete} at a uniform position; substituted and inserted symbols come from the collection's
    character distribution (a substitute always differs from the symbol it replaces).

    Random numbers are drawn from the generator in blocks and consumed in order, so a collection
    is still a deterministic function of its seed."""

    _BLOCK = 1 << 16

    def __init__(self, rng, symbols, probs):
        self.rng = rng
        self.symbols = symbols
        self.probs = probs
        self._u = np.empty(0)
        self._ui = 0
        self._s = np.empty(0, dtype=np.uint8)
        self._si = 0

    def _int(self, m: int) -> int:
        """Uniform integer in [0, m)."""
        if self._ui >= len(self._u):
            self._u = self.rng.random(self._BLOCK)
            self._ui = 0
        u = self._u[self._ui]
        self._ui += 1
        return min(int(u * m), m - 1)

    def _sym(self) -> int:
        if self._si >= len(self._s):
            self._s = self.symbols[self.rng.choice(len(self.symbols), size=self._BLOCK,
                                                   p=self.probs)]
            self._si = 0
        c = int(self._s[self._si])
        self._si += 1
        return c

    def edit(self, s: bytes, k: int) -> bytes:
        b = bytearray(s)
        for _ in range(k):
            op = self._int(3)
            if len(b) == 0:
                op = 1
            if op == 0:      # substitute
                pos = self._int(len(b))
                c = self._sym()
                while c == b[pos] and len(self.symbols) > 1:
                    c = self._sym()
                b[pos] = c
            elif op == 1:    # insert
                pos = self._int(len(b) + 1)
                b.insert(pos, self._sym())
            else:            # delete
                pos = self._int(len(b))
                del b[pos]
        return bytes(b)

    def near_dup(self, s: bytes, kmin: int, kmax: int, lmin: int | None, lmax: int | None) -> bytes:
        """An edited copy with k ~ U{kmin..kmax}; redrawn (up to 100 tries, else an exact copy)
        when the result leaves [lmin, lmax]."""
        for _ in range(100):
            k = kmin + self._int(kmax - kmin + 1)
            t = self.edit(s, k)
            if (lmin is None or len(t) >= lmin) and (lmax is None or len(t) <= lmax):
                return t
        return s


def _finish(rng, strings: list[bytes], name: str, meta: dict) -> Collection:
    perm = rng.permutation(len(strings))
    col = from_list([strings[k] for k in perm], name=name)
    col.meta = dict(meta)
    col.meta["sha256"] = col.sha256()
    return col


def cfg1(n: int = 10_000, seed: int | None = None) -> Collection:
    """Small uniform collection: n/2 base strings, lengths U{8..20}, chars uniform over a-z and
    space; one copy of each base with U{0..3} random edits (copies are not length-clamped)."""
    rng = np.random.default_rng(BASE_SEED + 1 if seed is None else seed)
    nb = n // 2
    lens = rng.integers(8, 21, size=nb)
    base = _iid_strings(rng, lens, ALPHA27, np.full(27, 1 / 27))
    ed = _Editor(rng, ALPHA27, np.full(27, 1 / 27))
    copies = [ed.edit(s, int(rng.integers(0, 4))) for s in base]
    extra = [] if n % 2 == 0 else [base[0]]
    return _finish(rng, base + copies + extra, "uniform27-short", {"cfg": 1})


def cfg2(n: int = 1_000_000, seed: int | None = None) -> Collection:
    """Short strings shaped like DBLP Author: 70% originals with length round(N(15, 4)) clamped to
    [5, 40], chars i.i.d. over a-z + space with English letter frequencies (space 0.18); 30%
    near-duplicates of uniformly chosen originals with U{1..4} edits."""
    rng = np.random.default_rng(BASE_SEED + 2 if seed is None else seed)
    probs = english27_probs()
    n_orig = int(round(0.7 * n))
    lens = np.clip(np.rint(rng.normal(15, 4, size=n_orig)), 5, 40).astype(np.int64)
    orig = _iid_strings(rng, lens, ALPHA27, probs)
    ed = _Editor(rng, ALPHA27, probs)
    src = rng.integers(0, n_orig, size=n - n_orig)
    dups = [ed.near_dup(orig[int(j)], 1, 4, 5, 40) for j in src]
    return _finish(rng, orig + dups, "english27-short", {"cfg": 2, "probs": probs.tolist()})


def cfg3(n: int = 500_000, seed: int | None = None) -> Collection:
    """Medium strings shaped like the AOL Query Log: 80% originals with length round(N(45, 15))
    clamped to [10, 120] over 40 symbols with Zipf(1.1) rank frequencies; 20% near-duplicates with
    U{1..8} edits."""
    rng = np.random.default_rng(BASE_SEED + 3 if seed is None else seed)
    probs = zipf_probs(40, 1.1)
    n_orig = int(round(0.8 * n))
    lens = np.clip(np.rint(rng.normal(45, 15, size=n_orig)), 10, 120).astype(np.int64)
    orig = _iid_strings(rng, lens, ALPHA40, probs)
    ed = _Editor(rng, ALPHA40, probs)
    src = rng.integers(0, n_orig, size=n - n_orig)
    dups = [ed.near_dup(orig[int(j)], 1, 8, 10, 120) for j in src]
    return _finish(rng, orig + dups, "zipf40-medium", {"cfg": 3})


def cfg4(n: int = 100_000, seed: int | None = None, vocab: int = 20_000,
         median: float = 700.0, sigma: float = 0.5) -> Collection:
    """Long strings built from words: a vocabulary of 20,000 words (lengths U{2..12}, chars uniform
    a-z) drawn with Zipf(1.0) rank frequencies, joined by single spaces and cut to a target length
    round(LogNormal(ln 700, 0.5)) clamped to [200, 2000]; 90% originals, 10% near-duplicates with
    U{1..40} edits."""
    rng = np.random.default_rng(BASE_SEED + 4 if seed is None else seed)
    letters = ALPHA27[:26]
    wlen = rng.integers(2, 13, size=vocab)
    wflat = letters[rng.integers(0, 26, size=int(wlen.sum()))]
    # Each vocabulary word followed by one space, stored flat.
    wl1 = wlen + 1
    woff = np.zeros(vocab + 1, dtype=np.int64)
    np.cumsum(wl1, out=woff[1:])
    vflat = np.empty(int(woff[-1]), dtype=np.uint8)
    src_off = np.concatenate([[0], np.cumsum(wlen)[:-1]])
    for w in range(vocab):
        vflat[woff[w]:woff[w] + wlen[w]] = wflat[src_off[w]:src_off[w] + wlen[w]]
        vflat[woff[w] + wlen[w]] = ord(" ")
    wprobs = zipf_probs(vocab, 1.0)
    n_orig = int(round(0.9 * n))
    targets = np.clip(np.rint(rng.lognormal(np.log(median), sigma, size=n_orig)), 200, 2000)
    targets = targets.astype(np.int64)
    mean_w = float(np.dot(wprobs, wl1))
    n_words = int(targets.sum() / mean_w * 1.15) + 10_000
    while True:
        wids = rng.choice(vocab, size=n_words, p=wprobs)
        lens = wl1[wids]
        pos = np.zeros(n_words + 1, dtype=np.int64)
        np.cumsum(lens, out=pos[1:])
        starts = np.empty(n_orig, dtype=np.int64)
        w = 0
        ok = True
        for j in range(n_orig):
            if w >= n_words:
                ok = False
                break
            starts[j] = pos[w]
            w = int(np.searchsorted(pos, pos[w] + targets[j], side="left"))
        if ok and starts[-1] + targets[-1] <= pos[-1]:
            break
        n_words = int(n_words * 1.5)
    total = int(pos[-1])
    rep_start = woff[wids] - pos[:-1]
    stream = vflat[np.repeat(rep_start, lens) + np.arange(total, dtype=np.int64)]
    sb = stream.tobytes()
    orig = [sb[starts[j]:starts[j] + targets[j]] for j in range(n_orig)]
    del stream, sb
    cprobs = np.full(27, 1 / 27)
    ed = _Editor(rng, ALPHA27, cprobs)
    src = rng.integers(0, n_orig, size=n - n_orig)
    dups = [ed.near_dup(orig[int(j)], 1, 40, 200, 2000) for j in src]
    return _finish(rng, orig + dups, "zipfwords-long", {"cfg": 4, "sigma": sigma})


def cfg5_index(n: int = 1_000_000, seed: int | None = None) -> Collection:
    """Serving index: lengths U{10..120}, chars i.i.d. with the English-frequency 27-symbol
    distribution."""
    rng = np.random.default_rng(BASE_SEED + 5 if seed is None else seed)
    lens = rng.integers(10, 121, size=n)
    return _finish(rng, _iid_strings(rng, lens, ALPHA27, english27_probs()), "serving-index",
                   {"cfg": 5})


def cfg5_batch(rng, index: Collection, mean: float = 64.0, tau_max: int = 8):
    """One serving batch: Poisson(mean) queries (0 is redrawn), each with tau ~ U{1..tau_max} and
    length U{10..120}; half are random strings, half are copies of a uniformly chosen indexed
    string with U{1..tau} edits.  Returns (Collection, taus int32[m])."""
    m = 0
    while m == 0:
        m = int(rng.poisson(mean))
    probs = english27_probs()
    ed = _Editor(rng, ALPHA27, probs)
    taus = rng.integers(1, tau_max + 1, size=m).astype(np.int32)
    out = []
    for q in range(m):
        if rng.random() < 0.5:
            ln = int(rng.integers(10, 121))
            out.append(_iid_strings(rng, [ln], ALPHA27, probs)[0])
        else:
            src = index.get(int(rng.integers(index.n)))
            out.append(ed.near_dup(src, 1, int(taus[q]), 10, 120))
    return from_list(out, name="serving-batch"), taus


def cfg5_queries(index: Collection, batches: int = 32, seed: int | None = None):
    """A fixed serving stream for parity checks: `batches` batches drawn by cfg5_batch from one
    seeded generator (seed 71715 + 100 by default).  Returns the list of (Collection, taus)."""
    rng = np.random.default_rng(BASE_SEED + 105 if seed is None else seed)
    return [cfg5_batch(rng, index) for _ in range(batches)]


def concat(parts) -> Collection:
    """The collections' strings back to back (ids renumbered in order)."""
    chars = np.concatenate([p.chars for p in parts]) if parts else np.empty(0, np.uint8)
    offs = [np.zeros(1, dtype=np.int64)]
    base = 0
    for p in parts:
        offs.append(p.offsets[1:].astype(np.int64) + base)
        base += int(p.offsets[-1])
    return Collection(chars.astype(np.uint8), np.concatenate(offs).astype(np.int32), "concat")


def random_small(rng, n: int, alphabet: bytes = b"ab", lmin: int = 0, lmax: int = 8,
                 dup_frac: float = 0.3, kmax: int = 2) -> Collection:
    """Tiny collections over a small alphabet with many repeats and near-duplicates, for
    exhaustive checks; lengths may be below tau + 1."""
    sym = np.frombuffer(alphabet, dtype=np.uint8)
    probs = np.full(len(sym), 1 / len(sym))
    ed = _Editor(rng, sym, probs)
    out: list[bytes] = []
    for _ in range(n):
        if out and rng.random() < dup_frac:
            src = out[int(rng.integers(len(out)))]
            out.append(ed.edit(src, int(rng.integers(0, kmax + 1))))
        else:
            ln = int(rng.integers(lmin, lmax + 1))
            out.append(bytes(sym[rng.integers(0, len(sym), size=ln)]))
    return from_list(out, name="random-small")


CONFIGS = {1: cfg1, 2: cfg2, 3: cfg3, 4: cfg4}
TAUS = {1: (2,), 2: (1, 2, 3, 4), 3: (2, 4, 6, 8), 4: (8, 16, 32)}
