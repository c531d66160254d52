#!/usr/bin/env python3
"""Writes tests/golden/fullsize.json: the oracle's exact results on every workload at its full
size, for the GPU parity tests (tests/test_gpu_golden.py).

For each (workload, tau): the number of pairs and the SHA-256 of the sorted pair list (rows of
two little-endian int32, (a, b) with a < b for a self-join, (query, indexed id) for the serving
stream), and the oracle's selected-substring, candidate, cell and side-path counts.  The result
of Definition 1 is a set with one canonical order (Theorem 6 makes Pass-Join reach exactly it),
so the hash pins the whole list.

Only oracle/ and workloads/ are used.  The oracle runs unchanged, split over processes by probe
string (oracle.self_join_pj_parallel): each process indexes every string and probes with its
share, and the shares' pairs are disjoint.

Usage: python tests/golden/make_fullsize.py [--procs N] [--only cfg2:4,cfg4:32,cfg5 ...]
The file is updated entry by entry, so a run can be split.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O      # noqa: E402
import workloads as W   # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fullsize.json")
CFG5_BATCHES = 32


def pairs_sha256(pairs: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(pairs, dtype="<i4").tobytes()).hexdigest()


def load() -> dict:
    if os.path.exists(OUT):
        with open(OUT) as f:
            return json.load(f)
    return {}


def save(d: dict) -> None:
    tmp = OUT + ".tmp"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
        f.write("\n")
    os.replace(tmp, OUT)


def entry(r: O.JoinResult, secs: float) -> dict:
    return {"pairs": int(len(r.pairs)), "pairs_sha256": pairs_sha256(r.pairs),
            "candidates": int(r.candidates), "cells": int(r.cells),
            "selected": int(r.selected), "side_pairs": int(r.side_pairs),
            "oracle_seconds": round(secs, 1)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=os.cpu_count() or 1)
    ap.add_argument("--only", default="", help="comma list of cfgN:tau or cfg5")
    args = ap.parse_args()
    only = set(x for x in args.only.split(",") if x)
    d = load()
    for cfg, taus in W.TAUS.items():
        name = f"cfg{cfg}"
        want = [t for t in taus if not only or f"{name}:{t}" in only or name in only]
        if not want:
            continue
        print(f"{name}: generating", flush=True)
        col = W.CONFIGS[cfg]()
        rec = d.setdefault(name, {})
        rec["n"] = col.n
        rec["arena_sha256"] = col.sha256()
        rec.setdefault("taus", {})
        for t in want:
            t0 = time.time()
            r = O.self_join_pj_parallel(col, t, procs=args.procs)
            e = entry(r, time.time() - t0)
            rec["taus"][str(t)] = e
            print(f"{name} tau={t}: {e}", flush=True)
            save(d)
    if not only or "cfg5" in only:
        print("cfg5: generating index and query stream", flush=True)
        S = W.cfg5_index()
        batches = W.cfg5_queries(S, CFG5_BATCHES)
        Q = W.concat([q for q, _ in batches])
        taus = np.concatenate([t for _, t in batches]).astype(np.int32)
        t0 = time.time()
        parts, cand, cells, sel, side = [], 0, 0, 0, 0
        for t in range(1, 9):
            ids = np.nonzero(taus == t)[0]
            if len(ids) == 0:
                continue
            r = O.join_pj_parallel(Q.subset(ids), S, t, procs=args.procs)
            p = r.pairs.copy()
            p[:, 0] = ids[p[:, 0]]
            parts.append(p)
            cand += r.candidates
            cells += r.cells
            sel += r.selected
            side += r.side_pairs
            print(f"cfg5 tau={t}: {len(ids)} queries, {len(p)} pairs", flush=True)
        pairs = np.concatenate(parts) if parts else np.empty((0, 2), np.int32)
        key = pairs[:, 0].astype(np.int64) << 32 | pairs[:, 1].astype(np.int64)
        pairs = pairs[np.argsort(key, kind="stable")]
        res = O.JoinResult(pairs, cand, cells, sel, side)
        e = entry(res, time.time() - t0)
        e.update({"index_n": S.n, "index_sha256": S.sha256(), "batches": CFG5_BATCHES,
                  "queries": Q.n, "queries_sha256": Q.sha256(),
                  "taus_sha256": hashlib.sha256(taus.astype("<i4").tobytes()).hexdigest()})
        d["cfg5"] = e
        print(f"cfg5: {e}", flush=True)
        save(d)


if __name__ == "__main__":
    main()
