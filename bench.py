#!/usr/bin/env python3
"""Benchmark: Pass-Join self-join of the short-string collection on one MI355X.

One step = the self-join of 1,000,000 synthetic short strings (lengths ~N(15, 4) in [5, 40],
27 symbols with English letter frequencies, 30% near-duplicates with 1-4 edits) at every
threshold tau in {1, 2, 3, 4}: all phases (arena, index, probe, verify, short path, dedupe) run
on the GPU with inputs resident in HBM and the pairs left in HBM.

Prints ONE JSON line on stdout.  `value` is candidates verified per second over the whole
step (the candidate count is the paper's: every (y, x, i, p) the multi-match probe generates).
The line also carries a serving measurement (p50/p99 latency at fixed arrival rates over a
resident index; see serving_bench) unless --no-serve is given.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X published peaks used for the roofline
PEAK_HBM_GBS = 8000.0
CUS, CLOCK_GHZ, LANES_PER_CU = 256, 2.4, 64
PEAK_INT32_TOPS = CUS * LANES_PER_CU * CLOCK_GHZ / 1000.0      # 39.3 T int32 lane-ops/s
OPS_PER_CELL = 7   # recurrence: compare, add, min, add, min; expected distance: add, min

WORKLOAD = ("cfg2 short-string self-join: 1,000,000 strings, lengths round(N(15,4)) in [5,40], "
            "27 symbols (a-z, space) with English letter frequencies, 30% near-duplicates with "
            "1-4 edits, tau in {1,2,3,4}")
# other workloads (--workload): generator, default size, default taus, description
OTHER_WORKLOADS = {
    "cfg3": ("cfg3", 500_000, "2,4,6,8",
             "cfg3 medium-string self-join: 500,000 strings, lengths round(N(45,15)) in [10,120], "
             "40 symbols with Zipf(1.1) frequencies, 20% near-duplicates with 1-8 edits"),
    "cfg4": ("cfg4", 100_000, "8,16,32",
             "cfg4 long-string self-join: 100,000 strings of words from a 20,000-word Zipf(1.0) "
             "vocabulary, lengths round(LogNormal(ln 700, 0.5)) in [200,2000], 10% "
             "near-duplicates with 1-40 edits"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


DEVICE_SOURCES = ("pj_device.hip", "pj_device_common.h", "pj_internal.h")


def kernel_source_sha() -> str:
    """Hash of the device sources (the kernels' code); host-side changes do not alter it."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1111_7171_amd", "csrc")
    for f in DEVICE_SOURCES:
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel: str, sha: str, workload: str):
    """HBM traffic per launch measured by rocprofv3 PMC runs (profiles/traffic.json) for this
    kernel on this workload, only if the kernels have not changed since."""
    p = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    e = d.get(kernel)
    if not e or e.get("source_sha") != sha or e.get("workload_key") != workload:
        return None
    return e.get("bytes_per_launch")


def cpu_info() -> dict:
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"cpu_model": model, "nproc": os.cpu_count(), "usable_cpus": usable}


# Probe-share sampling of the oracle (a share = the probe strings at visiting ranks r = w mod K;
# every process still indexes all strings): K per tau for the all-core leg (as a multiple of the
# process count) and for the one-core leg.
CPU_SHARES_ALL = {1: 1, 2: 1, 3: 8, 4: 80}
CPU_SHARES_ONE = {1: 1, 2: 8, 3: 60, 4: 400}


def cpu_baseline(col, taus):
    """The oracle's Pass-Join (plain C, unchanged) on a bounded sample of the same workload,
    on all usable host cores (one process per core, each probing its own shares) and on one
    core.  Returns candidates per second of the all-core leg, with the one-core leg beside it."""
    import oracle as O
    info = cpu_info()
    procs = max(1, min(16, info["usable_cpus"]))
    legs = {}
    for leg, nproc, table in (("all_cores", procs, CPU_SHARES_ALL), ("one_core", 1, CPU_SHARES_ONE)):
        cands, secs, parts = 0, 0.0, []
        for t in taus:
            k = table.get(t, 200) * (nproc if leg == "all_cores" else 1)
            only = list(range(nproc)) if leg == "all_cores" else [0]
            t0 = time.perf_counter()
            r = O.self_join_pj_parallel(col, t, procs=nproc, shares=k, only=only)
            dt = time.perf_counter() - t0
            cands += r.candidates
            secs += dt
            parts.append(f"tau={t}: {len(only)}/{k} of the probe strings, {r.candidates} "
                         f"candidates, {dt:.1f}s")
            log(f"cpu baseline ({leg}, {nproc} process(es))", parts[-1])
        legs[leg] = {"value": cands / secs, "cores": nproc, "seconds": round(secs, 2),
                     "sample": "; ".join(parts)}
    a = legs["all_cores"]
    return {"value": a["value"], "unit": "candidates/s", "cores": a["cores"], "kind": "oracle",
            "sample": "all 1,000,000 strings indexed by every process (Algorithm 1 order), "
                      "probe strings sampled by visiting rank; time includes each process's "
                      "index build. " + a["sample"],
            "one_core": legs["one_core"], **info}


# Fixed serving arrival rates (batches/s): 50% and 80% of the closed-loop saturation of the
# captured path measured on one MI355X (8,300 batches/s), frozen so that every run reports its
# latency at the same QPS.
SERVE_LAMBDAS = (4150.0, 6640.0)


def serving_bench(P, W, n_index: int, seconds: float, slots: int, compare_eager: bool = True):
    """Open-loop serving: batches of Poisson(64) queries (tau U{1..8}, lengths U{10..120}, half
    edited copies of indexed strings) arrive as a Poisson process against a resident index of
    n_index strings, at the fixed rates SERVE_LAMBDAS.  The closed-loop saturation throughput is
    measured too.  Latency = submit -> pairs in host memory (server clock), per batch and per
    query (a query's latency is its batch's), split into the wait for a slot (submit -> admit)
    and the batch's service time (admit -> done); admission deferrals are counted.  The
    uncaptured path is also measured at the lower rate."""
    import threading

    import numpy as np
    log(f"serving: building index of {n_index} strings, tau 1..8")
    S = W.cfg5_index(n_index)
    t0 = time.perf_counter()
    idx = P.pj_build_index(S, 1, 8)
    build_s = time.perf_counter() - t0
    info = idx.info()
    rng = np.random.default_rng(71715)
    pool = [W.cfg5_batch(rng, S) for _ in range(256)]
    out = {"index_strings": n_index, "index_build_s": round(build_s, 3),
           "index_device_bytes": info["device_bytes"], "slots": slots}

    def open_loop(srv, lam, seed, label):
        ids, lock = [], threading.Lock()
        stop = threading.Event()
        lats, waits, svcs, nq, batch_sizes, qsz, defer, defer_mem = [], [], [], [0], [], [], [0], [0]

        def collector():
            j = 0
            while True:
                with lock:
                    have = j < len(ids)
                if not have:
                    if stop.is_set():
                        with lock:
                            if j >= len(ids):
                                return
                    time.sleep(0.0005)
                    continue
                rid, m = ids[j]
                _, inf = srv.wait(rid)
                lats.append(inf["t_done_ms"] - inf["t_submit_ms"])
                waits.append(inf["t_admit_ms"] - inf["t_submit_ms"])
                svcs.append(inf["t_done_ms"] - inf["t_admit_ms"])
                batch_sizes.append(inf["batch_requests"])
                qsz.append(m)
                defer[0] += inf["deferrals"]
                defer_mem[0] += inf["deferred_by_memory"]
                nq[0] += m
                j += 1

        th = threading.Thread(target=collector)
        th.start()
        arr = np.random.default_rng(seed)
        t0 = time.perf_counter()
        t_next = t0
        k = 0
        while t_next - t0 < seconds:
            now = time.perf_counter()
            if now < t_next:
                time.sleep(min(t_next - now, 0.002))
                continue
            q, t = pool[k % len(pool)]
            rid = srv.submit(q, t)
            with lock:
                ids.append((rid, q.n))
            k += 1
            t_next += arr.exponential(1.0 / lam)
        stop.set()
        th.join()
        wall = time.perf_counter() - t0
        L, Wt, Sv = np.array(lats), np.array(waits), np.array(svcs)
        Lq = np.repeat(L, np.array(qsz, dtype=np.int64))        # per query
        pc = lambda a, q: round(float(np.percentile(a, q)), 3)
        rec = {
            "lambda_batches_per_s": round(lam, 2), "batches": len(L), "queries": int(len(Lq)),
            "p50_ms": pc(L, 50), "p99_ms": pc(L, 99), "p999_ms": pc(L, 99.9),
            "query_p50_ms": pc(Lq, 50), "query_p99_ms": pc(Lq, 99),
            "deferred_requests": int(defer[0]), "deferred_for_memory": int(defer_mem[0]),
            "queue_wait_p50_ms": pc(Wt, 50), "queue_wait_p99_ms": pc(Wt, 99),
            "service_p50_ms": pc(Sv, 50), "service_p99_ms": pc(Sv, 99),
            "batches_per_s": round(len(L) / wall, 2), "queries_per_s": round(nq[0] / wall, 1),
            "mean_requests_per_device_batch": round(float(np.mean(batch_sizes)), 2),
        }
        log("serving", label, rec)
        return rec

    with P.Server(idx, slots=slots, max_batch_queries=512, mem_budget=8 << 30) as srv:
        for k in range(8):                                   # warm the slots' scratch
            srv.wait(srv.submit(*pool[k]))
        # closed loop: keep 2 * slots batches outstanding
        t_end = time.perf_counter() + max(2.0, seconds / 4)
        pend, done, k = [], 0, 0
        t0 = time.perf_counter()
        while time.perf_counter() < t_end or pend:
            while time.perf_counter() < t_end and len(pend) < 2 * slots:
                pend.append(srv.submit(*pool[k % len(pool)]))
                k += 1
            srv.wait(pend.pop(0))
            done += 1
        sat = done / (time.perf_counter() - t0)
        out["saturation_batches_per_s"] = round(sat, 2)
        levels = []
        for k, lam in enumerate(SERVE_LAMBDAS):
            rec = open_loop(srv, lam, 50 + 30 * k, f"captured {lam:g}/s")
            rec["load_of_measured_saturation"] = round(lam / sat, 3)
            levels.append(rec)
        out["levels"] = levels
    if compare_eager:
        # the same arrival rate (50% of the captured saturation) with uncaptured batches
        with P.Server(idx, slots=slots, max_batch_queries=512, mem_budget=8 << 30,
                      eager=True) as srv:
            for k in range(8):
                srv.wait(srv.submit(*pool[k]))
            rec = open_loop(srv, SERVE_LAMBDAS[0], 50, f"uncaptured {SERVE_LAMBDAS[0]:g}/s")
            rec["load_of_captured_saturation"] = round(SERVE_LAMBDAS[0] / sat, 3)
            out["uncaptured"] = rec
    idx.free()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--taus", default=None, help="default: 1,2,3,4 (cfg2)")
    ap.add_argument("--n", type=int, default=None, help="default: 1,000,000 (cfg2)")
    ap.add_argument("--workload", default="cfg2", choices=["cfg2"] + sorted(OTHER_WORKLOADS),
                    help="cfg2 (the default benchmark) or another synthetic workload")
    ap.add_argument("--mode", type=int, default=0,
                    help="0 auto, 1 plain, 2 batched, 3 batched with shared-prefix lists")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run a plain device copy of this size (PMC calibration)")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--no-graph", action="store_true",
                    help="skip the timing of hipGraph-replayed self-joins (pj_plan_run)")
    ap.add_argument("--no-e2e", action="store_true",
                    help="skip the end-to-end (host arrays in, host pairs out) timings")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-n", type=int, default=1_000_000)
    ap.add_argument("--serve-slots", type=int, default=4)
    ap.add_argument("--no-tune", action="store_true",
                    help="skip autotuning the launch parameters (built-in defaults)")
    ap.add_argument("--selection", type=int, default=0,
                    help="substring selection: 0 multi-match (default), 1 position, 2 shift, "
                         "3 every substring (Sec. 4)")
    ap.add_argument("--window-bytes", type=int, default=0,
                    help="time pj_self_join_streamed with length windows of at most this many "
                         "string bytes instead (host inputs and outputs: includes the copies)")
    ap.add_argument("--tune-cache", default=None,
                    help="autotune cache file (written when tuning; with --no-tune it is only "
                         "read).  Default: a fresh file in the temp directory")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the Pass-Join hot path here is a single-GPU build "
              "(multi-GPU sharding is a design note, not implemented).", file=sys.stderr)
        sys.exit(2)

    import numpy as np

    import workloads as W

    workload = WORKLOAD
    if args.workload == "cfg2":
        args.n = args.n or 1_000_000
        args.taus = args.taus or "1,2,3,4"
        gen = W.cfg2
    else:
        name, n0, taus0, workload = OTHER_WORKLOADS[args.workload]
        args.n = args.n or n0
        args.taus = args.taus or taus0
        gen = getattr(W, name)
        # the CPU baseline's sampling and the serving run are sized for cfg2
        args.no_cpu = True
        args.no_serve = True
    taus = [int(t) for t in args.taus.split(",")]
    log(f"generating workload {args.workload} n={args.n}")
    col = gen(args.n)
    # the CPU baseline runs first: its worker processes fork from a process that has not
    # touched the GPU (so they hold no device handles), and nothing else competes for the CPU
    cpu = None if args.no_cpu else cpu_baseline(col, taus)

    import torch

    import paper_1111_7171_amd as P
    dev = torch.device("cuda:0")
    chars = torch.from_numpy(col.chars.copy()).to(dev)
    offs = torch.from_numpy(col.offsets.copy()).to(dev)
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    if args.calib_copy_mib:
        # a plain elementwise kernel of known traffic (one dispatch reads and writes nbytes):
        # the runtime's device-to-device copy may split a copy or hand parts of it to a DMA
        # engine, so it is not used for this
        nbytes = args.calib_copy_mib << 20
        a = torch.ones(nbytes // 4, dtype=torch.int32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            torch.add(a, 1, out=b)
        torch.cuda.synchronize()
        log(f"calibration kernel: {nbytes} bytes read and written, x 3")

    # autotuning (outside the timed region): launch parameters per (GPU, tau, length bucket),
    # searched on this workload; the timed joins read them from the cache file
    tuning = None
    cache = args.tune_cache if args.mode != P.MODE_PLAIN else None
    if not args.no_tune and args.mode != P.MODE_PLAIN:
        import tempfile
        cache = args.tune_cache or os.path.join(tempfile.mkdtemp(prefix="pj_tune_"), "tune.txt")
        tuning = {}
        for t in taus:
            r = P.pj_tune(col, t, tune_cache=cache)
            tuning[str(t)] = r
            log(f"tuned tau={t}: {r}")

    class _HostPairs:
        def free(self):
            pass

    def step(collect):
        outs = []
        for t in taus:
            if args.window_bytes:
                P.pj_self_join_streamed(col, t, args.window_bytes, mode=args.mode,
                                        tune_cache=cache, selection=args.selection)
                r = _HostPairs()
            else:
                r = P.pj_self_join((chars, offs), t, mode=args.mode, outputs_on_device=True,
                                   stream=stream, tune_cache=cache, selection=args.selection)
            st = P.pj_last_stats()
            outs.append(r)
            if collect is not None:
                collect.append((t, st))
        return outs

    for w in range(args.warmup):
        for r in step(None):
            r.free()
        log(f"warmup {w + 1}/{args.warmup} done")

    torch.cuda.synchronize()
    stats = []
    keep = []
    t0 = time.perf_counter()
    for k in range(args.steps):
        keep.extend(step(stats))
        log(f"step {k + 1}/{args.steps} done")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    for r in keep:
        r.free()

    cand = sum(s["candidates"] for _, s in stats)
    cells = sum(s["cells"] for _, s in stats)
    verify_ms = sum(s["ms_verify_kernel"] for _, s in stats)
    probe_ms = sum(s["ms_probe_kernel"] for _, s in stats)
    # the dominant kernel: list-segment verification (k_verify_segs)
    list_ms = sum(s["ms_list_kernel"] for _, s in stats)
    list_cells = sum(s["list_cells"] for _, s in stats)
    list_launches = sum(s["list_launches"] for _, s in stats)
    # per tau: the median wall time over the timed steps, the counts and phase times of the
    # last step
    per_tau = {}
    for t, s in stats[-len(taus):]:
        med = float(np.median([x["ms_total"] for tt, x in stats if tt == t]))
        per_tau[str(t)] = {
            "ms": round(med, 3), "ms_last": round(s["ms_total"], 3),
            "candidates": s["candidates"], "cells": s["cells"],
            "pairs": s["pairs"], "selected": s["selected"], "hits": s["hits"],
            "index_entries": s["index_entries"],
            "ms_index": round(s["ms_index"], 3), "ms_probe": round(s["ms_probe"], 3),
            "ms_verify": round(s["ms_verify"], 3), "ms_output": round(s["ms_output"], 3),
            "ms_verify_kernel": round(s["ms_verify_kernel"], 3),
            "shared_rows": s["shared_rows"], "shared_cells": s["shared_cells"],
            "key_collisions": s["key_collisions"],
            "candidates_per_s": s["candidates"] / max(med, 1e-9) * 1e3,
            "gcups": s["cells"] / max(s["ms_verify_kernel"], 1e-9) / 1e6,
        }

    # end to end (host arrays in -> sorted host pairs out, as the C ABI returns them; PCIe
    # copies included), outside the timed region: median of 5 per tau, beside the
    # device-resident time of the timed steps
    end_to_end = {}
    if not args.window_bytes and not args.no_e2e:
        for t in taus:
            runs, m = [], 0
            for _ in range(5):
                t0 = time.perf_counter()
                hp = P.pj_self_join_host(col, t, mode=args.mode, tune_cache=cache,
                                         selection=args.selection)
                runs.append((time.perf_counter() - t0) * 1e3)
                m = hp.count
                hp.free()
            end_to_end[str(t)] = {"ms": round(float(np.median(runs)), 3), "pairs": m,
                                  "device_resident_ms": per_tau[str(t)]["ms"]}
            log(f"end to end tau={t}: {end_to_end[str(t)]}")

    # the same self-joins replayed from hipGraphs (pj_self_join_plan / pj_plan_run: each tau's
    # launches captured once, then replayed after a device checksum of the strings), outside the
    # timed region: median of the replays, beside the eager time of the timed steps
    graph = {}
    if not args.window_bytes and not args.no_graph:
        step_ms = 0.0
        for t in taus:
            plan = P.Plan((chars, offs), t, mode=args.mode, stream=stream, tune_cache=cache,
                          selection=args.selection)
            plan.run().free()
            runs = []
            for _ in range(max(args.steps, 3)):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r = plan.run()
                runs.append((time.perf_counter() - t0) * 1e3)
                if P.pj_last_stats()["replayed"] != 1:
                    raise RuntimeError("the plan did not replay")
                r.free()
            plan.free()
            ms = float(np.median(runs))
            graph[str(t)] = {"ms": round(ms, 3), "eager_ms": per_tau[str(t)]["ms"]}
            step_ms += ms
            log(f"graph replay tau={t}: {graph[str(t)]}")
        graph["step_ms"] = round(step_ms, 3)
        graph["host_syncs_per_call"] = 2

    sha = kernel_source_sha()
    # dominant verification kernel: the list-segment kernel (k_verify_segs) when it takes most
    # of the verification time, else candidate by candidate verification -- the long-string
    # path (k_verify_cont passes, indexed strings longer than 128 bytes) or k_verify_batched.
    # Algorithmic work = OPS_PER_CELL integer ops per DP cell the kernel evaluates (counted on
    # the device per kernel).
    other_ms = max(verify_ms - list_ms, 0.0)
    if list_ms >= other_ms and list_launches > 0:
        rk, k_ms, k_cells, k_launches = "k_verify_segs", list_ms, list_cells, list_launches
    else:
        rk = "k_verify_cont" if int(col.lengths().max(initial=0)) > 128 else "k_verify_batched"
        k_ms, k_cells = other_ms, cells - list_cells
        k_launches = len(stats)      # one verification call per self-join
    per_launch_s = k_ms / 1e3 / max(k_launches, 1)
    ops_per_launch = OPS_PER_CELL * k_cells / max(k_launches, 1)
    achieved = ops_per_launch / max(per_launch_s, 1e-12) / 1e12
    # the counters were taken on one configuration: the workload with its size, taus,
    # selection and mode
    traffic = load_traffic(rk, sha, f"{args.workload} n={args.n} taus={args.taus} "
                                    f"selection={args.selection} mode={args.mode}")
    line = {
        "metric": "self-join wall time, candidates/s, GCUPS; serving p50/p99 latency at fixed QPS",
        "value": cand / elapsed,
        "unit": "candidates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": workload, "n": args.n, "taus": taus, "mode": args.mode,
                   **({"selection": args.selection} if args.selection else {}),
                   **({"window_bytes": args.window_bytes, "inputs": "host"}
                      if args.window_bytes else {})},
        "gcups": cells / max(verify_ms, 1e-9) / 1e6,
        "self_join_ms": {k: v["ms"] for k, v in per_tau.items()},
        "end_to_end_ms": {k: v["ms"] for k, v in end_to_end.items()},
        "end_to_end": end_to_end,
        "graph_replay": graph,
        "per_tau": per_tau,
        "probe_kernel_ms_per_step": probe_ms / args.steps,
        "verify_kernel_ms_per_step": verify_ms / args.steps,
        "roofline": {
            "kernel": rk,
            "bound": "alu",
            "achieved": achieved,
            "peak": PEAK_INT32_TOPS,
            "unit": "TOP/s",
            "frac": achieved / PEAK_INT32_TOPS,
            "traffic": traffic,
            "ops_per_cell": OPS_PER_CELL,
            "launches": k_launches,
            "avg_launch_ms": per_launch_s * 1e3,
            "cells_per_launch": k_cells / max(k_launches, 1),
            "share_of_verify_time": k_ms / max(verify_ms, 1e-9),
        },
        "kernel_source_sha": sha,
        "tuning": tuning,
    }
    if not args.no_serve:
        line["serving"] = serving_bench(P, W, args.serve_n, args.serve_seconds, args.serve_slots)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
