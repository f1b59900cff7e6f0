#!/usr/bin/env python3
"""Benchmark of the gate-sweep hot path on one MI355X.

A step is one solve: a random circuit of G = 4*nq dense gates (k = 1, 2, 3
with probabilities .50/.35/.15, random ordered targets, random unitaries)
applied in place to one nq-qubit complex FP64 state that is already resident
in HBM.  The default workload is the largest single state the 64 GB device
budget admits, nq = 31 (2^31 amplitudes, 32 GiB), seed 1, run by the fused
multi-gate path (qcw_circuit_fused_ex with all plan flags: gates on disjoint
qubits reordered into fewer passes, gates merged inside a pass, the
three-product complex arithmetic; --plan 0 for the bit-exact list-order
passes, --path plain for one sweep per gate).

Prints ONE JSON line with the throughput (solves/s), the roofline of the
dominant kernel (algorithmic bytes 32 * 2^nq per launch -- one pass reads and
writes every amplitude once -- over its launch durations, measured with HIP
events recorded by the library on the launch stream), the CPU oracle timed on
a bounded sample of the same solve, and sections for the batched (4096
instances) and served (open-loop Poisson) forms.

--counters runs each kernel once at nq = 28 beside a plain copy of known size
(the sweep for k = 1, 2, 3, once more on the three lowest qubits, and one fused
solve),
for rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs; it prints what it launched.
--section NAME runs one of the extra sections alone (e.g. multiverse_nq12) and
prints its JSON object, for profiling that section's kernels.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "solves/sec batched vs plain GPU at stated error; p50/p99 latency; % roofline"


def _args():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=5)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--nq", type=int, default=31)
    p.add_argument("--gates", type=int, default=0, help="gates per circuit (default 4*nq)")
    p.add_argument("--seed", type=int, default=1)
    p.add_argument("--path", choices=["fused", "plain"], default="fused",
                   help="fused multi-gate passes (default) or one sweep per gate")
    p.add_argument("--tile-bits", type=int, default=0)
    p.add_argument("--plan", type=int, choices=range(8), default=7,
                   help="fused plan flags: 1 = QCW_PLAN_COMMUTE, 2 = QCW_PLAN_FUSE, "
                        "4 = QCW_PLAN_3M (default all three)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sample-log2", type=int, default=26,
                   help="contiguous outputs per gate timed on the CPU oracle")
    p.add_argument("--serve-seconds", type=float, default=60.0,
                   help="length of the open-loop serving run (config 3: 60 s)")
    p.add_argument("--serve-rate", type=float, default=2000.0)
    p.add_argument("--serve-sweep-seconds", type=float, default=2.0,
                   help="seconds per offered rate in the serving rate sweep (0: skip)")
    p.add_argument("--no-compare", action="store_true",
                   help="skip the untimed comparison solves (plain path, list-order plan) and the "
                        "error checks, so a kernel trace holds only the timed launches")
    p.add_argument("--oracle-check-nq", type=int, default=28,
                   help="size of the oracle check of the timed plan (0: skip)")
    p.add_argument("--skip-extra", action="store_true",
                   help="only the headline workload (no batched/serving sections)")
    p.add_argument("--section", default="",
                   help="run one of the extra sections alone and print its JSON (for profiling)")
    p.add_argument("--counters", action="store_true",
                   help="launch each kernel once at nq=28 next to a 2 GiB copy, then exit")
    p.add_argument("--tune-table", default=os.path.join(ROOT, "paper_1101_1785_amd", "tune",
                                                        "gfx950.txt"))
    return p.parse_args()


KERNEL_SOURCES = {"sweep": ("sweep.hip", "qcw_device.h"), "fused": ("fused.hip", "qcw_device.h")}


def _source_hash(kernel: str) -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1101_1785_amd", "csrc")
    for f in KERNEL_SOURCES[kernel]:
        h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def _traffic(kernel: str, nq: int):
    """HBM bytes per launch from the committed rocprofv3 counter record (bytes per
    amplitude measured at nq = 28, times 2^nq), or None when the kernel's sources
    changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    e = d.get(kernel)
    if not e or e.get("source_hash") != _source_hash(kernel):
        return None
    return e["bytes_per_amplitude"] * float(1 << nq)


def cpu_baseline(circ, psi_host, sample_log2: int):
    """Oracle time for a bounded sample: a contiguous block of 2^s outputs of every
    gate of the circuit, evaluated from the input state, scaled to a whole solve."""
    import oracle
    nq = circ.nq
    N = 1 << nq
    S = min(N, 1 << sample_log2)
    start = (N // 2) - S // 2 if N > S else 0
    idx = np.arange(start, start + S, dtype=np.uint64)
    oracle.apply_at(circ.mats[0], circ.targets[0], psi_host, idx[:1024], nq=nq)  # warm
    t0 = time.perf_counter()
    for U, t in zip(circ.mats, circ.targets):
        oracle.apply_at(U, t, psi_host, idx, nq=nq)
    dt = time.perf_counter() - t0
    per_solve = dt * (N / S)
    cores = oracle.threads()
    # the same on one thread, over a 16x smaller sample
    S1 = max(1, S // 16)
    idx1 = idx[:S1]
    oracle.set_threads(1)
    try:
        t1 = time.perf_counter()
        for U, t in zip(circ.mats, circ.targets):
            oracle.apply_at(U, t, psi_host, idx1, nq=nq)
        dt1 = time.perf_counter() - t1
    finally:
        oracle.set_threads(cores)
    return {"value": 1.0 / per_solve, "unit": "solves/s", "cores": cores,
            "kind": "oracle",
            "sample": f"{S} contiguous outputs (2^{sample_log2}) of each of the {len(circ)} gates "
                      f"at nq={nq}, {dt:.2f} s of CPU work, scaled by 2^{nq}/{S} to one solve",
            "one_core": {"value": 1.0 / (dt1 * (N / S1)), "unit": "solves/s", "cores": 1,
                         "sample": f"{S1} outputs of each gate, {dt1:.2f} s, scaled to one solve"}}


FP64_PEAK_TFLOPS = 78.6


def _flops_per_solve(circ):
    """8m - 2 real flops per amplitude per gate (m complex products and m - 1 sums)."""
    N = 1 << circ.nq
    return sum(N * (8 * (1 << k) - 2) for k in circ.ks)


def _time_batch(torch, b, reps):
    """Per-execution ms of the batch: replayed as its hipGraph (one execution per
    graph launch), as one graph of 8 executions in a row (qcw_batch_run_repeat),
    and enqueued as one eager kernel launch (the same kernel and work); plus the
    host time each enqueue costs (a graph launch costs the HIP runtime tens of
    microseconds of host time, so back-to-back replays of a batch that runs
    for less than that are host-bound)."""
    out, host = {}, {}
    modes = (("graph", b.run, 1), ("graph_x8", lambda: b.run_repeat(8), 8),
             ("eager", b.run_eager, 1))
    for mode, fn, per in modes:
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        fn()
        torch.cuda.synchronize()
        n = max(1, reps // per)
        e0.record()
        c0 = time.perf_counter()
        for _ in range(n):
            fn()
        c1 = time.perf_counter()
        e1.record()
        torch.cuda.synchronize()
        out[mode] = e0.elapsed_time(e1) / (n * per)
        host[mode] = (c1 - c0) / n * 1e6
    return out, host


def bench_batched(torch, L, qi, seed, count, lo, hi, tune_table, reps=50, plain=True,
                  check=256, label=""):
    """One persistent launch over `count` instances vs sequential plain circuits."""
    import oracle
    print(f"[bench] batched {label}: generating {count} instances nq {lo}..{hi}",
          file=sys.stderr, flush=True)
    inst = qi.batch(seed, count, lo, hi)
    flat = np.concatenate([p for _, p, _ in inst])
    # error vs the oracle after exactly one application
    states = torch.from_numpy(flat).to("cuda")
    b = L.Batch([(nq, c) for nq, _, c in inst], states, tune_table=tune_table)
    b.run()
    torch.cuda.synchronize()
    got = states.cpu().numpy()
    offs = np.concatenate([[0], np.cumsum([1 << nq for nq, _, _ in inst])])
    sub = list(range(0, count, max(1, count // check)))[:check]
    refs = oracle.circuit_batch([inst[i] for i in sub])
    err = max(np.linalg.norm(got[offs[i]:offs[i + 1]] - r) / np.linalg.norm(r)
              for i, r in zip(sub, refs))
    tm, host_us = _time_batch(torch, b, reps)
    launch = "graph"          # the captured hipGraph replay is the batched form's figure
    ms = tm[launch]
    info = b.info(hi)
    # graph replays rotating over independent copies (own states and tables)
    # totalling at least 1 GiB, four times the 256 MB last-level cache, so
    # that replays start from HBM rather than from cache
    per_copy = 16 * flat.size + 64 * b.gates.size + 16 * b.mats.size
    rot = int(min(64, max(10, -(-(1 << 30) // per_copy))))
    copies, handles = [], []
    for _ in range(rot):
        st = torch.from_numpy(flat).to("cuda")
        copies.append(st)
        handles.append(L.qcw_batch_create(b.inst, len(b.inst), b.gates, b.gates.size, b.mats,
                                          b.mats.size, st, st.numel(), tune_table, None))
    for h in handles:
        L.qcw_batch_run(h)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    rounds = 5
    e0.record()
    for _ in range(rounds):
        for h in handles:
            L.qcw_batch_run(h)
    e1.record()
    torch.cuda.synchronize()
    cold_us = e0.elapsed_time(e1) / (rounds * rot) * 1e3
    for h in handles:
        L.qcw_batch_destroy(h)
    del copies
    b.close()
    flops = sum(_flops_per_solve(c) for _, _, c in inst)
    hbm = sum(32 * (1 << nq) + sum(16 * U.size + 64 for U in c.mats) for nq, _, c in inst)
    out = {
        "instances": count, "nq_range": [lo, hi], "gates_per_instance": "4*nq", "seed": seed,
        "batched_solves_per_s": count / (ms * 1e-3), "batched_us_per_launch": ms * 1e3,
        "launch": launch, "graph_us": tm["graph"] * 1e3, "eager_us": tm["eager"] * 1e3,
        "graph_x8_us_per_execution": tm["graph_x8"] * 1e3,
        "graph_x8_solves_per_s": count / (tm["graph_x8"] * 1e-3),
        "host_enqueue_us": host_us,
        "fp64_tflops": flops / (ms * 1e-3) / 1e12,
        "fp64_frac": flops / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
        "hbm_gbs_algorithmic": hbm / (ms * 1e-3) / 1e9,
        "max_rel_err_vs_oracle": err, "checked_instances": len(sub),
        "rotating_copies": rot, "rotating_copies_graph_us": cold_us,
        "rotating_copies_solves_per_s": count / (cold_us * 1e-6),
        "tile_shape_at_max_nq": L.qcw_batch_variant_name(info[0]),
        "grid_blocks": info[1], "lds_bytes_per_block": info[2],
        "tune_table": os.path.relpath(tune_table, ROOT) if tune_table else None,
    }
    if plain:
        packed = [L.pack_circuit(c) for _, _, c in inst]
        psis = [torch.from_numpy(p).to("cuda") for _, p, _ in inst]
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for (nq, _, c), (g, m), ps in zip(inst, packed, psis):
            L.qcw_circuit(ps, nq, g, len(c), m, m.size)
        e1.record()
        torch.cuda.synchronize()
        pm = e0.elapsed_time(e1)
        out["plain_solves_per_s"] = count / (pm * 1e-3)
        out["batched_over_plain"] = out["batched_solves_per_s"] / out["plain_solves_per_s"]
        pg = np.concatenate([p.cpu().numpy() for p in psis])
        out["batched_equals_plain_bitwise"] = bool(np.array_equal(pg, got))
        out["max_abs_diff_vs_plain"] = float(np.max(np.abs(pg - got)))
        # one persistent-kernel launch per instance (eager), over the first
        # `single` instances; set-up outside the timed region
        single = min(count, 512)
        one = [L.Batch([(nq, c)], ps, tune_table=tune_table)
               for (nq, _, c), ps in zip(inst[:single], psis[:single])]
        for x in one:
            x.run_eager()
        torch.cuda.synchronize()
        e0.record()
        for x in one:
            x.run_eager()
        e1.record()
        torch.cuda.synchronize()
        sm = e0.elapsed_time(e1)
        for x in one:
            x.close()
        out["single_launch_per_instance_solves_per_s"] = single / (sm * 1e-3)
        out["single_launch_instances_timed"] = single
    return out


def bench_serving(L, qi, seed, rate, seconds, lo, hi, tune_table, pool=4096):
    """Open-loop Poisson arrivals; latency from each request's scheduled arrival."""
    import threading
    arr = qi.poisson_arrivals(seed, rate, seconds)
    print(f"[bench] serving: {arr.size} arrivals at {rate}/s for {seconds}s "
          f"(request pool {pool})", file=sys.stderr, flush=True)
    inst = qi.batch(seed, pool, lo, hi)
    reqs = [(nq, p, *L.pack_circuit(c)) for nq, p, c in inst]
    s = L.Server(hbm_budget_bytes=1 << 30, max_slots=1024, gates_per_tick=0, max_nq=hi,
                 tune_table=tune_table)
    # warm the path (kernel load, plan cache)
    for nq, p, g, m in reqs[:64]:
        s.wait(s.submit(nq, psi0=p, gates=g, mats=m), nq)
    tickets = [None] * arr.size
    done_ns = np.zeros(arr.size, np.int64)
    status = np.zeros(arr.size, np.int64)
    t0 = time.monotonic_ns() + 20_000_000
    sched = t0 + (arr * 1e9).astype(np.int64)
    ready = threading.Semaphore(0)

    submit_s = [0.0]

    def client():
        for i in range(arr.size):
            dt = (sched[i] - time.monotonic_ns()) / 1e9
            if dt > 0:
                time.sleep(dt)
            nq, p, g, m = reqs[i % pool]
            c0 = time.perf_counter()
            tickets[i] = s.submit(nq, psi0=p, gates=g, mats=m)
            submit_s[0] += time.perf_counter() - c0
            ready.release()

    def collector():
        for i in range(arr.size):
            ready.acquire()
            nq = reqs[i % pool][0]
            out, st = s.wait(tickets[i], nq, timeout_s=120.0)
            done_ns[i] = st.t_done_ns
            status[i] = 0 if out is not None else st.status

    tc, tr = threading.Thread(target=client), threading.Thread(target=collector)
    tc.start(); tr.start(); tc.join(); tr.join()
    cnt = s.counters()
    s.close()
    lat = (done_ns - sched) / 1e6
    span = (done_ns.max() - sched.min()) / 1e9
    return {
        "rate_per_s": rate, "seconds": seconds, "requests": int(arr.size),
        "nq_range": [lo, hi], "gates_per_request": "4*nq", "seed": seed,
        "request_pool": pool,
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "max_ms": float(lat.max()), "solves_per_s": float(arr.size / span),
        "failed": int(np.count_nonzero(status)), "ticks": int(cnt["ticks"]),
        "peak_active": int(cnt["peak_active"]), "peak_pending": int(cnt["peak_pending"]),
        "client_submit_us": submit_s[0] / arr.size * 1e6,
        "latency_from": "scheduled arrival to completion (open loop)",
    }


def bench_plain_serving(torch, L, qi, seed, rate, seconds, lo, hi, pool=4096):
    """The same open-loop arrivals served one request at a time on the plain path:
    copy the state in, one sweep per gate (qcw_circuit), copy the result out.
    Device and pinned host buffers are allocated once per qubit count."""
    arr = qi.poisson_arrivals(seed, rate, seconds)
    inst = qi.batch(seed, pool, lo, hi)
    reqs = [(nq, torch.from_numpy(p).pin_memory(), *L.pack_circuit(c), len(c))
            for nq, p, c in inst]
    dev = {q: torch.empty(1 << q, dtype=torch.complex128, device="cuda") for q in range(lo, hi + 1)}
    out = {q: torch.empty(1 << q, dtype=torch.complex128).pin_memory() for q in range(lo, hi + 1)}

    def serve(nq, p, g, m, G):
        psi = dev[nq]
        psi.copy_(p, non_blocking=True)
        L.qcw_circuit(psi, nq, g, G, m, m.size)
        out[nq].copy_(psi, non_blocking=True)
        torch.cuda.current_stream().synchronize()

    for r in reqs[:64]:                                  # warm
        serve(*r)
    done_ns = np.zeros(arr.size, np.int64)
    t0 = time.monotonic_ns() + 20_000_000
    sched = t0 + (arr * 1e9).astype(np.int64)
    for i in range(arr.size):
        dt = (sched[i] - time.monotonic_ns()) / 1e9
        if dt > 0:
            time.sleep(dt)
        serve(*reqs[i % pool])
        done_ns[i] = time.monotonic_ns()
    lat = (done_ns - sched) / 1e6
    span = (done_ns.max() - sched.min()) / 1e9
    return {"rate_per_s": rate, "requests": int(arr.size),
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "solves_per_s": float(arr.size / span)}


def bench_serving_sweep(torch, L, qi, tt, seconds, rates=(2000, 8000, 12000, 16000, 24000),
                        plain_rates=(1000, 2000, 4000, 6000, 8000)):
    """Raise the offered rate until p99 diverges, for the continuous-batching server
    and for the plain one-request-at-a-time path.  A rate counts as sustained when
    nothing failed, at least 95% of the offered rate completed, and p99 stayed
    within 20x the p99 at the lowest rate."""
    def sweep(run, rs):
        rows, best, base = [], None, None
        for r in rs:
            d = run(r)
            rows.append({k: d[k] for k in ("rate_per_s", "p50_ms", "p99_ms", "solves_per_s")
                         if k in d} | ({"client_submit_us": d["client_submit_us"]}
                                       if "client_submit_us" in d else {}))
            base = base if base is not None else d["p99_ms"]
            ok = d.get("failed", 0) == 0 and d["solves_per_s"] >= 0.95 * r and \
                d["p99_ms"] <= 20 * base
            if not ok:
                break
            best = r
        return rows, best
    srv, srv_best = sweep(lambda r: bench_serving(L, qi, 3, r, seconds, 3, 9, tt), rates)
    pln, pln_best = sweep(lambda r: bench_plain_serving(torch, L, qi, 3, r, seconds, 3, 9),
                          plain_rates)
    return {"seconds_per_rate": seconds, "nq_range": [3, 9], "seed": 3,
            "server": srv, "plain": pln,
            "max_sustained_rate_server": srv_best, "max_sustained_rate_plain": pln_best,
            "criterion": "no failures, >= 95% of offered rate completed, p99 <= 20x the "
                         "lowest-rate p99; sweep stops at the first rate that misses",
            "client": "one Python thread submits (client_submit_us per request, including "
                      "the host-side fusion of the request's circuit) and one collects; above "
                      "~1/client_submit_us the client, not the server, sets the rate"}


def bench_serving_native(L, qi, tt, seconds, rates=(16000, 32000, 64000, 96000, 128000, 192000),
                         clients=2, pool=4096, seed=3, lo=3, hi=9):
    """Config 3 driven by the native open-loop load generator (serve_load, built
    beside the library): requests submitted from `clients` C++ threads at
    Poisson arrival times, results copied to host memory in submission order.
    Same request mix and server settings as bench_serving; latency from each
    request's scheduled arrival to its completion."""
    import subprocess
    import tempfile
    exe = os.path.join(ROOT, "paper_1101_1785_amd", "serve_load")
    if not os.path.exists(exe):
        return {"skipped": "serve_load not built"}
    inst = qi.batch(seed, pool, lo, hi)
    out = {"seconds_per_rate": seconds, "client_threads": clients, "nq_range": [lo, hi],
           "seed": seed, "request_pool": pool, "server": []}
    with tempfile.TemporaryDirectory() as d:
        pool_path = os.path.join(d, "pool.bin")
        with open(pool_path, "wb") as f:
            np.array([pool], dtype=np.int32).tofile(f)
            for nq, p, c in inst:
                g, m = L.pack_circuit(c)
                np.array([nq, len(g)], dtype=np.int32).tofile(f)
                np.array([m.size], dtype=np.int64).tofile(f)
                g.tofile(f)
                np.ascontiguousarray(m, dtype=np.complex128).tofile(f)
                np.ascontiguousarray(p, dtype=np.complex128).tofile(f)
        rec = np.dtype([("sched", "<i8"), ("done", "<i8"), ("status", "<i4")])
        for rate in rates:
            print(f"[bench] serving (native client): {rate}/s for {seconds}s", file=sys.stderr,
                  flush=True)
            arr = qi.poisson_arrivals(seed, rate, seconds)
            arr_path, res_path = os.path.join(d, "arr.bin"), os.path.join(d, "res.bin")
            with open(arr_path, "wb") as f:
                np.array([arr.size], dtype=np.int64).tofile(f)
                arr.astype(np.float64).tofile(f)
            r = subprocess.run([exe, pool_path, arr_path, res_path, str(1 << 30), "1024", str(hi),
                                tt or "-", str(clients)], capture_output=True, text=True,
                               timeout=seconds * 10 + 120)
            if r.returncode not in (0, 1) or not os.path.exists(res_path):
                out["server"].append({"rate_per_s": rate, "error": r.stderr[-300:]})
                break
            raw = np.fromfile(res_path, dtype=np.uint8)
            n, ticks, peak = np.frombuffer(raw[:24].tobytes(), dtype=np.int64)
            recs = np.frombuffer(raw[24:].tobytes(), dtype=rec)
            okm = recs["status"] == 0
            lat = (recs["done"][okm] - recs["sched"][okm]) / 1e6
            span = (recs["done"][okm].max() - recs["sched"].min()) / 1e9
            out["server"].append({
                "rate_per_s": rate, "requests": int(n), "failed": int((~okm).sum()),
                "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                "solves_per_s": float(okm.sum() / span), "ticks": int(ticks),
                "peak_active": int(peak)})
    return out


def bench_grover(torch, L, qi, tt, count=1024, n=6, seed=9):
    """Textbook Grover search (qcw_inputs.workloads) over n data qubits, at the
    optimal iteration count, for `count` random marked items in one batched
    launch; every result checked against the closed form."""
    from qcw_inputs import workloads as W
    k = W.grover_optimal_iterations(n)
    rng = np.random.default_rng([seed, 3])
    marked = rng.integers(0, 1 << n, count)
    cache = {}
    circs = []
    for m in marked:
        if int(m) not in cache:
            cache[int(m)] = W.grover(n, int(m), k)
        circs.append(cache[int(m)])
    nq = circs[0].nq
    psi0 = np.zeros(1 << nq, complex)
    psi0[0] = 1.0
    states = torch.from_numpy(np.tile(psi0, count)).to("cuda")
    b = L.Batch([(nq, c) for c in circs], states, tune_table=tt)
    b.run()
    torch.cuda.synchronize()
    flat = states.cpu().numpy().reshape(count, 1 << nq)
    a, o = W.grover_amplitudes(n, k)
    err = 0.0
    for i, m in enumerate(marked):
        ref = np.zeros(1 << nq, complex)
        ref[np.arange(1 << n) << (nq - n)] = o
        ref[int(m) << (nq - n)] = a
        err = max(err, float(np.max(np.abs(flat[i] - ref))))
    tm, _ = _time_batch(torch, b, 24)
    b.close()
    ms = tm["graph"]
    return {"data_qubits": n, "qubits": nq, "iterations": k, "gates_per_search": len(circs[0]),
            "searches": count, "us_per_launch": ms * 1e3, "searches_per_s": count / (ms * 1e-3),
            "success_probability": a * a, "max_abs_err_vs_closed_form": err,
            "launch": "graph", "eager_us_per_launch": tm["eager"] * 1e3,
            "graph_x8_us_per_execution": tm["graph_x8"] * 1e3}


def bench_shard(torch, L, qi, nq=32):
    """One GPU's kernel for gates on the top qubit of a 32-qubit state split over
    two GPUs (qcw_op_shard): its 2^31-amplitude half updated from itself and the
    partner's staged half.  Algorithmic traffic 48 B per local amplitude."""
    h = 1 << (nq - 1)
    free, _ = torch.cuda.mem_get_info()
    if free < 2 * 16 * h + (8 << 30):
        return {"skipped": "not enough device memory"}
    loc = torch.zeros(h, dtype=torch.complex128, device="cuda")
    rem = torch.zeros_like(loc)
    rng = np.random.default_rng(12)
    out = {"nq_total": nq, "amplitudes_per_gpu": h, "bytes_per_amplitude": 48}
    for k, t in ((1, (1,)), (2, (1, 17)), (3, (5, 1, 30))):
        U = qi.random_unitary(rng, 1 << k)
        L.qcw_op_shard(k, t, U, 0, loc, rem, nq)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            L.qcw_op_shard(k, t, U, 0, loc, rem, nq)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 5
        out[f"k{k}_targets"] = list(t)
        out[f"k{k}_ms"] = ms
        out[f"k{k}_gbs"] = 48 * h / (ms * 1e-3) / 1e9
    del loc, rem
    torch.cuda.empty_cache()
    return out


def bench_multiverse(torch, L, qi, nq, seed, n_p=16, eps=0.2, steps=20, noise="pauli", kernel=-1):
    """Multiverse density-matrix steps (Eq. rhoE4): channel of n_p single-hit and
    n_p double-hit paths (weights eps*p_s/n_p, p1=.95, p2=.05, p_keep=1-eps) whose
    hit operators are Pauli operators or (noise="rotation") random rotations
    exp(-i theta n.sigma/2), then one algorithm gate (H_1 or a CNOT of the GHZ
    chain) by conjugation, both in one call (qcw_channel_apply_gate: a CNOT is
    folded into the channel's pass when the compiled tiled kernel runs)."""
    rng = np.random.default_rng([seed, 7])
    P = [qi.X, qi.Y, qi.Z]

    def hit():
        return qi.random_rotation(rng) if noise == "rotation" else P[int(rng.integers(3))]
    terms = []
    for s, ps in ((1, 0.95), (2, 0.05)):
        for _ in range(n_p):
            qs = [int(x) + 1 for x in rng.choice(nq, s, replace=False)]
            terms.append((eps * ps / n_p, {q: hit() for q in qs}))
    ch = L.Channel(nq, 1 - eps, terms)
    ch.plan(kernel)
    psi0 = qi.basis_state(nq, 0)
    a = torch.from_numpy(np.outer(psi0, psi0.conj()).reshape(-1)).to("cuda")
    b2 = torch.empty_like(a)
    gates = [(qi.H, (1,))] + [(qi.CNOT, (1, t)) for t in range(2, nq + 1)]

    def step(i, x, y):
        # one call: a permutation gate (the CNOTs) is folded into the channel's
        # stores when the compiled tiled kernel runs; H takes a second pass
        U, t = gates[i % len(gates)]
        ch.apply_gate(x, y, U, t)

    for i in range(min(len(gates), steps)):  # compiles each gate's kernel before the timing
        step(i, a, b2)
    torch.cuda.synchronize()
    a.copy_(torch.from_numpy(np.outer(psi0, psi0.conj()).reshape(-1)))
    L.qcw_timing_reset()
    L.qcw_timing_enable(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    x, y = a, b2
    for i in range(steps):
        step(i, x, y)
        x, y = y, x
    e1.record()
    torch.cuda.synchronize()
    L.qcw_timing_enable(False)
    ms = e0.elapsed_time(e1) / steps
    n, cms = L.qcw_timing_read(L.QCW_KERNEL_CHANNEL)
    n_conj, conj_ms = L.qcw_timing_read(L.QCW_KERNEL_CONJ)
    ob = L.qcw_rho_observables(x, psi0=psi0)
    spectral = {}
    if nq <= 6:
        ev, S = L.qcw_rho_eigvals(x)
        rho0 = torch.from_numpy(np.outer(psi0, psi0.conj()).reshape(-1)).to("cuda")
        t0 = time.perf_counter()
        F = L.qcw_rho_fidelity(x, rho0)
        spectral = {"entropy_bits_after": S, "entropy_nats_after": S * float(np.log(2.0)),
                    "max_eigenvalue_after": float(ev[-1]),
                    "general_fidelity_after": F,
                    "fidelity_call_ms": (time.perf_counter() - t0) * 1e3}
    NN = 1 << (2 * nq)
    fl = ch.flops_per_element() * NN
    cavg = cms / max(n, 1)
    plan = ch.plan()
    kernel = ("gather" if plan["gather_kernel"] else
              "tiled, compiled for the channel" if plan["compiled_kernel"] else "tiled, generic")
    ch.close()
    return {"nq": nq, "paths": 2 * n_p, "noise": noise, "steps_per_s": 1e3 / ms, "ms_per_step": ms,
            "channel_ms": cavg, "channel_fp64_tflops": fl / (cavg * 1e-3) / 1e12,
            "channel_fp64_frac": fl / (cavg * 1e-3) / 1e12 / FP64_PEAK_TFLOPS,
            "channel_gbs_read_write_once": 32 * NN / (cavg * 1e-3) / 1e9,
            "channel_hbm_frac": 32 * NN / (cavg * 1e-3) / 1e9 / HBM_PEAK_GBS,
            # the binding roof: the longer of the flop time and the byte time
            "channel_bound": "fp64" if fl / FP64_PEAK_TFLOPS / 1e12 > 32 * NN / HBM_PEAK_GBS / 1e9
                             else "hbm",
            "channel_roof_frac": max(fl / FP64_PEAK_TFLOPS / 1e12, 32 * NN / HBM_PEAK_GBS / 1e9)
                                 / (cavg * 1e-3),
            "channel_kernel": kernel, "channel_grid": plan["grid"], "channel_vgprs": plan["vgprs"],
            "channel_flops_per_element": ch_flops if (ch_flops := fl // NN) else None,
            "gate_passes": n_conj, "gate_pass_ms": conj_ms / max(n_conj, 1) if n_conj else None,
            "steps_with_gate_in_channel_pass": steps - n_conj if n_conj <= steps else None,
            "trace_after": ob["trace"].real, "purity_after": ob["purity"],
            "fidelity_after": ob["fidelity"], **spectral}


def bench_multiverse_obs(torch, L, qi, nq, seed, steps=10, n_p=16, eps=0.2):
    """Multiverse steps with the observables of §5 (trace, purity, fidelity
    against |0..0>, polarisations) after every step.  qcw_channel_step_obs sums them in the
    channel's own pass (asynchronously, into device memory), against the
    step followed by qcw_rho_observables (a further pass over rho, and a
    synchronisation) every step.  The same channel and GHZ-chain gates as
    the multiverse sections."""
    rng = np.random.default_rng([seed, 7])
    P = [qi.X, qi.Y, qi.Z]
    terms = []
    for s_, ps in ((1, 0.95), (2, 0.05)):
        for _ in range(n_p):
            qs = [int(x) + 1 for x in rng.choice(nq, s_, replace=False)]
            terms.append((eps * ps / n_p, {q: P[int(rng.integers(3))] for q in qs}))
    ch = L.Channel(nq, 1 - eps, terms)
    psi0 = qi.basis_state(nq, 0)
    psi0_d = torch.from_numpy(psi0).to("cuda")
    rho0 = torch.from_numpy(np.outer(psi0, psi0.conj()).reshape(-1)).to("cuda")
    a, b = rho0.clone(), torch.empty_like(rho0)
    obs = torch.empty(4 + 3 * nq, dtype=torch.float64, device="cuda")
    gates = [(qi.H, (1,))] + [(qi.CNOT, (1, t)) for t in range(2, nq + 1)]
    hist = np.empty((steps, 4 + 3 * nq))
    for i in range(min(len(gates), steps)):  # compile both kernels of each gate before the timing
        U, t = gates[i]
        ch.step_obs(a, b, obs, U, t, psi0=psi0_d)
        ch.apply_gate(a, b, U, t)
    torch.cuda.synchronize()

    def run(fused):
        x, y = a, b
        x.copy_(rho0)
        torch.cuda.synchronize()
        L.qcw_timing_reset()
        L.qcw_timing_enable(True)
        t0 = time.perf_counter()
        for i in range(steps):
            U, t = gates[i % len(gates)]
            if fused:
                ch.step_obs(x, y, obs, U, t, psi0=psi0_d)
                hist[i] = obs.cpu().numpy()  # read back each step, as a driver loop would
            else:
                ch.apply_gate(x, y, U, t)
                o = L.qcw_rho_observables(y, psi0=psi0)
                hist[i] = [o["trace"].real, o["trace"].imag, o["purity"], o["fidelity"],
                           *o["polarization"].reshape(-1)]
            x, y = y, x
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps * 1e3
        L.qcw_timing_enable(False)
        n, cms = L.qcw_timing_read(L.QCW_KERNEL_CHANNEL)
        return dt, hist.copy(), cms / max(n, 1)

    ms_f, h_f, ch_f = run(True)
    ms_s, h_s, ch_s = run(False)
    ch.close()
    return {"nq": nq, "steps": steps, "ms_per_step_observed_in_pass": ms_f,
            "ms_per_step_with_observables_call": ms_s,
            "channel_ms_observing": ch_f, "channel_ms_plain": ch_s,
            "speedup": ms_s / ms_f,
            "max_abs_diff_observables": float(np.max(np.abs(h_f - h_s))),
            "fidelity_after": float(h_f[-1, 3]), "purity_after": float(h_f[-1, 2]),
            "what": "host clock per step including reading the observables back every step"}


def bench_multiverse_low_gates(torch, L, qi, nq, seed, reps=20, n_p=16, eps=0.2):
    """Multiverse steps whose gate mixes basis states on the last qubits (H,
    a random two-qubit and a random three-qubit unitary, the compiled kernel
    applying it to each tile's outputs in LDS), in one call
    (qcw_channel_apply_gate) against the channel followed by
    qcw_rho_conjugate; both must give the same bits.  The same channel as
    the multiverse sections; rho is random."""
    rng = np.random.default_rng([seed, 7])
    P = [qi.X, qi.Y, qi.Z]
    terms = []
    for s_, ps in ((1, 0.95), (2, 0.05)):
        for _ in range(n_p):
            qs = [int(x) + 1 for x in rng.choice(nq, s_, replace=False)]
            terms.append((eps * ps / n_p, {q: P[int(rng.integers(3))] for q in qs}))
    ch = L.Channel(nq, 1 - eps, terms)
    NN = 1 << (2 * nq)
    g = torch.Generator(device="cuda").manual_seed(seed)
    a = torch.complex(torch.randn(NN, dtype=torch.float64, device="cuda", generator=g),
                      torch.randn(NN, dtype=torch.float64, device="cuda", generator=g))
    b, c = torch.empty_like(a), torch.empty_like(a)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)

    def timed(fn):
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    out = {"nq": nq, "reps": reps}
    for name, U, t in (("H_on_qubit_nq", qi.H, (nq,)),
                       ("u2_on_last_qubits", qi.random_unitary(rng, 4), (nq, nq - 3)),
                       ("u3_on_last_qubits", qi.random_unitary(rng, 8), (nq - 1, nq - 3, nq))):
        print(f"[bench] multiverse nq={nq}: {name} in the channel's pass", file=sys.stderr, flush=True)
        ch.apply_gate(a, b, U, t)  # compiles the kernel for these targets
        ch.apply(a, c)
        L.qcw_rho_conjugate(len(t), t, U, c)
        torch.cuda.synchronize()
        one = timed(lambda: ch.apply_gate(a, b, U, t))
        two = timed(lambda: (ch.apply(a, c), L.qcw_rho_conjugate(len(t), t, U, c)))
        out[name] = {"ms_one_pass": one, "ms_channel_then_conjugation": two,
                     "bit_equal": bool(torch.equal(b, c))}
    out["channel_alone_ms"] = timed(lambda: ch.apply(a, c))
    ch.close()
    return out


def bench_config0(torch, L, qi, reps=10000):
    """Config 0: the paper's first worked-example size (nq = 3), one 12-gate
    random circuit (seed 0) on the plain path, one solve at a time: latency of
    single solves (host clock around a solve and its synchronisation; p50/p99
    over `reps`), throughput of back-to-back solves, and the error of one solve
    against the oracle."""
    import oracle
    nq, G = 3, 12
    psi0 = qi.state(0, nq)
    c = qi.circuit(0, nq, G)
    g, m = L.pack_circuit(c)
    psi = torch.from_numpy(psi0).to("cuda")
    L.qcw_circuit(psi, nq, g, len(c), m, m.size)
    torch.cuda.synchronize()
    ref = oracle.circuit(c, psi0)
    err = float(np.linalg.norm(psi.cpu().numpy() - ref) / np.linalg.norm(ref))
    lat = np.empty(reps)
    for i in range(reps):
        t0 = time.perf_counter()
        L.qcw_circuit(psi, nq, g, len(c), m, m.size)
        torch.cuda.synchronize()
        lat[i] = time.perf_counter() - t0
    t0 = time.perf_counter()
    for _ in range(reps):
        L.qcw_circuit(psi, nq, g, len(c), m, m.size)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"nq": nq, "gates": G, "seed": 0, "solves": reps,
            "p50_us": float(np.percentile(lat, 50) * 1e6),
            "p99_us": float(np.percentile(lat, 99) * 1e6),
            "back_to_back_solves_per_s": reps / dt,
            "rel_err_vs_oracle": err}


def bench_sweeps(torch, L, qi, sizes=(26, 28, 30, 31), reps=5):
    """Config 1 as single sweeps: one gate per launch, k = 1, 2, 3 with targets
    on the lowest qubits, the highest, or both ends, at several sizes; GB/s
    (32 B per amplitude) against the 8 TB/s peak and against a plain copy
    kernel measured here (torch copy_ of 16 GiB).  Also OmegaALL (H on every
    qubit) at the largest size, as fused passes and as one sweep per qubit."""
    print("[bench] sweeps: copy kernel", file=sys.stderr, flush=True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    a = torch.zeros(1 << 30, dtype=torch.complex128, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(3):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    copy_gbs = 3 * 2 * a.numel() * 16 / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    rng = np.random.default_rng(1)
    rows = []
    omega = None
    for nq in sizes:
        print(f"[bench] sweeps: nq={nq}", file=sys.stderr, flush=True)
        N = 1 << nq
        psi = torch.randn(N, dtype=torch.complex128, device="cuda")
        for k in (1, 2, 3):
            classes = (("lowest", tuple(range(nq, nq - k, -1))),
                       ("highest", tuple(range(1, k + 1))),
                       ("mixed", ((nq // 2,), (1, nq), (1, nq // 2, nq))[k - 1]))
            for cls, targets in classes:
                U = qi.random_unitary(rng, 1 << k)
                L.qcw_opk(k, targets, U, psi)
                torch.cuda.synchronize()
                e0.record()
                for _ in range(reps):
                    L.qcw_opk(k, targets, U, psi)
                e1.record()
                torch.cuda.synchronize()
                ms = e0.elapsed_time(e1) / reps
                gbs = 32 * N / (ms * 1e-3) / 1e9
                rows.append({"nq": nq, "k": k, "targets": cls, "qubits": list(targets),
                             "ms": ms, "GB/s": gbs, "frac_of_8TBs": gbs / HBM_PEAK_GBS,
                             "frac_of_copy": gbs / copy_gbs})
        if nq == sizes[-1]:
            L.qcw_omega_all(qi.H, psi)
            torch.cuda.synchronize()
            e0.record()
            L.qcw_omega_all(qi.H, psi)
            e1.record()
            torch.cuda.synchronize()
            fused_ms = e0.elapsed_time(e1)
            e0.record()
            for q in range(1, nq + 1):
                L.qcw_op1(qi.H, q, psi)
            e1.record()
            torch.cuda.synchronize()
            omega = {"nq": nq, "fused_passes_ms": fused_ms,
                     "one_sweep_per_qubit_ms": e0.elapsed_time(e1)}
        del psi
        torch.cuda.empty_cache()
    return {"copy_kernel_GB/s": copy_gbs, "rows": rows, "omega_all_H": omega}


def bench_plain_small(torch, L, qi, nq, seed, reps=2000):
    """Literal paper size: one nq-qubit state, one 4*nq-gate circuit per solve."""
    psi = torch.from_numpy(qi.state(seed, nq)).to("cuda")
    c = qi.circuit(seed, nq, 4 * nq)
    g, m = L.pack_circuit(c)
    L.qcw_circuit(psi, nq, g, len(c), m, m.size)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        L.qcw_circuit(psi, nq, g, len(c), m, m.size)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"nq": nq, "gates": len(c), "plain_solves_per_s": reps / dt,
            "us_per_solve": dt / reps * 1e6}


def _diff_stats(torch, x, y, chunk=1 << 26):
    """Relative 2-norm difference, max |x - y| over |y|, and bitwise equality of
    two device vectors, in chunks (temporaries of 1 GiB)."""
    num = den = mx = 0.0
    equal = True
    for i in range(0, x.numel(), chunk):
        xs, ys = x[i:i + chunk], y[i:i + chunk]
        d = xs - ys
        num += torch.linalg.vector_norm(d).item() ** 2
        den += torch.linalg.vector_norm(ys).item() ** 2
        mx = max(mx, d.abs().max().item())
        equal = equal and torch.equal(xs, ys)
        del d
    den = den ** 0.5
    return {"rel_err_2norm": (num ** 0.5) / den, "max_abs_err_over_norm": mx / den,
            "bitwise_equal": equal}


def compare_paths(torch, L, psi, psi_host, nq, gates, mats, G, a, stream):
    """After the timed region, from the same input in separate buffers: one
    solve of the timed plan, one plain solve (one sweep per gate) and one
    list-order fused solve.  Returns the comparison solves/s and the timed
    plan's error against the plain path (the list-order passes must equal the
    plain path bit for bit)."""
    def once(fn):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        return 1.0 / (time.perf_counter() - t1)

    src = torch.from_numpy(psi_host).to("cuda")
    psi.copy_(src)
    once(lambda: L.qcw_circuit_fused_ex(psi, nq, gates, G, mats, mats.size, a.tile_bits, 0, 0,
                                        a.plan, stream))
    plain = src.clone()
    plain_rate = once(lambda: L.qcw_circuit(plain, nq, gates, G, mats, mats.size, stream))
    plan_err = _diff_stats(torch, psi, plain)
    lo_rate = once(lambda: L.qcw_circuit_fused_ex(src, nq, gates, G, mats, mats.size,
                                                  a.tile_bits, 0, 0, 0, stream))
    lo = _diff_stats(torch, src, plain)
    del src, plain
    torch.cuda.empty_cache()
    G64 = max(1.0, G / 64)
    other = {
        "plain_one_sweep_per_gate_solves_per_s": plain_rate,
        "fused_list_order_bit_exact_solves_per_s": lo_rate,
        "fused_list_order_passes": L.qcw_fused_pass_count(nq, gates, G, a.tile_bits, 0, 0),
    }
    checks = {
        "timed_plan_vs_plain": {**{k: v for k, v in plan_err.items() if k != "bitwise_equal"},
                                "tolerance_2norm": 1e-12 * G64,
                                "what": "one solve of the timed plan against one plain solve "
                                        "(one sweep per gate) of the same input, "
                                        "the whole 2^nq-amplitude state"},
        "list_order_equals_plain_bitwise": lo["bitwise_equal"],
    }
    return other, checks


def oracle_check(torch, L, qi, nq, a, seed=1):
    """The timed configuration (same plan flags and tiles) on a state the oracle
    finishes in under a minute on the host: one 4*nq-gate solve against the
    oracle's circuit, element by element."""
    import oracle
    G = 4 * nq
    print(f"[bench] oracle check of the timed plan at nq={nq}", file=sys.stderr, flush=True)
    psi0 = qi.state(seed, nq)
    c = qi.circuit(seed, nq, G)
    g, m = L.pack_circuit(c)
    x = torch.from_numpy(psi0).to("cuda")
    L.qcw_circuit_fused_ex(x, nq, g, G, m, m.size, a.tile_bits, 0, 0, a.plan)
    torch.cuda.synchronize()
    got = x.cpu().numpy()
    del x
    torch.cuda.empty_cache()
    t0 = time.perf_counter()
    ref = oracle.circuit(c, psi0)
    dt = time.perf_counter() - t0
    nr = np.linalg.norm(ref)
    return {"nq": nq, "gates": G, "seed": seed,
            "passes": L.qcw_fused_pass_count(nq, g, G, a.tile_bits, 0, a.plan),
            "rel_err_2norm": float(np.linalg.norm(got - ref) / nr),
            "max_abs_err_over_norm": float(np.max(np.abs(got - ref)) / nr),
            "tolerance_2norm": 1e-12 * max(1.0, G / 64), "tolerance_elementwise": 1e-12,
            "oracle_s": dt, "oracle_threads": oracle.threads()}


def _executed_flops(L, circ, gates, mats, a):
    """FP64 flops the fused passes execute per launch (average over the plan's
    passes), from the device tables of the plan: per amplitude 8m - 2 for a
    gate in the direct form, 6m + 1 in the three-product form."""
    tb = L.qcw_debug_fused_tables(circ.nq, gates, len(circ), mats, a.tile_bits, 0, a.plan)
    N = 1 << circ.nq
    tot = sum(N * ((6 * (1 << g["k"]) + 1) if g["m3"] else (8 * (1 << g["k"]) - 2))
              for g in tb["gates"])
    return tot / max(1, len(tb["passes"]))


def bench_eigen(torch, L, nq, count=4096, seed=8, reps=5, check=64):
    """Batched eigenvalues with entropies, and batched fidelities, of `count`
    density matrices of nq qubits (ranks 1, 2, 3 and full in turn), one
    persistent launch each (the observables the paper follows per step, §5);
    errors against numpy's Hermitian solver on a sample."""
    rng = np.random.default_rng([seed, nq])
    n = 1 << nq
    ranks = [1, 2, 3, n]
    rhos = np.empty((count, n, n), np.complex128)
    for i in range(count):
        r = min(ranks[i % 4], n)
        A = rng.normal(size=(n, r)) + 1j * rng.normal(size=(n, r))
        R = A @ A.conj().T
        rhos[i] = R / np.trace(R).real
    d = torch.from_numpy(rhos.reshape(-1)).to("cuda")
    eig = torch.empty((count, n), dtype=torch.float64, device="cuda")
    ent = torch.empty(count, dtype=torch.float64, device="cuda")
    fid = torch.empty(count, dtype=torch.float64, device="cuda")
    psi0 = np.zeros(n, complex)
    psi0[0] = 1
    ref0 = torch.from_numpy(np.outer(psi0, psi0).reshape(-1)).to("cuda")
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_eig = timed(lambda: L.qcw_rho_eigvals_batch(d, nq, count, eig=eig, entropy=ent))
    ms_fid_pair = timed(lambda: L.qcw_rho_fidelity_batch(d, d, nq, count, out=fid))
    ms_fid_pure = timed(lambda: L.qcw_rho_fidelity_batch(d, ref0, nq, count, rho0_stride=0,
                                                          out=fid))
    ev = eig.cpu().numpy()
    S = ent.cpu().numpy()
    F = fid.cpu().numpy()
    sub = range(0, count, max(1, count // check))
    err_ev = max(float(np.max(np.abs(ev[i] - np.linalg.eigvalsh(rhos[i])))) for i in sub)
    err_S = 0.0
    for i in sub:
        lam = np.linalg.eigvalsh(rhos[i])
        lam = lam[lam > 1e-300]
        err_S = max(err_S, abs(S[i] + float(np.sum(lam * np.log2(lam)))))
    err_F = max(abs(F[i] - np.sqrt(rhos[i][0, 0].real)) for i in sub)
    del d, eig, ent, fid
    torch.cuda.empty_cache()
    return {"nq": nq, "matrices": count, "ranks": "1, 2, 3, full in turn",
            "eig_ms": ms_eig, "eig_matrices_per_s": count / (ms_eig * 1e-3),
            "fidelity_pairs_ms": ms_fid_pair, "fidelity_pure_reference_ms": ms_fid_pure,
            "fidelity_pure_reference_per_s": count / (ms_fid_pure * 1e-3),
            "max_abs_err_eigenvalues_vs_lapack": err_ev, "max_abs_err_entropy_bits": err_S,
            "max_abs_err_fidelity_vs_closed_form": float(err_F), "checked_matrices": len(sub)}


def key_figures(extra, checks, cpu):
    """A compact copy of the figures of every configuration, kept with the
    workload description so that they survive in short records."""
    def pick(sec, *keys):
        d = extra.get(sec) or {}
        return {k: d[k] for k in keys if k in d} or None
    k = {
        "config0_plain_nq3": pick("config0_plain_nq3", "p50_us", "p99_us",
                                  "back_to_back_solves_per_s", "rel_err_vs_oracle"),
        "config2_batched_4096_nq3_7": pick("batched_config2", "graph_us", "eager_us",
                                           "graph_x8_us_per_execution",
                                           "batched_solves_per_s", "plain_solves_per_s",
                                           "batched_over_plain", "max_rel_err_vs_oracle",
                                           "fp64_frac"),
        "config3_served_poisson": pick("serving_config3", "rate_per_s", "seconds", "requests",
                                       "failed", "p50_ms", "p99_ms", "solves_per_s",
                                       "peak_active"),
        "config4_batched_4096_nq9": pick("batched_config4", "graph_us", "eager_us",
                                         "graph_x8_us_per_execution",
                                         "batched_solves_per_s", "plain_solves_per_s",
                                         "batched_over_plain", "max_rel_err_vs_oracle",
                                         "fp64_frac"),
        "eigen_batch_nq5": pick("eigen_batch_nq5", "eig_matrices_per_s",
                                "max_abs_err_eigenvalues_vs_lapack"),
        "channel_nq13": pick("multiverse_nq13", "channel_ms", "channel_bound",
                             "channel_roof_frac", "channel_gbs_read_write_once"),
        "timed_plan_vs_plain_rel_err": (checks.get("timed_plan_vs_plain") or {}).get(
            "rel_err_2norm"),
        "timed_plan_vs_oracle_rel_err": (checks.get("oracle_check") or {}).get("rel_err_2norm"),
        "cpu_oracle_solves_per_s": (cpu or {}).get("value"),
    }
    return {a: b for a, b in k.items() if b is not None}


def counters_run(torch, L, qi):
    """One launch of each kernel family at a known size, for hardware counters."""
    nq = 28
    N = 1 << nq
    src = torch.zeros(1 << 27, dtype=torch.complex128, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)                                   # copy: 2 GiB read + 2 GiB written
    torch.cuda.synchronize()
    del src, dst
    psi = torch.from_numpy(qi.state(1, nq)).to("cuda")
    rng = np.random.default_rng(0)
    for k, t in ((1, (14,)), (2, (3, 20)), (3, (10, 4, 25)), (3, (nq, nq - 1, nq - 2))):
        L.qcw_opk(k, t, qi.random_unitary(rng, 1 << k), psi)
    c = qi.circuit(1, nq, 4 * nq)
    g, m = L.pack_circuit(c)
    L.qcw_circuit_fused_ex(psi, nq, g, len(c), m, m.size, 0, 0, 0, 7)
    torch.cuda.synchronize()
    print(json.dumps({"counters_run": {
        "copy_bytes_read": 16 << 27, "copy_bytes_written": 16 << 27,
        "sweep_launches": 4, "sweep_bytes_per_launch": 32 * N,
        "fused_passes": L.qcw_fused_pass_count(nq, g, len(c), 0, 0, 7),
        "fused_bytes_per_pass": 32 * N, "nq": nq}}), flush=True)


def extra_sections(torch, L, qi, a):
    """The sections reported beside the headline, in report order (name -> run)."""
    tt = a.tune_table if a.tune_table and os.path.exists(a.tune_table) else None
    secs = {
        "batched_config2": lambda: bench_batched(torch, L, qi, 2, 4096, 3, 7, tt,
                                                 label="4096 x nq 3..7"),
        "batched_config4": lambda: bench_batched(torch, L, qi, 4, 4096, 9, 9, tt,
                                                 label="4096 x nq 9"),
        "config0_plain_nq3": lambda: bench_config0(torch, L, qi),
        "sweeps_config1": lambda: bench_sweeps(torch, L, qi),
        "plain_nq9": lambda: bench_plain_small(torch, L, qi, 9, 1),
        "grover_n6": lambda: bench_grover(torch, L, qi, tt),
        "shard_nq32": lambda: bench_shard(torch, L, qi),
        "multiverse_nq12": lambda: bench_multiverse(torch, L, qi, 12, 5),
        "multiverse_nq13": lambda: bench_multiverse(torch, L, qi, 13, 5, steps=10),
        "multiverse_nq13_generic": lambda: bench_multiverse(torch, L, qi, 13, 5, steps=10, kernel=2),
        "multiverse_nq14": lambda: bench_multiverse(torch, L, qi, 14, 5, steps=5),
        "multiverse_nq13_observed": lambda: bench_multiverse_obs(torch, L, qi, 13, 5),
        "multiverse_nq13_last_qubit_gates": lambda: bench_multiverse_low_gates(torch, L, qi, 13, 5),
        "multiverse_nq15": lambda: bench_multiverse(torch, L, qi, 15, 5, steps=3),
        "eigen_batch_nq5": lambda: bench_eigen(torch, L, 5),
        "eigen_batch_nq6": lambda: bench_eigen(torch, L, 6),
        "multiverse_nq5": lambda: bench_multiverse(torch, L, qi, 5, 5, steps=200),
        "multiverse_nq5_rotation_noise": lambda: bench_multiverse(torch, L, qi, 5, 6, steps=200,
                                                                  noise="rotation"),
        "multiverse_nq10_rotation_noise": lambda: bench_multiverse(torch, L, qi, 10, 6, steps=20,
                                                                   noise="rotation"),
        "serving_config3": lambda: bench_serving(L, qi, 3, a.serve_rate, a.serve_seconds, 3, 9,
                                                 tt),
    }
    if a.serve_sweep_seconds > 0:
        secs["serving_rate_sweep"] = lambda: bench_serving_sweep(torch, L, qi, tt,
                                                                 a.serve_sweep_seconds)
        secs["serving_native_sweep"] = lambda: bench_serving_native(L, qi, tt,
                                                                    a.serve_sweep_seconds)
    return secs


def main():
    a = _args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    from paper_1101_1785_amd import _lib as L
    import qcw_inputs as qi

    if a.counters:
        counters_run(torch, L, qi)
        return
    if a.section:
        # One section alone (for profiling it): its JSON object, not the
        # headline record.
        secs = extra_sections(torch, L, qi, a)
        if a.section not in secs:
            print(f"unknown section {a.section!r}; one of: {', '.join(secs)}", file=sys.stderr)
            sys.exit(2)
        print(json.dumps({a.section: secs[a.section]()}))
        return

    nq = a.nq
    G = a.gates or 4 * nq
    N = 1 << nq
    print(f"[bench] generating nq={nq} state and a {G}-gate circuit (seed {a.seed})",
          file=sys.stderr, flush=True)
    psi_host = qi.state(a.seed, nq)
    circ = qi.circuit(a.seed, nq, G)
    gates, mats = L.pack_circuit(circ)
    psi = torch.from_numpy(psi_host).to("cuda")
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()

    def solve():
        if a.path == "fused":
            L.qcw_circuit_fused_ex(psi, nq, gates, G, mats, mats.size, a.tile_bits, 0, 0, a.plan,
                                   stream)
        else:
            L.qcw_circuit(psi, nq, gates, G, mats, mats.size, stream)

    print(f"[bench] warmup {a.warmup}", file=sys.stderr, flush=True)
    for _ in range(a.warmup):
        solve()
    torch.cuda.synchronize()

    print(f"[bench] timing {a.steps} steps ({a.path})", file=sys.stderr, flush=True)
    L.qcw_timing_reset()
    L.qcw_timing_enable(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(a.steps):
        solve()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    L.qcw_timing_enable(False)
    ms_total = e0.elapsed_time(e1)
    ms_step = ms_total / a.steps

    bytes_per_launch = 32.0 * N
    per_k = {}
    if a.path == "fused":
        launches, kms = L.qcw_timing_read(L.QCW_KERNEL_FUSED)
        npass = L.qcw_fused_pass_count(nq, gates, G, a.tile_bits, 0, a.plan)
        kernel = "qcw::fused_pass_kernel (one pass = a run of gates over the state in LDS tiles)"
        unit_note = f"one pass over the state; {npass} passes per {G}-gate solve"
    else:
        launches, kms = 0, 0.0
        for k, fam in ((1, L.QCW_KERNEL_SWEEP1), (2, L.QCW_KERNEL_SWEEP2), (3, L.QCW_KERNEL_SWEEP3)):
            n, ms = L.qcw_timing_read(fam)
            launches += n
            kms += ms
            if n:
                per_k[f"k{k}"] = {"launches": n, "avg_ms": ms / n,
                                  "GB/s": 32.0 * N * n / (ms * 1e-3) / 1e9}
        npass = G
        kernel = "qcw::sweep_kernel (k=1,2,3)"
        unit_note = "one gate over the state"
    avg_ms = kms / max(launches, 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    # the circuit's algorithmic flops (its gates as listed, 8m - 2 per amplitude
    # per gate), spread over the launches
    flops_per_launch = _flops_per_solve(circ) / max(npass, 1)
    fp64_tflops = flops_per_launch / (avg_ms * 1e-3) / 1e12
    # the binding roof: the larger of the two minimum times per launch
    t_hbm = bytes_per_launch / (HBM_PEAK_GBS * 1e9)
    t_fp64 = flops_per_launch / (FP64_PEAK_TFLOPS * 1e12)
    executed = _executed_flops(L, circ, gates, mats, a) if a.path == "fused" else None
    norm = torch.linalg.vector_norm(psi).item()

    # the other paths, and the error of the timed plan, outside the timed region
    other, checks = {}, {"final_norm": norm, "wall_s": wall}
    if a.path == "fused" and not a.no_compare:
        print("[bench] comparison solves and error checks", file=sys.stderr, flush=True)
        other, chk = compare_paths(torch, L, psi, psi_host, nq, gates, mats, G, a, stream)
        checks.update(chk)
    del psi
    torch.cuda.empty_cache()
    if a.path == "fused" and not a.no_compare and a.oracle_check_nq > 0:
        checks["oracle_check"] = oracle_check(torch, L, qi, a.oracle_check_nq, a)

    cpu = None
    if not a.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline(circ, psi_host, a.cpu_sample_log2)
    del psi_host

    extra = {}
    if not a.skip_extra:
        for name, fn in extra_sections(torch, L, qi, a).items():
            print(f"[bench] section {name}", file=sys.stderr, flush=True)
            extra[name] = fn()

    hbm = {"achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": achieved / HBM_PEAK_GBS,
           "traffic": _traffic("fused" if a.path == "fused" else "sweep", nq),
           "algorithmic_bytes_per_launch": bytes_per_launch, "min_ms_per_launch": t_hbm * 1e3}
    fp64 = {"achieved": fp64_tflops, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": fp64_tflops / FP64_PEAK_TFLOPS,
            "algorithmic_flops_per_launch": flops_per_launch, "min_ms_per_launch": t_fp64 * 1e3}
    if t_fp64 > t_hbm:
        roof = {"bound": "alu", **fp64, "traffic": hbm["traffic"],
                "why": "the circuit's FP64 flops per pass need more time at 78.6 TFLOP/s than "
                       "its 32 B per amplitude at 8 TB/s (FP64 vector peak; the FP64 matrix "
                       "cores share that throughput)"}
    else:
        roof = {"bound": "hbm", **hbm}
    roofline = {
        **roof,
        "hbm": hbm, "fp64": fp64,
        "kernel": kernel, "unit_of_work": unit_note, "launches": launches,
        "avg_launch_ms": avg_ms, "per_k": per_k or None,
        "executed_flops_per_launch": executed,
    }
    key = key_figures(extra, checks, cpu)
    out = {
        "metric": METRIC,
        "value": a.steps / (ms_total * 1e-3),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"single {nq}-qubit complex FP64 state ({16 * N / 2**30:.0f} GiB) "
                        f"resident in HBM; a solve = one {G}-gate random circuit "
                        f"(k=1/2/3 at .50/.35/.15, random ordered targets, random unitaries); "
                        f"seed {a.seed}",
            "nq": nq, "gates": G, "seed": a.seed,
            "path": "qcw_circuit_fused_ex" if a.path == "fused" else "qcw_circuit",
            "plan": (("|".join(n for b, n in ((1, "QCW_PLAN_COMMUTE"), (2, "QCW_PLAN_FUSE"),
                                               (4, "QCW_PLAN_3M")) if a.plan & b)
                      or "list order (bit-exact)") if a.path == "fused" else None),
            "passes_per_solve": npass,
            **other,
            "key_figures": key,
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "checks": checks,
        **extra,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
