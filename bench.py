#!/usr/bin/env python3
"""Benchmark of the gate-sweep hot path on one MI355X.

A step is one solve: a random circuit of G = 4*nq dense gates (k = 1, 2, 3
with probabilities .50/.35/.15, random ordered targets, random unitaries)
applied in place to one nq-qubit complex FP64 state that is already resident
in HBM.  The default workload is the largest single state the 64 GB device
budget admits, nq = 31 (2^31 amplitudes, 32 GiB), seed 1.

Prints ONE JSON line with the throughput (solves/s), the roofline of the
dominant kernel (the one-gate sweep; algorithmic bytes 32 * 2^nq per launch,
measured with HIP events recorded by the library on the launch stream) and
the CPU oracle timed on a bounded sample of the same solve.
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
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-sample-log2", type=int, default=26,
                   help="contiguous outputs per gate timed on the CPU oracle")
    return p.parse_args()


def _source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1101_1785_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h", ".cpp")):
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def _traffic(kernel: str, nq: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None
    when the kernels changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        d = json.load(open(path))
    except (OSError, ValueError):
        return None
    e = d.get(kernel)
    if not e or e.get("source_hash") != _source_hash() or e.get("nq") != nq:
        return None
    return e.get("bytes_per_launch")


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
    return {"value": 1.0 / per_solve, "unit": "solves/s", "cores": oracle.threads(),
            "kind": "oracle",
            "sample": f"{S} contiguous outputs (2^{sample_log2}) of each of the {len(circ)} gates "
                      f"at nq={nq}, {dt:.2f} s of CPU work, scaled by 2^{nq}/{S} to one solve"}


def main():
    a = _args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    from paper_1101_1785_amd import _lib as L
    import qcw_inputs as qi

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

    print(f"[bench] warmup {a.warmup}", file=sys.stderr, flush=True)
    for _ in range(a.warmup):
        L.qcw_circuit(psi, nq, gates, G, mats, mats.size, stream)
    torch.cuda.synchronize()

    print(f"[bench] timing {a.steps} steps", file=sys.stderr, flush=True)
    L.qcw_timing_reset()
    L.qcw_timing_enable(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(a.steps):
        L.qcw_circuit(psi, nq, gates, G, mats, mats.size, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    L.qcw_timing_enable(False)
    ms_total = e0.elapsed_time(e1)
    ms_step = ms_total / a.steps

    launches, kms = 0, 0.0
    per_k = {}
    for k, fam in ((1, L.QCW_KERNEL_SWEEP1), (2, L.QCW_KERNEL_SWEEP2), (3, L.QCW_KERNEL_SWEEP3)):
        n, ms = L.qcw_timing_read(fam)
        launches += n
        kms += ms
        if n:
            per_k[f"k{k}"] = {"launches": n, "avg_ms": ms / n,
                              "GB/s": 32.0 * N * n / (ms * 1e-3) / 1e9}
    bytes_per_launch = 32.0 * N
    avg_ms = kms / max(launches, 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    norm = torch.linalg.vector_norm(psi).item()

    cpu = None
    if not a.no_cpu_baseline:
        print("[bench] timing the CPU oracle on a sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline(circ, psi_host, a.cpu_sample_log2)

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
            "workload": f"plain path, one {nq}-qubit complex FP64 state ({16 * N / 2**30:.0f} GiB) "
                        f"resident in HBM; a solve = one {G}-gate random circuit "
                        f"(k=1/2/3 at .50/.35/.15, random ordered targets, random unitaries), "
                        f"one in-place sweep per gate; seed {a.seed}",
            "nq": nq, "gates": G, "seed": a.seed, "path": "qcw_circuit (one sweep per gate)",
        },
        "roofline": {
            "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": _traffic("sweep", nq),
            "kernel": "qcw::sweep_kernel (k=1,2,3)", "launches": launches,
            "avg_launch_ms": avg_ms, "algorithmic_bytes_per_launch": bytes_per_launch,
            "per_k": per_k,
        },
        "cpu_baseline": cpu,
        "checks": {"final_norm": norm, "wall_s": wall},
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
