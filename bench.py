"""Throughput benchmark of the sketching estimators on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload torus] [--m 1024]
                    [--samples S] [--batch B] [--no-cpu-baseline]

A step is one full pass of the estimator over one batch of synthetic input
already resident in HBM: hash generation, the sketching pass over every tensor,
the DFT/product/sum combine and the per-network mean/variance, for every
sample of every network in the batch.  Prints one JSON line.

Workloads:
  torus    4 x 4 periodic lattice of order-4 tensors, bond 16, FP32 U[0,1),
           cyclic estimator; a batch of B independent tori (B = 256: 1 GiB).
  triangle three 64 x 64 FP64 N(0,1) matrices, tr(ABC), m = 256.
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

METRIC = "sketch estimates/s at 1e-2 rel. error; % HBM roofline; batched/learned vs plain"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="torus", choices=["torus", "triangle"])
    ap.add_argument("--m", type=int, default=None)
    ap.add_argument("--samples", type=int, default=None)
    ap.add_argument("--batch", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    return ap.parse_args()


def build_workload(a):
    import numpy as np
    import tn_workloads as W
    if a.workload == "torus":
        m = a.m or 1024
        B = a.batch or 256
        S = a.samples or 8
        nets = [W.torus(L=4, D=16, seed=2 + b) for b in range(B)]
        name = f"torus4x4_D16_fp32_uniform_m{m}"
        dtype = "float32"
    else:
        m = a.m or 256
        B = a.batch or 64
        S = a.samples or 64
        nets = [W.triangle(64, seed=1 + b) for b in range(B)]
        name = f"triangle64_fp64_normal_m{m}"
        dtype = "float64"
    return nets, m, S, name, dtype


def _cpu_worker(args):
    workload, m, seed, samples = args
    import oracle
    import tn_workloads as W
    net = W.torus(L=4, D=16, seed=2) if workload == "torus" else W.triangle(64, seed=1)
    t0 = time.perf_counter()
    for r in samples:
        oracle.m1_estimate(net, m, seed, r, combine="dft")
    return len(samples), time.perf_counter() - t0


def cpu_baseline(workload, m, seconds):
    """The FP64 oracle (Eq. (1) with its DFT) on the host cores: one process per
    core, each timing sketch estimates of one network for ~`seconds`."""
    import oracle
    import tn_workloads as W
    oracle.build()
    net = W.torus(L=4, D=16, seed=2) if workload == "torus" else W.triangle(64, seed=1)
    t0 = time.perf_counter()
    oracle.m1_estimate(net, m, 0, 0, combine="dft")
    one = max(time.perf_counter() - t0, 1e-6)
    cores = max(1, min(16, os.cpu_count() or 1))
    per = max(1, int(seconds / one))
    jobs = [(workload, m, 0, list(range(c * per, (c + 1) * per))) for c in range(cores)]
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(cores) as pool:
        res = pool.map(_cpu_worker, jobs)
    wall = time.perf_counter() - t0
    n = sum(r[0] for r in res)
    return {"value": n / wall, "unit": "estimates/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} estimates of one {workload} network (m={m}, FP64, DFT combine), "
                      f"{per} per process on {cores} processes, {wall:.1f} s wall"}


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch
    import paper_2603_07387_amd as T
    torch.cuda.set_device(0)
    nets, m, S, name, dtype = build_workload(a)
    td = getattr(torch, dtype)
    specs = []
    for n in nets:
        ts = [torch.from_numpy(np.ascontiguousarray(x)).to("cuda", td) for x in n.data]
        specs.append(T.NetworkSpec.from_network(n, ts))
    torch.cuda.synchronize()
    flags = T.TN_FLAG_PROFILE | (0 if os.environ.get("TN_SCATTER_SB") else T.TN_FLAG_AUTOTUNE)
    plan = T.Plan(specs, T.TN_CYCLIC, m, S, 0, flags=flags)
    stats = torch.empty(2 * len(nets), dtype=torch.float64, device="cuda")
    for _ in range(a.warmup):
        plan.estimate(stats)
    torch.cuda.synchronize()
    for k in range(4):
        plan.kernel_time(k)     # drop warm-up records
    t0 = time.perf_counter()
    for _ in range(a.steps):
        plan.estimate(stats)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall * 1e3 / a.steps
    est_total = len(nets) * S * a.steps
    value = est_total / wall
    sk_ms, sk_n = plan.kernel_time(T.TN_KERNEL_SKETCH)
    kt = {"hash": plan.kernel_time(T.TN_KERNEL_HASH), "combine": plan.kernel_time(T.TN_KERNEL_COMBINE),
          "stats": plan.kernel_time(T.TN_KERNEL_STATS)}
    # Algorithmic bytes of one sketching launch: every tensor entry once per pass of
    # `sb` samples, the packed hash tables of each sample, the m-float sketch of
    # each (slot, sample).
    entries = sum(n.nnz() for n in nets)
    esize = np.dtype(dtype).itemsize
    W_ = plan.query(0)
    sb, chunk = plan.query(8), plan.query(9)
    passes = -(-chunk // sb)
    sketch_bytes = plan.query(6) * m * (8 if dtype == "float64" else 4)
    launch_bytes = passes * entries * esize + chunk * W_ * 4 + chunk * sketch_bytes
    avg_ms = sk_ms / max(1, sk_n)
    achieved = launch_bytes / (avg_ms * 1e-3) / 1e9
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "estimates/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if dtype == "float32" else "f64",
        "data": "synthetic",
        "config": {"workload": name, "networks": len(nets), "samples_per_network": S, "m": m,
                   "entries": entries, "bytes_resident": entries * esize},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "m1_scatter", "avg_launch_ms": avg_ms, "launches": sk_n,
                     "algorithmic_bytes_per_launch": launch_bytes, "samples_per_pass": sb},
        "kernel_ms_per_step": {"sketch": sk_ms / a.steps,
                               **{k: v[0] / a.steps for k, v in kt.items()}},
    }
    plan.close()
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(a.workload, m, a.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
