"""Throughput benchmark of the sketching estimators on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload batched|torus|ttcat|triangle|ladder]
                    [--m M] [--samples S] [--batch B] [--products fp32|fp64|bf16] [--dft fft|bf16|fp8]
                    [--persistent] [--error-curve] [--no-cpu-baseline] [--no-plain]

A step is one full pass of the estimator over one batch of synthetic input
already resident in HBM: hash generation, the sketching pass over every tensor,
the combine and the per-network mean/variance, for every sample of every
network in the batch.  Prints one JSON line.

Workloads (all inputs seeded and synthetic):
  batched   4096 random connected cyclic networks, 3-12 tensors, bonds
            U{2..32}, FP32 N(0,1), cyclic estimator, m = 1024, S = 16
            (1.16 GB resident); the combine's DFTs on the BF16 matrix cores
            unless --dft fft (or --persistent: that kernel has its own FFT).  Default.
  torus     4 x 4 periodic lattice of order-4 tensors, bond 16, FP32 U[0,1),
            cyclic estimator, m = 1024; a batch of B independent tori
            (B = 256: 1 GiB resident).
  ttcat     tensor-train caterpillar (32 cores (1,64,64)..(64,64,1) with their
            physical legs contracted against vectors), FP32 N(0,1/64), acyclic
            estimator, m = 4096, S = 4096 samples; products on the FP32 matrix
            cores unless --products says otherwise.
  triangle  three 64 x 64 FP64 N(0,1) matrices, tr(ABC), m = 256.
  ladder    the literal inner product of two such tensor trains (a cyclic
            ladder of 64 cores, 94 contractions), cyclic estimator,
            m = 4096, S = 64.
Single-network workloads (ttcat, ladder) also report the output-relative
error against the exact FP64 contraction (tn_contract_exact): their
input-relative scale prod ||X_k||_F dwarfs the value itself.
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
FP64_MFMA_PEAK_TFLOPS = 78.6   # dense FP64 matrix cores (the same figure as FP64 vector)
FP32_MFMA_PEAK_TFLOPS = 157.3   # dense FP32 matrix cores
BF16_MFMA_PEAK_TFLOPS = 2500.0  # dense BF16 matrix cores

METRIC = "sketch estimates/s at 1e-2 rel. error; % HBM roofline; batched/learned vs plain"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="batched", choices=["torus", "batched", "ttcat", "triangle", "ladder"])
    ap.add_argument("--m", type=int, default=None)
    ap.add_argument("--samples", type=int, default=None)
    ap.add_argument("--batch", type=int, default=None)
    ap.add_argument("--products", default="fp32", choices=["fp64", "fp32", "bf16"],
                    help="acyclic method: SMVP products on the FP32 (default; exact operands for FP32 "
                         "data), FP64 (the reference mode) or BF16 matrix cores")
    ap.add_argument("--dft", default=None, choices=["fft", "bf16", "fp8"],
                    help="cyclic method, m = 1024: the combine's DFTs as an LDS FFT or as 32 x 32 products "
                         "on the BF16 (TN_FLAG_DFT_BF16) or FP8 (TN_FLAG_DFT_FP8) matrix cores; default bf16 "
                         "for the batched workload (its configuration names BF16 matrix-core contractions), "
                         "fft otherwise")
    ap.add_argument("--persistent", action="store_true",
                    help="cyclic method: the persistent fused kernel (TN_FLAG_PERSISTENT)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--error-curve", action="store_true",
                    help="torus: the exact FP64 contraction of the first torus (tn_contract_exact) and the "
                         "relative error of the mean of S estimates against it, S = 1 .. 4096, at "
                         "m = 1024, 16384 and 65536")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the unbatched comparison (one plan per network)")
    ap.add_argument("--cpu-seconds", type=float, default=8.0,
                    help="seconds of oracle work per leg (one process, then all cores)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run 5 device copies of 1 GiB (reference for HBM byte counters)")
    return ap.parse_args()


def copy_calibration():
    """Plain 1 GiB device-to-device copies: the reference kernel whose FETCH_SIZE
    and WRITE_SIZE counters calibrate the HBM traffic of the estimator kernels."""
    import torch
    n = (1 << 30) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "copies": 5}))


def build_workload(a):
    import tn_workloads as W
    if a.workload == "torus":
        m, B, S = a.m or 1024, a.batch or 256, a.samples or 32
        nets = [W.torus(L=4, D=16, seed=2 + b) for b in range(B)]
        return nets, m, S, f"torus4x4_D16_fp32_uniform_m{m}_x{B}", "float32", "cyclic"
    if a.workload == "batched":
        m, B, S = a.m or 1024, a.batch or 4096, a.samples or 16
        nets = W.random_batch(count=B, seed=4)
        return nets, m, S, f"random_cyclic_3to12_bond2to32_fp32_m{m}_x{B}", "float32", "cyclic"
    if a.workload == "ttcat":
        m, B, S = a.m or 4096, a.batch or 1, a.samples or 4096
        nets = [W.tt_caterpillar(seed=3 + b) for b in range(B)]
        return nets, m, S, f"tt_caterpillar32_bond64_phys64_fp32_m{m}_x{B}", "float32", "acyclic"
    if a.workload == "ladder":
        m, B, S = a.m or 4096, a.batch or 1, a.samples or 64
        nets = [W.tt_ladder(seed=3 + b) for b in range(B)]
        return nets, m, S, f"tt_ladder32_bond64_phys64_fp32_m{m}_x{B}", "float32", "cyclic"
    m, B, S = a.m or 256, a.batch or 64, a.samples or 256
    nets = [W.triangle(64, seed=1 + b) for b in range(B)]
    return nets, m, S, f"triangle64_fp64_normal_m{m}_x{B}", "float64", "cyclic"


def _oracle_net(workload, j):
    """Network j of the workload as the oracle sees it (the batched workload's
    networks differ; the other workloads repeat one network)."""
    import tn_workloads as W
    if workload == "batched":
        return W.random_network(4, j)
    return {"torus": lambda: W.torus(L=4, D=16, seed=2), "ttcat": lambda: W.tt_caterpillar(seed=3),
            "triangle": lambda: W.triangle(64, seed=1), "ladder": lambda: W.tt_ladder(seed=3)}[workload]()


def _cpu_worker(args):
    """Estimates of (network j, sample r) pairs until `seconds` of oracle time
    have passed (building the networks' inputs is not counted)."""
    workload, m, jobs, seconds = args
    import oracle
    done, spent = 0, 0.0
    cache = {}
    for (j, r) in jobs:
        if j not in cache:
            cache.clear()
            cache[j] = _oracle_net(workload, j)
        net = cache[j]
        t0 = time.perf_counter()
        if workload == "ttcat":
            oracle.m2_estimate(net, m, j, r)
        else:
            oracle.m1_estimate(net, m, j, r, combine="dft")
        spent += time.perf_counter() - t0
        done += 1
        if spent >= seconds:
            break
    return done, spent


def _jobs(workload, S, worker, workers, count):
    """(network, sample) pairs in the GPU's order: every sample of network 0,
    then of network 1, ...  The batched workload's 4096 networks are split
    into one contiguous run per worker; the other workloads have one network
    and each worker takes its own run of samples."""
    if workload == "batched":
        start = worker * (4096 // workers) * S
        return [((start + i) // S % 4096, (start + i) % S) for i in range(count)]
    return [(0, worker * count + i) for i in range(count)]


def cpu_baseline(workload, m, S, seconds):
    """The FP64 oracle on the host cores: one process for `seconds`, then one
    process per core (up to the box's share of 16) for `seconds` each, all on
    the workload's (network, sample) pairs.  The rate of the parallel leg is
    its estimates over the longest worker's oracle time."""
    import oracle
    oracle.build()
    nproc = os.cpu_count() or 1
    cores = max(1, min(16, nproc))
    cap = 1 << 20
    n1, w1 = _cpu_worker((workload, m, _jobs(workload, S, 0, 1, cap), seconds))
    jobs = [(workload, m, _jobs(workload, S, c, cores, cap), seconds) for c in range(cores)]
    with mp.get_context("spawn").Pool(cores) as pool:
        res = pool.map(_cpu_worker, jobs)
    n = sum(r[0] for r in res)
    wall = max(r[1] for r in res)
    how = "Method 2, Alg. 2-5" if workload == "ttcat" else "Eq. (1) with its DFT"
    what = ("networks of the batch in order, S samples each" if workload == "batched"
            else f"one {workload} network")
    return {"value": n / wall, "unit": "estimates/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} estimates ({what}; m={m}, FP64, {how}) on {cores} processes, "
                      f"{wall:.1f} s of oracle time in the longest process",
            "nproc": nproc,
            "single_thread": {"value": n1 / w1, "unit": "estimates/s", "cores": 1,
                              "sample": f"{n1} estimates ({what}) in {w1:.1f} s on one process"}}


def source_hash(kernel_sources):
    import hashlib
    d = hashlib.sha256()
    for src in kernel_sources:
        d.update(open(os.path.join(ROOT, src), "rb").read())
    return d.hexdigest()[:16]


def measured_traffic(workload_name, samples_per_pass, kernel_sources):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    summary, if it was taken on this workload, schedule and kernel sources."""
    import glob
    h = source_hash(kernel_sources)
    for path in glob.glob(os.path.join(ROOT, "profiles", "*.md")):
        for line in open(path):
            if not line.startswith("machine-readable:"):
                continue
            kv = dict(tok.split("=", 1) for tok in line.split()[1:] if "=" in tok)
            if (kv.get("workload") == workload_name and kv.get("samples_per_pass") == str(samples_per_pass)
                    and kv.get("kernel_source_sha256_16") == h):
                return float(kv["traffic_bytes_per_launch"]), os.path.basename(path)
    return None, None


def m2_products(net, root=0):
    """(rows, cols) of w_k = mat(X_k) G for every tensor with children when the
    tree is rooted at `root`: rows is the size of the parent mode (1 at the
    root), cols the product of the child modes."""
    import numpy as np
    owner = [k for k in range(net.p) for _ in range(net.orders[k])]
    partner = {}
    for (u, v) in net.edges:
        partner[u], partner[v] = v, u
    parent_mode = {root: None}
    order = [root]
    for k in order:
        for u in net.modes(k):
            l = owner[partner[u]]
            if u != parent_mode[k] and l not in parent_mode:
                parent_mode[l] = partner[u]
                order.append(l)
    out = []
    for k in range(net.p):
        rows = 1 if parent_mode[k] is None else net.dims[parent_mode[k]]
        cols = int(np.prod([net.dims[u] for u in net.modes(k) if u != parent_mode[k]], dtype=np.int64))
        if net.orders[k] > (0 if parent_mode[k] is None else 1):
            out.append((rows, cols))
    return out


def plain_form(T, specs, meth, m, S, flags, steps, limit=256):
    """The unbatched form on the same GPU: one plan per network (the first
    `limit` networks of the workload), estimated one after another on the same
    stream, same m, samples and flags.  Returns its estimates/s."""
    import torch
    specs = specs[:limit]
    plans = [T.Plan([sp], meth, m, S, 0, flags=flags) for sp in specs]
    stats = torch.empty(2, dtype=torch.float64, device="cuda")
    for pl in plans:                       # warm-up (and the autotuner's runs)
        pl.estimate(stats)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for pl in plans:
            pl.estimate(stats)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for pl in plans:
        pl.close()
    return {"value": len(specs) * S * steps / wall, "unit": "estimates/s", "networks": len(specs),
            "form": "one plan per network, estimated in turn on one stream"}


def kernel_breakdown(T, specs, meth, m, S, flags, steps):
    """Device ms per step of each kernel kind, from a separate untimed pass of
    `steps` estimates with HIP events around every launch."""
    import torch
    plan = T.Plan(specs, meth, m, S, 0, flags=flags)
    stats = torch.empty(2 * len(specs), dtype=torch.float64, device="cuda")
    plan.estimate(stats)
    torch.cuda.synchronize()
    kinds = {"sketch": T.TN_KERNEL_SKETCH, "hash": T.TN_KERNEL_HASH, "combine": T.TN_KERNEL_COMBINE,
             "stats": T.TN_KERNEL_STATS}
    for k in kinds.values():
        plan.kernel_time(k)
    for _ in range(steps):
        plan.estimate(stats)
    torch.cuda.synchronize()
    out = {name: plan.kernel_time(k)[0] / steps for name, k in kinds.items()}
    plan.close()
    return out


def error_curve(T, spec, torch):
    """The 4 x 4 bond-16 torus against its exact value: the relative error of
    the mean of the first S estimates (fresh plans, seed 5) for S = 4^j, and
    the spread of one estimate, at three sketch sizes.  Uniform[0,1) tensors
    are dominated by their all-ones part, so single estimates are heavy-tailed
    (Lemma 7's regime) and the error falls slowly and unevenly with S."""
    import numpy as np
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    z = T.tn_contract_exact(spec)
    t_exact = time.perf_counter() - t0
    res = {"exact": z, "exact_seconds": t_exact,
           "exact_main_product_flops": 4.0 * 16.0 ** 12,  # two 65536^3 products on the FP64 matrix cores
           "m": {}}
    S = 4096
    for m in (1024, 16384, 65536):
        plan = T.Plan([spec], T.TN_CYCLIC, m, S, 5)
        smp = torch.empty(S, dtype=torch.float64, device="cuda")
        plan.estimate(samples_out=smp)
        y = smp.cpu().numpy()
        plan.close()
        sizes = [4 ** j for j in range(7)]
        res["m"][str(m)] = {
            "S": sizes,
            "rel_error_of_mean": [float(abs(y[:k].mean() - z) / z) for k in sizes],
            "rel_std_of_one_estimate": float(y.std(ddof=1) / z),
            "rel_error_median_of_means_64_groups": float(abs(np.median(y.reshape(64, -1).mean(axis=1)) - z) / z),
        }
    return res


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    import numpy as np
    import torch
    import paper_2603_07387_amd as T
    torch.cuda.set_device(0)
    if a.copy_calibration:
        copy_calibration()
        return
    nets, m, S, name, dtype, method = build_workload(a)
    td = getattr(torch, dtype)
    specs = []
    for n in nets:
        ts = [torch.from_numpy(np.ascontiguousarray(x)).to("cuda", td) for x in n.data]
        specs.append(T.NetworkSpec.from_network(n, ts))
    torch.cuda.synchronize()
    # Timed region: HIP events around the sketching launches only (each event
    # costs device time); the per-kind breakdown comes from a second pass below.
    base_flags = 0 if os.environ.get("TN_SCATTER_SB") else T.TN_FLAG_AUTOTUNE
    flags = base_flags | T.TN_FLAG_PROFILE | T.TN_FLAG_PROFILE_SKETCH
    bf16_products = a.products == "bf16" and method == "acyclic"
    if bf16_products:
        flags |= T.TN_FLAG_MFMA_BF16
    f32_products = a.products == "fp32" and method == "acyclic" and dtype != "float64"
    if f32_products:
        flags |= T.TN_FLAG_MFMA_F32
    # the persistent kernel carries its own FFT combine
    dft = a.dft or ("bf16" if a.workload == "batched" and m == 1024 and dtype != "float64" and not a.persistent
                    else "fft")
    dft_bf16 = dft == "bf16" and method == "cyclic"
    if dft_bf16:
        flags |= T.TN_FLAG_DFT_BF16
    dft_fp8 = dft == "fp8" and method == "cyclic"
    if dft_fp8:
        flags |= T.TN_FLAG_DFT_FP8
    persistent = a.persistent and method == "cyclic"
    if persistent:
        flags |= T.TN_FLAG_PERSISTENT
    meth = T.TN_CYCLIC if method == "cyclic" else T.TN_ACYCLIC
    plan = T.Plan(specs, meth, m, S, 0, flags=flags)
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
    value = len(nets) * S * a.steps / wall
    sk_ms, sk_n = plan.kernel_time(T.TN_KERNEL_SKETCH)
    avg_ms = sk_ms / max(1, sk_n)
    kt = kernel_breakdown(T, specs, meth, m, S, (flags & ~T.TN_FLAG_PROFILE_SKETCH), a.steps)
    plain = None
    if len(specs) > 1 and not a.no_plain:
        plain = plain_form(T, specs, meth, m, S, flags & ~(T.TN_FLAG_PROFILE | T.TN_FLAG_PROFILE_SKETCH),
                           min(a.steps, 5))
        plain["batched_over_plain"] = value / plain["value"]
    entries = sum(n.nnz() for n in nets)
    esize = np.dtype(dtype).itemsize
    if method == "cyclic":
        # Algorithmic bytes of one sketching launch: every tensor entry once per
        # pass of `sb` samples, the packed hash tables of each sample, the m-word
        # sketch of each (slot, sample).
        # (The persistent kernel writes estimates only: no sketch vectors.)
        sb, chunk, banks = plan.query(8), plan.query(9), plan.query(10)
        passes = -(-chunk // sb)
        sketch_bytes = 0 if persistent else plan.query(6) * m * (8 if dtype == "float64" else 4)
        launch_units = passes * entries * esize + chunk * plan.query(0) * 4 + chunk * sketch_bytes
        achieved = launch_units / (avg_ms * 1e-3) / 1e9
        kname = "m1_fused_kernel" if persistent else "m1_scatter_kernel"
        src = ["paper_2603_07387_amd/csrc/fused.hip" if persistent else "paper_2603_07387_amd/csrc/m1.hip",
               "paper_2603_07387_amd/csrc/m1_device.h"]
        traffic, tsrc = measured_traffic(name, sb, src)
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "traffic_source": tsrc,
                "kernel": kname,
                "avg_launch_ms": avg_ms, "launches": sk_n, "algorithmic_bytes_per_launch": launch_units,
                "samples_per_pass": sb, "accumulator_banks": banks}
    else:
        # One product launch per tree depth: w_k = mat(X_k) G for every tensor
        # with children, rows x cols times cols x S.
        prods = [rc for n in nets for rc in m2_products(n)]
        flops_step = 2.0 * sum(r * c for r, c in prods) * S
        if bf16_products:
            # BF16 matrix cores are ~30x faster than the FP64 ones: the launch is
            # bound by reading G (cols x S; stored as BF16 for FP32/BF16 data,
            # FP64 for FP64 data), X once and writing w.
            gsize = 8 if dtype == "float64" else 2
            wsize = 8 if dtype == "float64" else 4
            bytes_step = sum(S * c * gsize + r * c * esize + S * r * wsize for r, c in prods)
            achieved = bytes_step / (sk_ms / a.steps * 1e-3) / 1e9
            roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": achieved / HBM_PEAK_GBS, "traffic": None, "kernel": "m2_gemm16_kernel<BF16>",
                    "avg_launch_ms": avg_ms, "launches": sk_n, "algorithmic_bytes_per_step": bytes_step,
                    "flops_per_step": flops_step}
        else:
            achieved = flops_step / (sk_ms / a.steps * 1e-3) / 1e12
            peak = FP32_MFMA_PEAK_TFLOPS if f32_products else FP64_MFMA_PEAK_TFLOPS
            roof = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                    "frac": achieved / peak, "traffic": None,
                    "kernel": "m2_gemm16_kernel<F32>" if f32_products else "m2_gemm16_kernel",
                    "avg_launch_ms": avg_ms, "launches": sk_n, "flops_per_step": flops_step}
    st = stats.cpu().numpy().reshape(-1, 2)
    norms = np.array([n.input_norm() for n in nets])
    # input-relative std of one estimate (Def. 4's error scale), and the samples
    # a network needs for a mean within 1e-2 of it (one standard error)
    rel_std = np.sqrt(np.maximum(st[:, 1], 0)) / norms
    need = np.maximum(1.0, np.ceil((rel_std / 1e-2) ** 2))
    exact = None
    if a.workload in ("ttcat", "ladder"):
        # output-relative error against the exact FP64 contraction of each network
        vals = np.array([T.tn_contract_exact(sp) for sp in specs])
        rel_out = np.abs(st[:, 0] - vals) / np.abs(vals)
        std_out = np.sqrt(np.maximum(st[:, 1], 0)) / np.abs(vals)
        exact = {"exact": [float(v) for v in vals[:4]],
                 "mean_estimate": [float(v) for v in st[:4, 0]],
                 "output_relative_error_of_mean": float(np.median(rel_out)),
                 "output_relative_std_of_one_estimate": float(np.median(std_out)),
                 "samples_for_1e-2_output_relative": float(np.median(np.maximum(1.0, np.ceil((std_out / 1e-2) ** 2))))}
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
        "config": {"workload": name, "method": method, "networks": len(nets),
                   "samples_per_network": S, "m": m, "entries": entries,
                   **({"products": "bf16 matrix cores, fp32 accumulation"} if bf16_products else {}),
                   **({"products": "fp32 matrix cores, fp32 accumulation"} if f32_products else {}),
                   **({"dft": "bf16 matrix cores (32 x 32 four-step), fp32 accumulation"} if dft_bf16 else {}),
                   **({"dft": "fp8 (e4m3) matrix cores (32 x 32 four-step), fp32 accumulation"} if dft_fp8 else {}),
                   "bytes_resident": entries * esize},
        "roofline": roof,
        "at_1e-2": {"median_input_relative_std": float(np.median(rel_std)),
                    "median_samples_needed": float(np.median(need)),
                    "networks_per_s": float(len(nets) / np.sum(need) * value)},
        "kernel_ms_per_step": kt,
        "plain": plain,
        **({"output_relative": exact} if exact is not None else {}),
    }
    plan.close()
    if a.error_curve and a.workload == "torus":
        out["error_curve"] = error_curve(T, specs[0], torch)
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(a.workload, m, S, a.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
