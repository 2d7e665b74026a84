"""Benchmark of the Fastfood hot path on one MI355X.

Workload (MNIST-shaped synthetic input, the paper's data shape): 8192 rows of
784 pixels (80 % zeros, else uniform [0, 1]) padded to n = 1024, E = 16
expansions (32768 features per row), RBF sigma = 2, seed 1398239763.

A step is one forward pass x -> phi over the batch (one kernel launch); the
fwd+bwd step adds the adjoint (dx and the batch-summed dB, dG, dS).  Inputs
are resident in HBM before timing.  Prints one JSON line.

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--cpu-seconds S]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

BATCH, D, N, E, SIGMA = 8192, 784, 1024, 16, 2.0
FWD_BYTES_PER_VECTOR = 4 * D + 8 * N * E          # read x, write phi
BWD_BYTES_PER_VECTOR = 8 * D + 8 * N * E          # read x and dphi, write dx
HBM_PEAK_GBS = 8000.0
METRIC = "Fastfood vectors/s + %HBM peak at n=1024 E=16, fwd and fwd+bwd vs oracle error"


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--only", choices=["fwd", "bwd", "all"], default="all",
                    help="time only one pass (for profiling); the JSON line then lacks the other")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also time a plain 1 GiB device copy and fill (bandwidth calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(rows would shard with zero communication; see DESIGN.md)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1702_08159_amd as mk
    import workloads

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    seed = workloads.FASTFOOD_SEED
    x_np = workloads.mnist_sparse(BATCH)
    x = torch.from_numpy(x_np).to(dev)
    phi = torch.empty((BATCH, 2 * N * E), dtype=torch.float32, device=dev)
    dphi = torch.from_numpy(workloads.grad_features(BATCH, 2 * N * E)).to(dev)
    dx = torch.empty_like(x)
    log("inputs resident; building plan")
    mk.forward(x, E, seed, SIGMA, out=phi)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream(dev)

    def fwd():
        mk.forward(x, E, seed, SIGMA, out=phi)

    def bwd():
        return mk.backward(x, dphi, E, seed, SIGMA, need_dx=True, need_params=True)

    use_graph = not args.no_graph
    graph = None
    if use_graph:
        # one hipGraph launch per forward step (the plan is already cached)
        s = torch.cuda.Stream(dev)
        s.wait_stream(stream)
        with torch.cuda.stream(s):
            for _ in range(2):
                fwd()
        stream.wait_stream(s)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            fwd()
        torch.cuda.synchronize()

    def run_fwd():
        if graph is not None:
            graph.replay()
        else:
            fwd()

    t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0.record(stream)
        for _ in range(steps):
            fn()
        t1.record(stream)
        torch.cuda.synchronize()
        return t0.elapsed_time(t1) / steps

    if args.copy_probe:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        b = torch.empty_like(a)
        cp_ms = timed(lambda: b.copy_(a), 20, 3)
        fill_ms = timed(lambda: b.fill_(2.0), 20, 3)
        log("copy 1 GiB: %.3f ms (%.0f GB/s read+write); fill 1 GiB: %.3f ms (%.0f GB/s)"
            % (cp_ms, 2 * (1 << 30) / cp_ms / 1e6, fill_ms, (1 << 30) / fill_ms / 1e6))
        del a, b

    fwd_ms = bwd_ms = float("nan")
    if args.only in ("fwd", "all"):
        fwd_ms = timed(run_fwd, args.steps, args.warmup)
        log("forward %.3f ms/step" % fwd_ms)
    if args.only in ("bwd", "all"):
        bwd_ms = timed(bwd, args.steps, max(1, args.warmup // 2))
        log("backward %.3f ms/step" % bwd_ms)

    fwd_vps = BATCH / (fwd_ms * 1e-3)
    fb_ms = fwd_ms + bwd_ms
    fb_vps = BATCH / (fb_ms * 1e-3)
    fwd_gbs = FWD_BYTES_PER_VECTOR * BATCH / (fwd_ms * 1e-3) / 1e9
    fb_bytes = (FWD_BYTES_PER_VECTOR + BWD_BYTES_PER_VECTOR) * BATCH
    fb_gbs = fb_bytes / (fb_ms * 1e-3) / 1e9

    cpu = None
    err = None
    if not args.no_cpu_baseline and args.only != "bwd":
        import oracle

        oracle.build(force=False)
        phi_host = phi.cpu().numpy()
        p = oracle.params(seed, N, E, SIGMA)
        xs = x_np.astype(np.float64)
        t = time.perf_counter()
        oracle.forward(xs[:64], E, seed, SIGMA, p=p)
        per_row = (time.perf_counter() - t) / 64
        rows = int(min(BATCH, max(64, args.cpu_seconds / per_row)))
        worst = 0.0
        t = time.perf_counter()
        for r0 in range(0, rows, 512):
            r1 = min(rows, r0 + 512)
            ref, _, _ = oracle.forward(xs[r0:r1], E, seed, SIGMA, p=p)
            dif = np.linalg.norm(phi_host[r0:r1].astype(np.float64) - ref, axis=1) / np.linalg.norm(ref, axis=1)
            worst = max(worst, float(dif.max()))
        cpu_s = time.perf_counter() - t
        log("oracle: %d rows in %.1f s" % (rows, cpu_s))
        cpu = {"value": rows / cpu_s, "unit": "vectors/s", "cores": 1, "kind": "oracle",
               "sample": "first %d of the %d rows, forward, FP64 C oracle, one thread" % (rows, BATCH)}
        err = worst

    line = {
        "metric": METRIC,
        "value": fwd_vps,
        "unit": "vectors/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": fwd_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "fastfood-forward mnist-shaped 8192x784 (80% zeros) n=1024 E=16 sigma=2",
                   "batch": BATCH, "d": D, "n": N, "E": E, "sigma": SIGMA, "graph": use_graph},
        "fwd_hbm_frac": fwd_gbs / HBM_PEAK_GBS,
        "fwd_bwd_vectors_per_s": fb_vps,
        "fwd_bwd_ms_per_step": fb_ms,
        "fwd_bwd_hbm_frac": fb_gbs / HBM_PEAK_GBS,
        "bwd_ms_per_step": bwd_ms,
        "max_row_rel_err_vs_oracle": err,
        "roofline": {"bound": "hbm", "achieved": fwd_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": fwd_gbs / HBM_PEAK_GBS, "traffic": None},
        "cpu_baseline": cpu,
    }
    def clean(o):
        if isinstance(o, dict):
            return {k: clean(v) for k, v in o.items()}
        if isinstance(o, float) and not math.isfinite(o):
            return None
        return o

    print(json.dumps(clean(line)), flush=True)


if __name__ == "__main__":
    main()
