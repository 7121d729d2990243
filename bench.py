#!/usr/bin/env python
"""Throughput of the PeriDEM step loop on one MI355X.

One step is one pass of the whole hot path (velocity-Verlet position update,
cell-key radix sort and cell starts, contact + walls + bond forces + velocity
update) over the settling bed of 100 particles (equal thirds of disks, plus
shapes and rings, R ~ U[0.8, 1.2] mm, h = 0.0904 mm, horizon 3h, contact
radius 0.95h, 30 x 60 mm box, gravity 9.81 m/s^2, dt = 1e-7 s, plain FP64),
with all inputs resident in device memory.

Prints one JSON line: bond interactions/s (unordered reference bonds x
steps/s) as the value, steps/s beside it, the roofline of the dominant
kernel (force kernel: algorithmic bytes per launch / mean launch time from
HIP events on the library's stream) and the FP64 CPU oracle timed on the
host cores over a bounded sample of the same workload.
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

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
BYTES_PER_NODE_FORCE = 16 + 16 + 16 + 16 + 48  # x, u, v, a read; u, v, a written
BYTES_PER_BOND = 4  # one 32-bit slot per directed bond (partner index + broken bit)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2108_07212_amd", "csrc", "pd_kernels.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they
    were taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    e = rec.get(kernel, {}).get(workload)
    if not e or e.get("kernel_source") != kernel_source_hash():
        return None
    return e.get("hbm_bytes_per_launch")


def cpu_baseline(prob, seconds: float, n_pairs: int):
    """The FP64 oracle on the host cores, a bounded number of steps."""
    from oracle import Oracle
    threads = min(os.cpu_count() or 1, 16)
    o = Oracle(prob, contact_mode=1, n_threads=threads)
    o.step(2)
    t0 = time.perf_counter()
    n = 0
    while True:
        o.step(5)
        n += 5
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    sps = n / el
    return {"value": n_pairs * sps, "unit": "bond interactions/s", "cores": threads,
            "kind": "oracle", "steps_per_s": sps,
            "sample": f"{n} steps of the same settling bed (FP64 oracle, bucket-grid contact, "
                      f"OpenMP over nodes), {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=500)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-steps", type=int, default=500)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the path has no "
              "multi-GPU form in this build", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2108_07212_amd import pd
    from paper_2108_07212_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(3)
    torch.cuda.set_device(0)
    prob = W.settling()
    g = pd.PD(prob)
    sizes = g.sizes()
    N, n_dir = sizes["nodes"], sizes["bonds"]
    n_pairs = n_dir // 2
    def timed(steps):
        torch.cuda.synchronize()
        r0 = g.sizes()["list_rebuilds"]
        t0 = time.perf_counter()
        g.step(steps)  # returns after the stream is drained
        torch.cuda.synchronize()
        return steps / (time.perf_counter() - t0), g.sizes()["list_rebuilds"] - r0

    # the contact set evaluated from exact distances every step, over the
    # candidate lists (rebuilt by the cell-key radix sort when stale)
    g.step(args.warmup)
    sps, rebuilds = timed(args.steps)
    # per-kernel mean launch time (HIP events on the library's stream)
    kt = g.time_kernels(args.kernel_steps)
    force_ms = kt["force"][0]
    # the same loop with the cell search run every step (skin 0)
    tun = g.tuning()
    g.set_tuning(skin_factor=0.0)
    g.step(max(10, args.warmup // 10))
    sps0, _ = timed(max(100, args.steps // 10))
    g.set_tuning(**tun)
    force_bytes = BYTES_PER_NODE_FORCE * N + BYTES_PER_BOND * n_dir
    achieved = force_bytes / (force_ms * 1e-3) / 1e9
    traffic = measured_traffic("force", "settling_100")
    out = {
        "metric": "PD bond interactions/s (plain FP64, settling bed)",
        "value": n_pairs * sps,
        "unit": "bond interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 / sps,
        "steps_per_s": sps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded settling bed, lattice nodes, RSA placement)",
        "config": {"workload": "settling_100", "particles": prob.n_particles, "nodes": N,
                   "directed_bonds": n_dir, "unordered_bonds": n_pairs, "dt": prob.dt,
                   "gravity": prob.gravity[1], "precision": "fp64", "tuning": g.tuning()},
        "roofline": {"bound": "hbm", "kernel": "k_force<double,M_STEP>", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "bytes_per_launch": force_bytes,
                     "mean_launch_ms": force_ms},
        "kernels_ms": {k: v[0] for k, v in kt.items()},
        "kernel_launches_per_step": {k: v[1] / args.kernel_steps for k, v in kt.items()},
        "list_rebuilds_per_1000_steps": 1000.0 * rebuilds / args.steps,
        "every_step_search": {"value": n_pairs * sps0, "steps_per_s": sps0,
                              "note": "same step with the cell-key sort and cell search "
                                      "every step (skin 0)"},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(W.settling(), args.cpu_seconds, n_pairs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
