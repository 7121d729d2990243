#!/usr/bin/env python
"""Throughput of the PeriDEM step loop on one MI355X.

One step is one pass of the whole hot path (velocity-Verlet position update,
contact candidates (cell-key radix sort when a list goes stale), contact +
walls + bond forces with breaking, velocity update) over 64 independent
settling aggregates of 50-400 particles each (disks, plus shapes and rings,
R ~ U[0.8, 1.2] mm, h = 0.078 mm, horizon 3h, contact radius 0.95h,
gravity 9.81 m/s^2, dt = 1e-7 s): 6.4M nodes and 130M directed bonds in
plain FP64, with all inputs resident in device memory.

Prints one JSON line: bond interactions/s (unordered reference bonds x
steps/s) as the value, steps/s beside it, the roofline of the dominant
kernel (force kernel: algorithmic bytes per launch / its mean duration in
graph replays, HIP events on the library's stream) and the FP64 CPU oracle
timed on the host cores over one aggregate of the same workload.  Secondary
legs: the 30k-node settling bed (FP64; also with the cell search every
step), the FP32-force split on the compaction bed, the batch with FP32
forces against its aggregates run one by one, the modal closure, the
notched-square impact and the jammed shape beds.
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# algorithmic bytes of one step: per node x, u, v, a read (64 B), u, v, a
# written (48 B), cell key and permutation (16 B); FP32 force split: a in
# FP32 (16 B less); per directed bond one 32-bit slot (partner + broken bit)
BYTES_PER_NODE = {0: 128, 1: 112}
BYTES_PER_BOND = 4


def kernel_source_hash() -> str:
    """First 16 hex digits of the SHA-256 of pd_kernels.hip's code: comments
    and blank lines taken out, so that a comment edit leaves the traffic
    records valid and any change to the code does not."""
    with open(os.path.join(ROOT, "paper_2108_07212_amd", "csrc", "pd_kernels.hip")) as f:
        src = f.read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = re.sub(r"//[^\n]*", "", src)
    code = "\n".join(ln.rstrip() for ln in src.splitlines() if ln.strip())
    return hashlib.sha256(code.encode()).hexdigest()[:16]


def tuning_key(t: dict) -> str:
    return (f"bn{int(t['block_nodes'])}_lds{int(t['use_lds'])}_lpn{int(t.get('lanes_per_node', 4))}"
            f"_wp{int(t.get('wall_pass', 0))}_sk{float(t.get('skin_factor', 1.0)):g}")


def parse_tuning(text: str) -> dict:
    """'block_nodes=128,use_lds=1,skin_factor=0.5' -> dict"""
    out = {}
    for part in filter(None, text.split(",")):
        k, v = part.split("=")
        out[k.strip()] = float(v) if k.strip() in ("skin_factor", "cell_factor") else int(v)
    return out


def measured_traffic(kernel: str, workload: str, tuning: dict):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they
    were taken on the current kernel source with the same launch
    configuration (nodes per workgroup, LDS staging, lanes per node, wall
    pass, skin)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    e = rec.get(kernel, {}).get(workload, {}).get(tuning_key(tuning))
    if not e or e.get("kernel_source") != kernel_source_hash():
        return None
    return e.get("hbm_bytes_per_launch")


def host_cpu():
    """The host's core count and CPU model (the oracle's machine)."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "model": model}


def cpu_baseline(prob, seconds: float, sample: str):
    """The FP64 oracle on the host cores (OpenMP over nodes, up to 16
    threads), a bounded number of steps of `prob`; then a shorter
    single-thread run.  Rates in bond interactions/s (the sample's unordered
    bonds x its steps/s), which are comparable across problem sizes."""
    from oracle import Oracle

    def run(threads, secs):
        o = Oracle(prob, contact_mode=1, n_threads=threads)
        n_pairs = len(o.bonds()[1]) // 2
        o.step(2)
        t0 = time.perf_counter()
        n = 0
        while True:
            o.step(5)
            n += 5
            el = time.perf_counter() - t0
            if el >= secs:
                break
        return n, el, n_pairs

    threads = min(os.cpu_count() or 1, 16)
    n, el, n_pairs = run(threads, seconds)
    n1, el1, _ = run(1, max(2.0, seconds / 3))
    sps, sps1 = n / el, n1 / el1
    return {"value": n_pairs * sps, "unit": "bond interactions/s", "cores": threads,
            "kind": "oracle", "steps_per_s": sps,
            "single_thread": {"value": n_pairs * sps1, "steps_per_s": sps1,
                              "sample": f"{n1} steps, {el1:.1f} s"},
            "host": host_cpu(),
            "sample": f"{sample}: {prob.n_nodes} nodes, {n_pairs} unordered bonds, {n} steps "
                      f"in {el:.1f} s (FP64 oracle, bucket-grid contact, OpenMP over nodes)"}


def precision_split(pd, W, torch, steps):
    """The compaction run with damage (Sec. 7.4), FP32 force arithmetic
    (FP64 state and FP64 break decisions) against plain FP64: 509 mixed
    particles (178k nodes) from the jammed start of Sec. 7.1; the top wall
    comes down at 1 m/s (the paper's compaction speed) for 5 mm, and from that
    checkpoint at 0.1 m/s until the bonds break.  Along the 0.1 m/s run, at
    every sample: the FP32 force error at the FP64 run's state (max-norm,
    relative), broken bonds of the FP64 and FP32 runs, the top-wall force
    and the volume fraction; the step rates of both.  Then the same error on
    the herded compaction bed (particles pushed into each other at t = 0),
    a stress case."""
    import numpy as np
    pre_steps = 50000
    prob = W.jammed_compaction(wall_speed=1.0)
    g = pd.PD(prob, precision=0)
    g.step(20)
    tun = g.autotune(50)
    t0 = time.perf_counter()
    g.step(pre_steps - 20)
    torch.cuda.synchronize()
    t_pre = time.perf_counter() - t0
    ck = g.get_state()
    wall = float(g.observables()["top_wall_y"][0])
    del g
    run = W.restart_with_wall(prob, ck, wall, 0.1)
    ck0 = dict(ck, step=0)
    ctx = {}
    for prec in (0, 1):
        c = pd.PD(run, precision=prec)
        c.set_tuning(**tun)
        c.set_state(ck0)
        ctx[prec] = c
    probe = pd.PD(run, precision=1)
    probe.set_tuning(**tun)
    series, t_run = [], {0: 0.0, 1: 0.0}
    chunk, done, first = 10000, 0, None
    while done < steps:
        for prec in (0, 1):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            ctx[prec].step(chunk)
            torch.cuda.synchronize()
            t_run[prec] += time.perf_counter() - t1
        done += chunk
        s64 = ctx[0].get_state()
        probe.set_state(s64)
        f64 = ctx[0].forces(pd.TERM_ALL)
        f32 = probe.forces(pd.TERM_ALL)
        scale = max(np.abs(f64[0]).max(), np.abs(f64[1]).max())
        ob = ctx[0].observables()
        nb64, nb32 = int(ctx[0].damage()[1]), int(ctx[1].damage()[1])
        series.append({"step": done, "wall_travel_mm": 1e3 * (run.box[0, 3] - float(ob["top_wall_y"][0])),
                       "force_rel_err_fp32": float(max(np.abs(f32[0] - f64[0]).max(),
                                                       np.abs(f32[1] - f64[1]).max()) / scale),
                       "broken_directed_fp64": nb64, "broken_directed_fp32": nb32,
                       "top_wall_force_y": float(ob["wall_force"][0, 3, 1]),
                       "volume_fraction": float(ob["volume_fraction"][0])})
        if nb64 > 0 and first is None:
            first = done
        if first is not None and done >= first + 3 * chunk:
            break
    n_pairs = ctx[0].sizes()["bonds"] // 2
    res = {"workload": "jammed_compaction (509 particles, 40 x 40 mm, h = 0.070 mm)",
           "nodes": prob.n_nodes, "tuning": tun,
           "precompaction": {"wall_speed": 1.0, "steps": pre_steps, "seconds": t_pre},
           "wall_speed": 0.1, "steps": done, "first_break_step": first, "series": series,
           "fp64": {"steps_per_s": done / t_run[0], "bond_interactions_per_s": n_pairs * done / t_run[0]},
           "fp32": {"steps_per_s": done / t_run[1], "bond_interactions_per_s": n_pairs * done / t_run[1]},
           "max_force_rel_err_fp32": max(e["force_rel_err_fp32"] for e in series)}
    del ctx, probe
    herd = W.herd(W.compaction(), 0.30)
    g64, g32 = pd.PD(herd, precision=0), pd.PD(herd, precision=1)
    f64, f32 = g64.forces(pd.TERM_ALL), g32.forces(pd.TERM_ALL)
    scale = max(np.abs(f64[0]).max(), np.abs(f64[1]).max())
    res["herded_stress_case"] = {
        "nodes": herd.n_nodes,
        "force_rel_err_fp32": float(max(np.abs(f32[0] - f64[0]).max(), np.abs(f32[1] - f64[1]).max()) / scale)}
    return res


def timed_steps(g, torch, steps):
    """steps/s of exactly `steps` steps of context g (the stream drained on
    both sides), and the candidate-list rebuilds among them."""
    torch.cuda.synchronize()
    r0 = g.sizes()["list_rebuilds"]
    t0 = time.perf_counter()
    g.step(steps)  # returns after the stream is drained
    torch.cuda.synchronize()
    return steps / (time.perf_counter() - t0), g.sizes()["list_rebuilds"] - r0


def step_kernel_name(tuning: dict, precision: int) -> str:
    """The step kernel a tuning launches (list mode: with or without the pass
    of walls and contact candidates before it)."""
    r = "double" if precision == 0 else "float"
    if tuning.get("wall_pass") and tuning.get("skin_factor", 0.0) > 0.0:
        return f"k_force_wp<{r},{tuning['lanes_per_node']}>"
    if tuning.get("skin_factor", 0.0) > 0.0:
        return f"k_force<{r},M_STEP,list,{tuning['lanes_per_node']}>"
    return f"k_force<{r},M_STEP>"


def force_roofline(g, kernel_steps, precision, workload):
    """Roofline of the step kernel: algorithmic bytes per launch over its
    mean duration in graph replays (HIP events on the library's stream).
    With the pass of walls and contact candidates, that pass is a launch of
    its own before each step kernel (kernels_ms.pass): inside ms_per_step,
    outside this kernel's time."""
    sizes = g.sizes()
    tun = g.tuning()
    kt = g.time_kernels(kernel_steps)
    ms = kt["force"][0]
    fb = BYTES_PER_NODE[precision] * sizes["nodes"] + BYTES_PER_BOND * sizes["bonds"]
    ach = fb / (ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": step_kernel_name(tun, precision), "achieved": ach,
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
            "traffic": measured_traffic("force", workload, tun),
            "bytes_per_launch": fb, "mean_launch_ms": ms,
            "bytes_per_node": BYTES_PER_NODE[precision], "bytes_per_directed_bond": BYTES_PER_BOND,
            "timed_launches": kt["force"][1], "pass_ms": kt["pass"][0]}, kt


def headline(pd, W, torch, args, prob):
    """The 64 batched settling aggregates (6.4M nodes) in plain FP64: the
    library's autotuner, W warmup steps and one untimed pass of K steps
    (captures the K-step replay), then exactly K timed steps; five more
    windows of K steps for the spread; the force kernel's roofline."""
    g = pd.PD(prob, precision=0)
    sizes = g.sizes()
    g.step(min(args.warmup, 20) if args.warmup > 0 else 0)
    t0 = time.perf_counter()
    if args.tuning:
        g.set_tuning(**parse_tuning(args.tuning))
    else:
        g.autotune(10)
    t_tune = time.perf_counter() - t0
    if args.warmup > 0:
        g.step(args.warmup)
    g.step(args.steps)
    sps, rebuilds = timed_steps(g, torch, args.steps)
    rep = sorted(timed_steps(g, torch, args.steps)[0] for _ in range(5))
    roof, kt = force_roofline(g, args.kernel_steps, 0, "batched_64_fp64")
    n_pairs = sizes["bonds"] // 2
    out = {
        "metric": "PD bond interactions/s (plain FP64, 64 batched settling aggregates)",
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
        "data": "synthetic (seeded aggregates, lattice nodes, RSA placement)",
        "config": {"workload": "batched_64", "aggregates": prob.n_aggregates,
                   "particles": prob.n_particles, "nodes": sizes["nodes"],
                   "directed_bonds": sizes["bonds"], "unordered_bonds": n_pairs, "dt": prob.dt,
                   "gravity": prob.gravity[1], "precision": "fp64", "tuning": g.tuning(),
                   "autotune_s": t_tune},
        "roofline": roof,
        "kernels_ms": {k: v[0] for k, v in kt.items()},
        "kernel_launches_per_step": {k: v[1] / args.kernel_steps for k, v in kt.items()},
        "list_rebuilds_in_timed_steps": rebuilds,
        "repeats": {"n": 5, "steps_each": args.steps, "steps_per_s_median": rep[2],
                    "steps_per_s_min": rep[0], "steps_per_s_max": rep[4]},
        "bond_evaluations_per_s": sizes["bonds"] * sps,
    }
    del g
    return out


def settling_leg(pd, W, torch, args):
    """The 30k-node settling bed (100 particles, plain FP64): candidate lists
    with the autotuner's skin, then the cell search every step (skin 0, the
    cell size chosen among 1, 2 and 3 contact radii)."""
    prob = W.settling()
    g = pd.PD(prob)
    sizes = g.sizes()
    n_pairs = sizes["bonds"] // 2
    g.step(100)
    if args.tuning:
        g.set_tuning(**parse_tuning(args.tuning))
    else:
        g.autotune(50)
    steps = args.settling_steps
    g.step(500)
    g.step(steps)
    sps, rebuilds = timed_steps(g, torch, steps)
    rep = sorted(timed_steps(g, torch, max(1, steps // 5))[0] for _ in range(5))
    roof, kt = force_roofline(g, 512, 0, "settling_100")
    tun = g.tuning()
    best0 = None
    for cf in (1.0, 2.0, 3.0):
        g.set_tuning(skin_factor=0.0, cell_factor=cf)
        g.step(50)
        s_cf, _ = timed_steps(g, torch, max(100, steps // 50))
        if best0 is None or s_cf > best0[1]:
            best0 = (cf, s_cf)
    g.set_tuning(skin_factor=0.0, cell_factor=best0[0])
    sps0, _ = timed_steps(g, torch, max(100, steps // 10))
    g.set_tuning(**tun)
    res = {"workload": "settling_100", "nodes": sizes["nodes"], "directed_bonds": sizes["bonds"],
           "steps": steps, "steps_per_s": sps, "bond_interactions_per_s": n_pairs * sps,
           "ms_per_step": 1e3 / sps, "tuning": tun, "roofline": roof,
           "kernels_ms": {k: v[0] for k, v in kt.items()},
           "list_rebuilds_per_1000_steps": 1000.0 * rebuilds / steps,
           "repeats": {"n": 5, "steps_each": max(1, steps // 5), "steps_per_s_median": rep[2],
                       "steps_per_s_min": rep[0], "steps_per_s_max": rep[4]},
           "every_step_search": {"bond_interactions_per_s": n_pairs * sps0, "steps_per_s": sps0,
                                 "cell_factor": best0[0],
                                 "note": "the same step with the cell-key sort and cell search "
                                         "every step (skin 0)"}}
    del g
    return res


def settling_g5000(pd, W, torch, args):
    """The settling bed at the paper's gravity of 5000 m/s^2 (Sec. 7.3):
    after 2 ms of fall the lower particles pile up on the floor, contacts
    are everywhere and the candidate lists go stale every few steps.  Steps/s
    with the lists, rebuilds per 1000 steps, contact pairs per step."""
    prob = W.settling(gravity=-5000.0)
    g = pd.PD(prob)
    sizes = g.sizes()
    n_pairs = sizes["bonds"] // 2
    g.step(100)
    if args.tuning:
        g.set_tuning(**parse_tuning(args.tuning))
    else:
        g.autotune(50)
    g.step(20000)
    steps = max(1000, args.settling_steps // 4)
    # timed without event counting (its atomics slow the step); the contact
    # pairs are counted over the next window of as many steps
    s0 = g.get_state()
    sps, rebuilds = timed_steps(g, torch, steps)
    g.set_state(s0)
    g.set_counting(True)
    c0 = g.counters()
    g.step(steps)
    c1 = g.counters()
    g.set_counting(False)
    res = {"workload": "settling_100_g5000", "gravity": -5000.0, "t_start_ms": 2.0,
           "steps": steps, "steps_per_s": sps, "bond_interactions_per_s": n_pairs * sps,
           "ms_per_step": 1e3 / sps, "tuning": g.tuning(),
           "list_rebuilds_per_1000_steps": 1000.0 * rebuilds / steps,
           "contact_pairs_per_step": float(c1["inter"] - c0["inter"] + c1["self_"] - c0["self_"]) / steps}
    del g
    return res


def batched_fp32(pd, W, torch, steps, prob, tuning_fixed=None):
    """The 64 aggregates with FP32 force arithmetic (FP64 state and break
    decisions): steps/s of the batch, the roofline of its force kernel, and
    the time of the same 64 aggregates run one after another, each in a
    context of its own."""
    g = pd.PD(prob, precision=1)
    g.step(20)
    t0 = time.perf_counter()
    if tuning_fixed:
        g.set_tuning(**tuning_fixed)
        tuning = g.tuning()
    else:
        tuning = g.autotune(10)
    t_tune = time.perf_counter() - t0
    g.step(20)
    g.step(steps)
    sizes = g.sizes()
    sps, _ = timed_steps(g, torch, steps)
    roof, _ = force_roofline(g, 128, 1, "batched_64")
    res = {"workload": "batched_64", "precision": "fp32_force", "aggregates": prob.n_aggregates,
           "nodes": sizes["nodes"], "tuning": tuning, "autotune_s": t_tune,
           "directed_bonds": sizes["bonds"], "steps_per_s": sps,
           "bond_interactions_per_s": sizes["bonds"] // 2 * sps,
           "force_kernel": roof}
    del g
    seq = 0.0
    sub_steps = max(20, steps // 2)
    for a in range(prob.n_aggregates):
        ga = pd.PD(W.subproblem_aggregate(prob, a), precision=1)
        ga.set_tuning(**tuning)
        ga.step(5)
        ga.step(sub_steps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ga.step(sub_steps)
        torch.cuda.synchronize()
        seq += (time.perf_counter() - t0) / sub_steps
        del ga
    res["sequential_ms_per_step"] = 1e3 * seq
    res["batched_ms_per_step"] = 1e3 / sps
    res["speedup_vs_sequential"] = seq * sps
    return res


def modal_excitation(prob, modes, seed, strain_range):
    """u0 of every closure particle in its rigid + modal space: R(theta_p) Phi q
    with seeded q scaled so that the first-order stretch bound sum |q| sigma
    is uniform in strain_range (input generation: the modes are the
    library's)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    sp = prob.meta["shape_of_particle"]
    po = prob.particle_offset
    rho = prob.materials[0].rho
    first = {}
    ux, uy = np.zeros(prob.n_nodes), np.zeros(prob.n_nodes)
    for p in range(prob.n_particles):
        s = int(sp[p])
        sl = slice(po[p], po[p + 1])
        m = rho * prob.vol[sl]
        xy = np.stack([prob.x[sl], prob.y[sl]], axis=1)
        X = xy - (m[:, None] * xy).sum(0) / m.sum()
        if s not in first:
            first[s] = X
        T = first[s]
        th = np.arctan2((m * (T[:, 0] * X[:, 1] - T[:, 1] * X[:, 0])).sum(),
                        (m * (T[:, 0] * X[:, 0] + T[:, 1] * X[:, 1])).sum())
        phi, lam, sig, nm = modes[s]
        q = rng.normal(0, 1, 32) / (1.0 + np.arange(32))
        q[nm:] = 0.0
        q *= rng.uniform(*strain_range) / (np.abs(q) * sig).sum()
        u = np.einsum("nkc,k->nc", phi, q)
        c, sn = np.cos(th), np.sin(th)
        ux[sl] = c * u[:, 0] - sn * u[:, 1]
        uy[sl] = sn * u[:, 0] + c * u[:, 1]
    prob.u0x, prob.u0y = ux, uy
    return prob


def closure(pd, W, torch, steps, train_iters):
    """The learned modal closure on 2000 particles of four fixed shapes
    (disk, plus, ring, L; about 390 nodes each, 781 500 nodes) in a packed
    bed (security disks at 0.85 of the default box scale) under gravity
    (5 000 m/s^2), seeded rigid velocities up to 1 m/s and the top wall
    coming down at 1 m/s: snapshots of a plain run of that settling and
    compaction (from a seeded modal excitation) train each shape's network
    on the GPU; then plain, linear-closure and learned-closure runs from
    another excitation are timed, in the nodal form and in the reduced form
    (rigid + modal state, boundary nodes only), with the closure checked
    against the plain bond force every 100 steps; contacts make particles
    fall back to the plain force during the timed runs."""
    import numpy as np
    mk = lambda: W.closure_bed(vmax=1.0, fill_scale=0.85, gravity=-5000.0, wall_speed=1.0)
    prob = mk()
    sp = prob.meta["shape_of_particle"]
    g = pd.PD(prob)
    t0 = time.perf_counter()
    g.closure_setup(sp)
    t_modes = time.perf_counter() - t0
    modes = {s: g.closure_modes(s) for s in range(4)}
    del g
    strain = (0.01, 0.03)
    train = modal_excitation(mk(), modes, 51, strain)
    g = pd.PD(train)
    g.closure_setup(sp)
    Q, G = [], []
    for _ in range(200):
        g.step(5)
        q, gg = g.closure_snapshot(device=True)
        Q.append(q)
        G.append(gg)
    Q, G = torch.cat(Q), torch.cat(G)
    _, s_of, _ = g.closure_particles()
    rows = torch.from_numpy(np.tile(s_of, len(Q) // len(s_of))).cuda()
    res = {"workload": "closure_2000 (packed bed: gravity 5000 m/s^2, rigid velocities <= 1 m/s, top wall 1 m/s)", "nodes": prob.n_nodes,
           "particles": prob.n_particles, "modes_setup_s": t_modes,
           "snapshots_per_shape": int(len(Q) // 4)}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    params = {}
    losses = {}
    for s in range(4):
        sel = torch.nonzero(rows == s).flatten()
        L = g.closure_train(s, Q[sel], G[sel], iters=train_iters, batch=1024, lr=2e-3, seed=s)
        losses[s] = [float(L[0]), float(L[:50].mean()), float(L[-50:].mean())]
        params[s] = g.closure_get(s)
        res.setdefault("sigma_r_mean", {})[s] = float(params[s][2].mean())
        res.setdefault("samples", {})[s] = int(sel.numel())
    torch.cuda.synchronize()
    res["train_s"] = time.perf_counter() - t0
    res["train_loss_first_head_last"] = losses
    # held-out snapshots: learned vs linear closure against the plain force
    test = modal_excitation(mk(), modes, 52, strain)
    gt = pd.PD(test)
    gt.closure_setup(sp)
    for s in range(4):
        gt.closure_load(s, *params[s])
    e_n = e_l = n2 = 0.0
    for _ in range(20):
        gt.step(10)
        q, gg = gt.closure_snapshot(device=True)
        for s in range(4):
            sel = torch.from_numpy(np.nonzero(s_of == s)[0]).cuda()
            qs, gs = q[sel], gg[sel]
            gn = gt.closure_forward(s, qs)
            lam = torch.from_numpy(modes[s][1]).cuda()
            e_n += float(((gn - gs) ** 2).sum())
            e_l += float(((-lam * qs - gs) ** 2).sum())
            n2 += float((gs ** 2).sum())
    res["heldout_modal_force_err"] = {"learned": (e_n / n2) ** 0.5, "linear": (e_l / n2) ** 0.5}
    del gt
    # timed runs from the held-out excitation
    R = pd.CLOSURE_REDUCED
    for name, mode in (("plain", 0), ("linear", 1), ("learned", 2), ("reduced_linear", 1 | R),
                       ("reduced_learned", 2 | R)):
        gr = pd.PD(modal_excitation(mk(), modes, 52, strain))
        gr.closure_setup(sp)
        for s in range(4):
            gr.closure_load(s, *params[s])
        gr.closure_enable(mode)
        gr.step(100)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        gr.step(steps)
        torch.cuda.synchronize()
        sps = steps / (time.perf_counter() - t0)
        st = gr.closure_stats()
        n_pairs = gr.sizes()["bonds"] // 2
        res[name] = {"steps_per_s": sps, "bond_interactions_per_s": n_pairs * sps,
                     "list_rebuilds": gr.sizes()["list_rebuilds"],
                     "active": st["active"], "fallbacks": st["fallbacks"], "checks": st["checks"],
                     "check_err": st["err"] if mode else None,
                     "check_err_linear": st["err_linear"] if mode else None}
        del gr
    for name in ("linear", "learned", "reduced_linear", "reduced_learned"):
        res[f"speedup_{name}_vs_plain"] = res[name]["steps_per_s"] / res["plain"]["steps_per_s"]
    return res


def fragmentation(pd, W, torch, micro_s):
    """The notched square of side 1 mm struck from above and below by two
    1 x 0.5 mm rectangles at 20 m/s (4000 nodes, M1 material, h = 25 um,
    horizon 3h, dt = 2 ns), for the two toughness values of the paper: the
    child particles of the square (components of its intact-bond graph
    holding at least 1% of its nodes), all components, broken bonds and the
    step rate, after micro_s microseconds."""
    import numpy as np
    res = {"workload": "notched_impact (side 1 mm, 20 m/s, h = 25 um)", "t_us": micro_s}
    for Gc in (135.0, 13.5):
        prob = W.notched_impact(Gc=Gc, n_side=40, dt=2e-9)
        g = pd.PD(prob)
        steps = int(round(micro_s * 1e-6 / prob.dt))
        n_a = int(prob.particle_offset[1])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        g.step(steps)
        torch.cuda.synchronize()
        sps = steps / (time.perf_counter() - t0)
        lab, cnt, nc = g.fragments(min_nodes=max(1, n_a // 100))
        sizes = np.bincount(lab[:n_a], minlength=n_a)
        big = sorted((int(v) for v in sizes[sizes > 0]), reverse=True)
        res[f"Gc_{Gc:g}"] = {"children_of_square": int(cnt[0]),
                             "children_of_rectangles": [int(cnt[1]), int(cnt[2])],
                             "components_all": int(nc), "largest_pieces_of_square": big[:4],
                             "broken_directed": int(g.damage()[1]), "steps": steps,
                             "steps_per_s": sps}
        del g
    return res


def settle_shapes(pd, W, torch, micro_s, every_us):
    """Settling of beds of one shape each from jammed security disks (perturbed
    disks, squares, plus shapes, rings; 25 x 50 mm container, the parameters
    of Sec. 7.3: eps = 0.5 mm, h = eps/8, R_c = eps/5, mu = r_d = 0.8,
    5000 m/s^2, dt = 70 ns, FP64): packing of the security disks, the bed's
    volume fraction at the start and after micro_s microseconds (particle area
    over width x bed height, and the same with rings counted as full disks),
    its kinetic energy series, broken bonds and the step rate."""
    import numpy as np
    res = {"workload": "jammed_settling (25 x 50 mm, eps = 0.5 mm, h = eps/8)", "t_us": micro_s}
    for shape in W.SETTLE_SHAPES:
        prob = W.jammed_settling(shape)
        g = pd.PD(prob)
        width = prob.box[0, 1] - prob.box[0, 0]
        sizes = g.sizes()

        def frac(uy):
            H = float(np.max(prob.y + uy))
            return (float(prob.vol.sum()) / (width * H), prob.meta["filled_area"] / (width * H), H)

        phi0 = frac(np.zeros(prob.n_nodes))
        g.step(20)
        tun = g.autotune(50)
        every = int(round(every_us * 1e-6 / prob.dt))
        n_chunks = max(1, int(round(micro_s / every_us)))
        ke = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(n_chunks):
            g.step(every)
            s = g.get_state()
            ke.append(float(0.5 * 1200.0 * np.sum(prob.vol * (s["vx"] ** 2 + s["vy"] ** 2))))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        phi1 = frac(s["uy"])
        res[shape] = {"particles": prob.n_particles, "nodes": sizes["nodes"],
                      "directed_bonds": sizes["bonds"], "packing": prob.meta["packing"],
                      "phi_start": phi0[0], "phi_end": phi1[0],
                      "phi_filled_start": phi0[1], "phi_filled_end": phi1[1],
                      "bed_height_mm_end": 1e3 * phi1[2], "kinetic_energy_series": ke,
                      "broken_directed": int(g.damage()[1]), "tuning": tun,
                      "steps": every * n_chunks, "steps_per_s": every * n_chunks / wall}
        del g
    return res


def hbm_probe(pd, torch, mib=1024, reps=10):
    """The library's streaming probe (hand-written read-only and copy
    kernels) over buffers of `mib` MiB, four times the 256 MB on-package
    cache: the device's achievable bandwidth, and the known traffic that
    scales a profiler's byte counters (a read pass moves `mib` MiB, a copy
    twice that)."""
    n = mib * 1024 * 1024
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    pd.stream_probe(0, src, dst, 2)
    pd.stream_probe(1, src, dst, 2)
    ms_r = pd.stream_probe(0, src, dst, reps)
    ms_c = pd.stream_probe(1, src, dst, reps)
    del src, dst
    torch.cuda.empty_cache()
    return {"bytes": n, "passes": reps,
            "read_ms": ms_r, "read_GBs": n / (ms_r * 1e-3) / 1e9,
            "copy_ms": ms_c, "copy_GBs": 2 * n / (ms_c * 1e-3) / 1e9}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200,
                    help="timed steps of the headline (the 64 batched aggregates, FP64)")
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--kernel-steps", type=int, default=128)
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--settling-steps", type=int, default=20000)
    ap.add_argument("--split-steps", type=int, default=600000,
                    help="most steps of the 0.1 m/s compaction run (it stops 30k steps after "
                         "the first break)")
    ap.add_argument("--batched-steps", type=int, default=200)
    ap.add_argument("--closure-steps", type=int, default=3000)
    ap.add_argument("--train-iters", type=int, default=2000)
    ap.add_argument("--impact-us", type=float, default=40.0)
    ap.add_argument("--tuning", default="",
                    help="fixed tuning instead of the autotuner for the run's contexts, e.g. "
                         "block_nodes=128,use_lds=1,skin_factor=0.5 (profiling runs)")
    ap.add_argument("--settle-us", type=float, default=10000.0)
    ap.add_argument("--settle-every-us", type=float, default=1000.0)
    ap.add_argument("--workload", choices=("batched", "settling", "settling_g5000", "compaction",
                                           "batched_fp32",
                                           "closure", "fragmentation", "settle_shapes"),
                    default="batched",
                    help="batched: the headline line (plus the secondary legs unless "
                         "--no-variants); any other: only that leg")
    ap.add_argument("--hbm-probe", action="store_true",
                    help="only run the streaming probe (1 GiB read-only and copy passes): "
                         "achievable bandwidth and profiler counter calibration")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the step loop has "
              "no multi-GPU form (its sharding is a design only)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2108_07212_amd import pd
    from paper_2108_07212_amd import workloads as W

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(3)
    torch.cuda.set_device(0)
    fixed = parse_tuning(args.tuning) if args.tuning else None
    if args.hbm_probe:
        print(json.dumps({"hbm_probe": hbm_probe(pd, torch)}), flush=True)
        return
    legs = {
        "settling": lambda: settling_leg(pd, W, torch, args),
        "settling_g5000": lambda: settling_g5000(pd, W, torch, args),
        "compaction": lambda: precision_split(pd, W, torch, args.split_steps),
        "batched_fp32": lambda: batched_fp32(pd, W, torch, args.batched_steps,
                                             W.batched(precision=1), fixed),
        "closure": lambda: closure(pd, W, torch, args.closure_steps, args.train_iters),
        "fragmentation": lambda: fragmentation(pd, W, torch, args.impact_us),
        "settle_shapes": lambda: settle_shapes(pd, W, torch, args.settle_us, args.settle_every_us),
    }
    if args.workload != "batched":
        print(json.dumps({args.workload: legs[args.workload]()}), flush=True)
        return
    def progress(what, t0):
        # one line per finished leg on stderr (the JSON line stays alone on stdout)
        print(f"[bench] {what} done in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    prob = W.batched(precision=0)
    out = headline(pd, W, torch, args, prob)
    out["hbm_measured"] = hbm_probe(pd, torch)
    progress("headline", t0)
    if not args.no_variants:
        for key, run in (("settling_100", legs["settling"]), ("settling_g5000", legs["settling_g5000"]),
                         ("precision_split", legs["compaction"]),
                         ("batched_fp32", lambda: batched_fp32(pd, W, torch, args.batched_steps, prob,
                                                               fixed)),
                         ("closure", legs["closure"]), ("fragmentation", legs["fragmentation"]),
                         ("settle_shapes", legs["settle_shapes"])):
            t0 = time.perf_counter()
            out[key] = run()
            progress(key, t0)
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        # one aggregate of the same batch, of about the batch's mean size
        sizes = np.diff(prob.particle_offset)
        agg_nodes = np.bincount(prob.particle_aggregate, weights=sizes)
        k = int(np.argmin(np.abs(agg_nodes - agg_nodes.mean())))
        out["cpu_baseline"] = cpu_baseline(
            W.subproblem_aggregate(prob, k), args.cpu_seconds,
            f"aggregate {k} of the 64 batched settling aggregates (of mean size)")
        progress("cpu_baseline", t0)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
