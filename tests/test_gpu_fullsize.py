"""Parity at the benchmark's full sizes, in the launch configuration the
benchmark times for each workload (the headline and the batched run: 128
nodes per workgroup, LDS staging, candidate lists with skin 0.5, graph
replays of 64 steps; the precision split's bed: two lanes per node, as its
autotuner picks; its stress case and the closure: the library's default
tuning).

* The settling bed of 100 particles (30 075 nodes, 594 576 directed bonds),
  with seeded nodal noise (displacements of 2 um, velocities of 0.05 m/s;
  from rest every bond force stays exactly zero for many steps): the whole
  problem against the FP64 oracle -- reference bonds and contact sets
  bit-exact, per-term forces to 1e-12, a 200-step trajectory to 1e-9 (also
  in the two tunings the autotuner has picked for the settling leg).
* The settling bed under the paper's 5 000 m/s^2 (the contact-active
  leg): the oracle falls for 2 ms (20 100 steps), then ten windows of 100
  steps, each started by the library from the oracle's state, in the
  autotuner's tuning there (four lanes per node) and with one lane and the
  pass: trajectories to 1e-9 and broken bonds bit-exact at each window's
  end, with list rebuilds and contact inside the windows.
* The FP32 / FP64 precision split's bed (509 particles from the jammed
  start, 178k nodes) at its start in that leg's tuning, and its stress case
  (500 particles herded into one another, 245k nodes), whole against the
  oracle.
* The closure workload of 2 000 particles, reduced and nodal forms, whole
  against the oracle's closure steppers.
* The notched impact at its benchmark resolution, whole against the oracle
  through first contact and the bulk of the fractures.
* The four jammed shape beds of the settling study, whole against the oracle.
* The 64 batched aggregates (6.4 M nodes, 130 M directed bonds), FP64 and
  FP32 forces each with one lane per node and the pass of walls and contact
  candidates (the autotuner's pick at this size in both precisions), FP64
  with one lane and FP32 with two without the pass, with the
  same noise and seeded rigid particle velocities: aggregates never
  interact, so three sampled aggregates (the smallest, the largest, the
  first) are each run by the oracle alone and compared with their slice of
  the batched run: bonds bit-exact; FP64 100-step trajectory to 1e-9; the
  FP32-force mode (the benchmark's) 100-step trajectory to 1e-5 (FP32 force
  rounding, about 3e-7 of the largest force per step, adds up over the
  steps; measured 1e-7 to 7e-7) and, at the oracle's final state (loaded
  into the aggregate alone), per-term FP32 forces to 2e-5, the FP32 force
  bar.
"""
import sys

import numpy as np
import pytest

from oracle import Oracle
from paper_2108_07212_amd import workloads as W

pytestmark = pytest.mark.gpu

BENCH_TUNING = dict(block_nodes=128, use_lds=1, use_graph=1, skin_factor=0.5)
TERMS = (1, 2, 4, 8, 16)


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pdmod():
    import torch
    assert torch.cuda.is_available(), "GPU test without a GPU"
    from paper_2108_07212_amd import pd
    pd.load_library()
    return pd


def _relerr(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def test_settling_100_full_size(pdmod):
    _say("case: settling bed, full size, benchmark tuning")
    prob = W.perturb(W.settling(), 9, du=2e-6, dv=0.05)
    g = pdmod.PD(prob)
    g.set_tuning(**BENCH_TUNING)
    o = Oracle(prob, contact_mode=1, n_threads=16)
    rg, cg = g.bonds()
    ro, co = o.bonds()
    assert np.array_equal(rg, ro) and np.array_equal(cg, co)
    assert len(cg) == 594576
    for t in TERMS:
        gx, gy = g.forces(t)
        ox, oy = o.forces(t)
        scale = max(np.abs(ox).max(), np.abs(oy).max())
        if scale == 0.0:
            assert np.abs(gx).max() == 0.0 and np.abs(gy).max() == 0.0, t
            continue
        assert max(np.abs(gx - ox).max(), np.abs(gy - oy).max()) <= 1e-12 * scale, t
    assert np.abs(o.forces(1)[0]).max() > 0.0  # the noise strains the bonds
    assert g.step(200, check=False) == o.step(200)
    sg, so = g.get_state(), o.get_state()
    for k in ("ux", "uy", "vx", "vy"):
        assert _relerr(sg[k], so[k]) <= 1e-9, k
    assert np.array_equal(sg["broken"], so["broken"])
    cg_ = g.contacts()
    co_ = o.contacts()
    assert np.array_equal(cg_[0], co_[0]) and np.array_equal(cg_[1], co_[1])
    # the settling leg's own picks of the autotuner (four lanes per node)
    for tun in (dict(block_nodes=64, skin_factor=1.0), dict(block_nodes=128, skin_factor=2.0)):
        h = pdmod.PD(prob)
        h.set_tuning(**dict(BENCH_TUNING, **tun), lanes_per_node=4, wall_pass=0)
        assert h.step(200, check=False) == 0
        sh = h.get_state()
        for k in ("ux", "uy", "vx", "vy"):
            assert _relerr(sh[k], so[k]) <= 1e-9, (tun, k)
        assert np.array_equal(sh["broken"], so["broken"]), tun
        del h


# the contact-active leg's tunings: the autotuner's pick there, and one lane
# per node with the pass
G5000_TUNINGS = (dict(block_nodes=64, use_lds=1, use_graph=1, skin_factor=1.0, lanes_per_node=4,
                      wall_pass=0),
                 dict(block_nodes=128, use_lds=1, use_graph=1, skin_factor=0.5, lanes_per_node=1,
                      wall_pass=1))


def test_settling_g5000_window_full_size(pdmod):
    _say("case: settling bed under 5000 m/s^2, full size, windows from the oracle at t = 2 ms")
    prob = W.settling(gravity=-5000.0)
    o = Oracle(prob, contact_mode=1, n_threads=16)
    for k in range(10):
        assert o.step(2010) == 0
        _say(f"  oracle fall: {(k + 1) * 2010} steps")
    runs = []
    for tun in G5000_TUNINGS:
        g = pdmod.PD(prob)
        g.set_tuning(**tun)
        g.set_counting(True)
        runs.append(g)
    so = o.get_state()
    for k in range(10):
        start = so
        assert o.step(100) == 0
        so = o.get_state()
        for tun, g in zip(G5000_TUNINGS, runs):
            g.set_state(start)
            assert g.step(100, check=False) == 0
            sg = g.get_state()
            err = max(_relerr(sg[key], so[key]) for key in ("ux", "uy", "vx", "vy"))
            _say(f"  segment {k}, {tun['lanes_per_node']} lane(s), pass {tun['wall_pass']}: {err:.2e}")
            assert err <= 1e-9, (k, tun, err)
            assert np.array_equal(sg["broken"], so["broken"]), (k, tun)
    for g in runs:
        # the lists went stale inside the segments, and contact acted
        assert g.sizes()["list_rebuilds"] > 2 * 10
        assert g.counters()["inter"] > 0
    assert o.counters()["inter"] > 0


def test_jammed_compaction_full_size(pdmod):
    """The precision-split leg's bed (509 particles from the jammed start of
    Sec. 7.1, 178k nodes, top wall at 1 m/s) at its start, with seeded nodal
    noise, in that leg's autotuned tuning (two lanes per node): FP64 against
    the oracle -- bonds bit-exact, per-term forces to 1e-12, 100 steps to
    1e-9, broken bonds equal; FP32 forces per term to 2e-5."""
    _say("case: jammed compaction, full size, the precision split's start")
    prob = W.perturb(W.jammed_compaction(wall_speed=1.0), 10, du=2e-6, dv=0.05)
    tun = dict(BENCH_TUNING, lanes_per_node=2, wall_pass=0)
    o = Oracle(prob, contact_mode=1, n_threads=16)
    g = pdmod.PD(prob, precision=W.PREC_FP64)
    g.set_tuning(**tun)
    g32 = pdmod.PD(prob, precision=W.PREC_FP32_FORCE)
    g32.set_tuning(**tun)
    rg, cg = g.bonds()
    ro, co = o.bonds()
    assert np.array_equal(rg, ro) and np.array_equal(cg, co)
    for t in TERMS:
        ox, oy = o.forces(t)
        scale = max(np.abs(ox).max(), np.abs(oy).max())
        if scale == 0.0:
            continue
        for gg, tol in ((g, 1e-12), (g32, 2e-5)):
            gx, gy = gg.forces(t)
            e = max(np.abs(gx - ox).max(), np.abs(gy - oy).max()) / scale
            _say(f"    term {t}: {e:.2e}")
            assert e <= tol, (t, tol, e)
    assert np.abs(o.forces(1)[0]).max() > 0.0  # the noise strains the bonds
    assert g.step(100, check=False) == o.step(100)
    sg, so = g.get_state(), o.get_state()
    for k in ("ux", "uy", "vx", "vy"):
        e = _relerr(sg[k], so[k])
        _say(f"    {k}: {e:.2e}")
        assert e <= 1e-9, k
    assert np.array_equal(sg["broken"], so["broken"])


def test_compaction_500_full_size(pdmod):
    """The precision-split leg's stress case (500 particles, about 245k
    nodes, herded into one another at t = 0, top wall at 0.1 m/s) in the
    library's default tuning: FP64 against the oracle -- bonds and contact
    sets bit-exact, per-term forces to 1e-12, 100 steps to 1e-9, broken bonds
    equal.  The FP32-force mode: per-term forces against the oracle to 2e-5
    at the start and at its own final state; its 100-step trajectory to
    1e-3 only: this packed start amplifies any perturbation (about 2 million
    contact evaluations in 100 steps, a third of them at the friction law's
    stick/slip threshold) -- the FP64 oracle itself, with its start
    accelerations perturbed by 3e-7 of their largest value, moves its
    velocities by 1.6e-3 to 2.5e-3 in 100 steps; FP32 forces measured 1.5e-4
    and 1.7e-4 against the oracle, displacements 2e-8."""
    _say("case: compaction 500, full size, packed start")
    prob = W.herd(W.compaction(), 0.30)
    prob.top_wall_speed = np.array([0.1])
    o = Oracle(prob, contact_mode=1, n_threads=16)
    g = pdmod.PD(prob, precision=W.PREC_FP64)
    rg, cg = g.bonds()
    ro, co = o.bonds()
    assert np.array_equal(rg, ro) and np.array_equal(cg, co)
    for t in TERMS:
        gx, gy = g.forces(t)
        ox, oy = o.forces(t)
        scale = max(np.abs(ox).max(), np.abs(oy).max())
        if scale == 0.0:
            continue
        assert max(np.abs(gx - ox).max(), np.abs(gy - oy).max()) <= 1e-12 * scale, t
    c0 = o.contacts()
    assert len(c0[0]) > 0  # packed: contacts from the start
    gc = g.contacts()
    assert np.array_equal(gc[0], c0[0]) and np.array_equal(gc[1], c0[1])
    g32 = pdmod.PD(prob, precision=W.PREC_FP32_FORCE)

    def fp32_forces(label):
        for t in TERMS:
            gx, gy = g32.forces(t)
            ox, oy = o.forces(t)
            scale = max(np.abs(ox).max(), np.abs(oy).max())
            if scale == 0.0:
                continue
            e = max(np.abs(gx - ox).max(), np.abs(gy - oy).max()) / scale
            _say(f"    fp32 forces {label} term {t}: {e:.2e}")
            assert e < 2e-5, (label, t, e)

    fp32_forces("start")
    steps = 100
    assert g.step(steps, check=False) == 0 and g32.step(steps, check=False) == 0
    assert o.step(steps) == 0
    so = o.get_state()
    for gg, tol in ((g, 1e-9), (g32, 1e-3)):
        sg = gg.get_state()
        for k in ("ux", "uy", "vx", "vy"):
            e = _relerr(sg[k], so[k])
            _say(f"    {k}: {e:.2e}")
            assert e <= tol, (k, e)
    assert np.array_equal(g.get_state()["broken"], so["broken"])
    # the FP32 forces at the oracle's final state (the library is put there)
    g32.set_state(so)
    fp32_forces("final")


def _aggregate_ranges(prob):
    pa = np.asarray(prob.particle_aggregate)
    po = np.asarray(prob.particle_offset)
    out = []
    for a in range(prob.n_aggregates):
        sel = np.nonzero(pa == a)[0]
        out.append((int(po[sel[0]]), int(po[sel[-1] + 1])))
    return out


def test_batched_64_full_size_sampled(pdmod):
    _say("case: 64 batched aggregates, full size, benchmark tuning, sampled aggregates")
    prob = W.perturb(W.particle_velocities(W.batched(), 7, 3.0), 8, du=2e-6, dv=0.05)
    ranges = _aggregate_ranges(prob)
    sizes = [n1 - n0 for n0, n1 in ranges]
    sample = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 0})
    steps = 100
    runs = {}
    # (precision, lanes per node, the pass of walls and contact candidates):
    # one lane with the pass is what the autotuner picks at this size in both
    # precisions; two lanes without it for the FP32-force mode
    configs = ((W.PREC_FP64, 1, 1), (W.PREC_FP64, 1, 0), (W.PREC_FP32_FORCE, 1, 1),
               (W.PREC_FP32_FORCE, 2, 0))
    for prec, lanes, wp in configs:
        _say(f"  library run: precision {prec}, {lanes} lane(s), pass {wp}")
        g = pdmod.PD(prob, precision=prec)
        g.set_tuning(**BENCH_TUNING, lanes_per_node=lanes, wall_pass=wp)
        if prec == W.PREC_FP64 and wp == 0:
            rg, cg = g.bonds()
        g.set_counting(True)
        assert g.step(steps, check=False) == 0
        runs[prec, lanes, wp] = (g.get_state(), g.counters()["inter"])
        del g
    for a in sample:
        _say(f"  aggregate {a}: nodes {sizes[a]}")
        n0, n1 = ranges[a]
        sub = W.subproblem_aggregate(prob, a)
        o = Oracle(sub, contact_mode=1, n_threads=16)
        ro, co = o.bonds()
        assert np.array_equal(cg[rg[n0]:rg[n1]] - n0, co), a
        assert np.array_equal(rg[n0:n1 + 1] - rg[n0], ro), a
        assert o.step(steps) == 0
        so = o.get_state()
        for prec, lanes, wp in configs:
            tol = 1e-9 if prec == W.PREC_FP64 else 1e-5
            sg = runs[prec, lanes, wp][0]
            for k in ("ux", "uy", "vx", "vy"):
                e = _relerr(sg[k][n0:n1], so[k])
                _say(f"    prec {prec} lanes {lanes} pass {wp} {k}: {e:.2e}")
                assert e <= tol, (a, prec, lanes, wp, k, e)
            assert np.array_equal(sg["broken"][cg_slice(rg, n0, n1)], so["broken"]), (a, prec, lanes, wp)
        # FP32 forces at the oracle's final state: the aggregate alone in the
        # library (aggregates never interact), FP32 forces, put at that state
        ga = pdmod.PD(sub, precision=W.PREC_FP32_FORCE)
        ga.set_tuning(**BENCH_TUNING, lanes_per_node=2)
        ga.set_state(so)
        for t in TERMS:
            ox, oy = o.forces(t)
            gx, gy = ga.forces(t)
            scale = max(np.abs(ox).max(), np.abs(oy).max())
            if scale == 0.0:
                continue
            e = max(np.abs(gx - ox).max(), np.abs(gy - oy).max()) / scale
            _say(f"    fp32 forces term {t}: {e:.2e}")
            assert e < 2e-5, (a, t, e)
        assert np.abs(ga.forces(1)[0]).max() > 0.0  # bond forces act
        del ga


def cg_slice(rg, n0, n1):
    return slice(int(rg[n0]), int(rg[n1]))


def test_closure_2000_full_size_reduced(pdmod):
    """The closure workload (2 000 particles of four shapes, 781 500 nodes,
    seeded rigid velocities) started in each particle's rigid + modal space,
    against the oracle's closure steppers over 20 steps: the reduced form
    with the linear closure to 1e-9 and with seeded network weights to 1e-6,
    the nodal form with the linear closure to 1e-9 (the bars of the
    small-bed tests)."""
    import os
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import test_gpu_closure as TC
    from oracle import closure as CL
    _say("case: closure 2000 particles, full size, reduced form")
    base = W.closure_bed(vmax=0.5)
    o0 = Oracle(base, contact_mode=1, n_threads=16)
    modes = TC.oracle_modes(base, o0)
    s0 = float(o0.constants()["s0"][0])
    del o0
    S = len(modes)
    steps = 20
    learned = {s: TC.rand_params(70 + s) for s in modes}
    for reduced, mode, tol, params in ((True, 1, 1e-9, None), (True, 2, 1e-6, learned),
                                       (False, 1, 1e-9, None)):
        prob = TC.modal_deformation(W.closure_bed(vmax=0.5), modes, 69, (0.05, 0.3), s0)
        sp = prob.meta["shape_of_particle"]
        g = pdmod.PD(prob)
        g.closure_setup(sp, gate_frac=0.5, tau_c=[TC.BIG] * S, check_every=0)
        TC.load_modes(g, modes)
        sq = sr = None
        if params is not None:
            qs = TC.initial_q(prob, modes)
            sq = {s: np.sqrt((qs[s] ** 2).mean(0)).astype(np.float32).astype(np.float64) for s in modes}
            sr = {s: (3e-2 * modes[s][1] * sq[s]).astype(np.float32).astype(np.float64) for s in modes}
            for s in modes:
                g.closure_load(s, params[s], sq[s], sr[s])
        g.closure_enable(mode | (pdmod.CLOSURE_REDUCED if reduced else 0))
        o = Oracle(prob, contact_mode=1, n_threads=16)
        Stepper = CL.ReducedStepper if reduced else CL.ClosureStepper
        st = Stepper(o, prob, sp, modes, [s0] * S, [TC.BIG] * S, 0.5, params=params,
                     sig_q=sq, sig_r=sr)
        off = []
        for _ in range(steps):
            off += st.step()
        assert g.step(steps, check=False) == 0
        a, b = g.get_state(), o.get_state()
        for k in ("ux", "uy", "vx", "vy"):
            e = _relerr(a[k], b[k])
            _say(f"    {'reduced' if reduced else 'nodal'} mode {mode} {k}: {e:.2e}")
            assert e < tol, (mode, k, e)
        assert g.closure_stats()["fallbacks"] == len(off)
        del g, o, st


@pytest.mark.parametrize("Gc", [135.0, 13.5])
def test_notched_impact_full_size(pdmod, Gc):
    """The three-particle impact at the benchmark's resolution (1 mm squares
    of 40 x 40 nodes, 20 m/s, dt = 2 ns), whole against the oracle through
    first contact (about step 600) and the bulk of the fractures: states to
    1e-9 and broken flags bit-exact every 250 steps up to step 1 250, then
    the fragment labels and the child counts from the same broken flags."""
    from oracle import child_counts, components
    _say(f"case: notched impact full size Gc={Gc}")
    prob = W.notched_impact(Gc=Gc, n_side=40, dt=2e-9)
    g, o = pdmod.PD(prob), Oracle(prob, contact_mode=1, n_threads=16)
    row, col = o.bonds()
    for k in range(5):
        assert g.step(250, check=False) == o.step(250)
        sg, so = g.get_state(), o.get_state()
        eu = max(_relerr(sg["ux"], so["ux"]), _relerr(sg["uy"], so["uy"]))
        ev = max(_relerr(sg["vx"], so["vx"]), _relerr(sg["vy"], so["vy"]))
        nb = int(so["broken"].sum())
        _say(f"    step {250 * (k + 1)}: eu={eu:.2e} ev={ev:.2e} broken={nb}")
        assert eu <= 1e-9 and ev <= 1e-9, (k, eu, ev)
        assert np.array_equal(sg["broken"], so["broken"]), k
    assert nb > 1000
    ref = components(row, col, so["broken"], prob.n_nodes)
    lab, cnt, nc = g.fragments(min_nodes=1)
    assert np.array_equal(lab, ref)
    assert np.array_equal(cnt, child_counts(ref, prob.particle_offset, 1))


@pytest.mark.parametrize("shape", ["pdisk", "square", "plus", "ring"])
def test_jammed_settling_full_size(pdmod, shape):
    """The four shape beds of the benchmark (25 x 50 mm, jammed security-disk
    start, 70k-142k nodes) with seeded rigid velocities in [-3, 3]^2 m/s plus
    2 m/s downward and the nodal noise above: whole against the oracle over
    300 steps, through the first contacts -- bond sets bit-exact, states to
    1e-9, broken flags bit-exact."""
    _say(f"case: jammed settling full size {shape}")
    prob = W.perturb(W.particle_velocities(W.jammed_settling(shape), 9, 3.0), 10, du=2e-6, dv=0.05)
    prob.v0y = prob.v0y - 2.0
    g, o = pdmod.PD(prob), Oracle(prob, contact_mode=1, n_threads=16)
    # bond sets bit-exact (the annulus's nodes lie on radial lines through the
    # hole's vertices, so bonds run along the cusps' bisector rays)
    rg, cg = g.bonds()
    ro, co = o.bonds()
    assert np.array_equal(rg, ro) and np.array_equal(cg, co)
    g.set_counting(True)
    assert g.step(300, check=False) == o.step(300)
    sg, so = g.get_state(), o.get_state()
    eu = max(_relerr(sg["ux"], so["ux"]), _relerr(sg["uy"], so["uy"]))
    ev = max(_relerr(sg["vx"], so["vx"]), _relerr(sg["vy"], so["vy"]))
    _say(f"    nodes {prob.n_nodes}: eu={eu:.2e} ev={ev:.2e} contacts={g.counters()['inter']}")
    assert eu <= 1e-9 and ev <= 1e-9, (eu, ev)
    assert np.array_equal(sg["broken"], so["broken"])
