"""Parity window of the compaction run with damage (Sec. 7.4): the top wall
driven down at 0.1 m/s through the first bond breaks, on a small bed from
the jammed start of Sec. 7.1 (26 mixed particles, 5 906 nodes, 8 x 8 mm).

The oracle makes its own checkpoint: the wall at 1 m/s (the paper's
compaction speed) for 18 500 steps, then at 0.1 m/s until its first break.
From its state one to two thousand steps before that break it runs 3 000
steps in segments of 250.  At the start of each segment the library (FP64,
one and four lanes per node; FP32 forces) takes the oracle's state and runs
the segment: FP64 trajectories to 1e-9 and broken bonds bit-exact at its
end (the same bar as for 100-step trajectories; over the whole window the
breaks' release makes rounding differences grow about tenfold per 500
steps, in the oracle as well), the FP32-force mode with the same broken
bonds; the breaks happen inside the window.  At the window's end the
FP32-force mode's forces are within 2e-5 of the oracle's.
"""
import sys

import numpy as np
import pytest

from oracle import Oracle
from paper_2108_07212_amd import workloads as W

pytestmark = pytest.mark.gpu

TRAJ_TOL = 1e-9


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


def _checkpoint():
    """The oracle's run to just before its first break at 0.1 m/s."""
    fast = W.jammed_compaction(width=8e-3, height=8e-3, mesh_size=2.5e-3, wall_speed=1.0)
    o = Oracle(fast, contact_mode=1, n_threads=16)
    pre = 18500
    assert o.step(pre) == 0
    s = o.get_state()
    assert int(s["broken"].sum()) == 0
    wall = fast.box[0, 3] - 1.0 * pre * fast.dt
    slow = W.restart_with_wall(fast, s, wall, 0.1)
    o = Oracle(slow, contact_mode=1, n_threads=16)
    s["step"] = 0
    o.set_state(s)
    hist = [o.get_state()]
    for _ in range(120):
        assert o.step(1000) == 0
        st = o.get_state()
        if int(st["broken"].sum()) > 0:
            break
        hist.append(st)
    else:
        pytest.fail("no bond broke in 120 000 steps at 0.1 m/s")
    return slow, hist[max(0, len(hist) - 2)]


def test_compaction_window_through_first_breaks(pdmod):
    _say("case: compaction window at 0.1 m/s through the first breaks (oracle checkpoint)")
    prob, ck = _checkpoint()
    _say(f"  window starts at step {ck['step']} of the 0.1 m/s run")
    o = Oracle(prob, contact_mode=1, n_threads=16)
    o.set_state(ck)
    runs = {}
    for lanes in (1, 4):
        g = pdmod.PD(prob)
        g.set_tuning(lanes_per_node=lanes)
        runs[lanes] = g
    g32 = pdmod.PD(prob, precision=W.PREC_FP32_FORCE)
    so = o.get_state()
    for k in range(12):
        start = so
        assert o.step(250) == 0
        so = o.get_state()
        for lanes, g in runs.items():
            g.set_state(start)
            assert g.step(250, check=False) == 0
            sg = g.get_state()
            err = max(_relerr(sg[key], so[key]) for key in ("ux", "uy", "vx", "vy"))
            _say(f"  segment {k}, {lanes} lane(s): max relative error {err:.2e}")
            assert err <= TRAJ_TOL, (k, lanes, err)
            assert np.array_equal(sg["broken"], so["broken"]), (k, lanes)
        g32.set_state(start)
        assert g32.step(250, check=False) == 0
        assert np.array_equal(g32.get_state()["broken"], so["broken"]), k
        _say(f"  {(k + 1) * 250} steps: broken {int(so['broken'].sum())}")
    assert int(so["broken"].sum()) > 0
    assert o.counters()["inter"] > 0
    # FP32 forces at the oracle's state at the window's end
    g32.set_state(so)
    for t in (1, 2, 4, 8):
        gx, gy = g32.forces(t)
        ox, oy = o.forces(t)
        scale = max(np.abs(ox).max(), np.abs(oy).max())
        if scale == 0.0:
            continue
        e = max(np.abs(gx - ox).max(), np.abs(gy - oy).max()) / scale
        assert e < 2e-5, (t, e)
