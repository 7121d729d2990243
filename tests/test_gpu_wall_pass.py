"""The wall pass (tuning wall_pass = 1): the wall forces (Sec. 4.5) of the
nodes near a wall and the contact forces of the nodes with candidates
evaluated in a launch of their own before each list-mode step, the step
kernel reading them.  Beds pressed into a corner of the floor
and the left wall and into the top wall moving down at 2 m/s, against the
oracle (trajectories to 1e-9 through list rebuilds, among them those the
moving wall forces), and against the same run with the walls inside the step
kernel: bit for bit at four lanes per node (the pass sums the four wall
regions in the order of the step kernel's four lanes), within rounding at one
lane."""
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


def _pressed(where):
    h = 0.12e-3
    parts, bx = W.mixed_bed(8, h, 14e-3, 14e-3, 51, shapes=("disk", "plus", "ring"))
    prob = W.assemble(parts, h, [W.Material(horizon=3 * h)], bx, contact_radius=0.95 * h,
                      friction_mu=0.5, damping_ratio=0.8, dt=1e-7, gravity=(0.0, -5000.0),
                      top_wall_speed=[2.0])
    xlo, ylo, ytop = prob.box[0, 0], prob.box[0, 2], prob.box[0, 3]
    if where == "corner":
        prob.u0x = np.full(prob.n_nodes, -(prob.x.min() - xlo) + 0.3 * h)
        prob.u0y = np.full(prob.n_nodes, -(prob.y.min() - ylo) + 0.3 * h)
    else:  # against the moving top wall
        prob.u0x = np.zeros(prob.n_nodes)
        prob.u0y = np.full(prob.n_nodes, (ytop - prob.y.max()) - 0.3 * h)
    W.perturb(prob, 52, dv=0.5)
    return prob


@pytest.mark.parametrize("where", ["corner", "top"])
@pytest.mark.parametrize("lanes", [1, 4])
def test_wall_pass_follows_the_oracle(pdmod, where, lanes):
    _say(f"case: wall pass, bed pressed into the {where}, {lanes} lane(s) per node")
    prob = _pressed(where)
    g, o = pdmod.PD(prob), Oracle(prob)
    g.set_tuning(lanes_per_node=lanes, wall_pass=1)
    for k in range(3):
        assert g.step(40, check=False) == o.step(40)
        sg, so = g.get_state(), o.get_state()
        for key in ("ux", "uy", "vx", "vy"):
            e = _relerr(sg[key], so[key])
            assert e <= TRAJ_TOL, (k, key, e)
        assert np.array_equal(sg["broken"], so["broken"]), k
    R = o.wall_reactions()
    assert np.abs(R).max() > 0.0  # the walls act
    assert g.sizes()["list_rebuilds"] >= 1


@pytest.mark.parametrize("where", ["corner", "top"])
def test_wall_pass_matches_inline_walls(pdmod, where):
    _say(f"case: wall pass against inline walls, bed pressed into the {where}")
    prob = _pressed(where)
    out = {}
    for wp in (0, 1):
        g = pdmod.PD(prob)
        g.set_tuning(lanes_per_node=4, wall_pass=wp)
        assert g.step(150, check=False) == 0
        out[wp] = g.get_state()
    for key in ("ux", "uy", "vx", "vy", "ax", "ay"):
        assert np.array_equal(out[0][key], out[1][key]), key
    assert np.array_equal(out[0]["broken"], out[1]["broken"])


def test_wall_pass_kernel_timing(pdmod):
    _say("case: wall pass timing classes")
    prob = _pressed("corner")
    g = pdmod.PD(prob)
    g.set_tuning(lanes_per_node=1, wall_pass=1)
    g.step(5)
    kt = g.time_kernels(64)
    assert kt["pass"][1] > 0 and kt["pass"][0] > 0.0
    assert kt["force"][1] > 0 and kt["force"][0] > 0.0
    g.set_tuning(wall_pass=0)
    assert g.time_kernels(64)["pass"][1] == 0
