"""Parity of the HIP path with the FP64 oracle on the particle shapes and
initial configurations of Sec. 7.1-7.3: perturbed disks (a random
non-convex 20-gon per particle), squares, and beds started from jammed
security disks with the horizon of Sec. 7.3 (eps = 8h).

Bars: bond sets bit-exact; per-term forces 1e-12 relative to the largest;
trajectories max|u_gpu - u_oracle| / max|u_oracle| <= 1e-9 (same for v).
"""
import sys

import numpy as np
import pytest

from oracle import Oracle
from paper_2108_07212_amd import workloads as W

pytestmark = pytest.mark.gpu

FORCE_TOL = 1e-12
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


def _small(shape, seed=6):
    return W.jammed_settling(shape, width=8e-3, height=12e-3, mesh_size=2.4e-3, r_min=0.3e-3,
                             seed=seed)


@pytest.mark.parametrize("shape", W.SETTLE_SHAPES)
def test_jammed_shapes_bonds_and_forces(pdmod, shape):
    _say(f"case: jammed {shape} bonds and forces")
    prob = _small(shape)
    g, o = pdmod.PD(prob), Oracle(prob)
    rg, cg = g.bonds()
    ro, co = o.bonds()
    assert np.array_equal(rg, ro) and np.array_equal(cg, co)
    # some displacement so that every term is non-trivial
    W.perturb(prob, 5, du=0.02 * prob.meta["h"], dv=0.05)
    g, o = pdmod.PD(prob), Oracle(prob)
    for t in (1, 2, 4, 8, 16):
        gx, gy = g.forces(t)
        ox, oy = o.forces(t)
        scale = max(np.abs(ox).max(), np.abs(oy).max())
        if scale == 0.0:
            assert np.abs(gx).max() == 0.0 and np.abs(gy).max() == 0.0, t
            continue
        e = max(np.abs(gx - ox).max(), np.abs(gy - oy).max()) / scale
        assert e <= FORCE_TOL, (t, e)


@pytest.mark.parametrize("shape", ["pdisk", "square"])
def test_jammed_settling_trajectory(pdmod, shape):
    """Particles fall from the jammed start under 5000 m/s^2 with seeded
    rigid velocities in [-3, 3]^2 m/s plus 2 m/s downward, so that they reach
    the floor and each other within the run (the start is contact-free)."""
    _say(f"case: jammed {shape} trajectory")
    prob = W.particle_velocities(_small(shape), 9, 3.0)
    prob.v0y = prob.v0y - 2.0
    g, o = pdmod.PD(prob), Oracle(prob)
    for k in range(4):
        assert g.step(150, check=False) == o.step(150)
        sg, so = g.get_state(), o.get_state()
        eu = max(_relerr(sg["ux"], so["ux"]), _relerr(sg["uy"], so["uy"]))
        ev = max(_relerr(sg["vx"], so["vx"]), _relerr(sg["vy"], so["vy"]))
        _say(f"  step {150 * (k + 1)}: eu={eu:.2e} ev={ev:.2e}")
        assert eu <= TRAJ_TOL and ev <= TRAJ_TOL, (k, eu, ev)
        assert np.array_equal(sg["broken"], so["broken"])
    c = o.counters()
    assert c["wall"] > 0 and c["inter"] > 0
