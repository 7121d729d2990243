"""Parity of the HIP path (libpd through its C ABI) with the FP64 oracle.

Bars: reference bond sets and contact sets bit-exact; per-step forces
||F_gpu - F_oracle||_inf / ||F_oracle||_inf <= 1e-12 per term; 100-step
trajectories max|u_gpu - u_oracle| / max|u_oracle| <= 1e-9 (same for v).
"""
import math
import sys

import numpy as np
import pytest

from oracle import Oracle
from paper_2108_07212_amd import workloads as W

pytestmark = pytest.mark.gpu

FORCE_TOL = 1e-12
TRAJ_TOL = 1e-9
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


def _bed(n, seed, h=0.12e-3, box=(14e-3, 14e-3), g=(0.0, 0.0), mu=0.5, rd=0.8, dt=1e-7,
         shapes=("disk", "plus", "ring"), vtop=0.0, precision=W.PREC_FP64):
    parts, bx = W.mixed_bed(n, h, box[0], box[1], seed, shapes=shapes)
    return W.assemble(parts, h, [W.Material(horizon=3 * h)], bx, contact_radius=0.95 * h,
                      friction_mu=mu, damping_ratio=rd, dt=dt, gravity=g,
                      top_wall_speed=[vtop], precision=precision)


def _herd(prob, alpha, seed=0, dv=0.0):
    """Translate each particle rigidly toward the bed centre so particles
    overlap (contacts without bond strain); optional random velocities."""
    cx, cy = prob.x.mean(), prob.y.mean()
    po = prob.particle_offset
    ux, uy = np.zeros(prob.n_nodes), np.zeros(prob.n_nodes)
    for p in range(prob.n_particles):
        s = slice(po[p], po[p + 1])
        ux[s] = -alpha * (prob.x[s].mean() - cx)
        uy[s] = -alpha * (prob.y[s].mean() - cy)
    prob.u0x, prob.u0y = ux, uy
    if dv:
        W.perturb(prob, seed, dv=dv)
    return prob


def _relerr(a, b):
    scale = max(np.abs(b).max(), 1e-300)
    return np.abs(a - b).max() / scale


def _check_forces(g, o, label):
    worst = 0.0
    for t in TERMS:
        gx, gy = g.forces(t)
        ox, oy = o.forces(t)
        scale = max(np.abs(ox).max(), np.abs(oy).max())
        if scale == 0.0:
            assert np.abs(gx).max() == 0.0 and np.abs(gy).max() == 0.0, (label, t)
            continue
        e = max(np.abs(gx - ox).max(), np.abs(gy - oy).max()) / scale
        worst = max(worst, e)
        assert e <= FORCE_TOL, (label, t, e)
    return worst


def _check_bonds(g, o, label):
    rg, cg = g.bonds()
    ro, co = o.bonds()
    assert np.array_equal(rg, ro), label
    assert np.array_equal(cg, co), label


# ---------------------------------------------------------------------------
def test_bond_sets_two_disks(pdmod):
    _say("case: bond sets, two disks")
    prob = W.two_disks()
    g = pdmod.PD(prob)
    o = Oracle(prob)
    _check_bonds(g, o, "two_disks")
    assert len(g.bonds()[1]) == 7952


@pytest.mark.parametrize("seed", [1, 2])
def test_bond_sets_mixed_shapes(pdmod, seed):
    """The extended-boundary / cusp-bisector detector (GPU) gives exactly the
    plain-definition bond set (oracle) on plus, ring and L shapes."""
    _say(f"case: bond sets, mixed shapes seed={seed}")
    prob = _bed(12, seed, shapes=("plus", "ring", "lshape", "disk"))
    g = pdmod.PD(prob)
    o = Oracle(prob)
    _check_bonds(g, o, f"mixed{seed}")
    assert len(o.bonds()[1]) > 1000


def test_bond_sets_lattice_aligned(pdmod):
    """Unrotated shapes whose corners sit on lattice lines."""
    _say("case: bond sets, lattice aligned")
    h = 0.125e-3
    parts = [W.Particle("plus", 1e-3, (3e-3, 3e-3), 0.0), W.Particle("lshape", 1e-3, (6e-3, 3e-3), 0.0),
             W.Particle("ring", 1e-3, (3e-3, 6e-3), 0.0), W.Particle("plus", 1e-3, (6e-3, 6e-3), math.pi / 4)]
    prob = W.assemble(parts, h, [W.Material(horizon=3 * h)], [0, 9e-3, 0, 9e-3],
                      contact_radius=0.95 * h, friction_mu=0.5, damping_ratio=0.5, dt=1e-7)
    _check_bonds(pdmod.PD(prob), Oracle(prob), "aligned")


def _translated(prob, shifts):
    """Each particle moved rigidly by shifts[p] = (dx, dy), its nodes and its
    boundary loops alike."""
    po, lo, vo = prob.particle_offset, prob.loop_offset, prob.loop_vertex_offset
    for p, (dx, dy) in enumerate(shifts):
        s = slice(po[p], po[p + 1])
        prob.x[s] += dx
        prob.y[s] += dy
        v0, v1 = int(vo[lo[p]]), int(vo[lo[p + 1]])
        prob.loop_xy[2 * v0:2 * v1:2] += dx
        prob.loop_xy[2 * v0 + 1:2 * v1:2] += dy
    return prob


@pytest.mark.parametrize("case", ["toward_centre", "seeded_0", "seeded_1", "seeded_2"])
def test_bond_sets_translated_particles(pdmod, case):
    """Bond sets do not depend on where a particle sits.  A ring's hole is a
    regular polygon of an even vertex count, so each cusp's bisector ray runs
    through the opposite vertex; at some positions rounding put that vertex
    just outside both of its edges and the ray ran on through the material
    behind (104 bonds of one ring lost, first seen with the particles of the
    closure test bed moved a quarter of the way toward its centre, kept here
    as a case)."""
    _say(f"case: bond sets of translated particles, {case}")
    prob = W.closure_bed(n_per_shape=3, h=0.08e-3, nodes=60, seed=21, wall_speed=0.0, vmax=0.3)
    P = prob.n_particles
    if case == "toward_centre":
        cx, cy = prob.x.mean(), prob.y.mean()
        po = prob.particle_offset
        shifts = [(-0.25 * (prob.x[po[p]:po[p + 1]].mean() - cx),
                   -0.25 * (prob.y[po[p]:po[p + 1]].mean() - cy)) for p in range(P)]
    else:
        # seeded shifts of up to 1 mm, each within the room its particle has
        # in the box (a margin of one contact radius)
        rng = np.random.default_rng(100 + int(case[-1]))
        xlo, xhi, ylo, yhi = prob.box[0]
        m = prob.contact_radius
        po = prob.particle_offset
        shifts = []
        for p in range(P):
            xs, ys = prob.x[po[p]:po[p + 1]], prob.y[po[p]:po[p + 1]]
            lx, hx = max(xlo + m - xs.min(), -1e-3), min(xhi - m - xs.max(), 1e-3)
            ly, hy = max(ylo + m - ys.min(), -1e-3), min(yhi - m - ys.max(), 1e-3)
            shifts.append((rng.uniform(lx, hx) if lx < hx else 0.0,
                           rng.uniform(ly, hy) if ly < hy else 0.0))
    prob = _translated(prob, shifts)
    _check_bonds(pdmod.PD(prob), Oracle(prob), case)


def test_forces_t0_two_disks(pdmod):
    _say("case: forces t0 two disks")
    prob = W.two_disks()
    _check_forces(pdmod.PD(prob), Oracle(prob), "two_disks")


@pytest.mark.parametrize("seed,alpha", [(3, 0.45), (5, 0.5)])
def test_forces_contact_active(pdmod, seed, alpha):
    """Per-step forces with inter-particle contact, self-contact after damage,
    friction in both regimes, damping and walls, at a herded state."""
    _say(f"case: forces contact-active seed={seed}")
    prob = _herd(_bed(10, seed), alpha, seed=seed, dv=0.5)
    g, o = pdmod.PD(prob), Oracle(prob)
    g.set_counting(True)
    _check_forces(g, o, f"herd{seed}")
    pi, pj = g.contacts()
    qi, qj = o.contacts()
    assert len(qi) > 100
    assert np.array_equal(pi, qi) and np.array_equal(pj, qj)


def _wall_probe(vtop=0.0, seed=0):
    """Single-node particles at signed distances -0.8 R_c .. 0.97 R_c from each
    wall and in each corner zone, with random velocities."""
    h = 1e-4
    Rc = 0.95 * h
    L = 4e-3
    rng = np.random.default_rng(seed)
    pts = []
    for d in np.linspace(-0.8, 0.97, 13) * Rc:
        s = rng.uniform(0.2, 0.8) * L
        pts += [(d, s), (L - d, s), (s, d), (s, L - d)]
    for _ in range(24):
        da, db = rng.uniform(-0.7, 0.95, 2) * Rc
        pts += [(da, db), (L - da, db), (L - da, L - db), (da, L - db)]
    vel = [tuple(v) for v in rng.uniform(-0.5, 0.5, (len(pts), 2))]
    prob = W.single_node_particles(pts, vel, h * h, [0, L, 0, L], contact_radius=Rc, h=h,
                                   friction_mu=0.4, damping_ratio=0.6, dt=1e-8)
    prob.top_wall_speed = np.array([vtop])
    return prob


@pytest.mark.parametrize("vtop", [0.0, 2.0])
def test_forces_walls_and_corners(pdmod, vtop):
    """Wall and corner regions (Sec. 4.5) with damping and friction, including
    a moving top wall evaluated at a later time."""
    _say(f"case: forces walls vtop={vtop}")
    prob = _wall_probe(vtop)
    o = Oracle(prob)
    g = pdmod.PD(prob)
    _check_forces(g, o, "walls")
    if vtop:
        s = o.get_state()
        s["step"] = 3  # top wall moved by 3 dt vtop
        o.set_state(s)
        g.set_state(s)
        _check_forces(g, o, "walls-later")
    wx, wy = o.forces(8)
    assert np.count_nonzero(wx) + np.count_nonzero(wy) > 100


def test_forces_corner_overlap_beyond_one_wall(pdmod):
    """Nodes beyond one wall near a corner whose other segment the first
    wall's line misses (the overlap is that whole segment), and beyond both
    walls with the corner outside the contact disk (the disk minus two caps):
    the two segments overlap although d_a^2 + d_b^2 >= R_c^2."""
    _say("case: forces corner overlap beyond a wall")
    h = 1e-4
    Rc = 0.95 * h
    L = 4e-3
    pts = []
    for da, db in [(-0.3, 0.97), (-0.5, 0.9), (-0.2, 0.99), (0.95, -0.4), (-0.75, -0.75),
                   (-0.6, -0.85), (-0.72, -0.7), (-0.05, 0.999)]:
        da, db = da * Rc, db * Rc
        pts += [(da, db), (L - da, db), (L - da, L - db), (da, L - db)]
    rng = np.random.default_rng(7)
    vel = [tuple(v) for v in rng.uniform(-0.5, 0.5, (len(pts), 2))]
    prob = W.single_node_particles(pts, vel, h * h, [0, L, 0, L], contact_radius=Rc, h=h,
                                   friction_mu=0.4, damping_ratio=0.6, dt=1e-8)
    _check_forces(pdmod.PD(prob), Oracle(prob), "corner-overlap")


def _two_material_bed(seed, kn_mode=W.KN_SELF_CONSISTENT, dt=1e-7, conic=True, alpha=0.45):
    """A herded bed whose particles alternate between two materials: the
    configs' material (constant micromodulus) and a stiffer, denser one with
    the conic micromodulus (Table tab:2d-peri) and a larger horizon."""
    h = 0.12e-3
    parts, bx = W.mixed_bed(10, h, 14e-3, 14e-3, seed)
    for k, p in enumerate(parts):
        p.material = k % 2
    mats = [W.Material(horizon=3 * h),
            W.Material(rho=2400.0, bulk_k=6.0e7, Gc=80.0, horizon=3.5 * h,
                       micro=W.MICRO_CONIC if conic else W.MICRO_CONST)]
    prob = W.assemble(parts, h, mats, bx, contact_radius=0.95 * h, friction_mu=0.5,
                      damping_ratio=0.8, dt=dt, gravity=(0.0, -5000.0), kn_mode=kn_mode)
    return _herd(prob, alpha, seed=seed, dv=0.5)


@pytest.mark.parametrize("seed", [61, 62])
def test_two_materials_conic(pdmod, seed):
    """Two materials, one with the conic micromodulus: per-term forces (the
    harmonic-mean stiffness of Sec. 4.1 between particles of the two
    materials), bond sets and a 100-step trajectory with breaking."""
    _say(f"case: two materials, conic micromodulus seed={seed}")
    prob = _two_material_bed(seed)
    g, o = pdmod.PD(prob), Oracle(prob)
    _check_bonds(g, o, "two-materials")
    g.set_counting(True)
    _check_forces(g, o, "two-materials t0")
    eu, ev, sg, so = _traj(g, o, 100)
    assert eu <= TRAJ_TOL and ev <= TRAJ_TOL, (eu, ev)
    assert np.array_equal(sg["broken"], so["broken"])
    assert o.counters()["inter"] > 0
    g.set_state(so)
    _check_forces(g, o, "two-materials t100")


def test_kn_paper_3d(pdmod):
    """K_n = 18 k / (pi eps^5) as printed (Sec. 4.1), at a step small enough
    for its stiffness (dt = 1e-8 s), with two materials: forces and a 100-step
    trajectory against the oracle (particles pushed together less than in the
    other beds: this stiffness turns the same overlaps into ~1000x the
    force)."""
    _say("case: K_n as printed (3-D)")
    prob = _two_material_bed(63, kn_mode=W.KN_PAPER_3D, dt=1e-8, conic=False, alpha=0.15)
    g, o = pdmod.PD(prob), Oracle(prob)
    c = o.constants()
    assert c["Kn"][0] == pytest.approx(18 * 2.16e7 / (math.pi * prob.materials[0].horizon ** 5),
                                       rel=1e-14)
    _check_forces(g, o, "kn3d t0")
    eu, ev, sg, so = _traj(g, o, 100)
    assert eu <= TRAJ_TOL and ev <= TRAJ_TOL, (eu, ev)
    assert o.counters()["inter"] > 0


def _traj(g, o, steps):
    assert g.step(steps, check=False) == o.step(steps)
    sg, so = g.get_state(), o.get_state()
    eu = max(_relerr(sg["ux"], so["ux"]), _relerr(sg["uy"], so["uy"]))
    ev = max(_relerr(sg["vx"], so["vx"]), _relerr(sg["vy"], so["vy"]))
    return eu, ev, sg, so


def test_trajectory_two_disks_100(pdmod):
    _say("case: trajectory two disks")
    prob = W.two_disks()
    g, o = pdmod.PD(prob), Oracle(prob)
    eu, ev, sg, so = _traj(g, o, 100)
    assert eu <= TRAJ_TOL and ev <= TRAJ_TOL, (eu, ev)


def test_trajectory_two_disks_contact_1000(pdmod):
    """The contact-active two-disk case through first contact (~step 500)."""
    _say("case: trajectory two disks contact")
    prob = W.two_disks(contact_active=True)
    g, o = pdmod.PD(prob), Oracle(prob)
    for k in range(10):
        eu, ev, sg, so = _traj(g, o, 100)
        assert eu <= TRAJ_TOL and ev <= TRAJ_TOL, (k, eu, ev)
    assert o.counters()["inter"] > 0
    assert np.array_equal(sg["broken"], so["broken"])


@pytest.mark.parametrize("lanes,wall_pass", [(4, 0), (1, 0), (4, 1), (1, 1)])
def test_breaks_during_list_steps(pdmod, lanes, wall_pass):
    """A 40 m/s head-on impact breaks bonds while the candidate lists are in
    use: each broken pair joins its nodes' lists in the step it breaks (no
    rebuild).  The first 75 steps (bonds break, fragments touch) follow the
    oracle; after that, contact onsets near ties make any rounding difference
    grow about a thousandfold per 25 steps, in the oracle as well, so the
    remaining check is the list path against the every-step cell search on
    the GPU (with fewer lanes per node, whose sums run in another order,
    against lists of a wider skin), which must give the same states and
    broken bonds.  With the wall pass the contacts of the nodes with
    candidates are evaluated in the pass before each step kernel, and a node
    whose first candidates come from a break joins the pass's list."""
    _say(f"case: breaks during list steps, {lanes} lanes per node, wall pass {wall_pass}")

    def impact():
        prob = W.two_disks(contact_active=True)
        vy = np.zeros(prob.n_nodes)
        vy[prob.particle_offset[1]:] = -40.0
        prob.v0y = vy
        return prob

    prob = impact()
    g, o = pdmod.PD(prob), Oracle(prob)
    g.set_tuning(lanes_per_node=lanes, wall_pass=wall_pass)
    assert g.tuning()["skin_factor"] > 0
    for k in range(3):
        eu, ev, sg, so = _traj(g, o, 25)
        assert eu <= TRAJ_TOL and ev <= TRAJ_TOL, (k, eu, ev)
        assert np.array_equal(sg["broken"], so["broken"]), k
    assert int(so["broken"].sum()) > 50
    assert o.counters()["self_"] > 0
    # against the cell search every step (four lanes per node); with fewer
    # lanes, whose per-node sums run in another order, against the same lane
    # count with a four times wider skin (other lists, other rebuild steps)
    lst, srch = pdmod.PD(impact()), pdmod.PD(impact())
    lst.set_tuning(lanes_per_node=lanes, wall_pass=wall_pass)
    if lanes == 4:
        srch.set_tuning(skin_factor=0.0)
    else:
        srch.set_tuning(lanes_per_node=lanes, wall_pass=wall_pass,
                        skin_factor=4 * lst.tuning()["skin_factor"])
    r0 = lst.sizes()["list_rebuilds"]
    for k in range(3):
        lst.step(50)
        srch.step(50)
        a, b = lst.get_state(), srch.get_state()
        assert np.array_equal(a["broken"], b["broken"]), k
        eu = max(_relerr(a["ux"], b["ux"]), _relerr(a["uy"], b["uy"]))
        ev = max(_relerr(a["vx"], b["vx"]), _relerr(a["vy"], b["vy"]))
        assert eu <= TRAJ_TOL and ev <= TRAJ_TOL, (k, eu, ev)
    assert int(a["broken"].sum()) > 200
    lst.step(150)
    # rebuilds come from motion (a node moving half the skin), not from the
    # hundreds of steps with a break
    assert lst.sizes()["list_rebuilds"] - r0 < 40


@pytest.mark.parametrize("lanes", [1, 2, 4])
def test_contact_pass_matches_inline_contacts(pdmod, lanes):
    """The pass before the step kernel (tuning wall_pass = 1) evaluates the
    contact forces of the nodes with candidates on the step kernel's lanes
    and in its order: a herded bed away from the walls (contacts, friction,
    damping, bonds breaking and their pairs joining the lists) gives the same
    states bit for bit as contact inside the step kernel, at every lane
    count."""
    _say(f"case: contact pass against inline contacts, {lanes} lane(s) per node")
    prob = _herd(_bed(10, 13), 0.45, seed=13, dv=2.0)
    out, cnt = {}, {}
    for wp in (0, 1):
        g = pdmod.PD(prob)
        g.set_tuning(lanes_per_node=lanes, wall_pass=wp)
        g.set_counting(True)
        assert g.step(200, check=False) == 0
        out[wp] = g.get_state()
        cnt[wp] = g.counters()
    for key in ("ux", "uy", "vx", "vy", "ax", "ay"):
        assert np.array_equal(out[0][key], out[1][key]), key
    assert np.array_equal(out[0]["broken"], out[1]["broken"])
    assert cnt[0] == cnt[1]
    assert cnt[1]["inter"] > 0 and cnt[1]["self_"] > 0 and cnt[1]["broken"] > 0
    assert cnt[1]["wall"] == 0


@pytest.mark.parametrize("seed,lanes", [(11, 4), (12, 4), (11, 1), (12, 2)])
def test_trajectory_bed_100(pdmod, seed, lanes):
    """A herded bed with gravity 5000 m/s^2: contact, friction, damping,
    walls and bond breaking over 100 steps, with 4, 2 or 1 lanes per node in
    the list-mode step."""
    _say(f"case: trajectory bed seed={seed} lanes={lanes}")
    prob = _herd(_bed(10, seed, g=(0.0, -5000.0)), 0.45, seed=seed, dv=0.5)
    g, o = pdmod.PD(prob), Oracle(prob)
    g.set_tuning(lanes_per_node=lanes)
    eu, ev, sg, so = _traj(g, o, 100)
    assert eu <= TRAJ_TOL and ev <= TRAJ_TOL, (eu, ev)
    assert np.array_equal(sg["broken"], so["broken"])
    pg, nbg = g.damage()
    po, nbo = o.damage()
    assert nbg == nbo
    assert np.array_equal(pg, po)


@pytest.mark.parametrize("seed", [41, 42])
def test_unequal_volumes_and_offlattice_nodes(pdmod, seed):
    """Nodal volumes jittered by up to 40 % and disk nodes moved off the
    lattice: bond sets bit-exact, per-term forces and a 100-step trajectory
    with friction, damping and gravity (whose coefficients use the volume of
    the node they act on, so V_i != V_j shows) against the oracle."""
    _say(f"case: unequal volumes seed={seed}")
    prob = W.jitter_nodes(_herd(_bed(10, seed, g=(0.0, -5000.0)), 0.45, seed=seed, dv=0.5), seed)
    g, o = pdmod.PD(prob), Oracle(prob)
    rg, cg = g.bonds()
    ro, co = o.bonds()
    assert np.array_equal(rg, ro) and np.array_equal(cg, co)
    _check_forces(g, o, "t0")
    eu, ev, sg, so = _traj(g, o, 100)
    assert eu <= TRAJ_TOL and ev <= TRAJ_TOL, (eu, ev)
    assert np.array_equal(sg["broken"], so["broken"])
    assert o.counters()["inter"] > 0 and o.counters()["slip"] + o.counters()["stick"] > 0
    # per-step forces at the oracle's state after the run
    g.set_state(so)
    _check_forces(g, o, "t100")


@pytest.mark.parametrize("vtop", [0.0, 2.0])
def test_compaction_observables(pdmod, vtop):
    """Wall reactions, bond counts, volume fraction and per-particle damage of
    a bed pressed into the floor and the left wall (top wall moving down at
    vtop) against the oracle's wall split and the plain definitions."""
    _say(f"case: observables vtop={vtop}")
    h = 0.12e-3
    prob = _bed(8, 51, h=h, g=(0.0, -5000.0), vtop=vtop)
    xlo, ylo = prob.box[0, 0], prob.box[0, 2]
    prob.u0x = np.full(prob.n_nodes, -(prob.x.min() - xlo) + 0.3 * h)
    prob.u0y = np.full(prob.n_nodes, -(prob.y.min() - ylo) + 0.3 * h)
    W.perturb(prob, 52, dv=0.5)
    g, o = pdmod.PD(prob), Oracle(prob)
    for k in range(3):
        eu, ev, sg, so = _traj(g, o, 40)
        assert eu <= TRAJ_TOL and ev <= TRAJ_TOL, (k, eu, ev)
        obs = g.observables()
        R = o.wall_reactions()
        scale = np.abs(R).max()
        assert scale > 0
        assert np.abs(obs["wall_force"] - R).max() <= 1e-12 * scale, k
        row, col = o.bonds()
        assert obs["reference"][0] == len(col)
        assert obs["broken"][0] == int(so["broken"].sum())
        t = so["step"] * prob.dt
        ytop = prob.box[0, 3] - vtop * t
        area = (prob.box[0, 1] - prob.box[0, 0]) * (ytop - prob.box[0, 2])
        assert abs(obs["top_wall_y"][0] - ytop) <= 1e-15 * abs(ytop)
        assert abs(obs["volume_fraction"][0] - prob.vol.sum() / area) <= 1e-13
        # per-particle damage: broken / reference directed bonds of its nodes
        rows = np.repeat(np.arange(prob.n_nodes), np.diff(row))
        part = np.repeat(np.arange(prob.n_particles), np.diff(prob.particle_offset))
        nb = np.bincount(part[rows], weights=so["broken"].astype(float), minlength=prob.n_particles)
        nr = np.bincount(part[rows], minlength=prob.n_particles)
        ref = np.where(nr > 0, nb / np.maximum(nr, 1), 0.0)
        np.testing.assert_array_equal(g.particle_damage(), ref)


def test_damage_after_breaking(pdmod):
    _say("case: damage")
    h = 0.125e-3
    parts = [W.Particle("disk", 1e-3, (3e-3, 3e-3))]
    prob = W.assemble(parts, h, [W.Material(horizon=3 * h)], [0, 6e-3, 0, 6e-3],
                      contact_radius=0.95 * h, friction_mu=0, damping_ratio=0, dt=1e-8)
    prob.u0x = np.zeros(prob.n_nodes)
    prob.u0x[100] = 12 * h
    g, o = pdmod.PD(prob), Oracle(prob)
    pg, nbg = g.damage()
    po, nbo = o.damage()
    assert nbg == nbo > 0 and np.array_equal(pg, po)


@pytest.mark.parametrize("prec", [W.PREC_FP64, W.PREC_FP32_FORCE])
def test_carried_displacement_is_bitwise(pdmod, prec):
    """Launches after the first of a list-mode replay read the advanced
    displacement the previous launch wrote; one-step replays evaluate it from
    u, v and a every time.  Both give the same states bit for bit, with
    contacts (a herd of particles driven together)."""
    _say(f"case: carried displacement prec={prec}")
    prob = _herd(_bed(10, 24, g=(0.0, -5000.0), precision=prec), 0.45, seed=24, dv=3.0)
    long_, short = pdmod.PD(prob), pdmod.PD(prob)
    long_.set_counting(True)
    short.set_counting(True)
    long_.step(160)
    for _ in range(160):
        short.step(1)
    a, b = long_.get_state(), short.get_state()
    for k in ("ux", "uy", "vx", "vy", "ax", "ay", "broken"):
        assert np.array_equal(a[k], b[k]), k
    assert long_.counters()["inter"] > 0


@pytest.mark.parametrize("skin", [1.0, 0.0])
def test_determinism_graph_and_tuning(pdmod, skin):
    """Bitwise equal results: two runs; graph vs direct launches; every block
    size and LDS staging choice (for a fixed skin and lane count).  Lane
    counts (list mode) change only the order of the per-node sums: their
    trajectories agree to 1e-9 and their broken bonds exactly."""
    _say(f"case: determinism skin={skin}")
    prob = _herd(_bed(10, 21, g=(0.0, -5000.0)), 0.45, seed=21, dv=0.5)
    first = None
    for lanes in ((4, 2, 1) if skin > 0 else (4,)):
        ref = None
        for bn in (256, 128, 64):
            for lds in (1, 0):
                for graph in (1, 0):
                    g = pdmod.PD(prob)
                    g.set_tuning(block_nodes=bn, use_lds=lds, use_graph=graph, skin_factor=skin,
                                 lanes_per_node=lanes)
                    g.step(137)
                    s = g.get_state()
                    if ref is None:
                        ref = s
                    else:
                        for k in ("ux", "uy", "vx", "vy", "ax", "ay", "broken"):
                            assert np.array_equal(ref[k], s[k]), (lanes, bn, lds, graph, k)
        if first is None:
            first = ref
        else:
            assert np.array_equal(first["broken"], ref["broken"]), lanes
            for k in ("ux", "uy", "vx", "vy"):
                assert _relerr(ref[k], first[k]) <= TRAJ_TOL, (lanes, k)


@pytest.mark.parametrize("skin", [0.0, 0.25, 2.0])
def test_trajectory_skins(pdmod, skin):
    """Every skin (0: cell search every step) gives the oracle trajectory;
    a small skin forces many candidate-list rebuilds, a wide one lists longer
    than their initial slots."""
    _say(f"case: trajectory skin={skin}")
    prob = _herd(_bed(10, 13, g=(0.0, -5000.0)), 0.45, seed=13, dv=2.0)
    g, o = pdmod.PD(prob), Oracle(prob)
    g.set_tuning(skin_factor=skin)
    eu, ev, sg, so = _traj(g, o, 150)
    assert eu <= TRAJ_TOL and ev <= TRAJ_TOL, (eu, ev)
    assert np.array_equal(sg["broken"], so["broken"])
    if skin == 0.25:
        assert g.sizes()["list_rebuilds"] > 3
    if skin == 2.0:
        # some node has more candidates than the 16 initial slots: the lists
        # grew after a rebuild queued ahead of a replay overflowed them
        assert g.sizes()["list_slots"] > 16


def test_autotune_keeps_state(pdmod):
    """The autotuner times candidates on a copy of the state: afterwards the
    state and the forces are bitwise what they were, and stepping on with the
    chosen tuning equals a fresh context run with that tuning."""
    _say("case: autotune")
    prob = _herd(_bed(10, 14), 0.3, seed=14, dv=0.3)
    g = pdmod.PD(prob)
    g.step(10)
    s0 = g.get_state()
    f0 = g.forces()
    best = g.autotune(6)
    assert best["block_nodes"] in (64, 128, 256)
    s1 = g.get_state()
    f1 = g.forces()
    for k in ("ux", "uy", "vx", "vy", "ax", "ay", "broken"):
        assert np.array_equal(s0[k], s1[k]), k
    # the chosen cell size may reorder contact sums: equal up to rounding
    scale = max(np.abs(f0[0]).max(), np.abs(f0[1]).max())
    assert max(np.abs(f0[0] - f1[0]).max(), np.abs(f0[1] - f1[1]).max()) <= 1e-13 * scale
    h = pdmod.PD(prob)
    h.step(10)
    h.set_tuning(**best)
    g.step(40)
    h.step(40)
    sg, sh = g.get_state(), h.get_state()
    for k in ("ux", "uy", "vx", "vy", "broken"):
        assert np.array_equal(sg[k], sh[k]), k


def test_cell_factor_changes_only_rounding(pdmod):
    _say("case: cell factor")
    prob = _herd(_bed(10, 22), 0.45, seed=22, dv=0.5)
    o = Oracle(prob)
    for cf in (1.0, 1.5, 2.0, 3.0):
        g = pdmod.PD(prob)
        g.set_tuning(cell_factor=cf)
        _check_forces(g, o, f"cf{cf}")
        assert np.array_equal(g.contacts()[0], o.contacts()[0])


def test_checkpoint_restart(pdmod):
    _say("case: checkpoint")
    prob = _herd(_bed(8, 23, g=(0.0, -5000.0)), 0.4, seed=23, dv=0.3)
    a = pdmod.PD(prob)
    a.step(50)
    b = pdmod.PD(prob)
    b.step(25)
    s = b.get_state()
    c = pdmod.PD(prob)
    c.set_state(s)
    c.step(25)
    sa, sc = a.get_state(), c.get_state()
    for k in ("ux", "uy", "vx", "vy", "ax", "ay", "broken"):
        assert np.array_equal(sa[k], sc[k]), k


def test_oracle_state_handoff(pdmod):
    """The GPU continues from an oracle state (and vice versa) with parity."""
    _say("case: state handoff")
    prob = _herd(_bed(8, 24, g=(0.0, -5000.0)), 0.45, seed=24, dv=0.3)
    o = Oracle(prob)
    o.step(30)
    g = pdmod.PD(prob)
    g.set_state(o.get_state())
    _check_forces(g, o, "handoff")
    eu, ev, _, _ = _traj(g, o, 50)
    assert eu <= TRAJ_TOL and ev <= TRAJ_TOL


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7])
@pytest.mark.parametrize("lanes,wall_pass", [(4, 0), (1, 0), (4, 1), (1, 1)])
def test_tiny_problems_list_steps(pdmod, n, lanes, wall_pass):
    """A handful of single-node particles (no bonds) in contact with each
    other and with the walls, stepped with candidate lists: node counts that
    fill neither a list-build workgroup (four nodes) nor a SELL slice, with
    and without the pass, against the oracle."""
    _say(f"case: tiny problem n={n} lanes={lanes} wall_pass={wall_pass}")
    h = 1e-4
    Rc = 0.95 * h
    L = 12 * Rc
    rng = np.random.default_rng(40 + n)
    pts = [(0.6 * Rc, 0.7 * Rc)]
    while len(pts) < n:  # a chain, each node 0.8 R_c from the last
        ang = rng.uniform(0.0, 0.5 * math.pi)
        pts.append((pts[-1][0] + 0.8 * Rc * math.cos(ang), pts[-1][1] + 0.8 * Rc * math.sin(ang)))
    vel = [tuple(v) for v in rng.uniform(-0.3, 0.3, (n, 2))]
    prob = W.single_node_particles(pts, vel, h * h, [0, L, 0, L], contact_radius=Rc, h=h,
                                   friction_mu=0.4, damping_ratio=0.6, dt=1e-8,
                                   gravity=(0.0, -5000.0))
    g, o = pdmod.PD(prob), Oracle(prob)
    g.set_tuning(lanes_per_node=lanes, wall_pass=wall_pass)
    assert g.tuning()["skin_factor"] > 0
    eu, ev, sg, so = _traj(g, o, 60)
    assert eu <= TRAJ_TOL and ev <= TRAJ_TOL, (eu, ev)
    c = o.counters()
    assert c["wall"] > 0
    if n > 1:
        assert c["inter"] > 0


def test_escape_status(pdmod):
    _say("case: escape")
    h = 1e-4
    Rc = 0.95 * h
    prob = W.single_node_particles([(5e-3, 0.5 * Rc), (5e-3, 5e-3)], [(0, 0.0), (0, 0)], h * h,
                                   [0, 1e-2, 0, 1e-2], contact_radius=Rc, h=h, dt=1e-8)
    g = pdmod.PD(prob)
    s = g.get_state()
    s["uy"][0] = -2.0 * Rc
    g.set_state(s)
    assert g.step(1, check=False) == pdmod.PD_E_ESCAPED
    assert g.step(1, check=False) == pdmod.PD_E_ESCAPED  # sticky


def test_invalid_problem_rejected(pdmod):
    prob = W.two_disks()
    prob.dt = -1.0
    with pytest.raises(pdmod.PDError) as e:
        pdmod.PD(prob)
    assert e.value.status == pdmod.PD_E_INVALID


# ---------------------------------------------------------------------------
# FP32 force accumulation with FP64 state and FP64 break decisions
# ---------------------------------------------------------------------------
def _near_critical(seed, scale=1.0, noise=3e-8):
    """Particles stretched homogeneously so that bond stretches cluster within
    about 1e-7 of s0: every break decision is a near tie."""
    h = 0.12e-3
    parts, box = W.mixed_bed(6, h, 12e-3, 12e-3, seed)
    prob = W.assemble(parts, h, [W.Material(horizon=3 * h)], box, contact_radius=0.95 * h,
                      friction_mu=0.5, damping_ratio=0.8, dt=1e-7)
    s0 = Oracle(prob).constants()["s0"][0]
    rng = np.random.default_rng(seed)
    ux, uy = np.zeros(prob.n_nodes), np.zeros(prob.n_nodes)
    po = prob.particle_offset
    for p in range(prob.n_particles):
        sl = slice(po[p], po[p + 1])
        cx, cy = prob.x[sl].mean(), prob.y[sl].mean()
        k = s0 * scale * (1.0 + noise * rng.standard_normal(po[p + 1] - po[p]))
        ux[sl] = k * (prob.x[sl] - cx)
        uy[sl] = k * (prob.y[sl] - cy)
    prob.u0x, prob.u0y = ux, uy
    return prob


@pytest.mark.parametrize("precision", [0, 1])
def test_break_decisions_at_near_ties(pdmod, precision):
    """With stretches within ~1e-7 of s0, the bonds broken at t = 0 are exactly
    the oracle's, in FP64 and in the FP32-force mode (FP64 recheck)."""
    _say(f"case: near-tie breaks precision={precision}")
    prob = _near_critical(31)
    o = Oracle(prob)
    g = pdmod.PD(prob, precision=precision)
    bo, bg = o.get_state()["broken"], g.get_state()["broken"]
    assert 0 < bo.sum() < len(bo)  # a genuine mix of broken and intact bonds
    assert np.array_equal(bo, bg)
    o.step(3)
    g.step(3)
    assert np.array_equal(o.get_state()["broken"], g.get_state()["broken"])


def test_fp32_forces_close_to_fp64(pdmod):
    """FP32 force arithmetic and accumulation: per-term force error against the
    FP64 oracle at the same state stays at FP32 level (max-norm relative)."""
    _say("case: fp32 forces")
    prob = _herd(_bed(10, 33), 0.45, seed=33, dv=0.5)
    W.perturb(prob, 34, du=2e-6)
    o = Oracle(prob)
    g = pdmod.PD(prob, precision=1)
    for t in TERMS:
        gx, gy = g.forces(t)
        ox, oy = o.forces(t)
        scale = max(np.abs(ox).max(), np.abs(oy).max())
        if scale == 0:
            continue
        e = max(np.abs(gx - ox).max(), np.abs(gy - oy).max()) / scale
        assert e < 2e-5, (t, e)


# ---------------------------------------------------------------------------
# batched aggregates
# ---------------------------------------------------------------------------
def _small_batch(seed=41, n_agg=3):
    prob = W.batched(n_aggregates=n_agg, h=0.15e-3, seed=seed, n_range=(6, 12), dt=4e-7,
                     gravity=-5000.0, precision=W.PREC_FP64)
    return W.particle_velocities(prob, seed, 3.0)


def test_batched_aggregates_match_alone(pdmod):
    """Aggregates of uneven size in one problem evolve as they do alone:
    bond sets and broken bonds bit-exact, trajectories to 1e-9."""
    _say("case: batched vs alone")
    prob = _small_batch()
    gb = pdmod.PD(prob)
    gb.step(500)
    sb = gb.get_state()
    rb, cb = gb.bonds()
    n0 = 0
    b0 = 0
    for a in range(prob.n_aggregates):
        sub = W.subproblem_aggregate(prob, a)
        ga = pdmod.PD(sub)
        ra, ca = ga.bonds()
        n1 = n0 + sub.n_nodes
        assert np.array_equal(cb[rb[n0]:rb[n1]] - n0, ca)
        ga.step(500)
        sa = ga.get_state()
        for k in ("ux", "uy", "vx", "vy"):
            e = _relerr(sb[k][n0:n1], sa[k])
            assert e <= TRAJ_TOL, (a, k, e)
        nb = len(ca)
        assert np.array_equal(sb["broken"][b0:b0 + nb], sa["broken"])
        n0, b0 = n1, b0 + nb
    assert gb.counters()["steps"] == 500


def test_batched_oracle_parity(pdmod):
    _say("case: batched vs oracle")
    prob = _small_batch(seed=41, n_agg=3)
    g, o = pdmod.PD(prob), Oracle(prob)
    g.set_counting(True)
    eu, ev, sg, so = _traj(g, o, 500)
    assert eu <= TRAJ_TOL and ev <= TRAJ_TOL, (eu, ev)
    assert np.array_equal(sg["broken"], so["broken"])
    assert g.counters()["inter"] > 0  # the aggregates' particles touch
