"""Pins of the oracle's self-contact law (Sec. 4.4) and of the pair stiffness
between two materials (Sec. 4.1), each against something the paper or the
mechanics fixes rather than the oracle's own formula:

* the closing remark of Sec. 4.4: for nodes whose reference distance is at
  least R_c, self-contact is the inter-particle law once c_w / R_c = K_n;
* below R_c the self-contact law is a compression-only spring of rest length
  |xi| (the reference distance): a pair released from compression separates
  with the speed energy conservation gives, after a quarter period, and a
  shattered particle at rest feels no force at all;
* two single-node particles of different materials collide as one spring
  whose stiffness is the harmonic mean of theirs: the contact lasts pi/omega
  with omega^2 = K_n V_i V_j (m_i + m_j) / (m_i m_j), which tells the
  harmonic mean from the geometric and arithmetic ones.
"""
import math

import numpy as np
import pytest

from oracle import Oracle
from oracle.oracle import T_NBR, T_SELF
from paper_2108_07212_amd import workloads as W


def _pair_problem(nodes, same_particle, h, Rc, v, mats=None, mat_of=(0, 0), rd=0.0, mu=0.0,
                  dt=1e-9, vol=None):
    """Two nodes, either one particle of two nodes or two one-node particles."""
    mats = mats or [W.Material(horizon=3 * h)]
    vol = h * h if vol is None else vol
    if same_particle:
        nb = np.array(nodes, dtype=float) - np.array(nodes[0], dtype=float)
        parts = [W.Particle("disk", 0.0, tuple(nodes[0]), 0.0, mat_of[0], nodes_body=nb,
                            loops_body=[])]
    else:
        parts = [W.Particle("disk", 0.0, tuple(p), 0.0, m, nodes_body=np.zeros((1, 2)),
                            loops_body=[]) for p, m in zip(nodes, mat_of)]
    prob = W.assemble(parts, h, mats, [0.0, 1e-2, 0.0, 1e-2], contact_radius=Rc,
                      friction_mu=mu, damping_ratio=rd, dt=dt, vol=vol)
    prob.v0x = np.array([v[0][0], v[1][0]])
    prob.v0y = np.array([v[0][1], v[1][1]])
    return prob


def _break_all(o):
    s = o.get_state()
    s["broken"][:] = 1
    o.set_state(s)


@pytest.mark.parametrize("L_over_h,d_over_h", [(2.0, 0.6), (1.0, 0.3), (2.5, 0.9)])
def test_self_contact_equals_inter_particle_beyond_rc(L_over_h, d_over_h):
    """Sec. 4.4, last remark: with |xi| >= R_c and K_n = c_w / R_c the
    self-contact force (repulsion, damping, friction) equals the force
    between the same two nodes in different particles."""
    h = 1e-4
    Rc = 0.95 * h
    x0 = np.array([5e-3, 5e-3])
    ref = [tuple(x0), tuple(x0 + [L_over_h * h, 0.0])]
    th = 0.4
    cur = [tuple(x0), tuple(x0 + d_over_h * h * np.array([math.cos(th), math.sin(th)]))]
    v = [(0.3, -0.2), (-0.5, 0.4)]
    same = _pair_problem(ref, True, h, Rc, v, rd=0.7, mu=0.4, dt=1e-8)
    o = Oracle(same)
    assert len(o.bonds()[1]) == 2  # the two nodes are bonded in the reference
    _break_all(o)
    s = o.get_state()
    s["ux"][1] = cur[1][0] - ref[1][0]
    s["uy"][1] = cur[1][1] - ref[1][1]
    o.set_state(s)
    fs = o.forces(T_SELF)
    sep = _pair_problem(cur, False, h, Rc, v, rd=0.7, mu=0.4, dt=1e-8)
    on = Oracle(sep)
    fn = on.forces(T_NBR)
    assert np.abs(fs[0]).max() > 0
    for k in range(2):
        np.testing.assert_allclose(fs[k], fn[k], rtol=1e-14, atol=1e-14 * np.abs(fn[k]).max())
    # and the bonded pair feels no contact at all
    o2 = Oracle(_pair_problem(ref, True, h, Rc, v, rd=0.7, mu=0.4, dt=1e-8))
    s2 = o2.get_state()
    s2["ux"][1], s2["uy"][1] = s["ux"][1], s["uy"][1]
    o2.set_state(s2)
    assert np.abs(o2.forces(T_SELF)[0]).max() == 0.0


def test_self_contact_below_rc_is_compression_spring():
    """|xi| < R_c: two nodes of one particle at reference distance L, bond
    broken, released at rest from distance d0 < L, separate as a
    compression-only spring of rest length L and stiffness c_w V^2 / L:
    relative speed (L - d0) omega when the distance reaches L, after a
    quarter period pi / (2 omega), omega^2 = 2 c_w V / (rho L); and no force
    once the distance is at least L."""
    h = 1e-4
    Rc = 0.95 * h
    L = 0.5 * h
    d0 = 0.3 * h
    x0 = np.array([5e-3, 5e-3])
    out = []
    for dt in (4e-10, 2e-10):
        prob = _pair_problem([tuple(x0), tuple(x0 + [L, 0.0])], True, h, Rc, [(0, 0), (0, 0)],
                             dt=dt)
        o = Oracle(prob)
        _break_all(o)
        s = o.get_state()
        s["ux"][0], s["ux"][1] = 0.5 * (L - d0), -0.5 * (L - d0)
        o.set_state(s)
        cw = o.constants()["cw"][0]
        V = h * h
        m = prob.materials[0].rho * V
        om = math.sqrt(2 * cw * V / (prob.materials[0].rho * L))
        assert om == pytest.approx(math.sqrt(2 * (cw * V * V / L) / m), rel=1e-14)
        n = 0
        while True:
            o.step(1)
            n += 1
            s = o.get_state()
            d = (x0[0] + L + s["ux"][1]) - (x0[0] + s["ux"][0])
            if d >= L:
                break
            assert n < 100000
        vrel = s["vx"][1] - s["vx"][0]
        out.append((vrel, n * dt))
        assert vrel == pytest.approx((L - d0) * om, rel=2e-2)
        assert n * dt == pytest.approx(math.pi / (2 * om), rel=2e-2)
        # separated past the rest length: no force, constant velocity
        o.step(20)
        s2 = o.get_state()
        assert s2["vx"][1] - s2["vx"][0] == pytest.approx(vrel, rel=1e-12)
    e = [abs(r[0] - (L - d0) * om) for r in out]
    assert e[1] < e[0]


def test_shattered_particle_at_rest_feels_no_force():
    """Every bond of a lattice disk broken, at rest, with a contact radius of
    1.5 h (nearest and diagonal neighbours within R_c, each at its own
    reference distance): the self-contact law gives zero force, and the
    particle stays exactly where it is."""
    h = 1e-4
    parts = [W.Particle("disk", 8 * h, (5e-3, 5e-3), 0.0)]
    prob = W.assemble(parts, h, [W.Material(horizon=3 * h)], [0.0, 1e-2, 0.0, 1e-2],
                      contact_radius=1.5 * h, friction_mu=0.5, damping_ratio=0.8, dt=1e-8)
    o = Oracle(prob)
    _break_all(o)
    assert o.counters()["self_"] == 0
    fx, fy = o.forces(T_SELF)
    assert np.abs(fx).max() == 0.0 and np.abs(fy).max() == 0.0
    o.step(50)
    s = o.get_state()
    assert np.abs(s["ux"]).max() == 0.0 and np.abs(s["vy"]).max() == 0.0
    assert o.counters()["self_"] > 0  # the pairs were evaluated, and gave nothing


@pytest.mark.parametrize("ratio,rho_b", [(4.0, 1200.0), (9.0, 3000.0)])
def test_two_material_head_on_harmonic_mean(ratio, rho_b):
    """Sec. 4.1: between materials a and b the repulsion stiffness is
    K = 2 K_a K_b / (K_a + K_b).  Two single-node particles meeting head on
    (no damping, no friction) stay in contact for pi / omega with
    omega^2 = K V_a V_b (1/m_a + 1/m_b), and leave with the entry speed."""
    h = 1e-4
    Rc = 0.95 * h
    V = h * h
    mats = [W.Material(horizon=3 * h), W.Material(bulk_k=2.16e7 * ratio, rho=rho_b, horizon=3 * h)]
    x0 = np.array([5e-3, 5e-3])
    gap = Rc + 0.1 * h
    vin = 1.0
    prob = _pair_problem([tuple(x0), tuple(x0 + [gap, 0.0])], False, h, Rc,
                         [(0.5 * vin, 0.0), (-0.5 * vin, 0.0)], mats=mats, mat_of=(0, 1),
                         dt=5e-10)
    o = Oracle(prob)
    Ka, Kb = o.constants()["Kn"]
    assert Kb == pytest.approx(ratio * Ka, rel=1e-12)
    ma, mb = mats[0].rho * V, rho_b * V

    def duration(K):
        return math.pi / math.sqrt(K * V * V * (1 / ma + 1 / mb))

    t_in = t_out = None
    n = 0
    while n < 200000:
        o.step(1)
        n += 1
        s = o.get_state()
        d = (x0[0] + gap + s["ux"][1]) - (x0[0] + s["ux"][0])
        if t_in is None and d < Rc:
            t_in = n
        if t_in is not None and d >= Rc:
            t_out = n
            break
    T = (t_out - t_in) * prob.dt
    harmonic = 2 * Ka * Kb / (Ka + Kb)
    assert T == pytest.approx(duration(harmonic), rel=1e-2)
    for other in (math.sqrt(Ka * Kb), 0.5 * (Ka + Kb), min(Ka, Kb)):
        assert abs(T - duration(other)) > 5e-2 * duration(other)
    vout = s["vx"][1] - s["vx"][0]
    assert vout == pytest.approx(vin, rel=1e-2)
