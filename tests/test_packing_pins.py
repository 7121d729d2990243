"""Pins of the initial-configuration geometry of Sec. 7.1-7.2: incircles,
jammed security disks, the perturbed-disk and square shapes, and the settling
workload built on them (geometry only; no force law is involved).

Checked against closed forms (incircles of an equilateral and a 3-4-5
triangle, the square's area and lattice count, the expected area of the
random polygon), brute force (the nodal circles' optimum against a dense
grid search of the centre) and the construction's own requirements
(disjoint disks inside the box, gaps of at least R_c between particles and
to the walls at t = 0).
"""
import math

import numpy as np
import pytest
from scipy.spatial import cKDTree

from paper_2108_07212_amd import workloads as W


def test_incircle_closed_forms():
    a = 2.0
    pts = np.array([(0.0, 0.0), (a, 0.0), (0.5 * a, a * math.sqrt(3) / 2), (0.0, 3.0), (4.0, 0.0)])
    c, r = W.triangle_incircles(pts, np.array([[0, 1, 2], [0, 4, 3]]))
    np.testing.assert_allclose(r[0], a / (2 * math.sqrt(3)), rtol=1e-14)
    np.testing.assert_allclose(c[0], pts[:3].mean(axis=0), rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(r[1], 1.0, rtol=1e-14)  # legs 3 and 4: r = (3 + 4 - 5) / 2
    np.testing.assert_allclose(c[1], (1.0, 1.0), rtol=1e-14)


@pytest.fixture(scope="module")
def jam():
    w, h, m = 8e-3, 12e-3, 1.6e-3
    c, r, st, origin = W.jammed_disks(w, h, m, seed=3)
    return w, h, m, c, r, st, origin


def test_jammed_disks_are_disjoint_and_inside(jam):
    w, h, m, c, r, st, origin = jam
    d = np.sqrt(((c[:, None, :] - c[None, :, :]) ** 2).sum(-1))
    np.fill_diagonal(d, np.inf)
    assert (r[:, None] + r[None, :] - d).max() <= 1e-15 * m
    tol = 1e-15 * m
    assert (c[:, 0] - r).min() >= -tol and (c[:, 1] - r).min() >= -tol
    assert (c[:, 0] + r).max() <= w + tol and (c[:, 1] + r).max() <= h + tol
    # maximising the nodal circles fills most of what the incircles leave
    # (the paper's figure: 0.69 with the first nodal circles, 0.80 after)
    assert st["packing_incircles"] < 0.62 < 0.74 < st["packing_jammed"] < 0.84


def test_nodal_circles_against_grid_search(jam):
    """The Nelder-Mead optimum of a few interior nodal circles against a
    dense grid over the node's star (same objective, brute force)."""
    w, h, m, c, r, st, origin = jam
    rng = np.random.default_rng(3)
    pts, tri = W._box_mesh(w, h, m, rng)
    cT, rT = W.triangle_incircles(pts, tri)
    interior = [v for v in range(len(pts)) if 1.5 * m < pts[v, 0] < w - 1.5 * m
                and 1.5 * m < pts[v, 1] < h - 1.5 * m]
    checked = 0
    for v in interior:
        ts = np.nonzero((tri == v).any(axis=1))[0]
        ring = np.nonzero(np.isin(tri, np.unique(tri[ts])).any(axis=1))[0]
        g = np.linspace(-0.6 * m, 0.6 * m, 241)
        X, Y = np.meshgrid(pts[v, 0] + g, pts[v, 1] + g)
        P = np.stack([X.ravel(), Y.ravel()], 1)
        inside = np.zeros(len(P), dtype=bool)
        for t in ts:
            A, B, C = pts[tri[t]]
            d1 = (B[0] - A[0]) * (P[:, 1] - A[1]) - (B[1] - A[1]) * (P[:, 0] - A[0])
            d2 = (C[0] - B[0]) * (P[:, 1] - B[1]) - (C[1] - B[1]) * (P[:, 0] - B[0])
            d3 = (A[0] - C[0]) * (P[:, 1] - C[1]) - (A[1] - C[1]) * (P[:, 0] - C[0])
            inside |= ((d1 >= 0) & (d2 >= 0) & (d3 >= 0)) | ((d1 <= 0) & (d2 <= 0) & (d3 <= 0))
        P = P[inside]
        gap = (np.sqrt(((P[:, None, :] - cT[ring][None]) ** 2).sum(-1)) - rT[ring]).min(1)
        best = gap.max()
        k = int(np.nonzero(origin == v)[0][0])
        # a nodal circle that overlapped a neighbouring one gave part of its
        # radius up; the others are the optimum
        others = np.nonzero(origin >= 0)[0]
        others = others[others != k]
        dn = np.hypot(*(c[others] - c[k]).T) - r[others] - r[k]
        if dn.min() < 1e-9 * m:
            continue
        assert r[k] >= best * (1 - 1e-3), (v, r[k], best)
        assert r[k] <= best + 2 * (g[1] - g[0])
        checked += 1
    assert checked >= 4


def test_square_shape():
    R = 1e-3
    lp = W.shape_loops("square", R)[0]
    np.testing.assert_allclose(np.hypot(lp[:, 0], lp[:, 1]), R, rtol=1e-15)
    np.testing.assert_allclose(W.polygon_area([lp]), 2 * R * R, rtol=1e-14)
    h = 0.13e-3
    k = int(math.floor(R / math.sqrt(2) / h))
    assert len(W.body_nodes("square", R, h)) == (2 * k + 1) ** 2


def test_plus_and_ring_of_the_settling_study():
    """Plus with inner radius cR: re-entrant corners at distance cR, tips on
    the circle, area 8 L w - 4 w^2 (two crossed 2L x 2w bars); annulus area
    of the polygons against pi R^2 (1 - tau^2) up to the 64-gon's deficit."""
    R, c = 1.0, 0.2
    lp = W.plus_loop(R, c)
    rr = np.hypot(lp[:, 0], lp[:, 1])
    np.testing.assert_allclose(np.sort(rr)[:4], c * R, rtol=1e-14)
    np.testing.assert_allclose(np.sort(rr)[4:], R, rtol=1e-14)
    w = c * R / math.sqrt(2)
    L = math.sqrt(R * R - w * w)
    np.testing.assert_allclose(W.polygon_area([lp]), 8 * L * w - 4 * w * w, rtol=1e-14)
    n = 64
    poly = 0.5 * n * math.sin(2 * math.pi / n)  # area of the unit n-gon
    np.testing.assert_allclose(W.polygon_area(W.ring_loops(R, 0.6, n)), poly * (1 - 0.36), rtol=1e-13)


def test_perturbed_disk_shape():
    """Vertex radii in [phi R, R]; mean area of the random 20-gon equals
    (n/2) sin(2 pi/n) R^2 E[1 - X]^2 with X ~ U[0, 1 - phi] (independent
    neighbouring radii), E[1 - X] = (1 + phi)/2."""
    R, n, phi = 1.0, 20, 0.6
    rng = np.random.default_rng(11)
    areas = []
    for _ in range(4000):
        lp = W.perturbed_disk_loop(R, rng, n, phi)
        rr = np.hypot(lp[:, 0], lp[:, 1])
        assert rr.min() >= phi * R - 1e-15 and rr.max() <= R + 1e-15
        areas.append(W.polygon_area([lp]))
    expect = 0.5 * n * math.sin(2 * math.pi / n) * R * R * ((1 + phi) / 2) ** 2
    assert abs(np.mean(areas) - expect) < 0.005 * expect


@pytest.mark.parametrize("shape", W.SETTLE_SHAPES)
def test_jammed_settling_starts_free_of_contact(shape):
    prob = W.jammed_settling(shape, width=8e-3, height=12e-3, mesh_size=2.4e-3, r_min=0.3e-3)
    Rc = prob.contact_radius
    po = prob.particle_offset
    part = np.repeat(np.arange(prob.n_particles), np.diff(po))
    P = np.stack([prob.x, prob.y], 1)
    # every node in its security disk
    cen = np.array([(prob.x[po[p]:po[p + 1]].mean(), 0.0) for p in range(prob.n_particles)])
    assert prob.n_particles >= 5
    pairs = cKDTree(P).query_pairs(Rc, output_type="ndarray")
    assert not np.any(part[pairs[:, 0]] != part[pairs[:, 1]])
    b = prob.box[0]
    gap = np.minimum.reduce([prob.x - b[0], b[1] - prob.x, prob.y - b[2], b[3] - prob.y])
    assert gap.min() >= Rc
    del cen
