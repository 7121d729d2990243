"""Seeded synthetic workloads for the PeriDEM step loop.

Geometry and placement only: particle boundary polygons (disk, plus, ring,
L-shape), nodes on a uniform lattice inside each particle, random sequential
placement of non-overlapping security disks, and the problem record that both
the GPU library and the CPU oracle consume.  Nothing here evaluates a force
law, a stretch, a neighbour set or an integrator step; random numbers that
the method itself would need are never drawn here.

The paper meshes particles with Gmsh (Sec. 5, last paragraph); here the nodes
are lattice points of spacing h inside the particle, each with nodal area
h^2 (in 2-D "volume" means area, Sec. 7 intro).  Shapes follow Sec. 7.2:
plus-shaped particles with arm half-length R and arm width R/2, rings with
inner radius R/2, plus an L-shape (union of [0,R]x[0,R/2] and [0,R/2]x[0,R]).
The initial packing of Sec. 7.1 (jammed security disks from a triangle mesh)
is replaced by random sequential placement of security disks of radius 1.1 R.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SHAPES = ("disk", "plus", "ring", "lshape", "square")

# enum values shared with the C records (see include/pd.h)
MICRO_CONST, MICRO_CONIC = 0, 1
PREC_FP64, PREC_FP32_FORCE = 0, 1
KN_SELF_CONSISTENT, KN_PAPER_3D = 0, 1


# ----------------------------------------------------------------------------
# shapes (body frame, centroid at the origin)
# ----------------------------------------------------------------------------
def _circle(radius: float, nv: int, ccw: bool) -> np.ndarray:
    ang = 2.0 * np.pi * np.arange(nv) / nv
    pts = np.stack([radius * np.cos(ang), radius * np.sin(ang)], axis=1)
    return pts if ccw else pts[::-1].copy()


def shape_loops(shape: str, R: float, n_circle: int = 64) -> list:
    """Boundary loops of a shape: outer loop counter-clockwise, holes clockwise.

    A disk returns no loop: it is convex, so no bond can leave it and no
    line-of-sight filtering applies (Sec. 5: the non-bond set is empty on
    convex domains).
    """
    if shape == "disk":
        return []
    if shape == "plus":
        b = 0.25 * R  # half of the arm width R/2
        v = [(R, -b), (R, b), (b, b), (b, R), (-b, R), (-b, b), (-R, b),
             (-R, -b), (-b, -b), (-b, -R), (b, -R), (b, -b)]
        return [np.array(v, dtype=np.float64)]
    if shape == "ring":
        return [_circle(R, n_circle, True), _circle(0.5 * R, n_circle, False)]
    if shape == "square":
        a = R / math.sqrt(2.0)  # inscribed in the circle of radius R (Sec. 7.2)
        return [np.array([(-a, -a), (a, -a), (a, a), (-a, a)], dtype=np.float64)]
    if shape == "lshape":
        h2 = 0.5 * R
        v = np.array([(0, 0), (R, 0), (R, h2), (h2, h2), (h2, R), (0, R)], dtype=np.float64)
        # centroid of the union of two rectangles minus their overlap
        a1, c1 = R * h2, (0.5 * R, 0.5 * h2)
        a2, c2 = h2 * R, (0.5 * h2, 0.5 * R)
        a3, c3 = h2 * h2, (0.5 * h2, 0.5 * h2)
        A = a1 + a2 - a3
        cx = (a1 * c1[0] + a2 * c2[0] - a3 * c3[0]) / A
        cy = (a1 * c1[1] + a2 * c2[1] - a3 * c3[1]) / A
        return [v - np.array([cx, cy])]
    raise ValueError(f"unknown shape {shape!r}")


def shape_area(shape: str, R: float) -> float:
    if shape == "disk":
        return math.pi * R * R
    if shape == "plus":
        return 1.75 * R * R
    if shape == "ring":
        return math.pi * R * R * 0.75
    if shape == "lshape":
        return 0.75 * R * R
    if shape == "square":
        return 2.0 * R * R
    raise ValueError(shape)


def perturbed_disk_loop(R: float, rng: np.random.Generator, n: int = 20,
                        phi: float = 0.6) -> np.ndarray:
    """Sec. 7.2: the polygon with vertices r_k (cos t_k, sin t_k), t_k = 2 pi k / n,
    r_k = R (1 - X_k), X_k ~ U[0, 1 - phi] independent (counter-clockwise,
    about the centre of the disk of radius R that bounds it)."""
    t = 2.0 * np.pi * np.arange(n) / n
    r = R * (1.0 - rng.uniform(0.0, 1.0 - phi, size=n))
    return np.stack([r * np.cos(t), r * np.sin(t)], axis=1)


def plus_loop(R: float, c: float = 0.2) -> np.ndarray:
    """Sec. 7.2 plus shape inscribed in the circle of radius R with inner
    radius cR: the re-entrant corners lie at distance cR from the centre (arm
    half-width w = cR / sqrt 2) and the arm tips' corners on the circle
    (arm half-length sqrt(R^2 - w^2)); counter-clockwise."""
    w = c * R / math.sqrt(2.0)
    L = math.sqrt(R * R - w * w)
    v = [(L, -w), (L, w), (w, w), (w, L), (-w, L), (-w, w), (-L, w), (-L, -w), (-w, -w),
         (-w, -L), (w, -L), (w, -w)]
    return np.array(v, dtype=np.float64)


def ring_loops(R: float, tau: float = 0.6, n_circle: int = 64) -> list:
    """Sec. 7.2 annulus: outer radius R, inner radius tau R (hole clockwise)."""
    return [_circle(R, n_circle, True), _circle(tau * R, n_circle, False)]


def polygon_area(loops: list) -> float:
    """Signed-area sum of the loops (outer counter-clockwise, holes clockwise)."""
    a = 0.0
    for lp in loops:
        x, y = lp[:, 0], lp[:, 1]
        a += 0.5 * float(np.sum(x * np.roll(y, -1) - np.roll(x, -1) * y))
    return a


def _inside_even_odd(px: np.ndarray, py: np.ndarray, loops: list) -> np.ndarray:
    """Even-odd rule: crossings of the horizontal ray to +x with every edge
    (all edges of a loop at once, the same expressions per edge)."""
    inside = np.zeros(px.shape, dtype=bool)
    qx, qy = px[:, None], py[:, None]
    for lp in loops:
        a = lp
        b = np.roll(lp, -1, axis=0)
        ax, ay, bx, by = a[:, 0], a[:, 1], b[:, 0], b[:, 1]
        cond = (ay > qy) != (by > qy)
        with np.errstate(divide="ignore", invalid="ignore"):
            xint = ax + (qy - ay) * (bx - ax) / (by - ay)
        inside ^= (np.count_nonzero(cond & (qx < xint), axis=1) & 1).astype(bool)
    return inside


def _dist_to_loops(px: np.ndarray, py: np.ndarray, loops: list) -> np.ndarray:
    """Distance of each point to the nearest edge of the loops."""
    d = np.full(px.shape, np.inf)
    qx0, qy0 = px[:, None], py[:, None]
    for lp in loops:
        a = lp
        b = np.roll(lp, -1, axis=0)
        ax, ay = a[:, 0], a[:, 1]
        ex, ey = b[:, 0] - ax, b[:, 1] - ay
        L2 = ex * ex + ey * ey
        t = np.minimum(np.maximum(((qx0 - ax) * ex + (qy0 - ay) * ey) / L2, 0.0), 1.0)
        qx, qy = ax + t * ex - qx0, ay + t * ey - qy0
        d = np.minimum(d, np.sqrt(qx * qx + qy * qy).min(axis=1))
    return d


def body_nodes(shape: str, R: float, h: float, margin: float = 1e-3) -> np.ndarray:
    """Lattice points (i h, j h) inside the shape, body frame, row-major order.

    Disk: points with |x| <= R (boundary points included).  Polygonal shapes:
    points strictly inside with distance to the boundary above margin*h, so
    that no node sits on the boundary.
    """
    n = int(math.ceil(R / h)) + 1
    ii = np.arange(-n, n + 1)
    jj, iig = np.meshgrid(ii, ii, indexing="ij")  # row-major: j outer, i inner
    px = (iig * h).ravel().astype(np.float64)
    py = (jj * h).ravel().astype(np.float64)
    if shape == "disk":
        keep = (iig.ravel() ** 2 + jj.ravel() ** 2) * (h * h) <= R * R * (1.0 + 1e-9)
        return np.stack([px[keep], py[keep]], axis=1)
    return loop_nodes(shape_loops(shape, R), R, h, margin)


def loop_nodes(loops: list, R: float, h: float, margin: float = 1e-3) -> np.ndarray:
    """Lattice points (i h, j h) strictly inside the loops (even-odd rule) and
    farther than margin*h from them, row-major; the loops lie within the
    circle of radius R about the origin."""
    n = int(math.ceil(R / h)) + 1
    ii = np.arange(-n, n + 1)
    jj, iig = np.meshgrid(ii, ii, indexing="ij")
    px = (iig * h).ravel().astype(np.float64)
    py = (jj * h).ravel().astype(np.float64)
    # points beyond the circle through the farthest vertex are outside; the
    # rest get the even-odd test, and the points inside the distance test
    rmax = max(float(np.sqrt((lp * lp).sum(axis=1)).max()) for lp in loops)
    keep = px * px + py * py <= (1.001 * rmax) ** 2
    idx = np.nonzero(keep)[0]
    keep[idx] = _inside_even_odd(px[idx], py[idx], loops)
    idx = np.nonzero(keep)[0]
    keep[idx] = _dist_to_loops(px[idx], py[idx], loops) > margin * h
    return np.stack([px[keep], py[keep]], axis=1)


# ----------------------------------------------------------------------------
# problem record
# ----------------------------------------------------------------------------
@dataclass
class Material:
    rho: float = 1200.0
    bulk_k: float = 2.16e7
    young_E: float = 0.0  # <= 0: E = 4k/3 (2-D, nu = 1/3)
    Gc: float = 50.0
    horizon: float = 0.0
    micro: int = MICRO_CONST


@dataclass
class Problem:
    """Everything pd_setup / the oracle need, as numpy arrays (SoA)."""
    x: np.ndarray
    y: np.ndarray
    vol: np.ndarray
    particle_offset: np.ndarray
    particle_material: np.ndarray
    particle_aggregate: np.ndarray
    materials: list
    loop_offset: np.ndarray
    loop_vertex_offset: np.ndarray
    loop_xy: np.ndarray
    box: np.ndarray  # [n_aggregates, 4] xlo, xhi, ylo, yhi at t = 0
    top_wall_speed: np.ndarray  # [n_aggregates], downward, m/s
    contact_radius: float
    friction_mu: float
    damping_ratio: float
    dt: float
    gravity: tuple = (0.0, 0.0)
    kn_mode: int = KN_SELF_CONSISTENT
    precision: int = PREC_FP64
    u0x: np.ndarray | None = None
    u0y: np.ndarray | None = None
    v0x: np.ndarray | None = None
    v0y: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def n_nodes(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_particles(self) -> int:
        return int(self.particle_offset.shape[0] - 1)

    @property
    def n_aggregates(self) -> int:
        return int(self.box.shape[0])


@dataclass
class Particle:
    shape: str
    R: float
    center: tuple
    theta: float = 0.0
    material: int = 0
    aggregate: int = 0
    velocity: tuple = (0.0, 0.0)
    nodes_body: np.ndarray | None = None  # override the lattice (tests)
    loops_body: list | None = None


def assemble(particles: list, h: float, materials: list, box, *, contact_radius: float,
             friction_mu: float, damping_ratio: float, dt: float, gravity=(0.0, 0.0),
             top_wall_speed=None, kn_mode: int = KN_SELF_CONSISTENT,
             precision: int = PREC_FP64, vol: float | None = None, meta=None) -> Problem:
    """Rotate/translate each particle's lattice and loops into the world frame."""
    xs, ys, offs, vxs, vys = [], [], [0], [], []
    loop_off, vert_off, loop_xy = [0], [0], []
    for p in particles:
        nb = p.nodes_body if p.nodes_body is not None else body_nodes(p.shape, p.R, h)
        lps = p.loops_body if p.loops_body is not None else shape_loops(p.shape, p.R)
        c, s = math.cos(p.theta), math.sin(p.theta)
        wx = p.center[0] + c * nb[:, 0] - s * nb[:, 1]
        wy = p.center[1] + s * nb[:, 0] + c * nb[:, 1]
        xs.append(wx)
        ys.append(wy)
        vxs.append(np.full(len(nb), p.velocity[0]))
        vys.append(np.full(len(nb), p.velocity[1]))
        offs.append(offs[-1] + len(nb))
        for lp in lps:
            lx = p.center[0] + c * lp[:, 0] - s * lp[:, 1]
            ly = p.center[1] + s * lp[:, 0] + c * lp[:, 1]
            loop_xy.append(np.stack([lx, ly], axis=1).ravel())
            vert_off.append(vert_off[-1] + len(lp))
        loop_off.append(loop_off[-1] + len(lps))
    x = np.concatenate(xs)
    y = np.concatenate(ys)
    box = np.asarray(box, dtype=np.float64).reshape(-1, 4)
    n_agg = box.shape[0]
    if top_wall_speed is None:
        top_wall_speed = np.zeros(n_agg)
    v0x = np.concatenate(vxs)
    v0y = np.concatenate(vys)
    return Problem(
        x=x, y=y,
        vol=np.full(x.shape, (h * h) if vol is None else vol, dtype=np.float64),
        particle_offset=np.asarray(offs, dtype=np.int32),
        particle_material=np.asarray([p.material for p in particles], dtype=np.int32),
        particle_aggregate=np.asarray([p.aggregate for p in particles], dtype=np.int32),
        materials=list(materials),
        loop_offset=np.asarray(loop_off, dtype=np.int32),
        loop_vertex_offset=np.asarray(vert_off, dtype=np.int32),
        loop_xy=(np.concatenate(loop_xy) if loop_xy else np.zeros(0)).astype(np.float64),
        box=box, top_wall_speed=np.asarray(top_wall_speed, dtype=np.float64).reshape(n_agg),
        contact_radius=float(contact_radius), friction_mu=float(friction_mu),
        damping_ratio=float(damping_ratio), dt=float(dt), gravity=tuple(gravity),
        kn_mode=kn_mode, precision=precision,
        u0x=None, u0y=None,
        v0x=v0x if np.any(v0x) else None, v0y=v0y if np.any(v0y) else None,
        meta=dict(meta or {}, h=h),
    )


# ----------------------------------------------------------------------------
# placement
# ----------------------------------------------------------------------------
def rsa_place(rng: np.random.Generator, radii: np.ndarray, width: float, height: float,
              x0: float = 0.0, y0: float = 0.0, factor: float = 1.1,
              max_tries: int = 100_000) -> np.ndarray:
    """Random sequential placement of non-overlapping security disks.

    Disk k has radius factor*radii[k]; its centre is drawn uniformly in the box
    shrunk by that radius and rejected while it overlaps an accepted disk.
    """
    centers = np.zeros((len(radii), 2))
    rs = factor * np.asarray(radii)
    # uniform grid of buckets for the overlap test
    cell = 2.0 * rs.max() if len(rs) else 1.0
    nbx = max(1, int(width / cell) + 1)
    buckets: dict = {}
    for k, r in enumerate(rs):
        if 2 * r > width or 2 * r > height:
            raise ValueError("security disk larger than the box")
        for _ in range(max_tries):
            cx = x0 + r + (width - 2 * r) * rng.random()
            cy = y0 + r + (height - 2 * r) * rng.random()
            bx, by = int((cx - x0) / cell), int((cy - y0) / cell)
            ok = True
            for dbx in (-1, 0, 1):
                for dby in (-1, 0, 1):
                    for m in buckets.get((bx + dbx) + nbx * (by + dby), ()):
                        if (cx - centers[m, 0]) ** 2 + (cy - centers[m, 1]) ** 2 < (r + rs[m]) ** 2:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if ok:
                centers[k] = (cx, cy)
                buckets.setdefault(bx + nbx * by, []).append(k)
                break
        else:
            raise RuntimeError(f"placement failed for disk {k}")
    return centers


# ----------------------------------------------------------------------------
# the configurations
# ----------------------------------------------------------------------------
def _material(h: float, micro: int = MICRO_CONST) -> Material:
    return Material(rho=1200.0, bulk_k=2.16e7, young_E=0.0, Gc=50.0, horizon=3.0 * h, micro=micro)


def two_disks(contact_active: bool = False, kn_mode: int = KN_SELF_CONSISTENT,
              dt: float = 1e-7) -> Problem:
    """Two disks of radius R = 1 mm, h = R/8, horizon 3h.

    Disk A rests on the floor of a 4R x 8R box with its lowest node at height
    R_c; disk B starts 0.5R above A moving down at 1 m/s under gravity.  The
    contact-active variant puts B at a surface gap of R_c + 0.05R and turns
    gravity off, so that the disks meet within about 500 steps.
    """
    R = 1e-3
    h = R / 8
    Rc = 0.95 * h
    yA = R + Rc
    gap = (Rc + 0.05 * R) if contact_active else 0.5 * R
    yB = yA + 2 * R + gap
    parts = [Particle("disk", R, (2 * R, yA)),
             Particle("disk", R, (2 * R, yB), velocity=(0.0, -1.0))]
    g = (0.0, 0.0) if contact_active else (0.0, -9.81)
    return assemble(parts, h, [_material(h)], [0.0, 4 * R, 0.0, 8 * R], contact_radius=Rc,
                    friction_mu=0.5, damping_ratio=0.8, dt=dt, gravity=g, kn_mode=kn_mode,
                    meta=dict(name="two_disks_contact" if contact_active else "two_disks",
                              steps=1000, R=R))


def mixed_bed(n_particles: int, h: float, box_w: float, box_h: float, seed: int, *,
              shapes=("disk", "plus", "ring"), R_range=(0.8e-3, 1.2e-3), gravity=-9.81,
              top_wall_speed: float = 0.0, dt: float = 1e-7, precision: int = PREC_FP64,
              aggregate: int = 0, x0: float = 0.0, y0: float = 0.0, rng=None,
              micro: int = MICRO_CONST, name: str = "mixed_bed") -> tuple:
    """A bed of mixed shapes in equal shares, placed by security-disk RSA.

    Draw order with numpy default_rng(seed): shape list shuffled, then per
    particle R ~ U[R_range], theta ~ U[0, 2 pi), then the placement attempts.
    Returns (particles, box).
    """
    rng = np.random.default_rng(seed) if rng is None else rng
    k = len(shapes)
    counts = [n_particles // k + (1 if i < n_particles % k else 0) for i in range(k)]
    kinds = []
    for s, c in zip(shapes, counts):
        kinds += [s] * c
    kinds = [kinds[i] for i in rng.permutation(len(kinds))]
    Rs = rng.uniform(R_range[0], R_range[1], size=n_particles)
    th = rng.uniform(0.0, 2 * np.pi, size=n_particles)
    centers = rsa_place(rng, Rs, box_w, box_h, x0=x0, y0=y0)
    parts = [Particle(kinds[i], float(Rs[i]), (float(centers[i, 0]), float(centers[i, 1])),
                      float(th[i]), 0, aggregate) for i in range(n_particles)]
    box = [x0, x0 + box_w, y0, y0 + box_h]
    return parts, box


def settling(n_particles: int = 100, h: float = 0.0904e-3, gravity: float = -9.81,
             seed: int = 2, dt: float = 1e-7, precision: int = PREC_FP64) -> Problem:
    """Plain FP64 settling: equal thirds of disks, plus shapes and rings in a 30R x 60R box."""
    Rn = 1e-3
    parts, box = mixed_bed(n_particles, h, 30 * Rn, 60 * Rn, seed)
    return assemble(parts, h, [_material(h)], box, contact_radius=0.95 * h, friction_mu=0.5,
                    damping_ratio=0.8, dt=dt, gravity=(0.0, gravity), precision=precision,
                    meta=dict(name=f"settling_{n_particles}", seed=seed, steps=20000))


def compaction(n_particles: int = 500, h: float = 0.070e-3, seed: int = 3,
               wall_speed: float = 0.1, dt: float = 1e-7, precision: int = PREC_FP64,
               box_scale: float | None = None) -> Problem:
    """Compaction: mixed shapes, no gravity, top wall moving down at wall_speed.

    The box keeps the settling bed's fill fraction: 30R x 60R scaled by
    sqrt(n/100).
    """
    Rn = 1e-3
    sc = math.sqrt(n_particles / 100.0) if box_scale is None else box_scale
    parts, box = mixed_bed(n_particles, h, 30 * Rn * sc, 60 * Rn * sc, seed)
    return assemble(parts, h, [_material(h)], box, contact_radius=0.95 * h, friction_mu=0.5,
                    damping_ratio=0.8, dt=dt, gravity=(0.0, 0.0), precision=precision,
                    top_wall_speed=[wall_speed],
                    meta=dict(name=f"compaction_{n_particles}", seed=seed))


def batched(n_aggregates: int = 64, h: float = 0.078e-3, seed: int = 4,
            n_range=(50, 400), dt: float = 1e-7, gravity: float = -9.81,
            precision: int = PREC_FP32_FORCE) -> Problem:
    """Independent settling aggregates of uneven size in one problem.

    Aggregate a has n_a ~ U{n_range} particles drawn uniformly from disk, plus
    and ring, in its own box 30R sqrt(n_a/100) x 60R sqrt(n_a/100); the boxes
    are laid side by side (they never interact: each aggregate has its own
    walls and its own cells).
    """
    Rn = 1e-3
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_range[0], n_range[1] + 1, size=n_aggregates)
    parts, boxes = [], []
    xoff = 0.0
    for a, na in enumerate(ns):
        sc = math.sqrt(na / 100.0)
        w, hh = 30 * Rn * sc, 60 * Rn * sc
        kinds = rng.choice(np.array(["disk", "plus", "ring"]), size=na)
        Rs = rng.uniform(0.8e-3, 1.2e-3, size=na)
        th = rng.uniform(0.0, 2 * np.pi, size=na)
        centers = rsa_place(rng, Rs, w, hh, x0=xoff, y0=0.0)
        parts += [Particle(str(kinds[i]), float(Rs[i]), (float(centers[i, 0]), float(centers[i, 1])),
                           float(th[i]), 0, a) for i in range(na)]
        boxes.append([xoff, xoff + w, 0.0, hh])
        xoff += w + 10 * Rn
    return assemble(parts, h, [_material(h)], boxes, contact_radius=0.95 * h, friction_mu=0.5,
                    damping_ratio=0.8, dt=dt, gravity=(0.0, gravity), precision=precision,
                    meta=dict(name=f"batched_{n_aggregates}", seed=seed,
                              particles_per_aggregate=ns.tolist()))


def subproblem_aggregate(prob: Problem, a: int) -> Problem:
    """The nodes, particles and box of aggregate a alone, as a problem of its own."""
    pa = prob.particle_aggregate
    sel = np.nonzero(pa == a)[0]
    p0, p1 = int(sel[0]), int(sel[-1]) + 1
    assert np.all(np.diff(sel) == 1)
    n0, n1 = int(prob.particle_offset[p0]), int(prob.particle_offset[p1])
    l0, l1 = int(prob.loop_offset[p0]), int(prob.loop_offset[p1])
    v0, v1 = int(prob.loop_vertex_offset[l0]), int(prob.loop_vertex_offset[l1])

    def cut(arr):
        return None if arr is None else arr[n0:n1].copy()

    return Problem(
        x=prob.x[n0:n1].copy(), y=prob.y[n0:n1].copy(), vol=prob.vol[n0:n1].copy(),
        particle_offset=(prob.particle_offset[p0:p1 + 1] - n0).astype(np.int32),
        particle_material=prob.particle_material[p0:p1].copy(),
        particle_aggregate=np.zeros(p1 - p0, dtype=np.int32),
        materials=prob.materials,
        loop_offset=(prob.loop_offset[p0:p1 + 1] - l0).astype(np.int32),
        loop_vertex_offset=(prob.loop_vertex_offset[l0:l1 + 1] - v0).astype(np.int32),
        loop_xy=prob.loop_xy[2 * v0:2 * v1].copy(),
        box=prob.box[a:a + 1].copy(), top_wall_speed=prob.top_wall_speed[a:a + 1].copy(),
        contact_radius=prob.contact_radius, friction_mu=prob.friction_mu,
        damping_ratio=prob.damping_ratio, dt=prob.dt, gravity=prob.gravity,
        kn_mode=prob.kn_mode, precision=prob.precision,
        u0x=cut(prob.u0x), u0y=cut(prob.u0y), v0x=cut(prob.v0x), v0y=cut(prob.v0y),
        meta=dict(prob.meta, aggregate=a),
    )


def herd(prob: Problem, alpha: float) -> Problem:
    """Translate every particle rigidly toward the bed centre by the fraction
    alpha of its distance: a synthetic packed state with contacts (and
    overlaps) at t = 0, a stress case for contact and breaking."""
    cx, cy = prob.x.mean(), prob.y.mean()
    po = prob.particle_offset
    ux, uy = np.zeros(prob.n_nodes), np.zeros(prob.n_nodes)
    for p in range(prob.n_particles):
        sl = slice(po[p], po[p + 1])
        ux[sl] = -alpha * (prob.x[sl].mean() - cx)
        uy[sl] = -alpha * (prob.y[sl].mean() - cy)
    prob.u0x, prob.u0y = ux, uy
    return prob


def single_node_particles(points, velocities, vol: float, box, *, contact_radius: float,
                          h: float, friction_mu=0.0, damping_ratio=0.0, dt=1e-8,
                          gravity=(0.0, 0.0), kn_mode=KN_SELF_CONSISTENT,
                          material: Material | None = None) -> Problem:
    """Particles of one node each (no bonds): the contact law in isolation."""
    mat = material or _material(h)
    parts = [Particle("disk", 0.0, tuple(p), 0.0, velocity=tuple(v),
                      nodes_body=np.zeros((1, 2)), loops_body=[])
             for p, v in zip(points, velocities)]
    return assemble(parts, h, [mat], box, contact_radius=contact_radius,
                    friction_mu=friction_mu, damping_ratio=damping_ratio, dt=dt,
                    gravity=gravity, kn_mode=kn_mode, vol=vol)


def perturb(prob: Problem, seed: int, du: float = 0.0, dv: float = 0.0) -> Problem:
    """Add seeded uniform noise of amplitude du to u0 and dv to v0 (test inputs)."""
    rng = np.random.default_rng(seed)
    n = prob.n_nodes
    if du:
        prob.u0x = (prob.u0x if prob.u0x is not None else 0.0) + du * rng.uniform(-1, 1, n)
        prob.u0y = (prob.u0y if prob.u0y is not None else 0.0) + du * rng.uniform(-1, 1, n)
    if dv:
        prob.v0x = (prob.v0x if prob.v0x is not None else 0.0) + dv * rng.uniform(-1, 1, n)
        prob.v0y = (prob.v0y if prob.v0y is not None else 0.0) + dv * rng.uniform(-1, 1, n)
    return prob


def particle_velocities(prob: Problem, seed: int, vmax: float) -> Problem:
    """Give every particle a seeded rigid velocity, uniform in [-vmax, vmax]^2."""
    rng = np.random.default_rng(seed)
    vel = rng.uniform(-vmax, vmax, size=(prob.n_particles, 2))
    counts = np.diff(prob.particle_offset)
    prob.v0x = np.repeat(vel[:, 0], counts)
    prob.v0y = np.repeat(vel[:, 1], counts)
    return prob


CLOSURE_SHAPES = ("disk", "plus", "ring", "lshape")


def closure_radius(shape: str, h: float, nodes: int) -> float:
    """The size R at which the shape's lattice holds about `nodes` nodes
    (area / h^2 = nodes)."""
    return h * math.sqrt(nodes / shape_area(shape, 1.0))


def closure_bed(n_per_shape: int = 500, h: float = 0.08e-3, nodes: int = 400, seed: int = 5,
                wall_speed: float = 0.1, vmax: float = 0.0, fill_scale: float = 1.0,
                gravity: float = 0.0, dt: float = 1e-7, shapes=CLOSURE_SHAPES) -> Problem:
    """Fixed shapes for the modal closure: n_per_shape particles of each shape,
    every instance of a shape with the same size R (so the same body-frame
    node set, and one mode basis per shape), random orientation, placed by
    security-disk RSA in a box 30 x 60 R_mean scaled by sqrt(n/100) x
    fill_scale, top wall moving down at wall_speed, optional seeded rigid
    velocities uniform in [-vmax, vmax]^2.

    Draw order with default_rng(seed): shape list shuffled, theta per
    particle, placement attempts, then the velocities.
    """
    rng = np.random.default_rng(seed)
    Rs = {s: closure_radius(s, h, nodes) for s in shapes}
    kinds = []
    for s in shapes:
        kinds += [s] * n_per_shape
    kinds = [kinds[i] for i in rng.permutation(len(kinds))]
    n = len(kinds)
    th = rng.uniform(0.0, 2 * np.pi, size=n)
    # security disks bound the particle: the L shape's farthest vertex from
    # its centroid is beyond R
    bound = {s: max(np.hypot(lp[:, 0], lp[:, 1]).max() for lp in shape_loops(s, Rs[s]))
             if shape_loops(s, Rs[s]) else Rs[s] for s in shapes}
    radii = np.array([bound[k] for k in kinds])
    Rm = float(np.mean(radii))
    sc = math.sqrt(n / 100.0) * fill_scale
    w, hh = 30 * Rm * sc, 60 * Rm * sc
    centers = rsa_place(rng, radii, w, hh)
    parts = [Particle(kinds[i], Rs[kinds[i]], (float(centers[i, 0]), float(centers[i, 1])),
                      float(th[i]), 0, 0) for i in range(n)]
    prob = assemble(parts, h, [_material(h)], [0.0, w, 0.0, hh], contact_radius=0.95 * h,
                    friction_mu=0.5, damping_ratio=0.8, dt=dt, gravity=(0.0, gravity),
                    top_wall_speed=[wall_speed],
                    meta=dict(name=f"closure_{n}", seed=seed, shapes=list(shapes),
                              R=Rs, kinds=kinds))
    prob.meta["shape_of_particle"] = np.array([list(shapes).index(k) for k in kinds], dtype=np.int32)
    if vmax > 0:
        vel = rng.uniform(-vmax, vmax, size=(n, 2))
        counts = np.diff(prob.particle_offset)
        prob.v0x = np.repeat(vel[:, 0], counts)
        prob.v0y = np.repeat(vel[:, 1], counts)
    return prob


def jitter_nodes(prob: Problem, seed: int, vol_frac: float = 0.4, pos_frac: float = 0.25) -> Problem:
    """Unstructured-like nodes: every nodal volume scaled by a seeded factor
    uniform in [1 - vol_frac, 1 + vol_frac], and the nodes of particles
    without boundary loops (disks) moved by a seeded offset uniform in
    [-pos_frac h, pos_frac h]^2 (such a particle has no boundary a node could
    cross).  Draw order: volumes, then offsets."""
    rng = np.random.default_rng(seed)
    h = prob.meta["h"]
    prob.vol = prob.vol * rng.uniform(1.0 - vol_frac, 1.0 + vol_frac, prob.n_nodes)
    dx = rng.uniform(-pos_frac * h, pos_frac * h, (prob.n_nodes, 2))
    lo = prob.loop_offset
    po = prob.particle_offset
    x, y = prob.x.copy(), prob.y.copy()
    for p in range(prob.n_particles):
        if lo[p + 1] == lo[p]:
            s = slice(po[p], po[p + 1])
            x[s] += dx[s, 0]
            y[s] += dx[s, 1]
    prob.x, prob.y = x, y
    prob.meta = dict(prob.meta, jitter=(seed, vol_frac, pos_frac))
    return prob


# ----------------------------------------------------------------------------
# notched square hit by two rectangles (Sec. 7.3)
# ----------------------------------------------------------------------------
def cell_nodes(half_w: float, half_h: float, h: float) -> np.ndarray:
    """Cell centres ((i + 1/2) h, (j + 1/2) h) of the uniform grid that tiles
    the rectangle [-half_w, half_w] x [-half_h, half_h], body frame, row-major
    (j outer).  No node lies on the rectangle's edges or on its mid-lines."""
    nx, ny = int(round(half_w / h)), int(round(half_h / h))
    if nx < 1 or ny < 1 or abs(nx * h - half_w) > 1e-9 * h or abs(ny * h - half_h) > 1e-9 * h:
        raise ValueError("half sizes must be whole multiples of h")
    xs = (np.arange(-nx, nx) + 0.5) * h
    ys = (np.arange(-ny, ny) + 0.5) * h
    gy, gx = np.meshgrid(ys, xs, indexing="ij")
    return np.stack([gx.ravel(), gy.ravel()], axis=1)


def notched_square_loop(R: float, notch_half_width: float) -> np.ndarray:
    """Counter-clockwise boundary of the square [-R, R]^2 with a slot of
    half-width notch_half_width along y = 0 from the left edge to the
    centre."""
    w = notch_half_width
    return np.array([(-R, -R), (R, -R), (R, R), (-R, R), (-R, w), (0.0, w), (0.0, -w), (-R, -w)],
                    dtype=np.float64)


def notched_impact(Gc: float = 135.0, side: float = 1e-3, n_side: int = 50, speed: float = 20.0,
                   horizon_factor: float = 3.0, dt: float = 2e-9, gap: float | None = None,
                   material: str = "M1", precision: int = PREC_FP64) -> Problem:
    """Sec. 7.3: a square particle A of side `side` with a notch from the
    middle of its left edge to its centre, struck at the same time from above
    and below by rectangles B and C of side x side/2 moving at +-`speed`
    toward it; friction and damping off, no gravity.

    The paper gives neither the mesh size nor the horizon.  Here the nodes
    are the cell centres of a grid of spacing h = side / n_side (so no node
    lies on the notch line), the horizon is horizon_factor * h, and the notch
    is a slot of width h/5 (narrower than the node spacing: it removes
    exactly the bonds that cross the notch line left of the centre).  The
    material is M1 of Tab. tab:material (E = 191 GPa, k = 159.2 GPa,
    rho = 8000 kg/m^3), the one the paper assigns to its two- and
    three-particle tests, or M2 (E = 1.23 GPa, k = 2 GPa, rho = 1200 kg/m^3),
    with the given toughness Gc.  B and C start with a
    surface gap of `gap` (default h) to A.  Particle order: A, B, C.
    """
    h = side / n_side
    R = 0.5 * side
    if n_side % 2:
        raise ValueError("n_side must be even (the notch runs between node rows)")
    g = h if gap is None else gap
    rho, k, E = {"M1": (8000.0, 159.2e9, 191e9), "M2": (1200.0, 2e9, 1.23e9)}[material]
    mat = Material(rho=rho, bulk_k=k, young_E=E, Gc=Gc, horizon=horizon_factor * h)
    nodes_a = cell_nodes(R, R, h)
    nodes_r = cell_nodes(R, 0.5 * R, h)
    rect = [np.array([(-R, -0.5 * R), (R, -0.5 * R), (R, 0.5 * R), (-R, 0.5 * R)])]
    L = 6.0 * R
    yb = R + g + 0.5 * R
    parts = [Particle("notched", R, (0.0, 0.0), nodes_body=nodes_a,
                      loops_body=[notched_square_loop(R, 0.1 * h)]),
             Particle("rect", R, (0.0, yb), velocity=(0.0, -speed), nodes_body=nodes_r,
                      loops_body=rect),
             Particle("rect", R, (0.0, -yb), velocity=(0.0, speed), nodes_body=nodes_r,
                      loops_body=rect)]
    return assemble(parts, h, [mat], [-L, L, -L, L], contact_radius=0.95 * h, friction_mu=0.0,
                    damping_ratio=0.0, dt=dt, gravity=(0.0, 0.0), precision=precision,
                    meta=dict(name=f"notched_impact_{material}_Gc{Gc:g}", Gc=Gc, side=side,
                              n_side=n_side, speed=speed, material=material))


# ----------------------------------------------------------------------------
# jammed security disks (Sec. 7.1)
# ----------------------------------------------------------------------------
def triangle_incircles(pts: np.ndarray, tri: np.ndarray):
    """Incircle of every triangle (Sec. 7.1, step 2): centre
    (v1 l1 + v2 l2 + v3 l3) / (l1 + l2 + l3) with l_k the length of the side
    opposite v_k, radius 2 |T| / (l1 + l2 + l3)."""
    v1, v2, v3 = pts[tri[:, 0]], pts[tri[:, 1]], pts[tri[:, 2]]
    l1 = np.linalg.norm(v2 - v3, axis=1)
    l2 = np.linalg.norm(v1 - v3, axis=1)
    l3 = np.linalg.norm(v1 - v2, axis=1)
    per = l1 + l2 + l3
    c = (v1 * l1[:, None] + v2 * l2[:, None] + v3 * l3[:, None]) / per[:, None]
    area = 0.5 * np.abs((v2[:, 0] - v1[:, 0]) * (v3[:, 1] - v1[:, 1])
                        - (v3[:, 0] - v1[:, 0]) * (v2[:, 1] - v1[:, 1]))
    return c, 2.0 * area / per


def _box_mesh(width: float, height: float, size: float, rng: np.random.Generator,
              jitter: float = 0.15):
    """Triangular mesh of the box [0, width] x [0, height]: nodes every ~size
    along the edges (corners included) and a jittered triangular lattice of
    spacing size inside, kept half a spacing from the edges; Delaunay
    triangles (the box is convex, so they tile it)."""
    from scipy.spatial import Delaunay
    nx = max(1, int(round(width / size)))
    ny = max(1, int(round(height / size)))
    bx = np.linspace(0.0, width, nx + 1)
    by = np.linspace(0.0, height, ny + 1)[1:-1]
    bnd = np.concatenate([np.stack([bx, np.zeros_like(bx)], 1), np.stack([bx, np.full_like(bx, height)], 1),
                          np.stack([np.zeros_like(by), by], 1), np.stack([np.full_like(by, width), by], 1)])
    dy = size * math.sqrt(3.0) / 2.0
    rows = []
    for r in range(int(height / dy) + 2):
        y = r * dy
        xs = np.arange(0.0, width + size, size) + (0.5 * size if r % 2 else 0.0)
        rows.append(np.stack([xs, np.full_like(xs, y)], 1))
    inner = np.concatenate(rows)
    inner = inner + rng.uniform(-jitter * size, jitter * size, inner.shape)
    m = 0.5 * size
    keep = ((inner[:, 0] > m) & (inner[:, 0] < width - m) & (inner[:, 1] > m)
            & (inner[:, 1] < height - m))
    pts = np.concatenate([bnd, inner[keep]])
    tri = Delaunay(pts).simplices
    v1, v2, v3 = pts[tri[:, 0]], pts[tri[:, 1]], pts[tri[:, 2]]
    area = 0.5 * np.abs((v2[:, 0] - v1[:, 0]) * (v3[:, 1] - v1[:, 1])
                        - (v3[:, 0] - v1[:, 0]) * (v2[:, 1] - v1[:, 1]))
    return pts, tri[area > 1e-9 * size * size]


def jammed_disks(width: float, height: float, mesh_size: float, seed: int, shrink: float = 0.0,
                 x0: float = 0.0, y0: float = 0.0):
    """Security disks by the construction of Sec. 7.1: a triangular mesh of the
    box, the incircle of every triangle, and for every mesh node v the largest
    circle centred in the star of v (the triangles at v) that meets no
    incircle of the triangles at v or next to them and stays in the box: its
    centre c maximises min(min_T |c - c_T| - r_T, distance to the box edges),
    found by Nelder-Mead from v; nodal circles that still overlap one another
    give up the overlap in equal parts.  Then every radius shrinks by
    `shrink` (R_c / 2 in the paper); disks left with no positive radius are
    dropped.  Returns (centres [n, 2], radii [n], stats, origin [n]) with
    origin -1 for an incircle and the mesh node for a nodal circle."""
    from scipy.optimize import minimize
    rng = np.random.default_rng(seed)
    pts, tri = _box_mesh(width, height, mesh_size, rng)
    cT, rT = triangle_incircles(pts, tri)
    star = [[] for _ in range(len(pts))]
    for t, (a, b, c) in enumerate(tri):
        star[a].append(t)
        star[b].append(t)
        star[c].append(t)
    box_area = width * height
    phi_incircles = float(np.sum(np.pi * rT ** 2) / box_area)
    cn = np.zeros_like(pts)
    rn = np.zeros(len(pts))
    for v in range(len(pts)):
        ts = np.array(star[v], dtype=np.int64)
        ring = np.unique(np.concatenate([star[w] for w in np.unique(tri[ts])]))
        cc, rr = cT[ring], rT[ring]
        A, B, Cc = pts[tri[ts, 0]], pts[tri[ts, 1]], pts[tri[ts, 2]]

        def in_star(c):
            d1 = (B[:, 0] - A[:, 0]) * (c[1] - A[:, 1]) - (B[:, 1] - A[:, 1]) * (c[0] - A[:, 0])
            d2 = (Cc[:, 0] - B[:, 0]) * (c[1] - B[:, 1]) - (Cc[:, 1] - B[:, 1]) * (c[0] - B[:, 0])
            d3 = (A[:, 0] - Cc[:, 0]) * (c[1] - Cc[:, 1]) - (A[:, 1] - Cc[:, 1]) * (c[0] - Cc[:, 0])
            neg = (d1 < 0) | (d2 < 0) | (d3 < 0)
            pos = (d1 > 0) | (d2 > 0) | (d3 > 0)
            return bool(np.any(~(neg & pos)))

        def gap(c):
            if not in_star(c):
                return -1.0
            d = np.sqrt((cc[:, 0] - c[0]) ** 2 + (cc[:, 1] - c[1]) ** 2) - rr
            return min(d.min(), c[0], width - c[0], c[1], height - c[1])

        # start a hair inside the star (boundary nodes sit on the box edge)
        start = pts[v] + 1e-3 * (cT[ts].mean(axis=0) - pts[v])
        r0 = gap(start)
        res = minimize(lambda c: -gap(c), start, method="Nelder-Mead",
                       options=dict(xatol=1e-9 * mesh_size, fatol=1e-12 * mesh_size, maxiter=4000))
        cn[v], rn[v] = (res.x, -res.fun) if -res.fun > r0 else (start, r0)
    # nodal circles of neighbouring nodes may still meet: split each overlap
    from scipy.spatial import cKDTree
    tree = cKDTree(cn)
    overlaps = 0
    for a, b in sorted(tree.query_pairs(2.0 * max(rn.max(), 1e-300))):
        d = float(np.hypot(*(cn[a] - cn[b])))
        o = rn[a] + rn[b] - d
        if o > 0:
            overlaps += 1
            rn[a] -= 0.5 * o
            rn[b] -= 0.5 * o
    centres = np.concatenate([cT, cn])
    radii = np.concatenate([rT, rn])
    # what the optimiser's tolerance leaves of overlaps with incircles farther
    # away: the nodal circle gives it up
    nT = len(rT)
    tree = cKDTree(centres)
    for a, b in sorted(tree.query_pairs(2.0 * float(radii.max()))):
        o = radii[a] + radii[b] - float(np.hypot(*(centres[a] - centres[b])))
        if o > 0:
            k = b if b >= nT else a
            if k < nT:
                raise RuntimeError("incircles of a triangulation overlap")
            radii[k] -= o
    phi_jammed = float(np.sum(np.pi * radii[radii > 0] ** 2) / box_area)
    radii = radii - shrink
    keep = radii > 0
    stats = dict(mesh_nodes=int(len(pts)), triangles=int(len(tri)),
                 packing_incircles=phi_incircles, packing_jammed=phi_jammed,
                 packing_final=float(np.sum(np.pi * radii[keep] ** 2) / box_area),
                 nodal_overlaps_split=overlaps, dropped=int((~keep).sum()))
    centres = centres[keep] + np.array([x0, y0])
    origin = np.concatenate([np.full(len(rT), -1), np.arange(len(rn))])[keep]
    return centres, radii[keep], stats, origin


def jammed_compaction(width: float = 40e-3, height: float = 40e-3, mesh_size: float = 3.2e-3,
                      seed: int = 3, h: float = 0.070e-3, r_min: float = 0.4e-3,
                      wall_speed: float = 0.1, dt: float = 1e-7,
                      precision: int = PREC_FP64) -> Problem:
    """Compaction of mixed particles from a jammed start (Sec. 7.4 with the
    initial configuration of Sec. 7.1): security disks of jammed_disks over
    the container inset by R_c / 2, shrunk by R_c / 2 and kept if of radius
    >= r_min (510 in a 40 x 40 mm box with mesh size 3.2 mm); in each an
    equal-thirds mix of disks, plus shapes (half-length R, arm width R/2) and
    rings (inner radius R/2) whose farthest point lies on the disk's circle,
    randomly oriented;
    h = 0.070 mm, horizon 3h, R_c = 0.95 h, the configs' material (G_c =
    50 J/m^2), mu = 0.5, r_d = 0.8, no gravity, the top wall moving down at
    wall_speed.

    Draw order: the mesh jitter (default_rng(seed)), then default_rng(seed +
    1) for the shape list's shuffle and the orientations."""
    Rc = 0.95 * h
    centres, radii, st, _ = jammed_disks(width - Rc, height - Rc, mesh_size, seed,
                                         shrink=0.5 * Rc, x0=0.5 * Rc, y0=0.5 * Rc)
    keep = radii >= r_min
    centres, radii = centres[keep], radii[keep]
    n = len(radii)
    rng = np.random.default_rng(seed + 1)
    kinds = [("disk", "plus", "ring")[k % 3] for k in range(n)]
    kinds = [kinds[i] for i in rng.permutation(n)]
    th = rng.uniform(0.0, 2.0 * np.pi, size=n)
    # a plus of half-length R reaches sqrt(1 + 1/16) R at its arm corners:
    # scaled so that its farthest point lies on the disk's circle
    reach = {"disk": 1.0, "ring": 1.0, "plus": math.sqrt(1.0 + 1.0 / 16.0)}
    parts = [Particle(kinds[k], float(radii[k]) / reach[kinds[k]],
                      (float(centres[k, 0]), float(centres[k, 1])), float(th[k])) for k in range(n)]
    return assemble(parts, h, [_material(h)], [0.0, width, 0.0, height], contact_radius=Rc,
                    friction_mu=0.5, damping_ratio=0.8, dt=dt, gravity=(0.0, 0.0),
                    top_wall_speed=[wall_speed], precision=precision,
                    meta=dict(name="jammed_compaction", seed=seed, packing=st,
                              dropped_small=int((~keep).sum())))


def restart_with_wall(prob: Problem, state: dict, wall_y: float, speed: float) -> Problem:
    """The same nodes, particles and materials, with the displacement and
    velocity of `state` as the initial condition and the top wall of the
    (single) aggregate at height wall_y moving down at `speed`: a run that
    continues from a checkpoint with a new wall motion (the checkpoint's
    accelerations and broken bonds are loaded with pd_set_state)."""
    import copy
    out = copy.copy(prob)
    out.box = prob.box.copy()
    out.box[0, 3] = wall_y
    out.top_wall_speed = np.array([speed], dtype=np.float64)
    out.u0x, out.u0y = np.asarray(state["ux"]).copy(), np.asarray(state["uy"]).copy()
    out.v0x, out.v0y = np.asarray(state["vx"]).copy(), np.asarray(state["vy"]).copy()
    out.meta = dict(prob.meta, restart=True)
    return out


SETTLE_SHAPES = ("pdisk", "square", "plus", "ring")


def jammed_settling(shape: str, width: float = 25e-3, height: float = 50e-3,
                    mesh_size: float = 3.2e-3, seed: int = 6, eps: float = 0.5e-3,
                    r_min: float = 0.4e-3, gravity: float = -5000.0, dt: float = 70e-9,
                    Gc: float | None = None, precision: int = PREC_FP64) -> Problem:
    """Settling of one particle shape from jammed security disks (Sec. 7.3):
    the disks of jammed_disks over the container inset by R_c / 2 (mesh size
    mesh_size), shrunk by R_c / 2 and keeping those of radius >= r_min; in each a
    particle whose farthest point lies on the disk's circle, randomly
    oriented about the disk's centre.  Shapes with the parameters of Sec. 7.2:
    "pdisk" (perturbed disk, 20 vertices, phi = 0.6, a polygon of its own per
    particle), "square" (side sqrt(2) R), "plus" (inner radius 0.2 R),
    "ring" (inner radius 0.6 R), and "disk".  Parameters of Sec. 7.3: eps = 0.5 mm, h = eps/8,
    R_c = eps/5, mu = 0.8, r_d = 0.8, g = 5000 m/s^2, dt = 70 ns, material M2
    of Tab. tab:material (E = 1.23 GPa, k = 2 GPa, rho = 1200 kg/m^3).  The
    paper turns damage on only for its compaction study (Sec. 7.4), so by
    default bonds do not break here (Gc = None: a toughness so large that
    the critical stretch is never reached); a value turns damage on.

    Draw order: the mesh jitter (default_rng(seed)), then default_rng(seed + 1)
    for the orientations and, for perturbed disks, the vertex radii
    particle by particle."""
    h = eps / 8.0
    Rc = eps / 5.0
    # jammed in the container inset by R_c / 2, then shrunk by R_c / 2: every
    # gap between particles and to the walls is at least R_c, so no contact or
    # wall force acts at t = 0
    centres, radii, st, _ = jammed_disks(width - Rc, height - Rc, mesh_size, seed,
                                         shrink=0.5 * Rc, x0=0.5 * Rc, y0=0.5 * Rc)
    keep = radii >= r_min
    centres, radii = centres[keep], radii[keep]
    rng = np.random.default_rng(seed + 1)
    th = rng.uniform(0.0, 2.0 * np.pi, size=len(radii))
    parts = []
    for k, (c, rs) in enumerate(zip(centres, radii)):
        cen = (float(c[0]), float(c[1]))
        if shape == "pdisk":
            lp = perturbed_disk_loop(float(rs), rng)
            parts.append(Particle("pdisk", float(rs), cen, float(th[k]), loops_body=[lp],
                                  nodes_body=loop_nodes([lp], float(rs), h)))
        elif shape in ("plus", "ring"):
            lps = [plus_loop(float(rs))] if shape == "plus" else ring_loops(float(rs))
            parts.append(Particle(shape, float(rs), cen, float(th[k]), loops_body=lps,
                                  nodes_body=loop_nodes(lps, float(rs), h)))
        elif shape in ("square", "disk"):
            parts.append(Particle(shape, float(rs), cen, float(th[k])))
        else:
            raise ValueError(f"unknown shape {shape!r}")
    mat = Material(rho=1200.0, bulk_k=2e9, young_E=1.23e9, Gc=1e30 if Gc is None else Gc,
                   horizon=eps)
    prob = assemble(parts, h, [mat], [0.0, width, 0.0, height], contact_radius=Rc,
                    friction_mu=0.8, damping_ratio=0.8, dt=dt, gravity=(0.0, gravity),
                    precision=precision,
                    meta=dict(name=f"jammed_settling_{shape}", shape=shape, seed=seed,
                              security_radii=radii, packing=st, dropped_small=int((~keep).sum())))
    # area the particle occupies inside its outer boundary (holes filled):
    # the paper's annulus fractions count the hole as particle volume
    prob.meta["filled_area"] = float(sum(
        abs(polygon_area([p.loops_body[0] if p.loops_body else shape_loops(p.shape, p.R)[0]]))
        for p in parts))
    return prob
