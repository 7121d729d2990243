"""FP64 reference of the learned modal closure -- TEST INFRASTRUCTURE.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark
use this module; the library never imports it.

The paper has no reduced-order model: this follows the project's own
definition of one, written out plainly (numpy / scipy, float64):

* the linearized bond force of eq. (peri) about the reference configuration
  gives a stiffness K per particle shape; with the lumped mass M = diag(rho V)
  the lowest non-rigid solutions of K phi = lambda M phi (three rigid modes
  excluded), normalised phi^T M phi = 1, are the modes;
* a particle's deformation is read in its best-fit rotated frame (weighted
  2-D Procrustes about the mass centroid), projected on the modes
  (q = Phi^T M u), and its internal force is replaced by M Phi g(q) rotated
  back, with g(q) = -lambda q (linear closure) or -lambda q + sigma_r
  MLP(q / sigma_q) (learned closure);
* the particle moves as a rigid body plus those modes: the external nodal
  forces are split into total force, torque about the centroid and modal
  force, and the nodal acceleration is rebuilt from them (Galerkin
  projection; coupling between the rotation and the modal inertia is left
  out).

The MLP is 32 -> 256 -> 256 -> 32 with SiLU after the two hidden layers.
Weights are stored [out][in]; the packed order is W1, b1, W2, b2, W3, b3.
With bf16=True the forward and backward round the operands of every matrix
product to bfloat16 (round to nearest even) at the same points as the GPU
kernels: the normalised input, the weights, the two hidden activations and
the three back-propagated signals dy, dz2, dz1; sums are exact (float64)
here, float32 on the GPU.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

N_RIGID = 3
N_IN = 32
N_HID = 256
LAYERS = ((N_HID, N_IN), (N_HID, N_HID), (N_IN, N_HID))  # (out, in) per layer
N_PARAMS = sum(o * i + o for o, i in LAYERS)


# ----------------------------------------------------------------------------
# shapes, stiffness and modes
# ----------------------------------------------------------------------------
def particle_range(prob, p):
    return int(prob.particle_offset[p]), int(prob.particle_offset[p + 1])


def node_masses(prob, p):
    n0, n1 = particle_range(prob, p)
    rho = prob.materials[int(prob.particle_material[p])].rho
    return rho * prob.vol[n0:n1]


def reference_frame(prob, p):
    """Mass centroid and centred reference coordinates of particle p."""
    n0, n1 = particle_range(prob, p)
    m = node_masses(prob, p)
    xy = np.stack([prob.x[n0:n1], prob.y[n0:n1]], axis=1)
    c0 = (m[:, None] * xy).sum(0) / m.sum()
    return c0, xy - c0


def best_fit_angle(X, Y, m):
    """Angle of the rotation R minimising sum m |R X - Y|^2 (X, Y centred):
    R(phi) X . Y = cos(phi) sum m X.Y + sin(phi) sum m X x Y is largest at
    phi = atan2(sum m X x Y, sum m X.Y)."""
    cross = (m * (X[:, 0] * Y[:, 1] - X[:, 1] * Y[:, 0])).sum()
    dot = (m * (X[:, 0] * Y[:, 0] + X[:, 1] * Y[:, 1])).sum()
    return float(np.arctan2(cross, dot))


def rot(phi, V):
    c, s = np.cos(phi), np.sin(phi)
    return np.stack([c * V[:, 0] - s * V[:, 1], s * V[:, 0] + c * V[:, 1]], axis=1)


def stiffness(prob, p, row, col, cw, horizon, micro):
    """K of particle p (2n x 2n, dof order x0, y0, x1, y1, ...): the bond
    force c_w w s V_i V_j e of eq. (peri) with the stretch linearised,
    s = (u_j - u_i).e / |xi|, gives on node i the force
    k (e e^T)(u_j - u_i), k = c_w w V_i V_j / |xi|, and K = -dF/du."""
    n0, n1 = particle_range(prob, p)
    n = n1 - n0
    K = np.zeros((2 * n, 2 * n))
    for i in range(n0, n1):
        for k in range(row[i], row[i + 1]):
            j = int(col[k])
            dx, dy = prob.x[j] - prob.x[i], prob.y[j] - prob.y[i]
            L = np.hypot(dx, dy)
            e = np.array([dx / L, dy / L])
            w = 1.0 if micro == 0 else 1.0 - L / horizon
            kk = cw * w * prob.vol[i] * prob.vol[j] / L
            B = kk * np.outer(e, e)
            a, b = 2 * (i - n0), 2 * (j - n0)
            K[a:a + 2, a:a + 2] += B
            K[a:a + 2, b:b + 2] -= B
    return K


def modes(K, m, n_modes=N_IN):
    """Lowest n_modes non-rigid solutions of K phi = lambda M phi,
    M = diag(m_0, m_0, m_1, m_1, ...), with phi^T M phi = I (scipy's
    generalized symmetric eigensolver). Returns (lambda, Phi [2n x n_modes],
    all eigenvalues)."""
    M = np.repeat(m, 2)
    lam, vec = scipy.linalg.eigh(K, np.diag(M))
    return lam[N_RIGID:N_RIGID + n_modes].copy(), vec[:, N_RIGID:N_RIGID + n_modes].copy(), lam


def stretch_bound(prob, p, row, col, Phi):
    """sigma_k = max over the particle's bonds of |linear stretch of mode k|:
    for amplitudes q, max |s| <= sum_k |q_k| sigma_k to first order."""
    n0, n1 = particle_range(prob, p)
    P = Phi.reshape(n1 - n0, 2, -1)
    sig = np.zeros(Phi.shape[1])
    for i in range(n0, n1):
        for k in range(row[i], row[i + 1]):
            j = int(col[k])
            dx, dy = prob.x[j] - prob.x[i], prob.y[j] - prob.y[i]
            L2 = dx * dx + dy * dy
            d = P[j - n0] - P[i - n0]
            sig = np.maximum(sig, np.abs(d[0] * dx + d[1] * dy) / L2)
    return sig


# ----------------------------------------------------------------------------
# projection of a particle's state
# ----------------------------------------------------------------------------
def project(X, m, Phi, y, v, F):
    """Rigid + modal reading of a particle at positions y, velocities v,
    external nodal forces F (all [n, 2]); X = template coordinates, centred.

    Returns c (centroid), vc, phi (best-fit angle), I (polar moment about c),
    Omega (angular velocity from the angular momentum), Ftot, torque,
    q = Phi^T M u_body and gext = Phi^T f_body, with u_body = R(-phi)(y - c) - X
    and f_body = R(-phi) F.
    """
    M = m.sum()
    c = (m[:, None] * y).sum(0) / M
    vc = (m[:, None] * v).sum(0) / M
    Y = y - c
    phi = best_fit_angle(X, Y, m)
    I = (m * (Y ** 2).sum(1)).sum()
    dv = v - vc
    Lz = (m * (Y[:, 0] * dv[:, 1] - Y[:, 1] * dv[:, 0])).sum()
    Ftot = F.sum(0)
    tau = (Y[:, 0] * F[:, 1] - Y[:, 1] * F[:, 0]).sum()
    ub = rot(-phi, Y) - X
    fb = rot(-phi, F)
    q = Phi.T @ (np.repeat(m, 2) * ub.ravel())
    gext = Phi.T @ fb.ravel()
    return dict(c=c, vc=vc, phi=phi, I=I, Omega=Lz / I, Ftot=Ftot, tau=tau, M=M, Y=Y,
                q=q, gext=gext)


def modal_force(Phi, phi, F):
    """Phi^T R(-phi) F: the modal part of nodal forces F (e.g. the PD force)."""
    return Phi.T @ rot(-phi, F).ravel()


def closure_accel(pr, Phi, qdd, gravity):
    """Nodal acceleration of a closure particle: translation by Ftot/M,
    rotation alpha = tau/I about the centroid with the centripetal term of
    the angular velocity Omega, and the modal acceleration R(phi) Phi qdd,
    plus the body force."""
    Y = pr["Y"]
    alpha = pr["tau"] / pr["I"]
    Om = pr["Omega"]
    a = np.empty_like(Y)
    a[:, 0] = pr["Ftot"][0] / pr["M"] - alpha * Y[:, 1] - Om * Om * Y[:, 0]
    a[:, 1] = pr["Ftot"][1] / pr["M"] + alpha * Y[:, 0] - Om * Om * Y[:, 1]
    a += rot(pr["phi"], (Phi @ qdd).reshape(-1, 2))
    a[:, 0] += gravity[0]
    a[:, 1] += gravity[1]
    return a


# ----------------------------------------------------------------------------
# the MLP
# ----------------------------------------------------------------------------
def bf16_round(a):
    """Round to the nearest bfloat16 (ties to even), returned as float64.
    The input is first rounded to float32, as the GPU holds it."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if nan.any():
        out[nan] = np.nan
    return out.reshape(np.shape(a))


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def unpack(params):
    """Packed float array -> [(W1, b1), (W2, b2), (W3, b3)], W as [out, in]."""
    params = np.asarray(params, dtype=np.float64)
    out, k = [], 0
    for o, i in LAYERS:
        W = params[k:k + o * i].reshape(o, i)
        k += o * i
        b = params[k:k + o]
        k += o
        out.append((W, b))
    assert k == params.size
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in layers])


def mlp_forward(params, x, bf16=False):
    """y = W3 h2 + b3, h2 = silu(W2 h1 + b2), h1 = silu(W1 x + b1); x [B, 32]."""
    r = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    (W1, b1), (W2, b2), (W3, b3) = unpack(params)
    xb = r(x)
    z1 = xb @ r(W1).T + b1
    h1 = r(silu(z1))
    z2 = h1 @ r(W2).T + b2
    h2 = r(silu(z2))
    y = h2 @ r(W3).T + b3
    return y, dict(x=xb, z1=z1, h1=h1, z2=z2, h2=h2)


def mlp_backward(params, cache, dy, bf16=False):
    """Gradients of sum(y * dy) with respect to the packed parameters (the
    chain rule through the three layers), same packing as params."""
    r = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    (W1, b1), (W2, b2), (W3, b3) = unpack(params)
    dyb = r(dy)
    gW3 = dyb.T @ cache["h2"]
    gb3 = np.asarray(dy).sum(0)
    dz2 = (dyb @ r(W3)) * dsilu(cache["z2"])
    dz2b = r(dz2)
    gW2 = dz2b.T @ cache["h1"]
    gb2 = dz2.sum(0)
    dz1 = (dz2b @ r(W2)) * dsilu(cache["z1"])
    dz1b = r(dz1)
    gW1 = dz1b.T @ cache["x"]
    gb1 = dz1.sum(0)
    return pack([(gW1, gb1), (gW2, gb2), (gW3, gb3)])


def loss_and_grads(params, q, r, sig_q, sig_r, bf16=False):
    """Training objective on a batch: mean over samples and outputs of
    (MLP(q / sigma_q) - r / sigma_r)^2, r = g + lambda q being the part of the
    modal force the linear closure misses. Returns (loss, gradients)."""
    x = np.asarray(q, dtype=np.float64) / sig_q
    t = np.asarray(r, dtype=np.float64) / sig_r
    y, cache = mlp_forward(params, x, bf16=bf16)
    d = y - t
    B = x.shape[0]
    loss = float((d * d).sum() / (B * N_IN))
    dy = 2.0 * d / (B * N_IN)
    return loss, mlp_backward(params, cache, dy, bf16=bf16)


def closure_modal_force(q, lam, params=None, sig_q=None, sig_r=None, bf16=True):
    """g(q) = -lambda q, plus sigma_r MLP(q / sigma_q) for the learned closure;
    q [B, 32]."""
    q = np.atleast_2d(np.asarray(q, dtype=np.float64))
    g = -lam * q
    if params is not None:
        y, _ = mlp_forward(params, q / sig_q, bf16=bf16)
        g = g + sig_r * y
    return g


# ----------------------------------------------------------------------------
# a time step with closure particles
# ----------------------------------------------------------------------------
class ClosureStepper:
    """Velocity-Verlet steps of a problem in which the particles listed in
    `shape_of_particle` (>= 0) take their internal force from the closure and
    move as rigid body + modes, the others by the plain force of the C oracle
    (Algorithm alg:buildtree).  Forces of every term come from the C oracle at
    the advanced positions with the previous velocities; the wall is at
    t_{n+1}.  Gate after each step: a closure particle whose bound
    sum |q_k| sigma_k passes gate_frac s0 or whose contact load sum |F_i|
    passes tau_c uses the plain force from the next step on.  Bonds must not
    break (the C oracle's force evaluation does not commit breaks)."""

    def __init__(self, o, prob, shape_of_particle, modes, s0, tau_c, gate_frac,
                 params=None, sig_q=None, sig_r=None):
        from .oracle import T_PD, T_SELF, T_NBR, T_WALL  # noqa: F401
        self.o, self.prob = o, prob
        self.sp = np.asarray(shape_of_particle)
        self.modes = modes            # shape -> (Phi [2n, K], lam [K], sig [K])
        self.s0, self.tau_c, self.gate = s0, tau_c, gate_frac
        self.params, self.sig_q, self.sig_r = params, sig_q, sig_r
        self.templates = {}
        for s in sorted(set(self.sp[self.sp >= 0].tolist())):
            pt = int(np.nonzero(self.sp == s)[0][0])
            self.templates[s] = reference_frame(prob, pt)[1]
        self.active = self.sp >= 0
        rho = np.array([prob.materials[int(m)].rho for m in prob.particle_material])
        self.rho_node = np.repeat(rho, np.diff(prob.particle_offset))

    def _g(self, s, q):
        Phi, lam, _ = self.modes[s]
        if self.params is None:
            return closure_modal_force(q, lam)[0]
        return closure_modal_force(q, lam, self.params[s], self.sig_q[s], self.sig_r[s])[0]

    def step(self):
        from .oracle import T_PD, T_SELF, T_NBR, T_WALL
        o, prob = self.o, self.prob
        st = o.get_state()
        dt = prob.dt
        ux = (st["ux"] + dt * st["vx"]) + (0.5 * dt * dt) * st["ax"]
        uy = (st["uy"] + dt * st["vy"]) + (0.5 * dt * dt) * st["ay"]
        tmp = dict(st, ux=ux, uy=uy, step=st["step"] + 1)
        o.set_state(tmp)
        fpx, fpy = o.forces(T_PD)
        fcx, fcy = o.forces(T_SELF | T_NBR | T_WALL)
        gx, gy = prob.gravity
        ax = (fpx + fcx) / self.rho_node + gx
        ay = (fpy + fcy) / self.rho_node + gy
        gate_off = []
        for p in np.nonzero(self.active)[0]:
            s = int(self.sp[p])
            n0, n1 = particle_range(prob, p)
            m = node_masses(prob, p)
            V = prob.vol[n0:n1]
            Phi, lam, sig = self.modes[s]
            y = np.stack([prob.x[n0:n1] + ux[n0:n1], prob.y[n0:n1] + uy[n0:n1]], axis=1)
            v = np.stack([st["vx"][n0:n1], st["vy"][n0:n1]], axis=1)
            F = np.stack([fcx[n0:n1] * V, fcy[n0:n1] * V], axis=1)
            pr = project(self.templates[s], m, Phi, y, v, F)
            qdd = self._g(s, pr["q"]) + pr["gext"]
            a = closure_accel(pr, Phi, qdd, (gx, gy))
            ax[n0:n1], ay[n0:n1] = a[:, 0], a[:, 1]
            strain = float((np.abs(pr["q"]) * sig).sum())
            load = float(np.sqrt((F ** 2).sum(1)).sum())
            if strain > self.gate * self.s0[s] or load > self.tau_c[s]:
                gate_off.append(p)
        vx = st["vx"] + (0.5 * dt) * (st["ax"] + ax)
        vy = st["vy"] + (0.5 * dt) * (st["ay"] + ay)
        o.set_state(dict(st, ux=ux, uy=uy, vx=vx, vy=vy, ax=ax, ay=ay, step=st["step"] + 1))
        for p in gate_off:
            self.active[p] = False
        return gate_off

    def check(self, err_tol):
        """The periodic check at the current state: modal PD force vs the
        closure's, per active particle; returns (sum |g - g_pd|^2,
        sum |g_pd|^2, sum |-lambda q - g_pd|^2, particles that fall back)."""
        from .oracle import T_PD
        o, prob = self.o, self.prob
        st = o.get_state()
        fpx, fpy = o.forces(T_PD)
        e2 = n2 = l2 = 0.0
        out = []
        for p in np.nonzero(self.active)[0]:
            s = int(self.sp[p])
            n0, n1 = particle_range(prob, p)
            m = node_masses(prob, p)
            V = prob.vol[n0:n1]
            Phi, lam, sig = self.modes[s]
            y = np.stack([prob.x[n0:n1] + st["ux"][n0:n1], prob.y[n0:n1] + st["uy"][n0:n1]], axis=1)
            z = np.zeros_like(y)
            F = np.stack([fpx[n0:n1] * V, fpy[n0:n1] * V], axis=1)
            pr = project(self.templates[s], m, Phi, y, z, F)
            g_pd = pr["gext"]
            gh = self._g(s, pr["q"])
            lq = -lam * pr["q"]
            de, dn, dl = ((gh - g_pd) ** 2).sum(), (g_pd ** 2).sum(), ((lq - g_pd) ** 2).sum()
            e2, n2, l2 = e2 + de, n2 + dn, l2 + dl
            smax = max_stretch(prob, p, st)
            if smax > self.gate * self.s0[s] or np.sqrt(de) > err_tol * max(np.sqrt(dn), np.linalg.norm(lq)):
                out.append(p)
        for p in out:
            self.active[p] = False
        return e2, n2, l2, out


def max_stretch(prob, p, st, row=None, col=None, _cache={}):
    """Largest |stretch| over the particle's intact bonds at state st
    (eq. (peri): s = (|xi + eta| - |xi|) / |xi|), for the check."""
    key = id(prob)
    if key not in _cache:
        from .oracle import Oracle
        oo = Oracle(prob, contact_mode=1)
        _cache[key] = oo.bonds()
    row, col = _cache[key]
    n0, n1 = particle_range(prob, p)
    x, y = prob.x, prob.y
    brk = st.get("broken")
    best = 0.0
    for i in range(n0, n1):
        for k in range(row[i], row[i + 1]):
            if brk is not None and brk[k]:
                continue
            j = int(col[k])
            X, Y = x[j] - x[i], y[j] - y[i]
            L = np.hypot(X, Y)
            l = np.hypot(X + st["ux"][j] - st["ux"][i], Y + st["uy"][j] - st["uy"][i])
            best = max(best, abs(l - L) / L)
    return best


# ----------------------------------------------------------------------------
# reduced form: rigid + modal state integrated directly
# ----------------------------------------------------------------------------
class ReducedStepper:
    """The closure's reduced form (a step in the same order as the library's):
    each closure particle's state is its centroid c, rotation angle phi about
    its shape's template, modal amplitudes q, and their rates and
    accelerations.  At start, from the nodal state: mass centroid, velocity
    and acceleration of the centroid, best-fit angle, angular velocity and
    acceleration from the angular momentum and its rate about the centroid,
    q, q' and q'' as projections of the body-frame deformation, velocity and
    acceleration left after the rigid motion.  A step: nodal positions
    advanced (u + dt v + dt^2/2 a); c, phi, q advanced the same way; contact
    and wall forces from the C oracle at those positions (previous
    velocities); the nodal forces reduced to F, the torque about c (arms from
    the advanced nodal positions) and Phi^T R(-phi) f; accelerations
    F/M + g, tau / I(q) with I(q) = I0 + 2 b.q + q.q (b_k = sum m X.phi_k),
    g(q) + Phi^T R(-phi) f; rates by the trapezoidal rule; the gate; every
    node of the particle reconstructed (x + u = c + R(phi)(X + Phi q),
    velocity and acceleration by differentiation, without the Coriolis term
    of the modal rate)."""

    def __init__(self, o, prob, shape_of_particle, modes, s0, tau_c, gate_frac,
                 params=None, sig_q=None, sig_r=None, active=None):
        """active: which closure particles start in the closure (default all)"""
        self.o, self.prob = o, prob
        self.sp = np.asarray(shape_of_particle)
        self.modes = modes
        self.s0, self.tau_c, self.gate = s0, tau_c, gate_frac
        self.params, self.sig_q, self.sig_r = params, sig_q, sig_r
        self.templates, self.I0, self.b, self.M = {}, {}, {}, {}
        for s in sorted(set(self.sp[self.sp >= 0].tolist())):
            pt = int(np.nonzero(self.sp == s)[0][0])
            X = reference_frame(prob, pt)[1]
            m = node_masses(prob, pt)
            Phi = modes[s][0]
            self.templates[s] = X
            self.M[s] = m.sum()
            self.I0[s] = (m * (X ** 2).sum(1)).sum()
            self.b[s] = Phi.T @ (np.repeat(m, 2) * X.ravel())
        self.active = (self.sp >= 0) if active is None else np.asarray(active, dtype=bool).copy()
        rho = np.array([prob.materials[int(mm)].rho for mm in prob.particle_material])
        self.rho_node = np.repeat(rho, np.diff(prob.particle_offset))
        self.state = {}
        st = o.get_state()
        for p in np.nonzero(self.active)[0]:
            self.state[p] = self._init(p, st)
        self._write_all(st)

    def _g(self, s, q):
        Phi, lam, _ = self.modes[s]
        if self.params is None:
            return closure_modal_force(q, lam)[0]
        return closure_modal_force(q, lam, self.params[s], self.sig_q[s], self.sig_r[s])[0]

    def _init(self, p, st):
        prob = self.prob
        s = int(self.sp[p])
        n0, n1 = particle_range(prob, p)
        m = node_masses(prob, p)
        M = m.sum()
        X = self.templates[s]
        Phi = self.modes[s][0]
        y = np.stack([prob.x[n0:n1] + st["ux"][n0:n1], prob.y[n0:n1] + st["uy"][n0:n1]], 1)
        v = np.stack([st["vx"][n0:n1], st["vy"][n0:n1]], 1)
        a = np.stack([st["ax"][n0:n1], st["ay"][n0:n1]], 1)
        c = (m[:, None] * y).sum(0) / M
        vc = (m[:, None] * v).sum(0) / M
        ac = (m[:, None] * a).sum(0) / M
        Y = y - c
        phi = best_fit_angle(X, Y, m)
        I = (m * (Y ** 2).sum(1)).sum()
        dv, da = v - vc, a - ac
        om = (m * (Y[:, 0] * dv[:, 1] - Y[:, 1] * dv[:, 0])).sum() / I
        al = (m * (Y[:, 0] * da[:, 1] - Y[:, 1] * da[:, 0])).sum() / I
        zY = np.stack([-Y[:, 1], Y[:, 0]], 1)  # z x Y
        body = lambda w: rot(-phi, w).ravel()
        mm = np.repeat(m, 2)
        q = Phi.T @ (mm * (rot(-phi, Y) - X).ravel())
        qv = Phi.T @ (mm * body(dv - om * zY))
        qa = Phi.T @ (mm * body(da - al * zY + om * om * Y))
        return dict(c=c, vc=vc, ac=ac, phi=phi, om=om, al=al, q=q, qv=qv, qa=qa)

    def _nodes(self, p):
        """positions, velocities, accelerations of every node of p"""
        s = int(self.sp[p])
        r = self.state[p]
        X = self.templates[s]
        Phi = self.modes[s][0]
        Z = X + (Phi @ r["q"]).reshape(-1, 2)
        Y = rot(r["phi"], Z)
        zY = np.stack([-Y[:, 1], Y[:, 0]], 1)
        pos = r["c"] + Y
        vel = r["vc"] + r["om"] * zY + rot(r["phi"], (Phi @ r["qv"]).reshape(-1, 2))
        acc = r["ac"] + r["al"] * zY - r["om"] ** 2 * Y + rot(r["phi"], (Phi @ r["qa"]).reshape(-1, 2))
        return pos, vel, acc

    def _write(self, p, arrs):
        prob = self.prob
        n0, n1 = particle_range(prob, p)
        pos, vel, acc = self._nodes(p)
        arrs["ux"][n0:n1] = pos[:, 0] - prob.x[n0:n1]
        arrs["uy"][n0:n1] = pos[:, 1] - prob.y[n0:n1]
        arrs["vx"][n0:n1], arrs["vy"][n0:n1] = vel[:, 0], vel[:, 1]
        arrs["ax"][n0:n1], arrs["ay"][n0:n1] = acc[:, 0], acc[:, 1]

    def _write_all(self, st):
        arrs = {k: st[k].copy() for k in ("ux", "uy", "vx", "vy", "ax", "ay")}
        for p in np.nonzero(self.active)[0]:
            self._write(p, arrs)
        self.o.set_state(dict(st, **arrs))

    def step(self):
        from .oracle import T_PD, T_SELF, T_NBR, T_WALL
        o, prob = self.o, self.prob
        st = o.get_state()
        dt = prob.dt
        h2 = 0.5 * dt * dt
        ux = (st["ux"] + dt * st["vx"]) + h2 * st["ax"]
        uy = (st["uy"] + dt * st["vy"]) + h2 * st["ay"]
        o.set_state(dict(st, ux=ux, uy=uy, step=st["step"] + 1))
        fpx, fpy = o.forces(T_PD)
        fcx, fcy = o.forces(T_SELF | T_NBR | T_WALL)
        gx, gy = prob.gravity
        ax = (fpx + fcx) / self.rho_node + gx
        ay = (fpy + fcy) / self.rho_node + gy
        vx = st["vx"] + (0.5 * dt) * (st["ax"] + ax)
        vy = st["vy"] + (0.5 * dt) * (st["ay"] + ay)
        arrs = dict(ux=ux, uy=uy, vx=vx, vy=vy, ax=ax, ay=ay)
        gate_off = []
        for p in np.nonzero(self.active)[0]:
            s = int(self.sp[p])
            r = self.state[p]
            Phi, lam, sig = self.modes[s]
            X = self.templates[s]
            n0, n1 = particle_range(prob, p)
            V = prob.vol[n0:n1]
            r["c"] = (r["c"] + dt * r["vc"]) + h2 * r["ac"]
            r["phi"] = (r["phi"] + dt * r["om"]) + h2 * r["al"]
            r["q"] = (r["q"] + dt * r["qv"]) + h2 * r["qa"]
            f = np.stack([fcx[n0:n1] * V, fcy[n0:n1] * V], 1)
            Y = np.stack([prob.x[n0:n1] + ux[n0:n1], prob.y[n0:n1] + uy[n0:n1]], 1) - r["c"]
            F = f.sum(0)
            tau = (Y[:, 0] * f[:, 1] - Y[:, 1] * f[:, 0]).sum()
            load = np.sqrt((f ** 2).sum(1)).sum()
            gext = Phi.T @ rot(-r["phi"], f).ravel()
            q = r["q"]
            I = self.I0[s] + 2.0 * (self.b[s] @ q) + q @ q
            ac = F / self.M[s] + np.array([gx, gy])
            al = tau / I
            qa = self._g(s, q) + gext
            r["vc"] = r["vc"] + (0.5 * dt) * (r["ac"] + ac)
            r["om"] = r["om"] + (0.5 * dt) * (r["al"] + al)
            r["qv"] = r["qv"] + (0.5 * dt) * (r["qa"] + qa)
            r["ac"], r["al"], r["qa"] = ac, al, qa
            self._write(p, arrs)
            strain = float((np.abs(q) * sig).sum())
            if strain > self.gate * self.s0[s] or load > self.tau_c[s]:
                gate_off.append(p)
        o.set_state(dict(st, step=st["step"] + 1, **arrs))
        for p in gate_off:
            self.active[p] = False
        return gate_off

    def check(self, err_tol):
        """The periodic check at the current (reconstructed) nodal state, as
        ClosureStepper.check."""
        return ClosureStepper.check(self, err_tol)
