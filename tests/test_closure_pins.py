"""Pins of the closure oracle (oracle/closure.py) against things other than
itself: library conversions and autograd, finite differences, rigid-body
closed forms, brute-force minimisation, and the oracle's own PD force (pinned
in test_oracle_pins.py) along each mode."""
import math

import numpy as np
import pytest
import scipy.optimize
import torch

from oracle import Oracle, T_PD
from oracle import closure as CL
from paper_2108_07212_amd import workloads as W

H = 0.08e-3


@pytest.fixture(scope="module")
def small_bed():
    """One particle of each closure shape, about 80 nodes each."""
    prob = W.closure_bed(n_per_shape=1, h=H, nodes=80, seed=11)
    o = Oracle(prob, contact_mode=1)
    row, col = o.bonds()
    k = o.constants()
    return prob, o, row, col, k


def _template(prob, o, row, col, k, p):
    mat = prob.materials[int(prob.particle_material[p])]
    K = CL.stiffness(prob, p, row, col, k["cw"][0], mat.horizon, mat.micro)
    m = CL.node_masses(prob, p)
    lam, Phi, alllam = CL.modes(K, m)
    c0, X = CL.reference_frame(prob, p)
    return K, m, lam, Phi, alllam, c0, X


# ----------------------------------------------------------------------------
# bfloat16 rounding and the MLP against torch
# ----------------------------------------------------------------------------
def test_bf16_round_matches_torch():
    rng = np.random.default_rng(0)
    a = np.concatenate([rng.normal(0, 1, 5000), rng.normal(0, 1e-30, 100),
                        rng.normal(0, 1e30, 100), [0.0, -0.0, 1.0, -2.5, 65504.0]])
    # exact ties: float32 values halfway between two bfloat16 neighbours
    base = (np.arange(200, dtype=np.uint32) << 16) + (0x3F80 << 16)
    ties = (base + 0x8000).view(np.float32).astype(np.float64)
    a = np.concatenate([a, ties, -ties])
    ref = torch.tensor(a.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(CL.bf16_round(a), ref)


def _rand_params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    out = []
    for o, i in CL.LAYERS:
        out.append((scale * rng.normal(0, 1 / math.sqrt(i), (o, i)), 0.1 * rng.normal(0, 1, o)))
    return CL.pack(out)


def _torch_mlp(params, x):
    (W1, b1), (W2, b2), (W3, b3) = [(torch.tensor(W, requires_grad=True),
                                     torch.tensor(b, requires_grad=True))
                                    for W, b in CL.unpack(params)]
    h1 = torch.nn.functional.silu(torch.nn.functional.linear(torch.tensor(x), W1, b1))
    h2 = torch.nn.functional.silu(torch.nn.functional.linear(h1, W2, b2))
    y = torch.nn.functional.linear(h2, W3, b3)
    return y, [W1, b1, W2, b2, W3, b3]


def test_mlp_forward_matches_torch():
    p = _rand_params(1)
    x = np.random.default_rng(2).normal(0, 1, (17, CL.N_IN))
    y, _ = CL.mlp_forward(p, x)
    yt, _ = _torch_mlp(p, x)
    np.testing.assert_allclose(y, yt.detach().numpy(), rtol=1e-13, atol=1e-14)


def test_silu_special_values():
    assert CL.silu(0.0) == 0.0
    assert abs(CL.silu(40.0) - 40.0) < 1e-15 * 40
    assert abs(CL.silu(-40.0)) < 1e-15
    # derivative against a central difference
    z = np.linspace(-6, 6, 25)
    fd = (CL.silu(z + 1e-6) - CL.silu(z - 1e-6)) / 2e-6
    np.testing.assert_allclose(CL.dsilu(z), fd, rtol=1e-8, atol=1e-9)


def test_mlp_backward_matches_torch_autograd():
    p = _rand_params(3)
    rng = np.random.default_rng(4)
    x = rng.normal(0, 1, (9, CL.N_IN))
    dy = rng.normal(0, 1, (9, CL.N_IN))
    y, cache = CL.mlp_forward(p, x)
    g = CL.mlp_backward(p, cache, dy)
    yt, ts = _torch_mlp(p, x)
    (yt * torch.tensor(dy)).sum().backward()
    gt = np.concatenate([t.grad.numpy().ravel() for t in ts])
    np.testing.assert_allclose(g, gt, rtol=1e-12, atol=1e-14)


def test_loss_gradient_against_finite_differences():
    p = _rand_params(5)
    rng = np.random.default_rng(6)
    q = rng.normal(0, 2.0, (6, CL.N_IN))
    r = rng.normal(0, 0.5, (6, CL.N_IN))
    sq, sr = np.full(CL.N_IN, 2.0), np.full(CL.N_IN, 0.5)
    _, g = CL.loss_and_grads(p, q, r, sq, sr)
    idx = rng.choice(CL.N_PARAMS, 60, replace=False)
    idx = np.concatenate([idx, [0, CL.N_PARAMS - 1, 256 * 32 + 3]])  # a W1, b3, b1 entry
    for k in idx:
        e = 1e-6
        pp, pm = p.copy(), p.copy()
        pp[k] += e
        pm[k] -= e
        fd = (CL.loss_and_grads(pp, q, r, sq, sr)[0] - CL.loss_and_grads(pm, q, r, sq, sr)[0]) / (2 * e)
        assert abs(fd - g[k]) <= 1e-6 * max(1e-3, abs(g[k])) + 1e-10, (k, fd, g[k])


def test_bf16_backward_reduces_to_exact_on_representable_values():
    """When every rounded quantity is already a bfloat16 value, the bf16 path
    equals the exact one: weights and inputs bf16, and a linear last layer
    probed through dy that is bf16-representable."""
    p = CL.bf16_round(_rand_params(7))
    x = CL.bf16_round(np.random.default_rng(8).normal(0, 1, (5, CL.N_IN)))
    y1, c1 = CL.mlp_forward(p, x, bf16=True)
    # the hidden activations of the exact path are not bf16 values, so only
    # the first layer's pre-activation agrees exactly
    y0, c0 = CL.mlp_forward(p, x, bf16=False)
    np.testing.assert_allclose(c1["z1"], c0["z1"], rtol=1e-15, atol=1e-15)
    # and the bf16 forward equals the exact forward evaluated on its rounded
    # activations, layer by layer
    (W1, b1), (W2, b2), (W3, b3) = CL.unpack(p)
    np.testing.assert_allclose(c1["z2"], c1["h1"] @ W2.T + b2, rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(y1, c1["h2"] @ W3.T + b3, rtol=1e-14, atol=1e-14)
    assert np.abs(y1 - y0).max() < 0.05 * np.abs(y0).max()


# ----------------------------------------------------------------------------
# stiffness and modes against the oracle's PD force
# ----------------------------------------------------------------------------
def _pd_nodal_force(o, prob, n0, n1, ux, uy):
    s = o.get_state()
    s2 = dict(s)
    s2["ux"] = s["ux"].copy()
    s2["uy"] = s["uy"].copy()
    s2["ux"][n0:n1] = ux
    s2["uy"][n0:n1] = uy
    o.set_state(s2)
    fx, fy = o.forces(T_PD)
    o.set_state(s)
    V = prob.vol[n0:n1]
    return np.stack([fx[n0:n1] * V, fy[n0:n1] * V], axis=1)


@pytest.mark.parametrize("p", [0, 1, 2, 3])
def test_stiffness_is_the_linearised_pd_force(small_bed, p):
    prob, o, row, col, k = small_bed
    K, m, lam, Phi, alllam, c0, X = _template(prob, o, row, col, k, p)
    np.testing.assert_allclose(K, K.T, rtol=0, atol=1e-12 * np.abs(K).max())
    n0, n1 = CL.particle_range(prob, p)
    rng = np.random.default_rng(20 + p)
    u = rng.normal(0, 1, (n1 - n0, 2))
    errs = []
    for eps in (1e-6 * H, 0.5e-6 * H):
        F = _pd_nodal_force(o, prob, n0, n1, eps * u[:, 0], eps * u[:, 1])
        lin = -(K @ (eps * u).ravel()).reshape(-1, 2)
        errs.append(np.abs(F - lin).max() / np.abs(lin).max())
    # the remainder is second order: it halves with the amplitude
    assert errs[0] < 2e-4
    assert 1.6 < errs[0] / errs[1] < 2.4


@pytest.mark.parametrize("p", [0, 1, 2, 3])
def test_rigid_modes_and_normalisation(small_bed, p):
    prob, o, row, col, k = small_bed
    K, m, lam, Phi, alllam, c0, X = _template(prob, o, row, col, k, p)
    n = len(m)
    tx = np.tile([1.0, 0.0], n)
    ty = np.tile([0.0, 1.0], n)
    rz = np.stack([-X[:, 1], X[:, 0]], axis=1).ravel()
    scale = np.abs(K).max()
    for r in (tx, ty, rz):
        assert np.abs(K @ r).max() < 1e-12 * scale * np.abs(r).max()
    assert np.all(np.abs(alllam[:3]) < 1e-10 * lam[0])
    assert lam[0] > 0 and np.all(np.diff(lam) >= 0)
    M = np.repeat(m, 2)
    G = Phi.T @ (M[:, None] * Phi)
    np.testing.assert_allclose(G, np.eye(Phi.shape[1]), atol=1e-10)
    # modes carry no net momentum or angular momentum
    for r in (tx, ty, rz):
        assert np.abs(Phi.T @ (M * r)).max() < 1e-9 * math.sqrt((M * r * r).sum())


@pytest.mark.parametrize("p", [0, 1, 2, 3])
def test_pd_force_along_each_mode(small_bed, p):
    """F_pd(eps phi_k) / eps -> -lambda_k M phi_k: the linear closure is the
    PD force to first order."""
    prob, o, row, col, k = small_bed
    K, m, lam, Phi, alllam, c0, X = _template(prob, o, row, col, k, p)
    n0, n1 = CL.particle_range(prob, p)
    M = np.repeat(m, 2)
    for kk in (0, 7, 31):
        ph = Phi[:, kk]
        eps = 1e-7 * H / np.abs(ph).max()
        F = _pd_nodal_force(o, prob, n0, n1, eps * ph[0::2], eps * ph[1::2]).ravel()
        ref = -eps * lam[kk] * M * ph
        assert np.abs(F - ref).max() < 1e-4 * np.abs(ref).max(), kk


def test_stretch_bound_is_tight_for_one_mode(small_bed):
    prob, o, row, col, k = small_bed
    p = 1
    K, m, lam, Phi, alllam, c0, X = _template(prob, o, row, col, k, p)
    sig = CL.stretch_bound(prob, p, row, col, Phi)
    n0, n1 = CL.particle_range(prob, p)
    xs, ys = prob.x[n0:n1], prob.y[n0:n1]
    for kk in (0, 5, 20):
        eps = 1e-8 / sig[kk]
        ux, uy = eps * Phi[0::2, kk], eps * Phi[1::2, kk]
        smax = 0.0
        for i in range(n0, n1):
            for b in range(row[i], row[i + 1]):
                j = int(col[b])
                L = math.hypot(xs[j - n0] - xs[i - n0], ys[j - n0] - ys[i - n0])
                l = math.hypot(xs[j - n0] + ux[j - n0] - xs[i - n0] - ux[i - n0],
                               ys[j - n0] + uy[j - n0] - ys[i - n0] - uy[i - n0])
                smax = max(smax, abs(l - L) / L)
        assert abs(smax / eps - sig[kk]) < 1e-5 * sig[kk]


# ----------------------------------------------------------------------------
# best-fit frame, projection and the rigid-body acceleration
# ----------------------------------------------------------------------------
def test_instances_share_the_template(small_bed):
    """Every instance of a shape is its template rotated and translated."""
    prob = W.closure_bed(n_per_shape=3, h=H, nodes=80, seed=12)
    sp = prob.meta["shape_of_particle"]
    for s in range(4):
        ps = np.nonzero(sp == s)[0]
        _, Xt = CL.reference_frame(prob, ps[0])
        m = CL.node_masses(prob, ps[0])
        for p in ps[1:]:
            c0, Xp = CL.reference_frame(prob, p)
            th = CL.best_fit_angle(Xt, Xp, m)
            assert np.abs(CL.rot(th, Xt) - Xp).max() < 1e-15 * 1e3


def test_best_fit_angle_against_brute_force_minimisation():
    rng = np.random.default_rng(30)
    X = rng.normal(0, 1, (40, 2))
    m = rng.uniform(0.5, 2.0, 40)
    X -= (m[:, None] * X).sum(0) / m.sum()
    for th in (0.3, -2.9, 3.1):
        Y = CL.rot(th, X) + 0.05 * rng.normal(0, 1, X.shape)
        Y -= (m[:, None] * Y).sum(0) / m.sum()
        f = lambda a: (m * ((CL.rot(a, X) - Y) ** 2).sum(1)).sum()
        grid = np.linspace(-math.pi, math.pi, 2001)
        a0 = grid[np.argmin([f(a) for a in grid])]
        res = scipy.optimize.minimize_scalar(f, bracket=(a0 - 0.01, a0, a0 + 0.01), tol=1e-12)
        d = (CL.best_fit_angle(X, Y, m) - res.x + math.pi) % (2 * math.pi) - math.pi
        assert abs(d) < 1e-6


def test_projection_recovers_frame_and_amplitudes(small_bed):
    prob, o, row, col, k = small_bed
    p = 2
    K, m, lam, Phi, alllam, c0, X = _template(prob, o, row, col, k, p)
    rng = np.random.default_rng(31)
    q0 = rng.normal(0, 1e-3, Phi.shape[1]) * H / np.abs(Phi).max()
    th, c = 1.234, np.array([3e-3, -2e-3])
    y = c + CL.rot(th, X + (Phi @ q0).reshape(-1, 2))
    z = np.zeros_like(y)
    pr = CL.project(X, m, Phi, y, z, z)
    assert abs(pr["phi"] - th) < 1e-13
    assert np.abs(pr["c"] - c).max() < 1e-15 * 10
    np.testing.assert_allclose(pr["q"], q0, rtol=0, atol=1e-9 * np.abs(q0).max())


def test_rigid_body_accelerations(small_bed):
    prob, o, row, col, k = small_bed
    p = 3
    K, m, lam, Phi, alllam, c0, X = _template(prob, o, row, col, k, p)
    th, c = -0.7, np.array([1e-3, 2e-3])
    y = c + CL.rot(th, X)
    Y = y - c
    z = np.zeros_like(y)
    g = (0.0, -9.81)
    # uniform body force: pure translation
    a0 = np.array([3.0, -4.0])
    pr = CL.project(X, m, Phi, y, z, m[:, None] * a0)
    assert np.abs(pr["gext"]).max() < 1e-10 * np.abs(m[:, None] * a0).sum() / np.sqrt(m.sum())
    a = CL.closure_accel(pr, Phi, np.zeros(Phi.shape[1]), g)
    np.testing.assert_allclose(a, np.broadcast_to(a0 + np.array(g), a.shape), rtol=1e-12, atol=1e-12)
    # tangential forces m alpha (z x Y): pure angular acceleration alpha
    al = 250.0
    F = m[:, None] * al * np.stack([-Y[:, 1], Y[:, 0]], axis=1)
    pr = CL.project(X, m, Phi, y, z, F)
    a = CL.closure_accel(pr, Phi, np.zeros(Phi.shape[1]), (0.0, 0.0))
    np.testing.assert_allclose(a, F / m[:, None], rtol=1e-10, atol=1e-12 * np.abs(a).max())
    # rigid rotation at Omega with no force: centripetal acceleration
    Om = 40.0
    v = Om * np.stack([-Y[:, 1], Y[:, 0]], axis=1)
    pr = CL.project(X, m, Phi, y, v, z)
    assert abs(pr["Omega"] - Om) < 1e-12 * Om
    a = CL.closure_accel(pr, Phi, np.zeros(Phi.shape[1]), (0.0, 0.0))
    np.testing.assert_allclose(a, -Om * Om * Y, rtol=1e-12, atol=1e-12 * Om * Om * np.abs(Y).max())


def test_linear_closure_modal_force_matches_pd(small_bed):
    """For a small deformation in the mode span, the projected PD force is
    -lambda q to first order; the relative error halves with the amplitude."""
    prob, o, row, col, k = small_bed
    p = 0
    K, m, lam, Phi, alllam, c0, X = _template(prob, o, row, col, k, p)
    n0, n1 = CL.particle_range(prob, p)
    rng = np.random.default_rng(32)
    dirn = rng.normal(0, 1, Phi.shape[1])
    errs = []
    for amp in (1e-4, 5e-5):
        q0 = amp * H * dirn / np.abs(Phi @ dirn).max()
        u = (Phi @ q0).reshape(-1, 2)
        F = _pd_nodal_force(o, prob, n0, n1, u[:, 0], u[:, 1])
        g = CL.modal_force(Phi, 0.0, F)
        gl = CL.closure_modal_force(q0, lam)[0]
        errs.append(np.linalg.norm(g - gl) / np.linalg.norm(gl))
    assert errs[0] < 1e-3
    assert 1.6 < errs[0] / errs[1] < 2.4
