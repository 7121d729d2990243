"""GPU test of pd_forces_noalloc, the allocation-free variant of pd_forces.

Through the C ABI: its output must equal pd_forces(on_device=1) of the same
context bit for bit (the same kernels on the same state; only the workspace
differs), on two calls in a row whose second input is smaller than the
first (the workspace keeps the first call's contents), on every term mask;
a problem larger than the workspace is refused before anything runs.
"""
import numpy as np
import pytest

from paper_2108_07212_amd import workloads as W

pytestmark = pytest.mark.gpu


def _torch():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _pd():
    from paper_2108_07212_amd import pd
    return pd


def _check(g, torch, pd, masks):
    for mask in masks:
        ex, ey = g.forces(mask, device=True)
        fx = torch.full((g.N,), np.nan, dtype=torch.float64, device="cuda")
        fy = torch.full((g.N,), np.nan, dtype=torch.float64, device="cuda")
        g.forces_noalloc(fx, fy, mask)
        torch.cuda.synchronize()
        assert torch.equal(fx, ex) and torch.equal(fy, ey), f"mask {mask}"
        assert bool(torch.isfinite(fx).all()) and bool(torch.isfinite(fy).all())


def test_noalloc_forces_equal_pd_forces_larger_then_smaller_input():
    torch = _torch()
    pd = _pd()
    print("noalloc: settling bed (perturbed), then two disks", flush=True)
    big = W.perturb(W.settling(), seed=11, du=2e-6, dv=0.05)
    g1 = pd.PD(big)
    g1.step(30)
    _check(g1, torch, pd, (pd.TERM_ALL, pd.TERM_PD, pd.TERM_WALL | pd.TERM_NBR))
    small = W.two_disks(contact_active=True)
    g2 = pd.PD(small)
    g2.step(600)  # into the collision: contact and PD terms both non-zero
    assert g2.N < g1.N
    _check(g2, torch, pd, (pd.TERM_ALL, pd.TERM_PD, pd.TERM_NBR, pd.TERM_SELF))
    # and the first context again, after the smaller call
    _check(g1, torch, pd, (pd.TERM_ALL,))


def test_noalloc_refuses_a_problem_larger_than_its_workspace():
    torch = _torch()
    pd = _pd()
    print("noalloc: 422 500 single-node particles (over the workspace)", flush=True)
    h = 1e-4
    n = 650
    pts = np.stack(np.meshgrid(np.arange(n), np.arange(n)), -1).reshape(-1, 2) * h + h
    prob = W.single_node_particles(pts, np.zeros_like(pts), h * h,
                                   (0.0, (n + 1) * h, 0.0, (n + 1) * h),
                                   contact_radius=0.95 * h, h=h)
    g = pd.PD(prob)
    fx = torch.zeros(g.N, dtype=torch.float64, device="cuda")
    fy = torch.zeros(g.N, dtype=torch.float64, device="cuda")
    with pytest.raises(pd.PDError) as ei:
        g.forces_noalloc(fx, fy)
    assert ei.value.status == pd.PD_E_INVALID
    assert "workspace" in str(ei.value)
    assert float(fx.abs().max()) == 0.0  # nothing ran
