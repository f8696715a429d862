"""Adjoint of the step (frozen dt and cascade choice) through the C-ABI.

L = <g, x(T)> for a fixed random g.  The adjoint gradients with respect to
the per-cell shear modulus and the initial cell and node velocities are
checked along random directions against central differences of the GPU
forward pass replayed with the recorded dt and masks (Richardson
extrapolated), and, component by component, against central differences of
the CPU oracle run with the same recorded dt and masks.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2104_02139_amd import hyperlag as H
from paper_2104_02139_amd import workloads as W

pytestmark = pytest.mark.gpu


def _case(kind):
    if kind == "cube3d":
        w = W.rotating_cube_3d(n=3, jitter=0.15, omega=3.0)
        w.mu = W.shear_modulus_field(w.n_cells, mu0=8.2e5, seed=3)
        rng = np.random.default_rng(4)
        w.v_cell = w.v_cell * 20 + rng.normal(0, 0.5, w.v_cell.shape)
        w.v_node = w.v_node * 20
        return w, 8, 3
    if kind == "plate2d":
        # detection off: every cell second order, so the initial node velocity
        # enters every Crank-Nicolson update of the first step
        w = W.plane_wave_2d(n=6, amp=0.05)
        rng = np.random.default_rng(5)
        w.mu = w.mu * np.exp(0.2 * rng.standard_normal(w.n_cells))
        return w, 10, 4
    if kind == "bar3d_mood":
        w = W.impact_bar_3d(nx=8, ny=2, graded=False)
        w.mu = w.mu * np.exp(0.1 * np.random.default_rng(6).standard_normal(w.n_cells))
        return w, 6, 2
    raise KeyError(kind)


def _loss(ctx, w, g, mu, vc, vn):
    ctx.init_state(w.rho0, mu, w.lam, vc, vn, ctx.params)
    ctx.forward_replay()
    return float(np.sum(g * ctx.query("x")))


def _fd(ctx, w, g, base, which, direction, eps):
    def at(s):
        mu, vc, vn = (a.copy() for a in base)
        if which == "mu":
            mu = mu * (1.0 + s * direction)
        elif which == "vc":
            vc = vc + s * direction
        else:
            vn = vn + s * direction
        return _loss(ctx, w, g, mu, vc, vn)

    d1 = (at(eps) - at(-eps)) / (2 * eps)
    d2 = (at(eps / 2) - at(-eps / 2)) / eps
    return (4 * d2 - d1) / 3, abs(d2 - d1)


@pytest.mark.parametrize("kind", ["cube3d", "plate2d", "bar3d_mood"])
def test_adjoint_matches_finite_differences(kind):
    w, steps, every = _case(kind)
    ctx = H.from_workload(w, params=H.default_params(w.dim, detect=(kind != "plate2d"), c_cfl=w.c_cfl))
    ctx.forward_record(steps, every)
    masks = [ctx.tape(n)[0] for n in range(steps)]
    print(f"[adjoint] {kind}: {w.n_cells} cells, {steps} steps, first-order cells per step "
          f"{[int(m.sum()) for m in masks]}", flush=True)
    rng = np.random.default_rng(7)
    g = rng.standard_normal((w.n_nodes, w.dim))
    gmu, gvc, gvn = ctx.adjoint_run(g)
    assert np.all(np.isfinite(gmu)) and np.all(np.isfinite(gvc)) and np.all(np.isfinite(gvn))
    base = (w.mu.copy(), w.v_cell.copy(), w.v_node.copy())
    vscale = max(np.abs(w.v_cell).max(), 1e-3)
    # steps large enough that <g, x> changes far above its roundoff
    # (~1e-15 here); Richardson extrapolation removes the O(eps^2) error
    for which, grad, eps in (("mu", gmu * w.mu, 1e-3), ("vc", gvc, 1e-2 * vscale),
                             ("vn", gvn, 1e-1 * vscale)):
        for t in range(2):
            shape = w.mu.shape if which == "mu" else (w.v_cell.shape if which == "vc" else w.v_node.shape)
            dirn = rng.standard_normal(shape)
            adj = float(np.sum(grad * dirn))
            fd, spread = _fd(ctx, w, g, base, which, dirn, eps)
            rel = abs(adj - fd) / max(abs(fd), 1e-300)
            print(f"  {which}: adjoint {adj:.12e} fd {fd:.12e} rel {rel:.2e} (fd spread {spread:.1e})",
                  flush=True)
            # 1e-6 relative, or within the finite differences' own noise
            # (the spread between the two step sizes) when the derivative
            # is at their roundoff floor
            assert abs(adj - fd) <= 1e-6 * abs(fd) + 3 * spread, (which, adj, fd, spread)


def test_adjoint_against_oracle_gradient():
    """CPU reference: central differences of the oracle with the GPU's
    recorded dt and cascade masks, per cell shear modulus."""
    w, steps, every = _case("cube3d")
    ctx = H.from_workload(w)
    ctx.forward_record(steps, every)
    tapes = [ctx.tape(n) for n in range(steps)]
    rng = np.random.default_rng(8)
    g = rng.standard_normal((w.n_nodes, w.dim))
    gmu, _, _ = ctx.adjoint_run(g)

    def oracle_loss(mu):
        import copy
        ww = copy.copy(w)
        ww.mu = mu
        prob = O.Problem(ww, O.default_params(w.c_cfl))
        for mask, dt in tapes:
            prob.step(float(dt[0]), mask=mask, replay=True)
        return float(np.sum(g * prob.state.x))

    for c in (0, 37, w.n_cells - 1):
        h = 1e-4 * w.mu[c]
        mp, mm = w.mu.copy(), w.mu.copy()
        mp[c] += h
        mm[c] -= h
        fd = (oracle_loss(mp) - oracle_loss(mm)) / (2 * h)
        rel = abs(gmu[c] - fd) / max(abs(fd), 1e-300)
        print(f"  cell {c}: adjoint {gmu[c]:.10e} oracle fd {fd:.10e} rel {rel:.2e}", flush=True)
        assert rel <= 1e-5


def test_autograd_function_identification_step():
    """torch.autograd through the library: L = sum |x(T) - x_target|^2 with
    x_target from another shear-modulus field; the gradient from backward
    equals the adjoint of dL/dx = 2 (x(T) - x_target), and a small step
    along -grad lowers L (replayed with the recorded dt and masks)."""
    import torch
    from paper_2104_02139_amd.autograd import run

    w = W.identification_cube_3d(n=3, steps=12)
    dev = torch.device("cuda:0")
    hctx = H.from_workload(w)
    # target: final positions with a second seeded modulus field
    mu_t = torch.tensor(W.shear_modulus_field(w.n_cells, seed=9), dtype=torch.float64, device=dev)
    vc = torch.tensor(w.v_cell * 50.0, dtype=torch.float64, device=dev)
    vn = torch.tensor(w.v_node * 50.0, dtype=torch.float64, device=dev)
    with torch.no_grad():
        x_target = run(mu_t, vc, vn, hctx, w, 12, 5).clone()
    mu = torch.tensor(w.mu, dtype=torch.float64, device=dev, requires_grad=True)
    x = run(mu, vc, vn, hctx, w, 12, 5)
    loss = ((x - x_target) ** 2).sum()
    loss.backward()
    g = mu.grad.detach().cpu().numpy()
    assert np.all(np.isfinite(g)) and np.abs(g).max() > 0
    gmu, _, _ = hctx.adjoint_run((2 * (x - x_target)).detach())
    assert np.allclose(g, gmu.cpu().numpy(), rtol=1e-12, atol=0)
    # descent along -grad with the recorded dt / masks
    mu_np = mu.detach().cpu().numpy()
    mu2 = mu_np - 1e-3 * mu_np.max() * g / np.abs(g).max()
    hctx.init_state(w.rho0, mu2, w.lam, vc.cpu().numpy(), vn.cpu().numpy(), hctx.params)
    hctx.forward_replay()
    l2 = float(np.sum((hctx.query("x") - x_target.cpu().numpy()) ** 2))
    print(f"  L {float(loss):.6e} -> {l2:.6e}", flush=True)
    assert l2 < float(loss)
