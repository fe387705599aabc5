"""Hand-written adjoint of the GPU step vs reference gradients.

dL/dG_w from lbm_forward_ckpt + lbm_backward (HIP) against (i) autograd through the PyTorch CPU
oracle on small lattices, to 1e-9 relative to the gradient's largest entry, and (ii) FP64 central
finite differences of the GPU forward at the full 256x128, 4,000-step, K = 200 configuration on
16 seeded wall nodes, to 1e-6 relative.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def gpu_case(orc, gpu, p, gw, centres, radii, seed):
    q = orc.make_params(p)
    rho0 = synth.droplet_rho(q.nx, q.ny, q.rho_l, q.rho_v, centres, radii, seed=seed)
    pg = dict(p, rho_l=q.rho_l, rho_v=q.rho_v)
    return q, gpu.Sim(pg, gw, rho0), orc.init_rest(q, rho0)


def gpu_grad(sim, nsteps, K, wc=1.0, wwet=1.0):
    ws = sim.adjoint_workspace(nsteps, K)
    blob = sim.save_state()
    sim.forward_ckpt(nsteps, K, ws)
    L = sim.loss(wc, wwet)
    g = sim.backward(nsteps, K, ws, wc, wwet).cpu().numpy()
    sim.load_state(blob)
    return L, g


@pytest.mark.parametrize("form,ghost,tau_v,nsteps,K", [
    ("modpsi", 1, 1.1, 150, 37), ("rho", 1, 1.1, 150, 50), ("psi", 1, 1.1, 150, 150),
    ("modpsi", 0, 1.1, 100, 30), ("modpsi", 1, 2.0, 150, 40), ("rho", 1, 2.0, 1, 1),
    ("psi", 1, 0.6, 60, 200)])
def test_adjoint_matches_autograd(orc, gpu, form, ghost, tau_v, nsteps, K):
    from oracle import grad_oracle as G
    nx, ny = 70, 26
    p = synth.base_params(nx=nx, ny=ny, wall_force=form, ghost=ghost, tau_v=tau_v)
    gw = synth.gw_smooth(nx, {"rho": 0.05, "psi": -0.02, "modpsi": 0.1}[form], 0.03, seed=4)
    gw[1] = np.linspace(-0.03, 0.02, nx)
    c, R = ((35.0, 0.5), 10.0) if ghost else ((35.0, 13.0), 6.0)  # see test_grad_oracle
    q, sim, f0 = gpu_case(orc, gpu, p, gw, [c], [R], seed=8)
    L_ref, g_ref = G.loss_and_grad(f0, gw, q, nsteps, 0.7, 1.3)
    L, g = gpu_grad(sim, nsteps, K, 0.7, 1.3)
    scale = np.abs(g_ref).max()
    err = np.abs(g - g_ref).max() / scale
    print(f"{form} ghost={ghost} tau_v={tau_v} N={nsteps} K={K}: L {L} vs {L_ref}, "
          f"max |dg|/max|g| = {err:.3e}")
    assert abs(L - L_ref) <= 1e-9 * abs(L_ref)
    assert err <= 1e-9


@pytest.mark.parametrize("form,gw_mean", [("modpsi", 0.3), ("rho", 0.15), ("psi", -1.0)])
def test_adjoint_matches_autograd_piecewise_eos(orc, gpu, form, gw_mean):
    """The paper's Eq. (15) EOS at 500/1 (sigma = 0.084, viscosity ratio 5): every form, 90
    steps, checkpoint every 17 (a ragged last segment)."""
    from oracle import grad_oracle as G
    nx, ny, n, K = 70, 26, 90, 17
    p = dict(nx=nx, ny=ny, walls=1, ghost=1, eos="piecewise", th_v=0.64 / 3, th_m=-0.04 / 3,
             th_l=1 / 3, rho_v=1.0, rho_l=500.0, G=-1.0, sigma=0.084, tau_l=1.1, tau_v=2.0,
             wall_force=form, **synth.RATES)
    q = orc.make_params(p)
    rho0 = synth.droplet_rho(nx, ny, q.rho_l, q.rho_v, [(35.0, 0.5)], [10.0], width=4.0, seed=8)
    gw = synth.gw_smooth(nx, gw_mean, abs(gw_mean) * 0.3, seed=4)
    gw[1] = np.linspace(-0.03, 0.02, nx)
    sim = gpu.Sim(dict(p, rho_l=q.rho_l, rho_v=q.rho_v), gw, rho0)
    L_ref, g_ref = G.loss_and_grad(orc.init_rest(q, rho0), gw, q, n, 0.7, 1.3)
    L, g = gpu_grad(sim, n, K, 0.7, 1.3)
    err = np.abs(g - g_ref).max() / np.abs(g_ref).max()
    print(f"Eq. 15 {form}: L {L} vs {L_ref}, max |dg|/max|g| = {err:.3e}")
    assert abs(L - L_ref) <= 1e-9 * abs(L_ref)
    assert err <= 1e-9


def test_adjoint_c4_vs_finite_differences(orc, gpu):
    """256x128, droplet R = 40, modified form, smooth bottom G_w pattern (mean -0.1, amplitude
    0.05), 4,000 steps, checkpoint every 200: adjoint vs central differences (h = 1e-5, checked
    against h = 2e-5) on 16 seeded bottom-wall nodes."""
    cfg = synth.c4_adjoint()
    p, gw, N, K = cfg["params"], cfg["gw"], cfg["steps"], cfg["K"]
    q, sim, _ = gpu_case(orc, gpu, p, gw, cfg["centres"], cfg["radii"], cfg["seed"])
    L, g = gpu_grad(sim, N, K)
    blob = sim.save_state()
    d = synth.Draws(cfg["seed"] + 77)
    nodes = sorted({int(d.u01() * q.nx) for _ in range(40)})[:16]
    scale = np.abs(g[0]).max()

    def loss_at(gg):
        sim.load_state(blob)
        sim.set_gw(gg)
        sim.step(N)
        return sim.loss()

    worst = 0.0
    for x in nodes:
        fds = []
        for h in (1e-5, 2e-5):
            gp, gm = gw.copy(), gw.copy()
            gp[0, x] += h
            gm[0, x] -= h
            fds.append((loss_at(gp) - loss_at(gm)) / (2 * h))
        rel = abs(g[0, x] - fds[0]) / scale
        worst = max(worst, rel)
        print(f"node {x}: adjoint {g[0, x]:.10e} fd {fds[0]:.10e} (h=2e-5: {fds[1]:.10e}) "
              f"rel {rel:.2e}")
        assert rel <= 1e-6
    sim.set_gw(gw)
    print("L", L, "max |g|", scale, "worst rel", worst)


def test_autograd_function(orc, gpu):
    import torch
    from paper_1410_2569_amd.autograd import lbm_run
    nx, ny = 64, 24
    p = synth.base_params(nx=nx, ny=ny, wall_force="modpsi")
    gw0 = synth.gw_smooth(nx, -0.05, 0.02, seed=6)
    q, sim, _ = gpu_case(orc, gpu, p, gw0, [(32.0, 0.5)], [9.0], seed=9)
    state0 = sim.save_state()
    gw = torch.tensor(gw0, dtype=torch.float64, device="cuda", requires_grad=True)
    L = lbm_run(gw, sim, state0, 120, 40)
    L.backward()
    sim.load_state(state0)
    L2, g2 = gpu_grad(sim, 120, 40)
    assert abs(float(L) - L2) <= 1e-12 * abs(L2)
    assert np.array_equal(gw.grad.cpu().numpy(), g2)


def test_backward_requires_matching_forward(orc, gpu):
    p = synth.base_params(nx=32, ny=16, wall_force="modpsi")
    q, sim, _ = gpu_case(orc, gpu, p, synth.gw_uniform(32, 0.0), [(16.0, 0.5)], [5.0], seed=1)
    ws = sim.adjoint_workspace(20, 5)
    with pytest.raises(gpu.LBMError) as e:
        sim.backward(20, 5, ws)
    assert e.value.code == -6
    sim.forward_ckpt(20, 5, ws)
    sim.step(1)
    with pytest.raises(gpu.LBMError):
        sim.backward(20, 5, ws)


def test_batch_adjoint_bitwise_equals_single(orc, gpu):
    """The ensemble adjoint (every instance's reverse steps in one launch over a shared work-list)
    against each lattice's own lbm_backward: uneven bounce-back lattices, three forms, viscosity
    ratios, an odd step count and a ragged last segment; losses and gradients bit for bit."""
    d = synth.Draws(21)
    cases = []
    for i, (nx, ny) in enumerate(((70, 26), (130, 41), (37, 12))):
        form = synth.FORMS[i % 3]
        p = synth.base_params(nx=nx, ny=ny, wall_force=form, tau_v=(1.1, 2.0, 0.6)[i])
        q = orc.make_params(p)
        rho0 = synth.droplet_rho(nx, ny, q.rho_l, q.rho_v, [(nx / 2.0, 0.5)],
                                 [max(3.0, 0.35 * min(nx, ny))], seed=30 + i)
        gw = synth.gw_smooth(nx, {"rho": 0.05, "psi": -0.02, "modpsi": 0.1}[form], 0.03,
                             seed=int(d.u01() * 1000))
        cases.append((dict(p, rho_l=q.rho_l, rho_v=q.rho_v), gw, rho0))
    N, K = 61, 13
    b = gpu.Batch([c[0] for c in cases], [c[1] for c in cases], [c[2] for c in cases],
                  tune={"tile": 1, "schedule": 2})
    b.step(9)
    states = [b.save_state(i) for i in range(len(cases))]
    ws = b.adjoint_workspace(N, K)
    b.forward_ckpt(N, K, ws)
    Lb = b.loss(0.7, 1.3)
    gb = [g.cpu().numpy() for g in b.backward(N, K, ws, 0.7, 1.3)]
    for i, (p, gw, rho0) in enumerate(cases):
        sim = gpu.Sim(p, gw, rho0)
        sim.load_state(states[i])
        L, g = gpu_grad(sim, N, K, 0.7, 1.3)
        print(f"instance {i}: L {L} vs {Lb[i]}, max |g| {np.abs(g).max():.3e}")
        assert L == Lb[i]
        assert np.array_equal(g, gb[i]), (i, np.abs(g - gb[i]).max())
