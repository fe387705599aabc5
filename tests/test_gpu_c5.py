"""The largest workload at full size: 8 lattices of 2048 x 1024 (six droplets each on a striped
wall, modified form) advanced as one ensemble in the launch configuration the benchmark times
(two steps per launch, 64 x 8 output tiles, 768-thread workgroups, most of them interior).

Checks: the populations of the first and last instance against the oracle element by element
after an odd number of steps (two-step launches plus a single-step remainder); mass conservation
of every instance over 200 steps (an invariant at any size); and the adjoint gradient of the
wetting objective at full size against central differences on wall nodes under droplets.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

RTOL = 1e-9  # max over fluid nodes of max_a |df_a| / rho, as in test_gpu_parity


def c5_cases(orc):
    out = []
    for e in synth.c5_batch():
        q = orc.make_params(e["params"])
        rho0 = synth.droplet_rho(q.nx, q.ny, q.rho_l, q.rho_v, e["centres"], e["radii"],
                                 seed=e["seed"])
        out.append((dict(e["params"], rho_l=q.rho_l, rho_v=q.rho_v), e["gw"], rho0, q, e))
    return out


@pytest.fixture(scope="module")
def c5(orc, gpu):
    cases = c5_cases(orc)
    b = gpu.Batch([c[0] for c in cases], [c[1] for c in cases], [c[2] for c in cases],
                  tune={"tile": 1, "schedule": 2})
    return cases, b


def test_c5_full_size_parity(orc, c5):
    cases, b = c5
    steps = 21
    b.step(steps)
    assert b.current_step == steps
    for i in (0, len(cases) - 1):
        _, gw, rho0, q, _ = cases[i]
        f = orc.run(q, gw, orc.init_rest(q, rho0), steps)
        g = b.f(i)
        fl = orc.fluid_mask(q)
        rel = float((np.abs(g - f).max(0)[fl] / f.sum(0)[fl]).max())
        print(f"c5 instance {i}: {steps} steps, max |df|/rho = {rel:.3e}", flush=True)
        assert rel <= RTOL


def test_c5_mass_conservation(orc, c5):
    cases, b = c5
    m0 = [float(c[2][1:-1].sum()) for c in cases]
    b.step(200 - b.current_step)
    obs = b.observables(allow_nonfinite=True)
    for i, o in enumerate(obs):
        assert o["nonfinite"] == 0
        assert abs(o["mass"] - m0[i]) <= 1e-12 * m0[i], (i, o["mass"], m0[i])


def test_c5_parity_after_200_steps(orc, c5):
    """The first instance against the oracle after the 200 steps of the mass test."""
    cases, b = c5
    assert b.current_step == 200
    _, gw, rho0, q, _ = cases[0]
    f = orc.run(q, gw, orc.init_rest(q, rho0), 200)
    fl = orc.fluid_mask(q)
    rel = float((np.abs(b.f(0) - f).max(0)[fl] / f.sum(0)[fl]).max())
    print(f"c5 instance 0: 200 steps, max |df|/rho = {rel:.3e}", flush=True)
    assert rel <= RTOL


def test_c5_adjoint_full_size(orc, gpu, c5):
    """dL/dG_w of instance 0 over 200 steps from its state after the ensemble's steps (checkpoint
    every 20) against central differences of the forward run on wall nodes under droplets."""
    import torch
    cases, b = c5
    p, gw, rho0, q, e = cases[0]
    state = b.save_state(0)
    sim = gpu.Sim(p, gw, rho0)
    sim.load_state(state)
    n, K = 200, 20
    ws = sim.adjoint_workspace(n, K)
    sim.forward_ckpt(n, K, ws)
    sim.loss()
    g = sim.backward(n, K, ws).cpu().numpy()
    torch.cuda.synchronize()
    assert np.isfinite(g).all()
    scale = np.abs(g[0]).max()
    assert scale > 0
    nodes = [int(round(xc + s * 0.8 * r)) for (xc, _), r in zip(e["centres"][:2], e["radii"][:2])
             for s in (-1, 1)]
    h = 1e-5
    errs = []
    for x in nodes:
        vals = []
        for sgn in (1, -1):
            gg = gw.copy()
            gg[0, x] += sgn * h
            sim.load_state(state)
            sim.set_gw(gg)
            sim.step(n)
            vals.append(sim.loss())
        fd = (vals[0] - vals[1]) / (2 * h)
        errs.append(abs(g[0, x] - fd) / scale)
        print(f"node {x}: adjoint {g[0, x]:.6e}, FD {fd:.6e}", flush=True)
    print("c5 adjoint vs FD, max rel err", max(errs))
    assert max(errs) <= 1e-6


def test_c5_batched_adjoint_full_size(orc, gpu, c5):
    """The ensemble adjoint over all eight 2048 x 1024 lattices at once (200 steps from the state
    after the tests above, checkpoint every 20): instance 0's gradient bit for bit equal to its
    lattice's own lbm_backward, and every instance's gradient finite and non-zero."""
    cases, b = c5
    p, gw, rho0, q, e = cases[0]
    state = b.save_state(0)
    sim = gpu.Sim(p, gw, rho0)
    sim.load_state(state)
    n, K = 200, 20
    ws1 = sim.adjoint_workspace(n, K)
    sim.forward_ckpt(n, K, ws1)
    L1 = sim.loss()
    g1 = sim.backward(n, K, ws1).cpu().numpy()
    del ws1, sim
    ws = b.adjoint_workspace(n, K)
    b.forward_ckpt(n, K, ws)
    Lb = b.loss()
    gb = [g.cpu().numpy() for g in b.backward(n, K, ws)]
    del ws
    print(f"c5 batched adjoint: L0 {Lb[0]} vs {L1}, max |dg| {np.abs(gb[0] - g1).max():.3e}")
    assert Lb[0] == L1
    assert np.array_equal(gb[0], g1)
    for g in gb:
        assert np.isfinite(g).all() and np.abs(g[0]).max() > 0
