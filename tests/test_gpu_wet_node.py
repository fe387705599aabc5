"""GPU parity of the non-slip wet-node wall scheme of Sec. III.A (walls = 2) against the oracle.

The boundary nodes on the wall planes (rows 1 and ny-2) rebuild the populations arriving from the
solid from the streamed ones and their force of the previous step; the GPU keeps that force as
part of the state, so these tests also cover odd step counts, every tile shape and schedule (the
two-step kernel keeps the intermediate force in LDS), state save/load, and ensembles that mix
both wall schemes. Tolerances as in test_gpu_parity.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

RTOL = 1e-9


def wet_case(orc, nx, ny, form, seed, gwv=0.1, eos="cs"):
    if eos == "cs":
        p = synth.base_params(nx=nx, ny=ny, walls=2, wall_force=form)
    else:
        p = synth.paper_params(nx=nx, ny=ny, wall_force=form)
    q = orc.make_params(p)
    # one droplet on each wall so that both reconstructions see liquid and a contact line
    rho0 = synth.droplet_rho(nx, ny, q.rho_l, q.rho_v,
                             [(nx / 2.0, 1.0), (nx / 5.0, ny - 2.0)],
                             [min(nx, ny) / 3.0, min(nx, ny) / 5.0], seed=seed)
    gw = synth.gw_smooth(nx, gwv, 0.4 * abs(gwv), seed=seed)
    gw[1] = -0.5 * gw[0][::-1]
    pg = dict(p, rho_l=q.rho_l, rho_v=q.rho_v)
    if eos != "cs":
        pg.update(rho1=q.rho1, rho2=q.rho2)
    return q, pg, gw, rho0


def assert_close(q, f_gpu, f_orc, what):
    fl = orc_fluid(q)
    rel = float((np.abs(f_gpu - f_orc).max(0)[fl] / f_orc.sum(0)[fl]).max())
    print(f"{what}: max |df|/rho = {rel:.3e}", flush=True)
    assert rel <= RTOL, f"{what}: {rel:.3e}"


def orc_fluid(q):
    m = np.ones((q.ny, q.nx), bool)
    m[0] = m[-1] = False
    return m


@pytest.mark.parametrize("form", ["rho", "psi", "modpsi"])
@pytest.mark.parametrize("schedule", ["fused", "two_pass", "two_step"])
def test_wet_node_parity(orc, gpu, form, schedule):
    """Ragged 150 x 41 lattice, patterned G_w on both walls, 301 steps (odd)."""
    nx, ny, steps = 150, 41, 301
    gwv = {"rho": 0.1, "psi": -0.03, "modpsi": 0.2}[form]
    q, pg, gw, rho0 = wet_case(orc, nx, ny, form, seed=31, gwv=gwv)
    sim = gpu.Sim(pg, gw, rho0)
    sim.set_schedule(schedule)
    sim.step(steps)
    f = orc.run(q, gw, orc.init_rest(q, rho0), steps)
    assert_close(q, sim.f(), f, f"wet {form}/{schedule}")
    o, oo = sim.observables(), orc.observables(q, gw, f)
    for k in ("rho_min", "rho_max", "mass"):
        assert abs(o[k] - oo[k]) <= RTOL * abs(oo[k]), k
    # contact angle of the bottom droplet: fit window around it (the top droplet is left out)
    lo, hi = nx / 2.0 - 25.0, nx / 2.0 + 25.0
    ow = sim.observables(lo, hi)
    th, _, _, _, n = orc.contact_angle(q, f.sum(0), lo, hi)
    assert ow["n_fit"] == n and n >= 6
    assert abs(ow["theta_deg"] - th) <= 0.1, (ow["theta_deg"], th)


def test_wet_node_parity_paper_eos(orc, gpu):
    """The paper's own EOS, Eq. (15), with the wet-node wall and the modified psi-based force."""
    q, pg, gw, rho0 = wet_case(orc, 90, 40, "modpsi", seed=4, gwv=0.3, eos="piecewise")
    sim = gpu.Sim(pg, gw, rho0)
    sim.step(400)
    f = orc.run(q, gw, orc.init_rest(q, rho0), 400)
    assert_close(q, sim.f(), f, "wet piecewise")


def test_wet_node_every_tile_bitwise(orc, gpu):
    """Every fused tile, every two-step tile and the two-pass schedule give the same bits."""
    q, pg, gw, rho0 = wet_case(orc, 200, 70, "rho", seed=13, gwv=0.1)
    steps = 151
    ref = None
    for sched in [16 + t for t in range(8)] + [32 + t for t in range(8)] + [1]:
        sim = gpu.Sim(pg, gw, rho0)
        sim.set_schedule(sched)
        sim.step(steps)
        f = sim.f()
        if ref is None:
            ref = f
            assert_close(q, f, orc.run(q, gw, orc.init_rest(q, rho0), steps), "wet tiles")
        else:
            assert np.array_equal(f, ref), f"schedule {sched} differs"


@pytest.mark.parametrize("nx,ny", [(3, 4), (5, 6), (61, 9), (125, 17)])
def test_wet_node_tiny_lattices(orc, gpu, nx, ny):
    """Smallest lattices: with ny = 4 both fluid rows are boundary nodes."""
    p = synth.base_params(nx=nx, ny=ny, walls=2, wall_force="modpsi")
    q = orc.make_params(p)
    rho0 = synth.droplet_rho(nx, ny, q.rho_l, q.rho_v, [(nx / 2.0, 1.0)],
                             [max(1.0, min(nx, ny) / 3.0)], jitter=1e-2, seed=nx + ny)
    gw = np.random.default_rng(nx * 7 + ny).uniform(-0.1, 0.1, (2, nx))
    pg = dict(p, rho_l=q.rho_l, rho_v=q.rho_v)
    f = orc.run(q, gw, orc.init_rest(q, rho0), 40)
    for sched in [0, 1, 2] + [16 + t for t in range(8)] + [32 + t for t in range(8)]:
        sim = gpu.Sim(pg, gw, rho0)
        sim.set_schedule(sched)
        sim.step(40)
        assert_close(q, sim.f(), f, f"wet {nx}x{ny} schedule {sched}")


def test_wet_node_save_load_carries_wall_force(orc, gpu):
    """The wall force is part of the state: 60 steps, save, 61 more, reload, 61 more -> same bits."""
    q, pg, gw, rho0 = wet_case(orc, 96, 30, "psi", seed=8, gwv=-0.03)
    sim = gpu.Sim(pg, gw, rho0)
    sim.step(60)
    blob = sim.save_state()
    sim.step(61)
    a = sim.f()
    sim.load_state(blob)
    sim.step(61)
    assert np.array_equal(sim.f(), a)
    assert_close(q, a, orc.run(q, gw, orc.init_rest(q, rho0), 121), "wet save/load")


@pytest.mark.parametrize("schedule,tile", [(0, 0), (1, 1), (2, 1), (1, 4), (2, 4)])
def test_batch_mixing_wall_schemes(orc, gpu, schedule, tile):
    """An ensemble with both wall schemes: each instance bit-identical to its lone run (per-step
    launches, the persistent launch, two steps per launch)."""
    cases = []
    for i, (nx, ny, walls, form) in enumerate([(64, 24, 2, "rho"), (96, 41, 1, "psi"),
                                               (37, 12, 2, "modpsi"), (130, 64, 2, "psi")]):
        p = synth.base_params(nx=nx, ny=ny, walls=walls, wall_force=form)
        q = orc.make_params(p)
        y0 = 1.0 if walls == 2 else 0.5
        rho0 = synth.droplet_rho(nx, ny, q.rho_l, q.rho_v, [(nx / 2, y0)], [min(nx, ny) / 3],
                                 seed=i)
        g = synth.gw_smooth(nx, {"rho": 0.05, "psi": -0.02, "modpsi": 0.1}[form], 0.02, seed=i)
        cases.append((dict(p, rho_l=q.rho_l, rho_v=q.rho_v), g, rho0))
    steps = 131
    b = gpu.Batch([c[0] for c in cases], [c[1] for c in cases], [c[2] for c in cases],
                  tune={"tile": tile, "schedule": schedule})
    b.step(steps)
    for i, (p, g, r) in enumerate(cases):
        s = gpu.Sim(p, g, r)
        s.step(steps)
        assert np.array_equal(b.f(i), s.f()), f"instance {i} (walls {p['walls']})"
