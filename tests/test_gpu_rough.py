"""GPU parity of the solid-mask geometry (rough surfaces, Sec. III.B) against the oracle.

Pillared lattices with every wall force, the fused schedule with each of its tile shapes, the
two-pass schedule and two steps per launch with each output tile; the channel expressed as a mask
against the bounce-back channel without ghost rows; the paper's 300 x 150 pillared surface at full
size (where most two-step tiles see no solid node and take the interior variant); state round
trips; masked ensembles; and the entry points that do not take a mask. Tolerances as in
test_gpu_parity.
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

RTOL = 1e-9


def pillar_case(orc, form, nx=63, ny=40, height=6):
    gwv = {"rho": 0.03, "psi": -0.01, "modpsi": -0.05}[form]
    m = synth.pillar_mask(nx, ny, height=height, width=3, gap=4)
    p = synth.base_params(nx=nx, ny=ny, walls=3, ghost=0, wall_force=form, solid=m)
    q = orc.make_params(p)
    rho0 = synth.droplet_rho(nx, ny, q.rho_l, q.rho_v, [(nx / 2.0, height + 0.5 + 8.0)], [10.0],
                             seed=7, walls=False)
    rho0[m != 0] = 0.0
    gw = np.where(m != 0, gwv, 0.0)
    gw[m != 0] += 0.2 * gwv * np.sin(np.nonzero(m)[1] / 5.0)  # a pattern along the surface
    pg = dict(p, rho_l=q.rho_l, rho_v=q.rho_v)
    return q, pg, m, gw, rho0


def rel_err(q, f_gpu, f_orc):
    fl = orc_fluid(q)
    return float((np.abs(f_gpu - f_orc).max(0)[fl] / f_orc.sum(0)[fl]).max())


def orc_fluid(q):
    return q._solid == 0


@pytest.mark.parametrize("form", ["rho", "psi", "modpsi"])
def test_mask_parity_all_schedules(orc, gpu, form):
    q, pg, m, gw, rho0 = pillar_case(orc, form)
    steps = 301
    f = orc.run(q, gw, orc.init_rest(q, rho0), steps)
    ref = None
    for sched in (16, 17, 18, 19, 1, 2, 32, 33, 34, 35, 36, 37, 38, 39):
        sim = gpu.Sim(pg, gw, rho0)
        sim.set_schedule(sched)
        sim.step(steps)
        g = sim.f()
        rel = rel_err(q, g, f)
        print(f"mask {form} schedule {sched}: {rel:.3e}", flush=True)
        assert rel <= RTOL
        assert not g[:, m != 0].any()
        if ref is None:
            ref = g
        else:
            assert np.array_equal(g, ref), f"schedule {sched} differs from tile 0"
    o = sim.observables(y_wall=6.5)
    oo = orc.observables(q, gw, f, y_wall=6.5)
    for k in ("rho_min", "rho_max", "mass"):
        assert abs(o[k] - oo[k]) <= RTOL * abs(oo[k]), k
    assert o["n_fit"] == oo["n_fit"]
    if np.isnan(oo["theta"]):  # the fitted circle misses the contact plane on both sides
        assert np.isnan(o["theta_deg"]) and abs(o["yc"] - oo["yc"]) <= 1e-6 * abs(oo["yc"])
    else:
        assert abs(o["theta_deg"] - oo["theta"]) <= 0.1


def test_row_mask_matches_bounce_back_channel(orc, gpu):
    """A mask of the two wall rows is the bounce-back channel without ghost rows."""
    nx, ny = 70, 30
    p = synth.base_params(nx=nx, ny=ny, walls=1, ghost=0, wall_force="modpsi")
    q = orc.make_params(p)
    rho0 = synth.droplet_rho(nx, ny, q.rho_l, q.rho_v, [(35.0, 15.0)], [7.0], seed=2)
    gw_rows = synth.gw_smooth(nx, 0.05, 0.02, seed=3)
    gw_rows[1] = -gw_rows[0]
    pg = dict(p, rho_l=q.rho_l, rho_v=q.rho_v)
    a = gpu.Sim(pg, gw_rows, rho0)
    a.set_schedule("fused")
    a.step(250)
    m = np.zeros((ny, nx), np.uint8)
    m[0] = m[-1] = 1
    gw_nodes = np.zeros((ny, nx))
    gw_nodes[0], gw_nodes[-1] = gw_rows[0], gw_rows[1]
    b = gpu.Sim(dict(pg, walls=3), gw_nodes, rho0, solid=m)
    b.step(250)
    fa, fb = a.f(), b.f()
    fl = np.ones((ny, nx), bool)
    fl[0] = fl[-1] = False
    rel = float((np.abs(fa - fb).max(0)[fl] / fa.sum(0)[fl]).max())
    print("row mask vs channel", rel)
    assert rel <= 1e-12
    f = orc.run(q, gw_rows, orc.init_rest(q, rho0), 250)
    assert float((np.abs(fb - f).max(0)[fl] / f.sum(0)[fl]).max()) <= RTOL


def test_paper_rough_surface_full_size(orc, gpu):
    """300 x 150 with pillars 20 high, 6 wide, gaps of 3, Eq. (15), density-based force: GPU
    against the oracle after 201 steps; two steps per launch (every output tile, most of them
    interior) give the fused schedule's bits."""
    c = synth.rough_setup("rho", -1.85, gw_scale=1.0)
    q = orc.make_params(c["params"])
    pg = dict(c["params"], rho1=q.rho1, rho2=q.rho2)
    sim = gpu.Sim(pg, c["gw"], c["rho0"])
    sim.set_schedule("fused")
    sim.step(201)
    ref = sim.f()
    f = orc.run(q, c["gw"], orc.init_rest(q, c["rho0"]), 201)
    rel = rel_err(q, ref, f)
    print("rough full size", rel)
    assert rel <= RTOL
    for sched in (2, 33, 34, 35, 36, 37, 38, 39):
        s2 = gpu.Sim(pg, c["gw"], c["rho0"])
        s2.set_schedule(sched)
        s2.step(201)
        assert np.array_equal(s2.f(), ref), f"schedule {sched}"


def test_mask_save_load_and_set_gw(orc, gpu):
    q, pg, m, gw, rho0 = pillar_case(orc, "modpsi")
    sim = gpu.Sim(pg, gw, rho0)
    sim.step(50)
    blob = sim.save_state()
    sim.step(51)
    a = sim.f()
    sim.load_state(blob)
    sim.step(51)
    assert np.array_equal(sim.f(), a)
    # changing G_w mid-run equals the oracle run with the same change
    gw2 = 0.5 * gw
    sim.load_state(blob)
    sim.set_gw(gw2)
    sim.step(40)
    f = orc.run(q, gw, orc.init_rest(q, rho0), 50)
    f = orc.run(q, gw2, f, 40)
    assert rel_err(q, sim.f(), f) <= RTOL


def test_mask_rejected_where_unsupported(orc, gpu):
    q, pg, m, gw, rho0 = pillar_case(orc, "rho")
    sim = gpu.Sim(pg, gw, rho0)
    for sched in (20, 21, 22, 23):  # the overlapped fused tiles
        with pytest.raises(gpu.LBMError):
            sim.set_schedule(sched)
    with pytest.raises(gpu.LBMError):
        sim.adjoint_workspace(100, 10)


@pytest.mark.parametrize("tile,schedule", [(0, 0), (1, 0), (2, 0), (3, 0), (1, 1), (0, 2), (1, 2),
                                           (2, 2), (3, 2), (4, 1), (4, 2)])
def test_masked_ensemble_bitwise_equals_lone_runs(orc, gpu, tile, schedule):
    """Pillared lattices of several sizes and forms as one ensemble: every instance carries the
    same bits as the lattice stepped alone, and the per-instance contact planes feed the fits."""
    cases = []
    for i, (form, nx, ny, h) in enumerate([("rho", 63, 40, 6), ("modpsi", 49, 30, 4),
                                           ("psi", 77, 33, 8)]):
        q, pg, m, gw, rho0 = pillar_case(orc, form, nx=nx, ny=ny, height=h)
        cases.append((pg, m, gw, rho0, h + 0.5))
    steps = 131
    b = gpu.Batch([c[0] for c in cases], [c[2] for c in cases], [c[3] for c in cases],
                  tune={"tile": tile, "schedule": schedule}, solids=[c[1] for c in cases])
    b.step(steps)
    obs = b.observables(y_wall=[c[4] for c in cases], allow_nonfinite=True)
    for i, (pg, m, gw, rho0, yw) in enumerate(cases):
        s = gpu.Sim(pg, gw, rho0, solid=m)
        s.step(steps)
        assert np.array_equal(b.f(i), s.f()), f"instance {i}"
        o = s.observables(y_wall=yw, allow_nonfinite=True)
        assert o["rho_min"] == obs[i]["rho_min"] and o["n_fit"] == obs[i]["n_fit"]


def test_masked_ensemble_rejects_mixing(orc, gpu):
    q, pg, m, gw, rho0 = pillar_case(orc, "rho")
    flat = synth.base_params(nx=40, ny=20)
    rf = synth.droplet_rho(40, 20, q.rho_l, q.rho_v, [(20.0, 0.5)], [6.0])
    with pytest.raises((gpu.LBMError, AssertionError)):  # the binding or the library refuses
        gpu.Batch([pg, dict(flat, rho_l=q.rho_l, rho_v=q.rho_v)], [gw, np.zeros((2, 40))],
                  [rho0, rf])
