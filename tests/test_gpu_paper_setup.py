"""The paper's own simulations on the GPU (Sec. III.A): Eq. (15) EOS at rho_L/rho_V = 500/1,
sigma = 0.084, the wet-node wall, 300 x 100 fluid nodes, a droplet of R = 30 centred 25 nodes
above the wall, every printed G_w of Figs. 2-4 advanced as one ensemble.

Checks, in this order: element-wise parity with the oracle at the full lattice size; the
neutral wall (89.3 degrees printed, 90 analytic); the printed static angles of Figs. 2-4 with
the G_w scale per interaction (synth.PAPER_GW_SCALE); the behaviour at the ends of the ranges
(full spreading, 180 degrees, the pseudopotential-based form's limits, Fig. 5); and the density
extremes of Table I (values at 90 degrees, orderings elsewhere).
"""
import json
import math
import os

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
KEY = {"rho": "rho_based", "psi": "psi_based", "modpsi": "modified_psi_based"}
STEPS = 30_000


def printed(form, g):
    return dict(GOLD["wetting_trend"][KEY[form]]).get(g)


def test_paper_setup_parity_full_size(orc, gpu):
    """300 x 102, density-based form at the printed G_w = 0.21: GPU against the oracle, element
    by element after 400 steps (two-step schedule, even and odd splits)."""
    c = synth.paper_setup("rho", 0.21)
    q = orc.make_params(c["params"])
    pg = dict(c["params"], rho1=q.rho1, rho2=q.rho2)
    sim = gpu.Sim(pg, c["gw"], c["rho0"])
    sim.step(201)
    sim.step(199)
    f = orc.run(q, c["gw"], orc.init_rest(q, c["rho0"]), 400)
    fl = orc.fluid_mask(q)
    rel = float((np.abs(sim.f() - f).max(0)[fl] / f.sum(0)[fl]).max())
    print("paper setup parity", rel)
    assert rel <= 1e-9
    o, oo = sim.observables(), orc.observables(q, c["gw"], f)
    assert abs(o["rho_max"] - oo["rho_max"]) <= 1e-9 * oo["rho_max"]
    assert abs(o["theta_deg"] - oo["theta"]) <= 0.1


@pytest.fixture(scope="module")
def figures(gpu):
    cases = synth.paper_figures()
    b = gpu.Batch([c["params"] for c in cases], [c["gw"] for c in cases],
                  [c["rho0"] for c in cases])
    b.step(STEPS)
    obs = b.observables(allow_nonfinite=True)
    out = {}
    for c, o in zip(cases, obs):
        out[(c["form"], c["gw_printed"])] = o
        print(c["form"], c["gw_printed"], "theta", round(o["theta_deg"], 2), "printed",
              printed(c["form"], c["gw_printed"]), "rho", o["rho_min"], o["rho_max"], flush=True)
    return out


def test_neutral_wall(figures):
    """G_w = 0: 90 degrees analytically, 89.3 printed (Fig. 1); identical for the three forms."""
    th = [figures[(f, 0.0)]["theta_deg"] for f in synth.FORMS]
    assert th[0] == th[1] == th[2]
    assert abs(th[0] - GOLD["neutral_wall"]["theta_paper"]) <= 1.0
    assert abs(th[0] - GOLD["neutral_wall"]["theta_analytic"]) <= 1.5


@pytest.mark.parametrize("form,tol", [("rho", 2.0), ("modpsi", 2.0), ("psi", 3.5)])
def test_printed_static_angles(figures, form, tol):
    """Figs. 2-4: every printed angle between 40 and 150 degrees, within tol."""
    n = 0
    for g in synth.PAPER_GW[form]:
        p = printed(form, g)
        if p is None or not 40.0 <= p <= 150.0:
            continue
        th = figures[(form, g)]["theta_deg"]
        assert abs(th - p) <= tol, (form, g, th, p)
        n += 1
    assert n >= 4


def test_range_ends(figures):
    """Strong wetting spreads below 30 degrees (printed 17.6 and 19.0, still spreading at this
    step count); the density-based and modified forms reach 180 degrees (the fitted circle no
    longer cuts the wall plane at y = 1); the pseudopotential-based form still holds the droplet
    at the printed G_w = 3.6 (165.6 degrees, Fig. 3) and its printed G_w = -3.0 lies past the
    stability limit of this model."""
    for form, g in (("rho", -0.21), ("modpsi", -0.3)):
        assert figures[(form, g)]["theta_deg"] < 30.0
    for form, g in (("rho", 0.36), ("modpsi", 0.53)):
        o = figures[(form, g)]
        assert math.isnan(o["theta_deg"]) and o["yc"] - 1.0 > o["r"] - 0.5, o
        assert o["nonfinite"] == 0
    assert figures[("psi", 3.6)]["theta_deg"] >= 155.0
    assert figures[("psi", -3.0)]["nonfinite"] > 0


def test_table1_density_extremes(figures):
    """Table I: at 90 degrees rho_min = 1.00 and rho_max = 500.5; non-wetting walls keep rho_max
    near rho_L and lower rho_min as the angle grows, wetting walls raise rho_max; at about 150
    degrees the vapour density drops least with the modified form and most with the
    pseudopotential-based one (4 %, 13 %, 79 % printed)."""
    t = GOLD["table1_neutral_row"]
    o = figures[("rho", 0.0)]
    assert abs(o["rho_min"] - t["rho_min"]) <= 0.01 and abs(o["rho_max"] - t["rho_max"]) <= 0.5
    for form in synth.FORMS:
        pts = [(figures[(form, g)]["theta_deg"], figures[(form, g)]) for g in synth.PAPER_GW[form]
               if figures[(form, g)]["nonfinite"] == 0 and not math.isnan(figures[(form, g)]["theta_deg"])]
        pts.sort(key=lambda p: p[0])
        wet = [o["rho_max"] for th, o in pts if th < 85.0]
        dry = [o for th, o in pts if th > 95.0]
        assert all(a > b for a, b in zip(wet, wet[1:])), (form, wet)
        assert all(500.0 < o["rho_max"] < 502.0 for o in dry), form
        mins = [o["rho_min"] for o in dry]
        assert all(a > b for a, b in zip(mins, mins[1:])), (form, mins)
    m150 = {f: figures[(f, g)]["rho_min"] for f, g in (("modpsi", 0.3), ("rho", 0.21), ("psi", 3.0))}
    assert m150["modpsi"] > m150["rho"] > m150["psi"]
