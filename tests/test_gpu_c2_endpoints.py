"""The 1024 x 512 sweep at full length: the two end-point runs (the most wetting density-based G_w
and the most non-wetting modified G_w) for all 50,000 steps in the benchmark's launch
configuration, against the oracle's end state stored in tests/golden/c2_endpoints.json (written
by tests/golden/make_c2_endpoints.py from the oracle alone): the density at 64 seeded fluid
nodes, the density extremes, the mass and the contact angle. Round-off differences grow slowly
through 50,000 steps (3e-13 to 2e-10 relative observed at the sampled nodes); the bound is 1e-8.
"""
import json
import math
import os

import pytest

import synth

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "c2_endpoints.json")


def test_c2_endpoints_full_length(orc, gpu):
    with open(GOLD) as fh:
        gold = json.load(fh)
    runs = synth.c2_sweep()
    for g in gold["runs"]:
        r = runs[g["index"]]
        assert r["form"] == g["form"] and abs(r["G_w"] - g["G_w"]) < 1e-12
        q = orc.make_params(r["params"])
        rho0 = synth.droplet_rho(q.nx, q.ny, q.rho_l, q.rho_v, r["centres"], r["radii"],
                                 seed=r["seed"])
        sim = gpu.Sim(dict(r["params"], rho_l=q.rho_l, rho_v=q.rho_v), r["gw"], rho0)
        sim.step(gold["steps"])
        rho = sim.rho()
        rel = max(abs(rho[y, x] - v) / v for (x, y), v in zip(g["nodes"], g["rho"]))
        o, oo = sim.observables(), g["observables"]
        print(f"{g['form']} G_w={g['G_w']}: sampled rho {rel:.3e}, theta {o['theta_deg']:.4f} "
              f"(oracle {oo['theta']:.4f})", flush=True)
        assert rel <= 1e-8
        for k in ("rho_min", "rho_max", "mass"):
            assert abs(o[k] - oo[k]) <= 1e-8 * abs(oo[k]), k
        assert not math.isnan(oo["theta"]) and abs(o["theta_deg"] - oo["theta"]) <= 1e-3
