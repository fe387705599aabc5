"""Writes c2_endpoints.json: the oracle's state after the full 50,000 steps of two end-point runs
of the 1024 x 512 sweep (the most wetting density-based G_w and the most non-wetting modified
G_w): the observables and the density at 64 seeded fluid nodes. Calls only the oracle and the
input generators; takes about an hour on eight cores.

    python tests/golden/make_c2_endpoints.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

STEPS = 50_000
PICK = (("rho", -0.14), ("modpsi", 0.4))
NODES = 64


def sample_nodes(nx: int, ny: int, seed: int = 77):
    d = synth.Draws(seed)
    return [(int(d.u01() * nx), 1 + int(d.u01() * (ny - 2))) for _ in range(NODES)]


def main():
    runs = synth.c2_sweep()
    out = {"steps": STEPS, "runs": []}
    for form, g in PICK:
        idx = next(i for i, r in enumerate(runs) if r["form"] == form and abs(r["G_w"] - g) < 1e-9)
        r = runs[idx]
        q = oracle.make_params(r["params"])
        rho0 = synth.droplet_rho(q.nx, q.ny, q.rho_l, q.rho_v, r["centres"], r["radii"],
                                 seed=r["seed"])
        f = oracle.init_rest(q, rho0)
        t0 = time.time()
        for k in range(0, STEPS, 5_000):
            f = oracle.run(q, r["gw"], f, 5_000)
            print(f"{form} {g}: {k + 5_000} steps, {time.time() - t0:.0f} s", flush=True)
        o = oracle.observables(q, r["gw"], f)
        rho = oracle.fields(q, r["gw"], f)["rho"]
        nodes = sample_nodes(q.nx, q.ny)
        out["runs"].append({"index": idx, "form": form, "G_w": g, "observables": o,
                            "nodes": nodes, "rho": [float(rho[y, x]) for x, y in nodes]})
        print(form, g, {k: o[k] for k in ("theta", "rho_min", "rho_max", "mass")}, flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_endpoints.json"),
              "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
