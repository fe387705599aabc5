"""Writes c2_endpoints.json: the oracle's state after the full 50,000 steps of the end-point runs
of the 1024 x 512 sweep (the smallest and the largest G_w of each wall-force form): the
observables and the density at 64 seeded fluid nodes. Calls only the oracle and the input
generators; each run takes about 26 minutes on eight cores. Runs named on the command line
(form:G_w) are computed and merged into the existing file; with no arguments, all six.

    python tests/golden/make_c2_endpoints.py [form:G_w ...]
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
PICK = (("rho", -0.14), ("modpsi", 0.4), ("rho", 0.28), ("modpsi", -0.2), ("psi", -0.1),
        ("psi", 0.04))
NODES = 64


def sample_nodes(nx: int, ny: int, seed: int = 77):
    d = synth.Draws(seed)
    return [(int(d.u01() * nx), 1 + int(d.u01() * (ny - 2))) for _ in range(NODES)]


def main():
    runs = synth.c2_sweep()
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_endpoints.json")
    pick = PICK
    out = {"steps": STEPS, "runs": []}
    if len(sys.argv) > 1:
        pick = [(a.split(":")[0], float(a.split(":")[1])) for a in sys.argv[1:]]
        if os.path.exists(path):
            with open(path) as fh:
                out = json.load(fh)
    for form, g in pick:
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
        out["runs"] = [e for e in out["runs"] if e["index"] != idx]
        out["runs"].append({"index": idx, "form": form, "G_w": g, "observables": o,
                            "nodes": nodes, "rho": [float(rho[y, x]) for x, y in nodes]})
        out["runs"].sort(key=lambda e: [(f, v) for f, v in PICK].index((e["form"], e["G_w"])))
        print(form, g, {k: o[k] for k in ("theta", "rho_min", "rho_max", "mass")}, flush=True)
        with open(path, "w") as fh:  # after every run, so that finished runs are kept
            json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
