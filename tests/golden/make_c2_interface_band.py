"""Writes c2_interface_band.json: the oracle's density after the full 50,000 steps of one run of
the 1024 x 512 sweep (pseudopotential-based G_w = -0.1, the end-point run whose round-off grows
fastest) at every fluid node within 4 nodes (Chebyshev distance) of a lattice edge that crosses
the rho_mid = (rho_l + rho_v)/2 contour, where the interface's steep gradients amplify round-off
differences most. Calls only the oracle and the input generators; about 26 minutes on eight
cores.

    python tests/golden/make_c2_interface_band.py
"""
import json
import os
import sys
import time

import numpy as np
from scipy import ndimage

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

STEPS = 50_000
FORM, GW = "psi", -0.1
BAND = 4


def band_nodes(q, rho):
    """Fluid nodes within BAND of a node whose right or upper fluid neighbour lies on the other
    side of rho_mid."""
    mid = 0.5 * (q.rho_l + q.rho_v)
    fl = oracle.fluid_mask(q)
    liq = rho >= mid
    edge = np.zeros_like(fl)
    edge[:, :-1] |= (liq[:, :-1] != liq[:, 1:]) & fl[:, :-1] & fl[:, 1:]
    edge[:-1, :] |= (liq[:-1, :] != liq[1:, :]) & fl[:-1, :] & fl[1:, :]
    near = ndimage.binary_dilation(edge, structure=np.ones((3, 3), bool), iterations=BAND)
    ys, xs = np.nonzero(near & fl)
    return list(zip(xs.tolist(), ys.tolist()))


def main():
    runs = synth.c2_sweep()
    idx = next(i for i, r in enumerate(runs) if r["form"] == FORM and abs(r["G_w"] - GW) < 1e-9)
    r = runs[idx]
    q = oracle.make_params(r["params"])
    rho0 = synth.droplet_rho(q.nx, q.ny, q.rho_l, q.rho_v, r["centres"], r["radii"],
                             seed=r["seed"])
    f = oracle.init_rest(q, rho0)
    t0 = time.time()
    for k in range(0, STEPS, 5_000):
        f = oracle.run(q, r["gw"], f, 5_000)
        print(f"{FORM} {GW}: {k + 5_000} steps, {time.time() - t0:.0f} s", flush=True)
    rho = oracle.fields(q, r["gw"], f)["rho"]
    nodes = band_nodes(q, rho)
    out = {"steps": STEPS, "index": idx, "form": FORM, "G_w": GW, "band": BAND,
           "x": [x for x, _ in nodes], "y": [y for _, y in nodes],
           "rho": [float(rho[y, x]) for x, y in nodes]}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_interface_band.json")
    with open(path, "w") as fh:
        json.dump(out, fh)
    print(f"{len(nodes)} band nodes written to {path}", flush=True)


if __name__ == "__main__":
    main()
