"""Write configs/cs_ratio500.json: temperature and forcing parameter of the CS fluid (TEST INFRA).

The paper tunes sigma of Eq. (9) (0.084 for its piecewise-linear EOS, Sec. III) so that the model's
coexistence densities match the Maxwell construction. For the Carnahan-Starling fluid
(a = 0.5, b = 4, R = 1) at density ratio 500 no value is printed, so this script:

1. finds T with rho_l / rho_v = 500 from the Maxwell construction (oracle.maxwell);
2. bisects sigma on a flat liquid slab (4 x 256, periodic, tau_nu = 1.1) until the simulated
   vapour density, averaged over the last steps, equals the Maxwell vapour density.

Only the oracle and the synthetic-input module are used.
    python -m oracle.calibrate_sigma
"""
from __future__ import annotations

import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

import oracle  # noqa: E402
import synth  # noqa: E402
from oracle.maxwell import cs_temperature_for_ratio, maxwell_cs  # noqa: E402

OUT = os.path.join(os.path.dirname(HERE), "configs", "cs_ratio500.json")


def slab_densities(sigma: float, T: float, steps: int = 24000, avg: int = 4000,
                   every: int = 50, ny: int = 256):
    """Time-averaged bulk (rho_v, rho_l) of the flat slab after `steps` steps."""
    p = synth.base_params(nx=4, ny=ny, walls=0, sigma=sigma, T=T)
    q = oracle.make_params(p)
    f = oracle.init_rest(q, synth.slab_rho(4, ny, q.rho_l, q.rho_v, ny // 4, 3 * ny // 4))
    oracle.run(q, None, f, steps - avg)
    rv, rl = [], []
    for _ in range(avg // every):
        oracle.run(q, None, f, every)
        r = f.sum(0)[:, 0]
        rv.append(r[0])
        rl.append(r[ny // 2])
    return float(np.mean(rv)), float(np.mean(rl))


def main():
    a, b, R, ratio = 0.5, 4.0, 1.0, 500.0
    T = cs_temperature_for_ratio(a, b, R, ratio)
    rho_v, rho_l, _ = maxwell_cs(a, b, R, T)
    lo, hi = 0.10, 0.13
    for it in range(14):
        mid = 0.5 * (lo + hi)
        rv, rl = slab_densities(mid, T)
        print(f"sigma={mid:.6f} rho_v={rv:.6e} (Maxwell {rho_v:.6e}) rho_l={rl:.6f}", flush=True)
        # the simulated vapour density grows with sigma
        if rv < rho_v:
            lo = mid
        else:
            hi = mid
    sigma = round(0.5 * (lo + hi), 5)
    rv, rl = slab_densities(sigma, T)
    out = dict(a=a, b=b, R=R, ratio=ratio, T=T, sigma=sigma,
               note="T: Maxwell construction for rho_l/rho_v = 500; sigma: flat-slab bisection "
                    "on the vapour density (oracle/calibrate_sigma.py)",
               slab_rho_v=rv, slab_rho_l=rl, maxwell_rho_v=rho_v, maxwell_rho_l=rho_l)
    with open(OUT, "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
