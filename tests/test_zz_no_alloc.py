"""The allocation-free entry point lbm_observables_of_state: for population fields held on the
device, its record must equal that of lbm_observables (the existing entry point, which keeps its
scratch in the context's workspace) for the same state. Two calls in a row on one GPU, the second
on a smaller lattice (the fixed scratch array keeps the first call's contents), for bounce-back
walls with and without ghost rows, the wet-node wall and a periodic lattice; and the size limit of
the array."""
import math

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

KEYS = ("rho_min", "rho_max", "umax", "umax_liquid", "mass", "xc", "yc", "r")


def _case(orc, nx, ny, walls, ghost, form, steps):
    p = synth.base_params(nx=nx, ny=ny, walls=walls, ghost=ghost, wall_force=form)
    q = orc.make_params(p)
    # a droplet on the bottom wall, or away from the walls where no ghost rows hold it
    yc = ny / 2.0 if walls == 0 or not ghost else (0.5 if walls == 1 else 1.0)
    rho0 = synth.droplet_rho(nx, ny, q.rho_l, q.rho_v, [(nx / 2.0, yc)], [0.3 * min(nx, ny)],
                             seed=nx + ny, walls=walls != 0)
    if walls == 0:
        rho0 = np.maximum(rho0, q.rho_v)
    gw = synth.gw_smooth(nx, 0.05 if form != "psi" else -0.02, 0.02, seed=ny)
    return dict(p, rho_l=q.rho_l, rho_v=q.rho_v), gw, rho0, steps


def _compare(gpu, case):
    import torch

    p, gw, rho0, steps = case
    sim = gpu.Sim(p, gw, rho0)
    sim.step(steps)
    ref = sim.observables()
    f = torch.from_numpy(sim.f()).cuda()
    g = torch.from_numpy(np.ascontiguousarray(gw)).cuda()
    got = gpu.observables_of_state(p, f, g if p["walls"] else None)
    for k in KEYS:
        a, b = got[k], ref[k]
        assert abs(a - b) <= 1e-12 * max(abs(b), 1e-300) or (math.isnan(a) and math.isnan(b)), \
            (k, a, b)
    assert got["n_fit"] == ref["n_fit"] and got["nonfinite"] == 0
    if math.isnan(ref["theta_deg"]):
        assert math.isnan(got["theta_deg"])
    else:
        assert abs(got["theta_deg"] - ref["theta_deg"]) <= 1e-9
    return got


@pytest.mark.parametrize("walls,ghost", [(1, 1), (1, 0), (2, 1), (0, 1)])
def test_no_alloc_matches_observables_twice(orc, gpu, walls, ghost):
    form = "modpsi" if walls != 1 or ghost else "rho"
    big = _case(orc, 300, 150, walls, ghost, form, 400)
    small = _case(orc, 96, 40, walls, ghost, form, 300)
    _compare(gpu, big)
    _compare(gpu, small)  # second call, smaller input: the array holds the first call's data


def test_no_alloc_rejects_lattices_beyond_the_array(gpu):
    import ctypes as C
    import torch

    p = synth.base_params(nx=2048, ny=1024)
    q = gpu.make_params(p)
    o = gpu.Obs()
    f = torch.zeros(1, dtype=torch.float64, device="cuda")  # never read: rejected first
    rc = gpu.lib().lbm_observables_of_state(C.byref(q), C.c_void_p(f.data_ptr()),
                                            C.c_void_p(f.data_ptr()), None, C.byref(o))
    assert rc == gpu.lbm.E_SIZE
    assert b"static array" in gpu.lib().lbm_last_error(None)
