"""Pins of the oracle's solid-mask geometry (rough surfaces, Sec. III.B), no GPU.

A mask holding only the rows y = 0 and y = ny-1 is the bounce-back channel without a ghost layer:
the two geometry paths must give the same bits. Pillars must conserve mass exactly (halfway
bounce-back), keep a mirror-symmetric state symmetric, and Cassie's law, Eq. (17), must reproduce
the printed apparent angles from the printed flat ones (the closed form that the GPU test of the
rough surface checks against simulated angles).
"""
import json
import math
import os

import numpy as np
import pytest

import synth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def channel_case(orc, nx=48, ny=26, form="modpsi"):
    p = synth.base_params(nx=nx, ny=ny, walls=1, ghost=0, wall_force=form)
    q = orc.make_params(p)
    rho0 = synth.droplet_rho(nx, ny, q.rho_l, q.rho_v, [(nx / 2.0, ny / 2.0)], [ny / 4.0],
                             seed=3)
    return p, q, rho0


@pytest.mark.parametrize("form", ["rho", "psi", "modpsi"])
def test_row_mask_equals_bounce_back_channel(orc, form):
    p, q, rho0 = channel_case(orc, form=form)
    nx, ny = q.nx, q.ny
    mean = {"rho": 0.05, "psi": -0.02, "modpsi": 0.05}[form]
    gw_rows = synth.gw_smooth(nx, mean, 0.5 * abs(mean), seed=4)
    gw_rows[1] = -0.5 * gw_rows[0][::-1]
    f1 = orc.run(q, gw_rows, orc.init_rest(q, rho0), 300)
    m = np.zeros((ny, nx), np.uint8)
    m[0] = m[-1] = 1
    qm = orc.make_params(dict(p, walls=3, solid=m))
    gw_nodes = np.zeros((ny, nx))
    gw_nodes[0], gw_nodes[-1] = gw_rows[0], gw_rows[1]
    f2 = orc.run(qm, gw_nodes, orc.init_rest(qm, rho0), 300)
    assert np.array_equal(f1, f2)


def pillar_case(orc, form="modpsi", gwv=-0.05, nx=63, ny=40, height=6):
    m = synth.pillar_mask(nx, ny, height=height, width=3, gap=4)
    p = synth.base_params(nx=nx, ny=ny, walls=3, ghost=0, wall_force=form, solid=m)
    q = orc.make_params(p)
    rho0 = synth.droplet_rho(nx, ny, q.rho_l, q.rho_v, [(nx // 2, height + 0.5 + 8.0)], [10.0],
                             jitter=0.0, walls=False)
    rho0[m != 0] = 0.0
    gw = np.where(m != 0, gwv, 0.0)
    return q, m, gw, rho0


def test_pillars_conserve_mass(orc):
    q, m, gw, rho0 = pillar_case(orc)
    f = orc.init_rest(q, rho0)
    m0 = f.sum()
    orc.run(q, gw, f, 500)
    assert abs(f.sum() - m0) <= 1e-12 * m0
    assert not f[:, m != 0].any(), "solid nodes hold no populations"


def test_pillars_mirror_symmetry(orc):
    """63 columns, pillars of 3 with gaps of 4 centred on x = 31 (period 7 divides 63), no
    jitter: the state stays mirror-symmetric about x = 31 (pillar tops, sides and corners)."""
    q, m, gw, rho0 = pillar_case(orc, form="rho", gwv=0.03)
    idx = (62 - np.arange(q.nx)) % q.nx
    assert np.array_equal(m, m[:, idx])
    f = orc.run(q, gw, orc.init_rest(q, rho0), 600)
    r = f.sum(0)
    assert np.abs(r - r[:, idx]).max() <= 1e-11 * r.max()
    assert np.abs(r).max() > 0


def test_cassie_law_reproduces_printed_angles():
    """Eq. (17) with f' = a/(a + b) = 6/9: 138.5 -> 146.4 and 138 -> 146.0 degrees (Sec. III.B)."""
    f = 6.0 / 9.0
    for flat, rough in ((138.5, 146.4), (138.0, 146.0)):
        c = f * math.cos(math.radians(flat)) + f - 1.0
        assert abs(math.degrees(math.acos(c)) - rough) <= 0.05


def test_pillar_mask_geometry():
    m = synth.pillar_mask()
    assert m.shape == (150, 300)
    assert m[0].all() and m[-1].all()
    col = m[1:21].all(0)           # pillar columns are solid over their whole height
    assert not m[21:-1].any()      # nothing above the pillar tops
    runs = np.diff(np.flatnonzero(np.diff(np.r_[0, col.astype(int), 0])))
    assert set(runs[1:-1].tolist()) <= {6, 3}, "pillars 6 wide, gaps 3 wide (away from the seam)"
    assert col[150] and col[147] and col[152]  # centred on x = 150
