"""Pins of the dynamic-wetting measurement (Sec. III.B), no GPU: the oracle's contact line, the
Laplace-law surface tension and the power-law fit against closed forms."""
import math

import numpy as np

import synth


def test_contact_line_linear_crossings(orc):
    """On a row that is linear through rho_mid near each crossing, linear interpolation is exact:
    crossings at x = 10.3 (rising) and 30.7 (falling)."""
    q = orc.make_params(synth.paper_params(nx=48, ny=12))
    mid = 0.5 * (q.rho_l + q.rho_v)
    x = np.arange(48, dtype=float)
    row = np.where(x < 20.5, mid + (x - 10.3), mid - (x - 30.7))
    rho = np.full((12, 48), 1.0)
    rho[1] = row
    left, right = orc.contact_line(q, rho, 1)
    assert abs(left - 10.3) <= 1e-12 and abs(right - 30.7) <= 1e-12
    assert all(math.isnan(v) for v in orc.contact_line(q, np.ones((12, 48)), 1))


def test_contact_line_of_a_symmetric_droplet(orc):
    """A droplet centred on column 24, no jitter: the crossings are mirror images (left + right
    = 48), after the droplet has spread for a while."""
    p = synth.base_params(nx=48, ny=20, walls=2, wall_force="modpsi")
    q = orc.make_params(p)
    rho0 = synth.droplet_rho(48, 20, q.rho_l, q.rho_v, [(24.0, 1.0)], [8.0], jitter=0.0)
    f = orc.run(q, synth.gw_uniform(48, -0.05, 0.0), orc.init_rest(q, rho0), 300)
    left, right = orc.contact_line(q, f.sum(0), 1)
    assert right > left and abs(left + right - 48.0) <= 1e-9


def test_power_law_fit_recovers_exponent():
    from paper_1410_2569_amd import analysis as A
    t = np.linspace(10.0, 3000.0, 300)
    r = 0.37 * t ** 0.485
    r[:5] = np.nan  # not yet in contact
    C, n, k = A.fit_power_law(t, r, 100.0, 2000.0)
    assert abs(n - 0.485) <= 1e-12 and abs(C - 0.37) <= 1e-12 and k > 100


def test_laplace_fit_recovers_gamma():
    from paper_1410_2569_amd import analysis as A
    R = np.array([18.0, 22.0, 26.0, 30.0, 34.0])
    g, c = A.laplace_gamma(R, 6.8 / R + 0.015)
    assert abs(g - 6.8) <= 1e-12 and abs(c - 0.015) <= 1e-13
    assert abs(A.inertial_time(500.0, 30.0, 6.8) - math.sqrt(500.0 * 27000.0 / 6.8)) <= 1e-9


def test_spreading_setup_releases_above_the_wall():
    """The droplet's lowest point lies 2 nodes (half the ~4-node interface) above the wall
    plane: rho at that height is the midpoint density."""
    c = synth.spreading_setup(-0.1)
    rho0 = c["rho0"]
    col = rho0[:, 150]
    mid = 0.5 * (500.0 + 1.0)
    y = np.arange(len(col), dtype=float)
    k = int(np.argmax(col[1:40] >= mid)) + 1  # first row at or above the midpoint density
    yc = y[k - 1] + (mid - col[k - 1]) / (col[k] - col[k - 1])
    assert abs(yc - 3.0) <= 0.01
    assert c["gw"][0, 0] == synth.PAPER_GW_SCALE["modpsi"] * -0.1
