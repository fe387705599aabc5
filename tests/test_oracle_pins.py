"""Pins of the CPU oracle against what the paper and the mathematics fix (no GPU).

Each test checks the oracle against something other than itself: values printed in the paper
(tests/golden/paper_values.json), closed forms, textbook special cases and invariants. They are
chosen so that a dropped term, a wrong sign or index, or a transposed operand in the oracle fails
at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest

import synth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
CS2 = 1.0 / 3.0
EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
T9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def pw_params(**over):
    g = GOLD["eq15_spinodals"]
    p = dict(nx=4, ny=256, walls=0, ghost=1, eos="piecewise", th_v=g["th_v_over_cs2"] * CS2,
             th_m=g["th_m_over_cs2"] * CS2, th_l=g["th_l_over_cs2"] * CS2, rho_v=g["rho_v"],
             rho_l=g["rho_l"], G=-1.0, sigma=0.084, tau_l=1.1, tau_v=1.1, wall_force="psi",
             **synth.RATES)
    p.update(over)
    return p


# ------------------------------------------------------------------------------------------
# Thermodynamics
# ------------------------------------------------------------------------------------------

def test_eq15_spinodals_match_printed(orc):
    """Maxwell construction of Eq. (15) at (rho_V, rho_L) = (1, 500) -> (1.36, 481.04)."""
    g = GOLD["eq15_spinodals"]
    r1, r2 = orc.piecewise_spinodals(g["rho_v"], g["rho_l"], g["th_v_over_cs2"] * CS2,
                                     g["th_m_over_cs2"] * CS2, g["th_l_over_cs2"] * CS2)
    half_ulp = 0.5 * 10 ** -g["printed_decimals"]
    assert abs(r1 - g["rho1"]) <= half_ulp and abs(r2 - g["rho2"]) <= half_ulp, (r1, r2)


def test_cs_maxwell_closed_form_residuals(orc):
    """CS coexistence: equal pressures and the equal-area rule evaluated with the closed-form
    antiderivative of p/rho^2 (the oracle itself integrates numerically)."""
    a, b, R = 0.5, 4.0, 1.0
    T = orc.cs_temperature_for_ratio(a, b, R, 500.0)
    rv, rl, p0 = orc.maxwell_cs(a, b, R, T)
    assert abs(rl / rv - 500.0) < 1e-9 * 500
    p = lambda r: orc.cs_pressure(r, a, b, R, T)  # noqa: E731
    # p is a difference of terms of size a rho^2, so its round-off is relative to that scale
    assert abs(p(rv) - p0) <= 1e-14 * a * rv ** 2 + 1e-15 * p0
    assert abs(p(rl) - p0) <= 1e-14 * a * rl ** 2

    def Phi(r):  # d/drho Phi = p / rho^2 for Carnahan-Starling
        e = b * r / 4
        return R * T * (math.log(e) + (4 * e - 3 * e * e) / (1 - e) ** 2) - a * r

    area = (Phi(rl) - Phi(rv)) - p0 * (1 / rv - 1 / rl)
    assert abs(area) <= 1e-10 * p0 / rv
    # textbook critical point of Carnahan-Starling: T_c = 0.3773 a/(b R), rho_c = 0.5218/b
    Tc, rc = orc.maxwell.cs_critical(a, b, R)
    assert abs(Tc * b * R / a - 0.3773) < 1e-4 and abs(rc * b - 0.5218) < 1e-4
    assert T < Tc


def test_psi_definition_vapour_branch(orc):
    """psi = sqrt(2 (p_EOS - rho c_s^2)/(G c^2)): on the vapour branch of Eq. (15),
    psi^2 = 2 (1/3 - theta_V) rho for G = -1."""
    q = orc.make_params(pw_params())
    for rho in (0.1, 0.7, 1.3):
        ps = orc.lib().orc_psi(q, rho)
        assert abs(ps * ps - 2 * (CS2 - q.th_v) * rho) <= 1e-14


# ------------------------------------------------------------------------------------------
# Moment basis, equilibria and forcing (Eqs. 2-4, 9)
# ------------------------------------------------------------------------------------------

def tables(orc):
    import ctypes as C
    M = np.zeros(81); ex = (C.c_int * 9)(); ey = (C.c_int * 9)(); op = (C.c_int * 9)()
    w = np.zeros(9)
    orc.lib().orc_tables(M.ctypes.data_as(C.POINTER(C.c_double)), ex, ey, op,
                         w.ctypes.data_as(C.POINTER(C.c_double)))
    return M.reshape(9, 9), np.array(ex[:]), np.array(ey[:]), np.array(op[:]), w


def feq_textbook(rho, v):
    """Second-order D2Q9 equilibrium with t = 4/9, 1/9, 1/36."""
    eu = EX * v[0] + EY * v[1]
    return T9 * rho * (1 + 3 * eu + 4.5 * eu ** 2 - 1.5 * (v[0] ** 2 + v[1] ** 2))


def test_moment_basis_reproduces_eq3(orc):
    M, ex, ey, op, w = tables(orc)
    assert (ex == EX).all() and (ey == EY).all()
    assert all(ex[op[a]] == -ex[a] and ey[op[a]] == -ey[a] for a in range(9))
    assert np.allclose(w, [0] + [1 / 3] * 4 + [1 / 12] * 4, rtol=0, atol=0)
    G = M @ M.T
    assert np.array_equal(G, np.diag(np.diag(G))), "rows of M must be orthogonal"
    rng = np.random.default_rng(0)
    for _ in range(20):
        rho, v = rng.uniform(0.1, 2.0), rng.uniform(-0.1, 0.1, 2)
        v2 = v @ v
        eq3 = rho * np.array([1, -2 + 3 * v2, 1 - 3 * v2, v[0], -v[0], v[1], -v[1],
                              v[0] ** 2 - v[1] ** 2, v[0] * v[1]])
        assert np.allclose(M @ feq_textbook(rho, v), eq3, rtol=0, atol=1e-14)


def bgk_guo(f, F, s):
    """Textbook single-relaxation-time collision with Guo's forcing term (rate s = 1/tau)."""
    rho = f.sum()
    v = np.array([(EX * f).sum() + F[0] / 2, (EY * f).sum() + F[1] / 2]) / rho
    eu = EX * v[0] + EY * v[1]
    eF = EX * F[0] + EY * F[1]
    force = T9 * (3 * ((EX - v[0]) * F[0] + (EY - v[1]) * F[1]) + 9 * eu * eF)
    return f - s * (f - feq_textbook(rho, v)) + (1 - s / 2) * force


def test_mrt_reduces_to_bgk_guo(orc):
    """With every rate equal and sigma = 0, Eqs. (1)-(4), (9) are single-relaxation-time LB with
    Guo's forcing; this pins M, M^-1, Eq. (3) and Eq. (9) together."""
    import ctypes as C
    rng = np.random.default_rng(1)
    for s in (0.6, 1.0, 1.7):
        p = pw_params(sigma=0.0, s_rho=s, s_e=s, s_zeta=s, s_j=s, s_q=s, tau_l=1 / s, tau_v=1 / s)
        q = orc.make_params(p)
        for _ in range(10):
            f = feq_textbook(rng.uniform(0.5, 2), rng.uniform(-0.05, 0.05, 2)) * \
                (1 + 0.05 * rng.standard_normal(9))
            F = rng.uniform(-0.01, 0.01, 2)
            out = np.zeros(9)
            dp = C.POINTER(C.c_double)
            orc.lib().orc_collide_node(q, f.ctypes.data_as(dp), 1.0, F.ctypes.data_as(dp),
                                       F.ctypes.data_as(dp), out.ctypes.data_as(dp))
            assert np.allclose(out, bgk_guo(f, F, s), rtol=0, atol=1e-14)


def test_sigma_term_moves_only_energy_moments(orc):
    """Eq. (9): sigma enters the e and epsilon rows only, with opposite signs and the factors
    1/(tau_e - 1/2) and 1/(tau_zeta - 1/2); mass and momentum of f* do not depend on it."""
    import ctypes as C
    dp = C.POINTER(C.c_double)
    M, *_ = tables(orc)
    f = feq_textbook(1.3, np.array([0.02, -0.01])) * (1 + 0.01 * np.arange(9))
    Fm = np.array([0.003, -0.004]); psi = 0.7
    outs = []
    for sig in (0.0, 0.1):
        q = orc.make_params(pw_params(sigma=sig, s_e=0.8, s_zeta=0.5))
        out = np.zeros(9)
        orc.lib().orc_collide_node(q, f.ctypes.data_as(dp), psi, Fm.ctypes.data_as(dp),
                                   Fm.ctypes.data_as(dp), out.ctypes.data_as(dp))
        outs.append(M @ out)
    d = outs[1] - outs[0]
    assert np.allclose(d[[0, 3, 4, 5, 6, 7, 8]], 0, atol=1e-15)
    Q = 12 * 0.1 * (Fm @ Fm) / psi ** 2
    # m*_k gains (1 - s_k/2) S_k; tau_e = 1.25, tau_zeta = 2
    assert abs(d[1] - (1 - 0.4) * Q / (1.25 - 0.5)) < 1e-15
    assert abs(d[2] + (1 - 0.25) * Q / (2.0 - 0.5)) < 1e-15


# ------------------------------------------------------------------------------------------
# Force stencils (Eqs. 7, 10, 11, 14)
# ------------------------------------------------------------------------------------------

def rho_for_psi_vapour(psi, th_v):
    """Inverse of psi(rho) on the vapour branch of Eq. (15) with G = -1."""
    return psi ** 2 / (2 * (CS2 - th_v))


def test_cohesive_force_of_linear_psi(orc):
    """sum_a w_a e_a e_a = I for w = 1/3, 1/12, so a linear psi field gives exactly
    F_m = -G psi grad(psi) (Eq. 7) away from the periodic seam."""
    nx, ny = 40, 30
    q = orc.make_params(pw_params(nx=nx, ny=ny))
    y, x = np.mgrid[0:ny, 0:nx].astype(float)
    gx, gy = 0.001, 0.002
    psi_lin = 0.3 + gx * x + gy * y
    rho = rho_for_psi_vapour(psi_lin, q.th_v)
    fd = orc.fields(q, None, orc.init_rest(q, rho))
    assert np.allclose(fd["psi"], psi_lin, rtol=1e-13, atol=0)
    inner = (slice(1, ny - 1), slice(1, nx - 1))
    assert np.allclose(fd["Fm"][0][inner], (psi_lin * gx)[inner], rtol=1e-11, atol=0)
    assert np.allclose(fd["Fm"][1][inner], (psi_lin * gy)[inner], rtol=1e-11, atol=0)


@pytest.mark.parametrize("form", ["rho", "psi", "modpsi"])
def test_flat_wall_adhesion_closed_form(orc, form):
    """Flat bottom wall: F_ads = -P (sum of omega_a G_w(x + e_a) e_a over a = 4, 7, 8), i.e.
    F_x = -P (G_w(x+1) - G_w(x-1))/36, F_y = P (G_w(x)/9 + (G_w(x-1) + G_w(x+1))/36), and the
    mirror image at the top wall, with P = rho, psi, psi^2 (Eqs. 10, 11, 14)."""
    nx, ny = 24, 10
    q = orc.make_params(pw_params(nx=nx, ny=ny, walls=1, wall_force=form))
    rng = np.random.default_rng(3)
    gw = rng.uniform(-0.3, 0.3, (2, nx))
    rho = np.full((ny, nx), 1.1) * (1 + 0.05 * rng.random((ny, nx)))
    rho[0] = rho[-1] = 0
    fd = orc.fields(q, gw, orc.init_rest(q, rho))
    P = {"rho": fd["rho"], "psi": fd["psi"], "modpsi": fd["psi"] ** 2}[form]
    for row, g, sgn in ((1, gw[0], 1.0), (ny - 2, gw[1], -1.0)):
        gm, gp = np.roll(g, 1), np.roll(g, -1)
        Fx = -P[row] * (gp - gm) / 36
        Fy = sgn * P[row] * (g / 9 + (gm + gp) / 36)
        assert np.allclose(fd["Fads"][0][row], Fx, rtol=1e-13, atol=1e-17)
        assert np.allclose(fd["Fads"][1][row], Fy, rtol=1e-13, atol=1e-17)
    assert not fd["Fads"][:, 2:ny - 2].any(), "no adhesion away from the walls"
    # uniform G_w: F_ads = (0, G_w P / 6) at the bottom wall
    gu = np.full((2, nx), 0.12)
    fd = orc.fields(q, gu, orc.init_rest(q, rho))
    P = {"rho": fd["rho"], "psi": fd["psi"], "modpsi": fd["psi"] ** 2}[form]
    assert np.allclose(fd["Fads"][1][1], 0.12 * P[1] / 6, rtol=1e-13)


# ------------------------------------------------------------------------------------------
# Invariants of the scheme
# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("walls", [0, 1])
def test_rest_state_stays_at_rest(orc, walls):
    nx, ny = 16, 12
    q = orc.make_params(synth.base_params(nx=nx, ny=ny, walls=walls, wall_force="psi"))
    rho = np.full((ny, nx), 0.3)
    if walls:
        rho[0] = rho[-1] = 0
    f = orc.run(q, np.zeros((2, nx)), orc.init_rest(q, rho), 1000)
    fd = orc.fields(q, np.zeros((2, nx)), f)
    fl = orc.fluid_mask(q)
    assert not fd["v"][:, fl].any(), "velocity must stay exactly zero"
    assert np.abs(fd["rho"][fl] - 0.3).max() <= 1e-14 * 0.3


def droplet_case(orc, nx=64, ny=40, walls=1, form="modpsi", gwv=0.1, R=12.0, steps=1500,
                 jitter=1e-3, x0=None, **over):
    p = synth.base_params(nx=nx, ny=ny, walls=walls, wall_force=form, **over)
    q = orc.make_params(p)
    y0 = 0.5 if walls else ny / 2
    c = [((nx / 2.0) if x0 is None else x0, y0)]
    rho0 = synth.droplet_rho(nx, ny, q.rho_l, q.rho_v, c, [R], jitter=jitter, seed=5,
                             walls=bool(walls))
    gw = synth.gw_uniform(nx, gwv)
    f0 = orc.init_rest(q, rho0)
    return q, gw, f0


def test_mass_conservation(orc):
    q, gw, f = droplet_case(orc, gwv=-0.1)
    fl = orc.fluid_mask(q)
    m0 = f.sum(0)[fl].sum()
    orc.run(q, gw, f, 3000)
    assert abs(f.sum(0)[fl].sum() - m0) <= 1e-12 * m0


def test_momentum_conservation_periodic(orc):
    """Fully periodic: sum of F_m vanishes (pairwise antisymmetry of Eq. 7), so the total
    momentum sum(e f) + sum(F)/2 is constant."""
    q, gw, f = droplet_case(orc, nx=48, ny=48, walls=0, R=10, x0=20.3)
    def mom(f):
        fd = orc.fields(q, None, f)
        F = fd["Fm"] + fd["Fads"]
        return np.array([(EX[:, None, None] * f).sum() + F[0].sum() / 2,
                         (EY[:, None, None] * f).sum() + F[1].sum() / 2])
    P0 = mom(f)
    scale = f.sum()
    orc.run(q, None, f, 1500)
    assert np.abs(mom(f) - P0).max() <= 1e-12 * scale


def test_mirror_symmetry(orc):
    """Droplet centred on a node column, no jitter: rho stays mirror-symmetric about x0 and v_x
    antisymmetric, to round-off."""
    nx = 64
    q, gw, f = droplet_case(orc, nx=nx, jitter=0.0, x0=32.0, form="psi", gwv=-0.03)
    orc.run(q, gw, f, 1500)
    fd = orc.fields(q, gw, f)
    idx = (2 * 32 - np.arange(nx)) % nx
    fl = orc.fluid_mask(q)
    r = fd["rho"]
    assert np.abs(r - r[:, idx])[fl].max() <= 1e-12 * r.max()
    vx = fd["v"][0]
    assert np.abs(vx + vx[:, idx])[fl].max() <= 1e-12


# ------------------------------------------------------------------------------------------
# Coexistence, Laplace law, neutral wall, wetting trend
# ------------------------------------------------------------------------------------------

def slab_average(orc, q, steps, avg=4000, every=50):
    ny = q.ny
    f = orc.init_rest(q, synth.slab_rho(q.nx, ny, q.rho_l, q.rho_v, ny // 4, 3 * ny // 4))
    orc.run(q, None, f, steps - avg)
    rv, rl = [], []
    for _ in range(avg // every):
        orc.run(q, None, f, every)
        r = f.sum(0)[:, 0]
        rv.append(r[0]); rl.append(r[ny // 2])
    return float(np.mean(rv)), float(np.mean(rl)), f


@pytest.mark.slow
def test_flat_interface_eq15_matches_table1(orc):
    """Eq. (15) with sigma = 0.084: a flat interface reaches the neutral-row densities of Table I
    (rho_min = 1.00, rho_max = 500.5): thermodynamic consistency of the forcing of Eq. (9)."""
    t = GOLD["table1_neutral_row"]
    q = orc.make_params(pw_params(sigma=t["sigma"]))
    rv, rl, _ = slab_average(orc, q, 30000)
    print("Eq.15 slab rho_v, rho_l =", rv, rl)
    # The flat slab's vapour density sits 2.2% below the printed (droplet) value for every sigma
    # inside the printed rounding 0.0835..0.0845 (0.977..0.980), hence 2.5%. The pin still
    # separates the forcing term sharply: without the sigma term, with half of it or with its
    # sign flipped psi becomes undefined, and doubling it gives rho_v = 1.29.
    assert abs(rl - t["rho_max"]) <= 0.005 * t["rho_max"]
    assert abs(rv - t["rho_min"]) <= 0.025 * t["rho_min"]


@pytest.mark.slow
def test_flat_interface_cs_calibrated(orc):
    """CS fluid with the calibrated sigma: the liquid density (not the calibration target) meets
    the Maxwell construction within 0.5%."""
    q = orc.make_params(synth.base_params(nx=4, ny=256, walls=0))
    rv, rl, _ = slab_average(orc, q, 24000)
    assert abs(rl - q.rho_l) <= 0.005 * q.rho_l
    assert abs(rv - q.rho_v) <= 0.01 * q.rho_v


@pytest.mark.slow
def test_laplace_law(orc):
    """Free droplets (periodic): Delta p = p_in - p_out with p = rho c_s^2 + G psi^2 / 2 (Eq. 8)
    is linear in 1/R, with slope close to the flat-interface surface tension
    gamma = -(G/6) integral (dpsi/dy)^2 dy from the pressure tensor of Eq. (8)."""
    q = orc.make_params(synth.base_params(nx=4, ny=128, walls=0))
    _, _, fs = slab_average(orc, q, 12000, avg=50)
    psi = orc.fields(q, None, fs)["psi"][:, 0]
    dpsi = (np.roll(psi, -1) - np.roll(psi, 1)) / 2
    gamma = -(q.G / 6) * (dpsi ** 2).sum() / 2  # the slab has two interfaces
    inv_r, dp = [], []
    n = 112
    for R in (12.0, 16.0, 22.0):
        qd = orc.make_params(synth.base_params(nx=n, ny=n, walls=0))
        rho0 = synth.droplet_rho(n, n, qd.rho_l, qd.rho_v, [(n / 2, n / 2)], [R], jitter=0,
                                 walls=False)
        f = orc.run(qd, None, orc.init_rest(qd, rho0), 8000)
        fd = orc.fields(qd, None, f)
        p = fd["rho"] / 3 + qd.G * fd["psi"] ** 2 / 2
        # radius from the rho_mid area, pressures from the centre and a far corner
        rm = 0.5 * (qd.rho_l + qd.rho_v)
        Req = math.sqrt((fd["rho"] >= rm).sum() / math.pi)
        inv_r.append(1 / Req)
        dp.append(p[n // 2, n // 2] - p[0, 0])
    slope, icpt = np.polyfit(inv_r, dp, 1)
    resid = np.array(dp) - (slope * np.array(inv_r) + icpt)
    print("gamma_flat", gamma, "slope", slope, "intercept", icpt, "dp", dp)
    assert np.abs(resid).max() <= 0.02 * max(dp)
    assert abs(icpt) <= 0.05 * max(dp)
    assert abs(slope - gamma) <= 0.10 * gamma


@pytest.mark.slow
def test_neutral_wall_is_90_degrees(orc):
    """G_w = 0 with Eq. (7) applied at the wall (mirrored ghost psi): 90 degrees analytically."""
    cfg = synth.c1_small()
    q = orc.make_params(cfg["params"])
    rho0 = synth.droplet_rho(q.nx, q.ny, q.rho_l, q.rho_v, cfg["centres"], cfg["radii"],
                             seed=cfg["seed"])
    gw = synth.gw_uniform(q.nx, 0.0)
    f = orc.run(q, gw, orc.init_rest(q, rho0), 6000)
    o = orc.observables(q, gw, f)
    target = GOLD["neutral_wall"]["theta_analytic"]
    print("neutral wall theta", o["theta"])
    assert abs(o["theta"] - target) <= 1.0


@pytest.mark.slow
@pytest.mark.parametrize("form,values", [("rho", (-0.08, 0.0, 0.12)),
                                         ("psi", (-0.04, 0.0, 0.04)),
                                         ("modpsi", (-0.15, 0.0, 0.25))])
def test_angle_increases_with_gw(orc, form, values):
    """The static angle grows strictly with G_w for each interaction (Sec. II.B, Figs. 2-4)."""
    th = []
    for g in values:
        q, gw, f = droplet_case(orc, nx=80, ny=40, form=form, gwv=g, R=14.0)
        orc.run(q, gw, f, 3000)
        th.append(orc.observables(q, gw, f)["theta"])
    print(form, values, th)
    assert th[0] < th[1] < th[2]
    assert th[0] < 90.0 < th[2]
