"""Pins of the oracle parts that no invariant of the step reaches: the phase-interpolated shear
viscosity (Sec. III.C), the wetting objective and the contact-angle geometry (Figs. 1-4).

Each is checked against a closed form that does not restate the oracle's code:
* viscosity: the hydrodynamic decay rate nu k^2 of a shear wave in a uniform fluid at rest
  density rho, with nu = nu_V + clamp((rho - rho_V)/(rho_L - rho_V), 0, 1) (nu_L - nu_V) (the
  viscosity reading of Sec. III.C) and nu = (tau_nu - 1/2) c_s^2 (Sec. II.A);
* objective: slabs and single nodes whose centroid height and wetted length are known exactly;
* contact angle: density fields built from a circle that cuts the wall plane at a chosen angle.

Every pin is then shown to fail when a plausible mistake is planted in a copy of the oracle (the
C source recompiled, or the Python function rebuilt from its edited source): viscosities of the
two phases swapped, the clamp of the phase fraction removed, the wall plane at 0, the band
excluded next to the wall one node too thin, the wrong row for the wetted length.
"""
import inspect
import math
import subprocess
import textwrap

import numpy as np
import pytest

import oracle
import synth

E = np.array([[0, 0], [1, 0], [0, 1], [-1, 0], [0, -1], [1, 1], [-1, 1], [-1, -1], [1, -1]],
             dtype=np.float64)
T9 = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
NU_L = 1.0 / 30.0  # liquid kinematic viscosity of Sec. III.C (tau_nu = 0.6)


# ------------------------------------------------------------------------------------------
# planted mistakes
# ------------------------------------------------------------------------------------------

def _mutant_c_library(tmp_path, old: str, new: str) -> str:
    src = open(oracle.SRC).read()
    assert src.count(old) == 1, old
    c = tmp_path / "mutant.c"
    c.write_text(src.replace(old, new))
    so = tmp_path / "mutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fopenmp", "-shared",
                           "-fPIC", str(c), "-o", str(so), "-lm"])
    return str(so)


def _use_c_library(monkeypatch, so: str):
    monkeypatch.setattr(oracle, "build", lambda force=False: so)
    monkeypatch.setattr(oracle, "_lib", None)


def _mutant_function(fn, old: str, new: str):
    src = textwrap.dedent(inspect.getsource(fn))
    assert src.count(old) == 1, old
    ns = dict(fn.__globals__)
    exec(compile(src.replace(old, new), f"<mutant {fn.__name__}>", "exec"), ns)
    return ns[fn.__name__]


# ------------------------------------------------------------------------------------------
# shear viscosity between the phases (Sec. III.C)
# ------------------------------------------------------------------------------------------

def shear_wave_viscosity(rho0: float, tau_l: float, tau_v: float, ny: int = 256,
                         steps: int = 3000, u0: float = 1e-4) -> float:
    """Kinematic viscosity measured from the decay of u_x = u0 sin(k y), k = 2 pi/ny, in a fully
    periodic fluid of uniform density rho0 (no force acts: psi is uniform and there is no wall).
    The amplitude decays as exp(-nu k^2 t); nu is the fitted rate over k^2."""
    p = synth.base_params(nx=3, ny=ny, walls=0, tau_l=tau_l, tau_v=tau_v)
    q = oracle.make_params(p)
    k = 2.0 * np.pi / ny
    ux = u0 * np.sin(k * np.arange(ny))[:, None] * np.ones((1, q.nx))
    f = np.empty((9, ny, q.nx))
    for a in range(9):  # second-order equilibrium at (rho0, u)
        eu = E[a, 0] * ux
        f[a] = T9[a] * rho0 * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * ux * ux)
    f = np.ascontiguousarray(f)
    s = np.sin(k * np.arange(ny))
    t, amp = [], []
    for n in range(0, steps + 1, 100):
        if n:
            try:
                oracle.run(q, None, f, 100)
            except oracle.OracleError:
                return math.nan
        v = oracle.fields(q, None, f)["v"][0][:, 0]
        t.append(n)
        amp.append(float((v * s).sum() / (s * s).sum()))
    t, amp = np.array(t[5:], dtype=np.float64), np.array(amp[5:])
    if not (np.all(np.isfinite(amp)) and np.all(amp > 0)):
        return math.nan
    slope = np.polyfit(t, np.log(amp), 1)[0]
    return -slope / k ** 2


def viscosity_cases():
    """(ratio nu_V/nu_L, rest density, expected nu): vapour, liquid, a density between the
    liquid spinodal and rho_L (phase fraction 0.85, a uniform state that does not separate), and
    a compressed liquid at 1.05 rho_L (phase fraction above 1: clamped)."""
    q = oracle.make_params(synth.base_params())
    rv, rl = q.rho_v, q.rho_l
    out = []
    for ratio in (5.0, 15.0):
        nu_v = ratio * NU_L
        for rho in (rv, rl, 0.38, 1.05 * rl):
            phi = min(max((rho - rv) / (rl - rv), 0.0), 1.0)
            out.append((ratio, rho, nu_v + phi * (NU_L - nu_v)))
    return out


def worst_viscosity_error() -> float:
    worst = 0.0
    for ratio, rho, nu in viscosity_cases():
        got = shear_wave_viscosity(rho, 3.0 * NU_L + 0.5, 3.0 * ratio * NU_L + 0.5)
        err = abs(got / nu - 1.0) if math.isfinite(got) else math.inf
        worst = max(worst, err)
    return worst


def test_shear_wave_decay_follows_phase_interpolated_viscosity(orc):
    """nu_V/nu_L = 5 and 15 with nu_L = 1/30: the measured viscosity matches the interpolation
    within 1% in the vapour, the liquid, between them and past rho_L (clamp)."""
    assert worst_viscosity_error() < 0.01


@pytest.mark.parametrize("old,new", [
    # viscosities of the two phases swapped
    ("double nu = nu_v + phi * (nu_l - nu_v);", "double nu = nu_l + phi * (nu_v - nu_l);"),
    # the phase fraction not clamped at 1
    ("if (phi > 1.0) phi = 1.0;", ""),
], ids=["nu_swapped", "clamp_removed"])
def test_shear_wave_pin_catches_planted_mistakes(orc, tmp_path, monkeypatch, old, new):
    _use_c_library(monkeypatch, _mutant_c_library(tmp_path, old, new))
    assert worst_viscosity_error() > 0.05


# ------------------------------------------------------------------------------------------
# wetting objective
# ------------------------------------------------------------------------------------------

def _objective_params():
    return oracle.make_params(synth.base_params(nx=37, ny=24))


def _vapour(q):
    rho = np.full((q.ny, q.nx), q.rho_v)
    rho[0, :] = rho[-1, :] = 0.0
    return rho


def objective_errors(loss) -> float:
    """Largest deviation of (y_c, l_w) from their closed forms over slabs and single nodes."""
    q = _objective_params()
    err = 0.0
    for k in (1, 2, 5, 11):  # liquid slab on rows 1..k: y_c = k/2, l_w = nx
        rho = _vapour(q)
        rho[1:k + 1, :] = q.rho_l
        err = max(err, abs(loss(q, rho, 1.0, 0.0) - k / 2.0),
                  abs(loss(q, rho, 0.0, 1.0) - q.nx))
    for x, y in ((0, 1), (5, 2), (36, 7), (18, 22)):  # one liquid node: y_c = y - 1/2
        rho = _vapour(q)
        rho[y, x] = q.rho_l
        err = max(err, abs(loss(q, rho, 1.0, 0.0) - (y - 0.5)),
                  abs(loss(q, rho, 0.0, 1.0) - (1.0 if y == 1 else 0.0)))
    # partial phase fractions: phi = 1 at row 2 and 1/2 at row 5 of one column
    rho = _vapour(q)
    rho[2, 3] = q.rho_l
    rho[5, 3] = q.rho_v + 0.5 * (q.rho_l - q.rho_v)
    err = max(err, abs(loss(q, rho, 1.0, 0.0) - (1.5 + 0.5 * 4.5) / 1.5))
    return err


def test_objective_closed_forms(orc):
    assert objective_errors(oracle.loss) < 1e-12


@pytest.mark.parametrize("old,new", [
    ("[:, None] - 0.5", "[:, None] - 0.0"),  # wall plane at row 0 instead of y = 1/2
    ("phi[1, :]", "phi[2, :]"),  # wetted length on the wrong row
], ids=["wall_offset", "wet_row"])
def test_objective_pin_catches_planted_mistakes(orc, old, new):
    assert objective_errors(_mutant_function(oracle.loss, old, new)) > 0.4


# ------------------------------------------------------------------------------------------
# contact angle (Figs. 1-4): circles cutting the wall plane at a chosen angle
# ------------------------------------------------------------------------------------------

CAPS = ((30.0, 100.0), (60.0, 60.0), (90.0, 40.0), (120.0, 40.0), (150.0, 40.0))


def cap_density(q, theta_deg: float, r: float, y_wall: float, width: float = 4.0):
    """Liquid cap whose rho_mid contour is the circle of radius r centred at
    (nx/2, y_wall - r cos theta), which meets the wall plane y = y_wall at angle theta (measured
    through the liquid); tanh profile across the contour. One node of debris just below the
    fitted band (at y_wall + 2.5, density a tenth of the density range above rho_mid) must be
    ignored by the fit."""
    th = math.radians(theta_deg)
    yc = y_wall - r * math.cos(th)
    y, x = np.meshgrid(np.arange(q.ny, dtype=np.float64), np.arange(q.nx, dtype=np.float64),
                       indexing="ij")
    d = np.hypot(x - q.nx / 2.0, y - yc)
    mid, span = 0.5 * (q.rho_l + q.rho_v), q.rho_l - q.rho_v
    rho = mid - 0.5 * span * np.tanh(2.0 * (d - r) / width)
    rho[int(y_wall + 2.5), 20] = mid + 0.1 * span
    rho[0, :] = rho[-1, :] = 0.0
    return rho


def angle_errors(contact_angle) -> float:
    err = 0.0
    for walls in (1, 2):  # wall planes y = 0.5 (bounce-back) and y = 1 (wet-node)
        q = oracle.make_params(synth.base_params(nx=400, ny=160, walls=walls))
        yw = 0.5 if walls == 1 else 1.0
        for th, r in CAPS:
            got = contact_angle(q, cap_density(q, th, r, yw))[0]
            err = max(err, abs(got - th) if math.isfinite(got) else math.inf)
    return err


def test_contact_angle_of_circular_caps(orc):
    """theta within 0.1 degree for 30 ... 150 degrees on both wall planes."""
    assert angle_errors(oracle.contact_angle) < 0.1


def test_contact_angle_pin_catches_wall_plane_at_zero(orc, monkeypatch):
    monkeypatch.setattr(oracle, "wall_plane", lambda q: 0.0)
    assert angle_errors(oracle.contact_angle) > 0.4


@pytest.mark.parametrize("old,new", [
    ("yb + 3.0", "yb + 2.0"),  # fitted band starts one node too close to the wall
    ("(yb - yc) / r", "(yc - yb) / r"),  # sign of the cosine
], ids=["band", "sign"])
def test_contact_angle_pin_catches_planted_mistakes(orc, old, new):
    assert angle_errors(_mutant_function(oracle.contact_angle, old, new)) > 0.4
