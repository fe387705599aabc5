"""C ABI of liblbm without a GPU: every declared symbol is exported, parameter validation runs
before any HIP call, and the host-side thermodynamics agree with the oracle."""
import ctypes as C
import math
import os
import re
import subprocess

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


@pytest.fixture(scope="module")
def L():
    import paper_1410_2569_amd as L
    return L


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", src)))


def test_every_declared_symbol_is_exported(L):
    lib = L.lib()
    names = declared_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, f"declared but not exported: {missing}"
    # the binding knows every entry point's signature
    assert set(names) <= set(L.lbm.SIGNATURES), set(names) - set(L.lbm.SIGNATURES)
    out = subprocess.run(["nm", "-D", "--defined-only", L.lbm.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r"\b(lbm_[a-z_0-9]+)\b", out))
    assert set(names) <= exported


def test_struct_layout_matches_header(L):
    # 8 int32 then 20 doubles
    assert C.sizeof(L.Params) == 8 * 4 + 20 * 8
    assert C.sizeof(L.Obs) == 8 + 9 * 8 + 2 * 4


def good_params(L, **over):
    p = synth.base_params(nx=64, ny=32)
    p.update(over)
    return L.make_params(p)


def test_workspace_size_scales(L):
    a = L.workspace_size(good_params(L, nx=64, ny=32))
    b = L.workspace_size(good_params(L, nx=1024, ny=512))
    # two population buffers of 9 planes dominate
    assert b > 2 * 9 * 1024 * 512 * 8 and a < b


@pytest.mark.parametrize("field,value,code", [
    ("abi_version", 99, -5), ("nx", 2, -1), ("ny", 3, -1), ("walls", 3, -1), ("walls", -1, -1),
    ("ghost_psi", 7, -1), ("eos", 5, -1), ("wall_force", 3, -1), ("reserved", 1, -1),
    ("G", 1.0, -1), ("G", float("nan"), -1), ("sigma", float("inf"), -1),
    ("s_e", 0.0, -1), ("s_q", 2.0, -1), ("tau_l", 0.5, -1), ("tau_v", 0.4, -1),
    ("rho_v", 0.0, -1), ("rho_l", 1e-5, -1), ("T", -1.0, -1),
])
def test_invalid_parameters_rejected_without_gpu(L, field, value, code):
    q = good_params(L)
    setattr(q, field, value)
    n = C.c_size_t()
    assert L.lib().lbm_workspace_size(C.byref(q), C.byref(n)) == code
    h = C.c_void_p()
    rho0 = np.full((q.ny, q.nx), 0.3); gw = np.zeros((2, q.nx))
    dp = C.POINTER(C.c_double)
    rc = L.lib().lbm_create(C.byref(q), gw.ctypes.data_as(dp), rho0.ctypes.data_as(dp),
                            C.c_void_p(256), 1 << 40, None, C.byref(h))
    assert rc == code and not h.value


def test_wet_node_accepted_but_not_for_the_adjoint(L):
    """walls = 2 (wet-node scheme) is a valid geometry; the objective and adjoint support
    bounce-back walls only and say so before any GPU call."""
    q = good_params(L, walls=2)
    n = C.c_size_t()
    assert L.lib().lbm_workspace_size(C.byref(q), C.byref(n)) == 0
    assert L.lib().lbm_adjoint_workspace_size(C.byref(q), 100, 10, C.byref(n)) == -1
    q = good_params(L, walls=1)
    assert L.lib().lbm_adjoint_workspace_size(C.byref(q), 100, 10, C.byref(n)) == 0


def test_create_rejects_bad_buffers_without_gpu(L):
    q = good_params(L)
    need = L.workspace_size(q)
    dp = C.POINTER(C.c_double)
    rho0 = np.full((q.ny, q.nx), 0.3); gw = np.zeros((2, q.nx))
    h = C.c_void_p()
    lib = L.lib()
    # workspace too small
    assert lib.lbm_create(C.byref(q), gw.ctypes.data_as(dp), rho0.ctypes.data_as(dp),
                          C.c_void_p(256), need - 1, None, C.byref(h)) == -2
    # misaligned workspace, missing arrays
    assert lib.lbm_create(C.byref(q), gw.ctypes.data_as(dp), rho0.ctypes.data_as(dp),
                          C.c_void_p(8), need, None, C.byref(h)) == -1
    assert lib.lbm_create(C.byref(q), None, rho0.ctypes.data_as(dp), C.c_void_p(256), need,
                          None, C.byref(h)) == -1
    assert lib.lbm_create(C.byref(q), gw.ctypes.data_as(dp), None, C.c_void_p(256), need,
                          None, C.byref(h)) == -1
    # non-positive density in the fluid, non-finite G_w
    bad = rho0.copy(); bad[5, 5] = 0.0
    assert lib.lbm_create(C.byref(q), gw.ctypes.data_as(dp), bad.ctypes.data_as(dp),
                          C.c_void_p(256), need, None, C.byref(h)) == -1
    # a density outside the pseudopotential's domain (Carnahan-Starling: psi is real only below
    # about 0.593 at these constants)
    bad = rho0.copy(); bad[7, 9] = 0.7
    assert lib.lbm_create(C.byref(q), gw.ctypes.data_as(dp), bad.ctypes.data_as(dp),
                          C.c_void_p(256), need, None, C.byref(h)) == -1
    # droplets whose jitter would leave that domain, or an invalid description
    for kw in (dict(jitter=0.5), dict(width=-1.0), dict(radii=[0.0])):
        args = dict(centres=[(32.0, 0.5)], radii=[8.0], width=2.0, jitter=1e-3, seed=1)
        args.update(kw)
        d = L.make_droplets(**args)
        assert lib.lbm_create_droplets(C.byref(q), gw.ctypes.data_as(dp), C.byref(d),
                                       C.c_void_p(256), need, None, C.byref(h)) == -1, kw
    d = L.make_droplets([(32.0, 0.5)], [8.0])
    assert lib.lbm_create_droplets(C.byref(q), gw.ctypes.data_as(dp), C.byref(d),
                                   C.c_void_p(256), need - 1, None, C.byref(h)) == -2
    g2 = gw.copy(); g2[0, 3] = math.nan
    assert lib.lbm_create(C.byref(q), g2.ctypes.data_as(dp), rho0.ctypes.data_as(dp),
                          C.c_void_p(256), need, None, C.byref(h)) == -1
    # null handles
    assert lib.lbm_step(None, 1) == -1
    assert lib.lbm_observables(None, None) == -1
    assert lib.lbm_destroy(None) == -1
    assert lib.lbm_strerror(-4) == b"non-finite state"


def test_maxwell_matches_oracle(L, orc):
    """The library solves the equal-area rule with the closed-form antiderivative; the oracle with
    adaptive quadrature. They must agree."""
    for T in (0.024461878423483633, 0.03, 0.04):
        a = L.maxwell_cs(0.5, 4.0, 1.0, T)
        b = orc.maxwell_cs(0.5, 4.0, 1.0, T)
        assert np.allclose(a, b, rtol=1e-10, atol=0), (T, a, b)
    T_lib = L.cs_temperature(0.5, 4.0, 1.0, 500.0)
    T_orc = orc.cs_temperature_for_ratio(0.5, 4.0, 1.0, 500.0)
    assert abs(T_lib - T_orc) <= 1e-12 * T_orc
    # above the critical temperature there is no coexistence
    with pytest.raises(L.LBMError):
        L.maxwell_cs(0.5, 4.0, 1.0, 0.05)
