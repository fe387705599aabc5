"""Python binding of liblbm (argument marshalling only: every step of the path runs in the HIP
kernels of the library; torch supplies device memory and the stream).

The library must be built (``python -m paper_1410_2569_amd.build``); importing fails loudly when
it is missing, and there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

ABI_VERSION = 1
OK, E_INVAL, E_SIZE, E_HIP, E_NONFINITE, E_ABI, E_STATE = 0, -1, -2, -3, -4, -5, -6
WALL = {"rho": 0, "psi": 1, "modpsi": 2}
EOS = {"cs": 0, "piecewise": 1}
WALLS = {"periodic": 0, "bounce_back": 1, "wet_node": 2, "mask": 3}
SCHEDULE = {"fused": 0, "two_pass": 1, "two_step": 2}


class LBMError(RuntimeError):
    def __init__(self, code: int, msg: str = ""):
        self.code = code
        super().__init__(f"liblbm error {code}: {msg}")


class Params(C.Structure):
    _fields_ = [("abi_version", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
                ("walls", C.c_int32), ("ghost_psi", C.c_int32), ("eos", C.c_int32),
                ("wall_force", C.c_int32), ("reserved", C.c_int32),
                ("a", C.c_double), ("b", C.c_double), ("R", C.c_double), ("T", C.c_double),
                ("rho1", C.c_double), ("rho2", C.c_double), ("th_v", C.c_double),
                ("th_m", C.c_double), ("th_l", C.c_double),
                ("G", C.c_double), ("sigma", C.c_double),
                ("s_rho", C.c_double), ("s_e", C.c_double), ("s_zeta", C.c_double),
                ("s_j", C.c_double), ("s_q", C.c_double),
                ("tau_l", C.c_double), ("tau_v", C.c_double),
                ("rho_l", C.c_double), ("rho_v", C.c_double)]


class Tune(C.Structure):
    _fields_ = [("tile", C.c_int32), ("reserved", C.c_int32), ("waves_per_cu", C.c_int32),
                ("schedule", C.c_int32)]

    def as_dict(self) -> dict:
        return {"tile": self.tile, "waves_per_cu": self.waves_per_cu, "schedule": self.schedule}


class Droplets(C.Structure):
    _fields_ = [("count", C.c_int32), ("reserved", C.c_int32),
                ("x0", C.c_double * 64), ("y0", C.c_double * 64), ("radius", C.c_double * 64),
                ("width", C.c_double), ("jitter", C.c_double), ("seed", C.c_uint64)]


def make_droplets(centres, radii, width=2.0, jitter=1e-3, seed=1) -> Droplets:
    """lbm_droplets for lbm_create_droplets: centres [(x0, y0), ...] and radii in lattice units."""
    d = Droplets()
    assert 1 <= len(centres) == len(radii) <= 64
    d.count = len(centres)
    for k, ((x0, y0), r) in enumerate(zip(centres, radii)):
        d.x0[k], d.y0[k], d.radius[k] = float(x0), float(y0), float(r)
    d.width, d.jitter, d.seed = float(width), float(jitter), int(seed) & 0xFFFFFFFFFFFFFFFF
    return d


class Obs(C.Structure):
    _fields_ = [("step", C.c_int64), ("rho_min", C.c_double), ("rho_max", C.c_double),
                ("umax", C.c_double), ("umax_liquid", C.c_double), ("mass", C.c_double),
                ("theta_deg", C.c_double), ("xc", C.c_double), ("yc", C.c_double),
                ("r", C.c_double), ("n_fit", C.c_int32), ("nonfinite", C.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


# name -> (restype, argtypes); the exported C ABI of include/lbm.h
_dp = C.POINTER(C.c_double)
_P = C.POINTER(Params)
SIGNATURES = {
    "lbm_maxwell_cs": (C.c_int, [C.c_double, C.c_double, C.c_double, C.c_double, _dp, _dp, _dp]),
    "lbm_cs_temperature": (C.c_int, [C.c_double, C.c_double, C.c_double, C.c_double, _dp]),
    "lbm_piecewise_spinodals": (C.c_int, [C.c_double] * 5 + [_dp, _dp]),
    "lbm_pressure": (C.c_int, [_P, C.c_double, _dp]),
    "lbm_workspace_size": (C.c_int, [_P, C.POINTER(C.c_size_t)]),
    "lbm_create": (C.c_int, [_P, _dp, _dp, C.c_void_p, C.c_size_t, C.c_void_p,
                             C.POINTER(C.c_void_p)]),
    "lbm_step": (C.c_int, [C.c_void_p, C.c_int64]),
    "lbm_observables": (C.c_int, [C.c_void_p, C.POINTER(Obs)]),
    "lbm_observables_window": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.POINTER(Obs)]),
    "lbm_observables_plane": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_double,
                                        C.POINTER(Obs)]),
    "lbm_observables_of_state": (C.c_int, [_P, C.c_void_p, C.c_void_p, C.c_void_p,
                                           C.POINTER(Obs)]),
    "lbm_record_contact_line": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.c_int32,
                                          C.c_void_p, C.c_size_t]),
    "lbm_batch_create_masked": (C.c_int, [_P, C.c_int32, C.POINTER(C.c_void_p), C.POINTER(_dp),
                                          C.POINTER(_dp), C.c_void_p, C.c_void_p, C.c_size_t,
                                          C.c_void_p, C.POINTER(C.c_void_p)]),
    "lbm_batch_observables_plane": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_void_p]),
    "lbm_batch_record_contact_line": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32,
                                                C.POINTER(C.c_int32), C.c_void_p, C.c_size_t]),
    "lbm_create_masked": (C.c_int, [_P, C.c_void_p, _dp, _dp, C.c_void_p, C.c_size_t, C.c_void_p,
                                    C.POINTER(C.c_void_p)]),
    "lbm_create_droplets": (C.c_int, [_P, _dp, C.POINTER(Droplets), C.c_void_p, C.c_size_t,
                                      C.c_void_p, C.POINTER(C.c_void_p)]),
    "lbm_read_rho": (C.c_int, [C.c_void_p, _dp, C.c_size_t]),
    "lbm_read_f": (C.c_int, [C.c_void_p, _dp, C.c_size_t]),
    "lbm_state_size": (C.c_int, [C.c_void_p, C.POINTER(C.c_size_t)]),
    "lbm_save_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "lbm_load_state": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "lbm_set_gw": (C.c_int, [C.c_void_p, _dp]),
    "lbm_set_schedule": (C.c_int, [C.c_void_p, C.c_int32]),
    "lbm_current_step": (C.c_int64, [C.c_void_p]),
    "lbm_adjoint_workspace_size": (C.c_int, [_P, C.c_int64, C.c_int32, C.POINTER(C.c_size_t)]),
    "lbm_forward_ckpt": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_size_t]),
    "lbm_loss": (C.c_int, [C.c_void_p, C.c_double, C.c_double, _dp]),
    "lbm_backward": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_size_t,
                               C.c_double, C.c_double, C.c_void_p]),
    "lbm_batch_workspace_size": (C.c_int, [_P, C.c_int32, C.c_void_p, C.POINTER(C.c_size_t)]),
    "lbm_batch_create": (C.c_int, [_P, C.c_int32, C.POINTER(_dp), C.POINTER(_dp), C.c_void_p,
                                   C.c_void_p, C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]),
    "lbm_batch_step": (C.c_int, [C.c_void_p, C.c_int64]),
    "lbm_batch_observables": (C.c_int, [C.c_void_p, C.c_void_p]),
    "lbm_batch_adjoint_workspace_size": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32,
                                                   C.POINTER(C.c_size_t)]),
    "lbm_batch_forward_ckpt": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.c_void_p,
                                         C.c_size_t]),
    "lbm_batch_loss": (C.c_int, [C.c_void_p, C.c_double, C.c_double, _dp]),
    "lbm_batch_backward": (C.c_int, [C.c_void_p, C.c_int64, C.c_int32, C.c_void_p, C.c_size_t,
                                     C.c_double, C.c_double, C.c_void_p]),
    "lbm_batch_read_f": (C.c_int, [C.c_void_p, C.c_int32, _dp, C.c_size_t]),
    "lbm_batch_save_state": (C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_size_t]),
    "lbm_batch_current_step": (C.c_int64, [C.c_void_p]),
    "lbm_batch_get_tune": (C.c_int, [C.c_void_p, C.c_void_p, C.POINTER(C.c_int32)]),
    "lbm_batch_destroy": (C.c_int, [C.c_void_p]),
    "lbm_batch_last_error": (C.c_char_p, [C.c_void_p]),
    "lbm_autotune": (C.c_int, [_P, C.c_int32, C.POINTER(_dp), C.POINTER(_dp), C.c_void_p,
                               C.c_size_t, C.c_void_p, C.c_int32, C.c_void_p,
                               C.POINTER(C.c_double)]),
    "lbm_fp64_probe": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t,
                                 C.c_void_p]),
    "lbm_destroy": (C.c_int, [C.c_void_p]),
    "lbm_strerror": (C.c_char_p, [C.c_int]),
    "lbm_last_error": (C.c_char_p, [C.c_void_p]),
}

_lib = None


def lib() -> C.CDLL:
    """Load liblbm.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_1410_2569_amd.build`")
        # torch ships its own HIP runtime under the same soname as the system one liblbm.so was
        # linked against; loading torch first makes both use torch's (loading liblbm.so first
        # would bind torch to the system runtime, which then finds no device)
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _dptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def check(rc: int, ctx=None):
    """Raise LBMError for a failed call; the message adds the context's last error, or (without a
    context) the reason of the last failed creation on this thread."""
    if rc != OK:
        msg = lib().lbm_strerror(rc).decode()
        extra = lib().lbm_last_error(ctx)
        if extra:
            msg += ": " + extra.decode()
        raise LBMError(rc, msg)


def maxwell_cs(a: float, b: float, R: float, T: float):
    """(rho_v, rho_l, p0) of the Carnahan-Starling Maxwell construction (library's solver)."""
    rv, rl, p0 = C.c_double(), C.c_double(), C.c_double()
    check(lib().lbm_maxwell_cs(a, b, R, T, C.byref(rv), C.byref(rl), C.byref(p0)))
    return rv.value, rl.value, p0.value


def cs_temperature(a: float, b: float, R: float, ratio: float) -> float:
    T = C.c_double()
    check(lib().lbm_cs_temperature(a, b, R, ratio, C.byref(T)))
    return T.value


def piecewise_spinodals(rho_v: float, rho_l: float, th_v: float, th_m: float, th_l: float):
    """(rho1, rho2) of Eq. (15) for coexistence densities (rho_v, rho_l) (library's solver)."""
    r1, r2 = C.c_double(), C.c_double()
    check(lib().lbm_piecewise_spinodals(rho_v, rho_l, th_v, th_m, th_l, C.byref(r1),
                                        C.byref(r2)))
    return r1.value, r2.value


def pressure(q, rho: float) -> float:
    """p_EOS(rho) of parameter block q (library's host EOS)."""
    q = q if isinstance(q, Params) else make_params(q)
    out = C.c_double()
    check(lib().lbm_pressure(C.byref(q), float(rho), C.byref(out)))
    return out.value


def make_params(p: dict) -> Params:
    """C parameter block from a parameter dict (keys as in synth.base_params). rho_l/rho_v
    default to the library's own Maxwell construction for the Carnahan-Starling EOS; rho1/rho2
    of Eq. (15) to the library's spinodal solver. walls: 0 periodic, 1 bounce-back, 2 wet-node
    (or the names in WALLS)."""
    q = Params()
    q.abi_version = ABI_VERSION
    q.nx, q.ny = int(p["nx"]), int(p["ny"])
    w = p.get("walls", 1)
    q.walls = WALLS[w] if isinstance(w, str) else int(w)
    q.ghost_psi = int(p.get("ghost", 1))
    q.eos = EOS[p.get("eos", "cs")]
    q.wall_force = WALL[p.get("wall_force", "psi")]
    for k in ("a", "b", "R", "T", "rho1", "rho2", "th_v", "th_m", "th_l"):
        setattr(q, k, float(p.get(k, 0.0)))
    if q.eos == EOS["piecewise"] and "rho1" not in p:
        q.rho1, q.rho2 = piecewise_spinodals(float(p["rho_v"]), float(p["rho_l"]), q.th_v,
                                             q.th_m, q.th_l)
    q.G = float(p.get("G", -1.0))
    q.sigma = float(p["sigma"])
    for k in ("s_rho", "s_e", "s_zeta", "s_j", "s_q", "tau_l", "tau_v"):
        setattr(q, k, float(p[k]))
    if "rho_l" in p and "rho_v" in p:
        q.rho_l, q.rho_v = float(p["rho_l"]), float(p["rho_v"])
    elif q.eos == EOS["cs"]:
        q.rho_v, q.rho_l, _ = maxwell_cs(q.a, q.b, q.R, q.T)
    else:
        raise ValueError("piecewise EOS needs rho_l and rho_v")
    return q


def _use_on(t, stream):
    """Make a freshly allocated tensor t safe to use on `stream`: torch's caching allocator hands
    out a block that is free only with respect to the current stream, so `stream` first waits for
    the current stream; record_stream keeps the block from being reused until the work queued on
    `stream` has finished."""
    import torch

    cur = torch.cuda.current_stream(t.device)
    if stream.cuda_stream != cur.cuda_stream:
        stream.wait_stream(cur)
        t.record_stream(stream)
    return t


def _done_on(t, stream):
    """Hand a tensor written by work queued on `stream` back to the caller: the current stream
    waits for `stream`, so torch work queued after this call (a copy to the host, arithmetic)
    reads the finished values."""
    import torch

    cur = torch.cuda.current_stream(t.device)
    if stream.cuda_stream != cur.cuda_stream:
        cur.wait_stream(stream)
    return t


def fp64_probe(a, b, stream=None):
    """sqrt(a) and a / b computed by the library's device code (contiguous float64 device
    tensors of one shape); returns the two result tensors."""
    import torch

    assert a.is_cuda and a.dtype == torch.float64 and a.is_contiguous() and a.shape == b.shape
    assert b.is_cuda and b.dtype == torch.float64 and b.is_contiguous()
    st = stream if stream is not None else torch.cuda.current_stream(a.device)
    sq, qt = torch.empty_like(a), torch.empty_like(a)
    check(lib().lbm_fp64_probe(C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()),
                               C.c_void_p(sq.data_ptr()), C.c_void_p(qt.data_ptr()), a.numel(),
                               C.c_void_p(st.cuda_stream)))
    return sq, qt


def workspace_size(q: Params) -> int:
    n = C.c_size_t()
    check(lib().lbm_workspace_size(C.byref(q), C.byref(n)))
    return n.value


def observables_of_state(params, f, gw=None, stream=None, allow_nonfinite=False) -> dict:
    """Observables of pre-collision populations the caller holds on the device: f a contiguous
    float64 tensor of shape (9, ny, nx) (the layout of Sim.f()), gw (2, nx) on the same device or
    None with periodic y. Runs the library's allocation-free entry point (its scratch is a fixed
    device array of the library)."""
    import torch

    q = params if isinstance(params, Params) else make_params(params)
    assert f.is_cuda and f.dtype == torch.float64 and f.is_contiguous()
    assert tuple(f.shape) == (9, q.ny, q.nx)
    if gw is not None:
        assert gw.is_cuda and gw.dtype == torch.float64 and gw.is_contiguous()
        assert tuple(gw.shape) == (2, q.nx) and gw.device == f.device
    st = stream if stream is not None else torch.cuda.current_stream(f.device)
    o = Obs()
    rc = lib().lbm_observables_of_state(C.byref(q), C.c_void_p(f.data_ptr()),
                                        C.c_void_p(gw.data_ptr() if gw is not None else 0),
                                        C.c_void_p(st.cuda_stream), C.byref(o))
    if not (rc == E_NONFINITE and allow_nonfinite):
        check(rc)
    return o.as_dict()


class Sim:
    """One lattice on the current HIP device, in a torch-allocated workspace. rho0: the initial
    density, shape (ny, nx), or a Droplets description (make_droplets) whose density the library
    generates on the device. With walls = 3 ("mask") pass the solid mask ((ny, nx), nonzero =
    solid) as `solid` (or under params["solid"]) and G_w per node, shape (ny, nx)."""

    def __init__(self, params, gw, rho0, device="cuda", stream=None, solid=None):
        import torch

        if solid is None and isinstance(params, dict):
            solid = params.get("solid")
        self.q = params if isinstance(params, Params) else make_params(params)
        self.nx, self.ny = self.q.nx, self.q.ny
        self.masked = self.q.walls == WALLS["mask"]
        nbytes = workspace_size(self.q)
        # 256-byte aligned: torch's caching allocator hands out 512-byte aligned blocks
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.ws.device)
        _use_on(self.ws, self.stream)
        gshape = (self.ny, self.nx) if self.masked else (2, self.nx)
        g = np.ascontiguousarray(gw if gw is not None else np.zeros(gshape), dtype=np.float64)
        assert g.shape == gshape
        h = C.c_void_p()
        ws, st = C.c_void_p(self.ws.data_ptr()), C.c_void_p(self.stream.cuda_stream)
        if isinstance(rho0, Droplets):  # initial density generated on the device
            check(lib().lbm_create_droplets(C.byref(self.q), _dptr(g), C.byref(rho0), ws, nbytes,
                                            st, C.byref(h)))
            self.h = h
            return
        r = np.ascontiguousarray(rho0, dtype=np.float64)
        assert r.shape == (self.ny, self.nx)
        if self.masked:
            m = np.ascontiguousarray(np.asarray(solid) != 0, dtype=np.uint8)
            assert m.shape == (self.ny, self.nx)
            check(lib().lbm_create_masked(C.byref(self.q), m.ctypes.data_as(C.c_void_p),
                                          _dptr(g), _dptr(r), ws, nbytes, st, C.byref(h)))
        else:
            check(lib().lbm_create(C.byref(self.q), _dptr(g), _dptr(r), ws, nbytes, st,
                                   C.byref(h)))
        self.h = h

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            lib().lbm_destroy(h)
            self.h = None

    def _chk(self, rc):
        check(rc, self.h)

    def set_schedule(self, schedule):
        s = SCHEDULE[schedule] if isinstance(schedule, str) else int(schedule)
        self._chk(lib().lbm_set_schedule(self.h, s))

    def step(self, n: int = 1):
        self._chk(lib().lbm_step(self.h, int(n)))

    @property
    def current_step(self) -> int:
        return lib().lbm_current_step(self.h)

    def observables(self, x_lo=-math.inf, x_hi=math.inf, allow_nonfinite=False,
                    y_wall=None) -> dict:
        """Observables; y_wall: contact plane of the angle fit (default: the wall plane)."""
        o = Obs()
        if y_wall is None:
            rc = lib().lbm_observables_window(self.h, x_lo, x_hi, C.byref(o))
        else:
            rc = lib().lbm_observables_plane(self.h, x_lo, x_hi, float(y_wall), C.byref(o))
        if rc == E_NONFINITE and allow_nonfinite:
            return o.as_dict()
        self._chk(rc)
        return o.as_dict()

    def record_contact_line(self, n: int, every: int, row: int = 1, out=None):
        """Advance n steps recording the contact line on `row` every `every` steps (device-side;
        no host synchronisation). Returns a (n/every + 1, 2) float64 device tensor of
        (left, right) crossings, filled asynchronously on the context stream (the current stream
        is made to wait for it)."""
        import torch
        k = n // every + 1
        if out is None:
            out = _use_on(torch.empty((k, 2), dtype=torch.float64, device=self.ws.device),
                          self.stream)
        assert out.is_contiguous() and out.dtype == torch.float64
        self._chk(lib().lbm_record_contact_line(self.h, int(n), int(every), int(row),
                                                C.c_void_p(out.data_ptr()), out.numel()))
        return _done_on(out, self.stream)

    def rho(self) -> np.ndarray:
        out = np.empty((self.ny, self.nx))
        self._chk(lib().lbm_read_rho(self.h, _dptr(out), out.size))
        return out

    def f(self) -> np.ndarray:
        out = np.empty((9, self.ny, self.nx))
        self._chk(lib().lbm_read_f(self.h, _dptr(out), out.size))
        return out

    def save_state(self) -> bytes:
        n = C.c_size_t()
        self._chk(lib().lbm_state_size(self.h, C.byref(n)))
        buf = C.create_string_buffer(n.value)
        self._chk(lib().lbm_save_state(self.h, buf, n.value))
        return buf.raw

    def load_state(self, blob: bytes):
        self._chk(lib().lbm_load_state(self.h, C.c_char_p(blob), len(blob)))

    def set_gw(self, gw):
        g = np.ascontiguousarray(gw, dtype=np.float64)
        assert g.shape == ((self.ny, self.nx) if self.masked else (2, self.nx))
        self._chk(lib().lbm_set_gw(self.h, _dptr(g)))

    # ---- adjoint -----------------------------------------------------------------------------
    def adjoint_workspace(self, nsteps: int, K: int):
        """A device workspace (torch uint8 tensor) for lbm_forward_ckpt / lbm_backward."""
        import torch
        n = C.c_size_t()
        check(lib().lbm_adjoint_workspace_size(C.byref(self.q), int(nsteps), int(K), C.byref(n)))
        return _use_on(torch.empty(n.value, dtype=torch.uint8, device=self.ws.device),
                       self.stream)

    def forward_ckpt(self, nsteps: int, K: int, ws):
        self._chk(lib().lbm_forward_ckpt(self.h, int(nsteps), int(K), C.c_void_p(ws.data_ptr()),
                                         ws.numel()))

    def loss(self, w_centroid: float = 1.0, w_wet: float = 1.0) -> float:
        L = C.c_double()
        self._chk(lib().lbm_loss(self.h, w_centroid, w_wet, C.byref(L)))
        return L.value

    def backward(self, nsteps: int, K: int, ws, w_centroid: float = 1.0, w_wet: float = 1.0):
        """dL/dG_w as a (2, nx) float64 device tensor (row 0 bottom wall, row 1 top wall)."""
        import torch
        g = _use_on(torch.empty((2, self.nx), dtype=torch.float64, device=self.ws.device),
                    self.stream)
        self._chk(lib().lbm_backward(self.h, int(nsteps), int(K), C.c_void_p(ws.data_ptr()),
                                     ws.numel(), w_centroid, w_wet, C.c_void_p(g.data_ptr())))
        return _done_on(g, self.stream)


class Batch:
    """An ensemble of uneven lattices advanced together by the batch kernels. An ensemble of solid
    masks (walls = 3 for every instance) takes the masks as `solids` (or params["solid"]) and G_w
    per node."""

    def __init__(self, params_list, gw_list, rho0_list, tune=None, device="cuda", stream=None,
                 solids=None):
        import torch

        self.n = len(params_list)
        if solids is None and all(isinstance(pr, dict) and "solid" in pr for pr in params_list):
            solids = [pr["solid"] for pr in params_list]
        arr = (Params * self.n)()
        for i, pr in enumerate(params_list):
            arr[i] = pr if isinstance(pr, Params) else make_params(pr)
        self.params = arr
        self.masked = solids is not None
        shape = (lambda q: (q.ny, q.nx)) if self.masked else (lambda q: (2, q.nx))
        self._gw = [np.ascontiguousarray(g if g is not None else np.zeros(shape(arr[i])),
                                         dtype=np.float64) for i, g in enumerate(gw_list)]
        self._rho = [np.ascontiguousarray(r, dtype=np.float64) for r in rho0_list]
        for i in range(self.n):
            assert self._gw[i].shape == shape(arr[i])
            assert self._rho[i].shape == (arr[i].ny, arr[i].nx)
        if self.masked:
            self._solid = [np.ascontiguousarray(np.asarray(m) != 0, dtype=np.uint8) for m in solids]
            sp = (C.c_void_p * self.n)(*[m.ctypes.data for m in self._solid])
        gwp = (_dp * self.n)(*[_dptr(g) for g in self._gw])
        rp = (_dp * self.n)(*[_dptr(r) for r in self._rho])
        t = None
        if tune is not None:
            t = tune if isinstance(tune, Tune) else Tune(int(tune.get("tile", 1)), 0,
                                                          int(tune.get("waves_per_cu", 0)),
                                                          int(tune.get("schedule", 0)))
        tp = C.byref(t) if t is not None else None
        nbytes = C.c_size_t()
        check(lib().lbm_batch_workspace_size(arr, self.n, tp, C.byref(nbytes)))
        self.ws = torch.empty(nbytes.value, dtype=torch.uint8, device=device)
        # a stream of its own (default priority): the legacy default stream cannot be captured
        # into the hipGraphs the ensemble replays
        self.stream = stream if stream is not None else torch.cuda.Stream(self.ws.device)
        _use_on(self.ws, self.stream)
        h = C.c_void_p()
        ws, st = C.c_void_p(self.ws.data_ptr()), C.c_void_p(self.stream.cuda_stream)
        if self.masked:
            rc = lib().lbm_batch_create_masked(arr, self.n, sp, gwp, rp, tp, ws, nbytes.value, st,
                                               C.byref(h))
        else:
            rc = lib().lbm_batch_create(arr, self.n, gwp, rp, tp, ws, nbytes.value, st,
                                        C.byref(h))
        check(rc)
        self.h = h

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            lib().lbm_batch_destroy(h)
            self.h = None

    def _chk(self, rc):
        if rc != OK:
            msg = lib().lbm_strerror(rc).decode()
            extra = lib().lbm_batch_last_error(self.h)
            raise LBMError(rc, msg + (": " + extra.decode() if extra else ""))

    def step(self, n: int = 1):
        self._chk(lib().lbm_batch_step(self.h, int(n)))

    @property
    def current_step(self) -> int:
        return lib().lbm_batch_current_step(self.h)

    def tune(self):
        t, g = Tune(), C.c_int32()
        self._chk(lib().lbm_batch_get_tune(self.h, C.byref(t), C.byref(g)))
        return dict(t.as_dict(), grid=g.value)

    def observables(self, allow_nonfinite=False, y_wall=None) -> list:
        """Observables of every instance; y_wall: contact plane per instance (default planes)."""
        out = (Obs * self.n)()
        if y_wall is None:
            rc = lib().lbm_batch_observables(self.h, out)
        else:
            yw = (C.c_double * self.n)(*[float(v) for v in y_wall])
            rc = lib().lbm_batch_observables_plane(self.h, yw, out)
        if not (rc == E_NONFINITE and allow_nonfinite):
            self._chk(rc)
        return [o.as_dict() for o in out]

    def record_contact_line(self, n: int, every: int, rows, out=None):
        """Advance n steps recording every instance's contact line on rows[i] every `every`
        steps (device-side). Returns a (n/every + 1, count, 2) float64 device tensor."""
        import torch
        k = n // every + 1
        if out is None:
            out = _use_on(torch.empty((k, self.n, 2), dtype=torch.float64, device=self.ws.device),
                          self.stream)
        assert out.is_contiguous() and out.dtype == torch.float64
        rw = (C.c_int32 * self.n)(*[int(r) for r in rows])
        self._chk(lib().lbm_batch_record_contact_line(self.h, int(n), int(every), rw,
                                                      C.c_void_p(out.data_ptr()), out.numel()))
        return _done_on(out, self.stream)

    # ---- adjoint of every instance ---------------------------------------------------------------
    def adjoint_workspace(self, nsteps: int, K: int):
        """A device workspace (torch uint8 tensor) for forward_ckpt / backward of the ensemble."""
        import torch
        n = C.c_size_t()
        self._chk(lib().lbm_batch_adjoint_workspace_size(self.h, int(nsteps), int(K), C.byref(n)))
        return _use_on(torch.empty(n.value, dtype=torch.uint8, device=self.ws.device), self.stream)

    def forward_ckpt(self, nsteps: int, K: int, ws):
        self._chk(lib().lbm_batch_forward_ckpt(self.h, int(nsteps), int(K),
                                               C.c_void_p(ws.data_ptr()), ws.numel()))

    def loss(self, w_centroid: float = 1.0, w_wet: float = 1.0) -> list:
        L = (C.c_double * self.n)()
        self._chk(lib().lbm_batch_loss(self.h, w_centroid, w_wet, L))
        return list(L)

    def backward(self, nsteps: int, K: int, ws, w_centroid: float = 1.0, w_wet: float = 1.0):
        """dL/dG_w of every instance: a list of (2, nx_i) float64 device tensors (views of one
        buffer), row 0 bottom wall, row 1 top wall."""
        import torch
        sizes = [2 * q.nx for q in self.params]
        g = _use_on(torch.empty(sum(sizes), dtype=torch.float64, device=self.ws.device),
                    self.stream)
        self._chk(lib().lbm_batch_backward(self.h, int(nsteps), int(K), C.c_void_p(ws.data_ptr()),
                                           ws.numel(), w_centroid, w_wet,
                                           C.c_void_p(g.data_ptr())))
        _done_on(g, self.stream)
        out, o = [], 0
        for q, n in zip(self.params, sizes):
            out.append(g[o:o + n].view(2, q.nx))
            o += n
        return out

    def save_state(self, index: int) -> bytes:
        """Checkpoint blob of one instance, loadable by Sim.load_state."""
        q = self.params[index]
        n = 32 + 9 * q.nx * q.ny * 8
        buf = C.create_string_buffer(n)
        self._chk(lib().lbm_batch_save_state(self.h, int(index), buf, n))
        return buf.raw

    def f(self, index: int) -> np.ndarray:
        q = self.params[index]
        out = np.empty((9, q.ny, q.nx))
        self._chk(lib().lbm_batch_read_f(self.h, int(index), _dptr(out), out.size))
        return out


def autotune(params_list, gw_list, rho0_list, steps=200, device="cuda"):
    """Fastest lbm_tune for this ensemble (every tile shape x schedule timed on the device)."""
    import torch

    n = len(params_list)
    arr = (Params * n)()
    for i, pr in enumerate(params_list):
        arr[i] = pr if isinstance(pr, Params) else make_params(pr)
    gws = [np.ascontiguousarray(g, dtype=np.float64) for g in gw_list]
    rhos = [np.ascontiguousarray(r, dtype=np.float64) for r in rho0_list]
    gwp = (_dp * n)(*[_dptr(g) for g in gws])
    rp = (_dp * n)(*[_dptr(r) for r in rhos])
    need = 0
    for tile in range(5):
        b = C.c_size_t()
        t = Tune(tile, 0, 0, 0)
        check(lib().lbm_batch_workspace_size(arr, n, C.byref(t), C.byref(b)))
        need = max(need, b.value)
    ws = torch.empty(need, dtype=torch.uint8, device=device)
    best, ms = Tune(), C.c_double()
    stream = torch.cuda.Stream(ws.device)  # capturable (see Batch)
    _use_on(ws, stream)
    check(lib().lbm_autotune(arr, n, gwp, rp, C.c_void_p(ws.data_ptr()), need,
                             C.c_void_p(stream.cuda_stream), int(steps), C.byref(best),
                             C.byref(ms)))
    return dict(best.as_dict(), ms=ms.value, steps=steps)
