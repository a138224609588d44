"""ctypes binding of libpplbm.so (include/pplbm.h), same function names as the C ABI.

Argument marshalling only: every step of the method runs in the library's HIP kernels.
torch provides device memory and the stream (``Lattice``); nothing falls back to a CPU path
-- if the library is missing, importing this module fails loudly.
"""
from __future__ import annotations

import atexit
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpplbm.so")

LBM_OK, LBM_EINVAL, LBM_ENOMEM, LBM_EHIP, LBM_EUNSTABLE, LBM_ENOTCONVERGED, LBM_ESTATE = \
    0, -1, -2, -3, -4, -5, -6
LBM_EOS_CARNAHAN_STARLING, LBM_EOS_SBRAGAGLIA_SHAN = 0, 1
LBM_FORCE_EDM, LBM_FORCE_GUO, LBM_FORCE_GUO_LI, LBM_FORCE_SC = 0, 1, 2, 3
LBM_COEX_MAXWELL, LBM_COEX_MECHANICAL = 0, 1
LBM_COLL_BGK, LBM_COLL_MRT = 0, 1
LBM_PREC_F64, LBM_PREC_MIXED = 1, 2
LBM_LAYOUT_PLANES, LBM_LAYOUT_ROWS = 0, 1
LBM_KERNEL_TWO_PASS, LBM_KERNEL_SWEEP, LBM_KERNEL_SWEEP2 = 0, 1, 2
LBM_LAUNCH_NONTEMPORAL, LBM_LAUNCH_XCD_ORDER, LBM_LAUNCH_SHALLOW = 1, 2, 4
LBM_LAUNCH_SERIAL_KINDS = 8
LBM_LAUNCH_TWO_STEP = 16

SCHEMES = {"EDM": LBM_FORCE_EDM, "GUO": LBM_FORCE_GUO, "GUO_LI": LBM_FORCE_GUO_LI,
           "SC": LBM_FORCE_SC}
COLLISIONS = {"BGK": LBM_COLL_BGK, "MRT": LBM_COLL_MRT}


class lbm_eos(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("a", ctypes.c_double), ("b", ctypes.c_double),
                ("R", ctypes.c_double), ("T_over_Tc", ctypes.c_double), ("K", ctypes.c_double),
                ("eps", ctypes.c_double)]


class lbm_force(ctypes.Structure):
    _fields_ = [("scheme", ctypes.c_int), ("A", ctypes.c_double), ("sigma", ctypes.c_double),
                ("G", ctypes.c_double)]


class lbm_collision(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("s_rho", ctypes.c_double), ("s_e", ctypes.c_double),
                ("s_eps", ctypes.c_double), ("s_j", ctypes.c_double), ("s_q", ctypes.c_double)]


class lbm_stats_t(ctypes.Structure):
    _fields_ = [("mass", ctypes.c_double), ("rho_min", ctypes.c_double),
                ("rho_max", ctypes.c_double), ("rho_probe_a", ctypes.c_double),
                ("rho_probe_b", ctypes.c_double), ("ratio", ctypes.c_double),
                ("us_max", ctypes.c_double), ("dv_max", ctypes.c_double),
                ("step", ctypes.c_longlong), ("nonfinite", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# torch (the source of device memory and streams) must bring up the GPU before this library's
# HIP runtime does: a process where the library initialises HIP first cannot start torch's.
try:
    import torch as _torch
    _torch.cuda.is_available()
except ImportError:  # torch is optional for the C ABI itself
    pass

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1412_5170_amd.build` "
                      "(there is no CPU fallback)")
_lib = ctypes.CDLL(LIB_PATH)

# Objects still alive when the interpreter exits are not destroyed through the library: the
# module's globals and the HIP runtime may already be gone, and the process frees everything.
_LIVE = [True]
atexit.register(_LIVE.__setitem__, 0, False)

_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_SIG = {
    "lbm_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.POINTER(lbm_eos),
                                  ctypes.POINTER(lbm_force), ctypes.POINTER(lbm_collision),
                                  ctypes.c_double, ctypes.POINTER(_P)]),
    "lbm_destroy": (None, [_P]),
    "lbm_layout": (ctypes.c_int, [_P] + [ctypes.POINTER(ctypes.c_size_t)] * 4),
    "lbm_attach": (ctypes.c_int, [_P, _P, _P, _P, _P]),
    "lbm_set_stream": (ctypes.c_int, [_P, _P]),
    "lbm_set_precision": (ctypes.c_int, [_P, ctypes.c_int]),
    "lbm_set_layout": (ctypes.c_int, [_P, ctypes.c_int]),
    "lbm_strides": (ctypes.c_int, [_P] + [ctypes.POINTER(ctypes.c_size_t)] * 2),
    "lbm_set_tile": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int]),
    "lbm_set_launch": (ctypes.c_int, [_P] + [ctypes.c_int] * 4),
    "lbm_get_launch": (ctypes.c_int, [_P] + [ctypes.POINTER(ctypes.c_int)] * 4),
    "lbm_set_probes": (ctypes.c_int, [_P] + [ctypes.c_int] * 4),
    "lbm_init": (ctypes.c_int, [_P, _D, _D]),
    "lbm_step": (ctypes.c_int, [_P, ctypes.c_int]),
    "lbm_read": (ctypes.c_int, [_P, _D, _D]),
    "lbm_populations": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_float)]),
    "lbm_set_populations": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_float)]),
    "lbm_stats": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(lbm_stats_t)]),
    "lbm_stats_noalloc": (ctypes.c_int, [_P, ctypes.POINTER(lbm_stats_t)]),
    "lbm_timing_enable": (ctypes.c_int, [_P, ctypes.c_int]),
    "lbm_timing": (ctypes.c_int, [_P, _D, _D, ctypes.POINTER(ctypes.c_longlong)]),
    "lbm_eos_critical": (ctypes.c_int, [ctypes.POINTER(lbm_eos), _D, _D, _D]),
    "lbm_eos_maxwell": (ctypes.c_int, [ctypes.POINTER(lbm_eos), _D, _D]),
    "lbm_eos_pressure": (ctypes.c_int, [ctypes.POINTER(lbm_eos), ctypes.POINTER(lbm_force),
                                        ctypes.c_double, _D]),
    "lbm_coexistence": (ctypes.c_int, [ctypes.POINTER(lbm_eos), ctypes.POINTER(lbm_force),
                                       ctypes.c_int, ctypes.c_double, _D, _D]),
    "lbm_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "lbm_last_error": (ctypes.c_char_p, [_P]),
    "lbm_copy_f32": (ctypes.c_int, [_P, _P, ctypes.c_size_t, _P]),
}
for _name, (_res, _args) in _SIG.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args
    globals()[_name] = _fn


class LBMError(RuntimeError):
    def __init__(self, code, msg=""):
        self.code = code
        super().__init__(f"{lbm_strerror(code).decode()} ({code}): {msg}")


def check(code, handle=None):
    if code != LBM_OK:
        msg = lbm_last_error(handle).decode() if handle else ""
        raise LBMError(code, msg)
    return code


def _dptr(a):
    if a is None:
        return ctypes.cast(None, _D)
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


def make_eos(T_over_Tc, K=1.0, a=1.0, b=4.0, R=1.0):
    """Carnahan-Starling EOS (Eq. 29-30) at T/Tc, psi from Eq. 7."""
    return lbm_eos(LBM_EOS_CARNAHAN_STARLING, a, b, R, T_over_Tc, K, 0.0)


def make_ss_eos(eps):
    """Effective density of Eq. 33 with exponent eps (0: exp(-1/rho)); pressure from Eq. 7."""
    return lbm_eos(LBM_EOS_SBRAGAGLIA_SHAN, 1.0, 4.0, 1.0, 0.5, 1.0, eps)


def make_force(scheme="GUO", A=0.0, sigma=0.0, G=-1.0):
    return lbm_force(SCHEMES[scheme] if isinstance(scheme, str) else scheme, A, sigma, G)


def make_collision(kind="BGK", s=(1.0, 1.1, 1.1, 1.0, 1.1)):
    """s = (s_rho, s_e, s_eps, s_j, s_q); s_nu = 1/tau is implied (Eq. 35)."""
    return lbm_collision(COLLISIONS[kind] if isinstance(kind, str) else kind, *s)


def eos_critical(eos: lbm_eos):
    rc, Tc, pc = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    check(lbm_eos_critical(ctypes.byref(eos), ctypes.byref(rc), ctypes.byref(Tc), ctypes.byref(pc)))
    return rc.value, Tc.value, pc.value


def coexistence(eos: lbm_eos, force: lbm_force, rule="maxwell", eps_mech=0.0):
    """Flat-interface coexistence densities (rho_g, rho_l): rule 'maxwell' (Eq. 19) or
    'mechanical' (Eq. 18 with exponent eps_mech)."""
    g, l = ctypes.c_double(), ctypes.c_double()
    r = LBM_COEX_MAXWELL if rule == "maxwell" else LBM_COEX_MECHANICAL
    check(lbm_coexistence(ctypes.byref(eos), ctypes.byref(force), r, float(eps_mech),
                          ctypes.byref(g), ctypes.byref(l)))
    return g.value, l.value


def eos_pressure(eos: lbm_eos, force: lbm_force, rho):
    """Bulk pressure p0(rho) of the EOS (Eq. 30, or Eq. 7 with Eq. 33's psi)."""
    p = ctypes.c_double()
    check(lbm_eos_pressure(ctypes.byref(eos), ctypes.byref(force), float(rho), ctypes.byref(p)))
    return p.value


def eos_maxwell(eos: lbm_eos):
    g, l = ctypes.c_double(), ctypes.c_double()
    check(lbm_eos_maxwell(ctypes.byref(eos), ctypes.byref(g), ctypes.byref(l)))
    return g.value, l.value


class Lattice:
    """One periodic lattice whose buffers and stream come from torch (device memory only)."""

    def __init__(self, nx, ny, eos, force, collision, tau, precision=LBM_PREC_MIXED,
                 tile=None, device="cuda:0", stream=None, layout=LBM_LAYOUT_ROWS):
        import torch  # torch supplies device memory and the stream
        self.nx, self.ny = nx, ny
        h = _P()
        check(lbm_create(nx, ny, ctypes.byref(eos), ctypes.byref(force), ctypes.byref(collision),
                         float(tau), ctypes.byref(h)))
        self.h = h
        pitch, plane, fb, pb = (ctypes.c_size_t() for _ in range(4))
        check(lbm_layout(h, ctypes.byref(pitch), ctypes.byref(plane), ctypes.byref(fb),
                         ctypes.byref(pb)), h)
        self.pitch, self.plane = pitch.value, plane.value
        dev = torch.device(device)
        self.f_a = torch.zeros(fb.value // 4, dtype=torch.float32, device=dev)
        self.f_b = torch.zeros(fb.value // 4, dtype=torch.float32, device=dev)
        self.psi = torch.zeros(pb.value // 4, dtype=torch.float32, device=dev)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        check(lbm_attach(h, self.f_a.data_ptr(), self.f_b.data_ptr(), self.psi.data_ptr(),
                         self.stream.cuda_stream), h)
        check(lbm_set_precision(h, precision), h)
        check(lbm_set_layout(h, layout), h)
        if tile is not None:
            check(lbm_set_tile(h, *tile), h)

    def __del__(self, _live=_LIVE):
        h = getattr(self, "h", None)
        if h and _live[0]:
            lbm_destroy(h)
            self.h = None

    def init(self, rho0, u0=None):
        rho0 = np.ascontiguousarray(rho0, dtype=np.float64)
        assert rho0.shape == (self.ny, self.nx)
        u0 = None if u0 is None else np.ascontiguousarray(u0, dtype=np.float64)
        check(lbm_init(self.h, _dptr(rho0), _dptr(u0)), self.h)

    def step(self, n=1):
        check(lbm_step(self.h, int(n)), self.h)

    def read(self):
        rho = np.empty((self.ny, self.nx))
        u = np.empty((self.ny, self.nx, 2))
        check(lbm_read(self.h, _dptr(rho), _dptr(u)), self.h)
        return rho, u

    def populations(self):
        f = np.empty((9, self.ny, self.nx), dtype=np.float32)
        check(lbm_populations(self.h, f.ctypes.data_as(ctypes.POINTER(ctypes.c_float))), self.h)
        return f

    def save(self, path):
        """Checkpoint (populations, step count, parameters) to a file."""
        check(lbm_save(self.h, os.fsencode(path)), self.h)

    def load(self, path):
        """Restore a checkpoint written by `save` for a lattice of the same size and parameters."""
        check(lbm_load(self.h, os.fsencode(path)), self.h)

    def set_populations(self, f):
        f = np.ascontiguousarray(f, dtype=np.float32)
        assert f.shape == (9, self.ny, self.nx)
        check(lbm_set_populations(self.h, f.ctypes.data_as(ctypes.POINTER(ctypes.c_float))), self.h)

    def stats(self, track_dv=False, allow_unstable=False):
        s = lbm_stats_t()
        rc = lbm_stats(self.h, int(track_dv), ctypes.byref(s))
        if rc != LBM_OK and not (allow_unstable and rc == LBM_EUNSTABLE):
            check(rc, self.h)
        return s.as_dict()

    def stats_noalloc(self, allow_unstable=False):
        """lbm_stats without allocating (the library's fixed device array; no dv)."""
        s = lbm_stats_t()
        rc = lbm_stats_noalloc(self.h, ctypes.byref(s))
        if rc != LBM_OK and not (allow_unstable and rc == LBM_EUNSTABLE):
            check(rc, self.h)
        return s.as_dict()

    def set_probes(self, xa, ya, xb, yb):
        check(lbm_set_probes(self.h, xa, ya, xb, yb), self.h)

    def set_tile(self, tx, ty):
        check(lbm_set_tile(self.h, tx, ty), self.h)

    def set_launch(self, kernel, tx, ty, flags=0):
        check(lbm_set_launch(self.h, kernel, tx, ty, flags), self.h)

    def autotune(self, cache_path=None, trial_steps=20):
        """Pick the fastest sweep launch by timed trials on the current state (restored
        afterwards) and apply it; returns ms per step of the winner (-1: cache hit)."""
        ms = ctypes.c_double(0.0)
        path = None if cache_path is None else os.fsencode(cache_path)
        check(lbm_autotune(self.h, path, int(trial_steps), ctypes.byref(ms)), self.h)
        return ms.value

    def get_launch(self):
        v = [ctypes.c_int() for _ in range(4)]
        check(lbm_get_launch(self.h, *(ctypes.byref(x) for x in v)), self.h)
        return tuple(x.value for x in v)

    def set_precision(self, precision):
        check(lbm_set_precision(self.h, precision), self.h)

    def timing_enable(self, on=True):
        check(lbm_timing_enable(self.h, int(on)), self.h)

    def timing(self):
        a, b, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_longlong()
        check(lbm_timing(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(n)), self.h)
        return a.value, b.value, n.value


# ---- batched sweep -------------------------------------------------------------------------
_BSIG = {
    "lbm_batch_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(ctypes.c_int), ctypes.POINTER(lbm_eos),
                                        ctypes.POINTER(lbm_force), ctypes.POINTER(lbm_collision),
                                        _D, ctypes.POINTER(_P)]),
    "lbm_batch_destroy": (None, [_P]),
    "lbm_batch_set_launch": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "lbm_batch_set_segment": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int]),
    "lbm_batch_init": (ctypes.c_int, [_P, ctypes.c_int, _D, _D]),
    "lbm_autotune": (ctypes.c_int, [_P, ctypes.c_char_p, ctypes.c_int, _D]),
    "lbm_batch_autotune": (ctypes.c_int, [_P, ctypes.c_char_p, ctypes.c_int, _D]),
    "lbm_batch_init_rest": (ctypes.c_int, [_P, ctypes.c_int, _D]),
    "lbm_batch_init_tanh": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_int]),
    "lbm_save": (ctypes.c_int, [_P, ctypes.c_char_p]),
    "lbm_load": (ctypes.c_int, [_P, ctypes.c_char_p]),
    "lbm_batch_init_profile": (ctypes.c_int, [_P, ctypes.c_int, _D, ctypes.c_double,
                                              ctypes.c_double, ctypes.c_double, _D]),
    "lbm_batch_set_active": (ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int]),
    "lbm_batch_step": (ctypes.c_int, [_P, ctypes.c_int]),
    "lbm_batch_stats": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(lbm_stats_t)]),
    "lbm_batch_run": (ctypes.c_int, [_P, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                     ctypes.c_longlong,
                                     ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_int)]),
    "lbm_batch_read": (ctypes.c_int, [_P, ctypes.c_int, _D, _D]),
    "lbm_batch_populations": (ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_float)]),
    "lbm_batch_steps": (ctypes.c_longlong, [_P, ctypes.c_int]),
    "lbm_batch_sync": (ctypes.c_int, [_P]),
    "lbm_batch_last_error": (ctypes.c_char_p, [_P]),
}
for _name, (_res, _args) in _BSIG.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args
    globals()[_name] = _fn


def bcheck(code, b=None):
    if code != LBM_OK:
        raise LBMError(code, lbm_batch_last_error(b).decode() if b else "")
    return code


class Batch:
    """Independent lattices advanced together (lbm_batch_*).  members: list of dicts with nx,
    ny, T_over_Tc, K, scheme, A, sigma, collision, s (5 MRT rates), tau; "psi_eps" (with "G")
    selects the effective density of Eq. 33 instead of the Carnahan-Starling EOS."""

    def __init__(self, members, tx=256, groups=0, flags=LBM_LAUNCH_TWO_STEP):
        n = len(members)
        self.members = members
        nx = (ctypes.c_int * n)(*[m["nx"] for m in members])
        ny = (ctypes.c_int * n)(*[m["ny"] for m in members])
        eos = (lbm_eos * n)(*[make_ss_eos(m["psi_eps"]) if "psi_eps" in m else
                              make_eos(m["T_over_Tc"], K=m.get("K", 1.0)) for m in members])
        frc = (lbm_force * n)(*[make_force(m.get("scheme", "GUO"), A=m.get("A", 0.0),
                                           sigma=m.get("sigma", 0.0), G=m.get("G", -1.0))
                                for m in members])
        col = (lbm_collision * n)(*[make_collision(m.get("collision", "BGK"),
                                                   s=m.get("s", (1.0, 1.1, 1.1, 1.0, 1.1)))
                                    for m in members])
        tau = (ctypes.c_double * n)(*[m["tau"] for m in members])
        b = _P()
        check(lbm_batch_create(n, nx, ny, eos, frc, col, tau, ctypes.byref(b)))
        self.b = b
        bcheck(lbm_batch_set_launch(b, tx, groups, flags), b)

    def __del__(self, _live=_LIVE):
        b = getattr(self, "b", None)
        if b and _live[0]:
            lbm_batch_destroy(b)
            self.b = None

    def set_segment(self, i, rows):
        bcheck(lbm_batch_set_segment(self.b, i, rows), self.b)

    def init(self, i, rho0, u0=None):
        m = self.members[i]
        rho0 = np.ascontiguousarray(rho0, dtype=np.float64)
        assert rho0.shape == (m["ny"], m["nx"])
        u0 = None if u0 is None else np.ascontiguousarray(u0, dtype=np.float64)
        bcheck(lbm_batch_init(self.b, i, _dptr(rho0), _dptr(u0)), self.b)

    def init_rest(self, i, rho0):
        """f = f^eq(rho0, -F/(2 rho0)): the density at physical rest (v = 0)."""
        m = self.members[i]
        rho0 = np.ascontiguousarray(rho0, dtype=np.float64)
        assert rho0.shape == (m["ny"], m["nx"])
        bcheck(lbm_batch_init_rest(self.b, i, _dptr(rho0)), self.b)

    def init_tanh(self, i, R, W=5.0, droplet=True):
        """The plain start: a tanh droplet (or bubble) of radius R between the Maxwell densities
        of the lattice's EOS, at physical rest."""
        bcheck(lbm_batch_init_tanh(self.b, i, float(R), float(W), int(droplet)), self.b)

    def init_profile(self, i, log_rho, r0, dr, mass=0.0):
        """Warm start from 64 values of log rho at r_k = r0 + k dr; with mass > 0 the profile is
        shifted radially to carry exactly that total mass.  Returns the shift."""
        log_rho = np.ascontiguousarray(log_rho, dtype=np.float64)
        assert log_rho.shape == (64,)
        shift = ctypes.c_double(0.0)
        bcheck(lbm_batch_init_profile(self.b, i, _dptr(log_rho), float(r0), float(dr),
                                      float(mass), ctypes.byref(shift)), self.b)
        return shift.value

    def autotune(self, cache_path=None, trial_steps=20):
        """Pick strip width, prefetch depth and segment heights per size class by timed trials
        (state restored afterwards); returns ms per step of the winner (-1: cache hit)."""
        ms = ctypes.c_double(0.0)
        path = None if cache_path is None else os.fsencode(cache_path)
        bcheck(lbm_batch_autotune(self.b, path, int(trial_steps), ctypes.byref(ms)), self.b)
        return ms.value

    def set_active(self, i, on):
        bcheck(lbm_batch_set_active(self.b, i, int(on)), self.b)

    def step(self, n):
        bcheck(lbm_batch_step(self.b, int(n)), self.b)

    def sync(self):
        bcheck(lbm_batch_sync(self.b), self.b)

    def stats(self, track_dv=False, allow_unstable=True):
        out = (lbm_stats_t * len(self.members))()
        rc = lbm_batch_stats(self.b, int(track_dv), out)
        if rc != LBM_OK and not (allow_unstable and rc == LBM_EUNSTABLE):
            bcheck(rc, self.b)
        return [s.as_dict() for s in out]

    def run(self, tol, check_every=100, max_steps=2_000_000, tol_rho=0.0):
        n = len(self.members)
        steps = (ctypes.c_longlong * n)()
        status = (ctypes.c_int * n)()
        bcheck(lbm_batch_run(self.b, tol, tol_rho, check_every, max_steps, steps, status), self.b)
        return list(steps), list(status)

    def read(self, i):
        m = self.members[i]
        rho = np.empty((m["ny"], m["nx"]))
        u = np.empty((m["ny"], m["nx"], 2))
        bcheck(lbm_batch_read(self.b, i, _dptr(rho), _dptr(u)), self.b)
        return rho, u

    def populations(self, i):
        m = self.members[i]
        f = np.empty((9, m["ny"], m["nx"]), dtype=np.float32)
        bcheck(lbm_batch_populations(self.b, i, f.ctypes.data_as(ctypes.POINTER(ctypes.c_float))),
               self.b)
        return f

    def steps(self, i):
        return int(lbm_batch_steps(self.b, i))


# ---- learned warm start network ----------------------------------------------------------------
_MSIG = {
    "lbm_mlp_create": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(_P)]),
    "lbm_mlp_destroy": (None, [_P]),
    "lbm_mlp_param_count": (ctypes.c_size_t, [_P]),
    "lbm_mlp_set_params": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_float)]),
    "lbm_mlp_get_params": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_float)]),
    "lbm_mlp_forward": (ctypes.c_int, [_P, _P, ctypes.c_int, _P, _P]),
    "lbm_mlp_gradient": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, _P, _P]),
    "lbm_mlp_train_step": (ctypes.c_int, [_P, _P, _P, ctypes.c_int, ctypes.c_float,
                                          ctypes.POINTER(ctypes.c_float), _P]),
    "lbm_mlp_last_error": (ctypes.c_char_p, [_P]),
}
for _name, (_res, _args) in _MSIG.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args
    globals()[_name] = _fn


class MLP:
    """The library's GPU network; inputs and outputs are torch CUDA float32 tensors."""

    def __init__(self, dims, seed=0):
        self.dims = list(dims)
        arr = (ctypes.c_int * len(dims))(*dims)
        n = _P()
        check(lbm_mlp_create(len(dims) - 1, arr, ctypes.byref(n)))
        self.n = n
        self.nparam = int(lbm_mlp_param_count(n))
        # Glorot-uniform weights, zero biases (seeded).
        rng = np.random.default_rng(seed)
        parts = []
        for i, o in zip(dims[:-1], dims[1:]):
            lim = np.sqrt(6.0 / (i + o))
            parts += [rng.uniform(-lim, lim, size=o * i), np.zeros(o)]
        self.set_params(np.concatenate(parts).astype(np.float32))

    def __del__(self, _live=_LIVE):
        n = getattr(self, "n", None)
        if n and _live[0]:
            lbm_mlp_destroy(n)
            self.n = None

    def _check(self, rc):
        if rc != LBM_OK:
            raise LBMError(rc, lbm_mlp_last_error(self.n).decode())

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        assert p.size == self.nparam
        self._check(lbm_mlp_set_params(self.n, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))

    def get_params(self):
        p = np.empty(self.nparam, dtype=np.float32)
        self._check(lbm_mlp_get_params(self.n, p.ctypes.data_as(ctypes.POINTER(ctypes.c_float))))
        return p

    @staticmethod
    def _stream():
        import torch
        return torch.cuda.current_stream().cuda_stream

    def forward(self, x):
        import torch
        x = x.contiguous().float()
        y = torch.empty((x.shape[0], self.dims[-1]), dtype=torch.float32, device=x.device)
        self._check(lbm_mlp_forward(self.n, x.data_ptr(), x.shape[0], y.data_ptr(), self._stream()))
        return y

    def gradient(self, x, dy):
        import torch
        x = x.contiguous().float()
        dy = dy.contiguous().float()
        g = torch.empty(self.nparam, dtype=torch.float32, device=x.device)
        self._check(lbm_mlp_gradient(self.n, x.data_ptr(), dy.data_ptr(), x.shape[0], g.data_ptr(),
                                     self._stream()))
        return g

    def train_step(self, x, target, lr):
        loss = ctypes.c_float()
        self._check(lbm_mlp_train_step(self.n, x.data_ptr(), target.data_ptr(), x.shape[0],
                                       float(lr), ctypes.byref(loss), self._stream()))
        return loss.value
