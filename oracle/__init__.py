"""Oracle for the pseudo-potential D2Q9 lattice Boltzmann step of arXiv:1412.5170.

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the CPU-baseline leg of
the benchmark are the only callers.  Nothing here is shared with, or imported by, the
HIP library or its Python binding.

* ``lbm_oracle.c``  -- plain FP64 time step (Sec. 2-4), loaded through ctypes here.
* ``thermo``        -- Carnahan-Starling EOS, exact critical point, Maxwell equal-area
                       coexistence (Eq. 19), mechanical stability condition (Eq. 18),
                       parameter maps (Table 1, Eq. 32).
* ``bruteforce``    -- the literal equations with explicit tensor sums on tiny lattices,
                       used to pin the C stepper.
* ``mlp``           -- FP64 reference of the warm-start network's forward/backward pass.
* ``profile``       -- the warm-start initial state: radial profile to lattice, mass matching.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

EDM, GUO, GUO_LI, SC = 0, 1, 2, 3
BGK, MRT = 0, 1

# D2Q9 velocity order used by the oracle's population arrays ([9][ny][nx]).
EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])


def build(force: bool = False) -> str:
    """Compile lbm_oracle.c into liboracle.so with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
             "-shared", "-std=c11", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("a", ctypes.c_double), ("b", ctypes.c_double), ("R", ctypes.c_double),
                ("T", ctypes.c_double), ("K", ctypes.c_double), ("G", ctypes.c_double),
                ("A", ctypes.c_double), ("sigma", ctypes.c_double), ("tau", ctypes.c_double),
                ("scheme", ctypes.c_int), ("collision", ctypes.c_int),
                ("s", ctypes.c_double * 9),
                ("psi_kind", ctypes.c_int), ("psi_eps", ctypes.c_double)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(_Params)
        _lib.orc_step.argtypes = [pp, dp, ctypes.c_int]
        _lib.orc_collide.argtypes = [pp, dp, dp]
        _lib.orc_fields.argtypes = [pp, dp] + [dp] * 8
        _lib.orc_init_feq.argtypes = [ctypes.c_int, dp, dp, dp, dp]
        _lib.orc_feq.argtypes = [ctypes.c_double] * 3 + [dp]
        _lib.orc_pressure.argtypes = [pp, ctypes.c_double]
        _lib.orc_pressure.restype = ctypes.c_double
        _lib.orc_psi.argtypes = [pp, ctypes.c_double]
        _lib.orc_psi.restype = ctypes.c_double
        _lib.orc_mrt_matrix.argtypes = [dp, dp]
        _lib.orc_guo_bracket.argtypes = [ctypes.c_double] * 4 + [dp]
        _lib.orc_threads.restype = ctypes.c_int
        _lib.orc_set_threads.argtypes = [ctypes.c_int]
    return _lib


def threads() -> int:
    """OpenMP threads the stepper runs on."""
    return int(lib().orc_threads())


def set_threads(n: int) -> None:
    """Run the stepper's later parallel loops on n threads."""
    lib().orc_set_threads(int(n))


class OracleError(RuntimeError):
    pass


_ERR = {-1: "invalid parameters", -2: "unstable state (psi^2 <= 0, eta >= 1 or non-finite)",
        -3: "out of memory"}


def _check(rc):
    if rc != 0:
        raise OracleError(_ERR.get(rc, "error %d" % rc))


@dataclass
class Params:
    """Physical and numerical parameters of one lattice (absolute temperature T)."""
    nx: int
    ny: int
    T: float
    tau: float = 1.0
    scheme: int = GUO
    collision: int = BGK
    a: float = 1.0
    b: float = 4.0
    R: float = 1.0
    K: float = 1.0
    G: float = -1.0
    A: float = 0.0
    sigma: float = 0.0
    s: tuple = field(default_factory=lambda: (1.0,) * 9)
    psi_kind: int = 0     # 0: psi from the EOS (Eq. 7); 1: psi of Eq. 33
    psi_eps: float = 1.0  # Eq. 33 exponent (psi_kind 1)

    def c(self) -> _Params:
        return _Params(self.nx, self.ny, self.a, self.b, self.R, self.T, self.K, self.G,
                       self.A, self.sigma, self.tau, self.scheme, self.collision,
                       (ctypes.c_double * 9)(*self.s), self.psi_kind, self.psi_eps)


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def init_feq(rho, ux=None, uy=None) -> np.ndarray:
    """Populations f = f^eq(rho, u) (Eq. 2), shape [9, ny, nx]."""
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    n = rho.size
    f = np.empty((9,) + rho.shape, dtype=np.float64)
    ux = None if ux is None else np.ascontiguousarray(ux, dtype=np.float64)
    uy = None if uy is None else np.ascontiguousarray(uy, dtype=np.float64)
    null = ctypes.POINTER(ctypes.c_double)()
    lib().orc_init_feq(n, _ptr(rho), _ptr(ux) if ux is not None else null,
                       _ptr(uy) if uy is not None else null, _ptr(f))
    return f


def feq(rho: float, ux: float, uy: float) -> np.ndarray:
    out = np.empty(9)
    lib().orc_feq(rho, ux, uy, _ptr(out))
    return out


def pressure(p: Params, rho: float) -> float:
    pc = p.c()
    return lib().orc_pressure(ctypes.byref(pc), rho)


def psi(p: Params, rho: float) -> float:
    pc = p.c()
    return lib().orc_psi(ctypes.byref(pc), rho)


def step(p: Params, f: np.ndarray, nsteps: int = 1) -> np.ndarray:
    """Advance a copy of f ([9, ny, nx]) by nsteps time steps and return it."""
    g = np.array(f, dtype=np.float64, order="C", copy=True)
    assert g.shape == (9, p.ny, p.nx)
    pc = p.c()
    _check(lib().orc_step(ctypes.byref(pc), _ptr(g), int(nsteps)))
    return g


def collide(p: Params, f: np.ndarray) -> np.ndarray:
    """Post-collision populations f* (before streaming)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.empty_like(f)
    pc = p.c()
    _check(lib().orc_collide(ctypes.byref(pc), _ptr(f), _ptr(out)))
    return out


def fields(p: Params, f: np.ndarray) -> dict:
    """rho, psi, F, u and v = u + F/(2 rho) of the populations f."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    shp = (p.ny, p.nx)
    out = {k: np.empty(shp) for k in ("rho", "psi", "Fx", "Fy", "ux", "uy", "vx", "vy")}
    pc = p.c()
    _check(lib().orc_fields(ctypes.byref(pc), _ptr(f), *[_ptr(out[k]) for k in
                                                         ("rho", "psi", "Fx", "Fy", "ux", "uy",
                                                          "vx", "vy")]))
    return out


def mrt_matrix():
    M = np.empty((9, 9))
    Minv = np.empty((9, 9))
    _check(lib().orc_mrt_matrix(_ptr(M), _ptr(Minv)))
    return M, Minv


def guo_bracket(Fx: float, Fy: float, Vx: float, Vy: float) -> np.ndarray:
    """Guo's bracket B_a(F, V) of Eq. 23 (without the 1 - 1/(2 tau) factor), nine values."""
    out = np.empty(9)
    lib().orc_guo_bracket(Fx, Fy, Vx, Vy, _ptr(out))
    return out


def stats(p: Params, f: np.ndarray, probes=None) -> dict:
    """Observables of Sec. 4 in FP64: total mass, min/max rho, Us_max = max |v|, probe
    densities.  ``probes`` maps a name to an (x, y) node."""
    fl = fields(p, f)
    rho = fl["rho"]
    vmag = np.hypot(fl["vx"], fl["vy"])
    out = {"mass": float(rho.sum()), "rho_min": float(rho.min()), "rho_max": float(rho.max()),
           "us_max": float(vmag.max())}
    for name, (x, y) in (probes or {}).items():
        out[name] = float(rho[y, x])
    return out
