"""Plain FP64 CPU oracle of the D2Q13 energy-conserving lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()``
and by the ``cpu_baseline`` leg of ``bench.py``; never by the product package.

The arithmetic lives in ``oracle13.c`` (plain C, per-node loops, no FMA
contraction, OpenMP over nodes).  This module only builds it with gcc and
marshals numpy arrays through ctypes.  Populations are dense ``(13, ny, nx)``
float64 arrays holding the pre-collision state f(t).

Paper: Lallemand & Dubois, "Comparison of Simulations of Convective Flows",
sec. 2 (scheme), secs. 5 and 8 (forces), sec. 7 (walls, T), Table 1 (Nusselt).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle13.c")
_LIB = os.path.join(_HERE, "liboracle13.so")

PERIODIC, ADIABATIC, DIRICHLET_T = 0, 1, 2
WEST, EAST, SOUTH, NORTH = 0, 1, 2, 3


class Params(ctypes.Structure):
    """Free parameters of the scheme (sec. 2) plus the body forces (secs. 5, 8)."""

    _fields_ = [
        ("Pr", ctypes.c_double), ("E0", ctypes.c_double), ("c1", ctypes.c_double),
        ("k2", ctypes.c_double), ("c_epsE", ctypes.c_double),
        ("c_varpi_rho", ctypes.c_double), ("c_varpi_E", ctypes.c_double),
        ("s_XX", ctypes.c_double), ("s_rx", ctypes.c_double), ("s_eps", ctypes.c_double),
        ("s_varpi", ctypes.c_double), ("s_XXe", ctypes.c_double),
        ("F0x", ctypes.c_double), ("F0y", ctypes.c_double),
        ("gx", ctypes.c_double), ("gy", ctypes.c_double), ("rho0", ctypes.c_double),
        ("collide", ctypes.c_int),
        ("Q_E", ctypes.c_double),
    ]


class Sides(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int * 4), ("u_t", ctypes.c_double * 4), ("T_w", ctypes.c_double * 4)]


class Derived(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in (
        "A", "Y", "h1", "k1", "h2", "c2", "c_eps_rho", "sigma_XX", "sigma_q", "s_q",
        "nu", "kappa", "cs2", "B", "kappa_E")]


def build(force: bool = False) -> str:
    """Compile oracle13.c with gcc into liboracle13.so (plain -O2, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        L.or13_matrix.argtypes = [dp, dp]
        L.or13_velocities.argtypes = [ctypes.POINTER(ctypes.c_int)] * 2
        L.or13_derive.argtypes = [ctypes.POINTER(Params), ctypes.POINTER(Derived)]
        L.or13_derive.restype = ctypes.c_int
        L.or13_equilibrium_moments.argtypes = [ctypes.POINTER(Params)] + [ctypes.c_double] * 4 + [dp]
        L.or13_init.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, dp, ctypes.POINTER(Params), dp]
        L.or13_collide.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.POINTER(Params), dp]
        L.or13_stream.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, ctypes.POINTER(Params),
                                  ctypes.POINTER(Sides), dp]
        L.or13_step.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.POINTER(Params),
                                ctypes.POINTER(Sides), dp, dp]
        L.or13_step.restype = ctypes.c_int
        L.or13_run.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.POINTER(Params),
                               ctypes.POINTER(Sides), ctypes.c_long]
        L.or13_run.restype = ctypes.c_int
        L.or13_moments.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.POINTER(Params), dp, dp, dp, dp]
        L.or13_diagnostics.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.POINTER(Params),
                                       ctypes.POINTER(Sides), dp]
        L.or13_num_threads.restype = ctypes.c_int
        L.or13_set_num_threads.argtypes = [ctypes.c_int]
        L.or13_fourier.argtypes = [ctypes.c_int, ctypes.c_int, dp, ctypes.POINTER(Params), ctypes.c_int,
                                   ctypes.c_int, dp]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# Free-parameter set used by default.  The paper prints no values (sec. 2 says
# they were chosen by a linear-stability heuristic); this set was chosen the same
# way (roots of the linear dispersion relation over the Brillouin zone) and gives
# A = 13 c1 + 95 + 2 E0 = 52, i.e. cs^2 = 1, and positive rest populations.
DEFAULTS = dict(Pr=0.71, E0=-2.0, c1=-3.0, k2=-2.5, c_epsE=-2.5, c_varpi_rho=-6.0, c_varpi_E=-0.5,
                s_XX=1.6, s_rx=1.05, s_eps=1.0, s_varpi=1.0, s_XXe=1.5,
                F0x=0.0, F0y=0.0, gx=0.0, gy=0.0, rho0=1.0, collide=1, Q_E=0.0)


def params(**kw) -> Params:
    d = dict(DEFAULTS)
    for k, v in kw.items():
        if k not in d:
            raise KeyError(k)
        d[k] = v
    return Params(**d)


def sides(kinds=(PERIODIC,) * 4, u_t=(0.0,) * 4, T_w=(0.0,) * 4) -> Sides:
    s = Sides()
    for w in range(4):
        s.kind[w] = int(kinds[w])
        s.u_t[w] = float(u_t[w])
        s.T_w[w] = float(T_w[w])
    return s


def matrix():
    """(M, D, vx, vy): moment matrix rows k, columns j; D_k = sum_j M_kj^2."""
    M = np.zeros(169)
    D = np.zeros(13)
    lib().or13_matrix(_p(M), _p(D))
    vx = (ctypes.c_int * 13)()
    vy = (ctypes.c_int * 13)()
    lib().or13_velocities(vx, vy)
    return M.reshape(13, 13), D, np.array(vx[:]), np.array(vy[:])


def derive(p: Params):
    """Derived coefficients; returns (status, dict)."""
    d = Derived()
    st = lib().or13_derive(ctypes.byref(p), ctypes.byref(d))
    return st, {n: getattr(d, n) for n, _ in Derived._fields_}


def equilibrium_moments(p: Params, rho, jx, jy, E):
    out = np.zeros(13)
    lib().or13_equilibrium_moments(ctypes.byref(p), rho, jx, jy, E, _p(out))
    return out


def init(rho, ux, uy, T, p: Params) -> np.ndarray:
    rho, ux, uy, T = (np.ascontiguousarray(a, dtype=np.float64) for a in (rho, ux, uy, T))
    ny, nx = rho.shape
    f = np.zeros((13, ny, nx))
    lib().or13_init(nx, ny, _p(rho), _p(ux), _p(uy), _p(T), ctypes.byref(p), _p(f))
    return f


def collide(f: np.ndarray, p: Params) -> np.ndarray:
    f = np.ascontiguousarray(f, dtype=np.float64)
    _, ny, nx = f.shape
    out = np.empty_like(f)
    lib().or13_collide(nx, ny, _p(f), ctypes.byref(p), _p(out))
    return out


def step(f: np.ndarray, p: Params, s: Sides, return_fstar: bool = False):
    f = np.ascontiguousarray(f, dtype=np.float64)
    _, ny, nx = f.shape
    out = np.empty_like(f)
    fs = np.empty_like(f)
    st = lib().or13_step(nx, ny, _p(f), ctypes.byref(p), ctypes.byref(s), _p(out), _p(fs))
    if st:
        raise MemoryError("oracle step failed")
    return (out, fs) if return_fstar else out


def run(f: np.ndarray, p: Params, s: Sides, steps: int) -> np.ndarray:
    g = np.array(f, dtype=np.float64, order="C", copy=True)
    _, ny, nx = g.shape
    if lib().or13_run(nx, ny, _p(g), ctypes.byref(p), ctypes.byref(s), int(steps)):
        raise MemoryError("oracle run failed")
    return g


def moments(f: np.ndarray, p: Params):
    f = np.ascontiguousarray(f, dtype=np.float64)
    _, ny, nx = f.shape
    rho, ux, uy, T = (np.empty((ny, nx)) for _ in range(4))
    lib().or13_moments(nx, ny, _p(f), ctypes.byref(p), _p(rho), _p(ux), _p(uy), _p(T))
    return rho, ux, uy, T


DIAG_NAMES = ("sum_rho", "sum_jx", "sum_jy", "sum_E", "heat_flux", "Nu_mean", "u_max",
              "asym_abs", "asym_rel", "nonfinite", "rho_min", "Nu_west", "Nu_east", "wall_energy_in",
              "wall_mass_in")


def diagnostics(f: np.ndarray, p: Params, s: Sides) -> dict:
    f = np.ascontiguousarray(f, dtype=np.float64)
    _, ny, nx = f.shape
    out = np.zeros(16)
    lib().or13_diagnostics(nx, ny, _p(f), ctypes.byref(p), ctypes.byref(s), _p(out))
    return dict(zip(DIAG_NAMES, out[:len(DIAG_NAMES)]))


def fourier(f: np.ndarray, p: Params, kx: int, ky: int) -> dict:
    """sum q exp(-2 pi i (kx x/nx + ky y/ny)) for q = rho, ux, uy, E (complex)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    _, ny, nx = f.shape
    out = np.zeros(8)
    lib().or13_fourier(nx, ny, _p(f), ctypes.byref(p), int(kx), int(ky), _p(out))
    return {q: complex(out[2 * k], out[2 * k + 1]) for k, q in enumerate(("rho", "ux", "uy", "E"))}


def num_threads() -> int:
    return int(lib().or13_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops from now on (timing only: results do not depend on it)."""
    lib().or13_set_num_threads(int(n))
