"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle runs.

This module holds no arithmetic of the scheme: it only draws macroscopic
initial fields (rho, ux, uy, T on an (ny, nx) grid, float64) and domain
descriptors.  Each side (oracle, HIP library) turns them into populations with
its own code.  Recipes:

* ``periodic_wave``      -- nonlinear wave on a periodic box: rho = 1 + a cos(kx),
                            ux = b cos(kx), T uniform (sec. 4 style test, no walls).
* ``shear_acoustic``     -- ux = 0.01 sin(2 pi y / L), rho = 1 + 1e-3 cos(2 pi x / L),
                            T uniform (transverse shear wave + sound wave, sec. 6).
* ``thermal_mode``       -- T = T0 + dT cos(kx), rho = 1 - (T - T0)/28, at rest: the
                            non-acoustic diffusive state of sec. 4 (eigenvector
                            (1, 0, -28) of the first-order system, sec. 6).
* ``transverse_wave``    -- v_y = V0 cos(kx), rho = 1 + (13/56) v_y^2, T uniform: the sec. 6
                            transverse wave with the initial pressure made uniform.
* ``cavity_fields``      -- heated cavity at rest, T = T0 + 1e-3 dT U[-1, 1) noise with
                            rho = 1 - (T - T0)/28 (numpy default_rng(seed)), sec. 10.
* ``cavity_batch``       -- square cavities, side ~ U{64..512}, Ra log-uniform in
                            [1e3, 1e6], Pr ~ U[0.5, 7], one draw order per cavity.
* ``channel_batch``      -- channels periodic along y: length ~ U{256..2048}, width ~
                            U{32..256}; even index Couette (west wall velocity ~
                            U[0.01, 0.05]), odd index Poiseuille (force ~ U[1e-6, 1e-5]);
                            walls T0 +- dT with dT = 0.01 (secs. 7, 8).
"""
from __future__ import annotations

import numpy as np


def _grid(nx: int, ny: int):
    x = np.broadcast_to(np.arange(nx, dtype=np.float64)[None, :], (ny, nx))
    y = np.broadcast_to(np.arange(ny, dtype=np.float64)[:, None], (ny, nx))
    return x, y


def periodic_wave(n: int = 32, T0: float = -2.0, a_rho: float = 0.05, a_u: float = 0.02):
    x, _ = _grid(n, n)
    c = np.cos(2.0 * np.pi * x / n)
    return (1.0 + a_rho * c, a_u * c, np.zeros((n, n)), np.full((n, n), T0))


def shear_acoustic(nx: int, ny: int | None = None, T0: float = -2.0, a_u: float = 0.01, a_rho: float = 1e-3):
    ny = nx if ny is None else ny
    x, y = _grid(nx, ny)
    return (1.0 + a_rho * np.cos(2.0 * np.pi * x / nx), a_u * np.sin(2.0 * np.pi * y / ny),
            np.zeros((ny, nx)), np.full((ny, nx), T0))


def thermal_mode(nx: int, ny: int, T0: float = -2.0, dT: float = 1e-4, K: int = 1):
    x, _ = _grid(nx, ny)
    dE = dT * np.cos(2.0 * np.pi * K * x / nx)
    return (1.0 - dE / 28.0, np.zeros((ny, nx)), np.zeros((ny, nx)), T0 + dE)


def transverse_wave(nx: int, ny: int, V0: float = 0.02, T0: float = -2.0, a: float = 13.0 / 56.0):
    """Sec. 6 initial state: v_y = V0 cos(k x), rho = 1 + a v_y^2, uniform T.
    a = 13/56 makes the initial pressure (14/13) rho + E/26 - u_y^2/2 uniform
    (first-order system of sec. 6 and XX^eq = -rho u_y^2), so no 2k sound."""
    x, _ = _grid(nx, ny)
    uy = V0 * np.cos(2.0 * np.pi * x / nx)
    return (1.0 + a * uy * uy, np.zeros((ny, nx)), uy, np.full((ny, nx), T0))


def cavity_fields(n: int, T0: float = -2.0, dT: float = 0.01, seed: int = 0, ny: int | None = None):
    ny = n if ny is None else ny
    rng = np.random.default_rng(seed)
    dE = 1e-3 * dT * rng.uniform(-1.0, 1.0, size=(ny, n))
    return (1.0 - dE / 28.0, np.zeros((ny, n)), np.zeros((ny, n)), T0 + dE)


def cavity_batch(count: int = 64, seed: int = 4, side_lo: int = 64, side_hi: int = 512):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        side = int(rng.integers(side_lo, side_hi + 1))
        Ra = float(10.0 ** rng.uniform(3.0, 6.0))
        Pr = float(rng.uniform(0.5, 7.0))
        out.append(dict(nx=side, ny=side, Ra=Ra, Pr=Pr))
    return out


def channel_batch(count: int = 128, seed: int = 5, len_lo: int = 256, len_hi: int = 2048,
                  w_lo: int = 32, w_hi: int = 256, dT: float = 0.01):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(count):
        L = int(rng.integers(len_lo, len_hi + 1))
        W = int(rng.integers(w_lo, w_hi + 1))
        if i % 2 == 0:
            out.append(dict(nx=W, ny=L, kind="couette", U=float(rng.uniform(0.01, 0.05)), F=0.0, dT=dT))
        else:
            out.append(dict(nx=W, ny=L, kind="poiseuille", U=0.0, F=float(rng.uniform(1e-6, 1e-5)), dT=dT))
    return out


def rest_fields(nx: int, ny: int, T0: float = -2.0):
    return (np.ones((ny, nx)), np.zeros((ny, nx)), np.zeros((ny, nx)), np.full((ny, nx), T0))


def cavity_forcing(L: int, Ra: float, Pr: float, nu: float, kappa: float, eps_h: float = 0.2,
                   dT_min: float = 0.01, dT_max: float = 1.0, mach_max: float = 0.1, cs: float = 1.0):
    """Temperature difference and gravity for a heated cavity of side L at Rayleigh
    number Ra (eq intro-rayleigh with beta = 1/28: an isobaric change dE of the
    D2Q13 energy changes rho by -dE/28).

    |g| = 28 Ra nu kappa / (dT L^3).  Two limits make the run meaningful: the
    hydrostatic parameter |g| L / cs^2 (density scale height over cavity size)
    stays <= eps_h, and the free-fall Mach number sqrt(Ra/Pr) nu / (L cs) stays
    <= mach_max.  dT is the smallest value in [dT_min, dT_max] meeting the
    first; when no dT does, or the Mach limit is broken, Ra is lowered to the
    largest feasible value and `clamped` is set.  Inputs nu, kappa come from the
    caller's own parameter derivation."""
    Ra_eff = float(Ra)
    ra_mach = Pr * (mach_max * L * cs / nu) ** 2
    ra_hydro = eps_h * cs * cs * dT_max * L * L / (28.0 * nu * kappa)
    Ra_eff = min(Ra_eff, ra_mach, ra_hydro)
    dT = min(dT_max, max(dT_min, 28.0 * Ra_eff * nu * kappa / (eps_h * cs * cs * L * L)))
    g = 28.0 * Ra_eff * nu * kappa / (dT * L ** 3)
    return dict(dT=dT, g=g, Ra=Ra_eff, Ra_requested=float(Ra), clamped=Ra_eff < Ra,
                hydro=g * L / (cs * cs), mach=(Ra_eff / Pr) ** 0.5 * nu / (L * cs))


def cavity_dT_cap(L: int, grad_max: float = 1.5e-3, dT_abs_max: float = 0.6) -> float:
    """Largest wall temperature difference a cavity of side L of the batched
    workload may use: at most 0.6 (wall energies within E0 +- 0.3, the range in
    which the parameter sets were scanned) and at most grad_max L (a mean wall
    gradient of 1.5e-3 per node).  Anti-bounce-back walls let mass through in
    proportion to the wall temperature jump, and cavities with a larger jump
    per node drift and then diverge: with the cap every cavity of the 64-cavity
    batch stays finite with its mean density within 2 % over 10^5 steps, while
    dT = 1 on a 67^2 cavity diverges after about 1.1 x 10^4."""
    return min(dT_abs_max, grad_max * L)


def channel_viscosity(W: int, F: float, u_max: float = 0.05, nu_lo: float = 0.0625, nu_hi: float = 0.25):
    """Viscosity for a Poiseuille channel of width W under force F so that the
    steady centre-line speed F W^2 / (8 nu) stays <= u_max; nu is clamped to
    [nu_lo, nu_hi] (the linearly stable range of the default parameter set) and
    F is lowered when even nu_hi is not enough (`clamped`)."""
    nu = min(nu_hi, max(nu_lo, F * W * W / (8.0 * u_max)))
    F_eff = min(F, 8.0 * nu * u_max / (W * W))
    return dict(nu=nu, F=F_eff, clamped=F_eff < F)


def s_xx_for_nu(nu: float, A: float = 52.0) -> float:
    """Relaxation rate s_XX giving shear viscosity nu = (1/s_XX - 1/2) A / 104
    for A = 13 c1 + 95 + 2 E0 (the default set has A = 52)."""
    return 1.0 / (nu * 104.0 / A + 0.5)


# Free-parameter sets (the paper prints none: sec. 2 chooses them from the roots
# of the linear dispersion relation over wave vectors of magnitude 0..2 pi, which
# is how these were found).  LOW_PR (the default): linearly stable for Pr <= 1,
# s_XX <= 1.6, |u| <= 0.05.  HIGH_PR: stable for Pr in [0.5, 7], s_XX <= 1.5,
# |u| <= 0.05, energy offsets |E - E0| <= 0.3.  The CPU test suite re-checks
# these claims and those of the cavity sets below.
LOW_PR_SET = dict(E0=-2.0, c1=-3.0, k2=-2.5, c_epsE=-2.5, c_varpi_rho=-6.0, c_varpi_E=-0.5,
                  s_rx=1.05, s_eps=1.0, s_varpi=1.0, s_XXe=1.5)
HIGH_PR_SET = dict(E0=-0.22, c1=-3.11, k2=-1.78, c_epsE=-3.77, c_varpi_rho=-0.98, c_varpi_E=-0.09,
                   s_rx=0.92, s_eps=0.91, s_varpi=1.29, s_XXe=1.75)


# Free parameters for the heated cavity at Pr = 0.71 with s_XX = 1.9 (nu = 0.0144,
# cs^2 = 1.097): found by the same search of the linear dispersion relation,
# run for Pr = 0.71 and s_XX = 1.9 over random draws of the ten other free
# parameters (linearly stable for |u| <= 0.07 and energy offsets up to 0.1;
# unstable at other Prandtl numbers), then kept because the 256^2 cavity at
# Ra = 1e3 to 1e6 runs with it for 6 x 10^5 steps with the mean density within
# 0.7 % (the default set at s_XX = 1.7 gains 8 % at Ra = 1e5 over 1.2 x 10^6
# steps).  Its lower viscosity lets the feasible forcing use a ten times smaller
# wall temperature difference at Ra = 1e5 (dT = 0.057 against 0.59), and the
# anti-bounce-back walls exchange correspondingly less mass.
CAVITY_PR071_SET = dict(E0=0.275, c1=-2.962, k2=0.697, c_epsE=1.384, c_varpi_rho=-0.553, c_varpi_E=-0.143,
                        s_rx=0.453, s_eps=1.192, s_varpi=1.268, s_XXe=1.372, s_XX=1.9, Pr=0.71)


# Free parameters for the batched cavities (every Pr in [0.5, 7]) with s_XX =
# 1.8 (nu = 0.0256, cs^2 = 0.920): the same search run over Pr = 1, 2, 4, 7 at
# once (linearly stable for Pr in [0.5, 7], |u| <= 0.07 and energy offsets up
# to 0.3); kept because the 64-cavity batch runs 1.2 x 10^5 steps with every
# mean density within 0.2 %, and its lower viscosity leaves 5 of the 64
# cavities with a lowered Ra instead of 20 (with LOW_PR_SET at s_XX = 1.6 for
# Pr <= 1 and HIGH_PR_SET at s_XX = 1.5 above).
CAVITY_BATCH_SET = dict(E0=-2.812, c1=-3.194, k2=-0.947, c_epsE=-5.399, c_varpi_rho=-3.717, c_varpi_E=0.203,
                        s_rx=0.948, s_eps=0.617, s_varpi=1.453, s_XXe=1.411)


def cavity_parameter_set(Pr: float) -> dict:
    """Free parameters for a cavity of the batched workload at Prandtl number Pr."""
    return dict(CAVITY_BATCH_SET, Pr=float(Pr), s_XX=1.8)
