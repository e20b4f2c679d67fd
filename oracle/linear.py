"""Linear (von Neumann) analysis of the D2Q13 scheme, in NumPy.

TEST INFRASTRUCTURE ONLY.  Sec. 2 of the paper chooses the free parameters by
computing the roots of the linear dispersion relation for wave vectors of
magnitude 0..2pi in several directions.  This module builds the amplification
matrix of one time step linearised about a uniform state,

    A(k) = diag(exp(-i k.v_j)) M^-1 (I - S (I - J)) M,

where J is the Jacobian of the equilibrium moments (eq d2q13-moments-equil) with
respect to the conserved moments (rho, E, jx, jy), and S the diagonal of
relaxation rates.  Its eigenvalues give the exact per-step damping and phase of
every linear mode at finite k; they are what small-amplitude oracle runs must
reproduce.  The moment matrix is rebuilt here in floating point directly from the
polynomials of eq (d2q13-polynomes), independently of the C oracle; only the
derived coefficients come from the oracle.
"""
from __future__ import annotations

import numpy as np

import oracle

VEL = np.array([(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1),
                (2, 0), (0, 2), (-2, 0), (0, -2)], dtype=float)


def moment_matrix() -> np.ndarray:
    x, y = VEL[:, 0], VEL[:, 1]
    r = x * x + y * y
    rows = [np.ones(13), -28 + 13 * r, 140 + r * (-361 / 2 + 77 / 2 * r),
            -12 + r * (581 / 12 + r * (-273 / 8 + 137 / 24 * r)), x, y, x * (r - 3), y * (r - 3),
            x * (101 / 6 + r * (-63 / 4 + 35 / 12 * r)), y * (101 / 6 + r * (-63 / 4 + 35 / 12 * r)),
            x * x - y * y, x * y, (x * x - y * y) * (-65 / 12 + 17 / 12 * r)]
    return np.round(np.array(rows))


def _meq(m, p, d):
    rho, E, jx, jy = m[0], m[1], m[4], m[5]
    out = m.copy()
    out[2] = d["c_eps_rho"] * rho + p.c_epsE * E
    out[3] = p.c_varpi_rho * rho + p.c_varpi_E * E
    a = p.c1 + d["h1"] * rho + d["k1"] * E
    b = d["c2"] + d["h2"] * rho + p.k2 * E
    out[6], out[7], out[8], out[9] = jx * a, jy * a, jx * b, jy * b
    out[10] = (jx * jx - jy * jy) / rho
    out[11] = jx * jy / rho
    out[12] = 0.0
    return out


def amplification(p, k, U=(0.0, 0.0), rho=1.0, E=None, derived=None):
    """Amplification matrix for wave vector k about (rho, j = rho U, E).

    `derived` replaces the oracle's derived coefficients (h1, k1, h2, c2, ...)
    when given.  The Jacobian is taken by a complex step (the equilibria are
    rational in the conserved moments), exact to rounding."""
    d = oracle.derive(p)[1] if derived is None else derived
    M = moment_matrix()
    D = (M * M).sum(1)
    Minv = M.T / D
    if E is None:
        E = p.E0
    m0 = np.zeros(13, dtype=complex)
    m0[0], m0[1], m0[4], m0[5] = rho, E, rho * U[0], rho * U[1]
    J = np.zeros((13, 13))
    h = 1e-30
    for c in (0, 1, 4, 5):
        e = np.zeros(13, dtype=complex)
        e[c] = 1j * h
        J[:, c] = _meq(m0 + e, p, d).imag / h
    s = np.array([0, 0, p.s_eps, p.s_varpi, 0, 0, d["s_q"], d["s_q"], p.s_rx, p.s_rx,
                  p.s_XX, p.s_XX, p.s_XXe])
    C = Minv @ (np.eye(13) - np.diag(s) @ (np.eye(13) - J)) @ M
    ph = np.exp(-1j * (VEL @ np.asarray(k, dtype=float)))
    return ph[:, None] * C


def hydro_modes(p, k, U=(0.0, 0.0)):
    """The four least-damped eigenvalues (hydrodynamic modes) as (damping/step, phase/step)."""
    lam = np.linalg.eigvals(amplification(p, k, U))
    lam = sorted(lam, key=lambda z: -abs(z))[:4]
    return [(-np.log(abs(z)), np.angle(z)) for z in lam]


def max_amplification(p, n=33, U=(0.0, 0.0)) -> float:
    """max |lambda| over a grid of the wedge 0 <= ky <= kx <= pi (the zone's symmetric part)."""
    worst = 0.0
    for kx in np.linspace(0.0, np.pi, n):
        for ky in np.linspace(0.0, kx, n):
            worst = max(worst, float(np.abs(np.linalg.eigvals(amplification(p, (kx, ky), U))).max()))
    return worst
