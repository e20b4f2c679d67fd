"""Analytic start-up solutions for channels between walls at xi = 0 and xi = W
(halfway walls: xi = x + 1/2), used by the channel tests (secs. 7, 8)."""
import numpy as np


def startup_couette(xi, W, U, nu, t, terms=400):
    n = np.arange(1, terms + 1)[:, None]
    return U * (1 - xi / W) - (2 * U / np.pi) * (np.sin(n * np.pi * xi / W) / n *
                                                 np.exp(-nu * (n * np.pi / W) ** 2 * t)).sum(0)


def startup_poiseuille(xi, W, F, nu, t, terms=401):
    n = np.arange(1, terms + 1, 2)[:, None]
    return F * xi * (W - xi) / (2 * nu) - (4 * F * W ** 2 / (nu * np.pi ** 3) * np.sin(n * np.pi * xi / W) / n ** 3 *
                                            np.exp(-nu * (n * np.pi / W) ** 2 * t)).sum(0)


def startup_conduction(xi, W, T0, dT, kappa, t, terms=400):
    n = np.arange(2, terms + 1, 2)[:, None]
    return T0 + dT * (1 - 2 * xi / W) - dT * (4 / (n * np.pi) * np.sin(n * np.pi * xi / W) *
                                             np.exp(-kappa * (n * np.pi / W) ** 2 * t)).sum(0)
