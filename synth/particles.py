"""Seeded particle initial conditions (positions and momenta).

Momenta are u = gamma * v in m/s, given in the local cylindrical basis
(u_rho, u_phi, u_z) at each particle's position.
"""

from __future__ import annotations

import numpy as np

C_LIGHT = 299792458.0
EPS0 = 8.8541878128e-12
MU0 = 1.0 / (EPS0 * C_LIGHT * C_LIGHT)
ELECTRON_CHARGE = -1.602176634e-19
ELECTRON_MASS = 9.1093837015e-31
ELECTRON_REST_KEV = ELECTRON_MASS * C_LIGHT ** 2 / 1.602176634e-16


def gamma_beta_from_kev(kev):
    """(gamma, beta) of an electron of kinetic energy kev."""
    g = 1.0 + kev / ELECTRON_REST_KEV
    return g, np.sqrt(1.0 - 1.0 / g ** 2)


def disk_beam(n, rho_max, z0, z1, beta, seed):
    """n particles uniform in volume inside rho < rho_max, z0 < z < z1,
    moving along +z with speed beta*c.  Returns (zr (n,2), u (n,3))."""
    rng = np.random.default_rng(seed)
    rho = rho_max * np.sqrt(rng.uniform(0.0, 1.0, n))
    z = rng.uniform(z0, z1, n)
    g = 1.0 / np.sqrt(1.0 - beta * beta)
    u = np.zeros((n, 3))
    u[:, 2] = g * beta * C_LIGHT
    return np.stack([z, rho], axis=1), u


def annular_beam(n, r_in, r_out, z0, z1, kev, seed):
    """n particles uniform in volume in r_in < rho < r_out, z0 < z < z1,
    moving along +z with kinetic energy kev."""
    rng = np.random.default_rng(seed)
    rho = np.sqrt(rng.uniform(r_in * r_in, r_out * r_out, n))
    z = rng.uniform(z0, z1, n)
    g, b = gamma_beta_from_kev(kev)
    u = np.zeros((n, 3))
    u[:, 2] = g * b * C_LIGHT
    return np.stack([z, rho], axis=1), u


def random_momenta(n, u_scale, seed):
    """Isotropic-ish random momenta with |u| up to u_scale (for tests)."""
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, u_scale / np.sqrt(3.0), (n, 3))
