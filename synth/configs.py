"""Seeded synthetic workloads (meshes, particles, initial fields).

  cavity  : PEC pillbox, rho in [0, 1 cm], z in [0, 2 cm], ~2,000 faces;
            TM010 field (E0 = 1 MV/m); 10,000 electrons (weight 1e4) uniform
            in volume in rho < 2 mm with v_z = 0.5 c.
  diode   : planar gap z in [0, 1 cm], rho in [0, 5 cm], ~20,000 faces;
            cathode z = 0 (emitting for rho < 2 cm), anode z = 1 cm,
            free outer boundary; 100 kV applied as a uniform E_z.
  bwo     : rippled-wall tube R(z) = 1.5 cm + 0.25 cm sin(2 pi (z - z0)/1.67 cm)
            over 10 periods (amplitude ramped over the first and last half
            period) between a 2 cm upstream and a 3 cm downstream drift of
            radius 1.5 cm; ~200,000 faces; PEC wall and end plates; annular
            500 keV beam r in [0.9, 1.1] cm, ~8M macro-electrons; B_z = 1 T.
  variant : one member of the batched sweep (ripple amplitude 0.1-0.4 cm,
            period 1.2-2.0 cm, taper 0-30 %, beam 300-600 keV, 20k-300k faces,
            ~25 particles per face).
"""

from __future__ import annotations

import numpy as np

from .meshes import rect_mesh, rippled_mesh, BC_PEC, BC_AXIS, BC_EMITTER, BC_OPEN
from .particles import ELECTRON_CHARGE, ELECTRON_MASS, C_LIGHT, disk_beam, annular_beam, gamma_beta_from_kev

CAVITY_A = 0.01
CAVITY_H = 0.02
CAVITY_DT = 1.87e-13          # 0.5 x leapfrog limit of the cavity mesh (3.743e-13 s)


def cavity_mesh(seed=0, h=0.49e-3):
    return rect_mesh(0.0, CAVITY_H, CAVITY_A, h, seed=seed)


def cavity_beam(n=10000, seed=1):
    zr, u = disk_beam(n, 0.002, 0.0, CAVITY_H, 0.5, seed)
    return zr, u


CAVITY_WEIGHT = 10000


def diode_mesh(seed=0, h=0.24e-3, emitter_radius=0.02):
    def tag(side, z, r):
        if side == "bottom":
            return BC_AXIS
        if side == "left":
            return BC_EMITTER if r < emitter_radius else BC_PEC
        if side == "right":
            return BC_PEC
        return BC_OPEN
    return rect_mesh(0.0, 0.01, 0.05, h, seed=seed, tags=tag)


DIODE_VOLTS = 1.0e5
DIODE_GAP = 0.01


def bwo_radius_fn(amp=0.0025, period=0.0167, n_periods=10, r0=0.015, up=0.02, taper=0.0):
    z0 = up
    z1 = up + n_periods * period

    def R(z):
        z = np.asarray(z, dtype=np.float64)
        x = (z - z0) / period
        env = np.clip(x * 2.0, 0.0, 1.0) * np.clip((n_periods - x) * 2.0, 0.0, 1.0)
        env = 0.5 - 0.5 * np.cos(np.pi * env)               # raised-cosine ramp over half a period
        a = amp * (1.0 - taper * np.clip(x / n_periods, 0.0, 1.0))
        inside = (z > z0) & (z < z1)
        return r0 + np.where(inside, a * env * np.sin(2 * np.pi * x), 0.0)

    return R, z1


def bwo_mesh(seed=3, h=0.19e-3, amp=0.0025, period=0.0167, n_periods=10, taper=0.0, up=0.02, down=0.03,
             emitter=None):
    """The rippled-wall tube; emitter=(r_in, r_out) tags that annulus of the
    upstream end plate as an emitting conductor (the beam's replenishment)."""
    R, z1 = bwo_radius_fn(amp, period, n_periods, 0.015, up, taper)
    L = z1 + down
    tags = None
    if emitter is not None:
        r_in, r_out = emitter

        def tags(side, z, rho):
            if side == "bottom":
                return BC_AXIS
            if side == "left" and r_in <= rho <= r_out:
                return BC_EMITTER
            return BC_PEC
    return rippled_mesh(R, 0.0, L, h, seed=seed, tags=tags,
                        meta=dict(amp=amp, period=period, n_periods=n_periods, taper=taper, length=L))


BWO_BZ = 1.0
BWO_KEV = 500.0


def bwo_beam(n, length, kev=BWO_KEV, seed=3, r_in=0.009, r_out=0.011):
    return annular_beam(n, r_in, r_out, 0.0005, length - 0.0005, kev, seed)


def bwo_weight(n, length, kev=BWO_KEV, current=1500.0):
    """Integer weight giving the stated beam current for n macro-electrons."""
    g, b = gamma_beta_from_kev(kev)
    charge = current * length / (b * C_LIGHT)
    return max(1, int(round(charge / (n * abs(ELECTRON_CHARGE)))))


def variant_params(i):
    """Parameters of member i (0..63) of the batched sweep (seeded)."""
    rng = np.random.default_rng(7000 + i)
    return dict(amp=float(rng.uniform(0.001, 0.004)), period=float(rng.uniform(0.012, 0.020)),
                taper=float(rng.uniform(0.0, 0.3)), kev=float(rng.uniform(300.0, 600.0)),
                faces=int(rng.uniform(20000, 300000)), seed=2000 + i)


def variant_mesh(i):
    p = variant_params(i)
    length = 0.02 + 10 * p["period"] + 0.03
    area = length * 0.015
    h = np.sqrt(4 * area / np.sqrt(3) / p["faces"])
    return bwo_mesh(seed=p["seed"], h=h, amp=p["amp"], period=p["period"], taper=p["taper"]), p
