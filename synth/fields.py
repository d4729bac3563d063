"""Analytic initial fields projected onto mesh cells by plain quadrature.

Edge values are line integrals of E along each edge from its tail node to its
head node (the pairing of a 1-form with an oriented edge); face values are
area integrals of B_phi over each counter-clockwise (z, rho) triangle (the
pairing of a 2-form with an oriented face).  Only quadrature lives here.
"""

from __future__ import annotations

import numpy as np
import scipy.special

from .particles import C_LIGHT

# first zero of J0, used for the TM010 mode of a pillbox of radius a
J0_FIRST_ZERO = 2.404825557695773


def _gauss01(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def edge_line_integrals(nodes, edges, field_fn, n=8):
    """int_tail^head E . dl for every edge; field_fn(z, rho) -> (E_z, E_rho)."""
    x, w = _gauss01(n)
    a = nodes[edges[:, 0]]
    b = nodes[edges[:, 1]]
    d = b - a
    pts = a[:, None, :] + x[None, :, None] * d[:, None, :]
    ez, er = field_fn(pts[..., 0], pts[..., 1])
    integrand = ez * d[:, None, 0] + er * d[:, None, 1]
    return integrand @ w


def face_flux_integrals(nodes, tris, fn, n=6):
    """int_T fn(z, rho) dA for every triangle, by a collapsed (Duffy) product
    Gauss rule: exact for polynomials of degree <= 2n-2."""
    x, w = _gauss01(n)
    p = nodes[tris]
    v0, v1, v2 = p[:, 0], p[:, 1], p[:, 2]
    twice_area = ((v1[:, 0] - v0[:, 0]) * (v2[:, 1] - v0[:, 1])
                  - (v2[:, 0] - v0[:, 0]) * (v1[:, 1] - v0[:, 1]))
    total = np.zeros(len(tris))
    for xu, wu in zip(x, w):
        for xv, wv in zip(x, w):
            l1 = xu
            l2 = (1.0 - xu) * xv
            l0 = 1.0 - l1 - l2
            q = l0[..., None] * v0 + l1 * v1 + l2 * v2 if np.ndim(l0) else l0 * v0 + l1 * v1 + l2 * v2
            total += wu * wv * (1.0 - xu) * fn(q[:, 0], q[:, 1])
    return total * twice_area


def uniform_field_dofs(nodes, edges, e_z, e_rho):
    """Edge values of a uniform field: E0 . (r_head - r_tail), exact."""
    d = nodes[edges[:, 1]] - nodes[edges[:, 0]]
    return d[:, 0] * e_z + d[:, 1] * e_rho


def tm010_fields(nodes, tris, edges, a, e0, dt):
    """TM010 standing wave of a pillbox of radius a at t = 0 (E) and
    t = -dt/2 (B):  E_z = e0 J0(k rho) cos(w t),
    B_phi = -(e0/c) J1(k rho) sin(w t),  k = 2.4048/a,  w = c k.

    Returns (E edge values at t=0, B face fluxes at t=-dt/2, omega)."""
    k = J0_FIRST_ZERO / a
    omega = C_LIGHT * k
    E = edge_line_integrals(nodes, edges,
                            lambda z, r: (e0 * scipy.special.j0(k * r), np.zeros_like(r)))
    s = np.sin(omega * (-0.5 * dt))
    B = face_flux_integrals(nodes, tris, lambda z, r: -(e0 / C_LIGHT) * scipy.special.j1(k * r) * s)
    return E, B, omega
