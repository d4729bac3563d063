"""Continuous emission from emitter edges, FP64 (reading of the injection
step of the diode / gun configurations, Sec. 4).

TEST INFRASTRUCTURE ONLY (see the package header).

Each step starts by placing per_step macro-particles on the emitter edges
(boundary edges tagged EMITTER), uniformly per unit area of the emitting
surface of revolution: an edge with probability proportional to its length
times its mean radius, a point on it with density proportional to rho.  The
particle takes its charge from the wall charge of the edge's two nodes in
proportion to its barycentric coordinates, so nodal charge is unchanged by
the emission.  Momentum u_mean + u_spread * U[-1, 1]^3 in the frame
(tangent tail -> head, phi, inward normal).

Random numbers: draw d of particle i at step n is output
c = 2^32 n + 8 i + d + 1 of SplitMix64 (Steele, Lea and Flood, 2014) with
the given seed: z = seed + c * 0x9E3779B97F4A7C15, then the generator's
output mix, as (z >> 11) * 2^-53.
"""

from __future__ import annotations

import numpy as np

from .topology import EMITTER

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, c):
    """Output number c (uint64 array, c >= 1) of SplitMix64 seeded with seed."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + np.asarray(c, dtype=np.uint64) * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def uniform(seed, c):
    return (splitmix64(seed, c) >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


class Emitter:
    def __init__(self, topo):
        edges = np.flatnonzero(topo.edge_tag == EMITTER)          # canonical order
        nodes = topo.nodes
        # the face next to each boundary edge
        face = np.full(topo.n1, -1, dtype=np.int64)
        for t in range(topo.n2):
            for e in topo.tri_edges[t]:
                face[e] = t
        self.edges = edges
        self.tail = topo.edges[edges, 0]
        self.head = topo.edges[edges, 1]
        za, ra = nodes[self.tail, 0], nodes[self.tail, 1]
        zb, rb = nodes[self.head, 0], nodes[self.head, 1]
        dz, dr = zb - za, rb - ra
        length = np.sqrt(dz * dz + dr * dr)
        self.weight_cdf = np.cumsum(length * (ra + rb) * 0.5)
        self.ra, self.rb = ra, rb
        self.za, self.zb = za, zb
        self.t = np.stack([dz / length, dr / length], axis=1)            # (z, rho)
        self.face = face[edges]
        n = np.stack([-self.t[:, 1], self.t[:, 0]], axis=1)
        tri = topo.tris[self.face]
        opp = np.array([[v for v in tri[q] if v != self.tail[q] and v != self.head[q]][0] for q in range(len(edges))])
        to_opp = nodes[opp] - nodes[self.tail]
        flip = (n * to_opp).sum(axis=1) < 0
        n[flip] *= -1.0
        self.n = n

    def emit(self, step, per_step, seed, u_mean, u_spread):
        """Returns (z, rho, face, u[k][3] = (u_rho, u_phi, u_z), weight of the tail node)."""
        i = np.arange(per_step, dtype=np.uint64)
        c0 = (np.uint64(step) << np.uint64(32)) + np.uint64(8) * i + np.uint64(1)
        u0, u1 = uniform(seed, c0), uniform(seed, c0 + np.uint64(1))
        x = u0 * self.weight_cdf[-1]
        e = np.searchsorted(self.weight_cdf, x, side="right")
        ra, rb = self.ra[e], self.rb[e]
        # inverse of the rho-weighted distribution along the edge
        s = u1 * (ra + rb) / (ra + np.sqrt(ra * ra + (rb - ra) * u1 * (ra + rb)))
        s = np.clip(s, 0.0, 1.0)
        z = self.za[e] + s * (self.zb[e] - self.za[e])
        rho = ra + s * (rb - ra)
        ut = u_mean[0] + u_spread * (2.0 * uniform(seed, c0 + np.uint64(2)) - 1.0)
        uph = u_mean[1] + u_spread * (2.0 * uniform(seed, c0 + np.uint64(3)) - 1.0)
        un = u_mean[2] + u_spread * (2.0 * uniform(seed, c0 + np.uint64(4)) - 1.0)
        tz, tr = self.t[e, 0], self.t[e, 1]
        nz, nr = self.n[e, 0], self.n[e, 1]
        u = np.stack([ut * tr + un * nr, uph, ut * tz + un * nz], axis=1)
        return z, rho, self.face[e], u, self.tail[e], self.head[e], 1.0 - s
