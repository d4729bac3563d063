// Continuous emission from emitter edges: counter-based random draws and
// the sampling of an emission point and momentum (shared by both steps).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "device.h"

namespace axp {

// Output number c (c >= 1) of the SplitMix64 generator seeded with `seed`
// (Steele, Lea and Flood, OOPSLA 2014): mix(seed + c * golden gamma), as a
// uniform double in [0, 1).  Draw d of particle i at step n uses
// c = 2^32 n + 8 i + d + 1.
__device__ __forceinline__ double splitmix_uniform(unsigned long long seed, unsigned long long c) {
    unsigned long long z = seed + c * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

struct Emission {
    int e;                     // emitter edge
    double s;                  // position tail -> head in [0, 1]
    double ur, up, uz;         // momentum / c, (rho, phi, z)
};

// Edge by inverse CDF of the weights, position with density proportional
// to rho along the edge (uniform per unit area of the emitting surface of
// revolution), momentum uniform in a box around the mean.
__device__ __forceinline__ Emission sample_emission(const EmitEdge *ee, const InjParams &p, unsigned long long step,
                                                    int i) {
    const unsigned long long c0 = (step << 32) + 8ull * (unsigned long long)i + 1ull;
    const double u0 = splitmix_uniform(p.seed, c0), u1 = splitmix_uniform(p.seed, c0 + 1);
    const double x = u0 * p.total;
    int lo = 0, hi = p.n_edges - 1;          // first edge with cdf > x
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (ee[mid].cdf > x) hi = mid;
        else lo = mid + 1;
    }
    const EmitEdge &E = ee[lo];
    const double ra = E.ra, rb = E.rb;
    // solve (ra s + (rb - ra) s^2 / 2) / ((ra + rb) / 2) = u1 without cancellation
    const double s = u1 * (ra + rb) / (ra + sqrt(ra * ra + (rb - ra) * u1 * (ra + rb)));
    Emission em;
    em.e = lo;
    em.s = fmin(fmax(s, 0.0), 1.0);
    const double ut = p.um[0] + p.spread * (2.0 * splitmix_uniform(p.seed, c0 + 2) - 1.0);
    const double uph = p.um[1] + p.spread * (2.0 * splitmix_uniform(p.seed, c0 + 3) - 1.0);
    const double un = p.um[2] + p.spread * (2.0 * splitmix_uniform(p.seed, c0 + 4) - 1.0);
    em.uz = ut * E.tz + un * E.nz;
    em.ur = ut * E.tr + un * E.nr;
    em.up = uph;
    return em;
}

}  // namespace axp
