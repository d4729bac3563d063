// Reductions of the diagnostics shared by the two precisions' kernels
// (device code only).
#pragma once

#include <hip/hip_runtime.h>

#include "device.h"

namespace axp {

__device__ __forceinline__ unsigned long long dbits(double v) { return (unsigned long long)__double_as_longlong(v); }

// Partials of an evaluation.  Each node-pass block also takes a fixed slice
// of the step's particle-kernel, face-pass and edge-pass partials, so the
// final reduction only sees one partial per node-pass block.  Reductions run
// in a fixed order.  Maxima are bit patterns of non-negative doubles (the
// mixed continuity residual: an integer): 0 drift, 1 |res|, 2 scale, 3 dce,
// 4 qmax.
enum {
    kSumQ = 0,          // total charge of the evaluated level
    kSumWEnow = 1,      // 1/2 E D of the evaluated level
    kSumWE = 2,         // energy record of the step's start level: 1/2 E^n D^n (edge pass)
    kSumWB = 3,         //   1/2 B^{n+1/2} H B^{n-1/2} (face pass)
    kSumWK = 4,         //   1/2 (K^{n-1/2} + K^{n+1/2}) (particle kernel)
    kSumLiveStart = 5,  //   live particles at the start level
    kSumLiveNow = 6,    // live particles at the evaluated level
    kDiagSums = 7,
    kDiagMaxes = 5
};
static_assert(kDiagSums + kDiagMaxes <= kDiagSlots, "partial slots");

struct DiagVals {
    double sum[kDiagSums];
    unsigned long long mx[kDiagMaxes];
};

// Adds this block's slices of the particle partials (3 per particle block:
// W_K, live at the start, live at the end; on demand only the last is
// written), the face partials and the edge partials to v.
__device__ __forceinline__ void fold_slices(const DevState &s, DiagVals &v, int in_step, int nb_face, int nb_edge,
                                            int nb_node) {
    const long long ns = (long long)s.ctr->n_slots;
    const int nb_part = (int)((ns + 1023) / 1024);
    const int kp = (nb_part + nb_node - 1) / nb_node;
    for (int i = threadIdx.x; i < kp; i += blockDim.x) {
        const int b = blockIdx.x * kp + i;
        if (b < nb_part) {
            if (in_step) {
                v.sum[kSumWK] += s.part_kin[3 * b];
                v.sum[kSumLiveStart] += s.part_kin[3 * b + 1];
            }
            v.sum[kSumLiveNow] += s.part_kin[3 * b + 2];
        }
    }
    if (!in_step) return;
    const int kf = (nb_face + nb_node - 1) / nb_node;
    for (int i = threadIdx.x; i < kf; i += blockDim.x) {
        const int b = blockIdx.x * kf + i;
        if (b < nb_face) v.sum[kSumWB] += s.part_face[b];
    }
    const int ke = (nb_edge + nb_node - 1) / nb_node;
    for (int i = threadIdx.x; i < ke; i += blockDim.x) {
        const int b = blockIdx.x * ke + i;
        if (b < nb_edge) v.sum[kSumWE] += s.part_edge[b];
    }
}

// Butterfly over the 64 lanes of a wave (fixed order): sum, and max of bit patterns.
__device__ __forceinline__ double wave_sum64d(double x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    return x;
}

__device__ __forceinline__ unsigned long long wave_max64(unsigned long long x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const unsigned long long o = __shfl_xor(x, off, 64);
        x = o > x ? o : x;
    }
    return x;
}

// Fixed-order reduction of DiagVals over a block of 256 threads: the values
// are staged in LDS, each wave reduces whole slots (four entries per lane in
// order, then a butterfly).  Thread 0 receives the result.
__device__ __forceinline__ DiagVals block_reduce_diag(const DiagVals &v) {
    constexpr int NV = kDiagSums + kDiagMaxes;
    __shared__ double sh[NV][256];
    __shared__ double res[NV];
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < kDiagSums; ++k) sh[k][t] = v.sum[k];
#pragma unroll
    for (int k = 0; k < kDiagMaxes; ++k) sh[kDiagSums + k][t] = __longlong_as_double((long long)v.mx[k]);
    __syncthreads();
    const int w = t >> 6, l = t & 63;
    for (int k = w; k < NV; k += 4) {                 // wave-uniform
        if (k < kDiagSums) {
            const double x = wave_sum64d(((sh[k][l] + sh[k][l + 64]) + sh[k][l + 128]) + sh[k][l + 192]);
            if (l == 0) res[k] = x;
        } else {
            unsigned long long x = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const unsigned long long y = dbits(sh[k][l + 64 * q]);
                x = y > x ? y : x;
            }
            x = wave_max64(x);
            if (l == 0) res[k] = __longlong_as_double((long long)x);
        }
    }
    __syncthreads();
    DiagVals r{};
    if (t == 0) {
#pragma unroll
        for (int k = 0; k < kDiagSums; ++k) r.sum[k] = res[k];
#pragma unroll
        for (int k = 0; k < kDiagMaxes; ++k) r.mx[k] = dbits(res[kDiagSums + k]);
    }
    return r;
}

// Stores a block's partials slot-major (slot k of block b at k * nb + b), so
// the final reduction reads each slot with coalesced loads.
__device__ __forceinline__ void store_partials(double *part, int b, int nb, const DiagVals &r) {
#pragma unroll
    for (int k = 0; k < kDiagSums; ++k) part[(size_t)k * nb + b] = r.sum[k];
#pragma unroll
    for (int k = 0; k < kDiagMaxes; ++k) part[(size_t)(kDiagSums + k) * nb + b] = __longlong_as_double((long long)r.mx[k]);
}

}  // namespace axp
