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

// Reductions over the 64 lanes of a wave in a fixed order, by DPP moves (no
// LDS round trip): inclusive scans within each row of 16 lanes (row_shr by
// 1, 2, 4, 8), then lane 15 into row 1 and lane 47 into row 3 (row_bcast:15),
// then lane 31 into rows 2 and 3 (row_bcast:31); lane 63 ends with the
// result, which every lane receives.  Lanes that receive nothing get 0, the
// identity of both the sum and the max of non-negative bit patterns.  The
// whole wave must be active.  GFX9 DPP controls: row_shr:n = 0x110 + n,
// row_bcast:15 = 0x142, row_bcast:31 = 0x143.
template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned long long dpp64(unsigned long long v) {
    return (unsigned long long)__builtin_amdgcn_update_dpp((long long)0, (long long)v, CTRL, ROWS, 0xF, true);
}

__device__ __forceinline__ unsigned long long lane63(unsigned long long v) {
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)v, 63);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(v >> 32), 63);
    return ((unsigned long long)hi << 32) | lo;
}

template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_add(double x) {
    return x + __longlong_as_double((long long)dpp64<CTRL, ROWS>(dbits(x)));
}

__device__ __forceinline__ double wave_sum64d(double x) {
    x = dpp_add<0x111, 0xF>(x);
    x = dpp_add<0x112, 0xF>(x);
    x = dpp_add<0x114, 0xF>(x);
    x = dpp_add<0x118, 0xF>(x);
    x = dpp_add<0x142, 0xA>(x);
    x = dpp_add<0x143, 0xC>(x);
    return __longlong_as_double((long long)lane63(dbits(x)));
}

template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned long long dpp_max(unsigned long long x) {
    const unsigned long long y = dpp64<CTRL, ROWS>(x);
    return y > x ? y : x;
}

__device__ __forceinline__ unsigned long long wave_max64(unsigned long long x) {
    x = dpp_max<0x111, 0xF>(x);
    x = dpp_max<0x112, 0xF>(x);
    x = dpp_max<0x114, 0xF>(x);
    x = dpp_max<0x118, 0xF>(x);
    x = dpp_max<0x142, 0xA>(x);
    x = dpp_max<0x143, 0xC>(x);
    return lane63(x);
}

// Fixed-order reduction of DiagVals over a block of 256 threads (four
// waves): each wave reduces every value, then thread 0 combines the four
// waves in order.  Thread 0 receives the result.
__device__ __forceinline__ DiagVals block_reduce_diag(const DiagVals &v) {
    constexpr int NV = kDiagSums + kDiagMaxes;
    __shared__ double sh[NV][4];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    double sm[kDiagSums];
    unsigned long long mx[kDiagMaxes];
#pragma unroll
    for (int k = 0; k < kDiagSums; ++k) sm[k] = wave_sum64d(v.sum[k]);
#pragma unroll
    for (int k = 0; k < kDiagMaxes; ++k) mx[k] = wave_max64(v.mx[k]);
    if (l == 0) {
#pragma unroll
        for (int k = 0; k < kDiagSums; ++k) sh[k][w] = sm[k];
#pragma unroll
        for (int k = 0; k < kDiagMaxes; ++k) sh[kDiagSums + k][w] = __longlong_as_double((long long)mx[k]);
    }
    __syncthreads();
    DiagVals r{};
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < kDiagSums; ++k) r.sum[k] = ((sh[k][0] + sh[k][1]) + sh[k][2]) + sh[k][3];
#pragma unroll
        for (int k = 0; k < kDiagMaxes; ++k) {
            unsigned long long x = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const unsigned long long y = dbits(sh[kDiagSums + k][q]);
                x = y > x ? y : x;
            }
            r.mx[k] = x;
        }
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
