// Mixed-precision HIP kernels of one time step (gfx950, wave64).
//
//   k_tri_pass    Faraday update of face fluxes, eq. (full_d_dfl), and the
//                 per-face gather tile of the Whitney expansions (Sec. 3.2).
//   k_particles   gather + relativistic Boris (eqs. DNE, DLE) + axisymmetric
//                 position update + walk across faces with the charge-
//                 conserving edge current of eq. (current), in 64-bit
//                 fixed point on element-local coordinates.
//   k_edge_pass   D += dt C^T H B^{n+1/2} - dt J (eq. full_d_dal, D-form).
//   k_spmv        E = M D with the SPAI matrix in sliced ELL (FP32).
//   sort          counting sort of particles by face (compacts the dead).
//   diagnostics   nodal charge, discrete continuity (eq. DCE), Gauss-law
//                 residual (eq. DGL_RSD_REL), energies.
//
// Element-local positions: a particle is (face T, Lambda_0, Lambda_1) with
// Lambda_k = lambda_k 2^23 exactly (Lambda_2 = 2^23 - Lambda_0 - Lambda_1).
// A straight piece of path from Lambda^s to Lambda^e inside T contributes
// Lambda^s_{k+1} Lambda^e_{k+2} - Lambda^s_{k+2} Lambda^e_{k+1} (units 2^-46)
// to the current of side k (oriented from local node k+1 to k+2); the
// sum of these over a node's sides is exactly 2^23 times the change of the
// node's Lambda, so the continuity equation holds bit-exactly.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "device.h"
#include "diag.h"
#include "inject.h"

namespace axp {

constexpr int kS = 1 << 23;                  // element-local fixed point: lambda * 2^23
constexpr float kInvS = 1.0f / 8388608.0f;
constexpr int kTagAxis = 2;

__device__ __forceinline__ int xcd_block(int bid, int nb) {
    // consecutive logical blocks on the same XCD (blocks are dealt round-robin over 8 XCDs)
    int x = bid & 7, i = bid >> 3, per = nb >> 3, rem = nb & 7;
    return x < rem ? x * (per + 1) + i : rem * (per + 1) + (x - rem) * per + i;
}

__device__ __forceinline__ int sel3(int k, int a, int b, int c) { return k == 0 ? a : (k == 1 ? b : c); }

// ------------------------------------------------------------------ faces
// magnetic current of point source k at step n (Sec. 4.1)
__device__ __forceinline__ double source_current(const FieldSrc &fs, int k, unsigned long long n) {
    const double tt = double(n) * fs.dt - fs.t0[k];
    const double a = tt / (2.0 * fs.sig[k]);
    return fs.amp[k] * exp(-a * a) * cos(fs.w[k] * tt);
}

// Sum of v over the 256 threads of a block in a fixed order (deterministic);
// every thread of the block must call it.
__device__ __forceinline__ double block_sum256(double v) {
    __shared__ double sh[256];
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// One face: returns 1/2 B^{n+1/2} H B^{n-1/2}, its share of the magnetic energy of level n.
__device__ __forceinline__ double tri_pass_face(const DevMesh &m, const DevState &s, const FieldSrc &fs,
                                                const DevLayers &lay, int t, bool diag) {
    const int4 e = m.tedge[t];
    const int inst = m.tinst ? m.tinst[t] : 0;
    const double dt = m.inst[inst].dt;
    float E0 = s.E[e.x], E1 = s.E[e.y], E2 = s.E[e.z];
    if (e.w & 1) E0 = -E0;
    if (e.w & 2) E1 = -E1;
    if (e.w & 4) E2 = -E2;
    const double bo = s.B[t];
    double bn = bo - dt * ((double)E0 + (double)E1 + (double)E2);   // circulation along the CCW boundary
    for (int k = 0; k < fs.n_src; ++k)
        if (t == fs.src_face[k]) bn -= dt * source_current(fs, k, s.ctr->step);
    s.B[t] = bn;
    s.Bprev[t] = bo;
    const int il = lay.n ? lay.face_layer[t] : -1;
    if (il < 0) {
        s.HBdt[t] = m.Hdt[t] * bn;
    } else {                                    // layer face: s_z h = H B, trapezoidal in time
        const double b = lay.beta[il];
        const double hn = ((1.0 - b) * lay.h[il] + lay.Hf[il] * (bn - bo)) / (1.0 + b);
        lay.h[il] = hn;
        s.HBdt[t] = dt * hn;
    }
    const float4 g = m.gS[t];
    const float4 r = m.rho4[t];
    const float g0z = g.x * kInvS, g0r = g.y * kInvS, g1z = g.z * kInvS, g1r = g.w * kInvS;
    const float g2z = -(g0z + g1z), g2r = -(g0r + g1r);
    // E(lambda) = sum_j lambda_j a_j,  a_j = E_{j-1} grad lam_{j+1} - E_{j+1} grad lam_{j-1}
    float4 f0, f1;
    f0.x = E2 * g1z - E1 * g2z;
    f0.y = E2 * g1r - E1 * g2r;
    f0.z = E0 * g2z - E2 * g0z;
    f0.w = E0 * g2r - E2 * g0r;
    f1.x = E1 * g0z - E0 * g1z;
    f1.y = E1 * g0r - E0 * g1r;
    f1.z = (float)((bn + bo) * (double)r.w);     // B_phi = (B^{n+1/2} + B^{n-1/2}) / (2 area)
    f1.w = 0.0f;
    s.f0[t] = f0;
    s.f1[t] = f1;
    if (t == fs.probe_face) {                   // E^n at the probe point (Whitney gather)
        const long long i = (long long)s.ctr->step - fs.probe_start;
        if (i >= 0 && i < fs.probe_cap) {
            const double l0 = fs.probe_l0, l1 = fs.probe_l1, l2 = 1.0 - l0 - l1;
            fs.probe[2 * i] = l0 * f0.x + l1 * f0.z + l2 * f1.x;
            fs.probe[2 * i + 1] = l0 * f0.y + l1 * f0.w + l2 * f1.y;
        }
    }
    s.Jloc[3 * t] = 0ull;
    s.Jloc[3 * t + 1] = 0ull;
    s.Jloc[3 * t + 2] = 0ull;
    if (!diag) return 0.0;
    s.Qloc[3 * t] = 0ull;                       // the particle kernel adds the charge of level n
    s.Qloc[3 * t + 1] = 0ull;
    s.Qloc[3 * t + 2] = 0ull;
    return 0.5 * (m.Hdt[t] / dt) * bn * bo;
}

// Faraday update of every face (and its gather tile).  diag: the step
// evaluates the diagnostics of its start level; the face pass then clears
// the corner charges and leaves one partial of W_B per block.
// Emission of one step by one block (the step's count n_slots, the draws'
// counter inj_step): particle n_slots + i at its emission point on an
// emitter edge (the face's third coordinate 0), its charge taken from the
// edge's tail and head nodes' wall charge in fixed point (the nodal charge
// is unchanged), summed per edge end in LDS (s_q, 2 per edge) and added with
// one atomic per edge end; then the block commits the count.
constexpr int kInjMaxEdges = 1024;

__device__ __forceinline__ void inject_block(const DevState &s, const EmitEdge *ee, const InjParams &p,
                                             unsigned long long *s_q) {
    for (int k = threadIdx.x; k < 2 * p.n_edges; k += blockDim.x) s_q[k] = 0ull;
    const unsigned long long step = s.ctr->inj_step;
    const long long base = (long long)s.ctr->n_slots;
    __syncthreads();
    const int c = s.cur;
    for (int i = threadIdx.x; i < p.per_step; i += blockDim.x) {
        const long long q = base + i;
        const Emission em = sample_emission(ee, p, step, i);
        const EmitEdge E = ee[em.e];
        int La = (int)rint((1.0 - em.s) * (double)kS);
        La = La < 0 ? 0 : (La > kS ? kS : La);
        const int Lb = kS - La;
        const int L0 = E.ka == 0 ? La : (E.kb == 0 ? Lb : 0);
        const int L1 = E.ka == 1 ? La : (E.kb == 1 ? Lb : 0);
        s.cell[c][q] = E.face | (p.species << kCellBits);
        s.L0[c][q] = (uint32_t)L0;
        s.L1[c][q] = (uint32_t)L1;
        s.ur[c][q] = (float)em.ur;
        s.up[c][q] = (float)em.up;
        s.uz[c][q] = (float)em.uz;
        atomicAdd(&s_q[2 * em.e], (unsigned long long)(-(long long)La * p.kq));
        atomicAdd(&s_q[2 * em.e + 1], (unsigned long long)(-(long long)Lb * p.kq));
    }
    __syncthreads();
    for (int k = threadIdx.x; k < 2 * p.n_edges; k += blockDim.x)
        if (s_q[k]) {
            const EmitEdge &E = ee[k >> 1];
            atomicAdd((unsigned long long *)&s.Qres[(k & 1) ? E.nb : E.na], s_q[k]);
        }
    if (threadIdx.x == 0) {
        s.ctr->n_slots = (unsigned long long)base + (unsigned long long)p.per_step;
        s.ctr->inj_step = step + 1ull;
    }
}

// final reduction of a diagnostic step's evaluation by one block (defined with the diagnostics)
__device__ void final_block(DevState s, int nb_node, int nb_we);

// The face pass.  With fin_nb_node > 0 one extra block is the final reduction
// of the last diagnostic step, with ip.per_step > 0 one more is the step's
// emission: both are independent of the faces, so they overlap them and cost
// no launch.

__global__ __launch_bounds__(256) void k_tri_pass(DevMesh m, DevState s, FieldSrc fs, DevLayers lay, int diag,
                                                  const EmitEdge *ee, InjParams ip, int fin_nb_node, int fin_nb_we) {
    // the final reduction, then the emission, take the first blocks, so that
    // their chains of dependent loads start with the grid instead of after
    // the face blocks
    int bid = blockIdx.x;
    if (fin_nb_node > 0) {
        if (bid == 0) {
            final_block(s, fin_nb_node, fin_nb_we);
            return;
        }
        --bid;
    }
    if (ip.per_step > 0) {
        if (bid == 0) {
            __shared__ unsigned long long s_q[2 * kInjMaxEdges];
            inject_block(s, ee, ip, s_q);
            return;
        }
        --bid;
    }
    const int t = bid * blockDim.x + threadIdx.x;
    const double wb = t < m.n2 ? tri_pass_face(m, s, fs, lay, t, diag != 0) : 0.0;
    if (!diag) return;                          // uniform across the grid
    const double tot = block_sum256(wb);
    if (threadIdx.x == 0) s.part_face[bid] = tot;
}

// -------------------------------------------------------------- particles
// One kernel, k_particles, over blocks of 1024 consecutive particles (4 per
// thread).  Phase 1 (push): gather, Boris, position update; a particle whose
// path ends in its own face deposits the single piece's current into the
// thread's register accumulator (consecutive particles share faces), reduced
// per face across the wave into the block's LDS window; a particle that
// leaves its face is queued in LDS.  Phase 2 (walk): the block's threads walk
// the queued particles face by face, each piece's current going into the same
// window.  Phase 3: owners take their movers' final coordinates back, store
// their four particles with vector stores, and the window is added to the
// global face currents once.
constexpr int kPPT = 4;          // particles per thread (consecutive in storage)
constexpr int kWG = 256;

// exact 48-bit product of two coordinates in [0, 2^23] (full-rate 24-bit multiplies)
__device__ __forceinline__ long long m24(int a, int b) {
    return (long long)((unsigned long long)((unsigned)a & 0xFFFFFFu) * ((unsigned)b & 0xFFFFFFu));
}

// current of the straight piece s -> e inside one face, per side k
__device__ __forceinline__ void piece_current(int s0, int s1, int s2, int e0, int e1, int e2, int kq,
                                              long long &c0, long long &c1, long long &c2) {
    c0 = m24(s1, e2) - m24(s2, e1);
    c1 = m24(s2, e0) - m24(s0, e2);
    c2 = m24(s0, e1) - m24(s1, e0);
    if (kq != 1) { c0 *= kq; c1 *= kq; c2 *= kq; }
}

// Sum of a 64-bit value over the lanes of the wave (butterfly of shuffles).
__device__ __forceinline__ long long wave_sum64(long long v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Per-block accumulation window: the fixed-point currents and sort counts of
// kWin consecutive faces live in LDS; faces outside the window go straight to
// global memory.  A block's particles are sorted by face, so nearly all of
// its deposits land in the window, and the window is added to global memory
// once per face at the end of the block.  Between sorts the particles drift
// off their faces' order; 512 faces still hold most of them 16 steps after
// a sort.  With the walk queue that is 24.6 KB of LDS per block, which keeps
// the 6 waves per SIMD the registers allow.
constexpr int kWin = 512;
constexpr int kWinLead = 192;    // default: the window starts this many faces before the block's first face

struct Win {
    unsigned long long *jl;      // LDS, 3 * kWin
    int *cl;                     // LDS, kWin
    int base;
};

__device__ __forceinline__ void win_add_j(const Win &w, unsigned long long *J, int t, long long a0, long long a1,
                                          long long a2) {
    const int rel = t - w.base;
    if (rel >= 0 && rel < kWin) {
        if (a0) atomicAdd(&w.jl[3 * rel], (unsigned long long)a0);
        if (a1) atomicAdd(&w.jl[3 * rel + 1], (unsigned long long)a1);
        if (a2) atomicAdd(&w.jl[3 * rel + 2], (unsigned long long)a2);
    } else {
        if (a0) atomicAdd(&J[3 * t], (unsigned long long)a0);
        if (a1) atomicAdd(&J[3 * t + 1], (unsigned long long)a1);
        if (a2) atomicAdd(&J[3 * t + 2], (unsigned long long)a2);
    }
}

__device__ __forceinline__ void win_add_c(const Win &w, int *cnt, int t, int v) {
    const int rel = t - w.base;
    if (rel >= 0 && rel < kWin) atomicAdd(&w.cl[rel], v);
    else atomicAdd(&cnt[t], v);
}

// Deposit every lane's (face t, 3 side currents): sums over runs of
// consecutive lanes holding the same face (lanes follow the particle order,
// which is sorted by face), after which the last lane of each run adds the
// run's total.  Cost is independent of how many faces the wave holds.  Lanes
// with t < 0 hold nothing.  All lanes of the wave must call this together.
//
// Values move between lanes with DPP (data-parallel primitives of the VALU,
// no LDS round trip): shifts by 1, 2, 4 and 8 lanes within each row of 16,
// then the last lane of a row broadcast into the next row (row_bcast:15,
// rows 1 and 3) and lane 31 into the upper half (row_bcast:31, rows 2 and
// 3); lanes outside a move's source range receive 0.
// GFX9 DPP controls: row_shr:n = 0x110 + n, wave_shl:1 = 0x130,
// wave_shr:1 = 0x138, row_bcast:15 = 0x142, row_bcast:31 = 0x143.
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_mov(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xF, true);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned dpp_mov(unsigned v) {
    return (unsigned)dpp_mov<CTRL, ROWS>((int)v);
}

// (64-bit: one move per 32-bit half; the 64-bit form of the builtin keeps the
// halves in one register pair, so a following 64-bit add is one instruction)
template <int CTRL, int ROWS>
__device__ __forceinline__ long long dpp_mov(long long v) {
    return __builtin_amdgcn_update_dpp((long long)0, v, CTRL, ROWS, 0xF, true);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ unsigned long long dpp_mov(unsigned long long v) {
    return (unsigned long long)dpp_mov<CTRL, ROWS>((long long)v);
}

__device__ __forceinline__ bool run_tail(int t) {
    const int lane = threadIdx.x & 63;
    const int tn = dpp_mov<0x130, 0xF>(t);                   // lane + 1 (lane 63: tail anyway)
    return lane == 63 || tn != t;
}

// ds_bpermute of a lane's value from the lane at byte address addr (4 x lane)
__device__ __forceinline__ int bperm(int addr, int v) { return __builtin_amdgcn_ds_bpermute(addr, v); }
__device__ __forceinline__ unsigned bperm(int addr, unsigned v) { return (unsigned)bperm(addr, (int)v); }
__device__ __forceinline__ long long bperm(int addr, long long v) {
    const unsigned lo = bperm(addr, (unsigned)(unsigned long long)v);
    const unsigned hi = bperm(addr, (unsigned)((unsigned long long)v >> 32));
    return (long long)(((unsigned long long)hi << 32) | lo);
}
__device__ __forceinline__ unsigned long long bperm(int addr, unsigned long long v) {
    return (unsigned long long)bperm(addr, (long long)v);
}

template <int CTRL, int ROWS, class V, int N>
__device__ __forceinline__ void scan_step(V (&a)[N]) {
#pragma unroll
    for (int k = 0; k < N; ++k) a[k] += dpp_mov<CTRL, ROWS>(a[k]);
}

// Sums of a[] over runs of consecutive lanes holding the same key t: each
// lane receives the sum over its run up to itself, so a run's last lane
// holds the run's total.  Integer sums, exact in any order (modular for the
// unsigned types, whose run totals stay below 2^32): an inclusive scan over
// the whole wave (row shifts, then the row broadcasts), after which each
// lane subtracts the scan value of the lane just before its run's first lane
// (one ds_bpermute per 32-bit word).  All lanes of the wave must call this
// together.
template <class V, int N>
__device__ __forceinline__ void run_totals(int t, V (&a)[N]) {
    const int lane = threadIdx.x & 63;
    const int tp = dpp_mov<0x138, 0xF>(t);                   // lane - 1 (lane 0: a head anyway)
    const unsigned long long heads = __ballot(lane == 0 || tp != t);
    const int head = 63 - __clzll(heads & ((2ull << lane) - 1ull));   // first lane of this lane's run
    scan_step<0x111, 0xF>(a);
    scan_step<0x112, 0xF>(a);
    scan_step<0x114, 0xF>(a);
    scan_step<0x118, 0xF>(a);
    scan_step<0x142, 0xA>(a);
    scan_step<0x143, 0xC>(a);
    const int src = (head > 0 ? head - 1 : 0) << 2;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const V before = bperm(src, a[k]);
        if (head > 0) a[k] -= before;
    }
}

__device__ __forceinline__ void wave_deposit(const Win &w, unsigned long long *J, int t, long long a0, long long a1,
                                             long long a2) {
    long long a[3] = {a0, a1, a2};
    run_totals<long long, 3>(t, a);
    if (run_tail(t) && t >= 0) win_add_j(w, J, t, a[0], a[1], a[2]);
}

// Charge of the particles' end positions in a diagnostic step (eq. charge):
// per face of the window its three corner sums kq Lambda_k (units 2^-23 of
// the charge unit), in LDS words of type QA.  Single case (charge multiple 1):
// 32-bit words, every added value below 2^32 and non-negative, a wrap-around
// carried exactly into the 64-bit global accumulator; otherwise 64-bit words.
template <class QA>
struct QWinL {
    QA *ql;                      // LDS, 3 * kWin
    int base;
};

__device__ __forceinline__ void qadd1(unsigned *l, unsigned long long *g, long long q) {
    if (!q) return;
    const unsigned v = (unsigned)q;
    const unsigned old = atomicAdd(l, v);
    if ((unsigned)(old + v) < old) atomicAdd(g, 1ull << 32);
}

__device__ __forceinline__ void qadd1(unsigned long long *l, unsigned long long *g, long long q) {
    if (q) atomicAdd(l, (unsigned long long)q);
}

template <class QA>
__device__ __forceinline__ void qwin_add3(const QWinL<QA> &w, unsigned long long *Qloc, int t, long long q0,
                                          long long q1, long long q2) {
    const int rel = t - w.base;
    if (rel >= 0 && rel < kWin) {
        qadd1(&w.ql[3 * rel], &Qloc[3 * t], q0);
        qadd1(&w.ql[3 * rel + 1], &Qloc[3 * t + 1], q1);
        qadd1(&w.ql[3 * rel + 2], &Qloc[3 * t + 2], q2);
    } else {
        if (q0) atomicAdd(&Qloc[3 * t], (unsigned long long)q0);
        if (q1) atomicAdd(&Qloc[3 * t + 1], (unsigned long long)q1);
        if (q2) atomicAdd(&Qloc[3 * t + 2], (unsigned long long)q2);
    }
}

// Same for a count per face (histogram of the counting sort).
__device__ __forceinline__ void wave_count(const Win &w, int *cnt, int t, int c) {
    int a[1] = {c};
    run_totals<int, 1>(t, a);
    if (run_tail(t) && t >= 0 && a[0]) win_add_c(w, cnt, t, a[0]);
}

// (blocks of kWG threads: each thread takes fixed rows of the window, and
// reads all of its rows before the first atomic)
static_assert((3 * kWin) % kWG == 0 && kWin % kWG == 0, "window rows per thread");

__device__ __forceinline__ void win_zero(const Win &w) {
#pragma unroll
    for (int r = 0; r < 3 * kWin / kWG; ++r) w.jl[threadIdx.x + r * kWG] = 0ull;
#pragma unroll
    for (int r = 0; r < kWin / kWG; ++r) w.cl[threadIdx.x + r * kWG] = 0;
}

// after a barrier: add the window to the global arrays (3 n2 < 2^31)
__device__ __forceinline__ void win_flush(const Win &w, unsigned long long *J, int *cnt, int n2, bool counts) {
    constexpr int R = 3 * kWin / kWG, RC = kWin / kWG;
    unsigned long long v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = w.jl[threadIdx.x + r * kWG];
    int c[RC];
#pragma unroll
    for (int r = 0; r < RC; ++r) c[r] = counts ? w.cl[threadIdx.x + r * kWG] : 0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int gi = 3 * w.base + (int)threadIdx.x + r * kWG;
        if (v[r] != 0ull && gi >= 0 && gi < 3 * n2) atomicAdd(&J[gi], v[r]);
    }
#pragma unroll
    for (int r = 0; r < RC; ++r) {
        const int t = w.base + (int)threadIdx.x + r * kWG;
        if (c[r] != 0 && t >= 0 && t < n2) atomicAdd(&cnt[t], c[r]);
    }
}

// Particle streams are loaded and stored non-temporally: each word is read
// and written once per step, and without the hint the 400 MB a step moves
// evicts the faces' and edges' tables from L2 and the last-level cache
// (measured: particle kernel 108.8 -> 105.7 us, SpMV 20.3 -> 16.1 us, face
// pass 13.9 -> 12.6 us, the step 0.155 -> 0.146 ms).  Native vector types,
// which the non-temporal builtins take.
typedef int nt_i4 __attribute__((ext_vector_type(4)));
typedef unsigned nt_u4 __attribute__((ext_vector_type(4)));
typedef float nt_f4 __attribute__((ext_vector_type(4)));

struct Particle {
    int cell;
    uint32_t L0, L1;
    float ur, up, uz;
};

struct PushConst {
    float qe, qb, cdt, bz;
    int kq;
    float mw;        // m w c^2 / (2 pi) of the species [J/rad] (kinetic-energy diagnostic; 1 in the single case)
};

template <bool SINGLE>
__device__ __forceinline__ PushConst push_const(const DevMesh &m, const PushConst &k0, int T, int sp) {
    if (SINGLE) return k0;
    const InstConst &ic = m.inst[m.tinst ? m.tinst[T] : 0];
    return PushConst{ic.qe[sp], ic.qb[sp], ic.cdt, ic.bz, ic.kq[sp], (float)ic.mw[sp]};
}

// Gather, momentum push (relativistic Boris, or Vay's pusher when VAY) and
// the axisymmetric position update of one particle: returns the meridian
// displacement (dz, drho) and updates u.
template <bool VAY>
__device__ __forceinline__ void push(const DevState &s, Particle &P, const PushConst &ic, const float4 f0,
                                     const float4 f1, const float4 r4, int L0, int L1, int L2, float &fz, float &fr) {
    const float qe = ic.qe, qb = ic.qb;
    const float l0 = L0 * kInvS, l1 = L1 * kInvS, l2 = L2 * kInvS;
    // Whitney 1-form E, face-constant B_phi, external B_z
    const float Ez = l0 * f0.x + l1 * f0.z + l2 * f1.x;
    const float Er = l0 * f0.y + l1 * f0.w + l2 * f1.y;
    const float Bp = f1.z, Bz = ic.bz;
    // u normalised by c; basis (rho, phi, z); qe E = q dt E / (2 m c), tau = q dt B / (2 m)
    float ur, up, uz;
    if (!VAY) {
        // relativistic Boris: half kick, rotation about B, half kick
        const float umr = P.ur + qe * Er, ump = P.up, umz = P.uz + qe * Ez;
        const float igm = __builtin_amdgcn_rsqf(1.0f + umr * umr + ump * ump + umz * umz);
        const float tp = qb * Bp * igm, tz = qb * Bz * igm;
        const float f = 2.0f * __builtin_amdgcn_rcpf(1.0f + tp * tp + tz * tz);
        const float sp_ = f * tp, sz = f * tz;
        const float vr = umr + (ump * tz - umz * tp);
        const float vp = ump - umr * tz;
        const float vz = umz + umr * tp;
        ur = umr + (vp * sz - vz * sp_) + qe * Er;
        up = ump - vr * sz;
        uz = umz + vr * sp_ + qe * Ez;
    } else {
        // Vay: u' = u + 2 qe E + (u / gamma) x tau, then the new gamma from
        // the quadratic in gamma^2 and the exact solve of u = u' + (u / gamma) x tau
        const float taup = qb * Bp, tauz = qb * Bz;
        const float ig0 = __builtin_amdgcn_rsqf(1.0f + P.ur * P.ur + P.up * P.up + P.uz * P.uz);
        const float vr = P.ur * ig0, vp = P.up * ig0, vz = P.uz * ig0;
        const float ar = P.ur + 2.0f * qe * Er + (vp * tauz - vz * taup);
        const float ap = P.up - vr * tauz;
        const float az = P.uz + 2.0f * qe * Ez + vr * taup;
        const float tau2 = taup * taup + tauz * tauz;
        const float ustar = ap * taup + az * tauz;
        const float sigma = 1.0f + ar * ar + ap * ap + az * az - tau2;
        const float g2 = 0.5f * (sigma + __builtin_sqrtf(sigma * sigma + 4.0f * (tau2 + ustar * ustar)));
        const float ign = __builtin_amdgcn_rsqf(g2);
        const float tp = taup * ign, tz = tauz * ign;
        const float sc = __builtin_amdgcn_rcpf(1.0f + tp * tp + tz * tz);
        const float at = ustar * ign;                    // u' . t
        ur = sc * (ar + (ap * tz - az * tp));
        up = sc * (ap + at * tp - ar * tz);
        uz = sc * (az + at * tz + ar * tp);
    }
    if (!(ur * ur + up * up + uz * uz < 3.0e38f)) {   // non-finite or absurd momentum: count, stop
        atomicAdd(&s.ctr->nan_count, 1ull);
        ur = up = uz = 0.0f;
    }
    // move in the local Cartesian frame, rotate back to the meridian plane
    const float ig = __builtin_amdgcn_rsqf(1.0f + ur * ur + up * up + uz * uz) * ic.cdt;
    const float rho = l0 * r4.x + l1 * r4.y + l2 * r4.z;
    const float dr = ur * ig, dp = up * ig;
    fz = uz * ig;
    const float X = rho + dr;
    const float r2 = X * X + dp * dp;
    const float ir = r2 > 0.0f ? __builtin_amdgcn_rsqf(r2) : 0.0f;
    if (r2 > 0.0f) {
        const float cs = X * ir, sn = dp * ir;
        const float nr = cs * ur + sn * up;
        up = -sn * ur + cs * up;
        ur = nr;
    }
    const float den = r2 * ir + rho;              // rho' + rho
    fr = den > 0.0f ? (2.0f * rho * dr + dr * dr + dp * dp) * __builtin_amdgcn_rcpf(den) : 0.0f;
    P.ur = ur; P.up = up; P.uz = uz;
}

// integer change of the barycentric coordinates for a displacement in face t
__device__ __forceinline__ void lam_change(const float4 g, float fz, float fr, int &d0, int &d1, int &d2) {
    const float d0f = fminf(fmaxf(g.x * fz + g.y * fr, -1.0e9f), 1.0e9f);
    const float d1f = fminf(fmaxf(g.z * fz + g.w * fr, -1.0e9f), 1.0e9f);
    d0 = (int)__builtin_rintf(d0f);
    d1 = (int)__builtin_rintf(d1f);
    d2 = -d0 - d1;
}

constexpr int kChunk = kWG * kPPT;   // particles per block
// LDS walk queue entries per block.  About a fifth of the particles leave
// their face in a step at half the stability limit; a block with more than
// kQCap of them has its owners walk the rest themselves.  A queue for the
// whole chunk would take 20 KB of LDS and cost a resident block per CU.
constexpr int kQCap = 512;

// queued particle of the walk phase (LDS)
struct Mover {
    int cell, L0, L1;
    float fz, fr;        // remaining meridian displacement
};

// Walks one particle that leaves its face: straight pieces face by face,
// each piece's current into the block's window (or global memory), until
// the path ends inside a face, is absorbed by a conductor or open boundary
// edge (its charge kept on the wall nodes), stops on the axis, or hits the
// piece cap.  mv holds the start (face, coordinates, remaining
// displacement) and receives the final cell word and coordinates.
template <bool SINGLE, bool DIAG>
__device__ __forceinline__ void walk_mover(const DevMesh &m, const DevState &s, const Win &w, const PushConst &k0,
                                           int max_walk, int *nabs, Mover &mv) {
    int t = mv.cell & kCellMask;
    const int sp = (mv.cell >> kCellBits) & 15;
    const int kq = SINGLE ? 1 : push_const<SINGLE>(m, k0, t, sp).kq;
    int L0 = mv.L0, L1 = mv.L1, L2 = kS - L0 - L1, entry = -1;
    float fz = mv.fz, fr = mv.fr;
    int newcell = -2;                   // -2: still walking
    // the face's gradients and neighbours are fetched together, so each
    // piece waits for one memory latency, not two in a row
    float4 g = m.gS[t];
    int4 nb = m.nbr[t];
    for (int seg = 0; newcell == -2; ++seg) {
        long long c0 = 0, c1 = 0, c2 = 0;
        const int tf = t;
        int d0, d1, d2;
        lam_change(g, fz, fr, d0, d1, d2);
        // never leave through the side just entered (rounding); slide along it instead
        if (entry == 0 && d0 < 0) { d0 = 0; d2 = -d1; }
        if (entry == 1 && d1 < 0) { d1 = 0; d2 = -d0; }
        if (entry == 2 && d2 < 0) { d2 = 0; d1 = -d0; }
        const int e0 = L0 + d0, e1 = L1 + d1, e2 = L2 + d2;
        if (e0 >= 0 && e1 >= 0 && e2 >= 0) {
            piece_current(L0, L1, L2, e0, e1, e2, kq, c0, c1, c2);
            L0 = e0; L1 = e1; L2 = e2;
            newcell = t | (sp << kCellBits);
        } else {
            // exit side: smallest Lambda_k / (-d_k) among the coordinates going negative
            // (float comparison: any valid choice keeps the walk charge-conserving)
            int kx = -1;
            float best = 3.0e38f;
            if (e0 < 0) { kx = 0; best = (float)L0 * __builtin_amdgcn_rcpf((float)(-d0)); }
            if (e1 < 0) { const float v = (float)L1 * __builtin_amdgcn_rcpf((float)(-d1)); if (v < best) { kx = 1; best = v; } }
            if (e2 < 0) { const float v = (float)L2 * __builtin_amdgcn_rcpf((float)(-d2)); if (v < best) { kx = 2; best = v; } }
            const float sx = fminf(best, 1.0f);
            // crossing point: Lambda_kx = 0, the other two keep their sum
            const int ka = kx == 2 ? 0 : kx + 1;
            const int kb = kx == 0 ? 2 : kx - 1;
            const int La = sel3(ka, L0, L1, L2), da = sel3(ka, d0, d1, d2);
            int xa = La + (int)__builtin_rintf(sx * (float)da);
            xa = xa < 0 ? 0 : (xa > kS ? kS : xa);
            const int xb = kS - xa;
            const int x0 = ka == 0 ? xa : (kb == 0 ? xb : 0);
            const int x1 = ka == 1 ? xa : (kb == 1 ? xb : 0);
            const int x2 = ka == 2 ? xa : (kb == 2 ? xb : 0);
            piece_current(L0, L1, L2, x0, x1, x2, kq, c0, c1, c2);
            const float rem = 1.0f - sx;
            fz *= rem;
            fr *= rem;
            const int nn = sel3(kx, nb.x, nb.y, nb.z);
            if (nn < 0) {
                if (-nn == kTagAxis) {          // rho = 0 cannot be crossed: stay on it
                    L0 = x0; L1 = x1; L2 = x2;
                    newcell = t | (sp << kCellBits);
                } else {                        // absorbed; its charge stays on the wall nodes
                    const int4 tn = m.tnodes[t];
                    const int na = sel3(ka, tn.x, tn.y, tn.z), nbn = sel3(kb, tn.x, tn.y, tn.z);
                    atomicAdd((unsigned long long *)&s.Qres[na], (unsigned long long)((long long)xa * kq));
                    atomicAdd((unsigned long long *)&s.Qres[nbn], (unsigned long long)((long long)xb * kq));
                    atomicAdd(&s.ctr->n_absorbed, 1ull);
                    if (DIAG) atomicAdd(nabs, 1);
                    newcell = -1;
                }
            } else {
                const unsigned map = ((unsigned)nb.w >> (4 * kx)) & 15u;
                const int pa = map & 3, pb = map >> 2, q = 3 - pa - pb;
                L0 = pa == 0 ? xa : (pb == 0 ? xb : 0);
                L1 = pa == 1 ? xa : (pb == 1 ? xb : 0);
                L2 = pa == 2 ? xa : (pb == 2 ? xb : 0);
                entry = q;
                t = nn;
                if (seg + 1 >= max_walk) {      // cut: the particle stops at the crossing
                    atomicAdd(&s.ctr->walk_overflow, 1ull);
                    newcell = t | (sp << kCellBits);
                } else {
                    g = m.gS[t];
                    nb = m.nbr[t];
                }
            }
        }
        win_add_j(w, s.Jloc, tf, c0, c1, c2);
    }
    mv.cell = newcell;
    mv.L0 = L0;
    mv.L1 = L1;
}

// Sums of N values over runs of consecutive lanes holding the same key t
// (run_totals); the run's last lane then holds the run's sums.  All lanes of
// the wave must call it together.
template <class V, int N>
__device__ __forceinline__ void wave_run_sums(int t, V (&a)[N]) {
    run_totals<V, N>(t, a);
}

__device__ __forceinline__ void corner_add(unsigned long long *Qloc, int t, long long q0, long long q1, long long q2) {
    if (q0) atomicAdd(&Qloc[3 * t], (unsigned long long)q0);
    if (q1) atomicAdd(&Qloc[3 * t + 1], (unsigned long long)q1);
    if (q2) atomicAdd(&Qloc[3 * t + 2], (unsigned long long)q2);
}

// Charge window of a block: the corner charges of `len` consecutive faces
// from base on accumulate in LDS; other faces go to global memory.
struct QWin {
    unsigned long long *ql;      // LDS, 3 * len
    int base, len;
};

__device__ __forceinline__ void qwin_add(const QWin &w, unsigned long long *Qloc, int t, long long q0, long long q1,
                                         long long q2) {
    const int rel = t - w.base;
    if (rel >= 0 && rel < w.len) {
        if (q0) atomicAdd(&w.ql[3 * rel], (unsigned long long)q0);
        if (q1) atomicAdd(&w.ql[3 * rel + 1], (unsigned long long)q1);
        if (q2) atomicAdd(&w.ql[3 * rel + 2], (unsigned long long)q2);
    } else {
        corner_add(Qloc, t, q0, q1, q2);
    }
}

// after a barrier: add the charge window to the corner accumulators
__device__ __forceinline__ void qwin_flush(const QWin &w, unsigned long long *Qloc, int n2) {
    for (int i = threadIdx.x; i < 3 * w.len; i += blockDim.x) {
        const unsigned long long v = w.ql[i];
        const long long gi = 3ll * w.base + i;
        if (v != 0ull && gi >= 0 && gi < 3ll * n2) atomicAdd(&Qloc[gi], v);
    }
}

// Nodal charge of the particles at their current positions, eq. (charge):
// a particle in face T adds kq Lambda_k (units 2^-23 of the charge unit) to
// corner k of T.  The thread folds its particles face by face, the wave sums
// runs of lanes holding the same face, and each run's last lane adds the
// three sums to the block's charge window (the particles are sorted by face,
// so a wave holds a few runs and a block a few dozen faces).  In the single
// case (charge multiple 1) a wave's sums stay below 2^32 (256 particles of at
// most 2^23 each) and the scan runs on 32-bit words.
template <bool SINGLE>
__device__ __forceinline__ void charge_deposit(const DevMesh &m, const QWin &w, unsigned long long *Qloc,
                                               const Particle (&P)[kPPT]) {
    using Acc = typename std::conditional<SINGLE, unsigned, long long>::type;
    int qt = -1;
    Acc q[3] = {0, 0, 0};
#pragma unroll
    for (int j = 0; j < kPPT; ++j) {
        if (P[j].cell < 0) continue;
        const int T = P[j].cell & kCellMask;
        if (T != qt) {
            if (qt >= 0) qwin_add(w, Qloc, qt, (long long)q[0], (long long)q[1], (long long)q[2]);
            qt = T;
            q[0] = q[1] = q[2] = 0;
        }
        const Acc L0 = (Acc)P[j].L0, L1 = (Acc)P[j].L1, L2 = (Acc)kS - L0 - L1;
        if (SINGLE) {
            q[0] += L0; q[1] += L1; q[2] += L2;
        } else {
            const InstConst &ic = m.inst[m.tinst ? m.tinst[T] : 0];
            const Acc kq = (Acc)ic.kq[(P[j].cell >> kCellBits) & 15];
            q[0] += kq * L0; q[1] += kq * L1; q[2] += kq * L2;
        }
    }
    wave_run_sums<Acc, 3>(qt, q);
    if (run_tail(qt) && qt >= 0) qwin_add(w, Qloc, qt, (long long)q[0], (long long)q[1], (long long)q[2]);
}

// gamma - 1 of u / c without cancellation for slow particles
__device__ __forceinline__ float gamma_m1(float ur, float up, float uz) {
    const float u2 = ur * ur + up * up + uz * uz;
    const float w = 1.0f + u2;
    return u2 * __builtin_amdgcn_rcpf(w * __builtin_amdgcn_rsqf(w) + 1.0f);   // u^2 / (gamma + 1)
}

// Per-wave sums in a fixed butterfly (deterministic); every lane gets the total.
// Sum over the 64 lanes of a wave in a fixed order, returned to every lane.
__device__ __forceinline__ double wave_sum_d(double v) { return wave_sum64d(v); }

__device__ __forceinline__ int wave_sum_i(int v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Charge of the particles' end positions (level n+1, eq. charge) in a
// diagnostic step: the thread folds its particles face by face, the wave
// sums runs of lanes holding the same face, and each run's last lane adds
// the three corner sums kq Lambda_k to the block's charge window.  Done after
// the walk, when the push's registers are free.  With QA = 32-bit words a
// wave's sums stay below 2^32 (256 particles of at most 2^23 each).
template <bool SINGLE, class QA>
__device__ __forceinline__ void end_charge(const DevMesh &m, const PushConst &k0, const QWinL<QA> &qw,
                                           unsigned long long *Qloc, const Particle (&P)[kPPT]) {
    int qt = -1;
    QA q[3] = {0, 0, 0};
#pragma unroll
    for (int j = 0; j < kPPT; ++j) {
        if (P[j].cell < 0) continue;
        const int T = P[j].cell & kCellMask;
        if (T != qt) {
            if (qt >= 0) qwin_add3(qw, Qloc, qt, (long long)q[0], (long long)q[1], (long long)q[2]);
            qt = T;
            q[0] = q[1] = q[2] = 0;
        }
        const QA L0 = (QA)P[j].L0, L1 = (QA)P[j].L1, L2 = (QA)kS - L0 - L1;
        if (SINGLE) {
            q[0] += L0; q[1] += L1; q[2] += L2;
        } else {
            const QA kq = (QA)(long long)push_const<SINGLE>(m, k0, T, (P[j].cell >> kCellBits) & 15).kq;
            q[0] += kq * L0; q[1] += kq * L1; q[2] += kq * L2;
        }
    }
    wave_run_sums<QA, 3>(qt, q);
    if (run_tail(qt) && qt >= 0) qwin_add3(qw, Qloc, qt, (long long)q[0], (long long)q[1], (long long)q[2]);
}

// Q32: every species' charge multiple is 0 or 1, so the end-position charge
// of a diagnostic step accumulates in 32-bit LDS words (always so in the
// single case).
template <bool SINGLE, bool VAY, bool DIAG, bool Q32>
// Occupancy: 6 waves per SIMD (80 VGPRs) for the plain step.  The diagnostic
// step is bounded at 5 waves (96 VGPRs) so that its extra live values never
// spill (forced to 80, an earlier form spilled: scratch traffic 1.2x the
// kernel's bytes, 20 % slower); with the momenta stored before its walk the
// single-species form needs 80 and runs at 6 waves as well.
__global__ __launch_bounds__(kWG, DIAG ? 5 : 6) void k_particles(DevMesh m, DevState s, int max_walk, int do_count,
                                                      PushConst k0, int win_lead) {
    __shared__ int s_nmv;
    __shared__ int s_base;
    __shared__ unsigned long long s_jl[3 * kWin];
    __shared__ int s_cl[kWin];
    // diagnostic steps: the end positions' charge window (32-bit words: in
    // the walk queue's LDS once the walk is over, so that the block keeps
    // the LDS footprint that allows 6 blocks per CU), per wave the kinetic
    // energy and live count, the block's absorbed count
    using QA = typename std::conditional<SINGLE || Q32, unsigned, unsigned long long>::type;
    constexpr bool kQInQueue = sizeof(QA) * 3 * kWin <= sizeof(Mover) * kQCap;
    __shared__ __align__(16) unsigned char s_queue[sizeof(Mover) * kQCap];
    __shared__ QA s_qown[DIAG && !kQInQueue ? 3 * kWin : 1];
    Mover *const s_mv = reinterpret_cast<Mover *>(s_queue);
    QA *const s_ql = kQInQueue ? reinterpret_cast<QA *>(s_queue) : s_qown;
    __shared__ double s_wk[kWG / 64];
    __shared__ double s_wk1[kWG / 64];   // single case: K^{n-1/2} in s_wk, K^{n+1/2} here
    __shared__ int s_nl[kWG / 64];
    __shared__ int s_nabs;
    // The grid covers the buffer's capacity (a graph replays one launch
    // while emission and sorts change the count): only the first nbv blocks
    // have particles, and they are spread over all XCDs in contiguous chunks.
    const long long n = (long long)s.ctr->n_slots;
    const int nbv = (int)((n + kChunk - 1) / kChunk);
    if ((int)blockIdx.x >= nbv) return;                     // whole block past the end
    const int chunk = xcd_block(blockIdx.x, nbv);
    const long long p0 = ((long long)chunk * kWG + threadIdx.x) * kPPT;
    const int c = s.cur;
    int32_t *cell = s.cell[c];
    uint32_t *L0a = s.L0[c], *L1a = s.L1[c];
    float *ura = s.ur[c], *upa = s.up[c], *uza = s.uz[c];
    const bool full = p0 + kPPT <= n;
    Particle P[kPPT];
    if (full) {
        const nt_i4 cc = __builtin_nontemporal_load(reinterpret_cast<const nt_i4 *>(cell + p0));
        const nt_u4 a = __builtin_nontemporal_load(reinterpret_cast<const nt_u4 *>(L0a + p0));
        const nt_u4 b = __builtin_nontemporal_load(reinterpret_cast<const nt_u4 *>(L1a + p0));
        const nt_f4 x = __builtin_nontemporal_load(reinterpret_cast<const nt_f4 *>(ura + p0));
        const nt_f4 y = __builtin_nontemporal_load(reinterpret_cast<const nt_f4 *>(upa + p0));
        const nt_f4 z = __builtin_nontemporal_load(reinterpret_cast<const nt_f4 *>(uza + p0));
        P[0] = {cc.x, a.x, b.x, x.x, y.x, z.x};
        P[1] = {cc.y, a.y, b.y, x.y, y.y, z.y};
        P[2] = {cc.z, a.z, b.z, x.z, y.z, z.z};
        P[3] = {cc.w, a.w, b.w, x.w, y.w, z.w};
    } else {
#pragma unroll
        for (int j = 0; j < kPPT; ++j) {
            const long long p = p0 + j;
            if (p < n) P[j] = {cell[p], L0a[p], L1a[p], ura[p], upa[p], uza[p]};
            else P[j] = {-1, 0u, 0u, 0.f, 0.f, 0.f};
        }
    }
    // thread 0 holds the block's first particle: the window starts at its face
    if (threadIdx.x == 0) {
        s_nmv = 0;
        s_nabs = 0;
        s_base = (P[0].cell >= 0 ? (P[0].cell & kCellMask) : 0) - win_lead;
    }
    Win w{s_jl, s_cl, 0};
    win_zero(w);
    if (DIAG) {                      // particles pushed in the step (live at its start), per wave
        int nl = 0;
#pragma unroll
        for (int j = 0; j < kPPT; ++j) nl += __popcll(__ballot(P[j].cell >= 0));
        if ((threadIdx.x & 63) == 0) s_nl[threadIdx.x >> 6] = nl;
    }
    if (DIAG && SINGLE) {            // K^{n-1/2} of those particles, before the push needs the registers
        double k = 0.0;
#pragma unroll
        for (int j = 0; j < kPPT; ++j)
            if (P[j].cell >= 0) k += (double)gamma_m1(P[j].ur, P[j].up, P[j].uz);
        const double v = wave_sum_d(k);
        if ((threadIdx.x & 63) == 0) s_wk[threadIdx.x >> 6] = v;
    }
    __syncthreads();
    w.base = s_base;
    const QWinL<QA> qw{s_ql, s_base};
    // ---- phase 1: push
    int acc_t = -1;
    long long a0 = 0, a1 = 0, a2 = 0;
    int ct = -1, cc = 0;             // run-length count of the new faces (stayers only)
    bool mover[kPPT];
    float mfz[kPPT], mfr[kPPT];
    double kin = 0.0;                // diagnostic steps, several species: sum of mw (gamma - 1) at n-1/2 and n+1/2
    int Tc = -1;                     // face data cached across the thread's particles
    float4 cf0 = make_float4(0.f, 0.f, 0.f, 0.f), cf1 = cf0, cr4 = cf0, cg = cf0;
    int ic_key = -1;                 // cell word (face, species) the constants below belong to
    PushConst ic = k0;
#pragma unroll
    for (int j = 0; j < kPPT; ++j) {
        mover[j] = false;
        mfz[j] = mfr[j] = 0.0f;
        if (P[j].cell < 0) continue;
        const int T = P[j].cell & kCellMask;
        const int sp = (P[j].cell >> kCellBits) & 15;
        if (T != Tc) {
            Tc = T;
            cf0 = s.f0[T]; cf1 = s.f1[T]; cr4 = m.rho4[T]; cg = m.gS[T];
        }
        if (!SINGLE && P[j].cell != ic_key) {
            ic_key = P[j].cell;
            ic = push_const<SINGLE>(m, k0, T, sp);
        }
        const int L0 = (int)P[j].L0, L1 = (int)P[j].L1, L2 = kS - L0 - L1;
        float fz, fr;
        if (DIAG && !SINGLE) {       // W_K = 1/2 (K^{n-1/2} + K^{n+1/2}), absorbed particles included
            kin += (double)(ic.mw * gamma_m1(P[j].ur, P[j].up, P[j].uz));
        }
        push<VAY>(s, P[j], ic, cf0, cf1, cr4, L0, L1, L2, fz, fr);
        if (DIAG && !SINGLE) kin += (double)(ic.mw * gamma_m1(P[j].ur, P[j].up, P[j].uz));
        int d0, d1, d2;
        lam_change(cg, fz, fr, d0, d1, d2);
        const int e0 = L0 + d0, e1 = L1 + d1, e2 = L2 + d2;
        if (e0 >= 0 && e1 >= 0 && e2 >= 0) {
            long long c0, c1, c2;
            piece_current(L0, L1, L2, e0, e1, e2, SINGLE ? 1 : ic.kq, c0, c1, c2);
            if (T != acc_t) {
                if (acc_t >= 0) win_add_j(w, s.Jloc, acc_t, a0, a1, a2);
                acc_t = T; a0 = a1 = a2 = 0;
            }
            a0 += c0; a1 += c1; a2 += c2;
            P[j].L0 = (uint32_t)e0;
            P[j].L1 = (uint32_t)e1;
            if (do_count) {
                if (T == ct) ++cc;
                else {
                    if (ct >= 0) win_add_c(w, s.cnt, ct, cc);
                    ct = T; cc = 1;
                }
            }
        } else {
            mover[j] = true;
            mfz[j] = fz;
            mfr[j] = fr;
        }
    }
    wave_deposit(w, s.Jloc, acc_t, a0, a1, a2);
    if (DIAG && !SINGLE) {
        const double v = wave_sum_d(kin);
        if ((threadIdx.x & 63) == 0) s_wk[threadIdx.x >> 6] = v;
    }
    if (do_count) wave_count(w, s.cnt, ct, cc);
    // Momenta are final after the push (the walk moves particles, not
    // momenta).  The diagnostic step of the single case sums K^{n+1/2} of the
    // particles live at the start and stores the momenta now, which frees
    // their registers for the walk and the charge pass.
    constexpr bool kEarlyU = DIAG && SINGLE;
    if (kEarlyU) {
        double k = 0.0;
#pragma unroll
        for (int j = 0; j < kPPT; ++j)
            if (P[j].cell >= 0) k += (double)gamma_m1(P[j].ur, P[j].up, P[j].uz);
        const double v = wave_sum_d(k);
        if ((threadIdx.x & 63) == 0) s_wk1[threadIdx.x >> 6] = v;
        if (full) {
            __builtin_nontemporal_store((nt_f4){P[0].ur, P[1].ur, P[2].ur, P[3].ur}, reinterpret_cast<nt_f4 *>(ura + p0));
            __builtin_nontemporal_store((nt_f4){P[0].up, P[1].up, P[2].up, P[3].up}, reinterpret_cast<nt_f4 *>(upa + p0));
            __builtin_nontemporal_store((nt_f4){P[0].uz, P[1].uz, P[2].uz, P[3].uz}, reinterpret_cast<nt_f4 *>(uza + p0));
        } else {
#pragma unroll
            for (int j = 0; j < kPPT; ++j)
                if (p0 + j < n) { ura[p0 + j] = P[j].ur; upa[p0 + j] = P[j].up; uza[p0 + j] = P[j].uz; }
        }
    }
    // queue the movers in LDS (one LDS atomic per wave and particle slot)
    const int lane = threadIdx.x & 63;
    int slot[kPPT];
#pragma unroll
    for (int j = 0; j < kPPT; ++j) {
        slot[j] = -1;
        const unsigned long long mask = __ballot(mover[j]);
        if (mask == 0ull) continue;
        int base = 0;
        if (lane == __ffsll((long long)mask) - 1) base = atomicAdd(&s_nmv, __popcll(mask));
        base = __shfl(base, __ffsll((long long)mask) - 1, 64);
        if (mover[j]) {
            const int q = base + __popcll(mask & ((1ull << lane) - 1ull));
            if (q < kQCap) {
                slot[j] = q;
                s_mv[q] = Mover{P[j].cell, (int)P[j].L0, (int)P[j].L1, mfz[j], mfr[j]};
            } else slot[j] = -2;
        }
    }
    __syncthreads();
    // ---- phase 2: walk of the queued particles (any thread, any mover); movers
    // that found the queue full are walked by their owners
    const int nmv = min(s_nmv, kQCap);
    if (s_nmv > kQCap) {
#pragma unroll
        for (int j = 0; j < kPPT; ++j)
            if (slot[j] == -2) {
                Mover mv{P[j].cell, (int)P[j].L0, (int)P[j].L1, mfz[j], mfr[j]};
                walk_mover<SINGLE, DIAG>(m, s, w, k0, max_walk, &s_nabs, mv);
                P[j].cell = mv.cell; P[j].L0 = (uint32_t)mv.L0; P[j].L1 = (uint32_t)mv.L1;
                if (do_count && mv.cell >= 0) win_add_c(w, s.cnt, mv.cell & kCellMask, 1);
            }
    }
    for (int i = threadIdx.x; i < nmv; i += kWG) {
        Mover mv = s_mv[i];
        walk_mover<SINGLE, DIAG>(m, s, w, k0, max_walk, &s_nabs, mv);
        s_mv[i] = mv;
        if (do_count && mv.cell >= 0) win_add_c(w, s.cnt, mv.cell & kCellMask, 1);
    }
    __syncthreads();
    // ---- phase 3: movers' final coordinates back to their owners; stores; window flush
#pragma unroll
    for (int j = 0; j < kPPT; ++j)
        if (slot[j] >= 0) {
            P[j].cell = s_mv[slot[j]].cell;
            P[j].L0 = (uint32_t)s_mv[slot[j]].L0;
            P[j].L1 = (uint32_t)s_mv[slot[j]].L1;
        }
    if (DIAG) {
        // level n+1: the end positions' charge (absorbed particles, cell -1, hold none)
        __syncthreads();             // the owners have read the queue: its LDS becomes the charge window
#pragma unroll
        for (int r = 0; r < 3 * kWin / kWG; ++r) s_ql[threadIdx.x + r * kWG] = 0;
        __syncthreads();
        end_charge<SINGLE, QA>(m, k0, qw, s.Qloc, P);
        __syncthreads();
    }
    win_flush(w, s.Jloc, s.cnt, m.n2, do_count != 0);
    if (DIAG) {                      // the charge window, and the block's partials of level n and n+1
        constexpr int R = 3 * kWin / kWG;
        unsigned long long q[R];
#pragma unroll
        for (int r = 0; r < R; ++r) q[r] = (unsigned long long)s_ql[threadIdx.x + r * kWG];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int gi = 3 * w.base + (int)threadIdx.x + r * kWG;
            if (q[r] != 0ull && gi >= 0 && gi < 3 * m.n2) atomicAdd(&s.Qloc[gi], q[r]);
        }
        if (threadIdx.x == 0) {
            double v = 0.0;
            int nl = 0;
#pragma unroll
            for (int k = 0; k < kWG / 64; ++k) { v += SINGLE ? s_wk[k] + s_wk1[k] : s_wk[k]; nl += s_nl[k]; }
            v *= 0.5;                // W_K = 1/2 (K^{n-1/2} + K^{n+1/2})
            s.part_kin[3 * chunk] = SINGLE ? v * m.inst[0].mw[0] : v;
            s.part_kin[3 * chunk + 1] = (double)nl;
            s.part_kin[3 * chunk + 2] = (double)(nl - s_nabs);
        }
    }
    if (full) {
        __builtin_nontemporal_store((nt_i4){P[0].cell, P[1].cell, P[2].cell, P[3].cell}, reinterpret_cast<nt_i4 *>(cell + p0));
        __builtin_nontemporal_store((nt_u4){P[0].L0, P[1].L0, P[2].L0, P[3].L0}, reinterpret_cast<nt_u4 *>(L0a + p0));
        __builtin_nontemporal_store((nt_u4){P[0].L1, P[1].L1, P[2].L1, P[3].L1}, reinterpret_cast<nt_u4 *>(L1a + p0));
        if (!kEarlyU) {
            __builtin_nontemporal_store((nt_f4){P[0].ur, P[1].ur, P[2].ur, P[3].ur}, reinterpret_cast<nt_f4 *>(ura + p0));
            __builtin_nontemporal_store((nt_f4){P[0].up, P[1].up, P[2].up, P[3].up}, reinterpret_cast<nt_f4 *>(upa + p0));
            __builtin_nontemporal_store((nt_f4){P[0].uz, P[1].uz, P[2].uz, P[3].uz}, reinterpret_cast<nt_f4 *>(uza + p0));
        }
    } else {
#pragma unroll
        for (int j = 0; j < kPPT; ++j) {
            const long long p = p0 + j;
            if (p < n) {
                cell[p] = P[j].cell; L0a[p] = P[j].L0; L1a[p] = P[j].L1;
                if (!kEarlyU) { ura[p] = P[j].ur; upa[p] = P[j].up; uza[p] = P[j].uz; }
            }
        }
    }
}

// ------------------------------------------------------------------ edges
// etri.z packs: bits 0-1 side in left face, 2-3 side in right face,
// bit 4 left sign negative, bit 5 right sign negative, bit 6 free edge.
// diag: the step evaluates the energies of its start level n; the edge pass
// reads D^n and E^n before the update and leaves 1/2 E^n D^n per block.
__device__ __forceinline__ double edge_update(const DevMesh &m, const DevState &s, int e, int keep_j, bool diag) {
    const int4 et = m.etri[e];
    const int inst = et.w;
    const double js = m.inst[inst].jscale;
    const int kl = et.z & 3, kr = (et.z >> 2) & 3;
    const long long jl = (long long)s.Jloc[3 * et.x + kl];
    const double sl = (et.z & 16) ? -1.0 : 1.0;
    double acc = sl * (s.HBdt[et.x] - js * (double)jl);
    long long jfx = (et.z & 16) ? -jl : jl;
    if (et.y >= 0) {
        const long long jr = (long long)s.Jloc[3 * et.y + kr];
        const double sr = (et.z & 32) ? -1.0 : 1.0;
        acc += sr * (s.HBdt[et.y] - js * (double)jr);
        jfx += (et.z & 32) ? -jr : jr;
    }
    if (jfx > (1ll << 62) || jfx < -(1ll << 62)) atomicAdd(&s.ctr->fixed_overflow, 1ull);
    if (keep_j) s.Jfx[e] = jfx;        // every edge: conductor edges carry current too (continuity check)
    if (!(et.z & 64)) return 0.0;      // conductor edge: tangential E stays 0
    const double dn = s.D[e];
    const double d = dn + acc;
    s.D[e] = d;
    s.D32[e] = (float)d;
    return diag ? 0.5 * (double)s.E[e] * dn : 0.0;
}

__global__ __launch_bounds__(256) void k_edge_pass(DevMesh m, DevState s, int keep_j, int diag) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e == 0) s.ctr->step = s.ctr->step + 1ull;   // the face pass of this step has read it
    const double we = e < m.n1 ? edge_update(m, s, e, keep_j, diag != 0) : 0.0;
    if (!diag) return;                              // uniform across the grid
    const double tot = block_sum256(we);
    if (threadIdx.x == 0) s.part_edge[blockIdx.x] = tot;
}

// ------------------------------------------------------------------- SpMV
// Row i of E = M D in the sliced ELL layout (FP32, D read as its FP32 copy).
__device__ __forceinline__ float spmv_row(const DevMesh &m, const DevState &s, int i) {
    const int sl = i >> 6, lane = i & 63;
    const int64_t beg = m.m_sptr[sl];
    const int len = m.m_slen[sl];
    const float *v = m.m_val + beg + lane;
    const int32_t *c = m.m_col + beg + lane;
    float acc = 0.0f;
    // four entries per trip, their loads issued before the gathers that depend on them
    int j = 0;
    for (; j + 4 <= len; j += 4) {
        const int c0 = c[64 * j], c1 = c[64 * (j + 1)], c2 = c[64 * (j + 2)], c3 = c[64 * (j + 3)];
        const float v0 = v[64 * j], v1 = v[64 * (j + 1)], v2 = v[64 * (j + 2)], v3 = v[64 * (j + 3)];
        const float x0 = s.D32[c0], x1 = s.D32[c1], x2 = s.D32[c2], x3 = s.D32[c3];
        acc = fmaf(v0, x0, acc);
        acc = fmaf(v1, x1, acc);
        acc = fmaf(v2, x2, acc);
        acc = fmaf(v3, x3, acc);
    }
    for (; j < len; ++j) acc = fmaf(v[64 * j], s.D32[c[64 * j]], acc);
    return acc;
}

__global__ __launch_bounds__(256) void k_spmv(DevMesh m, DevState s) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m.n1) return;
    s.E[i] = spmv_row(m, s, i);
}

// ------------------------------------------------------------------- sort
__global__ __launch_bounds__(256) void k_zero_i32(int32_t *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// Counting-sort passes over blocks of kSortChunk consecutive particles.  A
// block's particles usually lie in few consecutive faces (the array is kept
// sorted), so counts and slot reservations go through an LDS window of faces
// and only one global atomic per (block, face) is needed.
constexpr int kSortChunk = 1024;
constexpr int kSortWin = 4096;

// Runs of consecutive lanes with equal key (keys < 0 never merge: callers
// give such lanes a unique negative key).  Returns the lane's offset in its
// run; the run's last lane gets the run length in *len (others 0) and its
// index in *tail.
__device__ __forceinline__ int run_offset(int key, int *len, int *tail) {
    const int lane = threadIdx.x & 63;
    const int kp = __shfl_up(key, 1, 64);
    const unsigned long long heads = __ballot(lane == 0 || kp != key);
    const unsigned long long tails = (heads >> 1) | (1ull << 63);
    const int start = 63 - __clzll(heads & ((2ull << lane) - 1ull));
    const int end = __ffsll(tails & (~0ull << lane)) - 1;
    *tail = end;
    *len = lane == end ? end - start + 1 : 0;
    return lane - start;
}

__global__ __launch_bounds__(256) void k_count(DevState s, int n2) {
    __shared__ int lcnt[kSortWin];
    __shared__ int s_base;
    const long long n = (long long)s.ctr->n_slots;
    const long long pb = (long long)blockIdx.x * kSortChunk;
    if (pb >= n) return;
    const int32_t *__restrict__ cell = s.cell[s.cur];
    if (threadIdx.x == 0) {
        const int c0 = cell[pb];
        s_base = (c0 >= 0 ? (c0 & kCellMask) : 0) - kSortWin / 8;
    }
    for (int i = threadIdx.x; i < kSortWin; i += 256) lcnt[i] = 0;
    __syncthreads();
    const int base = s_base;
    const int lane = threadIdx.x & 63;
    for (int j = threadIdx.x; j < kSortChunk; j += 256) {
        const long long p = pb + j;
        const int c = p < n ? cell[p] : -1;
        const int t = c & kCellMask, rel = t - base;
        const bool inwin = c >= 0 && rel >= 0 && rel < kSortWin;
        if (c >= 0 && !inwin) atomicAdd(&s.cnt[t], 1);
        int len, tail;
        run_offset(inwin ? t : -2 - lane, &len, &tail);
        if (inwin && len) atomicAdd(&lcnt[rel], len);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < kSortWin; i += 256) {
        const int v = lcnt[i], t = base + i;
        if (v != 0 && t >= 0 && t < n2) atomicAdd(&s.cnt[t], v);
    }
}

// exclusive scan of cnt[0..n) in blocks of 1024; block totals to blk
__global__ __launch_bounds__(256) void k_scan_local(int32_t *cnt, int32_t *blk, int n) {
    __shared__ int32_t sh[256];
    const int base = blockIdx.x * 1024 + threadIdx.x * 4;
    int v[4], sum = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) { v[j] = (base + j < n) ? cnt[base + j] : 0; sum += v[j]; }
    sh[threadIdx.x] = sum;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        int x = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
        __syncthreads();
        sh[threadIdx.x] += x;
        __syncthreads();
    }
    int run = sh[threadIdx.x] - sum;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (base + j < n) cnt[base + j] = run;
        run += v[j];
    }
    if (threadIdx.x == 255) blk[blockIdx.x] = sh[255];
}

__global__ __launch_bounds__(256) void k_scan_blocks(int32_t *blk, int nb, int32_t *total_out, DevState s) {
    __shared__ int32_t sh[256];
    int carry = 0;
    for (int b0 = 0; b0 < nb; b0 += 256) {
        const int i = b0 + threadIdx.x;
        const int v = i < nb ? blk[i] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            int x = threadIdx.x >= off ? sh[threadIdx.x - off] : 0;
            __syncthreads();
            sh[threadIdx.x] += x;
            __syncthreads();
        }
        if (i < nb) blk[i] = carry + sh[threadIdx.x] - v;
        const int tot = sh[255];
        __syncthreads();
        carry += tot;
    }
    if (threadIdx.x == 0) *total_out = carry;
}

__global__ __launch_bounds__(256) void k_scan_add(int32_t *cnt, const int32_t *blk, int n) {
    const int i = blockIdx.x * 1024 + threadIdx.x * 4;
#pragma unroll
    for (int j = 0; j < 4; ++j)
        if (i + j < n) cnt[i + j] += blk[blockIdx.x];
}

// Payload of the particle move: NF arrays of W (4- or 8-byte words).
template <class W, int NF>
struct Payload {
    const W *src[NF];
    W *dst[NF];
};

template <class W, int NF>
__global__ __launch_bounds__(256) void k_scatter(DevState s, int n2, Payload<W, NF> pl) {
    __shared__ int lcnt[kSortWin];
    __shared__ int s_base;
    constexpr int K = kSortChunk / 256;
    const long long n = (long long)s.ctr->n_slots;
    const long long pb = (long long)blockIdx.x * kSortChunk;
    if (pb >= n) return;
    const int a = s.cur, b = 1 - s.cur;
    const int32_t *__restrict__ cell_a = s.cell[a];
    int32_t *__restrict__ cell_b = s.cell[b];
    if (threadIdx.x == 0) {
        const int c0 = cell_a[pb];
        s_base = (c0 >= 0 ? (c0 & kCellMask) : 0) - kSortWin / 8;
    }
    for (int i = threadIdx.x; i < kSortWin; i += 256) lcnt[i] = 0;
    // the payload is loaded up front: its latency overlaps the ranking and
    // the slot reservations, which do not depend on it.  The loads are
    // non-temporal (each word is read once); the scattered stores are not
    // (non-temporal, they doubled the scatter's time: 50 -> 103 us)
    int cv[K];
    W v[NF][K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const long long p = pb + threadIdx.x + 256 * k;
        cv[k] = p < n ? __builtin_nontemporal_load(&cell_a[p]) : -1;
#pragma unroll
        for (int f = 0; f < NF; ++f) v[f][k] = p < n ? __builtin_nontemporal_load(&pl.src[f][p]) : W(0);
    }
    __syncthreads();
    const int base = s_base;
    const int lane = threadIdx.x & 63;
    int rank[K];
    // 1. rank of each particle among the block's particles of the same face:
    //    lanes of a wave holding the same face are ranked by ballot, and the
    //    wave takes its range of the block's count with one LDS atomic
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const int c = cv[k];
        const int t = c & kCellMask, rel = t - base;
        const bool inwin = c >= 0 && rel >= 0 && rel < kSortWin;
        rank[k] = -1;
        if (c >= 0 && !inwin) rank[k] = -2 - atomicAdd(&s.cnt[t], 1);   // outside the window: global slot
        // one LDS reservation per run of lanes holding the same face
        int len, tail;
        const int off = run_offset(inwin ? t : -2 - lane, &len, &tail);
        int base_run = 0;
        if (inwin && len) base_run = atomicAdd(&lcnt[rel], len);
        base_run = __shfl(base_run, tail, 64);
        if (inwin) rank[k] = base_run + off;
    }
    __syncthreads();
    // 2. one global reservation per face of the window
    for (int i = threadIdx.x; i < kSortWin; i += 256) {
        const int v = lcnt[i], t = base + i;
        if (v != 0) lcnt[i] = atomicAdd(&s.cnt[t], v);
    }
    __syncthreads();
    // 3. move
    int q[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
        q[k] = -1;
        if (rank[k] == -1) continue;
        q[k] = rank[k] >= 0 ? lcnt[(cv[k] & kCellMask) - base] + rank[k] : -2 - rank[k];
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
        if (q[k] < 0) continue;
        const int qq = q[k];
        cell_b[qq] = cv[k];
#pragma unroll
        for (int f = 0; f < NF; ++f) pl.dst[f][qq] = v[f][k];
    }
}

__global__ void k_set_slots(DevState s, const int32_t *total) { s.ctr->n_slots = (unsigned long long)(*total); }

// adds delta to the face index of every live cell word (pooling of instances)
__global__ __launch_bounds__(256) void k_offset_cells(int32_t *cell, int64_t n, int32_t delta) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && cell[i] >= 0) cell[i] += delta;
}

// ------------------------------------------------------------ diagnostics
// An evaluation at time level n.  In a diagnostic step the face pass and the
// particle kernel have left the corner charges of level n, the W_B and W_K
// partials and the live counts; on demand k_charge_now leaves the charges and
// counts.  k_node_diag then runs while D^n and J^{n-1/2} (the last step's
// edge current) are still in place, and k_diag_final reduces the partials.

// on-demand charge of the current positions (blocks of kChunk particles, as
// k_particles, with the same charge window) and the live count
template <bool SINGLE>
__global__ __launch_bounds__(kWG) void k_charge_now(DevMesh m, DevState s) {
    __shared__ unsigned long long s_q[3 * kWin];
    __shared__ int s_base;
    __shared__ int s_nl[kWG / 64];
    const long long n = (long long)s.ctr->n_slots;
    const int chunk = blockIdx.x;
    if ((long long)chunk * kChunk >= n) return;
    const long long p0 = ((long long)chunk * kWG + threadIdx.x) * kPPT;
    const int c = s.cur;
    Particle P[kPPT];
    int live = 0;
#pragma unroll
    for (int j = 0; j < kPPT; ++j) {
        const long long q = p0 + j;
        P[j] = {-1, 0u, 0u, 0.f, 0.f, 0.f};
        if (q < n) { P[j].cell = s.cell[c][q]; P[j].L0 = s.L0[c][q]; P[j].L1 = s.L1[c][q]; }
        live += P[j].cell >= 0;
    }
    for (int i = threadIdx.x; i < 3 * kWin; i += kWG) s_q[i] = 0ull;
    if (threadIdx.x == 0) s_base = (P[0].cell >= 0 ? (P[0].cell & kCellMask) : 0) - kWinLead;
    const int nl = wave_sum_i(live);
    if ((threadIdx.x & 63) == 0) s_nl[threadIdx.x >> 6] = nl;
    __syncthreads();
    const QWin qw{s_q, s_base, kWin};
    charge_deposit<SINGLE>(m, qw, s.Qloc, P);
    __syncthreads();
    qwin_flush(qw, s.Qloc, m.n2);
    if (threadIdx.x == 0) {
        int t = 0;
#pragma unroll
        for (int k = 0; k < kWG / 64; ++k) t += s_nl[k];
        s.part_kin[3 * chunk + 2] = (double)t;
    }
}

constexpr int kNodeCols = 4;   // list entries a node loads in one go (a mesh node has about six)

// Node i of an evaluation at level n = ctr->step: nodal charge (wall charge
// plus the corners of its faces), the Gauss residual against its reference
// and its scale, the continuity residual against the last evaluated level,
// and the charge in charge units.
__device__ __forceinline__ void node_vals(const DevMesh &m, DevState &s, int i, bool have_prev, bool first,
                                          DiagVals &v) {
    const int inst = m.ninst ? m.ninst[i] : 0;
    long long Q = s.Qres[i];
    // the node's slice of the padded lists, kNodeCols entries at a time: the
    // index loads of a chunk, then its value loads, are in flight together
    // (the mesh's longest lists are kernel arguments, so no load bounds the
    // chunks); the sums keep the list order
    const size_t sl = (size_t)(i >> 6), l = (size_t)(i & 63);
    const int32_t *cp = m.ncorner_ell + sl * (size_t)m.nwc * 64 + l;
    const int32_t *ep = m.nedge_ell + sl * (size_t)m.nwe * 64 + l;
    const int ncol = m.nwc > m.nwe ? m.nwc : m.nwe;
    double div = 0.0, mag = 0.0;
    long long divj = 0;
    for (int j0 = 0; j0 < ncol; j0 += kNodeCols) {
        int ci[kNodeCols], ei[kNodeCols];
#pragma unroll
        for (int j = 0; j < kNodeCols; ++j) {
            ci[j] = j0 + j < m.nwc ? cp[64 * (j0 + j)] : -1;
            ei[j] = j0 + j < m.nwe ? ep[64 * (j0 + j)] : 0;
        }
        long long qv[kNodeCols], jv[kNodeCols];
        double d[kNodeCols];
#pragma unroll
        for (int j = 0; j < kNodeCols; ++j) {
            const int e = (ei[j] < 0 ? -ei[j] : ei[j]) - 1;
            qv[j] = ci[j] >= 0 ? (long long)s.Qloc[ci[j]] : 0ll;
            d[j] = ei[j] ? s.D[e] : 0.0;
            jv[j] = ei[j] ? s.Jfx[e] : 0ll;
        }
#pragma unroll
        for (int j = 0; j < kNodeCols; ++j) {
            Q += qv[j];
            if (ei[j]) {
                div += ei[j] > 0 ? d[j] : -d[j];
                mag += fabs(d[j]);
                divj += ei[j] > 0 ? jv[j] : -jv[j];
            }
        }
    }
    const double q = (double)Q * m.inst[inst].qscale;
    if (have_prev) {
        const long long r = (long long)kS * (Q - s.Qprev[i]) + divj;
        v.mx[3] = (unsigned long long)(r < 0 ? -r : r);
    }
    s.Qprev[i] = Q;
    s.Qfx[i] = Q;
    if (m.nfree[i]) {
        const double g = div - q;
        if (first) s.g0[i] = g;
        v.mx[0] = dbits(fabs(g - s.g0[i]));
        v.mx[1] = dbits(fabs(g));
        v.mx[2] = dbits(mag);
    }
    v.sum[0] = q;
}

// Node pass of an evaluation at level n = ctr->step, on demand or (in_step)
// after the field update of a diagnostic step with absorbing layers: Q^n
// from the wall charge and the corner charges, the Gauss residual
// res = Ddiv D^n - Q^n (Sec. 3.5.2) and its drift from the reference level,
// the continuity residual 2^23 (Q^n - Q^{n-1}) + Ddiv J^{n-1/2} (Sec. 3.5.1)
// when level n-1 was evaluated, the total charge; per edge 1/2 E^n D^n (W_E
// with the scheme's [*eps]_a).  Each block also folds its slice of the
// step's particle, face and edge partials (in_step).
__global__ __launch_bounds__(256) void k_node_diag(DevMesh m, DevState s, int in_step, int nb_face, int nb_edge) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned long long n = s.ctr->step;
    const bool have_prev = s.ctr->diag_level1 == n && n > 0;
    const bool first = s.ctr->g0_set == 0;
    DiagVals v{};
    if (i < m.n0) node_vals(m, s, i, have_prev, first, v);
    if (i < m.n1) v.sum[1] = 0.5 * (double)s.E[i] * s.D[i];
    fold_slices(s, v, in_step, nb_face, nb_edge, gridDim.x);
    const DiagVals r = block_reduce_diag(v);
    if (threadIdx.x == 0) store_partials(s.part_node, blockIdx.x, gridDim.x, r);
}

// The bookkeeping of an evaluation (one thread): res holds the kDiagSums
// sums and the kDiagMaxes maxima (bit patterns as doubles), cur the step,
// the continuity reference, the energy count and the running maxima.
__device__ __forceinline__ void finish_eval(DevState s, const double *res, const unsigned long long *cur, int in_step,
                                         int plain) {
    DiagVals r{};
#pragma unroll
    for (int k = 0; k < kDiagSums; ++k) r.sum[k] = res[k];
#pragma unroll
    for (int k = 0; k < kDiagMaxes; ++k) r.mx[k] = dbits(res[kDiagSums + k]);
    DevCounters &ctr = *s.ctr;
    DevDiag &d = *s.diag;
    const unsigned long long n = cur[0];
    const bool have_prev = cur[1] == n && n > 0;
    d.level = (long long)n;
    d.n_live = (long long)r.sum[kSumLiveNow];
    d.q_total = r.sum[kSumQ];
    d.WE_now = r.sum[kSumWEnow];
    d.gauss_abs = __longlong_as_double((long long)r.mx[1]);
    d.gauss_scale = __longlong_as_double((long long)r.mx[2]);
    const double qmax = __longlong_as_double((long long)r.mx[4]);
    d.qmax = qmax;
    if (r.mx[0] > cur[3]) d.gauss_drift_max_bits = r.mx[0];
    if (have_prev) {
        const unsigned long long x = r.mx[3];
        d.dce_last = (long long)x;
        if (x > cur[4]) d.dce_max = x;
        if (plain) {
            const double rel = __longlong_as_double((long long)x) / (qmax > 0.0 ? qmax : 1.0);
            if (dbits(rel) > cur[5]) d.dce_rel_max_bits = dbits(rel);
        }
    } else {
        d.dce_last = -1;
    }
    d.n_evals = cur[6] + 1;
    if (in_step) {
        DevEnergy e;
        e.level = (long long)n - 1;
        e.n_live = (long long)r.sum[kSumLiveStart];
        e.WE = r.sum[kSumWE];
        e.WB = r.sum[kSumWB];
        e.WK = r.sum[kSumWK];
        e.Qtot = 0.0;
        s.energy[cur[2] % kEnergyRing] = e;
        ctr.energy_count = cur[2] + 1;
        d.energy = e;
    }
    ctr.diag_level1 = n + 1;
    ctr.g0_set = 1;
}

__device__ __forceinline__ void load_eval_state(const DevState &s, int l, unsigned long long *cur) {
    const unsigned long long *src[7] = {&s.ctr->step, &s.ctr->diag_level1, &s.ctr->energy_count,
                                        &s.diag->gauss_drift_max_bits, &s.diag->dce_max, &s.diag->dce_rel_max_bits,
                                        &s.diag->n_evals};
    cur[l] = *src[l];
}

// Reduces the node-pass partials of an evaluation at level n = ctr->step in
// a fixed order into DevDiag; in a step (whose start level is n - 1),
// appends the energy record of level n - 1 to the ring.  Sets the reference
// flags of the next evaluation.  plain: the FP64 step's continuity residual
// is a double (|dQ + Ddiv J| in charge units) judged against max |Q|.
constexpr int kFinalThreads = 64 * kDiagSlots;      // one wave per slot

// Slots of the evaluation's partials reduced in a fixed order: lane l sums
// (or takes the largest of) entries l, l + 64, l + 128, ... in that order,
// then a butterfly over the wave.  A lane loads kSlotChunk entries of every
// slot it reduces before it adds any, so they are in flight together.  Slot
// kSumWEnow comes from the SpMV blocks' nb_we partials when nb_we > 0.
constexpr int kSlotChunk = 8;

__device__ __forceinline__ const double *slot_src(const DevState &s, int k, int nb_node, int nb_we, int &nb) {
    const bool we = k == kSumWEnow && nb_we > 0;
    nb = we ? nb_we : nb_node;
    return we ? s.part_wenow : s.part_node + (size_t)k * nb_node;
}

// slots k0, k0 + 4, ..., k0 + 4 (NS - 1) by one wave (lane l)
template <int NS>
__device__ __forceinline__ void reduce_slots(const DevState &s, int k0, int l, int nb_node, int nb_we,
                                             double (&out)[NS]) {
    const double *p[NS];
    int nb[NS];
    double x[NS];
    unsigned long long mx[NS];
    int nbmax = 0;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
        p[i] = slot_src(s, k0 + 4 * i, nb_node, nb_we, nb[i]);
        x[i] = 0.0;
        mx[i] = 0ull;
        nbmax = nb[i] > nbmax ? nb[i] : nbmax;
    }
    for (int b = l; b < nbmax; b += 64 * kSlotChunk) {
        double v[NS][kSlotChunk];
#pragma unroll
        for (int i = 0; i < NS; ++i)
#pragma unroll
            for (int u = 0; u < kSlotChunk; ++u) v[i][u] = b + 64 * u < nb[i] ? p[i][b + 64 * u] : 0.0;
#pragma unroll
        for (int i = 0; i < NS; ++i) {
            if (k0 + 4 * i < kDiagSums) {
#pragma unroll
                for (int u = 0; u < kSlotChunk; ++u) x[i] += v[i][u];
            } else {
#pragma unroll
                for (int u = 0; u < kSlotChunk; ++u) {
                    const unsigned long long y = dbits(v[i][u]);
                    mx[i] = y > mx[i] ? y : mx[i];
                }
            }
        }
    }
#pragma unroll
    for (int i = 0; i < NS; ++i)
        out[i] = k0 + 4 * i < kDiagSums ? wave_sum64d(x[i]) : __longlong_as_double((long long)wave_max64(mx[i]));
}

// k_diag_final of a diagnostic step by one block of 256 threads riding in the
// next face pass: each wave reduces three slots together (the same per-slot
// order, so the same results).
__device__ void final_block(DevState s, int nb_node, int nb_we) {
    static_assert(kDiagSums + kDiagMaxes == 12, "three slots per wave");
    __shared__ double res[kDiagSlots];
    __shared__ unsigned long long cur[7];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    if (w == 0 && l < 7) load_eval_state(s, l, cur);
    double r[3];
    reduce_slots<3>(s, w, l, nb_node, nb_we, r);
    if (l == 0)
#pragma unroll
        for (int i = 0; i < 3; ++i) res[w + 4 * i] = r[i];
    __syncthreads();
    if (threadIdx.x == 0) finish_eval(s, res, cur, 1, 0);
}

__global__ __launch_bounds__(kFinalThreads) void k_diag_final(DevState s, int nb_node, int in_step, int plain,
                                                               int nb_we) {
    __shared__ double res[kDiagSlots];
    __shared__ unsigned long long cur[7];     // the counters and running values thread 0 updates
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;   // wave w reduces slot w over the node-pass blocks
    if (w == kDiagSlots - 1 && l < 7) load_eval_state(s, l, cur);   // in parallel with the reduction
    if (w < kDiagSums + kDiagMaxes) {
        double t[1];
        reduce_slots<1>(s, w, l, nb_node, nb_we, t);
        if (l == 0) res[w] = t[0];
    }
    __syncthreads();
    if (threadIdx.x == 0) finish_eval(s, res, cur, in_step, plain);
}

// E = M D of a diagnostic step, with 1/2 E D of the new level summed per
// block of rows b (the energy the evaluation reports for that level).
__device__ __forceinline__ void spmv_we_block(const DevMesh &m, DevState &s, int b) {
    __shared__ double wsum[4];
    const int t = threadIdx.x, l = t & 63, w = t >> 6;
    const int i = b * 256 + t;
    double we = 0.0;
    if (i < m.n1) {
        const float e = spmv_row(m, s, i);
        s.E[i] = e;
        we = 0.5 * (double)e * s.D[i];
    }
    we = wave_sum64d(we);
    if (l == 0) wsum[w] = we;
    __syncthreads();
    if (t == 0) s.part_wenow[b] = ((wsum[0] + wsum[1]) + wsum[2]) + wsum[3];
}

// The node pass of a diagnostic step, block b of nb_node: one thread per
// node only (the energy of the new level comes from the SpMV blocks).
__device__ __forceinline__ void node_step_block(const DevMesh &m, DevState &s, int nb_node, int nb_face,
                                                int nb_edge) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned long long n = s.ctr->step;
    const bool have_prev = s.ctr->diag_level1 == n && n > 0;
    const bool first = s.ctr->g0_set == 0;
    DiagVals v{};
    if (i < m.n0) node_vals(m, s, i, have_prev, first, v);
    fold_slices(s, v, 1, nb_face, nb_edge, nb_node);
    const DiagVals r = block_reduce_diag(v);
    if (threadIdx.x == 0) store_partials(s.part_node, blockIdx.x, nb_node, r);
}

// Both in one launch: blocks 0 .. nb_node - 1 are the node pass (chains of
// dependent gathers, so they start first), the rest the SpMV.  They share no
// array (the SpMV reads D and writes E; the node pass reads D, the charges
// and the edge currents).  A separate node-pass launch after the SpMV took
// 12.8 us of its own.
__global__ __launch_bounds__(256) void k_spmv_node(DevMesh m, DevState s, int nb_node, int nb_face, int nb_edge) {
    if ((int)blockIdx.x < nb_node) node_step_block(m, s, nb_node, nb_face, nb_edge);
    else spmv_we_block(m, s, (int)blockIdx.x - nb_node);
}

__global__ __launch_bounds__(256) void k_zero_u64(unsigned long long *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// ------------------------------------------------------- absorbing layers
// After E^{n+1} = M (D^n + dt rhs): per layer face, with e its side values,
//   q^{n+1} = ((1 - beta) q^n + A_z (e^{n+1} - e^n)) / (1 + beta)
//   corr_k  = 2 beta ((A_rho e^{n+1})_k - q_k^{n+1} / (1 + beta));
// then D -= corr on every free side (each edge adds its faces' corrections in
// a fixed order, so the update is deterministic).  E values are taken as
// stored (edge orientation), as the local matrices are.
template <class T>
__global__ __launch_bounds__(256) void k_layer_faces(DevMesh m, const T *E, DevLayers lay) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= lay.n) return;
    const int4 te = m.tedge[lay.face[i]];
    const double en[3] = {(double)E[te.x], (double)E[te.y], (double)E[te.z]};
    double de[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) de[k] = en[k] - lay.eprev[3 * i + k];
    const double b = lay.beta[i];
    const double *Az = lay.Az + 9 * i, *Ar = lay.Ar + 9 * i;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double az = Az[3 * k] * de[0] + Az[3 * k + 1] * de[1] + Az[3 * k + 2] * de[2];
        const double ar = Ar[3 * k] * en[0] + Ar[3 * k + 1] * en[1] + Ar[3 * k + 2] * en[2];
        const double qn = ((1.0 - b) * lay.q[3 * i + k] + az) / (1.0 + b);
        lay.q[3 * i + k] = qn;
        lay.corr[3 * i + k] = 2.0 * b * (ar - qn / (1.0 + b));
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) lay.eprev[3 * i + k] = en[k];
}

__global__ __launch_bounds__(256) void k_layer_edges(DevMesh m, DevState s, DevLayers lay) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= lay.n_edges) return;
    const int4 r = lay.edges[j];
    if (!(m.etri[r.x].z & 64)) return;          // conductor edge: D stays
    double c = lay.corr[3 * (r.y >> 2) + (r.y & 3)];
    if (r.z >= 0) c += lay.corr[3 * (r.z >> 2) + (r.z & 3)];
    s.D[r.x] -= c;
}

// --------------------------------------------------------------- launchers
static inline unsigned nblk(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

bool emission_fits_face_pass(const InjParams &p) {
    return p.per_step > 0 && p.per_step <= 4096 && p.n_edges <= kInjMaxEdges;
}

void launch_tri_pass(const DevMesh &m, DevState &s, const FieldSrc &fs, const DevLayers &lay, bool diag,
                     const EmitEdge *ee, const InjParams *emit, bool final_prev, hipStream_t st) {
    if (m.n2 == 0) {
        if (final_prev) launch_step_final(m, s, st);
        return;
    }
    InjParams ip{};
    if (emit && emission_fits_face_pass(*emit)) ip = *emit;
    const unsigned nb = (unsigned)nblk(m.n2, 256) + (final_prev ? 1u : 0u) + (ip.per_step > 0 ? 1u : 0u);
    const int fin_nb_node = final_prev ? (int)nblk(m.n0, 256) : 0, fin_nb_we = (int)nblk(m.n1, 256);
    hipLaunchKernelGGL(k_tri_pass, dim3(nb), dim3(256), 0, st, m, s, fs, lay, diag ? 1 : 0, ee, ip, fin_nb_node,
                       fin_nb_we);
}

template <class T>
void layers_post(const DevMesh &m, DevState &s, const T *E, const DevLayers &lay, hipStream_t st) {
    if (lay.n == 0) return;
    hipLaunchKernelGGL((k_layer_faces<T>), dim3(nblk(lay.n, 256)), dim3(256), 0, st, m, E, lay);
    hipLaunchKernelGGL(k_layer_edges, dim3(nblk(lay.n_edges, 256)), dim3(256), 0, st, m, s, lay);
}

void launch_layers_post(const DevMesh &m, DevState &s, const float *E, const DevLayers &lay, hipStream_t st) {
    layers_post(m, s, E, lay, st);
}

void launch_layers_post(const DevMesh &m, DevState &s, const double *E, const DevLayers &lay, hipStream_t st) {
    layers_post(m, s, E, lay, st);
}

// single: one instance with one species whose charge multiple is 1; its
// constants travel as kernel arguments (scalar registers) instead of a
// per-particle table lookup.
template <bool SINGLE, bool VAY>
static void launch_particles_t(const DevMesh &m, DevState &s, int max_walk, int dc, PushConst k0, bool diag,
                               bool q32, int wl, dim3 grid, hipStream_t st) {
    if (!diag)
        hipLaunchKernelGGL((k_particles<SINGLE, VAY, false, true>), grid, dim3(kWG), 0, st, m, s, max_walk, dc, k0, wl);
    else if (SINGLE || q32)
        hipLaunchKernelGGL((k_particles<SINGLE, VAY, true, true>), grid, dim3(kWG), 0, st, m, s, max_walk, dc, k0, wl);
    else hipLaunchKernelGGL((k_particles<SINGLE, VAY, true, false>), grid, dim3(kWG), 0, st, m, s, max_walk, dc, k0, wl);
}

void launch_particles(const DevMesh &m, DevState &s, int max_walk, bool count, const InstConst *single, bool vay,
                      bool diag, bool q32, int win_lead, hipStream_t st) {
    if (s.capacity == 0) return;
    const dim3 grid(nblk(s.capacity, kChunk));
    const int dc = count ? 1 : 0;
    const int wl = win_lead < 0 ? 0 : (win_lead >= kWin ? kWin - 1 : win_lead);
    if (single) {
        const PushConst k0{single->qe[0], single->qb[0], single->cdt, single->bz, 1, 1.0f};
        if (vay) launch_particles_t<true, true>(m, s, max_walk, dc, k0, diag, true, wl, grid, st);
        else launch_particles_t<true, false>(m, s, max_walk, dc, k0, diag, true, wl, grid, st);
    } else {
        const PushConst k0{0.f, 0.f, 0.f, 0.f, 1, 1.0f};
        if (vay) launch_particles_t<false, true>(m, s, max_walk, dc, k0, diag, q32, wl, grid, st);
        else launch_particles_t<false, false>(m, s, max_walk, dc, k0, diag, q32, wl, grid, st);
    }
}

void launch_sort_zero(const DevMesh &m, DevState &s, hipStream_t st) {
    hipLaunchKernelGGL(k_zero_i32, dim3(nblk(m.n2 + 1, 256)), dim3(256), 0, st, s.cnt, (int64_t)m.n2 + 1);
}

void launch_edge_pass(const DevMesh &m, DevState &s, bool keep_j, bool diag, hipStream_t st) {
    hipLaunchKernelGGL(k_edge_pass, dim3(nblk(m.n1, 256)), dim3(256), 0, st, m, s, keep_j ? 1 : 0, diag ? 1 : 0);
}

void launch_spmv(const DevMesh &m, DevState &s, hipStream_t st) {
    hipLaunchKernelGGL(k_spmv, dim3(nblk(m.n1, 256)), dim3(256), 0, st, m, s);
}

// counted: the particle kernel of this step already histogrammed the faces
void launch_sort_payload(const DevMesh &m, DevState &s, bool counted, int width, int n_fields, void *const *src,
                         void *const *dst, hipStream_t st) {
    if (s.capacity == 0) return;
    const int n = m.n2;
    const int nb = (int)nblk(n, 1024);
    if (!counted) {
        launch_sort_zero(m, s, st);
        hipLaunchKernelGGL(k_count, dim3(nblk(s.capacity, kSortChunk)), dim3(256), 0, st, s, n);
    }
    hipLaunchKernelGGL(k_scan_local, dim3(nb), dim3(256), 0, st, s.cnt, s.blk, n);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(256), 0, st, s.blk, nb, s.cnt + n, s);
    hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(256), 0, st, s.cnt, s.blk, n);
    const dim3 grid(nblk(s.capacity, kSortChunk));
    if (width == 4 && n_fields == 5) {
        Payload<uint32_t, 5> pl;
        for (int f = 0; f < 5; ++f) { pl.src[f] = (const uint32_t *)src[f]; pl.dst[f] = (uint32_t *)dst[f]; }
        hipLaunchKernelGGL((k_scatter<uint32_t, 5>), grid, dim3(256), 0, st, s, n, pl);
    } else if (width == 8 && n_fields == 5) {
        Payload<unsigned long long, 5> pl;
        for (int f = 0; f < 5; ++f) {
            pl.src[f] = (const unsigned long long *)src[f];
            pl.dst[f] = (unsigned long long *)dst[f];
        }
        hipLaunchKernelGGL((k_scatter<unsigned long long, 5>), grid, dim3(256), 0, st, s, n, pl);
    }
    hipLaunchKernelGGL(k_set_slots, dim3(1), dim3(1), 0, st, s, s.cnt + n);
    s.cur = 1 - s.cur;
}

// ------------------------------------------------------------- emission
// Appends particle n_slots + i at its emission point on an emitter edge (the
// coordinate of the face's third node is 0) and takes its charge from the
// tail and head nodes' wall charge in fixed point, so the nodal charge is
// unchanged.
__global__ __launch_bounds__(256) void k_inject(DevMesh m, DevState s, const EmitEdge *ee, InjParams p) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.per_step) return;
    const unsigned long long step = s.ctr->inj_step;
    const long long q = (long long)s.ctr->n_slots + i;
    const Emission em = sample_emission(ee, p, step, i);
    const EmitEdge E = ee[em.e];
    int La = (int)rint((1.0 - em.s) * (double)kS);
    La = La < 0 ? 0 : (La > kS ? kS : La);
    const int Lb = kS - La;
    const int L0 = E.ka == 0 ? La : (E.kb == 0 ? Lb : 0);
    const int L1 = E.ka == 1 ? La : (E.kb == 1 ? Lb : 0);
    const int c = s.cur;
    s.cell[c][q] = E.face | (p.species << kCellBits);
    s.L0[c][q] = (uint32_t)L0;
    s.L1[c][q] = (uint32_t)L1;
    s.ur[c][q] = (float)em.ur;
    s.up[c][q] = (float)em.up;
    s.uz[c][q] = (float)em.uz;
    atomicAdd((unsigned long long *)&s.Qres[E.na], (unsigned long long)(-(long long)La * p.kq));
    atomicAdd((unsigned long long *)&s.Qres[E.nb], (unsigned long long)(-(long long)Lb * p.kq));
}

__global__ void k_inject_commit(DevState s, int per_step) {
    s.ctr->n_slots += (unsigned long long)per_step;
    s.ctr->inj_step += 1ull;
}

// The emission alone, in one block (sizes too large for the face pass's
// block take the multi-block kernel and the commit above).
constexpr int kInjBlock = 1024, kInjMaxOne = 16 * kInjBlock;

__global__ __launch_bounds__(kInjBlock) void k_inject_one(DevMesh m, DevState s, const EmitEdge *ee, InjParams p) {
    __shared__ unsigned long long s_q[2 * kInjMaxEdges];
    inject_block(s, ee, p, s_q);
}

void launch_inject(const DevMesh &m, DevState &s, const EmitEdge *ee, const InjParams &p, hipStream_t st) {
    if (p.per_step <= 0) return;
    if (p.per_step <= kInjMaxOne && p.n_edges <= kInjMaxEdges) {
        hipLaunchKernelGGL(k_inject_one, dim3(1), dim3(kInjBlock), 0, st, m, s, ee, p);
        return;
    }
    hipLaunchKernelGGL(k_inject, dim3(nblk(p.per_step, 256)), dim3(256), 0, st, m, s, ee, p);
    hipLaunchKernelGGL(k_inject_commit, dim3(1), dim3(1), 0, st, s, p.per_step);
}

void launch_offset_cells(int32_t *cell, int64_t n, int32_t delta, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_offset_cells, dim3(nblk(n, 256)), dim3(256), 0, st, cell, n, delta);
}

void launch_sort(const DevMesh &m, DevState &s, bool counted, hipStream_t st) {
    const int a = s.cur, b = 1 - s.cur;
    void *const src[5] = {s.L0[a], s.L1[a], s.ur[a], s.up[a], s.uz[a]};
    void *const dst[5] = {s.L0[b], s.L1[b], s.ur[b], s.up[b], s.uz[b]};
    launch_sort_payload(m, s, counted, 4, 5, src, dst, st);
}

void launch_zero_u64(unsigned long long *p, int64_t n, hipStream_t st) {
    if (n > 0) hipLaunchKernelGGL(k_zero_u64, dim3(nblk(n, 256)), dim3(256), 0, st, p, n);
}

static int node_blocks(const DevMesh &m) { return (int)nblk(m.n0 > m.n1 ? m.n0 : m.n1, 256); }

void launch_diag_final(const DevMesh &m, DevState &s, bool in_step, bool plain, hipStream_t st) {
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(kFinalThreads), 0, st, s, node_blocks(m), in_step ? 1 : 0,
                       plain ? 1 : 0, 0);
}

void launch_diag_in_step(const DevMesh &m, DevState &s, hipStream_t st) {
    hipLaunchKernelGGL(k_node_diag, dim3(node_blocks(m)), dim3(256), 0, st, m, s, 1, (int)nblk(m.n2, 256),
                       (int)nblk(m.n1, 256));
    launch_diag_final(m, s, true, false, st);
}

void launch_spmv_diag(const DevMesh &m, DevState &s, hipStream_t st) {
    const int nb_node = (int)nblk(m.n0, 256), nb_spmv = (int)nblk(m.n1, 256);
    hipLaunchKernelGGL(k_spmv_node, dim3(nb_node + nb_spmv), dim3(256), 0, st, m, s, nb_node, (int)nblk(m.n2, 256),
                       nb_spmv);
}

void launch_step_final(const DevMesh &m, DevState &s, hipStream_t st) {
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(kFinalThreads), 0, st, s, (int)nblk(m.n0, 256), 1, 0,
                       (int)nblk(m.n1, 256));
}

void launch_diag_now(const DevMesh &m, DevState &s, hipStream_t st) {
    launch_zero_u64(s.Qloc, 3ll * m.n2, st);
    if (s.capacity)   // general charge multiples (the on-demand path is not the hot one)
        hipLaunchKernelGGL(k_charge_now<false>, dim3(nblk(s.capacity, kChunk)), dim3(kWG), 0, st, m, s);
    hipLaunchKernelGGL(k_node_diag, dim3(node_blocks(m)), dim3(256), 0, st, m, s, 0, 0, 0);
    launch_diag_final(m, s, false, false, st);
}

}  // namespace axp
