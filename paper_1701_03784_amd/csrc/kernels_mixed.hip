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
// Lambda_k = lambda_k 2^24 exactly (Lambda_2 = 2^24 - Lambda_0 - Lambda_1).
// A straight piece of path from Lambda^s to Lambda^e inside T contributes
// Lambda^s_{k+1} Lambda^e_{k+2} - Lambda^s_{k+2} Lambda^e_{k+1} (units 2^-48)
// to the current of side k (oriented from local node k+1 to k+2); the
// sum of these over a node's sides is exactly 2^24 times the change of the
// node's Lambda, so the continuity equation holds bit-exactly.
#include <hip/hip_runtime.h>

#include "device.h"

namespace axp {

constexpr int kS = 1 << 24;
constexpr float kInvS = 1.0f / 16777216.0f;
constexpr int kTagAxis = 2;

__device__ __forceinline__ int xcd_block(int bid, int nb) {
    // consecutive logical blocks on the same XCD (blocks are dealt round-robin over 8 XCDs)
    int x = bid & 7, i = bid >> 3, per = nb >> 3, rem = nb & 7;
    return x < rem ? x * (per + 1) + i : rem * (per + 1) + (x - rem) * per + i;
}

__device__ __forceinline__ int sel3(int k, int a, int b, int c) { return k == 0 ? a : (k == 1 ? b : c); }

// ------------------------------------------------------------------ faces
__global__ __launch_bounds__(256) void k_tri_pass(DevMesh m, DevState s) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m.n2) return;
    const int4 e = m.tedge[t];
    const int inst = m.tinst ? m.tinst[t] : 0;
    const double dt = m.inst[inst].dt;
    float E0 = s.E[e.x], E1 = s.E[e.y], E2 = s.E[e.z];
    if (e.w & 1) E0 = -E0;
    if (e.w & 2) E1 = -E1;
    if (e.w & 4) E2 = -E2;
    const double bo = s.B[t];
    const double bn = bo - dt * ((double)E0 + (double)E1 + (double)E2);   // circulation along the CCW boundary
    s.B[t] = bn;
    s.Bprev[t] = bo;
    s.HBdt[t] = m.Hdt[t] * bn;
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
    s.Jloc[3 * t] = 0ull;
    s.Jloc[3 * t + 1] = 0ull;
    s.Jloc[3 * t + 2] = 0ull;
}

// -------------------------------------------------------------- particles
constexpr int kPPT = 4;          // particles per thread (consecutive in storage)
constexpr int kWG = 256;
constexpr int kWin = 512;        // faces in the LDS current window

struct WinAcc {
    unsigned long long *lds;
    int base;
    unsigned long long *glob;
};

__device__ __forceinline__ void dep3(const WinAcc &w, int t, long long c0, long long c1, long long c2) {
    const int rel = t - w.base;
    if (rel >= 0 && rel < kWin) {
        if (c0) atomicAdd(&w.lds[3 * rel], (unsigned long long)c0);
        if (c1) atomicAdd(&w.lds[3 * rel + 1], (unsigned long long)c1);
        if (c2) atomicAdd(&w.lds[3 * rel + 2], (unsigned long long)c2);
    } else {
        if (c0) atomicAdd(&w.glob[3 * t], (unsigned long long)c0);
        if (c1) atomicAdd(&w.glob[3 * t + 1], (unsigned long long)c1);
        if (c2) atomicAdd(&w.glob[3 * t + 2], (unsigned long long)c2);
    }
}

// current of the straight piece s -> e inside one face, per side k
__device__ __forceinline__ void piece_current(int s0, int s1, int s2, int e0, int e1, int e2, int kq,
                                              long long &c0, long long &c1, long long &c2) {
    c0 = ((long long)s1 * e2 - (long long)s2 * e1) * kq;
    c1 = ((long long)s2 * e0 - (long long)s0 * e2) * kq;
    c2 = ((long long)s0 * e1 - (long long)s1 * e0) * kq;
}

struct Particle {
    int cell;
    uint32_t L0, L1;
    float ur, up, uz;
};

// Push one particle and walk it; first-piece current goes to the register
// accumulator (acc_t, a0..a2), the rest to the window / global arrays.
__device__ __forceinline__ void push_walk(const DevMesh &m, const DevState &s, Particle &P, const WinAcc &w,
                                          int &acc_t, long long &a0, long long &a1, long long &a2, int max_walk) {
    if (P.cell < 0) return;
    const int T = P.cell & kCellMask;
    const int sp = (P.cell >> kCellBits) & 15;
    const int inst = m.tinst ? m.tinst[T] : 0;
    const InstConst &ic = m.inst[inst];
    const float qe = ic.qe[sp], qb = ic.qb[sp];
    const int kq = ic.kq[sp];
    int L0 = (int)P.L0, L1 = (int)P.L1, L2 = kS - L0 - L1;
    const float l0 = L0 * kInvS, l1 = L1 * kInvS, l2 = L2 * kInvS;
    // gather (Whitney 1-form E, face-constant B_phi, external B_z)
    const float4 f0 = s.f0[T], f1 = s.f1[T];
    const float Ez = l0 * f0.x + l1 * f0.z + l2 * f1.x;
    const float Er = l0 * f0.y + l1 * f0.w + l2 * f1.y;
    const float Bp = f1.z, Bz = ic.bz;
    // relativistic Boris with u normalised by c; basis (rho, phi, z)
    const float umr = P.ur + qe * Er, ump = P.up, umz = P.uz + qe * Ez;
    const float igm = __builtin_amdgcn_rsqf(1.0f + umr * umr + ump * ump + umz * umz);
    const float tp = qb * Bp * igm, tz = qb * Bz * igm;
    const float f = 2.0f / (1.0f + tp * tp + tz * tz);
    const float sp_ = f * tp, sz = f * tz;
    const float vr = umr + (ump * tz - umz * tp);
    const float vp = ump - umr * tz;
    const float vz = umz + umr * tp;
    float ur = umr + (vp * sz - vz * sp_) + qe * Er;
    float up = ump - vr * sz;
    float uz = umz + vr * sp_ + qe * Ez;
    const float u2 = ur * ur + up * up + uz * uz;
    if (!(u2 < 3.0e38f)) {     // non-finite or absurd momentum: count, stop the particle
        atomicAdd(&s.ctr->nan_count, 1ull);
        ur = up = uz = 0.0f;
    }
    const float ig = __builtin_amdgcn_rsqf(1.0f + ur * ur + up * up + uz * uz);
    // move in the local Cartesian frame, rotate back to the meridian plane
    const float4 r4 = m.rho4[T];
    const float rho = l0 * r4.x + l1 * r4.y + l2 * r4.z;
    const float dr = ur * ig * ic.cdt, dp = up * ig * ic.cdt, dz = uz * ig * ic.cdt;
    const float X = rho + dr;
    const float r1 = __builtin_sqrtf(X * X + dp * dp);
    if (r1 > 0.0f) {
        const float ir = 1.0f / r1;
        const float cs = X * ir, sn = dp * ir;
        const float nr = cs * ur + sn * up;
        up = -sn * ur + cs * up;
        ur = nr;
    }
    const float den = r1 + rho;
    float fr = den > 0.0f ? (2.0f * rho * dr + dr * dr + dp * dp) / den : 0.0f;
    float fz = dz;
    P.ur = ur; P.up = up; P.uz = uz;

    // walk across faces; element-local integer coordinates
    int t = T, entry = -1;
    bool first = true;
    for (int seg = 0;; ++seg) {
        const float4 g = m.gS[t];
        const float d0f = fminf(fmaxf(g.x * fz + g.y * fr, -1.0e9f), 1.0e9f);
        const float d1f = fminf(fmaxf(g.z * fz + g.w * fr, -1.0e9f), 1.0e9f);
        int d0 = (int)__builtin_rintf(d0f), d1 = (int)__builtin_rintf(d1f), d2 = -d0 - d1;
        // never leave through the side just entered (rounding); slide along it instead
        if (entry == 0 && d0 < 0) { d0 = 0; d2 = -d1; }
        if (entry == 1 && d1 < 0) { d1 = 0; d2 = -d0; }
        if (entry == 2 && d2 < 0) { d2 = 0; d1 = -d0; }
        const int e0 = L0 + d0, e1 = L1 + d1, e2 = L2 + d2;
        long long c0, c1, c2;
        if (e0 >= 0 && e1 >= 0 && e2 >= 0) {
            piece_current(L0, L1, L2, e0, e1, e2, kq, c0, c1, c2);
            if (first && t == acc_t) { a0 += c0; a1 += c1; a2 += c2; }
            else if (first) { dep3(w, acc_t, a0, a1, a2); acc_t = t; a0 = c0; a1 = c1; a2 = c2; }
            else dep3(w, t, c0, c1, c2);
            L0 = e0; L1 = e1; L2 = e2;
            break;
        }
        // exit side: smallest Lambda_k / (-d_k) among the coordinates going negative (ties: lower k)
        int kx = -1;
        long long num = 0, dd = 1;
        if (e0 < 0) { kx = 0; num = L0; dd = -(long long)d0; }
        if (e1 < 0 && (kx < 0 || (long long)L1 * dd < num * (-(long long)d1))) { kx = 1; num = L1; dd = -(long long)d1; }
        if (e2 < 0 && (kx < 0 || (long long)L2 * dd < num * (-(long long)d2))) { kx = 2; num = L2; dd = -(long long)d2; }
        const float sx = (float)num / (float)dd;
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
        if (first && t == acc_t) { a0 += c0; a1 += c1; a2 += c2; }
        else if (first) { dep3(w, acc_t, a0, a1, a2); acc_t = t; a0 = c0; a1 = c1; a2 = c2; }
        else dep3(w, t, c0, c1, c2);
        first = false;
        const float rem = 1.0f - sx;
        fz *= rem;
        fr *= rem;
        const int4 nb = m.nbr[t];
        const int n = sel3(kx, nb.x, nb.y, nb.z);
        if (n < 0) {
            if (-n == kTagAxis) {           // rho = 0 cannot be crossed: stay on it
                L0 = x0; L1 = x1; L2 = x2;
                break;
            }
            // conductor / open boundary: absorbed; its charge stays on the wall nodes
            const int4 tn = m.tnodes[t];
            const int na = sel3(ka, tn.x, tn.y, tn.z), nbn = sel3(kb, tn.x, tn.y, tn.z);
            atomicAdd((unsigned long long *)&s.Qres[na], (unsigned long long)((long long)xa * kq));
            atomicAdd((unsigned long long *)&s.Qres[nbn], (unsigned long long)((long long)xb * kq));
            atomicAdd(&s.ctr->n_absorbed, 1ull);
            P.cell = -1;
            return;
        }
        const unsigned map = ((unsigned)nb.w >> (4 * kx)) & 15u;
        const int pa = map & 3, pb = map >> 2, q = 3 - pa - pb;
        L0 = pa == 0 ? xa : (pb == 0 ? xb : 0);
        L1 = pa == 1 ? xa : (pb == 1 ? xb : 0);
        L2 = pa == 2 ? xa : (pb == 2 ? xb : 0);
        entry = q;
        t = n;
        if (seg + 1 >= max_walk) {          // cut: the particle stops at the crossing
            atomicAdd(&s.ctr->walk_overflow, 1ull);
            break;
        }
    }
    P.cell = t | (sp << kCellBits);
    P.L0 = (uint32_t)L0;
    P.L1 = (uint32_t)L1;
}

__global__ __launch_bounds__(kWG) void k_particles(DevMesh m, DevState s, int max_walk) {
    __shared__ unsigned long long lacc[3 * kWin];
    __shared__ int s_base;
    const int chunk = xcd_block(blockIdx.x, gridDim.x);
    const long long n = (long long)s.ctr->n_slots;
    const long long pb = (long long)chunk * kWG * kPPT;
    if (pb >= n) return;
    const int c = s.cur;
    int32_t *cell = s.cell[c];
    uint32_t *L0 = s.L0[c], *L1 = s.L1[c];
    float *ur = s.ur[c], *up = s.up[c], *uz = s.uz[c];
    if (threadIdx.x == 0) {
        const int c0 = cell[pb];
        s_base = (c0 >= 0 ? (c0 & kCellMask) : 0) - kWin / 8;
    }
    for (int i = threadIdx.x; i < 3 * kWin; i += kWG) lacc[i] = 0ull;
    __syncthreads();
    WinAcc w{lacc, s_base, s.Jloc};
    const long long p0 = pb + (long long)threadIdx.x * kPPT;
    Particle P[kPPT];
    if (p0 + kPPT <= n) {
        const int4 cc = *reinterpret_cast<const int4 *>(cell + p0);
        const uint4 a = *reinterpret_cast<const uint4 *>(L0 + p0);
        const uint4 b = *reinterpret_cast<const uint4 *>(L1 + p0);
        const float4 x = *reinterpret_cast<const float4 *>(ur + p0);
        const float4 y = *reinterpret_cast<const float4 *>(up + p0);
        const float4 z = *reinterpret_cast<const float4 *>(uz + p0);
        P[0] = {cc.x, a.x, b.x, x.x, y.x, z.x};
        P[1] = {cc.y, a.y, b.y, x.y, y.y, z.y};
        P[2] = {cc.z, a.z, b.z, x.z, y.z, z.z};
        P[3] = {cc.w, a.w, b.w, x.w, y.w, z.w};
    } else {
#pragma unroll
        for (int j = 0; j < kPPT; ++j) {
            const long long p = p0 + j;
            if (p < n) P[j] = {cell[p], L0[p], L1[p], ur[p], up[p], uz[p]};
            else P[j] = {-1, 0u, 0u, 0.f, 0.f, 0.f};
        }
    }
    int acc_t = -1;
    long long a0 = 0, a1 = 0, a2 = 0;
#pragma unroll
    for (int j = 0; j < kPPT; ++j) push_walk(m, s, P[j], w, acc_t, a0, a1, a2, max_walk);
    if (acc_t >= 0) dep3(w, acc_t, a0, a1, a2);
    if (p0 + kPPT <= n) {
        *reinterpret_cast<int4 *>(cell + p0) = make_int4(P[0].cell, P[1].cell, P[2].cell, P[3].cell);
        *reinterpret_cast<uint4 *>(L0 + p0) = make_uint4(P[0].L0, P[1].L0, P[2].L0, P[3].L0);
        *reinterpret_cast<uint4 *>(L1 + p0) = make_uint4(P[0].L1, P[1].L1, P[2].L1, P[3].L1);
        *reinterpret_cast<float4 *>(ur + p0) = make_float4(P[0].ur, P[1].ur, P[2].ur, P[3].ur);
        *reinterpret_cast<float4 *>(up + p0) = make_float4(P[0].up, P[1].up, P[2].up, P[3].up);
        *reinterpret_cast<float4 *>(uz + p0) = make_float4(P[0].uz, P[1].uz, P[2].uz, P[3].uz);
    } else {
#pragma unroll
        for (int j = 0; j < kPPT; ++j) {
            const long long p = p0 + j;
            if (p < n) {
                cell[p] = P[j].cell; L0[p] = P[j].L0; L1[p] = P[j].L1;
                ur[p] = P[j].ur; up[p] = P[j].up; uz[p] = P[j].uz;
            }
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 3 * kWin; i += kWG) {
        const unsigned long long v = lacc[i];
        const long long gi = 3ll * w.base + i;
        if (v != 0ull && gi >= 0 && gi < 3ll * m.n2) atomicAdd(&s.Jloc[gi], v);
    }
}

// ------------------------------------------------------------------ edges
// etri.z packs: bits 0-1 side in left face, 2-3 side in right face,
// bit 4 left sign negative, bit 5 right sign negative, bit 6 free edge.
__global__ __launch_bounds__(256) void k_edge_pass(DevMesh m, DevState s, int keep_j) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m.n1) return;
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
    if (!(et.z & 64)) return;          // conductor edge: tangential E stays 0
    const double d = s.D[e] + acc;
    s.D[e] = d;
    s.D32[e] = (float)d;
}

// ------------------------------------------------------------------- SpMV
__global__ __launch_bounds__(256) void k_spmv(DevMesh m, DevState s) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m.n1) return;
    const int sl = i >> 6, lane = i & 63;
    const int64_t beg = m.m_sptr[sl];
    const int len = m.m_slen[sl];
    const float *v = m.m_val + beg + lane;
    const int32_t *c = m.m_col + beg + lane;
    float acc = 0.0f;
    for (int j = 0; j < len; ++j) acc = fmaf(v[64 * j], s.D32[c[64 * j]], acc);
    s.E[i] = acc;
}

// ------------------------------------------------------------------- sort
__global__ __launch_bounds__(256) void k_zero_i32(int32_t *p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

__global__ __launch_bounds__(256) void k_count(DevState s) {
    const long long n = (long long)s.ctr->n_slots;
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int c = s.cell[s.cur][p];
    if (c >= 0) atomicAdd(&s.cnt[c & kCellMask], 1);
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

__global__ __launch_bounds__(256) void k_scatter(DevState s) {
    const long long n = (long long)s.ctr->n_slots;
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int a = s.cur, b = 1 - s.cur;
    const int c = s.cell[a][p];
    if (c < 0) return;
    const int q = atomicAdd(&s.cnt[c & kCellMask], 1);
    s.cell[b][q] = c;
    s.L0[b][q] = s.L0[a][p];
    s.L1[b][q] = s.L1[a][p];
    s.ur[b][q] = s.ur[a][p];
    s.up[b][q] = s.up[a][p];
    s.uz[b][q] = s.uz[a][p];
}

__global__ void k_set_slots(DevState s, const int32_t *total) { s.ctr->n_slots = (unsigned long long)(*total); }

// ------------------------------------------------------------ diagnostics
__global__ __launch_bounds__(256) void k_charge_init(DevMesh m, DevState s) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < m.n0) s.Qfx[v] = s.Qres[v];
}

__global__ __launch_bounds__(256) void k_charge(DevMesh m, DevState s) {
    const long long n = (long long)s.ctr->n_slots;
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int c = s.cell[s.cur][p];
    if (c < 0) return;
    const int T = c & kCellMask, sp = (c >> kCellBits) & 15;
    const int inst = m.tinst ? m.tinst[T] : 0;
    const long long kq = m.inst[inst].kq[sp];
    const long long L0 = s.L0[s.cur][p], L1 = s.L1[s.cur][p], L2 = kS - L0 - L1;
    const int4 tn = m.tnodes[T];
    atomicAdd((unsigned long long *)&s.Qfx[tn.x], (unsigned long long)(kq * L0));
    atomicAdd((unsigned long long *)&s.Qfx[tn.y], (unsigned long long)(kq * L1));
    atomicAdd((unsigned long long *)&s.Qfx[tn.z], (unsigned long long)(kq * L2));
}

__device__ __forceinline__ void atomic_max_pos(unsigned long long *a, double v) {
    atomicMax(a, (unsigned long long)__double_as_longlong(v));
}

// Gauss residual res_v = (Ddiv D)_v - Q_v, its drift from res^0, and the
// continuity residual 2^24 (Q^{n+1} - Q^n) + (Ddiv J)_v in fixed point.
__global__ __launch_bounds__(256) void k_node_diag(DevMesh m, DevState s, int have_prev, int first) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= m.n0) return;
    const int inst = m.ninst ? m.ninst[v] : 0;
    double div = 0.0, mag = 0.0;
    long long divj = 0;
    for (int k = m.nptr[v]; k < m.nptr[v + 1]; ++k) {
        const int e = m.nedge[k];
        const double d = s.D[e];
        div += m.nsign[k] > 0 ? d : -d;
        mag += fabs(d);
        if (have_prev) divj += m.nsign[k] > 0 ? s.Jfx[e] : -s.Jfx[e];
    }
    const double q = (double)s.Qfx[v] * m.inst[inst].qscale;
    const double g = div - q;
    if (have_prev) {
        const long long dce = (long long)kS * (s.Qfx[v] - s.Qprev[v]) + divj;
        atomicMax(&s.diag->dce_max, (unsigned long long)(dce < 0 ? -dce : dce));
    }
    s.Qprev[v] = s.Qfx[v];
    if (m.nfree[v]) {
        if (first) s.g0[v] = g;
        atomic_max_pos(&s.diag->gauss_drift_bits, fabs(g - s.g0[v]));
        atomic_max_pos(&s.diag->gauss_abs_bits, fabs(g));
        atomic_max_pos(&s.diag->gauss_scale_bits, mag);
    }
    atomicAdd(&s.diag->Qtot, q);
}

__device__ __forceinline__ double block_sum(double v) {
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

__global__ __launch_bounds__(256) void k_energy_fields(DevMesh m, DevState s) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    double we = 0.0, wb = 0.0;
    if (i < m.n1) {
        double ae = 0.0;
        for (int64_t k = m.a_ptr[i]; k < m.a_ptr[i + 1]; ++k) ae += m.a_val[k] * (double)s.E[m.a_col[k]];
        we = 0.5 * (double)s.E[i] * ae;
    }
    if (i < m.n2) {
        const int inst = m.tinst ? m.tinst[i] : 0;
        wb = 0.5 * (m.Hdt[i] / m.inst[inst].dt) * s.B[i] * s.Bprev[i];
    }
    we = block_sum(we);
    wb = block_sum(wb);
    if (threadIdx.x == 0) {
        atomicAdd(&s.diag->WE, we);
        atomicAdd(&s.diag->WB, wb);
    }
}

__global__ __launch_bounds__(256) void k_energy_kin(DevMesh m, DevState s) {
    const long long n = (long long)s.ctr->n_slots;
    const long long p = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double wk = 0.0;
    if (p < n) {
        const int c = s.cell[s.cur][p];
        if (c >= 0) {
            const int T = c & kCellMask, sp = (c >> kCellBits) & 15;
            const int inst = m.tinst ? m.tinst[T] : 0;
            const double a = s.ur[s.cur][p], b = s.up[s.cur][p], z = s.uz[s.cur][p];
            const double u2 = a * a + b * b + z * z;
            wk = m.inst[inst].mw[sp] * (u2 / (sqrt(1.0 + u2) + 1.0));   // (gamma - 1) without cancellation
        }
    }
    wk = block_sum(wk);
    if (threadIdx.x == 0) atomicAdd(&s.diag->WK, wk);
}

// --------------------------------------------------------------- launchers
static inline unsigned nblk(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

void launch_tri_pass(const DevMesh &m, DevState &s, hipStream_t st) {
    if (m.n2 == 0) return;
    hipLaunchKernelGGL(k_tri_pass, dim3(nblk(m.n2, 256)), dim3(256), 0, st, m, s);
}

void launch_particles(const DevMesh &m, DevState &s, int max_walk, hipStream_t st) {
    if (s.capacity == 0) return;
    hipLaunchKernelGGL(k_particles, dim3(nblk(s.capacity, kWG * kPPT)), dim3(kWG), 0, st, m, s, max_walk);
}

void launch_edge_pass(const DevMesh &m, DevState &s, bool keep_j, hipStream_t st) {
    hipLaunchKernelGGL(k_edge_pass, dim3(nblk(m.n1, 256)), dim3(256), 0, st, m, s, keep_j ? 1 : 0);
}

void launch_spmv(const DevMesh &m, DevState &s, hipStream_t st) {
    hipLaunchKernelGGL(k_spmv, dim3(nblk(m.n1, 256)), dim3(256), 0, st, m, s);
}

void launch_sort(const DevMesh &m, DevState &s, hipStream_t st) {
    if (s.capacity == 0) return;
    const int n = m.n2;
    const int nb = (int)nblk(n, 1024);
    hipLaunchKernelGGL(k_zero_i32, dim3(nblk(n + 1, 256)), dim3(256), 0, st, s.cnt, (int64_t)n + 1);
    hipLaunchKernelGGL(k_count, dim3(nblk(s.capacity, 256)), dim3(256), 0, st, s);
    hipLaunchKernelGGL(k_scan_local, dim3(nb), dim3(256), 0, st, s.cnt, s.blk, n);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(256), 0, st, s.blk, nb, s.cnt + n, s);
    hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(256), 0, st, s.cnt, s.blk, n);
    hipLaunchKernelGGL(k_scatter, dim3(nblk(s.capacity, 256)), dim3(256), 0, st, s);
    hipLaunchKernelGGL(k_set_slots, dim3(1), dim3(1), 0, st, s, s.cnt + n);
    s.cur = 1 - s.cur;
}

void launch_diag(const DevMesh &m, DevState &s, bool have_prev_q, bool first, hipStream_t st) {
    (void)hipMemsetAsync(s.diag, 0, sizeof(DevDiag), st);
    hipLaunchKernelGGL(k_charge_init, dim3(nblk(m.n0, 256)), dim3(256), 0, st, m, s);
    if (s.capacity) hipLaunchKernelGGL(k_charge, dim3(nblk(s.capacity, 256)), dim3(256), 0, st, m, s);
    hipLaunchKernelGGL(k_node_diag, dim3(nblk(m.n0, 256)), dim3(256), 0, st, m, s, have_prev_q ? 1 : 0, first ? 1 : 0);
    const int64_t ne = m.n1 > m.n2 ? m.n1 : m.n2;
    hipLaunchKernelGGL(k_energy_fields, dim3(nblk(ne, 256)), dim3(256), 0, st, m, s);
    if (s.capacity) hipLaunchKernelGGL(k_energy_kin, dim3(nblk(s.capacity, 256)), dim3(256), 0, st, m, s);
}

}  // namespace axp
