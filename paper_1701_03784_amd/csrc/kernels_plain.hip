// FP64 variant of the time step: the reference point of the mixed step.
// Same kernels and data flow (face pass, particle kernel with an LDS walk
// queue and current window, edge pass, sliced-ELL SpMV, counting sort by
// face), but every quantity is FP64: barycentric positions, momenta, the
// gather tile, the SPAI values, E, and the currents, which are summed with
// FP64 atomics (so their order, and the last bits, vary from run to run).
//
//   k_tri_pass_d   eq. (full_d_dfl) and the Whitney gather tile (Sec. 3.2)
//   k_particles_d  gather, relativistic Boris or Vay push (eqs. DNE, DLE), axisymmetric
//                  position update, walk with the current of eq. (current)
//   k_edge_pass_d  D += dt C^T H B^{n+1/2} - dt J (eq. full_d_dal, D-form)
//   k_spmv_d       E = M D
#include <hip/hip_runtime.h>

#include "device.h"
#include "diag.h"
#include "inject.h"

namespace axp {

namespace {

constexpr int kTagAxisD = 2;
constexpr int kWGd = 256;
constexpr int kChunkD = 1024;          // particles per block (as the mixed step)
constexpr int kPPTd = kChunkD / kWGd;

__device__ __forceinline__ double sel3d(int k, double a, double b, double c) { return k == 0 ? a : (k == 1 ? b : c); }
__device__ __forceinline__ int sel3i(int k, int a, int b, int c) { return k == 0 ? a : (k == 1 ? b : c); }

__device__ __forceinline__ void fadd(double *a, double v) {
    if (v != 0.0) unsafeAtomicAdd(a, v);       // hardware FP64 atomic add
}

__device__ __forceinline__ double block_sum_d(double v) {
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

// one face of the FP64 face pass; returns 1/2 B^{n+1/2} H B^{n-1/2} when diag
__device__ __forceinline__ double tri_face_d(const DevMesh &m, const DevState &s, const DevPlain &p, double dt,
                                             const FieldSrc &fs, const DevLayers &lay, int t, bool diag) {
    const int4 e = m.tedge[t];
    double E0 = p.E[e.x], E1 = p.E[e.y], E2 = p.E[e.z];
    if (e.w & 1) E0 = -E0;
    if (e.w & 2) E1 = -E1;
    if (e.w & 4) E2 = -E2;
    const double bo = s.B[t];
    double bn = bo - dt * (E0 + E1 + E2);
    for (int k = 0; k < fs.n_src; ++k)          // magnetic point sources (Sec. 4.1)
        if (t == fs.src_face[k]) {
            const double tt = double(s.ctr->step) * fs.dt - fs.t0[k];
            const double a = tt / (2.0 * fs.sig[k]);
            bn -= dt * fs.amp[k] * exp(-a * a) * cos(fs.w[k] * tt);
        }
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
    const double4 g = p.grad[t];
    const double g0z = g.x, g0r = g.y, g1z = g.z, g1r = g.w;
    const double g2z = -(g0z + g1z), g2r = -(g0r + g1r);
    // E(lambda) = sum_j lambda_j a_j,  a_j = E_{j-1} grad lam_{j+1} - E_{j+1} grad lam_{j-1}
    double4 f0, f1;
    f0.x = E2 * g1z - E1 * g2z;
    f0.y = E2 * g1r - E1 * g2r;
    f0.z = E0 * g2z - E2 * g0z;
    f0.w = E0 * g2r - E2 * g0r;
    f1.x = E1 * g0z - E0 * g1z;
    f1.y = E1 * g0r - E0 * g1r;
    f1.z = (bn + bo) * p.rho[t].w;          // B_phi = (B^{n+1/2} + B^{n-1/2}) / (2 area)
    f1.w = 0.0;
    p.f0[t] = f0;
    p.f1[t] = f1;
    if (t == fs.probe_face) {                   // E^n at the probe point (Whitney gather)
        const long long i = (long long)s.ctr->step - fs.probe_start;
        if (i >= 0 && i < fs.probe_cap) {
            const double l0 = fs.probe_l0, l1 = fs.probe_l1, l2 = 1.0 - l0 - l1;
            fs.probe[2 * i] = l0 * f0.x + l1 * f0.z + l2 * f1.x;
            fs.probe[2 * i + 1] = l0 * f0.y + l1 * f0.w + l2 * f1.y;
        }
    }
    p.Jloc[3 * t] = 0.0;
    p.Jloc[3 * t + 1] = 0.0;
    p.Jloc[3 * t + 2] = 0.0;
    return diag ? 0.5 * (m.Hdt[t] / dt) * bn * bo : 0.0;
}

__global__ __launch_bounds__(256) void k_tri_pass_d(DevMesh m, DevState s, DevPlain p, double dt, FieldSrc fs,
                                                    DevLayers lay, int diag) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const double wb = t < m.n2 ? tri_face_d(m, s, p, dt, fs, lay, t, diag != 0) : 0.0;
    if (!diag) return;                          // uniform across the grid
    const double tot = block_sum_d(wb);
    if (threadIdx.x == 0) s.part_face[blockIdx.x] = tot;
}

// current of the straight piece s -> e inside one face, per side k
// (side k runs from local node k+1 to k+2), times the charge multiple
__device__ __forceinline__ void piece_d(double s0, double s1, double s2, double e0, double e1, double e2, double kq,
                                        double &c0, double &c1, double &c2) {
    c0 = kq * (s1 * e2 - s2 * e1);
    c1 = kq * (s2 * e0 - s0 * e2);
    c2 = kq * (s0 * e1 - s1 * e0);
}

// ---------------------------------------------------------------- particles
// k_particles_d: the structure of the mixed step's particle kernel in FP64.
// Blocks of 1024 consecutive particles, 4 per thread.  Phase 1: gather,
// Boris, position update; the current of a path that stays in its face is
// folded per face by a segmented scan across the wave into the block's LDS
// window (FP64 LDS atomics); a particle that leaves its face is queued in
// LDS.  Phase 2: the block walks the queue.  Phase 3: owners store their
// particles, and the window is added to the face currents with FP64 global
// atomics (whose order, and so the last bits, vary from run to run).
constexpr int kWinD = 512;
constexpr int kWinLeadD = 192;

typedef __attribute__((address_space(3))) double lds_double;

struct WinD {
    lds_double *jl;  // LDS, 3 * kWinD (typed as LDS so that its adds stay ds_add_f64)
    int *cl;         // LDS, kWinD
    int base;
};

__device__ __forceinline__ void lds_fadd(lds_double *a, double v) {
    if (v != 0.0) __builtin_amdgcn_ds_atomic_fadd_f64(a, v);
}

__device__ __forceinline__ void win_add_j_d(const WinD &w, double *J, int t, double a0, double a1, double a2) {
    const int rel = t - w.base;
    if (rel >= 0 && rel < kWinD) {
        lds_fadd(&w.jl[3 * rel], a0);
        lds_fadd(&w.jl[3 * rel + 1], a1);
        lds_fadd(&w.jl[3 * rel + 2], a2);
    } else {
        fadd(&J[3 * t], a0);
        fadd(&J[3 * t + 1], a1);
        fadd(&J[3 * t + 2], a2);
    }
}

__device__ __forceinline__ void win_add_c_d(const WinD &w, int *cnt, int t, int v) {
    const int rel = t - w.base;
    if (rel >= 0 && rel < kWinD) atomicAdd(&w.cl[rel], v);
    else atomicAdd(&cnt[t], v);
}

__device__ __forceinline__ int lane_run_d(int t) {
    const int lane = threadIdx.x & 63;
    const int tp = __shfl_up(t, 1, 64);
    const unsigned long long heads = __ballot(lane == 0 || tp != t);
    return __popcll(heads & ((2ull << lane) - 1ull));
}

__device__ __forceinline__ bool run_tail_d(int t) {
    const int lane = threadIdx.x & 63;
    const int tn = __shfl_down(t, 1, 64);
    return lane == 63 || tn != t;
}

// segmented scan over runs of lanes with the same face; the run's last lane deposits
__device__ __forceinline__ void wave_deposit_d(const WinD &w, double *J, int t, double a0, double a1, double a2) {
    const int lane = threadIdx.x & 63;
    const int run = lane_run_d(t);
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int ro = __shfl_up(run, off, 64);
        const double b0 = __shfl_up(a0, off, 64);
        const double b1 = __shfl_up(a1, off, 64);
        const double b2 = __shfl_up(a2, off, 64);
        if (lane >= off && ro == run) { a0 += b0; a1 += b1; a2 += b2; }
    }
    if (run_tail_d(t) && t >= 0) win_add_j_d(w, J, t, a0, a1, a2);
}

__device__ __forceinline__ void wave_count_d(const WinD &w, int *cnt, int t, int c) {
    const int lane = threadIdx.x & 63;
    const int run = lane_run_d(t);
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int ro = __shfl_up(run, off, 64);
        const int b = __shfl_up(c, off, 64);
        if (lane >= off && ro == run) c += b;
    }
    if (run_tail_d(t) && t >= 0 && c) win_add_c_d(w, cnt, t, c);
}

// LDS walk queue entries per block (about a fifth of the particles leave
// their face in a step at half the stability limit); a block with more
// movers has its owners walk the rest
constexpr int kQCapD = 512;

struct MoverD {
    int cell;
    double l0, l1, fz, fr;
};

struct ParticleD {
    int cell;
    double l0, l1, ur, up, uz;
};

// gather, momentum push with u normalised by c in (rho, phi, z) (relativistic
// Boris, or Vay's pusher when VAY), push in the local Cartesian frame and
// rotate back: returns the meridian displacement
template <bool VAY>
__device__ __forceinline__ void push_d(const DevState &s, ParticleD &P, const PlainConst &k, int sp, const double4 f0,
                                       const double4 f1, const double4 r4, double &fz, double &fr) {
    const double l0 = P.l0, l1 = P.l1, l2 = 1.0 - l0 - l1;
    const double Ez = l0 * f0.x + l1 * f0.z + l2 * f1.x;
    const double Er = l0 * f0.y + l1 * f0.w + l2 * f1.y;
    const double Bp = f1.z, Bz = k.bz;
    const double qe = k.qe[sp], qb = k.qb[sp];
    double ur, up, uz;
    if (!VAY) {
        const double umr = P.ur + qe * Er, ump = P.up, umz = P.uz + qe * Ez;
        const double igm = 1.0 / sqrt(1.0 + umr * umr + ump * ump + umz * umz);
        const double tp = qb * Bp * igm, tz = qb * Bz * igm;
        const double f = 2.0 / (1.0 + tp * tp + tz * tz);
        const double sp_ = f * tp, sz = f * tz;
        const double vr = umr + (ump * tz - umz * tp);
        const double vp = ump - umr * tz;
        const double vz = umz + umr * tp;
        ur = umr + (vp * sz - vz * sp_) + qe * Er;
        up = ump - vr * sz;
        uz = umz + vr * sp_ + qe * Ez;
    } else {
        // u' = u + 2 qe E + (u / gamma) x tau; new gamma from the quadratic in
        // gamma^2; exact solve of u = u' + (u / gamma) x tau
        const double taup = qb * Bp, tauz = qb * Bz;
        const double ig0 = 1.0 / sqrt(1.0 + P.ur * P.ur + P.up * P.up + P.uz * P.uz);
        const double vr = P.ur * ig0, vp = P.up * ig0, vz = P.uz * ig0;
        const double ar = P.ur + 2.0 * qe * Er + (vp * tauz - vz * taup);
        const double ap = P.up - vr * tauz;
        const double az = P.uz + 2.0 * qe * Ez + vr * taup;
        const double tau2 = taup * taup + tauz * tauz;
        const double ustar = ap * taup + az * tauz;
        const double sigma = 1.0 + ar * ar + ap * ap + az * az - tau2;
        const double gn = sqrt(0.5 * (sigma + sqrt(sigma * sigma + 4.0 * (tau2 + ustar * ustar))));
        const double tp = taup / gn, tz = tauz / gn;
        const double sc = 1.0 / (1.0 + tp * tp + tz * tz);
        const double at = ustar / gn;
        ur = sc * (ar + (ap * tz - az * tp));
        up = sc * (ap + at * tp - ar * tz);
        uz = sc * (az + at * tz + ar * tp);
    }
    if (!(ur * ur + up * up + uz * uz < 1.0e300)) {
        atomicAdd(&s.ctr->nan_count, 1ull);
        ur = up = uz = 0.0;
    }
    const double ig = k.cdt / sqrt(1.0 + ur * ur + up * up + uz * uz);
    const double rho = l0 * r4.x + l1 * r4.y + l2 * r4.z;
    const double dr = ur * ig, dp = up * ig;
    fz = uz * ig;
    const double X = rho + dr;
    const double r1 = sqrt(X * X + dp * dp);
    if (r1 > 0.0) {
        const double cs = X / r1, sn = dp / r1;
        const double nr = cs * ur + sn * up;
        up = -sn * ur + cs * up;
        ur = nr;
    }
    const double den = r1 + rho;
    fr = den > 0.0 ? (2.0 * rho * dr + dr * dr + dp * dp) / den : 0.0;
    P.ur = ur; P.up = up; P.uz = uz;
}

// walk of one particle that leaves its face (see the mixed step)
__device__ __forceinline__ void walk_mover_d(const DevMesh &m, const DevState &s, const DevPlain &p, const WinD &w,
                                             const PlainConst &k, int max_walk, MoverD &mv) {
    int t = mv.cell & kCellMask;
    const int sp = (mv.cell >> kCellBits) & 15;
    const double kq = k.kq[sp];
    double l0 = mv.l0, l1 = mv.l1, l2 = 1.0 - l0 - l1;
    double fz = mv.fz, fr = mv.fr;
    int entry = -1;
    int newcell = -2;
    double4 g = p.grad[t];
    int4 nb = m.nbr[t];
    for (int seg = 0; newcell == -2; ++seg) {
        double d0 = g.x * fz + g.y * fr, d1 = g.z * fz + g.w * fr, d2 = -d0 - d1;
        // never leave through the side just entered (rounding): slide along it
        if (entry == 0 && d0 < 0.0) { d0 = 0.0; d2 = -d1; }
        if (entry == 1 && d1 < 0.0) { d1 = 0.0; d2 = -d0; }
        if (entry == 2 && d2 < 0.0) { d2 = 0.0; d1 = -d0; }
        const double e0 = l0 + d0, e1 = l1 + d1, e2 = l2 + d2;
        double c0, c1, c2;
        const int tf = t;
        // the path leaves through side k only if lambda_k decreases and goes negative
        if ((e0 >= 0.0 || d0 >= 0.0) && (e1 >= 0.0 || d1 >= 0.0) && (e2 >= 0.0 || d2 >= 0.0)) {
            piece_d(l0, l1, l2, e0, e1, e2, kq, c0, c1, c2);
            l0 = e0; l1 = e1; l2 = e2;
            newcell = t | (sp << kCellBits);
            win_add_j_d(w, p.Jloc, tf, c0, c1, c2);
            break;
        }
        // exit side: smallest lambda_k / (-d_k) among the coordinates going negative
        int kx = -1;
        double best = 3.0;
        if (e0 < 0.0 && d0 < 0.0) { kx = 0; best = l0 / (-d0); }
        if (e1 < 0.0 && d1 < 0.0) { const double v = l1 / (-d1); if (v < best) { kx = 1; best = v; } }
        if (e2 < 0.0 && d2 < 0.0) { const double v = l2 / (-d2); if (v < best) { kx = 2; best = v; } }
        if (kx < 0) {                               // non-finite displacement: stop here
            atomicAdd(&s.ctr->nan_count, 1ull);
            newcell = t | (sp << kCellBits);
            break;
        }
        const double sx = fmin(fmax(best, 0.0), 1.0);
        const int ka = kx == 2 ? 0 : kx + 1, kb = kx == 0 ? 2 : kx - 1;
        double xa = sel3d(ka, l0, l1, l2) + sx * sel3d(ka, d0, d1, d2);
        xa = fmin(fmax(xa, 0.0), 1.0);
        const double xb = 1.0 - xa;
        const double x0 = ka == 0 ? xa : (kb == 0 ? xb : 0.0);
        const double x1 = ka == 1 ? xa : (kb == 1 ? xb : 0.0);
        const double x2 = ka == 2 ? xa : (kb == 2 ? xb : 0.0);
        piece_d(l0, l1, l2, x0, x1, x2, kq, c0, c1, c2);
        win_add_j_d(w, p.Jloc, tf, c0, c1, c2);
        fz *= (1.0 - sx);
        fr *= (1.0 - sx);
        const int nn = sel3i(kx, nb.x, nb.y, nb.z);
        if (nn < 0) {
            if (-nn == kTagAxisD) {                 // rho = 0 cannot be crossed: stay on it
                l0 = x0; l1 = x1; l2 = x2;
                newcell = t | (sp << kCellBits);
            } else {                                // absorbed; its charge stays on the wall nodes
                const int4 tn = m.tnodes[t];
                fadd(&p.Qres[sel3i(ka, tn.x, tn.y, tn.z)], kq * xa);
                fadd(&p.Qres[sel3i(kb, tn.x, tn.y, tn.z)], kq * xb);
                atomicAdd(&s.ctr->n_absorbed, 1ull);
                newcell = -1;
            }
            break;
        }
        const unsigned map = ((unsigned)nb.w >> (4 * kx)) & 15u;
        const int pa = map & 3, pb = map >> 2, q = 3 - pa - pb;
        l0 = pa == 0 ? xa : (pb == 0 ? xb : 0.0);
        l1 = pa == 1 ? xa : (pb == 1 ? xb : 0.0);
        l2 = pa == 2 ? xa : (pb == 2 ? xb : 0.0);
        entry = q;
        t = nn;
        if (seg + 1 >= max_walk) {                  // cut: the particle stops at the crossing
            atomicAdd(&s.ctr->walk_overflow, 1ull);
            newcell = t | (sp << kCellBits);
            break;
        }
        g = p.grad[t];
        nb = m.nbr[t];
    }
    mv.cell = newcell;
    mv.l0 = l0;
    mv.l1 = l1;
}

// gamma - 1 of u / c without cancellation for slow particles
__device__ __forceinline__ double gamma_m1_d(double ur, double up, double uz) {
    const double u2 = ur * ur + up * up + uz * uz;
    return u2 / (sqrt(1.0 + u2) + 1.0);
}

// DIAG: the step evaluates the diagnostics of its start level; the kernel
// then leaves per block W_K = 1/2 (K^{n-1/2} + K^{n+1/2}) over the particles
// it pushes and their count (each wave summed by a fixed butterfly, the
// waves in order).
template <bool VAY, bool DIAG>
__global__ __launch_bounds__(kWGd) void k_particles_d(DevMesh m, DevState s, DevPlain p, PlainConst k, int max_walk,
                                                      int do_count) {
    __shared__ double s_wk[kWGd / 64];
    __shared__ int s_nl[kWGd / 64];
    __shared__ int s_nmv;
    __shared__ int s_base;
    __shared__ double s_jl[3 * kWinD];
    __shared__ int s_cl[kWinD];
    __shared__ MoverD s_mv[kQCapD];
    const int chunk = blockIdx.x;
    const long long n = (long long)s.ctr->n_slots;
    const long long p0 = ((long long)chunk * kWGd + threadIdx.x) * kPPTd;
    if ((long long)chunk * kChunkD >= n) return;
    const int c = s.cur;
    int32_t *cell = s.cell[c];
    double *l0a = p.l0[c], *l1a = p.l1[c], *ura = p.ur[c], *upa = p.up[c], *uza = p.uz[c];
    ParticleD P[kPPTd];
#pragma unroll
    for (int j = 0; j < kPPTd; ++j) {
        const long long q = p0 + j;
        if (q < n) P[j] = {cell[q], l0a[q], l1a[q], ura[q], upa[q], uza[q]};
        else P[j] = {-1, 0.0, 0.0, 0.0, 0.0, 0.0};
    }
    // thread 0 holds the block's first particle: the window starts at its face
    if (threadIdx.x == 0) {
        s_nmv = 0;
        s_base = (P[0].cell >= 0 ? (P[0].cell & kCellMask) : 0) - kWinLeadD;
    }
    for (int i = threadIdx.x; i < 3 * kWinD; i += kWGd) s_jl[i] = 0.0;
    for (int i = threadIdx.x; i < kWinD; i += kWGd) s_cl[i] = 0;
    __syncthreads();
    const WinD w{(lds_double *)s_jl, s_cl, s_base};
    // ---- phase 1: push
    int acc_t = -1;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    int ct = -1, cc = 0;
    bool mover[kPPTd];
    double mfz[kPPTd], mfr[kPPTd];
    int Tc = -1;
    double4 cf0 = make_double4(0.0, 0.0, 0.0, 0.0), cf1 = cf0, cr4 = cf0, cg = cf0;
    double wk = 0.0;
    int nlive = 0;
#pragma unroll
    for (int j = 0; j < kPPTd; ++j) {
        mover[j] = false;
        mfz[j] = mfr[j] = 0.0;
        if (P[j].cell < 0) continue;
        const int T = P[j].cell & kCellMask;
        const int sp = (P[j].cell >> kCellBits) & 15;
        if (T != Tc) {
            Tc = T;
            cf0 = p.f0[T]; cf1 = p.f1[T]; cr4 = p.rho[T]; cg = p.grad[T];
        }
        double fz, fr;
        const double l0 = P[j].l0, l1 = P[j].l1, l2 = 1.0 - l0 - l1;
        if (DIAG) {
            ++nlive;
            wk += k.mw[sp] * gamma_m1_d(P[j].ur, P[j].up, P[j].uz);
        }
        push_d<VAY>(s, P[j], k, sp, cf0, cf1, cr4, fz, fr);
        if (DIAG) wk += k.mw[sp] * gamma_m1_d(P[j].ur, P[j].up, P[j].uz);
        const double d0 = cg.x * fz + cg.y * fr, d1 = cg.z * fz + cg.w * fr, d2 = -d0 - d1;
        const double e0 = l0 + d0, e1 = l1 + d1, e2 = l2 + d2;
        if ((e0 >= 0.0 || d0 >= 0.0) && (e1 >= 0.0 || d1 >= 0.0) && (e2 >= 0.0 || d2 >= 0.0)) {
            double c0, c1, c2;
            piece_d(l0, l1, l2, e0, e1, e2, k.kq[sp], c0, c1, c2);
            if (T != acc_t) {
                if (acc_t >= 0) win_add_j_d(w, p.Jloc, acc_t, a0, a1, a2);
                acc_t = T; a0 = a1 = a2 = 0.0;
            }
            a0 += c0; a1 += c1; a2 += c2;
            P[j].l0 = e0;
            P[j].l1 = e1;
            if (do_count) {
                if (T == ct) ++cc;
                else {
                    if (ct >= 0) win_add_c_d(w, s.cnt, ct, cc);
                    ct = T; cc = 1;
                }
            }
        } else {
            mover[j] = true;
            mfz[j] = fz;
            mfr[j] = fr;
        }
    }
    wave_deposit_d(w, p.Jloc, acc_t, a0, a1, a2);
    if (do_count) wave_count_d(w, s.cnt, ct, cc);
    if (DIAG) {
        double v = 0.5 * wk;
        int nl = nlive;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            v += __shfl_xor(v, off, 64);
            nl += __shfl_xor(nl, off, 64);
        }
        if ((threadIdx.x & 63) == 0) { s_wk[threadIdx.x >> 6] = v; s_nl[threadIdx.x >> 6] = nl; }
    }
    const int lane = threadIdx.x & 63;
    int slot[kPPTd];
#pragma unroll
    for (int j = 0; j < kPPTd; ++j) {
        slot[j] = -1;
        const unsigned long long mask = __ballot(mover[j]);
        if (mask == 0ull) continue;
        int base = 0;
        if (lane == __ffsll((long long)mask) - 1) base = atomicAdd(&s_nmv, __popcll(mask));
        base = __shfl(base, __ffsll((long long)mask) - 1, 64);
        if (mover[j]) {
            const int q = base + __popcll(mask & ((1ull << lane) - 1ull));
            if (q < kQCapD) {
                slot[j] = q;
                s_mv[q] = MoverD{P[j].cell, P[j].l0, P[j].l1, mfz[j], mfr[j]};
            } else slot[j] = -2;
        }
    }
    __syncthreads();
    // ---- phase 2: walk of the queued particles; movers that found the queue
    // full are walked by their owners
    const int nmv = min(s_nmv, kQCapD);
    if (s_nmv > kQCapD) {
#pragma unroll
        for (int j = 0; j < kPPTd; ++j)
            if (slot[j] == -2) {
                MoverD mv{P[j].cell, P[j].l0, P[j].l1, mfz[j], mfr[j]};
                walk_mover_d(m, s, p, w, k, max_walk, mv);
                P[j].cell = mv.cell; P[j].l0 = mv.l0; P[j].l1 = mv.l1;
                if (do_count && mv.cell >= 0) win_add_c_d(w, s.cnt, mv.cell & kCellMask, 1);
            }
    }
    for (int i = threadIdx.x; i < nmv; i += kWGd) {
        MoverD mv = s_mv[i];
        walk_mover_d(m, s, p, w, k, max_walk, mv);
        s_mv[i] = mv;
        if (do_count && mv.cell >= 0) win_add_c_d(w, s.cnt, mv.cell & kCellMask, 1);
    }
    __syncthreads();
    // ---- phase 3: owners take their movers back; stores; window flush
#pragma unroll
    for (int j = 0; j < kPPTd; ++j)
        if (slot[j] >= 0) {
            P[j].cell = s_mv[slot[j]].cell;
            P[j].l0 = s_mv[slot[j]].l0;
            P[j].l1 = s_mv[slot[j]].l1;
        }
    for (int i = threadIdx.x; i < 3 * kWinD; i += kWGd) {
        const double v = s_jl[i];
        const long long gi = 3ll * w.base + i;
        if (v != 0.0 && gi >= 0 && gi < 3ll * m.n2) unsafeAtomicAdd(&p.Jloc[gi], v);
    }
    if (do_count)
        for (int i = threadIdx.x; i < kWinD; i += kWGd) {
            const int v = s_cl[i], t = w.base + i;
            if (v != 0 && t >= 0 && t < m.n2) atomicAdd(&s.cnt[t], v);
        }
    if (DIAG && threadIdx.x == 0) {
        double v = 0.0;
        int nl = 0;
#pragma unroll
        for (int q = 0; q < kWGd / 64; ++q) { v += s_wk[q]; nl += s_nl[q]; }
        s.part_kin[3 * chunk] = v;
        s.part_kin[3 * chunk + 1] = (double)nl;
    }
#pragma unroll
    for (int j = 0; j < kPPTd; ++j) {
        const long long q = p0 + j;
        if (q < n) {
            cell[q] = P[j].cell;
            l0a[q] = P[j].l0; l1a[q] = P[j].l1;
            ura[q] = P[j].ur; upa[q] = P[j].up; uza[q] = P[j].uz;
        }
    }
}

// diag: also 1/2 E^n D^n per block, read before the update (the energy
// record of the step's start level)
__device__ __forceinline__ double edge_update_d(const DevMesh &m, const DevState &s, const DevPlain &p, double qunit,
                                                int e, bool diag) {
    const int4 et = m.etri[e];
    const int kl = et.z & 3, kr = (et.z >> 2) & 3;
    const double jl = p.Jloc[3 * et.x + kl];
    const double sl = (et.z & 16) ? -1.0 : 1.0;
    double acc = sl * (s.HBdt[et.x] - qunit * jl);
    double jfx = sl * jl;
    if (et.y >= 0) {
        const double jr = p.Jloc[3 * et.y + kr];
        const double sr = (et.z & 32) ? -1.0 : 1.0;
        acc += sr * (s.HBdt[et.y] - qunit * jr);
        jfx += sr * jr;
    }
    p.Jfx[e] = jfx;                    // every edge: conductor edges carry current too (continuity check)
    if (!(et.z & 64)) return 0.0;      // conductor edge: tangential E stays 0
    const double dn = s.D[e];
    s.D[e] = dn + acc;
    return diag ? 0.5 * p.E[e] * dn : 0.0;
}

__global__ __launch_bounds__(256) void k_edge_pass_d(DevMesh m, DevState s, DevPlain p, double qunit, int diag) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e == 0) s.ctr->step = s.ctr->step + 1ull;   // the face pass of this step has read it
    const double we = e < m.n1 ? edge_update_d(m, s, p, qunit, e, diag != 0) : 0.0;
    if (!diag) return;                              // uniform across the grid
    const double tot = block_sum_d(we);
    if (threadIdx.x == 0) s.part_edge[blockIdx.x] = tot;
}

__global__ __launch_bounds__(256) void k_spmv_d(DevMesh m, DevState s, DevPlain p) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m.n1) return;
    const int sl = i >> 6, lane = i & 63;
    const int64_t beg = m.m_sptr[sl];
    const int len = m.m_slen[sl];
    const double *v = p.m_val + beg + lane;
    const int32_t *cc = m.m_col + beg + lane;
    double acc = 0.0;
    int j = 0;
    for (; j + 4 <= len; j += 4) {
        const int c0 = cc[64 * j], c1 = cc[64 * (j + 1)], c2 = cc[64 * (j + 2)], c3 = cc[64 * (j + 3)];
        const double v0 = v[64 * j], v1 = v[64 * (j + 1)], v2 = v[64 * (j + 2)], v3 = v[64 * (j + 3)];
        const double x0 = s.D[c0], x1 = s.D[c1], x2 = s.D[c2], x3 = s.D[c3];
        acc = fma(v0, x0, acc);
        acc = fma(v1, x1, acc);
        acc = fma(v2, x2, acc);
        acc = fma(v3, x3, acc);
    }
    for (; j < len; ++j) acc = fma(v[64 * j], s.D[cc[64 * j]], acc);
    p.E[i] = acc;
}

// ------------------------------------------------------------ diagnostics
// Nodal charge of the particles at their current positions, eq. (charge),
// plus the wall charge: Q = Qres + sum_p kq lambda_k (charge units, FP64
// atomics).  Blocks of kChunkD particles; each block also leaves its live
// count.
__global__ __launch_bounds__(256) void k_charge_init_d(DevMesh m, DevPlain p) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    if (v < m.n0) p.Q[v] = p.Qres[v];
}

__global__ __launch_bounds__(kWGd) void k_charge_d(DevMesh m, DevState s, DevPlain p, PlainConst k) {
    __shared__ int s_nl[kWGd / 64];
    const long long n = (long long)s.ctr->n_slots;
    const int chunk = blockIdx.x;
    if ((long long)chunk * kChunkD >= n) return;
    int live = 0;
    for (int j = 0; j < kPPTd; ++j) {
        const long long i = ((long long)chunk * kWGd + threadIdx.x) * kPPTd + j;
        const int c = i < n ? s.cell[s.cur][i] : -1;
        if (c < 0) continue;
        ++live;
        const int T = c & kCellMask, sp = (c >> kCellBits) & 15;
        const double kq = k.kq[sp];
        const double l0 = p.l0[s.cur][i], l1 = p.l1[s.cur][i];
        const int4 tn = m.tnodes[T];
        fadd(&p.Q[tn.x], kq * l0);
        fadd(&p.Q[tn.y], kq * l1);
        fadd(&p.Q[tn.z], kq * (1.0 - l0 - l1));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) live += __shfl_xor(live, off, 64);
    if ((threadIdx.x & 63) == 0) s_nl[threadIdx.x >> 6] = live;
    __syncthreads();
    if (threadIdx.x == 0) {
        int nl = 0;
        for (int q = 0; q < kWGd / 64; ++q) nl += s_nl[q];
        s.part_kin[3 * chunk + 2] = (double)nl;
    }
}

// Node pass of an evaluation at level n = ctr->step (the FP64 step's
// version of k_node_diag): Q^n from k_charge_d, the Gauss residual and its
// drift, |Q^n - Q^{n-1} + Ddiv J^{n-1/2}| when level n-1 was evaluated, the
// total charge, max |Q|; per edge 1/2 E^n D^n; and this block's slice of the
// face and particle partials.  Block partials in the layout k_diag_final
// reads.
__global__ __launch_bounds__(256) void k_node_diag_d(DevMesh m, DevState s, DevPlain p, double qunit, int in_step,
                                                     int nb_face, int nb_edge) {
    const int v = blockIdx.x * blockDim.x + threadIdx.x;
    const unsigned long long n = s.ctr->step;
    const bool have_prev = s.ctr->diag_level1 == n && n > 0;
    const bool first = s.ctr->g0_set == 0;
    DiagVals d{};
    if (v < m.n0) {
        double div = 0.0, mag = 0.0, divj = 0.0;
        for (int q = m.nptr[v]; q < m.nptr[v + 1]; ++q) {
            const int e = m.nedge[q];
            const double x = s.D[e];
            div += m.nsign[q] > 0 ? x : -x;
            mag += fabs(x);
            divj += m.nsign[q] > 0 ? p.Jfx[e] : -p.Jfx[e];
        }
        const double Qv = p.Q[v];
        if (have_prev) d.mx[3] = dbits(fabs((Qv - p.Qprev[v]) + divj));
        d.mx[4] = dbits(fabs(Qv));
        p.Qprev[v] = Qv;
        if (m.nfree[v]) {
            const double g = div - Qv * qunit;
            if (first) s.g0[v] = g;
            d.mx[0] = dbits(fabs(g - s.g0[v]));
            d.mx[1] = dbits(fabs(g));
            d.mx[2] = dbits(mag);
        }
        d.sum[kSumQ] = Qv * qunit;
    }
    if (v < m.n1) d.sum[kSumWEnow] = 0.5 * p.E[v] * s.D[v];
    fold_slices(s, d, in_step, nb_face, nb_edge, gridDim.x);
    const DiagVals r = block_reduce_diag(d);
    if (threadIdx.x == 0) store_partials(s.part_node, blockIdx.x, gridDim.x, r);
}

// emission: as the mixed step, with FP64 coordinates and wall charge
__global__ __launch_bounds__(256) void k_inject_d(DevMesh m, DevState s, DevPlain pl, const EmitEdge *ee, InjParams p) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= p.per_step) return;
    const unsigned long long step = s.ctr->inj_step;
    const long long q = (long long)s.ctr->n_slots + i;
    const Emission em = sample_emission(ee, p, step, i);
    const EmitEdge E = ee[em.e];
    const double la = 1.0 - em.s, lb = em.s;
    const int c = s.cur;
    s.cell[c][q] = E.face | (p.species << kCellBits);
    pl.l0[c][q] = E.ka == 0 ? la : (E.kb == 0 ? lb : 0.0);
    pl.l1[c][q] = E.ka == 1 ? la : (E.kb == 1 ? lb : 0.0);
    pl.ur[c][q] = em.ur;
    pl.up[c][q] = em.up;
    pl.uz[c][q] = em.uz;
    unsafeAtomicAdd(&pl.Qres[E.na], -(double)p.kq * la);
    unsafeAtomicAdd(&pl.Qres[E.nb], -(double)p.kq * lb);
}

__global__ void k_inject_commit_d(DevState s, int per_step) {
    s.ctr->n_slots += (unsigned long long)per_step;
    s.ctr->inj_step += 1ull;
}

inline unsigned nb_(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

void launch_tri_pass_plain(const DevMesh &m, DevState &s, const DevPlain &p, const PlainConst &k, const FieldSrc &fs,
                           const DevLayers &lay, bool diag, hipStream_t st) {
    if (m.n2 == 0) return;
    hipLaunchKernelGGL(k_tri_pass_d, dim3(nb_(m.n2, 256)), dim3(256), 0, st, m, s, p, k.dt, fs, lay, diag ? 1 : 0);
}

template <bool VAY>
static void launch_particles_plain_t(const DevMesh &m, DevState &s, const DevPlain &p, const PlainConst &k,
                                     int max_walk, int dc, bool diag, dim3 grid, hipStream_t st) {
    if (diag) hipLaunchKernelGGL((k_particles_d<VAY, true>), grid, dim3(kWGd), 0, st, m, s, p, k, max_walk, dc);
    else hipLaunchKernelGGL((k_particles_d<VAY, false>), grid, dim3(kWGd), 0, st, m, s, p, k, max_walk, dc);
}

void launch_particles_plain(const DevMesh &m, DevState &s, const DevPlain &p, const PlainConst &k, int max_walk,
                            bool count, bool vay, bool diag, hipStream_t st) {
    if (s.capacity == 0) return;
    const dim3 grid(nb_(s.capacity, kChunkD));
    if (vay) launch_particles_plain_t<true>(m, s, p, k, max_walk, count ? 1 : 0, diag, grid, st);
    else launch_particles_plain_t<false>(m, s, p, k, max_walk, count ? 1 : 0, diag, grid, st);
}

void launch_edge_pass_plain(const DevMesh &m, DevState &s, const DevPlain &p, const PlainConst &k, bool diag,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_edge_pass_d, dim3(nb_(m.n1, 256)), dim3(256), 0, st, m, s, p, k.qunit, diag ? 1 : 0);
}

void launch_spmv_plain(const DevMesh &m, DevState &s, const DevPlain &p, hipStream_t st) {
    hipLaunchKernelGGL(k_spmv_d, dim3(nb_(m.n1, 256)), dim3(256), 0, st, m, s, p);
}

void launch_sort_plain(const DevMesh &m, DevState &s, DevPlain &p, bool counted, hipStream_t st) {
    const int a = s.cur, b = 1 - s.cur;
    void *const src[5] = {p.l0[a], p.l1[a], p.ur[a], p.up[a], p.uz[a]};
    void *const dst[5] = {p.l0[b], p.l1[b], p.ur[b], p.up[b], p.uz[b]};
    launch_sort_payload(m, s, counted, 8, 5, src, dst, st);
}

void launch_inject_plain(const DevMesh &m, DevState &s, const DevPlain &p, const EmitEdge *ee, const InjParams &ip,
                         hipStream_t st) {
    if (ip.per_step <= 0) return;
    hipLaunchKernelGGL(k_inject_d, dim3(nb_(ip.per_step, 256)), dim3(256), 0, st, m, s, p, ee, ip);
    hipLaunchKernelGGL(k_inject_commit_d, dim3(1), dim3(1), 0, st, s, ip.per_step);
}

void launch_charge_plain(const DevMesh &m, DevState &s, const DevPlain &p, const PlainConst &k, hipStream_t st) {
    hipLaunchKernelGGL(k_charge_init_d, dim3(nb_(m.n0, 256)), dim3(256), 0, st, m, p);
    if (s.capacity) hipLaunchKernelGGL(k_charge_d, dim3(nb_(s.capacity, kChunkD)), dim3(kWGd), 0, st, m, s, p, k);
}

void launch_diag_plain(const DevMesh &m, DevState &s, const DevPlain &p, const PlainConst &k, bool in_step,
                       hipStream_t st) {
    const int64_t nn = m.n0 > m.n1 ? m.n0 : m.n1;
    hipLaunchKernelGGL(k_node_diag_d, dim3(nb_(nn, 256)), dim3(256), 0, st, m, s, p, k.qunit, in_step ? 1 : 0,
                       (int)nb_(m.n2, 256), (int)nb_(m.n1, 256));
    launch_diag_final(m, s, in_step, true, st);
}

}  // namespace axp
