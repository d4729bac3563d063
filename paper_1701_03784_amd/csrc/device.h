// Device-side state of one (or a pool of) meridian devices and the host
// launchers of the HIP kernels.  Plain pointers only; the host owns them.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace axp {

constexpr int kCellBits = 27;                       // face index bits of a particle cell word
constexpr int32_t kCellMask = (1 << kCellBits) - 1; // species in bits 27..30, sign bit = dead
constexpr int kMaxSpecies = 16;

// Per-instance constants (one entry per device in a pooled batch).
struct InstConst {
    double dt;         // time step [s]
    double jscale;     // charge unit / (2 pi 2^46): fixed-point current -> D increment [C/rad]
    double qscale;     // charge unit / (2 pi 2^23): fixed-point charge -> C/rad
    float cdt;         // c dt [m]
    float bz;          // external B_z [T]
    int32_t n_species;
    int32_t pad;
    // per species: q dt/(2 m c) [1/(V/m)], q dt/(2 m) [1/T], integer charge multiple
    float qe[kMaxSpecies];
    float qb[kMaxSpecies];
    int32_t kq[kMaxSpecies];
    double mw[kMaxSpecies];   // m * weight * c^2 / (2 pi) for the kinetic energy [J/rad]
};

struct DevMesh {
    int32_t n0 = 0, n1 = 0, n2 = 0, n_inst = 1;
    // faces (internal order)
    const float4 *gS = nullptr;     // 2^23 grad lam0 (z, rho), 2^23 grad lam1 (z, rho)
    const float4 *rho4 = nullptr;   // rho of local nodes 0..2, 1/(2 area)
    const int4 *nbr = nullptr;      // face across side k (>= 0) or -tag; w: neighbour-local ids, 4 bits/side
    const int4 *tedge = nullptr;    // edge of side k; w: bit k set -> incidence sign -1
    const int4 *tnodes = nullptr;   // node ids of local nodes 0..2
    const double *Hdt = nullptr;    // dt [*mu^-1]_T
    const int32_t *tinst = nullptr; // instance of each face (pooled batches), or null
    // edges
    const int4 *etri = nullptr;     // left face, right face (-1), packed sides/signs/free, instance
    // nodes: incident edges with divergence sign; incident face corners (3 t + k)
    const int32_t *nptr = nullptr, *nedge = nullptr;
    const int32_t *ncptr = nullptr, *ncorner = nullptr;
    const int8_t *nsign = nullptr;
    const uint8_t *nfree = nullptr;
    const int32_t *ninst = nullptr; // instance of each node, or null
    // the same two lists in slices of 64 nodes, column-major (entry j of node
    // 64 s + l at (s * w + j) * 64 + l, w the longest list of the mesh): corner
    // ids with -1 as padding; edges as +-(e + 1) by divergence sign, 0 as padding
    const int32_t *ncorner_ell = nullptr, *nedge_ell = nullptr;
    int32_t nwc = 0, nwe = 0;
    // SPAI M in sliced-ELL (slices of 64 rows, column-major inside a slice)
    const int64_t *m_sptr = nullptr;
    const int32_t *m_slen = nullptr;
    const float *m_val = nullptr;
    const int32_t *m_col = nullptr;
    // [*eps] in CSR (energy diagnostic)
    const int64_t *a_ptr = nullptr;
    const int32_t *a_col = nullptr;
    const double *a_val = nullptr;
    const InstConst *inst = nullptr;
};

struct DevCounters {
    unsigned long long n_slots;       // particle slots in use (live + dead until the next sort)
    unsigned long long n_absorbed;
    unsigned long long walk_overflow;
    unsigned long long nan_count;
    unsigned long long fixed_overflow;
    unsigned long long inj_step;      // step index of the next emission (random-stream counter)
    unsigned long long step;          // index n of the step in flight (time t^n = n dt of sources and probe)
    unsigned long long diag_level1;   // 1 + time level of the last diagnostic evaluation (0: none, or
                                      // the continuity reference was invalidated)
    unsigned long long g0_set;        // the Gauss residual of the reference level is stored in g0
    unsigned long long energy_count;  // energy records written to the ring so far
    unsigned long long pad;
};

// Stretched-coordinate absorbing layers (the PML of the ports): per layer
// face i its internal face, beta = sigma dt / (2 eps0), H, the 3x3 z and rho
// parts of its local [*eps] (sides k, l), and the state h (H B / s_z), q
// (A_z e / s_z on its sides), eprev (its side values of E at the previous
// step) and corr (its three corrections of D in the step in flight).
// face_layer[t]: layer index of face t, or -1.  edges: per edge of a layer
// face, (edge, 4 i_a + k_a, 4 i_b + k_b or -1, 0).
struct DevLayers {
    int32_t n = 0, n_edges = 0;
    const int32_t *face = nullptr, *face_layer = nullptr;
    const double *beta = nullptr, *Hf = nullptr, *Az = nullptr, *Ar = nullptr;
    double *h = nullptr, *q = nullptr, *eprev = nullptr, *corr = nullptr;
    const int4 *edges = nullptr;
};

constexpr int kMaxSources = 8;

// Magnetic point sources and the field probe (Sec. 4.1), passed by value to
// the face pass.  Source k adds -dt M_k(t^n) to the flux of face src_face[k],
// M_k(t) = amp exp(-((t - t0) / (2 sig))^2) cos(w (t - t0)); the probe writes
// (E_z, E_rho) at barycentric (probe_l0, probe_l1) of probe_face at t^n into
// probe[2 (n - probe_start) + {0, 1}] while that index is below probe_cap.
struct FieldSrc {
    int32_t n_src = 0;
    int32_t src_face[kMaxSources] = {};
    double amp[kMaxSources] = {}, t0[kMaxSources] = {}, sig[kMaxSources] = {}, w[kMaxSources] = {};
    double dt = 0.0;
    int32_t probe_face = -1;
    double probe_l0 = 0.0, probe_l1 = 0.0;
    double *probe = nullptr;
    long long probe_cap = 0, probe_start = 0;
};

// Diagnostics.  An evaluation at time level n (a step's start, or the
// current state on demand) writes per-block partials; k_diag_final reduces
// them in a fixed order into DevDiag, so no value depends on the order in
// which blocks ran.  Maxima of non-negative doubles are kept as their bit
// patterns (which order like the values).
constexpr int kDiagSlots = 12;       // per node-pass block: sums Qtot, W_E, W_B, W_K, n_live; maxima drift,
                                     // |res|, scale, dce, qmax; 2 unused
constexpr int kEnergyRing = 4096;    // energy records kept on the device

struct DevEnergy {
    long long level;     // time level n
    long long n_live;    // live particles at level n
    double WE, WB, WK;   // 1/2 E^n [*eps]_a E^n, 1/2 B^{n+1/2} H B^{n-1/2}, 1/2 (K^{n-1/2} + K^{n+1/2})
    double Qtot;         // total charge incl. wall charge [C/rad]
};

struct DevDiag {
    long long level;                      // time level of the latest evaluation (-1: none)
    long long n_live;                     // live particles at that level
    double gauss_abs, gauss_scale;        // max over free nodes |res^n|, max of the summed |D| at a node
    double q_total, qmax;                 // total charge [C/rad]; FP64 step: max |Q| (charge units)
    double WE_now;                        // 1/2 E^n [*eps]_a E^n at that level
    long long dce_last;                   // max |2^23 dQ + Ddiv J| of that level (-1: no previous level)
    unsigned long long gauss_drift_max_bits;   // running maxima over every evaluation since the reference
    unsigned long long dce_max;                // mixed: fixed point; FP64 step: double bits of |dQ + Ddiv J|
    unsigned long long dce_rel_max_bits;       // FP64 step: running max of |dQ + Ddiv J| / max|Q|
    unsigned long long n_evals;                // evaluations since the reference
    DevEnergy energy;                     // latest energy record (level -1: none)
};

struct DevState {
    // fields
    double *B = nullptr;        // face flux, B^{n-1/2} before a step, B^{n+1/2} after its first kernel
    double *Bprev = nullptr;    // B^{n-1/2} of the last step
    double *HBdt = nullptr;     // dt H B^{n+1/2}
    float4 *f0 = nullptr, *f1 = nullptr;  // gather tile per face
    unsigned long long *Jloc = nullptr;   // fixed-point current per face side (3 per face)
    double *D = nullptr;        // [*eps]_a E on edges (FP64)
    float *D32 = nullptr;       // FP32 copy read by the SpMV
    float *E = nullptr;         // E on edges
    long long *Jfx = nullptr;   // fixed-point edge current of the last step (diagnostic)
    long long *Qres = nullptr;  // fixed-point wall/emitter charge per node (units 2^-23 charge unit)
    long long *Qfx = nullptr;   // fixed-point nodal charge (diagnostic)
    long long *Qprev = nullptr;
    double *g0 = nullptr;       // Gauss residual at the first diagnostic
    // particles (structure of arrays, two buffers for the sort)
    int32_t *cell[2] = {nullptr, nullptr};
    uint32_t *L0[2] = {nullptr, nullptr}, *L1[2] = {nullptr, nullptr};
    float *ur[2] = {nullptr, nullptr}, *up[2] = {nullptr, nullptr}, *uz[2] = {nullptr, nullptr};
    int cur = 0;
    int64_t capacity = 0;
    // sort scratch
    int32_t *cnt = nullptr;     // n2 + 1
    int32_t *blk = nullptr;     // scan block sums
    DevCounters *ctr = nullptr;
    DevDiag *diag = nullptr;
    // diagnostics: face-corner charge of the particles (3 per face, fixed
    // point), per-block partials and the ring of energy records
    unsigned long long *Qloc = nullptr;
    double *part_face = nullptr;   // W_B per face-pass block
    double *part_edge = nullptr;   // W_E per edge-pass block
    double *part_node = nullptr;   // kDiagSlots per node-pass block
    double *part_kin = nullptr;    // per particle block: W_K, live at the start, live at the end
    double *part_wenow = nullptr;  // 1/2 E D of the new level per block of the fused SpMV
    DevEnergy *energy = nullptr;   // kEnergyRing records
};

// Emitter edge of the continuous injector (canonical edge order).
struct EmitEdge {
    double cdf;                // inclusive cumulative emission weight  l (rho_t + rho_h) / 2
    double ra, rb;             // rho at tail and head
    double tz, tr, nz, nr;     // unit tangent tail -> head and inward unit normal, (z, rho)
    int32_t face, ka, kb;      // adjacent face and the local indices of tail and head in it
    int32_t na, nb;            // node ids of tail and head
    int32_t pad;
};

struct InjParams {
    unsigned long long seed;
    int32_t per_step, n_edges, species, kq;
    double um[3];              // mean momentum / c in the (tangent, phi, inward normal) frame
    double spread;             // half-width of the uniform spread, / c
    double total;              // total emission weight
};

// FP64 step (one instance): constants, geometry and state that differ from
// the mixed step.  B, Bprev, HBdt, D, g0, the sort scratch, counters and the
// particle cell words are shared with DevMesh / DevState.
struct PlainConst {
    double dt, cdt, bz;
    double qunit;            // charge unit / (2 pi) [C/rad]
    int32_t n_species, pad;
    double qe[kMaxSpecies];  // q dt / (2 m c)
    double qb[kMaxSpecies];  // q dt / (2 m)
    double kq[kMaxSpecies];  // macro charge / charge unit
    double mw[kMaxSpecies];  // m * weight * c^2 / (2 pi)
};

struct DevPlain {
    const double4 *grad = nullptr;   // grad lam0 (z, rho), grad lam1 (z, rho)
    const double4 *rho = nullptr;    // rho of local nodes 0..2, 1/(2 area)
    const double *m_val = nullptr;   // SPAI values in the same sliced ELL as DevMesh
    double *E = nullptr;             // E on edges
    double4 *f0 = nullptr, *f1 = nullptr;   // gather tile (f1.z = B_phi)
    double *Jloc = nullptr;          // current per face side, charge-unit * lambda products
    double *Jfx = nullptr;           // edge current of the last step (same units)
    double *Qres = nullptr;          // wall charge per node (charge units)
    double *Q = nullptr, *Qprev = nullptr;
    double *l0[2] = {nullptr, nullptr}, *l1[2] = {nullptr, nullptr};
    double *ur[2] = {nullptr, nullptr}, *up[2] = {nullptr, nullptr}, *uz[2] = {nullptr, nullptr};
};

// ---- launchers (kernels_mixed.hip) ----
// the face pass; with emit (1 to 4096 per step from an emitter of at most 1024
// edges) one extra block does the step's emission; with final_prev another
// does the final reduction the last diagnostic step's node pass left
// (launch_spmv_diag)
bool emission_fits_face_pass(const InjParams &p);
void launch_tri_pass(const DevMesh &m, DevState &s, const FieldSrc &fs, const DevLayers &lay, bool diag,
                     const EmitEdge *ee, const InjParams *emit, bool final_prev, hipStream_t st);
// layer update after E^{n+1}: q, eprev and the corrections of D (E: FP32 or FP64 edge values)
void launch_layers_post(const DevMesh &m, DevState &s, const float *E, const DevLayers &lay, hipStream_t st);
void launch_layers_post(const DevMesh &m, DevState &s, const double *E, const DevLayers &lay, hipStream_t st);
// gather, push and walk of every particle, with the charge-conserving current
// (q32: every charge multiple is 0 or 1; the single case implies it)
// (win_lead: faces of the accumulation window before the block's first face,
// a tuning knob that changes where sums land, never their values)
void launch_particles(const DevMesh &m, DevState &s, int max_walk, bool count, const InstConst *single, bool vay,
                      bool diag, bool q32, int win_lead, hipStream_t st);
void launch_sort_zero(const DevMesh &m, DevState &s, hipStream_t st);
void launch_edge_pass(const DevMesh &m, DevState &s, bool keep_j, bool diag, hipStream_t st);
void launch_spmv(const DevMesh &m, DevState &s, hipStream_t st);
void launch_sort(const DevMesh &m, DevState &s, bool counted, hipStream_t st);
// Diagnostics of a diagnostic step (the face pass, the particle kernel and
// the edge pass ran with diag on): the evaluation of its end level n + 1 and
// the energy record of its start level n, launched after the field update.
void launch_diag_in_step(const DevMesh &m, DevState &s, hipStream_t st);
// E = M D of a diagnostic step (no absorbing layers) with the energy of the
// new level per block of rows, and in the same launch the node pass over the
// nodes alone.  Its
// final reduction is left to the next face pass (final_prev) or to
// launch_step_final, which must run before anything reads the diagnostics.
void launch_spmv_diag(const DevMesh &m, DevState &s, hipStream_t st);
void launch_step_final(const DevMesh &m, DevState &s, hipStream_t st);
// Diagnostics of the current state (level = steps taken), on demand.
void launch_diag_now(const DevMesh &m, DevState &s, hipStream_t st);
// clears the face-corner charge accumulators (a fill kernel, graph-safe)
void launch_zero_u64(unsigned long long *p, int64_t n, hipStream_t st);
// reduces the partials of an evaluation (shared by both precisions)
void launch_diag_final(const DevMesh &m, DevState &s, bool in_step, bool plain, hipStream_t st);
// Counting sort of the particle arrays by face: cell words in s.cell plus
// n_fields payload arrays of `width` bytes (4 or 8) per particle, src[f] ->
// dst[f].  counted: s.cnt already holds the face histogram.
void launch_offset_cells(int32_t *cell, int64_t n, int32_t delta, hipStream_t st);
// Continuous emission: appends per_step particles before the step's push and
// takes their charge from the emitter nodes' wall charge.
void launch_inject(const DevMesh &m, DevState &s, const EmitEdge *ee, const InjParams &p, hipStream_t st);
void launch_sort_payload(const DevMesh &m, DevState &s, bool counted, int width, int n_fields, void *const *src,
                         void *const *dst, hipStream_t st);

// ---- launchers (kernels_plain.hip) ----
void launch_tri_pass_plain(const DevMesh &m, DevState &s, const DevPlain &p, const PlainConst &k, const FieldSrc &fs,
                           const DevLayers &lay, bool diag, hipStream_t st);
void launch_particles_plain(const DevMesh &m, DevState &s, const DevPlain &p, const PlainConst &k, int max_walk,
                            bool count, bool vay, bool diag, hipStream_t st);
// nodal charge Q^n of the particles at their current positions plus the wall charge
void launch_charge_plain(const DevMesh &m, DevState &s, const DevPlain &p, const PlainConst &k, hipStream_t st);
void launch_edge_pass_plain(const DevMesh &m, DevState &s, const DevPlain &p, const PlainConst &k, bool diag,
                            hipStream_t st);
void launch_spmv_plain(const DevMesh &m, DevState &s, const DevPlain &p, hipStream_t st);
void launch_sort_plain(const DevMesh &m, DevState &s, DevPlain &p, bool counted, hipStream_t st);
void launch_inject_plain(const DevMesh &m, DevState &s, const DevPlain &p, const EmitEdge *ee, const InjParams &ip,
                         hipStream_t st);
// FP64 step: node pass and reduction of an evaluation whose charge (launch_charge_plain)
// was computed at the level evaluated
void launch_diag_plain(const DevMesh &m, DevState &s, const DevPlain &p, const PlainConst &k, bool in_step,
                       hipStream_t st);

}  // namespace axp
