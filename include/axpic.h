/*
 * axpic — MI355X (gfx950) implementation of the per-time-step loop of the
 * axisymmetric, charge-conserving electromagnetic particle-in-cell method of
 * Na, Omelchenko, Moon, Borges and Teixeira, "Axisymmetric charge-conservative
 * electromagnetic particle simulation algorithm on unstructured grids"
 * (arXiv:1701.03784).
 *
 * The library keeps a meridian-plane (z, rho) triangle mesh, the field
 * degrees of freedom (E on edges, B_phi flux on faces), macro-particles and
 * the sparse approximate inverse (SPAI) of the permittivity Hodge matrix on
 * one GPU, and advances them with hand-written HIP kernels:
 *   Faraday update of face fluxes (Sec. 3.1, eq. full_d_dfl),
 *   Whitney-form gather of E and B_phi (Sec. 3.2),
 *   relativistic Boris push with an axisymmetric position update (Sec. 3.3),
 *   charge-conserving edge-current scatter along each particle's path
 *     across triangles (Sec. 3.4, eqs. current and DCE),
 *   Ampere update made explicit by the SPAI matrix (eq. full_d_dal).
 *
 * Conventions (all calls):
 *   - SI units.  Positions are (z, rho) pairs; momenta are u = gamma v in m/s
 *     in the local cylindrical basis (u_rho, u_phi, u_z).
 *   - Triangles must be counter-clockwise in the (z, rho) plane; face values
 *     are fluxes of B_phi through them.
 *   - Edge i of the mesh is the i-th pair (tail, head), tail < head, of the
 *     lexicographically sorted edge set (the orientation of App. D); edge
 *     values are line integrals of E from tail to head.  axp_get_edges
 *     returns that list.
 *   - Ring sources are per radian: a macro-particle of charge q deposits
 *     q/(2 pi) of charge and current.
 *   - Host pointers passed in are borrowed for the duration of the call only;
 *     the library copies what it keeps.  All device memory is owned by the
 *     context and released by axp_destroy.
 *   - Every call returns an axp_status; no C++ exception crosses the ABI.
 *     The message of the last failure is returned by axp_last_error.
 *     Argument and mesh errors leave the context usable.  AXP_E_HIP,
 *     AXP_E_NAN, AXP_E_WALK and AXP_E_FIXED_OVERFLOW are sticky: once
 *     raised (at axp_sync/axp_diag, from device flags) every later call that
 *     touches the device returns AXP_E_STATE.
 *   - One context per host thread; distinct contexts are independent.
 */
#ifndef AXPIC_H
#define AXPIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct axp_ctx axp_ctx;
typedef struct axp_batch axp_batch;
typedef int32_t axp_status;

enum {
    AXP_OK = 0,
    AXP_E_ARG = -1,            /* bad argument (null pointer, size, range) */
    AXP_E_MESH = -2,           /* invalid mesh: orientation, untagged boundary, non-manifold */
    AXP_E_SPAI = -3,           /* SPAI failed (singular least-squares block, not SPD) */
    AXP_E_UNSTABLE = -4,       /* dt above the leapfrog stability limit */
    AXP_E_OOM = -5,            /* device or host allocation failed */
    AXP_E_HIP = -6,            /* HIP runtime error */
    AXP_E_WALK = -7,           /* a particle path needed more than the segment cap */
    AXP_E_FIXED_OVERFLOW = -8, /* 64-bit fixed-point current or charge out of range */
    AXP_E_NAN = -9,            /* non-finite momentum or field */
    AXP_E_STATE = -10          /* call out of order, or a sticky error was raised before */
};

/* Boundary tags of boundary segments (axp_set_boundary). */
enum {
    AXP_BC_PEC = 1,     /* conductor: tangential E = 0; particles absorbed, charge kept on the wall */
    AXP_BC_AXIS = 2,    /* rho = 0: free (natural) edges; particles cannot cross */
    AXP_BC_EMITTER = 3, /* conductor that emits particles (axp_set_injector) */
    AXP_BC_OPEN = 4     /* free (natural, PMC-like) field boundary; particles absorbed */
};

/* Arithmetic of the time step. */
enum {
    AXP_PREC_PLAIN_FP64 = 0, /* FP64 gather/push/SpMV, FP64 barycentric positions, FP64 atomics */
    AXP_PREC_MIXED = 1       /* FP32 gather/push/SpMV; element-local fixed-point positions;
                                64-bit fixed-point current; FP64 D, B and diagnostics */
};

/* Momentum push (Sec. 3.3): the relativistic Boris rotation, or Vay's
 * pusher, which solves the time-centred momentum equation with the average
 * of the old and new velocities in the magnetic force exactly, so that a
 * particle at the E x B drift velocity feels no force at any energy. */
enum {
    AXP_PUSH_BORIS = 0,
    AXP_PUSH_VAY = 1
};

/* How the SPAI matrix was built (axp_info.spai_mode). */
enum {
    AXP_SPAI_PLAIN = 0,            /* least squares per column (Sec. 3.1) */
    AXP_SPAI_LEARNED = 1,          /* network guess + refinement, least-squares fallback per column */
    AXP_SPAI_LEARNED_REJECTED = 2, /* learned matrix failed the energy guard: plain SPAI used */
    AXP_SPAI_LEARNED_REVERTED = 3  /* learned matrix tripped the run-time energy guard: plain SPAI since */
};

typedef struct axp_mlp axp_mlp;

typedef void *(*axp_alloc_fn)(size_t bytes, void *user);
typedef void (*axp_free_fn)(void *ptr, void *user);

typedef struct {
    int32_t device;          /* HIP device ordinal */
    void *hip_stream;        /* hipStream_t the steps are enqueued on (NULL = default stream) */
    int32_t precision;       /* AXP_PREC_* */
    double dt;               /* time step [s]; <= 0: cfl_fraction * stability limit */
    double cfl_fraction;     /* used when dt <= 0 (default 0.5) */
    int32_t spai_level;      /* SPAI a-priori pattern level L (pattern of A^L), default 3 */
    double spai_drop_tol;    /* relative drop tolerance within each SPAI column, default 1e-3 */
    int32_t sort_period;     /* re-sort particles by triangle every this many steps (>= 1) */
    int32_t diag_every;      /* the step from level n to n+1 is a diagnostic step when n+1 is a multiple of
                                diag_every: inside its own kernels it evaluates level n+1 (charge, Gauss and
                                continuity residuals) and records the energies of level n (0: only axp_diag_get) */
    int32_t max_walk;        /* cap on path pieces per particle and step (default 64) */
    int32_t use_graph;       /* 1: capture axp_step's launches in a hipGraph and replay it */
    axp_alloc_fn alloc;      /* optional device allocator (NULL: hipMalloc) */
    axp_free_fn free;
    void *alloc_user;
    int32_t pusher;          /* AXP_PUSH_* (default AXP_PUSH_BORIS); a batch needs one pusher for all members */
} axp_config;

typedef struct {
    int64_t n_nodes, n_edges, n_faces;
    int64_t n_free_edges, n_free_nodes;
    int64_t spai_nnz;            /* non-zeros of M over free edges */
    double spai_fro_residual;    /* ||I - A M||_F / sqrt(n) over free edges */
    double spai_max_col_residual;
    double dt, dt_cfl;           /* time step in use and the leapfrog limit */
    double setup_seconds;        /* host time of axp_build */
    int64_t particle_capacity;
    int64_t n_particles;         /* live particles after the last sync */
    int64_t step;                /* steps taken */
    int32_t precision;
    int32_t n_species;
    int32_t spai_mode;               /* AXP_SPAI_* actually used */
    int32_t pad_;
    int64_t spai_fallback_columns;   /* learned SPAI: columns replaced by least squares */
    double spai_pred_resid_mean;     /* learned SPAI: mean ||e_k - A^ m_k|| of the network's columns */
    double spai_kept_resid_mean;     /* same after refinement, over the columns kept */
    double spai_energy_drift;        /* learned SPAI: relative energy drift of the guard run */
    double spai_seconds;             /* host time of the SPAI construction */
    int64_t n_layer_faces;           /* faces of the absorbing layers (axp_set_layers) */
    int64_t spai_guard_trip_step;    /* level at which the run-time guard tripped (-1: never) */
    double spai_run_drift;           /* largest total-energy drift the run-time guard has seen */
    double spai_feature_seconds;     /* learned SPAI: pair features (host) */
    double spai_infer_seconds;       /* learned SPAI: network inference (device, copies included) */
    double spai_solve_seconds;       /* least squares (plain); refinement, fallback and assembly (learned) */
    int32_t sort_period;             /* sort period in use (axp_config, or the autotuner's) */
    int32_t window_lead;             /* particle kernel's accumulation window: faces before a block's first */
} axp_info;

typedef struct {
    int64_t step;                /* time level evaluated: the number of steps taken */
    int64_t n_live;              /* live particles at that level */
    int64_t n_absorbed;          /* particles absorbed at walls (cumulative) */
    int64_t walk_overflow;       /* paths cut at the segment cap (cumulative) */
    int64_t nan_count;           /* non-finite momenta seen (cumulative) */
    int64_t fixed_overflow;      /* fixed-point headroom violations (cumulative) */
    int64_t dce_max_abs;         /* mixed: max over the evaluations since the reference of max over nodes
                                    |2^23 (Q^n - Q^{n-1}) + Ddiv J^{n-1/2}| in fixed point, taken where
                                    level n-1 was evaluated too (Sec. 3.5.1; 0 = exact) */
    double dce_max_rel;          /* FP64 step: the same maximum of |Q^n - Q^{n-1} + Ddiv J^{n-1/2}| / max|Q| */
    double gauss_max_drift;      /* max over the evaluations since the reference and over free nodes of
                                    |res^n - res^ref|, res = Ddiv [*eps]_a E - Q (Sec. 3.5.2) */
    double gauss_max_abs;        /* this level: max over free nodes |res^n| */
    double gauss_scale;          /* this level: max over free nodes of sum |D_e| at the node */
    double W_E, W_B, W_K;        /* energies per radian [J/rad] of level energy_step (the last diagnostic
                                    step): 1/2 E^n [*eps]_a E^n, 1/2 B^{n+1/2} H B^{n-1/2},
                                    1/2 (K^{n-1/2} + K^{n+1/2}) with K = sum w (gamma - 1) m c^2 / 2 pi */
    double Q_total;              /* this level: total charge per radian incl. wall charge [C/rad] */
    int64_t energy_step;         /* level of W_E, W_B, W_K; -1 before the first diagnostic step */
    int64_t n_evals;             /* evaluations since the reference */
    double W_E_now;              /* this level: 1/2 E^n [*eps]_a E^n [J/rad] */
} axp_diag;

/* Fills cfg with defaults: device 0, default stream, mixed precision,
 * dt = 0.5 x stability limit, SPAI level 3 / drop 1e-3, sort every 4 steps,
 * no periodic diagnostics, walk cap 64, graphs on, hipMalloc. */
void axp_config_default(axp_config *cfg);

/* Creates an empty context on cfg->device.  *out receives the handle. */
axp_status axp_create(const axp_config *cfg, axp_ctx **out);

/* Meridian mesh (Sec. 2.2, Fig. 2b; App. D): n_nodes points zr[n][2] =
 * (z, rho >= 0) and n_tris triangles tri[n][3] (node ids, counter-clockwise
 * in (z, rho)).  Copied.  AXP_E_MESH on clockwise or degenerate triangles. */
axp_status axp_set_mesh(axp_ctx *ctx, int32_t n_nodes, const double *zr, int32_t n_tris, const int32_t *tri);

/* Boundary segments seg_nodes[n][2] with tags tag[n] (AXP_BC_*).  Every
 * boundary edge of the mesh must be listed (AXP_E_MESH at axp_build if not). */
axp_status axp_set_boundary(axp_ctx *ctx, int32_t n_seg, const int32_t *seg_nodes, const uint8_t *tag);

/* Setup (host FP64 + uploads): topology and incidence (App. D), Hodge
 * matrices by exact quadrature of their defining integrals (Sec. 3.1, App. B),
 * SPAI of [*eps] (Sec. 3.1), the stability limit, locality renumbering,
 * device layouts.  Must precede every call below. */
axp_status axp_build(axp_ctx *ctx);

axp_status axp_info_get(const axp_ctx *ctx, axp_info *out);

/* Canonical edge list edges[n_edges][2] (tail, head), see Conventions. */
axp_status axp_get_edges(const axp_ctx *ctx, int32_t *edges);

/* The SPAI matrix M ~ [*eps]^-1 in CSR over canonical edge indices (zero rows
 * and columns on conductor edges).  rowptr[n_edges+1]; col/val hold
 * capacity entries; *nnz receives the count (AXP_E_ARG if it exceeds capacity,
 * with *nnz still set). */
axp_status axp_get_spai(const axp_ctx *ctx, int64_t capacity, int64_t *nnz, int64_t *rowptr, int32_t *col, double *val);

/* Fields at step 0: E0[n_edges] edge line integrals at t = 0 and
 * B_mhalf[n_faces] face fluxes at t = -dt/2 (face order of axp_set_mesh).
 * Conductor edge values are ignored (set to 0).  D^0 = [*eps]_a E^0 = M^-1 E^0
 * is solved by conjugate gradients in FP64. */
axp_status axp_set_fields(axp_ctx *ctx, const double *E0, const double *B_mhalf);

/* Electrostatic, Gauss-consistent fields at step 0.  The scheme keeps the
 * Gauss residual D~div [*eps]_a E - Q at its initial value (Sec. 3.5.2), so
 * it is zero for all steps only if it is zero at step 0; applied voltages
 * (the cathode-anode field of the diode, Sec. 4.2) enter as potentials of conductors.
 * Computes the nodal potential phi with phi = phi_conductor on conductor
 * nodes (nodes on AXP_BC_PEC or AXP_BC_EMITTER segments) such that
 * E^0 = -G phi (edge value phi_tail - phi_head; 0 on conductor edges) and
 * D^0 = M^-1 E^0 satisfy D~div D^0 = Q on every free node, to 1e-13 of the
 * larger of |Q| and the summed |D| at a node; sets E^0, D^0 and B^{-1/2} = 0.
 * E^0 is curl-free, so without particles the state does not move.
 *   phi_conductor  [n_nodes] volts, read on conductor nodes only; NULL: 0 V.
 *   with_charge    1: Q is the nodal charge of the particles present plus
 *                  the wall charge (per radian, as axp_get_sources returns);
 *                  0: Q = 0.
 *   phi_out        optional [n_nodes]: the potential on every node.
 * Host FP64 solve (setup): defect correction on D~div M^-1 D~div^T with the
 * rho-weighted P1 stiffness D~div A D~div^T as preconditioner.  Errors:
 * AXP_E_STATE before axp_build; AXP_E_NAN for a non-finite potential;
 * AXP_E_SPAI if the solve does not converge (fields unchanged). */
axp_status axp_set_electrostatic(axp_ctx *ctx, const double *phi_conductor, int32_t with_charge, double *phi_out);

/* Absorbing layers at the z ends of the domain (the PML terminating the
 * ports and the cathode side, Sec. 5.1), set before axp_build.  The layers
 * stretch z by s_z = 1 + sigma / (j omega eps0), i.e. the meridian medium
 * becomes eps_rho = eps0 s_z, eps_z = eps0 / s_z, mu_phi = mu0 s_z; sigma
 * grows as sigma_max (depth / thickness)^order from the layer's inner face
 * to the end of the mesh (faces with their centroid below z_left when bit 0
 * of sides is set, above z_right when bit 1 is set; sigma evaluated at the
 * centroid).  The step keeps D with E = M D, M the SPAI of the stretched
 * Hodge sum_T [(1 + beta) A_rho + A_z / (1 + beta)], beta = sigma dt /
 * (2 eps0), with auxiliary values on the layer faces: h (s_z h = H B) and
 * q (s_z q = A_z e), both by the trapezoidal rule, and the correction
 * D -= 2 beta (A_rho e - q / (1 + beta)) after E = M D.  The time step is
 * fixed first without the layers (axp_config), the stability limit checked
 * again with them (AXP_E_UNSTABLE).  The outer end of a layer should be a
 * conductor.  sigma_max [S/m] = 0 removes the layers.  Inside the layers
 * the conduction current changes the Gauss residual; outside it is kept.
 * Contexts with layers need the least-squares SPAI, cannot join a batch
 * and cannot be saved.  Errors: AXP_E_ARG (sides outside 0..3, order
 * outside 0..8, negative or non-finite values), AXP_E_STATE after axp_build. */
axp_status axp_set_layers(axp_ctx *ctx, int32_t sides, double z_left, double z_right, double sigma_max, int32_t order);

/* Magnetic point source (Sec. 4.1): a magnetic current M(t) at (z, rho)
 * [m], a ring about the axis, drives the flux of the face holding the
 * point: B_T^{n+1/2} = B_T^{n-1/2} - dt (C E^n)_T - dt M(t^n), t^n = n dt,
 * with the Gaussian-modulated pulse
 * M(t) = amplitude exp(-((t - t0) / (2 sigma))^2) cos(omega (t - t0))
 * (amplitude [V], t0 and sigma [s], omega [rad/s]).  Up to 8 sources;
 * they stay until axp_clear_point_sources and are not saved by axp_save.
 * Errors: AXP_E_ARG for a point outside the mesh, sigma <= 0, non-finite
 * values or a ninth source; AXP_E_STATE before axp_build.  Contexts with
 * sources cannot join a batch. */
axp_status axp_add_point_source(axp_ctx *ctx, double z, double rho, double amplitude, double t0, double sigma,
                                double omega);
axp_status axp_clear_point_sources(axp_ctx *ctx);

/* Field probe (Sec. 4.1): from the next step on, the E field at (z, rho)
 * (Whitney interpolation of the edge values, the gather of Sec. 3.2) is
 * recorded at t^n at the start of every step, for the next `capacity`
 * steps, in a device buffer the context owns (16 bytes per step).
 * capacity 0 removes the probe.  axp_get_probe copies the samples recorded
 * so far, (E_z, E_rho) [V/m] per step, into E_z_rho[2 * n]; *n receives
 * their count (with E_z_rho NULL only the count; AXP_E_ARG if it exceeds
 * capacity).  Not saved by axp_save; contexts with a probe cannot join a
 * batch. */
axp_status axp_set_probe(axp_ctx *ctx, double z, double rho, int64_t capacity);
axp_status axp_get_probe(axp_ctx *ctx, int64_t capacity, int64_t *n, double *E_z_rho);

/* Uniform static axial field B_z [T] added at the gather (beam focusing, Sec. 3.2). */
axp_status axp_set_external_bz(axp_ctx *ctx, double bz);

/* Particle species (the macro-particles of Sec. 2.2 and 3.3, rings of
 * charge about the axis): q [C] and m [kg] of one physical particle, and the
 * number of physical particles per macro-particle (weight >= 1).  In mixed
 * precision every species' macro charge q*weight must be an integer multiple
 * of the first species' macro charge (the fixed-point charge unit).
 * *species_id receives the new id (at most 16 species). */
axp_status axp_add_species(axp_ctx *ctx, double q, double m, int64_t weight, int32_t *species_id);

/* Adds n macro-particles at zr[n][2] (meridian positions (z, rho), rho >= 0)
 * with momenta u[n][3] = gamma v (u_rho, u_phi, u_z) [m/s], the state of the
 * push of Sec. 3.3 at t = -dt/2; each is located in the mesh (AXP_E_ARG if
 * outside or non-finite; nothing is added then) and stored element-local.
 * Host arrays are copied.  Breaks the continuity chain of the diagnostics
 * (the next evaluation has no previous level).  Synchronous. */
axp_status axp_inject(axp_ctx *ctx, int32_t species, int64_t n, const double *zr, const double *u);

/* Continuous injection from the AXP_BC_EMITTER boundary (the emission of
 * the diode and gun configurations, Sec. 4): at the start of every step,
 * per_step macro-particles of `species` are placed on emitter edges,
 * uniformly per unit area of the emitting surface of revolution (edge
 * chosen with probability proportional to its length times its mean rho,
 * position along it with density proportional to rho), in the face next to
 * the edge.  Momentum [kg m/s per kg, i.e. gamma v]: u_mean + u_spread *
 * (uniform in [-1, 1]^3), given in the edge frame (tangent tail -> head,
 * phi, inward normal); for an emitter on a z = const wall, u_mean[2] is the
 * momentum into the domain.  Each particle's charge is taken from the wall
 * charge of the edge's two nodes in proportion to its barycentric
 * coordinates, so the nodal charge, and the continuity equation, are
 * unchanged by the emission.  Random numbers: draw d (0..4: edge, position,
 * three momentum components) of particle i at step n is output
 * c = 2^32 n + 8 i + d + 1 of the SplitMix64 generator seeded with `seed`
 * (Steele, Lea and Flood 2014), as (out >> 11) * 2^-53.  per_step = 0
 * switches the injector off.  Not available to batch members. */
axp_status axp_set_injector(axp_ctx *ctx, int32_t species, int64_t per_step, const double u_mean[3],
                            double u_spread, uint64_t seed);

/* Enqueues n_steps time steps on cfg.hip_stream and returns (Sec. 3; the
 * order of one step n -> n+1): Faraday B^{n+1/2} = B^{n-1/2} - dt C E^n,
 * eq. (full_d_dfl); the gather of E^n and of the face field averaged over
 * B^{n-1/2}, B^{n+1/2} (Sec. 3.2); the relativistic push, eqs. (DNE)/(DLE)
 * (Sec. 3.3); the walk of each path across faces with the charge-conserving
 * edge current of eq. (current) (Sec. 3.4); Ampere
 * D^{n+1} = D^n + dt (C^T H B^{n+1/2} - J^{n+1/2}), E^{n+1} = M D^{n+1},
 * eq. (full_d_dal) with the SPAI M (Sec. 3.1).  Diagnostic steps (diag_every)
 * also evaluate their start level.  Errors raised by the kernels surface at
 * axp_sync.  AXP_E_ARG if n_steps < 0. */
axp_status axp_step(axp_ctx *ctx, int32_t n_steps);

/* Waits for the stream and raises sticky errors from device flags. */
axp_status axp_sync(axp_ctx *ctx);

/* Diagnostics of the current level n (the number of steps taken; evaluated
 * now unless the last diagnostic step or call already did), syncs first:
 * the nodal charge of eq. (charge) from the particles' element-local
 * coordinates plus the wall charge, the discrete Gauss law's residual and its
 * drift from the reference level (Sec. 3.5.2), the continuity residual
 * against level n-1 (Sec. 3.5.1), the total charge, and the energies of the
 * last diagnostic step.  The reference level is the first evaluation after
 * axp_set_fields / axp_set_electrostatic; axp_inject only breaks the
 * continuity chain.  Returns the sticky errors of axp_sync. */
axp_status axp_diag_get(axp_ctx *ctx, axp_diag *out);

/* Energy record of one diagnostic step n -> n+1 (its start level n), per radian. */
typedef struct {
    int64_t step;                /* level n */
    int64_t n_live;              /* live particles at level n */
    double W_E, W_B, W_K;        /* as in axp_diag */
    double Q_total;              /* reserved (0): the total charge is in axp_diag */
} axp_energy;

/* Energy records of the diagnostic steps not yet returned, oldest first:
 * at most capacity of them into out[capacity]; *n receives the count.  The
 * device keeps the last 4096 records; older ones not yet read are skipped.
 * W_E + W_B is the invariant of the leapfrog pair (full_d_dfl)/(full_d_dal)
 * without sources; with particles W_E + W_B + W_K is conserved up to the
 * push's and the deposit's time discretisation. */
axp_status axp_get_energies(axp_ctx *ctx, int64_t capacity, int64_t *n, axp_energy *out);

/* E^n[n_edges] (canonical edge order) and B^{n-1/2}[n_faces] (input face
 * order); either pointer may be NULL. */
axp_status axp_get_fields(axp_ctx *ctx, double *E, double *B_half);

/* D^n = [*eps]_a E^n (canonical edges), the last step's edge current
 * J^{n-1/2} times dt [C/rad] (canonical edges) and the nodal charge Q^n
 * [C/rad] (input node order, incl. wall charge).  Pointers may be NULL. */
axp_status axp_get_sources(axp_ctx *ctx, double *D, double *J_dt, double *Q);

/* Live particles: positions zr[cap][2], momenta u[cap][3], species[cap];
 * *n receives the live count (AXP_E_ARG if above cap, *n still set).  The
 * order is the library's storage order (grouped by triangle). */
axp_status axp_get_particles(axp_ctx *ctx, int64_t cap, int64_t *n, double *zr, double *u, int32_t *species);

/* Checkpoint of the complete state (fields, wall charge, particles, species,
 * B_z, injector, counters, step) to a file, and its restore into a context
 * built from the same mesh, boundary, precision and time step that has no
 * species yet (AXP_E_ARG on a mismatch).  A restored run continues exactly
 * as the saved one would have (bit for bit in mixed precision).  The file
 * layout is the library's own (native byte order). */
axp_status axp_save(axp_ctx *ctx, const char *path);
axp_status axp_load(axp_ctx *ctx, const char *path);

/* Per-phase kernel timing (observability).  While on, every phase of
 * axp_step is bracketed by HIP events recorded on cfg.hip_stream; the
 * accumulated device milliseconds and launch counts are returned (after a
 * stream sync) and reset by axp_set_timing(ctx, 1). */
enum {
    AXP_PHASE_FACE = 0,      /* Faraday + gather tile (per face) */
    AXP_PHASE_PARTICLES = 1, /* gather + push + in-face current (per particle) */
    AXP_PHASE_EDGE = 2,      /* D update (per edge) */
    AXP_PHASE_SPMV = 3,      /* E = M D (per edge row) */
    AXP_PHASE_SORT = 4,      /* counting sort of particles by face */
    AXP_PHASE_DIAG = 5,      /* diagnostics */
    AXP_PHASE_INJECT = 6,    /* continuous injection */
    AXP_PHASE_WALK = 7,      /* walk of the particles that leave their face (per mover) */
    AXP_N_PHASES = 8
};
axp_status axp_set_timing(axp_ctx *ctx, int32_t on);
axp_status axp_get_timing(axp_ctx *ctx, double *ms /*[AXP_N_PHASES]*/, int64_t *launches /*[AXP_N_PHASES]*/);

const char *axp_last_error(const axp_ctx *ctx);
void axp_destroy(axp_ctx *ctx);

/* ---- learned SPAI ------------------------------------------------------
 * A small network predicts the entries M^_kj of the Jacobi-scaled SPAI
 * matrix (A^ = S^-1/2 [*eps] S^-1/2 on the free edges, S = diag) for every
 * pair (k, j) of the level-L pattern, from 16 features of the pair, all
 * symmetric in (k, j):
 *   0-3  one-hot hop distance d(k, j) = 0..3 in the graph of A^
 *   4-6  (A^)_kj, (A^^2)_kj, (A^^3)_kj
 *   7    min/max of the two edge lengths (meridian plane)
 *   8    midpoint distance / (l_k + l_j)
 *   9    |cos| of the angle between the edges
 *   10   min/max of the midpoint radii rho (1 if both are 0)
 *   11   (l_k + l_j) / (rho_k + rho_j + l_k + l_j)
 *   12   (n_k + n_j)/20 and 13 |n_k - n_j|/10, n = entries in the row of A^
 *   14   mean over k, j of sum_i |A^_ki|, minus 1
 *   15   d / 3
 * Network: 16 -> H (tanh) -> ... -> H (tanh) -> 1 (linear), H = 32 or 64,
 * 1-4 hidden layers.  Parameter vector (FP32): per layer W[n_out][n_in]
 * row-major, then b[n_out].  Loss: sum_i w_i (p_i - y_i)^2 / sum_i w_i.
 * The training kernels (forward, backward, weight gradients on the matrix
 * cores, Adam) run on the network's device and stream. */
axp_status axp_mlp_create(int32_t device, void *hip_stream, int32_t n_in, int32_t n_hidden, int32_t n_layers,
                          int32_t spai_level, uint64_t seed, axp_mlp **out);
int64_t axp_mlp_n_params(const axp_mlp *net);
/* Host parameter vectors; set_params also clears the Adam state. */
axp_status axp_mlp_set_params(axp_mlp *net, const float *params);
axp_status axp_mlp_get_params(const axp_mlp *net, float *params);
/* X[n][16], y[n] and w[n] are DEVICE pointers (FP32). forward: y = net(X). */
axp_status axp_mlp_forward(axp_mlp *net, const float *X, int64_t n, float *y);
/* Loss and gradient over the n samples (device inputs); *loss and grad[n_params]
 * are host outputs and may be NULL (then nothing is synchronised). */
axp_status axp_mlp_loss_grad(axp_mlp *net, const float *X, const float *y, const float *w, int64_t n, double *loss,
                             float *grad);
/* Allocation-free variant of axp_mlp_loss_grad, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving or
 * training loops, harnesses that forbid hipMalloc.  Same kernels and
 * arithmetic as axp_mlp_loss_grad, so the same results bit for bit.
 *   X[n][16], y[n], w[n]   DEVICE inputs (FP32), as for axp_mlp_loss_grad
 *   loss_dev[2]            DEVICE output (FP64): weighted mean squared error,
 *                          then the sum of the weights (when that sum is not
 *                          positive, loss_dev[0] and grad_dev are 0)
 *   grad_dev[n_params]     DEVICE output (FP32): d loss / d parameters
 * Enqueued on the network's stream; nothing is synchronised or copied to the
 * host, and the network's own gradient (the one axp_mlp_adam_step uses) is
 * left as it was.  No device or host memory is allocated: the intermediate
 * activations, deltas and partial sums live in one static device array of
 * 32 MiB per device (held until the process ends), which a call of n samples
 * uses as 256-byte aligned pieces of 8 L H n, 4 n, 4 n, 16 ceil(n/256) and
 * 4 n_params ceil(n/512) bytes (L hidden layers of width H); at most
 * 31,234 samples at H = 64, L = 2 and 15,497 at H = 64, L = 4.  A call needing
 * more returns AXP_E_ARG before any launch (axp_mlp_last_error gives the
 * size).  Every byte a call reads from the array it has written first, but
 * all calls on one device share the array: calls that may overlap on one
 * device (other streams, other threads, other networks) race and must be
 * ordered by the caller.  AXP_E_ARG for null pointers or n < 1; AXP_E_HIP if
 * the launch fails. */
axp_status axp_mlp_loss_grad_noalloc(axp_mlp *net, const float *X, const float *y, const float *w, int64_t n,
                                     double *loss_dev, float *grad_dev);
/* One Adam step (bias-corrected) with the gradient of the last loss_grad call. */
axp_status axp_mlp_adam_step(axp_mlp *net, double lr, double beta1, double beta2, double eps);
axp_status axp_mlp_info(const axp_mlp *net, int32_t *n_in, int32_t *n_hidden, int32_t *n_layers, int32_t *spai_level,
                        int64_t *adam_steps);
axp_status axp_mlp_save(const axp_mlp *net, const char *path);
axp_status axp_mlp_load(int32_t device, void *hip_stream, const char *path, axp_mlp **out);
const char *axp_mlp_last_error(const axp_mlp *net);
void axp_mlp_destroy(axp_mlp *net);

/* Use the network for this context's SPAI (call before axp_build; NULL
 * restores the plain SPAI).  At axp_build the network's column m_k on the
 * level-L pattern J_k starts `iters` conjugate-gradient steps on the normal
 * equations of min ||e_k - A^(:, J_k) m||_2 (whose limit is the plain SPAI's
 * least-squares column); a column whose residual ||e_k - A^ m_k||_2 then
 * exceeds row_tol is replaced by its exact least-squares column; drop rule
 * and symmetric average as in the plain SPAI.  The result must then conserve
 * the discrete energy of a 64-step source-free leapfrog run to
 * energy_drift_tol (relative), else the plain SPAI is used
 * (AXP_SPAI_LEARNED_REJECTED).  The network is borrowed during axp_build. */
axp_status axp_set_spai_model(axp_ctx *ctx, axp_mlp *net, double row_tol, double energy_drift_tol, int32_t iters);

/* Run-time energy guard of the learned SPAI: the plain SPAI (Sec. 3.1) is
 * the fallback when the run's energy drifts.  Needs a context built with a
 * learned SPAI that the setup guard kept (AXP_SPAI_LEARNED) and diagnostic
 * steps (diag_every > 0); AXP_E_STATE otherwise.  drift_tol >= 0 arms the
 * guard, drift_tol < 0 disarms it.  While armed, axp_step works in chunks of
 * at most 2048 diagnostic steps: it first copies the state (fields, sources,
 * particles, counters; on the device, in memory allocated once and grown
 * with the particle buffers) as the chunk's checkpoint, runs the chunk, and
 * reads the energy records it produced.  The first record after arming sets
 * the reference W_ref of the total energy W = W_E + W_B + W_K; when a record
 * has |W - W_ref| > drift_tol |W_ref|, the context rebuilds M with the plain
 * SPAI, restores the checkpoint, keeps D (so Gauss's law and the continuity
 * equation carry over unchanged), sets E = M D with the new M, and runs the
 * chunk again.  The guard is then off, axp_info reports
 * AXP_SPAI_LEARNED_REVERTED and the level that tripped it.  Emission and
 * absorption exchange energy with the outside, so drift_tol must exceed what
 * the run's physics moves; the guard is meant for the growth of an unstable
 * M.  AXP_E_UNSTABLE (the state restored to the checkpoint, the learned M
 * kept) if dt exceeds the plain SPAI's stability limit.  A context with an
 * armed guard cannot join a batch. */
axp_status axp_set_spai_run_guard(axp_ctx *ctx, double drift_tol);

/* Loads a network saved by axp_mlp_save or axp_spai_model_train and uses it
 * for this context's SPAI as axp_set_spai_model does, with row_tol 0.01,
 * energy_drift_tol 1e-6 and 3 refinement steps.  The context owns the
 * network (freed by axp_destroy).  Call before axp_build.  Errors: AXP_E_ARG
 * (NULL argument, or a network of another SPAI level), AXP_E_STATE (after
 * axp_build), the status of axp_mlp_load for an unreadable file. */
axp_status axp_spai_model_load(axp_ctx *ctx, const char *model_path);

/* Trains a learned-SPAI network on device 0 (default stream) and saves it
 * to out_model (axp_mlp_save format).  mesh_list: a text file with one
 * mesh file per line (blank lines and lines starting with '#' are skipped).
 * A mesh file is text: "axpic-mesh 1", then "n_nodes n_tris n_seg", then
 * n_nodes lines "z rho" [m], n_tris lines of three node ids
 * (counter-clockwise) and n_seg boundary segments "a b tag" (AXP_BC_*),
 * as axp_set_mesh and axp_set_boundary take them.  For every mesh the plain
 * level-3 SPAI is built and at most 150,000 of its pattern pairs are drawn
 * (axp_spai_pairs); the network (16 -> 64 -> 64 -> 1) then takes 40 epochs
 * of Adam over minibatches of 4,096 after one shuffle, the learning rate
 * falling linearly from 3e-3 to 1e-4.  Random draws (pair samples, shuffle,
 * initial weights) follow `seed`.  Errors: AXP_E_ARG (unreadable list or
 * mesh file, no pairs), AXP_E_OOM, AXP_E_HIP, or the status of the first
 * failing library call (a bad mesh gives AXP_E_MESH). */
axp_status axp_spai_model_train(const char *mesh_list, const char *out_model, uint64_t seed);

/* Training data of a built context: features X[n][16] of every pattern pair,
 * the scaled entry y[n] = M^_kj of the context's SPAI (0 where dropped) and
 * the canonical edge indices kj[n][2].  *n receives the pair count; with
 * all outputs NULL only the count is returned (AXP_E_ARG if it exceeds
 * capacity). */
axp_status axp_spai_pairs(axp_ctx *ctx, int64_t capacity, int64_t *n, float *X, float *y, int32_t *kj);

/* Autotuner of two knobs of the step: runs about trial_steps real steps
 * (plus one settling window) under each of the sort periods 1, 2, 4, 8, 16,
 * keeps the fastest, then under each accumulation-window lead 64, 128, 192,
 * 256, 320 of the particle kernel (faces of the window before a block's first
 * particle's face) at that period, and keeps the fastest; timed with HIP
 * events (*sort_period receives the period, axp_info both).  The state
 * advances by those steps; since the current and the diagnostic charge are
 * summed in fixed point, the fields and particles after them do not depend
 * on the knobs (bit for bit; only the storage order of the particles does).
 * Cache: when the environment variable AXP_AUTOTUNE_CACHE names a file, a
 * line "key sort_period window_lead ms_per_step" is appended after the
 * trials, and a later call whose key (mesh, particle count to the nearest
 * power of two, precision, diagnostic cadence, pusher, GPU architecture)
 * is found there takes the knobs from the file's last such line and runs
 * no steps at all. */
axp_status axp_autotune(axp_ctx *ctx, int32_t trial_steps, int32_t *sort_period);

/* ---- batched sweep: many independent devices advanced together ---------
 * axp_batch_create pools n built mixed-precision contexts (each with fields,
 * a species and particles set) into one set of device arrays: faces, edges
 * and nodes of the members are concatenated, and every face, edge and node
 * carries its member's index for the per-member constants (dt, B_z, species).
 * axp_batch_step advances all members together with one launch per phase
 * for the whole pool; with cfg.use_graph of the first member the launches
 * of 2 x sort_period steps are captured in one hipGraph and replayed.  The
 * contexts are borrowed and must outlive the batch; their own state is
 * stale until axp_batch_sync copies the pooled state back (after which the
 * per-context getters and axp_diag_get see it).  Every member's result is
 * the same, bit for bit, as stepping that context alone.  The members must
 * share their diagnostic cadence (cfg.diag_every, else AXP_E_ARG); the pool's
 * diagnostic steps evaluate all members together (residual maxima over them,
 * charges and energies summed). */
axp_status axp_batch_create(axp_ctx *const *ctxs, int32_t n, axp_batch **out);
axp_status axp_batch_step(axp_batch *b, int32_t n_steps);
axp_status axp_batch_sync(axp_batch *b);
/* Autotuner and timing of the pool (as axp_autotune / axp_set_timing). */
axp_status axp_batch_autotune(axp_batch *b, int32_t trial_steps, int32_t *sort_period);
axp_status axp_batch_set_timing(axp_batch *b, int32_t on);
axp_status axp_batch_get_timing(axp_batch *b, double *ms /*[AXP_N_PHASES]*/, int64_t *launches /*[AXP_N_PHASES]*/);
/* Pool sizes, particle slots in use and steps taken; pointers may be NULL. */
axp_status axp_batch_info(axp_batch *b, int64_t *n_faces, int64_t *n_edges, int64_t *n_particles, int64_t *step);
const char *axp_batch_last_error(const axp_batch *b);
void axp_batch_destroy(axp_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* AXPIC_H */
