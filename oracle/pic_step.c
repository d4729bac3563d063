/*
 * FP64 reference of one time step of the axisymmetric charge-conserving
 * EM-PIC scheme (Na et al., arXiv:1701.03784).  TEST INFRASTRUCTURE ONLY:
 * the GPU library never links or calls this file.
 *
 * Order of one step n -> n+1 (Sec. 3.1-3.4):
 *   1. Faraday, eq. (full_d_dfl):   B^{n+1/2} = B^{n-1/2} - dt C E^n
 *      (- dt M(t^n) on the faces of magnetic point sources, Sec. 4.1)
 *   2. gather, Sec. 3.2:            E_p = sum_e E_e W1_e(r_p),
 *                                   B_p = sum_T (B^{n+1/2}+B^{n-1/2})_T/2 W2_T
 *      plus a static axial field B_z (beam focusing, Sec. 3.2);
 *   3. push, eqs. (DNE), (DLE):     relativistic Boris rotation, or Vay's
 *      pusher (the correction the paper cites for relativistic beams);
 *      axisymmetric position update: push in the local Cartesian frame
 *      (rho-hat, phi-hat, z-hat), then rotate back to the meridian plane;
 *   4. scatter, eq. (current):      J_e += (q/2pi/dt) int_path W1_e . dr,
 *      i.e. (q/2pi/dt)(lam_t^s lam_h^e - lam_h^s lam_t^e) on every straight
 *      piece of the path inside one triangle (t = tail, h = head of e);
 *   5. Ampere, eq. (full_d_dal):    E^{n+1} = E^n + dt M (C^T H B^{n+1/2} - J)
 *      with M the sparse approximate inverse of [*eps]; also
 *      D^{n+1} = D^n + dt (C^T H B^{n+1/2} - J), the quantity whose discrete
 *      divergence minus the nodal charge is invariant (Sec. 3.5.2).
 *
 * Charges and currents of a ring are per radian: a macro-particle of
 * charge q contributes q/(2 pi).  Units are SI; momenta are u = gamma v.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define O_PEC 1
#define O_AXIS 2
#define O_EMITTER 3
#define O_OPEN 4
#define O_MAXSEG 64

static const double O_C = 299792458.0;
static const double O_TWO_PI = 6.283185307179586476925286766559;

typedef struct {
    int64_t n0, n1, n2;
    const double *nodes;      /* [n0][2]: z, rho */
    const int64_t *tris;      /* [n2][3], counter-clockwise */
    const int64_t *edges;     /* [n1][2]: tail < head */
    const int64_t *tri_edges; /* [n2][3]: edge on side k = (node k, node k+1) */
    const int64_t *tri_signs; /* [n2][3]: C[T, edge] */
    const int64_t *tri_nbr;   /* [n2][3]: face across side k, -1 = boundary */
    const int64_t *edge_tag;  /* [n1]: 0 interior, else boundary tag */
    const uint8_t *edge_free; /* [n1]: 1 if E is unknown on the edge */
    const double *H;          /* [n2]: diagonal of [*mu^-1] */
    const int64_t *m_ptr;     /* M in CSR, n1 rows */
    const int64_t *m_col;
    const double *m_val;
} omesh;

typedef struct {
    int64_t n;
    double *z, *rho;          /* [n] global meridian position */
    int64_t *tri;             /* [n] containing triangle */
    double *u;                /* [n][3]: u_rho, u_phi, u_z (gamma v, m/s) */
    int8_t *alive;            /* [n] */
    const int64_t *species;   /* [n] */
    const double *sp_qm;      /* per species: q/m of the physical particle */
    const double *sp_qw;      /* per species: macro-particle charge */
} oparticles;

static double tri_area(const omesh *m, int64_t t)
{
    const int64_t *v = m->tris + 3 * t;
    const double *a = m->nodes + 2 * v[0], *b = m->nodes + 2 * v[1], *c = m->nodes + 2 * v[2];
    return 0.5 * ((b[0] - a[0]) * (c[1] - a[1]) - (c[0] - a[0]) * (b[1] - a[1]));
}

/* lam_i = area(r, r_j, r_k) / area(r_i, r_j, r_k), (i, j, k) cyclic */
static void bary(const omesh *m, int64_t t, double z, double r, double lam[3])
{
    const int64_t *v = m->tris + 3 * t;
    double A = tri_area(m, t);
    for (int i = 0; i < 3; ++i) {
        const double *pj = m->nodes + 2 * v[(i + 1) % 3];
        const double *pk = m->nodes + 2 * v[(i + 2) % 3];
        double a = 0.5 * ((pj[0] - z) * (pk[1] - r) - (pk[0] - z) * (pj[1] - r));
        lam[i] = a / A;
    }
}

/* grad lam_i = (rho_j - rho_k, z_k - z_j) / (2 area) */
static void grad_lambda(const omesh *m, int64_t t, double g[3][2])
{
    const int64_t *v = m->tris + 3 * t;
    double A2 = 2.0 * tri_area(m, t);
    for (int i = 0; i < 3; ++i) {
        const double *pj = m->nodes + 2 * v[(i + 1) % 3];
        const double *pk = m->nodes + 2 * v[(i + 2) % 3];
        g[i][0] = (pj[1] - pk[1]) / A2;
        g[i][1] = (pk[0] - pj[0]) / A2;
    }
}

/* local index (0..2) of global node id in triangle t */
static int local_of(const omesh *m, int64_t t, int64_t node)
{
    const int64_t *v = m->tris + 3 * t;
    for (int i = 0; i < 3; ++i)
        if (v[i] == node) return i;
    return -1;
}

/* E at a point of triangle t from the Whitney 1-form expansion */
static void gather_E(const omesh *m, int64_t t, const double lam[3], const double *E, double out[2])
{
    double g[3][2];
    grad_lambda(m, t, g);
    out[0] = out[1] = 0.0;
    for (int k = 0; k < 3; ++k) {
        int64_t e = m->tri_edges[3 * t + k];
        int a = local_of(m, t, m->edges[2 * e]);
        int b = local_of(m, t, m->edges[2 * e + 1]);
        for (int c = 0; c < 2; ++c)
            out[c] += E[e] * (lam[a] * g[b][c] - lam[b] * g[a][c]);
    }
}

/* current of one straight piece inside triangle t, from lam_s to lam_e */
static void deposit(const omesh *m, int64_t t, const double ls[3], const double le[3],
                    double coef, double *J)
{
    for (int k = 0; k < 3; ++k) {
        int64_t e = m->tri_edges[3 * t + k];
        int a = local_of(m, t, m->edges[2 * e]);     /* tail */
        int b = local_of(m, t, m->edges[2 * e + 1]); /* head */
        J[e] += coef * (ls[a] * le[b] - ls[b] * le[a]);
    }
}

/* cross product in the right-handed basis (rho, phi, z) */
static void cross3(const double a[3], const double b[3], double o[3])
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

/* Relativistic Boris: u^{n-1/2} -> u^{n+1/2} for E, B at r^n. k = q dt / (2 m). */
void oracle_boris(double u[3], const double E[3], const double B[3], double k)
{
    double um[3], t[3], s[3], up[3], c1[3], c2[3];
    for (int i = 0; i < 3; ++i) um[i] = u[i] + k * E[i];
    double gm = sqrt(1.0 + (um[0] * um[0] + um[1] * um[1] + um[2] * um[2]) / (O_C * O_C));
    for (int i = 0; i < 3; ++i) t[i] = k * B[i] / gm;
    double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    for (int i = 0; i < 3; ++i) s[i] = 2.0 * t[i] / (1.0 + t2);
    cross3(um, t, c1);
    for (int i = 0; i < 3; ++i) up[i] = um[i] + c1[i];
    cross3(up, s, c2);
    for (int i = 0; i < 3; ++i) u[i] = um[i] + c2[i] + k * E[i];
}

/* Vay's pusher: u^{n-1/2} -> u^{n+1/2} for E, B at r^n, k = q dt / (2 m).
 * It solves u^{n+1/2} - u^{n-1/2} = 2k (E + (v^{n+1/2} + v^{n-1/2})/2 x B)
 * for u^{n+1/2} in closed form: first u' = u^{n-1/2} + 2k E + k v^{n-1/2} x B,
 * then the remaining equation u^{n+1/2} = u' + k v^{n+1/2} x B, whose gamma
 * follows from a quadratic in gamma^2 (Vay, Phys. Plasmas 15, 056701, 2008). */
void oracle_vay(double u[3], const double E[3], const double B[3], double k)
{
    const double c2 = O_C * O_C;
    double g = sqrt(1.0 + (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) / c2);
    double v[3], vxb[3], up[3], tau[3];
    for (int i = 0; i < 3; ++i) v[i] = u[i] / g;
    cross3(v, B, vxb);
    for (int i = 0; i < 3; ++i) up[i] = u[i] + 2.0 * k * E[i] + k * vxb[i];
    for (int i = 0; i < 3; ++i) tau[i] = k * B[i];
    double tau2 = tau[0] * tau[0] + tau[1] * tau[1] + tau[2] * tau[2];
    double ustar = (up[0] * tau[0] + up[1] * tau[1] + up[2] * tau[2]) / O_C;
    double gp2 = 1.0 + (up[0] * up[0] + up[1] * up[1] + up[2] * up[2]) / c2;
    double sigma = gp2 - tau2;
    double gn = sqrt(0.5 * (sigma + sqrt(sigma * sigma + 4.0 * (tau2 + ustar * ustar))));
    double t[3], uxt[3];
    for (int i = 0; i < 3; ++i) t[i] = tau[i] / gn;
    double t2 = t[0] * t[0] + t[1] * t[1] + t[2] * t[2];
    double udt = up[0] * t[0] + up[1] * t[1] + up[2] * t[2];
    cross3(up, t, uxt);
    double s = 1.0 / (1.0 + t2);
    for (int i = 0; i < 3; ++i) u[i] = s * (up[i] + udt * t[i] + uxt[i]);
}

/* Move along rho-hat/phi-hat/z-hat by v dt, rotate (u_rho, u_phi) into the
 * frame of the new azimuth; returns the new (z, rho). */
void oracle_move(double z, double rho, double u[3], double dt, double *z_new, double *rho_new)
{
    double g = sqrt(1.0 + (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) / (O_C * O_C));
    double X = rho + u[0] / g * dt;
    double Y = u[1] / g * dt;
    double r1 = sqrt(X * X + Y * Y);
    if (r1 > 0.0) {
        double c = X / r1, s = Y / r1;
        double ur = c * u[0] + s * u[1];
        double up = -s * u[0] + c * u[1];
        u[0] = ur;
        u[1] = up;
    }
    *z_new = z + u[2] / g * dt;
    *rho_new = r1;
}

/* Walk particle p from its position to (ze, re), depositing the current of
 * each piece; returns pieces walked, or -1 on overflow. */
static int walk(const omesh *m, oparticles *P, int64_t p, double ze, double re,
                double coef_J, double q_ring, double *J, double *Qres, int64_t *stats)
{
    double zs = P->z[p], rs = P->rho[p];
    int64_t t = P->tri[p];
    int entered = -1;
    for (int seg = 0; seg < O_MAXSEG; ++seg) {
        double ls[3], le[3];
        bary(m, t, zs, rs, ls);
        bary(m, t, ze, re, le);
        int kx = -1;
        double sx = 2.0;
        for (int k = 0; k < 3; ++k) {
            if (k == entered || !(le[k] < 0.0)) continue;
            double s = ls[k] / (ls[k] - le[k]);
            if (s < sx) { sx = s; kx = k; }
        }
        if (kx < 0) {                       /* ends inside t */
            deposit(m, t, ls, le, coef_J, J);
            P->z[p] = ze; P->rho[p] = re; P->tri[p] = t;
            return seg + 1;
        }
        if (sx < 0.0) sx = 0.0;
        if (sx > 1.0) sx = 1.0;
        double lx[3];
        for (int k = 0; k < 3; ++k) lx[k] = ls[k] + sx * (le[k] - ls[k]);
        lx[kx] = 0.0;
        double zx = zs + sx * (ze - zs), rx = rs + sx * (re - rs);
        deposit(m, t, ls, lx, coef_J, J);
        int side = (kx + 1) % 3;            /* side (kx+1, kx+2) is opposite node kx */
        int64_t nb = m->tri_nbr[3 * t + side];
        if (nb < 0) {
            int64_t tag = m->edge_tag[m->tri_edges[3 * t + side]];
            if (tag == O_AXIS) {            /* cannot cross rho = 0: stop on it */
                P->z[p] = zx; P->rho[p] = rx; P->tri[p] = t;
                return seg + 1;
            }
            /* conductor or open boundary: absorbed; its charge stays on the wall nodes */
            const int64_t *v = m->tris + 3 * t;
            Qres[v[(kx + 1) % 3]] += q_ring * lx[(kx + 1) % 3];
            Qres[v[(kx + 2) % 3]] += q_ring * lx[(kx + 2) % 3];
            P->alive[p] = 0;
            P->z[p] = zx; P->rho[p] = rx; P->tri[p] = t;
            stats[1] += 1;
            return seg + 1;
        }
        const int64_t *v = m->tris + 3 * t;
        int64_t na = v[(kx + 1) % 3], nbn = v[(kx + 2) % 3];
        const int64_t *w = m->tris + 3 * nb;
        entered = -1;
        for (int i = 0; i < 3; ++i)
            if (w[i] != na && w[i] != nbn) entered = i;
        zs = zx; rs = rx; t = nb;
    }
    stats[2] += 1;
    P->z[p] = zs; P->rho[p] = rs; P->tri[p] = t;
    return -1;
}

/* Stretched-coordinate absorbing layer (the PML of the ports, Sec. 5.1):
 * the z coordinate is stretched by s_z = 1 + sigma / (j omega eps0) on the
 * layer's faces, i.e. eps_rho = eps0 s_z, eps_z = eps0 / s_z, mu_phi = mu0 s_z.
 * Per layer face f (n faces), beta = sigma dt / (2 eps0); Az, Ar: the z and
 * rho parts of eps0 int rho W1_k . W1_l over the face (3x3, its sides k, l);
 * h: the face's H-image flux (H B / s_z), q: (A_z / s_z) e on its sides,
 * eprev: its side values of E at the previous step. */
typedef struct {
    int64_t n;
    const int64_t *face;
    const double *beta;
    const double *Az;     /* [n][9] */
    const double *Ar;     /* [n][9] */
    double *h;            /* [n] */
    double *q;            /* [n][3] */
    double *eprev;        /* [n][3] */
} opml;

/*
 * One step.  E: E^n (n1) -> E^{n+1}.  B: B^{n-1/2} (n2) -> B^{n+1/2}.
 * D: D^n -> D^{n+1}.  J (n1) receives J^{n+1/2}.  Qres (n0) accumulates
 * the charge of absorbed particles.  Bh (n2) and rhs (n1) are scratch.
 * stats: [0] pieces walked, [1] absorbed, [2] walk overflows.
 * pusher: 0 relativistic Boris, 1 Vay.  src_face/src_val: the nsrc point
 * sources' faces and their magnetic currents at t^n.
 *
 * energy (may be NULL) receives the energies of time level n, the step's
 * start, per radian [J/rad]; a step is where their ingredients meet:
 *   [0] W_E = 1/2 E^n . D^n = 1/2 E^n [*eps]_a E^n  (the scheme's Hodge)
 *   [1] W_B = 1/2 B^{n+1/2} . H B^{n-1/2}
 *   [2] W_K = 1/2 (K^{n-1/2} + K^{n+1/2}),
 *       K = sum_p (m w c^2 / 2 pi)(gamma_p - 1) over the particles pushed
 *       (those absorbed during the step included)
 *   [3] K^{n+1/2}
 * Without sources W_E + W_B is the invariant of the leapfrog pair
 * (full_d_dfl)/(full_d_dal): its change over a step is
 * 1/2 (E^{n+1} + E^n) . dt C^T H B^{n+1/2} - 1/2 dt C (E^{n+1} + E^n) . H B^{n+1/2} = 0.
 */
/* gamma - 1 of momentum u = gamma v, without cancellation for slow particles */
static double gamma_m1(const double u[3])
{
    double w2 = (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) / (O_C * O_C);
    return w2 / (sqrt(1.0 + w2) + 1.0);
}

void oracle_step(const omesh *m, oparticles *P, double dt, double bz, int pusher,
                 int64_t nsrc, const int64_t *src_face, const double *src_val, const opml *pml,
                 double *E, double *B, double *D, double *J, double *Qres,
                 double *Bh, double *rhs, int64_t *stats, double *energy)
{
    double we = 0.0, wb = 0.0, k_old = 0.0, k_new = 0.0;
    if (energy)
        for (int64_t e = 0; e < m->n1; ++e) we += E[e] * D[e];
    /* 1. Faraday, with the magnetic point sources (Sec. 4.1): a magnetic
     *    current M(t^n) at a point drives the flux of the face holding it */
    for (int64_t t = 0; t < m->n2; ++t) {
        double circ = 0.0;
        for (int k = 0; k < 3; ++k)
            circ += (double)m->tri_signs[3 * t + k] * E[m->tri_edges[3 * t + k]];
        Bh[t] = B[t] - dt * circ;
    }
    for (int64_t k = 0; k < nsrc; ++k) Bh[src_face[k]] -= dt * src_val[k];
    if (energy)
        for (int64_t t = 0; t < m->n2; ++t) wb += Bh[t] * m->H[t] * B[t];
    memset(J, 0, sizeof(double) * m->n1);

    /* 2-4. gather, push, scatter.  Built with OpenMP (the timing form of the
     *     oracle) the particles are split statically over the threads, each
     *     with its own current, wall charge, counters and energy sums, added up
     *     in thread order afterwards: for a given thread count the result does
     *     not depend on scheduling, and with one thread it is the serial loop. */
    int nth = 1;
#ifdef _OPENMP
    nth = omp_get_max_threads();
#endif
    double *Jt = J, *Qt = Qres, *Kt = NULL;
    int64_t *St = stats;
    if (nth > 1) {
        Jt = (double *)calloc((size_t)nth * m->n1, sizeof(double));
        Qt = (double *)calloc((size_t)nth * m->n0, sizeof(double));
        St = (int64_t *)calloc((size_t)nth * 3, sizeof(int64_t));
    }
    Kt = (double *)calloc((size_t)nth * 2, sizeof(double));
#ifdef _OPENMP
#pragma omp parallel num_threads(nth)
#endif
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *Jl = nth > 1 ? Jt + (size_t)tid * m->n1 : J;
        double *Ql = nth > 1 ? Qt + (size_t)tid * m->n0 : Qres;
        int64_t *Sl = nth > 1 ? St + 3 * tid : stats;
        double kol = 0.0, knl = 0.0;
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
        for (int64_t p = 0; p < P->n; ++p) {
            if (!P->alive[p]) continue;
            int64_t t = P->tri[p];
            int64_t sp = P->species[p];
            double lam[3], e2[2];
            bary(m, t, P->z[p], P->rho[p], lam);
            gather_E(m, t, lam, E, e2);
            double bphi = 0.5 * (B[t] + Bh[t]) / tri_area(m, t);
            double Ev[3] = {e2[1], 0.0, e2[0]};          /* (E_rho, E_phi, E_z) */
            double Bv[3] = {0.0, bphi, bz};               /* (B_rho, B_phi, B_z) */
            double *u = P->u + 3 * p;
            /* m w c^2 / (2 pi) of the macro-particle: m w = (q w) / (q / m) */
            double mwc2 = P->sp_qw[sp] / P->sp_qm[sp] * O_C * O_C / O_TWO_PI;
            if (energy) kol += mwc2 * gamma_m1(u);
            if (pusher == 1) oracle_vay(u, Ev, Bv, P->sp_qm[sp] * dt * 0.5);
            else oracle_boris(u, Ev, Bv, P->sp_qm[sp] * dt * 0.5);
            if (energy) knl += mwc2 * gamma_m1(u);
            double ze, re;
            oracle_move(P->z[p], P->rho[p], u, dt, &ze, &re);
            double q_ring = P->sp_qw[sp] / O_TWO_PI;
            int nseg = walk(m, P, p, ze, re, q_ring / dt, q_ring, Jl, Ql, Sl);
            if (nseg > 0) Sl[0] += nseg;
        }
        Kt[2 * tid] = kol;
        Kt[2 * tid + 1] = knl;
    }
    for (int th = 0; th < nth; ++th) {
        k_old += Kt[2 * th];
        k_new += Kt[2 * th + 1];
    }
    free(Kt);
    if (nth > 1) {
        for (int th = 0; th < nth; ++th) {
            const double *Jl = Jt + (size_t)th * m->n1, *Ql = Qt + (size_t)th * m->n0;
            for (int64_t e = 0; e < m->n1; ++e) J[e] += Jl[e];
            for (int64_t v = 0; v < m->n0; ++v) Qres[v] += Ql[v];
            for (int k = 0; k < 3; ++k) stats[k] += St[3 * th + k];
        }
        free(Jt);
        free(Qt);
        free(St);
    }

    /* 5. Ampere: rhs = C^T H B^{n+1/2} - J on free edges; in the absorbing
     *    layer the face's H-image obeys s_z h = H B, integrated by the
     *    trapezoidal rule: h^{n+1/2} = ((1 - beta) h^{n-1/2} + H (B^{n+1/2} - B^{n-1/2})) / (1 + beta) */
    memset(rhs, 0, sizeof(double) * m->n1);
    for (int64_t t = 0; t < m->n2; ++t) {
        double hb = m->H[t] * Bh[t];
        for (int k = 0; k < 3; ++k)
            rhs[m->tri_edges[3 * t + k]] += (double)m->tri_signs[3 * t + k] * hb;
    }
    if (pml)
        for (int64_t i = 0; i < pml->n; ++i) {
            int64_t t = pml->face[i];
            double b = pml->beta[i];
            double hn = ((1.0 - b) * pml->h[i] + m->H[t] * (Bh[t] - B[t])) / (1.0 + b);
            double dh = hn - m->H[t] * Bh[t];          /* replace H B by h on this face */
            for (int k = 0; k < 3; ++k)
                rhs[m->tri_edges[3 * t + k]] += (double)m->tri_signs[3 * t + k] * dh;
            pml->h[i] = hn;
        }
    for (int64_t e = 0; e < m->n1; ++e)
        rhs[e] = m->edge_free[e] ? rhs[e] - J[e] : 0.0;
    if (!pml) {
        for (int64_t e = 0; e < m->n1; ++e) {
            if (!m->edge_free[e]) { E[e] = 0.0; continue; }
            double acc = 0.0;
            for (int64_t j = m->m_ptr[e]; j < m->m_ptr[e + 1]; ++j)
                acc += m->m_val[j] * rhs[m->m_col[j]];
            E[e] += dt * acc;
            D[e] += dt * rhs[e];
        }
    } else {
        /* D-form with the layer: D is the quantity with E = M D, M the SPAI
         * of the stretched Hodge sum_T [(1 + beta) A_rho + A_z / (1 + beta)].
         * After E^{n+1} = M (D^n + dt rhs), each layer face updates
         *   q^{n+1} = ((1 - beta) q^n + A_z (e^{n+1} - e^n)) / (1 + beta)
         *   D      -= 2 beta (A_rho e^{n+1} - q^{n+1} / (1 + beta))   on its sides */
        for (int64_t e = 0; e < m->n1; ++e) D[e] = m->edge_free[e] ? D[e] + dt * rhs[e] : 0.0;
        for (int64_t e = 0; e < m->n1; ++e) {
            if (!m->edge_free[e]) { E[e] = 0.0; continue; }
            double acc = 0.0;
            for (int64_t j = m->m_ptr[e]; j < m->m_ptr[e + 1]; ++j)
                acc += m->m_val[j] * D[m->m_col[j]];
            E[e] = acc;
        }
        for (int64_t i = 0; i < pml->n; ++i) {
            int64_t t = pml->face[i];
            double b = pml->beta[i], en[3], de[3];
            for (int k = 0; k < 3; ++k) {
                en[k] = E[m->tri_edges[3 * t + k]];
                de[k] = en[k] - pml->eprev[3 * i + k];
            }
            for (int k = 0; k < 3; ++k) {
                double az = 0.0, ar = 0.0;
                for (int l = 0; l < 3; ++l) {
                    az += pml->Az[9 * i + 3 * k + l] * de[l];
                    ar += pml->Ar[9 * i + 3 * k + l] * en[l];
                }
                double qn = ((1.0 - b) * pml->q[3 * i + k] + az) / (1.0 + b);
                pml->q[3 * i + k] = qn;
                int64_t e = m->tri_edges[3 * t + k];
                if (m->edge_free[e]) D[e] -= 2.0 * b * (ar - qn / (1.0 + b));
            }
            for (int k = 0; k < 3; ++k) pml->eprev[3 * i + k] = en[k];
        }
    }
    memcpy(B, Bh, sizeof(double) * m->n2);
    if (energy) {
        energy[0] = 0.5 * we;
        energy[1] = 0.5 * wb;
        energy[2] = 0.5 * (k_old + k_new);
        energy[3] = k_new;
    }
}

/* threads the step uses (1 without OpenMP) */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Nodal charge, eq. (charge): Q_v = sum_p (q/2pi) lam_v(r_p) + Qres_v */
void oracle_charge(const omesh *m, const oparticles *P, const double *Qres, double *Q)
{
    memcpy(Q, Qres, sizeof(double) * m->n0);
    for (int64_t p = 0; p < P->n; ++p) {
        if (!P->alive[p]) continue;
        double lam[3];
        bary(m, P->tri[p], P->z[p], P->rho[p], lam);
        const int64_t *v = m->tris + 3 * P->tri[p];
        double q = P->sp_qw[P->species[p]] / O_TWO_PI;
        for (int i = 0; i < 3; ++i) Q[v[i]] += q * lam[i];
    }
}

/* Field at points (for probes and tests): E (z, rho) and B_phi of the
 * Whitney expansions in the given triangles. */
void oracle_sample(const omesh *m, int64_t n, const int64_t *tri, const double *z, const double *rho,
                   const double *E, const double *Bface, double *out /* [n][3]: Ez, Erho, Bphi */)
{
    for (int64_t i = 0; i < n; ++i) {
        double lam[3], e2[2];
        bary(m, tri[i], z[i], rho[i], lam);
        gather_E(m, tri[i], lam, E, e2);
        out[3 * i] = e2[0];
        out[3 * i + 1] = e2[1];
        out[3 * i + 2] = Bface[tri[i]] / tri_area(m, tri[i]);
    }
}

/* Single-particle walk without fields (for brute-force current checks):
 * moves particle p to (ze, re) and deposits (q/2pi/dt) int W1 . dr. */
int oracle_walk_only(const omesh *m, oparticles *P, int64_t p, double ze, double re, double dt,
                     double *J, double *Qres, int64_t *stats)
{
    double q_ring = P->sp_qw[P->species[p]] / O_TWO_PI;
    return walk(m, P, p, ze, re, q_ring / dt, q_ring, J, Qres, stats);
}
