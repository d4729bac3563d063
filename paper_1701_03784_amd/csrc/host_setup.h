// Host-side (FP64) setup of the axisymmetric EM-PIC discretisation: mesh
// topology and locality order, Hodge matrices, SPAI, stability limit, CG.
#pragma once

#include <array>
#include <cstdint>
#include <string>
#include <vector>

namespace axp {

constexpr double kC = 299792458.0;
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kMu0 = 1.0 / (kEps0 * kC * kC);
constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr int kLamBits = 23;                       // element-local fixed point: lambda * 2^23
constexpr int64_t kLamOne = int64_t(1) << kLamBits;

enum Tag : int { TAG_NONE = 0, TAG_PEC = 1, TAG_AXIS = 2, TAG_EMITTER = 3, TAG_OPEN = 4 };

struct Csr {
    int64_t n = 0;
    std::vector<int64_t> ptr;
    std::vector<int32_t> col;
    std::vector<double> val;
    void spmv(const double *x, double *y) const;
};

struct SetupError {
    int code;
    std::string msg;
};

// Mesh in the library's internal numbering.  Local node k of a triangle is
// opposite its side k; side k runs from local node k+1 to k+2 (counter-
// clockwise), so its incidence sign is +1 when that direction agrees with
// the edge orientation tail -> head (tail < head, global node ids).
// Strip ordering of faces is used while a strip holds at most this many
// faces (about 2 x short extent / edge length): the neighbours of a face
// then stay inside the particle kernel's accumulation window.
constexpr int kStripMaxFaces = 224;

struct HostMesh {
    int32_t n0 = 0, n1 = 0, n2 = 0;
    std::vector<double> z, r;                      // node coordinates, user order
    std::vector<int32_t> tri_user;                 // internal face -> user face
    std::vector<int32_t> tri_int;                  // user face -> internal face
    bool strip_order = false;                      // faces in strips (else along a Hilbert curve)
    std::vector<std::array<int32_t, 3>> tv;        // internal face -> nodes (CCW)
    std::vector<std::array<int32_t, 2>> ev;        // internal edge -> (tail, head)
    std::vector<int32_t> edge_can;                 // internal edge -> canonical edge
    std::vector<int32_t> edge_int;                 // canonical edge -> internal edge
    std::vector<std::array<int32_t, 3>> tedge;     // face side k -> internal edge
    std::vector<std::array<int8_t, 3>> tsign;      // face side k -> incidence sign
    std::vector<std::array<int32_t, 3>> tnbr;      // face across side k, or -tag
    std::vector<uint32_t> tnbr_map;                // 4 bits per side: local ids in the neighbour
    std::vector<std::array<int32_t, 2>> etri;      // edge -> (left face, right face or -1)
    std::vector<std::array<int8_t, 2>> eside;      // side index of the edge in those faces
    std::vector<int32_t> etag;                     // 0 interior, else boundary tag
    std::vector<uint8_t> efree;                    // E unknown on the edge
    std::vector<uint8_t> nfree;                    // node touches no conductor edge
    std::vector<double> area;                      // face areas (internal)
    std::vector<std::array<double, 6>> grad;       // grad lambda_k (z, rho) per face
    std::vector<double> H;                         // [*mu^-1] diagonal (internal faces)
    Csr A;                                         // [*eps] over internal edges
    Csr M;                                         // SPAI of [*eps] (free rows/cols)
    double spai_fro = 0, spai_max_col = 0;
    int64_t spai_nnz = 0;
    int32_t n_free_edges = 0, n_free_nodes = 0;
    // node -> incident edges with divergence sign (+1 tail, -1 head)
    std::vector<int32_t> nptr, nedge;
    std::vector<int8_t> nsign;
    // point location grid
    double gz0 = 0, gr0 = 0, ghz = 1, ghr = 1;
    int32_t gnz = 0, gnr = 0;
    std::vector<int32_t> gptr, gtri;
};

// Jacobi-scaled [*eps] over the free edges: A^ = S^-1/2 A S^-1/2.
struct ScaledHodge {
    std::vector<int32_t> fidx;     // internal edge -> free index (-1: conductor edge)
    std::vector<int32_t> fedge;    // free index -> internal edge
    std::vector<double> s;         // diag(A)^-1/2
    std::vector<std::vector<std::pair<int32_t, double>>> adj;   // rows of A^ (free indices)
};

struct SpaiEntry {
    int32_t row, col;
    double v;
};

constexpr int kSpaiFeatures = 16;

// Pairs (k, j), j in the level-L pattern of free column k (sorted), and
// their network features X[pair][kSpaiFeatures].
struct PairSet {
    std::vector<int64_t> ptr;      // per free column
    std::vector<int32_t> j;
    std::vector<float> X;
};

struct LearnedSpaiStats {
    int64_t n_fallback = 0;        // columns replaced by least squares
    double pred_resid_mean = 0;    // mean ||e_k - A^ m_k|| of the network's columns
    double kept_resid_mean = 0;    // same after the refinement, over the kept columns
};

// Builds topology, locality order and incidence.  seg: boundary segments.
// Stretched-coordinate absorbing layers at the z ends (sides: bit 0 below
// z_left, bit 1 above z_right), conductivity sigma_max (depth/thickness)^order.
struct LayerConfig {
    int sides = 0;
    double z_left = 0.0, z_right = 0.0, sigma_max = 0.0;
    int order = 3;
};

// Faces of the layers: beta = sigma dt / (2 eps0), and the z and rho parts of
// their local [*eps] (9 values each, sides k, l of the face).
struct HostLayers {
    std::vector<int32_t> face;
    std::vector<double> beta, Az, Ar;
};

void build_topology(HostMesh &m, int32_t n_nodes, const double *zr, int32_t n_tris, const int32_t *tri,
                    int32_t n_seg, const int32_t *seg, const uint8_t *tag);
void assemble_hodge(HostMesh &m);
// eps0 int_T rho W_k . W_l on face t: comp 0 z parts, 1 rho parts, -1 all
void local_hodge(const HostMesh &m, int t, int comp, double out[3][3]);
// layer faces and the stretched Hodge K (the pattern of A, values changed on layer faces)
void build_layers(const HostMesh &m, double dt, const LayerConfig &cfg, HostLayers &L, Csr &K);
void build_spai(HostMesh &m, int level, double drop_tol, int n_threads);
void scaled_hodge(const HostMesh &m, ScaledHodge &h);
// least-squares columns (all free columns if cols is null), after the drop rule
void spai_ls_columns(const ScaledHodge &h, int level, double drop_tol, const std::vector<int32_t> *cols, int n_threads,
                     std::vector<SpaiEntry> &out);
// symmetric average, unscaling into m.M, residual statistics
void finish_spai(HostMesh &m, const ScaledHodge &h, std::vector<SpaiEntry> &entries, int n_threads);
void spai_pair_features(const HostMesh &m, const ScaledHodge &h, int level, int n_threads, PairSet &ps);
void learned_spai(HostMesh &m, const ScaledHodge &h, const PairSet &ps, const float *pred, int level, double drop_tol,
                  int iters, double row_tol, int n_threads, LearnedSpaiStats &st);
double leapfrog_energy_drift(const HostMesh &m, double dt, int steps, uint64_t seed);
double cfl_dt(const HostMesh &m, int iters);
// Solves M x = b on free edges (conjugate gradients, FP64); returns iterations.
int cg_solve_M(const HostMesh &m, const double *b, double *x, double rtol, int max_iter);
// Electrostatic initial state: potential phi (phi_c on conductor nodes),
// E = -G phi (zero on conductor edges), D = M^-1 E with D~div D = Q on the
// free nodes.  Returns the outer iterations, or -1 without convergence;
// res_rel receives max |D~div D - Q| over the free nodes / the D scale.
int electrostatic_state(const HostMesh &m, const double *phi_c, const double *Q, double rtol, int max_outer,
                        std::vector<double> &phi, std::vector<double> &E, std::vector<double> &D, double &res_rel);
void build_locator(HostMesh &m);
// Locates (z, rho); returns the internal face and barycentric coordinates, or -1.
int32_t locate_point(const HostMesh &m, double z, double rho, double lam[3]);

}  // namespace axp
