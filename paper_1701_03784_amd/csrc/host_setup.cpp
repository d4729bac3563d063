// Host-side FP64 setup: topology (App. D), Hodge matrices (Sec. 3.1, App. B),
// plain SPAI of [*eps] (Sec. 3.1), leapfrog stability limit, CG, locator.
#include "host_setup.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <thread>
#include <unordered_map>

#include "../../include/axpic.h"

namespace axp {

void Csr::spmv(const double *x, double *y) const {
    for (int64_t i = 0; i < n; ++i) {
        double s = 0;
        for (int64_t j = ptr[i]; j < ptr[i + 1]; ++j) s += val[j] * x[col[j]];
        y[i] = s;
    }
}

static inline uint64_t edge_key(int32_t a, int32_t b) {
    if (a > b) std::swap(a, b);
    return (uint64_t(uint32_t(a)) << 32) | uint32_t(b);
}

// Position of (x, y) on a Hilbert curve over a 2^order grid (iterative
// quadrant rotation of the classical construction).
static uint64_t hilbert_index(uint32_t x, uint32_t y, int order) {
    uint64_t d = 0;
    for (uint32_t s = 1u << (order - 1); s > 0; s >>= 1) {
        uint32_t rx = (x & s) ? 1 : 0;
        uint32_t ry = (y & s) ? 1 : 0;
        d += uint64_t(s) * uint64_t(s) * ((3 * rx) ^ ry);
        if (ry == 0) {
            if (rx == 1) {
                x = s - 1 - x;
                y = s - 1 - y;
            }
            std::swap(x, y);
        }
    }
    return d;
}

void build_topology(HostMesh &m, int32_t n_nodes, const double *zr, int32_t n_tris, const int32_t *tri,
                    int32_t n_seg, const int32_t *seg, const uint8_t *tag) {
    m.n0 = n_nodes;
    m.n2 = n_tris;
    m.z.resize(n_nodes);
    m.r.resize(n_nodes);
    for (int i = 0; i < n_nodes; ++i) {
        m.z[i] = zr[2 * i];
        m.r[i] = zr[2 * i + 1];
        if (!(m.r[i] >= 0.0) || !std::isfinite(m.z[i])) throw SetupError{AXP_E_MESH, "node with rho < 0 or non-finite"};
    }
    // Locality order of faces.  The particle kernel accumulates a block's
    // currents and charges in an LDS window of consecutive faces (from 192
    // before the block's first face to 320 after it); a path that ends in a
    // face outside it costs a global atomic.  Strips: columns about one edge
    // length wide across the long axis, each ordered along the short axis,
    // so a face's neighbours lie within about one column's face count of it.
    // Used while a column holds few enough faces for the window; wider
    // meshes take the Hilbert index of the centroid.
    double zmin = 1e300, zmax = -1e300, rmin = 1e300, rmax = -1e300;
    for (int i = 0; i < n_nodes; ++i) {
        zmin = std::min(zmin, m.z[i]); zmax = std::max(zmax, m.z[i]);
        rmin = std::min(rmin, m.r[i]); rmax = std::max(rmax, m.r[i]);
    }
    double ext = std::max(zmax - zmin, rmax - rmin);
    if (!(ext > 0)) throw SetupError{AXP_E_MESH, "degenerate node set"};
    double area_sum = 0.0;
    for (int t = 0; t < n_tris; ++t) {
        const int32_t *v = tri + 3 * t;
        area_sum += 0.5 * std::fabs((m.z[v[1]] - m.z[v[0]]) * (m.r[v[2]] - m.r[v[0]]) -
                                    (m.z[v[2]] - m.z[v[0]]) * (m.r[v[1]] - m.r[v[0]]));
    }
    const double hcol = std::sqrt(2.0 * area_sum / std::max(1, n_tris));   // about one edge length
    const bool z_long = (zmax - zmin) >= (rmax - rmin);
    const double short_ext = z_long ? rmax - rmin : zmax - zmin;
    const bool strips = hcol > 0.0 && 2.0 * short_ext / hcol <= double(kStripMaxFaces);
    m.strip_order = strips;
    std::vector<std::pair<uint64_t, int32_t>> order(n_tris);
    for (int t = 0; t < n_tris; ++t) {
        const int32_t *v = tri + 3 * t;
        for (int k = 0; k < 3; ++k)
            if (v[k] < 0 || v[k] >= n_nodes) throw SetupError{AXP_E_MESH, "triangle node id out of range"};
        double a2 = (m.z[v[1]] - m.z[v[0]]) * (m.r[v[2]] - m.r[v[0]]) - (m.z[v[2]] - m.z[v[0]]) * (m.r[v[1]] - m.r[v[0]]);
        if (!(a2 > 0)) throw SetupError{AXP_E_MESH, "triangle " + std::to_string(t) + " is not counter-clockwise in (z, rho)"};
        double cz = (m.z[v[0]] + m.z[v[1]] + m.z[v[2]]) / 3.0, cr = (m.r[v[0]] + m.r[v[1]] + m.r[v[2]]) / 3.0;
        uint32_t qx = uint32_t(std::min(65535.0, std::floor((cz - zmin) / ext * 65536.0)));
        uint32_t qy = uint32_t(std::min(65535.0, std::floor((cr - rmin) / ext * 65536.0)));
        if (strips) {
            const double cl = z_long ? cz - zmin : cr - rmin, cs = z_long ? cr - rmin : cz - zmin;
            const uint64_t col = uint64_t(cl / hcol);
            const uint64_t pos = uint64_t(std::min(4294967295.0, std::floor(cs / ext * 4294967296.0)));
            order[t] = {(col << 32) | pos, t};
        } else {
            order[t] = {hilbert_index(qx, qy, 16), t};
        }
    }
    std::sort(order.begin(), order.end());
    m.tri_user.resize(n_tris);
    m.tri_int.resize(n_tris);
    m.tv.resize(n_tris);
    for (int t = 0; t < n_tris; ++t) {
        int u = order[t].second;
        m.tri_user[t] = u;
        m.tri_int[u] = t;
        m.tv[t] = {tri[3 * u], tri[3 * u + 1], tri[3 * u + 2]};
    }
    // edges numbered by first appearance along the face order
    std::unordered_map<uint64_t, int32_t> eid;
    eid.reserve(size_t(n_tris) * 2);
    m.tedge.resize(n_tris);
    m.tsign.resize(n_tris);
    m.ev.clear();
    std::vector<std::array<int32_t, 2>> etri;
    std::vector<std::array<int8_t, 2>> eside;
    for (int t = 0; t < n_tris; ++t) {
        for (int k = 0; k < 3; ++k) {
            int32_t a = m.tv[t][(k + 1) % 3], b = m.tv[t][(k + 2) % 3];   // side k: a -> b (CCW)
            uint64_t key = edge_key(a, b);
            auto it = eid.find(key);
            int32_t e;
            if (it == eid.end()) {
                e = int32_t(m.ev.size());
                eid.emplace(key, e);
                m.ev.push_back({std::min(a, b), std::max(a, b)});
                etri.push_back({t, -1});
                eside.push_back({int8_t(k), int8_t(-1)});
            } else {
                e = it->second;
                if (etri[e][1] >= 0) throw SetupError{AXP_E_MESH, "edge shared by more than two triangles"};
                etri[e][1] = t;
                eside[e][1] = int8_t(k);
            }
            m.tedge[t][k] = e;
            m.tsign[t][k] = (a < b) ? 1 : -1;
        }
    }
    m.n1 = int32_t(m.ev.size());
    m.etri = etri;
    m.eside = eside;
    // canonical (sorted) edge order for the interface
    std::vector<int32_t> idx(m.n1);
    for (int i = 0; i < m.n1; ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](int32_t x, int32_t y) { return m.ev[x] < m.ev[y]; });
    m.edge_int = idx;
    m.edge_can.resize(m.n1);
    for (int c = 0; c < m.n1; ++c) m.edge_can[idx[c]] = c;
    // boundary tags
    std::unordered_map<uint64_t, int> stag;
    for (int s = 0; s < n_seg; ++s) stag[edge_key(seg[2 * s], seg[2 * s + 1])] = tag[s];
    m.etag.assign(m.n1, TAG_NONE);
    m.tnbr.resize(n_tris);
    m.tnbr_map.assign(n_tris, 0u);
    for (int e = 0; e < m.n1; ++e) {
        if (m.etri[e][1] < 0) {
            auto it = stag.find(edge_key(m.ev[e][0], m.ev[e][1]));
            if (it == stag.end())
                throw SetupError{AXP_E_MESH, "boundary edge (" + std::to_string(m.ev[e][0]) + "," +
                                                 std::to_string(m.ev[e][1]) + ") has no boundary tag"};
            if (it->second < TAG_PEC || it->second > TAG_OPEN) throw SetupError{AXP_E_MESH, "unknown boundary tag"};
            m.etag[e] = it->second;
        }
    }
    for (int t = 0; t < n_tris; ++t) {
        for (int k = 0; k < 3; ++k) {
            int e = m.tedge[t][k];
            int other = (m.etri[e][0] == t) ? m.etri[e][1] : m.etri[e][0];
            if (other < 0) {
                m.tnbr[t][k] = -m.etag[e];
            } else {
                m.tnbr[t][k] = other;
                int32_t a = m.tv[t][(k + 1) % 3], b = m.tv[t][(k + 2) % 3];
                uint32_t pa = 3, pb = 3;
                for (int j = 0; j < 3; ++j) {
                    if (m.tv[other][j] == a) pa = j;
                    if (m.tv[other][j] == b) pb = j;
                }
                m.tnbr_map[t] |= (pa | (pb << 2)) << (4 * k);
            }
        }
    }
    m.efree.resize(m.n1);
    m.nfree.assign(m.n0, 1);
    m.n_free_edges = 0;
    for (int e = 0; e < m.n1; ++e) {
        bool cond = (m.etag[e] == TAG_PEC || m.etag[e] == TAG_EMITTER);
        m.efree[e] = cond ? 0 : 1;
        m.n_free_edges += m.efree[e];
        if (cond) m.nfree[m.ev[e][0]] = m.nfree[m.ev[e][1]] = 0;
    }
    m.n_free_nodes = 0;
    for (int v = 0; v < m.n0; ++v) m.n_free_nodes += m.nfree[v];
    // node -> edges with divergence sign (+1 at the tail, -1 at the head)
    m.nptr.assign(m.n0 + 1, 0);
    for (int e = 0; e < m.n1; ++e) { m.nptr[m.ev[e][0] + 1]++; m.nptr[m.ev[e][1] + 1]++; }
    for (int v = 0; v < m.n0; ++v) m.nptr[v + 1] += m.nptr[v];
    m.nedge.resize(m.nptr[m.n0]);
    m.nsign.resize(m.nptr[m.n0]);
    std::vector<int32_t> cur(m.nptr.begin(), m.nptr.end() - 1);
    for (int e = 0; e < m.n1; ++e) {
        int c0 = cur[m.ev[e][0]]++, c1 = cur[m.ev[e][1]]++;
        m.nedge[c0] = e; m.nsign[c0] = 1;
        m.nedge[c1] = e; m.nsign[c1] = -1;
    }
    // geometry
    m.area.resize(n_tris);
    m.grad.resize(n_tris);
    for (int t = 0; t < n_tris; ++t) {
        double zz[3], rr[3];
        for (int k = 0; k < 3; ++k) { zz[k] = m.z[m.tv[t][k]]; rr[k] = m.r[m.tv[t][k]]; }
        double a2 = (zz[1] - zz[0]) * (rr[2] - rr[0]) - (zz[2] - zz[0]) * (rr[1] - rr[0]);
        m.area[t] = 0.5 * a2;
        for (int k = 0; k < 3; ++k) {
            int j = (k + 1) % 3, l = (k + 2) % 3;
            m.grad[t][2 * k] = (rr[j] - rr[l]) / a2;       // d lambda_k / dz
            m.grad[t][2 * k + 1] = (zz[l] - zz[j]) / a2;   // d lambda_k / drho
        }
    }
}

// int_T lambda_i lambda_j lambda_k dA = 2 Area (product of multiplicity factorials) / 5!
static double moment3(int i, int j, int k, double area) {
    int c[3] = {0, 0, 0};
    c[i]++; c[j]++; c[k]++;
    static const double fact[4] = {1, 1, 2, 6};
    return 2.0 * area * fact[c[0]] * fact[c[1]] * fact[c[2]] / 120.0;
}

void local_hodge(const HostMesh &m, int t, int comp, double out[3][3]) {
    // eps0 int_T rho W_k . W_l over the face's sides k, l (edge orientation of
    // each side), W_(a,b) = lam_a grad lam_b - lam_b grad lam_a; comp 0 keeps
    // the z components of the product only, 1 the rho components, -1 both
    const auto &g = m.grad[t];
    double gg[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            gg[a][b] = (comp != 1 ? g[2 * a] * g[2 * b] : 0.0) + (comp != 0 ? g[2 * a + 1] * g[2 * b + 1] : 0.0);
    const double rho[3] = {m.r[m.tv[t][0]], m.r[m.tv[t][1]], m.r[m.tv[t][2]]};
    int ta[3], hb[3];
    for (int k = 0; k < 3; ++k) {
        const int32_t e = m.tedge[t][k];
        const int la = (k + 1) % 3, lb = (k + 2) % 3;   // CCW side from la to lb
        if (m.tv[t][la] == m.ev[e][0]) { ta[k] = la; hb[k] = lb; } else { ta[k] = lb; hb[k] = la; }
    }
    const double A = m.area[t];
    for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) {
            const int a = ta[k], b = hb[k], c = ta[l], d = hb[l];
            double s = 0;
            for (int q = 0; q < 3; ++q)
                s += rho[q] * (moment3(q, a, c, A) * gg[b][d] - moment3(q, a, d, A) * gg[b][c] -
                               moment3(q, b, c, A) * gg[a][d] + moment3(q, b, d, A) * gg[a][c]);
            out[k][l] = kEps0 * s;
        }
}

void assemble_hodge(HostMesh &m) {
    // [*eps]_ij = eps0 int rho W_i . W_j, W_(a,b) = lam_a grad lam_b - lam_b grad lam_a
    std::vector<std::vector<std::pair<int32_t, double>>> rows(m.n1);
    for (auto &r : rows) r.reserve(5);
    m.H.resize(m.n2);
    for (int t = 0; t < m.n2; ++t) {
        double T[3][3];
        local_hodge(m, t, -1, T);
        for (int k = 0; k < 3; ++k) {
            for (int l = 0; l < 3; ++l) {
                int32_t ek = m.tedge[t][k], el = m.tedge[t][l];
                auto &row = rows[ek];
                bool found = false;
                for (auto &p : row)
                    if (p.first == el) { p.second += T[k][l]; found = true; break; }
                if (!found) row.push_back({el, T[k][l]});
            }
        }
        // [*mu^-1]_T = (1/mu0) int_T rho (W2)^2, W2 = 1/Area
        const double rho[3] = {m.r[m.tv[t][0]], m.r[m.tv[t][1]], m.r[m.tv[t][2]]};
        m.H[t] = (rho[0] + rho[1] + rho[2]) / (3.0 * kMu0 * m.area[t]);
    }
    m.A.n = m.n1;
    m.A.ptr.assign(m.n1 + 1, 0);
    for (int i = 0; i < m.n1; ++i) {
        std::sort(rows[i].begin(), rows[i].end());
        m.A.ptr[i + 1] = m.A.ptr[i] + int64_t(rows[i].size());
    }
    m.A.col.resize(m.A.ptr[m.n1]);
    m.A.val.resize(m.A.ptr[m.n1]);
    for (int i = 0; i < m.n1; ++i)
        for (size_t j = 0; j < rows[i].size(); ++j) {
            m.A.col[m.A.ptr[i] + j] = rows[i][j].first;
            m.A.val[m.A.ptr[i] + j] = rows[i][j].second;
        }
}

// Dense least squares min ||B x - b|| by Householder QR (B: rows x cols,
// column-major, modified in place).  Returns false if a pivot vanishes.
static bool householder_ls(int rows, int cols, double *B, double *b, double *x) {
    for (int j = 0; j < cols; ++j) {
        double *cj = B + size_t(j) * rows;
        double norm = 0;
        for (int i = j; i < rows; ++i) norm += cj[i] * cj[i];
        norm = std::sqrt(norm);
        if (norm == 0.0) return false;
        double alpha = cj[j] > 0 ? -norm : norm;
        double v0 = cj[j] - alpha;
        // v = (v0, cj[j+1..]); H = I - 2 v v^T / (v^T v)
        double vtv = v0 * v0;
        for (int i = j + 1; i < rows; ++i) vtv += cj[i] * cj[i];
        cj[j] = v0;
        for (int c = j + 1; c < cols; ++c) {
            double *cc = B + size_t(c) * rows;
            double s = 0;
            for (int i = j; i < rows; ++i) s += cj[i] * cc[i];
            s = 2.0 * s / vtv;
            for (int i = j; i < rows; ++i) cc[i] -= s * cj[i];
        }
        double s = 0;
        for (int i = j; i < rows; ++i) s += cj[i] * b[i];
        s = 2.0 * s / vtv;
        for (int i = j; i < rows; ++i) b[i] -= s * cj[i];
        cj[j] = alpha;   // R diagonal
    }
    for (int j = cols - 1; j >= 0; --j) {
        double s = b[j];
        for (int c = j + 1; c < cols; ++c) s -= B[size_t(c) * rows + j] * x[c];
        double d = B[size_t(j) * rows + j];
        if (d == 0.0) return false;
        x[j] = s / d;
    }
    return true;
}

void scaled_hodge(const HostMesh &m, ScaledHodge &h) {
    // free-edge numbering and Jacobi scaling A^ = S^-1/2 A S^-1/2
    h.fidx.assign(m.n1, -1);
    h.fedge.clear();
    for (int e = 0; e < m.n1; ++e)
        if (m.efree[e]) { h.fidx[e] = int32_t(h.fedge.size()); h.fedge.push_back(e); }
    const int nf = int(h.fedge.size());
    h.s.assign(nf, 0.0);
    h.adj.assign(nf, {});
    for (int i = 0; i < nf; ++i) {
        int e = h.fedge[i];
        double d = 0;
        for (int64_t j = m.A.ptr[e]; j < m.A.ptr[e + 1]; ++j)
            if (m.A.col[j] == e) d = m.A.val[j];
        if (!(d > 0)) throw SetupError{AXP_E_SPAI, "non-positive diagonal of [*eps]"};
        h.s[i] = 1.0 / std::sqrt(d);
    }
    for (int i = 0; i < nf; ++i) {
        int e = h.fedge[i];
        for (int64_t j = m.A.ptr[e]; j < m.A.ptr[e + 1]; ++j) {
            int c = h.fidx[m.A.col[j]];
            if (c >= 0 && m.A.val[j] != 0.0) h.adj[i].push_back({c, h.s[i] * m.A.val[j] * h.s[c]});
        }
    }
}

// Runs body(tid) on n_threads threads.
template <class F>
static void parallel(int n_threads, F &&body) {
    const int nt = std::max(1, n_threads);
    std::vector<std::thread> th;
    for (int t = 1; t < nt; ++t) th.emplace_back(body, t);
    body(0);
    for (auto &t : th) t.join();
}

// Columns J_k (free edges within `level` hops of k, sorted) with their hop
// distance; work arrays are per thread.
struct PatternWork {
    std::vector<int32_t> mark, dist, J, frontier, nxt;
    explicit PatternWork(int nf) : mark(nf, -1), dist(nf, 0) {}
    void column(const ScaledHodge &h, int k, int level) {
        J.clear(); frontier.clear();
        J.push_back(k); frontier.push_back(k); mark[k] = k; dist[k] = 0;
        for (int l = 0; l < level; ++l) {   // structure of A^level: within `level` hops
            nxt.clear();
            for (int u : frontier)
                for (auto &p : h.adj[u])
                    if (mark[p.first] != k) {
                        mark[p.first] = k;
                        dist[p.first] = l + 1;
                        nxt.push_back(p.first);
                        J.push_back(p.first);
                    }
            frontier.swap(nxt);
        }
        std::sort(J.begin(), J.end());
    }
};

void spai_ls_columns(const ScaledHodge &h, int level, double drop_tol, const std::vector<int32_t> *cols, int n_threads,
                     std::vector<SpaiEntry> &out) {
    const int nf = int(h.fedge.size());
    const int ncols = cols ? int(cols->size()) : nf;
    // column k: pattern J_k = nodes within `level` hops, rows I_k = J_k plus one more hop
    std::vector<std::vector<SpaiEntry>> per_thread(std::max(1, n_threads));
    std::atomic<int> next{0};
    std::atomic<bool> failed{false};
    parallel(n_threads, [&](int tid) {
        PatternWork pw(nf);
        std::vector<int32_t> rmark(nf, -1), I;
        std::vector<double> B, rhs, x;
        auto &o = per_thread[tid];
        for (;;) {
            int q0 = next.fetch_add(64);
            if (q0 >= ncols || failed.load()) break;
            for (int q = q0; q < std::min(ncols, q0 + 64); ++q) {
                const int k = cols ? (*cols)[q] : q;
                pw.column(h, k, level);
                const auto &J = pw.J;
                I.clear();
                for (int j : J)
                    for (auto &p : h.adj[j])
                        if (rmark[p.first] != k) { rmark[p.first] = k; I.push_back(p.first); }
                std::sort(I.begin(), I.end());
                const int nr = int(I.size()), nc = int(J.size());
                B.assign(size_t(nr) * nc, 0.0);
                for (int c = 0; c < nc; ++c) {
                    for (auto &p : h.adj[J[c]]) {
                        int r = int(std::lower_bound(I.begin(), I.end(), p.first) - I.begin());
                        B[size_t(c) * nr + r] = p.second;   // A^ symmetric: column J[c] = row J[c]
                    }
                }
                rhs.assign(nr, 0.0);
                rhs[std::lower_bound(I.begin(), I.end(), k) - I.begin()] = 1.0;
                x.assign(nc, 0.0);
                if (!householder_ls(nr, nc, B.data(), rhs.data(), x.data())) { failed = true; break; }
                double mx = 0;
                for (double v : x) mx = std::max(mx, std::fabs(v));
                for (int c = 0; c < nc; ++c)
                    if (std::fabs(x[c]) >= drop_tol * mx) o.push_back({J[c], k, x[c]});
            }
        }
    });
    if (failed) throw SetupError{AXP_E_SPAI, "rank-deficient SPAI least-squares block"};
    for (auto &v : per_thread) out.insert(out.end(), v.begin(), v.end());
}

void finish_spai(HostMesh &m, const ScaledHodge &h, std::vector<SpaiEntry> &entries, int n_threads) {
    const int nf = int(h.fedge.size());
    // symmetric average (M^ + M^T)/2: both halves of every entry, bucketed by
    // row (in any order: each row is sorted below)
    const int64_t ne = int64_t(entries.size());
    std::vector<std::atomic<int64_t>> slot(size_t(nf) + 1);
    for (auto &a : slot) a.store(0, std::memory_order_relaxed);
    auto over_entries = [&](auto &&body) {
        std::atomic<int64_t> next{0};
        parallel(n_threads, [&](int) {
            for (;;) {
                const int64_t q0 = next.fetch_add(65536);
                if (q0 >= ne) break;
                for (int64_t q = q0; q < std::min(ne, q0 + 65536); ++q) body(entries[size_t(q)]);
            }
        });
    };
    over_entries([&](const SpaiEntry &e) {
        slot[size_t(e.row) + 1].fetch_add(1, std::memory_order_relaxed);
        slot[size_t(e.col) + 1].fetch_add(1, std::memory_order_relaxed);
    });
    std::vector<int64_t> start(size_t(nf) + 1, 0);
    for (int i = 0; i < nf; ++i) start[i + 1] = start[i] + slot[size_t(i) + 1].load(std::memory_order_relaxed);
    for (int i = 0; i < nf; ++i) slot[i].store(start[i], std::memory_order_relaxed);
    std::vector<std::pair<int32_t, double>> pairs(static_cast<size_t>(start[nf]));
    over_entries([&](const SpaiEntry &e) {
        pairs[size_t(slot[e.row].fetch_add(1, std::memory_order_relaxed))] = {e.col, 0.5 * e.v};
        pairs[size_t(slot[e.col].fetch_add(1, std::memory_order_relaxed))] = {e.row, 0.5 * e.v};
    });
    entries.clear();
    entries.shrink_to_fit();
    // per row: sort by column and add the halves that meet (a + b: the sum
    // does not depend on the order the columns were solved in)
    std::vector<int64_t> cnt(nf, 0);
    {
        std::atomic<int> next{0};
        parallel(n_threads, [&](int) {
            for (;;) {
                const int i0 = next.fetch_add(1024);
                if (i0 >= nf) break;
                for (int i = i0; i < std::min(nf, i0 + 1024); ++i) {
                    const int64_t b = start[i], e = start[i + 1];
                    std::sort(pairs.begin() + b, pairs.begin() + e);
                    int64_t w = b;
                    for (int64_t q = b; q < e; ++q) {
                        if (w > b && pairs[size_t(w - 1)].first == pairs[size_t(q)].first)
                            pairs[size_t(w - 1)].second += pairs[size_t(q)].second;
                        else
                            pairs[size_t(w++)] = pairs[size_t(q)];
                    }
                    cnt[i] = w - b;
                }
            }
        });
    }
    // CSR over internal edges, unscaled
    m.M = Csr{};
    m.M.n = m.n1;
    m.M.ptr.assign(size_t(m.n1) + 1, 0);
    for (int e = 0; e < m.n1; ++e) {
        const int i = h.fidx[e];
        m.M.ptr[e + 1] = m.M.ptr[e] + (i >= 0 ? cnt[i] : 0);
    }
    m.M.col.resize(size_t(m.M.ptr[m.n1]));
    m.M.val.resize(size_t(m.M.ptr[m.n1]));
    std::vector<double> col2(m.n1, 0.0);
    {
        std::atomic<int> next{0};
        parallel(n_threads, [&](int) {
            std::vector<double> acc(m.n1, 0.0);
            std::vector<int32_t> touched;
            for (;;) {
                const int e0 = next.fetch_add(1024);
                if (e0 >= m.n1) break;
                for (int e = e0; e < std::min(m.n1, e0 + 1024); ++e) {
                    const int i = h.fidx[e];
                    if (i < 0) continue;
                    int64_t o = m.M.ptr[e];
                    for (int64_t q = start[i]; q < start[i] + cnt[i]; ++q, ++o) {
                        const auto &p = pairs[size_t(q)];
                        m.M.col[o] = h.fedge[p.first];
                        m.M.val[o] = h.s[i] * p.second * h.s[p.first];
                    }
                    // residual of the column: A m_e - e_e (M symmetric: column e = row e)
                    touched.clear();
                    for (int64_t j = m.M.ptr[e]; j < m.M.ptr[e + 1]; ++j) {
                        const int c = m.M.col[j];
                        for (int64_t q = m.A.ptr[c]; q < m.A.ptr[c + 1]; ++q) {
                            const int r = m.A.col[q];
                            if (!m.efree[r]) continue;
                            if (acc[r] == 0.0) touched.push_back(r);
                            acc[r] += m.A.val[q] * m.M.val[j];
                        }
                    }
                    acc[e] -= 1.0;
                    if (std::find(touched.begin(), touched.end(), e) == touched.end()) touched.push_back(e);
                    double s2 = 0;
                    for (int r : touched) { s2 += acc[r] * acc[r]; acc[r] = 0.0; }
                    col2[e] = s2;
                }
            }
        });
    }
    m.spai_nnz = m.M.ptr[m.n1];
    double fro = 0, mxc = 0;
    for (int e = 0; e < m.n1; ++e) {        // in edge order, whatever the thread count
        if (!m.efree[e]) continue;
        fro += col2[e];
        mxc = std::max(mxc, std::sqrt(col2[e]));
    }
    m.spai_fro = std::sqrt(fro / std::max(1, nf));
    m.spai_max_col = mxc;
}

void build_spai(HostMesh &m, int level, double drop_tol, int n_threads) {
    ScaledHodge h;
    scaled_hodge(m, h);
    std::vector<SpaiEntry> entries;
    spai_ls_columns(h, level, drop_tol, nullptr, n_threads, entries);
    finish_spai(m, h, entries, n_threads);
}

// ------------------------------------------------------- learned SPAI
// Features of the pairs (k, j), j in J_k, of every free column k; the list
// and its meaning are those of the network's training data.
void spai_pair_features(const HostMesh &m, const ScaledHodge &h, int level, int n_threads, PairSet &ps) {
    const int nf = int(h.fedge.size());
    // per free edge: length, midpoint, unit direction in the meridian plane; row count and |row| sum of A^
    std::vector<double> len(nf), mz(nf), mr(nf), dz(nf), dr(nf), rsum(nf);
    std::vector<int32_t> nrow(nf);
    for (int i = 0; i < nf; ++i) {
        const auto &ev = m.ev[h.fedge[i]];
        const double z0 = m.z[ev[0]], r0 = m.r[ev[0]], z1 = m.z[ev[1]], r1 = m.r[ev[1]];
        const double L = std::sqrt((z1 - z0) * (z1 - z0) + (r1 - r0) * (r1 - r0));
        len[i] = L; mz[i] = 0.5 * (z0 + z1); mr[i] = 0.5 * (r0 + r1);
        dz[i] = (z1 - z0) / L; dr[i] = (r1 - r0) / L;
        nrow[i] = int32_t(h.adj[i].size());
        double a = 0;
        for (auto &p : h.adj[i]) a += std::fabs(p.second);
        rsum[i] = a;
    }
    // pass 1: pattern sizes
    std::vector<int64_t> cnt(nf + 1, 0);
    std::atomic<int> next{0};
    parallel(n_threads, [&](int) {
        PatternWork pw(nf);
        for (;;) {
            int k0 = next.fetch_add(256);
            if (k0 >= nf) break;
            for (int k = k0; k < std::min(nf, k0 + 256); ++k) {
                pw.column(h, k, level);
                cnt[k + 1] = int64_t(pw.J.size());
            }
        }
    });
    ps.ptr.assign(nf + 1, 0);
    for (int k = 0; k < nf; ++k) ps.ptr[k + 1] = ps.ptr[k] + cnt[k + 1];
    const int64_t np = ps.ptr[nf];
    ps.j.assign(np, 0);
    ps.X.assign(size_t(np) * kSpaiFeatures, 0.0f);
    // pass 2: features; (A^^p)_jk by sparse products of column k
    next = 0;
    parallel(n_threads, [&](int) {
        PatternWork pw(nf);
        std::vector<double> v1(nf, 0.0), v2(nf, 0.0), v3(nf, 0.0);
        std::vector<int32_t> t1, t2, t3;
        std::vector<uint8_t> in1(nf, 0), in2(nf, 0), in3(nf, 0);
        auto spread = [&](const std::vector<int32_t> &src, const std::vector<double> &vs, std::vector<int32_t> &dst,
                          std::vector<double> &vd, std::vector<uint8_t> &in) {
            for (int c : src)
                for (auto &p : h.adj[c]) {
                    if (!in[p.first]) { in[p.first] = 1; dst.push_back(p.first); }
                    vd[p.first] += p.second * vs[c];
                }
        };
        for (;;) {
            int k0 = next.fetch_add(256);
            if (k0 >= nf) break;
            for (int k = k0; k < std::min(nf, k0 + 256); ++k) {
                pw.column(h, k, level);
                t1.clear(); t2.clear(); t3.clear();
                for (auto &p : h.adj[k]) { v1[p.first] = p.second; in1[p.first] = 1; t1.push_back(p.first); }
                spread(t1, v1, t2, v2, in2);
                spread(t2, v2, t3, v3, in3);
                int64_t o = ps.ptr[k];
                for (int j : pw.J) {
                    float *f = &ps.X[size_t(o) * kSpaiFeatures];
                    const int d = pw.dist[j];
                    if (d <= 3) f[d] = 1.0f;
                    f[4] = float(v1[j]);
                    f[5] = float(v2[j]);
                    f[6] = float(v3[j]);
                    f[7] = float(std::min(len[k], len[j]) / std::max(len[k], len[j]));
                    const double ddz = mz[k] - mz[j], ddr = mr[k] - mr[j];
                    f[8] = float(std::sqrt(ddz * ddz + ddr * ddr) / (len[k] + len[j]));
                    f[9] = float(std::fabs(dz[k] * dz[j] + dr[k] * dr[j]));
                    const double rmx = std::max(mr[k], mr[j]);
                    f[10] = float(rmx > 0 ? std::min(mr[k], mr[j]) / rmx : 1.0);
                    f[11] = float((len[k] + len[j]) / (mr[k] + mr[j] + len[k] + len[j]));
                    f[12] = float(double(nrow[k] + nrow[j]) / 20.0);
                    f[13] = float(std::fabs(double(nrow[k] - nrow[j])) / 10.0);
                    f[14] = float(0.5 * (rsum[k] + rsum[j]) - 1.0);
                    f[15] = float(double(d) / 3.0);
                    ps.j[o] = j;
                    ++o;
                }
                for (int c : t1) { v1[c] = 0.0; in1[c] = 0; }
                for (int c : t2) { v2[c] = 0.0; in2[c] = 0; }
                for (int c : t3) { v3[c] = 0.0; in3[c] = 0; }
            }
        }
    });
}

// Learned SPAI: the predicted Jacobi-scaled column m_k on the level-L
// pattern J_k is the starting point of `iters` conjugate-gradient steps on
// the normal equations of min ||e_k - A^(:, J_k) m||_2 (CGNR), whose limit is
// the plain SPAI's least-squares column; a column whose residual still
// exceeds row_tol is replaced by the exact least-squares column.  Drop rule,
// symmetric average and unscaling as for the plain SPAI.
void learned_spai(HostMesh &m, const ScaledHodge &h, const PairSet &ps, const float *pred, int level, double drop_tol,
                  int iters, double row_tol, int n_threads, LearnedSpaiStats &st) {
    const int nf = int(h.fedge.size());
    const int nt = std::max(1, n_threads);
    std::vector<std::vector<SpaiEntry>> per_thread(nt);
    std::vector<std::vector<int32_t>> fb_thread(nt);
    std::vector<double> res0_t(nt, 0.0), res_t(nt, 0.0);
    std::atomic<int> next{0};
    parallel(n_threads, [&](int tid) {
        // dense work vectors over free edges, with touched lists
        std::vector<double> r(nf, 0.0), ap(nf, 0.0);
        std::vector<uint8_t> inr(nf, 0), inap(nf, 0);
        std::vector<int32_t> tr, tap;
        std::vector<double> mv, g, pv;
        for (;;) {
            int k0 = next.fetch_add(128);
            if (k0 >= nf) break;
            for (int k = k0; k < std::min(nf, k0 + 128); ++k) {
                const int64_t b = ps.ptr[k], e = ps.ptr[k + 1];
                const int nc = int(e - b);
                const int32_t *J = ps.j.data() + b;
                mv.assign(nc, 0.0);
                for (int c = 0; c < nc; ++c) mv[c] = double(pred[b + c]);
                // r = e_k - A^ m
                for (int q : tr) { r[q] = 0.0; inr[q] = 0; }
                tr.clear();
                for (int c = 0; c < nc; ++c)
                    for (auto &p : h.adj[J[c]]) {
                        if (!inr[p.first]) { inr[p.first] = 1; tr.push_back(p.first); }
                        r[p.first] -= p.second * mv[c];
                    }
                if (!inr[k]) { inr[k] = 1; tr.push_back(k); }
                r[k] += 1.0;
                auto rnorm = [&]() {
                    double s2 = 0;
                    for (int q : tr) s2 += r[q] * r[q];
                    return std::sqrt(s2);
                };
                res0_t[tid] += rnorm();
                // g = (A^ r) on the pattern (A^ symmetric)
                auto grad = [&](std::vector<double> &out) {
                    out.assign(nc, 0.0);
                    for (int c = 0; c < nc; ++c) {
                        double v = 0;
                        for (auto &p : h.adj[J[c]]) v += p.second * r[p.first];
                        out[c] = v;
                    }
                };
                grad(g);
                pv = g;
                double gg = 0;
                for (double v : g) gg += v * v;
                const double floor = 1e-26 * gg;   // the column has converged below this
                for (int it = 0; it < iters && gg > floor; ++it) {
                    for (int q : tap) { ap[q] = 0.0; inap[q] = 0; }
                    tap.clear();
                    for (int c = 0; c < nc; ++c) {
                        if (pv[c] == 0.0) continue;
                        for (auto &p : h.adj[J[c]]) {
                            if (!inap[p.first]) { inap[p.first] = 1; tap.push_back(p.first); }
                            ap[p.first] += p.second * pv[c];
                        }
                    }
                    double den = 0;
                    for (int q : tap) den += ap[q] * ap[q];
                    if (!(den > 0)) break;
                    const double alpha = gg / den;
                    for (int c = 0; c < nc; ++c) mv[c] += alpha * pv[c];
                    for (int q : tap) {            // r -= alpha A^ p (support of A^ p lies in that of r)
                        if (!inr[q]) { inr[q] = 1; tr.push_back(q); }
                        r[q] -= alpha * ap[q];
                    }
                    grad(g);
                    double gn = 0;
                    for (double v : g) gn += v * v;
                    const double beta = gn / gg;
                    for (int c = 0; c < nc; ++c) pv[c] = g[c] + beta * pv[c];
                    gg = gn;
                }
                const double rn = rnorm();
                if (!(rn <= row_tol)) {           // also catches a non-finite prediction
                    fb_thread[tid].push_back(k);
                    continue;
                }
                res_t[tid] += rn;
                double mx = 0;
                for (double v : mv) mx = std::max(mx, std::fabs(v));
                for (int c = 0; c < nc; ++c)
                    if (std::fabs(mv[c]) >= drop_tol * mx) per_thread[tid].push_back({J[c], k, mv[c]});
            }
        }
    });
    std::vector<int32_t> fb;
    for (auto &v : fb_thread) fb.insert(fb.end(), v.begin(), v.end());
    std::sort(fb.begin(), fb.end());
    std::vector<SpaiEntry> entries;
    for (auto &v : per_thread) entries.insert(entries.end(), v.begin(), v.end());
    st.n_fallback = int64_t(fb.size());
    double r0 = 0, r1 = 0;
    for (double v : res0_t) r0 += v;
    for (double v : res_t) r1 += v;
    st.pred_resid_mean = nf ? r0 / nf : 0.0;
    st.kept_resid_mean = (nf - st.n_fallback) > 0 ? r1 / double(nf - st.n_fallback) : 0.0;
    if (!fb.empty()) spai_ls_columns(h, level, drop_tol, &fb, n_threads, entries);
    finish_spai(m, h, entries, n_threads);
}

// Source-free leapfrog in the D-form with the current M from a seeded random
// D^0 (B^{-1/2} = 0): returns max_n |W^n - W^0| / W^0 of the discrete energy
// W^n = 1/2 E^n . D^n + 1/2 B^{n+1/2} . H B^{n-1/2}, conserved by the
// scheme when M is symmetric positive definite and dt is below the limit.
double leapfrog_energy_drift(const HostMesh &m, double dt, int steps, uint64_t seed) {
    std::vector<double> D(m.n1, 0.0), E(m.n1, 0.0), B(m.n2, 0.0), Bo(m.n2, 0.0);
    uint64_t x = seed * 0x9E3779B97F4A7C15ull + 1;
    for (int e = 0; e < m.n1; ++e) {
        x ^= x << 13; x ^= x >> 7; x ^= x << 17;           // xorshift64
        D[e] = m.efree[e] ? double(x >> 11) * (1.0 / 9007199254740992.0) - 0.5 : 0.0;
    }
    // scale D so that E ~ 1 (keeps the energy O(1))
    m.M.spmv(D.data(), E.data());
    double w0 = -1, drift = 0;
    for (int n = 0; n <= steps; ++n) {
        // B^{n+1/2} = B^{n-1/2} - dt C E^n
        for (int t = 0; t < m.n2; ++t) {
            double c = 0;
            for (int k = 0; k < 3; ++k) c += m.tsign[t][k] * E[m.tedge[t][k]];
            Bo[t] = B[t];
            B[t] -= dt * c;
        }
        double w = 0;
        for (int e = 0; e < m.n1; ++e) w += 0.5 * E[e] * D[e];
        for (int t = 0; t < m.n2; ++t) w += 0.5 * B[t] * m.H[t] * Bo[t];
        if (!std::isfinite(w)) return INFINITY;
        if (w0 < 0) w0 = w;
        else drift = std::max(drift, std::fabs(w - w0) / w0);
        // D^{n+1} = D^n + dt C^T H B^{n+1/2}; E^{n+1} = M D^{n+1}
        for (int t = 0; t < m.n2; ++t) {
            const double hb = dt * m.H[t] * B[t];
            for (int k = 0; k < 3; ++k) {
                const int e = m.tedge[t][k];
                if (m.efree[e]) D[e] += m.tsign[t][k] * hb;
            }
        }
        m.M.spmv(D.data(), E.data());
    }
    return w0 > 0 ? drift : INFINITY;
}

// y = K x with K = C^T diag(H) C restricted to free edges
static void apply_K(const HostMesh &m, const double *x, double *y, std::vector<double> &tmp) {
    tmp.assign(m.n2, 0.0);
    for (int t = 0; t < m.n2; ++t) {
        double c = 0;
        for (int k = 0; k < 3; ++k) {
            int e = m.tedge[t][k];
            if (m.efree[e]) c += m.tsign[t][k] * x[e];
        }
        tmp[t] = m.H[t] * c;
    }
    for (int e = 0; e < m.n1; ++e) {
        double s = 0;
        if (m.efree[e])
            for (int q = 0; q < 2; ++q) {
                int t = m.etri[e][q];
                if (t < 0) continue;
                s += m.tsign[t][m.eside[e][q]] * tmp[t];
            }
        y[e] = s;
    }
}

double cfl_dt(const HostMesh &m, int iters) {
    std::vector<double> x(m.n1), y(m.n1), w(m.n1), tmp;
    uint64_t st = 0x9E3779B97F4A7C15ull;
    for (int e = 0; e < m.n1; ++e) {
        st ^= st << 13; st ^= st >> 7; st ^= st << 17;
        x[e] = m.efree[e] ? (double(st >> 11) / 9007199254740992.0 - 0.5) : 0.0;
    }
    double lam = 0;
    for (int it = 0; it < iters; ++it) {
        apply_K(m, x.data(), w.data(), tmp);
        m.M.spmv(w.data(), y.data());
        double n2 = 0, nx = 0;
        for (int e = 0; e < m.n1; ++e) { n2 += y[e] * y[e]; nx += x[e] * x[e]; }
        lam = std::sqrt(n2 / nx);
        double inv = 1.0 / std::sqrt(n2);
        for (int e = 0; e < m.n1; ++e) x[e] = y[e] * inv;
    }
    return 2.0 / std::sqrt(lam);
}

int cg_solve_M(const HostMesh &m, const double *b, double *x, double rtol, int max_iter) {
    const int n = m.n1;
    std::vector<double> r(n), p(n), q(n);
    for (int e = 0; e < n; ++e) x[e] = 0.0;
    double bb = 0;
    for (int e = 0; e < n; ++e) { r[e] = m.efree[e] ? b[e] : 0.0; p[e] = r[e]; bb += r[e] * r[e]; }
    if (bb == 0.0) return 0;
    double rr = bb;
    int it = 0;
    for (; it < max_iter && rr > rtol * rtol * bb; ++it) {
        m.M.spmv(p.data(), q.data());
        double pq = 0;
        for (int e = 0; e < n; ++e) pq += p[e] * q[e];
        double a = rr / pq;
        double rn = 0;
        for (int e = 0; e < n; ++e) { x[e] += a * p[e]; r[e] -= a * q[e]; rn += r[e] * r[e]; }
        double beta = rn / rr;
        rr = rn;
        for (int e = 0; e < n; ++e) p[e] = r[e] + beta * p[e];
    }
    return it;
}

// ------------------------------------------------------------ absorbing layers
void build_layers(const HostMesh &m, double dt, const LayerConfig &cfg, HostLayers &L, Csr &K) {
    double z0 = 1e300, z1 = -1e300;
    for (int v = 0; v < m.n0; ++v) { z0 = std::min(z0, m.z[v]); z1 = std::max(z1, m.z[v]); }
    L = HostLayers{};
    K = m.A;
    for (int t = 0; t < m.n2; ++t) {
        const double zc = (m.z[m.tv[t][0]] + m.z[m.tv[t][1]] + m.z[m.tv[t][2]]) / 3.0;
        double sig = 0.0;
        if ((cfg.sides & 1) && zc < cfg.z_left && cfg.z_left > z0)
            sig = cfg.sigma_max * std::pow((cfg.z_left - zc) / (cfg.z_left - z0), cfg.order);
        if ((cfg.sides & 2) && zc > cfg.z_right && cfg.z_right < z1)
            sig = cfg.sigma_max * std::pow((zc - cfg.z_right) / (z1 - cfg.z_right), cfg.order);
        if (!(sig > 0.0)) continue;
        const double beta = sig * dt / (2.0 * kEps0);
        double Az[3][3], Ar[3][3];
        local_hodge(m, t, 0, Az);
        local_hodge(m, t, 1, Ar);
        L.face.push_back(t);
        L.beta.push_back(beta);
        for (int k = 0; k < 3; ++k)
            for (int l = 0; l < 3; ++l) {
                L.Az.push_back(Az[k][l]);
                L.Ar.push_back(Ar[k][l]);
                // stretched Hodge: (1 + beta) A_rho + A_z / (1 + beta) on the face
                const double dk = beta * Ar[k][l] + (1.0 / (1.0 + beta) - 1.0) * Az[k][l];
                const int32_t ek = m.tedge[t][k], el = m.tedge[t][l];
                const int32_t *b = K.col.data() + K.ptr[ek], *e = K.col.data() + K.ptr[ek + 1];
                const int32_t *it = std::lower_bound(b, e, el);
                K.val[it - K.col.data()] += dk;
            }
    }
}

// ------------------------------------------------------------ electrostatics
// The scheme's Gauss law (Sec. 3.5.2) holds for all steps if the initial
// state satisfies D~div D = Q on the free nodes with D = [*eps]_a E = M^-1 E.
// With E = -G phi = D~div^T phi the field is curl-free (C G = 0) and
// K phi = Q with K = D~div M^-1 D~div^T (free nodes; phi fixed on conductor
// nodes).  K is applied through a CG solve with M; it is solved by defect
// correction preconditioned with L = D~div A D~div^T (the rho-weighted P1
// stiffness, close to K since M approximates A^-1), L itself by Jacobi PCG.
namespace {

// E = D~div^T phi on every edge (phi_tail - phi_head), 0 on conductor edges
void grad_field(const HostMesh &m, const double *phi, double *E) {
    for (int e = 0; e < m.n1; ++e) E[e] = m.efree[e] ? phi[m.ev[e][0]] - phi[m.ev[e][1]] : 0.0;
}

// y_v = (D~div x)_v on the free nodes (0 elsewhere)
void node_div(const HostMesh &m, const double *x, double *y) {
    for (int v = 0; v < m.n0; ++v) {
        double s = 0.0;
        if (m.nfree[v])
            for (int64_t q = m.nptr[v]; q < m.nptr[v + 1]; ++q) s += m.nsign[q] * x[m.nedge[q]];
        y[v] = s;
    }
}

double a_entry(const Csr &A, int e, int f) {
    const int32_t *b = A.col.data() + A.ptr[e], *en = A.col.data() + A.ptr[e + 1];
    const int32_t *it = std::lower_bound(b, en, f);
    return (it != en && *it == f) ? A.val[it - A.col.data()] : 0.0;
}

}  // namespace

int electrostatic_state(const HostMesh &m, const double *phi_c, const double *Q, double rtol, int max_outer,
                        std::vector<double> &phi, std::vector<double> &E, std::vector<double> &D, double &res_rel) {
    const int n0 = m.n0, n1 = m.n1;
    phi.assign(n0, 0.0);
    E.assign(n1, 0.0);
    D.assign(n1, 0.0);
    for (int v = 0; v < n0; ++v) phi[v] = m.nfree[v] ? 0.0 : phi_c[v];
    // Jacobi preconditioner of L: diag(L)_v = sum_{e,f at v} s_ve s_vf A_ef
    std::vector<double> dl(n0, 1.0);
    for (int v = 0; v < n0; ++v) {
        if (!m.nfree[v]) continue;
        double s = 0.0;
        for (int64_t a = m.nptr[v]; a < m.nptr[v + 1]; ++a)
            for (int64_t b = m.nptr[v]; b < m.nptr[v + 1]; ++b)
                s += m.nsign[a] * m.nsign[b] * a_entry(m.A, m.nedge[a], m.nedge[b]);
        dl[v] = s > 0.0 ? s : 1.0;
    }
    std::vector<double> te(n1), ta(n1), r(n0), x(n0), z(n0), p(n0), q(n0), dphi(n0);
    auto apply_L = [&](const double *in, double *out) {
        grad_field(m, in, te.data());
        m.A.spmv(te.data(), ta.data());
        node_div(m, ta.data(), out);
    };
    // Jacobi PCG for L x = b on the free nodes (x, b zero elsewhere)
    auto solve_L = [&](const double *b, double *xo, double tol) {
        double bb = 0.0;
        for (int v = 0; v < n0; ++v) { xo[v] = 0.0; r[v] = m.nfree[v] ? b[v] : 0.0; bb += r[v] * r[v]; }
        if (bb == 0.0) return;
        double rz = 0.0;
        for (int v = 0; v < n0; ++v) { z[v] = r[v] / dl[v]; p[v] = z[v]; rz += r[v] * z[v]; }
        for (int it = 0; it < 20 * n0 + 100; ++it) {
            apply_L(p.data(), q.data());
            double pq = 0.0;
            for (int v = 0; v < n0; ++v) pq += p[v] * q[v];
            if (!(pq > 0.0)) break;
            const double a = rz / pq;
            double rr = 0.0;
            for (int v = 0; v < n0; ++v) { xo[v] += a * p[v]; r[v] -= a * q[v]; rr += r[v] * r[v]; }
            if (rr <= tol * tol * bb) break;
            double rzn = 0.0;
            for (int v = 0; v < n0; ++v) { z[v] = r[v] / dl[v]; rzn += r[v] * z[v]; }
            const double beta = rzn / rz;
            rz = rzn;
            for (int v = 0; v < n0; ++v) p[v] = z[v] + beta * p[v];
        }
    };
    res_rel = 1e300;
    for (int outer = 0; outer < max_outer; ++outer) {
        grad_field(m, phi.data(), E.data());
        cg_solve_M(m, E.data(), D.data(), 1e-15, 20000);
        node_div(m, D.data(), x.data());
        double rmax = 0.0, scale = 0.0;
        for (int v = 0; v < n0; ++v) {
            if (!m.nfree[v]) continue;
            double sa = 0.0;                        // summed |D| at the node: the scale of its residual
            for (int64_t k = m.nptr[v]; k < m.nptr[v + 1]; ++k) sa += std::fabs(D[m.nedge[k]]);
            x[v] = Q[v] - x[v];
            rmax = std::max(rmax, std::fabs(x[v]));
            scale = std::max(scale, std::max(std::fabs(Q[v]), sa));
        }
        res_rel = scale > 0.0 ? rmax / scale : 0.0;
        if (res_rel <= rtol) return outer;
        std::vector<double> rhs(x.begin(), x.end());
        solve_L(rhs.data(), dphi.data(), 1e-10);
        for (int v = 0; v < n0; ++v)
            if (m.nfree[v]) phi[v] += dphi[v];
    }
    return -1;
}

void build_locator(HostMesh &m) {
    double zmin = 1e300, zmax = -1e300, rmin = 1e300, rmax = -1e300;
    for (int i = 0; i < m.n0; ++i) {
        zmin = std::min(zmin, m.z[i]); zmax = std::max(zmax, m.z[i]);
        rmin = std::min(rmin, m.r[i]); rmax = std::max(rmax, m.r[i]);
    }
    double area = (zmax - zmin) * (rmax - rmin);
    double cell = std::sqrt(std::max(area, 1e-300) / std::max(1, m.n2) * 2.0);
    m.gnz = std::max(1, int((zmax - zmin) / cell) + 1);
    m.gnr = std::max(1, int((rmax - rmin) / cell) + 1);
    m.gz0 = zmin; m.gr0 = rmin;
    m.ghz = (zmax - zmin) / m.gnz + 1e-300;
    m.ghr = (rmax - rmin) / m.gnr + 1e-300;
    std::vector<std::vector<int32_t>> cells(size_t(m.gnz) * m.gnr);
    for (int t = 0; t < m.n2; ++t) {
        double z0 = 1e300, z1 = -1e300, r0 = 1e300, r1 = -1e300;
        for (int k = 0; k < 3; ++k) {
            z0 = std::min(z0, m.z[m.tv[t][k]]); z1 = std::max(z1, m.z[m.tv[t][k]]);
            r0 = std::min(r0, m.r[m.tv[t][k]]); r1 = std::max(r1, m.r[m.tv[t][k]]);
        }
        int iz0 = std::max(0, int((z0 - m.gz0) / m.ghz)), iz1 = std::min(m.gnz - 1, int((z1 - m.gz0) / m.ghz));
        int ir0 = std::max(0, int((r0 - m.gr0) / m.ghr)), ir1 = std::min(m.gnr - 1, int((r1 - m.gr0) / m.ghr));
        for (int a = iz0; a <= iz1; ++a)
            for (int b = ir0; b <= ir1; ++b) cells[size_t(a) * m.gnr + b].push_back(t);
    }
    m.gptr.assign(cells.size() + 1, 0);
    for (size_t c = 0; c < cells.size(); ++c) m.gptr[c + 1] = m.gptr[c] + int32_t(cells[c].size());
    m.gtri.resize(m.gptr.back());
    for (size_t c = 0; c < cells.size(); ++c) std::copy(cells[c].begin(), cells[c].end(), m.gtri.begin() + m.gptr[c]);
}

int32_t locate_point(const HostMesh &m, double z, double rho, double lam[3]) {
    int iz = int((z - m.gz0) / m.ghz), ir = int((rho - m.gr0) / m.ghr);
    int best = -1;
    double bestv = -1e300, bl[3] = {0, 0, 0};
    for (int a = std::max(0, iz - 1); a <= std::min(m.gnz - 1, iz + 1); ++a)
        for (int b = std::max(0, ir - 1); b <= std::min(m.gnr - 1, ir + 1); ++b) {
            size_t c = size_t(a) * m.gnr + b;
            for (int32_t q = m.gptr[c]; q < m.gptr[c + 1]; ++q) {
                int t = m.gtri[q];
                double l[3];
                for (int k = 0; k < 3; ++k) {
                    int j = (k + 1) % 3, n = (k + 2) % 3;
                    double zj = m.z[m.tv[t][j]], rj = m.r[m.tv[t][j]], zn = m.z[m.tv[t][n]], rn = m.r[m.tv[t][n]];
                    l[k] = 0.5 * ((zj - z) * (rn - rho) - (zn - z) * (rj - rho)) / m.area[t];
                }
                double mn = std::min(l[0], std::min(l[1], l[2]));
                if (mn > bestv) { bestv = mn; best = t; bl[0] = l[0]; bl[1] = l[1]; bl[2] = l[2]; }
            }
        }
    if (best < 0 || bestv < -1e-9) return -1;
    for (int k = 0; k < 3; ++k) lam[k] = bl[k];
    return best;
}

}  // namespace axp
