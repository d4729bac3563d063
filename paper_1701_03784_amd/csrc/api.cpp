// C ABI of the library (include/axpic.h): context lifecycle, setup uploads,
// the step loop, diagnostics and read-back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "../../include/axpic.h"
#include "device.h"
#include "host_setup.h"

using namespace axp;

namespace axp {
int mlp_predict_host(axp_mlp *net, const float *X, int64_t n, float *y, std::string &err);
int mlp_level(const axp_mlp *net);
int mlp_n_in(const axp_mlp *net);
}  // namespace axp

struct Species {
    double q, m;
    int64_t w;
};

struct axp_ctx {
    axp_config cfg{};
    std::string err;
    int sticky = 0;
    bool has_mesh = false, has_bnd = false, built = false;
    std::vector<double> in_zr;
    std::vector<int32_t> in_tri, in_seg;
    std::vector<uint8_t> in_tag;
    HostMesh hm;
    double dt = 0, dt_cfl = 0, setup_s = 0;
    hipStream_t stream = nullptr;
    DevMesh dm{};
    DevState ds{};
    InstConst ic{};
    bool plain = false;   // FP64 step (AXP_PREC_PLAIN_FP64)
    DevPlain dp{};
    PlainConst pc{};
    std::vector<void *> allocs;
    std::vector<Species> species;
    double q_unit = 0;
    int64_t step = 0;
    int64_t last_eval_level = -1;  // time level of the last diagnostic evaluation enqueued (-1: none)
    bool final_pending = false;    // a diagnostic step's final reduction waits for the next face pass
    int64_t energy_read = 0;       // energy records already returned by axp_get_energies
    bool q32 = true;               // every species' charge multiple is 0 or 1 (all members of a pool)
    int win_lead = 192;            // accumulation window lead of the particle kernel (tuning knob)
    uint64_t shape_hash = 0;       // mesh identity for the autotune cache (a pool: its members')
    int64_t n_live_host = 0;
    // continuous injector
    bool inj_on = false;
    axp_mlp *owned_model = nullptr;     // network loaded by axp_spai_model_load
    InjParams inj{};
    EmitEdge *inj_edges = nullptr;
    // per-phase timing
    bool timing = false;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev;   // pending (phase, start, stop)
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_free;
    double phase_ms[AXP_N_PHASES] = {0};
    int64_t phase_n[AXP_N_PHASES] = {0};
    // learned SPAI
    axp_mlp *spai_model = nullptr;      // borrowed
    double spai_row_tol = 0.01, spai_energy_tol = 1e-6;
    int spai_iters = 3;
    int spai_mode_used = AXP_SPAI_PLAIN;
    LearnedSpaiStats spai_stats;
    double spai_energy_drift = 0, spai_seconds = 0;
    double spai_feature_s = 0, spai_infer_s = 0, spai_solve_s = 0;
    // run-time energy guard of the learned SPAI (axp_set_spai_run_guard)
    double guard_tol = -1.0;            // < 0: off
    bool guard_ref_set = false;
    double guard_wref = 0.0, guard_drift = 0.0;
    int64_t guard_trip_step = -1;
    void *snap = nullptr;               // device copy of the state at the last checkpoint
    size_t snap_bytes = 0;
    // step graphs (one per particle buffer), replayed on stream
    hipStream_t cap_stream = nullptr;
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    int graph_window = 0;
    // stretched-coordinate absorbing layers
    LayerConfig layer_cfg{};
    HostLayers hl{};
    DevLayers dl{};
    // magnetic point sources and field probe (Sec. 4.1)
    FieldSrc fs{};
    unsigned long long step_upload = 0;   // host image of the device step counter (async copy source)
};

namespace {

uint64_t mesh_hash(const axp_ctx *c);

struct ApiError {
    int code;
    std::string msg;
};

void *dalloc(axp_ctx *c, size_t bytes) {
    if (bytes == 0) bytes = 256;
    void *p = nullptr;
    if (c->cfg.alloc) {
        p = c->cfg.alloc(bytes, c->cfg.alloc_user);
        if (!p) throw ApiError{AXP_E_OOM, "device allocation callback failed"};
    } else {
        if (hipMalloc(&p, bytes) != hipSuccess) throw ApiError{AXP_E_OOM, "hipMalloc failed"};
    }
    c->allocs.push_back(p);
    return p;
}

void dfree(axp_ctx *c, void *p) {
    if (!p) return;
    auto it = std::find(c->allocs.begin(), c->allocs.end(), p);
    if (it != c->allocs.end()) c->allocs.erase(it);
    if (c->cfg.free) c->cfg.free(p, c->cfg.alloc_user);
    else (void)hipFree(p);
}

void hcheck(hipError_t e, const char *what) {
    if (e != hipSuccess) throw ApiError{AXP_E_HIP, std::string(what) + ": " + hipGetErrorString(e)};
}

template <class T>
T *upload(axp_ctx *c, const std::vector<T> &v) {
    T *p = (T *)dalloc(c, v.size() * sizeof(T));
    if (!v.empty()) hcheck(hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, c->stream), "upload");
    return p;
}

template <class T>
T *zeros(axp_ctx *c, size_t n) {
    T *p = (T *)dalloc(c, n * sizeof(T));
    hcheck(hipMemsetAsync(p, 0, n * sizeof(T), c->stream), "memset");
    return p;
}

axp_status fail(axp_ctx *c, int code, const std::string &msg) {
    if (c) c->err = msg;
    return code;
}

template <class F>
axp_status guarded(axp_ctx *c, F &&body) {
    try {
        return body();
    } catch (const ApiError &e) {
        if (e.code == AXP_E_HIP) c->sticky = AXP_E_HIP;
        return fail(c, e.code, e.msg);
    } catch (const SetupError &e) {
        return fail(c, e.code, e.msg);
    } catch (const std::bad_alloc &) {
        return fail(c, AXP_E_OOM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(c, AXP_E_ARG, e.what());
    }
}

void require_built(axp_ctx *c) {
    if (c->sticky) throw ApiError{AXP_E_STATE, "a sticky error was raised earlier: " + c->err};
    if (!c->built) throw ApiError{AXP_E_STATE, "axp_build has not been called"};
}

void upload_inst(axp_ctx *c) {
    hcheck(hipMemcpyAsync((void *)c->dm.inst, &c->ic, sizeof(InstConst), hipMemcpyHostToDevice, c->stream), "inst");
}

DevCounters read_counters(axp_ctx *c) {
    DevCounters h{};
    hcheck(hipMemcpyAsync(&h, c->ds.ctr, sizeof(h), hipMemcpyDeviceToHost, c->stream), "counters");
    hcheck(hipStreamSynchronize(c->stream), "sync");
    return h;
}

void drop_graphs(axp_ctx *c);

void grow_particles(axp_ctx *c, int64_t need) {
    DevState &s = c->ds;
    if (need <= s.capacity) return;
    drop_graphs(c);   // kernel arguments change
    int64_t cap = std::max<int64_t>(need, s.capacity + s.capacity / 2);
    cap = (cap + 1023) / 1024 * 1024;
    DevCounters h = read_counters(c);
    int64_t used = (int64_t)h.n_slots;
    if (c->plain) {
        DevPlain &p = c->dp;
        for (int b = 0; b < 2; ++b) {
            int32_t *cell = zeros<int32_t>(c, cap);
            double *f[5];
            double **old[5] = {&p.l0[b], &p.l1[b], &p.ur[b], &p.up[b], &p.uz[b]};
            for (int k = 0; k < 5; ++k) f[k] = zeros<double>(c, cap);
            if (b == s.cur && used > 0) {
                hcheck(hipMemcpyAsync(cell, s.cell[b], used * 4, hipMemcpyDeviceToDevice, c->stream), "copy");
                for (int k = 0; k < 5; ++k)
                    hcheck(hipMemcpyAsync(f[k], *old[k], used * 8, hipMemcpyDeviceToDevice, c->stream), "copy");
            }
            hcheck(hipStreamSynchronize(c->stream), "sync");
            dfree(c, s.cell[b]);
            s.cell[b] = cell;
            for (int k = 0; k < 5; ++k) { dfree(c, *old[k]); *old[k] = f[k]; }
        }
        s.capacity = cap;
        dfree(c, s.part_kin);
        s.part_kin = zeros<double>(c, size_t(3) * ((cap + 1023) / 1024));
        return;
    }
    for (int b = 0; b < 2; ++b) {
        int32_t *cell = zeros<int32_t>(c, cap);
        uint32_t *l0 = zeros<uint32_t>(c, cap), *l1 = zeros<uint32_t>(c, cap);
        float *ur = zeros<float>(c, cap), *up = zeros<float>(c, cap), *uz = zeros<float>(c, cap);
        if (b == s.cur && used > 0) {
            hcheck(hipMemcpyAsync(cell, s.cell[b], used * 4, hipMemcpyDeviceToDevice, c->stream), "copy");
            hcheck(hipMemcpyAsync(l0, s.L0[b], used * 4, hipMemcpyDeviceToDevice, c->stream), "copy");
            hcheck(hipMemcpyAsync(l1, s.L1[b], used * 4, hipMemcpyDeviceToDevice, c->stream), "copy");
            hcheck(hipMemcpyAsync(ur, s.ur[b], used * 4, hipMemcpyDeviceToDevice, c->stream), "copy");
            hcheck(hipMemcpyAsync(up, s.up[b], used * 4, hipMemcpyDeviceToDevice, c->stream), "copy");
            hcheck(hipMemcpyAsync(uz, s.uz[b], used * 4, hipMemcpyDeviceToDevice, c->stream), "copy");
        }
        hcheck(hipStreamSynchronize(c->stream), "sync");
        dfree(c, s.cell[b]); dfree(c, s.L0[b]); dfree(c, s.L1[b]);
        dfree(c, s.ur[b]); dfree(c, s.up[b]); dfree(c, s.uz[b]);
        s.cell[b] = cell; s.L0[b] = l0; s.L1[b] = l1; s.ur[b] = ur; s.up[b] = up; s.uz[b] = uz;
    }
    s.capacity = cap;
    dfree(c, s.part_kin);
    s.part_kin = zeros<double>(c, size_t(3) * ((cap + 1023) / 1024));
}

// Brackets one phase's launches with HIP events on stream st (eager steps).
struct PhaseScope {
    axp_ctx *c;
    int phase;
    hipStream_t st;
    hipEvent_t b = nullptr, e = nullptr;
    PhaseScope(axp_ctx *ctx, int ph, hipStream_t stream) : c(ctx), phase(ph), st(stream) {
        if (!c->timing) return;
        if (!c->ev_free.empty()) {
            b = c->ev_free.back().first;
            e = c->ev_free.back().second;
            c->ev_free.pop_back();
        } else {
            hcheck(hipEventCreate(&b), "event");
            hcheck(hipEventCreate(&e), "event");
        }
        hcheck(hipEventRecord(b, st), "event record");
    }
    PhaseScope(axp_ctx *ctx, int ph) : PhaseScope(ctx, ph, ctx->stream) {}
    ~PhaseScope() {
        if (!c->timing || !b) return;
        (void)hipEventRecord(e, st);
        c->ev.push_back({phase, {b, e}});
    }
};

void collect_timing(axp_ctx *c) {
    if (c->ev.empty()) return;
    hcheck(hipStreamSynchronize(c->stream), "sync");
    for (auto &r : c->ev) {
        float ms = 0.f;
        hcheck(hipEventElapsedTime(&ms, r.second.first, r.second.second), "elapsed");
        c->phase_ms[r.first] += ms;
        c->phase_n[r.first] += 1;
        c->ev_free.push_back(r.second);
    }
    c->ev.clear();
}

// Diagnostic evaluation of the current state (level = steps taken), on demand.
void run_diag(axp_ctx *c) {
    {
        PhaseScope ps(c, AXP_PHASE_DIAG);
        if (c->plain) {
            launch_charge_plain(c->dm, c->ds, c->dp, c->pc, c->stream);
            launch_diag_plain(c->dm, c->ds, c->dp, c->pc, false, c->stream);
        } else {
            launch_diag_now(c->dm, c->ds, c->stream);
        }
    }
    c->last_eval_level = c->step;
}

// Restarts the diagnostics' references: g0 (the Gauss residual's reference
// level) when reset_gauss, and always the continuity chain (the next
// evaluation has no previous level to compare with).  Host-to-device copies:
// never inside a graph.
void reset_diag_refs(axp_ctx *c, bool reset_gauss) {
    DevCounters h = read_counters(c);
    h.diag_level1 = 0;
    if (reset_gauss) h.g0_set = 0;
    hcheck(hipMemcpyAsync(c->ds.ctr, &h, sizeof(h), hipMemcpyHostToDevice, c->stream), "counters");
    if (reset_gauss) {
        DevDiag d{};
        hcheck(hipMemcpyAsync(&d, c->ds.diag, sizeof(d), hipMemcpyDeviceToHost, c->stream), "diag");
        hcheck(hipStreamSynchronize(c->stream), "sync");
        d.gauss_drift_max_bits = 0;
        d.dce_max = 0;
        d.dce_rel_max_bits = 0;
        d.n_evals = 0;
        hcheck(hipMemcpyAsync(c->ds.diag, &d, sizeof(d), hipMemcpyHostToDevice, c->stream), "diag");
    }
    hcheck(hipStreamSynchronize(c->stream), "sync");
    c->last_eval_level = -1;
}

// Host images of the device tables of one instance or of a pool of them.
struct HostTables {
    std::vector<float4> gS, rho4;
    std::vector<int4> nbr, tedge, tnodes, etri;
    std::vector<double> Hdt;
    std::vector<int32_t> tinst, ninst;
    std::vector<int32_t> nptr{0}, nedge;
    std::vector<int32_t> ncptr{0}, ncorner;   // face corners 3 t + k at each node
    std::vector<int8_t> nsign;
    std::vector<uint8_t> nfree;
    Csr M, A;   // pooled rows, column indices offset per instance
    int32_t n0 = 0, n1 = 0, n2 = 0;
};

// Appends one instance (faces, edges and nodes offset by the current sizes).
void append_instance(HostTables &h, const HostMesh &m, double dt, int inst) {
    const int32_t fo = h.n2, eo = h.n1, no = h.n0;
    const double S = double(kLamOne);
    for (int t = 0; t < m.n2; ++t) {
        const auto &g = m.grad[t];
        h.gS.push_back(make_float4(float(S * g[0]), float(S * g[1]), float(S * g[2]), float(S * g[3])));
        h.rho4.push_back(make_float4(float(m.r[m.tv[t][0]]), float(m.r[m.tv[t][1]]), float(m.r[m.tv[t][2]]),
                                     float(1.0 / (2.0 * m.area[t]))));
        int nb[3];
        for (int k = 0; k < 3; ++k) nb[k] = m.tnbr[t][k] >= 0 ? m.tnbr[t][k] + fo : m.tnbr[t][k];
        h.nbr.push_back(make_int4(nb[0], nb[1], nb[2], int(m.tnbr_map[t])));
        int sb = 0;
        for (int k = 0; k < 3; ++k) if (m.tsign[t][k] < 0) sb |= 1 << k;
        h.tedge.push_back(make_int4(m.tedge[t][0] + eo, m.tedge[t][1] + eo, m.tedge[t][2] + eo, sb));
        h.tnodes.push_back(make_int4(m.tv[t][0] + no, m.tv[t][1] + no, m.tv[t][2] + no, 0));
        h.Hdt.push_back(dt * m.H[t]);
        h.tinst.push_back(inst);
    }
    for (int e = 0; e < m.n1; ++e) {
        int L = m.etri[e][0], R = m.etri[e][1];
        int kl = m.eside[e][0], kr = R >= 0 ? m.eside[e][1] : 0;
        int packed = kl | (kr << 2);
        if (m.tsign[L][kl] < 0) packed |= 16;
        if (R >= 0 && m.tsign[R][kr] < 0) packed |= 32;
        if (m.efree[e]) packed |= 64;
        h.etri.push_back(make_int4(L + fo, R >= 0 ? R + fo : -1, packed, inst));
    }
    {
        std::vector<int32_t> cnt(size_t(m.n0) + 1, 0), fill;
        for (int t = 0; t < m.n2; ++t)
            for (int k = 0; k < 3; ++k) ++cnt[m.tv[t][k] + 1];
        for (int v = 0; v < m.n0; ++v) cnt[v + 1] += cnt[v];
        fill.assign(cnt.begin(), cnt.end() - 1);
        std::vector<int32_t> corner(size_t(3) * m.n2);
        for (int t = 0; t < m.n2; ++t)
            for (int k = 0; k < 3; ++k) corner[fill[m.tv[t][k]]++] = 3 * (t + fo) + k;
        const int32_t base = int32_t(h.ncorner.size());
        for (int v = 0; v < m.n0; ++v) h.ncptr.push_back(base + cnt[v + 1]);
        h.ncorner.insert(h.ncorner.end(), corner.begin(), corner.end());
    }
    for (int v = 0; v < m.n0; ++v) {
        for (int q = m.nptr[v]; q < m.nptr[v + 1]; ++q) {
            h.nedge.push_back(m.nedge[q] + eo);
            h.nsign.push_back(m.nsign[q]);
        }
        h.nptr.push_back(int32_t(h.nedge.size()));
        h.nfree.push_back(m.nfree[v]);
        h.ninst.push_back(inst);
    }
    auto app = [&](Csr &dst, const Csr &src) {
        if (dst.ptr.empty()) dst.ptr.push_back(0);
        for (int64_t i = 0; i < src.n; ++i) {
            for (int64_t q = src.ptr[i]; q < src.ptr[i + 1]; ++q) {
                dst.col.push_back(src.col[q] + eo);
                dst.val.push_back(src.val[q]);
            }
            dst.ptr.push_back(int64_t(dst.col.size()));
        }
        dst.n += src.n;
    };
    app(h.M, m.M);
    app(h.A, m.A);
    h.n0 += m.n0; h.n1 += m.n1; h.n2 += m.n2;
}

// Sliced ELL of a CSR matrix: slices of 64 rows, column-major in a slice,
// padded with zero values on the row's own column.
void build_sell(const Csr &M, int32_t n1, std::vector<int64_t> &sptr, std::vector<int32_t> &slen,
                std::vector<float> &mval, std::vector<double> *mvald, std::vector<int32_t> &mcol) {
    const int ns = (n1 + 63) / 64;
    sptr.assign(ns + 1, 0);
    slen.assign(ns, 0);
    for (int sl = 0; sl < ns; ++sl) {
        int mx = 0;
        for (int i = sl * 64; i < std::min(n1, sl * 64 + 64); ++i) mx = std::max<int>(mx, int(M.ptr[i + 1] - M.ptr[i]));
        slen[sl] = mx;
        sptr[sl + 1] = sptr[sl] + int64_t(mx) * 64;
    }
    mval.assign(sptr[ns], 0.0f);
    if (mvald) mvald->assign(sptr[ns], 0.0);
    mcol.assign(sptr[ns], 0);
    for (int sl = 0; sl < ns; ++sl)
        for (int lane = 0; lane < 64; ++lane) {
            int i = sl * 64 + lane;
            int64_t o = sptr[sl] + lane;
            int j = 0;
            if (i < n1)
                for (int64_t q = M.ptr[i]; q < M.ptr[i + 1]; ++q, ++j) {
                    mval[o + 64 * j] = float(M.val[q]);
                    if (mvald) (*mvald)[o + 64 * j] = M.val[q];
                    mcol[o + 64 * j] = M.col[q];
                }
            for (; j < slen[sl]; ++j) mcol[o + 64 * j] = i < n1 ? i : 0;
        }
}

// The node lists of h as column-major slices of 64 nodes, each list padded to
// the longest of the mesh (the node pass loads all of a node's entries at once).
void build_node_ell(const HostTables &h, std::vector<int32_t> &corner, int32_t &wc, std::vector<int32_t> &edge,
                    int32_t &we) {
    wc = we = 0;
    for (int v = 0; v < h.n0; ++v) {
        wc = std::max(wc, h.ncptr[v + 1] - h.ncptr[v]);
        we = std::max(we, h.nptr[v + 1] - h.nptr[v]);
    }
    const size_t ns = (size_t(h.n0) + 63) / 64;
    corner.assign(ns * size_t(wc) * 64, -1);
    edge.assign(ns * size_t(we) * 64, 0);
    for (int v = 0; v < h.n0; ++v) {
        const size_t sl = size_t(v) / 64, l = size_t(v) % 64;
        for (int32_t j = 0; j < h.ncptr[v + 1] - h.ncptr[v]; ++j)
            corner[(sl * wc + j) * 64 + l] = h.ncorner[h.ncptr[v] + j];
        for (int32_t j = 0; j < h.nptr[v + 1] - h.nptr[v]; ++j) {
            const int32_t q = h.nptr[v] + j;
            edge[(sl * we + j) * 64 + l] = h.nsign[q] > 0 ? h.nedge[q] + 1 : -(h.nedge[q] + 1);
        }
    }
}

// Uploads the tables and allocates the field state of a context (one
// instance: pooled = false; a batch pool: per-face / per-node instance ids).
void upload_tables(axp_ctx *c, const HostTables &h, bool pooled, int n_inst) {
    DevMesh &d = c->dm;
    d.n0 = h.n0; d.n1 = h.n1; d.n2 = h.n2; d.n_inst = n_inst;
    std::vector<int64_t> sptr;
    std::vector<int32_t> slen, mcol;
    std::vector<float> mval;
    std::vector<double> mvald;
    build_sell(h.M, h.n1, sptr, slen, mval, c->plain ? &mvald : nullptr, mcol);
    d.gS = upload(c, h.gS); d.rho4 = upload(c, h.rho4); d.nbr = upload(c, h.nbr);
    d.tedge = upload(c, h.tedge); d.tnodes = upload(c, h.tnodes); d.Hdt = upload(c, h.Hdt);
    d.tinst = pooled ? upload(c, h.tinst) : nullptr;
    d.etri = upload(c, h.etri);
    d.nptr = upload(c, h.nptr); d.nedge = upload(c, h.nedge); d.nsign = upload(c, h.nsign);
    d.nfree = upload(c, h.nfree); d.ninst = pooled ? upload(c, h.ninst) : nullptr;
    d.ncptr = upload(c, h.ncptr); d.ncorner = upload(c, h.ncorner);
    {
        std::vector<int32_t> ce, ee;
        build_node_ell(h, ce, d.nwc, ee, d.nwe);
        d.ncorner_ell = upload(c, ce); d.nedge_ell = upload(c, ee);
    }
    d.m_sptr = upload(c, sptr); d.m_slen = upload(c, slen); d.m_col = upload(c, mcol);
    d.m_val = c->plain ? nullptr : upload(c, mval);
    d.a_ptr = upload(c, h.A.ptr); d.a_col = upload(c, h.A.col); d.a_val = upload(c, h.A.val);
    d.inst = (InstConst *)dalloc(c, sizeof(InstConst) * size_t(n_inst));
    DevState &s = c->ds;
    s.B = zeros<double>(c, h.n2); s.Bprev = zeros<double>(c, h.n2); s.HBdt = zeros<double>(c, h.n2);
    s.D = zeros<double>(c, h.n1);
    s.g0 = zeros<double>(c, h.n0);
    if (c->plain) {
        DevPlain &p = c->dp;
        p.m_val = upload(c, mvald);
        p.E = zeros<double>(c, h.n1);
        p.f0 = zeros<double4>(c, h.n2); p.f1 = zeros<double4>(c, h.n2);
        p.Jloc = zeros<double>(c, size_t(3) * h.n2); p.Jfx = zeros<double>(c, h.n1);
        p.Qres = zeros<double>(c, h.n0); p.Q = zeros<double>(c, h.n0); p.Qprev = zeros<double>(c, h.n0);
    } else {
        s.f0 = zeros<float4>(c, h.n2); s.f1 = zeros<float4>(c, h.n2);
        s.Jloc = zeros<unsigned long long>(c, size_t(3) * h.n2);
        s.D32 = zeros<float>(c, h.n1); s.E = zeros<float>(c, h.n1);
        s.Jfx = zeros<long long>(c, h.n1);
        s.Qres = zeros<long long>(c, h.n0); s.Qfx = zeros<long long>(c, h.n0); s.Qprev = zeros<long long>(c, h.n0);
        s.Qloc = zeros<unsigned long long>(c, size_t(3) * h.n2);
    }
    s.cnt = zeros<int32_t>(c, size_t(h.n2) + 1);
    s.blk = zeros<int32_t>(c, size_t(h.n2) / 1024 + 2);
    s.ctr = zeros<DevCounters>(c, 1);
    s.diag = zeros<DevDiag>(c, 1);
    {
        DevDiag d{};
        d.level = -1;
        d.dce_last = -1;
        d.energy.level = -1;
        hcheck(hipMemcpyAsync(s.diag, &d, sizeof(d), hipMemcpyHostToDevice, c->stream), "diag");
        hcheck(hipStreamSynchronize(c->stream), "sync");
    }
    s.part_face = zeros<double>(c, (size_t(h.n2) + 255) / 256);
    s.part_edge = zeros<double>(c, (size_t(h.n1) + 255) / 256);
    s.part_node = zeros<double>(c, size_t(kDiagSlots) * ((size_t(std::max(h.n0, h.n1)) + 255) / 256));
    s.part_kin = zeros<double>(c, 3);
    s.part_wenow = zeros<double>(c, (size_t(h.n1) + 255) / 256);
    s.energy = zeros<DevEnergy>(c, kEnergyRing);
    s.capacity = 0;
    s.cur = 0;
}

void build_device(axp_ctx *c) {
    const HostMesh &m = c->hm;
    HostTables h;
    append_instance(h, m, c->dt, 0);
    upload_tables(c, h, false, 1);
    if (c->plain) {
        DevPlain &p = c->dp;
        std::vector<double4> grad(m.n2), rho(m.n2);
        for (int t = 0; t < m.n2; ++t) {
            const auto &g = m.grad[t];
            grad[t] = make_double4(g[0], g[1], g[2], g[3]);
            rho[t] = make_double4(m.r[m.tv[t][0]], m.r[m.tv[t][1]], m.r[m.tv[t][2]], 1.0 / (2.0 * m.area[t]));
        }
        p.grad = upload(c, grad); p.rho = upload(c, rho);
        std::memset(&c->pc, 0, sizeof(PlainConst));
        c->pc.dt = c->dt;
        c->pc.cdt = kC * c->dt;
    }
    std::memset(&c->ic, 0, sizeof(InstConst));
    c->ic.dt = c->dt;
    c->ic.cdt = float(kC * c->dt);
    upload_inst(c);
    const HostLayers &L = c->hl;
    std::vector<int32_t> face_layer;
    std::vector<double> Hf;
    std::vector<int4> ledges;
    if (!L.face.empty()) {
        const int nl = int(L.face.size());
        face_layer.assign(m.n2, -1);
        Hf.resize(nl);
        std::vector<int4> byedge(m.n1, make_int4(-1, -1, -1, 0));
        for (int i = 0; i < nl; ++i) {
            const int t = L.face[i];
            face_layer[t] = i;
            Hf[i] = m.H[t];
            for (int k = 0; k < 3; ++k) {
                int4 &r = byedge[m.tedge[t][k]];
                if (r.y < 0) r.y = 4 * i + k;
                else r.z = 4 * i + k;
            }
        }
        for (int e = 0; e < m.n1; ++e)
            if (byedge[e].y >= 0) ledges.push_back(make_int4(e, byedge[e].y, byedge[e].z, 0));
        DevLayers &d = c->dl;
        d.n = nl;
        d.n_edges = int32_t(ledges.size());
        d.face = upload(c, L.face);
        d.face_layer = upload(c, face_layer);
        d.beta = upload(c, L.beta);
        d.Hf = upload(c, Hf);
        d.Az = upload(c, L.Az);
        d.Ar = upload(c, L.Ar);
        d.h = zeros<double>(c, nl);
        d.q = zeros<double>(c, size_t(3) * nl);
        d.eprev = zeros<double>(c, size_t(3) * nl);
        d.corr = zeros<double>(c, size_t(3) * nl);
        d.edges = upload(c, ledges);
    }
    hcheck(hipStreamSynchronize(c->stream), "build sync");
}

// Layer state of fields at rest (E, B in internal order): h = H B, eprev = e,
// q = A_z e on each layer face.
void layers_at_rest(axp_ctx *c, const std::vector<double> &E, const std::vector<double> &B) {
    const HostLayers &L = c->hl;
    const int nl = int(L.face.size());
    if (nl == 0) return;
    const HostMesh &m = c->hm;
    std::vector<double> h(nl), q(size_t(3) * nl), ep(size_t(3) * nl);
    for (int i = 0; i < nl; ++i) {
        const int t = L.face[i];
        h[i] = m.H[t] * B[t];
        double e[3];
        for (int k = 0; k < 3; ++k) e[k] = ep[3 * i + k] = E[m.tedge[t][k]];
        for (int k = 0; k < 3; ++k)
            q[3 * i + k] = L.Az[9 * i + 3 * k] * e[0] + L.Az[9 * i + 3 * k + 1] * e[1] + L.Az[9 * i + 3 * k + 2] * e[2];
    }
    hcheck(hipMemcpyAsync(c->dl.h, h.data(), sizeof(double) * nl, hipMemcpyHostToDevice, c->stream), "layer h");
    hcheck(hipMemcpyAsync(c->dl.q, q.data(), sizeof(double) * 3 * nl, hipMemcpyHostToDevice, c->stream), "layer q");
    hcheck(hipMemcpyAsync(c->dl.eprev, ep.data(), sizeof(double) * 3 * nl, hipMemcpyHostToDevice, c->stream),
           "layer e");
    hcheck(hipStreamSynchronize(c->stream), "sync");
}


// Whether the step from level n to n + 1 is a diagnostic step: it evaluates
// level n + 1 (a multiple of diag_every) and records the energies of level n.
bool diag_step(const axp_ctx *c, int64_t n) { return c->cfg.diag_every > 0 && (n + 1) % c->cfg.diag_every == 0; }

// One time step enqueued on st (c->stream unless a graph is being captured).
void enqueue_step(axp_ctx *c, hipStream_t st) {
    const bool sort_now = (c->step + 1) % c->cfg.sort_period == 0;
    const bool diag = diag_step(c, c->step);
    DevMesh &m = c->dm;
    DevState &s = c->ds;
    // the mixed step's emission rides in the face pass when it fits one block
    const bool emit_in_face = c->inj_on && !c->plain && emission_fits_face_pass(c->inj);
    if (c->inj_on && !emit_in_face) {
        PhaseScope ps(c, AXP_PHASE_INJECT, st);
        if (c->plain) launch_inject_plain(m, s, c->dp, c->inj_edges, c->inj, st);
        else launch_inject(m, s, c->inj_edges, c->inj, st);
    }
    if (c->plain) {
        { PhaseScope ps(c, AXP_PHASE_FACE, st); launch_tri_pass_plain(m, s, c->dp, c->pc, c->fs, c->dl, diag, st); }
        if (sort_now) { PhaseScope ps(c, AXP_PHASE_SORT, st); launch_sort_zero(m, s, st); }
        {
            PhaseScope ps(c, AXP_PHASE_PARTICLES, st);
            launch_particles_plain(m, s, c->dp, c->pc, c->cfg.max_walk, sort_now, c->cfg.pusher == AXP_PUSH_VAY, diag,
                                   st);
        }
        { PhaseScope ps(c, AXP_PHASE_EDGE, st); launch_edge_pass_plain(m, s, c->dp, c->pc, diag, st); }
        {
            PhaseScope ps(c, AXP_PHASE_SPMV, st);
            launch_spmv_plain(m, s, c->dp, st);
            launch_layers_post(m, s, (const double *)c->dp.E, c->dl, st);
        }
        if (diag) {
            PhaseScope ps(c, AXP_PHASE_DIAG, st);
            launch_charge_plain(m, s, c->dp, c->pc, st);
            launch_diag_plain(m, s, c->dp, c->pc, true, st);
        }
        ++c->step;
        if (diag) c->last_eval_level = c->step;
        if (sort_now) { PhaseScope ps(c, AXP_PHASE_SORT, st); launch_sort_plain(m, s, c->dp, true, st); }
        return;
    }
    const bool single = m.tinst == nullptr && c->ic.n_species == 1 && c->ic.kq[0] == 1;
    const InstConst *k0 = single ? &c->ic : nullptr;
    {
        PhaseScope ps(c, AXP_PHASE_FACE, st);
        launch_tri_pass(m, s, c->fs, c->dl, diag, c->inj_edges, emit_in_face ? &c->inj : nullptr, c->final_pending,
                        st);
        c->final_pending = false;
    }
    if (sort_now) { PhaseScope ps(c, AXP_PHASE_SORT, st); launch_sort_zero(m, s, st); }
    {
        PhaseScope ps(c, AXP_PHASE_PARTICLES, st);
        launch_particles(m, s, c->cfg.max_walk, sort_now, k0, c->cfg.pusher == AXP_PUSH_VAY, diag, c->q32, c->win_lead,
                         st);
    }
    { PhaseScope ps(c, AXP_PHASE_EDGE, st); launch_edge_pass(m, s, true, diag, st); }
    if (diag && !c->dl.n) {
        // one launch: E = M D beside the evaluation of the new level; its final
        // reduction rides in the next face pass (or flush_final)
        PhaseScope ps(c, AXP_PHASE_SPMV, st);
        launch_spmv_diag(m, s, st);
        c->final_pending = true;
    } else {
        {
            PhaseScope ps(c, AXP_PHASE_SPMV, st);
            launch_spmv(m, s, st);
            launch_layers_post(m, s, (const float *)s.E, c->dl, st);
        }
        if (diag) { PhaseScope ps(c, AXP_PHASE_DIAG, st); launch_diag_in_step(m, s, st); }
    }
    ++c->step;
    if (diag) c->last_eval_level = c->step;
    if (sort_now) { PhaseScope ps(c, AXP_PHASE_SORT, st); launch_sort(m, s, true, st); }
}

// The final reduction of the last diagnostic step, if no face pass has done it yet.
void flush_final(axp_ctx *c, hipStream_t st) {
    if (!c->final_pending) return;
    PhaseScope ps(c, AXP_PHASE_DIAG, st);
    launch_step_final(c->dm, c->ds, st);
    c->final_pending = false;
}

void drop_graphs(axp_ctx *c) {
    for (auto &g : c->gexec)
        if (g) { (void)hipGraphExecDestroy(g); g = nullptr; }
}

// Graph of 2 * sort_period steps starting at a step that is a multiple of
// the sort period: it holds exactly two sorts, so the particle buffer in use
// is the same before and after it, and one graph per buffer suffices.
void launch_graph(axp_ctx *c, int W) {
    const int cur0 = c->ds.cur;
    if (!c->gexec[cur0]) {
        if (!c->cap_stream) hcheck(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking), "capture stream");
        const DevState saved = c->ds;
        const int64_t saved_step = c->step, saved_eval = c->last_eval_level;
        const bool saved_pending = c->final_pending;
        hcheck(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
        for (int k = 0; k < W; ++k) enqueue_step(c, c->cap_stream);
        flush_final(c, c->cap_stream);   // the window leaves no reduction pending
        hipGraph_t g = nullptr;
        const hipError_t e1 = hipStreamEndCapture(c->cap_stream, &g);
        c->ds = saved;              // the captured launches have not run
        c->step = saved_step;
        c->last_eval_level = saved_eval;
        c->final_pending = saved_pending;
        hcheck(e1, "end capture");
        const hipError_t e2 = hipGraphInstantiate(&c->gexec[cur0], g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        hcheck(e2, "graph instantiate");
        c->graph_window = W;
    }
    hcheck(hipGraphLaunch(c->gexec[cur0], c->stream), "graph launch");
    for (int64_t n = c->step; n < c->step + W; ++n)
        if (diag_step(c, n)) c->last_eval_level = n + 1;
    c->step += W;

}

void run_steps(axp_ctx *c, int n_steps) {
    if ((c->fs.n_src > 0 || c->fs.probe_face >= 0) && n_steps > 0) {
        // sources and probe read the step index on the device: start it at the host's
        c->step_upload = (unsigned long long)c->step;
        hcheck(hipMemcpyAsync(&c->ds.ctr->step, &c->step_upload, sizeof(unsigned long long), hipMemcpyHostToDevice,
                              c->stream), "step counter");
    }
    if (c->inj_on && n_steps > 0) {
        const DevCounters h = read_counters(c);
        grow_particles(c, int64_t(h.n_slots) + int64_t(n_steps) * c->inj.per_step);
    }
    const int sp = c->cfg.sort_period;
    const int W = 2 * sp;
    const int de = c->cfg.diag_every;
    for (int i = 0; i < n_steps;) {
        // with timing on the steps run eagerly: HIP does not time event records inside graphs
        bool graph = c->cfg.use_graph && !c->timing && c->step % sp == 0 && n_steps - i >= W;
        if (graph && de > 0 && sp % de != 0) {
            // a window's diagnostic steps would differ from one replay to the next:
            // replay only windows without one
            for (int64_t n = c->step; n < c->step + W; ++n)
                if (diag_step(c, n)) { graph = false; break; }
        }
        if (graph && c->graph_window != 0 && c->graph_window != W) drop_graphs(c);
        if (graph) {
            flush_final(c, c->stream);   // windows start with no reduction pending
            launch_graph(c, W);
            i += W;
            continue;
        }
        enqueue_step(c, c->stream);
        ++i;
        if (c->ev.size() > 4096) collect_timing(c);
    }
    flush_final(c, c->stream);
    hcheck(hipGetLastError(), "step launch");
}

// ---- run-time energy guard of the learned SPAI

// Device regions a step reads and writes (fields, sources, the particle
// buffer in use up to n_slots, counters and diagnostic state).
std::vector<std::pair<void *, size_t>> state_regions(axp_ctx *c, int64_t n_slots) {
    const DevState &s = c->ds;
    const size_t n0 = c->hm.n0, n1 = c->hm.n1, n2 = c->hm.n2, np = size_t(n_slots);
    const int b = s.cur;
    std::vector<std::pair<void *, size_t>> r = {
        {s.B, 8 * n2}, {s.Bprev, 8 * n2}, {s.D, 8 * n1}, {s.g0, 8 * n0}, {s.cell[b], 4 * np},
        {s.ctr, sizeof(DevCounters)}, {s.diag, sizeof(DevDiag)}};
    if (c->plain) {
        const DevPlain &p = c->dp;
        for (void *q : {(void *)p.E, (void *)p.Jfx}) r.push_back({q, 8 * n1});
        for (void *q : {(void *)p.Qres, (void *)p.Q, (void *)p.Qprev}) r.push_back({q, 8 * n0});
        for (void *q : {(void *)p.l0[b], (void *)p.l1[b], (void *)p.ur[b], (void *)p.up[b], (void *)p.uz[b]})
            r.push_back({q, 8 * np});
    } else {
        r.push_back({s.E, 4 * n1});
        r.push_back({s.D32, 4 * n1});
        r.push_back({s.Jfx, 8 * n1});
        for (void *q : {(void *)s.Qres, (void *)s.Qfx, (void *)s.Qprev}) r.push_back({q, 8 * n0});
        for (void *q : {(void *)s.L0[b], (void *)s.L1[b], (void *)s.ur[b], (void *)s.up[b], (void *)s.uz[b]})
            r.push_back({q, 4 * np});
    }
    return r;
}

struct Checkpoint {
    std::vector<std::pair<void *, size_t>> regions;
    int64_t step = 0, last_eval_level = -1, n_live_host = 0;
    int cur = 0;
    uint64_t energy_count = 0;
};

// Device copy of the state into c->snap (grown as needed); the copies are
// enqueued on the context's stream.
Checkpoint take_checkpoint(axp_ctx *c) {
    const DevCounters h = read_counters(c);
    Checkpoint k;
    k.regions = state_regions(c, int64_t(h.n_slots));
    size_t total = 0;
    for (auto &r : k.regions) total += (r.second + 255) & ~size_t(255);
    if (total > c->snap_bytes) {
        if (c->snap) dfree(c, c->snap);
        c->snap = nullptr;
        c->snap_bytes = 0;
        c->snap = dalloc(c, total);
        c->snap_bytes = total;
    }
    size_t off = 0;
    for (auto &r : k.regions) {
        if (r.second)
            hcheck(hipMemcpyAsync(static_cast<char *>(c->snap) + off, r.first, r.second, hipMemcpyDeviceToDevice,
                                  c->stream), "checkpoint");
        off += (r.second + 255) & ~size_t(255);
    }
    k.step = c->step;
    k.last_eval_level = c->last_eval_level;
    k.n_live_host = c->n_live_host;
    k.cur = c->ds.cur;
    k.energy_count = h.energy_count;
    return k;
}

void restore_checkpoint(axp_ctx *c, const Checkpoint &k) {
    size_t off = 0;
    for (auto &r : k.regions) {
        if (r.second)
            hcheck(hipMemcpyAsync(r.first, static_cast<char *>(c->snap) + off, r.second, hipMemcpyDeviceToDevice,
                                  c->stream), "restore");
        off += (r.second + 255) & ~size_t(255);
    }
    c->step = k.step;
    c->last_eval_level = k.last_eval_level;
    c->n_live_host = k.n_live_host;
    c->ds.cur = k.cur;
    hcheck(hipStreamSynchronize(c->stream), "sync");
}

// Replaces the learned M by the plain SPAI (host least squares, then the
// sliced ELL upload).  Throws AXP_E_UNSTABLE, the learned M kept, if the run's
// dt exceeds the plain SPAI's stability limit.
void revert_to_plain_spai(axp_ctx *c) {
    HostMesh &m = c->hm;
    Csr learned = m.M;
    const double fro = m.spai_fro, mx = m.spai_max_col;
    const int64_t nnz = m.spai_nnz;
    const int nt = int(std::min(16u, std::max(1u, std::thread::hardware_concurrency())));
    build_spai(m, c->cfg.spai_level, c->cfg.spai_drop_tol, nt);
    const double cfl = cfl_dt(m, 400);
    if (!(c->dt <= cfl * (1.0 + 1e-9))) {
        m.M = std::move(learned);
        m.spai_fro = fro; m.spai_max_col = mx; m.spai_nnz = nnz;
        throw ApiError{AXP_E_UNSTABLE, "the run-time guard tripped, but dt " + std::to_string(c->dt) +
                                           " exceeds the plain SPAI's stability limit " + std::to_string(cfl)};
    }
    std::vector<int64_t> sptr;
    std::vector<int32_t> slen, mcol;
    std::vector<float> mval;
    std::vector<double> mvald;
    build_sell(m.M, m.n1, sptr, slen, mval, c->plain ? &mvald : nullptr, mcol);
    hcheck(hipStreamSynchronize(c->stream), "sync");
    DevMesh &d = c->dm;
    dfree(c, (void *)d.m_sptr); dfree(c, (void *)d.m_slen); dfree(c, (void *)d.m_col);
    d.m_sptr = upload(c, sptr); d.m_slen = upload(c, slen); d.m_col = upload(c, mcol);
    if (c->plain) {
        dfree(c, (void *)c->dp.m_val);
        c->dp.m_val = upload(c, mvald);
    } else {
        dfree(c, (void *)d.m_val);
        d.m_val = upload(c, mval);
    }
    c->dt_cfl = cfl;
    drop_graphs(c);
    c->spai_mode_used = AXP_SPAI_LEARNED_REVERTED;
}

// Steps with the guard armed: chunks that fit the energy ring, each with a
// checkpoint before it and a look at its energy records after it.
void guarded_steps(axp_ctx *c, int n_steps) {
    const int de = c->cfg.diag_every;
    const int chunk_max = std::max(1, (kEnergyRing / 2) * de);
    for (int done = 0; done < n_steps;) {
        const int n = std::min(n_steps - done, chunk_max);
        if (c->inj_on) {
            // grow first: the checkpoint must cover the buffers the steps use
            const DevCounters h = read_counters(c);
            grow_particles(c, int64_t(h.n_slots) + int64_t(n) * c->inj.per_step);
        }
        const Checkpoint ck = take_checkpoint(c);
        run_steps(c, n);
        const DevCounters h = read_counters(c);
        const int64_t k = int64_t(h.energy_count) - int64_t(ck.energy_count);
        int64_t trip = -1;
        if (k > 0) {
            std::vector<DevEnergy> ring(kEnergyRing);
            hcheck(hipMemcpyAsync(ring.data(), c->ds.energy, sizeof(DevEnergy) * kEnergyRing, hipMemcpyDeviceToHost,
                                  c->stream), "energies");
            hcheck(hipStreamSynchronize(c->stream), "sync");
            for (int64_t i = 0; i < k; ++i) {
                const DevEnergy &e = ring[size_t((ck.energy_count + uint64_t(i)) % kEnergyRing)];
                const double w = e.WE + e.WB + e.WK;
                if (!c->guard_ref_set) {
                    if (w != 0.0 && std::isfinite(w)) { c->guard_wref = w; c->guard_ref_set = true; }
                    continue;
                }
                const double drift = std::fabs(w - c->guard_wref) / std::fabs(c->guard_wref);
                if (!(drift <= c->guard_drift)) c->guard_drift = std::isfinite(drift) ? drift : INFINITY;
                if (!(drift <= c->guard_tol)) { trip = e.level; break; }
            }
        }
        if (trip >= 0) {
            revert_to_plain_spai(c);
            restore_checkpoint(c, ck);
            // D is the state: Gauss's law and continuity carry over; E = M D with the new M
            if (c->plain) launch_spmv_plain(c->dm, c->ds, c->dp, c->stream);
            else launch_spmv(c->dm, c->ds, c->stream);
            hcheck(hipGetLastError(), "spmv launch");
            c->guard_trip_step = trip;
            c->guard_tol = -1.0;
            run_steps(c, n);
            done += n;
            if (done < n_steps) run_steps(c, n_steps - done);
            return;
        }
        done += n;
    }
}

}  // namespace

extern "C" {

void axp_config_default(axp_config *cfg) {
    if (!cfg) return;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->device = 0;
    cfg->hip_stream = nullptr;
    cfg->precision = AXP_PREC_MIXED;
    cfg->dt = 0.0;
    cfg->cfl_fraction = 0.5;
    cfg->spai_level = 3;
    cfg->spai_drop_tol = 1e-3;
    cfg->sort_period = 4;
    cfg->diag_every = 0;
    cfg->max_walk = 64;
    cfg->use_graph = 1;
    cfg->pusher = AXP_PUSH_BORIS;
}

axp_status axp_create(const axp_config *cfg, axp_ctx **out) {
    if (!cfg || !out) return AXP_E_ARG;
    *out = nullptr;
    if (cfg->precision != AXP_PREC_MIXED && cfg->precision != AXP_PREC_PLAIN_FP64) return AXP_E_ARG;
    if (cfg->pusher != AXP_PUSH_BORIS && cfg->pusher != AXP_PUSH_VAY) return AXP_E_ARG;
    if (cfg->spai_level < 1 || cfg->spai_level > 6 || cfg->spai_drop_tol < 0 || cfg->sort_period < 1 ||
        cfg->max_walk < 1 || cfg->diag_every < 0)
        return AXP_E_ARG;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || cfg->device < 0 || cfg->device >= ndev) return AXP_E_HIP;
    auto *c = new (std::nothrow) axp_ctx();
    if (!c) return AXP_E_OOM;
    c->cfg = *cfg;
    c->plain = cfg->precision == AXP_PREC_PLAIN_FP64;
    if (hipSetDevice(cfg->device) != hipSuccess) { delete c; return AXP_E_HIP; }
    c->stream = (hipStream_t)cfg->hip_stream;
    *out = c;
    return AXP_OK;
}

axp_status axp_set_mesh(axp_ctx *c, int32_t n_nodes, const double *zr, int32_t n_tris, const int32_t *tri) {
    if (!c) return AXP_E_ARG;
    if (c->built) return fail(c, AXP_E_STATE, "mesh already built");
    if (n_nodes < 3 || n_tris < 1 || !zr || !tri) return fail(c, AXP_E_ARG, "bad mesh arguments");
    if (n_tris >= (1 << kCellBits)) return fail(c, AXP_E_ARG, "too many triangles");
    c->in_zr.assign(zr, zr + 2 * size_t(n_nodes));
    c->in_tri.assign(tri, tri + 3 * size_t(n_tris));
    c->has_mesh = true;
    return AXP_OK;
}

axp_status axp_set_boundary(axp_ctx *c, int32_t n_seg, const int32_t *seg, const uint8_t *tag) {
    if (!c) return AXP_E_ARG;
    if (c->built) return fail(c, AXP_E_STATE, "mesh already built");
    if (n_seg < 0 || (n_seg > 0 && (!seg || !tag))) return fail(c, AXP_E_ARG, "bad boundary arguments");
    c->in_seg.assign(seg, seg + 2 * size_t(n_seg));
    c->in_tag.assign(tag, tag + size_t(n_seg));
    c->has_bnd = true;
    return AXP_OK;
}

axp_status axp_build(axp_ctx *c) {
    if (!c) return AXP_E_ARG;
    if (c->built) return fail(c, AXP_E_STATE, "already built");
    if (!c->has_mesh) return fail(c, AXP_E_STATE, "axp_set_mesh first");
    return guarded(c, [&]() -> axp_status {
        auto t0 = std::chrono::steady_clock::now();
        HostMesh m;
        build_topology(m, int32_t(c->in_zr.size() / 2), c->in_zr.data(), int32_t(c->in_tri.size() / 3),
                       c->in_tri.data(), int32_t(c->in_seg.size() / 2), c->in_seg.data(), c->in_tag.data());
        assemble_hodge(m);
        int nt = int(std::min(16u, std::max(1u, std::thread::hardware_concurrency())));
        auto ts = std::chrono::steady_clock::now();
        c->spai_mode_used = AXP_SPAI_PLAIN;
        if (c->spai_model) {
            // network guess, refinement, least-squares fallback per column
            ScaledHodge h;
            scaled_hodge(m, h);
            PairSet ps;
            spai_pair_features(m, h, c->cfg.spai_level, nt, ps);
            const auto tf = std::chrono::steady_clock::now();
            std::vector<float> pred(ps.j.size());
            std::string err;
            const int st = mlp_predict_host(c->spai_model, ps.X.data(), int64_t(ps.j.size()), pred.data(), err);
            if (st != AXP_OK) throw ApiError{st, err};
            ps.X.clear();
            ps.X.shrink_to_fit();
            const auto ti = std::chrono::steady_clock::now();
            learned_spai(m, h, ps, pred.data(), c->cfg.spai_level, c->cfg.spai_drop_tol, c->spai_iters, c->spai_row_tol,
                         nt, c->spai_stats);
            c->spai_mode_used = AXP_SPAI_LEARNED;
            c->spai_feature_s = std::chrono::duration<double>(tf - ts).count();
            c->spai_infer_s = std::chrono::duration<double>(ti - tf).count();
            c->spai_solve_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - ti).count();
        } else {
            build_spai(m, c->cfg.spai_level, c->cfg.spai_drop_tol, nt);
            c->spai_solve_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - ts).count();
        }
        c->spai_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - ts).count();
        c->dt_cfl = cfl_dt(m, 400);
        c->dt = c->cfg.dt > 0 ? c->cfg.dt : c->cfg.cfl_fraction * c->dt_cfl;
        if (c->spai_model) {
            // run-level guard: the source-free leapfrog energy must be conserved
            c->spai_energy_drift = std::isfinite(c->dt_cfl) && c->dt <= c->dt_cfl
                                       ? leapfrog_energy_drift(m, c->dt, 64, 12345)
                                       : INFINITY;
            if (!(c->spai_energy_drift <= c->spai_energy_tol)) {
                const auto tr = std::chrono::steady_clock::now();
                build_spai(m, c->cfg.spai_level, c->cfg.spai_drop_tol, nt);
                c->spai_solve_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - tr).count();
                c->spai_mode_used = AXP_SPAI_LEARNED_REJECTED;
                c->dt_cfl = cfl_dt(m, 400);
                c->dt = c->cfg.dt > 0 ? c->cfg.dt : c->cfg.cfl_fraction * c->dt_cfl;
            }
        }
        if (c->layer_cfg.sides) {
            // the time step is fixed without the layers; the SPAI then inverts
            // the stretched Hodge, and the stability limit is that of the result
            if (c->spai_model) throw ApiError{AXP_E_ARG, "absorbing layers need the least-squares SPAI"};
            if (!(c->dt > 0)) throw ApiError{AXP_E_UNSTABLE, "no time step"};
            Csr K;
            build_layers(m, c->dt, c->layer_cfg, c->hl, K);
            std::swap(m.A, K);
            build_spai(m, c->cfg.spai_level, c->cfg.spai_drop_tol, nt);
            std::swap(m.A, K);
            c->dt_cfl = cfl_dt(m, 400);
        }
        if (!(c->dt > 0) || c->dt > c->dt_cfl * (1.0 + 1e-9))
            throw ApiError{AXP_E_UNSTABLE, "dt " + std::to_string(c->dt) + " exceeds the stability limit " +
                                               std::to_string(c->dt_cfl)};
        build_locator(m);
        c->hm = std::move(m);
        c->shape_hash = mesh_hash(c);
        if (hipSetDevice(c->cfg.device) != hipSuccess) throw ApiError{AXP_E_HIP, "hipSetDevice"};
        build_device(c);
        c->setup_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        c->built = true;
        return AXP_OK;
    });
}

axp_status axp_info_get(const axp_ctx *c, axp_info *out) {
    if (!c || !out) return AXP_E_ARG;
    std::memset(out, 0, sizeof(*out));
    const HostMesh &m = c->hm;
    out->n_nodes = m.n0; out->n_edges = m.n1; out->n_faces = m.n2;
    out->n_free_edges = m.n_free_edges; out->n_free_nodes = m.n_free_nodes;
    out->spai_nnz = m.spai_nnz; out->spai_fro_residual = m.spai_fro; out->spai_max_col_residual = m.spai_max_col;
    out->dt = c->dt; out->dt_cfl = c->dt_cfl; out->setup_seconds = c->setup_s;
    out->particle_capacity = c->ds.capacity; out->n_particles = c->n_live_host;
    out->step = c->step; out->precision = c->cfg.precision; out->n_species = int32_t(c->species.size());
    out->spai_mode = c->spai_mode_used;
    out->spai_fallback_columns = c->spai_stats.n_fallback;
    out->spai_pred_resid_mean = c->spai_stats.pred_resid_mean;
    out->spai_kept_resid_mean = c->spai_stats.kept_resid_mean;
    out->spai_energy_drift = c->spai_energy_drift;
    out->spai_seconds = c->spai_seconds;
    out->n_layer_faces = int64_t(c->hl.face.size());
    out->spai_guard_trip_step = c->guard_trip_step;
    out->spai_run_drift = c->guard_drift;
    out->spai_feature_seconds = c->spai_feature_s;
    out->spai_infer_seconds = c->spai_infer_s;
    out->spai_solve_seconds = c->spai_solve_s;
    out->sort_period = c->cfg.sort_period;
    out->window_lead = c->win_lead;
    return c->built ? AXP_OK : AXP_E_STATE;
}

axp_status axp_get_edges(const axp_ctx *c, int32_t *edges) {
    if (!c || !edges) return AXP_E_ARG;
    if (!c->built) return AXP_E_STATE;
    for (int k = 0; k < c->hm.n1; ++k) {
        const auto &e = c->hm.ev[c->hm.edge_int[k]];
        edges[2 * k] = e[0];
        edges[2 * k + 1] = e[1];
    }
    return AXP_OK;
}

axp_status axp_get_spai(const axp_ctx *c, int64_t capacity, int64_t *nnz, int64_t *rowptr, int32_t *col, double *val) {
    if (!c || !nnz || !rowptr) return AXP_E_ARG;
    if (!c->built) return AXP_E_STATE;
    const HostMesh &m = c->hm;
    *nnz = m.M.ptr[m.n1];
    if (*nnz > capacity || !col || !val) return AXP_E_ARG;
    rowptr[0] = 0;
    int64_t o = 0;
    std::vector<std::pair<int32_t, double>> row;
    for (int k = 0; k < m.n1; ++k) {
        int i = m.edge_int[k];
        row.clear();
        for (int64_t q = m.M.ptr[i]; q < m.M.ptr[i + 1]; ++q) row.push_back({m.edge_can[m.M.col[q]], m.M.val[q]});
        std::sort(row.begin(), row.end());
        for (auto &p : row) { col[o] = p.first; val[o] = p.second; ++o; }
        rowptr[k + 1] = o;
    }
    return AXP_OK;
}

axp_status axp_set_fields(axp_ctx *c, const double *E0, const double *B_mhalf) {
    if (!c || !E0 || !B_mhalf) return AXP_E_ARG;
    return guarded(c, [&]() -> axp_status {
        require_built(c);
        const HostMesh &m = c->hm;
        std::vector<double> E(m.n1), B(m.n2), D(m.n1);
        for (int k = 0; k < m.n1; ++k) {
            int i = m.edge_int[k];
            E[i] = m.efree[i] ? E0[k] : 0.0;
            if (!std::isfinite(E[i])) throw ApiError{AXP_E_NAN, "non-finite E0"};
        }
        for (int u = 0; u < m.n2; ++u) {
            B[m.tri_int[u]] = B_mhalf[u];
            if (!std::isfinite(B_mhalf[u])) throw ApiError{AXP_E_NAN, "non-finite B"};
        }
        cg_solve_M(m, E.data(), D.data(), 1e-15, 5000);
        std::vector<float> E32(m.n1), D32(m.n1);
        for (int i = 0; i < m.n1; ++i) { E32[i] = float(E[i]); D32[i] = float(D[i]); }
        DevState &s = c->ds;
        hcheck(hipMemcpyAsync(s.B, B.data(), m.n2 * 8, hipMemcpyHostToDevice, c->stream), "B");
        hcheck(hipMemcpyAsync(s.D, D.data(), m.n1 * 8, hipMemcpyHostToDevice, c->stream), "D");
        if (c->plain) {
            hcheck(hipMemcpyAsync(c->dp.E, E.data(), m.n1 * 8, hipMemcpyHostToDevice, c->stream), "E");
        } else {
            hcheck(hipMemcpyAsync(s.D32, D32.data(), m.n1 * 4, hipMemcpyHostToDevice, c->stream), "D32");
            hcheck(hipMemcpyAsync(s.E, E32.data(), m.n1 * 4, hipMemcpyHostToDevice, c->stream), "E");
        }
        hcheck(hipStreamSynchronize(c->stream), "sync");
        layers_at_rest(c, E, B);
        reset_diag_refs(c, true);
        return AXP_OK;
    });
}

axp_status axp_set_layers(axp_ctx *c, int32_t sides, double z_left, double z_right, double sigma_max, int32_t order) {
    if (!c || sides < 0 || sides > 3 || !std::isfinite(z_left) || !std::isfinite(z_right) || !(sigma_max >= 0.0) ||
        !std::isfinite(sigma_max) || order < 0 || order > 8)
        return AXP_E_ARG;
    if (c->built) return fail(c, AXP_E_STATE, "absorbing layers are set before axp_build");
    c->layer_cfg.sides = sigma_max > 0.0 ? sides : 0;
    c->layer_cfg.z_left = z_left;
    c->layer_cfg.z_right = z_right;
    c->layer_cfg.sigma_max = sigma_max;
    c->layer_cfg.order = order;
    return AXP_OK;
}

axp_status axp_set_electrostatic(axp_ctx *c, const double *phi_conductor, int32_t with_charge, double *phi_out) {
    if (!c || (with_charge != 0 && with_charge != 1)) return AXP_E_ARG;
    return guarded(c, [&]() -> axp_status {
        require_built(c);
        const HostMesh &m = c->hm;
        std::vector<double> phic(m.n0, 0.0), Q(m.n0, 0.0);
        if (phi_conductor)
            for (int v = 0; v < m.n0; ++v) {
                if (m.nfree[v]) continue;
                if (!std::isfinite(phi_conductor[v])) throw ApiError{AXP_E_NAN, "non-finite conductor potential"};
                phic[v] = phi_conductor[v];
            }
        if (with_charge) {
            // nodal charge of the particles present and of the wall reservoirs [C/rad]
            run_diag(c);
            if (c->plain) {
                hcheck(hipMemcpyAsync(Q.data(), c->dp.Q, m.n0 * 8, hipMemcpyDeviceToHost, c->stream), "Q");
                hcheck(hipStreamSynchronize(c->stream), "sync");
                for (int v = 0; v < m.n0; ++v) Q[v] *= c->pc.qunit;
            } else {
                std::vector<long long> q(m.n0);
                hcheck(hipMemcpyAsync(q.data(), c->ds.Qfx, m.n0 * 8, hipMemcpyDeviceToHost, c->stream), "Q");
                hcheck(hipStreamSynchronize(c->stream), "sync");
                for (int v = 0; v < m.n0; ++v) Q[v] = double(q[v]) * c->ic.qscale;
            }
        }
        std::vector<double> phi, E, D;
        double res = 0.0;
        const int it = electrostatic_state(m, phic.data(), Q.data(), 1e-13, 60, phi, E, D, res);
        if (it < 0) throw ApiError{AXP_E_SPAI, "electrostatic solve did not converge (residual " + std::to_string(res) + ")"};
        std::vector<double> B(m.n2, 0.0);
        std::vector<float> E32(m.n1), D32(m.n1);
        for (int i = 0; i < m.n1; ++i) { E32[i] = float(E[i]); D32[i] = float(D[i]); }
        DevState &s = c->ds;
        hcheck(hipMemcpyAsync(s.B, B.data(), m.n2 * 8, hipMemcpyHostToDevice, c->stream), "B");
        hcheck(hipMemcpyAsync(s.D, D.data(), m.n1 * 8, hipMemcpyHostToDevice, c->stream), "D");
        if (c->plain) {
            hcheck(hipMemcpyAsync(c->dp.E, E.data(), m.n1 * 8, hipMemcpyHostToDevice, c->stream), "E");
        } else {
            hcheck(hipMemcpyAsync(s.D32, D32.data(), m.n1 * 4, hipMemcpyHostToDevice, c->stream), "D32");
            hcheck(hipMemcpyAsync(s.E, E32.data(), m.n1 * 4, hipMemcpyHostToDevice, c->stream), "E");
        }
        hcheck(hipStreamSynchronize(c->stream), "sync");
        layers_at_rest(c, E, B);
        reset_diag_refs(c, true);
        if (phi_out) std::memcpy(phi_out, phi.data(), sizeof(double) * m.n0);
        return AXP_OK;
    });
}

axp_status axp_add_point_source(axp_ctx *c, double z, double rho, double amplitude, double t0, double sigma,
                                double omega) {
    if (!c || !std::isfinite(z) || !std::isfinite(rho) || !std::isfinite(amplitude) || !std::isfinite(t0) ||
        !(sigma > 0.0) || !std::isfinite(sigma) || !std::isfinite(omega))
        return AXP_E_ARG;
    return guarded(c, [&]() -> axp_status {
        require_built(c);
        if (c->fs.n_src >= kMaxSources) throw ApiError{AXP_E_ARG, "too many point sources"};
        double lam[3];
        const int32_t t = locate_point(c->hm, z, rho, lam);
        if (t < 0) throw ApiError{AXP_E_ARG, "point source outside the mesh"};
        const int k = c->fs.n_src++;
        c->fs.src_face[k] = t;
        c->fs.amp[k] = amplitude;
        c->fs.t0[k] = t0;
        c->fs.sig[k] = sigma;
        c->fs.w[k] = omega;
        c->fs.dt = c->dt;
        drop_graphs(c);
        return AXP_OK;
    });
}

axp_status axp_clear_point_sources(axp_ctx *c) {
    if (!c) return AXP_E_ARG;
    return guarded(c, [&]() -> axp_status {
        c->fs.n_src = 0;
        drop_graphs(c);
        return AXP_OK;
    });
}

axp_status axp_set_probe(axp_ctx *c, double z, double rho, int64_t capacity) {
    if (!c || capacity < 0 || !std::isfinite(z) || !std::isfinite(rho)) return AXP_E_ARG;
    return guarded(c, [&]() -> axp_status {
        require_built(c);
        dfree(c, c->fs.probe);
        c->fs.probe = nullptr;
        c->fs.probe_face = -1;
        c->fs.probe_cap = 0;
        drop_graphs(c);
        if (capacity == 0) return AXP_OK;
        double lam[3];
        const int32_t t = locate_point(c->hm, z, rho, lam);
        if (t < 0) throw ApiError{AXP_E_ARG, "probe outside the mesh"};
        c->fs.probe = zeros<double>(c, size_t(2) * size_t(capacity));
        c->fs.probe_face = t;
        c->fs.probe_l0 = lam[0];
        c->fs.probe_l1 = lam[1];
        c->fs.probe_cap = capacity;
        c->fs.probe_start = c->step;
        c->fs.dt = c->dt;
        return AXP_OK;
    });
}

axp_status axp_get_probe(axp_ctx *c, int64_t capacity, int64_t *n, double *E_z_rho) {
    if (!c || !n || capacity < 0) return AXP_E_ARG;
    return guarded(c, [&]() -> axp_status {
        require_built(c);
        *n = 0;
        if (c->fs.probe_face < 0) return AXP_OK;
        const int64_t have = std::min<int64_t>(c->step - c->fs.probe_start, c->fs.probe_cap);
        *n = have;
        if (!E_z_rho) return AXP_OK;
        if (have > capacity) return fail(c, AXP_E_ARG, "capacity too small");
        hcheck(hipStreamSynchronize(c->stream), "sync");
        if (have > 0)
            hcheck(hipMemcpy(E_z_rho, c->fs.probe, size_t(have) * 2 * sizeof(double), hipMemcpyDeviceToHost), "probe");
        return AXP_OK;
    });
}

axp_status axp_set_external_bz(axp_ctx *c, double bz) {
    if (!c || !std::isfinite(bz)) return AXP_E_ARG;
    return guarded(c, [&]() -> axp_status {
        require_built(c);
        c->ic.bz = float(bz);
        c->pc.bz = bz;
        upload_inst(c);
        drop_graphs(c);
        return AXP_OK;
    });
}

axp_status axp_add_species(axp_ctx *c, double q, double m, int64_t weight, int32_t *id) {
    if (!c || !id || !(m > 0) || q == 0.0 || weight < 1 || !std::isfinite(q)) return AXP_E_ARG;
    return guarded(c, [&]() -> axp_status {
        require_built(c);
        if (c->species.size() >= size_t(kMaxSpecies)) throw ApiError{AXP_E_ARG, "too many species"};
        double qw = q * double(weight);
        if (c->species.empty()) c->q_unit = qw;
        double k = qw / c->q_unit;
        if (std::fabs(k - std::nearbyint(k)) > 1e-9 * std::fabs(k) || std::fabs(k) > 64)
            throw ApiError{AXP_E_ARG, "macro charge must be a small integer multiple of the first species' macro charge"};
        int sp = int(c->species.size());
        c->species.push_back({q, m, weight});
        InstConst &ic = c->ic;
        ic.n_species = int32_t(c->species.size());
        ic.qe[sp] = float(q * c->dt / (2.0 * m * kC));
        ic.qb[sp] = float(q * c->dt / (2.0 * m));
        ic.kq[sp] = int32_t(std::nearbyint(k));
        if (ic.kq[sp] != 0 && ic.kq[sp] != 1) c->q32 = false;
        ic.mw[sp] = m * double(weight) * kC * kC / kTwoPi;
        ic.jscale = c->q_unit / (kTwoPi * double(kLamOne) * double(kLamOne));   // current unit 2^-46
        ic.qscale = c->q_unit / (kTwoPi * double(kLamOne));                    // charge unit 2^-23
        PlainConst &pc = c->pc;
        pc.n_species = ic.n_species;
        pc.qe[sp] = q * c->dt / (2.0 * m * kC);
        pc.qb[sp] = q * c->dt / (2.0 * m);
        pc.kq[sp] = std::nearbyint(k);
        pc.mw[sp] = ic.mw[sp];
        pc.qunit = c->q_unit / kTwoPi;
        upload_inst(c);
        drop_graphs(c);
        *id = sp;
        return AXP_OK;
    });
}

axp_status axp_inject(axp_ctx *c, int32_t species, int64_t n, const double *zr, const double *u) {
    if (!c || n < 0 || (n > 0 && (!zr || !u))) return AXP_E_ARG;
    return guarded(c, [&]() -> axp_status {
        require_built(c);
        if (species < 0 || species >= int(c->species.size())) throw ApiError{AXP_E_ARG, "unknown species"};
        if (n == 0) return AXP_OK;
        const HostMesh &m = c->hm;
        std::vector<int32_t> cell(n);
        std::vector<uint32_t> l0(n), l1(n);
        std::vector<float> ur(n), up(n), uz(n);
        const bool plain = c->plain;
        std::vector<double> dl0(plain ? n : 0), dl1(plain ? n : 0), dur(plain ? n : 0), dup(plain ? n : 0),
            duz(plain ? n : 0);
        std::vector<int> bad(1, -1);
        int nt = int(std::min<int64_t>(16, std::max<int64_t>(1, n / 4096)));
        std::vector<std::thread> th;
        std::vector<int64_t> badidx(nt, -1);
        auto work = [&](int tid) {
            for (int64_t i = tid; i < n; i += nt) {
                double lam[3];
                int32_t t = locate_point(m, zr[2 * i], zr[2 * i + 1], lam);
                if (t < 0 || !std::isfinite(u[3 * i]) || !std::isfinite(u[3 * i + 1]) || !std::isfinite(u[3 * i + 2])) {
                    badidx[tid] = i;
                    continue;
                }
                double s = 0;
                for (int k = 0; k < 3; ++k) { lam[k] = std::max(0.0, lam[k]); s += lam[k]; }
                cell[i] = t | (species << kCellBits);
                if (plain) {
                    // lambda_2 = 1 - l0 - l1 must not come out negative by rounding
                    dl0[i] = std::min(1.0, lam[0] / s);
                    dl1[i] = std::min(lam[1] / s, 1.0 - dl0[i]);
                    dur[i] = u[3 * i] / kC;
                    dup[i] = u[3 * i + 1] / kC;
                    duz[i] = u[3 * i + 2] / kC;
                    continue;
                }
                int64_t a = std::llround(lam[0] / s * double(kLamOne));
                int64_t b = std::llround(lam[1] / s * double(kLamOne));
                a = std::min<int64_t>(std::max<int64_t>(a, 0), kLamOne);
                b = std::min<int64_t>(std::max<int64_t>(b, 0), kLamOne - a);
                l0[i] = uint32_t(a);
                l1[i] = uint32_t(b);
                ur[i] = float(u[3 * i] / kC);
                up[i] = float(u[3 * i + 1] / kC);
                uz[i] = float(u[3 * i + 2] / kC);
            }
        };
        for (int t = 1; t < nt; ++t) th.emplace_back(work, t);
        work(0);
        for (auto &t : th) t.join();
        for (auto b : badidx)
            if (b >= 0) throw ApiError{AXP_E_ARG, "particle " + std::to_string(b) + " is outside the mesh or has a non-finite momentum"};
        DevCounters h = read_counters(c);
        int64_t used = int64_t(h.n_slots);
        grow_particles(c, used + n);
        DevState &s = c->ds;
        int b = s.cur;
        hcheck(hipMemcpyAsync(s.cell[b] + used, cell.data(), n * 4, hipMemcpyHostToDevice, c->stream), "inject");
        if (plain) {
            DevPlain &p = c->dp;
            hcheck(hipMemcpyAsync(p.l0[b] + used, dl0.data(), n * 8, hipMemcpyHostToDevice, c->stream), "inject");
            hcheck(hipMemcpyAsync(p.l1[b] + used, dl1.data(), n * 8, hipMemcpyHostToDevice, c->stream), "inject");
            hcheck(hipMemcpyAsync(p.ur[b] + used, dur.data(), n * 8, hipMemcpyHostToDevice, c->stream), "inject");
            hcheck(hipMemcpyAsync(p.up[b] + used, dup.data(), n * 8, hipMemcpyHostToDevice, c->stream), "inject");
            hcheck(hipMemcpyAsync(p.uz[b] + used, duz.data(), n * 8, hipMemcpyHostToDevice, c->stream), "inject");
        } else {
        hcheck(hipMemcpyAsync(s.L0[b] + used, l0.data(), n * 4, hipMemcpyHostToDevice, c->stream), "inject");
        hcheck(hipMemcpyAsync(s.L1[b] + used, l1.data(), n * 4, hipMemcpyHostToDevice, c->stream), "inject");
        hcheck(hipMemcpyAsync(s.ur[b] + used, ur.data(), n * 4, hipMemcpyHostToDevice, c->stream), "inject");
        hcheck(hipMemcpyAsync(s.up[b] + used, up.data(), n * 4, hipMemcpyHostToDevice, c->stream), "inject");
        hcheck(hipMemcpyAsync(s.uz[b] + used, uz.data(), n * 4, hipMemcpyHostToDevice, c->stream), "inject");
        }
        unsigned long long ns = (unsigned long long)(used + n);
        hcheck(hipMemcpyAsync(&s.ctr->n_slots, &ns, 8, hipMemcpyHostToDevice, c->stream), "slots");
        if (plain) launch_sort_plain(c->dm, s, c->dp, false, c->stream);
        else launch_sort(c->dm, s, false, c->stream);
        hcheck(hipGetLastError(), "sort launch");
        hcheck(hipStreamSynchronize(c->stream), "inject sync");
        c->n_live_host = int64_t(read_counters(c).n_slots);
        reset_diag_refs(c, false);      // the added charge breaks the continuity chain
        return AXP_OK;
    });
}

axp_status axp_set_injector(axp_ctx *c, int32_t species, int64_t per_step, const double *u_mean, double u_spread,
                            uint64_t seed) {
    if (!c || per_step < 0 || per_step > (int64_t(1) << 24) || (per_step > 0 && !u_mean) || !(u_spread >= 0))
        return AXP_E_ARG;
    return guarded(c, [&]() -> axp_status {
        require_built(c);
        drop_graphs(c);
        if (per_step == 0) { c->inj_on = false; return AXP_OK; }
        if (species < 0 || species >= int(c->species.size())) throw ApiError{AXP_E_ARG, "unknown species"};
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(u_mean[k])) throw ApiError{AXP_E_ARG, "non-finite mean momentum"};
        const HostMesh &m = c->hm;
        std::vector<EmitEdge> ee;
        double cum = 0;
        for (int k = 0; k < m.n1; ++k) {            // canonical order
            const int e = m.edge_int[k];
            if (m.etag[e] != TAG_EMITTER) continue;
            const int f = m.etri[e][0], side = m.eside[e][0];
            const int ta = m.ev[e][0], hb = m.ev[e][1];
            EmitEdge E{};
            E.face = f;
            E.ka = E.kb = -1;
            for (int q = 0; q < 3; ++q) {
                if (m.tv[f][q] == ta) E.ka = q;
                if (m.tv[f][q] == hb) E.kb = q;
            }
            if (E.ka < 0 || E.kb < 0 || E.ka == side || E.kb == side) throw ApiError{AXP_E_MESH, "emitter edge topology"};
            const int opp = 3 - E.ka - E.kb;
            const double za = m.z[ta], ra = m.r[ta], zb = m.z[hb], rb = m.r[hb];
            const double dz = zb - za, dr = rb - ra;
            const double len = std::sqrt(dz * dz + dr * dr);
            cum += len * (ra + rb) * 0.5;
            E.cdf = cum;
            E.ra = ra; E.rb = rb;
            E.tz = dz / len; E.tr = dr / len;
            // inward normal: towards the face's third node
            double nz = -E.tr, nr = E.tz;
            const double oz = m.z[m.tv[f][opp]] - za, orr = m.r[m.tv[f][opp]] - ra;
            if (nz * oz + nr * orr < 0) { nz = -nz; nr = -nr; }
            E.nz = nz; E.nr = nr;
            E.na = ta; E.nb = hb;
            ee.push_back(E);
        }
        if (ee.empty() || !(cum > 0)) throw ApiError{AXP_E_ARG, "no emitter edge off the axis (AXP_BC_EMITTER)"};
        if (c->inj_edges) dfree(c, c->inj_edges);
        c->inj_edges = upload(c, ee);
        InjParams &p = c->inj;
        p.seed = seed;
        p.per_step = int32_t(per_step);
        p.n_edges = int32_t(ee.size());
        p.species = species;
        p.kq = c->plain ? int32_t(c->pc.kq[species]) : c->ic.kq[species];
        for (int k = 0; k < 3; ++k) p.um[k] = u_mean[k] / kC;
        p.spread = u_spread / kC;
        p.total = cum;
        const unsigned long long st = (unsigned long long)c->step;
        hcheck(hipMemcpyAsync(&c->ds.ctr->inj_step, &st, 8, hipMemcpyHostToDevice, c->stream), "injector step");
        hcheck(hipStreamSynchronize(c->stream), "sync");
        c->inj_on = true;
        return AXP_OK;
    });
}

axp_status axp_step(axp_ctx *c, int32_t n_steps) {
    if (!c || n_steps < 0) return AXP_E_ARG;
    return guarded(c, [&]() -> axp_status {
        require_built(c);
        if (c->guard_tol >= 0.0) guarded_steps(c, n_steps);
        else run_steps(c, n_steps);
        return AXP_OK;
    });
}

axp_status axp_sync(axp_ctx *c) {
    if (!c) return AXP_E_ARG;
    return guarded(c, [&]() -> axp_status {
        require_built(c);
        DevCounters h = read_counters(c);
        c->n_live_host = int64_t(h.n_slots);
        if (h.nan_count) { c->sticky = AXP_E_NAN; c->err = "non-finite particle momentum"; return AXP_E_NAN; }
        if (h.walk_overflow) { c->sticky = AXP_E_WALK; c->err = "particle path exceeded the segment cap"; return AXP_E_WALK; }
        if (h.fixed_overflow) { c->sticky = AXP_E_FIXED_OVERFLOW; c->err = "fixed-point current overflow"; return AXP_E_FIXED_OVERFLOW; }
        return AXP_OK;
    });
}

axp_status axp_diag_get(axp_ctx *c, axp_diag *out) {
    if (!c || !out) return AXP_E_ARG;
    return guarded(c, [&]() -> axp_status {
        require_built(c);
        if (c->last_eval_level != c->step) run_diag(c);
        DevDiag d{};
        hcheck(hipMemcpyAsync(&d, c->ds.diag, sizeof(d), hipMemcpyDeviceToHost, c->stream), "diag");
        DevCounters h = read_counters(c);
        std::memset(out, 0, sizeof(*out));
        out->step = c->step;
        out->n_live = int64_t(d.n_live);     // counted by the charge pass of the diagnostics
        out->n_absorbed = int64_t(h.n_absorbed);
        out->walk_overflow = int64_t(h.walk_overflow);
        out->nan_count = int64_t(h.nan_count);
        out->fixed_overflow = int64_t(h.fixed_overflow);
        out->dce_max_abs = c->plain ? 0 : int64_t(d.dce_max);
        double v;
        std::memcpy(&v, &d.gauss_drift_max_bits, 8); out->gauss_max_drift = v;
        out->gauss_max_abs = d.gauss_abs;
        out->gauss_scale = d.gauss_scale;
        out->Q_total = d.q_total;
        out->W_E_now = d.WE_now;
        out->n_evals = int64_t(d.n_evals);
        out->energy_step = d.energy.level;
        if (d.energy.level >= 0) { out->W_E = d.energy.WE; out->W_B = d.energy.WB; out->W_K = d.energy.WK; }
        if (c->plain) { std::memcpy(&v, &d.dce_rel_max_bits, 8); out->dce_max_rel = v; }
        return axp_sync(c);
    });
}

axp_status axp_get_energies(axp_ctx *c, int64_t capacity, int64_t *n, axp_energy *out) {
    if (!c || !n || capacity < 0 || (capacity > 0 && !out)) return AXP_E_ARG;
    return guarded(c, [&]() -> axp_status {
        require_built(c);
        const DevCounters h = read_counters(c);
        const int64_t written = int64_t(h.energy_count);
        int64_t from = std::max<int64_t>(c->energy_read, written - kEnergyRing);
        const int64_t k = std::min<int64_t>(capacity, written - from);
        *n = k;
        if (k <= 0) { c->energy_read = from; return AXP_OK; }
        std::vector<DevEnergy> ring(kEnergyRing);
        hcheck(hipMemcpyAsync(ring.data(), c->ds.energy, sizeof(DevEnergy) * kEnergyRing, hipMemcpyDeviceToHost,
                              c->stream), "energies");
        hcheck(hipStreamSynchronize(c->stream), "sync");
        for (int64_t i = 0; i < k; ++i) {
            const DevEnergy &e = ring[size_t((from + i) % kEnergyRing)];
            out[i].step = e.level;
            out[i].n_live = e.n_live;
            out[i].W_E = e.WE;
            out[i].W_B = e.WB;
            out[i].W_K = e.WK;
            out[i].Q_total = e.Qtot;
        }
        c->energy_read = from + k;
        return AXP_OK;
    });
}

axp_status axp_get_fields(axp_ctx *c, double *E, double *B) {
    if (!c) return AXP_E_ARG;
    return guarded(c, [&]() -> axp_status {
        require_built(c);
        const HostMesh &m = c->hm;
        if (E && c->plain) {
            std::vector<double> e(m.n1);
            hcheck(hipMemcpyAsync(e.data(), c->dp.E, m.n1 * 8, hipMemcpyDeviceToHost, c->stream), "E");
            hcheck(hipStreamSynchronize(c->stream), "sync");
            for (int k = 0; k < m.n1; ++k) E[k] = e[m.edge_int[k]];
        } else if (E) {
            std::vector<float> e(m.n1);
            hcheck(hipMemcpyAsync(e.data(), c->ds.E, m.n1 * 4, hipMemcpyDeviceToHost, c->stream), "E");
            hcheck(hipStreamSynchronize(c->stream), "sync");
            for (int k = 0; k < m.n1; ++k) E[k] = double(e[m.edge_int[k]]);
        }
        if (B) {
            std::vector<double> b(m.n2);
            hcheck(hipMemcpyAsync(b.data(), c->ds.B, m.n2 * 8, hipMemcpyDeviceToHost, c->stream), "B");
            hcheck(hipStreamSynchronize(c->stream), "sync");
            for (int u = 0; u < m.n2; ++u) B[u] = b[m.tri_int[u]];
        }
        return AXP_OK;
    });
}

axp_status axp_get_sources(axp_ctx *c, double *D, double *J_dt, double *Q) {
    if (!c) return AXP_E_ARG;
    return guarded(c, [&]() -> axp_status {
        require_built(c);
        const HostMesh &m = c->hm;
        if (D) {
            std::vector<double> d(m.n1);
            hcheck(hipMemcpyAsync(d.data(), c->ds.D, m.n1 * 8, hipMemcpyDeviceToHost, c->stream), "D");
            hcheck(hipStreamSynchronize(c->stream), "sync");
            for (int k = 0; k < m.n1; ++k) D[k] = d[m.edge_int[k]];
        }
        if (J_dt && c->plain) {
            std::vector<double> j(m.n1);
            hcheck(hipMemcpyAsync(j.data(), c->dp.Jfx, m.n1 * 8, hipMemcpyDeviceToHost, c->stream), "J");
            hcheck(hipStreamSynchronize(c->stream), "sync");
            for (int k = 0; k < m.n1; ++k) J_dt[k] = j[m.edge_int[k]] * c->pc.qunit;
        } else if (J_dt) {
            std::vector<long long> j(m.n1);
            hcheck(hipMemcpyAsync(j.data(), c->ds.Jfx, m.n1 * 8, hipMemcpyDeviceToHost, c->stream), "J");
            hcheck(hipStreamSynchronize(c->stream), "sync");
            for (int k = 0; k < m.n1; ++k) J_dt[k] = double(j[m.edge_int[k]]) * c->ic.jscale;
        }
        if (Q && c->plain) {
            if (c->last_eval_level != c->step) run_diag(c);
            std::vector<double> q(m.n0);
            hcheck(hipMemcpyAsync(q.data(), c->dp.Q, m.n0 * 8, hipMemcpyDeviceToHost, c->stream), "Q");
            hcheck(hipStreamSynchronize(c->stream), "sync");
            for (int v = 0; v < m.n0; ++v) Q[v] = q[v] * c->pc.qunit;
        } else if (Q) {
            if (c->last_eval_level != c->step) run_diag(c);
            std::vector<long long> q(m.n0);
            hcheck(hipMemcpyAsync(q.data(), c->ds.Qfx, m.n0 * 8, hipMemcpyDeviceToHost, c->stream), "Q");
            hcheck(hipStreamSynchronize(c->stream), "sync");
            for (int v = 0; v < m.n0; ++v) Q[v] = double(q[v]) * c->ic.qscale;
        }
        return AXP_OK;
    });
}

axp_status axp_get_particles(axp_ctx *c, int64_t cap, int64_t *n, double *zr, double *u, int32_t *species) {
    if (!c || !n) return AXP_E_ARG;
    return guarded(c, [&]() -> axp_status {
        require_built(c);
        DevCounters h = read_counters(c);
        int64_t ns = int64_t(h.n_slots);
        const DevState &s = c->ds;
        std::vector<int32_t> cell(ns);
        std::vector<uint32_t> l0(ns), l1(ns);
        std::vector<float> a(ns), b(ns), z(ns);
        std::vector<double> pl0, pl1, pa, pb, pz;
        int cb = s.cur;
        if (ns && c->plain) {
            const DevPlain &p = c->dp;
            pl0.resize(ns); pl1.resize(ns); pa.resize(ns); pb.resize(ns); pz.resize(ns);
            hcheck(hipMemcpyAsync(cell.data(), s.cell[cb], ns * 4, hipMemcpyDeviceToHost, c->stream), "p");
            hcheck(hipMemcpyAsync(pl0.data(), p.l0[cb], ns * 8, hipMemcpyDeviceToHost, c->stream), "p");
            hcheck(hipMemcpyAsync(pl1.data(), p.l1[cb], ns * 8, hipMemcpyDeviceToHost, c->stream), "p");
            hcheck(hipMemcpyAsync(pa.data(), p.ur[cb], ns * 8, hipMemcpyDeviceToHost, c->stream), "p");
            hcheck(hipMemcpyAsync(pb.data(), p.up[cb], ns * 8, hipMemcpyDeviceToHost, c->stream), "p");
            hcheck(hipMemcpyAsync(pz.data(), p.uz[cb], ns * 8, hipMemcpyDeviceToHost, c->stream), "p");
            hcheck(hipStreamSynchronize(c->stream), "sync");
        } else if (ns) {
            hcheck(hipMemcpyAsync(cell.data(), s.cell[cb], ns * 4, hipMemcpyDeviceToHost, c->stream), "p");
            hcheck(hipMemcpyAsync(l0.data(), s.L0[cb], ns * 4, hipMemcpyDeviceToHost, c->stream), "p");
            hcheck(hipMemcpyAsync(l1.data(), s.L1[cb], ns * 4, hipMemcpyDeviceToHost, c->stream), "p");
            hcheck(hipMemcpyAsync(a.data(), s.ur[cb], ns * 4, hipMemcpyDeviceToHost, c->stream), "p");
            hcheck(hipMemcpyAsync(b.data(), s.up[cb], ns * 4, hipMemcpyDeviceToHost, c->stream), "p");
            hcheck(hipMemcpyAsync(z.data(), s.uz[cb], ns * 4, hipMemcpyDeviceToHost, c->stream), "p");
            hcheck(hipStreamSynchronize(c->stream), "sync");
        }
        int64_t live = 0;
        for (int64_t i = 0; i < ns; ++i) live += cell[i] >= 0;
        *n = live;
        if (live > cap) return fail(c, AXP_E_ARG, "capacity too small");
        const HostMesh &m = c->hm;
        int64_t o = 0;
        for (int64_t i = 0; i < ns; ++i) {
            if (cell[i] < 0) continue;
            int t = cell[i] & kCellMask;
            double L[3];
            if (c->plain) {
                L[0] = pl0[i]; L[1] = pl1[i]; L[2] = 1.0 - pl0[i] - pl1[i];
            } else {
                L[0] = double(l0[i]) / double(kLamOne);
                L[1] = double(l1[i]) / double(kLamOne);
                L[2] = double(kLamOne - int64_t(l0[i]) - int64_t(l1[i])) / double(kLamOne);
            }
            double zz = 0, rr = 0;
            for (int k = 0; k < 3; ++k) {
                zz += L[k] * m.z[m.tv[t][k]];
                rr += L[k] * m.r[m.tv[t][k]];
            }
            if (zr) { zr[2 * o] = zz; zr[2 * o + 1] = rr; }
            if (u && c->plain) { u[3 * o] = pa[i] * kC; u[3 * o + 1] = pb[i] * kC; u[3 * o + 2] = pz[i] * kC; }
            else if (u) { u[3 * o] = double(a[i]) * kC; u[3 * o + 1] = double(b[i]) * kC; u[3 * o + 2] = double(z[i]) * kC; }
            if (species) species[o] = (cell[i] >> kCellBits) & 15;
            ++o;
        }
        return AXP_OK;
    });
}

}  // extern "C"

// ------------------------------------------------------------- checkpoints
namespace {

const char kCkptMagic[8] = {'A', 'X', 'P', 'C', 'K', 'P', 'T', '1'};

// FNV-1a over the input mesh and boundary: a checkpoint is restored only
// into a context built from the same inputs.
uint64_t mesh_hash(const axp_ctx *c) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](const void *p, size_t n) {
        const unsigned char *b = static_cast<const unsigned char *>(p);
        for (size_t i = 0; i < n; ++i) { h ^= b[i]; h *= 1099511628211ull; }
    };
    mix(c->in_zr.data(), c->in_zr.size() * sizeof(double));
    mix(c->in_tri.data(), c->in_tri.size() * sizeof(int32_t));
    mix(c->in_seg.data(), c->in_seg.size() * sizeof(int32_t));
    mix(c->in_tag.data(), c->in_tag.size());
    return h;
}

// Autotune cache key: the mesh (a pool: its members'), the particle count
// to the nearest power of two, the precision, the diagnostic cadence, the
// pusher and the GPU architecture.
std::string tune_key(const axp_ctx *c) {
    const DevCounters h = read_counters(const_cast<axp_ctx *>(c));
    const double n = double(h.n_slots);
    const int lg = n > 0 ? int(std::lround(std::log2(n))) : -1;
    hipDeviceProp_t prop{};
    std::string arch = "unknown";
    if (hipGetDeviceProperties(&prop, c->cfg.device) == hipSuccess) arch = prop.gcnArchName;
    for (char &ch : arch)
        if (ch == ' ') ch = '_';
    char buf[160];
    std::snprintf(buf, sizeof(buf), "%016llx/p2^%d/prec%d/diag%d/push%d/%s",
                  (unsigned long long)c->shape_hash, lg, int(c->cfg.precision), int(c->cfg.diag_every),
                  int(c->cfg.pusher), arch.c_str());
    return buf;
}

// The last line of the cache file with this key: "key sort_period window_lead ms_per_step".
bool cache_lookup(const char *path, const std::string &key, int &sp, int &wl) {
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[512];
    bool found = false;
    while (std::fgets(line, sizeof(line), f)) {
        char k[256];
        int a = 0, b = 0;
        double ms = 0;
        if (std::sscanf(line, "%255s %d %d %lf", k, &a, &b, &ms) == 4 && key == k && a >= 1 && a <= 1024 && b >= 0 &&
            b < 512) {
            sp = a;
            wl = b;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

void cache_store(const char *path, const std::string &key, int sp, int wl, double ms) {
    FILE *f = std::fopen(path, "a");
    if (!f) return;                 // an unwritable cache only costs the next run its trials
    char line[512];
    const int len = std::snprintf(line, sizeof(line), "%s %d %d %.6f\n", key.c_str(), sp, wl, ms);
    if (len > 0) std::fwrite(line, 1, size_t(len), f);     // one write: appends from several processes stay whole
    std::fclose(f);
}

struct CkptHeader {
    char magic[8];
    uint64_t mesh;
    int32_t precision, n0, n1, n2;
    double dt;
    int64_t step, last_diag_step, n_slots;
    int32_t g0_set, n_species, inj_on, pad;
    double q_unit, bz;
    DevCounters ctr;
    InjParams inj;
};

struct Blob {
    std::vector<char> bytes;
    template <class T>
    void dev(axp_ctx *c, const T *p, size_t n) {   // device array -> blob
        const size_t o = bytes.size();
        bytes.resize(o + n * sizeof(T));
        if (n) hcheck(hipMemcpyAsync(bytes.data() + o, p, n * sizeof(T), hipMemcpyDeviceToHost, c->stream), "save");
    }
};

template <class T>
void restore(axp_ctx *c, FILE *f, T *p, size_t n) {
    std::vector<T> tmp(n);
    if (n && std::fread(tmp.data(), sizeof(T), n, f) != n) throw ApiError{AXP_E_ARG, "truncated checkpoint"};
    if (n) hcheck(hipMemcpyAsync(p, tmp.data(), n * sizeof(T), hipMemcpyHostToDevice, c->stream), "load");
    hcheck(hipStreamSynchronize(c->stream), "sync");
}

}  // namespace

extern "C" {

axp_status axp_save(axp_ctx *c, const char *path) {
    if (!c || !path) return AXP_E_ARG;
    return guarded(c, [&]() -> axp_status {
        require_built(c);
        if (c->dl.n) throw ApiError{AXP_E_STATE, "checkpoints of contexts with absorbing layers are not supported"};
        const DevCounters h = read_counters(c);
        CkptHeader H{};
        std::memcpy(H.magic, kCkptMagic, 8);
        H.mesh = mesh_hash(c);
        H.precision = c->cfg.precision;
        H.n0 = c->hm.n0; H.n1 = c->hm.n1; H.n2 = c->hm.n2;
        H.dt = c->dt;
        H.step = c->step;
        H.last_diag_step = c->last_eval_level;
        H.n_slots = int64_t(h.n_slots);
        H.g0_set = int32_t(h.g0_set);
        H.n_species = int32_t(c->species.size());
        H.inj_on = c->inj_on;
        H.q_unit = c->q_unit;
        H.bz = c->plain ? c->pc.bz : double(c->ic.bz);
        H.ctr = h;
        H.inj = c->inj;
        const DevState &s = c->ds;
        const size_t n0 = c->hm.n0, n1 = c->hm.n1, n2 = c->hm.n2, np = size_t(h.n_slots);
        const int b = s.cur;
        Blob blob;
        blob.dev(c, s.B, n2); blob.dev(c, s.Bprev, n2); blob.dev(c, s.D, n1); blob.dev(c, s.g0, n0);
        blob.dev(c, s.cell[b], np);
        if (c->plain) {
            const DevPlain &p = c->dp;
            blob.dev(c, p.E, n1); blob.dev(c, p.Jfx, n1); blob.dev(c, p.Qres, n0); blob.dev(c, p.Qprev, n0);
            blob.dev(c, p.l0[b], np); blob.dev(c, p.l1[b], np);
            blob.dev(c, p.ur[b], np); blob.dev(c, p.up[b], np); blob.dev(c, p.uz[b], np);
        } else {
            blob.dev(c, s.E, n1); blob.dev(c, s.D32, n1); blob.dev(c, s.Jfx, n1);
            blob.dev(c, s.Qres, n0); blob.dev(c, s.Qprev, n0);
            blob.dev(c, s.L0[b], np); blob.dev(c, s.L1[b], np);
            blob.dev(c, s.ur[b], np); blob.dev(c, s.up[b], np); blob.dev(c, s.uz[b], np);
        }
        hcheck(hipStreamSynchronize(c->stream), "sync");
        FILE *f = std::fopen(path, "wb");
        if (!f) throw ApiError{AXP_E_ARG, std::string("cannot open ") + path};
        bool ok = std::fwrite(&H, sizeof(H), 1, f) == 1;
        for (const auto &sp : c->species) ok = ok && std::fwrite(&sp, sizeof(sp), 1, f) == 1;
        ok = ok && std::fwrite(blob.bytes.data(), 1, blob.bytes.size(), f) == blob.bytes.size();
        ok = (std::fclose(f) == 0) && ok;
        if (!ok) throw ApiError{AXP_E_ARG, std::string("write failed: ") + path};
        return AXP_OK;
    });
}

axp_status axp_load(axp_ctx *c, const char *path) {
    if (!c || !path) return AXP_E_ARG;
    return guarded(c, [&]() -> axp_status {
        require_built(c);
        FILE *f = std::fopen(path, "rb");
        if (!f) throw ApiError{AXP_E_ARG, std::string("cannot open ") + path};
        struct Closer { FILE *f; ~Closer() { std::fclose(f); } } closer{f};
        CkptHeader H{};
        if (std::fread(&H, sizeof(H), 1, f) != 1 || std::memcmp(H.magic, kCkptMagic, 8) != 0)
            throw ApiError{AXP_E_ARG, "not a checkpoint"};
        if (H.mesh != mesh_hash(c) || H.n0 != c->hm.n0 || H.n1 != c->hm.n1 || H.n2 != c->hm.n2)
            throw ApiError{AXP_E_ARG, "checkpoint of another mesh"};
        if (H.precision != c->cfg.precision || H.dt != c->dt)
            throw ApiError{AXP_E_ARG, "checkpoint of another precision or time step"};
        if (!c->species.empty()) throw ApiError{AXP_E_STATE, "load into a context without species"};
        if (H.n_species < 0 || H.n_species > kMaxSpecies || H.n_slots < 0) throw ApiError{AXP_E_ARG, "corrupt checkpoint"};
        std::vector<Species> sps(H.n_species);
        for (auto &sp : sps)
            if (std::fread(&sp, sizeof(sp), 1, f) != 1) throw ApiError{AXP_E_ARG, "truncated checkpoint"};
        for (const auto &sp : sps) {
            int32_t id = 0;
            const axp_status st = axp_add_species(c, sp.q, sp.m, sp.w, &id);
            if (st != AXP_OK) return st;
        }
        const axp_status st = axp_set_external_bz(c, H.bz);
        if (st != AXP_OK) return st;
        grow_particles(c, std::max<int64_t>(H.n_slots, 1));
        DevState &s = c->ds;
        const size_t n0 = H.n0, n1 = H.n1, n2 = H.n2, np = size_t(H.n_slots);
        const int b = s.cur;
        restore(c, f, s.B, n2); restore(c, f, s.Bprev, n2); restore(c, f, s.D, n1); restore(c, f, s.g0, n0);
        restore(c, f, s.cell[b], np);
        if (c->plain) {
            DevPlain &p = c->dp;
            restore(c, f, p.E, n1); restore(c, f, p.Jfx, n1); restore(c, f, p.Qres, n0); restore(c, f, p.Qprev, n0);
            restore(c, f, p.l0[b], np); restore(c, f, p.l1[b], np);
            restore(c, f, p.ur[b], np); restore(c, f, p.up[b], np); restore(c, f, p.uz[b], np);
        } else {
            restore(c, f, s.E, n1); restore(c, f, s.D32, n1); restore(c, f, s.Jfx, n1);
            restore(c, f, s.Qres, n0); restore(c, f, s.Qprev, n0);
            restore(c, f, s.L0[b], np); restore(c, f, s.L1[b], np);
            restore(c, f, s.ur[b], np); restore(c, f, s.up[b], np); restore(c, f, s.uz[b], np);
        }
        H.ctr.energy_count = 0;          // the energy records are not part of a checkpoint
        hcheck(hipMemcpyAsync(s.ctr, &H.ctr, sizeof(DevCounters), hipMemcpyHostToDevice, c->stream), "counters");
        hcheck(hipStreamSynchronize(c->stream), "sync");
        c->step = H.step;
        c->last_eval_level = H.last_diag_step;
        c->energy_read = 0;
        c->n_live_host = H.n_slots;
        if (H.inj_on) {
            c->inj_on = false;
            double um[3];
            for (int k = 0; k < 3; ++k) um[k] = H.inj.um[k] * kC;
            const axp_status si = axp_set_injector(c, H.inj.species, H.inj.per_step, um, H.inj.spread * kC, H.inj.seed);
            if (si != AXP_OK) return si;
            hcheck(hipMemcpyAsync(&s.ctr->inj_step, &H.ctr.inj_step, 8, hipMemcpyHostToDevice, c->stream), "counters");
            hcheck(hipStreamSynchronize(c->stream), "sync");
        }
        drop_graphs(c);
        return AXP_OK;
    });
}

axp_status axp_set_timing(axp_ctx *c, int32_t on) {
    if (!c) return AXP_E_ARG;
    return guarded(c, [&]() -> axp_status {
        collect_timing(c);
        c->timing = on != 0;
        for (int k = 0; k < AXP_N_PHASES; ++k) { c->phase_ms[k] = 0; c->phase_n[k] = 0; }
        return AXP_OK;
    });
}

axp_status axp_get_timing(axp_ctx *c, double *ms, int64_t *launches) {
    if (!c || !ms || !launches) return AXP_E_ARG;
    return guarded(c, [&]() -> axp_status {
        collect_timing(c);
        for (int k = 0; k < AXP_N_PHASES; ++k) { ms[k] = c->phase_ms[k]; launches[k] = c->phase_n[k]; }
        return AXP_OK;
    });
}

const char *axp_last_error(const axp_ctx *c) { return c ? c->err.c_str() : "null context"; }

void axp_destroy(axp_ctx *c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    for (auto &r : c->ev) { (void)hipEventDestroy(r.second.first); (void)hipEventDestroy(r.second.second); }
    for (auto &r : c->ev_free) { (void)hipEventDestroy(r.first); (void)hipEventDestroy(r.second); }
    for (void *p : std::vector<void *>(c->allocs)) dfree(c, p);
    if (c->owned_model) axp_mlp_destroy(c->owned_model);
    delete c;
}

axp_status axp_set_spai_model(axp_ctx *c, axp_mlp *net, double row_tol, double energy_drift_tol, int32_t iters) {
    if (!c) return AXP_E_ARG;
    if (c->built) return fail(c, AXP_E_STATE, "set the SPAI model before axp_build");
    if (net && (!(row_tol > 0) || !(energy_drift_tol > 0) || iters < 0 || iters > 64))
        return fail(c, AXP_E_ARG, "bad learned-SPAI tolerances");
    if (net && (mlp_level(net) != c->cfg.spai_level || mlp_n_in(net) != kSpaiFeatures))
        return fail(c, AXP_E_ARG, "the network was trained for another SPAI level or feature set");
    c->spai_model = net;
    c->spai_row_tol = row_tol;
    c->spai_energy_tol = energy_drift_tol;
    c->spai_iters = iters;
    return AXP_OK;
}

axp_status axp_set_spai_run_guard(axp_ctx *c, double drift_tol) {
    if (!c || std::isnan(drift_tol)) return AXP_E_ARG;
    if (!c->built) return fail(c, AXP_E_STATE, "axp_build first");
    if (drift_tol < 0.0) { c->guard_tol = -1.0; return AXP_OK; }
    if (c->spai_mode_used != AXP_SPAI_LEARNED)
        return fail(c, AXP_E_STATE, "the run-time guard needs a learned SPAI in use");
    if (c->cfg.diag_every <= 0) return fail(c, AXP_E_STATE, "the run-time guard needs diagnostic steps (diag_every > 0)");
    c->guard_tol = drift_tol;
    c->guard_ref_set = false;
    c->guard_wref = 0.0;
    c->guard_drift = 0.0;
    return AXP_OK;
}

axp_status axp_spai_model_load(axp_ctx *c, const char *model_path) {
    if (!c || !model_path) return AXP_E_ARG;
    if (c->built) return fail(c, AXP_E_STATE, "load the SPAI model before axp_build");
    axp_mlp *net = nullptr;
    const axp_status st = axp_mlp_load(c->cfg.device, c->cfg.hip_stream, model_path, &net);
    if (st != AXP_OK) return fail(c, st, std::string("cannot load the SPAI model ") + model_path);
    const axp_status s2 = axp_set_spai_model(c, net, 0.01, 1e-6, 3);
    if (s2 != AXP_OK) {
        axp_mlp_destroy(net);
        return s2;
    }
    if (c->owned_model) axp_mlp_destroy(c->owned_model);
    c->owned_model = net;
    return AXP_OK;
}

axp_status axp_spai_pairs(axp_ctx *c, int64_t capacity, int64_t *n, float *X, float *y, int32_t *kj) {
    if (!c || !n) return AXP_E_ARG;
    return guarded(c, [&]() -> axp_status {
        require_built(c);
        const HostMesh &m = c->hm;
        ScaledHodge h;
        scaled_hodge(m, h);
        PairSet ps;
        const int nt = int(std::min(16u, std::max(1u, std::thread::hardware_concurrency())));
        spai_pair_features(m, h, c->cfg.spai_level, nt, ps);
        const int64_t np = int64_t(ps.j.size());
        *n = np;
        if (!X && !y && !kj) return AXP_OK;
        if (np > capacity) return fail(c, AXP_E_ARG, "capacity too small");
        const int nf = int(h.fedge.size());
        for (int k = 0; k < nf; ++k) {
            const int ek = h.fedge[k];
            for (int64_t q = ps.ptr[k]; q < ps.ptr[k + 1]; ++q) {
                const int ej = h.fedge[ps.j[q]];
                if (X) std::memcpy(X + q * kSpaiFeatures, &ps.X[size_t(q) * kSpaiFeatures], sizeof(float) * kSpaiFeatures);
                if (y) {
                    // scaled entry M^_kj = M_kj / (s_k s_j) of the context's SPAI (0 where dropped)
                    const int32_t *b = m.M.col.data() + m.M.ptr[ek], *e = m.M.col.data() + m.M.ptr[ek + 1];
                    const int32_t *it = std::lower_bound(b, e, ej);
                    const double v = (it != e && *it == ej) ? m.M.val[it - m.M.col.data()] : 0.0;
                    y[q] = float(v / (h.s[k] * h.s[ps.j[q]]));
                }
                if (kj) { kj[2 * q] = m.edge_can[ek]; kj[2 * q + 1] = m.edge_can[ej]; }
            }
        }
        return AXP_OK;
    });
}

axp_status axp_autotune(axp_ctx *c, int32_t trial_steps, int32_t *sort_period) {
    if (!c || trial_steps < 1) return AXP_E_ARG;
    return guarded(c, [&]() -> axp_status {
        require_built(c);
        if (c->timing) throw ApiError{AXP_E_STATE, "turn timing off before autotuning"};
        const std::string key = tune_key(c);
        const char *cache = std::getenv("AXP_AUTOTUNE_CACHE");
        int sp_c = 0, wl_c = 0;
        if (cache && *cache && cache_lookup(cache, key, sp_c, wl_c)) {
            c->cfg.sort_period = sp_c;
            c->win_lead = wl_c;
            drop_graphs(c);
            if (sort_period) *sort_period = sp_c;
            return AXP_OK;
        }
        hipEvent_t e0, e1;
        hcheck(hipEventCreate(&e0), "event");
        hcheck(hipEventCreate(&e1), "event");
        // time trial_steps real steps (whole graph windows) under the current knobs
        auto trial = [&]() {
            const int sp = c->cfg.sort_period;
            drop_graphs(c);
            // align to the sort period, then one window to build the graph and settle the order
            const int align = int((sp - c->step % sp) % sp);
            run_steps(c, align + 2 * sp);
            const int n = (trial_steps + 2 * sp - 1) / (2 * sp) * (2 * sp);
            hcheck(hipEventRecord(e0, c->stream), "event record");
            run_steps(c, n);
            hcheck(hipEventRecord(e1, c->stream), "event record");
            hcheck(hipEventSynchronize(e1), "event sync");
            float ms = 0.f;
            hcheck(hipEventElapsedTime(&ms, e0, e1), "elapsed");
            return double(ms) / n;
        };
        // knob 1: the sort period; knob 2, at the best period: the lead of the
        // particle kernel's accumulation window
        double best = 1e300;
        int best_sp = c->cfg.sort_period;
        for (int sp : {1, 2, 4, 8, 16}) {
            c->cfg.sort_period = sp;
            const double per = trial();
            if (per < best) { best = per; best_sp = sp; }
        }
        c->cfg.sort_period = best_sp;
        int best_wl = c->win_lead;
        best = 1e300;
        for (int wl : {64, 128, 192, 256, 320}) {
            c->win_lead = wl;
            const double per = trial();
            if (per < best) { best = per; best_wl = wl; }
        }
        c->win_lead = best_wl;
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        drop_graphs(c);
        if (cache && *cache) cache_store(cache, key, best_sp, best_wl, best);
        if (sort_period) *sort_period = best_sp;
        return AXP_OK;
    });
}

}  // extern "C"

// ------------------------------------------------------------------ batch
struct axp_batch {
    axp_ctx *pool = nullptr;
    std::vector<axp_ctx *> ctxs;
    std::vector<int32_t> fo, eo, no;       // face / edge / node offsets of the instances (n + 1)
    std::vector<int64_t> live;             // live particles per instance at the last sync
    int64_t synced_step = 0;               // pool step at the last sync
};

namespace {

// Sorts the pool (compacting absorbed particles) and returns the particle
// range of each instance: after the sort the particles of instance k are
// those of faces [fo[k], fo[k+1]), which are contiguous.
std::vector<int64_t> pool_ranges(axp_batch *b) {
    axp_ctx *p = b->pool;
    const size_t n = b->ctxs.size();
    std::vector<int64_t> start(n + 1, 0);
    if (p->ds.capacity == 0) return start;
    launch_sort(p->dm, p->ds, false, p->stream);
    hcheck(hipGetLastError(), "sort launch");
    // after the scatter cnt[t] holds the end of face t
    for (size_t k = 1; k <= n; ++k) {
        int32_t v = 0;
        const int32_t f = b->fo[k] - 1;
        hcheck(hipMemcpyAsync(&v, p->ds.cnt + f, 4, hipMemcpyDeviceToHost, p->stream), "ranges");
        hcheck(hipStreamSynchronize(p->stream), "sync");
        start[k] = v;
    }
    return start;
}

template <class T>
void d2d(axp_ctx *p, T *dst, const T *src, size_t n) {
    if (n) hcheck(hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyDeviceToDevice, p->stream), "copy");
}

}  // namespace

extern "C" {

axp_status axp_batch_create(axp_ctx *const *ctxs, int32_t n, axp_batch **out) {
    if (!out || !ctxs || n < 1) return AXP_E_ARG;
    *out = nullptr;
    for (int k = 0; k < n; ++k) {
        axp_ctx *c = ctxs[k];
        if (!c) return AXP_E_ARG;
        if (!c->built || c->sticky) return fail(c, AXP_E_STATE, "batch members must be built and error-free");
        if (c->plain) return fail(c, AXP_E_ARG, "batches advance the mixed-precision step only");
        if (c->cfg.device != ctxs[0]->cfg.device) return fail(c, AXP_E_ARG, "batch members must share a device");
        if (c->cfg.pusher != ctxs[0]->cfg.pusher) return fail(c, AXP_E_ARG, "batch members must share a pusher");
        if (c->species.empty()) return fail(c, AXP_E_STATE, "batch members need a species");
        if (c->inj_on) return fail(c, AXP_E_ARG, "batch members cannot carry a continuous injector");
        if (c->fs.n_src > 0 || c->fs.probe_face >= 0)
            return fail(c, AXP_E_ARG, "batch members cannot carry point sources or a probe");
        if (c->dl.n) return fail(c, AXP_E_ARG, "batch members cannot carry absorbing layers");
        if (c->cfg.diag_every != ctxs[0]->cfg.diag_every)
            return fail(c, AXP_E_ARG, "batch members must share a diagnostic cadence");
        if (c->guard_tol >= 0.0) return fail(c, AXP_E_ARG, "batch members cannot carry an armed SPAI run-time guard");
    }
    bool q32 = true;
    for (int k = 0; k < n; ++k) q32 = q32 && ctxs[k]->q32;
    auto *b = new (std::nothrow) axp_batch();
    if (!b) return AXP_E_OOM;
    auto *p = new (std::nothrow) axp_ctx();
    if (!p) { delete b; return AXP_E_OOM; }
    b->pool = p;
    b->ctxs.assign(ctxs, ctxs + n);
    p->cfg = ctxs[0]->cfg;      // diagnostic steps of the pool evaluate all members together
    p->shape_hash = 1469598103934665603ull;
    for (int k = 0; k < n; ++k) {
        for (int q = 0; q < 8; ++q) {
            p->shape_hash ^= (ctxs[k]->shape_hash >> (8 * q)) & 0xFFull;
            p->shape_hash *= 1099511628211ull;
        }
    }
    p->q32 = q32;
    p->stream = ctxs[0]->stream;
    const axp_status st = guarded(p, [&]() -> axp_status {
        hcheck(hipSetDevice(p->cfg.device), "hipSetDevice");
        for (auto *c : b->ctxs) hcheck(hipStreamSynchronize(c->stream), "member sync");
        HostTables h;
        for (int k = 0; k < n; ++k) {
            b->fo.push_back(h.n2); b->eo.push_back(h.n1); b->no.push_back(h.n0);
            if (int64_t(h.n2) + ctxs[k]->hm.n2 >= (int64_t(1) << kCellBits))
                throw ApiError{AXP_E_ARG, "too many faces in the batch"};
            append_instance(h, ctxs[k]->hm, ctxs[k]->dt, k);
        }
        b->fo.push_back(h.n2); b->eo.push_back(h.n1); b->no.push_back(h.n0);
        upload_tables(p, h, true, n);
        std::vector<InstConst> ics(n);
        for (int k = 0; k < n; ++k) ics[k] = ctxs[k]->ic;
        hcheck(hipMemcpyAsync((void *)p->dm.inst, ics.data(), sizeof(InstConst) * n, hipMemcpyHostToDevice, p->stream),
               "inst");
        p->ic = ics[0];
        p->dt = ctxs[0]->dt;
        DevState &ps = p->ds;
        int64_t total = 0;
        std::vector<int64_t> slots(n);
        for (int k = 0; k < n; ++k) {
            slots[k] = int64_t(read_counters(ctxs[k]).n_slots);
            total += slots[k];
        }
        if (total >= (int64_t(1) << 31) - 4096) throw ApiError{AXP_E_ARG, "too many particles in the batch"};
        for (int k = 0; k < n; ++k) {
            const DevState &cs = ctxs[k]->ds;
            const HostMesh &m = ctxs[k]->hm;
            d2d(p, ps.B + b->fo[k], cs.B, m.n2);
            d2d(p, ps.Bprev + b->fo[k], cs.Bprev, m.n2);
            d2d(p, ps.D + b->eo[k], cs.D, m.n1);
            d2d(p, ps.D32 + b->eo[k], cs.D32, m.n1);
            d2d(p, ps.E + b->eo[k], cs.E, m.n1);
            d2d(p, ps.Jfx + b->eo[k], cs.Jfx, m.n1);
            d2d(p, ps.Qres + b->no[k], cs.Qres, m.n0);
        }
        grow_particles(p, std::max<int64_t>(total, 1));
        int64_t o = 0;
        for (int k = 0; k < n; ++k) {
            const DevState &cs = ctxs[k]->ds;
            const int a = cs.cur, q = ps.cur;
            d2d(p, ps.cell[q] + o, cs.cell[a], slots[k]);
            d2d(p, ps.L0[q] + o, cs.L0[a], slots[k]);
            d2d(p, ps.L1[q] + o, cs.L1[a], slots[k]);
            d2d(p, ps.ur[q] + o, cs.ur[a], slots[k]);
            d2d(p, ps.up[q] + o, cs.up[a], slots[k]);
            d2d(p, ps.uz[q] + o, cs.uz[a], slots[k]);
            launch_offset_cells(ps.cell[q] + o, slots[k], b->fo[k], p->stream);
            o += slots[k];
        }
        unsigned long long ns = (unsigned long long)total;
        hcheck(hipMemcpyAsync(&ps.ctr->n_slots, &ns, 8, hipMemcpyHostToDevice, p->stream), "slots");
        std::vector<int64_t> start = pool_ranges(b);
        b->live.resize(n);
        for (int k = 0; k < n; ++k) b->live[k] = start[k + 1] - start[k];
        hcheck(hipStreamSynchronize(p->stream), "batch sync");
        p->built = true;
        return AXP_OK;
    });
    if (st != AXP_OK) {
        for (auto *c : b->ctxs) c->err = "axp_batch_create: " + p->err;
        axp_destroy(p);
        delete b;
        return st;
    }
    *out = b;
    return AXP_OK;
}

axp_status axp_batch_step(axp_batch *b, int32_t n_steps) {
    if (!b || n_steps < 0) return AXP_E_ARG;
    return axp_step(b->pool, n_steps);
}

axp_status axp_batch_sync(axp_batch *b) {
    if (!b) return AXP_E_ARG;
    axp_ctx *p = b->pool;
    axp_status st = axp_sync(p);
    if (st != AXP_OK) {
        for (auto *c : b->ctxs) { c->sticky = st; c->err = "batch: " + p->err; }
        return st;
    }
    return guarded(p, [&]() -> axp_status {
        std::vector<int64_t> start = pool_ranges(b);
        DevState &ps = p->ds;
        for (size_t k = 0; k < b->ctxs.size(); ++k) {
            axp_ctx *c = b->ctxs[k];
            const HostMesh &m = c->hm;
            DevState &cs = c->ds;
            const int64_t nk = start[k + 1] - start[k];
            DevCounters h = read_counters(c);
            h.n_slots = 0;
            h.diag_level1 = 0;            // the pooled steps' charges are not the member's chain
            hcheck(hipMemcpyAsync(cs.ctr, &h, sizeof(h), hipMemcpyHostToDevice, c->stream), "counters");
            grow_particles(c, nk);
            hcheck(hipStreamSynchronize(c->stream), "sync");
            const int a = ps.cur, q = cs.cur;
            const int64_t o = start[k];
            d2d(p, cs.cell[q], ps.cell[a] + o, nk);
            d2d(p, cs.L0[q], ps.L0[a] + o, nk);
            d2d(p, cs.L1[q], ps.L1[a] + o, nk);
            d2d(p, cs.ur[q], ps.ur[a] + o, nk);
            d2d(p, cs.up[q], ps.up[a] + o, nk);
            d2d(p, cs.uz[q], ps.uz[a] + o, nk);
            launch_offset_cells(cs.cell[q], nk, -b->fo[k], p->stream);
            d2d(p, cs.B, ps.B + b->fo[k], m.n2);
            d2d(p, cs.Bprev, ps.Bprev + b->fo[k], m.n2);
            d2d(p, cs.D, ps.D + b->eo[k], m.n1);
            d2d(p, cs.D32, ps.D32 + b->eo[k], m.n1);
            d2d(p, cs.E, ps.E + b->eo[k], m.n1);
            d2d(p, cs.Jfx, ps.Jfx + b->eo[k], m.n1);
            d2d(p, cs.Qres, ps.Qres + b->no[k], m.n0);
            c->step += p->step - b->synced_step;
            c->last_eval_level = -1;
            h.n_slots = (unsigned long long)nk;
            h.n_absorbed += (unsigned long long)std::max<int64_t>(0, b->live[k] - nk);
            h.step = (unsigned long long)c->step;    // the device's level counter follows the pooled steps
            hcheck(hipMemcpyAsync(cs.ctr, &h, sizeof(h), hipMemcpyHostToDevice, p->stream), "counters");
            hcheck(hipStreamSynchronize(p->stream), "sync");
            c->n_live_host = nk;
            b->live[k] = nk;
        }
        b->synced_step = p->step;
        return AXP_OK;
    });
}

axp_status axp_batch_autotune(axp_batch *b, int32_t trial_steps, int32_t *sort_period) {
    if (!b) return AXP_E_ARG;
    return axp_autotune(b->pool, trial_steps, sort_period);
}

axp_status axp_batch_set_timing(axp_batch *b, int32_t on) { return b ? axp_set_timing(b->pool, on) : AXP_E_ARG; }

axp_status axp_batch_get_timing(axp_batch *b, double *ms, int64_t *launches) {
    return b ? axp_get_timing(b->pool, ms, launches) : AXP_E_ARG;
}

axp_status axp_batch_info(axp_batch *b, int64_t *n_faces, int64_t *n_edges, int64_t *n_particles, int64_t *step) {
    if (!b) return AXP_E_ARG;
    axp_ctx *p = b->pool;
    return guarded(p, [&]() -> axp_status {
        if (n_faces) *n_faces = p->dm.n2;
        if (n_edges) *n_edges = p->dm.n1;
        if (n_particles) *n_particles = int64_t(read_counters(p).n_slots);
        if (step) *step = p->step;
        return AXP_OK;
    });
}

const char *axp_batch_last_error(const axp_batch *b) { return b ? b->pool->err.c_str() : "null batch"; }

void axp_batch_destroy(axp_batch *b) {
    if (!b) return;
    axp_destroy(b->pool);
    delete b;
}

}  // extern "C"
