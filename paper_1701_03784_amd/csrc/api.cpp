// C ABI of the library (include/axpic.h): context lifecycle, setup uploads,
// the step loop, diagnostics and read-back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
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
    int64_t last_diag_step = -1;  // step at which Qprev was computed
    bool g0_set = false;
    int64_t n_live_host = 0;
    // injector
    bool inj_on = false;
    // per-phase timing
    bool timing = false;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev;   // pending (phase, start, stop)
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_free;
    double phase_ms[AXP_N_PHASES] = {0};
    int64_t phase_n[AXP_N_PHASES] = {0};
};

namespace {

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

void grow_particles(axp_ctx *c, int64_t need) {
    DevState &s = c->ds;
    if (need <= s.capacity) return;
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
        dfree(c, p.mv_p); dfree(c, p.mv_c); dfree(c, p.mv_l0); dfree(c, p.mv_l1); dfree(c, p.mv_fz); dfree(c, p.mv_fr);
        dfree(c, s.mv_n);
        s.mv_n = zeros<int32_t>(c, cap / 1024 + 1);
        p.mv_p = zeros<int32_t>(c, cap); p.mv_c = zeros<int32_t>(c, cap);
        p.mv_l0 = zeros<double>(c, cap); p.mv_l1 = zeros<double>(c, cap);
        p.mv_fz = zeros<double>(c, cap); p.mv_fr = zeros<double>(c, cap);
        s.capacity = cap;
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
    dfree(c, s.mv_p); dfree(c, s.mv_c); dfree(c, s.mv_l0); dfree(c, s.mv_l1); dfree(c, s.mv_fz); dfree(c, s.mv_fr);
    dfree(c, s.mv_n);
    s.mv_n = zeros<int32_t>(c, cap / 1024 + 1);
    s.mv_p = zeros<int32_t>(c, cap); s.mv_c = zeros<int32_t>(c, cap);
    s.mv_l0 = zeros<int32_t>(c, cap); s.mv_l1 = zeros<int32_t>(c, cap);
    s.mv_fz = zeros<float>(c, cap); s.mv_fr = zeros<float>(c, cap);
    s.capacity = cap;
}

struct PhaseScope {
    axp_ctx *c;
    int phase;
    hipEvent_t b = nullptr, e = nullptr;
    PhaseScope(axp_ctx *ctx, int ph) : c(ctx), phase(ph) {
        if (!c->timing) return;
        if (!c->ev_free.empty()) {
            b = c->ev_free.back().first;
            e = c->ev_free.back().second;
            c->ev_free.pop_back();
        } else {
            hcheck(hipEventCreate(&b), "event");
            hcheck(hipEventCreate(&e), "event");
        }
        hcheck(hipEventRecord(b, c->stream), "event record");
    }
    ~PhaseScope() {
        if (!c->timing || !b) return;
        (void)hipEventRecord(e, c->stream);
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

void run_diag(axp_ctx *c) {
    bool have_prev = (c->last_diag_step == c->step - 1) && c->step > 0;
    {
        PhaseScope ps(c, AXP_PHASE_DIAG);
        if (c->plain) launch_diag_plain(c->dm, c->ds, c->dp, c->pc, have_prev, !c->g0_set, c->stream);
        else launch_diag(c->dm, c->ds, have_prev, !c->g0_set, c->stream);
    }
    c->g0_set = true;
    c->last_diag_step = c->step;
}

void build_device(axp_ctx *c) {
    HostMesh &m = c->hm;
    DevMesh &d = c->dm;
    d.n0 = m.n0; d.n1 = m.n1; d.n2 = m.n2; d.n_inst = 1;
    const double S = double(kLamOne);
    std::vector<float4> gS(m.n2), rho4(m.n2);
    std::vector<int4> nbr(m.n2), tedge(m.n2), tnodes(m.n2);
    std::vector<double> Hdt(m.n2);
    for (int t = 0; t < m.n2; ++t) {
        const auto &g = m.grad[t];
        gS[t] = make_float4(float(S * g[0]), float(S * g[1]), float(S * g[2]), float(S * g[3]));
        rho4[t] = make_float4(float(m.r[m.tv[t][0]]), float(m.r[m.tv[t][1]]), float(m.r[m.tv[t][2]]),
                              float(1.0 / (2.0 * m.area[t])));
        nbr[t] = make_int4(m.tnbr[t][0], m.tnbr[t][1], m.tnbr[t][2], int(m.tnbr_map[t]));
        int sb = 0;
        for (int k = 0; k < 3; ++k) if (m.tsign[t][k] < 0) sb |= 1 << k;
        tedge[t] = make_int4(m.tedge[t][0], m.tedge[t][1], m.tedge[t][2], sb);
        tnodes[t] = make_int4(m.tv[t][0], m.tv[t][1], m.tv[t][2], 0);
        Hdt[t] = c->dt * m.H[t];
    }
    std::vector<int4> etri(m.n1);
    for (int e = 0; e < m.n1; ++e) {
        int L = m.etri[e][0], R = m.etri[e][1];
        int kl = m.eside[e][0], kr = R >= 0 ? m.eside[e][1] : 0;
        int packed = kl | (kr << 2);
        if (m.tsign[L][kl] < 0) packed |= 16;
        if (R >= 0 && m.tsign[R][kr] < 0) packed |= 32;
        if (m.efree[e]) packed |= 64;
        etri[e] = make_int4(L, R, packed, 0);
    }
    // SPAI in sliced ELL, 64 rows per slice, column-major within a slice
    const int ns = (m.n1 + 63) / 64;
    std::vector<int64_t> sptr(ns + 1, 0);
    std::vector<int32_t> slen(ns, 0);
    for (int sl = 0; sl < ns; ++sl) {
        int mx = 0;
        for (int i = sl * 64; i < std::min(m.n1, sl * 64 + 64); ++i) mx = std::max<int>(mx, int(m.M.ptr[i + 1] - m.M.ptr[i]));
        slen[sl] = mx;
        sptr[sl + 1] = sptr[sl] + int64_t(mx) * 64;
    }
    std::vector<float> mval(sptr[ns], 0.0f);
    std::vector<double> mvald(c->plain ? sptr[ns] : 0, 0.0);
    std::vector<int32_t> mcol(sptr[ns], 0);
    for (int sl = 0; sl < ns; ++sl)
        for (int lane = 0; lane < 64; ++lane) {
            int i = sl * 64 + lane;
            int64_t o = sptr[sl] + lane;
            int j = 0;
            if (i < m.n1)
                for (int64_t q = m.M.ptr[i]; q < m.M.ptr[i + 1]; ++q, ++j) {
                    mval[o + 64 * j] = float(m.M.val[q]);
                    if (c->plain) mvald[o + 64 * j] = m.M.val[q];
                    mcol[o + 64 * j] = m.M.col[q];
                }
            for (; j < slen[sl]; ++j) mcol[o + 64 * j] = i < m.n1 ? i : 0;
        }
    d.gS = upload(c, gS); d.rho4 = upload(c, rho4); d.nbr = upload(c, nbr);
    d.tedge = upload(c, tedge); d.tnodes = upload(c, tnodes); d.Hdt = upload(c, Hdt);
    d.tinst = nullptr;
    d.etri = upload(c, etri);
    d.nptr = upload(c, m.nptr); d.nedge = upload(c, m.nedge); d.nsign = upload(c, m.nsign);
    d.nfree = upload(c, m.nfree); d.ninst = nullptr;
    d.m_sptr = upload(c, sptr); d.m_slen = upload(c, slen); d.m_col = upload(c, mcol);
    d.m_val = c->plain ? nullptr : upload(c, mval);
    d.a_ptr = upload(c, m.A.ptr); d.a_col = upload(c, m.A.col); d.a_val = upload(c, m.A.val);
    std::memset(&c->ic, 0, sizeof(InstConst));
    c->ic.dt = c->dt;
    c->ic.cdt = float(kC * c->dt);
    d.inst = (InstConst *)dalloc(c, sizeof(InstConst));
    upload_inst(c);
    DevState &s = c->ds;
    s.B = zeros<double>(c, m.n2); s.Bprev = zeros<double>(c, m.n2); s.HBdt = zeros<double>(c, m.n2);
    s.D = zeros<double>(c, m.n1);
    s.g0 = zeros<double>(c, m.n0);
    if (c->plain) {
        DevPlain &p = c->dp;
        std::vector<double4> grad(m.n2), rho(m.n2);
        for (int t = 0; t < m.n2; ++t) {
            const auto &g = m.grad[t];
            grad[t] = make_double4(g[0], g[1], g[2], g[3]);
            rho[t] = make_double4(m.r[m.tv[t][0]], m.r[m.tv[t][1]], m.r[m.tv[t][2]], 1.0 / (2.0 * m.area[t]));
        }
        p.grad = upload(c, grad); p.rho = upload(c, rho); p.m_val = upload(c, mvald);
        p.E = zeros<double>(c, m.n1);
        p.f0 = zeros<double4>(c, m.n2); p.f1 = zeros<double4>(c, m.n2);
        p.Jloc = zeros<double>(c, size_t(3) * m.n2); p.Jfx = zeros<double>(c, m.n1);
        p.Qres = zeros<double>(c, m.n0); p.Q = zeros<double>(c, m.n0); p.Qprev = zeros<double>(c, m.n0);
        std::memset(&c->pc, 0, sizeof(PlainConst));
        c->pc.dt = c->dt;
        c->pc.cdt = kC * c->dt;
    } else {
        s.f0 = zeros<float4>(c, m.n2); s.f1 = zeros<float4>(c, m.n2);
        s.Jloc = zeros<unsigned long long>(c, size_t(3) * m.n2);
        s.D32 = zeros<float>(c, m.n1); s.E = zeros<float>(c, m.n1);
        s.Jfx = zeros<long long>(c, m.n1);
        s.Qres = zeros<long long>(c, m.n0); s.Qfx = zeros<long long>(c, m.n0); s.Qprev = zeros<long long>(c, m.n0);
    }
    s.cnt = zeros<int32_t>(c, size_t(m.n2) + 1);
    s.blk = zeros<int32_t>(c, size_t(m.n2) / 1024 + 2);
    s.ctr = zeros<DevCounters>(c, 1);
    s.diag = zeros<DevDiag>(c, 1);
    s.kin_part = zeros<double>(c, 1024);
    s.capacity = 0;
    s.cur = 0;
    hcheck(hipStreamSynchronize(c->stream), "build sync");
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
}

axp_status axp_create(const axp_config *cfg, axp_ctx **out) {
    if (!cfg || !out) return AXP_E_ARG;
    *out = nullptr;
    if (cfg->precision != AXP_PREC_MIXED && cfg->precision != AXP_PREC_PLAIN_FP64) return AXP_E_ARG;
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
        build_spai(m, c->cfg.spai_level, c->cfg.spai_drop_tol, nt);
        c->dt_cfl = cfl_dt(m, 400);
        c->dt = c->cfg.dt > 0 ? c->cfg.dt : c->cfg.cfl_fraction * c->dt_cfl;
        if (!(c->dt > 0) || c->dt > c->dt_cfl * (1.0 + 1e-9))
            throw ApiError{AXP_E_UNSTABLE, "dt " + std::to_string(c->dt) + " exceeds the stability limit " +
                                               std::to_string(c->dt_cfl)};
        build_locator(m);
        c->hm = std::move(m);
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
        c->g0_set = false;
        c->last_diag_step = -1;
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
                    dl0[i] = lam[0] / s;
                    dl1[i] = lam[1] / s;
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
        c->last_diag_step = -1;
        return AXP_OK;
    });
}

axp_status axp_set_injector(axp_ctx *c, int32_t, int64_t, const double *, double, uint64_t) {
    if (!c) return AXP_E_ARG;
    return fail(c, AXP_E_STATE, "continuous injection is not available in this build");
}

axp_status axp_step(axp_ctx *c, int32_t n_steps) {
    if (!c || n_steps < 0) return AXP_E_ARG;
    return guarded(c, [&]() -> axp_status {
        require_built(c);
        for (int i = 0; i < n_steps && c->plain; ++i) {
            const bool sort_now = (c->step + 1) % c->cfg.sort_period == 0;
            { PhaseScope ps(c, AXP_PHASE_FACE); launch_tri_pass_plain(c->dm, c->ds, c->dp, c->pc, c->stream); }
            if (sort_now) { PhaseScope ps(c, AXP_PHASE_SORT); launch_sort_zero(c->dm, c->ds, c->stream); }
            { PhaseScope ps(c, AXP_PHASE_PARTICLES); launch_push_plain(c->dm, c->ds, c->dp, c->pc, sort_now, c->stream); }
            {
                PhaseScope ps(c, AXP_PHASE_WALK);
                launch_walk_plain(c->dm, c->ds, c->dp, c->pc, c->cfg.max_walk, sort_now, c->stream);
            }
            { PhaseScope ps(c, AXP_PHASE_EDGE); launch_edge_pass_plain(c->dm, c->ds, c->dp, c->pc, c->stream); }
            { PhaseScope ps(c, AXP_PHASE_SPMV); launch_spmv_plain(c->dm, c->ds, c->dp, c->stream); }
            ++c->step;
            if (sort_now) { PhaseScope ps(c, AXP_PHASE_SORT); launch_sort_plain(c->dm, c->ds, c->dp, true, c->stream); }
            if (c->cfg.diag_every > 0 && c->step % c->cfg.diag_every == 0) run_diag(c);
            if (c->ev.size() > 4096) collect_timing(c);
        }
        for (int i = 0; i < n_steps && !c->plain; ++i) {
            const bool sort_now = (c->step + 1) % c->cfg.sort_period == 0;
            { PhaseScope ps(c, AXP_PHASE_FACE); launch_tri_pass(c->dm, c->ds, c->stream); }
            if (sort_now) { PhaseScope ps(c, AXP_PHASE_SORT); launch_sort_zero(c->dm, c->ds, c->stream); }
            const bool single = c->dm.tinst == nullptr && c->ic.n_species == 1 && c->ic.kq[0] == 1;
            {
                PhaseScope ps(c, AXP_PHASE_PARTICLES);
                launch_push(c->dm, c->ds, sort_now, single ? &c->ic : nullptr, c->stream);
            }
            {
                PhaseScope ps(c, AXP_PHASE_WALK);
                launch_walk(c->dm, c->ds, c->cfg.max_walk, sort_now, single ? &c->ic : nullptr, c->stream);
            }
            { PhaseScope ps(c, AXP_PHASE_EDGE); launch_edge_pass(c->dm, c->ds, true, c->stream); }
            { PhaseScope ps(c, AXP_PHASE_SPMV); launch_spmv(c->dm, c->ds, c->stream); }
            ++c->step;
            if (sort_now) {
                PhaseScope ps(c, AXP_PHASE_SORT);
                launch_sort(c->dm, c->ds, true, c->stream);
            }
            if (c->cfg.diag_every > 0 && c->step % c->cfg.diag_every == 0) run_diag(c);
            if (c->ev.size() > 4096) collect_timing(c);
        }
        hcheck(hipGetLastError(), "step launch");
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
        if (c->last_diag_step != c->step) run_diag(c);
        DevDiag d{};
        hcheck(hipMemcpyAsync(&d, c->ds.diag, sizeof(d), hipMemcpyDeviceToHost, c->stream), "diag");
        DevCounters h = read_counters(c);
        std::memset(out, 0, sizeof(*out));
        out->step = c->step;
        // live count: slots minus dead ones is not tracked per step; count after compaction
        out->n_live = int64_t(h.n_slots);
        out->n_absorbed = int64_t(h.n_absorbed);
        out->walk_overflow = int64_t(h.walk_overflow);
        out->nan_count = int64_t(h.nan_count);
        out->fixed_overflow = int64_t(h.fixed_overflow);
        out->dce_max_abs = int64_t(d.dce_max);
        double v;
        std::memcpy(&v, &d.gauss_drift_bits, 8); out->gauss_max_drift = v;
        std::memcpy(&v, &d.gauss_abs_bits, 8); out->gauss_max_abs = v;
        std::memcpy(&v, &d.gauss_scale_bits, 8); out->gauss_scale = v;
        out->W_E = d.WE; out->W_B = d.WB; out->W_K = d.WK; out->Q_total = d.Qtot;
        if (c->plain) {
            double da, qm;
            std::memcpy(&da, &d.dce_abs_bits, 8);
            std::memcpy(&qm, &d.qmax_bits, 8);
            out->dce_max_abs = 0;
            out->dce_max_rel = qm > 0 ? da / qm : da;
        }
        return axp_sync(c);
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
            if (c->last_diag_step != c->step) run_diag(c);
            std::vector<double> q(m.n0);
            hcheck(hipMemcpyAsync(q.data(), c->dp.Q, m.n0 * 8, hipMemcpyDeviceToHost, c->stream), "Q");
            hcheck(hipStreamSynchronize(c->stream), "sync");
            for (int v = 0; v < m.n0; ++v) Q[v] = q[v] * c->pc.qunit;
        } else if (Q) {
            if (c->last_diag_step != c->step) run_diag(c);
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

axp_status axp_save(axp_ctx *c, const char *) { return c ? fail(c, AXP_E_STATE, "checkpoints not available in this build") : AXP_E_ARG; }
axp_status axp_load(axp_ctx *c, const char *) { return c ? fail(c, AXP_E_STATE, "checkpoints not available in this build") : AXP_E_ARG; }

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
    for (auto &r : c->ev) { (void)hipEventDestroy(r.second.first); (void)hipEventDestroy(r.second.second); }
    for (auto &r : c->ev_free) { (void)hipEventDestroy(r.first); (void)hipEventDestroy(r.second); }
    for (void *p : std::vector<void *>(c->allocs)) dfree(c, p);
    delete c;
}

axp_status axp_batch_create(axp_ctx *const *, int32_t, axp_batch **out) {
    if (out) *out = nullptr;
    return AXP_E_STATE;
}
axp_status axp_batch_step(axp_batch *, int32_t) { return AXP_E_STATE; }
axp_status axp_batch_sync(axp_batch *) { return AXP_E_STATE; }
void axp_batch_destroy(axp_batch *) {}

}  // extern "C"
