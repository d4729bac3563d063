// Native trainer of the learned-SPAI network: the training loop over the
// library's own entry points (a context per mesh for the plain SPAI's pair
// features and targets, then Adam steps of the device MLP on minibatches).
// The network, its features and the refinement it feeds are described with
// axp_set_spai_model in include/axpic.h.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <fstream>
#include <numeric>
#include <random>
#include <string>
#include <vector>

#include "../../include/axpic.h"

namespace {

constexpr int kFeatures = 16;
constexpr int kHidden = 64, kLayers = 2, kLevel = 3;
constexpr int kEpochs = 40, kBatch = 4096;
constexpr double kLr0 = 3e-3, kLr1 = 1e-4;
constexpr int64_t kPairsPerMesh = 150000;

struct MeshFile {
    std::vector<double> zr;
    std::vector<int32_t> tri, seg;
    std::vector<uint8_t> tag;
};

// Text mesh: "axpic-mesh 1", then "n_nodes n_tris n_seg", then the node
// coordinates (z rho), the triangles (three node ids, counter-clockwise)
// and the boundary segments (two node ids and an AXP_BC_* tag).
bool read_mesh(const std::string &path, MeshFile &m) {
    std::ifstream f(path);
    if (!f) return false;
    std::string magic;
    int version = 0;
    long long nn = 0, nt = 0, ns = 0;
    f >> magic >> version >> nn >> nt >> ns;
    if (!f || magic != "axpic-mesh" || version != 1 || nn < 3 || nt < 1 || ns < 3 || nn > (1ll << 30) ||
        nt > (1ll << 30) || ns > (1ll << 30))
        return false;
    m.zr.resize(size_t(2 * nn));
    for (auto &v : m.zr) f >> v;
    m.tri.resize(size_t(3 * nt));
    for (auto &v : m.tri) f >> v;
    m.seg.resize(size_t(2 * ns));
    m.tag.resize(size_t(ns));
    for (long long i = 0; i < ns; ++i) {
        int t = 0;
        f >> m.seg[2 * i] >> m.seg[2 * i + 1] >> t;
        m.tag[i] = uint8_t(t);
    }
    return bool(f);
}

// Pair features and targets of one mesh's plain SPAI, at most kPairsPerMesh
// of them (a seeded sample without replacement).
axp_status mesh_pairs(const MeshFile &m, std::mt19937_64 &rng, std::vector<float> &X, std::vector<float> &y) {
    axp_config cfg;
    axp_config_default(&cfg);
    cfg.spai_level = kLevel;
    cfg.dt = 1e-30;                 // no time stepping: the stability check is moot
    axp_ctx *c = nullptr;
    axp_status st = axp_create(&cfg, &c);
    if (st != AXP_OK) return st;
    int64_t n = 0;
    std::vector<float> Xm, ym;
    do {
        if ((st = axp_set_mesh(c, int32_t(m.zr.size() / 2), m.zr.data(), int32_t(m.tri.size() / 3), m.tri.data())))
            break;
        if ((st = axp_set_boundary(c, int32_t(m.tag.size()), m.seg.data(), m.tag.data()))) break;
        if ((st = axp_build(c))) break;
        if ((st = axp_spai_pairs(c, 0, &n, nullptr, nullptr, nullptr))) break;
        Xm.resize(size_t(n) * kFeatures);
        ym.resize(size_t(n));
        st = axp_spai_pairs(c, n, &n, Xm.data(), ym.data(), nullptr);
    } while (false);
    axp_destroy(c);
    if (st != AXP_OK) return st;
    std::vector<int64_t> idx(static_cast<size_t>(n));
    std::iota(idx.begin(), idx.end(), 0);
    int64_t keep = n;
    if (n > kPairsPerMesh) {
        for (int64_t i = 0; i < kPairsPerMesh; ++i) {            // partial Fisher-Yates
            std::uniform_int_distribution<int64_t> d(i, n - 1);
            std::swap(idx[size_t(i)], idx[size_t(d(rng))]);
        }
        keep = kPairsPerMesh;
    }
    for (int64_t i = 0; i < keep; ++i) {
        const int64_t k = idx[size_t(i)];
        X.insert(X.end(), Xm.begin() + k * kFeatures, Xm.begin() + (k + 1) * kFeatures);
        y.push_back(ym[size_t(k)]);
    }
    return AXP_OK;
}

}  // namespace

extern "C" axp_status axp_spai_model_train(const char *mesh_list, const char *out_model, uint64_t seed) {
    if (!mesh_list || !out_model) return AXP_E_ARG;
    std::ifstream list(mesh_list);
    if (!list) return AXP_E_ARG;
    std::vector<std::string> paths;
    for (std::string line; std::getline(list, line);) {
        const size_t a = line.find_first_not_of(" \t\r");
        if (a == std::string::npos || line[a] == '#') continue;
        paths.push_back(line.substr(a, line.find_last_not_of(" \t\r") - a + 1));
    }
    if (paths.empty()) return AXP_E_ARG;
    std::mt19937_64 rng(seed);
    std::vector<float> X, y;
    for (const auto &p : paths) {
        MeshFile m;
        if (!read_mesh(p, m)) return AXP_E_ARG;
        const axp_status st = mesh_pairs(m, rng, X, y);
        if (st != AXP_OK) return st;
    }
    const int64_t n = int64_t(y.size());
    if (n == 0) return AXP_E_ARG;
    // one seeded shuffle, then sequential minibatches
    std::vector<int64_t> perm(static_cast<size_t>(n));
    std::iota(perm.begin(), perm.end(), 0);
    std::shuffle(perm.begin(), perm.end(), rng);
    std::vector<float> Xs(X.size()), ys(static_cast<size_t>(n)), ws(static_cast<size_t>(n), 1.0f);
    for (int64_t i = 0; i < n; ++i) {
        std::copy_n(X.begin() + perm[size_t(i)] * kFeatures, kFeatures, Xs.begin() + i * kFeatures);
        ys[size_t(i)] = y[size_t(perm[size_t(i)])];
    }
    float *dX = nullptr, *dy = nullptr, *dw = nullptr;
    axp_mlp *net = nullptr;
    axp_status st = AXP_OK;
    do {
        if (hipMalloc(&dX, Xs.size() * sizeof(float)) != hipSuccess || hipMalloc(&dy, ys.size() * sizeof(float)) != hipSuccess ||
            hipMalloc(&dw, ws.size() * sizeof(float)) != hipSuccess) {
            st = AXP_E_OOM;
            break;
        }
        if (hipMemcpy(dX, Xs.data(), Xs.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(dy, ys.data(), ys.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(dw, ws.data(), ws.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
            st = AXP_E_HIP;
            break;
        }
        if ((st = axp_mlp_create(0, nullptr, kFeatures, kHidden, kLayers, kLevel, seed, &net))) break;
        const int64_t per_epoch = (n + kBatch - 1) / kBatch, steps = int64_t(kEpochs) * per_epoch;
        int64_t k = 0;
        for (int ep = 0; ep < kEpochs && st == AXP_OK; ++ep)
            for (int64_t b0 = 0; b0 < n && st == AXP_OK; b0 += kBatch, ++k) {
                const int64_t nb = std::min<int64_t>(kBatch, n - b0);
                st = axp_mlp_loss_grad(net, dX + b0 * kFeatures, dy + b0, dw + b0, nb, nullptr, nullptr);
                const double a = double(k) / double(std::max<int64_t>(1, steps - 1));
                if (st == AXP_OK) st = axp_mlp_adam_step(net, kLr0 * (1.0 - a) + kLr1 * a, 0.9, 0.999, 1e-8);
            }
        if (st == AXP_OK) st = axp_mlp_save(net, out_model);
    } while (false);
    if (net) axp_mlp_destroy(net);
    (void)hipFree(dX);
    (void)hipFree(dy);
    (void)hipFree(dw);
    return st;
}
