// C ABI of the learned-SPAI network (include/axpic.h): parameters, device
// forward pass, loss and gradient, Adam, files.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <random>
#include <string>
#include <vector>

#include "../../include/axpic.h"
#include "mlp.h"

using namespace axp;

struct axp_mlp {
    int device = 0;
    hipStream_t stream = nullptr;
    int level = 3;
    MlpShape s;
    float *params = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
    double *loss = nullptr;
    MlpScratch k;
    void *static_scratch = nullptr;   // this device's copy of `scratch` (device address)
    int64_t t = 0;            // Adam steps taken
    std::string err;
};

namespace {

int hfail(axp_mlp *n, hipError_t e, const char *what) {
    if (n) n->err = std::string(what) + ": " + hipGetErrorString(e);
    return AXP_E_HIP;
}

#define MLP_HIP(net, call, what)                              \
    do {                                                      \
        hipError_t e_ = (call);                               \
        if (e_ != hipSuccess) return hfail(net, e_, what);    \
    } while (0)

void free_scratch(MlpScratch &k) {
    (void)hipFree(k.act); (void)hipFree(k.delta); (void)hipFree(k.pred); (void)hipFree(k.dout);
    (void)hipFree(k.loss_part); (void)hipFree(k.part);
    k = MlpScratch{};
}

int ensure_scratch(axp_mlp *net, int64_t n) {
    if (n <= net->k.cap) return AXP_OK;
    free_scratch(net->k);
    const int64_t cap = std::max<int64_t>(n, 1024);
    const int64_t nb = (cap + kMlpLossBlock - 1) / kMlpLossBlock, nc = (cap + kMlpChunk - 1) / kMlpChunk;
    MlpScratch &k = net->k;
    const size_t ah = sizeof(float) * size_t(net->s.L) * size_t(cap) * size_t(net->s.H);
    MLP_HIP(net, hipMalloc(&k.act, ah), "hipMalloc");
    MLP_HIP(net, hipMalloc(&k.delta, ah), "hipMalloc");
    MLP_HIP(net, hipMalloc(&k.pred, sizeof(float) * cap), "hipMalloc");
    MLP_HIP(net, hipMalloc(&k.dout, sizeof(float) * cap), "hipMalloc");
    MLP_HIP(net, hipMalloc(&k.loss_part, sizeof(double) * 2 * nb), "hipMalloc");
    MLP_HIP(net, hipMalloc(&k.part, sizeof(float) * size_t(nc) * net->s.np), "hipMalloc");
    k.cap = cap;
    return AXP_OK;
}

const char kMagic[8] = {'A', 'X', 'P', 'M', 'L', 'P', '1', '\0'};

// ---- static scratch of axp_mlp_loss_grad_noalloc
// One array per device, held until the process ends.  In host code
// `scratch` only stands for the symbol: its device address on a given device
// comes from hipGetSymbolAddress with that device current, done once per
// device when the first network is created there.
constexpr size_t kStaticScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxDevices] = {};

// The calling thread's current device must be net->device.
int resolve_static_scratch(axp_mlp *net) {
    if (net->device >= kMaxDevices) {
        net->err = "device ordinal beyond the static-scratch table";
        return AXP_E_ARG;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_addr[net->device]) {
        void *p = nullptr;
        MLP_HIP(net, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        if (!p) {
            net->err = "hipGetSymbolAddress(scratch) returned a null address";
            return AXP_E_HIP;
        }
        g_scratch_addr[net->device] = p;
    }
    net->static_scratch = g_scratch_addr[net->device];
    return AXP_OK;
}

// Places the loss/gradient scratch of n samples at base (256-byte aligned
// pieces, the layout ensure_scratch allocates) and returns the bytes used.
size_t carve_scratch(const MlpShape &s, int64_t n, unsigned char *base, MlpScratch &k) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        unsigned char *p = base + off;
        off += (bytes + 255) & ~size_t(255);
        return p;
    };
    const size_t nn = size_t(n);
    const size_t nb = (nn + kMlpLossBlock - 1) / kMlpLossBlock, nc = (nn + kMlpChunk - 1) / kMlpChunk;
    const size_t ah = sizeof(float) * size_t(s.L) * nn * size_t(s.H);
    k.cap = n;
    k.act = reinterpret_cast<float *>(take(ah));
    k.delta = reinterpret_cast<float *>(take(ah));
    k.pred = reinterpret_cast<float *>(take(sizeof(float) * nn));
    k.dout = reinterpret_cast<float *>(take(sizeof(float) * nn));
    k.loss_part = reinterpret_cast<double *>(take(sizeof(double) * 2 * nb));
    k.part = reinterpret_cast<float *>(take(sizeof(float) * nc * size_t(s.np)));
    return off;
}

}  // namespace

extern "C" {

axp_status axp_mlp_create(int32_t device, void *hip_stream, int32_t n_in, int32_t n_hidden, int32_t n_layers,
                          int32_t spai_level, uint64_t seed, axp_mlp **out) {
    if (!out) return AXP_E_ARG;
    *out = nullptr;
    if (!mlp_shape_supported(n_in, n_hidden, n_layers) || spai_level < 1 || spai_level > 3) return AXP_E_ARG;
    if (hipSetDevice(device) != hipSuccess) return AXP_E_HIP;
    auto *net = new (std::nothrow) axp_mlp();
    if (!net) return AXP_E_OOM;
    net->device = device;
    net->stream = (hipStream_t)hip_stream;
    net->level = spai_level;
    net->s.n_in = n_in; net->s.H = n_hidden; net->s.L = n_layers;
    net->s.np = mlp_param_count(n_in, n_hidden, n_layers);
    if (resolve_static_scratch(net) != AXP_OK) {
        axp_mlp_destroy(net);
        return AXP_E_HIP;
    }
    const size_t pb = sizeof(float) * net->s.np;
    if (hipMalloc(&net->params, pb) != hipSuccess || hipMalloc(&net->grad, pb) != hipSuccess ||
        hipMalloc(&net->m, pb) != hipSuccess || hipMalloc(&net->v, pb) != hipSuccess ||
        hipMalloc(&net->loss, 2 * sizeof(double)) != hipSuccess) {
        axp_mlp_destroy(net);
        return AXP_E_OOM;
    }
    // Glorot-uniform weights, zero biases
    std::vector<float> p(net->s.np, 0.0f);
    std::mt19937_64 rng(seed);
    int off = 0;
    auto layer = [&](int no, int ni) {
        const float a = std::sqrt(6.0f / float(no + ni));
        std::uniform_real_distribution<float> u(-a, a);
        for (int q = 0; q < no * ni; ++q) p[off + q] = u(rng);
        off += no * ni + no;
    };
    layer(n_hidden, n_in);
    for (int l = 1; l < n_layers; ++l) layer(n_hidden, n_hidden);
    layer(1, n_hidden);
    const axp_status st = axp_mlp_set_params(net, p.data());
    if (st != AXP_OK) { axp_mlp_destroy(net); return st; }
    *out = net;
    return AXP_OK;
}

int64_t axp_mlp_n_params(const axp_mlp *net) { return net ? net->s.np : 0; }

axp_status axp_mlp_set_params(axp_mlp *net, const float *params) {
    if (!net || !params) return AXP_E_ARG;
    for (int q = 0; q < net->s.np; ++q)
        if (!std::isfinite(params[q])) { net->err = "non-finite parameter"; return AXP_E_NAN; }
    const size_t pb = sizeof(float) * net->s.np;
    MLP_HIP(net, hipMemcpyAsync(net->params, params, pb, hipMemcpyHostToDevice, net->stream), "params");
    MLP_HIP(net, hipMemsetAsync(net->m, 0, pb, net->stream), "adam m");
    MLP_HIP(net, hipMemsetAsync(net->v, 0, pb, net->stream), "adam v");
    MLP_HIP(net, hipStreamSynchronize(net->stream), "sync");
    net->t = 0;
    return AXP_OK;
}

axp_status axp_mlp_get_params(const axp_mlp *net, float *params) {
    if (!net || !params) return AXP_E_ARG;
    auto *mut = const_cast<axp_mlp *>(net);
    MLP_HIP(mut, hipMemcpyAsync(params, net->params, sizeof(float) * net->s.np, hipMemcpyDeviceToHost, net->stream),
            "params");
    MLP_HIP(mut, hipStreamSynchronize(net->stream), "sync");
    return AXP_OK;
}

axp_status axp_mlp_forward(axp_mlp *net, const float *X, int64_t n, float *y) {
    if (!net || n < 0 || (n > 0 && (!X || !y))) return AXP_E_ARG;
    launch_mlp_forward(net->s, X, n, net->params, nullptr, y, net->stream);
    MLP_HIP(net, hipGetLastError(), "forward launch");
    return AXP_OK;
}

axp_status axp_mlp_loss_grad(axp_mlp *net, const float *X, const float *y, const float *w, int64_t n, double *loss,
                             float *grad) {
    if (!net || n < 1 || !X || !y || !w) return AXP_E_ARG;
    const int st = ensure_scratch(net, n);
    if (st != AXP_OK) return st;
    launch_mlp_loss_grad(net->s, X, y, w, n, net->params, net->k, net->grad, net->loss, net->stream);
    MLP_HIP(net, hipGetLastError(), "loss/grad launch");
    if (loss || grad) {
        double l[2] = {0, 0};
        MLP_HIP(net, hipMemcpyAsync(l, net->loss, sizeof(l), hipMemcpyDeviceToHost, net->stream), "loss");
        if (grad)
            MLP_HIP(net, hipMemcpyAsync(grad, net->grad, sizeof(float) * net->s.np, hipMemcpyDeviceToHost, net->stream),
                    "grad");
        MLP_HIP(net, hipStreamSynchronize(net->stream), "sync");
        if (loss) *loss = l[0];
        if (!(l[1] > 0)) { net->err = "sum of sample weights is not positive"; return AXP_E_ARG; }
    }
    return AXP_OK;
}

axp_status axp_mlp_loss_grad_noalloc(axp_mlp *net, const float *X, const float *y, const float *w, int64_t n,
                                     double *loss_dev, float *grad_dev) {
    if (!net || n < 1 || !X || !y || !w || !loss_dev || !grad_dev) return AXP_E_ARG;
    if (!net->static_scratch) {
        net->err = "the static scratch of this device was not resolved";
        return AXP_E_STATE;
    }
    // every sample takes more than one byte, so this bound keeps the size arithmetic in range
    if (n > int64_t(kStaticScratchBytes)) {
        net->err = "n = " + std::to_string(n) + " samples exceed the " + std::to_string(kStaticScratchBytes) +
                   "-byte static scratch";
        return AXP_E_ARG;
    }
    MlpScratch k;
    const size_t need = carve_scratch(net->s, n, static_cast<unsigned char *>(net->static_scratch), k);
    if (need > kStaticScratchBytes) {
        net->err = "n = " + std::to_string(n) + " samples need " + std::to_string(need) +
                   " bytes of scratch; the static scratch holds " + std::to_string(kStaticScratchBytes);
        return AXP_E_ARG;
    }
    launch_mlp_loss_grad(net->s, X, y, w, n, net->params, k, grad_dev, loss_dev, net->stream);
    MLP_HIP(net, hipGetLastError(), "loss/grad launch");
    return AXP_OK;
}

axp_status axp_mlp_adam_step(axp_mlp *net, double lr, double beta1, double beta2, double eps) {
    if (!net || !(lr > 0) || beta1 < 0 || beta1 >= 1 || beta2 < 0 || beta2 >= 1 || !(eps > 0)) return AXP_E_ARG;
    net->t += 1;
    const double c1 = 1.0 - std::pow(beta1, double(net->t)), c2 = 1.0 - std::pow(beta2, double(net->t));
    launch_mlp_adam(net->s.np, net->params, net->grad, net->m, net->v, float(lr), float(beta1), float(beta2), float(eps),
                    float(c1), float(c2), net->stream);
    MLP_HIP(net, hipGetLastError(), "adam launch");
    return AXP_OK;
}

axp_status axp_mlp_info(const axp_mlp *net, int32_t *n_in, int32_t *n_hidden, int32_t *n_layers, int32_t *spai_level,
                        int64_t *adam_steps) {
    if (!net) return AXP_E_ARG;
    if (n_in) *n_in = net->s.n_in;
    if (n_hidden) *n_hidden = net->s.H;
    if (n_layers) *n_layers = net->s.L;
    if (spai_level) *spai_level = net->level;
    if (adam_steps) *adam_steps = net->t;
    return AXP_OK;
}

axp_status axp_mlp_save(const axp_mlp *net, const char *path) {
    if (!net || !path) return AXP_E_ARG;
    std::vector<float> p(net->s.np);
    axp_status st = axp_mlp_get_params(net, p.data());
    if (st != AXP_OK) return st;
    FILE *f = std::fopen(path, "wb");
    if (!f) return AXP_E_ARG;
    const int32_t hdr[5] = {net->s.n_in, net->s.H, net->s.L, net->level, net->s.np};
    bool ok = std::fwrite(kMagic, 1, 8, f) == 8 && std::fwrite(hdr, sizeof(hdr), 1, f) == 1 &&
              std::fwrite(p.data(), sizeof(float), p.size(), f) == p.size();
    ok = (std::fclose(f) == 0) && ok;
    return ok ? AXP_OK : AXP_E_ARG;
}

axp_status axp_mlp_load(int32_t device, void *hip_stream, const char *path, axp_mlp **out) {
    if (!path || !out) return AXP_E_ARG;
    *out = nullptr;
    FILE *f = std::fopen(path, "rb");
    if (!f) return AXP_E_ARG;
    char magic[8];
    int32_t hdr[5];
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kMagic, 8) == 0 && std::fread(hdr, sizeof(hdr), 1, f) == 1;
    std::vector<float> p;
    if (ok && mlp_shape_supported(hdr[0], hdr[1], hdr[2]) && hdr[4] == mlp_param_count(hdr[0], hdr[1], hdr[2])) {
        p.resize(hdr[4]);
        ok = std::fread(p.data(), sizeof(float), p.size(), f) == p.size();
    } else {
        ok = false;
    }
    std::fclose(f);
    if (!ok) return AXP_E_ARG;
    axp_mlp *net = nullptr;
    axp_status st = axp_mlp_create(device, hip_stream, hdr[0], hdr[1], hdr[2], hdr[3], 0, &net);
    if (st != AXP_OK) return st;
    st = axp_mlp_set_params(net, p.data());
    if (st != AXP_OK) { axp_mlp_destroy(net); return st; }
    *out = net;
    return AXP_OK;
}

const char *axp_mlp_last_error(const axp_mlp *net) { return net ? net->err.c_str() : "null network"; }

void axp_mlp_destroy(axp_mlp *net) {
    if (!net) return;
    (void)hipStreamSynchronize(net->stream);
    free_scratch(net->k);
    (void)hipFree(net->params); (void)hipFree(net->grad); (void)hipFree(net->m); (void)hipFree(net->v);
    (void)hipFree(net->loss);
    delete net;
}

}  // extern "C"

// Library-internal: inference on host features (learned SPAI assembly).
namespace axp {

int mlp_predict_host(axp_mlp *net, const float *X, int64_t n, float *y, std::string &err) {
    if (n <= 0) return AXP_OK;
    float *dX = nullptr, *dy = nullptr;
    auto cleanup = [&]() { (void)hipFree(dX); (void)hipFree(dy); };
    if (hipMalloc(&dX, sizeof(float) * size_t(n) * net->s.n_in) != hipSuccess || hipMalloc(&dy, sizeof(float) * n) != hipSuccess) {
        cleanup();
        err = "hipMalloc of the feature buffer failed";
        return AXP_E_OOM;
    }
    hipError_t e = hipMemcpyAsync(dX, X, sizeof(float) * size_t(n) * net->s.n_in, hipMemcpyHostToDevice, net->stream);
    if (e == hipSuccess) {
        launch_mlp_forward(net->s, dX, n, net->params, nullptr, dy, net->stream);
        e = hipGetLastError();
    }
    if (e == hipSuccess) e = hipMemcpyAsync(y, dy, sizeof(float) * n, hipMemcpyDeviceToHost, net->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(net->stream);
    cleanup();
    if (e != hipSuccess) { err = std::string("network inference: ") + hipGetErrorString(e); return AXP_E_HIP; }
    return AXP_OK;
}

int mlp_level(const axp_mlp *net) { return net->level; }
int mlp_n_in(const axp_mlp *net) { return net->s.n_in; }

}  // namespace axp
