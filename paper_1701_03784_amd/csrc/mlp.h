// Learned-SPAI network: shapes, scratch buffers and kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace axp {

constexpr int kMlpChunk = 512;     // samples per partial-gradient chunk
constexpr int kMlpLossBlock = 256; // samples per loss partial (one workgroup)

struct MlpShape {
    int n_in = 16, H = 64, L = 2;  // inputs, hidden width, hidden layers
    int np = 0;                    // parameter count
};

inline int mlp_param_count(int n_in, int H, int L) { return H * n_in + H + (L - 1) * (H * H + H) + H + 1; }

// Device scratch of a loss/gradient evaluation over n samples.
struct MlpScratch {
    int64_t cap = 0;               // samples
    float *act = nullptr;          // [L][cap][H]
    float *delta = nullptr;        // [L][cap][H]
    float *pred = nullptr;         // [cap]
    float *dout = nullptr;         // [cap]
    double *loss_part = nullptr;   // [2 * blocks]
    float *part = nullptr;         // [chunks][np]
};

bool mlp_shape_supported(int n_in, int n_hidden, int n_layers);
void launch_mlp_forward(const MlpShape &s, const float *X, int64_t n, const float *params, float *act, float *out,
                        hipStream_t st);
// loss_dev[0] = weighted mean squared error, loss_dev[1] = sum of weights; grad = dL/dparams
void launch_mlp_loss_grad(const MlpShape &s, const float *X, const float *y, const float *w, int64_t n,
                          const float *params, MlpScratch &k, float *grad, double *loss_dev, hipStream_t st);
void launch_mlp_adam(int np, float *params, const float *grad, float *m, float *v, float lr, float b1, float b2,
                     float eps, float c1, float c2, hipStream_t st);

}  // namespace axp
