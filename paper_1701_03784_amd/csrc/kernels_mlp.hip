// Kernels of the small network that predicts entries of the Jacobi-scaled
// SPAI matrix (learned SPAI): forward, backward, weight gradients and Adam.
//
// Network: NIN -> H (tanh) -> ... -> H (tanh) -> 1 (linear), L hidden
// layers.  Parameters (FP32, one vector): layer 0 W[H][NIN], b[H]; layers
// 1..L-1 W[H][H], b[H]; output W[H], b.  Activations and deltas are stored
// sample-major ([layer][sample][H]).
//
//   k_mlp_fwd     one sample per thread; all parameters staged in LDS and
//                 read as wave-uniform broadcasts
//   k_mlp_bwd     one sample per thread: output residual, deltas of every
//                 hidden layer (tanh' = 1 - h^2), loss partial sums
//   k_mlp_wgrad   dW_l = sum_i delta_l[i]^T h_{l-1}[i] over a chunk of
//                 samples: a dense contraction over the sample axis on the
//                 matrix cores (v_mfma_f32_16x16x4_f32), one 16x16 tile per
//                 wave at a time; biases and the output layer by FMA
//   k_mlp_reduce  sum of the per-chunk partial gradients in chunk order
//                 (deterministic), divided by the total sample weight
//   k_mlp_adam    Adam with bias-corrected moments
#include <hip/hip_runtime.h>

#include "mlp.h"

namespace axp {

namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kMlpWG = 256;
static_assert(kMlpWG == kMlpLossBlock, "one loss partial per workgroup");

template <int NIN, int H>
__device__ __forceinline__ int out_offset(int L) {
    return H * NIN + H + (L - 1) * (H * H + H);
}

template <int NIN, int H>
__global__ __launch_bounds__(kMlpWG) void k_mlp_fwd(const float *__restrict__ X, int64_t n,
                                                    const float *__restrict__ params, int np, int L,
                                                    float *__restrict__ act, float *__restrict__ out) {
    extern __shared__ float sp[];
    for (int q = threadIdx.x; q < np; q += kMlpWG) sp[q] = params[q];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kMlpWG + threadIdx.x;
    if (i >= n) return;
    float x[NIN];
#pragma unroll
    for (int c = 0; c < NIN; c += 4) {
        const float4 v = *reinterpret_cast<const float4 *>(X + i * NIN + c);
        x[c] = v.x; x[c + 1] = v.y; x[c + 2] = v.z; x[c + 3] = v.w;
    }
    float h[H];
#pragma unroll
    for (int o = 0; o < H; ++o) {
        float z = sp[H * NIN + o];
#pragma unroll
        for (int c = 0; c < NIN; ++c) z = fmaf(sp[o * NIN + c], x[c], z);
        h[o] = tanhf(z);
    }
    if (act) {
        float *a = act + i * H;
#pragma unroll
        for (int o = 0; o < H; o += 4) *reinterpret_cast<float4 *>(a + o) = make_float4(h[o], h[o + 1], h[o + 2], h[o + 3]);
    }
    int off = H * NIN + H;
    for (int l = 1; l < L; ++l) {
        float g[H];
#pragma unroll
        for (int o = 0; o < H; ++o) {
            float z = sp[off + H * H + o];
#pragma unroll
            for (int c = 0; c < H; ++c) z = fmaf(sp[off + o * H + c], h[c], z);
            g[o] = tanhf(z);
        }
#pragma unroll
        for (int o = 0; o < H; ++o) h[o] = g[o];
        if (act) {
            float *a = act + ((int64_t)l * n + i) * H;
#pragma unroll
            for (int o = 0; o < H; o += 4) *reinterpret_cast<float4 *>(a + o) = make_float4(h[o], h[o + 1], h[o + 2], h[o + 3]);
        }
        off += H * H + H;
    }
    float z = sp[off + H];
#pragma unroll
    for (int c = 0; c < H; ++c) z = fmaf(sp[off + c], h[c], z);
    out[i] = z;
}

__device__ __forceinline__ double block_sum_mlp(double v, double *sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int off = kMlpWG / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

template <int NIN, int H>
__global__ __launch_bounds__(kMlpWG) void k_mlp_bwd(int64_t n, const float *__restrict__ params, int np, int L,
                                                    const float *__restrict__ act, const float *__restrict__ pred,
                                                    const float *__restrict__ y, const float *__restrict__ w,
                                                    float *__restrict__ delta, float *__restrict__ dout,
                                                    double *__restrict__ loss_part) {
    extern __shared__ float sp[];
    __shared__ double sh[kMlpWG];
    for (int q = threadIdx.x; q < np; q += kMlpWG) sp[q] = params[q];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * kMlpWG + threadIdx.x;
    const bool valid = i < n;
    float r = 0.f, wi = 0.f;
    if (valid) {
        r = pred[i] - y[i];
        wi = w[i];
    }
    const double lw = block_sum_mlp((double)wi * (double)r * (double)r, sh);
    const double sw = block_sum_mlp((double)wi, sh);
    if (threadIdx.x == 0) {
        loss_part[2 * blockIdx.x] = lw;
        loss_part[2 * blockIdx.x + 1] = sw;
    }
    if (!valid) return;
    const float d0 = 2.0f * wi * r;                  // dL/dp times sum(w)
    dout[i] = d0;
    const int off_out = out_offset<NIN, H>(L);
    float d[H], h[H];
    {
        const float *a = act + ((int64_t)(L - 1) * n + i) * H;
#pragma unroll
        for (int o = 0; o < H; o += 4) {
            const float4 v = *reinterpret_cast<const float4 *>(a + o);
            h[o] = v.x; h[o + 1] = v.y; h[o + 2] = v.z; h[o + 3] = v.w;
        }
#pragma unroll
        for (int o = 0; o < H; ++o) d[o] = d0 * sp[off_out + o] * (1.0f - h[o] * h[o]);
        float *dd = delta + ((int64_t)(L - 1) * n + i) * H;
#pragma unroll
        for (int o = 0; o < H; o += 4) *reinterpret_cast<float4 *>(dd + o) = make_float4(d[o], d[o + 1], d[o + 2], d[o + 3]);
    }
    for (int l = L - 1; l >= 1; --l) {
        const int off = H * NIN + H + (l - 1) * (H * H + H);     // W_l
        const float *a = act + ((int64_t)(l - 1) * n + i) * H;
#pragma unroll
        for (int c = 0; c < H; c += 4) {
            const float4 v = *reinterpret_cast<const float4 *>(a + c);
            h[c] = v.x; h[c + 1] = v.y; h[c + 2] = v.z; h[c + 3] = v.w;
        }
        float g[H];
#pragma unroll
        for (int c = 0; c < H; ++c) g[c] = 0.0f;
#pragma unroll
        for (int o = 0; o < H; ++o) {
#pragma unroll
            for (int c = 0; c < H; ++c) g[c] = fmaf(d[o], sp[off + o * H + c], g[c]);
        }
#pragma unroll
        for (int c = 0; c < H; ++c) d[c] = g[c] * (1.0f - h[c] * h[c]);
        float *dd = delta + ((int64_t)(l - 1) * n + i) * H;
#pragma unroll
        for (int c = 0; c < H; c += 4) *reinterpret_cast<float4 *>(dd + c) = make_float4(d[c], d[c + 1], d[c + 2], d[c + 3]);
    }
}

// Per-chunk partial gradients: part[chunk][np].
template <int NIN, int H>
__global__ __launch_bounds__(kMlpWG) void k_mlp_wgrad(const float *__restrict__ X, int64_t n, int L, int np,
                                                      const float *__restrict__ act, const float *__restrict__ delta,
                                                      const float *__restrict__ dout, int chunk,
                                                      float *__restrict__ part) {
    const int64_t i_beg = (int64_t)blockIdx.x * chunk;
    const int64_t i_end = i_beg + chunk < n ? i_beg + chunk : n;
    float *pb = part + (int64_t)blockIdx.x * np;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = lane >> 4;
    // weight tiles: layer 0 has (H/16) x (NIN/16) tiles, the others (H/16)^2
    constexpr int T0 = (H / 16) * (NIN / 16);
    constexpr int T1 = (H / 16) * (H / 16);
    const int n_tiles = T0 + (L - 1) * T1;
    for (int t = wave; t < n_tiles; t += kMlpWG / 64) {
        int l, tt, nin, woff;
        const float *hin;
        if (t < T0) {
            l = 0; tt = t; nin = NIN; woff = 0; hin = X;
        } else {
            l = 1 + (t - T0) / T1; tt = (t - T0) % T1; nin = H;
            woff = H * NIN + H + (l - 1) * (H * H + H);
            hin = act + (int64_t)(l - 1) * n * H;
        }
        const int o0 = (tt / (nin / 16)) * 16, c0 = (tt % (nin / 16)) * 16;
        const float *dl = delta + (int64_t)l * n * H;
        floatx4 acc = {0.f, 0.f, 0.f, 0.f};
        for (int64_t i0 = i_beg; i0 < i_end; i0 += 4) {
            const int64_t ii = i0 + lk;
            float a = 0.f, b = 0.f;
            if (ii < i_end) {
                a = dl[ii * H + o0 + lr];        // A[o][k] = delta_l[i0 + k][o]
                b = hin[ii * nin + c0 + lr];     // B[k][c] = h_{l-1}[i0 + k][c]
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
        }
        // D[o][c]: lane holds column c0 + (lane % 16), rows o0 + 4 (lane / 16) + r
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int o = o0 + 4 * lk + r, c = c0 + lr;
            pb[woff + o * nin + c] = acc[r];
        }
    }
    // biases of the hidden layers, output weights and bias
    const int n_items = L * H + H + 1;
    const int off_out = out_offset<NIN, H>(L);
    for (int q = threadIdx.x; q < n_items; q += kMlpWG) {
        float s = 0.f;
        if (q < L * H) {
            const int l = q / H, o = q % H;
            const float *dl = delta + (int64_t)l * n * H + o;
            for (int64_t i = i_beg; i < i_end; ++i) s += dl[i * H];
            const int boff = l == 0 ? H * NIN : H * NIN + H + (l - 1) * (H * H + H) + H * H;
            pb[boff + o] = s;
        } else if (q < L * H + H) {
            const int c = q - L * H;
            const float *a = act + (int64_t)(L - 1) * n * H + c;
            for (int64_t i = i_beg; i < i_end; ++i) s = fmaf(dout[i], a[i * H], s);
            pb[off_out + c] = s;
        } else {
            for (int64_t i = i_beg; i < i_end; ++i) s += dout[i];
            pb[off_out + H] = s;
        }
    }
}

__global__ __launch_bounds__(kMlpWG) void k_mlp_loss(const double *__restrict__ loss_part, int nblk,
                                                     double *__restrict__ out) {
    __shared__ double sh[kMlpWG];
    double a = 0.0, b = 0.0;
    for (int q = threadIdx.x; q < nblk; q += kMlpWG) {
        a += loss_part[2 * q];
        b += loss_part[2 * q + 1];
    }
    a = block_sum_mlp(a, sh);
    b = block_sum_mlp(b, sh);
    if (threadIdx.x == 0) {
        out[0] = b > 0.0 ? a / b : 0.0;
        out[1] = b;
    }
}

__global__ __launch_bounds__(kMlpWG) void k_mlp_reduce(const float *__restrict__ part, int nchunk, int np,
                                                       const double *__restrict__ loss, float *__restrict__ grad) {
    const int p = blockIdx.x * kMlpWG + threadIdx.x;
    if (p >= np) return;
    double s = 0.0;
    for (int b = 0; b < nchunk; ++b) s += (double)part[(int64_t)b * np + p];
    const double sw = loss[1];
    grad[p] = (float)(sw > 0.0 ? s / sw : 0.0);
}

__global__ __launch_bounds__(kMlpWG) void k_mlp_adam(float *__restrict__ params, const float *__restrict__ grad,
                                                     float *__restrict__ m, float *__restrict__ v, int np, float lr,
                                                     float b1, float b2, float eps, float c1, float c2) {
    const int p = blockIdx.x * kMlpWG + threadIdx.x;
    if (p >= np) return;
    const float g = grad[p];
    const float mm = b1 * m[p] + (1.0f - b1) * g;
    const float vv = b2 * v[p] + (1.0f - b2) * g * g;
    m[p] = mm;
    v[p] = vv;
    const float mh = mm / c1, vh = vv / c2;
    params[p] -= lr * mh / (sqrtf(vh) + eps);
}

inline unsigned nbk(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

bool mlp_shape_supported(int n_in, int n_hidden, int n_layers) {
    return n_in == 16 && (n_hidden == 32 || n_hidden == 64) && n_layers >= 1 && n_layers <= 4;
}

void launch_mlp_forward(const MlpShape &s, const float *X, int64_t n, const float *params, float *act, float *out,
                        hipStream_t st) {
    if (n <= 0) return;
    const size_t lds = sizeof(float) * s.np;
    if (s.H == 64)
        hipLaunchKernelGGL((k_mlp_fwd<16, 64>), dim3(nbk(n, kMlpWG)), dim3(kMlpWG), lds, st, X, n, params, s.np, s.L, act, out);
    else
        hipLaunchKernelGGL((k_mlp_fwd<16, 32>), dim3(nbk(n, kMlpWG)), dim3(kMlpWG), lds, st, X, n, params, s.np, s.L, act, out);
}

void launch_mlp_loss_grad(const MlpShape &s, const float *X, const float *y, const float *w, int64_t n,
                          const float *params, MlpScratch &k, float *grad, double *loss_dev, hipStream_t st) {
    const size_t lds = sizeof(float) * s.np;
    const unsigned nb = nbk(n, kMlpWG);
    launch_mlp_forward(s, X, n, params, k.act, k.pred, st);
    if (s.H == 64)
        hipLaunchKernelGGL((k_mlp_bwd<16, 64>), dim3(nb), dim3(kMlpWG), lds, st, n, params, s.np, s.L, k.act, k.pred, y, w,
                           k.delta, k.dout, k.loss_part);
    else
        hipLaunchKernelGGL((k_mlp_bwd<16, 32>), dim3(nb), dim3(kMlpWG), lds, st, n, params, s.np, s.L, k.act, k.pred, y, w,
                           k.delta, k.dout, k.loss_part);
    const int nchunk = (int)nbk(n, kMlpChunk);
    if (s.H == 64)
        hipLaunchKernelGGL((k_mlp_wgrad<16, 64>), dim3(nchunk), dim3(kMlpWG), 0, st, X, n, s.L, s.np, k.act, k.delta, k.dout,
                           kMlpChunk, k.part);
    else
        hipLaunchKernelGGL((k_mlp_wgrad<16, 32>), dim3(nchunk), dim3(kMlpWG), 0, st, X, n, s.L, s.np, k.act, k.delta, k.dout,
                           kMlpChunk, k.part);
    hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(kMlpWG), 0, st, k.loss_part, (int)nb, loss_dev);
    hipLaunchKernelGGL(k_mlp_reduce, dim3(nbk(s.np, kMlpWG)), dim3(kMlpWG), 0, st, k.part, nchunk, s.np, loss_dev, grad);
}

void launch_mlp_adam(int np, float *params, const float *grad, float *m, float *v, float lr, float b1, float b2,
                     float eps, float c1, float c2, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_adam, dim3(nbk(np, kMlpWG)), dim3(kMlpWG), 0, st, params, grad, m, v, np, lr, b1, b2, eps, c1,
                       c2);
}

}  // namespace axp
