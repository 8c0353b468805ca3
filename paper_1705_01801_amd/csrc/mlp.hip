// Surrogate MLP: dense layers with tanh hidden activations and a linear
// output, BF16 weights and activations, FP32 accumulation on MFMA, FP32
// master weights updated by Adam.  Trained on spectra produced by the batched
// LBM to map horn-profile parameters to resonant frequencies.
//
// Precision points (the CPU check follows the same ones): the input x, the
// weights used in products and the hidden activations are rounded to BF16;
// products accumulate in FP32; biases, pre-activations, loss and gradients
// are FP32; the output-layer gradient and the hidden-layer gradients are
// rounded to BF16 before they enter a product.
//
// GEMMs use v_mfma_f32_16x16x32_bf16: a wave computes one 16 x 16 tile of
// C = A B over K in steps of 32; lane l supplies row/column l % 16 and eight
// k values of group l / 16; the accumulator holds rows 4 (l / 16) + j,
// column l % 16.  Operands are read with arbitrary strides (the matrices are
// at most max_batch x 256) and out-of-range elements are read as zero.
#include <cmath>
#include <vector>

#include "host_util.h"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

using lbw::fail;
using lbw::hip_fail;

namespace {

constexpr int kEpiF32 = 0;           // out_f32 = acc
constexpr int kEpiBiasF32 = 1;       // out_f32 = acc + bias
constexpr int kEpiBiasTanhBF16 = 2;  // out_bf16 = bf16(tanh(acc + bias))

template <int EPI>
__global__ __launch_bounds__(256) void gemm_kernel(const __bf16* __restrict__ A, int64_t sam, int64_t sak,
                                                   const __bf16* __restrict__ B, int64_t sbk, int64_t sbn, int M,
                                                   int N, int K, const float* __restrict__ bias,
                                                   float* __restrict__ outf, __bf16* __restrict__ outb,
                                                   int64_t ldo) {
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int m0 = (blockIdx.x * 2 + (wave & 1)) * 16;
    const int n0 = (blockIdx.y * 2 + (wave >> 1)) * 16;
    const int r = lane % 16, grp = lane / 16;
    floatx4 acc = {0.f, 0.f, 0.f, 0.f};
    const int am = m0 + r, bn = n0 + r;
    for (int k0 = 0; k0 < K; k0 += 32) {
        bf16x8 a, b;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = k0 + 8 * grp + j;
            a[j] = (am < M && k < K) ? A[am * sam + k * sak] : (__bf16)0.0f;
            b[j] = (bn < N && k < K) ? B[k * sbk + bn * sbn] : (__bf16)0.0f;
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int m = m0 + 4 * grp + j, n = n0 + r;
        if (m < M && n < N) {
            const float v = acc[j];
            if (EPI == kEpiF32) outf[m * ldo + n] = v;
            else if (EPI == kEpiBiasF32) outf[m * ldo + n] = v + bias[n];
            else outb[m * ldo + n] = (__bf16)tanhf(v + bias[n]);
        }
    }
}

__global__ void to_bf16_kernel(const float* __restrict__ in, __bf16* __restrict__ out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = (__bf16)in[i];
}

// loss = sum w (y - t)^2 * inv_wsum;  dz = bf16(2 w (y - t) inv_wsum)
__global__ void loss_grad_kernel(const float* __restrict__ y, const float* __restrict__ t, const float* __restrict__ w,
                                 int64_t n, float inv_wsum, __bf16* __restrict__ dz, float* __restrict__ partial) {
    __shared__ float red[256];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    float l = 0.f;
    if (i < n) {
        const float d = y[i] - t[i];
        const float ww = w ? w[i] : 1.0f;
        l = ww * d * d;
        dz[i] = (__bf16)(2.0f * ww * d * inv_wsum);
    }
    red[threadIdx.x] = l;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void loss_sum_kernel(const float* __restrict__ partial, int n, float inv_wsum, float* __restrict__ loss) {
    __shared__ float red[256];
    float s = 0.f;
    for (int i = threadIdx.x; i < n; i += 256) s += partial[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = red[0] * inv_wsum;
}

// hidden layer: dz = bf16(dy (1 - y^2)), y the stored BF16 activation
__global__ void tanh_back_kernel(const float* __restrict__ dy, const __bf16* __restrict__ y,
                                 __bf16* __restrict__ dz, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) {
        const float yy = (float)y[i];
        dz[i] = (__bf16)(dy[i] * (1.0f - yy * yy));
    }
}

// db[n] = sum_b dz[b][n]
__global__ void bias_grad_kernel(const __bf16* __restrict__ dz, int B, int N, float* __restrict__ db) {
    const int n = blockIdx.x * 256 + threadIdx.x;
    if (n >= N) return;
    float s = 0.f;
    for (int b = 0; b < B; ++b) s += (float)dz[(int64_t)b * N + n];
    db[n] = s;
}

// Adam on FP32 master parameters; bias corrections passed in.
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1,
                            float c2) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Adam step whose learning rate and bias corrections come from a device step
// counter, so that a captured training step can be replayed unchanged: the
// step is the (*done + 1)-th Adam step of the network and the s-th of the
// schedule (s = *done - done0), with the cosine rate
// lr0 (1 + cos(pi s / total)) / 2 + lr_floor.  Same arithmetic as a host
// computing lr and the corrections in double and passing them as floats.
__global__ void adam_sched_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                  float* __restrict__ v, int64_t n, double lr0, double lr_floor, int64_t total,
                                  int64_t done0, float b1, float b2, float eps, const int64_t* __restrict__ done) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int64_t t = *done;
    const double sfrac = (double)(t - done0) / (double)total;
    const float lr = (float)(lr0 * 0.5 * (1.0 + cos(3.14159265358979323846 * sfrac)) + lr_floor);
    const float c1 = 1.0f - (float)pow((double)b1, (double)(t + 1));
    const float c2 = 1.0f - (float)pow((double)b2, (double)(t + 1));
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

__global__ void count_set_kernel(int64_t* c, int64_t value) {
    if (threadIdx.x == 0) *c = value;
}

__global__ void count_inc_kernel(int64_t* c) {
    if (threadIdx.x == 0) *c += 1;
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

template <int EPI>
hipError_t gemm(const __bf16* A, int64_t sam, int64_t sak, const __bf16* B, int64_t sbk, int64_t sbn, int M, int N,
                int K, const float* bias, float* outf, __bf16* outb, int64_t ldo, hipStream_t st) {
    dim3 grid((M + 31) / 32, (N + 31) / 32);
    hipLaunchKernelGGL(gemm_kernel<EPI>, grid, dim3(256), 0, st, A, sam, sak, B, sbk, sbn, M, N, K, bias, outf, outb,
                       ldo);
    return hipGetLastError();
}

}  // namespace

struct lbw_mlp {
    std::vector<int> w;     // widths, n_layers + 1
    int L = 0;              // layers
    int max_batch = 0;
    hipStream_t stream = nullptr;
    std::vector<int64_t> off;  // parameter offset of layer l (W then b)
    int64_t P = 0;
    float *p = nullptr, *g = nullptr, *m = nullptr, *v = nullptr;  // FP32 master, grad, Adam moments
    __bf16* wb = nullptr;        // BF16 copy of the weights (same offsets, biases unused)
    __bf16* act = nullptr;       // BF16 input and hidden activations, layer l at act_off[l]
    std::vector<int64_t> act_off;
    float* yout = nullptr;       // FP32 output of the last forward
    float* dy = nullptr;         // FP32 gradient w.r.t. a layer output
    __bf16* dz = nullptr;        // BF16 gradient w.r.t. a pre-activation
    float* partial = nullptr;
    float* loss_dev = nullptr;
    int64_t* d_steps = nullptr;  // Adam steps taken, on the device (scheduled training)
    int64_t steps = 0;
    bool have_grad = false;
};

namespace {

hipError_t refresh_bf16(lbw_mlp* M, hipStream_t st) {
    hipLaunchKernelGGL(to_bf16_kernel, dim3(nblk(M->P)), dim3(256), 0, st, M->p, M->wb, M->P);
    return hipGetLastError();
}
hipError_t refresh_bf16(lbw_mlp* M) { return refresh_bf16(M, M->stream); }

hipError_t forward(lbw_mlp* M, const float* x, int B, hipStream_t st) {
    hipLaunchKernelGGL(to_bf16_kernel, dim3(nblk((int64_t)B * M->w[0])), dim3(256), 0, st, x,
                       M->act + M->act_off[0], (int64_t)B * M->w[0]);
    hipError_t e = hipGetLastError();
    for (int l = 0; l < M->L && e == hipSuccess; ++l) {
        const int K = M->w[l], N = M->w[l + 1];
        const __bf16* X = M->act + M->act_off[l];
        const __bf16* W = M->wb + M->off[l];
        const float* bias = M->p + M->off[l] + (int64_t)N * K;
        if (l + 1 < M->L)
            e = gemm<kEpiBiasTanhBF16>(X, K, 1, W, 1, K, B, N, K, bias, nullptr, M->act + M->act_off[l + 1], N, st);
        else
            e = gemm<kEpiBiasF32>(X, K, 1, W, 1, K, B, N, K, bias, M->yout, nullptr, N, st);
    }
    return e;
}
hipError_t forward(lbw_mlp* M, const float* x, int B) { return forward(M, x, B, M->stream); }

// Loss, its gradient and the backward pass (after forward), on stream st.
hipError_t loss_and_backward(lbw_mlp* M, const float* t, const float* w, int B, float inv, hipStream_t st) {
    const int L = M->L;
    const int64_t n_out = (int64_t)B * M->w[L];
    hipLaunchKernelGGL(loss_grad_kernel, dim3(nblk(n_out)), dim3(256), 0, st, M->yout, t, w, n_out, inv, M->dz,
                       M->partial);
    hipLaunchKernelGGL(loss_sum_kernel, dim3(1), dim3(256), 0, st, M->partial, (int)nblk(n_out), inv, M->loss_dev);
    hipError_t e = hipGetLastError();
    for (int l = L - 1; l >= 0 && e == hipSuccess; --l) {
        const int K = M->w[l], N = M->w[l + 1];
        const __bf16* X = M->act + M->act_off[l];
        float* gW = M->g + M->off[l];
        float* gb = gW + (int64_t)N * K;
        // dW[n][k] = sum_b dz[b][n] X[b][k]
        e = gemm<kEpiF32>(M->dz, 1, N, X, K, 1, N, K, B, nullptr, gW, nullptr, K, st);
        if (e != hipSuccess) break;
        hipLaunchKernelGGL(bias_grad_kernel, dim3(nblk(N)), dim3(256), 0, st, M->dz, B, N, gb);
        e = hipGetLastError();
        if (e == hipSuccess && l > 0) {
            // dY_prev[b][k] = sum_n dz[b][n] W[n][k]
            e = gemm<kEpiF32>(M->dz, N, 1, M->wb + M->off[l], K, 1, B, K, N, nullptr, M->dy, nullptr, K, st);
            if (e != hipSuccess) break;
            hipLaunchKernelGGL(tanh_back_kernel, dim3(nblk((int64_t)B * K)), dim3(256), 0, st, M->dy, X, M->dz,
                               (int64_t)B * K);
            e = hipGetLastError();
        }
    }
    return e;
}

}  // namespace

extern "C" {

int lbw_mlp_create(const int32_t* widths, int n_layers, int max_batch, void* stream, lbw_mlp_t* out) {
    if (!out) return fail(LBW_EINVAL, "out is NULL");
    *out = nullptr;
    if (!widths || n_layers < 1 || n_layers > 16 || max_batch < 1) return fail(LBW_EINVAL, "invalid MLP shape");
    for (int l = 0; l <= n_layers; ++l)
        if (widths[l] < 1 || widths[l] > 4096) return fail(LBW_EINVAL, "layer width outside [1, 4096]");
    lbw_mlp* M = new lbw_mlp();
    M->w.assign(widths, widths + n_layers + 1);
    M->L = n_layers;
    M->max_batch = max_batch;
    M->stream = (hipStream_t)stream;
    int64_t P = 0, A = 0, maxw = 0;
    for (int l = 0; l < n_layers; ++l) {
        M->off.push_back(P);
        P += (int64_t)M->w[l] * M->w[l + 1] + M->w[l + 1];
    }
    for (int l = 0; l <= n_layers; ++l) {
        M->act_off.push_back(A);
        A += (int64_t)max_batch * M->w[l];
        if (M->w[l] > maxw) maxw = M->w[l];
    }
    M->P = P;
    const int64_t bw = (int64_t)max_batch * maxw;
    hipError_t e = hipMalloc(&M->p, sizeof(float) * P);
    if (e == hipSuccess) e = hipMalloc(&M->g, sizeof(float) * P);
    if (e == hipSuccess) e = hipMalloc(&M->m, sizeof(float) * P);
    if (e == hipSuccess) e = hipMalloc(&M->v, sizeof(float) * P);
    if (e == hipSuccess) e = hipMalloc(&M->wb, sizeof(__bf16) * P);
    if (e == hipSuccess) e = hipMalloc(&M->act, sizeof(__bf16) * A);
    if (e == hipSuccess) e = hipMalloc(&M->yout, sizeof(float) * (int64_t)max_batch * M->w[n_layers]);
    if (e == hipSuccess) e = hipMalloc(&M->dy, sizeof(float) * bw);
    if (e == hipSuccess) e = hipMalloc(&M->dz, sizeof(__bf16) * bw);
    if (e == hipSuccess) e = hipMalloc(&M->partial, sizeof(float) * (nblk(bw) + 1));
    if (e == hipSuccess) e = hipMalloc(&M->loss_dev, sizeof(float));
    if (e == hipSuccess) e = hipMalloc(&M->d_steps, sizeof(int64_t));
    if (e == hipSuccess) e = hipMemsetAsync(M->p, 0, sizeof(float) * P, M->stream);
    if (e == hipSuccess) e = hipMemsetAsync(M->m, 0, sizeof(float) * P, M->stream);
    if (e == hipSuccess) e = hipMemsetAsync(M->v, 0, sizeof(float) * P, M->stream);
    if (e == hipSuccess) e = refresh_bf16(M);
    if (e != hipSuccess) {
        lbw_mlp_free(M);
        return hip_fail(e, "lbw_mlp_create");
    }
    *out = M;
    return LBW_OK;
}

int lbw_mlp_param_count(lbw_mlp_t M, int64_t* count) {
    if (!M || !count) return fail(LBW_EINVAL, "NULL argument");
    *count = M->P;
    return LBW_OK;
}

int lbw_mlp_set_params(lbw_mlp_t M, const float* host) {
    if (!M || !host) return fail(LBW_EINVAL, "NULL argument");
    HIP_TRY(hipMemcpyAsync(M->p, host, sizeof(float) * M->P, hipMemcpyHostToDevice, M->stream), "lbw_mlp_set_params");
    HIP_TRY(hipMemsetAsync(M->m, 0, sizeof(float) * M->P, M->stream), "lbw_mlp_set_params");
    HIP_TRY(hipMemsetAsync(M->v, 0, sizeof(float) * M->P, M->stream), "lbw_mlp_set_params");
    HIP_TRY(refresh_bf16(M), "lbw_mlp_set_params");
    HIP_TRY(hipStreamSynchronize(M->stream), "lbw_mlp_set_params");
    M->steps = 0;
    M->have_grad = false;
    return LBW_OK;
}

int lbw_mlp_get_params(lbw_mlp_t M, float* host) {
    if (!M || !host) return fail(LBW_EINVAL, "NULL argument");
    HIP_TRY(hipMemcpyAsync(host, M->p, sizeof(float) * M->P, hipMemcpyDeviceToHost, M->stream), "lbw_mlp_get_params");
    HIP_TRY(hipStreamSynchronize(M->stream), "lbw_mlp_get_params");
    return LBW_OK;
}

int lbw_mlp_forward(lbw_mlp_t M, const float* x, int B, float* y) {
    if (!M || !x || !y) return fail(LBW_EINVAL, "NULL argument");
    if (B < 1 || B > M->max_batch) return fail(LBW_EINVAL, "batch %d outside [1, %d]", B, M->max_batch);
    HIP_TRY(forward(M, x, B), "lbw_mlp_forward");
    HIP_TRY(hipMemcpyAsync(y, M->yout, sizeof(float) * (int64_t)B * M->w[M->L], hipMemcpyDeviceToDevice, M->stream),
            "lbw_mlp_forward");
    return LBW_OK;
}

int lbw_mlp_loss_grad(lbw_mlp_t M, const float* x, const float* t, const float* w, int B, float weight_sum,
                      float* loss, float* grad) {
    if (!M || !x || !t) return fail(LBW_EINVAL, "NULL argument");
    if (B < 1 || B > M->max_batch) return fail(LBW_EINVAL, "batch %d outside [1, %d]", B, M->max_batch);
    if (!(weight_sum > 0.0f)) return fail(LBW_EINVAL, "weight_sum must be > 0");
    HIP_TRY(forward(M, x, B), "lbw_mlp_loss_grad");
    HIP_TRY(loss_and_backward(M, t, w, B, 1.0f / weight_sum, M->stream), "lbw_mlp_loss_grad");
    if (loss) HIP_TRY(hipMemcpyAsync(loss, M->loss_dev, sizeof(float), hipMemcpyDeviceToDevice, M->stream), "loss");
    if (grad) HIP_TRY(hipMemcpyAsync(grad, M->g, sizeof(float) * M->P, hipMemcpyDeviceToDevice, M->stream), "grad");
    M->have_grad = true;
    return LBW_OK;
}

int lbw_mlp_adam_step(lbw_mlp_t M, float lr, float beta1, float beta2, float eps) {
    if (!M) return fail(LBW_EINVAL, "NULL argument");
    if (!M->have_grad) return fail(LBW_ESTATE, "no gradient: call lbw_mlp_loss_grad first");
    if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return fail(LBW_EINVAL, "invalid Adam hyper-parameters");
    M->steps += 1;
    const float c1 = 1.0f - (float)std::pow((double)beta1, (double)M->steps);
    const float c2 = 1.0f - (float)std::pow((double)beta2, (double)M->steps);
    hipLaunchKernelGGL(adam_kernel, dim3(nblk(M->P)), dim3(256), 0, M->stream, M->p, M->g, M->m, M->v, M->P, lr,
                       beta1, beta2, eps, c1, c2);
    HIP_TRY(hipGetLastError(), "lbw_mlp_adam_step");
    HIP_TRY(refresh_bf16(M), "lbw_mlp_adam_step");
    return LBW_OK;
}

int lbw_mlp_train(lbw_mlp_t M, const float* x, const float* t, const float* w, int B, float weight_sum, int steps,
                  double lr, double lr_floor, float beta1, float beta2, float eps, float* loss) {
    if (!M || !x || !t) return fail(LBW_EINVAL, "NULL argument");
    if (B < 1 || B > M->max_batch) return fail(LBW_EINVAL, "batch %d outside [1, %d]", B, M->max_batch);
    if (!(weight_sum > 0.0f)) return fail(LBW_EINVAL, "weight_sum must be > 0");
    if (steps < 1) return fail(LBW_EINVAL, "steps must be >= 1");
    if (!(lr > 0.0) || !(lr_floor >= 0.0) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) ||
        !(eps > 0.f))
        return fail(LBW_EINVAL, "invalid Adam hyper-parameters");
    // the device counter starts at the network's step count; one training
    // step (forward, loss, backward, Adam, BF16 refresh, counter) is captured
    // on a private stream and replayed on the network's stream
    hipLaunchKernelGGL(count_set_kernel, dim3(1), dim3(64), 0, M->stream, M->d_steps, M->steps);
    HIP_TRY(hipGetLastError(), "lbw_mlp_train");
    hipStream_t cap = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "lbw_mlp_train");
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t le = forward(M, x, B, cap);
        if (le == hipSuccess) le = loss_and_backward(M, t, w, B, 1.0f / weight_sum, cap);
        if (le == hipSuccess) {
            hipLaunchKernelGGL(adam_sched_kernel, dim3(nblk(M->P)), dim3(256), 0, cap, M->p, M->g, M->m, M->v, M->P,
                               lr, lr_floor, (int64_t)steps, M->steps, beta1, beta2, eps, M->d_steps);
            le = hipGetLastError();
        }
        if (le == hipSuccess) le = refresh_bf16(M, cap);
        if (le == hipSuccess) {
            hipLaunchKernelGGL(count_inc_kernel, dim3(1), dim3(64), 0, cap, M->d_steps);
            le = hipGetLastError();
        }
        e = hipStreamEndCapture(cap, &graph);
        if (e == hipSuccess) e = le;
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    for (int i = 0; i < steps && e == hipSuccess; ++i) e = hipGraphLaunch(exec, M->stream);
    if (e == hipSuccess && loss) e = hipMemcpyAsync(loss, M->loss_dev, sizeof(float), hipMemcpyDeviceToDevice, M->stream);
    const hipError_t es = hipStreamSynchronize(M->stream);  // before the graph is destroyed
    if (e == hipSuccess) e = es;
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess) return hip_fail(e, "lbw_mlp_train");
    M->steps += steps;
    M->have_grad = true;
    return LBW_OK;
}

int lbw_mlp_free(lbw_mlp_t M) {
    if (!M) return LBW_OK;
    (void)hipStreamSynchronize(M->stream);
    for (void* ptr : {(void*)M->p, (void*)M->g, (void*)M->m, (void*)M->v, (void*)M->wb, (void*)M->act,
                      (void*)M->yout, (void*)M->dy, (void*)M->dz, (void*)M->partial, (void*)M->loss_dev,
                      (void*)M->d_steps})
        (void)hipFree(ptr);
    delete M;
    return LBW_OK;
}

}  // extern "C"
