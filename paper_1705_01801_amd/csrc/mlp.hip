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
// Every product is one kernel, gemm_kernel, with the elementwise work of the
// layer fused into its epilogue: bias + tanh (hidden forward), bias (output
// forward), bias + squared-error loss with the output gradient (training
// forward), tanh backward (hidden gradient), and the bias gradient as the row
// sums of the weight-gradient product.  A launch may carry two independent
// products (a layer's weight gradient and its input gradient), so a training
// step is L forward launches, L backward launches and one Adam launch.
//
// MFMA layout (v_mfma_f32_16x16x32_bf16): a wave computes one 16 x 16 tile
// of C = A B over K in steps of 32; lane l supplies row/column l % 16 and
// eight consecutive k values of group l / 16; the accumulator holds rows
// 4 (l / 16) + j, column l % 16.  A workgroup of four waves covers 32 x 32.
// The matrices are small (at most max_batch x 4096) and read with arbitrary
// strides: where an operand's k index is contiguous and its rows 16-byte
// aligned a lane reads its eight values with one 16-byte load, otherwise with
// eight 2-byte loads.  Loads are branch-free (an out-of-range element reads
// element 0 and is replaced by zero), and four K steps are loaded before
// their products, so a K of 128 costs one memory latency.
#include <cmath>
#include <cstdint>
#include <vector>

#include "host_util.h"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

using lbw::fail;
using lbw::hip_fail;

namespace {

constexpr int kEpiNone = -1;         // no second product
constexpr int kEpiBias = 0;          // outf = acc + bias
constexpr int kEpiBiasTanh = 1;      // outb = bf16(tanh(acc + bias))
constexpr int kEpiBiasLoss = 2;      // outf = y = acc + bias; dz, partial loss (below)
constexpr int kEpiWeightGrad = 3;    // outf = acc; rowsum[m] = sum_k A(m, k)
constexpr int kEpiTanhBack = 4;      // outb = bf16(acc (1 - y^2)), y = act[m][n]
constexpr int kKSteps = 4;           // K steps of 32 loaded before their products

// C[m][n] = sum_k A(m, k) B(k, n) over m < M, n < N, k < K, with
// A(m, k) = A[m sam + k sak] and B(k, n) = B[k sbk + n sbn]; C row stride ldo.
struct Gemm {
    const __bf16* A;
    int64_t sam, sak;
    const __bf16* B;
    int64_t sbk, sbn;
    int M, N, K;
    int64_t ldo;
    int tiles_m;           // ceil(M / 32); tile id = tile_n * tiles_m + tile_m
    const float* bias;     // [N]
    float* outf;           // FP32 output
    __bf16* outb;          // BF16 output
    const __bf16* act;     // tanh backward: stored activation, layout of C
    float* rowsum;         // weight gradient: bias gradient [M]
    const float* t;        // loss: targets, layout of C
    const float* w;        // loss: weights, layout of C, NULL = 1
    float inv;             // loss: 1 / sum of weights
    __bf16* dz;            // loss: bf16(2 w (y - t) inv), layout of C
    float* partial;        // loss: sum of w (y - t)^2 per tile
};

// Work done once per launch by workgroup 0 besides its tile.
struct Extra {
    int64_t* counter;           // += 1 (training step counter), or NULL
    const float* fin_partial;   // loss = inv * sum of fin_partial[0, fin_n), or NULL
    int fin_n;
    float fin_inv;
    float* fin_loss;
};

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Eight consecutive k values kb .. kb + 7 of row `row` of an operand with
// element (row, k) at P[row s_row + k s_k]; zero outside row < nrow, k < K.
// VEC: s_k == 1, K % 8 == 0 and every row start 16-byte aligned.
template <bool VEC>
__device__ __forceinline__ bf16x8 fragment(const __bf16* __restrict__ P, int64_t s_row, int64_t s_k, int row,
                                           int nrow, int kb, int K) {
    if constexpr (VEC) {
        const bool ok = row < nrow && kb < K;
        const int64_t idx = ok ? (int64_t)row * s_row + kb : 0;
        uint4 raw = *reinterpret_cast<const uint4*>(P + idx);
        raw.x = ok ? raw.x : 0u;
        raw.y = ok ? raw.y : 0u;
        raw.z = ok ? raw.z : 0u;
        raw.w = ok ? raw.w : 0u;
        return __builtin_bit_cast(bf16x8, raw);
    } else {
        bf16x8 out;
        const bool rok = row < nrow;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const bool ok = rok && kb + j < K;
            const int64_t idx = ok ? (int64_t)row * s_row + (int64_t)(kb + j) * s_k : 0;
            const __bf16 v = P[idx];
            out[j] = ok ? v : (__bf16)0.0f;
        }
        return out;
    }
}

template <int EPI, bool AV, bool BV>
__device__ __forceinline__ void gemm_tile(const Gemm& g, int tm, int tn) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = lane & 15, grp = lane >> 4;
    const int m0 = tm * 32 + (wave & 1) * 16, n0 = tn * 32 + (wave >> 1) * 16;
    const int am = m0 + r, bn = n0 + r;
    floatx4 acc = {0.f, 0.f, 0.f, 0.f}, accs = {0.f, 0.f, 0.f, 0.f};
    // the waves holding column 0 also multiply A by ones: row sums of A
    const bool sums = EPI == kEpiWeightGrad && g.rowsum && n0 == 0;
    bf16x8 ones;
#pragma unroll
    for (int j = 0; j < 8; ++j) ones[j] = sums ? (__bf16)1.0f : (__bf16)0.0f;
    // epilogue operands, loaded branch-free before the products
    const int n = n0 + r;
    const bool nok = n < g.N;
    float bias = 0.f, e1[4] = {0.f, 0.f, 0.f, 0.f}, e2[4] = {1.f, 1.f, 1.f, 1.f};
    if constexpr (EPI == kEpiBias || EPI == kEpiBiasTanh || EPI == kEpiBiasLoss) {
        const float bv = g.bias[nok ? n : 0];
        bias = nok ? bv : 0.f;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int m = m0 + 4 * grp + j;
        const bool ok = nok && m < g.M;
        const int64_t o = ok ? (int64_t)m * g.ldo + n : 0;
        if constexpr (EPI == kEpiTanhBack) e1[j] = (float)g.act[o];
        if constexpr (EPI == kEpiBiasLoss) {
            e1[j] = g.t[o];
            if (g.w) e2[j] = g.w[o];
        }
    }
    for (int k0 = 0; k0 < g.K; k0 += 32 * kKSteps) {
        bf16x8 a[kKSteps], b[kKSteps];
#pragma unroll
        for (int u = 0; u < kKSteps; ++u) {
            const int kb = k0 + 32 * u + 8 * grp;
            a[u] = fragment<AV>(g.A, g.sam, g.sak, am, g.M, kb, g.K);
            b[u] = fragment<BV>(g.B, g.sbn, g.sbk, bn, g.N, kb, g.K);
        }
#pragma unroll
        for (int u = 0; u < kKSteps; ++u) {
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[u], b[u], acc, 0, 0, 0);
            if constexpr (EPI == kEpiWeightGrad) accs = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[u], ones, accs, 0, 0, 0);
        }
    }
    float lsum = 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int m = m0 + 4 * grp + j;
        if (m < g.M && nok) {
            const int64_t o = (int64_t)m * g.ldo + n;
            const float v = acc[j];
            if constexpr (EPI == kEpiBias) {
                g.outf[o] = v + bias;
            } else if constexpr (EPI == kEpiBiasTanh) {
                g.outb[o] = (__bf16)tanhf(v + bias);
            } else if constexpr (EPI == kEpiBiasLoss) {
                const float y = v + bias;
                g.outf[o] = y;
                const float d = y - e1[j];
                const float ww = e2[j];
                lsum += ww * d * d;
                g.dz[o] = (__bf16)(2.0f * ww * d * g.inv);
            } else if constexpr (EPI == kEpiWeightGrad) {
                g.outf[o] = v;
            } else if constexpr (EPI == kEpiTanhBack) {
                const float y = e1[j];
                g.outb[o] = (__bf16)(v * (1.0f - y * y));
            }
        }
        if constexpr (EPI == kEpiWeightGrad)
            if (sums && r == 0 && m < g.M) g.rowsum[m] = accs[j];
    }
    if constexpr (EPI == kEpiBiasLoss) {
        __shared__ float red[4];
        lsum = wave_sum(lsum);
        if (lane == 0) red[wave] = lsum;
        __syncthreads();
        if (threadIdx.x == 0) g.partial[tn * g.tiles_m + tm] = ((red[0] + red[1]) + red[2]) + red[3];
    }
}

// Tiles [0, n1) of the grid compute g1, tiles [n1, n1 + n2) compute g2.
template <int E1, bool AV1, bool BV1, int E2, bool AV2, bool BV2>
__global__ __launch_bounds__(256) void gemm_kernel(Gemm g1, int n1, Gemm g2, Extra x) {
    const int id = blockIdx.x;
    if (id < n1) {
        gemm_tile<E1, AV1, BV1>(g1, id % g1.tiles_m, id / g1.tiles_m);
    } else if constexpr (E2 != kEpiNone) {
        const int id2 = id - n1;
        gemm_tile<E2, AV2, BV2>(g2, id2 % g2.tiles_m, id2 / g2.tiles_m);
    }
    if (blockIdx.x == 0 && threadIdx.x < 64) {
        if (x.counter && threadIdx.x == 0) *x.counter += 1;
        if (x.fin_partial) {
            float s = 0.f;
            for (int i = threadIdx.x; i < x.fin_n; i += 64) s += x.fin_partial[i];
            s = wave_sum(s);
            if (threadIdx.x == 0) x.fin_loss[0] = s * x.fin_inv;
        }
    }
}

__global__ void to_bf16_kernel(const float* __restrict__ in, __bf16* __restrict__ out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) out[i] = (__bf16)in[i];
}

// Adam on the FP32 master parameters, bias corrections passed in; refreshes
// the BF16 copy used by the products.
__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                            float* __restrict__ v, __bf16* __restrict__ pb, int64_t n, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
    pb[i] = (__bf16)pi;
}

// The same update inside a replayed training step: the step index t (from 1)
// is read from the device counter, the learning rate follows the cosine
// schedule lr0 (1 + cos(pi s / total)) / 2 + lr_floor with s = t - 1 - done0
// the step within this run, and the bias corrections are 1 - beta^t.
__global__ void adam_sched_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                  float* __restrict__ v, __bf16* __restrict__ pb, int64_t n, double lr0,
                                  double lr_floor, int64_t total, int64_t done0, float b1, float b2, float eps,
                                  const int64_t* __restrict__ counter) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int64_t t = *counter;
    const double sfrac = (double)(t - 1 - done0) / (double)total;
    const float lr = (float)(lr0 * 0.5 * (1.0 + cos(3.14159265358979323846 * sfrac)) + lr_floor);
    const float c1 = 1.0f - (float)pow((double)b1, (double)t);
    const float c2 = 1.0f - (float)pow((double)b2, (double)t);
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    p[i] = pi;
    pb[i] = (__bf16)pi;
}

__global__ void count_set_kernel(int64_t* c, int64_t value) {
    if (threadIdx.x == 0) *c = value;
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

inline bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

// Operand (row, k) at P[row s_row + k s_k] can take 16-byte loads.
inline bool vec_ok(const __bf16* P, int64_t s_row, int64_t s_k, int K) {
    return s_k == 1 && K % 8 == 0 && s_row % 8 == 0 && aligned16(P);
}

Gemm make_gemm(const __bf16* A, int64_t sam, int64_t sak, const __bf16* B, int64_t sbk, int64_t sbn, int M, int N,
               int K, int64_t ldo) {
    Gemm g{};
    g.A = A;
    g.sam = sam;
    g.sak = sak;
    g.B = B;
    g.sbk = sbk;
    g.sbn = sbn;
    g.M = M;
    g.N = N;
    g.K = K;
    g.ldo = ldo;
    g.tiles_m = (M + 31) / 32;
    return g;
}

inline int tiles(const Gemm& g) { return g.tiles_m * ((g.N + 31) / 32); }

template <int E1, bool AV1, bool BV1, int E2, bool AV2, bool BV2>
hipError_t launch(const Gemm& g1, const Gemm* g2, const Extra& x, hipStream_t st) {
    const int n1 = tiles(g1), n2 = g2 ? tiles(*g2) : 0;
    hipLaunchKernelGGL((gemm_kernel<E1, AV1, BV1, E2, AV2, BV2>), dim3(n1 + n2), dim3(256), 0, st, g1, n1,
                       g2 ? *g2 : g1, x);
    return hipGetLastError();
}

// One product with epilogue EPI; the two load paths picked from the operands.
template <int EPI>
hipError_t gemm1(const Gemm& g, const Extra& x, hipStream_t st) {
    const bool av = vec_ok(g.A, g.sam, g.sak, g.K), bv = vec_ok(g.B, g.sbn, g.sbk, g.K);
    if (av && bv) return launch<EPI, true, true, kEpiNone, false, false>(g, nullptr, x, st);
    if (av) return launch<EPI, true, false, kEpiNone, false, false>(g, nullptr, x, st);
    if (bv) return launch<EPI, false, true, kEpiNone, false, false>(g, nullptr, x, st);
    return launch<EPI, false, false, kEpiNone, false, false>(g, nullptr, x, st);
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
    float* yout = nullptr;       // FP32 output of the last training forward
    __bf16* dz[2] = {nullptr, nullptr};  // BF16 gradients w.r.t. pre-activations (alternating layers)
    float* partial = nullptr;    // per-tile loss sums of the output product
    int n_partial = 0;
    float* loss_dev = nullptr;
    int64_t* d_steps = nullptr;  // Adam steps taken, on the device (scheduled training)
    int64_t steps = 0;
    bool have_grad = false;
};

namespace {

hipError_t refresh_bf16(lbw_mlp* M) {
    hipLaunchKernelGGL(to_bf16_kernel, dim3(nblk(M->P)), dim3(256), 0, M->stream, M->p, M->wb, M->P);
    return hipGetLastError();
}

hipError_t cast_input(lbw_mlp* M, const float* x, int B, hipStream_t st) {
    hipLaunchKernelGGL(to_bf16_kernel, dim3(nblk((int64_t)B * M->w[0])), dim3(256), 0, st, x,
                       M->act + M->act_off[0], (int64_t)B * M->w[0]);
    return hipGetLastError();
}

// Layers 0 .. L-1 on the cast input.  The output layer writes y_out (FP32,
// [B][w_L]) when t is NULL, else the loss gradient and per-tile loss sums.
hipError_t forward_layers(lbw_mlp* M, int B, float* y_out, const float* t, const float* w, float inv,
                          int64_t* counter, hipStream_t st) {
    hipError_t e = hipSuccess;
    for (int l = 0; l < M->L && e == hipSuccess; ++l) {
        const int K = M->w[l], N = M->w[l + 1];
        Gemm g = make_gemm(M->act + M->act_off[l], K, 1, M->wb + M->off[l], 1, K, B, N, K, N);
        g.bias = M->p + M->off[l] + (int64_t)N * K;
        Extra x{};
        x.counter = l == 0 ? counter : nullptr;
        if (l + 1 < M->L) {
            g.outb = M->act + M->act_off[l + 1];
            e = gemm1<kEpiBiasTanh>(g, x, st);
        } else if (!t) {
            g.outf = y_out;
            e = gemm1<kEpiBias>(g, x, st);
        } else {
            g.outf = M->yout;
            g.t = t;
            g.w = w;
            g.inv = inv;
            g.dz = M->dz[0];
            g.partial = M->partial;
            M->n_partial = tiles(g);
            e = gemm1<kEpiBiasLoss>(g, x, st);
        }
    }
    return e;
}

// Gradients after a training forward: per layer (last first) one launch with
// dW = dz^T X and the bias gradient (row sums of dz^T), and, below the
// output layer, the next dz = (dz W) (1 - X^2) from the stored activation X.
// The first launch also reduces the loss.
hipError_t backward(lbw_mlp* M, int B, float inv, hipStream_t st) {
    hipError_t e = hipSuccess;
    int cur = 0;
    for (int l = M->L - 1; l >= 0 && e == hipSuccess; --l, cur ^= 1) {
        const int K = M->w[l], N = M->w[l + 1];
        const __bf16* X = M->act + M->act_off[l];
        const __bf16* dz = M->dz[cur];
        Gemm gw = make_gemm(dz, 1, N, X, K, 1, N, K, B, K);
        gw.outf = M->g + M->off[l];
        gw.rowsum = gw.outf + (int64_t)N * K;
        Extra x{};
        if (l == M->L - 1) {
            x.fin_partial = M->partial;
            x.fin_n = M->n_partial;
            x.fin_inv = inv;
            x.fin_loss = M->loss_dev;
        }
        if (l == 0) {
            e = launch<kEpiWeightGrad, false, false, kEpiNone, false, false>(gw, nullptr, x, st);
        } else {
            Gemm gy = make_gemm(dz, N, 1, M->wb + M->off[l], K, 1, B, K, N, K);
            gy.act = X;
            gy.outb = M->dz[cur ^ 1];
            if (vec_ok(gy.A, gy.sam, gy.sak, gy.K))
                e = launch<kEpiWeightGrad, false, false, kEpiTanhBack, true, false>(gw, &gy, x, st);
            else
                e = launch<kEpiWeightGrad, false, false, kEpiTanhBack, false, false>(gw, &gy, x, st);
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
        A += ((int64_t)max_batch * M->w[l] + 7) / 8 * 8;  // 16-byte aligned layers
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
    if (e == hipSuccess) e = hipMalloc(&M->dz[0], sizeof(__bf16) * bw);
    if (e == hipSuccess) e = hipMalloc(&M->dz[1], sizeof(__bf16) * bw);
    // one loss sum per 32 x 32 output tile
    if (e == hipSuccess)
        e = hipMalloc(&M->partial, sizeof(float) * (((int64_t)max_batch + 31) / 32) * ((M->w[n_layers] + 31) / 32));
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
    HIP_TRY(cast_input(M, x, B, M->stream), "lbw_mlp_forward");
    HIP_TRY(forward_layers(M, B, y, nullptr, nullptr, 0.f, nullptr, M->stream), "lbw_mlp_forward");
    return LBW_OK;
}

int lbw_mlp_loss_grad(lbw_mlp_t M, const float* x, const float* t, const float* w, int B, float weight_sum,
                      float* loss, float* grad) {
    if (!M || !x || !t) return fail(LBW_EINVAL, "NULL argument");
    if (B < 1 || B > M->max_batch) return fail(LBW_EINVAL, "batch %d outside [1, %d]", B, M->max_batch);
    if (!(weight_sum > 0.0f)) return fail(LBW_EINVAL, "weight_sum must be > 0");
    const float inv = 1.0f / weight_sum;
    HIP_TRY(cast_input(M, x, B, M->stream), "lbw_mlp_loss_grad");
    HIP_TRY(forward_layers(M, B, nullptr, t, w, inv, nullptr, M->stream), "lbw_mlp_loss_grad");
    HIP_TRY(backward(M, B, inv, M->stream), "lbw_mlp_loss_grad");
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
    hipLaunchKernelGGL(adam_kernel, dim3(nblk(M->P)), dim3(256), 0, M->stream, M->p, M->g, M->m, M->v, M->wb, M->P,
                       lr, beta1, beta2, eps, c1, c2);
    HIP_TRY(hipGetLastError(), "lbw_mlp_adam_step");
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
    // the input is cast once and the device counter starts at the network's
    // step count; one training step (forward with the counter increment and
    // the loss, backward, Adam with the BF16 refresh) is captured on a
    // private stream and replayed on the network's stream
    const float inv = 1.0f / weight_sum;
    HIP_TRY(cast_input(M, x, B, M->stream), "lbw_mlp_train");
    hipLaunchKernelGGL(count_set_kernel, dim3(1), dim3(64), 0, M->stream, M->d_steps, M->steps);
    HIP_TRY(hipGetLastError(), "lbw_mlp_train");
    hipStream_t cap = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "lbw_mlp_train");
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t le = forward_layers(M, B, nullptr, t, w, inv, M->d_steps, cap);
        if (le == hipSuccess) le = backward(M, B, inv, cap);
        if (le == hipSuccess) {
            hipLaunchKernelGGL(adam_sched_kernel, dim3(nblk(M->P)), dim3(256), 0, cap, M->p, M->g, M->m, M->v, M->wb,
                               M->P, lr, lr_floor, (int64_t)steps, M->steps, beta1, beta2, eps, M->d_steps);
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
                      (void*)M->yout, (void*)M->dz[0], (void*)M->dz[1], (void*)M->partial, (void*)M->loss_dev,
                      (void*)M->d_steps})
        (void)hipFree(ptr);
    delete M;
    return LBW_OK;
}

}  // extern "C"
