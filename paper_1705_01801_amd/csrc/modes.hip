// Resonant frequencies from probe traces, FP64 on the device.
//
// The paper locates resonances by driven frequency sweeps (Sec. IV.A and
// IV.C); for a freely ringing field the same peaks appear in the power
// spectrum of the probe signal.  Rule: per probe subtract the mean, apply
// the symmetric Hann window 1/2 - 1/2 cos(2 pi t / (T - 1)), zero-pad to
// nfft = 4 * nextpow2(T), FFT (radix-2 Stockham, natural-order output),
// P_k = sum over probes |X_k|^2 for k in [0, nfft/2]; peaks are bins
// b in [2, nfft/2 - 1] with P[b-1] < P[b] >= P[b+1] and P[b] > 1e-3 max P[2:],
// refined by a parabola through ln P (no refinement when a neighbour is 0).
#include "lbw_internal.h"

namespace lbw {
namespace {

constexpr int kBlock = 256;
constexpr int kPeakBlock = 1024;

int64_t nfft_for(int64_t T) {
    int64_t p = 1;
    while (p < T) p *= 2;
    return 4 * p;
}

// One block per probe: mean, then windowed and zero-padded complex input.
__global__ void prepare_kernel(const double* __restrict__ trace, int64_t T, int np, int64_t nfft, double2* __restrict__ x) {
    __shared__ double part[kBlock];
    const int p = blockIdx.x;
    double s = 0.0;
    for (int64_t t = threadIdx.x; t < T; t += kBlock) s += trace[t * np + p];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    const double mean = part[0] / (double)T;
    double2* xp = x + (size_t)p * nfft;
    for (int64_t t = threadIdx.x; t < nfft; t += kBlock) {
        double v = 0.0;
        if (t < T) {
            const double win = T > 1 ? 0.5 - 0.5 * cospi(2.0 * (double)t / (double)(T - 1)) : 1.0;
            v = (trace[t * np + p] - mean) * win;
        }
        xp[t] = make_double2(v, 0.0);
    }
}

// Radix-2 Stockham pass: Ns = size of the sub-transforms already formed.
__global__ void fft_pass_kernel(const double2* __restrict__ in, double2* __restrict__ out, int64_t nfft, int64_t Ns,
                                int np) {
    const int64_t half = nfft / 2;
    const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (gid >= half * np) return;
    const int64_t p = gid / half;
    const int64_t j = gid - p * half;
    const double2* ip = in + p * nfft;
    double2* op = out + p * nfft;
    const int64_t k = j % Ns;
    double2 a = ip[j];
    double2 b = ip[j + half];
    double sn, cs;
    sincospi(-(double)k / (double)Ns, &sn, &cs);  // exp(-2 pi i k / (2 Ns))
    const double2 bw = make_double2(b.x * cs - b.y * sn, b.x * sn + b.y * cs);
    const int64_t o = (j / Ns) * 2 * Ns + k;
    op[o] = make_double2(a.x + bw.x, a.y + bw.y);
    op[o + Ns] = make_double2(a.x - bw.x, a.y - bw.y);
}

__global__ void power_kernel(const double2* __restrict__ X, int64_t nfft, int np, double* __restrict__ P) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k > nfft / 2) return;
    double s = 0.0;
    for (int p = 0; p < np; ++p) {
        const double2 v = X[(size_t)p * nfft + k];
        s += v.x * v.x + v.y * v.y;
    }
    P[k] = s;
}

// Single block: global max over bins >= 2, then an ordered scan for peaks.
__global__ __launch_bounds__(kPeakBlock) void peaks_kernel(const double* __restrict__ P, int64_t nfft, int k,
                                                           double* __restrict__ freq, double* __restrict__ power) {
    __shared__ double red[kPeakBlock];
    __shared__ int cnt[kPeakBlock];
    __shared__ int found;
    const int64_t last = nfft / 2;  // P has last + 1 entries
    double m = 0.0;
    for (int64_t b = 2 + threadIdx.x; b <= last; b += kPeakBlock) m = fmax(m, P[b]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = kPeakBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
        __syncthreads();
    }
    const double thr = 1e-3 * red[0];
    for (int i = threadIdx.x; i < k; i += kPeakBlock) {
        freq[i] = __longlong_as_double(0x7ff8000000000000LL);
        power[i] = __longlong_as_double(0x7ff8000000000000LL);
    }
    if (threadIdx.x == 0) found = 0;
    __syncthreads();
    for (int64_t base = 2; base < last; base += kPeakBlock) {
        if (found >= k) break;  // uniform: found is read after a barrier
        const int64_t b = base + threadIdx.x;
        int flag = 0;
        if (b < last) flag = P[b - 1] < P[b] && P[b] >= P[b + 1] && P[b] > thr;
        cnt[threadIdx.x] = flag;
        __syncthreads();
        // inclusive scan (Hillis-Steele)
        for (int off = 1; off < kPeakBlock; off <<= 1) {
            const int v = threadIdx.x >= off ? cnt[threadIdx.x - off] : 0;
            __syncthreads();
            cnt[threadIdx.x] += v;
            __syncthreads();
        }
        const int slot = found + cnt[threadIdx.x] - 1;
        if (flag && slot < k) {
            const double pm = P[b - 1], p0 = P[b], pp = P[b + 1];
            const double l0 = log(p0);
            double delta = 0.0, lm = 0.0, lp = 0.0;
            if (pm > 0.0 && pp > 0.0) {
                lm = log(pm);
                lp = log(pp);
                const double den = lm - 2.0 * l0 + lp;
                delta = den != 0.0 ? 0.5 * (lm - lp) / den : 0.0;
            }
            freq[slot] = ((double)b + delta) / (double)nfft;
            power[slot] = exp(l0 - 0.25 * (lm - lp) * delta);
        }
        __syncthreads();
        if (threadIdx.x == kPeakBlock - 1) found += cnt[kPeakBlock - 1];
        __syncthreads();
    }
}

}  // namespace

size_t modes_work_bytes(int64_t T, int n_probes) {
    const int64_t nfft = nfft_for(T);
    return 2 * (size_t)nfft * n_probes * sizeof(double2) + (size_t)(nfft / 2 + 1) * sizeof(double);
}

hipError_t launch_modes(const double* trace, int64_t T, int np, int k, double* work, size_t work_bytes, double* freq,
                        double* power, hipStream_t st) {
    const int64_t nfft = nfft_for(T);
    if (work_bytes < modes_work_bytes(T, np)) return hipErrorInvalidValue;
    double2* x0 = reinterpret_cast<double2*>(work);
    double2* x1 = x0 + (size_t)nfft * np;
    double* P = reinterpret_cast<double*>(x1 + (size_t)nfft * np);
    hipLaunchKernelGGL(prepare_kernel, dim3(np), dim3(kBlock), 0, st, trace, T, np, nfft, x0);
    const unsigned fft_blocks = (unsigned)(((nfft / 2) * np + kBlock - 1) / kBlock);
    double2* src = x0;
    double2* dst = x1;
    for (int64_t Ns = 1; Ns < nfft; Ns *= 2) {
        hipLaunchKernelGGL(fft_pass_kernel, dim3(fft_blocks), dim3(kBlock), 0, st, src, dst, nfft, Ns, np);
        double2* t = src;
        src = dst;
        dst = t;
    }
    hipLaunchKernelGGL(power_kernel, dim3((unsigned)((nfft / 2 + 1 + kBlock - 1) / kBlock)), dim3(kBlock), 0, st, src,
                       nfft, np, P);
    hipLaunchKernelGGL(peaks_kernel, dim3(1), dim3(kPeakBlock), 0, st, P, nfft, k, freq, power);
    return hipGetLastError();
}

}  // namespace lbw
