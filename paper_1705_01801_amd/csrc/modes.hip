// Resonant frequencies from probe traces, FP64 on the device.
//
// The paper locates resonances by driven frequency sweeps (Sec. IV.A and
// IV.C); for a freely ringing field the same peaks appear in the power
// spectrum of the probe signal.  Rule: per probe subtract the mean, apply
// the symmetric Hann window 1/2 - 1/2 cos(2 pi t / (T - 1)), zero-pad to
// nfft = 4 * nextpow2(T), FFT (radix-2 Stockham, natural-order output),
// P_k = sum over a group's probes of |X_k|^2 for k in [0, nfft/2]; peaks are
// bins b in [16, nfft/2 - 1] with P[b-1] < P[b] >= P[b+1] and
// P[b] > 1e-3 max P[16:], refined by a parabola through ln P (no refinement
// when a neighbour is 0).  Bin 16 is the first bin outside the Hann window's
// DC main lobe (half-width 2/T cycles per step = at most 16 bins), where the
// leakage of a slow baseline drift would otherwise show up as a peak.
//
// A "group" is the set of probes of one geometry: consecutive columns of a
// trace whose rows hold `stride` values.  Groups are processed in chunks so
// that the FFT work space stays bounded.
#include <algorithm>
#include <mutex>
#include <vector>

#include "lbw_internal.h"

namespace lbw {
namespace {

constexpr int kBlock = 256;
constexpr int kPeakBlock = 1024;
constexpr int64_t kFirstBin = 16;
constexpr size_t kChunkBytes = size_t(1) << 30;  // FFT work space per chunk

// One block per column: mean, then windowed and zero-padded complex input.
__global__ void prepare_kernel(const double* __restrict__ trace, int64_t T, int64_t stride, int col_begin,
                               int64_t nfft, double2* __restrict__ x) {
    __shared__ double part[kBlock];
    const int64_t c = col_begin + blockIdx.x;
    double s = 0.0;
    for (int64_t t = threadIdx.x; t < T; t += kBlock) s += trace[t * stride + c];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    const double mean = part[0] / (double)T;
    double2* xp = x + (size_t)blockIdx.x * nfft;
    for (int64_t t = threadIdx.x; t < nfft; t += kBlock) {
        double v = 0.0;
        if (t < T) {
            const double win = T > 1 ? 0.5 - 0.5 * cospi(2.0 * (double)t / (double)(T - 1)) : 1.0;
            v = (trace[t * stride + c] - mean) * win;
        }
        xp[t] = make_double2(v, 0.0);
    }
}

// Radix-2 Stockham pass: Ns = size of the sub-transforms already formed.
__global__ void fft_pass_kernel(const double2* __restrict__ in, double2* __restrict__ out, int64_t nfft, int64_t Ns,
                                int ncols) {
    const int64_t half = nfft / 2;
    const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (gid >= half * ncols) return;
    const int64_t p = gid / half;
    const int64_t j = gid - p * half;
    const double2* ip = in + p * nfft;
    double2* op = out + p * nfft;
    const int64_t k = j % Ns;
    const double2 a = ip[j];
    const double2 b = ip[j + half];
    double sn, cs;
    sincospi(-(double)k / (double)Ns, &sn, &cs);  // exp(-2 pi i k / (2 Ns))
    const double2 bw = make_double2(b.x * cs - b.y * sn, b.x * sn + b.y * cs);
    const int64_t o = (j / Ns) * 2 * Ns + k;
    op[o] = make_double2(a.x + bw.x, a.y + bw.y);
    op[o + Ns] = make_double2(a.x - bw.x, a.y - bw.y);
}

// P[g][k] = sum over the group's columns of |X|^2; gcol[g] = first column of
// group g relative to the chunk, gcnt[g] = its column count.
__global__ void power_kernel(const double2* __restrict__ X, int64_t nfft, const int* __restrict__ gcol,
                             const int* __restrict__ gcnt, double* __restrict__ P) {
    const int g = blockIdx.y;
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t nb = nfft / 2 + 1;
    if (k >= nb) return;
    double s = 0.0;
    for (int p = 0; p < gcnt[g]; ++p) {
        const double2 v = X[(size_t)(gcol[g] + p) * nfft + k];
        s += v.x * v.x + v.y * v.y;
    }
    P[(size_t)g * nb + k] = s;
}

// One block per group: global max over bins >= 2, then an ordered scan.
__global__ __launch_bounds__(kPeakBlock) void peaks_kernel(const double* __restrict__ Pall, int64_t nfft, int k,
                                                           double* __restrict__ freq, double* __restrict__ power) {
    __shared__ double red[kPeakBlock];
    __shared__ int cnt[kPeakBlock];
    __shared__ int found;
    const int64_t last = nfft / 2;
    const double* P = Pall + (size_t)blockIdx.x * (last + 1);
    freq += (size_t)blockIdx.x * k;
    power += (size_t)blockIdx.x * k;
    double m = 0.0;
    for (int64_t b = kFirstBin + threadIdx.x; b <= last; b += kPeakBlock) m = fmax(m, P[b]);
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
    for (int64_t base = kFirstBin; base < last; base += kPeakBlock) {
        if (found >= k) break;  // uniform: found is read after a barrier
        const int64_t b = base + threadIdx.x;
        int flag = 0;
        if (b < last) flag = P[b - 1] < P[b] && P[b] >= P[b + 1] && P[b] > thr;
        cnt[threadIdx.x] = flag;
        __syncthreads();
        for (int off = 1; off < kPeakBlock; off <<= 1) {  // inclusive scan
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

// P[k] (+)= sum over columns [0, ncols) of |X|^2, for a single group whose
// columns are transformed in passes (accumulate = 0 on the first pass).
__global__ void power_accum_kernel(const double2* __restrict__ X, int64_t nfft, int ncols, int accumulate,
                                   double* __restrict__ P) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k > nfft / 2) return;
    double s = accumulate ? P[k] : 0.0;
    for (int p = 0; p < ncols; ++p) {
        const double2 v = X[(size_t)p * nfft + k];
        s += v.x * v.x + v.y * v.y;
    }
    P[k] = s;
}

// Work space of the allocation-free spectrum: a fixed array in device
// memory, one per GPU the library runs on, kept until the process ends.
// Host code never passes `scratch` itself to a kernel (on the host the name
// is only a stand-in for the symbol); it uses the device address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[kModesScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

hipError_t modes_scratch(void** ptr) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return hipSuccess;
}

int modes_static_cols(int64_t T) {
    const int64_t nfft = modes_nfft(T);
    const size_t per_col = 2 * (size_t)nfft * sizeof(double2);
    const size_t p_bytes = ((size_t)(nfft / 2 + 1) * sizeof(double) + 255) / 256 * 256;
    if (p_bytes + per_col > kModesScratchBytes) return 0;
    return (int)((kModesScratchBytes - p_bytes) / per_col);
}

hipError_t launch_modes_static(void* scratch_ptr, const double* trace, int64_t T, int64_t stride, int ncols, int k,
                               double* freq, double* power, hipStream_t st) {
    const int64_t nfft = modes_nfft(T);
    const int per_pass = modes_static_cols(T);
    if (per_pass < 1 || ncols < 1) return hipErrorInvalidValue;
    unsigned char* base = static_cast<unsigned char*>(scratch_ptr);
    double* P = reinterpret_cast<double*>(base);
    const size_t p_bytes = ((size_t)(nfft / 2 + 1) * sizeof(double) + 255) / 256 * 256;
    double2* x0 = reinterpret_cast<double2*>(base + p_bytes);
    double2* x1 = x0 + (size_t)nfft * per_pass;
    for (int c0 = 0; c0 < ncols; c0 += per_pass) {
        const int cols = std::min(per_pass, ncols - c0);
        hipLaunchKernelGGL(prepare_kernel, dim3(cols), dim3(kBlock), 0, st, trace, T, stride, c0, nfft, x0);
        double2* src = x0;
        double2* dst = x1;
        const unsigned fft_blocks = (unsigned)(((nfft / 2) * cols + kBlock - 1) / kBlock);
        for (int64_t Ns = 1; Ns < nfft; Ns *= 2) {
            hipLaunchKernelGGL(fft_pass_kernel, dim3(fft_blocks), dim3(kBlock), 0, st, src, dst, nfft, Ns, cols);
            std::swap(src, dst);
        }
        hipLaunchKernelGGL(power_accum_kernel, dim3((unsigned)((nfft / 2 + 1 + kBlock - 1) / kBlock)), dim3(kBlock),
                           0, st, src, nfft, cols, c0 > 0 ? 1 : 0, P);
    }
    hipLaunchKernelGGL(peaks_kernel, dim3(1), dim3(kPeakBlock), 0, st, P, nfft, k, freq, power);
    return hipGetLastError();
}

int64_t modes_nfft(int64_t T) {
    int64_t p = 1;
    while (p < T) p *= 2;
    return 4 * p;
}

size_t modes_work_bytes(int64_t T, int max_cols, int max_groups) {
    const int64_t nfft = modes_nfft(T);
    return 2 * (size_t)nfft * max_cols * sizeof(double2) + (size_t)(nfft / 2 + 1) * max_groups * sizeof(double) +
           2 * sizeof(int) * (size_t)max_groups + 256;
}

int modes_max_cols(int64_t T) {
    const size_t per_col = 2 * (size_t)modes_nfft(T) * sizeof(double2);
    return (int)std::max<size_t>(1, kChunkBytes / per_col);
}

hipError_t launch_modes_grouped(const double* trace, int64_t T, int64_t stride, const int* group_ncols, int groups,
                                int k, double* work, size_t work_bytes, double* freq, double* power,
                                hipStream_t st) {
    const int64_t nfft = modes_nfft(T);
    const int cap = modes_max_cols(T);
    int max_group = 0;
    for (int g = 0; g < groups; ++g) max_group = std::max(max_group, group_ncols[g]);
    if (max_group > cap) return hipErrorInvalidValue;
    int g0 = 0, col0 = 0;
    while (g0 < groups) {
        // chunk: groups [g0, g1) with at most cap columns
        int g1 = g0, cols = 0;
        while (g1 < groups && cols + group_ncols[g1] <= cap) cols += group_ncols[g1++];
        const int ng = g1 - g0;
        if (work_bytes < modes_work_bytes(T, cols, ng)) return hipErrorInvalidValue;
        double2* x0 = reinterpret_cast<double2*>(work);
        double2* x1 = x0 + (size_t)nfft * cols;
        double* P = reinterpret_cast<double*>(x1 + (size_t)nfft * cols);
        int* gcol = reinterpret_cast<int*>(P + (size_t)(nfft / 2 + 1) * ng);
        int* gcnt = gcol + ng;
        std::vector<int> h(2 * ng);
        for (int g = 0, c = 0; g < ng; ++g) {
            h[g] = c;
            h[ng + g] = group_ncols[g0 + g];
            c += group_ncols[g0 + g];
        }
        hipError_t e = hipMemcpyAsync(gcol, h.data(), sizeof(int) * 2 * ng, hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return e;
        double2* src = x0;
        double2* dst = x1;
        if (cols > 0) {
            hipLaunchKernelGGL(prepare_kernel, dim3(cols), dim3(kBlock), 0, st, trace, T, stride, col0, nfft, x0);
            const unsigned fft_blocks = (unsigned)(((nfft / 2) * cols + kBlock - 1) / kBlock);
            for (int64_t Ns = 1; Ns < nfft; Ns *= 2) {
                hipLaunchKernelGGL(fft_pass_kernel, dim3(fft_blocks), dim3(kBlock), 0, st, src, dst, nfft, Ns, cols);
                std::swap(src, dst);
            }
        }
        hipLaunchKernelGGL(power_kernel, dim3((unsigned)((nfft / 2 + 1 + kBlock - 1) / kBlock), ng), dim3(kBlock), 0,
                           st, src, nfft, gcol, gcnt, P);
        hipLaunchKernelGGL(peaks_kernel, dim3(ng), dim3(kPeakBlock), 0, st, P, nfft, k, freq + (size_t)g0 * k,
                           power + (size_t)g0 * k);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        // the host group table is reused next chunk: wait for the copy
        e = hipStreamSynchronize(st);
        if (e != hipSuccess) return e;
        g0 = g1;
        col0 += cols;
    }
    return hipSuccess;
}

}  // namespace lbw
