// Small reductions and per-point kernels around the sweeps: the wave
// model's point scales dt^2 / m, the data residual and misfit, and the
// on-demand scan of a field for non-finite values and its largest magnitude.
#include <algorithm>
#include <cstring>

#include "kernels.hpp"

namespace stn {

namespace {

// out[i] = dt2 / m[off[i]] (FP64): dt^2 v^2 at each listed interior point of
// a dense interior array m
__global__ void k_point_scale(const double* m, const int64_t* off, int64_t n, double dt2, double* out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = dt2 / m[off[i]];
}

// One workgroup of 256 threads: resid[i] = trace[i] - dobs[i] and
// misfit = 1/2 sum_i resid[i]^2 in FP64.  Thread t sums i = t, t + 256, ...
// in order; the 256 partial sums are added by a fixed pairwise tree, so the
// result does not depend on scheduling.
constexpr int kMisfitThreads = 256;

__global__ void __launch_bounds__(kMisfitThreads) k_misfit(const double* trace, const double* dobs, int64_t n,
                                                           double* resid, double* misfit) {
    __shared__ double part[kMisfitThreads];
    const int t = threadIdx.x;
    double acc = 0.0;
    for (int64_t i = t; i < n; i += kMisfitThreads) {
        const double r = trace[i] - dobs[i];
        resid[i] = r;
        acc = fma(r, r, acc);
    }
    part[t] = acc;
    __syncthreads();
    for (int w = kMisfitThreads / 2; w > 0; w >>= 1) {
        if (t < w) part[t] += part[t + w];
        __syncthreads();
    }
    if (t == 0) *misfit = 0.5 * part[0];
}

// Scan of a field's interior: out[0] += NaN count, out[1] += infinity count,
// out[2] = max(out[2], largest finite |value| as the bits of a non-negative
// double, whose integer order is the numeric order).
template <typename T>
__global__ void k_scan(const T* base, Grid3 g, unsigned long long* out) {
    const int64_t total = (int64_t)g.n[0] * g.n[1] * g.n[2];
    unsigned long long nan = 0, inf = 0;
    double mx = 0.0;
    for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < total;
         q += (int64_t)gridDim.x * blockDim.x) {
        const int64_t x = q % g.n[2], y = (q / g.n[2]) % g.n[1], z = q / ((int64_t)g.n[2] * g.n[1]);
        const float v = Storage<T>::load(base + g.origin + z * g.s[0] + y * g.s[1] + x);
        if (v != v) {
            nan++;
        } else if (fabsf(v) == __builtin_huge_valf()) {
            inf++;
        } else {
            mx = fmax(mx, (double)fabsf(v));
        }
    }
    if (nan) atomicAdd(&out[0], nan);
    if (inf) atomicAdd(&out[1], inf);
    if (mx > 0.0) atomicMax(&out[2], (unsigned long long)__double_as_longlong(mx));
}

unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// A chunk of 32-bit words carried by value in the kernel's arguments, so
// that host data reaches device memory without a host-to-device copy (and a
// captured launch keeps its own copy of the data).
constexpr int kFillWords = 512;
struct FillChunk {
    uint32_t n;
    uint32_t w[kFillWords];
};

__global__ void k_fill_words(uint32_t* dst, FillChunk c) {
    for (uint32_t i = threadIdx.x; i < c.n; i += blockDim.x) dst[i] = c.w[i];
}

}  // namespace

hipError_t launch_fill_words(void* dst, const void* src, size_t bytes, hipStream_t s) {
    if (bytes % 4) return hipErrorInvalidValue;
    const uint32_t* from = (const uint32_t*)src;
    uint32_t* to = (uint32_t*)dst;
    for (size_t done = 0; done < bytes / 4; done += kFillWords) {
        FillChunk c;
        c.n = (uint32_t)std::min<size_t>(kFillWords, bytes / 4 - done);
        std::memcpy(c.w, from + done, 4 * (size_t)c.n);
        hipLaunchKernelGGL(k_fill_words, dim3(1), dim3(256), 0, s, to + done, c);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_point_scale(const double* m, const int64_t* off, int64_t n, double dt2, double* out, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_point_scale, dim3(blocks_for(n, 64)), dim3(64), 0, s, m, off, n, dt2, out);
    return hipGetLastError();
}

hipError_t launch_misfit(const double* trace, const double* dobs, int64_t n, double* resid, double* misfit,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_misfit, dim3(1), dim3(kMisfitThreads), 0, s, trace, dobs, n, resid, misfit);
    return hipGetLastError();
}

hipError_t launch_scan(int dtype, const void* base, const Grid3& g, unsigned long long* out, hipStream_t s) {
    const int64_t total = (int64_t)g.n[0] * g.n[1] * g.n[2];
    if (total == 0) return hipSuccess;
    // a grid-stride loop over at most 4096 workgroups of 256 threads
    const unsigned nb = (unsigned)std::min<int64_t>(4096, blocks_for(total, 256));
    switch (dtype) {
        case DT_F32: hipLaunchKernelGGL(k_scan<float>, dim3(nb), dim3(256), 0, s, (const float*)base, g, out); break;
        case DT_BF16: hipLaunchKernelGGL(k_scan<bf16>, dim3(nb), dim3(256), 0, s, (const bf16*)base, g, out); break;
        case DT_F16: hipLaunchKernelGGL(k_scan<f16>, dim3(nb), dim3(256), 0, s, (const f16*)base, g, out); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace stn
