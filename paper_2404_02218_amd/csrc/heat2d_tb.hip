// Multi-step 2D heat sweep (FP32, zero halo).  A 2D field of a few hundred
// points per side sits in L2, so a sweep per launch is bound by launch
// latency, not by memory.  Here a workgroup loads its TX x TY tile plus a
// halo of R*T points into LDS, takes T steps there (step s is valid on the
// tile grown by R*(T-s) points; points outside the interior stay 0, the
// Dirichlet halo) and writes the tile, so one launch advances T steps.  The
// tiles overlap by the halo and recompute it (overlapped temporal blocking,
// the related work of Section 7).  Each point is evaluated in the canonical
// order of the plain sweep (centre, y pairs, x pairs), so T steps here equal
// T plain sweeps bit for bit.
#include "kernels.hpp"

namespace stn {

namespace {

// one thread per point of the region (up to 1024), so that a step is one
// point per thread between two barriers
template <int R, int T, int TX, int TY>
constexpr int threads_for() {
    const int n = (TX + 2 * R * T) * (TY + 2 * R * T);
    return n >= 1024 ? 1024 : (n + 63) / 64 * 64;
}

template <int R, int T, int TX, int TY>
__global__ __launch_bounds__((threads_for<R, T, TX, TY>())) void k_heat2d_tb(const float* __restrict__ in,
                                                                         float* __restrict__ out, Grid3 g,
                                                                         Coefs w) {
    constexpr int kThreads = threads_for<R, T, TX, TY>();
    constexpr int H = R * T, EX = TX + 2 * H, EY = TY + 2 * H, PX = EX + 1;
    __shared__ float A[EY * PX], B[EY * PX];
    const int nx = g.n[2], ny = g.n[1];
    const int ntx = (nx + TX - 1) / TX;
    const int X0 = (int)(blockIdx.x % ntx) * TX - H, Y0 = (int)(blockIdx.x / ntx) * TY - H;
    const int64_t sy = g.s[1];
    const float* U = in + g.origin;
    for (int i = threadIdx.x; i < EX * EY; i += kThreads) {
        const int ly = i / EX, lx = i - ly * EX, y = Y0 + ly, x = X0 + lx;
        A[ly * PX + lx] = (y >= 0 && y < ny && x >= 0 && x < nx) ? U[(int64_t)y * sy + x] : 0.f;
    }
    __syncthreads();
    auto step = [&](const float* S, float* D, int s) __attribute__((always_inline)) {
        const int lo = R * s, wx = EX - 2 * lo, wy = EY - 2 * lo;
        for (int i = threadIdx.x; i < wx * wy; i += kThreads) {
            const int ly = lo + i / wx, lx = lo + i % wx, y = Y0 + ly, x = X0 + lx;
            float v = 0.f;
            if (y >= 0 && y < ny && x >= 0 && x < nx) {
                const float* p = S + ly * PX + lx;
                const float c = p[0];
                float acc = w.cd0 * c, m[R], q[R];
#pragma unroll
                for (int k = 1; k <= R; k++) {
                    m[k - 1] = p[-k * PX];
                    q[k - 1] = p[k * PX];
                }
                acc = axis_sum<R>(acc, w, m, q);
#pragma unroll
                for (int k = 1; k <= R; k++) {
                    m[k - 1] = p[-k];
                    q[k - 1] = p[k];
                }
                acc = axis_sum<R>(acc, w, m, q);
                v = time_update<MODE_HEAT>(acc, c, 0.f, 0.f);
            }
            D[ly * PX + lx] = v;
        }
        __syncthreads();
    };
#pragma unroll
    for (int s = 1; s <= T; s++) {
        if (s & 1)
            step(A, B, s);
        else
            step(B, A, s);
    }
    const float* F = (T & 1) ? B : A;
    float* O = out + g.origin;
    for (int i = threadIdx.x; i < TX * TY; i += kThreads) {
        const int ly = H + i / TX, lx = H + i % TX, y = Y0 + ly, x = X0 + lx;
        if (y < ny && x < nx) O[(int64_t)y * sy + x] = F[ly * PX + lx];
    }
}

template <int R, int T, int TX, int TY>
hipError_t launch_cfg(const float* in, float* out, const Grid3& g, const Coefs& w, hipStream_t s) {
    const int64_t nb = (int64_t)((g.n[2] + TX - 1) / TX) * ((g.n[1] + TY - 1) / TY);
    if (nb == 0) return hipSuccess;
    hipLaunchKernelGGL((k_heat2d_tb<R, T, TX, TY>), dim3((unsigned)nb), dim3(threads_for<R, T, TX, TY>()), 0, s,
                       in, out, g, w);
    return hipGetLastError();
}

template <int R>
hipError_t launch_r(int cfg, const float* in, float* out, const Grid3& g, const Coefs& w, hipStream_t s) {
    static_assert(sizeof(kHeat2dCfgs) / sizeof(kHeat2dCfgs[0]) == 4, "one case per configuration");
    switch (cfg) {
        case 0: return launch_cfg<R, kHeat2dCfgs[0].t, kHeat2dCfgs[0].tx, kHeat2dCfgs[0].ty>(in, out, g, w, s);
        case 1: return launch_cfg<R, kHeat2dCfgs[1].t, kHeat2dCfgs[1].tx, kHeat2dCfgs[1].ty>(in, out, g, w, s);
        case 2: return launch_cfg<R, kHeat2dCfgs[2].t, kHeat2dCfgs[2].tx, kHeat2dCfgs[2].ty>(in, out, g, w, s);
        case 3: return launch_cfg<R, kHeat2dCfgs[3].t, kHeat2dCfgs[3].tx, kHeat2dCfgs[3].ty>(in, out, g, w, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_heat2d_tb(int cfg, int radius, const float* in, float* out, const Grid3& g, const Coefs& w,
                            hipStream_t s) {
    if (radius == 1) return launch_r<1>(cfg, in, out, g, w, s);
    if (radius == 2) return launch_r<2>(cfg, in, out, g, w, s);
    return hipErrorInvalidValue;
}

}  // namespace stn
