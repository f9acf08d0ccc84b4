// HIP kernels of the star-stencil sweep for gfx950 (CDNA4, 64-wide waves).
//
//  k_point   one thread per output point of a box: the general kernel for
//            1D/2D plans, sub-box applies, and variant 0 of 3D plans.
//  k_zmarch  the 3D sweep: each workgroup owns an xy tile (TX x TY) and marches
//            a chunk of z.  Every thread keeps the 2r+1 planes of its own
//            columns in registers (the z taps), stages the current plane with
//            its x/y halo in LDS (double-buffered, one barrier per plane) and
//            reads the in-plane taps from there as 16-byte LDS reads.  Loads of
//            plane z+r+1, the halo of plane z+1 and the centre values of the
//            previous level and beta are issued one plane ahead.  Workgroups are
//            remapped so that each XCD runs a contiguous range of tiles, whose
//            shared halo rows then hit that XCD's L2.  Sources are injected in
//            FP64 by the owning thread; receivers of the input level are read
//            by the first workgroup.
//  k_zmarch_batch  the same tile body over a flattened tile list of many
//            independent shots (one launch per step for all shots).
//  (k_zmarch and k_zmarch_batch are templates in zmarch.hpp, instantiated
//  per storage type in zmarch_*.hip; this file holds the rest.)
//  small kernels: source injection / receiver sampling for k_point runs, box
//            copies (halo pack, unpack, periodic self-exchange), zero fill,
//            beta from squared slowness, FP64 gradient flush.
#include <type_traits>

#include "kernels.hpp"

namespace stn {

// --------------------------------------------------------------- k_point
template <int MODE, int R, typename T, int ND>
__global__ __launch_bounds__(256) void k_point(ZView v, Coefs w, Box3 box) {
    using S = Storage<T>;
    const int64_t total = box.n[0] * box.n[1] * box.n[2];
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= total) return;
    const int64_t x = box.lo[2] + i % box.n[2];
    const int64_t y = box.lo[1] + (i / box.n[2]) % box.n[1];
    const int64_t z = box.lo[0] + i / (box.n[2] * box.n[1]);
    const int64_t off = v.g.origin + z * v.g.s[0] + y * v.g.s[1] + x;
    const T* U = (const T*)v.u;
    const float ctr = S::load(U + off);
    float acc = w.cd0 * ctr;
    float m[R], p[R];
    if constexpr (ND == 3) {
#pragma unroll
        for (int k = 1; k <= R; k++) {
            m[k - 1] = S::load(U + off - k * v.g.s[0]);
            p[k - 1] = S::load(U + off + k * v.g.s[0]);
        }
        acc = axis_sum<R>(acc, w, m, p);
    }
    if constexpr (ND >= 2) {
#pragma unroll
        for (int k = 1; k <= R; k++) {
            m[k - 1] = S::load(U + off - k * v.g.s[1]);
            p[k - 1] = S::load(U + off + k * v.g.s[1]);
        }
        acc = axis_sum<R>(acc, w, m, p);
    }
#pragma unroll
    for (int k = 1; k <= R; k++) {
        m[k - 1] = S::load(U + off - k);
        p[k - 1] = S::load(U + off + k);
    }
    acc = axis_sum<R>(acc, w, m, p);
    float prev = 0.f, beta = 0.f;
    if constexpr (MODE != MODE_HEAT) {
        prev = S::load((const T*)v.prev + off);
        beta = S::load((const T*)v.beta + off);
    }
    if constexpr (MODE == MODE_WAVE_DAMP) {
        const float g = (v.damp[z] + v.damp[v.g.n[0] + y]) + v.damp[v.g.n[0] + v.g.n[1] + x];
        S::store((T*)v.out + off, damped_update(acc, ctr, prev, beta, g));
    } else {
        S::store((T*)v.out + off, time_update<MODE>(acc, ctr, prev, beta));
    }
}

// ---------------------------------------------------------- small kernels
template <typename T>
__global__ void k_inject(T* base, SrcList src, int arow) {
    // one thread per distinct position: its entries in index order, as the
    // z-marching kernels inject them
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= src.ngrp) return;
    const int b = src.gbeg[g], e = src.gbeg[g + 1];
    T* p = base + src.off[src.grp[b]];
    float v = Storage<T>::load(p);
    for (int k = b; k < e; k++) v = inject<T>(v, src_amount(src, arow, src.grp[k]));
    Storage<T>::store(p, v);
}

template <typename T>
__global__ void k_record(const T* base, RecList rec, int trow) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rec.n) return;
    rec.trace[(int64_t)trow * rec.n + r] = (double)Storage<T>::load(base + rec.off[r]);
}

// element copies between boxes of a field and a contiguous buffer (C order)
template <typename T, int DIR>
__global__ void k_boxcopy(T* field, int64_t offset, int64_t s0, int64_t s1, CopyList L, T* buf) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= L.start[L.n]) return;
    int b = 0;
    while (b + 1 < L.n && i >= L.start[b + 1]) b++;
    const int64_t j = i - L.start[b];
    const int64_t nx = L.size[b][2], ny = L.size[b][1];
    const int64_t x = j % nx, y = (j / nx) % ny, z = j / (nx * ny);
    const int64_t src = offset + (L.src[b][0] + z) * s0 + (L.src[b][1] + y) * s1 + (L.src[b][2] + x);
    const int64_t dst = offset + (L.dst[b][0] + z) * s0 + (L.dst[b][1] + y) * s1 + (L.dst[b][2] + x);
    if constexpr (DIR == COPY_PACK)
        buf[i] = field[src];
    else if constexpr (DIR == COPY_UNPACK)
        field[dst] = buf[i];
    else
        field[dst] = field[src];
}

__global__ void k_zero(uint32_t* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

template <typename T>
__global__ void k_beta(const double* m, T* beta, Grid3 g, double scale) {
    const int64_t total = (int64_t)g.n[0] * g.n[1] * g.n[2];
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;
    const int64_t x = q % g.n[2], y = (q / g.n[2]) % g.n[1], z = q / ((int64_t)g.n[2] * g.n[1]);
    Storage<T>::store(beta + g.origin + z * g.s[0] + y * g.s[1] + x, (float)(scale / m[q]));
}

__global__ void k_flush(float* g32, double* grad, Grid3 g, double scale) {
    const int64_t total = (int64_t)g.n[0] * g.n[1] * g.n[2];
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;
    const int64_t x = q % g.n[2], y = (q / g.n[2]) % g.n[1], z = q / ((int64_t)g.n[2] * g.n[1]);
    float* p = g32 + g.origin + z * g.s[0] + y * g.s[1] + x;
    grad[q] += scale * (double)(*p);
    *p = 0.f;
}

// ----------------------------------------------------------- dispatchers
static inline unsigned blocks_for(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

template <int MODE, typename T, int R>
static hipError_t point_nd(const ZView& v, const Coefs& w, const Box3& box, hipStream_t s) {
    const int64_t total = box.n[0] * box.n[1] * box.n[2];
    if (total == 0) return hipSuccess;
    const unsigned nb = blocks_for(total, 256);
    if (v.g.nd == 3)
        hipLaunchKernelGGL((k_point<MODE, R, T, 3>), dim3(nb), dim3(256), 0, s, v, w, box);
    else if (v.g.nd == 2)
        hipLaunchKernelGGL((k_point<MODE, R, T, 2>), dim3(nb), dim3(256), 0, s, v, w, box);
    else
        hipLaunchKernelGGL((k_point<MODE, R, T, 1>), dim3(nb), dim3(256), 0, s, v, w, box);
    return hipGetLastError();
}

template <int MODE, typename T>
static hipError_t point_r(int radius, const ZView& v, const Coefs& w, const Box3& box, hipStream_t s) {
    switch (radius) {
        case 1: return point_nd<MODE, T, 1>(v, w, box, s);
        case 2: return point_nd<MODE, T, 2>(v, w, box, s);
        case 3: return point_nd<MODE, T, 3>(v, w, box, s);
        case 4: return point_nd<MODE, T, 4>(v, w, box, s);
    }
    return hipErrorInvalidValue;
}

template <typename T>
static hipError_t point_m(int mode, int radius, const ZView& v, const Coefs& w, const Box3& box, hipStream_t s) {
    if (mode == MODE_HEAT) return point_r<MODE_HEAT, T>(radius, v, w, box, s);
    if (mode == MODE_WAVE) return point_r<MODE_WAVE, T>(radius, v, w, box, s);
    if constexpr (std::is_same<T, float>::value)
        if (mode == MODE_WAVE_DAMP) return point_r<MODE_WAVE_DAMP, T>(radius, v, w, box, s);
    return hipErrorInvalidValue;
}

hipError_t launch_point(int mode, int radius, int dtype, const ZView& v, const Coefs& w, const Box3& box,
                        hipStream_t s) {
    switch (dtype) {
        case DT_F32: return point_m<float>(mode, radius, v, w, box, s);
        case DT_BF16: return point_m<bf16>(mode, radius, v, w, box, s);
        case DT_F16: return point_m<f16>(mode, radius, v, w, box, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_zmarch(int mode, int radius, int dtype, int cfg, const ZView& v, const Coefs& w, int parity,
                         int arow, int trow, hipStream_t s) {
    if (mode == MODE_WAVE_D || mode == MODE_WAVE_ADJ || mode == MODE_WAVE_DAMP) {
        // the adjoint path and the absorbing layer are FP32 only
        if (dtype != DT_F32) return hipErrorInvalidValue;
        return zmarch_adj_f32(mode, radius, cfg, v, w, parity, arow, trow, s);
    }
    switch (dtype) {
        case DT_F32: return zmarch_fwd_f32(mode, radius, cfg, v, w, parity, arow, trow, s);
        case DT_BF16: return zmarch_fwd_bf16(mode, radius, cfg, v, w, parity, arow, trow, s);
        case DT_F16: return zmarch_fwd_f16(mode, radius, cfg, v, w, parity, arow, trow, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_tb2(int mode, int radius, int dtype, const TBView& v, const Coefs& w, int arow, int trow_u,
                      int trow_p, hipStream_t s) {
    if (mode == MODE_WAVE && radius == 4) return tb2_wave(dtype, v, w, arow, trow_u, trow_p, s);
    if (mode == MODE_HEAT && dtype == DT_F32) return tb2_heat_f32(radius, v, w, s);
    return hipErrorInvalidValue;
}

hipError_t launch_zmarch_batch(int radius, int dtype, int cfg, const ZView* d_views, const int* d_block_map,
                               int nblocks, const Coefs& w, int parity, int arow, int trow, hipStream_t s) {
    switch (dtype) {
        case DT_F32: return zmarch_batch_f32(radius, cfg, d_views, d_block_map, nblocks, w, parity, arow, trow, s);
        case DT_BF16: return zmarch_batch_bf16(radius, cfg, d_views, d_block_map, nblocks, w, parity, arow, trow, s);
        case DT_F16: return zmarch_batch_f16(radius, cfg, d_views, d_block_map, nblocks, w, parity, arow, trow, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_inject(int dtype, void* out_base, const Grid3& g, const SrcList& src, int arow, hipStream_t s) {
    if (src.ngrp == 0) return hipSuccess;
    const unsigned nb = blocks_for(src.ngrp, 64);
    switch (dtype) {
        case DT_F32: hipLaunchKernelGGL(k_inject<float>, dim3(nb), dim3(64), 0, s, (float*)out_base + g.origin, src, arow); break;
        case DT_BF16: hipLaunchKernelGGL(k_inject<bf16>, dim3(nb), dim3(64), 0, s, (bf16*)out_base + g.origin, src, arow); break;
        case DT_F16: hipLaunchKernelGGL(k_inject<f16>, dim3(nb), dim3(64), 0, s, (f16*)out_base + g.origin, src, arow); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// interpolated receivers: trace[t][r] = sum over the nc corners c, in order,
// of w[r][c] * trace8[t][r][c] (FP64)
__global__ void k_gather(const double* trace8, const double* w, int nc, int64_t n, int64_t rows, double* trace) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows * n) return;
    const int64_t t = i / n, r = i - t * n;
    const double* v = trace8 + (t * n + r) * nc;
    double acc = 0.0;
    for (int c = 0; c < nc; c++) acc = fma(w[r * nc + c], v[c], acc);
    trace[i] = acc;
}

hipError_t launch_gather(const double* trace8, const double* w, int nc, int64_t n, int64_t rows, double* trace,
                         hipStream_t s) {
    if (n == 0 || rows == 0) return hipSuccess;
    const int64_t total = n * rows;
    hipLaunchKernelGGL(k_gather, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, trace8, w, nc, n, rows,
                       trace);
    return hipGetLastError();
}

hipError_t launch_record(int dtype, const void* base, const Grid3& g, const RecList& rec, int trow, hipStream_t s) {
    if (rec.n == 0) return hipSuccess;
    const unsigned nb = blocks_for(rec.n, 64);
    switch (dtype) {
        case DT_F32: hipLaunchKernelGGL(k_record<float>, dim3(nb), dim3(64), 0, s, (const float*)base + g.origin, rec, trow); break;
        case DT_BF16: hipLaunchKernelGGL(k_record<bf16>, dim3(nb), dim3(64), 0, s, (const bf16*)base + g.origin, rec, trow); break;
        case DT_F16: hipLaunchKernelGGL(k_record<f16>, dim3(nb), dim3(64), 0, s, (const f16*)base + g.origin, rec, trow); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T>
static hipError_t boxcopy_t(int dir, void* field, const Grid3& g, int64_t offset, const CopyList& L, void* buf,
                            hipStream_t s) {
    const int64_t total = L.start[L.n];
    if (total == 0) return hipSuccess;
    const unsigned nb = blocks_for(total, 256);
    T* f = (T*)field;
    T* b = (T*)buf;
    if (dir == COPY_PACK)
        hipLaunchKernelGGL((k_boxcopy<T, COPY_PACK>), dim3(nb), dim3(256), 0, s, f, offset, g.s[0], g.s[1], L, b);
    else if (dir == COPY_UNPACK)
        hipLaunchKernelGGL((k_boxcopy<T, COPY_UNPACK>), dim3(nb), dim3(256), 0, s, f, offset, g.s[0], g.s[1], L, b);
    else
        hipLaunchKernelGGL((k_boxcopy<T, COPY_FIELD>), dim3(nb), dim3(256), 0, s, f, offset, g.s[0], g.s[1], L, b);
    return hipGetLastError();
}

hipError_t launch_boxcopy(int dtype, int dir, void* field, const Grid3& g, int64_t offset, const CopyList& L,
                          void* buf, hipStream_t s) {
    // a copy moves storage bits, so 16-bit types share one instantiation
    if (dtype == DT_F32) return boxcopy_t<uint32_t>(dir, field, g, offset, L, buf, s);
    return boxcopy_t<uint16_t>(dir, field, g, offset, L, buf, s);
}

hipError_t launch_zero(void* p, int64_t bytes, hipStream_t s) {
    const int64_t n = bytes / 4;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero, dim3(blocks_for(n, 256)), dim3(256), 0, s, (uint32_t*)p, n);
    return hipGetLastError();
}

hipError_t launch_beta(int dtype, const double* m, void* beta, const Grid3& g, double scale, hipStream_t s) {
    const int64_t total = (int64_t)g.n[0] * g.n[1] * g.n[2];
    if (total == 0) return hipSuccess;
    const unsigned nb = blocks_for(total, 256);
    switch (dtype) {
        case DT_F32: hipLaunchKernelGGL(k_beta<float>, dim3(nb), dim3(256), 0, s, m, (float*)beta, g, scale); break;
        case DT_BF16: hipLaunchKernelGGL(k_beta<bf16>, dim3(nb), dim3(256), 0, s, m, (bf16*)beta, g, scale); break;
        case DT_F16: hipLaunchKernelGGL(k_beta<f16>, dim3(nb), dim3(256), 0, s, m, (f16*)beta, g, scale); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_flush(float* g32, double* grad, const Grid3& g, double scale, hipStream_t s) {
    const int64_t total = (int64_t)g.n[0] * g.n[1] * g.n[2];
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_flush, dim3(blocks_for(total, 256)), dim3(256), 0, s, g32, grad, g, scale);
    return hipGetLastError();
}

}  // namespace stn
