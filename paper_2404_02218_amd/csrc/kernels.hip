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
#include <algorithm>
#include <climits>
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
    for (int k = b; k < e; k++) {
        const int s = src.grp[k];
        v = inject<T>(v, src.amp[(int64_t)arow * src.n + s] * (src.scale ? src.scale[s] : 1.0));
    }
    Storage<T>::store(p, v);
}

template <typename T>
__global__ void k_record(const T* base, RecList rec, int trow) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rec.n) return;
    rec.trace[(int64_t)trow * rec.n + r] = (double)Storage<T>::load(base + rec.off[r]);
}

// Box copies between a field and a contiguous buffer (C order within a box,
// boxes one after another): pack, unpack, and field-to-field (periodic
// self-exchange).  A workgroup serves one box, so the box's parameters are
// uniform; a thread copies one unit, 4 elements where the box's rows are
// 16-byte aligned on both sides (the usual case: faces across x and y start
// at the aligned interior origin), else 1.  Unit -> (row, column) and
// row -> (z, y) use 32-bit division by precomputed multipliers.
struct FastDiv {
    uint32_t m, s, one;   // q = one ? n : (t + ((n - t) >> 1)) >> s, t = mulhi(n, m)
};

constexpr int kCopyBoxes = 8;
struct CopyBox {
    int64_t src, dst;      // field element offsets of the box's first source / destination element
    int64_t buf;           // buffer element of the box's first element
    uint32_t nx, ny, upr, units, vec;   // units per row, units in the box, 4 elements per unit
    FastDiv by_row, by_y;  // divide by upr, by ny
};
struct CopyPlan {
    int n;
    uint32_t bstart[kCopyBoxes + 1];   // first workgroup of each box
    CopyBox box[kCopyBoxes];
};

static FastDiv fast_div(uint32_t d) {
    FastDiv f{0, 0, 0};
    if (d <= 1) {
        f.one = 1;
        return f;
    }
    uint32_t l = 0;
    while ((uint64_t(1) << l) < d) l++;
    f.m = (uint32_t)(((uint64_t(1) << 32) * ((uint64_t(1) << l) - d)) / d + 1);
    f.s = l - 1;
    return f;
}

__device__ static inline uint32_t fdiv(uint32_t n, const FastDiv& f) {
    if (f.one) return n;
    const uint32_t t = __umulhi(n, f.m);
    return (t + ((n - t) >> 1)) >> f.s;
}

template <typename T> struct Vec4;
template <> struct Vec4<uint32_t> { using type = uint4; };
template <> struct Vec4<uint16_t> { using type = uint2; };

template <typename T, int DIR>
__global__ __launch_bounds__(256) void k_boxcopy(T* __restrict__ field, int64_t s0, int64_t s1, CopyPlan P,
                                                 T* __restrict__ buf) {
    using V = typename Vec4<T>::type;
    const uint32_t blk = blockIdx.x;
    int b = 0;
    while (b + 1 < P.n && blk >= P.bstart[b + 1]) b++;
    const CopyBox& B = P.box[b];
    const uint32_t u = (blk - P.bstart[b]) * 256u + threadIdx.x;
    if (u >= B.units) return;
    const uint32_t row = fdiv(u, B.by_row), col = u - row * B.upr;
    const uint32_t z = fdiv(row, B.by_y), y = row - z * B.ny;
    const uint32_t w = B.vec ? 4u : 1u;
    const int64_t fo = (int64_t)z * s0 + (int64_t)y * s1 + (int64_t)(col * w);
    const int64_t bo = B.buf + (int64_t)row * B.nx + (int64_t)(col * w);
    if (B.vec) {
        if constexpr (DIR == COPY_PACK)
            *reinterpret_cast<V*>(buf + bo) = *reinterpret_cast<const V*>(field + B.src + fo);
        else if constexpr (DIR == COPY_UNPACK)
            *reinterpret_cast<V*>(field + B.dst + fo) = *reinterpret_cast<const V*>(buf + bo);
        else
            *reinterpret_cast<V*>(field + B.dst + fo) = *reinterpret_cast<const V*>(field + B.src + fo);
    } else {
        if constexpr (DIR == COPY_PACK)
            buf[bo] = field[B.src + fo];
        else if constexpr (DIR == COPY_UNPACK)
            field[B.dst + fo] = buf[bo];
        else
            field[B.dst + fo] = field[B.src + fo];
    }
}

__global__ void k_zero(uint32_t* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// blockIdx.y: field f of `count` at `stride` elements from p; blockIdx.x:
// plane pz of the allocation, or the tail past the last plane when pz equals
// `planes`.  Halo planes are cleared whole, interior planes in their R halo
// rows and, in the other rows, in the columns outside [xlead, xlead + n2).
__global__ void k_zero_frame(uint32_t* p, int64_t stride, Grid3 g, int halo, int planes, int tail) {
    const int pz = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
    const int64_t s0 = g.s[0];
    const int rowlen = (int)g.rowlen;
    uint32_t* const plane = p + (int64_t)blockIdx.y * stride + (int64_t)pz * s0;
    if (pz == planes) {
        for (int c = tid; c < tail; c += nt) plane[c] = 0u;
        return;
    }
    if (pz < halo || pz >= halo + g.n[0]) {
        uint4* const q = reinterpret_cast<uint4*>(plane);   // s0 is a multiple of 4, the plane 16-byte aligned
        for (int64_t i = tid; i < s0 / 4; i += nt) q[i] = make_uint4(0u, 0u, 0u, 0u);
        return;
    }
    uint32_t* const bottom = plane + (int64_t)(halo + g.n[1]) * rowlen;
    for (int i = tid; i < halo * rowlen; i += nt) {
        plane[i] = 0u;
        bottom[i] = 0u;
    }
    const int xb = (int)g.xlead, xe = xb + g.n[2], npad = xb + rowlen - xe;
    for (int i = tid; i < g.n[1] * npad; i += nt) {
        const int r = i / npad, c = i - r * npad;
        plane[(int64_t)(halo + r) * rowlen + (c < xb ? c : xe + (c - xb))] = 0u;
    }
}

template <typename T>
__global__ void k_beta(const double* m, T* beta, Grid3 g, double scale) {
    const int64_t total = (int64_t)g.n[0] * g.n[1] * g.n[2];
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;
    const int64_t x = q % g.n[2], y = (q / g.n[2]) % g.n[1], z = q / ((int64_t)g.n[2] * g.n[1]);
    Storage<T>::store(beta + g.origin + z * g.s[0] + y * g.s[1] + x, (float)(scale / m[q]));
}

__global__ void k_flush(const float* g32, double* grad, Grid3 g, double scale) {
    const int64_t total = (int64_t)g.n[0] * g.n[1] * g.n[2];
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= total) return;
    const int64_t x = q % g.n[2], y = (q / g.n[2]) % g.n[1], z = q / ((int64_t)g.n[2] * g.n[1]);
    grad[q] += scale * (double)g32[g.origin + z * g.s[0] + y * g.s[1] + x];
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
    if (mode == MODE_WAVE_D || mode == MODE_WAVE_ADJ || mode == MODE_WAVE_ADJ2 || mode == MODE_WAVE_DAMP) {
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
    if (mode == MODE_WAVE_DAMP && radius == 4 && dtype == DT_F32) return tb2_wave_damp_f32(v, w, arow, trow_u, trow_p, s);
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

hipError_t launch_zmarch_batch_persistent(int radius, int dtype, int cfg, const ZView* d_views, const int* d_list,
                                          const int* d_off, int grid, const Coefs& w, int t0, int t1, int rec_on,
                                          int pmask, unsigned long long* d_sync, int spin_limit, hipStream_t s) {
    switch (dtype) {
        case DT_F32:
            return zmarch_batch_persistent_f32(radius, cfg, d_views, d_list, d_off, grid, w, t0, t1, rec_on, pmask,
                                               d_sync, spin_limit, s);
        case DT_BF16:
            return zmarch_batch_persistent_bf16(radius, cfg, d_views, d_list, d_off, grid, w, t0, t1, rec_on, pmask,
                                                d_sync, spin_limit, s);
        case DT_F16:
            return zmarch_batch_persistent_f16(radius, cfg, d_views, d_list, d_off, grid, w, t0, t1, rec_on, pmask,
                                               d_sync, spin_limit, s);
    }
    return hipErrorInvalidValue;
}

hipError_t zmarch_batch_persistent_per_cu(int radius, int dtype, int cfg, int* per_cu) {
    switch (dtype) {
        case DT_F32: return zmarch_batch_persistent_per_cu_f32(radius, cfg, per_cu);
        case DT_BF16: return zmarch_batch_persistent_per_cu_bf16(radius, cfg, per_cu);
        case DT_F16: return zmarch_batch_persistent_per_cu_f16(radius, cfg, per_cu);
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

// interpolated sources: amp8[t][e] = w[e] * amp[t][e >> shift] (FP64), the
// amount of corner entry e of source e >> shift
__global__ void k_spread(const double* amp, const double* w, int shift, int64_t n8, int64_t rows, double* amp8) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows * n8) return;
    const int64_t t = i / n8, e = i - t * n8;
    amp8[i] = w[e] * amp[t * (n8 >> shift) + (e >> shift)];
}

hipError_t launch_spread(const double* amp, const double* w, int shift, int64_t n8, int64_t rows, double* amp8,
                         hipStream_t s) {
    if (n8 == 0 || rows == 0) return hipSuccess;
    const int64_t total = n8 * rows;
    hipLaunchKernelGGL(k_spread, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, amp, w, shift, n8, rows,
                       amp8);
    return hipGetLastError();
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

template <typename T, int DIR>
static hipError_t boxcopy_launch(T* f, const Grid3& g, const CopyPlan& P, T* b, hipStream_t s) {
    if (P.n == 0 || P.bstart[P.n] == 0) return hipSuccess;
    hipLaunchKernelGGL((k_boxcopy<T, DIR>), dim3(P.bstart[P.n]), dim3(256), 0, s, f, g.s[0], g.s[1], P, b);
    return hipGetLastError();
}

template <typename T>
static hipError_t boxcopy_t(int dir, void* field, const Grid3& g, int64_t offset, const CopyList& L, void* buf,
                            hipStream_t s) {
    T* f = (T*)field;
    T* bp = (T*)buf;
    auto launch = [&](const CopyPlan& P) -> hipError_t {
        if (dir == COPY_PACK) return boxcopy_launch<T, COPY_PACK>(f, g, P, bp, s);
        if (dir == COPY_UNPACK) return boxcopy_launch<T, COPY_UNPACK>(f, g, P, bp, s);
        return boxcopy_launch<T, COPY_FIELD>(f, g, P, bp, s);
    };
    // rows of 4-element units must be 16-byte (4-element) aligned in every
    // buffer the direction touches
    const bool buf_ok = dir == COPY_FIELD || ((uintptr_t)buf % (4 * sizeof(T)) == 0);
    const bool strides_ok = g.s[0] % 4 == 0 && g.s[1] % 4 == 0;
    constexpr uint32_t kMaxUnits = 1u << 30;
    CopyPlan P{};
    for (int k = 0; k < L.n; k++) {
        const int64_t nz = L.size[k][0], ny = L.size[k][1], nx = L.size[k][2];
        if (nz <= 0 || ny <= 0 || nx <= 0) continue;
        const int64_t src0 = offset + L.src[k][0] * g.s[0] + L.src[k][1] * g.s[1] + L.src[k][2];
        const int64_t dst0 = offset + L.dst[k][0] * g.s[0] + L.dst[k][1] * g.s[1] + L.dst[k][2];
        bool vec = nx % 4 == 0 && strides_ok && buf_ok && L.start[k] % 4 == 0;
        if (dir != COPY_UNPACK) vec = vec && src0 % 4 == 0;
        if (dir != COPY_PACK) vec = vec && dst0 % 4 == 0;
        const int64_t upr = vec ? nx / 4 : nx;
        if (upr * ny >= kMaxUnits) return hipErrorInvalidValue;   // a plane of one box beyond 2^30 units
        // split along z so that each piece stays below 2^30 units
        const int64_t zstep = std::max<int64_t>(1, kMaxUnits / (upr * ny));
        for (int64_t z0 = 0; z0 < nz; z0 += zstep) {
            const int64_t zn = std::min(zstep, nz - z0);
            if (P.n == kCopyBoxes) {
                const hipError_t e = launch(P);
                if (e != hipSuccess) return e;
                P = CopyPlan{};
            }
            CopyBox& B = P.box[P.n];
            B.src = src0 + z0 * g.s[0];
            B.dst = dst0 + z0 * g.s[0];
            B.buf = L.start[k] + z0 * ny * nx;
            B.nx = (uint32_t)nx;
            B.ny = (uint32_t)ny;
            B.upr = (uint32_t)upr;
            B.units = (uint32_t)(upr * ny * zn);
            B.vec = vec ? 1u : 0u;
            B.by_row = fast_div(B.upr);
            B.by_y = fast_div(B.ny);
            P.bstart[P.n + 1] = P.bstart[P.n] + (B.units + 255u) / 256u;
            P.n++;
        }
    }
    return launch(P);
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

hipError_t launch_zero_frame(void* p, int count, int64_t stride_bytes, const Grid3& g, int halo, int64_t elems,
                             hipStream_t s) {
    const int64_t planes = g.n[0] + 2 * (int64_t)halo;
    const int64_t body = planes * g.s[0];
    if (count <= 0) return hipSuccess;
    if (g.nd != 3 || g.s[1] != g.rowlen || g.s[0] != (g.n[1] + 2 * halo) * g.rowlen || g.s[0] % 4 != 0 ||
        body > elems || elems - body > 1024 || planes >= INT_MAX || stride_bytes % 16 != 0 ||
        stride_bytes < elems * 4 || count > 65535 || (reinterpret_cast<uintptr_t>(p) & 15) != 0)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_zero_frame, dim3((unsigned)planes + 1, (unsigned)count), dim3(256), 0, s, (uint32_t*)p,
                       stride_bytes / 4, g, halo, (int)planes, (int)(elems - body));
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

hipError_t launch_flush(const float* g32, double* grad, const Grid3& g, double scale, hipStream_t s) {
    const int64_t total = (int64_t)g.n[0] * g.n[1] * g.n[2];
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_flush, dim3(blocks_for(total, 256)), dim3(256), 0, s, g32, grad, g, scale);
    return hipGetLastError();
}

}  // namespace stn
