// Temporal blocking of depth 2: one launch advances a sweep by two steps.
//  * radius-4 wave: reads u^n, u^{n-1} and beta once and writes u^{n+1} and
//    u^{n+2} to two other buffers, so a point-update moves 10 bytes of FP32
//    storage instead of 16;
//  * heat (any radius up to 4): reads u^n and writes u^{n+2}, 4 bytes per
//    point-update instead of 8.
//
// A workgroup owns a 64 x 32 tile of the xy plane and a z-chunk and marches up
// the chunk.  Its first 512 threads (8 wavefronts) own one 4-point group of
// the tile each (tile role); the next 256 own one group of the ring around the
// tile and one margin group of the u^n plane (ring role; the lanes beyond the
// 208 ring and 224 margin groups repeat the last group and write the same
// values to the same places, so that no wavefront branches on its lanes).
// Per plane z1:
//   stage 1 computes u^{n+1} at z1 on the extended region E = the tile plus a
//           ring of R points on each side in x and y.  Ring points are also
//           computed by the neighbouring tiles, with the same operations, so
//           every copy has the same bits.  E points outside the interior are
//           the zero halo of u^{n+1} and are set to 0;
//   stage 2 computes u^{n+2} at z = z1 - R on the tile: z taps from a register
//           ring of the group's own u^{n+1}, in-plane taps from an LDS ring of
//           the last R+1 planes of u^{n+1} over E, u^n at z from the group's
//           u^n register ring.
// Planes zb-R .. ze+R-1 of u^{n+1} are computed for a chunk [zb, ze); the 2R
// extra planes are recomputed by the neighbouring chunk in the same way.
//
// Every point is evaluated with the canonical operation order of the plain
// sweep (centre, z pairs, y pairs, x pairs, time update) and u^{n+1} passes
// through the storage type before stage 2 uses it, so two steps of this
// kernel equal two plain sweeps bit for bit.
#pragma once

#include <climits>
#include <type_traits>

#include "zmarch.hpp"

namespace stn {

template <int R_, bool WAVE_>
struct TB2 {
    static constexpr int R = R_, Q = 2 * R + 1;
    static constexpr bool WAVE = WAVE_;
    static constexpr int TX = 64, TY = 32;
    static constexpr int NTILE = (TX / 4) * TY;                       // 512 tile-role threads
    static constexpr int NRT = 256;                                   // ring-role threads
    static constexpr int NT = NTILE + NRT;
    static constexpr int EG = TX / 4 + 2, EY = TY + 2 * R;           // E: 18 groups x 40 rows
    static constexpr int W1 = TX + 16, H1 = TY + 4 * R, P1 = W1 * H1;  // u^n plane: E + R margin
    static constexpr int W2 = TX + 8, P2 = W2 * EY;                   // u^{n+1} plane over E
    static constexpr int NS1 = 2, NS2 = R + 1;   // NS2: u^{n+1} planes z1-R .. z1
    static constexpr int NRING = EG * EY - NTILE;                      // 208 ring groups
    static constexpr int NMX = 2 * EY, NMY = 2 * R * EG, NMARG = NMX + NMY;  // 224 margin groups
    // LDS: NS1 u^n planes, NS2 u^{n+1} planes, and (wave) NS2 planes of the
    // tile groups' own beta (each read back only by its thread)
    static constexpr int LDS_FLOATS = NS1 * P1 + NS2 * P2 + (WAVE ? NS2 * NTILE * 4 : 0);
    static_assert(R >= 1 && R <= 4, "the x ring and margins are one 4-point group wide");
    // waves per SIMD the register budget is sized for: the wave kernel needs
    // its registers at one workgroup per CU (3 waves per SIMD); the heat
    // kernel with r <= 2 fits two workgroups per CU (6 waves per SIMD)
    static constexpr int WAVES_PER_SIMD = (!WAVE && R <= 2) ? 6 : 3;
    static_assert(NRING <= NRT && NMARG <= NRT, "one ring and one margin group per ring-role thread");
    static_assert(NTILE % 64 == 0 && NRT % 64 == 0, "roles split at wavefront boundaries");
};

// ring group k of E as (ex, ey): R rows above, R rows below, then the left
// and right columns of the tile rows
template <int R>
__device__ static inline void tb2_ring_group(int k, int& ex, int& ey) {
    using Z = TB2<R, false>;
    constexpr int top = Z::EG * Z::R;
    if (k < top) {
        ey = k / Z::EG;
        ex = k % Z::EG;
    } else if (k < 2 * top) {
        ey = Z::R + Z::TY + (k - top) / Z::EG;
        ex = (k - top) % Z::EG;
    } else if (k < 2 * top + Z::TY) {
        ey = Z::R + (k - 2 * top);
        ex = 0;
    } else {
        ey = Z::R + (k - 2 * top - Z::TY);
        ex = Z::EG - 1;
    }
}

// Star update of one 4-point group.  zt(k) returns logical plane k of the
// group's z column (k = 0 .. 2R, centre k = R); `L` points at the group's own
// position in an LDS plane of pitch W (x taps from the groups on either side,
// y taps from the rows above and below).  The four points advance through
// the canonical order of each point's sum (centre, z pairs, y pairs, x pairs,
// k = 1 .. R within an axis).
template <int R, int MODE, class ZT>
__device__ __forceinline__ void tb2_star(const Coefs& w, ZT&& zt, const float* L, int W, const float4& prev,
                                         const float4& beta, const float4& gam, float (&o)[4]) {
    const float4 c = zt(R);
    float acc[4];
#pragma unroll
    for (int i = 0; i < 4; i++) acc[i] = w.cd0 * comp(c, i);
#pragma unroll
    for (int k = 1; k <= R; k++) {
        const float4 m = zt(R - k), p = zt(R + k);
#pragma unroll
        for (int i = 0; i < 4; i++) acc[i] = fmaf(w.c[k], comp(m, i) + comp(p, i), acc[i]);
    }
    if constexpr (MODE == MODE_HEAT) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 1; k <= R; k++) {
        const float4 m = *reinterpret_cast<const float4*>(L - k * W);
        const float4 p = *reinterpret_cast<const float4*>(L + k * W);
#pragma unroll
        for (int i = 0; i < 4; i++) acc[i] = fmaf(w.c[k], comp(m, i) + comp(p, i), acc[i]);
        // the heat kernels run at 6 waves per SIMD: keep one pair of taps in
        // registers at a time
        if constexpr (MODE == MODE_HEAT) __builtin_amdgcn_sched_barrier(0);
    }
    const float4 xl = *reinterpret_cast<const float4*>(L - 4);
    const float4 xr = *reinterpret_cast<const float4*>(L + 4);
    const float xv[12] = {xl.x, xl.y, xl.z, xl.w, c.x, c.y, c.z, c.w, xr.x, xr.y, xr.z, xr.w};
#pragma unroll
    for (int i = 0; i < 4; i++) {
        float m[R], p[R];
#pragma unroll
        for (int k = 1; k <= R; k++) {
            m[k - 1] = xv[4 + i - k];
            p[k - 1] = xv[4 + i + k];
        }
        acc[i] = axis_sum<R>(acc[i], w, m, p);
        if constexpr (MODE == MODE_WAVE_DAMP)
            o[i] = damped_update(acc[i], comp(c, i), comp(prev, i), comp(beta, i), comp(gam, i));
        else
            o[i] = time_update<MODE>(acc[i], comp(c, i), comp(prev, i), comp(beta, i));
    }
}

// Point lists and amplitudes are invariant during a launch: reading them
// through the constant address space makes them scalar loads, which the
// vector memory counter does not track.  (As vector loads whose results only
// some lanes use, they made the compiler wait for every outstanding load and
// store of the wave before stage 2.)
template <typename U>
__device__ __forceinline__ U tb2_ldc(const U* p) {
    return *(const __attribute__((address_space(4))) U*)p;
}

// first source of a tile's z-sorted list at or after plane z0
__device__ static inline void tb2_src_first(const SrcList& s, int tile, int z0, int& next, int& end, int& znext) {
    next = end = 0;
    znext = INT_MAX;
    if (s.n > 0) {
        next = tb2_ldc(s.tile_begin + tile);
        end = tb2_ldc(s.tile_begin + tile + 1);
        while (next < end && tb2_ldc(s.zyx4 + 4 * next) < z0) next++;
        znext = next < end ? tb2_ldc(s.zyx4 + 4 * next) : INT_MAX;
    }
}

// Raw buffer loads: a wave-uniform resource (base, byte range) in scalar
// registers, a wave-uniform byte offset (the plane) and a 32-bit byte offset
// per lane (the position in the plane).  Offsets past the range read as zero
// instead of faulting.
inline constexpr int kBufferConfig = 0x00020000;   // raw 32-bit data, gfx9 family

template <typename T>
__device__ __forceinline__ float4 tb2_bload4(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff);

template <>
__device__ __forceinline__ float4 tb2_bload4<float>(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    const f4 v = __builtin_bit_cast(f4, __builtin_amdgcn_raw_buffer_load_b128(r, off, soff, 0));
    return make_float4(v.x, v.y, v.z, v.w);
}

template <>
__device__ __forceinline__ float4 tb2_bload4<bf16>(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff) {
    typedef uint32_t u2 __attribute__((ext_vector_type(2)));
    const u2 v = __builtin_bit_cast(u2, __builtin_amdgcn_raw_buffer_load_b64(r, off, soff, 0));
    return make_float4(__uint_as_float(v.x << 16), __uint_as_float(v.x & 0xffff0000u), __uint_as_float(v.y << 16),
                       __uint_as_float(v.y & 0xffff0000u));
}

template <>
__device__ __forceinline__ float4 tb2_bload4<f16>(__amdgpu_buffer_rsrc_t r, uint32_t off, uint32_t soff) {
    typedef _Float16 h4 __attribute__((ext_vector_type(4)));
    const h4 v = __builtin_bit_cast(h4, __builtin_amdgcn_raw_buffer_load_b64(r, off, soff, 0));
    return make_float4((float)v.x, (float)v.y, (float)v.z, (float)v.w);
}

// The same loads without widening (RawGroup), for loads that stay in flight
// across a plane's compute: they are widened where the plane is consumed.
template <typename T>
__device__ __forceinline__ typename RawGroup<T>::type tb2_bload_raw(__amdgpu_buffer_rsrc_t r, uint32_t off,
                                                                     uint32_t soff) {
    if constexpr (std::is_same<T, float>::value) {
        return tb2_bload4<float>(r, off, soff);
    } else {
        return __builtin_bit_cast(u2v, __builtin_amdgcn_raw_buffer_load_b64(r, off, soff, 0));
    }
}

// Store a group of 4 points with the streaming hint at byte offset
// voff + soff of the field behind `r`.  full: every point of the group is
// interior (wave-uniform); otherwise points x0 + i >= nx are skipped.
inline constexpr int kStoreNT = 2;   // cache policy: non-temporal

template <typename T>
__device__ __forceinline__ void tb2_store(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, bool full, int x0,
                                          int nx, const float (&o)[4]) {
    if constexpr (std::is_same<T, float>::value) {
        if (full) {
            typedef uint32_t u4 __attribute__((ext_vector_type(4)));
            const u4 v = {__float_as_uint(o[0]), __float_as_uint(o[1]), __float_as_uint(o[2]), __float_as_uint(o[3])};
            __builtin_amdgcn_raw_buffer_store_b128(v, r, voff, soff, kStoreNT);
        } else {
#pragma unroll
            for (int i = 0; i < 4; i++)
                if (x0 + i < nx) __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(o[i]), r, voff + 4 * i, soff, kStoreNT);
        }
    } else {
        if (full) {
            typedef uint32_t u2 __attribute__((ext_vector_type(2)));
            const u2 v = {Storage<T>::pack2(o[0], o[1]), Storage<T>::pack2(o[2], o[3])};
            __builtin_amdgcn_raw_buffer_store_b64(v, r, voff, soff, kStoreNT);
        } else {
#pragma unroll
            for (int i = 0; i < 4; i++)
                if (x0 + i < nx)
                    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(uint16_t, Storage<T>::from_f(o[i])), r,
                                                          voff + 2 * i, soff, kStoreNT);
        }
    }
}

// One workgroup's tile and z-chunk (logical block lb of the field set v).
template <int MODE, int R_, typename T>
__device__ __forceinline__ void tb2_tile(const TBView& v, const Coefs& w, int lb, int arow, int trow_u, int trow_p,
                                         float* __restrict__ lds) {
    constexpr bool WAVE = MODE != MODE_HEAT, DAMP = MODE == MODE_WAVE_DAMP;
    // wave modes: a plane's stores go out after the next plane's loads (see
    // below); the heat form, with one load per plane and 6 waves per SIMD,
    // runs faster storing each plane as it is computed
    constexpr bool DEFER = WAVE;
    using Z = TB2<R_, WAVE>;
    using S = Storage<T>;
    constexpr int R = Z::R, Q = Z::Q, TX = Z::TX, TY = Z::TY, NT = Z::NT;
    constexpr int EG = Z::EG, EY = Z::EY, W1 = Z::W1, P1 = Z::P1, W2 = Z::W2, P2 = Z::P2, NS2 = Z::NS2;
    float* const U1 = lds;
    float* const U2 = lds + Z::NS1 * P1;
    float4* const BQ = reinterpret_cast<float4*>(U2 + NS2 * P2);

    const int tid = threadIdx.x;
    const int ntxy = v.ntx * v.nty;
    const int tile_x = lb % v.ntx, tile_y = (lb / v.ntx) % v.nty, zch = lb / ntxy;
    const int tile = tile_y * v.ntx + tile_x;
    const int X0 = tile_x * TX, Y0 = tile_y * TY;
    const int nx = v.g.n[2], ny = v.g.n[1], nz = v.g.n[0];
    const int zb = zch * v.zc;
    const int ze = min(zb + v.zc, nz);
    const int64_t sz = v.g.s[0], sy = v.g.s[1];
    const T* U = (const T*)v.u + v.g.origin;
    const T* P = (const T*)v.prev + v.g.origin;

    // receivers sample the two input levels (neither is written here)
    if (WAVE && lb == 0 && v.rec.n > 0) {
        for (int r = tid; r < v.rec.n; r += NT) {
            if (trow_u >= 0) v.rec.trace[(int64_t)trow_u * v.rec.n + r] = (double)S::load(U + v.rec.off[r]);
            if (trow_p >= 0) v.rec.trace[(int64_t)trow_p * v.rec.n + r] = (double)S::load(P + v.rec.off[r]);
        }
    }

    // Loads stay inside the field: rows and planes are clamped to the R-deep
    // halo, x groups to the last full group of the row (x >= X0 - 8 needs a
    // row lead of at least 8 elements, which the host checks).  Clamped
    // values only reach points that are forced to zero or not stored.
    // Every field is one buffer resource over its allocation (the host checks
    // it spans less than 2^31 bytes); a plane is a wave-uniform byte offset
    // (row -R, column -8 of the plane) and a lane adds its 32-bit position.
    const int xmax4 = (int)(v.g.rowlen - v.g.xlead) - 4;
    auto goff = [&](int x, int y) -> uint32_t {
        return (uint32_t)(((int64_t)(min(max(y, -R), ny + R - 1) + R) * sy + (min(x, xmax4) + 8)) * sizeof(T));
    };
    auto soff = [&](int z) -> uint32_t {
        return (uint32_t)((v.g.origin + (int64_t)min(max(z, -R), nz + R - 1) * sz - R * sy - 8) * sizeof(T));
    };
    auto rsrc = [&](const void* f) {
        return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(f), (short)0, (int)v.range, kBufferConfig);
    };
    const auto rU = rsrc(v.u), rO2 = rsrc(v.out2);
    const auto rP = WAVE ? rsrc(v.prev) : rU, rB = WAVE ? rsrc(v.beta) : rU, rO1 = WAVE ? rsrc(v.out1) : rO2;
    auto ld = [&](__amdgpu_buffer_rsrc_t r, int z, uint32_t off) -> float4 { return tb2_bload4<T>(r, off, soff(z)); };
    using Raw = typename RawGroup<T>::type;
    auto ldr = [&](__amdgpu_buffer_rsrc_t r, int z, uint32_t off) -> Raw { return tb2_bload_raw<T>(r, off, soff(z)); };

    // This thread's group of E (ex, ey): tile role (ex, ey) = (gx + 1, gy + R);
    // ring role: ring group k.  x0, y0: its first point.  Roles are per
    // wavefront (readfirstlane makes that visible to the compiler).
    const bool tile_role = __builtin_amdgcn_readfirstlane(tid >> 6) < Z::NTILE / 64;
    const int k = tid - Z::NTILE;                       // ring-role index
    int ex, ey;
    if (tile_role) {
        ex = tid % (TX / 4) + 1;
        ey = tid / (TX / 4) + R;
    } else {
        tb2_ring_group<R>(min(k, Z::NRING - 1), ex, ey);
    }
    const int x0 = X0 - 4 + 4 * ex, y0 = Y0 - R + ey;
    const uint32_t ag = goff(x0, y0);
    const int l1 = (ey + R) * W1 + 4 * ex + 4;          // position in a u^n plane
    const int l2 = ey * W2 + 4 * ex;                    // position in a u^{n+1} plane
    // margin group (ring role): 4 columns left and right of each E row, R
    // rows above and below E
    uint32_t am = 0;
    int lm = 0;
    if (!tile_role) {
        const int h = min(k, Z::NMARG - 1);
        if (h < Z::NMX) {
            const int r = h >> 1, side = h & 1;
            am = goff(side ? X0 + TX + 4 : X0 - 8, Y0 - R + r);
            lm = (r + R) * W1 + (side ? W1 - 4 : 0);
        } else {
            const int h2 = h - Z::NMX;
            const int i = h2 / EG, gxm = h2 % EG;
            const int row = i < R ? i : EY + i;
            am = goff(X0 - 4 + 4 * gxm, Y0 - 2 * R + row);
            lm = row * W1 + 4 * gxm + 4;
        }
    }
    bool in[4];
#pragma unroll
    for (int i = 0; i < 4; i++) in[i] = y0 >= 0 && y0 < ny && x0 + i >= 0 && x0 + i < nx;
    const bool store_ok = tile_role && y0 < ny && x0 < nx;   // then ag is unclamped
    const bool full_tile = X0 + TX <= nx && Y0 + TY <= ny;   // wave-uniform

    // qa: this group's u^n planes z1-R .. z1+R.  qx: tile role, the group's
    // u^{n+1} planes z1-2R .. z1; ring role, its margin group of u^n planes
    // z1-R .. z1+R (loaded with the leading plane, when the neighbouring
    // tiles load the same rows as their own, so they come from L2).  cp, cb:
    // u^{n-1} and beta at z1.  u^{n+1} plane p and the tile groups' beta at
    // p live in LDS slot (p - z1b) % (R + 1).
    const int z1b = zb - R, z1e = ze + R;
    float4 qa[Q], qx[Q];
#pragma unroll
    for (int j = 0; j < Q; j++) {
        qa[j] = ld(rU, z1b - R + j, ag);
        qx[j] = tile_role ? make_float4(0.f, 0.f, 0.f, 0.f) : ld(rU, z1b - R + j, am);
    }
    const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
    // absorbing layer: this group's row and column damping (clamped into the
    // interior: values outside it only feed points that are set to 0)
    float4 dgx = zero4;
    float dgy = 0.f;
    if constexpr (DAMP) {
        const float* D = v.damp + v.g.n[0];
        dgy = D[min(max(y0, 0), ny - 1)];
        dgx = make_float4(D[ny + min(max(x0, 0), nx - 1)], D[ny + min(max(x0 + 1, 0), nx - 1)],
                          D[ny + min(max(x0 + 2, 0), nx - 1)], D[ny + min(max(x0 + 3, 0), nx - 1)]);
    }
    auto gamma_at = [&](int z) -> float4 {
        if constexpr (DAMP) {
            const float g = v.damp[min(max(z, 0), nz - 1)] + dgy;
            return make_float4(g + dgx.x, g + dgx.y, g + dgx.z, g + dgx.w);
        } else {
            return zero4;
        }
    };
    float4 cp = zero4, cb = zero4;
    if constexpr (WAVE) {
        cp = ld(rP, z1b, ag);
        cb = ld(rB, z1b, ag);
    }

    // sources (wave): stage 1 walks the sources inside E, stage 2 the tile's own
    int e_next = 0, e_end = 0, e_z = INT_MAX, t_next = 0, t_end = 0, t_z = INT_MAX;
    if constexpr (WAVE) {
        tb2_src_first(v.src_e, tile, z1b, e_next, e_end, e_z);
        tb2_src_first(v.src_t, tile, zb, t_next, t_end, t_z);
    }

    float o2p[4] = {0.f, 0.f, 0.f, 0.f};   // u^{n+2} of the previous plane, stored with the next plane
    int it = 0;   // plane counter: u^n LDS slot it & 1
    int s2 = 0;   // LDS slot of u^{n+1} plane z1
    int z1 = z1b;
    // every call is inlined so that the register rings stay in registers
    auto step = [&](auto off_c) __attribute__((always_inline)) {
        // qa (and qx in the ring role) hold logical plane j (z1-R+j) at
        // (j + OFF) % Q; in the tile role qx holds logical plane j (z1-2R+j)
        // at (j + OFF2) % Q
        constexpr int OFF = decltype(off_c)::value;
        constexpr int OFF2 = (OFF + Q - 1) % Q;
        auto za = [&](int j) -> float4 { return qa[(j + OFF) % Q]; };
        auto zb2 = [&](int j) -> float4 { return qx[(j + OFF2) % Q]; };
        float* L1 = U1 + (it & 1) * P1;
        *reinterpret_cast<float4*>(&L1[l1]) = za(R);
        if (tile_role) {
            if constexpr (WAVE) BQ[s2 * Z::NTILE + tid] = cb;
        } else {
            *reinterpret_cast<float4*>(&L1[lm]) = qx[(R + OFF) % Q];
        }

        const bool more = z1 + 1 < z1e;
        // the next plane's loads, in flight during the compute (past the
        // chunk their planes are clamped and the values go unused)
        Raw nq, np, nb, nm;
        if (DEFER || more) {
            nq = ldr(rU, z1 + 1 + R, ag);
            if constexpr (WAVE) {
                np = ldr(rP, z1 + 1, ag);
                nb = ldr(rB, z1 + 1, ag);
            }
            if (!tile_role) nm = ldr(rU, z1 + 1 + R, am);
        }
        // the previous plane's stores, issued after these loads so that the
        // wait for the loads at the end of the plane does not also wait for
        // them: u^{n+1} at z1 - 1 (still in the column ring) and u^{n+2} at
        // z1 - 1 - R
        if (DEFER && tile_role && store_ok) {
            if (WAVE && z1 - 1 >= zb && z1 - 1 < ze) {
                const float4 p1 = zb2(2 * R - 1);
                const float o[4] = {p1.x, p1.y, p1.z, p1.w};
                tb2_store<T>(rO1, ag, soff(z1 - 1), full_tile, x0, nx, o);
            }
            if (z1 - 1 - R >= zb) tb2_store<T>(rO2, ag, soff(z1 - 1 - R), full_tile, x0, nx, o2p);
        }
        __syncthreads();

        // ---- stage 1: u^{n+1} at plane z1 over E (both roles)
        float4 r1;
        {
            const bool zin = z1 >= 0 && z1 < nz;
            float o[4];
            tb2_star<R, MODE>(w, za, L1 + l1, W1, cp, cb, gamma_at(z1), o);
            while (WAVE && e_z == z1) {
                const int* e = v.src_e.zyx4 + 4 * e_next;
                e_next++;
                e_z = e_next < e_end ? tb2_ldc(v.src_e.zyx4 + 4 * e_next) : INT_MAX;
                const int ey = tb2_ldc(e + 1), ex = tb2_ldc(e + 2);
                const double amt = tb2_ldc(v.src_e.amp + (int64_t)arow * v.src_e.n + tb2_ldc(e + 3));
#pragma unroll
                for (int i = 0; i < 4; i++)
                    if (ey == y0 && ex == x0 + i) o[i] = inject<T>(o[i], amt);
            }
            r1.x = zin && in[0] ? through<T>(o[0]) : 0.f;
            r1.y = zin && in[1] ? through<T>(o[1]) : 0.f;
            r1.z = zin && in[2] ? through<T>(o[2]) : 0.f;
            r1.w = zin && in[3] ? through<T>(o[3]) : 0.f;
            *reinterpret_cast<float4*>(&U2[s2 * P2 + l2]) = r1;
        }

        // ---- stage 2 (tile role): u^{n+2} at plane z = z1 - R
        if (tile_role) {
            qx[(2 * R + OFF2) % Q] = r1;
            const int z = z1 - R;
            if (z >= zb) {
                const int sz2 = s2 + 1 == NS2 ? 0 : s2 + 1;   // slot of plane z1 - R
                float o2[4];
                if constexpr (WAVE)
                    tb2_star<R, MODE>(w, zb2, U2 + sz2 * P2 + l2, W2, za(0), BQ[sz2 * Z::NTILE + tid], gamma_at(z),
                                      o2);
                else
                    tb2_star<R, MODE>(w, zb2, U2 + sz2 * P2 + l2, W2, zero4, zero4, zero4, o2);
                while (WAVE && t_z == z) {
                    const int* e = v.src_t.zyx4 + 4 * t_next;
                    t_next++;
                    t_z = t_next < t_end ? tb2_ldc(v.src_t.zyx4 + 4 * t_next) : INT_MAX;
                    const int ey = tb2_ldc(e + 1), ex = tb2_ldc(e + 2);
                    const double amt = tb2_ldc(v.src_t.amp + (int64_t)(arow + 1) * v.src_t.n + tb2_ldc(e + 3));
#pragma unroll
                    for (int i = 0; i < 4; i++)
                        if (ey == y0 && ex == x0 + i) o2[i] = inject<T>(o2[i], amt);
                }
                if constexpr (DEFER) {
#pragma unroll
                    for (int i = 0; i < 4; i++) o2p[i] = o2[i];
                } else if (store_ok) {
                    tb2_store<T>(rO2, ag, soff(z), full_tile, x0, nx, o2);
                }
            }
        }

        if (more) {
            qa[OFF] = widen4<T>(nq);
            if (!tile_role) qx[OFF] = widen4<T>(nm);
            if constexpr (WAVE) {
                cp = widen4<T>(np);
                cb = widen4<T>(nb);
            }
        }
        s2 = s2 + 1 == NS2 ? 0 : s2 + 1;
        it++;
        z1++;
    };
    while (z1 + Q <= z1e) StaticFor<0, Q>::run([&](auto c) __attribute__((always_inline)) { step(c); });
    StaticFor<0, Q - 1>::run([&](auto c) __attribute__((always_inline)) {
        if (z1 < z1e) step(c);
    });
    // the last plane's u^{n+2} (its u^{n+1} lies past the chunk)
    if (DEFER && tile_role && store_ok && z1 - 1 - R >= zb)
        tb2_store<T>(rO2, ag, soff(z1 - 1 - R), full_tile, x0, nx, o2p);
}

template <int MODE, int R, typename T>
__global__ __launch_bounds__(kTB2Threads, (TB2<R, MODE != MODE_HEAT>::WAVES_PER_SIMD)) void k_tb2(TBView v, Coefs w, int arow,
                                                                                               int trow_u, int trow_p) {
    extern __shared__ __attribute__((aligned(16))) float lds[];
    tb2_tile<MODE, R, T>(v, w, xcd_remap(blockIdx.x, gridDim.x), arow, trow_u, trow_p, lds);
}

// Batched shots: one launch covers the tiles of every shot; block_map as for
// k_zmarch_batch (laid out per XCD by the host; shot -1 pads).
template <typename T>
__global__ __launch_bounds__(kTB2Threads, 1) void k_tb2_batch(const TBView* __restrict__ views,
                                                         const int* __restrict__ block_map, Coefs w, int arow,
                                                         int trow_u, int trow_p) {
    extern __shared__ __attribute__((aligned(16))) float lds[];
    const int b = blockIdx.x;
    const int shot = block_map[2 * b];
    if (shot < 0) return;
    tb2_tile<MODE_WAVE, 4, T>(views[shot], w, block_map[2 * b + 1], arow, trow_u, trow_p, lds);
}

template <typename T>
static hipError_t tb2_batch_launch(const TBView* views, const int* bmap, int nblocks, const Coefs& w, int arow,
                                   int trow_u, int trow_p, hipStream_t s) {
    constexpr size_t lds = sizeof(float) * TB2<4, true>::LDS_FLOATS;
    if (nblocks == 0) return hipSuccess;
    auto k = k_tb2_batch<T>;
    static const hipError_t attr = allow_lds(k, lds);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL(k, dim3((unsigned)nblocks), dim3(kTB2Threads), lds, s, views, bmap, w, arow, trow_u, trow_p);
    return hipGetLastError();
}

template <int MODE, int R, typename T>
static hipError_t tb2_launch(const TBView& v, const Coefs& w, int arow, int trow_u, int trow_p, hipStream_t s) {
    constexpr size_t lds = sizeof(float) * TB2<R, MODE != MODE_HEAT>::LDS_FLOATS;
    const int64_t nb = (int64_t)v.ntx * v.nty * v.nzc;
    if (nb == 0) return hipSuccess;
    auto k = k_tb2<MODE, R, T>;
    static const hipError_t attr = allow_lds(k, lds);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL(k, dim3((unsigned)nb), dim3(kTB2Threads), lds, s, v, w, arow, trow_u, trow_p);
    return hipGetLastError();
}

}  // namespace stn
