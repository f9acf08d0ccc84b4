// Templates of the z-marching sweep kernels.  Each storage type (and the
// FP32 adjoint modes) is instantiated in its own translation unit so the
// library builds in parallel.
#pragma once

#include <climits>
#include <type_traits>

#include "kernels.hpp"

namespace stn {

__device__ static inline float comp(const float4& v, int i) {
    return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}

// Point lists and amplitudes are invariant during a launch: reading them
// through the constant address space makes them scalar loads, which the
// vector memory counter does not track (as vector loads used by some lanes
// only, they made the compiler wait for every outstanding load and store).
template <typename U>
__device__ __forceinline__ U ld_inv(const U* p) {
    return *(const __attribute__((address_space(4))) U*)p;
}

// FP16 operands through the mixed-precision FMA (v_fma_mix_f32): the named
// half (0 low, 1 high) of a 32-bit word is read as FP16, widened exactly
// inside the instruction, and the result rounds once in FP32.  Each form
// equals the FP32 arithmetic on widened operands bit for bit (1.0 * m and
// 2.0 * c are exact; a product plus -0 keeps the sign of a zero product).
template <int HM, int HP>
__device__ __forceinline__ float mix_add(uint32_t m, uint32_t p) {   // m + p
    float r;
    if constexpr (HM == 0 && HP == 0)
        asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel:[0,0,0] op_sel_hi:[1,0,1]" : "=v"(r) : "v"(m), "v"(p));
    else if constexpr (HM == 0)
        asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel:[0,0,1] op_sel_hi:[1,0,1]" : "=v"(r) : "v"(m), "v"(p));
    else if constexpr (HP == 0)
        asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,1]" : "=v"(r) : "v"(m), "v"(p));
    else
        asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel:[1,0,1] op_sel_hi:[1,0,1]" : "=v"(r) : "v"(m), "v"(p));
    return r;
}
template <int H>
__device__ __forceinline__ float mix_mul(float k, uint32_t c) {   // k * c
    float r;
    if constexpr (H == 0)
        asm("v_fma_mix_f32 %0, %1, %2, -%3 op_sel:[0,0,0] op_sel_hi:[0,1,0]" : "=v"(r) : "v"(k), "v"(c), "v"(0.0f));
    else
        asm("v_fma_mix_f32 %0, %1, %2, -%3 op_sel:[0,1,0] op_sel_hi:[0,1,0]" : "=v"(r) : "v"(k), "v"(c), "v"(0.0f));
    return r;
}
template <int HC, int HP>
__device__ __forceinline__ float mix_twice_minus(uint32_t c, uint32_t p) {   // 2c - p
    float r;
    if constexpr (HC == 0 && HP == 0)
        asm("v_fma_mix_f32 %0, 2.0, %1, -%2 op_sel:[0,0,0] op_sel_hi:[0,1,1]" : "=v"(r) : "v"(c), "v"(p));
    else if constexpr (HC == 0)
        asm("v_fma_mix_f32 %0, 2.0, %1, -%2 op_sel:[0,0,1] op_sel_hi:[0,1,1]" : "=v"(r) : "v"(c), "v"(p));
    else if constexpr (HP == 0)
        asm("v_fma_mix_f32 %0, 2.0, %1, -%2 op_sel:[0,1,0] op_sel_hi:[0,1,1]" : "=v"(r) : "v"(c), "v"(p));
    else
        asm("v_fma_mix_f32 %0, 2.0, %1, -%2 op_sel:[0,1,1] op_sel_hi:[0,1,1]" : "=v"(r) : "v"(c), "v"(p));
    return r;
}
template <int H>
__device__ __forceinline__ float mix_fma(uint32_t b, float a, float t) {   // b * a + t
    float r;
    if constexpr (H == 0)
        asm("v_fma_mix_f32 %0, %1, %2, %3 op_sel:[0,0,0] op_sel_hi:[1,0,0]" : "=v"(r) : "v"(b), "v"(a), "v"(t));
    else
        asm("v_fma_mix_f32 %0, %1, %2, %3 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(r) : "v"(b), "v"(a), "v"(t));
    return r;
}
template <int H>
__device__ __forceinline__ float mix_add_f(uint32_t c, float a) {   // c + a
    float r;
    if constexpr (H == 0)
        asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel:[0,0,0] op_sel_hi:[1,0,0]" : "=v"(r) : "v"(c), "v"(a));
    else
        asm("v_fma_mix_f32 %0, %1, 1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(r) : "v"(c), "v"(a));
    return r;
}
// word w (0, 1) of a group of four 16-bit values
__device__ __forceinline__ uint32_t word(const u2v& g, int w) { return w == 0 ? g.x : g.y; }

// compile-time loop: f(integral_constant<int, I>) for I = B .. E-1
template <int B, int E>
struct StaticFor {
    template <class F>
    __device__ __forceinline__ static void run(F&& f) {
        if constexpr (B < E) {
            f(std::integral_constant<int, B>{});
            StaticFor<B + 1, E>::run(f);
        }
    }
};

// Workgroups are dispatched round-robin over the 8 XCDs (block b -> XCD b%8).
// Give XCD x the contiguous logical range [x*q + min(x,r), ...) so that
// neighbouring tiles (which read each other's edge rows as halo) share an L2.
__device__ static inline int xcd_remap(int b, int nb) {
    const int q = nb >> 3, r = nb & 7;
    const int x = b & 7, i = b >> 3;
    return x * q + min(x, r) + i;
}

// -------------------------------------------------------------- k_zmarch
// LDS holds a ring of R+2 plane slots of (TY+2R) x (TX+8) values.  The halo
// part of a slot (the x and y margins of the tile) is written when its plane
// is the leading plane z+R, i.e. when the neighbouring tiles load the same
// rows as their own interior, so those rows are still in L2; the interior part
// is written when the plane becomes the current one.  With R+2 slots a single
// barrier per plane separates every write from the reads of the same slot.
template <int R, int BX, int BY, int VY, int VX>
struct ZTile {
    static constexpr int NT = BX * BY, TX = VX * BX, TY = BY * VY;
    static constexpr int LDX = TX + 8, LDY = TY + 2 * R, PLANE = LDX * LDY;
    static constexpr int NSLOT = R + 2;
    static constexpr int LDS_FLOATS = NSLOT * PLANE;
    // halo items are 4-element groups: one per side of each tile row, and
    // TX/4 per halo row above and below the tile
    static constexpr int NHX = 2 * TY, NHY = 2 * R * (TX / 4), NHT = NHX + NHY, NH = (NHT + NT - 1) / NT;
};

// LDS planes of 16-bit fields hold the storage values as loaded (half the
// LDS of FP32 planes, so more workgroups share a CU).  BF16 values are
// widened per read, one shift or mask per value; FP16 values stay 16-bit in
// registers too and enter the arithmetic through the mixed-precision FMA.
// Values pass through LDS unchanged either way.
//
// BF16 tiles with 8 points per lane keep FP32 planes instead and widen each
// value once, as it enters LDS: at that shape two workgroups share a compute
// unit either way, and widening per read cost more issue slots than the
// planes' extra LDS bytes.
template <typename T, int VX>
inline constexpr bool kLds16 =
    std::is_same<T, f16>::value || (std::is_same<T, bf16>::value && VX != 8);
// FP16: the z-queue, the taps and u_prev and beta stay in the storage type
template <typename T>
inline constexpr bool kMix = std::is_same<T, f16>::value;
template <typename T>
using QGroup = typename std::conditional<kMix<T>, u2v, float4>::type;
template <typename T, int VX>
using LdsT = typename std::conditional<kLds16<T, VX>, T, float>::type;
template <typename T, int VX>
__device__ __forceinline__ float4 lds_get4(const LdsT<T, VX>* p) {
    if constexpr (kLds16<T, VX>) return widen4<T>(*reinterpret_cast<const u2v*>(p));
    else return *reinterpret_cast<const float4*>(p);
}
template <typename T, int VX>
__device__ __forceinline__ void lds_put4_raw(LdsT<T, VX>* p, typename RawGroup<T>::type r) {
    if constexpr (kLds16<T, VX>) *reinterpret_cast<u2v*>(p) = r;
    else *reinterpret_cast<float4*>(p) = widen4<T>(r);
}
// a group of the z-queue into an LDS plane
template <typename T, int VX>
__device__ __forceinline__ void lds_put_q(LdsT<T, VX>* p, const QGroup<T>& g);
// a group of 4 values that came from storage of type T (exact in T)
template <typename T, int VX>
__device__ __forceinline__ void lds_put4(LdsT<T, VX>* p, float4 v) {
    if constexpr (kLds16<T, VX>) {
        const u2v r = {Storage<T>::pack2(v.x, v.y), Storage<T>::pack2(v.z, v.w)};
        *reinterpret_cast<u2v*>(p) = r;
    } else {
        *reinterpret_cast<float4*>(p) = v;
    }
}
template <typename T, int VX>
__device__ __forceinline__ void lds_put_q(LdsT<T, VX>* p, const QGroup<T>& g) {
    if constexpr (kMix<T>) *reinterpret_cast<u2v*>(p) = g;
    else lds_put4<T, VX>(p, g);
}
// a group of an LDS plane in the z-queue's form
template <typename T, int VX>
__device__ __forceinline__ QGroup<T> lds_get_q(const LdsT<T, VX>* p) {
    if constexpr (kMix<T>) return *reinterpret_cast<const u2v*>(p);
    else return lds_get4<T, VX>(p);
}

// Each thread owns VX consecutive x points (VX = 4 or 8) in VY consecutive
// rows (ty * VY .. ty * VY + VY - 1 of the tile), so the y taps of its rows
// overlap and every tap row is read from LDS once; a row's VX values travel
// as VX/4 float4.
template <int MODE, int R, typename T, int BX, int BY, int VY, int VX, bool NTH>
__device__ __forceinline__ void zmarch_tile(const ZView& v, const Coefs& w, int lb, int parity, int arow,
                                            int trow, float* __restrict__ lds) {
    using Z = ZTile<R, BX, BY, VY, VX>;
    constexpr int NT = Z::NT, TX = Z::TX, TY = Z::TY, LDX = Z::LDX, PLANE = Z::PLANE, NSLOT = Z::NSLOT;
    constexpr int NHX = Z::NHX, NHY = Z::NHY, NHT = Z::NHT, NH = Z::NH;
    constexpr int NV = VX / 4;
    constexpr bool WAVE = MODE != MODE_HEAT;
    // FP16: queue, taps, u_prev and beta stay 16-bit (QG); see mix_add
    constexpr bool MIX = kMix<T>;
    using QG = QGroup<T>;
    // adjoint with imaging; ADJ2 also images the input level (two steps'
    // imaging terms in one read and write of the partial g)
    constexpr bool ADJ = MODE == MODE_WAVE_ADJ || MODE == MODE_WAVE_ADJ2, ADJ2 = MODE == MODE_WAVE_ADJ2;
    // forward modes: a plane's output goes out after the next plane's loads,
    // which are issued on every plane, so the waits for those loads count the
    // same operations on every path and never wait for the stores
    constexpr bool DEFER = !ADJ && MODE != MODE_WAVE_D;
    using S = Storage<T>;
    using LT = LdsT<T, VX>;
    LT* const ldsT = reinterpret_cast<LT*>(lds);

    const int tid = threadIdx.x;
    const int tx = tid % BX, ty = tid / BX;
    const int ntxy = v.ntx * v.nty;
    const int tile_x = lb % v.ntx, tile_y = (lb / v.ntx) % v.nty, zch = lb / ntxy;
    const int X0 = tile_x * TX, Y0 = tile_y * TY;
    const int zb = zch * v.zc;
    const int ze = min(zb + v.zc, v.g.n[0]);
    const int nx = v.g.n[2], ny = v.g.n[1];
    const int64_t sz = v.g.s[0], sy = v.g.s[1];

    const T* U = (const T*)(parity ? v.prev : v.u) + v.g.origin;
    const T* P = (const T*)(parity ? v.u : v.prev) + v.g.origin;
    T* O = (T*)(parity ? (void*)v.u : v.out) + v.g.origin;
    const T* B = (const T*)v.beta + v.g.origin;

    // receivers sample the input level u^t (read-only during this launch)
    if (trow >= 0 && lb == 0) {
        for (int r = tid; r < v.rec.n; r += NT)
            v.rec.trace[(int64_t)trow * v.rec.n + r] = (double)S::load(U + v.rec.off[r]);
    }

    // every load stays inside the field: x groups are clamped to the row,
    // y rows to the last halo row; clamped values only feed masked outputs
    const int xmax4 = (int)(v.g.rowlen - v.g.xlead) - 4;
    const int xmaxv = (int)(v.g.rowlen - v.g.xlead) - VX;
    const int ymax = ny + R - 1;

    int64_t own[VY];
#pragma unroll
    for (int j = 0; j < VY; j++) {
        const int y = min(Y0 + ty * VY + j, ymax);
        own[j] = (int64_t)y * sy + min(X0 + VX * tx, xmaxv);
    }
    // absorbing layer: this thread's rows' and columns' damping profiles
    float dgy[VY], dgx[VX];
    if constexpr (MODE == MODE_WAVE_DAMP) {
#pragma unroll
        for (int j = 0; j < VY; j++) dgy[j] = v.damp[v.g.n[0] + min(Y0 + ty * VY + j, ny - 1)];
#pragma unroll
        for (int i = 0; i < VX; i++) dgx[i] = v.damp[v.g.n[0] + ny + min(X0 + VX * tx + i, nx - 1)];
    }
    int64_t hoff[NH];
    int hlds[NH];
    bool hon[NH];
#pragma unroll
    for (int m = 0; m < NH; m++) {
        const int h = tid + m * NT;
        hon[m] = h < NHT;
        if (h < NHX) {
            const int r = h >> 1, side = h & 1;
            const int y = min(Y0 + r, ymax);
            const int x = side ? min(X0 + TX, xmax4) : X0 - 4;
            hoff[m] = (int64_t)y * sy + x;
            hlds[m] = (R + r) * LDX + (side ? 4 + TX : 0);
        } else {
            const int h2 = min(h - NHX, NHY - 1);
            const int i = h2 / (TX / 4), g = h2 % (TX / 4);
            const int y = i < R ? Y0 - R + i : min(Y0 + TY + (i - R), ymax);
            hoff[m] = (int64_t)y * sy + min(X0 + 4 * g, xmax4);
            hlds[m] = (i < R ? i : TY + i) * LDX + 4 + 4 * g;
        }
    }

    // own columns of planes zb-R .. zb+R; halos of planes zb .. zb+R-1 go
    // straight to their slots, the halo of plane zb+R is in flight
    QG q[2 * R + 1][VY][NV];
#pragma unroll
    for (int k = 0; k < 2 * R + 1; k++)
#pragma unroll
        for (int j = 0; j < VY; j++) {
            if constexpr (MIX) load_vec_raw<T, VX, false>(U + (int64_t)(zb - R + k) * sz + own[j], q[k][j]);
            else load_vec<T, VX>(U + (int64_t)(zb - R + k) * sz + own[j], q[k][j], false);
        }
    for (int p = zb; p < min(zb + R, ze); p++) {
        LT* L = ldsT + ((p - zb) % NSLOT) * PLANE;
#pragma unroll
        for (int m = 0; m < NH; m++)
            if (hon[m]) lds_put4_raw<T, VX>(&L[hlds[m]], load4_raw<T, false>(U + (int64_t)p * sz + hoff[m]));
    }
    // loads in flight across a plane's compute stay in the storage type
    using Raw = typename RawGroup<T>::type;
    Raw hal[NH];
    if (zb + R < ze) {
#pragma unroll
        for (int m = 0; m < NH; m++)
            if (hon[m]) hal[m] = load4_raw<T, false>(U + (int64_t)(zb + R) * sz + hoff[m]);
    }
    QG cp[VY][NV], cb[VY][NV];
    if constexpr (WAVE) {
#pragma unroll
        for (int j = 0; j < VY; j++) {
            if constexpr (MIX) {
                load_vec_raw<T, VX, NTH>(P + (int64_t)zb * sz + own[j], cp[j]);
                load_vec_raw<T, VX, NTH>(B + (int64_t)zb * sz + own[j], cb[j]);
            } else {
                load_vec<T, VX>(P + (int64_t)zb * sz + own[j], cp[j], NTH);
                load_vec<T, VX>(B + (int64_t)zb * sz + own[j], cb[j], NTH);
            }
        }
    }

    // Prefetch distance 2 (forward sweeps of 16-bit fields, 8 points per
    // lane): plane zb + 1's loads are pending before the first plane, and each
    // plane issues plane z + 2's, so two planes of loads are in flight.  With
    // 16-byte loads of 16-bit values a plane's loads are half the bytes of
    // the FP32 form's; the second plane brings the bytes in flight back up
    // (512^3 BF16: 246 -> 210 us per sweep).  Other shapes and FP32 gain
    // nothing or lose, and keep distance 1.
    constexpr bool PD2 = DEFER && sizeof(T) == 2 && VX == 8;
    Raw pq[VY][NV], pp[VY][NV], pb[VY][NV], phal[NH];
    if constexpr (PD2) {
        const int64_t z1 = (int64_t)min(zb + 1, ze - 1) * sz;
#pragma unroll
        for (int j = 0; j < VY; j++) load_vec_raw<T, VX, false>(U + z1 + (int64_t)R * sz + own[j], pq[j]);
#pragma unroll
        for (int m = 0; m < NH; m++)
            if (hon[m]) phal[m] = load4_raw<T, false>(U + z1 + (int64_t)R * sz + hoff[m]);
        if constexpr (WAVE) {
#pragma unroll
            for (int j = 0; j < VY; j++) {
                load_vec_raw<T, VX, NTH>(P + z1 + own[j], pp[j]);
                load_vec_raw<T, VX, NTH>(B + z1 + own[j], pb[j]);
            }
        }
    }

    // adjoint: D and G of this thread's groups that lie wholly inside the
    // interior, at the current plane; like u_prev and beta they are loaded a
    // plane ahead, so their latency overlaps the compute (other groups read
    // them at the store); with gfresh the partial starts at zero and is not
    // read
    bool dg_ok[VY];
    int64_t dg_off[VY];
    float4 cd[VY][NV], cg[VY][NV], cd2[VY][NV];
    const bool gload = ADJ && !v.gfresh;
    if constexpr (ADJ) {
#pragma unroll
        for (int j = 0; j < VY; j++) {
            const int y = Y0 + ty * VY + j, x0 = X0 + VX * tx;
            dg_ok[j] = y < ny && x0 + VX - 1 < nx;
            dg_off[j] = v.g.origin + (int64_t)y * sy + x0;
            if (dg_ok[j] && zb < ze) {
#pragma unroll
                for (int c = 0; c < NV; c++) {
                    cd[j][c] = Storage<float>::load4_nt(v.dfield + dg_off[j] + (int64_t)zb * sz + 4 * c);
                    cg[j][c] = gload ? Storage<float>::load4_nt(v.gfield + dg_off[j] + (int64_t)zb * sz + 4 * c)
                                     : make_float4(0.f, 0.f, 0.f, 0.f);
                    if constexpr (ADJ2)
                        cd2[j][c] = Storage<float>::load4_nt(v.dfield2 + dg_off[j] + (int64_t)zb * sz + 4 * c);
                }
            }
        }
    }

    // This tile's sources, sorted by z on the host: `snext` indexes the next
    // one at or after the chunk start and `szn` holds its z in a register, so
    // planes without a source cost one compare and no memory access (a load
    // per plane would put its latency on this workgroup's critical path,
    // and the slowest workgroup sets the duration of the whole launch).
    int snext = 0, se = 0, szn = INT_MAX;
    if constexpr (WAVE) {
        if (v.src.n > 0) {
            const int tile = tile_y * v.ntx + tile_x;
            snext = ld_inv(v.src.tile_begin + tile);
            se = ld_inv(v.src.tile_begin + tile + 1);
            while (snext < se && ld_inv(v.src.zyx4 + 4 * snext) < zb) snext++;
            szn = snext < se ? ld_inv(v.src.zyx4 + 4 * snext) : INT_MAX;
        }
    }

    int slot = 0;             // slot of plane z
    int hslot = R % NSLOT;    // slot of plane z + R
    int z = zb;
    // One plane.  The z-queue is a ring of 2R+1 registers read through the
    // compile-time offset OFF (logical plane k lives in q[(k + OFF) % Q]); the
    // new leading plane overwrites the slot of the oldest one, so the queue
    // advances without register moves.  The plane loop below is unrolled
    // 2R+1 times so that every offset is a constant.
    constexpr int Q = 2 * R + 1;
    Raw nq[VY][NV];   // the next leading plane, in flight during the compute
    float o[VY][VX];  // the plane's output (DEFER: stored during the next plane)
    // store o as plane zs of the output (the rows and columns in the interior)
    auto store_out = [&](int zs) {
#pragma unroll
        for (int j = 0; j < VY; j++) {
            const int y = Y0 + ty * VY + j;
            const int x0 = X0 + VX * tx;
            if (y < ny && x0 < nx) {
                const int64_t off = (int64_t)zs * sz + (int64_t)y * sy + x0;
                if (x0 + VX - 1 < nx) {
                    float4 ov[NV];
#pragma unroll
                    for (int c = 0; c < NV; c++)
                        ov[c] = make_float4(o[j][4 * c], o[j][4 * c + 1], o[j][4 * c + 2], o[j][4 * c + 3]);
                    store_vec<T, VX>(O + off, ov, NTH && !ADJ);
                } else {
#pragma unroll
                    for (int i = 0; i < VX; i++)
                        if (x0 + i < nx) S::store(O + off + i, o[j][i]);
                }
            }
        }
    };
    auto step = [&](auto off_c) {
        constexpr int OFF = decltype(off_c)::value;
        auto qi = [&](int k) -> QG(&)[VY][NV] { return q[(k + OFF) % Q]; };
        LT* L = ldsT + slot * PLANE;
#pragma unroll
        for (int j = 0; j < VY; j++)
#pragma unroll
            for (int c = 0; c < NV; c++)
                lds_put_q<T, VX>(&L[(R + ty * VY + j) * LDX + 4 + VX * tx + 4 * c], qi(R)[j][c]);
        if (z + R < ze) {
            LT* H = ldsT + hslot * PLANE;
#pragma unroll
            for (int m = 0; m < NH; m++)
                if (hon[m]) lds_put4_raw<T, VX>(&H[hlds[m]], hal[m]);
        }

        const bool more = z + 1 < ze;
        Raw np[VY][NV], nb[VY][NV];
        float4 nd[VY][NV], ng[VY][NV], nd2[VY][NV];
        Raw n2q[VY][NV], n2p[VY][NV], n2b[VY][NV], n2h[NH];
        if constexpr (PD2) {
            const int64_t zn2 = (int64_t)min(z + 2, ze - 1) * sz;
#pragma unroll
            for (int j = 0; j < VY; j++) load_vec_raw<T, VX, false>(U + zn2 + (int64_t)R * sz + own[j], n2q[j]);
#pragma unroll
            for (int m = 0; m < NH; m++)
                if (hon[m]) n2h[m] = load4_raw<T, false>(U + zn2 + (int64_t)R * sz + hoff[m]);
            if constexpr (WAVE) {
#pragma unroll
                for (int j = 0; j < VY; j++) {
                    load_vec_raw<T, VX, NTH>(P + zn2 + own[j], n2p[j]);
                    load_vec_raw<T, VX, NTH>(B + zn2 + own[j], n2b[j]);
                }
            }
        } else if (DEFER || more) {
            // DEFER: past the chunk the loads re-read the current plane's
            // rows (in the field; the values go unused)
            const int64_t zn = (int64_t)(more ? z + 1 : z) * sz;
#pragma unroll
            for (int j = 0; j < VY; j++) load_vec_raw<T, VX, false>(U + zn + (int64_t)R * sz + own[j], nq[j]);
            if (DEFER || z + R + 1 < ze) {
#pragma unroll
                for (int m = 0; m < NH; m++)
                    if (hon[m]) hal[m] = load4_raw<T, false>(U + zn + (int64_t)R * sz + hoff[m]);
            }
            if constexpr (WAVE) {
#pragma unroll
                for (int j = 0; j < VY; j++) {
                    load_vec_raw<T, VX, NTH>(P + zn + own[j], np[j]);
                    load_vec_raw<T, VX, NTH>(B + zn + own[j], nb[j]);
                }
            }
            if constexpr (ADJ) {
#pragma unroll
                for (int j = 0; j < VY; j++)
                    if (dg_ok[j]) {
#pragma unroll
                        for (int c = 0; c < NV; c++) {
                            nd[j][c] = Storage<float>::load4_nt(v.dfield + dg_off[j] + zn + 4 * c);
                            ng[j][c] = gload ? Storage<float>::load4_nt(v.gfield + dg_off[j] + zn + 4 * c)
                                             : make_float4(0.f, 0.f, 0.f, 0.f);
                            if constexpr (ADJ2) nd2[j][c] = Storage<float>::load4_nt(v.dfield2 + dg_off[j] + zn + 4 * c);
                        }
                    }
            }
        }
        if constexpr (DEFER) {
            if (z > zb) store_out(z - 1);
        }
        __syncthreads();

        float dgz = 0.f;
        if constexpr (MODE == MODE_WAVE_DAMP) dgz = v.damp[z];
        float dv[VY][VX];
        // y tap rows row0 - R .. row0 + VY - 1 + R of this thread's columns:
        // its own rows from the z-queue, the 2R others from LDS, once each
        const int row0 = R + ty * VY;
        QG yr[VY + 2 * R][NV];
#pragma unroll
        for (int q2 = 0; q2 < VY + 2 * R; q2++)
#pragma unroll
            for (int c = 0; c < NV; c++) {
                if (q2 >= R && q2 < R + VY)
                    yr[q2][c] = qi(R)[q2 - R][c];
                else
                    yr[q2][c] = lds_get_q<T, VX>(L + (row0 - R + q2) * LDX + 4 + VX * tx + 4 * c);
            }
#pragma unroll
        for (int j = 0; j < VY; j++) {
            const int row = row0 + j;
            const LT* Lr = L + row * LDX + VX * tx;
            if constexpr (MIX) {
                // x taps as 16-bit halves of words: 4 left of the thread's
                // points (words 0, 1), its own VX, 4 right; the same
                // canonical order as below, each pair sum read straight
                // from the halves
                uint32_t xw[VX / 2 + 4];
                {
                    const u2v xl = *reinterpret_cast<const u2v*>(Lr);
                    const u2v xr = *reinterpret_cast<const u2v*>(Lr + 4 + VX);
                    xw[0] = xl.x;
                    xw[1] = xl.y;
#pragma unroll
                    for (int c = 0; c < NV; c++) {
                        xw[2 + 2 * c] = qi(R)[j][c].x;
                        xw[3 + 2 * c] = qi(R)[j][c].y;
                    }
                    xw[VX / 2 + 2] = xr.x;
                    xw[VX / 2 + 3] = xr.y;
                }
                StaticFor<0, VX>::run([&](auto ic) {
                    constexpr int i = decltype(ic)::value, c = i / 4, wd = (i % 4) / 2, h = i % 2;
                    float acc = mix_mul<h>(w.cd0, word(qi(R)[j][c], wd));
                    StaticFor<1, R + 1>::run([&](auto kc) {
                        constexpr int k = decltype(kc)::value;
                        acc = fmaf(w.c[k], mix_add<h, h>(word(qi(R - k)[j][c], wd), word(qi(R + k)[j][c], wd)), acc);
                    });
                    StaticFor<1, R + 1>::run([&](auto kc) {
                        constexpr int k = decltype(kc)::value;
                        acc = fmaf(w.c[k], mix_add<h, h>(word(yr[R + j - k][c], wd), word(yr[R + j + k][c], wd)), acc);
                    });
                    StaticFor<1, R + 1>::run([&](auto kc) {
                        constexpr int k = decltype(kc)::value, hm = 4 + i - k, hp = 4 + i + k;
                        acc = fmaf(w.c[k], mix_add<hm % 2, hp % 2>(xw[hm / 2], xw[hp / 2]), acc);
                    });
                    if constexpr (WAVE)
                        o[j][i] = mix_fma<h>(word(cb[j][c], wd), acc,
                                             mix_twice_minus<h, h>(word(qi(R)[j][c], wd), word(cp[j][c], wd)));
                    else
                        o[j][i] = mix_add_f<h>(word(qi(R)[j][c], wd), acc);
                });
            } else {
            // x taps: 4 left of the thread's points, its own VX, 4 right
            float xv[VX + 8];
            {
                const float4 xl = lds_get4<T, VX>(Lr);
                const float4 xr = lds_get4<T, VX>(Lr + 4 + VX);
                xv[0] = xl.x;
                xv[1] = xl.y;
                xv[2] = xl.z;
                xv[3] = xl.w;
#pragma unroll
                for (int i = 0; i < VX; i++) xv[4 + i] = comp(qi(R)[j][i / 4], i % 4);
                xv[VX + 4] = xr.x;
                xv[VX + 5] = xr.y;
                xv[VX + 6] = xr.z;
                xv[VX + 7] = xr.w;
            }
            QG ym[R][NV], yp[R][NV];
#pragma unroll
            for (int k = 1; k <= R; k++)
#pragma unroll
                for (int c = 0; c < NV; c++) {
                    ym[k - 1][c] = yr[R + j - k][c];
                    yp[k - 1][c] = yr[R + j + k][c];
                }
#pragma unroll
            for (int i = 0; i < VX; i++) {
                const int c = i / 4, e = i % 4;
                const float ctr = comp(qi(R)[j][c], e);
                float m[R], p[R];
                float acc = w.cd0 * ctr;
#pragma unroll
                for (int k = 1; k <= R; k++) {
                    m[k - 1] = comp(qi(R - k)[j][c], e);
                    p[k - 1] = comp(qi(R + k)[j][c], e);
                }
                acc = axis_sum<R>(acc, w, m, p);
#pragma unroll
                for (int k = 1; k <= R; k++) {
                    m[k - 1] = comp(ym[k - 1][c], e);
                    p[k - 1] = comp(yp[k - 1][c], e);
                }
                acc = axis_sum<R>(acc, w, m, p);
#pragma unroll
                for (int k = 1; k <= R; k++) {
                    m[k - 1] = xv[4 + i - k];
                    p[k - 1] = xv[4 + i + k];
                }
                acc = axis_sum<R>(acc, w, m, p);
                if constexpr (MODE == MODE_WAVE_DAMP) {
                    o[j][i] = damped_update(acc, ctr, comp(cp[j][c], e), comp(cb[j][c], e),
                                            (dgz + dgy[j]) + dgx[i]);
                } else if constexpr (WAVE) {
                    o[j][i] = time_update<MODE>(acc, ctr, comp(cp[j][c], e), comp(cb[j][c], e));
                    if constexpr (MODE == MODE_WAVE_D) dv[j][i] = comp(cb[j][c], e) * acc;
                } else {
                    o[j][i] = time_update<MODE>(acc, ctr, 0.f, 0.f);
                }
            }
            }
        }
        if constexpr (WAVE) {
            while (szn == z) {
                const int* e = v.src.zyx4 + 4 * snext;
                snext++;
                szn = snext < se ? ld_inv(v.src.zyx4 + 4 * snext) : INT_MAX;
                const int dy = ld_inv(e + 1) - Y0, dx = ld_inv(e + 2) - X0;
                const int idx = ld_inv(e + 3);
                const double amt =
                    ld_inv(v.src.amp + (int64_t)arow * v.src.n + idx) * (v.src.scale ? ld_inv(v.src.scale + idx) : 1.0);
#pragma unroll
                for (int j = 0; j < VY; j++)
#pragma unroll
                    for (int i = 0; i < VX; i++)
                        if (dy == ty * VY + j && dx == VX * tx + i) {
                            o[j][i] = inject<T>(o[j][i], amt);
                            if constexpr (MODE == MODE_WAVE_D) dv[j][i] = (float)((double)dv[j][i] + amt);
                        }
            }
        }

#pragma unroll
        for (int j = 0; j < VY; j++) {
            const int y = Y0 + ty * VY + j;
            const int x0 = X0 + VX * tx;
            if (y < ny && x0 < nx) {
                const int64_t off = (int64_t)z * sz + (int64_t)y * sy + x0;
                const bool full = x0 + VX - 1 < nx;
                if constexpr (!DEFER) {
                    if (full) {
                        float4 ov[NV];
#pragma unroll
                        for (int c = 0; c < NV; c++)
                            ov[c] = make_float4(o[j][4 * c], o[j][4 * c + 1], o[j][4 * c + 2], o[j][4 * c + 3]);
                        store_vec<T, VX>(O + off, ov, NTH && !ADJ);
                    } else {
#pragma unroll
                        for (int i = 0; i < VX; i++)
                            if (x0 + i < nx) S::store(O + off + i, o[j][i]);
                    }
                }
                // D (written by the recompute, read once by the adjoint many
                // steps later) and the imaging partial G (read and written once
                // per step) stream past the caches
                if constexpr (MODE == MODE_WAVE_D) {
                    float* D = v.dfield + v.g.origin + off;
                    if (full) {
#pragma unroll
                        for (int c = 0; c < NV; c++)
                            Storage<float>::store4_nt(D + 4 * c, make_float4(dv[j][4 * c], dv[j][4 * c + 1],
                                                                             dv[j][4 * c + 2], dv[j][4 * c + 3]));
                    } else {
#pragma unroll
                        for (int i = 0; i < VX; i++)
                            if (x0 + i < nx) D[i] = dv[j][i];
                    }
                }
                // ADJ2: the input level's term first, so that the partial
                // takes the same two roundings as after two ADJ steps
                if constexpr (ADJ) {
                    const float* D = v.dfield + v.g.origin + off;
                    float* G = v.gfield + v.g.origin + off;
                    if (full) {
#pragma unroll
                        for (int c = 0; c < NV; c++) {
                            const float4 d = cd[j][c];
                            float4 g = cg[j][c];
                            if constexpr (ADJ2) {
                                const float4 d2 = cd2[j][c], uc = qi(R)[j][c];
                                g.x = fmaf(uc.x, d2.x, g.x);
                                g.y = fmaf(uc.y, d2.y, g.y);
                                g.z = fmaf(uc.z, d2.z, g.z);
                                g.w = fmaf(uc.w, d2.w, g.w);
                            }
                            g.x = fmaf(o[j][4 * c], d.x, g.x);
                            g.y = fmaf(o[j][4 * c + 1], d.y, g.y);
                            g.z = fmaf(o[j][4 * c + 2], d.z, g.z);
                            g.w = fmaf(o[j][4 * c + 3], d.w, g.w);
                            Storage<float>::store4_nt(G + 4 * c, g);
                        }
                    } else {
                        const float* D2 = v.dfield2 + v.g.origin + off;
#pragma unroll
                        for (int i = 0; i < VX; i++)
                            if (x0 + i < nx) {
                                float g = gload ? G[i] : 0.f;
                                if constexpr (ADJ2) g = fmaf(comp(qi(R)[j][i / 4], i % 4), D2[i], g);
                                G[i] = fmaf(o[j][i], D[i], g);
                            }
                    }
                }
            }
        }

        if constexpr (PD2) {
            if (more) {
#pragma unroll
                for (int j = 0; j < VY; j++)
#pragma unroll
                    for (int c = 0; c < NV; c++) {
                        if constexpr (MIX) {
                            q[OFF][j][c] = pq[j][c];
                            if constexpr (WAVE) {
                                cp[j][c] = pp[j][c];
                                cb[j][c] = pb[j][c];
                            }
                        } else {
                            q[OFF][j][c] = widen4<T>(pq[j][c]);
                            if constexpr (WAVE) {
                                cp[j][c] = widen4<T>(pp[j][c]);
                                cb[j][c] = widen4<T>(pb[j][c]);
                            }
                        }
                    }
            }
#pragma unroll
            for (int m = 0; m < NH; m++) {
                hal[m] = phal[m];
                phal[m] = n2h[m];
            }
#pragma unroll
            for (int j = 0; j < VY; j++)
#pragma unroll
                for (int c = 0; c < NV; c++) {
                    pq[j][c] = n2q[j][c];
                    if constexpr (WAVE) {
                        pp[j][c] = n2p[j][c];
                        pb[j][c] = n2b[j][c];
                    }
                }
        } else if (more) {
#pragma unroll
            for (int j = 0; j < VY; j++)
#pragma unroll
                for (int c = 0; c < NV; c++) {
                    if constexpr (MIX) {
                        q[OFF][j][c] = nq[j][c];
                        if constexpr (WAVE) {
                            cp[j][c] = np[j][c];
                            cb[j][c] = nb[j][c];
                        }
                    } else {
                        q[OFF][j][c] = widen4<T>(nq[j][c]);
                        if constexpr (WAVE) {
                            cp[j][c] = widen4<T>(np[j][c]);
                            cb[j][c] = widen4<T>(nb[j][c]);
                        }
                    }
                    if constexpr (ADJ) {
                        cd[j][c] = nd[j][c];
                        cg[j][c] = ng[j][c];
                        if constexpr (ADJ2) cd2[j][c] = nd2[j][c];
                    }
                }
        }
        slot = slot + 1 == NSLOT ? 0 : slot + 1;
        hslot = hslot + 1 == NSLOT ? 0 : hslot + 1;
        z++;
    };
    while (z + Q <= ze) StaticFor<0, Q>::run([&](auto c) { step(c); });
    StaticFor<0, Q - 1>::run([&](auto c) {
        if (z < ze) step(c);
    });
    if constexpr (DEFER) {
        if (z > zb) store_out(z - 1);
    }
}

template <int MODE, int R, typename T, int BX, int BY, int VY, int VX, bool NTH>
__global__ __launch_bounds__(BX* BY) void k_zmarch(ZView v, Coefs w, int parity, int arow, int trow) {
    extern __shared__ __attribute__((aligned(16))) float lds[];
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    zmarch_tile<MODE, R, T, BX, BY, VY, VX, NTH>(v, w, lb, parity, arow, trow, lds);
}

// Batched shots: block_map[2 b], block_map[2 b + 1] = shot and block within
// the shot of workgroup b; shot -1 pads the map (the host lays it out per
// XCD, so it replaces xcd_remap here).
template <int R, typename T, int BX, int BY, int VY, int VX, bool NTH>
__global__ __launch_bounds__(BX* BY) void k_zmarch_batch(const ZView* __restrict__ views,
                                                        const int* __restrict__ block_map, Coefs w, int parity,
                                                        int arow, int trow) {
    extern __shared__ __attribute__((aligned(16))) float lds[];
    const int b = blockIdx.x;
    const int shot = block_map[2 * b], local = block_map[2 * b + 1];
    if (shot < 0) return;
    const ZView v = views[shot];
    zmarch_tile<MODE_WAVE, R, T, BX, BY, VY, VX, NTH>(v, w, local, parity, arow, trow, lds);
}

// Batched shots in one persistent launch: steps t0 .. t1 - 1 of every shot.
// The (shot, block) entries sit in 8 queues, one per XCD: queue x holds
// list[qoff[x]] .. list[qoff[x + 1] - 1], the entries the host laid out for
// XCD x, in map order.  Each step a workgroup takes entries one at a time
// from its own XCD's queue (the hardware register XCC_ID names the XCD) by
// an atomic ticket, and from the other queues in turn once that one is
// empty, so the XCD's compute units run a moving window of neighbouring
// tiles (their halo rows shared in the XCD's L2) and the work evens out as
// the hardware dispatcher evens out one launch's workgroups.  The next
// ticket is taken while the current entry runs.  Tickets count in
// sync[2 + 8 p + x] for step parity p; workgroup 0 clears the other
// parity's counters during a step, and the barrier after it orders the
// clearing before their next use.
// Between steps the grid meets at a barrier: arrivals count in sync[0]
// (each workgroup adds one per step; the barrier after step t opens at
// (t - t0 + 1) G), with an agent-scope release before the arrival and an
// acquire after the opening, so that a step's stores from any XCD reach the
// next step's loads on every other.  The wait is bounded: after spin_limit
// polls, or once another workgroup has given up, a workgroup sets sync[1]
// and leaves, and the host reports the error.  The host sizes the grid so
// that all of it is resident at once.  pmask: step t runs with parity
// t & pmask (0 for timing runs, which read the same levels every step and
// write a scratch output).
template <int R, typename T, int BX, int BY, int VY, int VX, bool NTH>
__global__ __launch_bounds__(BX* BY) void k_zmarch_batch_persistent(const ZView* __restrict__ views,
                                                                   const int* __restrict__ list,
                                                                   const int* __restrict__ qoff, Coefs w, int t0,
                                                                   int t1, int rec_on, int pmask,
                                                                   unsigned long long* sync, int spin_limit) {
    extern __shared__ __attribute__((aligned(16))) float lds[];
    __shared__ int give_up, next_entry;
    const int G = gridDim.x;
    // this workgroup's XCD (bits 3:0 of hardware register 20, XCC_ID)
    const int xcd = __builtin_amdgcn_s_getreg(0x1814) & 7;
    int q = xcd, tried = 0;
    unsigned long long* cnt = sync + 2;
    // thread 0: the next entry of the step's queues, or -1 when all are empty
    auto grab = [&](int par) -> int {
        while (tried < 8) {
            const unsigned long long k = atomicAdd(&cnt[8 * par + q], 1ull);
            if (k < (unsigned long long)(qoff[q + 1] - qoff[q])) return qoff[q] + (int)k;
            q = (q + 1) & 7;
            tried++;
        }
        return -1;
    };
    for (int t = t0; t < t1; t++) {
        const int par = t & 1;
        const int trow = (rec_on && t >= 1) ? t - 1 : -1;
        if (blockIdx.x == 0 && threadIdx.x < 8)
            __hip_atomic_store(&cnt[8 * (par ^ 1) + threadIdx.x], 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        q = xcd;
        tried = 0;
        if (threadIdx.x == 0) next_entry = grab(par);
        __syncthreads();
        int e = next_entry;
        while (e >= 0) {
            __syncthreads();   // every thread has read next_entry
            if (threadIdx.x == 0) next_entry = grab(par);
            const ZView v = views[list[2 * e]];
            zmarch_tile<MODE_WAVE, R, T, BX, BY, VY, VX, NTH>(v, w, list[2 * e + 1], t & pmask, t, trow, lds);
            __syncthreads();   // the next tile refills the LDS planes
            e = next_entry;
        }
        if (t + 1 == t1) break;
        // every wave's stores complete (in the L2), then one agent-scope
        // release per workgroup: the L2 write-back covers all its waves'
        // stores, and one per workgroup keeps the write-backs at each barrier
        // to the number of workgroups
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x < 64) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            __builtin_amdgcn_s_waitcnt(0);   // the write-back is done before the arrival below
        }
        if (threadIdx.x == 0) {
            // a workgroup that is not the last to arrive polls, at most
            // spin_limit times (so a zero limit makes the first arrival give up)
            const unsigned long long open = (unsigned long long)(t - t0 + 1) * (unsigned long long)G;
            const unsigned long long arrived = atomicAdd(&sync[0], 1ull) + 1ull;
            bool stop = false;
            if (arrived < open) {
                // sparse polls (a sleep of about 0.5 us between them, the
                // error flag every 64th) keep the waiting workgroups' coherent
                // loads from crowding the memory channel of the count
                for (int polls = 0;; polls++) {
                    if (polls >= spin_limit ||
                        ((polls & 63) == 0 && __hip_atomic_load(&sync[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
                        stop = true;
                        break;
                    }
                    if (__hip_atomic_load(&sync[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= open) break;
                    __builtin_amdgcn_s_sleep(20);
                }
            }
            if (stop) atomicOr(&sync[1], 1ull);
            give_up = stop;
        }
        __syncthreads();
        if (give_up) return;
        // one acquire per workgroup: it invalidates the compute unit's L1,
        // which the workgroup's waves share, and the L2 lines other XCDs may
        // have written; the barrier orders it before every wave's next loads
        if (threadIdx.x < 64) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __builtin_amdgcn_s_waitcnt(0);   // the invalidation is done before the barrier
        }
        __syncthreads();
    }
}

// dynamic LDS above 64 KiB must be enabled per kernel once
template <typename K>
static hipError_t allow_lds(K kernel, size_t bytes) {
    if (bytes <= 65536) return hipSuccess;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

template <int MODE, int R, typename T, int C>
static hipError_t zm_launch(const ZView& v, const Coefs& w, int parity, int arow, int trow, hipStream_t s) {
    constexpr TileCfg c = kTileCfgs[C];
    constexpr size_t lds = sizeof(LdsT<T, c.vx>) * ZTile<R, c.bx, c.by, c.vy, c.vx>::LDS_FLOATS;
    const int64_t nb = zmarch_blocks(v);
    if (nb == 0) return hipSuccess;
    auto k = k_zmarch<MODE, R, T, c.bx, c.by, c.vy, c.vx, c.nt>;
    static const hipError_t attr = allow_lds(k, lds);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL(k, dim3((unsigned)nb), dim3(c.bx * c.by), lds, s, v, w, parity, arow, trow);
    return hipGetLastError();
}

template <int MODE, int R, typename T>
static hipError_t zm_cfg(int cfg, const ZView& v, const Coefs& w, int parity, int arow, int trow, hipStream_t s) {
    switch (cfg) {
        case 0: return zm_launch<MODE, R, T, 0>(v, w, parity, arow, trow, s);
        case 1: return zm_launch<MODE, R, T, 1>(v, w, parity, arow, trow, s);
        case 2: return zm_launch<MODE, R, T, 2>(v, w, parity, arow, trow, s);
        case 3: return zm_launch<MODE, R, T, 3>(v, w, parity, arow, trow, s);
        case 4: return zm_launch<MODE, R, T, 4>(v, w, parity, arow, trow, s);
    }
    return hipErrorInvalidValue;
}

template <int MODE, typename T>
static hipError_t zm_r(int radius, int cfg, const ZView& v, const Coefs& w, int parity, int arow, int trow,
                       hipStream_t s) {
    switch (radius) {
        case 1: return zm_cfg<MODE, 1, T>(cfg, v, w, parity, arow, trow, s);
        case 2: return zm_cfg<MODE, 2, T>(cfg, v, w, parity, arow, trow, s);
        case 3: return zm_cfg<MODE, 3, T>(cfg, v, w, parity, arow, trow, s);
        case 4: return zm_cfg<MODE, 4, T>(cfg, v, w, parity, arow, trow, s);
    }
    return hipErrorInvalidValue;
}

template <int R, typename T, int C>
static hipError_t zb_launch(const ZView* views, const int* bmap, int nblocks, const Coefs& w, int parity, int arow,
                            int trow, hipStream_t s) {
    constexpr TileCfg c = kTileCfgs[C];
    constexpr size_t lds = sizeof(LdsT<T, c.vx>) * ZTile<R, c.bx, c.by, c.vy, c.vx>::LDS_FLOATS;
    if (nblocks == 0) return hipSuccess;
    auto k = k_zmarch_batch<R, T, c.bx, c.by, c.vy, c.vx, c.nt>;
    static const hipError_t attr = allow_lds(k, lds);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL(k, dim3((unsigned)nblocks), dim3(c.bx * c.by), lds, s, views, bmap, w, parity, arow, trow);
    return hipGetLastError();
}

template <typename T>
static hipError_t zb_cfg(int radius, int cfg, const ZView* views, const int* bmap, int nblocks, const Coefs& w,
                         int parity, int arow, int trow, hipStream_t s) {
    if (radius != 4) return hipErrorInvalidValue;
    switch (cfg) {
        case 0: return zb_launch<4, T, 0>(views, bmap, nblocks, w, parity, arow, trow, s);
        case 1: return zb_launch<4, T, 1>(views, bmap, nblocks, w, parity, arow, trow, s);
        case 2: return zb_launch<4, T, 2>(views, bmap, nblocks, w, parity, arow, trow, s);
        case 3: return zb_launch<4, T, 3>(views, bmap, nblocks, w, parity, arow, trow, s);
        case 4: return zb_launch<4, T, 4>(views, bmap, nblocks, w, parity, arow, trow, s);
    }
    return hipErrorInvalidValue;
}


template <typename T>
static hipError_t zbp_kernel(int radius, int cfg, const void*& k, size_t& lds, int& threads) {
    if (radius != 4 || cfg != kPersistentCfg) return hipErrorInvalidValue;
    constexpr TileCfg c = kTileCfgs[kPersistentCfg];
    lds = sizeof(LdsT<T, c.vx>) * ZTile<4, c.bx, c.by, c.vy, c.vx>::LDS_FLOATS;
    threads = c.bx * c.by;
    auto kf = k_zmarch_batch_persistent<4, T, c.bx, c.by, c.vy, c.vx, c.nt>;
    static const hipError_t attr = allow_lds(kf, lds);
    if (attr != hipSuccess) return attr;
    k = reinterpret_cast<const void*>(kf);
    return hipSuccess;
}

// workgroups of the persistent batched sweep one compute unit holds at once
template <typename T>
static hipError_t zbp_per_cu(int radius, int cfg, int& per_cu) {
    const void* k = nullptr;
    size_t lds = 0;
    int threads = 0;
    const hipError_t e = zbp_kernel<T>(radius, cfg, k, lds, threads);
    if (e != hipSuccess) return e;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, threads, lds);
}

template <typename T>
static hipError_t zbp_launch(int radius, int cfg, const ZView* views, const int* list, const int* qoff, int grid,
                             const Coefs& w, int t0, int t1, int rec_on, int pmask, unsigned long long* sync,
                             int spin_limit, hipStream_t s) {
    constexpr TileCfg c = kTileCfgs[kPersistentCfg];
    const void* k = nullptr;
    size_t lds = 0;
    int threads = 0;
    const hipError_t e = zbp_kernel<T>(radius, cfg, k, lds, threads);
    if (e != hipSuccess) return e;
    if (grid <= 0 || t1 <= t0) return hipSuccess;
    hipLaunchKernelGGL((k_zmarch_batch_persistent<4, T, c.bx, c.by, c.vy, c.vx, c.nt>), dim3((unsigned)grid),
                       dim3(threads), lds, s, views, list, qoff, w, t0, t1, rec_on, pmask, sync, spin_limit);
    return hipGetLastError();
}

// mode dispatch for one storage type and a set of modes
template <typename T>
static hipError_t zmarch_modes(int mode, int radius, int cfg, const ZView& v, const Coefs& w, int parity, int arow,
                               int trow, hipStream_t s) {
    switch (mode) {
        case MODE_HEAT: return zm_r<MODE_HEAT, T>(radius, cfg, v, w, parity, arow, trow, s);
        case MODE_WAVE: return zm_r<MODE_WAVE, T>(radius, cfg, v, w, parity, arow, trow, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace stn
