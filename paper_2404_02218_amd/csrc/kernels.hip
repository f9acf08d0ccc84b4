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
//  small kernels: source injection / receiver sampling for k_point runs, box
//            copies (halo pack, unpack, periodic self-exchange), zero fill,
//            beta from squared slowness, FP64 gradient flush.
#include <climits>

#include "kernels.hpp"

namespace stn {

__device__ static inline float comp(const float4& v, int i) {
    return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}

// Workgroups are dispatched round-robin over the 8 XCDs (block b -> XCD b%8).
// Give XCD x the contiguous logical range [x*q + min(x,r), ...) so that
// neighbouring tiles (which read each other's edge rows as halo) share an L2.
__device__ static inline int xcd_remap(int b, int nb) {
    const int q = nb >> 3, r = nb & 7;
    const int x = b & 7, i = b >> 3;
    return x * q + min(x, r) + i;
}

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
    S::store((T*)v.out + off, time_update<MODE>(acc, ctr, prev, beta));
}

// -------------------------------------------------------------- k_zmarch
// LDS holds a ring of R+2 plane slots of (TY+2R) x (TX+8) floats.  The halo
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

// Each thread owns VX consecutive x points (VX = 4 or 8) in VY rows strided
// by BY; a row's VX values travel as VX/4 float4.
template <int MODE, int R, typename T, int BX, int BY, int VY, int VX, bool NTH>
__device__ __forceinline__ void zmarch_tile(const ZView& v, const Coefs& w, int lb, int parity, int arow,
                                            int trow, float* __restrict__ lds) {
    using Z = ZTile<R, BX, BY, VY, VX>;
    constexpr int NT = Z::NT, TX = Z::TX, TY = Z::TY, LDX = Z::LDX, PLANE = Z::PLANE, NSLOT = Z::NSLOT;
    constexpr int NHX = Z::NHX, NHY = Z::NHY, NHT = Z::NHT, NH = Z::NH;
    constexpr int NV = VX / 4;
    constexpr bool WAVE = MODE != MODE_HEAT;
    using S = Storage<T>;

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
        const int y = min(Y0 + ty + j * BY, ymax);
        own[j] = (int64_t)y * sy + min(X0 + VX * tx, xmaxv);
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
    float4 q[2 * R + 1][VY][NV];
#pragma unroll
    for (int k = 0; k < 2 * R + 1; k++)
#pragma unroll
        for (int j = 0; j < VY; j++) load_vec<T, VX>(U + (int64_t)(zb - R + k) * sz + own[j], q[k][j], false);
    for (int p = zb; p < min(zb + R, ze); p++) {
        float* L = lds + ((p - zb) % NSLOT) * PLANE;
#pragma unroll
        for (int m = 0; m < NH; m++)
            if (hon[m]) *reinterpret_cast<float4*>(&L[hlds[m]]) = S::load4(U + (int64_t)p * sz + hoff[m]);
    }
    float4 hal[NH];
    if (zb + R < ze) {
#pragma unroll
        for (int m = 0; m < NH; m++)
            if (hon[m]) hal[m] = S::load4(U + (int64_t)(zb + R) * sz + hoff[m]);
    }
    float4 cp[VY][NV], cb[VY][NV];
    if constexpr (WAVE) {
#pragma unroll
        for (int j = 0; j < VY; j++) {
            load_vec<T, VX>(P + (int64_t)zb * sz + own[j], cp[j], NTH);
            load_vec<T, VX>(B + (int64_t)zb * sz + own[j], cb[j], NTH);
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
            snext = v.src.tile_begin[tile];
            se = v.src.tile_begin[tile + 1];
            while (snext < se && v.src.zyx4[4 * snext] < zb) snext++;
            szn = snext < se ? v.src.zyx4[4 * snext] : INT_MAX;
        }
    }

    int slot = 0;             // slot of plane z
    int hslot = R % NSLOT;    // slot of plane z + R
    for (int z = zb; z < ze; z++) {
        float* L = lds + slot * PLANE;
#pragma unroll
        for (int j = 0; j < VY; j++)
#pragma unroll
            for (int c = 0; c < NV; c++)
                *reinterpret_cast<float4*>(&L[(R + ty + j * BY) * LDX + 4 + VX * tx + 4 * c]) = q[R][j][c];
        if (z + R < ze) {
            float* H = lds + hslot * PLANE;
#pragma unroll
            for (int m = 0; m < NH; m++)
                if (hon[m]) *reinterpret_cast<float4*>(&H[hlds[m]]) = hal[m];
        }

        const bool more = z + 1 < ze;
        float4 nxt[VY][NV], np[VY][NV], nb[VY][NV];
        if (more) {
            const int64_t zn = (int64_t)(z + 1) * sz;
#pragma unroll
            for (int j = 0; j < VY; j++) load_vec<T, VX>(U + zn + (int64_t)R * sz + own[j], nxt[j], false);
            if (z + R + 1 < ze) {
#pragma unroll
                for (int m = 0; m < NH; m++)
                    if (hon[m]) hal[m] = S::load4(U + zn + (int64_t)R * sz + hoff[m]);
            }
            if constexpr (WAVE) {
#pragma unroll
                for (int j = 0; j < VY; j++) {
                    load_vec<T, VX>(P + zn + own[j], np[j], NTH);
                    load_vec<T, VX>(B + zn + own[j], nb[j], NTH);
                }
            }
        }
        __syncthreads();

        float o[VY][VX];
        float dv[VY][VX];
#pragma unroll
        for (int j = 0; j < VY; j++) {
            const int row = R + ty + j * BY;
            const float* Lr = L + row * LDX + VX * tx;
            // x taps: 4 left of the thread's points, its own VX, 4 right
            float xv[VX + 8];
            {
                const float4 xl = *reinterpret_cast<const float4*>(Lr);
                const float4 xr = *reinterpret_cast<const float4*>(Lr + 4 + VX);
                xv[0] = xl.x;
                xv[1] = xl.y;
                xv[2] = xl.z;
                xv[3] = xl.w;
#pragma unroll
                for (int i = 0; i < VX; i++) xv[4 + i] = comp(q[R][j][i / 4], i % 4);
                xv[VX + 4] = xr.x;
                xv[VX + 5] = xr.y;
                xv[VX + 6] = xr.z;
                xv[VX + 7] = xr.w;
            }
            float4 ym[R][NV], yp[R][NV];
#pragma unroll
            for (int k = 1; k <= R; k++)
#pragma unroll
                for (int c = 0; c < NV; c++) {
                    ym[k - 1][c] = *reinterpret_cast<const float4*>(L + (row - k) * LDX + 4 + VX * tx + 4 * c);
                    yp[k - 1][c] = *reinterpret_cast<const float4*>(L + (row + k) * LDX + 4 + VX * tx + 4 * c);
                }
#pragma unroll
            for (int i = 0; i < VX; i++) {
                const int c = i / 4, e = i % 4;
                const float ctr = comp(q[R][j][c], e);
                float m[R], p[R];
                float acc = w.cd0 * ctr;
#pragma unroll
                for (int k = 1; k <= R; k++) {
                    m[k - 1] = comp(q[R - k][j][c], e);
                    p[k - 1] = comp(q[R + k][j][c], e);
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
                if constexpr (WAVE) {
                    o[j][i] = time_update<MODE>(acc, ctr, comp(cp[j][c], e), comp(cb[j][c], e));
                    if constexpr (MODE == MODE_WAVE_D) dv[j][i] = comp(cb[j][c], e) * acc;
                } else {
                    o[j][i] = time_update<MODE>(acc, ctr, 0.f, 0.f);
                }
            }
        }

        if constexpr (WAVE) {
            while (szn == z) {
                const int* e = v.src.zyx4 + 4 * snext;
                snext++;
                szn = snext < se ? v.src.zyx4[4 * snext] : INT_MAX;
                const int dy = e[1] - Y0, dx = e[2] - X0;
                const int idx = e[3];
                const double amt = v.src.amp[(int64_t)arow * v.src.n + idx] * (v.src.scale ? v.src.scale[idx] : 1.0);
#pragma unroll
                for (int j = 0; j < VY; j++)
#pragma unroll
                    for (int i = 0; i < VX; i++)
                        if (dy == ty + j * BY && dx == VX * tx + i) {
                            o[j][i] = inject<T>(o[j][i], amt);
                            if constexpr (MODE == MODE_WAVE_D) dv[j][i] = (float)((double)dv[j][i] + amt);
                        }
            }
        }

#pragma unroll
        for (int j = 0; j < VY; j++) {
            const int y = Y0 + ty + j * BY;
            const int x0 = X0 + VX * tx;
            if (y < ny && x0 < nx) {
                const int64_t off = (int64_t)z * sz + (int64_t)y * sy + x0;
                const bool full = x0 + VX - 1 < nx;
                if (full) {
                    float4 ov[NV];
#pragma unroll
                    for (int c = 0; c < NV; c++)
                        ov[c] = make_float4(o[j][4 * c], o[j][4 * c + 1], o[j][4 * c + 2], o[j][4 * c + 3]);
                    store_vec<T, VX>(O + off, ov, NTH && MODE != MODE_WAVE_ADJ);
                } else {
#pragma unroll
                    for (int i = 0; i < VX; i++)
                        if (x0 + i < nx) S::store(O + off + i, o[j][i]);
                }
                if constexpr (MODE == MODE_WAVE_D) {
                    float* D = v.dfield + v.g.origin + off;
#pragma unroll
                    for (int i = 0; i < VX; i++)
                        if (x0 + i < nx) D[i] = dv[j][i];
                }
                if constexpr (MODE == MODE_WAVE_ADJ) {
                    const float* D = v.dfield + v.g.origin + off;
                    float* G = v.gfield + v.g.origin + off;
                    if (full) {
#pragma unroll
                        for (int c = 0; c < NV; c++) {
                            const float4 d = *reinterpret_cast<const float4*>(D + 4 * c);
                            float4 g = *reinterpret_cast<const float4*>(G + 4 * c);
                            g.x = fmaf(o[j][4 * c], d.x, g.x);
                            g.y = fmaf(o[j][4 * c + 1], d.y, g.y);
                            g.z = fmaf(o[j][4 * c + 2], d.z, g.z);
                            g.w = fmaf(o[j][4 * c + 3], d.w, g.w);
                            *reinterpret_cast<float4*>(G + 4 * c) = g;
                        }
                    } else {
#pragma unroll
                        for (int i = 0; i < VX; i++)
                            if (x0 + i < nx) G[i] = fmaf(o[j][i], D[i], G[i]);
                    }
                }
            }
        }

        if (more) {
#pragma unroll
            for (int k = 0; k < 2 * R; k++)
#pragma unroll
                for (int j = 0; j < VY; j++)
#pragma unroll
                    for (int c = 0; c < NV; c++) q[k][j][c] = q[k + 1][j][c];
#pragma unroll
            for (int j = 0; j < VY; j++)
#pragma unroll
                for (int c = 0; c < NV; c++) {
                    q[2 * R][j][c] = nxt[j][c];
                    if constexpr (WAVE) {
                        cp[j][c] = np[j][c];
                        cb[j][c] = nb[j][c];
                    }
                }
        }
        slot = slot + 1 == NSLOT ? 0 : slot + 1;
        hslot = hslot + 1 == NSLOT ? 0 : hslot + 1;
    }
}

template <int MODE, int R, typename T, int BX, int BY, int VY, int VX, bool NTH>
__global__ __launch_bounds__(BX* BY) void k_zmarch(ZView v, Coefs w, int parity, int arow, int trow) {
    extern __shared__ __attribute__((aligned(16))) float lds[];
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    zmarch_tile<MODE, R, T, BX, BY, VY, VX, NTH>(v, w, lb, parity, arow, trow, lds);
}

template <int R, typename T, int BX, int BY, int VY, int VX, bool NTH>
__global__ __launch_bounds__(BX* BY) void k_zmarch_batch(const ZView* __restrict__ views,
                                                        const int* __restrict__ block_start, int nshots,
                                                        Coefs w, int parity, int arow, int trow) {
    extern __shared__ __attribute__((aligned(16))) float lds[];
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    // shot owning logical block lb: block_start is the prefix sum of blocks per shot
    int lo = 0, hi = nshots - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (block_start[mid] <= lb)
            lo = mid;
        else
            hi = mid - 1;
    }
    const ZView v = views[lo];
    zmarch_tile<MODE_WAVE, R, T, BX, BY, VY, VX, NTH>(v, w, lb - block_start[lo], parity, arow, trow, lds);
}

// ---------------------------------------------------------- small kernels
template <typename T>
__global__ void k_inject(T* base, SrcList src, int arow) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= src.n) return;
    T* p = base + src.off[s];
    const double amt = src.amp[(int64_t)arow * src.n + s] * (src.scale ? src.scale[s] : 1.0);
    Storage<T>::store(p, inject<T>(Storage<T>::load(p), amt));
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
    constexpr size_t lds = sizeof(float) * ZTile<R, c.bx, c.by, c.vy, c.vx>::LDS_FLOATS;
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
        case 5: return zm_launch<MODE, R, T, 5>(v, w, parity, arow, trow, s);
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

hipError_t launch_zmarch(int mode, int radius, int dtype, int cfg, const ZView& v, const Coefs& w, int parity,
                         int arow, int trow, hipStream_t s) {
    if (mode == MODE_WAVE_D || mode == MODE_WAVE_ADJ) {
        // the adjoint path is FP32 only
        if (dtype != DT_F32) return hipErrorInvalidValue;
        if (mode == MODE_WAVE_D) return zm_r<MODE_WAVE_D, float>(radius, cfg, v, w, parity, arow, trow, s);
        return zm_r<MODE_WAVE_ADJ, float>(radius, cfg, v, w, parity, arow, trow, s);
    }
    switch (dtype) {
        case DT_F32:
            return mode == MODE_HEAT ? zm_r<MODE_HEAT, float>(radius, cfg, v, w, parity, arow, trow, s)
                                     : zm_r<MODE_WAVE, float>(radius, cfg, v, w, parity, arow, trow, s);
        case DT_BF16:
            return mode == MODE_HEAT ? zm_r<MODE_HEAT, bf16>(radius, cfg, v, w, parity, arow, trow, s)
                                     : zm_r<MODE_WAVE, bf16>(radius, cfg, v, w, parity, arow, trow, s);
        case DT_F16:
            return mode == MODE_HEAT ? zm_r<MODE_HEAT, f16>(radius, cfg, v, w, parity, arow, trow, s)
                                     : zm_r<MODE_WAVE, f16>(radius, cfg, v, w, parity, arow, trow, s);
    }
    return hipErrorInvalidValue;
}

template <int R, typename T, int C>
static hipError_t zb_launch(const ZView* views, const int* bs, int nshots, int nblocks, const Coefs& w,
                            int parity, int arow, int trow, hipStream_t s) {
    constexpr TileCfg c = kTileCfgs[C];
    constexpr size_t lds = sizeof(float) * ZTile<R, c.bx, c.by, c.vy, c.vx>::LDS_FLOATS;
    if (nblocks == 0) return hipSuccess;
    auto k = k_zmarch_batch<R, T, c.bx, c.by, c.vy, c.vx, c.nt>;
    static const hipError_t attr = allow_lds(k, lds);
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL(k, dim3((unsigned)nblocks), dim3(c.bx * c.by), lds, s, views, bs, nshots, w, parity, arow,
                       trow);
    return hipGetLastError();
}

template <typename T>
static hipError_t zb_cfg(int radius, int cfg, const ZView* views, const int* bs, int nshots, int nblocks,
                         const Coefs& w, int parity, int arow, int trow, hipStream_t s) {
    if (radius != 4) return hipErrorInvalidValue;
    switch (cfg) {
        case 0: return zb_launch<4, T, 0>(views, bs, nshots, nblocks, w, parity, arow, trow, s);
        case 1: return zb_launch<4, T, 1>(views, bs, nshots, nblocks, w, parity, arow, trow, s);
        case 2: return zb_launch<4, T, 2>(views, bs, nshots, nblocks, w, parity, arow, trow, s);
        case 3: return zb_launch<4, T, 3>(views, bs, nshots, nblocks, w, parity, arow, trow, s);
        case 4: return zb_launch<4, T, 4>(views, bs, nshots, nblocks, w, parity, arow, trow, s);
        case 5: return zb_launch<4, T, 5>(views, bs, nshots, nblocks, w, parity, arow, trow, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_zmarch_batch(int radius, int dtype, int cfg, const ZView* d_views, const int* d_block_start,
                               int nshots, int nblocks, const Coefs& w, int parity, int arow, int trow,
                               hipStream_t s) {
    switch (dtype) {
        case DT_F32: return zb_cfg<float>(radius, cfg, d_views, d_block_start, nshots, nblocks, w, parity, arow, trow, s);
        case DT_BF16: return zb_cfg<bf16>(radius, cfg, d_views, d_block_start, nshots, nblocks, w, parity, arow, trow, s);
        case DT_F16: return zb_cfg<f16>(radius, cfg, d_views, d_block_start, nshots, nblocks, w, parity, arow, trow, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_inject(int dtype, void* out_base, const Grid3& g, const SrcList& src, int arow, hipStream_t s) {
    if (src.n == 0) return hipSuccess;
    const unsigned nb = blocks_for(src.n, 64);
    switch (dtype) {
        case DT_F32: hipLaunchKernelGGL(k_inject<float>, dim3(nb), dim3(64), 0, s, (float*)out_base + g.origin, src, arow); break;
        case DT_BF16: hipLaunchKernelGGL(k_inject<bf16>, dim3(nb), dim3(64), 0, s, (bf16*)out_base + g.origin, src, arow); break;
        case DT_F16: hipLaunchKernelGGL(k_inject<f16>, dim3(nb), dim3(64), 0, s, (f16*)out_base + g.origin, src, arow); break;
        default: return hipErrorInvalidValue;
    }
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
