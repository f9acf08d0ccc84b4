// Stencil programs: several outputs over several input fields, each output a
// sum of linear or quadratic terms at arbitrary offsets (diagonals included).
//
// A workgroup owns a 64 x 16 tile and marches a z-chunk.  Every input's
// planes z-rz .. z+rz (the tile plus the program's reach in y and 4 columns
// either side in x) sit in an LDS ring of 2 rz + 2 slots, so one barrier per
// plane separates each slot's refill from its last reads.  A thread owns 4
// consecutive x points of one row and evaluates the terms in program order:
// a factor's 4 values are one or two aligned 16-byte LDS groups, picked apart
// by a wave-uniform switch on the x offset.  This kernel reads the terms at
// run time; program_rtc.cpp compiles the same tiling and arithmetic with the
// terms as constants.
#include "zmarch.hpp"

namespace stn {

namespace {

constexpr int TX = kProgTileX, TY = kProgTileY, NT = kProgThreads, LDX = TX + 8, GX = LDX / 4;
static_assert(NT == (TX / 4) * TY, "one 4-point group per thread");

// the 4 values at x0 + dx .. x0 + dx + 3 of an LDS row, where g points at
// the aligned group of x0 and |dx| <= 2 (dx is the same for every lane)
__device__ __forceinline__ float4 taps4(const float4* g, int dx) {
    const float4 c = g[0];
    switch (dx) {
        case -2: {
            const float4 p = g[-1];
            return make_float4(p.z, p.w, c.x, c.y);
        }
        case -1: {
            const float4 p = g[-1];
            return make_float4(p.w, c.x, c.y, c.z);
        }
        case 1: {
            const float4 n = g[1];
            return make_float4(c.y, c.z, c.w, n.x);
        }
        case 2: {
            const float4 n = g[1];
            return make_float4(c.z, c.w, n.x, n.y);
        }
        default:
            return c;
    }
}

__global__ __launch_bounds__(NT) void k_program(ProgView v) {
    extern __shared__ __attribute__((aligned(16))) float lds[];
    const int lb = xcd_remap(blockIdx.x, gridDim.x);
    const int tid = threadIdx.x, tx = tid % (TX / 4), ty = tid / (TX / 4);
    const int ntxy = v.ntx * v.nty;
    const int tile_x = lb % v.ntx, tile_y = (lb / v.ntx) % v.nty, zch = lb / ntxy;
    const int X0 = tile_x * TX, Y0 = tile_y * TY;
    const int nx = v.g.n[2], ny = v.g.n[1], nz = v.g.n[0];
    const int zb = zch * v.zc, ze = min(zb + v.zc, nz);
    const int rz = v.rz, ry = v.ry, NS = 2 * rz + 2;
    const int LDY = TY + 2 * ry, PLANE = LDY * LDX;
    const int64_t sz = v.g.s[0], sy = v.g.s[1];
    const int xmax4 = (int)(v.g.rowlen - v.g.xlead) - 4;

    // one plane of every input into its ring slot; rows and planes are
    // clamped into the halo, x groups to the last full group of the row
    // (clamped values only reach points that are not stored)
    auto load_plane = [&](int p) {
        const int pc = min(max(p, -rz), nz + rz - 1);
        const int slot = (p - zb + rz) % NS;
        const int ngroups = LDY * GX;
        for (int f = 0; f < v.nin; f++) {
            const float* base = v.in[f] + v.g.origin + (int64_t)pc * sz;
            float* L = lds + (f * NS + slot) * PLANE;
            for (int gi = tid; gi < ngroups; gi += NT) {
                const int row = gi / GX, cg = gi - row * GX;
                const int y = min(max(Y0 - ry + row, -ry), ny + ry - 1);
                const int x = min(X0 - 4 + 4 * cg, xmax4);
                *reinterpret_cast<float4*>(&L[row * LDX + 4 * cg]) =
                    *reinterpret_cast<const float4*>(base + (int64_t)y * sy + x);
            }
        }
    };

    for (int p = zb - rz; p < zb + rz; p++) load_plane(p);
    const int y = Y0 + ty, x0 = X0 + 4 * tx;
    const bool row_ok = y < ny && x0 < nx;
    for (int z = zb; z < ze; z++) {
        load_plane(z + rz);
        __syncthreads();
        float4 acc[kProgMaxFields];
#pragma unroll
        for (int o = 0; o < kProgMaxFields; o++) acc[o] = make_float4(0.f, 0.f, 0.f, 0.f);
        for (int t = 0; t < v.nterms; t++) {
            const ProgTerm& T = v.t[t];
            auto fac = [&](int f, const int (&o)[3]) -> float4 {
                const int slot = (z + o[0] - zb + rz) % NS;
                const float4* g = reinterpret_cast<const float4*>(lds + (f * NS + slot) * PLANE +
                                                                  (ty + ry + o[1]) * LDX + 4 + 4 * tx);
                return taps4(g, o[2]);
            };
            // s = fma(c, a, s) for one factor, fma(fl(c a), b, s) for two
            const float4 a = fac(T.in0, T.o0);
            float4 m = make_float4(T.coeff, T.coeff, T.coeff, T.coeff), b = a;
            if (T.nfac == 2) {
                b = fac(T.in1, T.o1);
                m = make_float4(__fmul_rn(T.coeff, a.x), __fmul_rn(T.coeff, a.y), __fmul_rn(T.coeff, a.z),
                                __fmul_rn(T.coeff, a.w));
            }
            // the output index is the same for every lane: a scalar branch
#pragma unroll
            for (int o = 0; o < kProgMaxFields; o++)
                if (T.out == o) {
                    acc[o].x = __builtin_fmaf(m.x, b.x, acc[o].x);
                    acc[o].y = __builtin_fmaf(m.y, b.y, acc[o].y);
                    acc[o].z = __builtin_fmaf(m.z, b.z, acc[o].z);
                    acc[o].w = __builtin_fmaf(m.w, b.w, acc[o].w);
                }
        }
        if (row_ok) {
            const int64_t off = v.g.origin + (int64_t)z * sz + (int64_t)y * sy + x0;
#pragma unroll
            for (int o = 0; o < kProgMaxFields; o++) {
                if (o >= v.nout) break;
                float* O = v.out[o] + off;
                if (x0 + 3 < nx) {
                    *reinterpret_cast<float4*>(O) = acc[o];
                } else {
                    const float r[4] = {acc[o].x, acc[o].y, acc[o].z, acc[o].w};
                    for (int i = 0; i < 4; i++)
                        if (x0 + i < nx) O[i] = r[i];
                }
            }
        }
    }
}

}  // namespace

hipError_t launch_program(const ProgView& v, hipStream_t s) {
    const int64_t nb = (int64_t)v.ntx * v.nty * v.nzc;
    if (nb == 0) return hipSuccess;
    const size_t lds = program_lds_bytes(v.nin, v.rz, v.ry);
    static const hipError_t attr = allow_lds(k_program, sizeof(float) * kProgMaxFields * (2 * kProgMaxR + 2) *
                                                            (kProgTileY + 2 * kProgMaxR) * (kProgTileX + 8));
    if (attr != hipSuccess) return attr;
    hipLaunchKernelGGL(k_program, dim3((unsigned)nb), dim3(kProgThreads), lds, s, v);
    return hipGetLastError();
}

}  // namespace stn
