// Launch descriptors and launcher entry points of the HIP kernels.  The host
// runtime (runtime.cpp) builds these descriptors after validating every
// argument, so the kernels themselves trust them.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <memory>
#include <string>
#include <vector>

#include "device.hpp"

namespace stn {

enum DType : int { DT_F32 = 0, DT_BF16 = 1, DT_F16 = 2 };

inline int dtype_size(int dt) { return dt == DT_F32 ? 4 : 2; }

// Padded field layout shared by every field of a plan.  Internal axes are
// (z, y, x); inactive leading axes of 1D/2D plans have extent 1 and stride 0.
struct Grid3 {
    int nd;          // active axes, 1..3 (the last nd of z, y, x)
    int n[3];        // interior extents
    int64_t s[3];    // strides in elements (s[2] == 1)
    int64_t origin;  // element offset of interior point (0,0,0) from the base
    int64_t xlead;   // elements from a row's first stored element to its first interior one
    int64_t rowlen;  // stored elements per row (the x pitch)
};

// Point sources of one field set.  zyx4 rows are (z, y, x, index) sorted by
// xy tile of the z-marching kernel, tile_begin is the CSR over tiles; off is
// the element offset (from the interior origin) of source `index`.
struct SrcList {
    int n;
    const int* zyx4;
    const int* tile_begin;
    const int64_t* off;
    const double* amp;    // [rows][n]; row chosen per launch
    const double* scale;  // [n] multiplier of amp, or null
    int ngrp;             // distinct positions
    const int* grp;       // entries ordered by (offset, index)
    const int* gbeg;      // [ngrp + 1] CSR of grp by position
};

struct RecList {
    int n;
    const int64_t* off;  // element offsets from the interior origin
    double* trace;       // [rows][n]
};

// One field set as the sweep kernels see it.  For in-place wave steps
// prev == out; a launch with parity 1 swaps the roles of u and prev/out.
struct ZView {
    const void* u;
    const void* prev;   // wave only
    const void* beta;   // wave only
    void* out;
    float* dfield;      // MODE_WAVE_D: written; MODE_WAVE_ADJ: read (same layout)
    float* gfield;      // MODE_WAVE_ADJ(2): imaging partial (same layout)
    const float* dfield2;  // MODE_WAVE_ADJ2: the second difference paired with the input level u
    int gfresh;            // MODE_WAVE_ADJ(2): the partial starts at zero (gfield is not read)
    const float* damp;  // MODE_WAVE_DAMP: per-axis damping [n0 | n1 | n2], gamma = (d0 + d1) + d2
    Grid3 g;
    int ntx, nty, zc, nzc;  // z-marching tiling: tiles along x, y; z-chunk length and count
    SrcList src;
    RecList rec;
};

// One field set as the depth-2 temporally blocked wave sweep sees it: inputs
// u^n, u^{n-1}, beta; outputs u^{n+1}, u^{n+2} in two buffers that alias none
// of the inputs.  Tiles are 64 x 32; src_t lists each tile's own sources,
// src_e the sources within R points of the tile in x and y (a source appears
// under every tile whose extended region holds it), both sorted by z.
struct TBView {
    const void* u;
    const void* prev;
    const void* beta;
    void* out1;
    void* out2;
    Grid3 g;
    int ntx, nty, zc, nzc;
    SrcList src_t;
    SrcList src_e;
    RecList rec;
    const float* damp;  // MODE_WAVE_DAMP: per-axis damping [n0 | n1 | n2]
    uint32_t range;   // bytes of each field's allocation (< 2^31)
};

// A stencil program: nout outputs, each a sum in program order of terms
// coeff * in[a](i + o_a) (* in[b](i + o_b)).  Offsets per internal axis
// (z, y, x), |offset| <= kProgMaxR.
inline constexpr int kProgMaxTerms = 64, kProgMaxFields = 4, kProgMaxR = 2;
inline constexpr int kProgTileX = 64, kProgTileY = 16, kProgThreads = 256;
struct ProgTerm {
    int out, nfac, in0, in1;
    int o0[3], o1[3];
    float coeff;
};
struct ProgView {
    const float* in[kProgMaxFields];
    float* out[kProgMaxFields];
    Grid3 g;
    int nin, nout, nterms;
    int rz, ry;              // reach of the program along z and y (0 on inactive axes)
    int ntx, nty, zc, nzc;   // tiling: 64 x 16 tiles, z-chunks
    ProgTerm t[kProgMaxTerms];
};
// dynamic LDS bytes of one workgroup of the program kernel
inline size_t program_lds_bytes(int nin, int rz, int ry) {
    return sizeof(float) * (size_t)nin * (2 * rz + 2) * (kProgTileY + 2 * ry) * (kProgTileX + 8);
}
hipError_t launch_program(const ProgView& v, hipStream_t s);
// the program compiled with its terms as constants (program_rtc.cpp):
// source text, compilation (shared by equal programs), launch on the
// current device (loads the code object there once)
struct RtcProgram;
// tile_y: 16 (256 threads) or 32 (512 threads); the tile is 64 points wide
std::string program_source(int nin, int nout, int rz, int ry, const std::vector<ProgTerm>& terms, bool tight,
                           int tile_y);
// LDS bytes of the compiled kernel's plane ring
inline size_t program_rtc_lds_bytes(int nin, int rz, int ry, bool tight, int tile_y) {
    return 16 * (size_t)nin * (2 * rz + (tight ? 1 : 2)) * (tile_y + 2 * ry) * ((kProgTileX + 8) / 4);
}
inline constexpr size_t kLdsPerCu = 160 * 1024;
std::shared_ptr<RtcProgram> program_compile(const std::string& src, int threads, std::string& log);
hipError_t launch_program_rtc(RtcProgram& rp, const ProgView& v, hipStream_t s);

// Tile shapes of the z-marching kernel: BX threads along x with VX points
// each, BY thread rows, each thread owning VY consecutive rows; nt: stream
// the once-read previous level and beta with non-temporal loads and the
// output with non-temporal stores.  VX = 8 gives 16-byte accesses for 16-bit
// storage (the fastest FP16 sweeps use it).
struct TileCfg {
    int bx, by, vy, vx;
    bool nt;
};
inline constexpr TileCfg kTileCfgs[] = {
    {16, 16, 2, 4, false},  // 64 x 32 tile, 256 threads
    {16, 16, 1, 4, true},   // 64 x 16 tile, 256 threads, streaming hints
    {8, 32, 1, 8, true},    // 64 x 32 tile, 256 threads, 8 points per lane, streaming hints
    {16, 16, 1, 4, false},  // 64 x 16 tile, 256 threads
    {16, 16, 1, 8, true},   // 128 x 16 tile, 256 threads, 8 points per lane, streaming hints
};
inline constexpr int kNumTileCfgs = sizeof(kTileCfgs) / sizeof(kTileCfgs[0]);
// the tile shape of the persistent batched sweep (64 x 16, streaming hints)
inline constexpr int kPersistentCfg = 1;
// 64-bit words of its barrier, error flag and per-XCD ticket counters
inline constexpr int kPersistentWords = 2 + 2 * 8;
// z-chunk lengths of the z-marching variants
inline constexpr int kZChunks[] = {256, 128, 64, 32};
inline constexpr int kNumZChunks = sizeof(kZChunks) / sizeof(kZChunks[0]);

inline int tile_tx(int cfg) { return kTileCfgs[cfg].vx * kTileCfgs[cfg].bx; }
inline int tile_ty(int cfg) { return kTileCfgs[cfg].by * kTileCfgs[cfg].vy; }
inline int tile_threads(int cfg) { return kTileCfgs[cfg].bx * kTileCfgs[cfg].by; }

struct Box3 {
    int64_t lo[3];
    int64_t n[3];
};

// up to 6 boxes per launch (the faces of a 3D box)
struct CopyList {
    int n;
    int64_t start[7];
    int64_t src[6][3];
    int64_t dst[6][3];
    int64_t size[6][3];
};

enum CopyDir : int { COPY_PACK = 0, COPY_UNPACK = 1, COPY_FIELD = 2 };

hipError_t launch_point(int mode, int radius, int dtype, const ZView& v, const Coefs& w, const Box3& box,
                        hipStream_t s);
hipError_t launch_zmarch(int mode, int radius, int dtype, int cfg, const ZView& v, const Coefs& w,
                         int parity, int arow, int trow, hipStream_t s);
// batched shots: d_block_map[2 b], d_block_map[2 b + 1] = shot and block within the shot of block b
hipError_t launch_zmarch_batch(int radius, int dtype, int cfg, const ZView* d_views, const int* d_block_map,
                               int nblocks, const Coefs& w, int parity, int arow, int trow, hipStream_t s);
// batched shots, steps t0 .. t1 - 1 in one persistent launch of `grid`
// workgroups (that the GPU holds at once); the (shot, block) pairs of XCD x
// are d_list[d_qoff[x]] .. d_list[d_qoff[x + 1] - 1] (8 queues, each in map
// order); step t has parity t & pmask, amplitude row t and, with rec_on,
// trace row t - 1.  d_sync: kPersistentWords zeroed words (barrier
// count, error flag, ticket counters; the flag is nonzero after the launch
// if a barrier wait gave up after spin_limit polls).  Radius 4, the 64 x 16
// streaming tile only.
hipError_t launch_zmarch_batch_persistent(int radius, int dtype, int cfg, const ZView* d_views, const int* d_list,
                                          const int* d_qoff, int grid, const Coefs& w, int t0, int t1, int rec_on,
                                          int pmask, unsigned long long* d_sync, int spin_limit, hipStream_t s);
// workgroups of that kernel one compute unit holds at once
hipError_t zmarch_batch_persistent_per_cu(int radius, int dtype, int cfg, int* per_cu);
// per-storage-type instantiations (zmarch_*.hip)
hipError_t zmarch_fwd_f32(int mode, int radius, int cfg, const ZView& v, const Coefs& w, int parity, int arow,
                          int trow, hipStream_t s);
hipError_t zmarch_fwd_bf16(int mode, int radius, int cfg, const ZView& v, const Coefs& w, int parity, int arow,
                           int trow, hipStream_t s);
hipError_t zmarch_fwd_f16(int mode, int radius, int cfg, const ZView& v, const Coefs& w, int parity, int arow,
                          int trow, hipStream_t s);
hipError_t zmarch_adj_f32(int mode, int radius, int cfg, const ZView& v, const Coefs& w, int parity, int arow,
                          int trow, hipStream_t s);
hipError_t zmarch_batch_f32(int radius, int cfg, const ZView* views, const int* bmap, int nblocks, const Coefs& w,
                            int parity, int arow, int trow, hipStream_t s);
hipError_t zmarch_batch_bf16(int radius, int cfg, const ZView* views, const int* bmap, int nblocks, const Coefs& w,
                             int parity, int arow, int trow, hipStream_t s);
hipError_t zmarch_batch_f16(int radius, int cfg, const ZView* views, const int* bmap, int nblocks, const Coefs& w,
                            int parity, int arow, int trow, hipStream_t s);
hipError_t zmarch_batch_persistent_f32(int radius, int cfg, const ZView* views, const int* list, const int* off, int grid,
                                      const Coefs& w, int t0, int t1, int rec_on, int pmask, unsigned long long* sync,
                                      int spin_limit, hipStream_t s);
hipError_t zmarch_batch_persistent_per_cu_f32(int radius, int cfg, int* per_cu);
hipError_t zmarch_batch_persistent_bf16(int radius, int cfg, const ZView* views, const int* list, const int* off, int grid,
                                      const Coefs& w, int t0, int t1, int rec_on, int pmask, unsigned long long* sync,
                                      int spin_limit, hipStream_t s);
hipError_t zmarch_batch_persistent_per_cu_bf16(int radius, int cfg, int* per_cu);
hipError_t zmarch_batch_persistent_f16(int radius, int cfg, const ZView* views, const int* list, const int* off, int grid,
                                      const Coefs& w, int t0, int t1, int rec_on, int pmask, unsigned long long* sync,
                                      int spin_limit, hipStream_t s);
hipError_t zmarch_batch_persistent_per_cu_f16(int radius, int cfg, int* per_cu);
// Depth-2 temporal blocking.  Wave (radius 4): steps arow and arow + 1;
// receivers record u^n as row trow_u and u^{n-1} as row trow_p (if >= 0).
// Heat (radius 1..4, FP32): u^{n+2} from u^n into out2.
hipError_t launch_tb2(int mode, int radius, int dtype, const TBView& v, const Coefs& w, int arow, int trow_u,
                      int trow_p, hipStream_t s);
hipError_t tb2_wave(int dtype, const TBView& v, const Coefs& w, int arow, int trow_u, int trow_p, hipStream_t s);
hipError_t tb2_heat_f32(int radius, const TBView& v, const Coefs& w, hipStream_t s);
hipError_t tb2_wave_damp_f32(const TBView& v, const Coefs& w, int arow, int trow_u, int trow_p, hipStream_t s);
// batched shots: d_views[nshots] (device), d_block_map as for launch_zmarch_batch
hipError_t tb2_batch(int dtype, const TBView* d_views, const int* d_block_map, int nblocks, const Coefs& w, int arow,
                     int trow_u, int trow_p, hipStream_t s);
// tile shape, threads and z-chunk lengths of the temporally blocked sweep
inline constexpr int kTB2TileX = 64, kTB2TileY = 32, kTB2Threads = 768;
// multi-step 2D heat (heat2d_tb.hip): T steps per launch on TX x TY tiles
struct Heat2dCfg {
    int t, tx, ty;
};
inline constexpr Heat2dCfg kHeat2dCfgs[] = {{4, 16, 16}, {8, 16, 16}, {8, 32, 32}, {16, 32, 32}};
inline constexpr int kNumHeat2dCfgs = sizeof(kHeat2dCfgs) / sizeof(kHeat2dCfgs[0]);
hipError_t launch_heat2d_tb(int cfg, int radius, const float* in, float* out, const Grid3& g, const Coefs& w,
                            hipStream_t s);

inline constexpr int kTB2ZChunks[] = {256, 128, 64};
inline constexpr int kNumTB2ZChunks = sizeof(kTB2ZChunks) / sizeof(kTB2ZChunks[0]);
hipError_t launch_inject(int dtype, void* out_base, const Grid3& g, const SrcList& src, int arow, hipStream_t s);
hipError_t launch_gather(const double* trace8, const double* w, int nc, int64_t n, int64_t rows, double* trace,
                         hipStream_t s);
hipError_t launch_spread(const double* amp, const double* w, int shift, int64_t n8, int64_t rows, double* amp8,
                         hipStream_t s);
hipError_t launch_record(int dtype, const void* base, const Grid3& g, const RecList& rec, int trow,
                         hipStream_t s);
hipError_t launch_boxcopy(int dtype, int dir, void* field, const Grid3& g, int64_t offset, const CopyList& L,
                          void* buf, hipStream_t s);
hipError_t launch_zero(void* p, int64_t bytes, hipStream_t s);
// zero every 32-bit element of `count` 3D FP32 field allocations of `elems`
// elements, stride_bytes apart from p, except their interiors (halo planes,
// rows and columns, the row padding and the tail), so that a sweep can write
// into them as its output
hipError_t launch_zero_frame(void* p, int count, int64_t stride_bytes, const Grid3& g, int halo, int64_t elems,
                             hipStream_t s);
hipError_t launch_beta(int dtype, const double* m, void* beta, const Grid3& g, double scale, hipStream_t s);
hipError_t launch_flush(const float* g32, double* grad, const Grid3& g, double scale, hipStream_t s);

// checks.hip: out[i] = dt2 / m[off[i]]; the data residual and its misfit
// 1/2 |trace - dobs|^2 (one workgroup, a fixed summation order); the scan of
// a field's interior (out[0] += NaNs, out[1] += infinities, out[2] = max of
// the largest finite |value| as the bits of a double)
hipError_t launch_point_scale(const double* m, const int64_t* off, int64_t n, double dt2, double* out, hipStream_t s);
hipError_t launch_misfit(const double* trace, const double* dobs, int64_t n, double* resid, double* misfit,
                         hipStream_t s);
hipError_t launch_scan(int dtype, const void* base, const Grid3& g, unsigned long long* out, hipStream_t s);
// copy `bytes` (a multiple of 4) of host data to device memory through the
// arguments of small kernels (512 words per launch)
hipError_t launch_fill_words(void* dst, const void* src, size_t bytes, hipStream_t s);

// blocks of one z-marching launch over a field set
inline int64_t zmarch_blocks(const ZView& v) { return (int64_t)v.ntx * v.nty * v.nzc; }

}  // namespace stn
