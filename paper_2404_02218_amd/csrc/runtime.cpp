// Host runtime behind the C ABI of libstencil.so: argument validation, the
// padded field layout, kernel-variant choice and autotuning, source/receiver
// tables, HIP-graph capture of time loops, halo exchange declarations, the
// batched-shot work list and the checkpointed adjoint driver.
//
// Every entry point validates all of its arguments before it enqueues any
// device work; errors are reported through a thread-local message.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <functional>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "kernels.hpp"
#include "stencil.h"

using namespace stn;

namespace {

thread_local std::string g_err;

stencil_status fail(stencil_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

#define HIP_TRY(expr)                                                                              \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return fail(STENCIL_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define ST_TRY(expr)                          \
    do {                                      \
        stencil_status s_ = (expr);           \
        if (s_ != STENCIL_OK) return s_;      \
    } while (0)

constexpr int64_t kMaxElems = int64_t(1) << 40;
constexpr int kAlignBytes = 128;  // first interior element of every row
constexpr int kPtrAlign = 256;    // field base pointers

int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

struct Layout {
    Grid3 g{};
    int ndim = 0;
    int halo = 0;
    int64_t extents[3] = {1, 1, 1};
    int64_t strides[3] = {0, 0, 0};
    int64_t offset = 0;
    int64_t elems = 0;
    int64_t bytes = 0;
};

stencil_status make_layout(int ndim, const int64_t* shape, int halo, int dtype, Layout& L) {
    const int es = dtype_size(dtype);
    const int64_t A = kAlignBytes / es;
    L = Layout{};
    L.ndim = ndim;
    L.halo = halo;
    int64_t n3[3] = {1, 1, 1};
    for (int i = 0; i < ndim; i++) {
        if (shape[i] < 0) return fail(STENCIL_E_INVALID, "shape entries must be >= 0");
        if (shape[i] > (int64_t(1) << 30)) return fail(STENCIL_E_NOMEM, "shape entry too large");
        n3[3 - ndim + i] = shape[i];
    }
    const int64_t xlead = round_up(halo, A);
    const int64_t ex = n3[2] + 2 * halo;
    const int64_t rowlen = round_up(xlead - halo + ex, A);
    const int64_t ey = ndim >= 2 ? n3[1] + 2 * halo : 1;
    const int64_t ez = ndim >= 3 ? n3[0] + 2 * halo : 1;
    if (ey > kMaxElems / rowlen || ez > kMaxElems / (ey * rowlen))
        return fail(STENCIL_E_NOMEM, "field would exceed 2^40 elements");
    L.offset = xlead - halo;
    int64_t s3[3] = {ndim >= 3 ? ey * rowlen : 0, ndim >= 2 ? rowlen : 0, 1};
    int64_t e3[3] = {ez, ey, ex};
    for (int i = 0; i < ndim; i++) {
        L.extents[i] = e3[3 - ndim + i];
        L.strides[i] = s3[3 - ndim + i];
    }
    L.elems = ez * ey * rowlen + A;
    L.bytes = L.elems * es;
    Grid3& g = L.g;
    g.nd = ndim;
    for (int a = 0; a < 3; a++) {
        g.n[a] = (int)n3[a];
        g.s[a] = s3[a];
    }
    const int64_t hz = ndim >= 3 ? halo : 0, hy = ndim >= 2 ? halo : 0;
    g.origin = L.offset + hz * s3[0] + hy * s3[1] + halo;
    g.xlead = xlead;
    g.rowlen = rowlen;
    return STENCIL_OK;
}

// device buffer owned by a plan
struct DevBuf {
    void* p = nullptr;
    size_t cap = 0;
    stencil_status ensure(size_t bytes) {
        if (bytes <= cap) return STENCIL_OK;
        if (p) {
            hipError_t e = hipDeviceSynchronize();
            if (e != hipSuccess) return fail(STENCIL_E_DEVICE, std::string("hipDeviceSynchronize: ") + hipGetErrorString(e));
            (void)hipFree(p);
            p = nullptr;
            cap = 0;
        }
        size_t want = std::max<size_t>(bytes, 256);
        hipError_t e = hipMalloc(&p, want);
        if (e != hipSuccess) {
            p = nullptr;
            return fail(STENCIL_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
        }
        cap = want;
        return STENCIL_OK;
    }
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

// Upload host bytes to a plan-owned device table.  The table may still be
// read by work enqueued earlier, so a changed table waits for the device.
struct DevTable {
    DevBuf buf;
    std::vector<char> host;
    bool valid = false;
    stencil_status upload(const void* data, size_t bytes) {
        if (valid && host.size() == bytes && (bytes == 0 || std::memcmp(host.data(), data, bytes) == 0))
            return STENCIL_OK;
        if (valid) {
            hipError_t e = hipDeviceSynchronize();
            if (e != hipSuccess) return fail(STENCIL_E_DEVICE, std::string("hipDeviceSynchronize: ") + hipGetErrorString(e));
        }
        ST_TRY(buf.ensure(bytes));
        if (bytes) {
            hipError_t e = hipMemcpy(buf.p, data, bytes, hipMemcpyHostToDevice);
            if (e != hipSuccess) return fail(STENCIL_E_DEVICE, std::string("hipMemcpy: ") + hipGetErrorString(e));
        }
        host.assign((const char*)data, (const char*)data + bytes);
        valid = true;
        return STENCIL_OK;
    }
};

// Variant numbers: 0 = point kernel; 1 .. kNumZVariants = z-marching
// (tile shape, z-chunk); then the depth-2 temporally blocked sweep, one per
// z-chunk, where the plan supports it.
struct Variant {
    bool zmarch = false;
    bool tb = false;   // depth-2 temporal blocking (tile 64 x 32 = tile shape 0)
    bool persistent = false;   // batch: every step in one launch with grid barriers
    int cfg = 0;
    int zc = 0;
};

constexpr int kNumZVariants = kNumTileCfgs * kNumZChunks;
// batch plans: persistent launches on the 64 x 16 streaming tile, one per
// z-chunk length
constexpr int kNumPersistent = kNumZChunks;
// steps of one tuning launch of a persistent variant
constexpr int kPersistentTuneSteps = 4;
// branches of the concurrent batch variant: the hardware queues a process
// gets by default
constexpr int kBranches = 4;

Variant variant_of(int v) {
    Variant r;
    if (v <= 0) return r;
    if (v > kNumZVariants) {
        r.tb = true;
        r.cfg = 0;
        r.zc = kTB2ZChunks[std::min(v - kNumZVariants - 1, kNumTB2ZChunks - 1)];
        return r;
    }
    r.zmarch = true;
    r.cfg = (v - 1) % kNumTileCfgs;
    r.zc = kZChunks[(v - 1) / kNumTileCfgs];
    return r;
}

// Default z-marching variant: the first tile shape, with the longest z-chunk
// that still gives at least 4 workgroups per compute unit (256 CUs).
int default_variant(const Layout& L) {
    if (L.ndim != 3) return 0;
    const int cfg = 0;
    const int64_t ntx = (L.g.n[2] + tile_tx(cfg) - 1) / tile_tx(cfg);
    const int64_t nty = (L.g.n[1] + tile_ty(cfg) - 1) / tile_ty(cfg);
    for (int zi = 0; zi < kNumZChunks; zi++) {
        const int64_t nzc = (L.g.n[0] + kZChunks[zi] - 1) / kZChunks[zi];
        if (ntx * nty * nzc >= 1024 || zi == kNumZChunks - 1) return 1 + zi * kNumTileCfgs + cfg;
    }
    return 1;
}

// Tuning choices per (device architecture, plan key): the variant's name,
// so that a cache file stays valid when variant numbers change.  Loaded once
// from $STENCIL_TUNE_CACHE (if set) and appended to after each tuning.
std::mutex g_tune_mu;
std::map<std::string, std::string> g_tune_cache;
bool g_tune_file_loaded = false;

const char* tune_cache_path() {
    const char* e = std::getenv("STENCIL_TUNE_CACHE");
    return (e && e[0]) ? e : nullptr;
}

// caller holds g_tune_mu.  Lines: "<arch> <plan key> <variant name>".
void load_tune_file() {
    if (g_tune_file_loaded) return;
    g_tune_file_loaded = true;
    const char* path = tune_cache_path();
    if (!path) return;
    std::ifstream in(path);
    std::string arch, key, name;
    while (in >> arch >> key >> name) g_tune_cache[arch + " " + key] = name;
}

void store_tune_choice(const std::string& full_key, const std::string& name) {
    g_tune_cache[full_key] = name;
    const char* path = tune_cache_path();
    if (!path) return;
    std::ofstream out(path, std::ios::app);
    if (out) out << full_key << " " << name << "\n";
}

}  // namespace

// One source/receiver table set (positions are host data, validated)
struct PointTables {
    DevTable zyx4, tiles, off;
    DevTable grp, gbeg;           // entries grouped by position (point-kernel injection)
    int n = 0, ngrp = 0;
    int cfg = -1;
};

struct stencil_plan_s {
    bool batch = false;
    bool program = false;   // a stencil program plan (stencil_program_create)
    int kind = 0, ndim = 0, radius = 0, halo = 0, dtype = 0, bc = 0;
    int64_t shape[3] = {0, 0, 0};
    double coeffs[5] = {0, 0, 0, 0, 0};
    Coefs w{};
    Layout L;
    int variant = 0;
    bool variant_forced = false;
    PointTables src, rec, adjrec;
    PointTables src_ext;   // sources listed under every tile within R of them (temporal blocking)
    // caller memory attached by stencil_set_workspace: the second field pair
    // of the temporally blocked wave sweep (per shot for a batch), zero halos
    void* ws = nullptr;
    size_t ws_bytes = 0;
    // source amounts scale[s] * amp[t][s] of a source with per-point scales
    DevBuf amp_scaled;
    std::vector<DevBuf> shot_amp_scaled;
    // offsets of stencil_wave_point_scale (two tables, reused while their
    // positions repeat) and of stencil_gradient's sources and receivers
    DevTable ps_off[2], gsrc_off, grec_off;
    int ps_next = 0;
    // stencil_gradient: source and receiver scales, residual; stencil_check:
    // NaN and infinity counts and the largest magnitude's bits
    DevBuf gsrc_scale, grec_scale, gresid, scan;
    // the workspace whose second-difference slots hold the last segment's
    // levels, written by the checkpointed forward (cleared once a recompute
    // overwrites them), with that forward's step count and interval
    const void* last_seg_ws = nullptr;
    int64_t last_seg_nsteps = 0, last_seg_k = 0;
    // interpolated sources and receivers (stencil_run_interp): corner
    // weights, the corners' amplitudes and the corner trace
    DevTable interp_sw, interp_rw;
    DevBuf interp_amp, interp_trace;
    // absorbing layer (stencil_wave_damping): FP32 profiles [n0 | n1 | n2]
    DevTable damp;
    bool damped = false;
    DevTable periodic_dummy;
    // graph cache of stencil_run
    hipStream_t cap = nullptr;
    hipGraphExec_t gexec = nullptr;
    std::vector<int64_t> gkey;
    // batch
    std::vector<Layout> shots;
    std::vector<PointTables> shot_src, shot_rec;
    DevTable views, block_map;   // block_map: (shot, block within the shot) per workgroup
    std::vector<int> bstart;
    int nblocks = 0;             // workgroups of a batched launch (with padding)
    // batched temporal blocking: per-shot extended source lists, the second
    // field pair of every shot, and the view tables of even and odd passes
    std::vector<PointTables> shot_src_ext;
    DevTable tbviews[2];
    // batch, concurrent variant: one sweep plan per shot with its own tuned
    // variant; the shots' runs go to kBranches streams, forked from and
    // joined back to the caller's stream (in one graph)
    std::vector<stencil_plan_s*> shot_plans;
    hipStream_t branch[kBranches] = {};
    hipEvent_t fork_ev = nullptr, join_ev[kBranches] = {};
    // the persistent batch variants: the barrier count and error flag
    // (device), the flag read back (pinned host), and the grid
    DevBuf bsync;
    unsigned long long* bsync_host = nullptr;
    int pgrid = 0;
    DevTable plist, poff;       // the per-XCD queues (entries, offsets)
    std::vector<int> hmap;      // the block map on the host
    // stencil program
    int nin = 0, nout = 0, reach[3] = {0, 0, 0};
    std::vector<ProgTerm> pterms;
    std::shared_ptr<RtcProgram> rtc;   // the compiled program (variant 0)
    std::shared_ptr<RtcProgram> rtc_tight;   // with the tight LDS ring (variant 2, compiled on first use)
    std::shared_ptr<RtcProgram> rtc_tall;    // 64 x 32 tiles of 512 threads (variant 3, compiled on first use)

    ~stencil_plan_s() {
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (cap) (void)hipStreamDestroy(cap);
        for (stencil_plan_s* q : shot_plans) delete q;
        for (hipStream_t b : branch)
            if (b) (void)hipStreamDestroy(b);
        if (fork_ev) (void)hipEventDestroy(fork_ev);
        for (hipEvent_t e : join_ev)
            if (e) (void)hipEventDestroy(e);
        if (bsync_host) (void)hipHostFree(bsync_host);
    }
};

namespace {

stencil_status check_plan(stencil_plan p, bool want_batch) {
    if (!p) return fail(STENCIL_E_INVALID, "plan is NULL");
    if (p->batch != want_batch)
        return fail(STENCIL_E_STATE, want_batch ? "not a batch plan" : "batch plan passed to a single-field call");
    return STENCIL_OK;
}

// The depth-2 temporally blocked sweep covers the 3D radius-4 wave (any
// storage type) and the 3D heat (FP32), with the zero halo.  Its loads start
// 8 elements left of a tile and address a field with 32-bit byte offsets.
bool tb_supported(const stencil_plan_s* p) {
    if (p->batch || p->ndim != 3 || p->bc != STENCIL_BC_DIRICHLET0) return false;
    const bool wave = p->kind == STENCIL_WAVE2 && p->radius == 4;
    const bool heat = p->kind == STENCIL_HEAT && p->dtype == STENCIL_F32;
    return (wave || heat) && p->L.g.xlead >= 8 && p->L.bytes < (int64_t(1) << 31);
}

bool tb_batch_supported(const stencil_plan_s* p) {
    if (!p->batch || p->radius != 4) return false;
    for (const Layout& L : p->shots)
        if (L.g.xlead < 8 || L.bytes >= (int64_t(1) << 31)) return false;
    return true;
}

// 2D heat, FP32, zero halo, radius <= 2: variants 1.. are the multi-step kernels
bool heat2d_supported(const stencil_plan_s* p) {
    return !p->batch && !p->program && p->ndim == 2 && p->kind == STENCIL_HEAT && p->dtype == STENCIL_F32 &&
           p->bc == STENCIL_BC_DIRICHLET0 && p->radius <= 2;
}

int variant_count_of(const stencil_plan_s* p) {
    if (p->program)
        return 3 + (program_rtc_lds_bytes(p->nin, p->reach[0], p->reach[1], false, 2 * kProgTileY) <= kLdsPerCu);
    // batch: z-marching and temporally blocked launches over all shots, then
    // the concurrent per-shot runs
    if (p->batch) return kNumZVariants + 1 + (tb_batch_supported(p) ? kNumTB2ZChunks : 0) + kNumPersistent + 1;
    if (p->ndim != 3) return heat2d_supported(p) ? 1 + kNumHeat2dCfgs : 1;
    return 1 + kNumZVariants + (tb_supported(p) ? kNumTB2ZChunks : 0);
}

// the batch variant that runs every shot with its own plan, concurrently
bool batch_concurrent(const stencil_plan_s* p, int v) { return p->batch && v == variant_count_of(p) - 1; }

// the batch variants that run every step in one persistent launch (just
// before the concurrent one)
bool batch_persistent(const stencil_plan_s* p, int v) {
    const int n = variant_count_of(p);
    return p->batch && v >= n - 1 - kNumPersistent && v < n - 1;
}

// variant v of plan p (batch plans add the persistent launches)
Variant plan_variant(const stencil_plan_s* p, int v) {
    if (!batch_persistent(p, v)) return variant_of(v);
    Variant r;
    r.zmarch = true;
    r.persistent = true;
    r.cfg = kPersistentCfg;
    r.zc = kZChunks[v - (variant_count_of(p) - 1 - kNumPersistent)];
    return r;
}

// plans of the sweep entry points (not stencil programs)
stencil_status check_sweep_plan(stencil_plan p) {
    ST_TRY(check_plan(p, false));
    if (p->program) return fail(STENCIL_E_STATE, "a stencil program plan takes stencil_program_apply");
    return STENCIL_OK;
}

stencil_status check_ptr(const void* p, const char* what) {
    if (!p) return fail(STENCIL_E_INVALID, std::string(what) + " is NULL");
    if (((uintptr_t)p) % kPtrAlign) return fail(STENCIL_E_INVALID, std::string(what) + " is not 256-byte aligned");
    return STENCIL_OK;
}

stencil_status set_coefs(stencil_plan p, int ndim, int radius, const double* coeffs) {
    if (!coeffs) return fail(STENCIL_E_INVALID, "coeffs is NULL");
    for (int k = 0; k <= radius; k++)
        if (!std::isfinite(coeffs[k])) return fail(STENCIL_E_INVALID, "coefficients must be finite");
    Coefs w{};
    for (int k = 0; k < 5; k++) w.c[k] = k <= radius ? (float)coeffs[k] : 0.f;
    w.cd0 = (float)(ndim * coeffs[0]);
    p->w = w;
    for (int k = 0; k < 5; k++) p->coeffs[k] = k <= radius ? coeffs[k] : 0.0;
    return STENCIL_OK;
}

// validate interior positions (host, [n][3]) against a layout
stencil_status check_positions(const Layout& L, int64_t n, const int64_t* pos, const char* what) {
    if (n < 0) return fail(STENCIL_E_INVALID, std::string(what) + ": negative count");
    if (n > (1 << 24)) return fail(STENCIL_E_INVALID, std::string(what) + ": too many points");
    if (n > 0 && !pos) return fail(STENCIL_E_INVALID, std::string(what) + ": positions are NULL");
    for (int64_t i = 0; i < n; i++)
        for (int d = 0; d < L.ndim; d++) {
            const int64_t c = pos[3 * i + d];
            if (c < 0 || c >= L.g.n[3 - L.ndim + d])
                return fail(STENCIL_E_INVALID, std::string(what) + ": position outside the interior");
        }
    return STENCIL_OK;
}

int64_t interior_offset(const Layout& L, const int64_t* p3) {
    int64_t off = 0;
    for (int d = 0; d < L.ndim; d++) off += p3[d] * L.g.s[3 - L.ndim + d];
    return off;
}

void zyx_of(const Layout& L, const int64_t* p3, int out[3]) {
    out[0] = out[1] = out[2] = 0;
    for (int d = 0; d < L.ndim; d++) out[3 - L.ndim + d] = (int)p3[d];
}

// Host tables of a point list for tile shape `cfg`: element offsets, the
// entries grouped by position (coincident entries are applied in index order
// by one thread), and for cfg >= 0 the CSR over xy tiles of the z-marching
// kernels, entries sorted by (tile, z).  ext > 0 lists a point under every
// tile whose box widened by `ext` in x and y holds it.
struct HostPoints {
    int n = 0, ngrp = 0;
    bool tiled = false;
    std::vector<int64_t> off;
    std::vector<int> grp, gbeg, zyx4, tiles;
};

void host_points(const Layout& L, int64_t n, const int64_t* pos, int cfg, HostPoints& H, int ext = 0) {
    H = HostPoints{};
    H.n = (int)n;
    H.off.assign((size_t)std::max<int64_t>(n, 1), 0);
    for (int64_t i = 0; i < n; i++) H.off[i] = interior_offset(L, pos + 3 * i);
    H.grp.assign((size_t)std::max<int64_t>(n, 1), 0);
    H.gbeg.assign(1, 0);
    for (int64_t i = 0; i < n; i++) H.grp[i] = (int)i;
    std::stable_sort(H.grp.begin(), H.grp.begin() + n, [&](int a, int b) { return H.off[a] < H.off[b]; });
    for (int64_t k = 1; k <= n; k++)
        if (k == n || H.off[H.grp[k]] != H.off[H.grp[k - 1]]) H.gbeg.push_back((int)k);
    H.ngrp = (int)H.gbeg.size() - 1;
    if (cfg < 0) return;
    H.tiled = true;
    const int TX = tile_tx(cfg), TY = tile_ty(cfg);
    const int ntx = std::max(1, (L.g.n[2] + TX - 1) / TX);
    const int nty = std::max(1, (L.g.n[1] + TY - 1) / TY);
    // sort by (xy tile, z): the kernel walks a tile's sources in z order
    std::vector<std::tuple<int, int, int>> order;
    order.reserve((size_t)n);
    for (int64_t i = 0; i < n; i++) {
        int zyx[3];
        zyx_of(L, pos + 3 * i, zyx);
        const int ty0 = std::max(0, (zyx[1] - ext) / TY), ty1 = std::min(nty - 1, (zyx[1] + ext) / TY);
        const int tx0 = std::max(0, (zyx[2] - ext) / TX), tx1 = std::min(ntx - 1, (zyx[2] + ext) / TX);
        for (int ty = ty0; ty <= ty1; ty++)
            for (int tx = tx0; tx <= tx1; tx++) order.emplace_back(ty * ntx + tx, zyx[0], (int)i);
    }
    std::stable_sort(order.begin(), order.end());
    const int64_t m = (int64_t)order.size();
    H.zyx4.assign((size_t)std::max<int64_t>(4 * m, 4), 0);
    H.tiles.assign((size_t)ntx * nty + 1, 0);
    for (int64_t k = 0; k < m; k++) {
        int zyx[3];
        const int i = std::get<2>(order[k]);
        zyx_of(L, pos + 3 * i, zyx);
        H.zyx4[4 * k + 0] = zyx[0];
        H.zyx4[4 * k + 1] = zyx[1];
        H.zyx4[4 * k + 2] = zyx[2];
        H.zyx4[4 * k + 3] = i;
        H.tiles[std::get<0>(order[k]) + 1]++;
    }
    for (size_t t = 1; t < H.tiles.size(); t++) H.tiles[t] += H.tiles[t - 1];
}

// Build the device tables of a point list (host_points, uploaded to the
// plan's tables).
stencil_status build_points(const Layout& L, int64_t n, const int64_t* pos, int cfg, PointTables& T, int ext = 0) {
    HostPoints H;
    host_points(L, n, pos, cfg, H, ext);
    T.n = H.n;
    T.ngrp = H.ngrp;
    ST_TRY(T.off.upload(H.off.data(), sizeof(int64_t) * (size_t)n));
    ST_TRY(T.grp.upload(H.grp.data(), sizeof(int) * (size_t)n));
    ST_TRY(T.gbeg.upload(H.gbeg.data(), sizeof(int) * H.gbeg.size()));
    if (H.tiled) {
        const int64_t m = H.tiles.back();
        ST_TRY(T.zyx4.upload(H.zyx4.data(), sizeof(int) * (size_t)(4 * m)));
        ST_TRY(T.tiles.upload(H.tiles.data(), sizeof(int) * H.tiles.size()));
    }
    T.cfg = cfg;
    return STENCIL_OK;
}

SrcList src_list(const PointTables& T, const double* amp, const double* scale) {
    SrcList s{};
    s.n = T.n;
    s.zyx4 = (const int*)T.zyx4.buf.p;
    s.tile_begin = (const int*)T.tiles.buf.p;
    s.off = (const int64_t*)T.off.buf.p;
    s.amp = amp;
    s.scale = scale;
    s.ngrp = T.ngrp;
    s.grp = (const int*)T.grp.buf.p;
    s.gbeg = (const int*)T.gbeg.buf.p;
    return s;
}

RecList rec_list(const PointTables& T, double* trace) {
    RecList r{};
    r.n = T.n;
    r.off = (const int64_t*)T.off.buf.p;
    r.trace = trace;
    return r;
}

// z-chunks: as many as chunks of at most `zc` planes need, of equal length
// (a short last chunk would pay the 2r warm-up planes for a few outputs)
void chunking(int nz, int zc, int& len, int& count) {
    const int c = std::max(1, std::min(zc, std::max(1, nz)));
    count = (nz + c - 1) / c;
    len = count > 0 ? (nz + count - 1) / count : c;
}

void set_tiling(ZView& v, const Layout& L, const Variant& var) {
    const int TX = tile_tx(var.cfg), TY = tile_ty(var.cfg);
    v.ntx = (L.g.n[2] + TX - 1) / TX;
    v.nty = (L.g.n[1] + TY - 1) / TY;
    chunking(L.g.n[0], var.zc, v.zc, v.nzc);
    if (L.g.n[0] == 0 || L.g.n[1] == 0 || L.g.n[2] == 0) v.ntx = v.nty = v.nzc = 0;
}

// Per-shot z-chunk lengths of a fused batch launch: the smallest shots,
// together at most 30% of the points, take 32-plane chunks and the others
// the variant's chunk length.  The block map puts the largest (shot, chunk)
// groups first on every XCD, so each launch ends with short workgroups that
// fill the compute units the long ones leave idle, while the large shots
// keep long chunks (fewer warm-up planes).
std::vector<int> batch_chunks(const std::vector<Layout>& shots, int zc) {
    const int ns = (int)shots.size();
    std::vector<int> out(ns, zc), order(ns);
    int64_t total = 0;
    for (int i = 0; i < ns; i++) {
        order[i] = i;
        total += (int64_t)shots[i].g.n[0] * shots[i].g.n[1] * shots[i].g.n[2];
    }
    auto pts = [&](int i) { return (int64_t)shots[i].g.n[0] * shots[i].g.n[1] * shots[i].g.n[2]; };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return pts(a) < pts(b); });
    int64_t acc = 0;
    for (int i : order) {
        acc += pts(i);
        if (10 * acc > 3 * total) break;
        out[i] = std::min(zc, 32);
    }
    return out;
}

// Copy list of the periodic self-exchange: each receive box takes the send
// box of the exchange facing the opposite way (internal z, y, x axes).
void periodic_copies(const Layout& L, int radius, std::vector<CopyList>& out);

// Exchange declarations of one rank: per axis and side, the r-thick face
// (star); with `box`, every neighbour direction d in {-1,0,1}^ndim \ {0}, so
// edges and corners too, in C order of d.
stencil_status exchanges_for(const Layout& L, int radius, const int32_t* grid, const int32_t* coord, int periodic,
                             std::vector<stencil_exchange>& ex, bool box = false) {
    ex.clear();
    for (int i = 0; i < L.ndim; i++) {
        if (grid[i] < 1 || coord[i] < 0 || coord[i] >= grid[i])
            return fail(STENCIL_E_INVALID, "rank coordinate outside the rank grid");
    }
    auto make = [&](const int* d) {
        stencil_exchange e;
        std::memset(&e, 0, sizeof(e));
        for (int j = 0; j < L.ndim; j++) {
            const int64_t n = L.g.n[3 - L.ndim + j];
            if (d[j] < 0) {
                e.at[j] = L.halo - radius;
                e.size[j] = radius;
                e.src_offset[j] = radius;
            } else if (d[j] > 0) {
                e.at[j] = L.halo + n;
                e.size[j] = radius;
                e.src_offset[j] = -radius;
            } else {
                e.at[j] = L.halo;
                e.size[j] = n;
            }
            e.to[j] = d[j];
        }
        ex.push_back(e);
    };
    auto has = [&](const int* d) {
        for (int j = 0; j < L.ndim; j++) {
            if (d[j] < 0 && !periodic && coord[j] == 0) return false;
            if (d[j] > 0 && !periodic && coord[j] == grid[j] - 1) return false;
        }
        return true;
    };
    if (!box) {
        for (int i = 0; i < L.ndim; i++)
            for (int side = 0; side < 2; side++) {
                int d[3] = {0, 0, 0};
                d[i] = side == 0 ? -1 : 1;
                if (has(d)) make(d);
            }
        return STENCIL_OK;
    }
    int ndir = 1;
    for (int i = 0; i < L.ndim; i++) ndir *= 3;
    for (int code = 0; code < ndir; code++) {
        int d[3] = {0, 0, 0}, rem = code;
        bool zero = true;
        for (int i = L.ndim - 1; i >= 0; i--) {
            d[i] = rem % 3 - 1;
            rem /= 3;
            zero &= d[i] == 0;
        }
        if (!zero && has(d)) make(d);
    }
    return STENCIL_OK;
}

void periodic_copies(const Layout& L, int radius, std::vector<CopyList>& out) {
    out.clear();
    int32_t grid[3] = {1, 1, 1}, coord[3] = {0, 0, 0};
    std::vector<stencil_exchange> ex;
    exchanges_for(L, radius, grid, coord, 1, ex);
    CopyList cl{};
    for (size_t k = 0; k < ex.size(); k++) {
        size_t partner = k;
        for (size_t j = 0; j < ex.size(); j++) {
            bool match = true;
            for (int i = 0; i < L.ndim; i++) match &= ex[j].to[i] == -ex[k].to[i];
            if (match) partner = j;
        }
        const int b = cl.n;
        int64_t vol = 1;
        for (int a = 0; a < 3; a++) {
            cl.src[b][a] = 0;
            cl.dst[b][a] = 0;
            cl.size[b][a] = 1;
        }
        for (int i = 0; i < L.ndim; i++) {
            const int a = 3 - L.ndim + i;
            cl.src[b][a] = ex[partner].at[i] + ex[partner].src_offset[i];
            cl.dst[b][a] = ex[k].at[i];
            cl.size[b][a] = ex[k].size[i];
            vol *= ex[k].size[i];
        }
        cl.start[b + 1] = cl.start[b] + vol;
        cl.n++;
    }
    out.push_back(cl);
}

// The point lists of one run: sources under their own tile (offsets and
// position groups for the point kernel), sources under every tile within R
// of them (temporal blocking) and receivers.
struct RunLists {
    SrcList st, se;
    RecList rl;
};

RunLists plan_lists(stencil_plan p, const stencil_source* src, const stencil_receivers* rec) {
    RunLists r;
    r.st = src_list(p->src, src ? src->amp : nullptr, nullptr);
    r.se = src_list(p->src_ext, src ? src->amp : nullptr, nullptr);
    r.rl = rec_list(p->rec, rec ? rec->trace : nullptr);
    return r;
}

// Depth-2 temporally blocked run.  Each pass reads one field pair and
// writes the other: the caller's (a, b) and the workspace pair alternate, so
// an even number of passes leaves u^{2K} in a and u^{2K-1} in b, as 2K plain
// in-place steps would.  Remaining steps (nsteps mod 4 of them when the pass
// count would be odd, else nsteps mod 2) run as plain z-marching sweeps on
// the same 64 x 32 tiles.  Receivers: pass k records its two input levels
// (rows 2k-1 and 2k-2); the level u^{2K-1} is recorded after the last pass.
stencil_status enqueue_run_tb(stencil_plan p, const Variant& var, void* a, void* b, const void* beta,
                              int64_t nsteps, const RunLists& RL, hipStream_t s) {
    const Layout& L = p->L;
    const SrcList& st = RL.st;
    const SrcList& se = RL.se;
    const RecList& rl = RL.rl;
    const int mode = p->damped ? MODE_WAVE_DAMP : MODE_WAVE;
    const float* damp = p->damped ? (const float*)p->damp.buf.p : nullptr;
    int64_t passes = nsteps / 2;
    if (passes & 1) passes--;
    void* pairs[2][2] = {{a, b}, {p->ws, (char*)p->ws + round_up(L.bytes, 256)}};
    void* newest = a;
    void* prev = b;
    for (int64_t k = 0; k < passes; k++) {
        void** dst = pairs[(k + 1) & 1];
        TBView v{};
        v.u = newest;
        v.prev = prev;
        v.beta = beta;
        v.out1 = dst[1];
        v.out2 = dst[0];
        v.g = L.g;
        v.ntx = (L.g.n[2] + kTB2TileX - 1) / kTB2TileX;
        v.nty = (L.g.n[1] + kTB2TileY - 1) / kTB2TileY;
        chunking(L.g.n[0], var.zc, v.zc, v.nzc);
        v.src_t = st;
        v.src_e = se;
        v.rec = rl;
        v.damp = damp;
        v.range = (uint32_t)L.bytes;
        const int tu = (rl.n > 0 && k >= 1) ? (int)(2 * k - 1) : -1;
        const int tp = (rl.n > 0 && k >= 1) ? (int)(2 * k - 2) : -1;
        HIP_TRY(launch_tb2(mode, p->radius, p->dtype, v, p->w, (int)(2 * k), tu, tp, s));
        newest = dst[0];
        prev = dst[1];
    }
    if (rl.n > 0 && passes > 0) HIP_TRY(launch_record(p->dtype, b, L.g, rl, (int)(2 * passes - 2), s));
    Variant plain;
    plain.zmarch = true;
    plain.cfg = var.cfg;
    plain.zc = var.zc;
    for (int64_t t = 2 * passes; t < nsteps; t++) {
        ZView v{};
        v.u = a;
        v.prev = b;
        v.out = b;
        v.beta = beta;
        v.g = L.g;
        set_tiling(v, L, plain);
        v.src = st;
        v.rec = rl;
        v.damp = damp;
        const int trow = (rl.n > 0 && t >= 1) ? (int)(t - 1) : -1;
        HIP_TRY(launch_zmarch(mode, p->radius, p->dtype, plain.cfg, v, p->w, (int)(t & 1), (int)t, trow, s));
    }
    if (rl.n > 0 && nsteps > 0) HIP_TRY(launch_record(p->dtype, (nsteps & 1) ? b : a, L.g, rl, (int)(nsteps - 1), s));
    return STENCIL_OK;
}

// 2D heat with the multi-step kernel: an even number of T-step passes
// between the two buffers (so, as after nsteps plain sweeps, the newest level
// is in a when nsteps is even), then plain sweeps for the rest.
static stencil_status enqueue_run_heat2d(stencil_plan p, void* a, void* b, int64_t nsteps, hipStream_t s) {
    const Layout& L = p->L;
    const int cfg = p->variant - 1;
    const int T = kHeat2dCfgs[cfg].t;
    int64_t passes = nsteps / T;
    if (passes & 1) passes--;
    void* cur = a;
    void* nxt = b;
    for (int64_t k = 0; k < passes; k++) {
        HIP_TRY(launch_heat2d_tb(cfg, p->radius, (const float*)cur, (float*)nxt, L.g, p->w, s));
        std::swap(cur, nxt);
    }
    Box3 box{};
    for (int a3 = 0; a3 < 3; a3++) {
        box.lo[a3] = 0;
        box.n[a3] = L.g.n[a3];
    }
    for (int64_t t = passes * T; t < nsteps; t++) {
        ZView v{};
        v.u = cur;
        v.prev = nxt;
        v.out = nxt;
        v.g = L.g;
        HIP_TRY(launch_point(MODE_HEAT, p->radius, p->dtype, v, p->w, box, s));
        std::swap(cur, nxt);
    }
    return STENCIL_OK;
}

// Enqueue nsteps sweeps of a single plan (no capture logic here).
stencil_status enqueue_run(stencil_plan p, void* a, void* b, const void* beta, int64_t nsteps,
                           const RunLists& RL, hipStream_t s) {
    const Layout& L = p->L;
    if (p->ndim == 2 && p->variant > 0 && heat2d_supported(p)) return enqueue_run_heat2d(p, a, b, nsteps, s);
    Variant var = variant_of(p->variant);
    const bool wave = p->kind == STENCIL_WAVE2;
    if (var.tb && wave) return enqueue_run_tb(p, var, a, b, beta, nsteps, RL, s);
    int64_t t0 = 0;
    if (var.tb) {
        // heat: an even number of two-step passes from one buffer into the
        // other (so u^{2K} is back in a), then plain sweeps on the same tiles
        int64_t passes = nsteps / 2;
        if (passes & 1) passes--;
        TBView v{};
        v.g = L.g;
        v.ntx = (L.g.n[2] + kTB2TileX - 1) / kTB2TileX;
        v.nty = (L.g.n[1] + kTB2TileY - 1) / kTB2TileY;
        chunking(L.g.n[0], var.zc, v.zc, v.nzc);
        v.range = (uint32_t)L.bytes;
        for (int64_t k = 0; k < passes; k++) {
            v.u = (k & 1) ? b : a;
            v.out2 = (k & 1) ? a : b;
            HIP_TRY(launch_tb2(MODE_HEAT, p->radius, p->dtype, v, p->w, 0, -1, -1, s));
        }
        t0 = 2 * passes;
        var.tb = false;
        var.zmarch = true;
    }
    const int mode = wave ? (p->damped ? MODE_WAVE_DAMP : MODE_WAVE) : MODE_HEAT;
    const float* damp = p->damped ? (const float*)p->damp.buf.p : nullptr;
    const SrcList& sl = RL.st;
    const RecList& rl = RL.rl;
    std::vector<CopyList> per;
    if (p->bc == STENCIL_BC_PERIODIC) periodic_copies(L, p->radius, per);
    for (int64_t t = t0; t < nsteps; t++) {
        const int parity = (int)(t & 1);
        void* cur = parity ? b : a;
        void* nxt = parity ? a : b;
        for (const CopyList& cl : per) HIP_TRY(launch_boxcopy(p->dtype, COPY_FIELD, cur, L.g, L.offset, cl, nullptr, s));
        if (var.zmarch) {
            ZView v{};
            v.u = a;
            v.prev = b;
            v.out = b;
            v.beta = beta;
            v.damp = damp;
            v.g = L.g;
            set_tiling(v, L, var);
            v.src = sl;
            v.rec = rl;
            const int trow = (rl.n > 0 && t >= 1) ? (int)(t - 1) : -1;
            HIP_TRY(launch_zmarch(mode, p->radius, p->dtype, var.cfg, v, p->w, parity, (int)t, trow, s));
        } else {
            ZView v{};
            v.u = cur;
            v.prev = nxt;
            v.out = nxt;
            v.beta = beta;
            v.damp = damp;
            v.g = L.g;
            Box3 box{};
            for (int a3 = 0; a3 < 3; a3++) {
                box.lo[a3] = 0;
                box.n[a3] = L.g.n[a3];
            }
            HIP_TRY(launch_point(mode, p->radius, p->dtype, v, p->w, box, s));
            if (sl.n) HIP_TRY(launch_inject(p->dtype, nxt, L.g, sl, (int)t, s));
            if (rl.n) HIP_TRY(launch_record(p->dtype, nxt, L.g, rl, (int)t, s));
        }
    }
    if (var.zmarch && rl.n > 0 && nsteps > 0) {
        void* newest = (nsteps & 1) ? b : a;
        HIP_TRY(launch_record(p->dtype, newest, L.g, rl, (int)(nsteps - 1), s));
    }
    return STENCIL_OK;
}

bool graphs_enabled() {
    const char* e = std::getenv("STENCIL_NO_GRAPH");
    return !(e && e[0] && e[0] != '0');
}

}  // namespace

// ------------------------------------------------------- allocation-free run
// The device memory stencil_run_noalloc works in: the point tables of a run
// and the formed source amounts.  Each GPU holds its own copy for the life
// of the process; host code reaches it only through the address
// hipGetSymbolAddress returns on that device (the array's name is a host
// stand-in).
constexpr size_t kNoAllocScratchBytes = size_t(8) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_ptr;   // device -> the array's address there

// the array's address on the current device, looked up once per device
stencil_status noalloc_scratch(void*& ptr) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it == g_scratch_ptr.end()) {
        void* q = nullptr;
        const hipError_t e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !q)
            return fail(STENCIL_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        it = g_scratch_ptr.emplace(dev, q).first;
    }
    ptr = it->second;
    return STENCIL_OK;
}

// Consecutive 256-byte aligned regions of the scratch array (base 0: only
// count the bytes).
struct ScratchCursor {
    uintptr_t base;
    size_t used = 0;
    char* take(size_t bytes) {
        const uintptr_t p = base + used;
        used += (bytes + 255) / 256 * 256;
        return (char*)p;
    }
};

// Device copies of one host point list in the scratch array: element
// offsets, position groups and (if tiled) the tile CSR.
struct ScratchPoints {
    char *off = nullptr, *grp = nullptr, *gbeg = nullptr, *zyx4 = nullptr, *tiles = nullptr;
};

void place_points(ScratchCursor& c, const HostPoints& H, ScratchPoints& P) {
    P.off = c.take(sizeof(int64_t) * H.off.size());
    P.grp = c.take(sizeof(int) * H.grp.size());
    P.gbeg = c.take(sizeof(int) * H.gbeg.size());
    if (H.tiled) {
        P.zyx4 = c.take(sizeof(int) * H.zyx4.size());
        P.tiles = c.take(sizeof(int) * H.tiles.size());
    }
}

hipError_t fill_points(const HostPoints& H, const ScratchPoints& P, hipStream_t s) {
    hipError_t e = launch_fill_words(P.off, H.off.data(), sizeof(int64_t) * H.off.size(), s);
    if (e == hipSuccess) e = launch_fill_words(P.grp, H.grp.data(), sizeof(int) * H.grp.size(), s);
    if (e == hipSuccess) e = launch_fill_words(P.gbeg, H.gbeg.data(), sizeof(int) * H.gbeg.size(), s);
    if (e == hipSuccess && H.tiled) e = launch_fill_words(P.zyx4, H.zyx4.data(), sizeof(int) * H.zyx4.size(), s);
    if (e == hipSuccess && H.tiled) e = launch_fill_words(P.tiles, H.tiles.data(), sizeof(int) * H.tiles.size(), s);
    return e;
}

SrcList scratch_src_list(const HostPoints& H, const ScratchPoints& P, const double* amp) {
    SrcList l{};
    l.n = H.n;
    l.zyx4 = (const int*)P.zyx4;
    l.tile_begin = (const int*)P.tiles;
    l.off = (const int64_t*)P.off;
    l.amp = amp;
    l.scale = nullptr;
    l.ngrp = H.ngrp;
    l.grp = (const int*)P.grp;
    l.gbeg = (const int*)P.gbeg;
    return l;
}

}  // namespace

// ======================================================================== C ABI
extern "C" {

const char* stencil_last_error(void) { return g_err.c_str(); }
int stencil_abi_version(void) { return 2; }

stencil_status stencil_create(stencil_plan* out, stencil_kind kind, int ndim, const int64_t* shape, int radius,
                              const double* coeffs, int halo, stencil_dtype dtype, stencil_bc bc) {
    if (!out) return fail(STENCIL_E_INVALID, "out is NULL");
    *out = nullptr;
    if (kind != STENCIL_HEAT && kind != STENCIL_WAVE2) return fail(STENCIL_E_INVALID, "unknown stencil kind");
    if (ndim < 1 || ndim > 3) return fail(ndim > 3 ? STENCIL_E_UNSUPPORTED : STENCIL_E_INVALID, "ndim must be 1, 2 or 3");
    if (!shape) return fail(STENCIL_E_INVALID, "shape is NULL");
    if (radius < 1 || radius > 4) return fail(STENCIL_E_UNSUPPORTED, "radius must be 1..4");
    if (halo < radius) return fail(STENCIL_E_INVALID, "halo must be >= radius (the largest access offset)");
    if (halo > 64) return fail(STENCIL_E_INVALID, "halo must be <= 64");
    if (dtype != STENCIL_F32 && dtype != STENCIL_BF16 && dtype != STENCIL_F16)
        return fail(STENCIL_E_INVALID, "unknown dtype");
    if (bc != STENCIL_BC_DIRICHLET0 && bc != STENCIL_BC_PERIODIC) return fail(STENCIL_E_INVALID, "unknown bc");
    stencil_plan p = new (std::nothrow) stencil_plan_s();
    if (!p) return fail(STENCIL_E_NOMEM, "out of host memory");
    p->kind = kind;
    p->ndim = ndim;
    p->radius = radius;
    p->halo = halo;
    p->dtype = dtype;
    p->bc = bc;
    for (int i = 0; i < ndim; i++) p->shape[i] = shape[i];
    stencil_status st = make_layout(ndim, shape, halo, dtype, p->L);
    if (st == STENCIL_OK) st = set_coefs(p, ndim, radius, coeffs);
    if (st == STENCIL_OK && bc == STENCIL_BC_PERIODIC) {
        for (int i = 0; i < ndim; i++)
            if (shape[i] < radius) st = fail(STENCIL_E_INVALID, "periodic axes need at least `radius` interior points");
    }
    if (st != STENCIL_OK) {
        delete p;
        return st;
    }
    p->variant = default_variant(p->L);
    if (heat2d_supported(p)) p->variant = 2;   // 8 steps per launch on 16 x 16 tiles
    *out = p;
    return STENCIL_OK;
}

stencil_status stencil_destroy(stencil_plan plan) {
    if (!plan) return fail(STENCIL_E_INVALID, "plan is NULL");
    delete plan;
    return STENCIL_OK;
}

static stencil_status layout_out(const Layout& L, int64_t* extents, int64_t* strides, int64_t* offset,
                                 int64_t* bytes) {
    for (int i = 0; i < L.ndim; i++) {
        if (extents) extents[i] = L.extents[i];
        if (strides) strides[i] = L.strides[i];
    }
    if (offset) *offset = L.offset;
    if (bytes) *bytes = L.bytes;
    return STENCIL_OK;
}

stencil_status stencil_layout(stencil_plan plan, int64_t* extents, int64_t* strides, int64_t* offset, int64_t* bytes) {
    ST_TRY(check_plan(plan, false));
    return layout_out(plan->L, extents, strides, offset, bytes);
}

stencil_status stencil_apply(stencil_plan p, void* out, const void* const* in, const int64_t* lo, const int64_t* hi,
                             void* stream) {
    ST_TRY(check_sweep_plan(p));
    if (!in) return fail(STENCIL_E_INVALID, "in is NULL");
    ST_TRY(check_ptr(out, "out"));
    ST_TRY(check_ptr(in[0], "in[0]"));
    const bool wave = p->kind == STENCIL_WAVE2;
    if (wave) {
        ST_TRY(check_ptr(in[1], "in[1]"));
        ST_TRY(check_ptr(in[2], "in[2]"));
        if (out == in[2]) return fail(STENCIL_E_INVALID, "out must not alias beta");
    }
    if (out == in[0]) return fail(STENCIL_E_INVALID, "out must not alias the level read at offsets");
    if (!lo || !hi) return fail(STENCIL_E_INVALID, "lo/hi are NULL");
    const Layout& L = p->L;
    Box3 box{};
    for (int a = 0; a < 3; a++) {
        box.lo[a] = 0;
        box.n[a] = 1;
    }
    for (int d = 0; d < L.ndim; d++) {
        const int a = 3 - L.ndim + d;
        if (lo[d] < 0 || hi[d] < lo[d] || hi[d] > L.g.n[a])
            return fail(STENCIL_E_INVALID, "box [lo, hi) must lie inside the interior");
        box.lo[a] = lo[d];
        box.n[a] = hi[d] - lo[d];
    }
    ZView v{};
    v.u = in[0];
    v.prev = wave ? in[1] : nullptr;
    v.beta = wave ? in[2] : nullptr;
    v.out = out;
    v.g = L.g;
    v.damp = p->damped ? (const float*)p->damp.buf.p : nullptr;
    const int mode = wave ? (p->damped ? MODE_WAVE_DAMP : MODE_WAVE) : MODE_HEAT;
    HIP_TRY(launch_point(mode, p->radius, p->dtype, v, p->w, box, (hipStream_t)stream));
    return STENCIL_OK;
}

static stencil_status run_args(stencil_plan p, void** fields, int64_t nsteps, const stencil_source* src,
                               const stencil_receivers* rec) {
    if (!fields) return fail(STENCIL_E_INVALID, "fields is NULL");
    const bool wave = p->kind == STENCIL_WAVE2;
    ST_TRY(check_ptr(fields[0], "fields[0]"));
    ST_TRY(check_ptr(fields[1], "fields[1]"));
    if (fields[0] == fields[1]) return fail(STENCIL_E_INVALID, "fields[0] and fields[1] must differ");
    if (wave) {
        ST_TRY(check_ptr(fields[2], "fields[2] (beta)"));
        if (fields[2] == fields[0] || fields[2] == fields[1]) return fail(STENCIL_E_INVALID, "beta must not alias a level");
    }
    if (nsteps < 0) return fail(STENCIL_E_INVALID, "nsteps must be >= 0");
    if (nsteps > (int64_t(1) << 30)) return fail(STENCIL_E_INVALID, "nsteps too large");
    if (src && src->n > 0) {
        ST_TRY(check_positions(p->L, src->n, src->pos, "sources"));
        if (!src->amp) return fail(STENCIL_E_INVALID, "source amplitudes are NULL");
    }
    if (rec && rec->n > 0) {
        ST_TRY(check_positions(p->L, rec->n, rec->pos, "receivers"));
        if (!rec->trace) return fail(STENCIL_E_INVALID, "receiver trace is NULL");
    }
    return STENCIL_OK;
}

static stencil_status prepare_points(stencil_plan p, const stencil_source* src, const stencil_receivers* rec) {
    const Variant var = variant_of(p->variant);
    const int cfg = (var.zmarch || var.tb) ? var.cfg : -1;
    ST_TRY(build_points(p->L, src ? src->n : 0, src ? src->pos : nullptr, cfg, p->src));
    if (var.tb) ST_TRY(build_points(p->L, src ? src->n : 0, src ? src->pos : nullptr, var.cfg, p->src_ext, 4));
    ST_TRY(build_points(p->L, rec ? rec->n : 0, rec ? rec->pos : nullptr, -1, p->rec));
    return STENCIL_OK;
}

// workspace bytes the plan's current variant needs: the second field pair
// of the temporally blocked wave sweep (one pair per shot for a batch)
static size_t run_workspace_bytes(const stencil_plan_s* p) {
    if (batch_concurrent(p, p->variant)) {
        // the shots whose own plan runs the temporally blocked sweep
        size_t b = 0;
        for (const stencil_plan_s* q : p->shot_plans) b += run_workspace_bytes(q);
        return b;
    }
    const Variant var = plan_variant(p, p->variant);
    if (!var.tb) return 0;
    if (p->batch) {
        size_t b = 0;
        for (const Layout& L : p->shots) b += 2 * (size_t)round_up(L.bytes, 256);
        return b;
    }
    if (p->kind != STENCIL_WAVE2 || p->ndim != 3) return 0;
    return 2 * (size_t)round_up(p->L.bytes, 256);
}

static stencil_status check_workspace(const stencil_plan_s* p) {
    const size_t need = run_workspace_bytes(p);
    if (need > 0 && (!p->ws || p->ws_bytes < need))
        return fail(STENCIL_E_STATE, "the temporally blocked variant needs a workspace of " + std::to_string(need) +
                                         " bytes (stencil_run_workspace, stencil_set_workspace)");
    return STENCIL_OK;
}

static stencil_status check_source_scale(const stencil_source* src) {
    if (src && src->n > 0 && src->scale && ((uintptr_t)src->scale & 7))
        return fail(STENCIL_E_INVALID, "source scales must be 8-byte aligned");
    return STENCIL_OK;
}

// A source with per-point scales: its amounts scale[s] * amp[t][s] (FP64)
// are formed once per call into `buf`, and `out` is the same source with
// those amounts and no scales.  Sources without scales pass through.
static stencil_status scaled_source(DevBuf& buf, const stencil_source* src, int64_t nsteps, stencil_source& out,
                                    const stencil_source*& use, hipStream_t s) {
    use = src;
    if (!src || src->n == 0 || !src->scale) return STENCIL_OK;
    ST_TRY(buf.ensure(sizeof(double) * (size_t)std::max<int64_t>(1, nsteps * src->n)));
    HIP_TRY(launch_spread(src->amp, src->scale, 0, src->n, nsteps, (double*)buf.p, s));
    out = *src;
    out.amp = (const double*)buf.p;
    out.scale = nullptr;
    use = &out;
    return STENCIL_OK;
}

static stencil_status run_common(stencil_plan p, void** fields, int64_t nsteps, const stencil_source* src_in,
                                 const stencil_receivers* rec, void* stream) {
    ST_TRY(run_args(p, fields, nsteps, src_in, rec));
    ST_TRY(check_source_scale(src_in));
    ST_TRY(check_workspace(p));
    ST_TRY(prepare_points(p, src_in, rec));
    hipStream_t s = (hipStream_t)stream;
    stencil_source scaled{};
    const stencil_source* src = src_in;
    ST_TRY(scaled_source(p->amp_scaled, src_in, nsteps, scaled, src, s));
    void* a = fields[0];
    void* b = fields[1];
    const void* beta = p->kind == STENCIL_WAVE2 ? fields[2] : nullptr;
    if (nsteps >= 2 && graphs_enabled()) {
        std::vector<int64_t> key = {(int64_t)(uintptr_t)a,
                                    (int64_t)(uintptr_t)b,
                                    (int64_t)(uintptr_t)beta,
                                    nsteps,
                                    p->variant,
                                    (int64_t)(uintptr_t)(src ? src->amp : nullptr),
                                    (int64_t)(uintptr_t)(rec ? rec->trace : nullptr),
                                    (int64_t)(uintptr_t)p->src.off.buf.p,
                                    (int64_t)(uintptr_t)p->rec.off.buf.p,
                                    (int64_t)(uintptr_t)p->src.zyx4.buf.p,
                                    (int64_t)(uintptr_t)p->src.tiles.buf.p,
                                    (int64_t)(uintptr_t)p->src_ext.zyx4.buf.p,
                                    (int64_t)(uintptr_t)p->src_ext.tiles.buf.p,
                                    (int64_t)(uintptr_t)p->ws,
                                    p->src.n,
                                    p->src.ngrp,
                                    p->src_ext.n,
                                    p->rec.n,
                                    (int64_t)(uintptr_t)p->src.grp.buf.p,
                                    (int64_t)(uintptr_t)p->src.gbeg.buf.p,
                                    (int64_t)p->damped,
                                    (int64_t)(uintptr_t)p->damp.buf.p};
        if (!p->gexec || key != p->gkey) {
            if (!p->cap) HIP_TRY(hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking));
            if (p->gexec) {
                HIP_TRY(hipStreamSynchronize(s));
                HIP_TRY(hipGraphExecDestroy(p->gexec));
                p->gexec = nullptr;
            }
            HIP_TRY(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
            stencil_status st = enqueue_run(p, a, b, beta, nsteps, plan_lists(p, src, rec), p->cap);
            hipGraph_t graph = nullptr;
            hipError_t e = hipStreamEndCapture(p->cap, &graph);
            if (st != STENCIL_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return st;
            }
            if (e != hipSuccess) return fail(STENCIL_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
            e = hipGraphInstantiate(&p->gexec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) {
                p->gexec = nullptr;
                return fail(STENCIL_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
            }
            p->gkey = key;
        }
        HIP_TRY(hipGraphLaunch(p->gexec, s));
    } else {
        ST_TRY(enqueue_run(p, a, b, beta, nsteps, plan_lists(p, src, rec), s));
    }
    if (nsteps & 1) std::swap(fields[0], fields[1]);
    return STENCIL_OK;
}

stencil_status stencil_run_noalloc(stencil_plan p, void** fields, int64_t nsteps, const stencil_source* src,
                                   const stencil_receivers* rec, void* stream) {
    ST_TRY(check_sweep_plan(p));
    ST_TRY(run_args(p, fields, nsteps, src, rec));
    ST_TRY(check_source_scale(src));
    ST_TRY(check_workspace(p));
    const Layout& L = p->L;
    const Variant var = variant_of(p->variant);
    const int cfg = (var.zmarch || var.tb) ? var.cfg : -1;
    const int64_t ns = src ? src->n : 0, nr = rec ? rec->n : 0;
    HostPoints hs, he, hr;
    host_points(L, ns, ns ? src->pos : nullptr, cfg, hs);
    if (var.tb) host_points(L, ns, ns ? src->pos : nullptr, var.cfg, he, 4);
    host_points(L, nr, nr ? rec->pos : nullptr, -1, hr);
    const bool scaled = ns > 0 && src->scale;
    // the regions this run needs, laid out from offset 0 first to size them
    ScratchCursor sizing{0};
    ScratchPoints ps, pe, pr;
    place_points(sizing, hs, ps);
    if (var.tb) place_points(sizing, he, pe);
    place_points(sizing, hr, pr);
    if (scaled) sizing.take(sizeof(double) * (size_t)(nsteps * ns));
    if (sizing.used > kNoAllocScratchBytes)
        return fail(STENCIL_E_NOMEM, "this run needs " + std::to_string(sizing.used) +
                                         " bytes of the static scratch; its maximum is " +
                                         std::to_string(kNoAllocScratchBytes) +
                                         " (fewer sources/receivers or steps per call, or stencil_run)");
    void* base = nullptr;
    ST_TRY(noalloc_scratch(base));
    ScratchCursor cur{(uintptr_t)base};
    place_points(cur, hs, ps);
    if (var.tb) place_points(cur, he, pe);
    place_points(cur, hr, pr);
    double* amounts = scaled ? (double*)cur.take(sizeof(double) * (size_t)(nsteps * ns)) : nullptr;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(fill_points(hs, ps, s));
    if (var.tb) HIP_TRY(fill_points(he, pe, s));
    HIP_TRY(fill_points(hr, pr, s));
    const double* amp = ns ? src->amp : nullptr;
    if (scaled) {
        HIP_TRY(launch_spread(src->amp, src->scale, 0, ns, nsteps, amounts, s));
        amp = amounts;
    }
    RunLists RL;
    RL.st = scratch_src_list(hs, ps, amp);
    RL.se = var.tb ? scratch_src_list(he, pe, amp) : SrcList{};
    RL.rl.n = hr.n;
    RL.rl.off = (const int64_t*)pr.off;
    RL.rl.trace = nr ? rec->trace : nullptr;
    ST_TRY(enqueue_run(p, fields[0], fields[1], p->kind == STENCIL_WAVE2 ? fields[2] : nullptr, nsteps, RL, s));
    if (nsteps & 1) std::swap(fields[0], fields[1]);
    return STENCIL_OK;
}

stencil_status stencil_wave_damping(stencil_plan p, const double* profile) {
    ST_TRY(check_sweep_plan(p));
    if (p->kind != STENCIL_WAVE2) return fail(STENCIL_E_STATE, "damping applies to wave plans");
    if (!profile) {
        p->damped = false;
        return STENCIL_OK;
    }
    if (p->dtype != STENCIL_F32) return fail(STENCIL_E_UNSUPPORTED, "the absorbing layer takes FP32 storage");
    const Grid3& g = p->L.g;
    std::vector<float> t((size_t)(g.n[0] + g.n[1] + g.n[2]), 0.f);
    size_t k = 0, base = 0;
    for (int a = 0; a < 3; a++) {
        const bool active = a >= 3 - p->ndim;
        for (int i = 0; i < g.n[a]; i++) {
            const double x = active ? profile[k++] : 0.0;
            if (!std::isfinite(x) || x < 0.0) return fail(STENCIL_E_INVALID, "damping must be finite and >= 0");
            t[base + (size_t)i] = (float)x;
        }
        base += (size_t)g.n[a];
    }
    ST_TRY(p->damp.upload(t.data(), sizeof(float) * std::max<size_t>(t.size(), 1)));
    p->damped = true;
    return STENCIL_OK;
}

stencil_status stencil_run(stencil_plan p, void** fields, int64_t nsteps, const stencil_source* src,
                           const stencil_receivers* rec, void* stream) {
    ST_TRY(check_sweep_plan(p));
    return run_common(p, fields, nsteps, src, rec, stream);
}

// Corners and multilinear weights of real interior positions ([n][3], the
// first ndim entries used): per axis base = min(floor(x), e - 2) (0 when
// e < 2), f = x - base; corner bit 0 -> (base, 1 - f), bit 1 ->
// (min(base + 1, e - 1), f); corners in C order of their bits.
static stencil_status interp_expand(const Layout& L, int64_t n, const double* pos, std::vector<int64_t>& cpos,
                                    std::vector<double>& w) {
    const int nd = L.ndim, nc = 1 << nd;
    if (n < 0 || n > (int64_t(1) << 24)) return fail(STENCIL_E_INVALID, "point count must be in [0, 2^24]");
    if (n > 0 && !pos) return fail(STENCIL_E_INVALID, "positions are NULL");
    cpos.assign((size_t)(n * nc * 3), 0);
    w.assign((size_t)(n * nc), 0.0);
    for (int64_t i = 0; i < n; i++) {
        int64_t base[3] = {0, 0, 0}, ext[3] = {1, 1, 1};
        double f[3] = {0, 0, 0};
        for (int j = 0; j < nd; j++) {
            ext[j] = L.g.n[3 - nd + j];
            const double x = pos[3 * i + j];
            if (!std::isfinite(x) || x < 0.0 || x > (double)(ext[j] - 1))
                return fail(STENCIL_E_INVALID, "an interpolated position lies outside the interior");
            if (ext[j] >= 2) {
                base[j] = std::min<int64_t>((int64_t)std::floor(x), ext[j] - 2);
                f[j] = x - (double)base[j];
            }
        }
        for (int c = 0; c < nc; c++) {
            double wt = 1.0;
            for (int j = 0; j < nd; j++) {
                const int bit = (c >> (nd - 1 - j)) & 1;
                cpos[(size_t)((i * nc + c) * 3 + j)] = bit ? std::min(base[j] + 1, ext[j] - 1) : base[j];
                wt *= bit ? f[j] : 1.0 - f[j];
            }
            w[(size_t)(i * nc + c)] = wt;
        }
    }
    return STENCIL_OK;
}

stencil_status stencil_interp_weights(stencil_plan p, int64_t n, const double* pos, int64_t* corners,
                                      double* weights) {
    ST_TRY(check_plan(p, false));
    if (!corners || !weights) return fail(STENCIL_E_INVALID, "corners and weights must be non-NULL");
    std::vector<int64_t> cp;
    std::vector<double> w;
    ST_TRY(interp_expand(p->L, n, pos, cp, w));
    std::copy(cp.begin(), cp.end(), corners);
    std::copy(w.begin(), w.end(), weights);
    return STENCIL_OK;
}

stencil_status stencil_run_interp(stencil_plan p, void** fields, int64_t nsteps, const stencil_source_interp* src,
                                  const stencil_receivers_interp* rec, void* stream) {
    ST_TRY(check_sweep_plan(p));
    ST_TRY(check_workspace(p));
    const int nd = p->ndim, nc = 1 << nd;
    const int64_t ns = src ? src->n : 0, nr = rec ? rec->n : 0;
    std::vector<int64_t> sp, rp;
    std::vector<double> sw, rw;
    ST_TRY(interp_expand(p->L, ns, src ? src->pos : nullptr, sp, sw));
    ST_TRY(interp_expand(p->L, nr, rec ? rec->pos : nullptr, rp, rw));
    if (ns > 0 && !src->amp) return fail(STENCIL_E_INVALID, "source amplitudes are NULL");
    if (nr > 0 && !rec->trace) return fail(STENCIL_E_INVALID, "receiver trace is NULL");
    if (nsteps < 0 || nsteps > (int64_t(1) << 30)) return fail(STENCIL_E_INVALID, "nsteps out of range");
    if (nr > 0 && nsteps * nr * nc > (int64_t(1) << 31)) return fail(STENCIL_E_NOMEM, "corner trace too large");
    ST_TRY(p->interp_sw.upload(sw.data(), sizeof(double) * sw.size()));
    ST_TRY(p->interp_rw.upload(rw.data(), sizeof(double) * rw.size()));
    if (ns > 0 && nsteps * ns * nc > (int64_t(1) << 31)) return fail(STENCIL_E_NOMEM, "corner amplitudes too large");
    ST_TRY(p->interp_trace.ensure(sizeof(double) * (size_t)std::max<int64_t>(1, nsteps * nr * nc)));
    ST_TRY(p->interp_amp.ensure(sizeof(double) * (size_t)std::max<int64_t>(1, nsteps * ns * nc)));
    // each corner entry's amount, w * amp (FP64), for the ordinary point-source path
    if (ns > 0)
        HIP_TRY(launch_spread(src->amp, (const double*)p->interp_sw.buf.p, nd, ns * nc, nsteps,
                              (double*)p->interp_amp.p, (hipStream_t)stream));
    const stencil_source s8{ns * nc, sp.data(), (const double*)p->interp_amp.p};
    const stencil_receivers r8{nr * nc, rp.data(), (double*)p->interp_trace.p};
    ST_TRY(run_common(p, fields, nsteps, ns ? &s8 : nullptr, nr ? &r8 : nullptr, stream));
    if (nr > 0)
        HIP_TRY(launch_gather((const double*)p->interp_trace.p, (const double*)p->interp_rw.buf.p, nc, nr, nsteps,
                              rec->trace, (hipStream_t)stream));
    return STENCIL_OK;
}

stencil_status stencil_exchanges(stencil_plan p, const int32_t* grid, const int32_t* coord, int periodic,
                                 stencil_exchange* out, int* n) {
    ST_TRY(check_plan(p, false));
    if (!grid || !coord || !n) return fail(STENCIL_E_INVALID, "grid, coord and n must be non-NULL");
    std::vector<stencil_exchange> ex;
    ST_TRY(exchanges_for(p->L, p->radius, grid, coord, periodic, ex));
    if (out && *n < (int)ex.size()) return fail(STENCIL_E_INVALID, "capacity of `out` is too small");
    if (out)
        for (size_t i = 0; i < ex.size(); i++) out[i] = ex[i];
    *n = (int)ex.size();
    return STENCIL_OK;
}

stencil_status stencil_exchanges_box(stencil_plan p, const int32_t* grid, const int32_t* coord, int periodic,
                                     stencil_exchange* out, int* n) {
    ST_TRY(check_plan(p, false));
    if (!grid || !coord || !n) return fail(STENCIL_E_INVALID, "grid, coord and n must be non-NULL");
    std::vector<stencil_exchange> ex;
    ST_TRY(exchanges_for(p->L, p->radius, grid, coord, periodic, ex, true));
    if (out && *n < (int)ex.size()) return fail(STENCIL_E_INVALID, "capacity of `out` is too small");
    if (out)
        for (size_t i = 0; i < ex.size(); i++) out[i] = ex[i];
    *n = (int)ex.size();
    return STENCIL_OK;
}

stencil_status stencil_program_create(stencil_plan* out, int ndim, const int64_t* shape, int halo, int nin,
                                      int nout, const stencil_term* terms, int nterms, stencil_dtype dtype) {
    if (!out) return fail(STENCIL_E_INVALID, "out is NULL");
    *out = nullptr;
    if (ndim < 1 || ndim > 3) return fail(ndim > 3 ? STENCIL_E_UNSUPPORTED : STENCIL_E_INVALID, "ndim must be 1, 2 or 3");
    if (!shape) return fail(STENCIL_E_INVALID, "shape is NULL");
    if (dtype != STENCIL_F32) return fail(STENCIL_E_UNSUPPORTED, "stencil programs take FP32 storage");
    if (halo < 1 || halo > 64) return fail(STENCIL_E_INVALID, "halo must be in [1, 64]");
    if (nin < 1 || nout < 1) return fail(STENCIL_E_INVALID, "nin and nout must be >= 1");
    if (nin > kProgMaxFields || nout > kProgMaxFields)
        return fail(STENCIL_E_UNSUPPORTED, "at most 4 input and 4 output fields");
    if (!terms || nterms < 1) return fail(STENCIL_E_INVALID, "a program needs at least one term");
    if (nterms > kProgMaxTerms) return fail(STENCIL_E_UNSUPPORTED, "at most 64 terms");
    const int lim = std::min(halo, kProgMaxR);
    std::vector<ProgTerm> pt((size_t)nterms);
    int reach[3] = {0, 0, 0};
    for (int t = 0; t < nterms; t++) {
        const stencil_term& T = terms[t];
        if (T.out < 0 || T.out >= nout) return fail(STENCIL_E_INVALID, "term output index out of range");
        if (T.nfac < 1 || T.nfac > 2) return fail(STENCIL_E_INVALID, "a term has 1 or 2 factors");
        if (!std::isfinite(T.coeff)) return fail(STENCIL_E_INVALID, "term coefficients must be finite");
        ProgTerm& P = pt[t];
        P.out = T.out;
        P.nfac = T.nfac;
        P.coeff = (float)T.coeff;
        for (int f = 0; f < 2; f++) {
            const bool used = f < T.nfac;
            const int in = used ? T.in[f] : 0;
            if (used && (in < 0 || in >= nin)) return fail(STENCIL_E_INVALID, "term input index out of range");
            int* o = f == 0 ? P.o0 : P.o1;
            for (int a = 0; a < 3; a++) {
                const int off = used ? T.off[f][a] : 0;
                if (a < 3 - ndim && off != 0) return fail(STENCIL_E_INVALID, "offset along an axis the grid lacks");
                if (off < -lim || off > lim)
                    return fail(off < -halo || off > halo ? STENCIL_E_INVALID : STENCIL_E_UNSUPPORTED,
                                "offsets must lie within min(halo, 2)");
                o[a] = off;
                reach[a] = std::max(reach[a], std::abs(off));
            }
            if (f == 0) P.in0 = in;
            else P.in1 = in;
        }
    }
    stencil_plan p = new (std::nothrow) stencil_plan_s();
    if (!p) return fail(STENCIL_E_NOMEM, "out of host memory");
    p->program = true;
    p->kind = -1;
    p->ndim = ndim;
    p->halo = halo;
    p->dtype = dtype;
    p->nin = nin;
    p->nout = nout;
    p->pterms = pt;
    for (int a = 0; a < 3; a++) p->reach[a] = reach[a];
    p->radius = std::max(1, std::max(reach[0], std::max(reach[1], reach[2])));
    for (int i = 0; i < ndim; i++) p->shape[i] = shape[i];
    stencil_status st = make_layout(ndim, shape, halo, dtype, p->L);
    if (st != STENCIL_OK) {
        delete p;
        return st;
    }
    std::string log;
    p->rtc = program_compile(program_source(nin, nout, reach[0], reach[1], pt, false, kProgTileY), kProgThreads, log);
    if (!p->rtc) {
        delete p;
        return fail(STENCIL_E_DEVICE, "compiling the stencil program failed: " + log);
    }
    *out = p;
    return STENCIL_OK;
}

stencil_status stencil_program_apply(stencil_plan p, void* const* outs, const void* const* ins, void* stream) {
    ST_TRY(check_plan(p, false));
    if (!p->program) return fail(STENCIL_E_STATE, "not a stencil program plan");
    if (!outs || !ins) return fail(STENCIL_E_INVALID, "outs and ins must be non-NULL");
    for (int f = 0; f < p->nin; f++) ST_TRY(check_ptr(ins[f], "input field"));
    for (int o = 0; o < p->nout; o++) {
        ST_TRY(check_ptr(outs[o], "output field"));
        for (int f = 0; f < p->nin; f++)
            if (outs[o] == ins[f]) return fail(STENCIL_E_INVALID, "an output aliases an input");
        for (int q = 0; q < o; q++)
            if (outs[o] == outs[q]) return fail(STENCIL_E_INVALID, "two outputs alias");
    }
    const Layout& L = p->L;
    ProgView v{};
    for (int f = 0; f < p->nin; f++) v.in[f] = (const float*)ins[f];
    for (int o = 0; o < p->nout; o++) v.out[o] = (float*)outs[o];
    v.g = L.g;
    v.nin = p->nin;
    v.nout = p->nout;
    v.nterms = (int)p->pterms.size();
    for (size_t t = 0; t < p->pterms.size(); t++) v.t[t] = p->pterms[t];
    v.rz = p->reach[0];
    v.ry = p->reach[1];
    const int ty = p->variant == 3 ? 2 * kProgTileY : kProgTileY;
    v.ntx = (L.g.n[2] + kProgTileX - 1) / kProgTileX;
    v.nty = (L.g.n[1] + ty - 1) / ty;
    chunking(L.g.n[0], 64, v.zc, v.nzc);
    if (L.g.n[0] == 0 || L.g.n[1] == 0 || L.g.n[2] == 0) return STENCIL_OK;
    std::shared_ptr<RtcProgram>* lazy = p->variant == 2 ? &p->rtc_tight : p->variant == 3 ? &p->rtc_tall : nullptr;
    if (lazy && !*lazy) {
        std::string log;
        *lazy = program_compile(program_source(p->nin, p->nout, p->reach[0], p->reach[1], p->pterms, p->variant == 2, ty),
                                16 * ty, log);
        if (!*lazy) return fail(STENCIL_E_DEVICE, "compiling the stencil program failed: " + log);
    }
    if (p->variant == 0) HIP_TRY(launch_program_rtc(*p->rtc, v, (hipStream_t)stream));
    else if (lazy) HIP_TRY(launch_program_rtc(**lazy, v, (hipStream_t)stream));
    else HIP_TRY(launch_program(v, (hipStream_t)stream));
    return STENCIL_OK;
}

// --------------------------------------------------------- exchange schedule
// directions (bit = C-order code over the plan's axes) in which a program
// reads input `field` outside the interior
static uint32_t program_dirs(const stencil_plan_s* p, int field) {
    const int nd = p->ndim;
    uint32_t m = 0;
    for (const ProgTerm& T : p->pterms)
        for (int k = 0; k < T.nfac; k++) {
            if ((k == 0 ? T.in0 : T.in1) != field) continue;
            const int* o = k == 0 ? T.o0 : T.o1;   // internal axes (z, y, x)
            // per axis the reachable d: 0 (if |o| < n) and sign(o) (if o != 0)
            int opts[3][2], nopt[3];
            for (int j = 0; j < nd; j++) {
                const int a = 3 - nd + j, off = o[a];
                nopt[j] = 0;
                if (std::abs(off) < p->L.g.n[a]) opts[j][nopt[j]++] = 0;
                if (off != 0) opts[j][nopt[j]++] = off > 0 ? 1 : -1;
            }
            int idx[3] = {0, 0, 0};
            for (;;) {
                int code = 0;
                bool zero = true, ok = true;
                for (int j = 0; j < nd; j++) {
                    if (nopt[j] == 0) {
                        ok = false;
                        break;
                    }
                    const int d = opts[j][idx[j]];
                    code = code * 3 + d + 1;
                    zero &= d == 0;
                }
                if (ok && !zero) m |= 1u << code;
                int j = nd - 1;
                while (j >= 0 && ++idx[j] >= nopt[j]) idx[j--] = 0;
                if (j < 0 || !ok) break;
            }
        }
    return m;
}

stencil_status stencil_program_halo_dirs(stencil_plan p, int field, uint32_t* dirs) {
    ST_TRY(check_plan(p, false));
    if (!p->program) return fail(STENCIL_E_STATE, "not a stencil program plan");
    if (!dirs) return fail(STENCIL_E_INVALID, "dirs is NULL");
    if (field < 0 || field >= p->nin) return fail(STENCIL_E_INVALID, "field index out of range");
    *dirs = program_dirs(p, field);
    return STENCIL_OK;
}

stencil_status stencil_schedule(const stencil_step* steps, int nsteps, int nfields, int loop,
                                stencil_action* prologue, int* nprologue, stencil_action* body, int* nbody) {
    if (!nprologue || !nbody) return fail(STENCIL_E_INVALID, "nprologue and nbody must be non-NULL");
    if (nsteps < 0 || (nsteps > 0 && !steps)) return fail(STENCIL_E_INVALID, "bad step list");
    if (nfields < 1 || nfields > 4096) return fail(STENCIL_E_INVALID, "nfields must be in [1, 4096]");
    // reads[k][f]: directions step k reads field f in; writes[k][f]
    std::vector<std::vector<uint32_t>> reads((size_t)nsteps, std::vector<uint32_t>((size_t)nfields, 0));
    std::vector<std::vector<char>> writes((size_t)nsteps, std::vector<char>((size_t)nfields, 0));
    int ndim = -1;
    for (int k = 0; k < nsteps; k++) {
        const stencil_plan p = steps[k].program;
        ST_TRY(check_plan(p, false));
        if (!p->program) return fail(STENCIL_E_INVALID, "a step's plan is not a stencil program");
        if (ndim >= 0 && p->ndim != ndim) return fail(STENCIL_E_STATE, "the programs differ in ndim");
        ndim = p->ndim;
        for (int i = 0; i < p->nin; i++) {
            const int f = steps[k].in[i];
            if (f < 0 || f >= nfields) return fail(STENCIL_E_INVALID, "input field id out of range");
            reads[k][f] |= program_dirs(p, i);
        }
        for (int o = 0; o < p->nout; o++) {
            const int f = steps[k].out[o];
            if (f < 0 || f >= nfields) return fail(STENCIL_E_INVALID, "output field id out of range");
            for (int i = 0; i < p->nin; i++)
                if (steps[k].in[i] == f) return fail(STENCIL_E_INVALID, "a step's output is one of its inputs");
            if (writes[k][f]) return fail(STENCIL_E_INVALID, "a step writes one field twice");
            writes[k][f] = 1;
        }
    }
    // directions read of f from step k on, up to its next write (wrapping
    // into the next iteration of a loop, at most once around)
    auto need_from = [&](int k, int f) {
        uint32_t m = 0;
        for (int i = 0; i < (loop ? nsteps : nsteps - k); i++) {
            const int j = (k + i) % nsteps;
            if (writes[j][f]) break;
            m |= reads[j][f];
        }
        return m;
    };
    auto simulate = [&](std::vector<uint32_t> fresh, std::vector<stencil_action>* out) {
        for (int k = 0; k < nsteps; k++) {
            for (int f = 0; f < nfields; f++)
                if (reads[k][f] & ~fresh[f]) {
                    const uint32_t d = need_from(k, f) & ~fresh[f];
                    if (out) out->push_back(stencil_action{STENCIL_ACT_EXCHANGE, k, f, d});
                    fresh[f] |= d;
                }
            if (out) out->push_back(stencil_action{STENCIL_ACT_APPLY, k, -1, 0});
            for (int f = 0; f < nfields; f++)
                if (writes[k][f]) fresh[f] = 0;
        }
        return fresh;
    };
    std::vector<uint32_t> entry((size_t)nfields, 0);
    if (loop && nsteps > 0) {
        // the state at the end of any iteration, restricted to what is read
        // before the field's first write in the body
        const std::vector<uint32_t> end = simulate(entry, nullptr);
        for (int f = 0; f < nfields; f++) entry[f] = end[f] & need_from(0, f);
    }
    std::vector<stencil_action> pro, bod;
    for (int f = 0; f < nfields; f++)
        if (entry[f]) pro.push_back(stencil_action{STENCIL_ACT_EXCHANGE, -1, f, entry[f]});
    simulate(entry, &bod);
    if ((prologue && *nprologue < (int)pro.size()) || (body && *nbody < (int)bod.size()))
        return fail(STENCIL_E_INVALID, "capacity of an action list is too small");
    if (prologue) std::copy(pro.begin(), pro.end(), prologue);
    if (body) std::copy(bod.begin(), bod.end(), body);
    *nprologue = (int)pro.size();
    *nbody = (int)bod.size();
    return STENCIL_OK;
}

static stencil_status halo_copy(stencil_plan p, void* field, const stencil_exchange* ex, int n, void* buf,
                                int dir, void* stream) {
    ST_TRY(check_plan(p, false));
    ST_TRY(check_ptr(field, "field"));
    if (n < 0 || (n > 0 && !ex)) return fail(STENCIL_E_INVALID, "bad exchange list");
    if (n > 0 && !buf) return fail(STENCIL_E_INVALID, "buf is NULL");
    const Layout& L = p->L;
    std::vector<CopyList> lists;
    CopyList cl{};
    for (int k = 0; k < n; k++) {
        int64_t vol = 1;
        const int b = cl.n;
        for (int a = 0; a < 3; a++) {
            cl.src[b][a] = cl.dst[b][a] = 0;
            cl.size[b][a] = 1;
        }
        for (int i = 0; i < L.ndim; i++) {
            const int a = 3 - L.ndim + i;
            const int64_t at = ex[k].at[i], sz = ex[k].size[i];
            const int64_t from = dir == COPY_PACK ? at + ex[k].src_offset[i] : at;
            if (sz < 0 || from < 0 || from + sz > L.extents[i])
                return fail(STENCIL_E_INVALID, "exchange box outside the field bounds");
            cl.src[b][a] = from;
            cl.dst[b][a] = from;
            cl.size[b][a] = sz;
            vol *= sz;
        }
        cl.start[b + 1] = cl.start[b] + vol;
        cl.n++;
        if (cl.n == 6 || k == n - 1) {
            lists.push_back(cl);
            const int64_t carry = cl.start[cl.n];
            cl = CopyList{};
            cl.start[0] = carry;
        }
    }
    // each list addresses buf from its own start offset
    for (CopyList& l : lists) {
        const int64_t base = l.start[0];
        for (int b = 0; b <= l.n; b++) l.start[b] -= base;
        char* bp = (char*)buf + base * dtype_size(p->dtype);
        HIP_TRY(launch_boxcopy(p->dtype, dir, field, L.g, L.offset, l, bp, (hipStream_t)stream));
    }
    return STENCIL_OK;
}

stencil_status stencil_halo_pack(stencil_plan p, const void* field, const stencil_exchange* ex, int n, void* buf,
                                 void* stream) {
    return halo_copy(p, (void*)field, ex, n, buf, COPY_PACK, stream);
}

stencil_status stencil_halo_unpack(stencil_plan p, void* field, const stencil_exchange* ex, int n, const void* buf,
                                   void* stream) {
    return halo_copy(p, field, ex, n, (void*)buf, COPY_UNPACK, stream);
}

// ------------------------------------------------------------------ batch
stencil_status stencil_batch_create(stencil_plan* out, int nshots, const int64_t* shapes, int radius,
                                    const double* coeffs, int halo, stencil_dtype dtype) {
    if (!out) return fail(STENCIL_E_INVALID, "out is NULL");
    *out = nullptr;
    if (nshots < 1 || nshots > 4096) return fail(STENCIL_E_INVALID, "nshots must be 1..4096");
    if (!shapes) return fail(STENCIL_E_INVALID, "shapes is NULL");
    if (radius != 4) return fail(STENCIL_E_UNSUPPORTED, "batched shots support radius 4 (space order 8)");
    if (halo < radius || halo > 64) return fail(STENCIL_E_INVALID, "halo must be in [radius, 64]");
    if (dtype != STENCIL_F32 && dtype != STENCIL_BF16 && dtype != STENCIL_F16)
        return fail(STENCIL_E_INVALID, "unknown dtype");
    stencil_plan p = new (std::nothrow) stencil_plan_s();
    if (!p) return fail(STENCIL_E_NOMEM, "out of host memory");
    p->batch = true;
    p->kind = STENCIL_WAVE2;
    p->ndim = 3;
    p->radius = radius;
    p->halo = halo;
    p->dtype = dtype;
    stencil_status st = set_coefs(p, 3, radius, coeffs);
    p->shots.resize(nshots);
    for (int s = 0; s < nshots && st == STENCIL_OK; s++) st = make_layout(3, shapes + 3 * s, halo, dtype, p->shots[s]);
    if (st != STENCIL_OK) {
        delete p;
        return st;
    }
    p->shot_src.resize(nshots);
    p->shot_rec.resize(nshots);
    p->shot_src_ext.resize(nshots);
    p->shot_amp_scaled.resize(nshots);
    // default: the 64x32 tile with 64-plane chunks
    p->variant = 1 + 2 * kNumTileCfgs + 0;
    *out = p;
    return STENCIL_OK;
}

stencil_status stencil_batch_layout(stencil_plan p, int shot, int64_t* extents, int64_t* strides, int64_t* offset,
                                    int64_t* bytes) {
    ST_TRY(check_plan(p, true));
    if (shot < 0 || shot >= (int)p->shots.size()) return fail(STENCIL_E_INVALID, "shot index out of range");
    return layout_out(p->shots[shot], extents, strides, offset, bytes);
}

// Block map of a batched launch: (shot, block within the shot) per
// workgroup, or shot -1 for a padding workgroup that exits at once.  The
// hardware hands workgroup b to XCD b % 8 and each XCD runs its workgroups in
// order, so the map is laid out per XCD: every (shot, z-chunk) group of tiles
// (neighbours that share halo rows, kept on one XCD for its L2) goes to the
// XCD with the least work so far, largest groups first, and each XCD's list
// is padded to the longest.  Work of a group = tiles x (chunk planes + 2r).
static stencil_status build_block_map_impl(const std::vector<ZView>& views, const std::vector<int>& nz, int radius,
                                           DevTable& table, int& nblocks, std::vector<int>* host_map = nullptr) {
    constexpr int kXcds = 8;
    struct Group {
        int shot, chunk, tiles;
        int64_t work;
    };
    std::vector<Group> groups;
    for (size_t sh = 0; sh < views.size(); sh++) {
        const ZView& v = views[sh];
        const int tiles = v.ntx * v.nty;
        for (int c = 0; c < v.nzc; c++) {
            const int len = std::min(v.zc, nz[sh] - c * v.zc);
            groups.push_back({(int)sh, c, tiles, (int64_t)tiles * (len + 2 * radius)});
        }
    }
    std::stable_sort(groups.begin(), groups.end(), [](const Group& a, const Group& b) { return a.work > b.work; });
    std::vector<std::vector<int>> lists(kXcds);
    std::vector<int64_t> load(kXcds, 0);
    for (const Group& g : groups) {
        const int x = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        load[x] += g.work;
        const int ntxy = g.tiles;
        for (int t = 0; t < ntxy; t++) {
            lists[x].push_back(g.shot);
            lists[x].push_back(g.chunk * ntxy + t);
        }
    }
    size_t len = 0;
    for (const auto& l : lists) len = std::max(len, l.size() / 2);
    if (len * kXcds > (size_t(1) << 30)) return fail(STENCIL_E_INVALID, "batch too large");
    nblocks = (int)(len * kXcds);
    std::vector<int> map(2 * std::max<size_t>(1, len * kXcds), -1);
    for (int x = 0; x < kXcds; x++)
        for (size_t i = 0; i < lists[x].size() / 2; i++) {
            const size_t b = i * kXcds + x;
            map[2 * b] = lists[x][2 * i];
            map[2 * b + 1] = lists[x][2 * i + 1];
        }
    if (host_map) *host_map = map;
    return table.upload(map.data(), sizeof(int) * map.size());
}

// The persistent batched sweep's queues: queue x holds the map's entries of
// XCD x (map index b with b % 8 == x, the pads dropped) in map order.
// list: (shot, block) pairs, qoff: 9 offsets.
static stencil_status build_persistent_queues(const std::vector<int>& map, DevTable& list, DevTable& qoff) {
    constexpr int kXcds = 8;
    std::vector<int> l, o(kXcds + 1, 0);
    for (int x = 0; x < kXcds; x++) {
        for (size_t b = x; 2 * b < map.size(); b += kXcds) {
            if (map[2 * b] < 0) continue;
            l.push_back(map[2 * b]);
            l.push_back(map[2 * b + 1]);
        }
        o[x + 1] = (int)(l.size() / 2);
    }
    if (l.empty()) l.assign(2, 0);
    ST_TRY(list.upload(l.data(), sizeof(int) * l.size()));
    return qoff.upload(o.data(), sizeof(int) * o.size());
}

static stencil_status batch_prepare(stencil_plan p, void** fields, int64_t nsteps, const stencil_source* src,
                                    const stencil_receivers* rec, const Variant& var, std::vector<ZView>& views) {
    const int ns = (int)p->shots.size();
    views.assign(ns, ZView{});
    p->bstart.assign(ns + 1, 0);
    const std::vector<int> zcs = batch_chunks(p->shots, var.zc);
    for (int s = 0; s < ns; s++) {
        const Layout& L = p->shots[s];
        ZView& v = views[s];
        v.u = fields[3 * s];
        v.prev = fields[3 * s + 1];
        v.out = fields[3 * s + 1];
        v.beta = fields[3 * s + 2];
        v.g = L.g;
        Variant vs = var;
        vs.zc = zcs[s];
        set_tiling(v, L, vs);
        const stencil_source* ss = src ? &src[s] : nullptr;
        const stencil_receivers* rr = rec ? &rec[s] : nullptr;
        ST_TRY(build_points(L, ss ? ss->n : 0, ss ? ss->pos : nullptr, var.cfg, p->shot_src[s]));
        if (var.tb) ST_TRY(build_points(L, ss ? ss->n : 0, ss ? ss->pos : nullptr, var.cfg, p->shot_src_ext[s], 4));
        ST_TRY(build_points(L, rr ? rr->n : 0, rr ? rr->pos : nullptr, -1, p->shot_rec[s]));
        v.src = src_list(p->shot_src[s], ss ? ss->amp : nullptr, nullptr);
        v.rec = rec_list(p->shot_rec[s], rr ? rr->trace : nullptr);
        const int64_t nb = zmarch_blocks(v);
        if ((int64_t)p->bstart[s] + nb > (int64_t(1) << 30)) return fail(STENCIL_E_INVALID, "batch too large");
        p->bstart[s + 1] = p->bstart[s] + (int)nb;
    }
    (void)nsteps;
    ST_TRY(p->views.upload(views.data(), sizeof(ZView) * views.size()));
    {
        std::vector<int> nz(ns);
        for (int s = 0; s < ns; s++) nz[s] = p->shots[s].g.n[0];
        ST_TRY(build_block_map_impl(views, nz, p->radius, p->block_map, p->nblocks, &p->hmap));
    }
    if (var.tb) {
        // pass k reads pair k & 1 (newest, previous) and writes the other pair
        // (u^{n+2} into its first buffer, u^{n+1} into its second)
        std::vector<TBView> tv[2];
        char* wsp = (char*)p->ws;
        for (int s = 0; s < ns; s++) {
            const Layout& L = p->shots[s];
            const int64_t fb = round_up(L.bytes, 256);
            void* pr[2][2] = {{fields[3 * s], fields[3 * s + 1]}, {wsp, wsp + fb}};
            wsp += 2 * fb;
            for (int par = 0; par < 2; par++) {
                TBView t{};
                t.u = pr[par][0];
                t.prev = pr[par][1];
                t.beta = fields[3 * s + 2];
                t.out2 = pr[1 - par][0];
                t.out1 = pr[1 - par][1];
                t.g = L.g;
                t.ntx = views[s].ntx;
                t.nty = views[s].nty;
                t.zc = views[s].zc;
                t.nzc = views[s].nzc;
                t.src_t = views[s].src;
                t.src_e = src_list(p->shot_src_ext[s], views[s].src.amp, nullptr);
                t.rec = views[s].rec;
                t.range = (uint32_t)L.bytes;
                tv[par].push_back(t);
            }
        }
        for (int par = 0; par < 2; par++) ST_TRY(p->tbviews[par].upload(tv[par].data(), sizeof(TBView) * tv[par].size()));
    }
    return STENCIL_OK;
}

// Polls a waiting workgroup makes at a persistent launch's grid barrier
// before it gives up: 2^20 polls, each a device-coherent load and a short
// sleep (about a microsecond or more), so about a second, against a few
// milliseconds for one step of the largest batch that fits in HBM.
// STENCIL_BARRIER_POLLS overrides it (the tests force the error path with 0).
static int barrier_polls() {
    const char* e = std::getenv("STENCIL_BARRIER_POLLS");
    if (e && *e) {
        const long v = std::strtol(e, nullptr, 10);
        if (v >= 0 && v <= (1L << 30)) return (int)v;
    }
    return 1 << 20;
}

// The persistent variants' grid: every map entry's workgroup if the GPU holds
// them all at once, else as many as it holds, rounded down to a multiple of
// 8 (each then takes several entries per step); the barrier words and the
// pinned flag on first use.
static stencil_status prepare_persistent(stencil_plan p, const Variant& var, const std::vector<int>& map, int nmap,
                                         DevTable& list, DevTable& qoff) {
    int per_cu = 0, dev = 0, cus = 0;
    HIP_TRY(zmarch_batch_persistent_per_cu(p->radius, p->dtype, var.cfg, &per_cu));
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int64_t resident = (int64_t)per_cu * cus / 8 * 8;
    if (resident < 8) return fail(STENCIL_E_DEVICE, "the persistent batched sweep does not fit 8 workgroups on the GPU");
    p->pgrid = (int)std::min<int64_t>(nmap, resident);
    ST_TRY(build_persistent_queues(map, list, qoff));
    ST_TRY(p->bsync.ensure(kPersistentWords * sizeof(unsigned long long)));
    if (!p->bsync_host) HIP_TRY(hipHostMalloc((void**)&p->bsync_host, 2 * sizeof(unsigned long long), hipHostMallocDefault));
    return STENCIL_OK;
}

// After a persistent launch: wait for it and report a barrier that gave up.
static stencil_status check_persistent(stencil_plan p, hipStream_t s) {
    HIP_TRY(hipMemcpyAsync(p->bsync_host, p->bsync.p, 2 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (p->bsync_host[1] != 0)
        return fail(STENCIL_E_DEVICE, "persistent batched sweep: a grid barrier gave up waiting (the grid of " +
                                          std::to_string(p->pgrid) +
                                          " workgroups was not resident at once); the fields are not valid");
    return STENCIL_OK;
}

static stencil_status enqueue_batch(stencil_plan p, const std::vector<ZView>& views, int64_t nsteps, const Variant& var,
                                    bool any_rec, hipStream_t s) {
    const int ns = (int)p->shots.size();
    const int nblocks = p->nblocks;
    int64_t t0 = 0;
    if (var.persistent) {
        // every step in one launch (the barrier words start at zero: a fill
        // kernel, which a graph replays correctly)
        HIP_TRY(launch_zero(p->bsync.p, kPersistentWords * sizeof(unsigned long long), s));
        HIP_TRY(launch_zmarch_batch_persistent(p->radius, p->dtype, var.cfg, (const ZView*)p->views.buf.p,
                                               (const int*)p->plist.buf.p, (const int*)p->poff.buf.p, p->pgrid, p->w,
                                               0, (int)nsteps, any_rec ? 1 : 0, 1, (unsigned long long*)p->bsync.p,
                                               barrier_polls(), s));
        t0 = nsteps;
    }
    if (var.tb) {
        // an even number of two-step passes (as in a single-plan run), then
        // plain batched sweeps on the 64 x 32 tiles for the rest
        int64_t passes = nsteps / 2;
        if (passes & 1) passes--;
        for (int64_t k = 0; k < passes; k++) {
            const int tu = (any_rec && k >= 1) ? (int)(2 * k - 1) : -1;
            const int tp = (any_rec && k >= 1) ? (int)(2 * k - 2) : -1;
            HIP_TRY(tb2_batch(p->dtype, (const TBView*)p->tbviews[k & 1].buf.p, (const int*)p->block_map.buf.p, nblocks,
                              p->w, (int)(2 * k), tu, tp, s));
        }
        if (any_rec && passes > 0) {
            for (int sh = 0; sh < ns; sh++) {
                const ZView& v = views[sh];
                if (v.rec.n > 0) HIP_TRY(launch_record(p->dtype, v.prev, v.g, v.rec, (int)(2 * passes - 2), s));
            }
        }
        t0 = 2 * passes;
    }
    for (int64_t t = t0; t < nsteps; t++) {
        const int trow = (any_rec && t >= 1) ? (int)(t - 1) : -1;
        HIP_TRY(launch_zmarch_batch(p->radius, p->dtype, var.cfg, (const ZView*)p->views.buf.p,
                                    (const int*)p->block_map.buf.p, nblocks, p->w, (int)(t & 1), (int)t, trow, s));
    }
    if (any_rec && nsteps > 0) {
        for (int sh = 0; sh < ns; sh++) {
            const ZView& v = views[sh];
            if (v.rec.n == 0) continue;
            const void* newest = (nsteps & 1) ? v.prev : v.u;
            HIP_TRY(launch_record(p->dtype, newest, v.g, v.rec, (int)(nsteps - 1), s));
        }
    }
    return STENCIL_OK;
}

// The concurrent batch variant's per-shot plans (created on first use with
// their default variant) and branch streams (default priority) and events.
static stencil_status ensure_shot_plans(stencil_plan p) {
    if (p->shot_plans.size() == p->shots.size()) return STENCIL_OK;
    for (size_t sh = p->shot_plans.size(); sh < p->shots.size(); sh++) {
        const Grid3& g = p->shots[sh].g;
        const int64_t shape[3] = {g.n[0], g.n[1], g.n[2]};
        stencil_plan q = nullptr;
        ST_TRY(stencil_create(&q, STENCIL_WAVE2, 3, shape, p->radius, p->coeffs, p->halo, (stencil_dtype)p->dtype,
                              STENCIL_BC_DIRICHLET0));
        p->shot_plans.push_back(q);
    }
    return STENCIL_OK;
}

static stencil_status ensure_branches(stencil_plan p) {
    for (hipStream_t& b : p->branch)
        if (!b) HIP_TRY(hipStreamCreateWithFlags(&b, hipStreamNonBlocking));
    if (!p->fork_ev) HIP_TRY(hipEventCreateWithFlags(&p->fork_ev, hipEventDisableTiming));
    for (hipEvent_t& e : p->join_ev)
        if (!e) HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    return STENCIL_OK;
}

// Shots with at least this many points fill the GPU on their own (about
// 32K points per compute unit).
constexpr int64_t kLargeShotPoints = int64_t(1) << 23;

// Shots to branches.  The large shots run one after another on the first
// branch, largest first, as the sequential runs do; the others are dealt
// largest first to the least-loaded of the remaining branches, where their
// launches take the compute units a large shot's launch leaves idle.  (Large
// shots spread over several branches compete for the caches and run slower
// than one after another.)  Without large shots every branch takes small ones.
static std::vector<std::vector<int>> branch_lists(const stencil_plan_s* p) {
    const int ns = (int)p->shots.size();
    std::vector<int> order(ns);
    for (int i = 0; i < ns; i++) order[i] = i;
    auto work = [&](int i) {
        const Grid3& g = p->shots[i].g;
        return (int64_t)g.n[0] * g.n[1] * g.n[2];
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work(a) > work(b); });
    std::vector<std::vector<int>> lists(kBranches);
    const int first_small = ns > 0 && work(order[0]) >= kLargeShotPoints ? 1 : 0;
    std::vector<int64_t> load(kBranches, 0);
    for (int i : order) {
        if (work(i) >= kLargeShotPoints) {
            lists[0].push_back(i);
            continue;
        }
        const int b = (int)(std::min_element(load.begin() + first_small, load.end()) - load.begin());
        load[b] += work(i);
        lists[b].push_back(i);
    }
    return lists;
}

// fork from `main` to the branches, run `body(branch, shot)` for each shot of
// each branch, join back
static stencil_status fork_join(stencil_plan p, hipStream_t main, const std::vector<std::vector<int>>& lists,
                                const std::function<stencil_status(hipStream_t, int)>& body) {
    HIP_TRY(hipEventRecord(p->fork_ev, main));
    for (int b = 0; b < kBranches; b++) HIP_TRY(hipStreamWaitEvent(p->branch[b], p->fork_ev, 0));
    for (int b = 0; b < kBranches; b++)
        for (int sh : lists[b]) ST_TRY(body(p->branch[b], sh));
    for (int b = 0; b < kBranches; b++) {
        HIP_TRY(hipEventRecord(p->join_ev[b], p->branch[b]));
        HIP_TRY(hipStreamWaitEvent(main, p->join_ev[b], 0));
    }
    return STENCIL_OK;
}

// Every shot's whole run with its own plan (its tuned variant, tables and
// workspace slice), the shots spread over kBranches streams so that their
// kernels overlap where one alone leaves compute units idle.  Arguments are
// validated by the caller.
static stencil_status batch_run_concurrent(stencil_plan p, void** fields, int64_t nsteps, const stencil_source* src,
                                           const stencil_receivers* rec, hipStream_t s) {
    ST_TRY(ensure_shot_plans(p));
    ST_TRY(ensure_branches(p));
    const int ns = (int)p->shots.size();
    std::vector<stencil_source> scaled(ns);
    std::vector<RunLists> lists(ns);
    char* wsp = (char*)p->ws;
    for (int sh = 0; sh < ns; sh++) {
        stencil_plan q = p->shot_plans[sh];
        const size_t need = run_workspace_bytes(q);
        q->ws = need ? wsp : nullptr;
        q->ws_bytes = need;
        wsp += need;
        const stencil_source* ss = src ? &src[sh] : nullptr;
        const stencil_receivers* rr = rec ? &rec[sh] : nullptr;
        ST_TRY(prepare_points(q, ss, rr));
        const stencil_source* use = ss;
        ST_TRY(scaled_source(q->amp_scaled, ss, nsteps, scaled[sh], use, s));
        lists[sh] = plan_lists(q, use, rr);
    }
    const std::vector<std::vector<int>> bl = branch_lists(p);
    auto body = [&](hipStream_t bs, int sh) -> stencil_status {
        return enqueue_run(p->shot_plans[sh], fields[3 * sh], fields[3 * sh + 1], fields[3 * sh + 2], nsteps, lists[sh],
                           bs);
    };
    if (nsteps >= 2 && graphs_enabled()) {
        std::vector<int64_t> key = {nsteps, p->variant, -1};
        for (int sh = 0; sh < ns; sh++) {
            const stencil_plan_s* q = p->shot_plans[sh];
            const RunLists& L = lists[sh];
            for (const void* ptr : {(const void*)fields[3 * sh], (const void*)fields[3 * sh + 1],
                                    (const void*)fields[3 * sh + 2], (const void*)q->ws, (const void*)L.st.zyx4,
                                    (const void*)L.st.tile_begin, (const void*)L.st.off, (const void*)L.st.amp,
                                    (const void*)L.st.grp, (const void*)L.st.gbeg, (const void*)L.se.zyx4,
                                    (const void*)L.se.tile_begin, (const void*)L.rl.off, (const void*)L.rl.trace})
                key.push_back((int64_t)(uintptr_t)ptr);
            key.push_back(q->variant);
            key.push_back(L.st.n);
            key.push_back(L.st.ngrp);
            key.push_back(L.se.n);
            key.push_back(L.rl.n);
        }
        if (!p->gexec || key != p->gkey) {
            if (!p->cap) HIP_TRY(hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking));
            if (p->gexec) {
                HIP_TRY(hipStreamSynchronize(s));
                HIP_TRY(hipGraphExecDestroy(p->gexec));
                p->gexec = nullptr;
            }
            HIP_TRY(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
            stencil_status st = fork_join(p, p->cap, bl, body);
            hipGraph_t graph = nullptr;
            hipError_t e = hipStreamEndCapture(p->cap, &graph);
            if (st != STENCIL_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return st;
            }
            if (e != hipSuccess) return fail(STENCIL_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
            e = hipGraphInstantiate(&p->gexec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) {
                p->gexec = nullptr;
                return fail(STENCIL_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
            }
            p->gkey = key;
        }
        HIP_TRY(hipGraphLaunch(p->gexec, s));
    } else {
        ST_TRY(fork_join(p, s, bl, body));
    }
    if (nsteps & 1)
        for (int sh = 0; sh < ns; sh++) std::swap(fields[3 * sh], fields[3 * sh + 1]);
    return STENCIL_OK;
}

stencil_status stencil_batch_run(stencil_plan p, void** fields, int64_t nsteps, const stencil_source* src,
                                 const stencil_receivers* rec, void* stream) {
    ST_TRY(check_plan(p, true));
    if (!fields) return fail(STENCIL_E_INVALID, "fields is NULL");
    if (nsteps < 0 || nsteps > (int64_t(1) << 30)) return fail(STENCIL_E_INVALID, "bad nsteps");
    const int ns = (int)p->shots.size();
    bool any_rec = false;
    for (int s = 0; s < ns; s++) {
        for (int k = 0; k < 3; k++) ST_TRY(check_ptr(fields[3 * s + k], "shot field"));
        if (fields[3 * s] == fields[3 * s + 1] || fields[3 * s + 2] == fields[3 * s] || fields[3 * s + 2] == fields[3 * s + 1])
            return fail(STENCIL_E_INVALID, "a shot's fields must be distinct");
        if (src && src[s].n > 0) {
            ST_TRY(check_positions(p->shots[s], src[s].n, src[s].pos, "sources"));
            if (!src[s].amp) return fail(STENCIL_E_INVALID, "source amplitudes are NULL");
            ST_TRY(check_source_scale(&src[s]));
        }
        if (rec && rec[s].n > 0) {
            ST_TRY(check_positions(p->shots[s], rec[s].n, rec[s].pos, "receivers"));
            if (!rec[s].trace) return fail(STENCIL_E_INVALID, "receiver trace is NULL");
            any_rec = true;
        }
    }
    ST_TRY(check_workspace(p));
    hipStream_t s = (hipStream_t)stream;
    if (batch_concurrent(p, p->variant)) return batch_run_concurrent(p, fields, nsteps, src, rec, s);
    const Variant var = plan_variant(p, p->variant);
    // shots whose sources carry per-point scales use their formed amounts
    std::vector<stencil_source> srcs;
    if (src) {
        srcs.assign(src, src + ns);
        for (int sh = 0; sh < ns; sh++) {
            stencil_source tmp{};
            const stencil_source* use = nullptr;
            ST_TRY(scaled_source(p->shot_amp_scaled[sh], &src[sh], nsteps, tmp, use, s));
            srcs[sh] = *use;
        }
    }
    std::vector<ZView> views;
    ST_TRY(batch_prepare(p, fields, nsteps, src ? srcs.data() : nullptr, rec, var, views));
    if (var.persistent) {
        if (nsteps > INT_MAX) return fail(STENCIL_E_INVALID, "the persistent batched sweep takes at most 2^31 - 1 steps");
        ST_TRY(prepare_persistent(p, var, p->hmap, p->nblocks, p->plist, p->poff));
    }
    if (nsteps >= 2 && graphs_enabled()) {
        std::vector<int64_t> key = {nsteps, p->variant, (int64_t)(uintptr_t)p->views.buf.p, any_rec,
                                    (int64_t)(uintptr_t)p->block_map.buf.p, (int64_t)(uintptr_t)p->ws, p->pgrid,
                                    (int64_t)(uintptr_t)p->bsync.p, barrier_polls(), (int64_t)(uintptr_t)p->plist.buf.p,
                                    (int64_t)(uintptr_t)p->poff.buf.p,
                                    (int64_t)(uintptr_t)p->tbviews[0].buf.p, (int64_t)(uintptr_t)p->tbviews[1].buf.p};
        for (const ZView& v : views) {
            key.push_back((int64_t)(uintptr_t)v.u);
            key.push_back((int64_t)(uintptr_t)v.prev);
            key.push_back((int64_t)(uintptr_t)v.beta);
            key.push_back((int64_t)(uintptr_t)v.src.amp);
            key.push_back((int64_t)(uintptr_t)v.rec.trace);
            key.push_back(v.src.n);
            key.push_back(v.rec.n);
            key.push_back((int64_t)(uintptr_t)v.src.zyx4);
            key.push_back((int64_t)(uintptr_t)v.src.tile_begin);
            key.push_back((int64_t)(uintptr_t)v.rec.off);
        }
        if (!p->gexec || key != p->gkey) {
            if (!p->cap) HIP_TRY(hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking));
            if (p->gexec) {
                HIP_TRY(hipStreamSynchronize(s));
                HIP_TRY(hipGraphExecDestroy(p->gexec));
                p->gexec = nullptr;
            }
            HIP_TRY(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
            stencil_status st = enqueue_batch(p, views, nsteps, var, any_rec, p->cap);
            hipGraph_t graph = nullptr;
            hipError_t e = hipStreamEndCapture(p->cap, &graph);
            if (st != STENCIL_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return st;
            }
            if (e != hipSuccess) return fail(STENCIL_E_DEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
            e = hipGraphInstantiate(&p->gexec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) {
                p->gexec = nullptr;
                return fail(STENCIL_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
            }
            p->gkey = key;
        }
        HIP_TRY(hipGraphLaunch(p->gexec, s));
    } else {
        ST_TRY(enqueue_batch(p, views, nsteps, var, any_rec, s));
    }
    if (nsteps & 1)
        for (int sh = 0; sh < ns; sh++) std::swap(fields[3 * sh], fields[3 * sh + 1]);
    if (var.persistent && nsteps > 0) ST_TRY(check_persistent(p, s));
    return STENCIL_OK;
}

// ---------------------------------------------------------------- adjoint
struct AdjLayout {
    int64_t fbytes = 0;  // one field, rounded up to 256 bytes
    int64_t nseg = 0;
    int64_t k = 0;
    // field slot indices
    int64_t ckpt0 = 0;     // 2*nseg slots
    int64_t seg0 = 0;      // k slots of second differences
    int64_t f0 = 0, f1 = 0, l0 = 0, l1 = 0, g = 0;
    int64_t slots = 0;
};

static stencil_status adj_layout(stencil_plan p, int64_t nsteps, int64_t k, AdjLayout& A) {
    if (p->kind != STENCIL_WAVE2 || p->ndim != 3) return fail(STENCIL_E_STATE, "adjoint needs a 3D wave plan");
    if (p->dtype != STENCIL_F32) return fail(STENCIL_E_STATE, "adjoint needs FP32 storage");
    if (p->bc != STENCIL_BC_DIRICHLET0) return fail(STENCIL_E_STATE, "adjoint needs the Dirichlet-zero boundary");
    if (nsteps < 1 || nsteps > (int64_t(1) << 24)) return fail(STENCIL_E_INVALID, "nsteps must be >= 1");
    if (k < 1 || k > nsteps) return fail(STENCIL_E_INVALID, "checkpoint_every must be in [1, nsteps]");
    A.fbytes = round_up(p->L.bytes, 256);
    A.k = k;
    A.nseg = (nsteps + k - 1) / k;
    A.ckpt0 = 0;
    A.seg0 = 2 * A.nseg;
    A.f0 = A.seg0 + k;
    A.f1 = A.f0 + 1;
    A.l0 = A.f1 + 1;
    A.l1 = A.l0 + 1;
    A.g = A.l1 + 1;
    A.slots = A.g + 1;
    return STENCIL_OK;
}

static char* slot(void* ws, const AdjLayout& A, int64_t i) { return (char*)ws + i * A.fbytes; }

stencil_status stencil_adjoint_workspace(stencil_plan p, int64_t nsteps, int64_t k, size_t* bytes) {
    ST_TRY(check_sweep_plan(p));
    if (p->damped) return fail(STENCIL_E_UNSUPPORTED, "the adjoint path has no absorbing layer");
    if (!bytes) return fail(STENCIL_E_INVALID, "bytes is NULL");
    AdjLayout A;
    ST_TRY(adj_layout(p, nsteps, k, A));
    *bytes = (size_t)(A.slots * A.fbytes);
    return STENCIL_OK;
}

static Variant adjoint_variant(stencil_plan p) {
    Variant var = variant_of(p->variant);
    if (!var.zmarch) var = variant_of(default_variant(p->L));
    return var;
}

// Forward run storing (u^c, u^{c-1}) every k steps (arguments validated)
// The buffers of one segment's levels: u^{t0} and u^{t0-1} in (cur, prv),
// then u^{t0+i} alternating between two other buffers, odd i in y and even
// i in x.  Step j reads levels j and j - 1 and writes level j + 1 (from the
// third step on, in place over level j - 1, as the plain run does).
struct SegLevels {
    void* cur;
    void* prv;
    void* x;
    void* y;
    void* at(int64_t i) const { return i < 0 ? prv : i == 0 ? cur : (i & 1) ? y : x; }
};

static stencil_status forward_ckpt_impl(stencil_plan p, void** fields, int64_t nsteps, int64_t k,
                                        const stencil_source* src, const stencil_receivers* rec, void* ws,
                                        const AdjLayout& A, hipStream_t s) {
    // until this forward completes, no workspace holds a last segment's
    // second differences this plan can vouch for
    p->last_seg_ws = nullptr;
    const Variant var = adjoint_variant(p);
    ST_TRY(build_points(p->L, src ? src->n : 0, src ? src->pos : nullptr, var.cfg, p->src));
    ST_TRY(build_points(p->L, rec ? rec->n : 0, rec ? rec->pos : nullptr, -1, p->rec));
    const Layout& L = p->L;
    void* a = fields[0];
    void* b = fields[1];
    const SrcList sl = src_list(p->src, src ? src->amp : nullptr, nullptr);
    const RecList rl = rec_list(p->rec, rec ? rec->trace : nullptr);
    // Checkpoint c is the slot pair (u^{ck}, u^{ck-1}).  Pair 0 is a copy of
    // the initial state; segment c then sweeps from pair c into pair c + 1,
    // so the sweeps write the later checkpoints themselves, and the last
    // segment sweeps into the caller's fields (u^N into a for even N, into b
    // for odd N, as the plain run leaves them).
    HIP_TRY(hipMemcpyAsync(slot(ws, A, A.ckpt0), a, L.bytes, hipMemcpyDeviceToDevice, s));
    HIP_TRY(hipMemcpyAsync(slot(ws, A, A.ckpt0 + 1), b, L.bytes, hipMemcpyDeviceToDevice, s));
    for (int64_t c0 = 2; c0 < 2 * A.nseg; c0 += 65535)
        HIP_TRY(launch_zero_frame(slot(ws, A, A.ckpt0 + c0), (int)std::min<int64_t>(65535, 2 * A.nseg - c0), A.fbytes,
                                  L.g, L.halo, L.elems, s));
    for (int64_t c = 0; c < A.nseg; c++) {
        const int64_t t0 = c * k, len = std::min(t0 + k, nsteps) - t0;
        const bool last = c + 1 == A.nseg;
        void* const cur = slot(ws, A, A.ckpt0 + 2 * c);
        void* const prv = slot(ws, A, A.ckpt0 + 2 * c + 1);
        void* const tu = last ? ((nsteps & 1) ? b : a) : slot(ws, A, A.ckpt0 + 2 * c + 2);
        void* const tp = last ? ((nsteps & 1) ? a : b) : slot(ws, A, A.ckpt0 + 2 * c + 3);
        const SegLevels lv{cur, prv, (len & 1) ? tp : tu, (len & 1) ? tu : tp};
        // the last segment also writes its second differences, which the
        // adjoint then takes without recomputing that segment
        for (int64_t j = 0; j < len; j++) {
            const int64_t t = t0 + j;
            ZView v{};
            v.u = lv.at(j);
            v.prev = lv.at(j - 1);
            v.out = lv.at(j + 1);
            v.beta = fields[2];
            v.g = L.g;
            if (last) v.dfield = (float*)slot(ws, A, A.seg0 + j);
            set_tiling(v, L, var);
            v.src = sl;
            v.rec = rl;
            HIP_TRY(launch_zmarch(last ? MODE_WAVE_D : MODE_WAVE, p->radius, p->dtype, var.cfg, v, p->w, 0, (int)t,
                                  (rl.n > 0 && t >= 1) ? (int)(t - 1) : -1, s));
        }
        // one-step segment: u^{t0} is still only in pair c
        if (len == 1) HIP_TRY(hipMemcpyAsync(tp, cur, L.bytes, hipMemcpyDeviceToDevice, s));
    }
    if (rl.n > 0) HIP_TRY(launch_record(p->dtype, (nsteps & 1) ? b : a, L.g, rl, (int)(nsteps - 1), s));
    if (nsteps & 1) std::swap(fields[0], fields[1]);
    p->last_seg_ws = ws;
    p->last_seg_nsteps = nsteps;
    p->last_seg_k = k;
    return STENCIL_OK;
}

// Adjoint sweep with fused imaging over the checkpointed segments, last to
// first (arguments validated); grad += -(1/dt^2) sum_n lam^n (u^{n+1} - 2u^n + u^{n-1})
static stencil_status adjoint_impl(stencil_plan p, const void* beta, int64_t nsteps, int64_t k,
                                   const stencil_source* src, int64_t nrec, const int64_t* rec_pos,
                                   const double* resid, const double* rec_scale, double dt, double* grad, void* ws,
                                   const AdjLayout& A, hipStream_t s) {
    const Variant var = adjoint_variant(p);
    ST_TRY(build_points(p->L, src ? src->n : 0, src ? src->pos : nullptr, var.cfg, p->src));
    ST_TRY(build_points(p->L, nrec, nrec ? rec_pos : nullptr, var.cfg, p->adjrec));
    const Layout& L = p->L;
    const SrcList fsrc = src_list(p->src, src ? src->amp : nullptr, nullptr);
    const SrcList asrc = src_list(p->adjrec, resid, rec_scale);
    const double grad_scale = -1.0 / (dt * dt);
    void* F0 = slot(ws, A, A.f0);
    void* F1 = slot(ws, A, A.f1);
    void* L0 = slot(ws, A, A.l0);
    void* L1 = slot(ws, A, A.l1);
    float* G = (float*)slot(ws, A, A.g);
    HIP_TRY(launch_zero(L0, L.bytes, s));
    HIP_TRY(launch_zero(L1, L.bytes, s));
    HIP_TRY(launch_zero_frame(F0, 2, A.fbytes, L.g, L.halo, L.elems, s));   // F0 and F1 (adjacent slots)
    const bool have_last = p->last_seg_ws == ws && p->last_seg_nsteps == nsteps && p->last_seg_k == k;
    int64_t j = 0;  // adjoint steps taken (parity of the lambda buffers)
    for (int64_t sg = A.nseg - 1; sg >= 0; sg--) {
        const int64_t c = sg * k, ce = std::min(c + k, nsteps);
        // the last segment's second differences may still be there from
        // the checkpointed forward
        if (sg != A.nseg - 1 || !have_last) {
            p->last_seg_ws = nullptr;
            // the recompute reads the checkpoint pair in place (it stays intact
            // for a later call) and sweeps on in F0 / F1
            const SegLevels lv{slot(ws, A, A.ckpt0 + 2 * sg), slot(ws, A, A.ckpt0 + 2 * sg + 1), F0, F1};
            for (int64_t t = c; t < ce; t++) {
                ZView v{};
                v.u = lv.at(t - c);
                v.prev = lv.at(t - c - 1);
                v.out = lv.at(t - c + 1);
                v.beta = beta;
                v.g = L.g;
                v.dfield = (float*)slot(ws, A, A.seg0 + (t - c));
                set_tiling(v, L, var);
                v.src = fsrc;
                HIP_TRY(launch_zmarch(MODE_WAVE_D, p->radius, p->dtype, var.cfg, v, p->w, 0, (int)t, -1, s));
            }
        }
        // Adjoint step kk produces lambda at level kk-1 and images it with
        // the second difference of that level.  Steps go in pairs: a plain
        // step (no imaging), then a step that images both its input level
        // and its output, so the partial G is read and written once per two
        // steps with the same roundings in the same order.  An odd remainder
        // takes the one-level imaging step.
        bool fresh = true;   // the segment's first imaging step starts the partial at zero
        for (int64_t kk = ce; kk > c;) {
            ZView v{};
            v.u = L0;
            v.prev = L1;
            v.out = L1;
            v.beta = beta;
            v.g = L.g;
            set_tiling(v, L, var);
            v.src = asrc;
            if (kk - 1 > c) {
                HIP_TRY(launch_zmarch(MODE_WAVE, p->radius, p->dtype, var.cfg, v, p->w, (int)(j & 1), (int)(kk - 1), -1, s));
                j++;
                v.dfield2 = (const float*)slot(ws, A, A.seg0 + (kk - 1 - c));
                v.dfield = (float*)slot(ws, A, A.seg0 + (kk - 2 - c));
                v.gfield = G;
                v.gfresh = fresh;
                fresh = false;
                HIP_TRY(launch_zmarch(MODE_WAVE_ADJ2, p->radius, p->dtype, var.cfg, v, p->w, (int)(j & 1), (int)(kk - 2), -1,
                                      s));
                j++;
                kk -= 2;
            } else {
                v.dfield = (float*)slot(ws, A, A.seg0 + (kk - 1 - c));
                v.gfield = G;
                v.gfresh = fresh;
                fresh = false;
                HIP_TRY(launch_zmarch(MODE_WAVE_ADJ, p->radius, p->dtype, var.cfg, v, p->w, (int)(j & 1), (int)(kk - 1), -1, s));
                j++;
                kk -= 1;
            }
        }
        HIP_TRY(launch_flush(G, grad, L.g, grad_scale, s));
    }
    return STENCIL_OK;
}

static stencil_status check_dt_h(double dt, double h) {
    if (!(dt > 0) || !(h > 0) || !std::isfinite(dt) || !std::isfinite(h))
        return fail(STENCIL_E_INVALID, "dt and h must be positive and finite");
    return STENCIL_OK;
}

stencil_status stencil_forward_ckpt(stencil_plan p, void** fields, int64_t nsteps, int64_t k, const stencil_source* src,
                                    const stencil_receivers* rec, void* ws, size_t ws_bytes, void* stream) {
    ST_TRY(check_sweep_plan(p));
    if (p->damped) return fail(STENCIL_E_UNSUPPORTED, "the adjoint path has no absorbing layer");
    AdjLayout A;
    ST_TRY(adj_layout(p, nsteps, k, A));
    ST_TRY(run_args(p, fields, nsteps, src, rec));
    ST_TRY(check_source_scale(src));
    ST_TRY(check_ptr(ws, "workspace"));
    if (ws_bytes < (size_t)(A.slots * A.fbytes)) return fail(STENCIL_E_INVALID, "workspace too small");
    hipStream_t s = (hipStream_t)stream;
    stencil_source scaled{};
    const stencil_source* use = src;
    ST_TRY(scaled_source(p->amp_scaled, src, nsteps, scaled, use, s));
    return forward_ckpt_impl(p, fields, nsteps, k, use, rec, ws, A, s);
}

stencil_status stencil_adjoint(stencil_plan p, const void* beta, int64_t nsteps, int64_t k, const stencil_source* src,
                               const stencil_receivers* rec, const double* resid, const double* rec_scale, double dt,
                               double* grad, void* ws, size_t ws_bytes, void* stream) {
    ST_TRY(check_sweep_plan(p));
    if (p->damped) return fail(STENCIL_E_UNSUPPORTED, "the adjoint path has no absorbing layer");
    AdjLayout A;
    ST_TRY(adj_layout(p, nsteps, k, A));
    ST_TRY(check_ptr(beta, "beta"));
    ST_TRY(check_ptr(ws, "workspace"));
    if (!grad) return fail(STENCIL_E_INVALID, "grad is NULL");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(STENCIL_E_INVALID, "dt must be positive and finite");
    if (ws_bytes < (size_t)(A.slots * A.fbytes)) return fail(STENCIL_E_INVALID, "workspace too small");
    if (src && src->n > 0) {
        ST_TRY(check_positions(p->L, src->n, src->pos, "sources"));
        if (!src->amp) return fail(STENCIL_E_INVALID, "source amplitudes are NULL");
        ST_TRY(check_source_scale(src));
    }
    const int64_t nrec = rec ? rec->n : 0;
    if (nrec > 0) {
        ST_TRY(check_positions(p->L, rec->n, rec->pos, "receivers"));
        if (!resid || !rec_scale) return fail(STENCIL_E_INVALID, "resid and rec_scale are required with receivers");
    }
    hipStream_t s = (hipStream_t)stream;
    stencil_source scaled{};
    const stencil_source* use = src;
    ST_TRY(scaled_source(p->amp_scaled, src, nsteps, scaled, use, s));
    return adjoint_impl(p, beta, nsteps, k, use, nrec, nrec ? rec->pos : nullptr, resid, rec_scale, dt, grad, ws, A, s);
}

stencil_status stencil_wave_beta(stencil_plan p, const double* m, double dt, double h, void* beta, void* stream) {
    ST_TRY(check_sweep_plan(p));
    if (p->kind != STENCIL_WAVE2) return fail(STENCIL_E_STATE, "not a wave plan");
    if (!m) return fail(STENCIL_E_INVALID, "m is NULL");
    ST_TRY(check_ptr(beta, "beta"));
    ST_TRY(check_dt_h(dt, h));
    HIP_TRY(launch_beta(p->dtype, m, beta, p->L.g, dt * dt / (h * h), (hipStream_t)stream));
    return STENCIL_OK;
}

// dense offsets of interior positions in an interior-shaped array
static std::vector<int64_t> dense_offsets(const stencil_plan_s* p, int64_t n, const int64_t* pos) {
    const Grid3& g = p->L.g;
    std::vector<int64_t> off((size_t)std::max<int64_t>(n, 1), 0);
    for (int64_t i = 0; i < n; i++) {
        int zyx[3];
        zyx_of(p->L, pos + 3 * i, zyx);
        off[(size_t)i] = ((int64_t)zyx[0] * g.n[1] + zyx[1]) * g.n[2] + zyx[2];
    }
    return off;
}

// the offsets in one of the plan's two point-scale tables: the one that
// already holds them, else the one used less recently
static stencil_status point_offsets(stencil_plan p, int64_t n, const int64_t* pos, const int64_t*& dev) {
    const std::vector<int64_t> off = dense_offsets(p, n, pos);
    const size_t bytes = sizeof(int64_t) * off.size();
    for (int i = 0; i < 2; i++) {
        DevTable& t = p->ps_off[i];
        if (t.valid && t.host.size() == bytes && std::memcmp(t.host.data(), off.data(), bytes) == 0) {
            dev = (const int64_t*)t.buf.p;
            p->ps_next = 1 - i;
            return STENCIL_OK;
        }
    }
    DevTable& t = p->ps_off[p->ps_next];
    p->ps_next ^= 1;
    ST_TRY(t.upload(off.data(), bytes));
    dev = (const int64_t*)t.buf.p;
    return STENCIL_OK;
}

stencil_status stencil_wave_point_scale(stencil_plan p, const double* m, double dt, int64_t n, const int64_t* pos,
                                        double* out, void* stream) {
    ST_TRY(check_sweep_plan(p));
    if (p->kind != STENCIL_WAVE2) return fail(STENCIL_E_STATE, "not a wave plan");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(STENCIL_E_INVALID, "dt must be positive and finite");
    if (n < 0) return fail(STENCIL_E_INVALID, "n must be >= 0");
    if (n == 0) return STENCIL_OK;
    if (!m || !out) return fail(STENCIL_E_INVALID, "m and out are required");
    ST_TRY(check_positions(p->L, n, pos, "positions"));
    const int64_t* off = nullptr;
    ST_TRY(point_offsets(p, n, pos, off));
    HIP_TRY(launch_point_scale(m, off, n, dt * dt, out, (hipStream_t)stream));
    return STENCIL_OK;
}

stencil_status stencil_gradient(stencil_plan p, void** fields, const double* m, double dt, double h, int64_t nsteps,
                                int64_t k, const stencil_source* src, const stencil_receivers* rec, const double* d_obs,
                                double* misfit, double* grad, void* ws, size_t ws_bytes, void* stream) {
    ST_TRY(check_sweep_plan(p));
    if (p->damped) return fail(STENCIL_E_UNSUPPORTED, "the adjoint path has no absorbing layer");
    AdjLayout A;
    ST_TRY(adj_layout(p, nsteps, k, A));
    ST_TRY(run_args(p, fields, nsteps, src, rec));
    ST_TRY(check_dt_h(dt, h));
    if (!m) return fail(STENCIL_E_INVALID, "m is NULL");
    if (src && src->n > 0 && src->scale)
        return fail(STENCIL_E_INVALID, "source scales come from m here; pass the wavelet with scale NULL");
    if (!rec || rec->n == 0) return fail(STENCIL_E_INVALID, "the misfit needs receivers");
    if (!d_obs || !misfit || !grad) return fail(STENCIL_E_INVALID, "d_obs, misfit and grad are required");
    ST_TRY(check_ptr(ws, "workspace"));
    if (ws_bytes < (size_t)(A.slots * A.fbytes)) return fail(STENCIL_E_INVALID, "workspace too small");
    const int64_t ns = src ? src->n : 0, nr = rec->n;
    if (nsteps * nr > (int64_t(1) << 31)) return fail(STENCIL_E_NOMEM, "trace too large");
    {
        const std::vector<int64_t> so = dense_offsets(p, ns, ns ? src->pos : nullptr);
        const std::vector<int64_t> ro = dense_offsets(p, nr, rec->pos);
        ST_TRY(p->gsrc_off.upload(so.data(), sizeof(int64_t) * so.size()));
        ST_TRY(p->grec_off.upload(ro.data(), sizeof(int64_t) * ro.size()));
    }
    const int64_t* soff = (const int64_t*)p->gsrc_off.buf.p;
    const int64_t* roff = (const int64_t*)p->grec_off.buf.p;
    ST_TRY(p->gsrc_scale.ensure(sizeof(double) * (size_t)std::max<int64_t>(1, ns)));
    ST_TRY(p->grec_scale.ensure(sizeof(double) * (size_t)nr));
    ST_TRY(p->gresid.ensure(sizeof(double) * (size_t)(nsteps * nr)));
    ST_TRY(p->amp_scaled.ensure(sizeof(double) * (size_t)std::max<int64_t>(1, nsteps * ns)));
    hipStream_t s = (hipStream_t)stream;
    const Layout& L = p->L;
    // u^0 = u^{-1} = 0; beta = dt^2 / (h^2 m); the source amounts
    // dt^2 / m_s * w(t) and receiver weights dt^2 / m_r
    HIP_TRY(launch_zero(fields[0], L.bytes, s));
    HIP_TRY(launch_zero(fields[1], L.bytes, s));
    HIP_TRY(launch_beta(p->dtype, m, fields[2], L.g, dt * dt / (h * h), s));
    HIP_TRY(launch_point_scale(m, roff, nr, dt * dt, (double*)p->grec_scale.p, s));
    stencil_source scaled{};
    const stencil_source* use = nullptr;
    if (ns > 0) {
        HIP_TRY(launch_point_scale(m, soff, ns, dt * dt, (double*)p->gsrc_scale.p, s));
        HIP_TRY(launch_spread(src->amp, (const double*)p->gsrc_scale.p, 0, ns, nsteps, (double*)p->amp_scaled.p, s));
        scaled = *src;
        scaled.amp = (const double*)p->amp_scaled.p;
        scaled.scale = nullptr;
        use = &scaled;
    }
    ST_TRY(forward_ckpt_impl(p, fields, nsteps, k, use, rec, ws, A, s));
    HIP_TRY(launch_misfit(rec->trace, d_obs, nsteps * nr, (double*)p->gresid.p, misfit, s));
    HIP_TRY(launch_zero(grad, sizeof(double) * L.g.n[0] * L.g.n[1] * L.g.n[2], s));
    return adjoint_impl(p, fields[2], nsteps, k, use, nr, rec->pos, (const double*)p->gresid.p,
                        (const double*)p->grec_scale.p, dt, grad, ws, A, s);
}

// ------------------------------------------------ workspace, stability, checks
stencil_status stencil_run_workspace(stencil_plan p, size_t* bytes) {
    if (!p) return fail(STENCIL_E_INVALID, "plan is NULL");
    if (!bytes) return fail(STENCIL_E_INVALID, "bytes is NULL");
    *bytes = p->program ? 0 : run_workspace_bytes(p);
    return STENCIL_OK;
}

stencil_status stencil_set_workspace(stencil_plan p, void* workspace, size_t bytes, void* stream) {
    if (!p) return fail(STENCIL_E_INVALID, "plan is NULL");
    if (p->program) return fail(STENCIL_E_STATE, "program plans take no workspace");
    if (!workspace) {
        p->ws = nullptr;
        p->ws_bytes = 0;
        return STENCIL_OK;
    }
    ST_TRY(check_ptr(workspace, "workspace"));
    if (bytes % 4) return fail(STENCIL_E_INVALID, "workspace bytes must be a multiple of 4");
    HIP_TRY(launch_zero(workspace, (int64_t)bytes, (hipStream_t)stream));
    p->ws = workspace;
    p->ws_bytes = bytes;
    return STENCIL_OK;
}

// Largest value over theta in [0, pi] of the symbol -(c0 + 2 sum_k c_k cos k theta)
// of the per-axis weights (sampled finely, and exactly at 0 and pi), times D.
static double stability_number(const stencil_plan_s* p) {
    double best = 0.0;
    const int ns = 4096;
    for (int i = 0; i <= ns; i++) {
        const double th = M_PI * i / ns;
        double v = p->coeffs[0];
        for (int k = 1; k <= p->radius; k++) v += 2.0 * p->coeffs[k] * std::cos(k * th);
        best = std::max(best, -v);
    }
    return p->ndim * best;
}

stencil_status stencil_stability(stencil_plan p, double* ds) {
    ST_TRY(check_sweep_plan(p));
    if (!ds) return fail(STENCIL_E_INVALID, "ds is NULL");
    *ds = stability_number(p);
    return STENCIL_OK;
}

stencil_status stencil_check(stencil_plan p, void* const* fields, stencil_check_report* out, void* stream) {
    ST_TRY(check_sweep_plan(p));
    if (!fields || !out) return fail(STENCIL_E_INVALID, "fields and out are required");
    const bool wave = p->kind == STENCIL_WAVE2;
    const int nlev = wave ? 2 : 1;
    for (int f = 0; f < nlev + (wave ? 1 : 0); f++) ST_TRY(check_ptr(fields[f], "field"));
    ST_TRY(p->scan.ensure(6 * sizeof(unsigned long long)));
    hipStream_t s = (hipStream_t)stream;
    unsigned long long* d = (unsigned long long*)p->scan.p;
    HIP_TRY(launch_zero(d, 6 * sizeof(unsigned long long), s));
    for (int f = 0; f < nlev; f++) HIP_TRY(launch_scan(p->dtype, fields[f], p->L.g, d, s));
    if (wave) HIP_TRY(launch_scan(p->dtype, fields[2], p->L.g, d + 3, s));
    unsigned long long h[6] = {0, 0, 0, 0, 0, 0};
    HIP_TRY(hipMemcpyAsync(h, d, sizeof h, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    std::memset(out, 0, sizeof *out);
    out->nan_count = (int64_t)h[0];
    out->inf_count = (int64_t)h[1];
    std::memcpy(&out->max_abs, &h[2], sizeof(double));
    const double ds = stability_number(p);
    if (wave) {
        std::memcpy(&out->beta_max, &h[5], sizeof(double));
        out->stability = out->beta_max * ds / 4.0;
        if (h[3] || h[4]) out->flags |= STENCIL_CHECK_BAD_BETA;
    } else {
        out->stability = ds / 2.0;
    }
    const double fmax = p->dtype == STENCIL_F16 ? 65504.0 : 3.4028234663852886e38;
    out->headroom = out->max_abs > 0 ? fmax / out->max_abs : HUGE_VAL;
    if (out->nan_count || out->inf_count) out->flags |= STENCIL_CHECK_NONFINITE;
    if (out->inf_count) out->flags |= STENCIL_CHECK_OVERFLOW;
    if (out->stability > 1.0) out->flags |= STENCIL_CHECK_UNSTABLE;
    return STENCIL_OK;
}

// --------------------------------------------------------------- variants
stencil_status stencil_variant_count(stencil_plan p, int* count) {
    if (!p) return fail(STENCIL_E_INVALID, "plan is NULL");
    if (!count) return fail(STENCIL_E_INVALID, "count is NULL");
    *count = variant_count_of(p);
    return STENCIL_OK;
}

stencil_status stencil_variant_name(stencil_plan p, int variant, char* buf, size_t len) {
    int n = 0;
    ST_TRY(stencil_variant_count(p, &n));
    if (variant < 0 || variant >= n) return fail(STENCIL_E_INVALID, "variant out of range");
    if (!buf || len == 0) return fail(STENCIL_E_INVALID, "buffer is NULL");
    std::string name;
    const std::string tile = std::to_string(kProgTileX) + "x" + std::to_string(kProgTileY) + "_t" +
                             std::to_string(kProgThreads);
    if (p->program) {
        name = variant == 3 ? "program_rtc_" + std::to_string(kProgTileX) + "x" + std::to_string(2 * kProgTileY) + "_t" +
                                  std::to_string(32 * kProgTileY)
                            : (variant == 0 ? "program_rtc_" : variant == 1 ? "program_interp_" : "program_rtc_tight_") +
                                  tile;
    } else if (batch_concurrent(p, variant)) {
        name = "shots_concurrent_" + std::to_string(kBranches);
    } else if (batch_persistent(p, variant)) {
        const Variant v = plan_variant(p, variant);
        name = "persistent_zmarch_" + std::to_string(tile_tx(v.cfg)) + "x" + std::to_string(tile_ty(v.cfg)) + "_t" +
               std::to_string(tile_threads(v.cfg)) + "_zc" + std::to_string(v.zc) + (kTileCfgs[v.cfg].nt ? "_nt" : "");
    } else if (p->ndim == 2 && variant > 0) {
        const Heat2dCfg& c = kHeat2dCfgs[variant - 1];
        name = "tb2d_t" + std::to_string(c.t) + "_" + std::to_string(c.tx) + "x" + std::to_string(c.ty);
    } else if (variant == 0) {
        name = "point";
    } else if (variant_of(variant).tb) {
        name = "tb2_" + std::to_string(kTB2TileX) + "x" + std::to_string(kTB2TileY) + "_t" +
               std::to_string(kTB2Threads) + "_zc" + std::to_string(variant_of(variant).zc);
    } else {
        const Variant v = variant_of(variant);
        name = "zmarch_" + std::to_string(tile_tx(v.cfg)) + "x" + std::to_string(tile_ty(v.cfg)) + "_t" +
               std::to_string(tile_threads(v.cfg)) + "_zc" + std::to_string(v.zc) +
               (kTileCfgs[v.cfg].vx == 8 ? "_p8" : "") + (kTileCfgs[v.cfg].nt ? "_nt" : "");
    }
    std::snprintf(buf, len, "%s", name.c_str());
    return STENCIL_OK;
}

stencil_status stencil_get_variant(stencil_plan p, int* variant) {
    if (!p) return fail(STENCIL_E_INVALID, "plan is NULL");
    if (!variant) return fail(STENCIL_E_INVALID, "variant is NULL");
    *variant = p->variant;
    return STENCIL_OK;
}

stencil_status stencil_set_variant(stencil_plan p, int variant) {
    int n = 0;
    ST_TRY(stencil_variant_count(p, &n));
    if (variant < 0 || variant >= n) return fail(STENCIL_E_INVALID, "variant out of range");
    if (p->batch && variant == 0) return fail(STENCIL_E_INVALID, "batch plans need a z-marching variant");
    p->variant = variant;
    p->variant_forced = true;
    return STENCIL_OK;
}

// Everything that decides which variants exist and how fast they run:
// device architecture, plan kind, dimensions, radius, halo, boundary,
// storage, damping and shapes (the field size also gates the temporally
// blocked sweep).
static std::string tune_key(stencil_plan p) {
    std::string arch = "unknown";
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
        arch = prop.gcnArchName;
        for (char& c : arch)
            if (c == ' ') c = '_';
    }
    std::string k = arch + " b" + std::to_string(p->batch) + ":k" + std::to_string(p->kind) + ":d" +
                    std::to_string(p->ndim) + ":r" + std::to_string(p->radius) + ":h" + std::to_string(p->halo) +
                    ":bc" + std::to_string(p->bc) + ":t" + std::to_string(p->dtype) + ":damp" +
                    std::to_string(p->damped);
    if (p->batch) {
        for (const Layout& L : p->shots)
            k += ":" + std::to_string(L.g.n[0]) + "x" + std::to_string(L.g.n[1]) + "x" + std::to_string(L.g.n[2]);
    } else {
        for (int a = 0; a < 3; a++) k += ":" + std::to_string(p->L.g.n[a]);
        k += ":B" + std::to_string(p->L.bytes);
    }
    return k;
}

// the plan's variant called `name`, or -1
static int variant_by_name(stencil_plan p, const std::string& name) {
    const int n = variant_count_of(p);
    char buf[96];
    for (int v = p->batch ? 1 : 0; v < n; v++)
        if (stencil_variant_name(p, v, buf, sizeof buf) == STENCIL_OK && name == buf) return v;
    return -1;
}

// A 2D heat run is launch-bound: time 96 steps of variant `var` the way a run
// executes them, as a captured graph replayed at least 10 times (eager launches
// leave larger gaps between kernels and would favour the deepest variants).
// The steps read `in` once and then alternate between the two scratch fields.
static stencil_status time_heat2d_graph(stencil_plan p, int var, const void* in, void* s0, void* s1, int reps,
                                        hipStream_t s, hipEvent_t e0, hipEvent_t e1, float& ms_per_step) {
    // 96 steps: 6 to 96 launches, enough that the per-replay cost of a graph
    // launch does not decide between depths
    constexpr int kSteps = 96;
    if (!p->cap) HIP_TRY(hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking));
    const int T = var == 0 ? 1 : kHeat2dCfgs[var - 1].t;
    Box3 box{};
    for (int a = 0; a < 3; a++) {
        box.lo[a] = 0;
        box.n[a] = p->L.g.n[a];
    }
    HIP_TRY(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    const void* src = in;
    void* dst = s0;
    for (int k = 0; k < kSteps / T && e == hipSuccess; k++) {
        if (var == 0) {
            ZView v{};
            v.u = src;
            v.prev = dst;
            v.out = dst;
            v.g = p->L.g;
            e = launch_point(MODE_HEAT, p->radius, p->dtype, v, p->w, box, p->cap);
        } else {
            e = launch_heat2d_tb(var - 1, p->radius, (const float*)src, (float*)dst, p->L.g, p->w, p->cap);
        }
        src = dst;
        dst = dst == s0 ? s1 : s0;
    }
    hipGraph_t graph = nullptr;
    const hipError_t ec = hipStreamEndCapture(p->cap, &graph);
    if (e == hipSuccess) e = ec;
    hipGraphExec_t ex = nullptr;
    if (e == hipSuccess) e = hipGraphInstantiate(&ex, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (e == hipSuccess) e = hipGraphLaunch(ex, s);   // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    const int nrep = std::max(reps, 10);
    for (int r = 0; r < nrep && e == hipSuccess; r++) e = hipGraphLaunch(ex, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (ex) (void)hipGraphExecDestroy(ex);
    if (e != hipSuccess) return fail(STENCIL_E_DEVICE, std::string("tuning graph: ") + hipGetErrorString(e));
    ms_per_step = ms / (float)(nrep * kSteps);
    return STENCIL_OK;
}

// The concurrent batch variant as a tuning candidate: each shot's own plan
// is tuned on its fields first (cached per shape); then every shot's kernel
// advances two steps (one temporally blocked launch, or two single-step
// launches) into scratch outputs, in the branches from fork to join, `reps`
// times.  scratch holds two fields per shot.  Result: ms per step.
static stencil_status time_batch_concurrent(stencil_plan p, void* const* fields, int reps, void* scratch, hipStream_t s,
                                            hipEvent_t e0, hipEvent_t e1, float& ms_per_step) {
    ST_TRY(ensure_shot_plans(p));
    ST_TRY(ensure_branches(p));
    const int ns = (int)p->shots.size();
    for (int sh = 0; sh < ns; sh++) ST_TRY(stencil_tune(p->shot_plans[sh], fields + 3 * sh, reps, s));
    std::vector<int64_t> off(ns);
    int64_t o = 0;
    for (int sh = 0; sh < ns; sh++) {
        off[sh] = o;
        o += 2 * round_up(p->shots[sh].bytes, 256);
    }
    const std::vector<std::vector<int>> bl = branch_lists(p);
    auto body = [&](hipStream_t bs, int sh) -> stencil_status {
        const stencil_plan_s* q = p->shot_plans[sh];
        const Layout& L = q->L;
        const Variant var = variant_of(q->variant);
        char* out = (char*)scratch + off[sh];
        if (var.tb) {
            TBView t{};
            t.u = fields[3 * sh];
            t.prev = fields[3 * sh + 1];
            t.beta = fields[3 * sh + 2];
            t.out1 = out;
            t.out2 = out + round_up(L.bytes, 256);
            t.g = L.g;
            t.ntx = (L.g.n[2] + kTB2TileX - 1) / kTB2TileX;
            t.nty = (L.g.n[1] + kTB2TileY - 1) / kTB2TileY;
            chunking(L.g.n[0], var.zc, t.zc, t.nzc);
            t.range = (uint32_t)L.bytes;
            HIP_TRY(launch_tb2(MODE_WAVE, q->radius, q->dtype, t, q->w, 0, -1, -1, bs));
            return STENCIL_OK;
        }
        for (int k = 0; k < 2; k++) {
            ZView v{};
            v.u = fields[3 * sh];
            v.prev = fields[3 * sh + 1];
            v.beta = fields[3 * sh + 2];
            v.out = out;
            v.g = L.g;
            if (var.zmarch) {
                set_tiling(v, L, var);
                HIP_TRY(launch_zmarch(MODE_WAVE, q->radius, q->dtype, var.cfg, v, q->w, 0, 0, -1, bs));
            } else {
                Box3 box{};
                for (int a = 0; a < 3; a++) {
                    box.lo[a] = 0;
                    box.n[a] = L.g.n[a];
                }
                HIP_TRY(launch_point(MODE_WAVE, q->radius, q->dtype, v, q->w, box, bs));
            }
        }
        return STENCIL_OK;
    };
    ST_TRY(fork_join(p, s, bl, body));   // warm-up
    HIP_TRY(hipEventRecord(e0, s));
    for (int r = 0; r < reps; r++) ST_TRY(fork_join(p, s, bl, body));
    HIP_TRY(hipEventRecord(e1, s));
    HIP_TRY(hipEventSynchronize(e1));
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    ms_per_step = ms / (2.0f * (float)reps);
    return STENCIL_OK;
}

// Program plans: fields = the nin inputs, then the nout outputs.  Each
// compiled variant (0, 2 and, where it exists, 3) is applied once untimed
// (that compiles and loads it) and then `reps` times on the caller's fields;
// the fastest is kept.  The outputs receive the program's result.
static stencil_status tune_program(stencil_plan p, void* const* fields, int reps, void* stream) {
    const void* ins[kProgMaxFields];
    void* outs[kProgMaxFields];
    for (int f = 0; f < p->nin; f++) ins[f] = fields[f];
    for (int o = 0; o < p->nout; o++) outs[o] = fields[p->nin + o];
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(STENCIL_E_DEVICE, "hipEventCreate failed");
    }
    const int keep = p->variant, n = variant_count_of(p);
    int best = keep;
    float best_ms = 1e30f;
    stencil_status st = STENCIL_OK;
    for (int v : {0, 2, 3}) {
        if (v >= n) continue;
        p->variant = v;
        st = stencil_program_apply(p, outs, ins, stream);
        if (st != STENCIL_OK) break;
        hipError_t e = hipEventRecord(e0, s);
        for (int r = 0; r < reps && e == hipSuccess && st == STENCIL_OK; r++) st = stencil_program_apply(p, outs, ins, stream);
        if (st != STENCIL_OK) break;
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
            st = fail(STENCIL_E_DEVICE, std::string("tuning a program: ") + hipGetErrorString(e));
            break;
        }
        if (ms < best_ms) {
            best_ms = ms;
            best = v;
        }
    }
    (void)hipStreamSynchronize(s);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    p->variant = st == STENCIL_OK ? best : keep;
    return st;
}

stencil_status stencil_tune(stencil_plan p, void* const* fields, int reps, void* stream) {
    if (!p) return fail(STENCIL_E_INVALID, "plan is NULL");
    if (!fields) return fail(STENCIL_E_INVALID, "fields is NULL");
    if (reps < 1 || reps > 1000) return fail(STENCIL_E_INVALID, "reps must be 1..1000");
    if (p->program) return tune_program(p, fields, reps, stream);
    int nvar = 0;
    ST_TRY(stencil_variant_count(p, &nvar));
    // the concurrent batch variant runs each shot with its own tuned plan
    auto tune_shot_plans = [&]() -> stencil_status {
        if (!batch_concurrent(p, p->variant)) return STENCIL_OK;
        ST_TRY(ensure_shot_plans(p));
        for (size_t sh = 0; sh < p->shots.size(); sh++) ST_TRY(stencil_tune(p->shot_plans[sh], fields + 3 * sh, reps, stream));
        return STENCIL_OK;
    };
    if (const char* force = std::getenv("STENCIL_FORCE_VARIANT")) {
        // a comma-separated list: the first name this plan offers wins
        std::string list(force);
        size_t at = 0;
        while (at <= list.size()) {
            const size_t end = std::min(list.find(',', at), list.size());
            const int v = variant_by_name(p, list.substr(at, end - at));
            if (v >= 0) {
                p->variant = v;
                return tune_shot_plans();
            }
            at = end + 1;
        }
    }
    const std::string key = tune_key(p);
    std::string cached;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        load_tune_file();
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) cached = it->second;
    }
    if (!cached.empty()) {
        // a cached name this plan does not offer is ignored and re-tuned
        const int v = variant_by_name(p, cached);
        if (v >= 0) {
            p->variant = v;
            return tune_shot_plans();
        }
    }
    if (nvar <= 1) return STENCIL_OK;
    hipStream_t s = (hipStream_t)stream;
    const bool wave = p->kind == STENCIL_WAVE2;
    const int mode = wave ? (p->damped ? MODE_WAVE_DAMP : MODE_WAVE) : MODE_HEAT;
    // scratch outputs: the caller's fields are only read
    std::vector<const Layout*> Ls;
    if (p->batch)
        for (const Layout& L : p->shots) Ls.push_back(&L);
    else
        Ls.push_back(&p->L);
    const int nf = p->batch ? 3 : (wave ? 3 : 2);
    for (size_t i = 0; i < Ls.size(); i++)
        for (int k = 0; k < (p->batch ? 3 : (wave ? 3 : 1)); k++) ST_TRY(check_ptr(fields[i * nf + k], "field"));
    // scratch outputs (two for the temporally blocked sweep)
    int64_t scratch_bytes = 0;
    for (const Layout* L : Ls) scratch_bytes += round_up(L->bytes, 256);
    scratch_bytes *= 2;
    void* scratch = nullptr;
    HIP_TRY(hipMalloc(&scratch, (size_t)scratch_bytes));
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    int best = p->variant;
    float best_ms = 1e30f;
    stencil_status st = STENCIL_OK;
    DevTable vt, bs, tvt, pl, po;
    for (int var_i = p->batch ? 1 : 0; var_i < nvar && st == STENCIL_OK; var_i++) {
        if (batch_concurrent(p, var_i)) {
            float ms = 0;
            st = time_batch_concurrent(p, fields, reps, scratch, s, e0, e1, ms);
            if (st == STENCIL_OK && ms < best_ms) {
                best_ms = ms;
                best = var_i;
            }
            continue;
        }
        if (heat2d_supported(p)) {
            float ms = 0;
            st = time_heat2d_graph(p, var_i, fields[0], scratch, (char*)scratch + round_up(p->L.bytes, 256), reps, s,
                                   e0, e1, ms);
            if (st == STENCIL_OK && ms < best_ms) {
                best_ms = ms;
                best = var_i;
            }
            continue;
        }
        const Variant var = plan_variant(p, var_i);
        std::vector<ZView> views;
        std::vector<int> bst(1, 0);
        int64_t off = 0;
        const std::vector<int> zcs = p->batch ? batch_chunks(p->shots, var.zc) : std::vector<int>(1, var.zc);
        for (size_t i = 0; i < Ls.size(); i++) {
            const Layout& L = *Ls[i];
            ZView v{};
            v.u = fields[i * nf + 0];
            v.prev = wave ? fields[i * nf + 1] : nullptr;
            v.beta = wave ? fields[i * nf + 2] : nullptr;
            v.damp = p->damped ? (const float*)p->damp.buf.p : nullptr;
            v.out = (char*)scratch + off;
            off += round_up(L.bytes, 256);
            v.g = L.g;
            Variant vs = var;
            vs.zc = zcs[i];
            if (var.zmarch || var.tb) set_tiling(v, L, vs);
            views.push_back(v);
            bst.push_back(bst.back() + (int)zmarch_blocks(v));
        }
        if (p->batch) {
            st = vt.upload(views.data(), sizeof(ZView) * views.size());
            int padded = 0;
            std::vector<int> hm;
            if (st == STENCIL_OK) {
                std::vector<int> nz;
                for (const Layout* L : Ls) nz.push_back(L->g.n[0]);
                st = build_block_map_impl(views, nz, p->radius, bs, padded, &hm);
            }
            bst.back() = padded;
            // a persistent variant the device cannot hold at once is skipped
            if (st == STENCIL_OK && var.persistent && prepare_persistent(p, var, hm, padded, pl, po) != STENCIL_OK)
                continue;
            if (st == STENCIL_OK && var.tb) {
                std::vector<TBView> tv;
                int64_t o2 = off;
                for (size_t i = 0; i < Ls.size(); i++) {
                    const Layout& L = *Ls[i];
                    TBView t{};
                    t.u = views[i].u;
                    t.prev = views[i].prev;
                    t.beta = views[i].beta;
                    t.out1 = views[i].out;
                    t.out2 = (char*)scratch + o2;
                    o2 += round_up(L.bytes, 256);
                    t.g = L.g;
                    t.ntx = views[i].ntx;
                    t.nty = views[i].nty;
                    t.zc = views[i].zc;
                    t.nzc = views[i].nzc;
                    t.range = (uint32_t)L.bytes;
                    tv.push_back(t);
                }
                st = tvt.upload(tv.data(), sizeof(TBView) * tv.size());
            }
            if (st != STENCIL_OK) break;
        }
        const bool heat2d = p->ndim == 2 && var_i > 0;
        auto launch = [&]() -> hipError_t {
            if (heat2d)
                return launch_heat2d_tb(var_i - 1, p->radius, (const float*)views[0].u, (float*)views[0].out, p->L.g,
                                        p->w, s);
            if (var.tb && p->batch)
                return tb2_batch(p->dtype, (const TBView*)tvt.buf.p, (const int*)bs.buf.p, bst.back(), p->w, 0, -1, -1, s);
            if (var.persistent) {
                // kPersistentTuneSteps steps in one launch, each reading the
                // caller's levels and writing the scratch output (parity 0)
                hipError_t e = launch_zero(p->bsync.p, kPersistentWords * sizeof(unsigned long long), s);
                if (e != hipSuccess) return e;
                return launch_zmarch_batch_persistent(p->radius, p->dtype, var.cfg, (const ZView*)vt.buf.p,
                                                      (const int*)pl.buf.p, (const int*)po.buf.p, p->pgrid, p->w, 0,
                                                      kPersistentTuneSteps, 0, 0, (unsigned long long*)p->bsync.p,
                                                      barrier_polls(), s);
            }
            if (var.tb) {
                const Layout& L = p->L;
                TBView t{};
                t.u = views[0].u;
                t.prev = views[0].prev;
                t.beta = views[0].beta;
                t.out1 = views[0].out;
                t.out2 = (char*)views[0].out + round_up(L.bytes, 256);
                t.g = L.g;
                t.ntx = (L.g.n[2] + kTB2TileX - 1) / kTB2TileX;
                t.nty = (L.g.n[1] + kTB2TileY - 1) / kTB2TileY;
                chunking(L.g.n[0], var.zc, t.zc, t.nzc);
                t.range = (uint32_t)L.bytes;
                t.damp = p->damped ? (const float*)p->damp.buf.p : nullptr;
                return launch_tb2(mode, p->radius, p->dtype, t, p->w, 0, -1, -1, s);
            }
            if (p->batch)
                return launch_zmarch_batch(p->radius, p->dtype, var.cfg, (const ZView*)vt.buf.p, (const int*)bs.buf.p,
                                           bst.back(), p->w, 0, 0, -1, s);
            if (var.zmarch) return launch_zmarch(mode, p->radius, p->dtype, var.cfg, views[0], p->w, 0, 0, -1, s);
            Box3 box{};
            for (int a = 0; a < 3; a++) {
                box.lo[a] = 0;
                box.n[a] = p->L.g.n[a];
            }
            return launch_point(mode, p->radius, p->dtype, views[0], p->w, box, s);
        };
        // a variant the runtime refuses to launch (e.g. more LDS than this
        // device allows) is skipped; any other error ends tuning
        hipError_t e = launch();
        if (e == hipErrorInvalidValue || e == hipErrorInvalidConfiguration || e == hipErrorLaunchOutOfResources) {
            (void)hipGetLastError();
            continue;
        }
        if (e == hipSuccess) e = hipEventRecord(e0, s);
        for (int r = 0; r < reps && e == hipSuccess; r++) e = launch();
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
            st = fail(STENCIL_E_DEVICE, std::string("tuning launch: ") + hipGetErrorString(e));
            break;
        }
        if (var.tb) ms *= 0.5f;   // one launch advances two steps
        if (var.persistent) {
            ms /= (float)kPersistentTuneSteps;
            const stencil_status cs = check_persistent(p, s);
            if (cs != STENCIL_OK) {
                st = cs;
                break;
            }
        }
        if (heat2d) ms /= (float)kHeat2dCfgs[var_i - 1].t;
        if (ms < best_ms) {
            best_ms = ms;
            best = var_i;
        }
    }
    (void)hipStreamSynchronize(s);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(scratch);
    if (st != STENCIL_OK) return st;
    p->variant = best;
    char name[96];
    if (stencil_variant_name(p, best, name, sizeof name) == STENCIL_OK) {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        store_tune_choice(key, name);
    }
    return STENCIL_OK;
}

}  // extern "C"
