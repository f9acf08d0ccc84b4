// Stencil programs compiled per program.  When a program plan is created the
// runtime writes a HIP kernel in which the terms are constants and compiles it
// for gfx950 with hiprtc; the code object is shared by every plan with the same
// program and loaded once per device at the first apply.  This is the
// counterpart of lowering one stencil program to one specialised GPU kernel
// (Section 4): the generic kernel in program.hip interprets the same terms.
//
// The generated kernel keeps that kernel's tiling (64 x 16 tiles, 256 threads,
// 4 x points per thread, an LDS ring of 2 rz + 2 planes per input; a taller
// form has 64 x 32 tiles of 512 threads, half the halo rows per point) and its
// arithmetic (terms in program order, one rounding per product and a fused
// multiply-add into the output), so the two agree bit for bit.  What the
// constants buy: the z loop is unrolled by the ring size, so every LDS read is
// a fixed offset from one per-thread address; each LDS group that several
// terms share is read once per plane; and the inputs' next plane is loaded
// into registers before the current plane is computed, so its HBM latency
// overlaps the arithmetic.
#include <hip/hiprtc.h>

#include <cstdio>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <sstream>
#include <string>
#include <vector>

#include "kernels.hpp"

namespace stn {

namespace {

constexpr int GX = (kProgTileX + 8) / 4;  // float4 groups per LDS row
constexpr int kMaxDevices = 64;

std::string flt(float c) {
    char b[64];
    std::snprintf(b, sizeof b, "%af", (double)c);  // hexadecimal: exact
    return b;
}

// per-thread offset (in float4 groups) of an LDS group from the thread's own
// group in slot 0 of input 0
int group_offset(int f, int slot, int dy, int gd, int ns, int plane4) {
    return (f * ns + slot) * plane4 + dy * GX + gd;
}

std::string gname(int off) { return off < 0 ? "gm" + std::to_string(-off) : "g" + std::to_string(off); }

}  // namespace

std::string program_source(int nin, int nout, int rz, int ry, const std::vector<ProgTerm>& terms, bool tight,
                           int tile_y) {
    // tight: a ring of 2 rz + 1 planes (less LDS, so more workgroups per CU)
    // whose refill waits for a second barrier after the compute
    // tile_y rows of 16 threads, each thread 4 consecutive x points of one row
    const int threads = 16 * tile_y;
    const int ns = 2 * rz + (tight ? 1 : 2), ldy = tile_y + 2 * ry, plane4 = ldy * GX;
    const int ngroups = plane4, nload = (ngroups + threads - 1) / threads;
    std::ostringstream s;
    s << "// generated stencil program: " << nin << " inputs, " << nout << " outputs, " << terms.size()
      << " terms, reach z " << rz << " y " << ry << (tight ? ", tight ring" : "") << ", tile 64x" << tile_y
      << "\n";
    s << "typedef float f4 __attribute__((ext_vector_type(4)));\n"
         "__device__ __forceinline__ f4 fma4(f4 a, f4 b, f4 c) {\n"
         "  return (f4){__builtin_fmaf(a.x, b.x, c.x), __builtin_fmaf(a.y, b.y, c.y),\n"
         "              __builtin_fmaf(a.z, b.z, c.z), __builtin_fmaf(a.w, b.w, c.w)};\n}\n";
    s << "extern \"C\" __global__ void __launch_bounds__(" << threads << ") stencil_program(";
    for (int f = 0; f < nin; f++) s << "const float* __restrict__ in" << f << ", ";
    for (int o = 0; o < nout; o++) s << "float* __restrict__ out" << o << ", ";
    s << "long long origin, long long sz, long long sy, int nx, int ny, int nz, int xmax4, int ntx, int nty, "
         "int zc) {\n";
    s << "  __shared__ f4 L[" << nin * ns * plane4 << "];\n";
    // XCD-aware tile order: hardware dispatches workgroup b to XCD b % 8, so
    // each XCD receives a contiguous range of logical tiles
    s << "  const int nb = (int)gridDim.x, b = (int)blockIdx.x, xq = nb >> 3, xr = nb & 7, xc = b & 7;\n"
         "  const int lb = xc * xq + min(xc, xr) + (b >> 3);\n"
         "  const int tid = (int)threadIdx.x, tx = tid & 15, ty = tid >> 4;\n"
         "  const int tile_x = lb % ntx, tile_y = (lb / ntx) % nty, zch = lb / (ntx * nty);\n"
         "  const int X0 = tile_x * "
      << kProgTileX << ", Y0 = tile_y * " << tile_y
      << ";\n"
         "  const int zb = zch * zc, ze = min(zb + zc, nz);\n";
    // the groups this thread loads: LDS group gi = row * GX + column; rows and
    // planes clamp into the halo, columns to the row's last full group
    for (int k = 0; k < nload; k++) {
        const bool always = (k + 1) * threads <= ngroups;
        s << "  const int gi" << k << " = tid + " << k * threads << ";\n";
        s << "  const bool ok" << k << " = " << (always ? "true" : "gi" + std::to_string(k) + " < " + std::to_string(ngroups))
          << ";\n";
        s << "  const long long go" << k << " = origin + (long long)min(max(Y0 - " << ry << " + gi" << k << " / " << GX
          << ", " << -ry << "), ny + " << ry - 1 << ") * sy + min(X0 - 4 + 4 * (gi" << k << " % " << GX
          << "), xmax4);\n";
        for (int f = 0; f < nin; f++) s << "  f4 pf" << f << "_" << k << ";\n";
    }
    auto gload = [&](const std::string& plane, const std::string& ind) {
        s << ind << "{ const long long pz = (long long)min(max(" << plane << ", " << -rz << "), nz + " << rz - 1
          << ") * sz;\n";
        for (int k = 0; k < nload; k++) {
            s << ind << "  if (ok" << k << ") {";
            for (int f = 0; f < nin; f++)
                s << " pf" << f << "_" << k << " = *(const f4*)(in" << f << " + go" << k << " + pz);";
            s << " }\n";
        }
        s << ind << "}\n";
    };
    auto lput = [&](int slot, const std::string& ind) {
        for (int k = 0; k < nload; k++) {
            s << ind << "if (ok" << k << ") {";
            for (int f = 0; f < nin; f++)
                s << " L[" << (f * ns + slot) * plane4 << " + gi" << k << "] = pf" << f << "_" << k << ";";
            s << " }\n";
        }
    };
    // prologue: planes zb - rz .. zb + rz into slots 0 .. 2 rz
    for (int sl = 0; sl <= 2 * rz; sl++) {
        gload("zb - " + std::to_string(rz - sl), "  ");
        lput(sl, "  ");
    }
    s << "  __syncthreads();\n";
    s << "  const int y = Y0 + ty, x0 = X0 + 4 * tx;\n"
         "  const bool row_ok = y < ny && x0 < nx, full = x0 + 3 < nx;\n"
         "  const long long obase = origin + (long long)y * sy + x0;\n"
         "  const f4* T0 = L + (ty + "
      << ry << ") * " << GX << " + 1 + tx;\n";
    s << "  for (int z = zb; z < ze; z += " << ns << ") {\n";
    for (int j = 0; j < ns; j++) {
        // plane zz = z + j; z - zb is a multiple of the ring size, so the
        // slot of plane zz + dz is (j + dz + rz) mod ns
        s << "    {\n      const int zz = z + " << j << ";\n      if (zz >= ze) break;\n"
          << "      const bool more = zz + 1 < ze;\n";
        s << "      if (more)\n";
        gload("zz + " + std::to_string(rz + 1), "      ");
        for (int o = 0; o < nout; o++) s << "      f4 acc" << o << " = (f4){0.f, 0.f, 0.f, 0.f};\n";
        std::set<int> have;
        auto group = [&](int off) {
            if (have.insert(off).second) s << "      const f4 " << gname(off) << " = T0[" << off << "];\n";
            return gname(off);
        };
        auto factor = [&](int f, const int (&o)[3]) {
            const int slot = ((j + o[0] + rz) % ns + ns) % ns;
            const int base = group_offset(f, slot, o[1], 0, ns, plane4);
            const std::string c = group(base);
            switch (o[2]) {
                case -2: {
                    const std::string p = group(base - 1);
                    return "(f4){" + p + ".z, " + p + ".w, " + c + ".x, " + c + ".y}";
                }
                case -1: {
                    const std::string p = group(base - 1);
                    return "(f4){" + p + ".w, " + c + ".x, " + c + ".y, " + c + ".z}";
                }
                case 1: {
                    const std::string n = group(base + 1);
                    return "(f4){" + c + ".y, " + c + ".z, " + c + ".w, " + n + ".x}";
                }
                case 2: {
                    const std::string n = group(base + 1);
                    return "(f4){" + c + ".z, " + c + ".w, " + n + ".x, " + n + ".y}";
                }
                default:
                    return c;
            }
        };
        for (const ProgTerm& T : terms) {
            const std::string a = factor(T.in0, T.o0);
            const std::string acc = "acc" + std::to_string(T.out);
            if (T.nfac == 1) {
                s << "      " << acc << " = fma4((f4)(" << flt(T.coeff) << "), " << a << ", " << acc << ");\n";
            } else {
                const std::string bb = factor(T.in1, T.o1);
                s << "      " << acc << " = fma4(" << flt(T.coeff) << " * " << a << ", " << bb << ", " << acc
                  << ");\n";
            }
        }
        s << "      if (row_ok) {\n        const long long oo = obase + (long long)zz * sz;\n"
             "        if (full) {\n";
        for (int o = 0; o < nout; o++)
            s << "          __builtin_nontemporal_store(acc" << o << ", (f4*)(out" << o << " + oo));\n";
        s << "        } else {\n";
        for (int o = 0; o < nout; o++)
            for (int i = 0; i < 4; i++)
                s << "          if (x0 + " << i << " < nx) out" << o << "[oo + " << i << "] = acc" << o << "[" << i
                  << "];\n";
        s << "        }\n      }\n";
        if (tight) s << "      __syncthreads();\n";
        s << "      if (more) {\n";
        lput((j + 2 * rz + 1) % ns, "        ");
        s << "      }\n      __syncthreads();\n    }\n";
    }
    s << "  }\n}\n";
    return s.str();
}

// ------------------------------------------------------------ compilation
struct RtcProgram {
    std::vector<char> code;
    int threads = 0;   // workgroup size
    std::mutex mu;
    hipModule_t mod[kMaxDevices] = {};
    hipFunction_t fn[kMaxDevices] = {};
};

namespace {
std::mutex g_rtc_mu;
std::map<std::string, std::shared_ptr<RtcProgram>> g_rtc;  // by source text
}  // namespace

std::shared_ptr<RtcProgram> program_compile(const std::string& src, int threads, std::string& log) {
    {
        std::lock_guard<std::mutex> lk(g_rtc_mu);
        auto it = g_rtc.find(src);
        if (it != g_rtc.end()) return it->second;
    }
    hiprtcProgram prog;
    if (hiprtcCreateProgram(&prog, src.c_str(), "stencil_program.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS) {
        log = "hiprtcCreateProgram failed";
        return nullptr;
    }
    const char* opts[] = {"--offload-arch=gfx950", "-O3",     "-std=c++17",      "-ffp-contract=off",
                          "-Xclang",               "-target-feature", "-Xclang", "-packed-fp32-ops"};
    const hiprtcResult r = hiprtcCompileProgram(prog, (int)(sizeof opts / sizeof opts[0]), opts);
    size_t n = 0;
    hiprtcGetProgramLogSize(prog, &n);
    log.assign(n, '\0');
    if (n) hiprtcGetProgramLog(prog, &log[0]);
    std::shared_ptr<RtcProgram> out;
    if (r == HIPRTC_SUCCESS) {
        size_t cs = 0;
        hiprtcGetCodeSize(prog, &cs);
        out = std::make_shared<RtcProgram>();
        out->threads = threads;
        out->code.resize(cs);
        hiprtcGetCode(prog, out->code.data());
    }
    hiprtcDestroyProgram(&prog);
    if (out) {
        std::lock_guard<std::mutex> lk(g_rtc_mu);
        auto it = g_rtc.emplace(src, out).first;  // a concurrent compile of the same text may have won
        out = it->second;
    }
    return out;
}

hipError_t launch_program_rtc(RtcProgram& rp, const ProgView& v, hipStream_t s) {
    const int64_t nb = (int64_t)v.ntx * v.nty * v.nzc;
    if (nb == 0) return hipSuccess;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    hipFunction_t fn;
    {
        std::lock_guard<std::mutex> lk(rp.mu);
        if (!rp.fn[dev]) {
            e = hipModuleLoadData(&rp.mod[dev], rp.code.data());
            if (e != hipSuccess) return e;
            e = hipModuleGetFunction(&rp.fn[dev], rp.mod[dev], "stencil_program");
            if (e != hipSuccess) {
                (void)hipModuleUnload(rp.mod[dev]);
                rp.mod[dev] = nullptr;
                rp.fn[dev] = nullptr;
                return e;
            }
        }
        fn = rp.fn[dev];
    }
    long long origin = v.g.origin, sz = v.g.s[0], sy = v.g.s[1];
    int nx = v.g.n[2], ny = v.g.n[1], nz = v.g.n[0];
    int xmax4 = (int)(v.g.rowlen - v.g.xlead) - 4, ntx = v.ntx, nty = v.nty, zc = v.zc;
    const float* in[kProgMaxFields];
    float* out[kProgMaxFields];
    void* args[2 * kProgMaxFields + 10];
    int na = 0;
    for (int f = 0; f < v.nin; f++) {
        in[f] = v.in[f];
        args[na++] = &in[f];
    }
    for (int o = 0; o < v.nout; o++) {
        out[o] = v.out[o];
        args[na++] = &out[o];
    }
    void* rest[] = {&origin, &sz, &sy, &nx, &ny, &nz, &xmax4, &ntx, &nty, &zc};
    for (void* a : rest) args[na++] = a;
    return hipModuleLaunchKernel(fn, (unsigned)nb, 1, 1, (unsigned)rp.threads, 1, 1, 0, s, args, nullptr);
}

}  // namespace stn
