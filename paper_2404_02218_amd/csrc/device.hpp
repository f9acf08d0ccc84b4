// Device-side building blocks shared by every sweep kernel: storage types,
// their FP32 widening / round-to-nearest-even narrowing, and the one
// per-point arithmetic of the star update.  Every kernel variant evaluates a
// point with exactly this sequence of operations, so all variants (plain,
// z-marching, batched, recompute) produce identical bits.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace stn {

// ---------------------------------------------------------------- storage
struct bf16 {
    uint16_t bits;
};
typedef _Float16 f16;

template <typename T>
struct Storage;

typedef float f4v __attribute__((ext_vector_type(4)));
typedef uint32_t u2v __attribute__((ext_vector_type(2)));

template <>
struct Storage<float> {
    __device__ static inline float load(const float* p) { return *p; }
    __device__ static inline float to_f(float v) { return v; }
    __device__ static inline float from_f(float v) { return v; }
    // four consecutive elements starting at a 16-byte aligned address
    __device__ static inline float4 load4(const float* p) { return *reinterpret_cast<const float4*>(p); }
    __device__ static inline void store4(float* p, float4 v) { *reinterpret_cast<float4*>(p) = v; }
    __device__ static inline void store(float* p, float v) { *p = v; }
    // streaming (non-temporal) forms for data touched once per sweep
    __device__ static inline void load8(const float* p, float4& a, float4& b, bool nt) {
        a = nt ? load4_nt(p) : load4(p);
        b = nt ? load4_nt(p + 4) : load4(p + 4);
    }
    __device__ static inline void store8(float* p, float4 a, float4 b, bool nt) {
        if (nt) {
            store4_nt(p, a);
            store4_nt(p + 4, b);
        } else {
            store4(p, a);
            store4(p + 4, b);
        }
    }
    __device__ static inline float4 load4_nt(const float* p) {
        const f4v r = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(p));
        return make_float4(r.x, r.y, r.z, r.w);
    }
    __device__ static inline void store4_nt(float* p, float4 v) {
        f4v r = {v.x, v.y, v.z, v.w};
        __builtin_nontemporal_store(r, reinterpret_cast<f4v*>(p));
    }
};

// bf16: widening is exact (the 16 bits are the top half of an FP32); narrowing
// is gfx950's conversion (v_cvt_pk_bf16_f32: round to nearest, ties to even; a
// NaN stays a quiet NaN), two values per instruction where they are stored
// together.  The FP32 value is pinned in a register first, as for f16 below,
// so that no kernel folds the narrowing into the producing operation.
__device__ static inline float bf16_to_f(uint16_t b) { return __uint_as_float(((uint32_t)b) << 16); }
__device__ static inline uint16_t f_to_bf16(float f) {
    asm volatile("" : "+v"(f));
    return __builtin_bit_cast(uint16_t, (__bf16)f);
}
__device__ static inline uint32_t f2_to_bf16x2(float a, float b) {
    asm volatile("" : "+v"(a), "+v"(b));
    typedef __bf16 b2 __attribute__((ext_vector_type(2)));
    const b2 r = {(__bf16)a, (__bf16)b};
    return __builtin_bit_cast(uint32_t, r);
}

template <>
struct Storage<bf16> {
    __device__ static inline float load(const bf16* p) { return bf16_to_f(p->bits); }
    __device__ static inline float to_f(bf16 v) { return bf16_to_f(v.bits); }
    __device__ static inline bf16 from_f(float v) { return bf16{f_to_bf16(v)}; }
    __device__ static inline float4 load4(const bf16* p) {
        uint2 r = *reinterpret_cast<const uint2*>(p);
        return make_float4(__uint_as_float(r.x << 16), __uint_as_float(r.x & 0xffff0000u),
                           __uint_as_float(r.y << 16), __uint_as_float(r.y & 0xffff0000u));
    }
    __device__ static inline void store4(bf16* p, float4 v) {
        uint2 r;
        r.x = f2_to_bf16x2(v.x, v.y);
        r.y = f2_to_bf16x2(v.z, v.w);
        *reinterpret_cast<uint2*>(p) = r;
    }
    __device__ static inline void store(bf16* p, float v) { p->bits = f_to_bf16(v); }
    __device__ static inline uint32_t pack2(float a, float b) { return f2_to_bf16x2(a, b); }
    // eight consecutive elements (16 bytes) as two float4
    __device__ static inline void load8(const bf16* p, float4& a, float4& b, bool nt) {
        typedef uint32_t u4v __attribute__((ext_vector_type(4)));
        const u4v r = nt ? __builtin_nontemporal_load(reinterpret_cast<const u4v*>(p)) : *reinterpret_cast<const u4v*>(p);
        a = make_float4(__uint_as_float(r.x << 16), __uint_as_float(r.x & 0xffff0000u),
                        __uint_as_float(r.y << 16), __uint_as_float(r.y & 0xffff0000u));
        b = make_float4(__uint_as_float(r.z << 16), __uint_as_float(r.z & 0xffff0000u),
                        __uint_as_float(r.w << 16), __uint_as_float(r.w & 0xffff0000u));
    }
    __device__ static inline void store8(bf16* p, float4 a, float4 b, bool nt) {
        typedef uint32_t u4v __attribute__((ext_vector_type(4)));
        u4v r;
        r.x = f2_to_bf16x2(a.x, a.y);
        r.y = f2_to_bf16x2(a.z, a.w);
        r.z = f2_to_bf16x2(b.x, b.y);
        r.w = f2_to_bf16x2(b.z, b.w);
        if (nt)
            __builtin_nontemporal_store(r, reinterpret_cast<u4v*>(p));
        else
            *reinterpret_cast<u4v*>(p) = r;
    }
    __device__ static inline float4 load4_nt(const bf16* p) {
        const u2v r = __builtin_nontemporal_load(reinterpret_cast<const u2v*>(p));
        return make_float4(__uint_as_float(r.x << 16), __uint_as_float(r.x & 0xffff0000u),
                           __uint_as_float(r.y << 16), __uint_as_float(r.y & 0xffff0000u));
    }
    __device__ static inline void store4_nt(bf16* p, float4 v) {
        u2v r;
        r.x = f2_to_bf16x2(v.x, v.y);
        r.y = f2_to_bf16x2(v.z, v.w);
        __builtin_nontemporal_store(r, reinterpret_cast<u2v*>(p));
    }
};

// f16: hardware conversions.  The FP32 value is pinned in a register before
// narrowing so that the compiler cannot fold the narrowing into the producing
// FMA (a mixed-precision FMA with an f16 result rounds once instead of twice);
// every kernel then rounds FP32 -> f16 identically.
__device__ static inline f16 f_to_f16(float v) {
    asm volatile("" : "+v"(v));
    return (f16)v;
}

template <>
struct Storage<f16> {
    __device__ static inline float load(const f16* p) { return (float)(*p); }
    __device__ static inline float to_f(f16 v) { return (float)v; }
    __device__ static inline f16 from_f(float v) { return f_to_f16(v); }
    __device__ static inline float4 load4(const f16* p) {
        typedef _Float16 h4 __attribute__((ext_vector_type(4)));
        h4 r = *reinterpret_cast<const h4*>(p);
        return make_float4((float)r.x, (float)r.y, (float)r.z, (float)r.w);
    }
    __device__ static inline void store4(f16* p, float4 v) {
        typedef _Float16 h4 __attribute__((ext_vector_type(4)));
        h4 r;
        r.x = f_to_f16(v.x);
        r.y = f_to_f16(v.y);
        r.z = f_to_f16(v.z);
        r.w = f_to_f16(v.w);
        *reinterpret_cast<h4*>(p) = r;
    }
    __device__ static inline void store(f16* p, float v) { *p = f_to_f16(v); }
    __device__ static inline uint32_t pack2(float a, float b) {
        return (uint32_t)__builtin_bit_cast(uint16_t, f_to_f16(a)) | ((uint32_t)__builtin_bit_cast(uint16_t, f_to_f16(b)) << 16);
    }
    __device__ static inline void load8(const f16* p, float4& a, float4& b, bool nt) {
        typedef _Float16 h8 __attribute__((ext_vector_type(8)));
        const h8 r = nt ? __builtin_nontemporal_load(reinterpret_cast<const h8*>(p)) : *reinterpret_cast<const h8*>(p);
        a = make_float4((float)r[0], (float)r[1], (float)r[2], (float)r[3]);
        b = make_float4((float)r[4], (float)r[5], (float)r[6], (float)r[7]);
    }
    __device__ static inline void store8(f16* p, float4 a, float4 b, bool nt) {
        typedef _Float16 h8 __attribute__((ext_vector_type(8)));
        h8 r;
        r[0] = f_to_f16(a.x);
        r[1] = f_to_f16(a.y);
        r[2] = f_to_f16(a.z);
        r[3] = f_to_f16(a.w);
        r[4] = f_to_f16(b.x);
        r[5] = f_to_f16(b.y);
        r[6] = f_to_f16(b.z);
        r[7] = f_to_f16(b.w);
        if (nt)
            __builtin_nontemporal_store(r, reinterpret_cast<h8*>(p));
        else
            *reinterpret_cast<h8*>(p) = r;
    }
    __device__ static inline float4 load4_nt(const f16* p) {
        typedef _Float16 h4 __attribute__((ext_vector_type(4)));
        const h4 r = __builtin_nontemporal_load(reinterpret_cast<const h4*>(p));
        return make_float4((float)r.x, (float)r.y, (float)r.z, (float)r.w);
    }
    __device__ static inline void store4_nt(f16* p, float4 v) {
        typedef _Float16 h4 __attribute__((ext_vector_type(4)));
        h4 r;
        r.x = f_to_f16(v.x);
        r.y = f_to_f16(v.y);
        r.z = f_to_f16(v.z);
        r.w = f_to_f16(v.w);
        __builtin_nontemporal_store(r, reinterpret_cast<h4*>(p));
    }
};

// VX consecutive elements (VX = 4 or 8) at an aligned address, as floats
template <typename T, int VX>
__device__ static inline void load_vec(const T* p, float4 (&v)[VX / 4], bool nt) {
    if constexpr (VX == 4)
        v[0] = nt ? Storage<T>::load4_nt(p) : Storage<T>::load4(p);
    else
        Storage<T>::load8(p, v[0], v[1], nt);
}
template <typename T, int VX>
__device__ static inline void store_vec(T* p, const float4 (&v)[VX / 4], bool nt) {
    if constexpr (VX == 4) {
        if (nt)
            Storage<T>::store4_nt(p, v[0]);
        else
            Storage<T>::store4(p, v[0]);
    } else {
        Storage<T>::store8(p, v[0], v[1], nt);
    }
}

// Loads that stay in flight across a compute phase are kept in the storage
// type and widened to FP32 where they are consumed: a conversion placed next
// to its load makes the wave wait for that load there.  RawGroup<T>::type
// holds 4 consecutive elements as loaded.
template <typename T>
struct RawGroup {
    typedef float4 type;
};
template <>
struct RawGroup<bf16> {
    typedef u2v type;
};
template <>
struct RawGroup<f16> {
    typedef u2v type;
};

// NT: the streaming (non-temporal) hint, fixed at compile time so that the
// hint cannot be lost when the compiler merges the two forms of the load
template <typename T, bool NT>
__device__ static inline typename RawGroup<T>::type load4_raw(const T* p) {
    if constexpr (std::is_same<T, float>::value) {
        if constexpr (NT) return Storage<float>::load4_nt(p);
        else return Storage<float>::load4(p);
    } else {
        if constexpr (NT) return __builtin_nontemporal_load(reinterpret_cast<const u2v*>(p));
        else return *reinterpret_cast<const u2v*>(p);
    }
}
template <typename T>
__device__ static inline float4 widen4(typename RawGroup<T>::type r) {
    if constexpr (std::is_same<T, float>::value) {
        return r;
    } else if constexpr (std::is_same<T, bf16>::value) {
        return make_float4(__uint_as_float(r.x << 16), __uint_as_float(r.x & 0xffff0000u), __uint_as_float(r.y << 16),
                           __uint_as_float(r.y & 0xffff0000u));
    } else {
        typedef _Float16 h4 __attribute__((ext_vector_type(4)));
        const h4 h = __builtin_bit_cast(h4, r);
        return make_float4((float)h.x, (float)h.y, (float)h.z, (float)h.w);
    }
}
template <typename T, int VX, bool NT>
__device__ static inline void load_vec_raw(const T* p, typename RawGroup<T>::type (&r)[VX / 4]) {
#pragma unroll
    for (int c = 0; c < VX / 4; c++) r[c] = load4_raw<T, NT>(p + 4 * c);
}

// value after a round trip through the storage type
template <typename T>
__device__ static inline float through(float v) {
    return Storage<T>::to_f(Storage<T>::from_f(v));
}

// ------------------------------------------------------------ coefficients
struct Coefs {
    float c[5];  // c_0..c_r (unused tail zero)
    float cd0;   // D * c_0, the centre weight of the D-axis star
};

enum Mode : int {
    MODE_HEAT = 0,      // out = u + L u
    MODE_WAVE = 1,      // out = 2u - u_prev + beta L u
    MODE_WAVE_D = 2,    // as MODE_WAVE, also writes beta L u (+ source) to a second-difference field
    MODE_WAVE_ADJ = 3,  // as MODE_WAVE, then g += out * d for an imaging field pair (g, d)
    MODE_WAVE_ADJ2 = 5, // as MODE_WAVE_ADJ, with g += u * d2 first: the input level paired with a second field d2
    MODE_WAVE_DAMP = 4, // the wave with an absorbing layer (damped_update), FP32
};

// Canonical accumulation: centre, then the z pairs, the y pairs, the x pairs,
// k = 1..r within an axis.  `m[k-1]`, `p[k-1]` are the taps at -k and +k.
template <int R>
__device__ static inline float axis_sum(float acc, const Coefs& w, const float* m, const float* p) {
#pragma unroll
    for (int k = 1; k <= R; k++) acc = fmaf(w.c[k], m[k - 1] + p[k - 1], acc);
    return acc;
}

// the per-point time update given L u (acc), the centre and the previous level
template <int MODE>
__device__ static inline float time_update(float acc, float centre, float prev, float beta) {
    if constexpr (MODE == MODE_HEAT) {
        return centre + acc;
    } else {
        float t = 2.0f * centre - prev;
        return fmaf(beta, acc, t);
    }
}

// The damped leapfrog of an absorbing layer: m u_tt + eta u_t = L u / h^2
// with u_t centred gives, for gamma = eta dt / (2 m),
//     u+ = (2u - (1 - gamma) u- + beta L u) / (1 + gamma),
// evaluated as ((2u - u-) + gamma u- + beta L u) / (1 + gamma).  Where gamma
// is 0 the result is the undamped update bit for bit.
__device__ static inline float damped_update(float acc, float centre, float prev, float beta, float gamma) {
    const float t = 2.0f * centre - prev;
    if (gamma == 0.0f) return fmaf(beta, acc, t);
    return fmaf(beta, acc, fmaf(gamma, prev, t)) / (1.0f + gamma);
}

// source injection: round to storage, widen, add the FP64 amount, round back
template <typename T>
__device__ static inline float inject(float v, double amount) {
    float s = through<T>(v);
    return (float)((double)s + amount);
}

}  // namespace stn
