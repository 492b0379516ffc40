// device_common.h -- device helpers shared by the image and scalar kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.h"

// Address-space views.  Data read through AS4 ("constant") is not written by
// the kernel reading it, so wave-uniform reads become scalar loads (operator
// weights, solve state, work lists); AS1 is plain global memory.
#define AS1 __attribute__((address_space(1)))
#define AS4 __attribute__((address_space(4)))
#define FI __device__ __forceinline__ __attribute__((always_inline))

namespace misr {

typedef long long i64;

FI int fdiv(int a, int b) {
    const int q = a / b;
    return (a % b != 0 && ((a < 0) != (b < 0))) ? q - 1 : q;
}
FI int cdiv(int a, int b) { return -fdiv(-a, b); }
FI int pmod(int a, int b) {
    const int r = a % b;
    return r < 0 ? r + b : r;
}
FI int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
FI float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
// v from the lane below: lane i receives lane i-1's value, lane 0 receives 0
// (a DPP wave shift right by one, full rate, no LDS traffic).
FI float wave_shr1(float v) {
    return __int_as_float(
        __builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x138, 0xf, 0xf, false));
}

template <class T>
FI const AS4 T *cst(const T *p) { return (const AS4 T *)p; }
template <class T>
FI const AS1 T *glb(const T *p) { return (const AS1 T *)p; }
template <class T>
FI AS1 T *glbw(T *p) { return (AS1 T *)p; }

// 32-bit mixing hash (the MurmurHash3 finaliser) of a pixel index and a seed:
// the counter-based source of the stochastic-rounding bits.
FI unsigned mix32(unsigned h) {
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}
FI unsigned pixel_hash(long long gidx, unsigned seed) {
    return mix32((unsigned)gidx * 0x9e3779b1u ^ mix32((unsigned)(gidx >> 32) + seed));
}

// Storage of x and y: float32, IEEE half or bfloat16.  rnd() rounds to the
// nearest representable value (ties to even); rnd_sr() rounds up with
// probability equal to the fraction of the spacing, from 16 hash bits.
struct StF32 {
    using raw = float;
    static constexpr int code = ST_F32;
    static FI float ld(const AS1 raw *p, i64 i) { return p[i]; }
    static FI float rnd(float v) { return v; }
    static FI float rnd_sr(float v, unsigned) { return v; }
    static FI void st(AS1 raw *p, i64 i, float v) { p[i] = v; }
};
struct StF16 {
    using raw = _Float16;
    static constexpr int code = ST_F16;
    static FI float ld(const AS1 raw *p, i64 i) { return (float)p[i]; }
    static FI float rnd(float v) { return (float)(_Float16)v; }
    static FI float rnd_sr(float v, unsigned h) {
        // spacing of half precision at v (subnormal spacing 2^-24 below 2^-14)
        const int e = (int)((__float_as_uint(v) >> 23) & 0xffu) - 127;
        const float ulp = __builtin_ldexpf(1.f, (e < -14 ? -14 : e) - 10);
        const float u = (float)(h & 0xffffu) * (1.f / 65536.f) - 0.5f;
        return (float)(_Float16)fmaf(u, ulp, v);
    }
    static FI void st(AS1 raw *p, i64 i, float v) { p[i] = (_Float16)v; }
};
// Detector counts: frames only (read, never written); the frame value is the
// count times the solve's y_scale, applied by the reader.
struct StU16 {
    using raw = unsigned short;
    static constexpr int code = ST_U16;
    static FI float ld(const AS1 raw *p, i64 i) { return (float)p[i]; }
};
struct StBF16 {
    using raw = unsigned short;
    static constexpr int code = ST_BF16;
    static FI unsigned short bits(float v) {
        unsigned u = __float_as_uint(v);
        if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
        u += 0x7fffu + ((u >> 16) & 1u);
        return (unsigned short)(u >> 16);
    }
    static FI float ld(const AS1 raw *p, i64 i) { return __uint_as_float((unsigned)p[i] << 16); }
    static FI float rnd(float v) { return __uint_as_float((unsigned)bits(v) << 16); }
    static FI float rnd_sr(float v, unsigned h) {
        unsigned u = __float_as_uint(v);
        if ((u & 0x7fffffffu) >= 0x7f800000u) return rnd(v);
        u += h & 0xffffu;
        return __uint_as_float(u & 0xffff0000u);
    }
    static FI void st(AS1 raw *p, i64 i, float v) { p[i] = bits(v); }
};

// Charbonnier penalty phi(z) = sqrt(z^2+e^2) - e and its derivative
// psi(z) = z / sqrt(z^2+e^2); e = 0 gives |z| and sign(z), sign(0) = 0.
FI void phi_psi(float z, float eps, float e2, float &phi, float &psi) {
    if (eps == 0.f) {
        phi = fabsf(z);
        psi = (z > 0.f) ? 1.f : ((z < 0.f) ? -1.f : 0.f);
        return;
    }
    const float d = fmaf(z, z, e2);
    const float r = rsq(d);
    psi = z * r;
    phi = z * psi / fmaf(eps, r, 1.f);
}

// (psi(b + h) - psi(b)) / h, the finite-difference quotient Moller's curvature
// takes along one BTV pair.  Closed form without cancellation:
//   (e^2 + C) / (A B (A + B)),  A = |(a, e)|, B = |(b, e)|, C = A B - a b,
// with C = (e^2 (a^2 + b^2) + e^4) / (A B + a b) when a b > 0.  When |h| is
// below 1e-3 B the Taylor series in h to third order is used instead (its
// remainder is below float32 rounding).
FI float psi_quot(float b, float h, float eps, float e2) {
    if (eps == 0.f) {
        if (h == 0.f) return 0.f;
        const float a = b + h;
        const float sa = (a > 0.f) ? 1.f : ((a < 0.f) ? -1.f : 0.f);
        const float sb = (b > 0.f) ? 1.f : ((b < 0.f) ? -1.f : 0.f);
        return (sa - sb) / h;
    }
    const float bb = fmaf(b, b, e2);
    const float rB = rsq(bb);
    const float rB2 = rB * rB;
    const float t = h * rB2;
    if (fabsf(h * rB) < 1e-3f) {
        const float poly = fmaf(0.5f * t * t, fmaf(4.f * b, b, -e2), fmaf(-1.5f * t, b, 1.f));
        return e2 * rB * rB2 * poly;
    }
    const float a = b + h;
    const float aa = fmaf(a, a, e2);
    const float rA = rsq(aa);
    const float A = aa * rA, B = bb * rB;
    const float AB = A * B, ab = a * b;
    const float C = (ab > 0.f) ? (e2 * (a * a + b * b) + e2 * e2) / (AB + ab) : AB - ab;
    return (e2 + C) * rA * rB / (A + B);
}

FI double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// Sums N per-thread values over an NT-thread workgroup in a fixed order and
// stores them to out[0..N) (threads 0..N-1 write).  red: LDS scratch of
// N * NT/64 doubles.
template <int N, int NT>
FI void block_sum_store(double (&v)[N], double *out, double *red) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = wave_sum(v[i]);
    if (lane == 0)
#pragma unroll
        for (int i = 0; i < N; ++i) red[wid * N + i] = v[i];
    __syncthreads();
    if (threadIdx.x < N) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < NT / 64; ++w) s += red[w * N + threadIdx.x];
        out[threadIdx.x] = s;
    }
    __syncthreads();
}

}  // namespace misr
