// llr_device.hpp -- device helpers for the gfx950 LLR kernels: the
// Philox4x32-10 counter generator, uniform conversions, precision-specific
// math, and the XCD-aware block remap.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace llr {

constexpr int kBlock = 256;           // threads per block of the lattice kernels
constexpr int kMaxLat = 8;            // lattices per context
constexpr int kVmCap = 64;            // heatbath sampler attempt cap

enum Kind : uint32_t { kSweep = 0, kInit = 1, kApproach = 2, kReplica = 3, kMlp = 4, kBoot = 5, kMuca = 6 };

// heatbath pass modes: the public LLR_MODE_* values 0-3 and the tuner's
// timing mode (proposals written, nothing accepted, no counters touched)
constexpr int kHbModeTune = 5;

__host__ __device__ inline uint32_t ctr1_word(uint32_t attempt_pair, uint32_t colour, uint32_t kind,
                                              uint32_t lat) {
    return (attempt_pair & 0xffu) | ((colour & 0xfu) << 8) | ((kind & 0xfu) << 12) | ((lat & 0xffu) << 16);
}

// a ^ b ^ c in one instruction: gfx950's three-input bitwise operation with
// the truth table of the three-way exclusive or (0x96)
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32->64
// multiplications with the published multipliers, key bumped by the published
// Weyl constants between rounds.  In the first two rounds some words are
// uniform over the wavefront (the sweep and interval counter words and the
// key), and the compiler keeps that work on the scalar unit; from the third
// round on every word differs per lane, and each round's two double xors are
// one three-input operation each.
__device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c.z;
        if (r < 2)
            c = make_uint4((uint32_t)(p1 >> 32) ^ c.y ^ k0, (uint32_t)p1, (uint32_t)(p0 >> 32) ^ c.w ^ k1,
                           (uint32_t)p0);
        else
            c = make_uint4(xor3((uint32_t)(p1 >> 32), c.y, k0), (uint32_t)p1, xor3((uint32_t)(p0 >> 32), c.w, k1),
                           (uint32_t)p0);
    }
    return c;
}

// Precision traits: FP64 uses full-precision math (the library's, and a
// range-specific sine and cosine of the same accuracy); FP32 uses the
// hardware transcendental unit (v_sin_f32/v_cos_f32 take revolutions) and
// approximate reciprocals where the sampler tolerates ulp-level error.
template <typename T> struct Math;

template <> struct Math<double> {
    static constexpr bool f32 = false;
    __device__ static __forceinline__ double unif(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }
    __device__ static __forceinline__ double sunif(uint32_t w) { return ((double)(int32_t)w + 0.5) * 0x1p-31; }
    // sin and cos of x for |x| <= 4 pi, which covers every caller (staple sums
    // of three angles in [-pi, pi), single angles): x = k pi + r with
    // |r| <= pi/2 by Cody and Waite's two-part reduction (pi_hi keeps 48
    // significant bits, so k pi_hi is exact for |k| <= 8), sin r and cos r by
    // their Taylor series through r^21 and r^22 (truncation below 2e-18 on
    // |r| <= pi/2), then the sign (-1)^k.  Measured error against the C
    // library: 2.7e-16 absolute over 2e7 points of |x| <= 3 pi.  The library
    // routine carries a large-argument path these angles never need.
    __device__ static __forceinline__ void sincos_rad(double x, double* s, double* c) {
        const double k = rint(x * 0.31830988618379067);           // 1/pi
        double r = __fma_rn(-k, 0x1.921fb54442d00p+1, x);          // pi_hi
        r = __fma_rn(-k, 0x1.8469898cc5170p-47, r);                // pi - pi_hi
        const double u = r * r;
        double p = 0x1.71b8ef6dcf572p-66;                           //  1/21!
        p = __fma_rn(p, u, -0x1.2f49b46814157p-57);                 // -1/19!
        p = __fma_rn(p, u, 0x1.952c77030ad4ap-49);                  //  1/17!
        p = __fma_rn(p, u, -0x1.ae7f3e733b81fp-41);                 // -1/15!
        p = __fma_rn(p, u, 0x1.6124613a86d09p-33);                  //  1/13!
        p = __fma_rn(p, u, -0x1.ae64567f544e4p-26);                 // -1/11!
        p = __fma_rn(p, u, 0x1.71de3a556c734p-19);                  //  1/9!
        p = __fma_rn(p, u, -0x1.a01a01a01a01ap-13);                 // -1/7!
        p = __fma_rn(p, u, 0x1.1111111111111p-7);                   //  1/5!
        p = __fma_rn(p, u, -0x1.5555555555555p-3);                  // -1/3!
        const double sr = __fma_rn(r * u, p, r);
        double q = -0x1.0ce396db7f853p-70;                          // -1/22!
        q = __fma_rn(q, u, 0x1.e542ba4020225p-62);                  //  1/20!
        q = __fma_rn(q, u, -0x1.6827863b97d97p-53);                 // -1/18!
        q = __fma_rn(q, u, 0x1.ae7f3e733b81fp-45);                  //  1/16!
        q = __fma_rn(q, u, -0x1.93974a8c07c9dp-37);                 // -1/14!
        q = __fma_rn(q, u, 0x1.1eed8eff8d898p-29);                  //  1/12!
        q = __fma_rn(q, u, -0x1.27e4fb7789f5cp-22);                 // -1/10!
        q = __fma_rn(q, u, 0x1.a01a01a01a01ap-16);                  //  1/8!
        q = __fma_rn(q, u, -0x1.6c16c16c16c17p-10);                 // -1/6!
        q = __fma_rn(q, u, 0x1.5555555555555p-5);                   //  1/4!
        q = __fma_rn(q, u, -0.5);
        q = __fma_rn(q, u, 1.0);
        const bool odd = ((int)k & 1) != 0;
        *s = odd ? -sr : sr;
        *c = odd ? -q : q;
    }
    // sin, cos of (pi/2) v for |v| < 1
    __device__ static __forceinline__ void sincos_halfpi(double v, double* s, double* c) { sincospi(0.5 * v, s, c); }
    // sin and cos of (pi/2) sunif(w)
    __device__ static __forceinline__ void sincos_halfpi_w(uint32_t w, double* s, double* c) {
        sincos_halfpi(sunif(w), s, c);
    }
    __device__ static __forceinline__ double atan2_(double y, double x) { return atan2(y, x); }
    __device__ static __forceinline__ double sqrt_(double x) { return sqrt(x); }
    __device__ static __forceinline__ double log_(double x) { return log(x); }
    __device__ static __forceinline__ double div_(double a, double b) { return a / b; }
    __device__ static __forceinline__ double pi() { return 3.14159265358979323846; }
    __device__ static __forceinline__ double fma_(double a, double b, double c) { return __fma_rn(a, b, c); }
};

template <> struct Math<float> {
    static constexpr bool f32 = true;
    // ((w >> 9) + 1/2) 2^-23 = (w >> 9) 2^-23 + 2^-24: exact, so one fma gives it
    __device__ static __forceinline__ float unif(uint32_t w) { return __fmaf_rn((float)(w >> 9), 0x1p-23f, 0x1p-24f); }
    __device__ static __forceinline__ float sunif(uint32_t w) { return ((float)((int32_t)w >> 9) + 0.5f) * 0x1p-22f; }
    __device__ static __forceinline__ void sincos_rad(float x, float* s, float* c) {
        const float r = x * 0.15915494309189535f;
        *s = __builtin_amdgcn_sinf(r);
        *c = __builtin_amdgcn_cosf(r);
    }
    // sin and cos of (pi/2) v, |v| < 1.  cos(pi v/2) = sin(pi (1 - |v|)/2) is
    // taken as a sine of the exact complement (v is a multiple of 2^-23), so a
    // small cosine keeps its relative accuracy: the proposal 2 atan2(q s, c)
    // amplifies the error of c by ~2/q, large at large coupling.
    __device__ static __forceinline__ void sincos_halfpi(float v, float* s, float* c) {
        const float r = 0.25f * v;
        *s = __builtin_amdgcn_sinf(r);
        *c = __builtin_amdgcn_sinf(0.25f - __builtin_fabsf(r));
    }
    // the same for v = sunif(w): the angle in revolutions, 0.25 ((w >> 9) + 1/2) 2^-22
    // = (w >> 9) 2^-24 + 2^-25, is exact and one fma from the integer
    __device__ static __forceinline__ void sincos_halfpi_w(uint32_t w, float* s, float* c) {
        const float r = __fmaf_rn((float)((int32_t)w >> 9), 0x1p-24f, 0x1p-25f);
        *s = __builtin_amdgcn_sinf(r);
        *c = __builtin_amdgcn_sinf(0.25f - __builtin_fabsf(r));
    }
    // atan2 from explicit instructions (the library version lowers its internal
    // division differently per call site, which changes last bits between
    // kernel instantiations): a = min/max by v_rcp_f32, atan(a) = a P(a^2)
    // with an odd degree-17 minimax polynomial on [0, 1] (fitted by Lawson's
    // iteration; max error 1.03e-7 rad in single precision), then octants.
    __device__ static __forceinline__ float atan2_(float y, float x) {
        const float ax = __builtin_fabsf(x), ay = __builtin_fabsf(y);
        const float mx = __builtin_fmaxf(ax, ay), mn = __builtin_fminf(ax, ay);
        const float a = mx > 0.f ? mn * __builtin_amdgcn_rcpf(mx) : 0.f;
        const float s = a * a;
        float p = 0.0024567251093685627f;
        p = __fmaf_rn(p, s, -0.014401360414922237f);
        p = __fmaf_rn(p, s, 0.039781227707862854f);
        p = __fmaf_rn(p, s, -0.07234857976436615f);
        p = __fmaf_rn(p, s, 0.10498946160078049f);
        p = __fmaf_rn(p, s, -0.14161229133605957f);
        p = __fmaf_rn(p, s, 0.19985906779766083f);
        p = __fmaf_rn(p, s, -0.33332598209381104f);
        p = __fmaf_rn(p, s, 0.9999998807907104f);
        float r = a * p;
        if (ay > ax) r = 1.57079632679489662f - r;
        if (x < 0.f) r = 3.14159265358979324f - r;
        return y < 0.f ? -r : r;
    }
    __device__ static __forceinline__ float sqrt_(float x) { return __builtin_amdgcn_sqrtf(x); }
    __device__ static __forceinline__ float log_(float x) { return __logf(x); }
    __device__ static __forceinline__ float div_(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
    __device__ static __forceinline__ float pi() { return 3.14159265f; }
    __device__ static __forceinline__ float fma_(float a, float b, float c) { return __fmaf_rn(a, b, c); }
};

// a b - c d and a b + c d with one rounding of the first product (explicit
// fused multiply-add: the kernels are compiled without contraction so that
// every instantiation performs identical operations).
template <typename T>
__device__ __forceinline__ T fms2(T a, T b, T c, T d) { return Math<T>::fma_(a, b, -(c * d)); }
template <typename T>
__device__ __forceinline__ T fma2(T a, T b, T c, T d) { return Math<T>::fma_(a, b, c * d); }

// Blocks are dispatched round-robin over the 8 XCDs; remap so that each XCD
// works on a contiguous range of logical blocks (neighbouring tiles of a chain
// share that XCD's L2).
__device__ __forceinline__ int xcd_remap(int b, int nb) {
    const int per = nb >> 3, rem = nb & 7;
    const int xcd = b & 7, idx = b >> 3;
    return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

// exact n / d for n < 2^32 / d via a precomputed m = ceil(2^32 / d)
__device__ __forceinline__ uint32_t fdiv(uint32_t n, uint32_t m) { return __umulhi(n, m); }

}  // namespace llr
