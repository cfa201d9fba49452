// Host stand-in for <hip/hip_runtime.h>, used only by the tests: it lets the
// device headers (set-up, lane formulas, Carlson functions) compile as plain C++ so
// that their arithmetic can be checked on a machine without a GPU.
// The hardware reciprocal / square-root / log2 / exp2 builtins map to the correctly
// rounded host operations; with COSMO_HOST_NOISE defined, each result is moved by a
// pseudo-random -1, 0 or +1 ulp, a model of the ~1 ulp hardware approximations.
#pragma once
#include <cmath>
#include <cstdint>
#include <math.h>
#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __constant__
#define __launch_bounds__(x)
#ifdef COSMO_HOST_NOISE
static inline int host_noise_pick() {
    static uint64_t s = 88172645463325252ull; // xorshift64
    s ^= s << 13; s ^= s >> 7; s ^= s << 17;
    return (int)(s % 3) - 1;
}
static inline float host_prim(float v) {
    int k = host_noise_pick();
    return k == 0 ? v : nextafterf(v, k > 0 ? INFINITY : -INFINITY);
}
#else
static inline float host_prim(float v) { return v; }
#endif
static inline float __builtin_amdgcn_sqrtf(float x) { return host_prim(std::sqrt(x)); }
static inline float __builtin_amdgcn_rcpf(float x) { return host_prim(1.0f / x); }
static inline float __builtin_amdgcn_rsqf(float x) { return host_prim(1.0f / std::sqrt(x)); }
static inline float __builtin_amdgcn_logf(float x) { return host_prim(std::log2(x)); }
static inline float __builtin_amdgcn_exp2f(float x) { return host_prim(std::exp2(x)); }
static inline double __builtin_amdgcn_rcp(double x) { return 1.0 / x; }
static inline double __builtin_amdgcn_rsq(double x) { return 1.0 / std::sqrt(x); }
// A host thread is a wave of one lane.
static inline unsigned long long __ballot(int p) { return p ? 1ull : 0ull; }
static inline double __builtin_amdgcn_frexp_mant(double x) { int e; return std::frexp(x, &e); }
static inline int __builtin_amdgcn_frexp_exp(double x) { int e; std::frexp(x, &e); return e; }
static inline double __builtin_amdgcn_ldexp(double x, int e) { return std::ldexp(x, e); }
// the opaque-constant hint of the device build (cmath.hpp: kc) has no host meaning
#define COSMO_KC_OPAQUE(c) ((void)0)
