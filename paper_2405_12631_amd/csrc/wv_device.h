// Device functions shared by several kernels.  Each computes its values with
// one fixed sequence of FP32 operations, so the encoder's and the decoder's
// kernels produce identical bits from identical inputs.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/wv.h"

namespace wv {

// The same pointer in the global address space, so that accesses through it
// compile to global_* instructions.  A pointer read from memory (a segment
// descriptor) is otherwise generic and its accesses flat_*, which count against
// the LDS wait counter as well: every wait for an LDS read in an MFMA loop would
// then also wait for the HBM loads in flight.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gmem(T* p) {
    return (__attribute__((address_space(1))) T*)p;
}
// Loads and stores of the HIP vector structs (uint4, float4, ...) through such a
// pointer, moved as a plain vector of 32-bit words.
template <class T>
__device__ __forceinline__ T ld_g(const T* p) {
    typedef uint32_t W __attribute__((ext_vector_type(sizeof(T) / 4)));
    return __builtin_bit_cast(T, *gmem(reinterpret_cast<const W*>(p)));
}
template <class T>
__device__ __forceinline__ void st_g(T* p, const T& v) {
    typedef uint32_t W __attribute__((ext_vector_type(sizeof(T) / 4)));
    *gmem(reinterpret_cast<W*>(p)) = __builtin_bit_cast(W, v);
}

// tanh x = 1 - 2 / (e^{2x} + 1) and the logistic 1 / (1 + e^{-x}) from the
// hardware exponential and reciprocal: absolute error about 1e-7, the exact
// limits for large |x| (e^{2x} overflowing to inf gives 1, underflowing to 0
// gives -1).
__device__ __forceinline__ float tanh_fast(float x) {
    return 1.0f - 2.0f * __builtin_amdgcn_rcpf(1.0f + __expf(2.0f * x));
}
__device__ __forceinline__ float sigmoid_fast(float x) { return __builtin_amdgcn_rcpf(1.0f + __expf(-x)); }

// Mixture head (Sec. 3.1 / 3.2 entropy parameters): raw 3K values ->
// w = softmax(v[0:K]), mu = v[K:2K], sigma = max(softplus(v[2K:3K]), sigma_min).
template <class OutPtr>
__device__ __forceinline__ void mixture_head(const float* v, int K, float sigma_min, OutPtr o) {
    float mx = v[0];
    for (int k = 1; k < K; ++k) mx = fmaxf(mx, v[k]);
    float e[4];
    float se = 0.f;
    for (int k = 0; k < K; ++k) {
        e[k] = __expf(v[k] - mx);
        se += e[k];
    }
    for (int k = 0; k < K; ++k) o[k] = e[k] / se;
    for (int k = 0; k < K; ++k) o[K + k] = v[K + k];
    for (int k = 0; k < K; ++k) {
        const float x = v[2 * K + k];
        const float sp = log1pf(__expf(-fabsf(x))) + fmaxf(x, 0.f);
        o[2 * K + k] = fmaxf(sp, sigma_min);
    }
}

// One row of the 16-bit CDF table (see wv_cdf_tables): setup from the
// parameters, then F_j before the running maximum.
template <int K, int DIST>
struct CdfRow {
    float w[K], mu[K], rs[K];   // weights, means, reciprocal scales
    float invS;
    int jlo, jhi, Fmax, smin;
};

// Smaller tail of a standard component at |z|: Gaussian 0.5 erfc(|z|/sqrt 2),
// Laplace 0.5 exp(-|z|).
template <int DIST>
__device__ __forceinline__ float tail_of(float az) {
    return DIST == WV_DIST_GAUSS ? 0.5f * erfcf(az * 0.70710678118654752f) : 0.5f * expf(-az);
}

template <int K, int DIST>
__device__ __forceinline__ void cdf_setup(const float* p, int smin, int nsym, CdfRow<K, DIST>& R) {
    // Beyond TZ scales every component's tail is below 1/F_max (F_max <= 2^16 - 2):
    // Gaussian 4.5 (Phi(-4.5) = 3.4e-6, at most 0.23 counts), Laplace 11
    // (exp(-11)/2 = 8.4e-6, at most 0.55 counts).  There floor(F_max C_j) is 0 below
    // the window and the upper-tail form gives F_max - 1 above it.
    constexpr float TZ = DIST == WV_DIST_GAUSS ? 4.5f : 11.0f;
    float S = 0.f, lo = 3.0e38f, hi = -3.0e38f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const float sg = p[2 * K + k];
        R.w[k] = p[k];
        R.mu[k] = p[K + k];
        R.rs[k] = 1.0f / sg;
        S += R.w[k];
        lo = fminf(lo, R.mu[k] - TZ * sg);
        hi = fmaxf(hi, R.mu[k] + TZ * sg);
    }
    R.invS = 1.0f / S;
    R.Fmax = 65536 - nsym;
    R.smin = smin;
    // Boundary b_j = smin + j - 0.5.  j < jlo: b_j <= lo; j > jhi: b_j >= hi.
    R.jlo = (int)fminf(fmaxf(floorf(lo - (float)smin + 0.5f) + 1.0f, 1.0f), (float)nsym);
    R.jhi = (int)fminf(fmaxf(ceilf(hi - (float)smin + 0.5f) - 1.0f, 0.0f), (float)(nsym - 1));
}

// F_j = floor(F_max C_j) as in exact arithmetic (lower tail where C_j <= 1/2, else
// F_max - ceil(F_max (1 - C_j)) with at least one count below F_max).
// Inside the window (jlo <= j <= jhi).
template <int K, int DIST>
__device__ __forceinline__ int cdf_F_in(const CdfRow<K, DIST>& R, int j) {
    const float b = (float)(R.smin + j) - 0.5f;
    float L = 0.f, U = 0.f;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        const float z = (b - R.mu[k]) * R.rs[k];
        const float tail = tail_of<DIST>(fabsf(z));
        if (z < 0.f) {
            L = fmaf(R.w[k], tail, L);
            U = fmaf(R.w[k], 1.0f - tail, U);
        } else {
            L = fmaf(R.w[k], 1.0f - tail, L);
            U = fmaf(R.w[k], tail, U);
        }
    }
    L *= R.invS;
    U *= R.invS;
    if (L <= U) return (int)floorf((float)R.Fmax * L);
    const int up = (int)ceilf((float)R.Fmax * U);
    return R.Fmax - (up < 1 ? 1 : up);
}

template <int K, int DIST>
__device__ __forceinline__ int cdf_F(const CdfRow<K, DIST>& R, int j) {
    if (j < R.jlo) return 0;
    if (j > R.jhi) return R.Fmax - 1;
    return cdf_F_in<K, DIST>(R, j);
}

}  // namespace wv
