// Discretised mixture (Gaussian or Laplacian components) -> 16-bit integer CDF tables.
//
// Row n (one coefficient) has N_s + 1 entries cdf[j] = j + F_j with
// F_j = floor(F_max * C_j), C_j the normalised mixture CDF at the boundary
// sym_min + j - 0.5, F_max = 2^16 - N_s; entry N_s (= 2^16) is stored as 0.
// The exact value of the floor is produced:
//   * outside [j_lo, j_hi], where every component is at least TZ scales away
//     from the boundary (TZ = 6 Gaussian, 12 Laplace), the value is known
//     without evaluating Phi: C_j <= Phi(-TZ) < 1/F_max gives F_j = 0 below,
//     and 0 < 1 - C_j < 1/F_max gives F_j = F_max - 1 above;
//   * inside, the lower tail sum is used when C_j <= 1/2, else the upper tail
//     (F_j = F_max - ceil(F_max * (1 - C_j)), at least one count below F_max),
//     so no digits are lost to 1 - tiny rounding to 1;
//   * a running maximum makes the row non-decreasing.
// One thread builds one row in LDS; the 64 rows of a workgroup are then
// written out as one contiguous, coalesced block.
#include "wv_internal.h"

namespace wv {
namespace {

constexpr int ROWS = 64;
constexpr int MAXE = 256;   // max entries per row (N_s + 1)

// Smaller tail of a standard component at |z|: Gaussian 0.5 erfc(|z|/sqrt 2),
// Laplace 0.5 exp(-|z|).  TAILZ: |z| beyond which the tail is < 1/(2^16 F_max)
// scale, i.e. 0 < tail * F_max < 1 (Gaussian 6: 1e-9; Laplace 12: 3e-6).
template <int DIST>
__device__ __forceinline__ float tail_of(float az) {
    return DIST == WV_DIST_GAUSS ? 0.5f * erfcf(az * 0.70710678118654752f) : 0.5f * expf(-az);
}

template <int K, int DIST>
__global__ __launch_bounds__(ROWS) void cdf_k(const float* __restrict__ params, long long n, int smin,
                                             int nsym, uint16_t* __restrict__ out) {
    extern __shared__ __attribute__((aligned(16))) uint16_t rows[];   // [ROWS][nsym + 1]
    const int t = threadIdx.x;
    const int E = nsym + 1;
    const long long row0 = (long long)blockIdx.x * ROWS;
    const long long row = row0 + t;
    const int nrows = (int)((n - row0) < ROWS ? (n - row0) : ROWS);
    uint16_t* my = rows + t * E;
    if (row < n) {
        const float* p = params + row * (3 * K);
        float w[K], mu[K], sg[K];
        float S = 0.f, lo = 3.0e38f, hi = -3.0e38f;
#pragma unroll
        for (int k = 0; k < K; ++k) {
            w[k] = p[k];
            mu[k] = p[K + k];
            sg[k] = p[2 * K + k];
            S += w[k];
            constexpr float TZ = DIST == WV_DIST_GAUSS ? 6.0f : 12.0f;
            lo = fminf(lo, mu[k] - TZ * sg[k]);
            hi = fmaxf(hi, mu[k] + TZ * sg[k]);
        }
        const float invS = 1.0f / S;
        const int Fmax = 65536 - nsym;
        // Boundary b_j = smin + j - 0.5.  j < jlo: b_j <= lo; j > jhi: b_j >= hi.
        const float flo = fminf(fmaxf(floorf(lo - (float)smin + 0.5f) + 1.0f, 1.0f), (float)nsym);
        const float fhi = fminf(fmaxf(ceilf(hi - (float)smin + 0.5f) - 1.0f, 0.0f), (float)(nsym - 1));
        const int jlo = (int)flo;
        const int jhi = (int)fhi;
        my[0] = 0;
        int F = 0;
        for (int j = 1; j < nsym; ++j) {
            int Fj;
            if (j < jlo) {
                Fj = 0;
            } else if (j > jhi) {
                Fj = Fmax - 1;
            } else {
                const float b = (float)(smin + j) - 0.5f;
                float L = 0.f, U = 0.f;
#pragma unroll
                for (int k = 0; k < K; ++k) {
                    const float z = (b - mu[k]) / sg[k];
                    const float tail = tail_of<DIST>(fabsf(z));
                    if (z < 0.f) {
                        L = fmaf(w[k], tail, L);
                        U = fmaf(w[k], 1.0f - tail, U);
                    } else {
                        L = fmaf(w[k], 1.0f - tail, L);
                        U = fmaf(w[k], tail, U);
                    }
                }
                L *= invS;
                U *= invS;
                if (L <= U) {
                    Fj = (int)floorf((float)Fmax * L);
                } else {
                    const int up = (int)ceilf((float)Fmax * U);
                    Fj = Fmax - (up < 1 ? 1 : up);
                }
            }
            F = Fj > F ? Fj : F;
            my[j] = (uint16_t)(j + F);
        }
        my[nsym] = 0;   // 2^16 mod 2^16
    }
    __syncthreads();
    // Contiguous copy of this block's rows.
    uint16_t* dst = out + row0 * E;
    const long long nel = (long long)nrows * E;
    if ((((uintptr_t)dst) & 15) == 0 && (nel & 7) == 0) {
        const uint4* src4 = reinterpret_cast<const uint4*>(rows);
        uint4* dst4 = reinterpret_cast<uint4*>(dst);
        for (long long i = t; i < nel / 8; i += ROWS) dst4[i] = src4[i];
    } else {
        for (long long i = t; i < nel; i += ROWS) dst[i] = rows[i];
    }
}

}  // namespace

hipError_t launch_cdf(const float* params, long long n, int K, int dist, int smin, int nsym,
                      uint16_t* cdf, hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (nsym + 1 > MAXE || nsym < 2) return hipErrorInvalidValue;
    const unsigned g = (unsigned)((n + ROWS - 1) / ROWS);
    const size_t lds = ((size_t)ROWS * (nsym + 1) * sizeof(uint16_t) + 15) & ~(size_t)15;
#define WV_CDF_CASE(KK, DD)                                                                   \
    if (K == KK && dist == DD) {                                                              \
        hipLaunchKernelGGL((cdf_k<KK, DD>), dim3(g), dim3(ROWS), lds, s, params, n, smin, nsym, cdf); \
        return hipGetLastError();                                                             \
    }
    WV_CDF_CASE(1, 0) WV_CDF_CASE(2, 0) WV_CDF_CASE(3, 0) WV_CDF_CASE(4, 0)
    WV_CDF_CASE(1, 1) WV_CDF_CASE(2, 1) WV_CDF_CASE(3, 1) WV_CDF_CASE(4, 1)
#undef WV_CDF_CASE
    return hipErrorInvalidValue;
}

}  // namespace wv
