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
#include "wv_device.h"
#include "wv_internal.h"

namespace wv {
namespace {

constexpr int ROWS = 64;
constexpr int MAXE = 256;   // max entries per row (N_s + 1)

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
        CdfRow<K, DIST> R;
        cdf_setup<K, DIST>(params + row * (3 * K), smin, nsym, R);
        my[0] = 0;
        int F = 0;
        for (int j = 1; j < nsym; ++j) {
            const int Fj = cdf_F<K, DIST>(R, j);
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
