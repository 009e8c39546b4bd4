// Discretised mixture (Gaussian or Laplacian components) -> 16-bit integer CDF tables.
//
// Row n (one coefficient) has N_s + 1 entries cdf[j] = j + F_j with
// F_j = floor(F_max * C_j), C_j the normalised mixture CDF at the boundary
// sym_min + j - 0.5, F_max = 2^16 - N_s; entry N_s (= 2^16) is stored as 0.
// The exact value of the floor is produced:
//   * outside [j_lo, j_hi], where every component is at least TZ scales away
//     from the boundary (TZ = 4.5 Gaussian, 11 Laplace), the value is known
//     without evaluating Phi: C_j <= Phi(-TZ) < 1/F_max gives F_j = 0 below,
//     and 0 < 1 - C_j < 1/F_max gives F_j = F_max - 1 above;
//   * inside, the lower tail sum is used when C_j <= 1/2, else the upper tail
//     (F_j = F_max - ceil(F_max * (1 - C_j)), at least one count below F_max),
//     so no digits are lost to 1 - tiny rounding to 1;
//   * a running maximum makes the row non-decreasing.
// A workgroup builds 64 rows in LDS, one thread per row, or (launches too small to
// fill the GPU, where one thread's 128 serial entries set the time) LPR lanes per
// row, each a contiguous slice of the entries, the running maximum completed by a
// prefix maximum over the row's lanes; either way the 64 rows are then written out
// as one contiguous, coalesced block, and the tables are the same.
#include "wv_device.h"
#include "wv_internal.h"

#include <mutex>

namespace wv {
namespace {

constexpr int ROWS = 64;
constexpr int MAXE = 256;   // max entries per row (N_s + 1)

template <int K, int DIST, int LPR>
__global__ __launch_bounds__(ROWS * LPR) void cdf_k(const float* __restrict__ params, long long n, int smin,
                                                   int nsym, uint16_t* __restrict__ out) {
    extern __shared__ __attribute__((aligned(16))) uint16_t rows[];   // [ROWS][nsym + 1]
    const int t = threadIdx.x / LPR;   // row of this lane in the block
    const int sl = threadIdx.x % LPR;  // its slice of the row's entries
    const int E = nsym + 1;
    const long long row0 = (long long)blockIdx.x * ROWS;
    const long long row = row0 + t;
    const int nrows = (int)((n - row0) < ROWS ? (n - row0) : ROWS);
    uint16_t* my = rows + t * E;
    // entries j = 1 .. nsym - 1 in LPR contiguous slices
    const int per = (nsym - 1 + LPR - 1) / LPR;
    const int ja = 1 + sl * per;
    const int jb = ja + per < nsym ? ja + per : nsym;
    int F = 0;
    if (row < n) {
        CdfRow<K, DIST> R;
        cdf_setup<K, DIST>(params + row * (3 * K), smin, nsym, R);
        // The slice in three runs, each lane with its own bounds, so a wave steps through
        // its longest window rather than the union of its rows' windows: F = 0 below the
        // window, evaluated inside it (running maximum within the slice), F_max - 1 above.
        const int j1 = min(max(R.jlo, ja), jb);
        const int j2 = max(min(R.jhi + 1, jb), j1);
        for (int j = ja; j < j1; ++j) my[j] = (uint16_t)(LPR > 1 ? 0 : j);
        for (int j = j1; j < j2; ++j) {
            const int Fj = cdf_F_in<K, DIST>(R, j);
            F = Fj > F ? Fj : F;
            my[j] = (uint16_t)(LPR > 1 ? F : j + F);
        }
        if (j2 < jb) F = max(F, R.Fmax - 1);
        for (int j = j2; j < jb; ++j) my[j] = (uint16_t)(LPR > 1 ? F : j + F);
    }
    if constexpr (LPR > 1) {
        // Maximum of F over the slices before this one: inclusive max-scan over the row's
        // lanes, shifted by one (F >= 0, so 0 is neutral).
        int incl = F;
#pragma unroll
        for (int d = 1; d < LPR; d <<= 1) {
            const int o = __shfl_up(incl, d, LPR);
            if (sl >= d) incl = o > incl ? o : incl;
        }
        int pre = __shfl_up(incl, 1, LPR);
        if (sl == 0) pre = 0;
        if (row < n)
            for (int j = ja; j < jb; ++j) {
                const int f = my[j];
                my[j] = (uint16_t)(j + (f > pre ? f : pre));
            }
    }
    if (row < n && sl == 0) {
        my[0] = 0;
        my[nsym] = 0;   // 2^16 mod 2^16
    }
    __syncthreads();
    // Contiguous copy of this block's rows.
    uint16_t* dst = out + row0 * E;
    const long long nel = (long long)nrows * E;
    if ((((uintptr_t)dst) & 15) == 0 && (nel & 7) == 0) {
        const uint4* src4 = reinterpret_cast<const uint4*>(rows);
        uint4* dst4 = reinterpret_cast<uint4*>(dst);
        for (long long i = threadIdx.x; i < nel / 8; i += ROWS * LPR) dst4[i] = src4[i];
    } else {
        for (long long i = threadIdx.x; i < nel; i += ROWS * LPR) dst[i] = rows[i];
    }
}

}  // namespace

hipError_t launch_cdf(const float* params, long long n, int K, int dist, int smin, int nsym,
                      uint16_t* cdf, hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (nsym + 1 > MAXE || nsym < 2) return hipErrorInvalidValue;
    const unsigned g = (unsigned)((n + ROWS - 1) / ROWS);
    const size_t lds = ((size_t)ROWS * (nsym + 1) * sizeof(uint16_t) + 15) & ~(size_t)15;
    // One lane per row once the launch has more than ~4 waves per SIMD of rows; below that
    // the serial row length sets the time and 4 lanes per row take a quarter of it each.
    const bool split = n <= 256ll * 1024;
#define WV_CDF_CASE(KK, DD)                                                                                  \
    if (K == KK && dist == DD) {                                                                             \
        if (split)                                                                                           \
            hipLaunchKernelGGL((cdf_k<KK, DD, 4>), dim3(g), dim3(ROWS * 4), lds, s, params, n, smin, nsym, cdf); \
        else                                                                                                 \
            hipLaunchKernelGGL((cdf_k<KK, DD, 1>), dim3(g), dim3(ROWS), lds, s, params, n, smin, nsym, cdf);     \
        return hipGetLastError();                                                                            \
    }
    WV_CDF_CASE(1, 0) WV_CDF_CASE(2, 0) WV_CDF_CASE(3, 0) WV_CDF_CASE(4, 0)
    WV_CDF_CASE(1, 1) WV_CDF_CASE(2, 1) WV_CDF_CASE(3, 1) WV_CDF_CASE(4, 1)
#undef WV_CDF_CASE
    return hipErrorInvalidValue;
}


// ---- lossless trim of CDF rows (for the copy to the host coder) ----------
// In a row, F_j = cdf[j] - j (j = 1 .. nsym-1) is non-decreasing, 0 below the
// mass window and F_max - 1 above it (F_max = 2^16 - nsym; the upper tail keeps
// at least one count, so F never reaches F_max).  The row is therefore fixed by
// lo = 1 + #{F_j = 0}, len = #{0 < F_j < F_max - 1} and F_lo .. F_{lo+len-1};
// both counts come from binary searches.  Rows go 256 to a block: the first kernel
// writes (lo, len) and the block's sum of len, the second scans the block sums,
// the third writes each row's F values at its offset.
namespace {

__global__ __launch_bounds__(256) void trim_len_k(const uint16_t* __restrict__ cdf, long long n, int nsym,
                                                  uint8_t* __restrict__ lolen, long long* __restrict__ bsum) {
    __shared__ int red[256];
    const long long row = (long long)blockIdx.x * 256 + threadIdx.x;
    int len = 0;
    if (row < n) {
        const uint16_t* r = cdf + row * (nsym + 1);
        const int ftop = 65536 - nsym - 1;   // F_max - 1
        // first j in [1, nsym) with F_j > 0 (nsym if none)
        int a = 1, b = nsym;
        while (a < b) {
            const int mid = (a + b) >> 1;
            if ((int)r[mid] - mid > 0) b = mid; else a = mid + 1;
        }
        const int lo = a;
        // first j in [lo, nsym) with F_j == F_max - 1 (nsym if none)
        b = nsym;
        while (a < b) {
            const int mid = (a + b) >> 1;
            if ((int)r[mid] - mid >= ftop) b = mid; else a = mid + 1;
        }
        len = a - lo;
        lolen[2 * row] = (uint8_t)lo;
        lolen[2 * row + 1] = (uint8_t)len;
    }
    red[threadIdx.x] = len;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) bsum[blockIdx.x] = red[0];
}

// Exclusive scan of nb block sums in place (one workgroup, chunks of 1024).
__global__ __launch_bounds__(1024) void trim_scan_k(long long* __restrict__ bsum, long long nb) {
    __shared__ long long sh[1024];
    long long carry = 0;
    for (long long base = 0; base < nb; base += 1024) {
        const long long i = base + threadIdx.x;
        const long long v = i < nb ? bsum[i] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {   // inclusive Hillis-Steele scan
            const long long add = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
            __syncthreads();
            sh[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < nb) bsum[i] = carry + sh[threadIdx.x] - v;
        const long long tot = sh[1023];
        __syncthreads();
        carry += tot;
    }
}

__global__ __launch_bounds__(256) void trim_write_k(const uint16_t* __restrict__ cdf, long long n, int nsym,
                                                    const uint8_t* __restrict__ lolen,
                                                    const long long* __restrict__ bsum,
                                                    uint16_t* __restrict__ packed) {
    __shared__ int sh[256];
    const long long row = (long long)blockIdx.x * 256 + threadIdx.x;
    const int len = row < n ? lolen[2 * row + 1] : 0;
    sh[threadIdx.x] = len;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const int add = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
        __syncthreads();
        sh[threadIdx.x] += add;
        __syncthreads();
    }
    if (row < n) {
        const long long off = bsum[blockIdx.x] + sh[threadIdx.x] - len;
        const int lo = lolen[2 * row];
        const uint16_t* r = cdf + row * (nsym + 1);
        for (int t = 0; t < len; ++t) packed[off + t] = (uint16_t)(r[lo + t] - (lo + t));
    }
}

}  // namespace

size_t cdf_trim_scratch_bytes(long long n) { return (size_t)((n + 255) / 256) * sizeof(long long); }

// Block sums of the trim for callers that cannot allocate: one array per GPU, held
// until the process ends.  Host code never passes `trim_scratch` itself (in host code
// the name is not a device address); it passes the address hipGetSymbolAddress gives
// for the current device, looked up once per device.
namespace {
__device__ __align__(256) long long trim_scratch[TRIM_STATIC_SCRATCH_BYTES / sizeof(long long)];
std::mutex g_trim_mu;
long long* g_trim_ptr[TRIM_MAX_DEVICES];
}  // namespace

hipError_t cdf_trim_static_scratch(long long** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= TRIM_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_trim_mu);
    if (!g_trim_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(trim_scratch));
        if (e != hipSuccess) return e;
        g_trim_ptr[dev] = static_cast<long long*>(p);
    }
    *out = g_trim_ptr[dev];
    return hipSuccess;
}

hipError_t launch_cdf_trim(const uint16_t* cdf, long long n, int nsym, uint8_t* lolen, uint16_t* packed,
                           long long* scratch, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const long long nb = (n + 255) / 256;
    hipLaunchKernelGGL(trim_len_k, dim3((unsigned)nb), dim3(256), 0, s, cdf, n, nsym, lolen, scratch);
    hipLaunchKernelGGL(trim_scan_k, dim3(1), dim3(1024), 0, s, scratch, nb);
    hipLaunchKernelGGL(trim_write_k, dim3((unsigned)nb), dim3(256), 0, s, cdf, n, nsym, lolen, scratch, packed);
    return hipGetLastError();
}

}  // namespace wv
