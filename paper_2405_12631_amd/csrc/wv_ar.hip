// Autoregressive context model of the LL subband (Sec. 3.2, Fig. 4a: LL is
// coded from its own causal spatial context only, one symbol at a time).
//
// Model: the 12 causal neighbours of a 5x5 window (two rows above, two
// positions to the left; zero outside the subband) -> A channels (ReLU) ->
// 1x1 A -> A (ReLU) -> 1x1 A -> 3K -> mixture head.  Every value is produced
// by the device functions below with a fixed FP32 operation order, so the
// encoder (all positions at once, one thread each) and the decoder (one
// wave per plane, one channel per lane) compute identical parameters, and
// the decoder's CDF row is built with the same functions as wv_cdf_tables.
//
// Decoder: the whole raster walk runs on the GPU, entropy decoding included
// (the rANS stream format of wv_rans_decode), so there is no host round trip
// per symbol.  One workgroup of one wave per plane.
#include "wv_device.h"
#include "wv_internal.h"

namespace wv {
namespace {

__constant__ int c_ar_dy[AR_TAPS] = {-2, -2, -2, -2, -2, -1, -1, -1, -1, -1, 0, 0};
__constant__ int c_ar_dx[AR_TAPS] = {-2, -1, 0, 1, 2, -2, -1, 0, 1, 2, -2, -1};

__device__ __forceinline__ float ar_h1(const float* W1, const float* b1, int k, const float* nb) {
    float s = b1[k];
#pragma unroll
    for (int t = 0; t < AR_TAPS; ++t) s = fmaf(W1[k * AR_TAPS + t], nb[t], s);
    return fmaxf(s, 0.f);
}

template <int A>
__device__ __forceinline__ float ar_h2(const float* W2, const float* b2, int k, const float* h1) {
    float s = b2[k];
#pragma unroll 8
    for (int j = 0; j < A; ++j) s = fmaf(W2[k * A + j], h1[j], s);
    return fmaxf(s, 0.f);
}

template <int A>
__device__ __forceinline__ float ar_out(const float* W3, const float* b3, int o, const float* h2) {
    float s = b3[o];
#pragma unroll 8
    for (int j = 0; j < A; ++j) s = fmaf(W3[o * A + j], h2[j], s);
    return s;
}

// Encoder side: parameters of every LL position from the known symbols.
template <int A>
__global__ __launch_bounds__(64) void ar_params_k(const ArModel M, const int16_t* __restrict__ q,
                                                 long long q_ps, int h, int w, int N,
                                                 float* __restrict__ params) {
    const long long idx = (long long)blockIdx.x * 64 + threadIdx.x;
    const long long nper = (long long)h * w;
    if (idx >= (long long)N * nper) return;
    const int n = (int)(idx / nper);
    const int p = (int)(idx - (long long)n * nper);
    const int r = p / w, c = p % w;
    const int16_t* qp = q + (long long)n * q_ps;
    float nb[AR_TAPS];
#pragma unroll
    for (int t = 0; t < AR_TAPS; ++t) {
        const int rr = r + c_ar_dy[t], cc = c + c_ar_dx[t];
        nb[t] = (rr >= 0 && cc >= 0 && cc < w) ? (float)qp[rr * w + cc] : 0.f;
    }
    float h1[A], h2[A], raw[12];
    for (int k = 0; k < A; ++k) h1[k] = ar_h1(M.w1, M.b1, k, nb);
    for (int k = 0; k < A; ++k) h2[k] = ar_h2<A>(M.w2, M.b2, k, h1);
    for (int o = 0; o < 3 * M.K; ++o) raw[o] = ar_out<A>(M.w3, M.b3, o, h2);
    mixture_head(raw, M.K, M.sigma_min, params + idx * 3 * M.K);
}

// Decoder: one wave per plane walks LL in raster order.
template <int A, int K, int DIST>
__global__ __launch_bounds__(64) void ar_decode_k(const ArModel M, const ArStreams S, int16_t* __restrict__ q,
                                                 long long q_ps, int h, int w, int smin, int nsym,
                                                 int* __restrict__ status) {
    constexpr uint32_t RL = 1u << 23;
    __shared__ float sw1[A * AR_TAPS], sb1[A], sw2[A * A], sb2[A], sw3[3 * K * A], sb3[3 * K];
    __shared__ float nb[AR_TAPS], h1[A], h2[A], raw[3 * K], prm[3 * K];
    __shared__ int Fj[256];
    __shared__ int sym_sh;
    extern __shared__ float rows3[];   // last three LL rows as floats, [3][w]
    const int lane = threadIdx.x;
    const int n = blockIdx.x;
    for (int i = lane; i < A * AR_TAPS; i += 64) sw1[i] = M.w1[i];
    for (int i = lane; i < A * A; i += 64) sw2[i] = M.w2[i];
    for (int i = lane; i < 3 * K * A; i += 64) sw3[i] = M.w3[i];
    for (int i = lane; i < A; i += 64) {
        sb1[i] = M.b1[i];
        sb2[i] = M.b2[i];
    }
    if (lane < 3 * K) sb3[lane] = M.b3[lane];
    const uint8_t* in = S.bytes + S.offs[n];
    const long long len = S.offs[n + 1] - S.offs[n];
    int16_t* qp = q + (long long)n * q_ps;
    uint32_t x = 0;
    long long pos = 4;
    int bad = 0;
    if (lane == 0) {
        if (len < 4) {
            bad = 1;
        } else {
            x = (uint32_t)in[0] | ((uint32_t)in[1] << 8) | ((uint32_t)in[2] << 16) | ((uint32_t)in[3] << 24);
            if (x < RL) bad = 1;
        }
    }
    __syncthreads();
    const long long npos = (long long)h * w;
    for (long long p = 0; p < npos; ++p) {
        const int r = (int)(p / w), c = (int)(p % w);
        if (lane < AR_TAPS) {
            const int rr = r + c_ar_dy[lane], cc = c + c_ar_dx[lane];
            nb[lane] = (rr >= 0 && cc >= 0 && cc < w) ? rows3[(rr % 3) * w + cc] : 0.f;
        }
        __syncthreads();
        if (lane < A) h1[lane] = ar_h1(sw1, sb1, lane, nb);
        __syncthreads();
        if (lane < A) h2[lane] = ar_h2<A>(sw2, sb2, lane, h1);
        __syncthreads();
        if (lane < 3 * K) raw[lane] = ar_out<A>(sw3, sb3, lane, h2);
        __syncthreads();
        if (lane == 0) mixture_head(raw, K, M.sigma_min, prm);
        __syncthreads();
        CdfRow<K, DIST> R;
        cdf_setup<K, DIST>(prm, smin, nsym, R);
        for (int j = 1 + lane; j < nsym; j += 64) Fj[j] = cdf_F<K, DIST>(R, j);
        __syncthreads();
        if (lane == 0) {
            int s = 0;
            if (!bad) {
                // cdf[j] = j + running max of F; find s with cdf[s] <= slot < cdf[s + 1].
                const uint32_t slot = x & 0xffffu;
                int F = 0;
                uint32_t start = 0, end = 65536;
                for (int j = 1; j <= nsym; ++j) {
                    uint32_t cj;
                    if (j < nsym) {
                        F = Fj[j] > F ? Fj[j] : F;
                        cj = (uint32_t)(j + F);
                    } else {
                        cj = 65536u;
                    }
                    if (cj > slot) {
                        s = j - 1;
                        end = cj;
                        break;
                    }
                    start = cj;
                }
                if (end <= start) {
                    bad = 1;
                } else {
                    x = (end - start) * (x >> 16) + slot - start;
                    while (x < RL) {
                        if (pos >= len) {
                            bad = 1;
                            break;
                        }
                        x = (x << 8) | in[pos++];
                    }
                }
            }
            sym_sh = s;
            qp[(long long)r * w + c] = (int16_t)(s + smin);
            rows3[(r % 3) * w + c] = (float)(s + smin);
        }
        __syncthreads();
    }
    if (lane == 0) status[n] = (bad || x != RL || pos != len) ? 1 : 0;
}

}  // namespace

hipError_t launch_ar_params(const ArModel& M, const int16_t* q, long long q_ps, int h, int w, int N,
                            float* params, hipStream_t s) {
    const long long n = (long long)N * h * w;
    if (n == 0) return hipSuccess;
    const unsigned g = (unsigned)((n + 63) / 64);
    if (M.A == 32)
        hipLaunchKernelGGL(ar_params_k<32>, dim3(g), dim3(64), 0, s, M, q, q_ps, h, w, N, params);
    else if (M.A == 64)
        hipLaunchKernelGGL(ar_params_k<64>, dim3(g), dim3(64), 0, s, M, q, q_ps, h, w, N, params);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_ar_decode(const ArModel& M, const ArStreams& S, int16_t* q, long long q_ps, int h,
                            int w, int N, int smin, int nsym, int* status, hipStream_t s) {
    if (N == 0) return hipSuccess;
    if (nsym > 255 || w > 4096) return hipErrorInvalidValue;
    const size_t lds = (size_t)3 * w * sizeof(float);
#define WV_AR_CASE(AA, KK, DD)                                                                   \
    if (M.A == AA && M.K == KK && M.dist == DD) {                                                 \
        hipLaunchKernelGGL((ar_decode_k<AA, KK, DD>), dim3(N), dim3(64), lds, s, M, S, q, q_ps, h, w, \
                           smin, nsym, status);                                                   \
        return hipGetLastError();                                                                 \
    }
    WV_AR_CASE(32, 1, 0) WV_AR_CASE(32, 2, 0) WV_AR_CASE(32, 3, 0) WV_AR_CASE(32, 4, 0)
    WV_AR_CASE(32, 1, 1) WV_AR_CASE(32, 2, 1) WV_AR_CASE(32, 3, 1) WV_AR_CASE(32, 4, 1)
    WV_AR_CASE(64, 1, 0) WV_AR_CASE(64, 2, 0) WV_AR_CASE(64, 3, 0) WV_AR_CASE(64, 4, 0)
    WV_AR_CASE(64, 1, 1) WV_AR_CASE(64, 2, 1) WV_AR_CASE(64, 3, 1) WV_AR_CASE(64, 4, 1)
#undef WV_AR_CASE
    return hipErrorInvalidValue;
}

}  // namespace wv
