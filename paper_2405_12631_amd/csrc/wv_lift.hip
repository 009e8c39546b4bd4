// Lifting filter end layers and elementwise kernels.
//
// A predict/update filter (Sec. 3.1) is conv(1 -> C), tanh, conv(C -> C),
// tanh, ..., conv(C -> 1).  The C -> C layers run on the MFMA conv kernel;
// the two end layers are thin (one input or one output channel) and run
// here on the vector ALUs, one thread per position.  The last layer also
// applies the lifting update in place of a separate pass:
//   predict: f = z + N(z); update: f = z/2 + N(z); optionally rounded;
//   out = A + sign * f.
#include "wv_device.h"
#include "wv_internal.h"

namespace wv {
namespace {

constexpr int BLK = 256;

inline unsigned nblocks(long long n) { return (unsigned)((n + BLK - 1) / BLK); }

template <int C>
__global__ __launch_bounds__(BLK) void lift_first_k(const VecLayer L, const CView z, int N, int h,
                                                   int w, float* __restrict__ a1) {
    const long long idx = (long long)blockIdx.x * BLK + threadIdx.x;
    const long long total = (long long)N * h * w;
    if (idx >= total) return;
    const int c = (int)(idx % w);
    const long long t = idx / w;
    const int r = (int)(t % h);
    const int n = (int)(t / h);
    const float* zp = z.p + (long long)n * z.ps;
    float zv[9];
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        const int rr = r + tap / 3 - 1;
        const int cc = c + tap % 3 - 1;
        zv[tap] = (rr >= 0 && rr < h && cc >= 0 && cc < w) ? zp[(long long)rr * z.rs + (long long)cc * z.cs]
                                                           : 0.f;
    }
    float* o = a1 + idx * C;
#pragma unroll
    for (int ch = 0; ch < C; ch += 4) {
        float v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            float s = L.bias[ch + j];
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) s = fmaf(L.w[tap * C + ch + j], zv[tap], s);
            v[j] = tanh_fast(s);
        }
        *reinterpret_cast<float4*>(o + ch) = make_float4(v[0], v[1], v[2], v[3]);
    }
}

template <int C>
__global__ __launch_bounds__(BLK) void lift_last_k(const VecLayer L, const float* __restrict__ a2,
                                                  const CView z, const CView A, const View out,
                                                  int N, int h, int w, int predict, float sign,
                                                  int lift_int) {
    const long long idx = (long long)blockIdx.x * BLK + threadIdx.x;
    const long long total = (long long)N * h * w;
    if (idx >= total) return;
    const int c = (int)(idx % w);
    const long long t = idx / w;
    const int r = (int)(t % h);
    const int n = (int)(t / h);
    float s = L.bias[0];
    for (int tap = 0; tap < 9; ++tap) {
        const int rr = r + tap / 3 - 1;
        const int cc = c + tap % 3 - 1;
        if (rr < 0 || rr >= h || cc < 0 || cc >= w) continue;
        const float4* p = reinterpret_cast<const float4*>(a2 + (((long long)n * h + rr) * w + cc) * C);
        const float* wt = L.w + tap * C;
#pragma unroll
        for (int j = 0; j < C / 4; ++j) {
            const float4 v = p[j];
            s = fmaf(wt[4 * j + 0], v.x, s);
            s = fmaf(wt[4 * j + 1], v.y, s);
            s = fmaf(wt[4 * j + 2], v.z, s);
            s = fmaf(wt[4 * j + 3], v.w, s);
        }
    }
    const float zz = z.p[(long long)n * z.ps + (long long)r * z.rs + (long long)c * z.cs];
    float f = predict ? zz + s : 0.5f * zz + s;
    if (lift_int) f = rintf(f);
    const float av = A.p[(long long)n * A.ps + (long long)r * A.rs + (long long)c * A.cs];
    out.p[(long long)n * out.ps + (long long)r * out.rs + (long long)c * out.cs] = av + sign * f;
}

// Depth-wise 3x3 conv: one thread per (position, 4 channels).
__global__ __launch_bounds__(BLK) void dwconv_k(const float* __restrict__ in, const float* __restrict__ w,
                                               const float* __restrict__ b, float* __restrict__ out,
                                               int N, int h, int wd, int C) {
    const int C4 = C / 4;
    const long long idx = (long long)blockIdx.x * BLK + threadIdx.x;
    const long long total = (long long)N * h * wd * C4;
    if (idx >= total) return;
    const int c4 = (int)(idx % C4);
    const long long p = idx / C4;
    const int c = (int)(p % wd);
    const long long t = p / wd;
    const int r = (int)(t % h);
    const int n = (int)(t / h);
    float4 acc = *reinterpret_cast<const float4*>(b + 4 * c4);
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        const int rr = r + tap / 3 - 1, cc = c + tap % 3 - 1;
        if (rr < 0 || rr >= h || cc < 0 || cc >= wd) continue;
        const float4 v = *reinterpret_cast<const float4*>(in + (((long long)n * h + rr) * wd + cc) * C + 4 * c4);
        const float4 k = *reinterpret_cast<const float4*>(w + tap * C + 4 * c4);
        acc.x = fmaf(k.x, v.x, acc.x);
        acc.y = fmaf(k.y, v.y, acc.y);
        acc.z = fmaf(k.z, v.z, acc.z);
        acc.w = fmaf(k.w, v.w, acc.w);
    }
    *reinterpret_cast<float4*>(out + p * C + 4 * c4) = acc;
}

__global__ __launch_bounds__(BLK) void center_u8_k(const uint8_t* __restrict__ x8,
                                                  float* __restrict__ xf, long long n) {
    const long long i = (long long)blockIdx.x * BLK + threadIdx.x;
    if (i < n) xf[i] = (float)x8[i] - 128.0f;
}

__global__ __launch_bounds__(BLK) void quantize_k(const float* __restrict__ y, int16_t* __restrict__ q,
                                                 long long total, long long per_plane, long long n_ll,
                                                 float dL, float dH, int smin, int smax, int* clip) {
    const long long i = (long long)blockIdx.x * BLK + threadIdx.x;
    if (i >= total) return;
    const float d = (i % per_plane) < n_ll ? dL : dH;
    const float v = rintf(y[i] * d);
    const bool out = v < (float)smin || v > (float)smax;
    q[i] = (int16_t)fminf(fmaxf(v, (float)smin), (float)smax);
    if (clip) {
        const unsigned long long m = __ballot(out);
        if (m && (threadIdx.x & 63) == __ffsll((long long)m) - 1) atomicAdd(clip, __popcll(m));
    }
}

__global__ __launch_bounds__(BLK) void dequantize_k(const int16_t* __restrict__ q, float* __restrict__ y,
                                                   long long total, long long per_plane, long long n_ll,
                                                   float dL, float dH) {
    const long long i = (long long)blockIdx.x * BLK + threadIdx.x;
    if (i >= total) return;
    const float d = (i % per_plane) < n_ll ? dL : dH;
    y[i] = (float)q[i] / d;
}

__global__ __launch_bounds__(BLK) void finalize_k(float* __restrict__ x, uint8_t* __restrict__ u8,
                                                 long long n, float offset) {
    const long long i = (long long)blockIdx.x * BLK + threadIdx.x;
    if (i >= n) return;
    const float v = x[i] + offset;
    x[i] = v;
    if (u8) u8[i] = (uint8_t)fminf(fmaxf(rintf(v), 0.f), 255.f);
}

// Step-g lattice of an h x w subband: row-major (r', c') with r = 2r' + g/2, c = 2c' + g%2.
__global__ __launch_bounds__(BLK) void scatter_k(const uint8_t* __restrict__ sym, int16_t* __restrict__ q,
                                                int N, long long q_ps, long long off, int h, int w,
                                                int gr, int gc, int hg, int wg, int smin) {
    const long long i = (long long)blockIdx.x * BLK + threadIdx.x;
    const long long ng = (long long)hg * wg;
    if (i >= (long long)N * ng) return;
    const int n = (int)(i / ng);
    const long long gi = i - (long long)n * ng;
    const int r = 2 * (int)(gi / wg) + gr;
    const int c = 2 * (int)(gi % wg) + gc;
    q[(long long)n * q_ps + off + (long long)r * w + c] = (int16_t)((int)sym[i] + smin);
}

__global__ __launch_bounds__(BLK) void gather_k(const int16_t* __restrict__ q, uint8_t* __restrict__ sym,
                                               int N, long long q_ps, long long off, int h, int w,
                                               int gr, int gc, int hg, int wg, int smin) {
    const long long i = (long long)blockIdx.x * BLK + threadIdx.x;
    const long long ng = (long long)hg * wg;
    if (i >= (long long)N * ng) return;
    const int n = (int)(i / ng);
    const long long gi = i - (long long)n * ng;
    const int r = 2 * (int)(gi / wg) + gr;
    const int c = 2 * (int)(gi % wg) + gc;
    sym[i] = (uint8_t)((int)q[(long long)n * q_ps + off + (long long)r * w + c] - smin);
}

// Temporal Haar lifting of T <= 32 frames; one thread owns one sample of every frame.
__global__ __launch_bounds__(BLK) void thaar_k(float* __restrict__ f, int T, long long n, int inverse) {
    const long long i = (long long)blockIdx.x * BLK + threadIdx.x;
    if (i >= n) return;
    float v[32], o[32];
    for (int t = 0; t < T; ++t) v[t] = f[(long long)t * n + i];
    if (!inverse) {
        // v holds the current low frames (m of them) at v[0..m); highs land at o[m/2..m).
        int m = T;
        while (m > 1) {
            const int hm = m / 2;
            for (int k = 0; k < hm; ++k) {
                const float hh = v[2 * k + 1] - v[2 * k];
                o[hm + k] = hh;
                v[k] = v[2 * k] + 0.5f * hh;
            }
            m = hm;
        }
        o[0] = v[0];
    } else {
        // Subbands [L_J, H_J, H_{J-1} (2), ..., H_1 (T/2)] -> frames.
        float cur[32];
        cur[0] = v[0];
        int m = 1;
        while (m < T) {
            for (int k = 0; k < m; ++k) {
                const float hh = v[m + k];
                const float e = cur[k] - 0.5f * hh;
                o[2 * k] = e;
                o[2 * k + 1] = hh + e;
            }
            m *= 2;
            for (int k = 0; k < m; ++k) cur[k] = o[k];
        }
    }
    for (int t = 0; t < T; ++t) f[(long long)t * n + i] = o[t];
}

// Subband impulse responses: per subband the key max over elements of
// (|q| << 32) | (0xffffffff - pooled cell index): the largest magnitude, and
// among equal magnitudes the first pooled cell in raster order.  atomicMax is
// order-independent, so the result is deterministic.
__global__ __launch_bounds__(BLK) void sir_keys_k(const int16_t* __restrict__ q,
                                                 unsigned long long* __restrict__ keys,
                                                 const SirMeta m) {
    const int i = blockIdx.y;
    const int h = m.h[i], w = m.w[i], sw = m.sw[i];
    const long long n = (long long)h * w;
    unsigned long long best = 0;
    for (long long e = (long long)blockIdx.x * BLK + threadIdx.x; e < n; e += (long long)gridDim.x * BLK) {
        const int r = (int)(e / w), c = (int)(e % w);
        const int v = abs((int)q[m.off[i] + e]);
        const unsigned cell = (unsigned)((r / m.ph) * sw + (c / m.pw));
        const unsigned long long key = ((unsigned long long)v << 32) | (0xffffffffull - cell);
        best = key > best ? key : best;
    }
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long other = __shfl_down(best, o);
        best = other > best ? other : best;
    }
    if ((threadIdx.x & 63) == 0 && best) atomicMax(keys + i, best);
}

// One S x S pyramid per subband: zero except the subband's own cell, which holds
// max |q_i| / Delta.  y: [nsub][S*S] packed in the S x S layout.
__global__ __launch_bounds__(BLK) void sir_pyramid_k(const unsigned long long* __restrict__ keys,
                                                    const SirMeta m, float dL, float dH,
                                                    float* __restrict__ y) {
    const int i = blockIdx.y;
    const int SS = m.S * m.S;
    for (int e = threadIdx.x; e < SS; e += BLK) y[(long long)i * SS + e] = 0.f;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long key = keys[i];
        const float v = (float)(unsigned)(key >> 32);
        const unsigned cell = key ? 0xffffffffu - (unsigned)(key & 0xffffffffull) : 0u;
        y[(long long)i * SS + m.soff[i] + cell] = v / (i == 0 ? dL : dH);
    }
}

// Zero fill with 16-byte stores and a byte tail (a kernel, so that it can sit in a
// captured graph where a memset node would not be replayed reliably).
__global__ __launch_bounds__(BLK) void zero_k(uint8_t* __restrict__ p, size_t bytes) {
    const size_t n16 = bytes >> 4;
    const size_t stride = (size_t)gridDim.x * BLK;
    for (size_t e = (size_t)blockIdx.x * BLK + threadIdx.x; e < n16; e += stride)
        reinterpret_cast<uint4*>(p)[e] = make_uint4(0, 0, 0, 0);
    const size_t t = (n16 << 4) + (size_t)blockIdx.x * BLK + threadIdx.x;
    if (t < bytes && t < (n16 << 4) + 16) p[t] = 0;
}

__global__ void fill_u64_k(unsigned long long* p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

}  // namespace

hipError_t launch_sir_keys(const int16_t* q, unsigned long long* keys, const SirMeta& m,
                           long long max_n, hipStream_t s) {
    hipLaunchKernelGGL(fill_u64_k, dim3(1), dim3(64), 0, s, keys, m.nsub);
    unsigned gx = (unsigned)((max_n + BLK - 1) / BLK);
    if (gx > 1024) gx = 1024;
    if (gx < 1) gx = 1;
    hipLaunchKernelGGL(sir_keys_k, dim3(gx, m.nsub), dim3(BLK), 0, s, q, keys, m);
    return hipGetLastError();
}

hipError_t launch_sir_pyramid(const unsigned long long* keys, const SirMeta& m, float dL, float dH,
                              float* y, hipStream_t s) {
    hipLaunchKernelGGL(sir_pyramid_k, dim3(1, m.nsub), dim3(BLK), 0, s, keys, m, dL, dH, y);
    return hipGetLastError();
}

hipError_t launch_lift_first(const VecLayer& L, CView z, int N, int h, int w, float* a1,
                             hipStream_t s) {
    const long long n = (long long)N * h * w;
    if (n == 0) return hipSuccess;
    if (L.ch == 16)
        hipLaunchKernelGGL(lift_first_k<16>, dim3(nblocks(n)), dim3(BLK), 0, s, L, z, N, h, w, a1);
    else if (L.ch == 32)
        hipLaunchKernelGGL(lift_first_k<32>, dim3(nblocks(n)), dim3(BLK), 0, s, L, z, N, h, w, a1);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_lift_last(const VecLayer& L, const float* a2, CView z, CView A, View out, int N,
                            int h, int w, int predict, float sign, int lift_int, hipStream_t s) {
    const long long n = (long long)N * h * w;
    if (n == 0) return hipSuccess;
    if (L.ch == 16)
        hipLaunchKernelGGL(lift_last_k<16>, dim3(nblocks(n)), dim3(BLK), 0, s, L, a2, z, A, out, N, h,
                           w, predict, sign, lift_int);
    else if (L.ch == 32)
        hipLaunchKernelGGL(lift_last_k<32>, dim3(nblocks(n)), dim3(BLK), 0, s, L, a2, z, A, out, N, h,
                           w, predict, sign, lift_int);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_dwconv(const float* in, const float* w, const float* b, float* out, int N, int h,
                         int w_, int C, hipStream_t s) {
    const long long n = (long long)N * h * w_ * (C / 4);
    if (n == 0) return hipSuccess;
    if (C % 4) return hipErrorInvalidValue;
    hipLaunchKernelGGL(dwconv_k, dim3(nblocks(n)), dim3(BLK), 0, s, in, w, b, out, N, h, w_, C);
    return hipGetLastError();
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
    if (!bytes) return hipSuccess;
    const size_t n16 = (bytes >> 4) + 1;
    const unsigned grid = (unsigned)std::min<size_t>((n16 + BLK - 1) / BLK, 4096);
    hipLaunchKernelGGL(zero_k, dim3(grid), dim3(BLK), 0, s, (uint8_t*)p, bytes);
    return hipGetLastError();
}

hipError_t launch_center_u8(const uint8_t* x8, float* xf, long long n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(center_u8_k, dim3(nblocks(n)), dim3(BLK), 0, s, x8, xf, n);
    return hipGetLastError();
}

hipError_t launch_quantize(const float* y, int16_t* q, int N, long long per_plane, long long n_ll,
                           float dL, float dH, int smin, int smax, int* clip, hipStream_t s) {
    const long long n = (long long)N * per_plane;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(quantize_k, dim3(nblocks(n)), dim3(BLK), 0, s, y, q, n, per_plane, n_ll, dL,
                       dH, smin, smax, clip);
    return hipGetLastError();
}

hipError_t launch_dequantize(const int16_t* q, float* y, int N, long long per_plane, long long n_ll,
                             float dL, float dH, hipStream_t s) {
    const long long n = (long long)N * per_plane;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(dequantize_k, dim3(nblocks(n)), dim3(BLK), 0, s, q, y, n, per_plane, n_ll, dL,
                       dH);
    return hipGetLastError();
}

hipError_t launch_finalize(float* x, uint8_t* u8, long long n, float offset, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(finalize_k, dim3(nblocks(n)), dim3(BLK), 0, s, x, u8, n, offset);
    return hipGetLastError();
}

hipError_t launch_scatter(const uint8_t* sym, int16_t* q, int N, long long q_ps, long long off, int h,
                          int w, int step, int smin, hipStream_t s) {
    const int gr = step >> 1, gc = step & 1;
    const int hg = (h - gr + 1) >> 1, wg = (w - gc + 1) >> 1;
    const long long n = (long long)N * hg * wg;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(scatter_k, dim3(nblocks(n)), dim3(BLK), 0, s, sym, q, N, q_ps, off, h, w, gr,
                       gc, hg, wg, smin);
    return hipGetLastError();
}

hipError_t launch_gather(const int16_t* q, uint8_t* sym, int N, long long q_ps, long long off, int h,
                         int w, int step, int smin, hipStream_t s) {
    const int gr = step >> 1, gc = step & 1;
    const int hg = (h - gr + 1) >> 1, wg = (w - gc + 1) >> 1;
    const long long n = (long long)N * hg * wg;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(gather_k, dim3(nblocks(n)), dim3(BLK), 0, s, q, sym, N, q_ps, off, h, w, gr, gc,
                       hg, wg, smin);
    return hipGetLastError();
}

hipError_t launch_thaar(float* f, float* /*tmp*/, int T, long long n, int inverse, hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (T < 1 || T > 32 || (T & (T - 1))) return hipErrorInvalidValue;
    hipLaunchKernelGGL(thaar_k, dim3(nblocks(n)), dim3(BLK), 0, s, f, T, n, inverse);
    return hipGetLastError();
}

}  // namespace wv
