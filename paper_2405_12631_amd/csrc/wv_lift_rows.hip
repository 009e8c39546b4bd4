// Row-streaming form of one predict/update filter application (Sec. 3.1), for the
// 32-channel filters over large arrays:
//   out = A + sign * f,  f = z + N(z) (predict) or z/2 + N(z) (update),
//   N = conv3x3(32 -> 1) . tanh . conv3x3(32 -> 32) . tanh . conv3x3(1 -> 32),
// every conv zero-padded at the array border.
//
// Why: the tiled kernel (lift_fused_k) recomputes the middle layer on a halo around
// each tile (1.25x-1.5x its outputs) and runs the vector layers and the matrix layer
// one after the other.  Here a workgroup walks a strip of 124 output columns down a
// segment of rows, and keeps each layer's recent rows in LDS rings: the middle layer
// runs on 128 positions per row (126 needed) for 124 outputs, on four waves, and the
// vector layers on the other four (layer 1 on 128 positions: one task per lane).
//
// Per row step t of an item with first output row y0 (one LDS-only barrier per step):
//   vector waves 4-7: store z row y0 - 3 + t (loaded the step before) and load the next;
//                     layer 1 on row y0 - 5 + t (128 positions, 32 channels, tanh);
//                     bias + tanh of the middle layer's row y0 - 8 + t (raw sums from the
//                     MFMA waves); layer 3 and the update on output row y0 - 10 + t
//                     (A and the output of that row read/written by the same lane);
//   MFMA waves 0-3:   middle layer on row y0 - 7 + t, wave w positions 32 w .. 32 w + 31
//                     (two M blocks of 16, both 16-channel output blocks), weights in
//                     registers for the whole launch, raw sums into the layer-2 ring.
// Every read in a step is of rows finished in earlier steps; the rings are large enough
// (z 8 rows, layer 1 4 rows, layer 2 5 rows) that no slot written in a step is read in it.
//
// Bits: each output takes the same arithmetic in the same order as lift_fused_k (the
// layer-1 FMA chain over taps 0..8, the middle layer's MFMA sequence over (tap, 16-channel
// chunk) steps with the same fragment layout, the layer-3 halves summed as there, the
// same tanh), so the two kernels give identical arrays.
#include "wv_device.h"
#include "wv_internal.h"
#include "wv_rows.h"

#include <atomic>

namespace wv {
namespace {

constexpr int LC = 32;            // filter channels
constexpr int NPOS = 128;         // middle-layer positions per row computed: 8 M blocks
constexpr int OUTW = LIFT_ROWS_OUTW;   // output columns per strip (124)
constexpr int A1C = OUTW + 4;     // layer-1 positions computed per row (128: one task per vector lane)
constexpr int A1N = NPOS + 2;     // layer-1 ring slots: the last two feed only unused positions
constexpr int ZN = OUTW + 6;      // z positions per row
constexpr int PB = LC * 4;        // bytes per position in the layer rings (8 chunks of 16 B)
constexpr int R1 = 4, R2 = 5, RZ = 8;
constexpr int NST = 9 * (LC / 16);   // (tap, 16-channel chunk) steps of the middle layer

__device__ __forceinline__ int rmod(int r, int n) { return (r + 8 * n) % n; }   // r >= -8 n

struct Item {
    int n, y0, R, c0;
};
__device__ __forceinline__ Item item_of(long long it, int nstrips, int nseg, int seg_rows, int h) {
    Item I;
    const int strip = (int)(it % nstrips);
    const long long rest = it / nstrips;
    const int seg = (int)(rest % nseg);
    I.n = (int)(rest / nseg);
    I.y0 = seg * seg_rows;
    I.R = min(seg_rows, h - I.y0);
    I.c0 = strip * OUTW;
    return I;
}

struct Smem {
    uint8_t (*a1)[A1N * PB];
    uint8_t (*a2)[NPOS * PB];
    float (*zr)[ZN];
    const float* w1s;
    const float* w3s;
    const float* b1s;
    const float* b2s;
};

// Middle layer, wave w of 0..3.
__device__ __forceinline__ void mfma_role(const MfmaLayer& L2, int h, int w, int nstrips, int nseg, int seg_rows,
                                          long long total, int wv, const Smem& S) {
    const int lane = lane_id();
    const int m = lane & 15, kk = lane >> 4;
    const int col = lane & 15, rowq = (lane >> 4) * 4;
    floatx4 wr[NST][2];
    const floatx4* wg = reinterpret_cast<const floatx4*>(L2.w);
#pragma unroll
    for (int st = 0; st < NST; ++st)
#pragma unroll
        for (int nb = 0; nb < 2; ++nb) wr[st][nb] = wg[(st * 2 + nb) * 64 + lane];
    for (long long it = blockIdx.x; it < total; it += gridDim.x) {
        const Item I = item_of(it, nstrips, nseg, seg_rows, h);
        const int T = I.R + 10;
        // The wave's positions are needed unless all of them lie right of the array.
        const bool need = I.c0 - 1 + 32 * wv < w;
        for (int t = 0; t < T; ++t) {
            const int x = I.y0 - 7 + t;
            if (t >= 6 && t <= I.R + 7 && x >= 0 && x < h && need) {
                floatx4 acc[2][2];
#pragma unroll
                for (int j = 0; j < 2; ++j)
#pragma unroll
                    for (int nb = 0; nb < 2; ++nb) acc[j][nb] = floatx4{0.f, 0.f, 0.f, 0.f};
                const uint8_t* r0 = S.a1[rmod(x - 1, R1)];
                const uint8_t* r1 = S.a1[rmod(x, R1)];
                const uint8_t* r2 = S.a1[rmod(x + 1, R1)];
                floatx4 afr[2][2];
                auto load = [&](int buf, int st) {
                    const int tap = st >> 1, cb = st & 1;
                    const uint8_t* rr = tap < 3 ? r0 : (tap < 6 ? r1 : r2);
                    const int dx = tap % 3;
#pragma unroll
                    for (int j = 0; j < 2; ++j)
                        afr[buf][j] = *reinterpret_cast<const floatx4*>(rr + swz(32 * wv + 16 * j + m + dx, 4 * cb + kk));
                };
                // The four accumulators' chains interleaved: each accumulator takes channel
                // offsets .x, .y, .z, .w of the step in that order.
                auto step = [&](int buf, int st) {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
#pragma unroll
                        for (int j = 0; j < 2; ++j)
#pragma unroll
                            for (int nb = 0; nb < 2; ++nb)
                                acc[j][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(afr[buf][j][e], wr[st][nb][e],
                                                                                 acc[j][nb], 0, 0, 0);
                };
                // The next step's two fragment reads issue ahead of this step's 16 MFMAs, so a
                // step of MFMAs covers their latency.
                load(0, 0);
                __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
#pragma unroll
                for (int st = 0; st < NST; st += 2) {
                    load(1, st + 1);
                    step(0, st);
                    __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
                    __builtin_amdgcn_sched_group_barrier(0x008, 16, 0);
                    if (st + 2 < NST) load(0, st + 2);
                    step(1, st + 1);
                    if (st + 2 < NST) __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
                    __builtin_amdgcn_sched_group_barrier(0x008, 16, 0);
                }
                // raw sums: position 32 wv + 16 j + rowq + i, channel 16 nb + col
                uint8_t* o = S.a2[rmod(x, R2)];
#pragma unroll
                for (int j = 0; j < 2; ++j)
#pragma unroll
                    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            const int p = 32 * wv + 16 * j + rowq + i;
                            const int ch = 16 * nb + col;
                            *reinterpret_cast<float*>(o + swz(p, ch >> 2) + (ch & 3) * 4) = acc[j][nb][i];
                        }
            }
            lds_barrier();
        }
    }
}

// Layer 1, the middle layer's bias and tanh, layer 3 and the update; vector lane v of 0..255.
__device__ __forceinline__ void vec_role(const VecLayer& L3, CView z, CView A, View out, int h, int w, int nstrips,
                                         int nseg, int seg_rows, int predict, float sign, int lift_int, long long total,
                                         int v, const Smem& S) {
    const float b3 = L3.bias[0];
    // This lane's layer-3 weights (its channel half, all taps) stay in registers.
    float4 w3r[9][LC / 8];
#pragma unroll
    for (int tap = 0; tap < 9; ++tap)
#pragma unroll
        for (int k = 0; k < LC / 8; ++k)
            w3r[tap][k] = *reinterpret_cast<const float4*>(S.w3s + tap * LC + (v & 1) * (LC / 2) + 4 * k);
    for (long long it = blockIdx.x; it < total; it += gridDim.x) {
        const Item I = item_of(it, nstrips, nseg, seg_rows, h);
        const int T = I.R + 10;
        const float* zp = z.p + (long long)I.n * z.ps;
        const float* ap = A.p + (long long)I.n * A.ps;
        float* op = out.p + (long long)I.n * out.ps;
        auto zload = [&](int r) {   // z row r at column c0 - 3 + v (lanes 0 .. ZN - 1)
            const int c = I.c0 - 3 + v;
            return (v < ZN && r >= 0 && r < h && c >= 0 && c < w) ? zp[(long long)r * z.rs + (long long)c * z.cs] : 0.f;
        };
        // layer-3 task of this lane: output column c0 + (v >> 1), channel half v & 1
        const int o = v >> 1, half = v & 1;
        const int oc = I.c0 + o;
        const bool owner = half == 0 && v < 2 * OUTW && oc < w;
        auto aload = [&](int r) {
            return (owner && r >= 0 && r < h) ? ap[(long long)r * A.rs + (long long)oc * A.cs] : 0.f;
        };
        float zn = zload(I.y0 - 3);
        float an = 0.f;
        float pend = 0.f;   // the previous step's output value
        for (int t = 0; t < T; ++t) {
            // What the previous step loaded is used before this step issues a global access:
            // loads and stores share one completion counter, so a wait for a load placed after
            // this step's store would also wait for the store.  For the same reason the output
            // is stored one step late, at the top of the next step.
            // ---- z ring: row y0 - 3 + t ----
            if (t <= I.R + 5 && v < ZN) S.zr[rmod(I.y0 - 3 + t, RZ)][v] = zn;
            const float acur = an;   // A of this step's output row
            wait_vm();
            if (t >= 11 && owner) op[(long long)(I.y0 - 11 + t) * out.rs + (long long)oc * out.cs] = pend;
            if (t + 1 <= I.R + 5) zn = zload(I.y0 - 2 + t);
            // ---- A of the next step's output row ----
            if (t + 1 >= 10 && t + 1 <= I.R + 9) an = aload(I.y0 - 9 + t);
            // ---- layer 1 on row y0 - 5 + t: tasks (position a, 16-channel half) ----
            if (t >= 3 && t <= I.R + 6) {
                const int r1 = I.y0 - 5 + t;
                const bool rin = r1 >= 0 && r1 < h;
                uint8_t* dst = S.a1[rmod(r1, R1)];
                const float* z0 = S.zr[rmod(r1 - 1, RZ)];
                const float* z1 = S.zr[rmod(r1, RZ)];
                const float* z2 = S.zr[rmod(r1 + 1, RZ)];
                {
                    const int a = v >> 1, hf = v & 1;   // 2 A1C = 256 tasks
                    static_assert(2 * A1C == 256, "one layer-1 task per vector lane");
                    const int c = I.c0 - 2 + a;
                    float4 res[4];
                    if (rin && c >= 0 && c < w) {
                        float zv[9];
#pragma unroll
                        for (int dx = 0; dx < 3; ++dx) {
                            zv[dx] = z0[a + dx];
                            zv[3 + dx] = z1[a + dx];
                            zv[6 + dx] = z2[a + dx];
                        }
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int c4 = 16 * hf + 4 * q;   // channels c4 .. c4 + 3
                            const float4 b = *reinterpret_cast<const float4*>(S.b1s + c4);
                            float s[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
                            for (int tap = 0; tap < 9; ++tap) {
                                const float4 wt = *reinterpret_cast<const float4*>(S.w1s + tap * LC + c4);
                                s[0] = fmaf(wt.x, zv[tap], s[0]);
                                s[1] = fmaf(wt.y, zv[tap], s[1]);
                                s[2] = fmaf(wt.z, zv[tap], s[2]);
                                s[3] = fmaf(wt.w, zv[tap], s[3]);
                            }
                            res[q] = make_float4(tanh_fast(s[0]), tanh_fast(s[1]), tanh_fast(s[2]), tanh_fast(s[3]));
                        }
                    } else {
#pragma unroll
                        for (int q = 0; q < 4; ++q) res[q] = make_float4(0.f, 0.f, 0.f, 0.f);
                    }
#pragma unroll
                    for (int q = 0; q < 4; ++q) *reinterpret_cast<float4*>(dst + swz(a, 4 * hf + q)) = res[q];
                }
            }
            // ---- middle layer, row y0 - 8 + t: bias and tanh in place (zero outside) ----
            if (t >= 7 && t <= I.R + 8) {
                const int r2 = I.y0 - 8 + t;
                const bool rin = r2 >= 0 && r2 < h;
                uint8_t* row = S.a2[rmod(r2, R2)];
#pragma unroll
                for (int k = 0; k < 4; ++k) {
                    const int idx = v + 256 * k;   // (position, chunk) of 16 B
                    const int p = idx >> 3, q = idx & 7;
                    const int c = I.c0 - 1 + p;
                    float4* ptr = reinterpret_cast<float4*>(row + swz(p, q));
                    float4 x = make_float4(0.f, 0.f, 0.f, 0.f);
                    if (rin && c >= 0 && c < w) {
                        const float4 raw = *ptr;
                        const float4 b = *reinterpret_cast<const float4*>(S.b2s + 4 * q);
                        x = make_float4(tanh_fast(raw.x + b.x), tanh_fast(raw.y + b.y), tanh_fast(raw.z + b.z),
                                        tanh_fast(raw.w + b.w));
                    }
                    *ptr = x;
                }
            }
            // ---- layer 3 and the update on output row y0 - 10 + t ----
            if (t >= 10) {
                const int r3 = I.y0 - 10 + t;
                float s = 0.f;
                if (v < 2 * OUTW) {
#pragma unroll
                    for (int tap = 0; tap < 9; ++tap) {
                        const uint8_t* row = S.a2[rmod(r3 - 1 + tap / 3, R2)];
                        const int p = o + tap % 3;
#pragma unroll
                        for (int k = 0; k < LC / 8; ++k) {
                            const float4 av = *reinterpret_cast<const float4*>(row + swz(p, 4 * half + k));
                            const float4 wv = w3r[tap][k];
                            s = fmaf(wv.x, av.x, s);
                            s = fmaf(wv.y, av.y, s);
                            s = fmaf(wv.z, av.z, s);
                            s = fmaf(wv.w, av.w, s);
                        }
                    }
                }
                const float other = __shfl_xor(s, 1);
                if (owner) {
                    const float vv = b3 + (s + other);
                    const float zz = S.zr[rmod(r3, RZ)][o + 3];
                    float f = predict ? zz + vv : 0.5f * zz + vv;
                    if (lift_int) f = rintf(f);
                    pend = acur + sign * f;
                }
            }
            lds_barrier();
        }
        if (owner) op[(long long)(I.y0 + I.R - 1) * out.rs + (long long)oc * out.cs] = pend;   // t = T - 1
    }
}

__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2))) void lift_rows_k(
    const VecLayer L1, const MfmaLayer L2, const VecLayer L3, const CView z, const CView A, const View out, int h,
    int w, int nstrips, int nseg, int seg_rows, int predict, float sign, int lift_int, long long total) {
    __shared__ __attribute__((aligned(16))) uint8_t a1[R1][A1N * PB];
    __shared__ __attribute__((aligned(16))) uint8_t a2[R2][NPOS * PB];
    __shared__ float zr[RZ][ZN];
    __shared__ __attribute__((aligned(16))) float w1s[9 * LC];
    __shared__ __attribute__((aligned(16))) float w3s[9 * LC];
    __shared__ __attribute__((aligned(16))) float b1s[LC];
    __shared__ __attribute__((aligned(16))) float b2s[LC];
    const int tid = threadIdx.x;
    for (int i = tid; i < 9 * LC; i += 512) {
        w1s[i] = L1.w[i];
        w3s[i] = L3.w[i];
    }
    if (tid < LC) {
        b1s[tid] = L1.bias[tid];
        b2s[tid] = L2.bias[tid];
    }
    __syncthreads();
    const Smem S{a1, a2, zr, w1s, w3s, b1s, b2s};
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    if (wave < 4)
        mfma_role(L2, h, w, nstrips, nseg, seg_rows, total, wave, S);
    else
        vec_role(L3, z, A, out, h, w, nstrips, nseg, seg_rows, predict, sign, lift_int, total, tid - 256, S);
}

}  // namespace

// Rows per item: each item pays 10 row steps of pipeline fill, and a launch takes as many
// rounds of the resident workgroups as its items need, so the number of row segments is the
// one that minimises rounds x (rows per segment + 10).
hipError_t launch_lift_rows(const VecLayer& L1, const MfmaLayer& L2, const VecLayer& L3, CView z, CView A, View out,
                            int N, int h, int w, int nstrips, int predict, float sign, int lift_int, hipStream_t s) {
    if ((long long)N * h * w == 0 || nstrips == 0) return hipSuccess;
    if (nstrips < 0 || (long long)(nstrips - 1) * OUTW >= w) return hipErrorInvalidValue;
    if (L1.ch != LC || L2.cin != LC || L2.nbt != 2) return hipErrorInvalidValue;
    // resident workgroups, cached per device
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    int resident = cache[dev].load(std::memory_order_relaxed);
    if (resident == 0) {
        int per_cu = 0, cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, lift_rows_k, 512, 0) != hipSuccess || per_cu < 1)
            return hipErrorInvalidValue;
        resident = per_cu * cus;
        cache[dev].store(resident, std::memory_order_relaxed);
    }
    const long long cols = (long long)nstrips * N;
    int seg_rows = h;
    long long best = -1;
    for (int ns = 1; ns <= h; ++ns) {
        const int r = (h + ns - 1) / ns;
        const long long items = cols * ((h + r - 1) / r);
        const long long rounds = (items + resident - 1) / resident;
        const long long cost = rounds * (r + 10);
        if (best < 0 || cost < best) {
            best = cost;
            seg_rows = r;
        }
        if (r <= 8) break;
    }
    const int nseg = (h + seg_rows - 1) / seg_rows;
    const long long total = cols * nseg;
    const long long g = total < resident ? total : resident;
    hipLaunchKernelGGL(lift_rows_k, dim3((unsigned)g), dim3(512), 0, s, L1, L2, L3, z, A, out, h, w, nstrips, nseg,
                       seg_rows, predict, sign, lift_int, total);
    return hipGetLastError();
}

}  // namespace wv
