// A whole coding-step stack of the context model (Sec. 3.2: the conv stack of one
// (subband type, step) and its mixture head) in one kernel, BF16 operands and
// activations, FP32 accumulation.  Model shape: 64 channels, three conv3x3
// layers with ReLU (the first one also reads the coded symbols of the earlier
// steps when step >= 1) and the head conv.
//
// Why fused: one 64 -> 64 BF16 conv layer does 288 FLOP per byte of activations
// it reads and writes, below the chip's ~312 FLOP/B balance, so a layer-by-layer
// stack is bound by HBM round trips of its intermediate activations.  Here they
// never leave LDS: a workgroup walks a strip of 58 output columns of one plane
// down its rows and keeps, for each layer input, a ring of 4 rows x 66 columns
// (64 BF16 channels per position).  Only the step's input l_i and the symbols
// come from HBM and only the parameters of the step's positions go back.
//
// Work split (8 waves, two per SIMD; wave w runs on SIMD w mod 4).  A row step is
// 12 units of matrix work (3 layers x 4 blocks of 16 output channels, 64 positions
// each), the head (16 padded output columns) on every other row, and the input loads:
//   SIMD 0: wave 0 layer 0 blocks 0-1, wave 4 the head (all 64 positions) and its epilogue;
//   SIMD 1: wave 1 layer 0 blocks 2-3, wave 5 the input rows and symbols of ring 0;
//   SIMD 2: wave 2 layer 1 blocks 0-1, wave 6 layer 2 blocks 0-1;
//   SIMD 3: wave 3 layer 1 blocks 2-3, wave 7 layer 2 blocks 2-3.
// Each wave keeps its blocks' weight fragments in registers for the whole launch (72
// VGPRs per block: 18 K steps of 32 input channels), so LDS carries only activations.
// A row step ends with one LDS-only workgroup barrier.  In step t layer l computes row
// y0 - 3 - 2 l + t (two rows behind layer l - 1), the loader stores input row y0 - 1 + t,
// and the head computes row y0 - 10 + t; layer 2 writes its row in the step after the
// one that computed it (its waves share SIMDs 2-3 with layer 1, and the deferred write
// overlaps their MFMAs).  Every read of a step therefore sees rows finished in earlier
// steps, and with 4-row rings no slot written in a step is one read in it.
//
// Bits: every output is accumulated with the same MFMA sequence as the
// layer-by-layer kernel (taps 0..8, 32-channel chunks in order, the symbol
// chunk last; the same fragment layout), then the same bias, ReLU and BF16
// rounding, and the head the same epilogue, so both forms give identical
// parameters.
#include "wv_device.h"
#include "wv_internal.h"
#include "wv_rows.h"

namespace wv {
namespace {

constexpr int SW = 64;             // positions a layer computes per row (4 blocks of 16)
constexpr int SLOTS = SW + 2;      // ring columns; slot k is image column c0 - 4 + k
constexpr int PSTR = 128;          // bytes per slot: 64 BF16 channels in 8 chunks of 16 bytes
constexpr int RROW = SLOTS * PSTR;
constexpr int RING = 4 * RROW;
constexpr int NCH = 64;            // channels of every layer input
constexpr int CC = NCH / 32;       // K chunks per tap
constexpr int NK = 9 * CC;         // K steps per layer

struct Item {
    int n, y0, R, c0;
};

__device__ __forceinline__ bool next_item(const StackSeg* segs, int nseg, long long it, long long total, int& si,
                                          Item& I) {
    if (it >= total) return false;
    int lo = 0, hi = nseg;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (segs[mid].item0 <= it) lo = mid; else hi = mid;
    }
    si = lo;
    const StackSeg& S = segs[lo];
    long long local = it - S.item0;
    const int sx = (int)(local % S.strips_x);
    local /= S.strips_x;
    const int sy = (int)(local % S.segs_y);
    I.n = (int)(local / S.segs_y);
    I.y0 = sy * S.seg_rows;
    I.R = min(S.seg_rows, S.h - I.y0);
    I.c0 = sx * (SW - 6);
    return true;
}

// K loop of one row of a layer: positions 0..63 of output row x (slots 1..64) from the
// input ring's rows x - 1, x, x + 1; NBL column blocks of weights in registers.
template <int MBN, int NBL>
__device__ __forceinline__ void row_mfma(const uint8_t* rin, int x, int mb0, const uint4 (&wr)[NK][NBL],
                                         floatx4 (&acc)[MBN][NBL], int lane) {
    const int m = lane & 15;
    const int kk = lane >> 4;
#pragma unroll
    for (int mb = 0; mb < MBN; ++mb)
#pragma unroll
        for (int nb = 0; nb < NBL; ++nb) acc[mb][nb] = floatx4{0.f, 0.f, 0.f, 0.f};
    uint4 a[2][MBN];
    auto load_a = [&](uint4 (&dst)[MBN], int st) {
        const int tap = st / CC, cc = st % CC;
        // blocks mb are 16 slots apart, which keeps slot & 7 and so the chunk swizzle
        const uint8_t* p = rin + ((x - 1 + tap / 3) & 3) * RROW + swz(mb0 * 16 + m + tap % 3, cc * 4 + kk);
#pragma unroll
        for (int mb = 0; mb < MBN; ++mb) dst[mb] = *reinterpret_cast<const uint4*>(p + mb * 16 * PSTR);
    };
    load_a(a[0], 0);
    __builtin_amdgcn_sched_group_barrier(0x100, MBN, 0);
#pragma unroll
    for (int st = 0; st < NK; ++st) {
        if (st + 1 < NK) load_a(a[(st + 1) & 1], st + 1);
#pragma unroll
        for (int mb = 0; mb < MBN; ++mb)
#pragma unroll
            for (int nb = 0; nb < NBL; ++nb) acc[mb][nb] = mfma_bf16(wr[st][nb], a[st & 1][mb], acc[mb][nb]);
        // Keep the next step's fragment reads ahead of this step's MFMAs (two fragment sets
        // live): the latency of an LDS read is then covered by a step of MFMAs.
        if (st + 1 < NK) __builtin_amdgcn_sched_group_barrier(0x100, MBN, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, MBN * NBL, 0);
    }
}

// Symbol chunk of layer 0 (after the taps, as in the layer-by-layer kernel): element j of
// lane group kk is tap 8 kk + j of the symbol channel (taps >= 9 zero).
template <int NBL>
__device__ __forceinline__ void row_sym(const uint16_t (*rs)[SLOTS], int x, const uint4 (&ws)[NBL],
                                        floatx4 (&acc)[4][NBL], int lane) {
    const int m = lane & 15;
    const int kk = lane >> 4;
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
        // All nine taps of position m read by every lane (addresses independent of the lane
        // group), then lane group 0 keeps taps 0..7, group 1 tap 8, groups 2-3 zeros.
        uint16_t v[9];
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) v[tap] = rs[(x - 1 + tap / 3) & 3][mb * 16 + m + tap % 3];
        uint16_t e[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) e[j] = kk == 0 ? v[j] : (kk == 1 && j == 0 ? v[8] : (uint16_t)0);
        const uint4 av = make_uint4(e[0] | ((uint32_t)e[1] << 16), e[2] | ((uint32_t)e[3] << 16),
                                    e[4] | ((uint32_t)e[5] << 16), e[6] | ((uint32_t)e[7] << 16));
#pragma unroll
        for (int nb = 0; nb < NBL; ++nb) acc[mb][nb] = mfma_bf16(ws[nb], av, acc[mb][nb]);
        __builtin_amdgcn_sched_barrier(0);   // one block's symbol reads at a time (register budget)
    }
}

struct Rings {
    uint8_t (*ring)[RING];
    uint16_t (*ring_s)[SLOTS];
    float (*head_st)[17];
};

// One wave's share of every row step (see the work split above): NBL output blocks from
// nb0 of layer l; with LOAD the input rows of ring 0; with HEADH >= 0 the head's
// positions 32 HEADH .. 32 HEADH + 31.  All waves walk the same items and row steps and
// meet at the same barriers.
template <bool SYM, int NBL, bool LOAD, int HEADH, int HEADM = 2, bool DEFER = false>
__device__ __forceinline__ void wave_run(const StackSeg* __restrict__ segs, int nseg, long long total, int l,
                                         int nb0, const Rings& rg) {
    const int lane = lane_id();
    const int col = lane & 15;
    const int rowq = (lane >> 4) * 4;
    constexpr int NV = (SLOTS * 8 + 63) / 64;   // 16-byte pieces per lane of an input row
    constexpr int NBX = NBL > 0 ? NBL : 1;   // array sizes (NBL = 0: no layer duty)
    uint4 wr[NK][NBX];
    uint4 ws[NBX];   // layer 0's symbol-chunk fragments (steps >= 1)
    uint4 wh[NK][1];
    const uint16_t* wcur = nullptr;
    // Accumulators are transposed (weights are the MFMA's first operand): lane holds
    // output channels 4 (lane / 16) .. + 3 of block nb for position lane % 16 of block mb.
    float bias[NBX][4];
    float hbias[4] = {0.f, 0.f, 0.f, 0.f};
    long long it = blockIdx.x;
    int si;
    Item I;
    while (next_item(segs, nseg, it, total, si, I)) {
        const StackSeg& S = segs[si];
        if (S.w16[l] != wcur) {   // every item of a launch uses one step's weights
            wcur = S.w16[l];
            const uint4* wg = reinterpret_cast<const uint4*>(wcur);
            if constexpr (NBL > 0) {
#pragma unroll
                for (int st = 0; st < NK; ++st)
#pragma unroll
                    for (int nb = 0; nb < NBL; ++nb) wr[st][nb] = ld_g(wg + (st * 4 + nb0 + nb) * 64 + lane);
#pragma unroll
                for (int nb = 0; nb < NBL; ++nb)
#pragma unroll
                    for (int k = 0; k < 4; ++k) bias[nb][k] = gmem(S.bias[l])[(nb0 + nb) * 16 + rowq + k];
            }
            if (NBL > 0 && SYM && l == 0) {
                const uint4* wsg = reinterpret_cast<const uint4*>(S.wsym);
#pragma unroll
                for (int nb = 0; nb < NBX; ++nb) ws[nb] = ld_g(wsg + (nb0 + nb) * 64 + lane);
            }
            if (HEADH >= 0) {
                const uint4* hg = reinterpret_cast<const uint4*>(S.w16[3]);
#pragma unroll
                for (int st = 0; st < NK; ++st) wh[st][0] = ld_g(hg + st * 64 + lane);
#pragma unroll
                for (int k = 0; k < 4; ++k) hbias[k] = gmem(S.bias[3])[rowq + k];
            }
        }
        // ---- input rows (64 BF16 channels) and masked symbols of ring 0 ----
        const uint16_t* in = S.in16 + (long long)I.n * S.in_ps;
        const auto sp = gmem(SYM ? S.sym + (long long)I.n * S.sym_ps : reinterpret_cast<const int16_t*>(S.in16));
        uint4 v[NV];
        int16_t sv[2];
        auto load = [&](int row) {
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                const int idx = lane + 64 * k;
                const int slot = idx >> 3;
                const int c = I.c0 - 4 + slot;
                v[k] = make_uint4(0, 0, 0, 0);
                if (idx < SLOTS * 8 && row >= 0 && row < S.h && c >= 0 && c < S.w)
                    v[k] = ld_g(reinterpret_cast<const uint4*>(in + ((long long)row * S.w + c) * NCH + (idx & 7) * 8));
            }
            if (SYM) {
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    const int c = I.c0 - 4 + lane + 64 * k;
                    const int rc = min(max(row, 0), S.h - 1), cc = min(max(c, 0), S.w - 1);
                    sv[k] = sp[(long long)rc * S.w + cc];
                }
            }
        };
        auto store = [&](int row) {
            uint8_t* dst = rg.ring[0] + (row & 3) * RROW;
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                const int idx = lane + 64 * k;
                if (idx < SLOTS * 8) *reinterpret_cast<uint4*>(dst + swz(idx >> 3, idx & 7)) = v[k];
            }
            if (SYM) {
#pragma unroll
                for (int k = 0; k < 2; ++k) {
                    const int slot = lane + 64 * k;
                    const int c = I.c0 - 4 + slot;
                    const bool ok = slot < SLOTS && row >= 0 && row < S.h && c >= 0 && c < S.w &&
                                    (2 * (row & 1) + (c & 1)) < S.step;
                    if (slot < SLOTS) rg.ring_s[row & 3][slot] = f2bf(ok ? (float)sv[k] : 0.f);
                }
            }
        };
        if constexpr (LOAD) {
            for (int r = I.y0 - 4; r <= I.y0 - 2; ++r) {
                load(r);
                store(r);
            }
            load(I.y0 - 1);
        }
        lds_barrier();
        const int T = I.R + 10;
        const int gr = S.step >> 1, gc = S.step & 1;
        floatx4 acc[4][NBX];
        bool pend = false;   // DEFER: a computed row waiting to be written
        int xpend = 0;
        const uint8_t* rin = rg.ring[NBL > 0 ? l : 0];
        uint8_t* rout = rg.ring[NBL > 0 ? l + 1 : 1];
        for (int t = 0; t < T; ++t) {
            if constexpr (LOAD) {
                if (t <= I.R + 4) store(I.y0 - 1 + t);
                if (t <= I.R + 3) load(I.y0 + t);
            }
            // ---- layer l: output row x (a deferred wave writes the row of the previous
            // step first, then computes this step's row into registers) ----
            if constexpr (NBL > 0) {
                const int x = I.y0 - 3 - 2 * l + t;
                const bool active = t >= 3 * l && t <= I.R + 5 + l;
                auto write_row = [&](int xw) {
                    // Lane: position p = 16 mb + lane % 16, channels 16 (nb0 + nb) + 4 (lane / 16)
                    // .. + 3, i.e. 8 bytes of chunk 2 (nb0 + nb) + lane / 32 at byte 8 ((lane / 16) & 1),
                    // swizzled by slot 1 + p (block mb adds 16 slots: swizzle unchanged).  The lane
                    // index is opaque to the loop optimiser here, so these offsets are recomputed
                    // per row instead of being hoisted into registers.
                    int ln = lane;
                    asm volatile("" : "+v"(ln));
                    const int pm = ln & 15, sl = 1 + pm;
                    uint8_t* orow = rout + (xw & 3) * RROW + sl * PSTR + ((ln >> 4) & 1) * 8;
                    const bool rok = xw >= 0 && xw < S.h;
#pragma unroll
                    for (int mb = 0; mb < 4; ++mb) {
                        const int c = I.c0 - 3 + mb * 16 + pm;
                        const bool ok = rok && c >= 0 && c < S.w;
#pragma unroll
                        for (int nb = 0; nb < NBL; ++nb) {
                            float v[4];
#pragma unroll
                            for (int k = 0; k < 4; ++k) v[k] = fmaxf(acc[mb][nb][k] + bias[nb][k], 0.f);
                            uint2 w = make_uint2(f2bf2(v[0], v[1]), f2bf2(v[2], v[3]));
                            if (!ok) w = make_uint2(0u, 0u);
                            const int chunk = 2 * (nb0 + nb) + (ln >> 5);
                            *reinterpret_cast<uint2*>(orow + mb * 16 * PSTR + ((chunk ^ (sl & 7)) << 4)) = w;
                        }
                    }
                };
                if (DEFER && pend) {
                    write_row(xpend);
                    pend = false;
                }
                if (active) {
                    if (x >= 0 && x < S.h) {
                        row_mfma<4, NBL>(rin, x, 0, wr, acc, lane);
                        if (SYM && l == 0) row_sym<NBL>(rg.ring_s, x, ws, acc, lane);
                    }
                    // rows outside the plane are written as zeros (the next layer's padding)
                    if (DEFER) {
                        pend = true;
                        xpend = x;
                    } else {
                        write_row(x);
                    }
                }
            }
            // ---- head: positions 32 HEADH .. + 31 of row xh, then the mixture epilogue ----
            if constexpr (HEADH >= 0) {
                const int xh = I.y0 - 10 + t;
                if (t >= 10 && (xh & 1) == gr) {
                    floatx4 acc[HEADM][1];
                    row_mfma<HEADM, 1>(rg.ring[3], xh, HEADM * HEADH, wh, acc, lane);
#pragma unroll
                    for (int mb = 0; mb < HEADM; ++mb)
#pragma unroll
                        for (int k = 0; k < 4; ++k)
                            rg.head_st[(HEADM * HEADH + mb) * 16 + col][rowq + k] = acc[mb][0][k] + hbias[k];
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    const int p = 16 * HEADM * HEADH + (lane & (16 * HEADM - 1));   // slot p + 1
                    const int c = I.c0 - 3 + p;
                    if (lane < 16 * HEADM && p >= 3 && p < SW - 3 && c < S.w && (c & 1) == gc) {
                        const int wg2 = (S.w - gc + 1) >> 1;
                        const int hg = (S.h - gr + 1) >> 1;
                        const long long gi = (long long)(xh >> 1) * wg2 + (c >> 1);
                        float* o = S.params + ((long long)I.n * hg * wg2 + gi) * 3 * S.K;
                        mixture_head(&rg.head_st[p][0], S.K, S.sigma_min, gmem(o));
                    }
                    __builtin_amdgcn_wave_barrier();
                }
            }
            lds_barrier();
        }
        it += gridDim.x;
    }
}

template <bool SYM>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2))) void stack_bf16_k(
    const StackSeg* __restrict__ segs, int nseg, long long total) {
    __shared__ __attribute__((aligned(16))) uint8_t ring[4][RING];
    __shared__ uint16_t ring_s[4][SLOTS];
    __shared__ float head_st[SW][17];
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);   // uniform: role values in scalar registers
    // Ring edge slots 0 and 65 of the layer outputs are never written; they feed only
    // outputs outside the strip's kept columns, but keep them finite.
    for (int k = tid; k < 4 * 4 * 2 * (PSTR / 4); k += 512) {
        const int r = k / (4 * 2 * (PSTR / 4));
        const int rem = k % (4 * 2 * (PSTR / 4));
        const int row = rem / (2 * (PSTR / 4));
        const int e = rem % (2 * (PSTR / 4));
        const int slot = e < PSTR / 4 ? 0 : SLOTS - 1;
        reinterpret_cast<uint32_t*>(ring[r] + row * RROW + slot * PSTR)[e % (PSTR / 4)] = 0u;
    }
    __syncthreads();
    const Rings rg{ring, ring_s, head_st};
    switch (wave) {   // wave w runs on SIMD w mod 4 (see the work split above)
        case 0: wave_run<SYM, 2, false, -1>(segs, nseg, total, 0, 0, rg); break;
        case 1: wave_run<SYM, 2, false, -1>(segs, nseg, total, 0, 2, rg); break;
        case 2: wave_run<SYM, 2, false, -1>(segs, nseg, total, 1, 0, rg); break;
        case 3: wave_run<SYM, 2, false, -1>(segs, nseg, total, 1, 2, rg); break;
        case 4: wave_run<SYM, 0, false, 0, 4>(segs, nseg, total, 3, 0, rg); break;
        case 5: wave_run<SYM, 0, true, -1>(segs, nseg, total, 0, 0, rg); break;
        case 6: wave_run<SYM, 2, false, -1, 2, true>(segs, nseg, total, 2, 0, rg); break;
        default: wave_run<SYM, 2, false, -1, 2, true>(segs, nseg, total, 2, 2, rg); break;
    }
}

}  // namespace

hipError_t launch_stack_bf16(const StackSeg* segs, int nseg, long long total, int has_sym, int grid,
                             hipStream_t s) {
    if (total <= 0 || nseg <= 0) return hipSuccess;
    if (grid < 1) grid = 1;
    if (has_sym)
        hipLaunchKernelGGL(stack_bf16_k<true>, dim3(grid), dim3(512), 0, s, segs, nseg, total);
    else
        hipLaunchKernelGGL(stack_bf16_k<false>, dim3(grid), dim3(512), 0, s, segs, nseg, total);
    return hipGetLastError();
}

}  // namespace wv
