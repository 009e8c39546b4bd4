// The ConvLSTM of the context model (Sec. 3.2: the long-term context l_i is the hidden
// state after subband i) as one row-streaming launch per subband, BF16 operands, FP32
// accumulation and cell state.  Gates = conv3x3 over [q_{i-1}, h_{i-1}] (65 -> 256
// channels), then c = sigma(f) c_prev + sigma(i) tanh(g), h = sigma(o) tanh(c).
//
// A workgroup walks a strip of 64 output columns of one plane down a segment of rows and
// keeps the last 4 input rows (66 columns x 64 BF16 channels, plus the symbols) in an LDS
// ring: in row step t every thread stores its share of input row y0 - 1 + t (loaded the
// step before) and loads the next, and the 8 waves compute output row y0 - 3 + t.  Wave w
// holds in registers, for the whole launch, the weights of 8 channels (its two 16-row
// blocks: 4 channels x 4 gates each); the weights are the MFMA's first operand, so a lane
// ends with the four gates of one channel at one position and applies the cell update
// without any exchange (channels 8 w + 2 q and + 1 for lane group q: the new c and h are
// written as float2 and two BF16).  One LDS-only barrier per row step.
//
// Bits: every gate takes the layer-by-layer kernel's MFMA sequence (taps 0..8, 32-channel
// chunks in order, the symbol chunk last, the same fragment layout), then the same bias,
// activations and cell arithmetic, so both forms give identical h and c.
#include "wv_device.h"
#include "wv_internal.h"
#include "wv_rows.h"

namespace wv {
namespace {

constexpr int SW = LSTM_STRIP;     // output positions per row (4 blocks of 16)
constexpr int SLOTS = SW + 2;      // ring slots: slot k is column c0 - 1 + k
constexpr int PSTR = 128;          // bytes per slot: 64 BF16 channels, 8 chunks of 16 bytes
constexpr int RROW = SLOTS * PSTR;
constexpr int NCH = 64;
constexpr int NK = 18;             // K steps: 9 taps x 2 chunks of 32 channels
constexpr int NBT = 16;            // 16-column blocks of the 256 gate columns
constexpr int NV = SLOTS * 8;      // 16-byte pieces of an input row (528)

// Packed gate column (block, column) of channel ch and gate g: the layer's packing puts
// gate g of channels 16 k .. 16 k + 15 in block 4 k + g.
__device__ __forceinline__ int pblock(int ch, int g) { return 4 * (ch >> 4) + g; }

struct Item {
    int n, y0, R, c0;
};
__device__ __forceinline__ bool next_item(const LstmSeg* segs, int nseg, long long it, long long total, int& si,
                                          Item& I) {
    if (it >= total) return false;
    int lo = 0, hi = nseg;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (segs[mid].item0 <= it) lo = mid; else hi = mid;
    }
    si = lo;
    const LstmSeg& S = segs[lo];
    long long local = it - S.item0;
    const int sx = (int)(local % S.strips_x);
    local /= S.strips_x;
    const int sy = (int)(local % S.segs_y);
    I.n = (int)(local / S.segs_y);
    I.y0 = sy * S.seg_rows;
    I.R = min(S.seg_rows, S.h - I.y0);
    I.c0 = sx * SW;
    return true;
}

// Gate sums of output row x, positions 16 mb0 .. 16 mb0 + 31 (two blocks of 16), for the
// wave's two 16-row weight blocks: the 18 K steps of the taps, then the symbol chunk.
__device__ __forceinline__ void row_gates(const uint8_t* ring, const uint16_t (*rs)[SLOTS], int x, int mb0,
                                          const uint4 (&wr)[NK][2], const uint4 (&ws)[2], floatx4 (&acc)[2][2],
                                          int lane) {
    const int m = lane & 15;
    const int kk = lane >> 4;
#pragma unroll
    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[mb][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    // Fragment reads run two K steps ahead (three sets live): a step is only 4 MFMAs, less
    // than an LDS read's latency.
    uint4 a[3][2];
    auto load_a = [&](uint4 (&dst)[2], int st) {
        const int tap = st >> 1, cc = st & 1;
        // blocks mb are 16 slots apart, which keeps slot & 7 and so the chunk swizzle
        const uint8_t* p = ring + ((x - 1 + tap / 3) & 3) * RROW + swz(mb0 * 16 + m + tap % 3, cc * 4 + kk);
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) dst[mb] = *reinterpret_cast<const uint4*>(p + mb * 16 * PSTR);
    };
    load_a(a[0], 0);
    load_a(a[1], 1);
    __builtin_amdgcn_sched_group_barrier(0x100, 4, 0);
#pragma unroll
    for (int st = 0; st < NK; ++st) {
        if (st + 2 < NK) load_a(a[(st + 2) % 3], st + 2);
#pragma unroll
        for (int mb = 0; mb < 2; ++mb)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[mb][j] = mfma_bf16(wr[st][j], a[st % 3][mb], acc[mb][j]);
        if (st + 2 < NK) __builtin_amdgcn_sched_group_barrier(0x100, 2, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, 4, 0);
    }
    // Symbol chunk: element e of lane group kk is tap 8 kk + e (taps >= 9 zero).
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
        uint16_t v[9];
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) v[tap] = rs[(x - 1 + tap / 3) & 3][(mb0 + mb) * 16 + m + tap % 3];
        uint16_t e[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) e[j] = kk == 0 ? v[j] : (kk == 1 && j == 0 ? v[8] : (uint16_t)0);
        const uint4 av = make_uint4(e[0] | ((uint32_t)e[1] << 16), e[2] | ((uint32_t)e[3] << 16),
                                    e[4] | ((uint32_t)e[5] << 16), e[6] | ((uint32_t)e[7] << 16));
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[mb][j] = mfma_bf16(ws[j], av, acc[mb][j]);
    }
}

__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2))) void lstm_bf16_k(
    const LstmSeg* __restrict__ segs, int nseg, long long total) {
    __shared__ __attribute__((aligned(16))) uint8_t ring[4 * RROW];
    __shared__ uint16_t ring_s[4][SLOTS];
    __shared__ float bias_s[4 * NCH];   // [channel][gate]
    // Rows of 64 positions staged in LDS so that HBM sees whole rows: the previous cell
    // states (two rows, FP32) and the new c and h (two rows each).  A position's 16-byte
    // chunks are stored at chunk ^ (position mod 16) (c) or ^ (position mod 8) (h), which
    // spreads the epilogue's 8- and 4-byte accesses of 16 positions over the banks.
    __shared__ __attribute__((aligned(16))) uint8_t cin_s[2][SW * 256];
    __shared__ __attribute__((aligned(16))) uint8_t cout_s[2][SW * 256];
    __shared__ __attribute__((aligned(16))) uint8_t hout_s[2][SW * 128];
    const int tid = threadIdx.x;
    const int lane = lane_id();
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    // Block j of this wave: row 4 q' + g is gate g of channel 8 wv + 2 q' + j.  Lane (row r,
    // K group kk) of the A fragment comes from the packed layer's block pblock(ch, g),
    // column ch % 16, lane ch % 16 + 16 kk.
    uint4 wr[NK][2];
    uint4 ws[2];
    const uint16_t* wcur = nullptr;
    long long it = blockIdx.x;
    int si;
    Item I;
    while (next_item(segs, nseg, it, total, si, I)) {
        const LstmSeg& S = segs[si];
        if (S.wt != wcur) {   // every segment of a launch has the same weights
            wcur = S.wt;
            int ln = lane;   // opaque: the lane offsets below are not kept across the loops
            asm volatile("" : "+v"(ln));
            const int r = ln & 15, kk = ln >> 4;
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                const int ch = 8 * wv + 2 * (r >> 2) + j;
                const int src = pblock(ch, r & 3) * 64 + (ch & 15) + 16 * kk;
#pragma unroll
                for (int st = 0; st < NK; ++st)
                    wr[st][j] = ld_g(reinterpret_cast<const uint4*>(S.wt) + (long long)st * NBT * 64 + src);
                ws[j] = ld_g(reinterpret_cast<const uint4*>(S.wsym) + src);
            }
            if (tid < 4 * NCH) bias_s[tid] = gmem(S.bias)[pblock(tid >> 2, tid & 3) * 16 + ((tid >> 2) & 15)];
            wait_vm();
        }
        // ---- input rows: thread tid owns 16-byte pieces tid and tid + 512 of a row ----
        const int win = S.w >> S.up;
        const uint8_t* inp =
            S.in16 ? reinterpret_cast<const uint8_t*>(S.in16) + (long long)I.n * S.in_ps * 2 : nullptr;
        const auto sp = gmem(S.sym ? S.sym + (long long)I.n * S.sym_ps : reinterpret_cast<const int16_t*>(S.wt));
        uint4 v[2];
        int16_t sv = 0;
        // The loader's and the epilogue's lane-dependent offsets are recomputed where they are
        // used (the thread index made opaque to the optimiser) instead of being held in
        // registers across the row loop, which the weights fill.
        auto opaque = [](int v) {
            asm volatile("" : "+v"(v));
            return v;
        };
        auto load = [&](int row) {
            const int tid_ = opaque(tid);
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int idx = tid_ + 512 * k;
                const int slot = idx >> 3;
                const int c = I.c0 - 1 + slot;
                v[k] = make_uint4(0, 0, 0, 0);
                if (idx < NV && inp && row >= 0 && row < S.h && c >= 0 && c < S.w)
                    v[k] = ld_g(reinterpret_cast<const uint4*>(
                        inp + ((long long)(row >> S.up) * win + (c >> S.up)) * NCH * 2 + (idx & 7) * 16));
            }
            if (tid_ < SLOTS) {
                const int c = I.c0 - 1 + tid_;
                const int rc = min(max(row, 0), S.h - 1), cc = min(max(c, 0), S.w - 1);
                sv = sp[S.sym ? (long long)(rc >> S.up) * win + (cc >> S.up) : 0ll];
            }
        };
        auto store = [&](int row) {
            const int tid_ = opaque(tid);
            uint8_t* dst = ring + (row & 3) * RROW;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int idx = tid_ + 512 * k;
                if (idx < NV) *reinterpret_cast<uint4*>(dst + swz(idx >> 3, idx & 7)) = v[k];
            }
            if (tid_ < SLOTS) {
                const int c = I.c0 - 1 + tid_;
                const bool ok = S.sym && row >= 0 && row < S.h && c >= 0 && c < S.w;   // |q| <= 256: exact
                ring_s[row & 3][tid_] = f2bf(ok ? (float)sv : 0.f);
            }
        };
        load(I.y0 - 1);
        lds_barrier();   // the previous item's last reads of the ring are done
        const int T = I.R + 3;
        const int wp = S.w >> S.up;
        // Previous cell states: row xr of 64 positions x 256 bytes, two 16-byte pieces per
        // thread, loaded a step before they are stored to LDS (at the current resolution: a
        // position reads its source column c >> up).
        uint4 cv[2];
        auto cload = [&](int xr) {
            const int tid_ = opaque(tid);
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int idx = tid_ + 512 * k;   // position idx / 16, piece idx % 16
                const int c = I.c0 + (idx >> 4);
                cv[k] = make_uint4(0, 0, 0, 0);
                if (S.c_prev && c < S.w)
                    cv[k] = ld_g(reinterpret_cast<const uint4*>(S.c_prev + (long long)I.n * S.cprev_ps +
                                                              ((long long)(xr >> S.up) * wp + (c >> S.up)) * NCH) +
                                 (idx & 15));
            }
        };
        auto cstore = [&](int xr) {
            const int tid_ = opaque(tid);
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int idx = tid_ + 512 * k;
                const int pos = idx >> 4;
                *reinterpret_cast<uint4*>(cin_s[xr & 1] + pos * 256 + (((idx & 15) ^ (pos & 15)) << 4)) = cv[k];
            }
        };
        // The staged c and h of output row xr to HBM: whole 256- and 128-byte positions.
        auto flush = [&](int xr) {
            const int tid_ = opaque(tid);
            const uint8_t* cs = cout_s[xr & 1];
            const uint8_t* hs = hout_s[xr & 1];
            const long long row0 = (long long)I.n * S.st_ps + ((long long)xr * S.w + I.c0) * NCH;
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const int idx = tid_ + 512 * k;
                const int pos = idx >> 4;
                if (I.c0 + pos < S.w)
                    st_g(reinterpret_cast<uint4*>(S.c_out + row0 + pos * NCH) + (idx & 15),
                         *reinterpret_cast<const uint4*>(cs + pos * 256 + (((idx & 15) ^ (pos & 15)) << 4)));
            }
            const int pos = tid_ >> 3;
            if (I.c0 + pos < S.w)
                st_g(reinterpret_cast<uint4*>(S.h_out + row0 + pos * NCH) + (tid_ & 7),
                     *reinterpret_cast<const uint4*>(hs + pos * 128 + (((tid_ & 7) ^ (pos & 7)) << 4)));
        };
        for (int t = 0; t < T; ++t) {
            const int x = I.y0 - 3 + t;   // output row of this step
            // Everything loaded in the previous step goes to LDS before this step issues any
            // global access: loads and stores share one completion counter, so a wait placed
            // after this step's loads and stores would wait for those too.
            if (t <= I.R + 1) store(I.y0 - 1 + t);
            if (t >= 2 && t <= I.R + 1) cstore(x + 1);
            wait_vm();   // already true here (the previous step's stores are a step old); it
                         // keeps later register reuse in this step from waiting on new loads
            // This step's global accesses: waves 0-3 issue theirs first, waves 4-7 (the other
            // wave of each SIMD) between the two halves of the row, so that one wave of a SIMD
            // issues MFMAs while the other waits on the memory pipeline.
            auto vmem = [&]() {
                if (t <= I.R) load(I.y0 + t);
                if (t >= 1 && t <= I.R) cload(I.y0 - 1 + t);
                if (t >= 4) flush(x - 1);
            };
            if (wv < 4) vmem();
            if (t < 3 && wv >= 4) vmem();   // no rows computed in this step
            if (t >= 3) {
                const uint8_t* cin = cin_s[x & 1];
                uint8_t* cout = cout_s[x & 1];
                uint8_t* hout = hout_s[x & 1];
#pragma unroll
                for (int half = 0; half < 2; ++half) {
                    if (half == 1 && wv >= 4) vmem();
                    floatx4 acc[2][2];
                    // The gate MFMAs at raised wave priority, the cell update at the normal one:
                    // a wave in its MFMAs goes first, and the other wave's epilogue fills the
                    // issue slots between them.
                    __builtin_amdgcn_s_setprio(1);
                    row_gates(ring, ring_s, x, 2 * half, wr, ws, acc, lane);
                    __builtin_amdgcn_s_setprio(0);
                    const int ln = opaque(lane);
                    const int ch0 = 8 * wv + 2 * (ln >> 4);   // this lane's two channels
#pragma unroll
                    for (int mb = 0; mb < 2; ++mb) {
                        const int pos = 16 * (2 * half + mb) + (ln & 15);
                        const floatx2 cp = *reinterpret_cast<const floatx2*>(
                            cin + pos * 256 + (((ch0 >> 2) ^ (pos & 15)) << 4) + (ch0 & 3) * 4);
                        float hn[2], cn[2];
#pragma unroll
                        for (int j = 0; j < 2; ++j) {
                            const float4 b = *reinterpret_cast<const float4*>(bias_s + 4 * (ch0 + j));
                            const float gi = sigmoid_fast(fmaf(acc[mb][j][0], 1.f, b.x));
                            const float gf = sigmoid_fast(fmaf(acc[mb][j][1], 1.f, b.y));
                            const float gg = tanh_fast(fmaf(acc[mb][j][2], 1.f, b.z));
                            const float go = sigmoid_fast(fmaf(acc[mb][j][3], 1.f, b.w));
                            const float cpv = j == 0 ? cp.x : cp.y;
                            cn[j] = fmaf(gf, cpv, gi * gg);   // as in the layer-by-layer kernel
                            hn[j] = go * tanh_fast(cn[j]);
                        }
                        *reinterpret_cast<floatx2*>(cout + pos * 256 + (((ch0 >> 2) ^ (pos & 15)) << 4) +
                                                    (ch0 & 3) * 4) = floatx2{cn[0], cn[1]};
                        *reinterpret_cast<uint32_t*>(hout + pos * 128 + (((ch0 >> 3) ^ (pos & 7)) << 4) +
                                                     (ch0 & 7) * 2) = f2bf2(hn[0], hn[1]);
                    }
                }
            }
            lds_barrier();
        }
        flush(I.y0 + I.R - 1);   // the last row (its staging buffer is not written again before
                                 // the next item's fourth step, three barriers later)
        it += gridDim.x;
    }
}

}  // namespace

hipError_t launch_lstm_bf16(const LstmSeg* segs, int nseg, long long total, int grid, hipStream_t s) {
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(lstm_bf16_k, dim3((unsigned)grid), dim3(512), 0, s, segs, nseg, total);
    return hipGetLastError();
}

}  // namespace wv
