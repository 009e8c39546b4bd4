// 3x3 convolution as an implicit GEMM on the gfx950 matrix cores with BF16 or
// FP8 (e4m3) operands and FP32 accumulation (precision variants of the context
// model).
//
// Same GEMM view and epilogues as the FP32 kernel (wv_conv.hip); what changes
// with v_mfma_f32_16x16x32_bf16 is the balance: one instruction covers 32
// input channels, so operand traffic rather than the matrix pipe becomes the
// limit.  The tile is therefore taller: a workgroup owns 16 x 16 positions,
// each of its 4 waves 4 rows x (16 NB) channels (16 accumulators for NB = 4).
// A fragments: one 16-byte LDS read = 8 channels of one position per lane;
// B fragments: per-tap weight slices staged in LDS in three buffers, read from
// HBM/L2 two taps ahead and stored to LDS one tap ahead.  Activations in and out are BF16 (NHWC), the
// LSTM cell state, every epilogue and the mixture parameters are FP32.
//
// FP8 form (F8): the same tiling, activations stored as e4m3 bytes, weights
// e4m3 with one FP32 scale per output channel applied to the accumulator
// before the bias.  With 64 input channels and no symbol channel one K step of
// v_mfma_scale_f32_16x16x128_f8f6f4 (unit block scales) covers two taps: lane
// group g = 0..3 holds tap 2s + g/2, channels 32 (g % 2) .. + 31 (32 bytes per
// lane), so nine taps take five steps (the tenth tap is zero) at twice the
// rate of v_mfma_f32_16x16x32_fp8_fp8, which the other layers keep (one
// 8-byte fragment of 8 channels per lane).  The symbol channel keeps its BF16
// MFMA chunk (its weights are packed divided by the channel scale), so symbols
// up to the int16 range stay exact.
#include "wv_device.h"
#include "wv_internal.h"

namespace wv {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef int intx8 __attribute__((ext_vector_type(8)));

typedef int intx4 __attribute__((ext_vector_type(4)));

constexpr int TH = 16;
constexpr int TW = 16;
constexpr int HH = TH + 2;
constexpr int HWD = TW + 2;
constexpr int HALO = HH * HWD;


__device__ __forceinline__ uint16_t f2bf(float f) {   // round to nearest even (v_cvt_pk_bf16_f32)
    return __builtin_bit_cast(uint16_t, (__bf16)f);
}

__device__ __forceinline__ bf16x8 as_bf(uint4 v) { return __builtin_bit_cast(bf16x8, v); }

// float -> e4m3 byte, round to nearest even, saturated to +-448 first.
__device__ __forceinline__ uint8_t f2e4m3(float f) {
    f = fminf(fmaxf(f, -448.f), 448.f);
    return (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(f, 0.f, 0, false) & 0xff);
}

// One lane's K = 128 operand (32 e4m3 bytes) from two aligned 16-byte loads.
__device__ __forceinline__ intx8 load32(const uint8_t* p) {
    const intx4* q = reinterpret_cast<const intx4*>(p);
    return __builtin_shufflevector(q[0], q[1], 0, 1, 2, 3, 4, 5, 6, 7);
}

__device__ __forceinline__ floatx4 mfma_f8k128(const intx8& a, const intx8& b, const floatx4& c) {
    // formats 0/0: e4m3 A and B; block scales 0x7f = 2^0
    return __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(a, b, c, 0, 0, 0, 0x7f7f7f7f, 0, 0x7f7f7f7f);
}

template <bool F8>
struct Frag;
template <>
struct Frag<false> { using T = uint4; };   // 8 bf16
template <>
struct Frag<true> { using T = uint2; };    // 8 e4m3

template <bool F8>
__device__ __forceinline__ floatx4 mfma_lp(const typename Frag<F8>::T& a, const typename Frag<F8>::T& b,
                                           const floatx4& c) {
    if constexpr (F8)
        return __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(__builtin_bit_cast(long, a), __builtin_bit_cast(long, b),
                                                          c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(a), as_bf(b), c, 0, 0, 0);
}

template <int CIN, int NB, bool SYM, int MODE, bool F8>
__device__ __forceinline__ void conv_tile_bf16(const MfmaLayer16& L, const ConvArgs& a, const int tile_idx,
                                               const int ycol) {
    using FragT = typename Frag<F8>::T;
    // Two taps per K = 128 step (see above) for the 64-channel step-stack layers without the
    // symbol channel (with it, or the ConvLSTM's 256 gate columns, the larger operands leave
    // the persistent form too few registers).  The weight packer applies the same rule.
    constexpr bool K128 = F8 && CIN == 64 && !SYM && MODE != CONV_LSTM;
    constexpr int ES = F8 ? 1 : 2;              // bytes per activation element
    constexpr int FB = 8 * ES;                  // bytes per operand fragment (8 K values)
    // bytes per halo position (conflict-free reads; 16-byte aligned for the 32-byte K128 reads)
    constexpr int STRIDE = K128 ? CIN + 16 : CIN * ES + 8 * ES;
    constexpr int CC = K128 ? 1 : CIN / 32;     // K chunks per staged B slice (a tap, or a K128 step)
    constexpr int BU = K128 ? 128 : FB * 64 / 16;   // uint4 per (chunk, 16-column block) of B
    constexpr int BV = CC * NB * BU;            // uint4 of B per tap (K128: per step) for this workgroup
    constexpr int NSTEP = K128 ? 5 : 9;         // staged B slices: taps, or K128 steps
    constexpr int BPT = (BV + 255) / 256;
    constexpr int NSY = (HALO + 255) / 256;     // symbol positions per thread
    constexpr int MB = (MODE == CONV_HEAD) ? 2 : 4;   // head: only the rows of its step's parity
    constexpr int OS = NB * 16 * ES + 16;       // bytes per position of the staged output tile
    static_assert(BPT <= 2, "B slice too large");
    // Input halo; after the MFMA loop it holds the output tile (RELU/TANH epilogue).
    constexpr int LDS_IN = HALO * STRIDE > TH * TW * OS ? HALO * STRIDE : TH * TW * OS;
    __shared__ __attribute__((aligned(16))) uint8_t lds_in[LDS_IN];
    __shared__ __attribute__((aligned(16))) uint4 lds_w[3][BV];
    __shared__ __attribute__((aligned(16))) uint4 lds_ws[SYM ? NB * 64 : 1];
    __shared__ uint16_t lds_s[SYM ? HALO : 1];
    __shared__ float lds_head[MODE == CONV_HEAD ? 8 * TW * 17 : 1];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    int t = tile_idx;
    const int tx = t % a.tiles_x;
    t /= a.tiles_x;
    const int ty = t % a.tiles_y;
    const int n = t / a.tiles_y;
    const int r0 = ty * TH;
    const int c0 = tx * TW;
    const int nblk0 = ycol * NB;
    // Rows of this wave: 4w .. 4w+3; the head keeps the two of parity step/2.
    const int gr = a.step >> 1;

    const uint4* wg = reinterpret_cast<const uint4*>(L.w);
    auto boff_of = [&](int k) -> long long {
        const int idx = (tid + k * 256) < BV ? tid + k * 256 : 0;
        const int cc = idx / (NB * BU);
        const int rem = idx - cc * (NB * BU);
        return ((long long)cc * L.nbt + nblk0) * BU + rem;
    };
    const long long bo0 = boff_of(0);
    const long long bo1 = BPT > 1 ? boff_of(1) : 0;
    const long long btap = (long long)CC * L.nbt * BU;
    // B slice k (a tap, or a K128 step) goes global -> registers (set k % 2) two slices ahead,
    // registers -> LDS buffer k % 3 one slice ahead.
    uint4 bq[2][2];
#define WV_LOAD_B(tp)                                       \
    {                                                       \
        const uint4* wt_ = wg + (long long)(tp) * btap;     \
        bq[(tp) & 1][0] = ld_g(wt_ + bo0);                  \
        if (BPT > 1) bq[(tp) & 1][1] = ld_g(wt_ + bo1);     \
    }
#define WV_STORE_B(tp)                                                                            \
    {                                                                                             \
        if (BV >= 256 || tid < BV) lds_w[(tp) % 3][tid] = bq[(tp) & 1][0];                        \
        if (BPT > 1 && (BV >= 512 || tid + 256 < BV)) lds_w[(tp) % 3][tid + 256] = bq[(tp) & 1][1]; \
    }
    WV_LOAD_B(0)

    {
        const int win = a.w >> a.in_up;
        const uint8_t* inp =
            a.in16 ? reinterpret_cast<const uint8_t*>(a.in16) + (long long)n * a.in_ps * ES : nullptr;
        constexpr int V = CIN * ES / 16;             // uint4 per position
        constexpr int NH = (HALO * V + 255) / 256;   // per thread: all loads in flight before any store
        uint4 hv[NH];
#pragma unroll
        for (int k = 0; k < NH; ++k) {
            const int idx = tid + k * 256;
            const int pos = idx / V;
            const int c16 = idx - pos * V;
            const int hy = pos / HWD;
            const int r = r0 + hy - 1;
            const int c = c0 + (pos - hy * HWD) - 1;
            hv[k] = make_uint4(0, 0, 0, 0);
            if (idx < HALO * V && inp && r >= 0 && r < a.h && c >= 0 && c < a.w)
                hv[k] = ld_g(reinterpret_cast<const uint4*>(
                    inp + ((long long)(r >> a.in_up) * win + (c >> a.in_up)) * CIN * ES + c16 * 16));
        }
        auto store_halo = [&]() {
#pragma unroll
            for (int k = 0; k < NH; ++k) {
                const int idx = tid + k * 256;
                if (idx < HALO * V) {
                    const int pos = idx / V;
                    uint8_t* dst = lds_in + pos * STRIDE + (idx - pos * V) * 16;
                    if constexpr (F8) {   // 8-byte aligned positions
                        reinterpret_cast<uint2*>(dst)[0] = make_uint2(hv[k].x, hv[k].y);
                        reinterpret_cast<uint2*>(dst)[1] = make_uint2(hv[k].z, hv[k].w);
                    } else {
                        *reinterpret_cast<uint4*>(dst) = hv[k];
                    }
                }
            }
        };
        if constexpr (SYM) {
            // Symbols of the halo (masked by coding step) and the symbol-channel weights: issued
            // right behind the halo loads, so that one wait covers all of them.
            // The loads are unconditional, from a clamped address (or, without symbols, from a
            // valid dummy one: the first weight), and the mask is applied after the wait: a
            // load under a branch whose result is converted there waits inside the branch.
            const bool has = a.sym != nullptr;
            const auto sp = gmem(has ? a.sym + (long long)n * a.sym_ps : reinterpret_cast<const int16_t*>(L.w));
            const int ws = a.w >> a.sym_up;
            int16_t sraw[NSY];
            bool sok[NSY];
#pragma unroll
            for (int k = 0; k < NSY; ++k) {
                const int pos = tid + k * 256;
                const int hy = pos / HWD;
                const int r = r0 + hy - 1;
                const int c = c0 + (pos - hy * HWD) - 1;
                sok[k] = has && pos < HALO && r >= 0 && r < a.h && c >= 0 && c < a.w &&
                         (2 * (r & 1) + (c & 1)) < a.sym_step;
                const int rc = min(max(r, 0), a.h - 1);
                const int cc = min(max(c, 0), a.w - 1);
                sraw[k] = sp[has ? (long long)(rc >> a.sym_up) * ws + (cc >> a.sym_up) : 0ll];
            }
            uint4 wsv = make_uint4(0, 0, 0, 0);
            if (tid < NB * 64) wsv = ld_g(reinterpret_cast<const uint4*>(L.wsym) + (long long)nblk0 * 64 + tid);
            store_halo();
#pragma unroll
            for (int k = 0; k < NSY; ++k)   // |symbol| <= 256: exact in BF16
                if (tid + k * 256 < HALO) lds_s[tid + k * 256] = f2bf(sok[k] ? (float)sraw[k] : 0.f);
            if (tid < NB * 64) lds_ws[tid] = wsv;
        } else {
            store_halo();
        }
    }
    WV_STORE_B(0)
    WV_LOAD_B(1)
    __syncthreads();

    floatx4 acc[MB][NB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = floatx4{0.f, 0.f, 0.f, 0.f};

    const int m = lane & 15;
    const int kk = lane >> 4;
    // tile row of accumulator block mb
    auto row_of = [&](int mb) { return MODE == CONV_HEAD ? wave * 4 + 2 * mb + gr : wave * 4 + mb; };

    // Steps (tap, 32-channel chunk) run in order; the A fragments of the next step
    // are read while this step's MFMAs run (the halo is not written in the loop,
    // so only the B slices need the per-tap barrier).  Fully unrolled so that the
    // fragment double buffer stays in registers.
  if constexpr (K128) {
    // Step s: lane group kk reads tap 2 s + kk / 2, channels 32 (kk % 2) .. + 31 of its position.
    const intx8 zero8 = {0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int st = 0; st < NSTEP; ++st) {
        if (st + 2 < NSTEP) {
            WV_LOAD_B(st + 2)
            __builtin_amdgcn_sched_barrier(0);   // keep the loads ahead of this step's MFMAs
        }
        const uint8_t* wb = reinterpret_cast<const uint8_t*>(lds_w[st % 3]);
        intx8 bv[NB];
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) bv[nb] = load32(wb + (nb * BU + 2 * lane) * 16);
        // Lane group kk: tap 2 st + kk / 2 (tap 9 is zero: read tap 8, then select zero).
        const int tp = 2 * st + (kk >> 1);
        const int tpc = tp < 9 ? tp : 8;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            intx8 av = load32(lds_in + ((row_of(mb) + tpc / 3) * HWD + m + tpc % 3) * STRIDE + 32 * (kk & 1));
            av = tp < 9 ? av : zero8;
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = mfma_f8k128(av, bv[nb], acc[mb][nb]);
        }
        if (st + 1 < NSTEP) {
            WV_STORE_B(st + 1)   // buffer (st + 1) % 3 was last read two steps ago
            __syncthreads();
        }
    }
  } else {
    FragT afr[2][MB];
#define WV_LOAD_A(dst, tp, ccv)                                                                      \
    _Pragma("unroll") for (int mb_ = 0; mb_ < MB; ++mb_) dst[mb_] = *reinterpret_cast<const FragT*>( \
        lds_in + ((row_of(mb_) + (tp) / 3) * HWD + m + (tp) % 3) * STRIDE + ((ccv) * 32 + kk * 8) * ES);
    WV_LOAD_A(afr[0], 0, 0)
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
        if (tap < 7) {
            WV_LOAD_B(tap + 2)
            __builtin_amdgcn_sched_barrier(0);   // keep the loads ahead of this tap's MFMAs
        }
        const FragT* wb = reinterpret_cast<const FragT*>(lds_w[tap % 3]);
        FragT bv[CC][NB];
#pragma unroll
        for (int cc = 0; cc < CC; ++cc)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) bv[cc][nb] = wb[(cc * NB + nb) * 64 + lane];
#pragma unroll
        for (int cc = 0; cc < CC; ++cc) {
            const int st = tap * CC + cc;
            if (cc + 1 < CC) {
                WV_LOAD_A(afr[(st + 1) & 1], tap, cc + 1)
            } else if (tap < 8) {
                WV_LOAD_A(afr[(st + 1) & 1], tap + 1, 0)
            }
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = mfma_lp<F8>(afr[st & 1][mb], bv[cc][nb], acc[mb][nb]);
        }
        if (tap < 8) {
            WV_STORE_B(tap + 1)   // buffer (tap + 1) % 3 was last read two taps ago
            __syncthreads();
        }
    }
#undef WV_LOAD_A
  }
#undef WV_LOAD_B
#undef WV_STORE_B
    if (SYM) {
        // One K = 32 chunk: element j of lane group kk is tap 8 kk + j (taps >= 9 are zero).
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            uint16_t e[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int tap = kk * 8 + j;
                e[j] = tap < 9 ? lds_s[(row_of(mb) + tap / 3) * HWD + m + tap % 3] : (uint16_t)0;
            }
            const uint4 av = make_uint4(e[0] | ((uint32_t)e[1] << 16), e[2] | ((uint32_t)e[3] << 16),
                                        e[4] | ((uint32_t)e[5] << 16), e[6] | ((uint32_t)e[7] << 16));
#pragma unroll
            for (int nb = 0; nb < NB; ++nb)
                acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf(av), as_bf(lds_ws[nb * 64 + lane]),
                                                                      acc[mb][nb], 0, 0, 0);
        }
    }

    const int col = lane & 15;
    const int rowq = (lane >> 4) * 4;
    // FP8: the accumulator of packed column nc is scaled by L.scale[nc] before the bias.
    float csc[NB];
#pragma unroll
    for (int nb = 0; nb < NB; ++nb) csc[nb] = F8 ? gmem(L.scale)[(nblk0 + nb) * 16 + col] : 1.f;
    if constexpr (MODE == CONV_RELU || MODE == CONV_TANH) {
        // Stage the output tile [256 positions][16 NB channels] in LDS (reusing the
        // halo buffer), then write 16-byte chunks: full, coalesced lines.
        static_assert(TH * TW * OS <= LDS_IN, "output tile does not fit the halo buffer");
        __syncthreads();
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const float b = gmem(L.bias)[(nblk0 + nb) * 16 + col];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    float v = F8 ? fmaf(acc[mb][nb][i], csc[nb], b) : acc[mb][nb][i] + b;
                    v = MODE == CONV_RELU ? fmaxf(v, 0.f) : tanh_fast(v);
                    uint8_t* dst = lds_in + (row_of(mb) * TW + rowq + i) * OS + (nb * 16 + col) * ES;
                    if constexpr (F8)
                        *dst = f2e4m3(v);
                    else
                        *reinterpret_cast<uint16_t*>(dst) = f2bf(v);
                }
            }
        __syncthreads();
        constexpr int V16 = NB * 16 * ES / 16;   // 16-byte chunks per position
        uint8_t* outp = reinterpret_cast<uint8_t*>(a.out16);
        for (int idx = tid; idx < TH * TW * V16; idx += 256) {
            const int pos = idx / V16;
            const int c16 = idx - pos * V16;
            const int r = r0 + pos / TW;
            const int c = c0 + pos % TW;
            if (r < a.h && c < a.w && (nblk0 * 16 + c16 * 16 / ES) < L.cout)
                st_g(reinterpret_cast<uint4*>(outp + ((long long)n * a.out_ps +
                                                      ((long long)r * a.w + c) * a.out_cs + nblk0 * 16) * ES +
                                              c16 * 16),
                     *reinterpret_cast<const uint4*>(lds_in + pos * OS + c16 * 16));
        }
    } else if constexpr (MODE == CONV_LSTM) {
        const int ch = ycol * 16 + col;
        const auto bias = gmem(L.bias);
        const float bi = bias[(nblk0 + 0) * 16 + col];
        const float bf = bias[(nblk0 + 1) * 16 + col];
        const float bg = bias[(nblk0 + 2) * 16 + col];
        const float bo = bias[(nblk0 + 3) * 16 + col];
        const int wp = a.w >> a.cprev_up;
        // All of this lane's previous cell states first (one wait for all of them, not one per
        // position; c_prev and c_out are different buffers).
        float cp[MB][4];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            const int r = r0 + row_of(mb);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int c = c0 + rowq + i;
                cp[mb][i] = 0.f;
                if (a.c_prev && r < a.h && c < a.w)
                    cp[mb][i] = gmem(a.c_prev)[(long long)n * a.cprev_ps +
                                               ((long long)(r >> a.cprev_up) * wp + (c >> a.cprev_up)) * a.C + ch];
            }
        }
        const auto c_out = gmem(a.c_out);
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            const int r = r0 + row_of(mb);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int c = c0 + rowq + i;
                if (r < a.h && c < a.w) {
                    const float gi = sigmoid_fast(fmaf(acc[mb][0][i], csc[0], bi));
                    const float gf = sigmoid_fast(fmaf(acc[mb][1][i], csc[1 % NB], bf));
                    const float gg = tanh_fast(fmaf(acc[mb][2][i], csc[2 % NB], bg));
                    const float go = sigmoid_fast(fmaf(acc[mb][3][i], csc[3 % NB], bo));
                    const float cn = fmaf(gf, cp[mb][i], gi * gg);   // one rounding order for every LSTM kernel
                    const float hn = go * tanh_fast(cn);
                    const long long o = (long long)n * a.st_ps + ((long long)r * a.w + c) * a.C + ch;
                    c_out[o] = cn;
                    if constexpr (F8)
                        gmem(reinterpret_cast<uint8_t*>(a.h16_out))[o] = f2e4m3(hn);
                    else
                        gmem(a.h16_out)[o] = f2bf(hn);
                }
            }
        }
    } else {  // CONV_HEAD
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                lds_head[((wave * 2 + mb) * TW + rowq + i) * 17 + col] =
                    F8 ? fmaf(acc[mb][0][i], csc[0], gmem(L.bias)[col]) : acc[mb][0][i] + gmem(L.bias)[col];
        __syncthreads();
        if (tid < 8 * TW) {
            const int rr = tid / TW;                       // 0..7: wave rr/2, block rr%2
            const int r = r0 + (rr >> 1) * 4 + 2 * (rr & 1) + gr;
            const int c = c0 + tid % TW;
            const int gc = a.step & 1;
            if (r < a.h && c < a.w && (c & 1) == gc) {
                const float* v = lds_head + tid * 17;
                const int K = a.K;
                const int wg2 = (a.w - gc + 1) >> 1;
                const int hg = (a.h - gr + 1) >> 1;
                const long long gi = (long long)(r >> 1) * wg2 + (c >> 1);
                float* o = a.params + ((long long)n * hg * wg2 + gi) * 3 * K;
                mixture_head(v, K, a.sigma_min, gmem(o));
            }
        }
    }
}

template <int CIN, int NB, bool SYM, int MODE, bool F8>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void conv3x3_mfma_bf16(
    const MfmaLayer16 L, const ConvArgs a) {
    long long tile;
    int ycol;
    conv_item_order(blockIdx.x, (long long)a.tiles_x * a.tiles_y * a.N, MODE == CONV_HEAD ? 1 : L.nbt / NB, tile,
                    ycol);
    conv_tile_bf16<CIN, NB, SYM, MODE, F8>(L, a, (int)tile, ycol);
}

// Persistent multi-segment form (see the FP32 kernel).
template <int CIN, int NB, bool SYM, int MODE, bool F8>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void conv3x3_mfma_bf16_seg(
    const ConvSeg16* __restrict__ segs, int nseg, long long total) {
    for (long long it = blockIdx.x; it < total; it += gridDim.x) {
        int lo = 0, hi = nseg;
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (segs[mid].item0 <= it) lo = mid; else hi = mid;
        }
        const ConvSeg16& S = segs[lo];
        const long long local = it - S.item0;
        long long tile;
        int ycol;
        conv_item_order(local, (long long)S.a.tiles_x * S.a.tiles_y * S.a.N, MODE == CONV_HEAD ? 1 : S.L.nbt / NB,
                        tile, ycol);
        conv_tile_bf16<CIN, NB, SYM, MODE, F8>(S.L, S.a, (int)tile, ycol);
        __syncthreads();
    }
}

template <int CIN, int NB, bool SYM, int MODE, bool F8>
hipError_t launch_t(const MfmaLayer16& L, const ConvArgs& a0, hipStream_t s) {
    ConvArgs a = a0;
    a.tiles_x = (a.w + TW - 1) / TW;
    a.tiles_y = (a.h + TH - 1) / TH;
    const int ncols = (MODE == CONV_HEAD) ? 1 : L.nbt / NB;
    dim3 grid((unsigned)(a.tiles_x * a.tiles_y * a.N * ncols));
    hipLaunchKernelGGL((conv3x3_mfma_bf16<CIN, NB, SYM, MODE, F8>), grid, dim3(256), 0, s, L, a);
    return hipGetLastError();
}

template <int CIN, int NB, bool SYM, bool F8>
hipError_t dispatch_mode(const MfmaLayer16& L, int mode, const ConvArgs& a, hipStream_t s) {
    switch (mode) {
        case CONV_RELU: return launch_t<CIN, NB, SYM, CONV_RELU, F8>(L, a, s);
        case CONV_LSTM: return NB == 4 ? launch_t<CIN, 4, SYM, CONV_LSTM, F8>(L, a, s) : hipErrorInvalidValue;
        case CONV_HEAD: return NB == 1 ? launch_t<CIN, 1, SYM, CONV_HEAD, F8>(L, a, s) : hipErrorInvalidValue;
    }
    return hipErrorInvalidValue;
}

template <int CIN, int NB, bool F8>
hipError_t dispatch_sym(const MfmaLayer16& L, int mode, const ConvArgs& a, hipStream_t s) {
    return L.has_sym ? dispatch_mode<CIN, NB, true, F8>(L, mode, a, s)
                     : dispatch_mode<CIN, NB, false, F8>(L, mode, a, s);
}

inline int pick_nb(const MfmaLayer16& L, int mode, const ConvArgs& a) {
    return conv_pick_nb(L.nbt, mode, (long long)((a.w + TW - 1) / TW) * ((a.h + TH - 1) / TH) * a.N, 1);
}

template <int CIN, bool F8>
hipError_t dispatch_nb(const MfmaLayer16& L, int mode, const ConvArgs& a, hipStream_t s) {
    switch (pick_nb(L, mode, a)) {
        case 1: return dispatch_sym<CIN, 1, F8>(L, mode, a, s);
        case 2: return dispatch_sym<CIN, 2, F8>(L, mode, a, s);
        case 4: return dispatch_sym<CIN, 4, F8>(L, mode, a, s);
    }
    return hipErrorInvalidValue;
}

template <int CIN, int NB, bool SYM, int MODE, bool F8>
hipError_t seg_t(const ConvSeg16* segs, int nseg, long long total, int grid, hipStream_t s) {
    if (grid < total && grid >= 8) grid &= ~7;   // columns of a tile on one XCD (conv_item_order)
    hipLaunchKernelGGL((conv3x3_mfma_bf16_seg<CIN, NB, SYM, MODE, F8>), dim3(grid), dim3(256), 0, s, segs, nseg,
                       total);
    return hipGetLastError();
}

template <int CIN, int NB, bool SYM, bool F8>
hipError_t seg_mode(const ConvSeg16* segs, int nseg, long long total, int mode, int grid, hipStream_t s) {
    switch (mode) {
        case CONV_RELU: return seg_t<CIN, NB, SYM, CONV_RELU, F8>(segs, nseg, total, grid, s);
        case CONV_LSTM:
            return NB == 4 ? seg_t<CIN, 4, SYM, CONV_LSTM, F8>(segs, nseg, total, grid, s) : hipErrorInvalidValue;
        case CONV_HEAD:
            return NB == 1 ? seg_t<CIN, 1, SYM, CONV_HEAD, F8>(segs, nseg, total, grid, s) : hipErrorInvalidValue;
    }
    return hipErrorInvalidValue;
}

template <int CIN, bool F8>
hipError_t seg_nb(const ConvSeg16* segs, int nseg, long long total, int sym, int mode, int nb, int grid,
                  hipStream_t s) {
#define WV_SEG_NB(NBV)                                                                         \
    if (nb == NBV) return sym ? seg_mode<CIN, NBV, true, F8>(segs, nseg, total, mode, grid, s) \
                              : seg_mode<CIN, NBV, false, F8>(segs, nseg, total, mode, grid, s);
    WV_SEG_NB(1) WV_SEG_NB(2) WV_SEG_NB(4)
#undef WV_SEG_NB
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_conv_seg_bf16(const ConvSeg16* segs, int nseg, long long total,
                                const MfmaLayer16& proto, int mode, int nb, int grid, hipStream_t s) {
    if (total <= 0 || nseg <= 0) return hipSuccess;
    const bool f8 = proto.scale != nullptr;
    switch (proto.cin) {
        case 32:
            return f8 ? seg_nb<32, true>(segs, nseg, total, proto.has_sym, mode, nb, grid, s)
                      : seg_nb<32, false>(segs, nseg, total, proto.has_sym, mode, nb, grid, s);
        case 64:
            return f8 ? seg_nb<64, true>(segs, nseg, total, proto.has_sym, mode, nb, grid, s)
                      : seg_nb<64, false>(segs, nseg, total, proto.has_sym, mode, nb, grid, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_conv_bf16(const MfmaLayer16& L, int mode, const ConvArgs& a, hipStream_t s) {
    if (a.N <= 0 || a.h <= 0 || a.w <= 0) return hipSuccess;
    if (mode == CONV_LSTM && L.nbt % 4 != 0) return hipErrorInvalidValue;
    const bool f8 = L.scale != nullptr;
    switch (L.cin) {
        case 32: return f8 ? dispatch_nb<32, true>(L, mode, a, s) : dispatch_nb<32, false>(L, mode, a, s);
        case 64: return f8 ? dispatch_nb<64, true>(L, mode, a, s) : dispatch_nb<64, false>(L, mode, a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace wv
