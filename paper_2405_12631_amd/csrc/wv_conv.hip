// 3x3 convolution as an implicit GEMM on the gfx950 matrix cores (FP32).
//
// Used by every dense contraction of the path: the ConvLSTM gate conv and
// the coding-step stacks of the context model (Sec. 3.2), and the C -> C
// layers of the lifting filters (Sec. 3.1).
//
// GEMM view: M = output positions, N = output channels, K = 9 taps x Cin.
// One workgroup (256 threads, 4 waves) works on an 8 x 16 position tile and
// 16*NB output channels at a time, walking its share of the tiles.  The (8+2) x (16+2) input halo of all Cin channels
// is staged once in LDS (NHWC, row stride Cin+4 floats); each wave computes
// two rows of 16 positions x NB blocks of 16 channels with
// v_mfma_f32_16x16x4f32, A fragments read from LDS as float4 (4 channels of
// one position per lane).  The weights of one tap (Cin x 16*NB, repacked as
// B fragments) are staged in LDS by the whole workgroup; the next tap's
// slice is fetched into registers while the current tap computes, so the
// MFMA loop reads only LDS.  The optional
// symbol channel (int16 symbols, masked by coding step) is a separate
// rank-9 update of three K=4 chunks.  Accumulation order is fixed, so a
// position's result does not depend on the tile, the grid or the batch.
#include "wv_device.h"
#include "wv_internal.h"

namespace wv {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int HALO_H = TILE_H + 2;
constexpr int HALO_W = TILE_W + 2;
constexpr int HALO = HALO_H * HALO_W;

// Persistent form for every launch: a workgroup walks items it = blockIdx.x,
// + gridDim.x, ... (item = (tile, column of NB 16-channel blocks) of one segment =
// one layer over one group of planes; a single-layer launch is one segment).
// The next item's halo is loaded into registers a slice per tap while this
// item's MFMAs run, next to that tap's weight load (so waiting for the weights
// never waits for a halo load issued later); at the last tap the next item's
// first weight slice and symbol inputs follow.  Static assignment, same bits.
struct ItemPosF {
    int n, r0, c0, ycol;
};

template <int NB, int MODE>
__device__ __forceinline__ ItemPosF item_pos_f32(const MfmaLayer& L, const ConvArgs& a, long long local) {
    const long long ntiles = (long long)a.tiles_x * a.tiles_y * a.N;
    long long tl;
    ItemPosF p;
    conv_item_order(local, ntiles, MODE == CONV_HEAD ? 1 : L.nbt / NB, tl, p.ycol);
    int t = (int)tl;
    const int tx = t % a.tiles_x;
    t /= a.tiles_x;
    const int ty = t % a.tiles_y;
    p.n = t / a.tiles_y;
    p.r0 = ty * TILE_H;
    p.c0 = tx * TILE_W;
    return p;
}

template <int CIN, int NB, bool SYM, int MODE, int TAPS, bool MULTI>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void conv3x3_f32p(
    const ConvSeg* __restrict__ segs, int nseg, const ConvSeg one, long long total) {
    // TAPS == 9: 3x3 conv; TAPS == 1: 1x1 conv (centre tap only, same data path).
    constexpr int STRIDE = CIN + 4;          // 68 floats for CIN = 64: conflict-free float4 reads
    constexpr int CB = CIN / 16;
    constexpr int BV4 = CB * NB * 64;        // float4 of B per tap for this workgroup's N blocks
    constexpr int BPT = (BV4 + 255) / 256;   // float4 per thread
    constexpr int MB = (MODE == CONV_HEAD) ? 1 : 2;   // head: only the row parity its step codes
    constexpr int V = CIN / 4;               // float4 per halo position
    constexpr int NH = (HALO * V + 255) / 256;
    constexpr int NS = (HALO + 255) / 256;
    constexpr int NWS = (3 * NB * 64 + 255) / 256;
    static_assert(BPT <= 4, "B slice larger than four float4 per thread");
    // Input halo; after the MFMA loop it holds the output tile (RELU/TANH epilogue).
    constexpr int LDS_IN = HALO * STRIDE > TILE_H * TILE_W * (NB * 16 + 4) ? HALO * STRIDE
                                                                            : TILE_H * TILE_W * (NB * 16 + 4);
    __shared__ __attribute__((aligned(16))) float lds_in[LDS_IN];
    __shared__ __attribute__((aligned(16))) float4 lds_w[BV4];
    __shared__ float lds_s[SYM ? HALO : 1];
    __shared__ float lds_ws[SYM ? 3 * NB * 64 : 1];
    __shared__ float lds_head[MODE == CONV_HEAD ? 4 * TILE_W * 17 : 1];

    long long it = blockIdx.x;
    if (it >= total) return;
    auto seg_index = [&](long long i) -> int {
        if constexpr (!MULTI) {
            return 0;
        } else {
            int lo = 0, hi = nseg;
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (segs[mid].item0 <= i) lo = mid; else hi = mid;
            }
            return lo;
        }
    };
#define WV_SEG(i) (MULTI ? segs[i] : one)
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int m = lane & 15;
    const int kk = lane >> 4;

    float4 hv[NH];
    int16_t sraw[NS];
    bool sok[NS];
    float wsv[NWS];
    float4 b0 = make_float4(0.f, 0.f, 0.f, 0.f), b1 = b0, b2 = b0, b3 = b0;
    // B fragments of tap tp for blocks [ycq NB, ycq NB + NB): global [tap][cb][nbt][64][4], LDS [cb][nb][64].
#define WV_LOAD_B(Lq, ycq, tp)                                                                     \
    {                                                                                              \
        const float4* wt_ = reinterpret_cast<const float4*>((Lq).w) + (long long)(tp) * CB * (Lq).nbt * 64; \
        _Pragma("unroll") for (int k_ = 0; k_ < BPT; ++k_) {                                       \
            const int idx_ = tid + k_ * 256;                                                       \
            if (idx_ < BV4) {                                                                      \
                const int cb_ = idx_ / (NB * 64);                                                  \
                const int rem_ = idx_ - cb_ * (NB * 64);                                           \
                const float4 v_ = ld_g(wt_ + ((long long)cb_ * (Lq).nbt + (ycq) * NB + (rem_ >> 6)) * 64 + (rem_ & 63)); \
                if (k_ == 0) b0 = v_; else if (k_ == 1) b1 = v_; else if (k_ == 2) b2 = v_; else b3 = v_; \
            }                                                                                      \
        }                                                                                          \
    }
#define WV_STORE_B()                                                       \
    {                                                                      \
        if (BV4 >= 256 || tid < BV4) lds_w[tid] = b0;                      \
        if (BPT > 1 && (BV4 >= 512 || tid + 256 < BV4)) lds_w[tid + 256] = b1; \
        if (BPT > 2 && (BV4 >= 768 || tid + 512 < BV4)) lds_w[tid + 512] = b2; \
        if (BPT > 3 && (BV4 >= 1024 || tid + 768 < BV4)) lds_w[tid + 768] = b3; \
    }
#define WV_LOAD_H(A, P, k)                                                                         \
    {                                                                                              \
        const int idx_ = tid + (k) * 256;                                                          \
        const int pos_ = idx_ / V;                                                                 \
        const int c4_ = idx_ - pos_ * V;                                                           \
        const int hy_ = pos_ / HALO_W;                                                             \
        const int r_ = (P).r0 + hy_ - 1;                                                           \
        const int c_ = (P).c0 + (pos_ - hy_ * HALO_W) - 1;                                         \
        hv[k] = make_float4(0.f, 0.f, 0.f, 0.f);                                                   \
        if (idx_ < HALO * V && (A).in && r_ >= 0 && r_ < (A).h && c_ >= 0 && c_ < (A).w)            \
            hv[k] = ld_g(reinterpret_cast<const float4*>(                                          \
                (A).in + (long long)(P).n * (A).in_ps +                                            \
                ((long long)(r_ >> (A).in_up) * ((A).w >> (A).in_up) + (c_ >> (A).in_up)) * CIN + c4_ * 4)); \
    }
#define WV_LOAD_S(A, Lq, P)                                                                        \
    if constexpr (SYM) {                                                                           \
        /* unconditional loads (clamped address; without symbols a valid dummy one, the first    \
           weight), masked when stored: a load under a branch that converts its result waits    \
           inside the branch, for every load in flight */                                        \
        const bool has_ = (A).sym != nullptr;                                                      \
        const auto sp_ = gmem(has_ ? (A).sym + (long long)(P).n * (A).sym_ps                        \
                                   : reinterpret_cast<const int16_t*>((Lq).w));                    \
        const int ws_ = (A).w >> (A).sym_up;                                                       \
        _Pragma("unroll") for (int k_ = 0; k_ < NS; ++k_) {                                        \
            const int pos_ = tid + k_ * 256;                                                       \
            const int hy_ = pos_ / HALO_W;                                                         \
            const int r_ = (P).r0 + hy_ - 1;                                                       \
            const int c_ = (P).c0 + (pos_ - hy_ * HALO_W) - 1;                                     \
            sok[k_] = has_ && pos_ < HALO && r_ >= 0 && r_ < (A).h && c_ >= 0 && c_ < (A).w &&      \
                      (2 * (r_ & 1) + (c_ & 1)) < (A).sym_step;                                    \
            const int rc_ = min(max(r_, 0), (A).h - 1);                                            \
            const int cc_ = min(max(c_, 0), (A).w - 1);                                            \
            sraw[k_] = sp_[has_ ? (long long)(rc_ >> (A).sym_up) * ws_ + (cc_ >> (A).sym_up) : 0ll]; \
        }                                                                                          \
        _Pragma("unroll") for (int k_ = 0; k_ < NWS; ++k_) {                                       \
            const int idx_ = tid + k_ * 256;                                                       \
            wsv[k_] = 0.f;                                                                         \
            if (idx_ < 3 * NB * 64) {                                                              \
                const int chunk_ = idx_ / (NB * 64);                                               \
                const int rem_ = idx_ - chunk_ * (NB * 64);                                        \
                wsv[k_] = gmem((Lq).wsym)[((long long)chunk_ * (Lq).nbt + (P).ycol * NB) * 64 + rem_]; \
            }                                                                                      \
        }                                                                                          \
    }

    int si = seg_index(it);
    {
        const ConvSeg& S0 = WV_SEG(si);
        const ItemPosF P0 = item_pos_f32<NB, MODE>(S0.L, S0.a, it - S0.item0);
#pragma unroll
        for (int k = 0; k < NH; ++k) WV_LOAD_H(S0.a, P0, k)
        WV_LOAD_S(S0.a, S0.L, P0)
        WV_LOAD_B(S0.L, P0.ycol, 0)
    }

    for (; it < total; it += gridDim.x) {
        const ConvSeg& S = WV_SEG(si);
        const MfmaLayer& L = S.L;
        const ConvArgs& a = S.a;
        const ItemPosF P = item_pos_f32<NB, MODE>(L, a, it - S.item0);
        const int n = P.n, r0 = P.r0, c0 = P.c0, ycol = P.ycol;
        const int nblk0 = ycol * NB;
        const int row0 = wave * 2 + (MODE == CONV_HEAD ? (a.step >> 1) : 0);   // first tile row of this wave

        __syncthreads();   // the previous item is done with every LDS buffer
#pragma unroll
        for (int k = 0; k < NH; ++k) {
            const int idx = tid + k * 256;
            if (idx < HALO * V) {
                const int pos = idx / V;
                *reinterpret_cast<float4*>(lds_in + pos * STRIDE + (idx - pos * V) * 4) = hv[k];
            }
        }
        if constexpr (SYM) {
#pragma unroll
            for (int k = 0; k < NS; ++k)
                if (tid + k * 256 < HALO) lds_s[tid + k * 256] = sok[k] ? (float)sraw[k] : 0.f;
#pragma unroll
            for (int k = 0; k < NWS; ++k)
                if (tid + k * 256 < 3 * NB * 64) lds_ws[tid + k * 256] = wsv[k];
        }
        WV_STORE_B()
        __syncthreads();

        const long long nx = it + gridDim.x;
        const bool has_next = nx < total;
        const int sn = has_next ? seg_index(nx) : si;
        const ConvSeg& SN = WV_SEG(sn);
        const ItemPosF PN = item_pos_f32<NB, MODE>(SN.L, SN.a, nx - SN.item0);

        floatx4 acc[MB][NB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = floatx4{0.f, 0.f, 0.f, 0.f};

#pragma unroll
        for (int tap = 0; tap < TAPS; ++tap) {
            if (tap < TAPS - 1) {
                WV_LOAD_B(L, ycol, tap + 1)   // in flight while this tap computes
            } else if (has_next) {
                WV_LOAD_B(SN.L, PN.ycol, 0)
                WV_LOAD_S(SN.a, SN.L, PN)
            }
            if (has_next) {   // this tap's share of the next item's halo
#pragma unroll
                for (int k = tap * NH / TAPS; k < (tap + 1) * NH / TAPS; ++k) WV_LOAD_H(SN.a, PN, k)
            }
            const int dy = TAPS == 1 ? 1 : tap / 3;
            const int dx = TAPS == 1 ? 1 : tap - dy * 3;
            const float* arow0 = lds_in + ((row0 + dy) * HALO_W + m + dx) * STRIDE + kk * 4;
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                float4 av[MB];
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
                    av[mb] = *reinterpret_cast<const float4*>(arow0 + mb * HALO_W * STRIDE + cb * 16);
                float4 bv[NB];
#pragma unroll
                for (int nb = 0; nb < NB; ++nb) bv[nb] = lds_w[(cb * NB + nb) * 64 + lane];
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb) {
                        acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[mb].x, bv[nb].x, acc[mb][nb], 0, 0, 0);
                        acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[mb].y, bv[nb].y, acc[mb][nb], 0, 0, 0);
                        acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[mb].z, bv[nb].z, acc[mb][nb], 0, 0, 0);
                        acc[mb][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[mb].w, bv[nb].w, acc[mb][nb], 0, 0, 0);
                    }
            }
            if (tap < TAPS - 1) {
                __syncthreads();   // every wave is done with this tap's B
                WV_STORE_B()
                __syncthreads();
            }
        }
    if (SYM) {
#pragma unroll
        for (int chunk = 0; chunk < 3; ++chunk) {
            const int tap = chunk * 4 + kk;
            const int dy = tap / 3;
            const int dx = tap - dy * 3;
            float av[MB];
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
                av[mb] = tap < 9 ? lds_s[(row0 + mb + dy) * HALO_W + m + dx] : 0.f;
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const float bv = lds_ws[(chunk * NB + nb) * 64 + lane];
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
                    acc[mb][nb] =
                        __builtin_amdgcn_mfma_f32_16x16x4f32(av[mb], bv, acc[mb][nb], 0, 0, 0);
            }
        }
    }

    // ---- epilogues.  Lane holds D[4*(lane/16) + i][lane % 16] of each block. ----
    const int col = lane & 15;
    const int rowq = (lane >> 4) * 4;
    if constexpr (MODE == CONV_RELU || MODE == CONV_TANH || MODE == CONV_RES) {
        // Stage the output tile [128 positions][16 NB channels] in LDS (reusing the
        // halo buffer), then write float4 chunks: full, coalesced lines.  CONV_RES
        // adds the skip tensor (same layout as the output) while storing.
        constexpr int OS = NB * 16 + 4;
        static_assert(TILE_H * TILE_W * OS <= LDS_IN, "output tile does not fit the halo buffer");
        __syncthreads();
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const float b = gmem(L.bias)[(nblk0 + nb) * 16 + col];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    float v = acc[mb][nb][i] + b;
                    if (MODE == CONV_RELU) v = fmaxf(v, 0.f);
                    if (MODE == CONV_TANH) v = tanh_fast(v);
                    lds_in[((row0 + mb) * TILE_W + rowq + i) * OS + nb * 16 + col] = v;
                }
            }
        __syncthreads();
        constexpr int V4 = NB * 4;   // float4 chunks per position
        for (int idx = tid; idx < TILE_H * TILE_W * V4; idx += 256) {
            const int pos = idx / V4;
            const int c4 = idx - pos * V4;
            const int r = r0 + pos / TILE_W;
            const int c = c0 + pos % TILE_W;
            if (r < a.h && c < a.w && (nblk0 * 16 + c4 * 4) < L.cout) {
                const long long o = (long long)n * a.out_ps + ((long long)r * a.w + c) * a.out_cs +
                                    nblk0 * 16 + c4 * 4;
                float4 v = *reinterpret_cast<const float4*>(lds_in + pos * OS + c4 * 4);
                if (MODE == CONV_RES) {
                    const float4 k = ld_g(reinterpret_cast<const float4*>(a.skip + o));
                    v = make_float4(v.x + k.x, v.y + k.y, v.z + k.z, v.w + k.w);
                }
                st_g(reinterpret_cast<float4*>(a.out + o), v);
            }
        }
    } else if constexpr (MODE == CONV_LSTM) {
        // Block nb of this workgroup is gate nb (input, forget, cell, output)
        // of channels 16*ycol .. +15 (the packer orders the columns so).
        const int ch = ycol * 16 + col;
        const auto bias = gmem(L.bias);
        const float bi = bias[(nblk0 + 0) * 16 + col];
        const float bf = bias[(nblk0 + 1) * 16 + col];
        const float bg = bias[(nblk0 + 2) * 16 + col];
        const float bo = bias[(nblk0 + 3) * 16 + col];
        const int wp = a.w >> a.cprev_up;
        // All of this lane's previous cell states first (one wait for all of them;
        // c_prev and c_out are different buffers).
        float cp[MB][4];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            const int r = r0 + row0 + mb;
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
        const auto h_out = gmem(a.h_out);
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
            const int r = r0 + row0 + mb;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int c = c0 + rowq + i;
                if (r < a.h && c < a.w) {
                    const float gi = sigmoid_fast(acc[mb][0][i] + bi);
                    const float gf = sigmoid_fast(acc[mb][1][i] + bf);
                    const float gg = tanh_fast(acc[mb][2][i] + bg);
                    const float go = sigmoid_fast(acc[mb][3][i] + bo);
                    const float cn = gf * cp[mb][i] + gi * gg;
                    const float hn = go * tanh_fast(cn);
                    const long long o = (long long)n * a.st_ps + ((long long)r * a.w + c) * a.C + ch;
                    c_out[o] = cn;
                    h_out[o] = hn;
                }
            }
        }
    } else {  // CONV_HEAD: raw 3K outputs of the coded row of each wave -> LDS -> step-g positions
#pragma unroll
        for (int i = 0; i < 4; ++i)
            lds_head[(wave * TILE_W + rowq + i) * 17 + col] = acc[0][0][i] + gmem(L.bias)[col];
        __syncthreads();
        if (tid < 4 * TILE_W) {
            const int wv = tid / TILE_W;
            const int r = r0 + wv * 2 + (a.step >> 1);
            const int c = c0 + tid % TILE_W;
            const int gr = a.step >> 1, gc = a.step & 1;
            if (r < a.h && c < a.w && (c & 1) == gc) {
                const float* v = lds_head + tid * 17;
                const int K = a.K;
                const int wg = (a.w - gc + 1) >> 1;
                const int hg = (a.h - gr + 1) >> 1;
                const long long gi = (long long)(r >> 1) * wg + (c >> 1);
                float* o = a.params + ((long long)n * hg * wg + gi) * 3 * K;
                mixture_head(v, K, a.sigma_min, gmem(o));
            }
        }
    }
        si = sn;
    }
#undef WV_SEG
#undef WV_LOAD_B
#undef WV_STORE_B
#undef WV_LOAD_H
#undef WV_LOAD_S
}

// Resident workgroups of one instantiation on the whole device (queried once).
template <int CIN, int NB, bool SYM, int MODE, int TAPS, bool MULTI>
int resident_f32() {
    static int n = 0;
    if (n == 0) {
        int per_cu = 0, cus = 0, dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, conv3x3_f32p<CIN, NB, SYM, MODE, TAPS, MULTI>, 256,
                                                         0) != hipSuccess ||
            per_cu < 1)
            return 256;
        n = per_cu * cus;
    }
    return n;
}

template <int CIN, int NB, bool SYM, int MODE, int TAPS = 9>
hipError_t launch_t(const MfmaLayer& L, const ConvArgs& a, hipStream_t s) {
    ConvSeg one{};
    one.L = L;
    one.a = a;
    one.item0 = 0;
    const int ncols = (MODE == CONV_HEAD) ? 1 : L.nbt / NB;
    const long long total = (long long)a.tiles_x * a.tiles_y * a.N * ncols;
    const long long res = resident_f32<CIN, NB, SYM, MODE, TAPS, false>();
    long long g = total < res ? total : res;
    if (g < total && g >= 8) g &= ~7ll;   // columns of a tile on one XCD (conv_item_order)
    const unsigned grid = (unsigned)g;
    hipLaunchKernelGGL((conv3x3_f32p<CIN, NB, SYM, MODE, TAPS, false>), dim3(grid), dim3(256), 0, s, nullptr, 0, one,
                       total);
    return hipGetLastError();
}

template <int CIN, int NB, bool SYM>
hipError_t dispatch_mode(const MfmaLayer& L, int mode, int taps, const ConvArgs& a, hipStream_t s) {
    if (taps == 1) {
        if (SYM) return hipErrorInvalidValue;
        switch (mode) {
            case CONV_RELU: return launch_t<CIN, NB, false, CONV_RELU, 1>(L, a, s);
            case CONV_RES: return launch_t<CIN, NB, false, CONV_RES, 1>(L, a, s);
        }
        return hipErrorInvalidValue;
    }
    switch (mode) {
        case CONV_RELU: return launch_t<CIN, NB, SYM, CONV_RELU>(L, a, s);
        case CONV_TANH: return launch_t<CIN, NB, SYM, CONV_TANH>(L, a, s);
        case CONV_RES: return SYM ? hipErrorInvalidValue : launch_t<CIN, NB, false, CONV_RES>(L, a, s);
        case CONV_LSTM: return NB == 4 ? launch_t<CIN, 4, SYM, CONV_LSTM>(L, a, s) : hipErrorInvalidValue;
        case CONV_HEAD: return NB == 1 ? launch_t<CIN, 1, SYM, CONV_HEAD>(L, a, s) : hipErrorInvalidValue;
    }
    return hipErrorInvalidValue;
}

template <int CIN, int NB>
hipError_t dispatch_sym(const MfmaLayer& L, int mode, int taps, const ConvArgs& a, hipStream_t s) {
    return L.has_sym ? dispatch_mode<CIN, NB, true>(L, mode, taps, a, s)
                     : dispatch_mode<CIN, NB, false>(L, mode, taps, a, s);
}

// Output blocks per workgroup.  Small subbands give few position tiles; there
// the output channels are spread over more workgroups (each output's
// accumulation order is unchanged, so the bits are too).
inline int pick_nb(const MfmaLayer& L, int mode, const ConvArgs& a) {
    return conv_pick_nb(L.nbt, mode, (long long)a.tiles_x * a.tiles_y * a.N, 0);
}

template <int CIN>
hipError_t dispatch_nb(const MfmaLayer& L, int mode, int taps, const ConvArgs& a, hipStream_t s) {
    const int nb = pick_nb(L, mode, a);
    switch (nb) {
        case 1: return dispatch_sym<CIN, 1>(L, mode, taps, a, s);
        case 2: return dispatch_sym<CIN, 2>(L, mode, taps, a, s);
        case 4: return dispatch_sym<CIN, 4>(L, mode, taps, a, s);
    }
    return hipErrorInvalidValue;
}

template <int CIN, int NB, bool SYM, int MODE, int TAPS = 9>
hipError_t seg_t(const ConvSeg* segs, int nseg, long long total, int grid, hipStream_t s) {
    const long long res = resident_f32<CIN, NB, SYM, MODE, TAPS, true>();
    long long g = grid < res ? grid : res;
    if (g > total) g = total;
    if (g < total && g >= 8) g &= ~7ll;   // columns of a tile on one XCD (conv_item_order)
    hipLaunchKernelGGL((conv3x3_f32p<CIN, NB, SYM, MODE, TAPS, true>), dim3((unsigned)g), dim3(256), 0, s, segs,
                       nseg, ConvSeg{}, total);
    return hipGetLastError();
}

template <int CIN, int NB, bool SYM>
hipError_t seg_mode(const ConvSeg* segs, int nseg, long long total, int mode, int taps, int grid,
                    hipStream_t s) {
    if (taps == 1) {
        if (SYM) return hipErrorInvalidValue;
        switch (mode) {
            case CONV_RELU: return seg_t<CIN, NB, false, CONV_RELU, 1>(segs, nseg, total, grid, s);
            case CONV_RES: return seg_t<CIN, NB, false, CONV_RES, 1>(segs, nseg, total, grid, s);
        }
        return hipErrorInvalidValue;
    }
    switch (mode) {
        case CONV_RELU: return seg_t<CIN, NB, SYM, CONV_RELU>(segs, nseg, total, grid, s);
        case CONV_RES: return SYM ? hipErrorInvalidValue : seg_t<CIN, NB, false, CONV_RES>(segs, nseg, total, grid, s);
        case CONV_LSTM: return NB == 4 ? seg_t<CIN, 4, SYM, CONV_LSTM>(segs, nseg, total, grid, s) : hipErrorInvalidValue;
        case CONV_HEAD: return NB == 1 ? seg_t<CIN, 1, SYM, CONV_HEAD>(segs, nseg, total, grid, s) : hipErrorInvalidValue;
    }
    return hipErrorInvalidValue;
}

template <int CIN>
hipError_t seg_nb(const ConvSeg* segs, int nseg, long long total, int sym, int mode, int taps, int nb,
                  int grid, hipStream_t s) {
#define WV_SEG_NB(NBV)                                                                   \
    if (nb == NBV) return sym ? seg_mode<CIN, NBV, true>(segs, nseg, total, mode, taps, grid, s) \
                              : seg_mode<CIN, NBV, false>(segs, nseg, total, mode, taps, grid, s);
    WV_SEG_NB(1) WV_SEG_NB(2) WV_SEG_NB(4)
#undef WV_SEG_NB
    return hipErrorInvalidValue;
}

}  // namespace

// Output-channel blocks per workgroup.  Four blocks reuse each A fragment most
// and win when the tiles fill the device for two or more rounds of resident
// workgroups (2 per CU); with fewer tiles, narrower blocks give more, shorter
// workgroups and a smaller last round (measured per level on the 512x768 image:
// FP32 best at one block, BF16/FP8 at two).  The choice never changes results.
int conv_pick_nb(int nbt, int mode, long long tiles, int lowp) {
    if (mode == CONV_HEAD) return 1;
    if (mode == CONV_LSTM) return 4;
    const int widest = nbt >= 4 ? 4 : nbt;
    if (tiles >= 1024) return widest;
    const int narrow = lowp ? 2 : 1;
    return narrow < widest ? narrow : widest;
}
int conv_tile_h(int bf16) { return bf16 ? 16 : TILE_H; }
int conv_tile_w(int bf16) { return bf16 ? 16 : TILE_W; }

hipError_t launch_conv_seg(const ConvSeg* segs, int nseg, long long total, const MfmaLayer& proto,
                           int mode, int nb, int grid, hipStream_t s) {
    if (total <= 0 || nseg <= 0) return hipSuccess;
    const int taps = proto.taps == 1 ? 1 : 9;
    switch (proto.cin) {
        case 16: return seg_nb<16>(segs, nseg, total, proto.has_sym, mode, taps, nb, grid, s);
        case 32: return seg_nb<32>(segs, nseg, total, proto.has_sym, mode, taps, nb, grid, s);
        case 64: return seg_nb<64>(segs, nseg, total, proto.has_sym, mode, taps, nb, grid, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_conv(const MfmaLayer& L, int mode, const ConvArgs& a, hipStream_t s) {
    if (a.N <= 0 || a.h <= 0 || a.w <= 0) return hipSuccess;
    if (mode == CONV_LSTM && L.nbt % 4 != 0) return hipErrorInvalidValue;
    const int taps = L.taps == 1 ? 1 : 9;
    switch (L.cin) {
        case 16: return dispatch_nb<16>(L, mode, taps, a, s);
        case 32: return dispatch_nb<32>(L, mode, taps, a, s);
        case 64: return dispatch_nb<64>(L, mode, taps, a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace wv
