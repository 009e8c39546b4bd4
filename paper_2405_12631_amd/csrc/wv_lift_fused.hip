// One predict/update filter application in a single kernel (Sec. 3.1):
//   out = A + sign * f,  f = z + N(z) (predict) or z/2 + N(z) (update),
//   N = conv3x3(C -> 1) . tanh . conv3x3(C -> C) . tanh . conv3x3(1 -> C),
// every conv zero-padded at the array border.  A workgroup owns an OH x OW
// output tile and keeps the whole chain in LDS: z on an (OH+6) x (OW+6) halo,
// the first layer on (OH+4) x (OW+4) positions (vector ALUs), the second on
// (OH+2) x (OW+2) positions as an implicit GEMM on v_mfma_f32_16x16x4f32 (its
// output then overwrites the first layer's buffer), the last layer and the
// update on the outputs.  Positions outside the array are zero in every layer,
// which is exactly the per-layer zero padding of the definition.
//
// Tile: 8 x 16 outputs and 4 waves (two workgroups per CU), or, for the
// 32-channel filters over large arrays, 16 x 32 outputs and 8 waves (layer 2
// on 612 positions = 39 of the 40 M blocks the waves take, 1.25x the outputs,
// where the 8 x 16 tile pays 1.5x).
//
// Persistent: a workgroup loads the three layers' weights into LDS once and
// then walks tiles blockIdx.x, + gridDim.x, ...; the next tile's z halo is
// read into registers while this tile's layer-2 MFMAs run.
#include "wv_device.h"
#include "wv_internal.h"

#include <atomic>

namespace wv {
namespace {

typedef float floatx4 __attribute__((ext_vector_type(4)));

template <int C, int OH, int OW, int NWV>
__global__ __launch_bounds__(64 * NWV) void lift_fused_k(const VecLayer L1, const MfmaLayer L2, const VecLayer L3,
                                                        const CView z, const CView A, const View out, int N,
                                                        int h, int w, int tiles_x, int tiles_y, int cbeg,
                                                        int predict, float sign, int lift_int, int total) {
    constexpr int NT = 64 * NWV;            // threads
    constexpr int ZH = OH + 6, ZW = OW + 6;   // z halo
    constexpr int AH = OH + 4, AW = OW + 4;   // first layer region
    constexpr int BH = OH + 2, BW = OW + 2;   // second layer region
    constexpr int S1 = C + 4;               // floats per position in the layer buffers
    constexpr int NP2 = BH * BW;            // second-layer positions
    constexpr int MB2 = (NP2 + 15) / 16;    // M blocks
    constexpr int CB = C / 16;              // K chunks (16 channels) per tap
    constexpr int NBT = C / 16;             // output blocks of 16
    constexpr int MBW = (MB2 + NWV - 1) / NWV;   // most M blocks a wave takes
    static_assert((2 * OH * OW) % NT == 0, "layer 3 takes two threads per output in whole rounds");
    __shared__ float zs[ZH * ZW];
    __shared__ __attribute__((aligned(16))) float act[AH * AW * S1];   // layer 1, then layer 2
    __shared__ __attribute__((aligned(16))) float4 w2s[9 * CB * NBT * 64];
    __shared__ float w1s[9 * C], b1s[C], b2s[C];
    __shared__ __attribute__((aligned(16))) float w3s[9 * C];

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    struct Tile { int n, r0, c0; };
    auto tile_of = [&](int t) {
        Tile T;
        const int tx = t % tiles_x;
        t /= tiles_x;
        const int ty = t % tiles_y;
        T.n = t / tiles_y;
        T.r0 = ty * OH;
        T.c0 = cbeg + tx * OW;
        return T;
    };
    // z halo of a tile, NZ positions per thread
    constexpr int NZ = (ZH * ZW + NT - 1) / NT;
    float zv_next[NZ];
    auto load_z = [&](const Tile& T) {
        const float* zp = z.p + (long long)T.n * z.ps;
#pragma unroll
        for (int k = 0; k < NZ; ++k) {
            const int i = tid + k * NT;
            const int r = T.r0 - 3 + i / ZW, c = T.c0 - 3 + i % ZW;
            zv_next[k] = 0.f;
            if (i < ZH * ZW && r >= 0 && r < h && c >= 0 && c < w)
                zv_next[k] = zp[(long long)r * z.rs + (long long)c * z.cs];
        }
    };

    if ((int)blockIdx.x >= total) return;
    load_z(tile_of(blockIdx.x));
    // weights, once per workgroup; every thread's loads are in flight before its first store
    {
        constexpr int NW = (9 * CB * NBT * 64 + NT - 1) / NT;
        float4 wv[NW];
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            const int i = tid + k * NT;
            wv[k] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (i < 9 * CB * NBT * 64) wv[k] = reinterpret_cast<const float4*>(L2.w)[i];
        }
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            const int i = tid + k * NT;
            if (i < 9 * CB * NBT * 64) w2s[i] = wv[k];
        }
    }
    for (int i = tid; i < 9 * C; i += NT) {
        w1s[i] = L1.w[i];
        w3s[i] = L3.w[i];
    }
    for (int i = tid; i < C; i += NT) {
        b1s[i] = L1.bias[i];
        b2s[i] = L2.bias[i];
    }
    const float b3 = L3.bias[0];
    constexpr int NTASK = 2 * OH * OW / NT;   // layer-3 rounds (two threads per output)

  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    const Tile T = tile_of(t);
    const int n = T.n, r0 = T.r0, c0 = T.c0;
    __syncthreads();   // the previous tile is done with zs and act (and the weights are in LDS)
#pragma unroll
    for (int k = 0; k < NZ; ++k)
        if (tid + k * NT < ZH * ZW) zs[tid + k * NT] = zv_next[k];
    __syncthreads();
    // The array this tile updates, one value per output of this thread's layer-3 rounds: read
    // now, used after layer 3.
    float apre[NTASK];
#pragma unroll
    for (int j = 0; j < NTASK; ++j) {
        const int o = (j * NT + tid) >> 1;
        const int r = r0 + o / OW, c = c0 + o % OW;
        apre[j] = 0.f;
        if (((j * NT + tid) & 1) == 0 && r < h && c < w)
            apre[j] = A.p[(long long)n * A.ps + (long long)r * A.rs + (long long)c * A.cs];
    }

    // layer 1 on the (OH+4) x (OW+4) region: tanh(b1 + sum_tap w1 z), zero outside the array.
    // A thread always takes the same four channels (NT is a multiple of C / 4), so their 36
    // weights and 4 biases are read from LDS once per tile.
    static_assert(NT % (C / 4) == 0, "fixed channel group per thread");
    {
        const int c4 = (tid % (C / 4)) * 4;
        float w1r[9][4], b1r[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            b1r[j] = b1s[c4 + j];
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) w1r[tap][j] = w1s[tap * C + c4 + j];
        }
        for (int pos = tid / (C / 4); pos < AH * AW; pos += NT / (C / 4)) {
            const int ay = pos / AW, ax = pos % AW;
            const int r = r0 - 2 + ay, c = c0 - 2 + ax;
            float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
            if (r >= 0 && r < h && c >= 0 && c < w) {
                float zv[9];
#pragma unroll
                for (int tap = 0; tap < 9; ++tap) zv[tap] = zs[(ay + tap / 3) * ZW + ax + tap % 3];
                float s[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    s[j] = b1r[j];
#pragma unroll
                    for (int tap = 0; tap < 9; ++tap) s[j] = fmaf(w1r[tap][j], zv[tap], s[j]);
                }
                v = make_float4(tanh_fast(s[0]), tanh_fast(s[1]), tanh_fast(s[2]), tanh_fast(s[3]));
            }
            *reinterpret_cast<float4*>(act + pos * S1 + c4) = v;
        }
    }
    __syncthreads();

    // layer 2 on the (OH+2) x (OW+2) region: MFMA over K = 9 taps x C channels
    const int m = lane & 15;
    const int kk = lane >> 4;
    // Wave w takes M blocks [mb0, mb0 + mcnt): MB2 split as evenly as whole blocks allow.
    const int mcnt = MB2 / NWV + (wave < MB2 % NWV ? 1 : 0);
    const int mb0 = wave * (MB2 / NWV) + (wave < MB2 % NWV ? wave : MB2 % NWV);
    floatx4 acc[MBW][NBT];
    int apos[MBW];
#pragma unroll
    for (int j = 0; j < MBW; ++j) {
        const int mb = mb0 + j;
        int p = mb * 16 + m;
        p = p < NP2 && j < mcnt ? p : NP2 - 1;              // dummy rows read a valid position
        apos[j] = (p / BW) * AW + (p % BW);
#pragma unroll
        for (int nb = 0; nb < NBT; ++nb) acc[j][nb] = floatx4{0.f, 0.f, 0.f, 0.f};
    }
    // (tap, 16-channel chunk) steps in order; the fragments of the next step are
    // read while this step's MFMAs run (fully unrolled: the double buffer stays
    // in registers).
    float4 afr[2][MBW], bfr[2][NBT];
#define WV_LOAD_F(buf, tp, cbv)                                                                     \
    {                                                                                               \
        _Pragma("unroll") for (int nb_ = 0; nb_ < NBT; ++nb_) bfr[buf][nb_] =                       \
            w2s[(((tp) * CB + (cbv)) * NBT + nb_) * 64 + lane];                                     \
        _Pragma("unroll") for (int j_ = 0; j_ < MBW; ++j_) afr[buf][j_] = *reinterpret_cast<const float4*>( \
            act + (apos[j_] + ((tp) / 3) * AW + (tp) % 3) * S1 + (cbv) * 16 + kk * 4);              \
    }
#define WV_STEP(cur, st)                                                                            \
    {                                                                                               \
        if ((st) + 1 < 9 * CB) WV_LOAD_F((cur) ^ 1, ((st) + 1) / CB, ((st) + 1) % CB)                 \
        _Pragma("unroll") for (int j = 0; j < MBW; ++j) if (MB2 % NWV == 0 || j < mcnt)             \
            _Pragma("unroll") for (int nb = 0; nb < NBT; ++nb) {                                    \
            acc[j][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(afr[cur][j].x, bfr[cur][nb].x, acc[j][nb], 0, 0, 0); \
            acc[j][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(afr[cur][j].y, bfr[cur][nb].y, acc[j][nb], 0, 0, 0); \
            acc[j][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(afr[cur][j].z, bfr[cur][nb].z, acc[j][nb], 0, 0, 0); \
            acc[j][nb] = __builtin_amdgcn_mfma_f32_16x16x4f32(afr[cur][j].w, bfr[cur][nb].w, acc[j][nb], 0, 0, 0); \
        }                                                                                           \
    }
    if (t + (int)gridDim.x < total) load_z(tile_of(t + gridDim.x));   // in flight during the MFMAs
    WV_LOAD_F(0, 0, 0)
    for (int st = 0; st + 1 < 9 * CB; st += 2) {   // pairs of steps: buffer 0, then buffer 1
        WV_STEP(0, st)
        WV_STEP(1, st + 1)
    }
    if ((9 * CB) & 1) WV_STEP(0, 9 * CB - 1)
#undef WV_STEP
#undef WV_LOAD_F
    __syncthreads();   // layer 1 is dead; its buffer takes layer 2
    const int col = lane & 15;
    const int rowq = (lane >> 4) * 4;
#pragma unroll
    for (int j = 0; j < MBW; ++j) {
        if (MB2 % NWV != 0 && j >= mcnt) continue;
        const int mb = mb0 + j;
#pragma unroll
        for (int nb = 0; nb < NBT; ++nb) {
            const int ch = nb * 16 + col;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int p = mb * 16 + rowq + i;
                if (p >= NP2) continue;
                const int r = r0 - 1 + p / BW, c = c0 - 1 + p % BW;
                const bool in = r >= 0 && r < h && c >= 0 && c < w;
                act[p * S1 + ch] = in ? tanh_fast(acc[j][nb][i] + b2s[ch]) : 0.f;
            }
        }
    }
    __syncthreads();

    // layer 3 and the lifting update: two threads per output, halves of the channels
#pragma unroll
    for (int j = 0; j < NTASK; ++j) {
        const int task = j * NT + tid;
        const int o = task >> 1;
        const int half = task & 1;
        const int oy = o / OW, ox = o % OW;
        float s = 0.f;
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const float4* ap = reinterpret_cast<const float4*>(act + ((oy + tap / 3) * BW + ox + tap % 3) * S1 +
                                                               half * (C / 2));
            const float4* wp = reinterpret_cast<const float4*>(w3s + tap * C + half * (C / 2));
#pragma unroll
            for (int k = 0; k < C / 8; ++k) {
                const float4 av = ap[k], wv = wp[k];
                s = fmaf(wv.x, av.x, s);
                s = fmaf(wv.y, av.y, s);
                s = fmaf(wv.z, av.z, s);
                s = fmaf(wv.w, av.w, s);
            }
        }
        const float other = __shfl_xor(s, 1);
        const int r = r0 + oy, c = c0 + ox;
        if (half == 0 && r < h && c < w) {
            const float v = b3 + (s + other);
            const float zz = zs[(oy + 3) * ZW + ox + 3];
            float f = predict ? zz + v : 0.5f * zz + v;
            if (lift_int) f = rintf(f);
            out.p[(long long)n * out.ps + (long long)r * out.rs + (long long)c * out.cs] = apre[j] + sign * f;
        }
    }
  }
}

template <int C, int OH, int OW, int NWV>
long long lift_resident() {   // resident workgroups, cached per device (256 if unknown)
    static std::atomic<long long> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    long long n = cache[dev].load(std::memory_order_relaxed);
    if (n == 0) {
        int per_cu = 0, cus = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, lift_fused_k<C, OH, OW, NWV>, 64 * NWV, 0) !=
                hipSuccess ||
            per_cu < 1)
            return 256;
        n = (long long)per_cu * cus;
        cache[dev].store(n, std::memory_order_relaxed);
    }
    return n;
}

template <int C, int OH, int OW, int NWV>
hipError_t lift_launch(const VecLayer& L1, const MfmaLayer& L2, const VecLayer& L3, CView z, CView A, View out, int N,
                       int h, int w, int predict, float sign, int lift_int, hipStream_t s, int cbeg = 0) {
    const int tx = (w - cbeg + OW - 1) / OW, ty = (h + OH - 1) / OH;
    const long long total = (long long)tx * ty * N;
    if (total >= (1ll << 31)) return hipErrorInvalidValue;
    const long long res = lift_resident<C, OH, OW, NWV>();
    const long long g = total < res ? total : res;
    hipLaunchKernelGGL((lift_fused_k<C, OH, OW, NWV>), dim3((unsigned)g), dim3(64 * NWV), 0, s, L1, L2, L3, z, A, out,
                       N, h, w, tx, ty, cbeg, predict, sign, lift_int, (int)total);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_lift_fused(const VecLayer& L1, const MfmaLayer& L2, const VecLayer& L3, CView z, CView A,
                             View out, int N, int h, int w, int predict, float sign, int lift_int,
                             hipStream_t s) {
    if ((long long)N * h * w == 0) return hipSuccess;
    if (L1.ch == 32 && L2.cin == 32 && L2.nbt == 2) {
        // Wide arrays stream rows (wv_lift_rows.hip) in 124-column strips; a last strip that
        // would be less than 70 % used is left to the tiles as a band of the remaining columns
        // (a whole strip costs the same however much of it is used).  Measured on the 64-image
        // batch: 1088 x 1920 arrays (960-, 480-, 240-, 120-column: last strips 74-97 % used) 13 %
        // faster in rows than in tiles; 512- and 384-column arrays 20-30 % slower in rows alone
        // (last strips 13 % and 10 % used), and with the band the batch's lifting went from
        // 115.3 to 110.9 ms.  WV_LIFT_FORM=tile / rows forces one form where it applies (tests
        // compare them bit for bit).
        const char* env = getenv("WV_LIFT_FORM");
        const bool force_tile = env && env[0] == 't', force_rows = env && env[0] == 'r';
        const int full = w / LIFT_ROWS_OUTW, rem = w - full * LIFT_ROWS_OUTW;
        const bool partial = 10 * rem >= 7 * LIFT_ROWS_OUTW;   // the last strip in rows too
        const int nrows = full + (partial ? 1 : 0);              // strips in rows
        if (!force_tile && nrows > 0 &&
            (force_rows || (long long)nrows * N * h >= LIFT_ROWS_MIN_STRIP_ROWS)) {
            hipError_t e = launch_lift_rows(L1, L2, L3, z, A, out, N, h, w, nrows, predict, sign, lift_int, s);
            if (e != hipSuccess || partial || rem == 0) return e;
            return lift_launch<32, 8, 16, 4>(L1, L2, L3, z, A, out, N, h, w, predict, sign, lift_int, s,
                                             full * LIFT_ROWS_OUTW);
        }
        // The 16 x 32 tile needs one 8-wave workgroup per CU, whose phases (vector layer 1, MFMA
        // layer 2, layer 3) no longer overlap with a second workgroup's; it pays off only where
        // its lower recompute has many rounds of tiles to work on (measured: 1088 x 1920 planes
        // 5.37 -> 4.63 ms per synthesis, 512 x 768 planes 1.26 -> 1.52 ms).
        const long long big = (long long)((w + 31) / 32) * ((h + 15) / 16) * N;
        if (big >= 2048)
            return lift_launch<32, 16, 32, 8>(L1, L2, L3, z, A, out, N, h, w, predict, sign, lift_int, s);
        return lift_launch<32, 8, 16, 4>(L1, L2, L3, z, A, out, N, h, w, predict, sign, lift_int, s);
    }
    if (L1.ch == 16 && L2.cin == 16 && L2.nbt == 1)
        return lift_launch<16, 8, 16, 4>(L1, L2, L3, z, A, out, N, h, w, predict, sign, lift_int, s);
    return hipErrorInvalidValue;
}

}  // namespace wv
