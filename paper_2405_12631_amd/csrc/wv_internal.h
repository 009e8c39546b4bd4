// Internal declarations shared by the C ABI (wv_api.hip) and the kernels
// (wv_conv.hip, wv_lift.hip, wv_cdf.hip).  Not installed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/wv.h"

namespace wv {

// Strided 2-D view of a stack of planes: element (n, r, c) lives at
// p[n * ps + r * rs + c * cs].  Used to read even/odd samples of a plane
// and to write subbands straight into the packed layout without copies.
struct View {
    float* p;
    long long ps;
    int rs, cs;
};
struct CView {
    const float* p;
    long long ps;
    int rs, cs;
};
inline CView cview(View v) { return CView{v.p, v.ps, v.rs, v.cs}; }

// Output tile of one conv workgroup: TILE_H x TILE_W positions, 4 waves, each
// wave two rows of 16 positions.
constexpr int TILE_H = 8;
constexpr int TILE_W = 16;

// Epilogue of the MFMA conv kernel.
// CONV_RES: out = skip + (conv + bias), no activation (residual blocks).
enum ConvMode { CONV_RELU = 0, CONV_TANH = 1, CONV_LSTM = 2, CONV_HEAD = 3, CONV_RES = 4 };

// One conv3x3 layer repacked for the MFMA kernel (see pack_mfma_layer):
//   w    : [9][cin/16][nbt][64 lanes][4]  float B fragments
//   wsym : [3][nbt][64 lanes]             symbol-channel B fragments or null
//   bias : [nbt * 16]
struct MfmaLayer {
    const float* w;
    const float* wsym;
    const float* bias;
    int cin;       // float input channels (multiple of 16)
    int cout;      // real output channels
    int nbt;       // output blocks of 16 (padded)
    int has_sym;   // 1: extra input channel 0 read from int16 symbols
    int taps;      // 9: 3x3 conv (w holds 9 taps); 1: 1x1 conv
};

// BF16 variant: w [9][cin/32][nbt][64 lanes][8 bf16], wsym [nbt][64 lanes][8 bf16]
// (element j of lane group kk is tap 8 kk + j), bias FP32 [nbt * 16].
// Reduced-precision layer: BF16 weights (scale == nullptr), or FP8 e4m3 weights
// with one FP32 scale per packed output column (the accumulator is multiplied by
// it before the bias).  The symbol-channel weights are BF16 in both cases (for
// FP8 already divided by the column's scale).
struct MfmaLayer16 {
    const uint16_t* w;
    const uint16_t* wsym;
    const float* bias;
    const float* scale;
    int cin, cout, nbt, has_sym;
};

// A 1 -> C or C -> 1 lifting conv for the vector kernels: w [9][C], bias [C] / [1].
struct VecLayer {
    const float* w;
    const float* bias;
    int ch;
};

struct ConvArgs {
    const float* in;       // NHWC float input [N][h >> in_up][w >> in_up][cin], or null (zeros)
    long long in_ps;       // plane stride (floats)
    int in_up;             // 1: nearest x2 upsampling on read
    const int16_t* sym;    // symbol channel base (plane 0 of this subband) or null (zeros)
    long long sym_ps;      // plane stride of the packed symbols
    int sym_up;            // 1: symbol plane at half resolution (nearest x2)
    int sym_step;          // positions with group >= sym_step read as zero
    float* out;            // NHWC output [N][h][w][out_cs]
    long long out_ps;
    int out_cs;
    const float* skip;     // CONV_RES: tensor added to the output (same layout)
    int N, h, w, tiles_x, tiles_y;
    // CONV_LSTM
    const float* c_prev;   // NHWC [N][h >> cprev_up][w >> cprev_up][C] or null (zeros)
    long long cprev_ps;
    int cprev_up;
    float* h_out;          // NHWC [N][h][w][C]
    float* c_out;
    long long st_ps;
    int C;
    // Reduced-precision kernels: activations / hidden state in BF16, or FP8 e4m3
    // (one byte) when the layer has scales; same strides, in elements.
    const uint16_t* in16;
    uint16_t* out16;
    uint16_t* h16_out;
    // CONV_HEAD
    float* params;         // [N][n_g][3K]
    int step, K;
    float sigma_min;
};

// Order of the work items (tile, channel column) of a conv launch with ncols
// columns per tile.  Workgroup i runs on XCD i mod 8, and every XCD has its own
// L2.  Here the ncols items of one tile get indices 8 apart and consecutive in
// their XCD's dispatch order.  In a grid of a multiple of 8 workgroups (or one
// item per workgroup) the columns of a tile then run at the same time on one
// XCD, and the tile's input halo comes from HBM once instead of ncols times.
// Tiles past the last full group of 8 keep the plain order.  The mapping is a
// bijection of [0, ntiles * ncols), so the results do not depend on it.
__device__ __forceinline__ void conv_item_order(long long local, long long ntiles, int ncols, long long& tile,
                                                int& ycol) {
    const long long t8 = ntiles & ~7ll;
    if (local < t8 * ncols) {
        const long long q = local >> 3;
        ycol = (int)(q % ncols);
        tile = (q / ncols) * 8 + (local & 7);
    } else {
        const long long r = local - t8 * ncols;
        const long long rest = ntiles - t8;
        ycol = (int)(r / rest);
        tile = t8 + r % rest;
    }
}

// One segment of a persistent multi-segment conv launch: its own layer (weights),
// arguments and first work item (items = tiles * columns of 16 NB channels).
struct ConvSeg {
    MfmaLayer L;
    ConvArgs a;
    long long item0;
};
struct ConvSeg16 {
    MfmaLayer16 L;
    ConvArgs a;
    long long item0;
};

// One segment of a fused step-stack launch (wv_stack_bf16.hip): a plane group's
// subband at one coding step.  Layers 0..2 (64 -> 64 BF16, ReLU; layer 0 with the
// symbol chunk wsym when step >= 1) and the head (64 -> 3K, one column block),
// packed as MfmaLayer16.  Work items: planes x vertical segments of seg_rows rows x
// strips of 58 columns.
struct StackSeg {
    const uint16_t* w16[4];
    const uint16_t* wsym;
    const float* bias[4];
    const uint16_t* in16;   // l_i, NHWC BF16 [N][h][w][64]
    long long in_ps;        // plane stride (elements)
    const int16_t* sym;     // this subband's symbols of plane 0 in the packed layout, or null
    long long sym_ps;
    float* params;          // [N][n_g][3K]
    int N, h, w, step, K;
    float sigma_min;
    int strips_x, segs_y, seg_rows;
    long long item0;
};
constexpr int STACK_STRIP = 58;   // output columns per strip

// One segment of a fused ConvLSTM launch (wv_lstm_bf16.hip): a plane group's subband at
// step 0.  Gates = conv3x3([q of the previous subband, h of the previous subband]) with the
// packed BF16 LSTM layer; inputs read at (r >> up, c >> up) when the resolution doubled.
// Work items: planes x vertical segments of seg_rows rows x strips of LSTM_STRIP columns.
struct LstmSeg {
    const uint16_t* wt;     // packed weights [tap][32-channel chunk][16-column block][64 lanes] (uint4)
    const uint16_t* wsym;   // symbol-channel weights [block][64 lanes] (uint4)
    const float* bias;      // [256] in packed column order
    const uint16_t* in16;   // h of the previous subband, NHWC BF16, or null (zeros)
    long long in_ps;
    const int16_t* sym;     // symbols of the previous subband (plane 0, packed layout), or null
    long long sym_ps;
    const float* c_prev;    // c of the previous subband, NHWC FP32, or null
    long long cprev_ps;
    uint16_t* h_out;        // NHWC BF16 [N][h][w][64]
    float* c_out;           // NHWC FP32
    long long st_ps;
    int N, h, w, up;        // up: inputs at half resolution (nearest x2)
    int strips_x, segs_y, seg_rows;
    long long item0;
};
constexpr int LSTM_STRIP = 64;   // output columns per strip

// Launchers (return hipSuccess or the launch error).
hipError_t launch_conv(const MfmaLayer& L, int mode, const ConvArgs& a, hipStream_t s);
hipError_t launch_conv_bf16(const MfmaLayer16& L, int mode, const ConvArgs& a, hipStream_t s);
// Persistent launches over device segment arrays.  `proto` gives the template
// shape shared by every segment (cin, has_sym, taps); nb output blocks per item.
hipError_t launch_conv_seg(const ConvSeg* segs, int nseg, long long total, const MfmaLayer& proto,
                           int mode, int nb, int grid, hipStream_t s);
hipError_t launch_conv_seg_bf16(const ConvSeg16* segs, int nseg, long long total,
                                const MfmaLayer16& proto, int mode, int nb, int grid, hipStream_t s);
// Fused BF16 step stacks over device segment arrays (has_sym: every segment has step >= 1).
hipError_t launch_stack_bf16(const StackSeg* segs, int nseg, long long total, int has_sym, int grid,
                             hipStream_t s);
// Fused BF16 ConvLSTM over device segment arrays.
hipError_t launch_lstm_bf16(const LstmSeg* segs, int nseg, long long total, int grid, hipStream_t s);
// Output blocks per workgroup chosen for a launch of `tiles` position tiles.
int conv_pick_nb(int nbt, int mode, long long tiles, int lowp);
int conv_tile_h(int bf16);
int conv_tile_w(int bf16);

// Lifting filter pieces.
//   first: a1[n][r][c][ch] = tanh(b[ch] + sum_tap w[tap][ch] z(n, r+dy-1, c+dx-1))
//   last : v = b + sum_tap,ch w[tap][ch] a2[n][r+dy-1][c+dx-1][ch];
//          f = (predict ? z + v : z/2 + v), rounded if lift_int;
//          out(n, r, c) = A(n, r, c) + sign * f
hipError_t launch_lift_first(const VecLayer& L, CView z, int N, int h, int w, float* a1,
                             hipStream_t s);
hipError_t launch_lift_last(const VecLayer& L, const float* a2, CView z, CView A, View out,
                            int N, int h, int w, int predict, float sign, int lift_int,
                            hipStream_t s);

// Depth-wise 3x3 conv, NHWC float, C channels: w [9][C], b [C].
hipError_t launch_dwconv(const float* in, const float* w, const float* b, float* out, int N, int h,
                         int w_, int C, hipStream_t s);
// Autoregressive LL model (wv_ar.hip): 12 causal taps of a 5x5 window.
constexpr int AR_TAPS = 12;
struct ArModel {
    const float *w1, *b1;   // [A][12] (taps in raster order of the window), [A]
    const float *w2, *b2;   // [A][A], [A]
    const float *w3, *b3;   // [3K][A], [3K]
    int A, K, dist;
    float sigma_min;
};
struct ArStreams {
    const uint8_t* bytes;    // all planes' LL streams back to back
    const long long* offs;   // device [N + 1]: plane n's stream is bytes[offs[n] .. offs[n+1])
};
hipError_t launch_ar_params(const ArModel& M, const int16_t* q, long long q_ps, int h, int w, int N,
                            float* params, hipStream_t s);
hipError_t launch_ar_decode(const ArModel& M, const ArStreams& S, int16_t* q, long long q_ps, int h,
                            int w, int N, int smin, int nsym, int* status, hipStream_t s);
// A whole three-layer predict/update filter and its lifting update in one kernel.
// Row-streaming form for 32-channel filters (wv_lift_rows.hip): the first `nstrips` strips of
// LIFT_ROWS_OUTW output columns (the last one may be partial); launch_lift_fused takes it for
// arrays of at least LIFT_ROWS_MIN_STRIP_ROWS (strip x row) units.
constexpr int LIFT_ROWS_OUTW = 124;
constexpr long long LIFT_ROWS_MIN_STRIP_ROWS = 2048;
hipError_t launch_lift_rows(const VecLayer& L1, const MfmaLayer& L2, const VecLayer& L3, CView z, CView A, View out,
                            int N, int h, int w, int nstrips, int predict, float sign, int lift_int, hipStream_t s);
hipError_t launch_lift_fused(const VecLayer& L1, const MfmaLayer& L2, const VecLayer& L3, CView z, CView A,
                             View out, int N, int h, int w, int predict, float sign, int lift_int,
                             hipStream_t s);
// Zero `bytes` bytes at p (16-byte aligned) with a kernel.
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_center_u8(const uint8_t* x8, float* xf, long long n, hipStream_t s);
hipError_t launch_quantize(const float* y, int16_t* q, int N, long long per_plane, long long n_ll,
                           float dL, float dH, int smin, int smax, int* clip, hipStream_t s);
hipError_t launch_dequantize(const int16_t* q, float* y, int N, long long per_plane,
                             long long n_ll, float dL, float dH, hipStream_t s);
hipError_t launch_finalize(float* x, uint8_t* u8, long long n, float offset, hipStream_t s);
// Subband impulse responses.  Per subband i: offset and size of q_i in the
// image's packed layout, offset and width of subband i in the S x S pyramid;
// (ph, pw) = (H / S, W / S) is the max-pooling window.
constexpr int MAX_SUB = 25;
struct SirMeta {
    long long off[MAX_SUB], soff[MAX_SUB];
    int h[MAX_SUB], w[MAX_SUB], sw[MAX_SUB];
    int nsub, S, ph, pw;
};
hipError_t launch_sir_keys(const int16_t* q, unsigned long long* keys, const SirMeta& m,
                           long long max_n, hipStream_t s);
hipError_t launch_sir_pyramid(const unsigned long long* keys, const SirMeta& m, float dL, float dH,
                              float* y, hipStream_t s);
hipError_t launch_scatter(const uint8_t* sym, int16_t* q, int N, long long q_ps, long long off,
                          int h, int w, int step, int smin, hipStream_t s);
hipError_t launch_gather(const int16_t* q, uint8_t* sym, int N, long long q_ps, long long off,
                         int h, int w, int step, int smin, hipStream_t s);
size_t cdf_trim_scratch_bytes(long long n);
// The trim's scratch as a file-scope device array (wv_cdf_trim_noalloc): its size, and
// its address on the current device (looked up once per device).
constexpr size_t TRIM_STATIC_SCRATCH_BYTES = 256 * 1024;
constexpr long long TRIM_STATIC_MAX_ROWS = (long long)(TRIM_STATIC_SCRATCH_BYTES / sizeof(long long)) * 256;
constexpr int TRIM_MAX_DEVICES = 64;
hipError_t cdf_trim_static_scratch(long long** out);
hipError_t launch_cdf_trim(const uint16_t* cdf, long long n, int nsym, uint8_t* lolen, uint16_t* packed,
                           long long* scratch, hipStream_t s);
hipError_t launch_cdf(const float* params, long long n, int K, int dist, int smin, int nsym,
                      uint16_t* cdf, hipStream_t s);
hipError_t launch_thaar(float* f, float* tmp, int T, long long n, int inverse, hipStream_t s);

}  // namespace wv
