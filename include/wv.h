/*
 * wv.h - C ABI of the MI355X (gfx950) four-step learned-wavelet decode path.
 *
 * Method: A. Meyer, S. Prativadibhayankaram, A. Kaup, "Efficient Learned
 * Wavelet Image and Video Coding", ICIP 2024 (arXiv 2405.12631).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Device memory is owned by the caller and passed as raw device pointers.
 *   The library allocates no device memory; it owns only host-side handles.
 * - Every GPU entry point enqueues work asynchronously on the caller's
 *   stream (a hipStream_t passed as void*, NULL = the default stream) and
 *   returns before the work finishes.  Inputs must stay valid until then.
 * - Return value: WV_OK (0) or a negative WV_E* code.  wv_last_error()
 *   returns a thread-local message for the last failure.  No entry point
 *   exits, aborts or throws.
 * - Shapes are checked on the host before any launch.  H and W must be
 *   divisible by 2^levels (WV_ESHAPE otherwise).  A device fault is reported
 *   as WV_EDEVICE by the call that observes it.
 * - "Plane": one colour component (Sec. 3.1 codes each YCbCr component as
 *   its own plane).  nplanes planes of one size are processed per call; all
 *   planes share the model.
 * - Subband order is the coding order LL_J, HL_J, LH_J, HH_J, ..., HL_1,
 *   LH_1, HH_1 (Sec. 3.1, Fig. 1; Fig. 11 caption).  A plane's quantised
 *   symbols are packed subband after subband, each row-major:
 *   q[plane][offset_i + r * w_i + c], offsets from wv_layout().
 * - Coding step g of a subband codes the positions with
 *   2 * (r mod 2) + (c mod 2) == g, in raster order (Sec. 3.2, Fig. 3:
 *   four steps, a quarter of the positions each, 0/2/6/8 coded 3x3
 *   neighbours).  n_g = ceil((h - g/2) / 2) * ceil((w - g%2) / 2).
 */
#ifndef WV_H
#define WV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    WV_OK = 0,
    WV_EINVAL = -1,       /* bad argument (null pointer, bad enum, bad config) */
    WV_ESHAPE = -2,       /* image or buffer shape not supported */
    WV_EORDER = -3,       /* subband/step out of range, or not the successor of the
                             last call on the same state buffer (coding order) */
    WV_EDEVICE = -4,      /* HIP runtime error or device fault */
    WV_ECORRUPT = -5,     /* corrupt or truncated bitstream */
    WV_EUNSUPPORTED = -6, /* configuration the kernels do not implement */
    WV_ENOMEM = -7        /* caller-provided buffer too small */
};

/* Arithmetic of the context-model convolutions (ConvLSTM and step stacks; the
 * lifting transform, the mixture head's epilogue and the CDF tables are FP32 in
 * every mode).  WV_BF16: BF16 operands and activations, FP32 accumulation.
 * WV_FP8: e4m3 weights with one FP32 scale per output channel (scale = max |w|
 * of the channel / 448), e4m3 activations (unscaled, saturated at +-448),
 * FP32 accumulation, symbols fed through a BF16 chunk so they stay exact.
 * Reduced precision needs ctx_ch of 32 or 64 and ctx_arch 0. */
typedef enum { WV_FP32 = 0, WV_BF16 = 1, WV_FP8 = 2 } wv_precision;

/* Component family of the per-coefficient mixture.  Sec. 3.1 uses a Laplacian
 * (mean and scale); the workload's default is a K-component Gaussian mixture. */
typedef enum { WV_DIST_GAUSS = 0, WV_DIST_LAPLACE = 1 } wv_dist;

/* Model hyper-parameters.  Sec. 3.1 (lifting), Sec. 3.2 (context model). */
typedef struct wv_config {
    int levels;      /* J decomposition levels (3J+1 subbands)                 */
    int lift_ch;     /* channels inside a predict/update filter (16 or 32)     */
    int lift_layers; /* conv3x3 layers per predict/update filter (>= 2)        */
    int ctx_ch;      /* C: ConvLSTM hidden channels = step-stack width (32/64) */
    int ctx_layers;  /* conv3x3 layers per coding-step stack (>= 2)            */
    int mix_k;       /* K Gaussian components per coefficient (1..4)           */
    int sym_min;     /* symbol alphabet [sym_min, sym_max], at most 255 symbols */
    int sym_max;
    int cdf_bits;    /* CDF precision: tables sum to 2^cdf_bits (16)           */
    float sigma_min; /* lower bound of the mixture scales, symbol units        */
    int lift_int;    /* 1: predict/update outputs rounded (lossless lifting)   */
    int dist;        /* wv_dist: mixture component family                     */
    int ctx_arch;    /* 0: plain conv stacks; 1: DepthConvBlock (step 0) and
                        Residual Block (steps 1-3) stacks, Sec. 3.2 (FP32 only) */
    int ll_ar;       /* 1: LL_J coded autoregressively in raster order (Sec. 3.2,
                        the paper's default) instead of in four steps      */
    int ar_ch;       /* channels of the autoregressive LL model (32 or 64)    */
} wv_config;

/* One subband of the packed layout. type: 0 LL, 1 HL, 2 LH, 3 HH. */
typedef struct wv_subband {
    int h, w, level, type;
    long long offset; /* first coefficient within a plane */
} wv_subband;

typedef struct wv_model wv_model;

const char* wv_last_error(void);
int wv_version(void);

/*
 * Weight blob.  A flat float32 array, tensors in this order, each conv as
 * weight [Cout][Cin][3][3] then bias [Cout]:
 *   P_row, U_row, P_col, U_col: lift_layers convs each,
 *       1 -> lift_ch, lift_ch -> lift_ch (lift_layers - 2 times), lift_ch -> 1;
 *   ConvLSTM gates: (1 + ctx_ch) -> 4 ctx_ch, gate blocks input, forget,
 *       cell, output; input channel 0 the previous subband's symbols;
 *   16 step stacks, subband type LL, HL, LH, HH (outer) x step 0..3 (inner),
 *       ctx_layers convs each: Cin_g -> ctx_ch, ctx_ch -> ctx_ch
 *       (ctx_layers - 2 times), ctx_ch -> 3K; Cin_0 = ctx_ch, Cin_g = 1 + ctx_ch
 *       for g >= 1 with channel 0 the current subband's coded symbols.
 *   With ctx_arch = 1 each stack is instead: in (3x3, Cin_g -> C); step 0 a
 *       DepthConvBlock p1a (1x1 [C][C][1][1]), dw (depth-wise [C][1][3][3]),
 *       p1b, p2a, p2b (1x1); steps 1-3 a Residual Block ra, rb (3x3 C -> C);
 *       out (3x3, C -> 3K).
 *   With ll_ar = 1, appended: ar.0 (5x5, 1 -> ar_ch; only the 12 causal taps,
 *       the two rows above and the two positions to the left, are used),
 *       ar.1 (1x1, ar_ch -> ar_ch), ar.2 (1x1, ar_ch -> 3K).
 * wv_weights_count: number of floats of that blob for cfg.
 */
int wv_weights_count(const wv_config* cfg, long long* n_floats);

/* Bytes of device memory the caller provides to wv_model_create for the
 * kernels' repacked weights. */
int wv_pack_bytes(const wv_config* cfg, int precision, size_t* bytes);

/*
 * Build a model handle.  d_weights: the blob above, in device memory
 * (read once, synchronously on `stream`, and not referenced afterwards).
 * d_pack: caller-owned device buffer of wv_pack_bytes() bytes that the model
 * reads for its whole lifetime.  The handle is immutable; concurrent calls on
 * different streams are safe if they use different workspaces.
 */
int wv_model_create(const wv_config* cfg, const float* d_weights, long long n_floats,
                    int precision, void* d_pack, size_t pack_bytes, void* stream,
                    wv_model** out);
void wv_model_destroy(wv_model* m);

/* Subband layout of an H x W plane: up to `cap` entries in coding order and the
 * number of coefficients per plane (= H * W). */
int wv_layout(const wv_config* cfg, int H, int W, wv_subband* out, int cap,
              long long* coefs_per_plane);

/* n_g of coding step `step` of an h x w subband. */
long long wv_group_count(int h, int w, int step);

/*
 * Device workspace sizes for nplanes planes of H x W:
 *   state_bytes   - ConvLSTM state (h, c), kept between wv_context_params calls;
 *   scratch_bytes - temporary memory of any single call (analyze, context,
 *                   synthesize); contents are not kept between calls.
 */
int wv_workspace_bytes(const wv_model* m, int nplanes, int H, int W,
                       size_t* state_bytes, size_t* scratch_bytes);

/*
 * Analysis transform and quantisation (encoder side).  Sec. 3.1, Fig. 2:
 * J levels of 1-D lifting row-wise then column-wise, HP = odd - P(even),
 * LP = even + U(HP), P(z) = z + N_P(z), U(z) = z/2 + N_U(z); then
 * q = clamp(round_half_even(y * Delta), sym_min, sym_max), Delta_L for LL_J,
 * Delta_H for the rest.
 *   d_x8   : uint8 planes [nplanes][H][W] (centred as x - 128), or NULL;
 *   d_xf   : float planes [nplanes][H][W] already centred, used if d_x8 NULL;
 *   d_q    : int16 [nplanes][H*W] packed symbols (output);
 *   d_y    : optional float [nplanes][H*W] packed unquantised subbands;
 *   d_clip : optional int32 counter; += number of clamped coefficients
 *            (the caller zeroes it).
 */
int wv_analyze(const wv_model* m, const uint8_t* d_x8, const float* d_xf, int nplanes,
               int H, int W, float delta_L, float delta_H, void* d_scratch,
               int16_t* d_q, float* d_y, int* d_clip, void* stream);

/*
 * Entropy parameters of coding step `step` of subband `subband` (Sec. 3.2).
 * step == 0 first advances the ConvLSTM long context (h, c) in d_state from
 * the previous subband to this one (input: the previous subband's symbols,
 * state and input upsampled x2 when the resolution doubles; zero state and
 * input for subband 0).  The step stack then reads the long context and, for
 * step >= 1, the symbols of steps < step of this subband; it never reads
 * positions of later steps or later subbands (causality).
 * Calls must come in coding order per plane set: (0,0), (0,1), ..., (0,3),
 * (1,0), ...; step 0 of subband i needs subband i-1 fully decoded in d_q.
 *   d_params : float [nplanes][n_g][3K] = (w_0..w_{K-1}, mu_0.., sigma_0..),
 *              w = softmax, mu raw, sigma = max(softplus, sigma_min),
 *              in symbol units.
 */
int wv_context_params(const wv_model* m, const int16_t* d_q, int nplanes, int H, int W,
                      int subband, int step, float* d_state, void* d_scratch,
                      float* d_params, void* stream);
/* Coding order (Sec. 3.2: each step reads the symbols of the steps before it, and
 * step 0 carries the long context over from the previous subband).  The library
 * remembers, per state buffer d_state, the (subband, step) of the last call that
 * returned WV_OK and returns WV_EORDER, launching nothing, for a call that is not
 * its successor: (i, g + 1) after (i, g) for g < 3, (i + 1, 0) after (i, 3).  (0, 0)
 * is accepted at any time and starts a new decode; after the last step of the
 * last subband only (0, 0) is.  With ll_ar = 1 the LL steps 1-3 are optional:
 * (1, 0) may follow any step of subband 0.  A call that fails leaves the cursor
 * where it was.  Calls on one state buffer must not overlap in time. */

/*
 * 16-bit CDF tables of n discretised K-component mixtures.  The paper
 * arithmetic-codes the symbols with the estimated distribution (Sec. 3.1);
 * the table format is this library's:
 *   N_s = sym_max - sym_min + 1, F_max = 2^cdf_bits - N_s,
 *   C_j = sum_k w_k Phi((sym_min + j - 0.5 - mu_k) / sigma_k) / sum_k w_k,
 *   Phi the standard normal CDF (dist = WV_DIST_GAUSS) or the standard
 *   Laplace CDF (WV_DIST_LAPLACE, sigma the Laplace scale),
 *   F_j = floor(F_max * C_j) (exact value: from the upper tail where
 *   C_j > 1/2, never F_max), running maximum, cdf[j] = j + F_j, j = 0..N_s-1;
 *   cdf[N_s] = 2^cdf_bits stored as 0 (mod 2^16).  Every symbol has
 *   frequency >= 1.
 *   d_params : float [n][3K];  d_cdf : uint16 [n][N_s + 1].
 * Requires cdf_bits == 16 and N_s <= 255.
 */
int wv_cdf_tables(const float* d_params, long long n, int mix_k, int dist, int sym_min,
                  int sym_max, int cdf_bits, uint16_t* d_cdf, void* stream);

/*
 * Autoregressive LL model (ll_ar = 1; Sec. 3.2, Fig. 4a: the LL subband is
 * coded from its own causal spatial context, one symbol at a time in raster
 * order).  Parameters of a position: its 12 causal neighbours in a 5x5 window
 * (zero outside the subband) -> ReLU(conv) -> ReLU(1x1) -> 1x1 -> the mixture
 * head of wv_context_params.
 *   wv_ar_params: encoder side; every LL position of every plane at once from
 *     the known symbols d_q; d_params float [nplanes][h_J * w_J][3K] in raster
 *     order (rows for wv_cdf_tables; the plane's stream is one rANS stream
 *     over the raster order).
 *   wv_ar_decode: decoder side; walks LL in raster order on the GPU, one
 *     workgroup per plane, computing each position's parameters and CDF row
 *     and rANS-decoding its symbol in the kernel (stream format of
 *     wv_rans_decode).  d_bytes: the planes' LL streams back to back,
 *     d_offsets int64 [nplanes + 1] (device); writes LL of d_q; d_status int
 *     [nplanes]: 0, or 1 for a corrupt or truncated stream (the walk still
 *     finishes).  Needs w_J <= 4096.
 */
int wv_ar_params(const wv_model* m, const int16_t* d_q, int nplanes, int H, int W,
                 float* d_params, void* stream);
int wv_ar_decode(const wv_model* m, const uint8_t* d_bytes, const long long* d_offsets,
                 int nplanes, int H, int W, int16_t* d_q, int* d_status, void* stream);

/*
 * Plans: several groups of planes of different sizes decoded together, each
 * layer of a coding step running as ONE persistent launch over all groups
 * (a work list of per-group segments, walked with a static stride: no
 * atomics, results bit-identical to the per-group calls).  A group is
 * nplanes planes of H x W with its own symbols and workspace, exactly the
 * buffers wv_context_params would take for it.  Segment descriptors for
 * every layer of every step are built once, on the host, and uploaded into
 * d_desc; afterwards a step launches with no copies, so a whole decode can be
 * captured in a graph and replayed.  Needs ctx_arch 0.
 *   nb_table: optional [levels] output-channel blocks per workgroup (1, 2, 4)
 *             of the inner layers of level j subbands, from an autotuner;
 *             NULL picks by occupancy.  The choice does not change results.
 *   wv_plan_bytes: descriptor bytes, and the largest row count of a step.
 *   wv_plan_create: d_params float [max_rows][3K]: the parameters of one
 *             step, group after group (group b from row group_first[b]).
 *   wv_plan_rows: rows of step (subband, step) and each group's first row.
 *   wv_plan_context_params: as wv_context_params for every group.
 *   wv_plan_scatter: d_sym uint8 laid out like the parameters' rows.
 */
typedef struct wv_group {
    int H, W, nplanes;
    int16_t* d_q;     /* [nplanes][H*W] */
    float* d_state;   /* wv_workspace_bytes(state) for this group */
    void* d_scratch;  /* wv_workspace_bytes(scratch) for this group */
} wv_group;
typedef struct wv_plan wv_plan;

int wv_plan_bytes(const wv_model* m, int ngroups, const wv_group* groups, const int* nb_table,
                  size_t* desc_bytes, long long* max_rows);
int wv_plan_create(const wv_model* m, int ngroups, const wv_group* groups, const int* nb_table,
                   void* d_desc, size_t desc_bytes, float* d_params, void* stream, wv_plan** out);
void wv_plan_destroy(wv_plan* p);
int wv_plan_rows(const wv_plan* p, int subband, int step, long long* rows, long long* group_first);
int wv_plan_context_params(wv_plan* p, int subband, int step, void* stream);
int wv_plan_scatter(const wv_plan* p, const uint8_t* d_sym, int subband, int step, void* stream);

/* wv_plan_context_params follows the coding order of wv_context_params, with one
 * cursor for all of the plan's groups (held by the plan). */

/*
 * Continuous batching: one call runs the coding step (subband, step) of each
 * item, where every item is a plane group (like a wv_group) at its own
 * position in its own decode.  The items' layers are grouped into one
 * persistent launch per role (ConvLSTM; first layer without / with the symbol
 * channel; each inner layer; the head), segments carrying their own weights.
 * Results are bit-identical to calling wv_context_params per item.
 * Descriptors are written to h_staging (pinned host memory the caller keeps
 * untouched until the stream has passed this call) and copied to d_desc
 * asynchronously; *used_bytes receives the bytes needed (n = 0 or
 * h_staging == NULL with d_desc == NULL queries them).  Needs ctx_arch 0.
 * Every item's (subband, step) must be the successor of the last call on its
 * d_state (the coding order of wv_context_params); if one is not, the call
 * returns WV_EORDER and launches nothing.  Two items may not share a d_state.
 */
typedef struct wv_step_item {
    int H, W, nplanes;
    int16_t* d_q;
    float* d_state;
    void* d_scratch;
    int subband, step;
    float* d_params;  /* [nplanes][n_g][3K] of this item */
} wv_step_item;

int wv_context_params_items(const wv_model* m, int n, const wv_step_item* items, void* h_staging,
                            size_t staging_bytes, void* d_desc, size_t desc_bytes,
                            size_t* used_bytes, void* stream);

/* Write decoded symbol indices (symbol - sym_min) of step `step` of subband
 * `subband` into the packed symbols: d_sym uint8 [nplanes][n_g]. */
int wv_scatter_symbols(const wv_config* cfg, const uint8_t* d_sym, int nplanes, int H, int W,
                       int subband, int step, int16_t* d_q, void* stream);

/* Encoder side: read the symbol indices of one step, d_sym uint8 [nplanes][n_g]. */
int wv_gather_symbols(const wv_config* cfg, const int16_t* d_q, int nplanes, int H, int W,
                      int subband, int step, uint8_t* d_sym, void* stream);

/*
 * Dequantisation and synthesis (Sec. 3.1): y_hat = q / Delta, then the exact
 * inverse of wv_analyze level by level, then + offset (128 undoes the
 * centring of uint8 input; 0 for planes analysed as centred floats).
 *   d_q or d_y (float packed subbands, used when d_q is NULL);
 *   d_xhat : float [nplanes][H][W];  d_u8 : optional uint8 clamp(rint(x_hat)).
 */
int wv_synthesize(const wv_model* m, const int16_t* d_q, const float* d_y, int nplanes,
                  int H, int W, float delta_L, float delta_H, float offset, void* d_scratch,
                  float* d_xhat, uint8_t* d_u8, void* stream);

/* Elementwise helpers of the video path: out = x - 128 (uint8 -> float), and
 * x += offset with an optional uint8 copy clamp(rint(x)). */
int wv_center_u8(const uint8_t* d_x8, long long n, float* d_out, void* stream);
int wv_add_offset(float* d_x, long long n, float offset, uint8_t* d_u8, void* stream);

/*
 * Subband impulse responses (Sec. 3.4) of one plane's quantised subbands
 * d_q [H*W] (packed layout).  For every subband i, the largest |q_i| is placed
 * into the i-th subband of an otherwise all-zero S x S pyramid, S = 2^levels
 * (the level-J subbands are 1 x 1); its cell is the arg-max of |q_i|
 * max-pooled by (H/S) x (W/S) windows, the first in raster order on ties.
 * The pyramid is dequantised (/ Delta) and inverse transformed without the
 * +128 offset.  d_out: float [3J+1][S][S].  d_scratch:
 * wv_impulse_scratch_bytes() bytes.
 */
int wv_impulse_scratch_bytes(const wv_model* m, size_t* bytes);
int wv_impulse_responses(const wv_model* m, const int16_t* d_q, int H, int W, float delta_L,
                         float delta_H, void* d_scratch, float* d_out, void* stream);

/*
 * Temporal Haar lifting over a GOP of T = 2^levels frames of n floats each
 * (lifting form of Sec. 3.3 without motion compensation): H = f_odd - f_even,
 * L = f_even + H/2, recursively on L.  Subband order: L_J, H_J, H_{J-1} (2),
 * ..., H_1 (T/2).  In place on d_frames [T][n]; T a power of two <= 32.
 */
int wv_temporal_haar_forward(float* d_frames, int T, long long n, void* stream);
int wv_temporal_haar_inverse(float* d_frames, int T, long long n, void* stream);

/*
 * Lossless trim of CDF rows for the copy to the host coder (the tables of
 * wv_cdf_tables, Sec. 3.1).  With F_j = cdf[j] - j (j = 1 .. nsym-1), F is
 * non-decreasing, 0 below the row's probability-mass window and F_max - 1
 * above it (F_max = 2^16 - nsym; the upper tail always keeps one count), so a
 * row is fixed by
 *   lo  = 1 + #{j : F_j = 0},   len = #{j : 0 < F_j < F_max - 1},
 * and F_lo .. F_{lo+len-1}.  wv_cdf_trim (device, stream-ordered) writes
 * d_lolen uint8 [n][2] = (lo, len) and the rows' F values back to back in row
 * order into d_packed (uint16; packed_cap >= n (nsym - 1), the worst case; only
 * the first sum(len) entries are written).  d_scratch: device buffer of
 * wv_cdf_trim_scratch_bytes(n) bytes.  The host recovers the offsets from the
 * lengths, so a copy needs 2 n + 2 sum(len) bytes instead of 2 n (nsym + 1).
 * wv_cdf_untrim (host) rebuilds the full tables (WV_ECORRUPT if (lo, len) are
 * out of range or sum(len) != packed_count).  wv_rans_encode_trim /
 * wv_rans_decode_trim: the coder below driven by trimmed tables; identical
 * streams and symbols to the full-table calls.
 */
int wv_cdf_trim_scratch_bytes(long long n, size_t* bytes);
int wv_cdf_trim(const uint16_t* d_cdf, long long n, int nsym, uint8_t* d_lolen, uint16_t* d_packed,
                long long packed_cap, void* d_scratch, size_t scratch_bytes, void* stream);
/*
 * wv_cdf_trim_noalloc: wv_cdf_trim for callers that cannot allocate device memory
 * (code under graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, results and stream order as wv_cdf_trim, without
 * the scratch argument: the block sums go to a 256 KiB array of the library's
 * own (a file-scope device array, one per GPU, held until the process ends), so
 * at most 8,388,608 rows per call (more: WV_ENOMEM, nothing launched).  The call
 * allocates nothing.  Every call on a GPU uses that GPU's one array and leaves
 * its contents behind (each entry a call reads it first writes, so nothing needs
 * clearing); calls that overlap in time on one GPU (two streams, two threads)
 * race on it and must be serialised by the caller.
 */
int wv_cdf_trim_noalloc(const uint16_t* d_cdf, long long n, int nsym, uint8_t* d_lolen, uint16_t* d_packed,
                        long long packed_cap, void* stream);
int wv_cdf_untrim(const uint8_t* lolen, const uint16_t* packed, long long packed_count, int nsym,
                  long long n, uint16_t* cdf_out);
int wv_rans_encode_trim(const uint8_t* lolen, const uint16_t* packed, long long packed_count, int nsym,
                        const uint8_t* sym, long long n, uint8_t* out, size_t cap, size_t* len);
int wv_rans_decode_trim(const uint8_t* lolen, const uint16_t* packed, long long packed_count, int nsym,
                        long long n, const uint8_t* in, size_t len, uint8_t* sym_out);

/*
 * Host rANS coder (no GPU).  Byte-wise renormalising rANS with a 32-bit state
 * in [2^23, 2^31) and M = 2^16: symbols are encoded last to first so the
 * decoder emits them in raster order; the stream starts with the final state
 * (4 bytes, little endian).  cdf rows as produced by wv_cdf_tables (row
 * stride nsym + 1, final entry 0 meaning 2^16).
 *   encode: out capacity `cap`; *len receives the stream length;
 *           WV_ENOMEM if cap is too small.
 *   decode: WV_ECORRUPT on a truncated or inconsistent stream.
 */
int wv_rans_encode(const uint16_t* cdf, int nsym, const uint8_t* sym, long long n,
                   uint8_t* out, size_t cap, size_t* len);
int wv_rans_decode(const uint16_t* cdf, int nsym, long long n, const uint8_t* in, size_t len,
                   uint8_t* sym_out);

/*
 * Graphs of library calls.  wv_graph_begin starts capturing the work that
 * library calls enqueue on `stream` (a stream created by the caller, not the
 * default stream; capture mode thread-local); wv_graph_end stops and
 * instantiates it.  Between the two the caller issues device entry points only
 * (no host synchronisation, no allocation, no host coder): for example one
 * coder-elided decode of a plan, every (subband, step)'s
 * wv_plan_context_params, wv_cdf_tables and wv_plan_scatter, then
 * wv_synthesize per group.  Host-side checks (shapes, coding order) run once,
 * at capture; wv_graph_launch replays the recorded kernels with the same
 * pointers, so every buffer must stay allocated while the graph lives.  Replays
 * on one stream run in order.  A failed call inside a capture leaves the
 * capture open: the caller still calls wv_graph_end (which then fails).
 *
 * wv_zero: zero `bytes` bytes at the 16-byte aligned device pointer d with a
 * kernel (replays correctly inside a graph, where memset nodes are avoided).
 */
typedef struct wv_graph wv_graph;
int wv_graph_begin(void* stream);
int wv_graph_end(void* stream, wv_graph** out);
int wv_graph_launch(const wv_graph* g, void* stream);
void wv_graph_destroy(wv_graph* g);
int wv_zero(void* d, size_t bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* WV_H */
