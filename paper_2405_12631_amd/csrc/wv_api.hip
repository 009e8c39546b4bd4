// C ABI of the four-step learned-wavelet decode path (declarations and
// documentation in include/wv.h).  Host code: argument checks, weight
// repacking, workspace layout and the launch sequence of each call.
#include <stdarg.h>
#include <algorithm>
#include <cmath>
#include <stdio.h>
#include <string.h>

#include <array>
#include <atomic>
#include <mutex>
#include <string>
#include <unordered_map>
#include <vector>

#include "wv_internal.h"
#include "wv_pieces.h"

using namespace wv;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_err;

static int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHK(expr)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(WV_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));     \
    } while (0)

extern "C" const char* wv_last_error(void) { return g_err.c_str(); }
extern "C" int wv_version(void) { return 100; }

// ---------------------------------------------------------------------------
// config, blob manifest
// ---------------------------------------------------------------------------
static int check_cfg(const wv_config* c) {
    if (!c) return fail(WV_EINVAL, "null config");
    if (c->levels < 1 || c->levels > 8) return fail(WV_EINVAL, "levels must be 1..8");
    if (c->lift_ch != 16 && c->lift_ch != 32) return fail(WV_EUNSUPPORTED, "lift_ch must be 16 or 32");
    if (c->lift_layers < 2) return fail(WV_EINVAL, "lift_layers must be >= 2");
    if (c->ctx_ch != 16 && c->ctx_ch != 32 && c->ctx_ch != 64)
        return fail(WV_EUNSUPPORTED, "ctx_ch must be 16, 32 or 64");
    if (c->ctx_layers < 2) return fail(WV_EINVAL, "ctx_layers must be >= 2");
    if (c->mix_k < 1 || c->mix_k > 4) return fail(WV_EUNSUPPORTED, "mix_k must be 1..4");
    const int nsym = c->sym_max - c->sym_min + 1;
    if (nsym < 2 || nsym > 255) return fail(WV_EUNSUPPORTED, "alphabet must have 2..255 symbols");
    if (c->sym_min < -32768 || c->sym_max > 32767) return fail(WV_EINVAL, "alphabet exceeds int16");
    if (c->cdf_bits != 16) return fail(WV_EUNSUPPORTED, "cdf_bits must be 16");
    if (!(c->sigma_min > 0.f)) return fail(WV_EINVAL, "sigma_min must be > 0");
    if (c->dist != WV_DIST_GAUSS && c->dist != WV_DIST_LAPLACE) return fail(WV_EINVAL, "bad dist");
    if (c->ctx_arch != 0 && c->ctx_arch != 1) return fail(WV_EINVAL, "bad ctx_arch");
    if (c->ll_ar != 0 && c->ll_ar != 1) return fail(WV_EINVAL, "bad ll_ar");
    if (c->ll_ar && c->ar_ch != 32 && c->ar_ch != 64) return fail(WV_EUNSUPPORTED, "ar_ch must be 32 or 64");
    return WV_OK;
}

namespace {

struct ConvShape {
    int cin, cout;
    long long w_off, b_off;   // float offsets in the blob
    int ks2 = 9;              // taps per filter (9 for 3x3, 1 for 1x1)
};

// Block architecture of one (type, step) stack, in blob order.
struct BlockShapes {
    ConvShape in, p1a, dw, p1b, p2a, p2b, ra, rb, out;   // dw: depth-wise [C][1][3][3]
};

struct Manifest {
    std::vector<ConvShape> lift[4];   // P_row, U_row, P_col, U_col
    ConvShape lstm;
    std::vector<ConvShape> ctx[4][4]; // [type][step], plain stacks
    BlockShapes blk[4][4];            // [type][step], ctx_arch == 1
    ConvShape ar0, ar1, ar2;          // ll_ar == 1: 5x5 (1 -> A), 1x1 (A -> A), 1x1 (A -> 3K)
    long long total = 0;
};

Manifest make_manifest(const wv_config& c) {
    Manifest m;
    long long off = 0;
    auto conv = [&](int cin, int cout, int ks2 = 9) {
        ConvShape s{cin, cout, off, 0, ks2};
        off += (long long)cout * cin * ks2;
        s.b_off = off;
        off += cout;
        return s;
    };
    for (int f = 0; f < 4; ++f) {
        std::vector<int> ch;
        ch.push_back(1);
        for (int l = 0; l < c.lift_layers - 1; ++l) ch.push_back(c.lift_ch);
        ch.push_back(1);
        for (size_t l = 0; l + 1 < ch.size(); ++l) m.lift[f].push_back(conv(ch[l], ch[l + 1]));
    }
    m.lstm = conv(1 + c.ctx_ch, 4 * c.ctx_ch);
    const int C = c.ctx_ch;
    for (int t = 0; t < 4; ++t)
        for (int g = 0; g < 4; ++g) {
            if (c.ctx_arch == 1) {
                BlockShapes& b = m.blk[t][g];
                b.in = conv(g == 0 ? C : C + 1, C);
                if (g == 0) {
                    b.p1a = conv(C, C, 1);
                    b.dw = conv(1, C);   // [C][1][3][3]
                    b.p1b = conv(C, C, 1);
                    b.p2a = conv(C, C, 1);
                    b.p2b = conv(C, C, 1);
                } else {
                    b.ra = conv(C, C);
                    b.rb = conv(C, C);
                }
                b.out = conv(C, 3 * c.mix_k);
                continue;
            }
            std::vector<int> ch;
            ch.push_back(g == 0 ? c.ctx_ch : 1 + c.ctx_ch);
            for (int l = 0; l < c.ctx_layers - 1; ++l) ch.push_back(c.ctx_ch);
            ch.push_back(3 * c.mix_k);
            for (size_t l = 0; l + 1 < ch.size(); ++l) m.ctx[t][g].push_back(conv(ch[l], ch[l + 1]));
        }
    if (c.ll_ar) {
        m.ar0 = conv(1, c.ar_ch, 25);
        m.ar1 = conv(c.ar_ch, c.ar_ch, 1);
        m.ar2 = conv(c.ar_ch, 3 * c.mix_k, 1);
    }
    m.total = off;
    return m;
}

// Host-side repacked model before upload.
struct PackBuf {
    std::vector<float> data;
    size_t add(size_t nfloats) {   // 256-byte aligned sub-buffer
        size_t off = (data.size() + 63) & ~(size_t)63;
        data.resize(off + nfloats, 0.f);
        return off;
    }
};

struct MfmaRef { size_t w, wsym, bias, scale; int cin, cout, nbt, has_sym, taps; };
struct VecRef { size_t w, bias; int ch; };

// Original output channel of packed column nc.  LSTM: columns are grouped by
// 64 = (input, forget, cell, output) x 16 channels so that one workgroup's
// accumulators hold all four gates of the same channels.
static int perm_col(int nc, int C, bool lstm) {
    if (!lstm) return nc;
    const int j = nc / 64, gate = (nc % 64) / 16, ch = 16 * j + nc % 16;
    return gate * C + ch;
}

MfmaRef pack_mfma(PackBuf& pb, const float* blob, const ConvShape& s, int has_sym, bool lstm,
                  int C) {
    MfmaRef r{};
    r.cin = s.cin - has_sym;
    r.cout = s.cout;
    r.nbt = (s.cout + 15) / 16;
    r.has_sym = has_sym;
    r.taps = s.ks2;
    const int CB = r.cin / 16;
    const int cin_total = s.cin;
    const int KS2 = s.ks2;
    const float* W = blob + s.w_off;
    const float* B = blob + s.b_off;
    r.w = pb.add((size_t)KS2 * CB * r.nbt * 256);
    r.wsym = has_sym ? pb.add((size_t)3 * r.nbt * 64) : 0;
    r.bias = pb.add((size_t)r.nbt * 16);
    float* pw = pb.data.data() + r.w;
    for (int tap = 0; tap < KS2; ++tap)
        for (int cb = 0; cb < CB; ++cb)
            for (int nb = 0; nb < r.nbt; ++nb)
                for (int lane = 0; lane < 64; ++lane)
                    for (int t = 0; t < 4; ++t) {
                        const int kk = lane >> 4, nn = lane & 15;
                        const int k = 16 * cb + 4 * kk + t;
                        const int nc = nb * 16 + nn;
                        float v = 0.f;
                        if (nc < s.cout) {
                            const int o = perm_col(nc, C, lstm);
                            v = W[((long long)o * cin_total + has_sym + k) * KS2 + tap];
                        }
                        pw[(((size_t)(tap * CB + cb) * r.nbt + nb) * 64 + lane) * 4 + t] = v;
                    }
    if (has_sym) {
        float* ps = pb.data.data() + r.wsym;
        for (int chunk = 0; chunk < 3; ++chunk)
            for (int nb = 0; nb < r.nbt; ++nb)
                for (int lane = 0; lane < 64; ++lane) {
                    const int kk = lane >> 4, nn = lane & 15;
                    const int tap = chunk * 4 + kk;
                    const int nc = nb * 16 + nn;
                    float v = 0.f;
                    if (tap < 9 && nc < s.cout)
                        v = W[((long long)perm_col(nc, C, lstm) * cin_total + 0) * 9 + tap];
                    ps[((size_t)chunk * r.nbt + nb) * 64 + lane] = v;
                }
    }
    float* pbias = pb.data.data() + r.bias;
    for (int nc = 0; nc < s.cout; ++nc) pbias[nc] = B[perm_col(nc, C, lstm)];
    return r;
}

static uint16_t host_f2bf(float f) {   // round to nearest even
    uint32_t u;
    memcpy(&u, &f, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// BF16 layer: B fragments of 8 consecutive K per lane, K chunk = 32 channels.
// Stored in the float pack buffer; offsets count floats, so 2 bf16 per float.
MfmaRef pack_mfma16(PackBuf& pb, const float* blob, const ConvShape& s, int has_sym, bool lstm,
                    int C) {
    MfmaRef r{};
    r.cin = s.cin - has_sym;
    r.cout = s.cout;
    r.nbt = (s.cout + 15) / 16;
    r.has_sym = has_sym;
    r.taps = 9;
    const int CC = r.cin / 32;
    const int cin_total = s.cin;
    const float* W = blob + s.w_off;
    const float* B = blob + s.b_off;
    r.w = pb.add((size_t)9 * CC * r.nbt * 64 * 4);          // 8 bf16 = 4 floats per lane
    r.wsym = has_sym ? pb.add((size_t)r.nbt * 64 * 4) : 0;
    r.bias = pb.add((size_t)r.nbt * 16);
    uint16_t* pw = reinterpret_cast<uint16_t*>(pb.data.data() + r.w);
    for (int tap = 0; tap < 9; ++tap)
        for (int cc = 0; cc < CC; ++cc)
            for (int nb = 0; nb < r.nbt; ++nb)
                for (int lane = 0; lane < 64; ++lane)
                    for (int j = 0; j < 8; ++j) {
                        const int kk = lane >> 4, nn = lane & 15;
                        const int k = 32 * cc + 8 * kk + j;
                        const int nc = nb * 16 + nn;
                        float v = 0.f;
                        if (nc < s.cout)
                            v = W[((long long)perm_col(nc, C, lstm) * cin_total + has_sym + k) * 9 + tap];
                        pw[((((size_t)(tap * CC + cc) * r.nbt + nb) * 64 + lane) * 8) + j] = host_f2bf(v);
                    }
    if (has_sym) {
        uint16_t* ps = reinterpret_cast<uint16_t*>(pb.data.data() + r.wsym);
        for (int nb = 0; nb < r.nbt; ++nb)
            for (int lane = 0; lane < 64; ++lane)
                for (int j = 0; j < 8; ++j) {
                    const int kk = lane >> 4, nn = lane & 15;
                    const int tap = 8 * kk + j;
                    const int nc = nb * 16 + nn;
                    float v = 0.f;
                    if (tap < 9 && nc < s.cout)
                        v = W[((long long)perm_col(nc, C, lstm) * cin_total + 0) * 9 + tap];
                    ps[((size_t)nb * 64 + lane) * 8 + j] = host_f2bf(v);
                }
    }
    float* pbias = pb.data.data() + r.bias;
    for (int nc = 0; nc < s.cout; ++nc) pbias[nc] = B[perm_col(nc, C, lstm)];
    return r;
}

// float -> OCP e4m3 (bias 7, 3 mantissa bits, no infinities, largest finite
// 448), round to nearest even, saturating.
static uint8_t host_f2e4m3(float f) {
    const uint8_t sign = std::signbit(f) ? 0x80 : 0;
    double a = std::fabs((double)f);
    if (std::isnan(f)) return 0x7f;
    if (a >= 448.0) return sign | 0x7e;
    if (a < std::ldexp(1.0, -6)) {                     // subnormal: multiples of 2^-9
        const double m = std::nearbyint(a * 512.0);     // ties to even (default rounding)
        return sign | (uint8_t)m;                        // m == 8 is the smallest normal
    }
    int e;
    const double fr = std::frexp(a, &e);                // a = fr 2^e, fr in [0.5, 1)
    double m = std::nearbyint((fr * 2.0 - 1.0) * 8.0);  // mantissa of 1.m x 2^(e-1)
    int ex = e - 1 + 7;
    if (m == 8.0) {
        m = 0.0;
        ++ex;
    }
    if (ex > 15 || (ex == 15 && m == 7.0)) return sign | 0x7e;
    return sign | (uint8_t)((ex << 3) | (int)m);
}

// FP8 layer: e4m3 B fragments of 8 consecutive K per lane (K chunk = 32
// channels, the BF16 order with bytes for elements), one FP32 scale per packed
// output column: scale = max |w| of the column / 448, w8 = e4m3(w / scale).  The
// symbol-channel chunk stays BF16 (divided by the same scale).
MfmaRef pack_mfma8(PackBuf& pb, const float* blob, const ConvShape& s, int has_sym, bool lstm, int C) {
    MfmaRef r{};
    r.cin = s.cin - has_sym;
    r.cout = s.cout;
    r.nbt = (s.cout + 15) / 16;
    r.has_sym = has_sym;
    r.taps = 9;
    const int CC = r.cin / 32;
    const int cin_total = s.cin;
    const float* W = blob + s.w_off;
    const float* B = blob + s.b_off;
    // Step-stack layers with 64 input channels and no symbol channel (the kernel's K128 rule):
    // [5 steps][nbt][64 lanes][32 bytes], step s = taps 2s, 2s + 1 (tap 9 zero), lane group
    // kk = tap 2s + kk/2, channels 32 (kk % 2) + j (the K = 128 MFMA); otherwise
    // [9 taps][cin/32][nbt][64 lanes][8 bytes] (the K = 32 MFMA).
    const bool k128 = r.cin == 64 && !has_sym && !lstm;
    r.w = k128 ? pb.add((size_t)5 * r.nbt * 64 * 8)          // 32 bytes = 8 floats per lane
               : pb.add((size_t)9 * CC * r.nbt * 64 * 2);   // 8 bytes = 2 floats per lane
    r.wsym = has_sym ? pb.add((size_t)r.nbt * 64 * 4) : 0;
    r.bias = pb.add((size_t)r.nbt * 16);
    r.scale = pb.add((size_t)r.nbt * 16);
    float* psc = pb.data.data() + r.scale;
    for (int nc = 0; nc < r.nbt * 16; ++nc) {
        float mx = 0.f;
        if (nc < s.cout) {
            const int o = perm_col(nc, C, lstm);
            for (int k = 0; k < r.cin; ++k)
                for (int tap = 0; tap < 9; ++tap)
                    mx = std::max(mx, std::fabs(W[((long long)o * cin_total + has_sym + k) * 9 + tap]));
        }
        psc[nc] = mx > 0.f ? mx / 448.f : 1.f;
    }
    uint8_t* pw = reinterpret_cast<uint8_t*>(pb.data.data() + r.w);
    if (k128)
        for (int st = 0; st < 5; ++st)
            for (int nb = 0; nb < r.nbt; ++nb)
                for (int lane = 0; lane < 64; ++lane)
                    for (int j = 0; j < 32; ++j) {
                        const int kk = lane >> 4, nn = lane & 15;
                        const int tap = 2 * st + (kk >> 1);
                        const int k = 32 * (kk & 1) + j;
                        const int nc = nb * 16 + nn;
                        float v = 0.f;
                        if (tap < 9 && nc < s.cout)
                            v = W[((long long)perm_col(nc, C, lstm) * cin_total + has_sym + k) * 9 + tap] / psc[nc];
                        pw[(((size_t)st * r.nbt + nb) * 64 + lane) * 32 + j] = host_f2e4m3(v);
                    }
    else
    for (int tap = 0; tap < 9; ++tap)
        for (int cc = 0; cc < CC; ++cc)
            for (int nb = 0; nb < r.nbt; ++nb)
                for (int lane = 0; lane < 64; ++lane)
                    for (int j = 0; j < 8; ++j) {
                        const int kk = lane >> 4, nn = lane & 15;
                        const int k = 32 * cc + 8 * kk + j;
                        const int nc = nb * 16 + nn;
                        float v = 0.f;
                        if (nc < s.cout)
                            v = W[((long long)perm_col(nc, C, lstm) * cin_total + has_sym + k) * 9 + tap] / psc[nc];
                        pw[((((size_t)(tap * CC + cc) * r.nbt + nb) * 64 + lane) * 8) + j] = host_f2e4m3(v);
                    }
    if (has_sym) {
        uint16_t* ps = reinterpret_cast<uint16_t*>(pb.data.data() + r.wsym);
        for (int nb = 0; nb < r.nbt; ++nb)
            for (int lane = 0; lane < 64; ++lane)
                for (int j = 0; j < 8; ++j) {
                    const int kk = lane >> 4, nn = lane & 15;
                    const int tap = 8 * kk + j;
                    const int nc = nb * 16 + nn;
                    float v = 0.f;
                    if (tap < 9 && nc < s.cout)
                        v = W[((long long)perm_col(nc, C, lstm) * cin_total + 0) * 9 + tap] / psc[nc];
                    ps[((size_t)nb * 64 + lane) * 8 + j] = host_f2bf(v);
                }
    }
    float* pbias = pb.data.data() + r.bias;
    for (int nc = 0; nc < s.cout; ++nc) pbias[nc] = B[perm_col(nc, C, lstm)];
    return r;
}

VecRef pack_vec_first(PackBuf& pb, const float* blob, const ConvShape& s) {
    VecRef r;
    r.ch = s.cout;
    r.w = pb.add((size_t)9 * s.cout);
    r.bias = pb.add((size_t)s.cout);
    for (int tap = 0; tap < 9; ++tap)
        for (int ch = 0; ch < s.cout; ++ch)
            pb.data[r.w + tap * s.cout + ch] = blob[s.w_off + (long long)ch * 9 + tap];
    for (int ch = 0; ch < s.cout; ++ch) pb.data[r.bias + ch] = blob[s.b_off + ch];
    return r;
}

VecRef pack_vec_last(PackBuf& pb, const float* blob, const ConvShape& s) {
    VecRef r;
    r.ch = s.cin;
    r.w = pb.add((size_t)9 * s.cin);
    r.bias = pb.add(4);
    for (int tap = 0; tap < 9; ++tap)
        for (int ch = 0; ch < s.cin; ++ch)
            pb.data[r.w + tap * s.cin + ch] = blob[s.w_off + (long long)ch * 9 + tap];
    pb.data[r.bias] = blob[s.b_off];
    return r;
}

struct BlockRefs {
    MfmaRef in, p1a, p1b, p2a, p2b, ra, rb, out;
    size_t dw_w, dw_b;   // depth-wise [9][C], [C]
};

struct HostModel {
    VecRef lift_first[4], lift_last[4];
    std::vector<MfmaRef> lift_mid[4];
    MfmaRef lstm;
    std::vector<MfmaRef> ctx[4][4];
    BlockRefs blk[4][4];
    size_t ar_w1, ar_b1, ar_w2, ar_b2, ar_w3, ar_b3;
};

// Raster-order offsets (dy, dx) of the 12 causal taps of the AR model's 5x5 window.
static const int kArDy[12] = {-2, -2, -2, -2, -2, -1, -1, -1, -1, -1, 0, 0};
static const int kArDx[12] = {-2, -1, 0, 1, 2, -2, -1, 0, 1, 2, -2, -1};

// Context layers are packed for the precision's kernel; lifting is always FP32.
HostModel pack_all(PackBuf& pb, const float* blob, const wv_config& c, int precision) {
    const Manifest mf = make_manifest(c);
    HostModel hm;
    for (int f = 0; f < 4; ++f) {
        const auto& v = mf.lift[f];
        hm.lift_first[f] = pack_vec_first(pb, blob, v.front());
        for (size_t l = 1; l + 1 < v.size(); ++l)
            hm.lift_mid[f].push_back(pack_mfma(pb, blob, v[l], 0, false, 0));
        hm.lift_last[f] = pack_vec_last(pb, blob, v.back());
    }
    auto ctxpack = precision == WV_BF16 ? pack_mfma16 : precision == WV_FP8 ? pack_mfma8 : pack_mfma;
    hm.lstm = ctxpack(pb, blob, mf.lstm, 1, true, c.ctx_ch);
    for (int t = 0; t < 4; ++t)
        for (int g = 0; g < 4; ++g) {
            if (c.ctx_arch == 1) {
                const BlockShapes& b = mf.blk[t][g];
                BlockRefs& r = hm.blk[t][g];
                r.in = pack_mfma(pb, blob, b.in, g > 0 ? 1 : 0, false, 0);
                if (g == 0) {
                    r.p1a = pack_mfma(pb, blob, b.p1a, 0, false, 0);
                    r.p1b = pack_mfma(pb, blob, b.p1b, 0, false, 0);
                    r.p2a = pack_mfma(pb, blob, b.p2a, 0, false, 0);
                    r.p2b = pack_mfma(pb, blob, b.p2b, 0, false, 0);
                    const int C = c.ctx_ch;
                    r.dw_w = pb.add((size_t)9 * C);
                    r.dw_b = pb.add((size_t)C);
                    for (int tap = 0; tap < 9; ++tap)
                        for (int ch = 0; ch < C; ++ch)
                            pb.data[r.dw_w + tap * C + ch] = blob[b.dw.w_off + (long long)ch * 9 + tap];
                    for (int ch = 0; ch < C; ++ch) pb.data[r.dw_b + ch] = blob[b.dw.b_off + ch];
                } else {
                    r.ra = pack_mfma(pb, blob, b.ra, 0, false, 0);
                    r.rb = pack_mfma(pb, blob, b.rb, 0, false, 0);
                }
                r.out = pack_mfma(pb, blob, b.out, 0, false, 0);
                continue;
            }
            const auto& v = mf.ctx[t][g];
            for (size_t l = 0; l < v.size(); ++l)
                hm.ctx[t][g].push_back(ctxpack(pb, blob, v[l], (l == 0 && g > 0) ? 1 : 0, false, 0));
        }
    if (c.ll_ar) {
        const int A = c.ar_ch, O3 = 3 * c.mix_k;
        hm.ar_w1 = pb.add((size_t)A * 12);
        hm.ar_b1 = pb.add(A);
        hm.ar_w2 = pb.add((size_t)A * A);
        hm.ar_b2 = pb.add(A);
        hm.ar_w3 = pb.add((size_t)O3 * A);
        hm.ar_b3 = pb.add(O3);
        for (int k = 0; k < A; ++k) {
            for (int t = 0; t < 12; ++t)
                pb.data[hm.ar_w1 + k * 12 + t] =
                    blob[mf.ar0.w_off + (long long)k * 25 + (kArDy[t] + 2) * 5 + (kArDx[t] + 2)];
            pb.data[hm.ar_b1 + k] = blob[mf.ar0.b_off + k];
            for (int j = 0; j < A; ++j) pb.data[hm.ar_w2 + k * A + j] = blob[mf.ar1.w_off + (long long)k * A + j];
            pb.data[hm.ar_b2 + k] = blob[mf.ar1.b_off + k];
        }
        for (int o = 0; o < O3; ++o) {
            for (int j = 0; j < A; ++j) pb.data[hm.ar_w3 + o * A + j] = blob[mf.ar2.w_off + (long long)o * A + j];
            pb.data[hm.ar_b3 + o] = blob[mf.ar2.b_off + o];
        }
    }
    return hm;
}

}  // namespace

struct wv_model {
    wv_config cfg;
    int precision;
    VecLayer lift_first[4], lift_last[4];
    std::vector<MfmaLayer> lift_mid[4];
    MfmaLayer lstm;                      // WV_FP32
    std::vector<MfmaLayer> ctx[4][4];
    MfmaLayer16 lstm16;                  // WV_BF16
    std::vector<MfmaLayer16> ctx16[4][4];
    struct Blocks {                      // ctx_arch == 1
        MfmaLayer in, p1a, p1b, p2a, p2b, ra, rb, out;
        const float* dw_w;
        const float* dw_b;
    } blk[4][4];
    ArModel ar;                          // ll_ar == 1
};

static int check_precision(const wv_config* c, int precision) {
    if (precision == WV_FP32) return WV_OK;
    if (precision == WV_BF16 || precision == WV_FP8) {
        const char* nm = precision == WV_BF16 ? "BF16" : "FP8";
        if (c->ctx_ch % 32) return fail(WV_EUNSUPPORTED, "%s context needs ctx_ch of 32 or 64", nm);
        if (c->ctx_arch != 0) return fail(WV_EUNSUPPORTED, "%s context needs ctx_arch 0", nm);
        return WV_OK;
    }
    return fail(WV_EUNSUPPORTED, "precision %d is not implemented", precision);
}

extern "C" int wv_weights_count(const wv_config* cfg, long long* n_floats) {
    int rc = check_cfg(cfg);
    if (rc) return rc;
    if (!n_floats) return fail(WV_EINVAL, "null output");
    *n_floats = make_manifest(*cfg).total;
    return WV_OK;
}

static size_t pack_floats(const wv_config& c, int precision) {
    // Pack a zero blob to measure the layout size (host only, cheap).
    const Manifest mf = make_manifest(c);
    std::vector<float> zero((size_t)mf.total, 0.f);
    PackBuf pb;
    pack_all(pb, zero.data(), c, precision);
    return pb.data.size();
}

extern "C" int wv_pack_bytes(const wv_config* cfg, int precision, size_t* bytes) {
    int rc = check_cfg(cfg);
    if (rc) return rc;
    rc = check_precision(cfg, precision);
    if (rc) return rc;
    if (!bytes) return fail(WV_EINVAL, "null output");
    *bytes = pack_floats(*cfg, precision) * sizeof(float);
    return WV_OK;
}

extern "C" int wv_model_create(const wv_config* cfg, const float* d_weights, long long n_floats,
                               int precision, void* d_pack, size_t pack_bytes, void* stream,
                               wv_model** out) {
    int rc = check_cfg(cfg);
    if (rc) return rc;
    if (!d_weights || !d_pack || !out) return fail(WV_EINVAL, "null pointer");
    rc = check_precision(cfg, precision);
    if (rc) return rc;
    const Manifest mf = make_manifest(*cfg);
    if (n_floats != mf.total)
        return fail(WV_EINVAL, "weight blob has %lld floats, config needs %lld", n_floats, mf.total);
    hipStream_t s = (hipStream_t)stream;
    std::vector<float> blob((size_t)mf.total);
    HIPCHK(hipMemcpyAsync(blob.data(), d_weights, blob.size() * sizeof(float), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    PackBuf pb;
    HostModel hm = pack_all(pb, blob.data(), *cfg, precision);
    if (pb.data.size() * sizeof(float) > pack_bytes)
        return fail(WV_ENOMEM, "pack buffer has %zu bytes, needs %zu", pack_bytes,
                    pb.data.size() * sizeof(float));
    HIPCHK(hipMemcpyAsync(d_pack, pb.data.data(), pb.data.size() * sizeof(float), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    const float* base = (const float*)d_pack;
    auto mfma = [&](const MfmaRef& r) {
        return MfmaLayer{base + r.w, r.has_sym ? base + r.wsym : nullptr, base + r.bias,
                         r.cin, r.cout, r.nbt, r.has_sym, r.taps};
    };
    auto vec = [&](const VecRef& r) { return VecLayer{base + r.w, base + r.bias, r.ch}; };
    auto mfma16 = [&](const MfmaRef& r) {
        return MfmaLayer16{reinterpret_cast<const uint16_t*>(base + r.w),
                           r.has_sym ? reinterpret_cast<const uint16_t*>(base + r.wsym) : nullptr,
                           base + r.bias, r.scale ? base + r.scale : nullptr, r.cin, r.cout, r.nbt,
                           r.has_sym};
    };
    wv_model* m = new wv_model();
    m->cfg = *cfg;
    m->precision = precision;
    for (int f = 0; f < 4; ++f) {
        m->lift_first[f] = vec(hm.lift_first[f]);
        m->lift_last[f] = vec(hm.lift_last[f]);
        for (auto& r : hm.lift_mid[f]) m->lift_mid[f].push_back(mfma(r));
    }
    if (precision != WV_FP32) {
        m->lstm16 = mfma16(hm.lstm);
        for (int t = 0; t < 4; ++t)
            for (int g = 0; g < 4; ++g)
                for (auto& r : hm.ctx[t][g]) m->ctx16[t][g].push_back(mfma16(r));
    } else {
        m->lstm = mfma(hm.lstm);
        for (int t = 0; t < 4; ++t)
            for (int g = 0; g < 4; ++g) {
                for (auto& r : hm.ctx[t][g]) m->ctx[t][g].push_back(mfma(r));
                if (cfg->ctx_arch == 1) {
                    const BlockRefs& r = hm.blk[t][g];
                    wv_model::Blocks& b = m->blk[t][g];
                    b.in = mfma(r.in);
                    b.out = mfma(r.out);
                    if (g == 0) {
                        b.p1a = mfma(r.p1a);
                        b.p1b = mfma(r.p1b);
                        b.p2a = mfma(r.p2a);
                        b.p2b = mfma(r.p2b);
                        b.dw_w = base + r.dw_w;
                        b.dw_b = base + r.dw_b;
                    } else {
                        b.ra = mfma(r.ra);
                        b.rb = mfma(r.rb);
                    }
                }
            }
    }
    if (cfg->ll_ar)
        m->ar = ArModel{base + hm.ar_w1, base + hm.ar_b1, base + hm.ar_w2, base + hm.ar_b2,
                        base + hm.ar_w3, base + hm.ar_b3, cfg->ar_ch, cfg->mix_k, cfg->dist,
                        cfg->sigma_min};
    *out = m;
    return WV_OK;
}

extern "C" void wv_model_destroy(wv_model* m) { delete m; }

// ---------------------------------------------------------------------------
// layout and workspace
// ---------------------------------------------------------------------------
namespace {

struct Sub { int h, w, level, type; long long off; };

int layout(const wv_config& c, int H, int W, std::vector<Sub>& out) {
    const int J = c.levels;
    if (H <= 0 || W <= 0) return fail(WV_ESHAPE, "empty image %dx%d", H, W);
    if (H % (1 << J) || W % (1 << J))
        return fail(WV_ESHAPE, "H=%d and W=%d must be divisible by 2^%d", H, W, J);
    out.clear();
    long long off = 0;
    auto add = [&](int lev, int t) {
        Sub s{H >> lev, W >> lev, lev, t, off};
        off += (long long)s.h * s.w;
        out.push_back(s);
    };
    add(J, 0);
    for (int j = J; j >= 1; --j) {
        add(j, 1);
        add(j, 2);
        add(j, 3);
    }
    return WV_OK;
}

// Float offsets of the per-call scratch regions (all 256-byte aligned).
struct Scratch {
    size_t X0, Xa, Xb, lbuf, hbuf, y, a1, a2;   // lifting
    size_t act0, act1, act2;                    // context
    size_t total;
};

inline size_t al(size_t x) { return (x + 63) & ~(size_t)63; }

Scratch scratch_layout(const wv_config& c, int N, int H, int W) {
    const size_t HW = (size_t)H * W;
    Scratch s{};
    size_t o = 0;
    // lifting (analysis and synthesis share the regions)
    s.X0 = o; o = al(o + N * HW);                 // centred input / dequantised subbands
    s.Xa = o; o = al(o + N * HW / 4);
    s.Xb = o; o = al(o + N * HW / 4);
    s.lbuf = o; o = al(o + N * HW / 2);
    s.hbuf = o; o = al(o + N * HW / 2);
    s.y = o; o = al(o + N * HW);
    s.a1 = o; o = al(o + N * HW / 2 * c.lift_ch);
    s.a2 = o; o = al(o + N * HW / 2 * c.lift_ch);
    const size_t lift_total = o;
    // context (reuses the same memory)
    o = 0;
    const size_t act = (size_t)N * (H / 2) * (W / 2) * c.ctx_ch;
    s.act0 = o; o = al(o + act);
    s.act1 = o; o = al(o + act);
    s.act2 = o; o = al(o + act);
    s.total = (lift_total > o ? lift_total : o) * sizeof(float);
    return s;
}

size_t state_floats(const wv_config& c, int N, int H, int W) {
    return (size_t)N * (H / 2) * (W / 2) * c.ctx_ch;   // one of h / c at the finest level
}

}  // namespace

extern "C" int wv_layout(const wv_config* cfg, int H, int W, wv_subband* out, int cap,
                         long long* coefs) {
    int rc = check_cfg(cfg);
    if (rc) return rc;
    std::vector<Sub> lay;
    rc = layout(*cfg, H, W, lay);
    if (rc) return rc;
    if (out) {
        if (cap < (int)lay.size()) return fail(WV_ENOMEM, "need %zu entries", lay.size());
        for (size_t i = 0; i < lay.size(); ++i)
            out[i] = wv_subband{lay[i].h, lay[i].w, lay[i].level, lay[i].type, lay[i].off};
    }
    if (coefs) *coefs = (long long)H * W;
    return WV_OK;
}

extern "C" long long wv_group_count(int h, int w, int step) {
    if (h < 0 || w < 0 || step < 0 || step > 3) return -1;
    const int gr = step >> 1, gc = step & 1;
    return (long long)((h - gr + 1) >> 1) * ((w - gc + 1) >> 1);
}

extern "C" int wv_workspace_bytes(const wv_model* m, int N, int H, int W, size_t* state_bytes,
                                  size_t* scratch_bytes) {
    if (!m) return fail(WV_EINVAL, "null model");
    if (N < 1) return fail(WV_ESHAPE, "nplanes must be >= 1");
    std::vector<Sub> lay;
    int rc = layout(m->cfg, H, W, lay);
    if (rc) return rc;
    if (state_bytes) *state_bytes = 4 * state_floats(m->cfg, N, H, W) * sizeof(float);
    if (scratch_bytes) *scratch_bytes = scratch_layout(m->cfg, N, H, W).total;
    return WV_OK;
}

// ---------------------------------------------------------------------------
// lifting
// ---------------------------------------------------------------------------
namespace {

enum { F_PROW = 0, F_UROW = 1, F_PCOL = 2, F_UCOL = 3 };

inline View vw(float* p, long long ps, int rs, int cs) { return View{p, ps, rs, cs}; }
inline CView cvw(const float* p, long long ps, int rs, int cs) { return CView{p, ps, rs, cs}; }

// out = A + sign * (predict ? z + N(z) : z/2 + N(z)) on an h x w array.
int run_filter(const wv_model* m, int f, CView z, CView A, View out, int N, int h, int w,
               int predict, float sign, float* a1, float* a2, hipStream_t s) {
    if (m->lift_mid[f].size() == 1) {   // three layers: the fused kernel keeps them in LDS
        HIPCHK(launch_lift_fused(m->lift_first[f], m->lift_mid[f][0], m->lift_last[f], z, A, out, N, h, w,
                                 predict, sign, m->cfg.lift_int, s));
        return WV_OK;
    }
    HIPCHK(launch_lift_first(m->lift_first[f], z, N, h, w, a1, s));
    float* cur = a1;
    float* oth = a2;
    const int C = m->cfg.lift_ch;
    for (const MfmaLayer& L : m->lift_mid[f]) {
        ConvArgs a{};
        a.in = cur;
        a.in_ps = (long long)h * w * C;
        a.out = oth;
        a.out_ps = (long long)h * w * C;
        a.out_cs = C;
        a.N = N;
        a.h = h;
        a.w = w;
        a.tiles_x = (w + TILE_W - 1) / TILE_W;
        a.tiles_y = (h + TILE_H - 1) / TILE_H;
        HIPCHK(launch_conv(L, CONV_TANH, a, s));
        float* t = cur;
        cur = oth;
        oth = t;
    }
    HIPCHK(launch_lift_last(m->lift_last[f], cur, z, A, out, N, h, w, predict, sign, m->cfg.lift_int, s));
    return WV_OK;
}

}  // namespace

extern "C" int wv_analyze(const wv_model* m, const uint8_t* d_x8, const float* d_xf, int N, int H,
                          int W, float dL, float dH, void* d_scratch, int16_t* d_q, float* d_y,
                          int* d_clip, void* stream) {
    if (!m) return fail(WV_EINVAL, "null model");
    if ((!d_x8 && !d_xf) || !d_scratch || !d_q) return fail(WV_EINVAL, "null pointer");
    if (N < 1) return fail(WV_ESHAPE, "nplanes must be >= 1");
    if (!(dL > 0.f) || !(dH > 0.f)) return fail(WV_EINVAL, "quantiser steps must be > 0");
    std::vector<Sub> lay;
    int rc = layout(m->cfg, H, W, lay);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const Scratch sc = scratch_layout(m->cfg, N, H, W);
    float* base = (float*)d_scratch;
    const long long HW = (long long)H * W;
    const float* X = d_xf;
    if (d_x8) {
        HIPCHK(launch_center_u8(d_x8, base + sc.X0, N * HW, s));
        X = base + sc.X0;
    }
    long long xps = HW;
    float* y = d_y ? d_y : base + sc.y;
    float* a1 = base + sc.a1;
    float* a2 = base + sc.a2;
    float* lb = base + sc.lbuf;
    float* hb = base + sc.hbuf;
    const int J = m->cfg.levels;
    // coding-order index of HL_j: 1 + 3 (J - j); LH, HH follow.
    for (int j = 1; j <= J; ++j) {
        const int hx = H >> (j - 1), wx = W >> (j - 1);
        const int hw2 = wx / 2;
        const long long hps = (long long)hx * hw2;
        // row step: h = odd - P_row(even); l = even + U_row(h)
        rc = run_filter(m, F_PROW, cvw(X, xps, wx, 2), cvw(X + 1, xps, wx, 2), vw(hb, hps, hw2, 1), N,
                        hx, hw2, 1, -1.f, a1, a2, s);
        if (rc) return rc;
        rc = run_filter(m, F_UROW, cvw(hb, hps, hw2, 1), cvw(X, xps, wx, 2), vw(lb, hps, hw2, 1), N, hx,
                        hw2, 0, 1.f, a1, a2, s);
        if (rc) return rc;
        const int hs = hx / 2, ws = hw2;
        const Sub& sHL = lay[1 + 3 * (J - j)];
        const Sub& sLH = lay[2 + 3 * (J - j)];
        const Sub& sHH = lay[3 + 3 * (J - j)];
        float* xn = (j == J) ? y + lay[0].off : base + ((j & 1) ? sc.Xa : sc.Xb);
        const long long xnps = (j == J) ? HW : (long long)hs * ws;
        // column step on l: LH = l_odd - P_col(l_even); LL = l_even + U_col(LH)
        rc = run_filter(m, F_PCOL, cvw(lb, hps, 2 * hw2, 1), cvw(lb + hw2, hps, 2 * hw2, 1),
                        vw(y + sLH.off, HW, ws, 1), N, hs, ws, 1, -1.f, a1, a2, s);
        if (rc) return rc;
        rc = run_filter(m, F_UCOL, cvw(y + sLH.off, HW, ws, 1), cvw(lb, hps, 2 * hw2, 1),
                        vw(xn, xnps, ws, 1), N, hs, ws, 0, 1.f, a1, a2, s);
        if (rc) return rc;
        // column step on h: HH = h_odd - P_col(h_even); HL = h_even + U_col(HH)
        rc = run_filter(m, F_PCOL, cvw(hb, hps, 2 * hw2, 1), cvw(hb + hw2, hps, 2 * hw2, 1),
                        vw(y + sHH.off, HW, ws, 1), N, hs, ws, 1, -1.f, a1, a2, s);
        if (rc) return rc;
        rc = run_filter(m, F_UCOL, cvw(y + sHH.off, HW, ws, 1), cvw(hb, hps, 2 * hw2, 1),
                        vw(y + sHL.off, HW, ws, 1), N, hs, ws, 0, 1.f, a1, a2, s);
        if (rc) return rc;
        X = xn;
        xps = xnps;
    }
    const long long n_ll = (long long)lay[0].h * lay[0].w;
    HIPCHK(launch_quantize(y, d_q, N, HW, n_ll, dL, dH, m->cfg.sym_min, m->cfg.sym_max, d_clip, s));
    return WV_OK;
}

static int synth_impl(const wv_model* m, const int16_t* d_q, const float* d_y, int N, int H, int W,
                      float dL, float dH, void* d_scratch, float* d_xhat, uint8_t* d_u8,
                      float offset, void* stream);

extern "C" int wv_synthesize(const wv_model* m, const int16_t* d_q, const float* d_y, int N, int H,
                             int W, float dL, float dH, float offset, void* d_scratch, float* d_xhat,
                             uint8_t* d_u8, void* stream) {
    return synth_impl(m, d_q, d_y, N, H, W, dL, dH, d_scratch, d_xhat, d_u8, offset, stream);
}

extern "C" int wv_center_u8(const uint8_t* d_x8, long long n, float* d_out, void* stream) {
    if (n < 0) return fail(WV_ESHAPE, "negative size");
    if (n > 0 && (!d_x8 || !d_out)) return fail(WV_EINVAL, "null pointer");
    HIPCHK(launch_center_u8(d_x8, d_out, n, (hipStream_t)stream));
    return WV_OK;
}

extern "C" int wv_add_offset(float* d_x, long long n, float offset, uint8_t* d_u8, void* stream) {
    if (n < 0) return fail(WV_ESHAPE, "negative size");
    if (n > 0 && !d_x) return fail(WV_EINVAL, "null pointer");
    HIPCHK(launch_finalize(d_x, d_u8, n, offset, (hipStream_t)stream));
    return WV_OK;
}

static int synth_impl(const wv_model* m, const int16_t* d_q, const float* d_y, int N, int H, int W,
                      float dL, float dH, void* d_scratch, float* d_xhat, uint8_t* d_u8,
                      float offset, void* stream) {
    if (!m) return fail(WV_EINVAL, "null model");
    if ((!d_q && !d_y) || !d_scratch || !d_xhat) return fail(WV_EINVAL, "null pointer");
    if (N < 1) return fail(WV_ESHAPE, "nplanes must be >= 1");
    if (d_q && (!(dL > 0.f) || !(dH > 0.f))) return fail(WV_EINVAL, "quantiser steps must be > 0");
    std::vector<Sub> lay;
    int rc = layout(m->cfg, H, W, lay);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    const Scratch sc = scratch_layout(m->cfg, N, H, W);
    float* base = (float*)d_scratch;
    const long long HW = (long long)H * W;
    const float* y = d_y;
    if (d_q) {
        const long long n_ll = (long long)lay[0].h * lay[0].w;
        HIPCHK(launch_dequantize(d_q, base + sc.X0, N, HW, n_ll, dL, dH, s));
        y = base + sc.X0;
    }
    float* a1 = base + sc.a1;
    float* a2 = base + sc.a2;
    float* lb = base + sc.lbuf;
    float* hb = base + sc.hbuf;
    const int J = m->cfg.levels;
    const float* X = y + lay[0].off;
    long long xps = HW;
    for (int j = J; j >= 1; --j) {
        const int hs = H >> j, ws = W >> j;
        const Sub& sHL = lay[1 + 3 * (J - j)];
        const Sub& sLH = lay[2 + 3 * (J - j)];
        const Sub& sHH = lay[3 + 3 * (J - j)];
        const long long bps = (long long)(2 * hs) * ws;
        // inverse column step on (LL, LH) -> l: even = LL - U_col(LH); odd = LH + P_col(even)
        rc = run_filter(m, F_UCOL, cvw(y + sLH.off, HW, ws, 1), cvw(X, xps, ws, 1),
                        vw(lb, bps, 2 * ws, 1), N, hs, ws, 0, -1.f, a1, a2, s);
        if (rc) return rc;
        rc = run_filter(m, F_PCOL, cvw(lb, bps, 2 * ws, 1), cvw(y + sLH.off, HW, ws, 1),
                        vw(lb + ws, bps, 2 * ws, 1), N, hs, ws, 1, 1.f, a1, a2, s);
        if (rc) return rc;
        // inverse column step on (HL, HH) -> h
        rc = run_filter(m, F_UCOL, cvw(y + sHH.off, HW, ws, 1), cvw(y + sHL.off, HW, ws, 1),
                        vw(hb, bps, 2 * ws, 1), N, hs, ws, 0, -1.f, a1, a2, s);
        if (rc) return rc;
        rc = run_filter(m, F_PCOL, cvw(hb, bps, 2 * ws, 1), cvw(y + sHH.off, HW, ws, 1),
                        vw(hb + ws, bps, 2 * ws, 1), N, hs, ws, 1, 1.f, a1, a2, s);
        if (rc) return rc;
        // inverse row step: even = l - U_row(h); odd = h + P_row(even)
        const int ho = 2 * hs, wo = 2 * ws;
        float* xo = (j == 1) ? d_xhat : base + ((j & 1) ? sc.Xa : sc.Xb);
        const long long ops = (long long)ho * wo;
        rc = run_filter(m, F_UROW, cvw(hb, bps, ws, 1), cvw(lb, bps, ws, 1), vw(xo, ops, wo, 2), N, ho,
                        ws, 0, -1.f, a1, a2, s);
        if (rc) return rc;
        rc = run_filter(m, F_PROW, cvw(xo, ops, wo, 2), cvw(hb, bps, ws, 1), vw(xo + 1, ops, wo, 2), N,
                        ho, ws, 1, 1.f, a1, a2, s);
        if (rc) return rc;
        X = xo;
        xps = ops;
    }
    HIPCHK(launch_finalize(d_xhat, d_u8, N * HW, offset, s));
    return WV_OK;
}

// ---------------------------------------------------------------------------
// subband impulse responses (Sec. 3.4)
// ---------------------------------------------------------------------------
namespace {
struct SirScratch { size_t keys, y, synth, total; };
SirScratch sir_layout(const wv_config& c, int S) {
    const int nsub = 3 * c.levels + 1;
    SirScratch r;
    r.keys = 0;
    r.y = al(32);                                   // 32 u64 keys = 64 floats ... 256-byte aligned
    r.synth = al(r.y + (size_t)nsub * S * S);
    r.total = (r.synth * sizeof(float)) + scratch_layout(c, nsub, S, S).total;
    return r;
}
}  // namespace

extern "C" int wv_impulse_scratch_bytes(const wv_model* m, size_t* bytes) {
    if (!m || !bytes) return fail(WV_EINVAL, "null pointer");
    *bytes = sir_layout(m->cfg, 1 << m->cfg.levels).total;
    return WV_OK;
}

extern "C" int wv_impulse_responses(const wv_model* m, const int16_t* d_q, int H, int W, float dL,
                                    float dH, void* d_scratch, float* d_out, void* stream) {
    if (!m) return fail(WV_EINVAL, "null model");
    if (!d_q || !d_scratch || !d_out) return fail(WV_EINVAL, "null pointer");
    if (!(dL > 0.f) || !(dH > 0.f)) return fail(WV_EINVAL, "quantiser steps must be > 0");
    std::vector<Sub> lay, play;
    int rc = layout(m->cfg, H, W, lay);
    if (rc) return rc;
    const int S = 1 << m->cfg.levels;
    rc = layout(m->cfg, S, S, play);
    if (rc) return rc;
    const int nsub = (int)lay.size();
    if (nsub > MAX_SUB) return fail(WV_EUNSUPPORTED, "too many subbands");
    SirMeta meta{};
    meta.nsub = nsub;
    meta.S = S;
    meta.ph = H / S;
    meta.pw = W / S;
    long long max_n = 0;
    for (int i = 0; i < nsub; ++i) {
        meta.off[i] = lay[i].off;
        meta.h[i] = lay[i].h;
        meta.w[i] = lay[i].w;
        meta.soff[i] = play[i].off;
        meta.sw[i] = play[i].w;
        const long long n = (long long)lay[i].h * lay[i].w;
        max_n = n > max_n ? n : max_n;
    }
    hipStream_t s = (hipStream_t)stream;
    const SirScratch sc = sir_layout(m->cfg, S);
    float* base = (float*)d_scratch;
    unsigned long long* keys = (unsigned long long*)(base + sc.keys);
    float* y = base + sc.y;
    HIPCHK(launch_sir_keys(d_q, keys, meta, max_n, s));
    HIPCHK(launch_sir_pyramid(keys, meta, dL, dH, y, s));
    return synth_impl(m, nullptr, y, nsub, S, S, dL, dH, base + sc.synth, d_out, nullptr, 0.0f, stream);
}

// ---------------------------------------------------------------------------
// coding order
// ---------------------------------------------------------------------------
// Sec. 3.2: step g of a subband reads the symbols its earlier steps decoded, and
// step 0 advances the ConvLSTM from the previous subband's state, so the calls
// on one state buffer must follow the coding order.  The library keeps, per
// state buffer, the position (subband * 4 + step) of the last call that
// succeeded; a decode that reaches its last step leaves the table.
namespace {
struct OrderTable {
    std::mutex mu;
    std::unordered_map<const void*, int> last;
};
OrderTable& order_table() {
    static OrderTable* t = new OrderTable();   // never destroyed: calls may come during exit
    return *t;
}

// Is (i, g) allowed after `last` (-1: no call yet)?  (0, 0) starts a new decode at
// any time.  With the autoregressive LL model subband 0 needs only its step 0 (the
// long context), so (1, 0) may follow any step of subband 0.
bool order_ok(int last, int i, int g, bool ll_ar) {
    if (i == 0 && g == 0) return true;
    if (last < 0) return false;
    const int li = last >> 2, lg = last & 3;
    if (ll_ar && li == 0 && i == 1 && g == 0) return true;
    return lg < 3 ? (i == li && g == lg + 1) : (i == li + 1 && g == 0);
}

int order_check(const void* key, int i, int g, bool ll_ar, const char* what) {
    OrderTable& t = order_table();
    std::lock_guard<std::mutex> lk(t.mu);
    auto it = t.last.find(key);
    const int last = it == t.last.end() ? -1 : it->second;
    if (order_ok(last, i, g, ll_ar)) return WV_OK;
    if (last < 0)
        return fail(WV_EORDER, "%s: (subband %d, step %d) before (0, 0) on this state buffer", what, i, g);
    return fail(WV_EORDER, "%s: (subband %d, step %d) does not follow (subband %d, step %d)", what, i, g,
                last >> 2, last & 3);
}

void order_commit(const void* key, int i, int g, int nsub) {
    OrderTable& t = order_table();
    std::lock_guard<std::mutex> lk(t.mu);
    if (i == nsub - 1 && g == 3) t.last.erase(key);
    else t.last[key] = i * 4 + g;
}
}  // namespace

// ---------------------------------------------------------------------------
// context model
// ---------------------------------------------------------------------------
static int context_params_impl(const wv_model* m, const int16_t* d_q, int N, int H, int W, int i, int g,
                               float* d_state, void* d_scratch, float* d_params, void* stream,
                               const std::vector<Sub>& lay);

extern "C" int wv_context_params(const wv_model* m, const int16_t* d_q, int N, int H, int W, int i,
                                 int g, float* d_state, void* d_scratch, float* d_params,
                                 void* stream) {
    if (!m) return fail(WV_EINVAL, "null model");
    if (!d_q || !d_state || !d_scratch) return fail(WV_EINVAL, "null pointer");
    if (N < 1) return fail(WV_ESHAPE, "nplanes must be >= 1");
    std::vector<Sub> lay;
    int rc = layout(m->cfg, H, W, lay);
    if (rc) return rc;
    if (i < 0 || i >= (int)lay.size() || g < 0 || g > 3)
        return fail(WV_EORDER, "subband %d / step %d out of range", i, g);
    if ((rc = order_check(d_state, i, g, m->cfg.ll_ar != 0, "wv_context_params"))) return rc;
    rc = context_params_impl(m, d_q, N, H, W, i, g, d_state, d_scratch, d_params, stream, lay);
    if (rc == WV_OK) order_commit(d_state, i, g, (int)lay.size());
    return rc;
}

static int context_params_impl(const wv_model* m, const int16_t* d_q, int N, int H, int W, int i, int g,
                               float* d_state, void* d_scratch, float* d_params, void* stream,
                               const std::vector<Sub>& lay) {
    const long long ng = wv_group_count(lay[i].h, lay[i].w, g);
    if (ng > 0 && !d_params) return fail(WV_EINVAL, "null pointer");
    if (ng == 0) return WV_OK;   // a 1-wide subband has no positions at this step
    hipStream_t s = (hipStream_t)stream;
    const int C = m->cfg.ctx_ch;
    const bool bf16 = m->precision != WV_FP32;   // h and activations stored as BF16 or FP8
    const long long HW = (long long)H * W;
    const size_t SS = state_floats(m->cfg, N, H, W);
    const Sub& S = lay[i];
    float* hcur = d_state + (size_t)(i & 1) * 2 * SS;
    float* ccur = hcur + SS;
    const long long st_ps = (long long)S.h * S.w * C;
    if (g == 0) {
        ConvArgs a{};
        a.N = N;
        a.h = S.h;
        a.w = S.w;
        a.tiles_x = (S.w + TILE_W - 1) / TILE_W;
        a.tiles_y = (S.h + TILE_H - 1) / TILE_H;
        a.sym_step = 4;
        a.h_out = hcur;
        a.c_out = ccur;
        a.st_ps = st_ps;
        a.C = C;
        if (i > 0) {
            const Sub& P = lay[i - 1];
            const int up = (S.h == 2 * P.h) ? 1 : 0;
            float* hold = d_state + (size_t)((i - 1) & 1) * 2 * SS;
            a.in = hold;
            a.in_ps = (long long)P.h * P.w * C;
            a.in_up = up;
            a.sym = d_q + P.off;
            a.sym_ps = HW;
            a.sym_up = up;
            a.c_prev = hold + SS;
            a.cprev_ps = (long long)P.h * P.w * C;
            a.cprev_up = up;
        }
        if (bf16) {
            a.in16 = reinterpret_cast<const uint16_t*>(a.in);
            a.in = nullptr;
            a.h16_out = reinterpret_cast<uint16_t*>(hcur);
            a.h_out = nullptr;
            HIPCHK(launch_conv_bf16(m->lstm16, CONV_LSTM, a, s));
        } else {
            HIPCHK(launch_conv(m->lstm, CONV_LSTM, a, s));
        }
    }
    float* base = (float*)d_scratch;
    const Scratch sc = scratch_layout(m->cfg, N, H, W);
    float* act[3] = {base + sc.act0, base + sc.act1, base + sc.act2};
    if (m->cfg.ctx_arch == 1) {
        // in -> block -> out (Sec. 3.2): step 0 a DepthConvBlock, steps 1-3 a Residual Block.
        const wv_model::Blocks& b = m->blk[S.type][g];
        auto run = [&](const MfmaLayer& L, int mode, const float* in, float* out,
                       const float* skip) -> int {
            ConvArgs a{};
            a.in = in;
            a.in_ps = st_ps;
            a.N = N;
            a.h = S.h;
            a.w = S.w;
            a.tiles_x = (S.w + TILE_W - 1) / TILE_W;
            a.tiles_y = (S.h + TILE_H - 1) / TILE_H;
            if (L.has_sym) {
                a.sym = d_q + S.off;
                a.sym_ps = HW;
                a.sym_step = g;
            }
            a.out = out;
            a.out_ps = st_ps;
            a.out_cs = C;
            a.skip = skip;
            a.params = d_params;
            a.step = g;
            a.K = m->cfg.mix_k;
            a.sigma_min = m->cfg.sigma_min;
            HIPCHK(launch_conv(L, mode, a, s));
            return WV_OK;
        };
        int rc2;
        if ((rc2 = run(b.in, CONV_RELU, hcur, act[0], nullptr))) return rc2;
        if (g == 0) {
            if ((rc2 = run(b.p1a, CONV_RELU, act[0], act[1], nullptr))) return rc2;
            HIPCHK(launch_dwconv(act[1], b.dw_w, b.dw_b, act[2], N, S.h, S.w, C, s));
            if ((rc2 = run(b.p1b, CONV_RES, act[2], act[1], act[0]))) return rc2;
            if ((rc2 = run(b.p2a, CONV_RELU, act[1], act[0], nullptr))) return rc2;
            if ((rc2 = run(b.p2b, CONV_RES, act[0], act[2], act[1]))) return rc2;
        } else {
            if ((rc2 = run(b.ra, CONV_RELU, act[0], act[1], nullptr))) return rc2;
            if ((rc2 = run(b.rb, CONV_RES, act[1], act[2], act[0]))) return rc2;
        }
        return run(b.out, CONV_HEAD, act[2], nullptr, nullptr);
    }
    const size_t nlayers = bf16 ? m->ctx16[S.type][g].size() : m->ctx[S.type][g].size();
    const float* in = hcur;
    for (size_t l = 0; l < nlayers; ++l) {
        const bool last = l + 1 == nlayers;
        ConvArgs a{};
        a.in = in;
        a.in_ps = st_ps;
        a.N = N;
        a.h = S.h;
        a.w = S.w;
        a.tiles_x = (S.w + TILE_W - 1) / TILE_W;
        a.tiles_y = (S.h + TILE_H - 1) / TILE_H;
        if (l == 0 && g > 0) {
            a.sym = d_q + S.off;
            a.sym_ps = HW;
            a.sym_step = g;
        }
        if (!last) {
            a.out = act[l & 1];
            a.out_ps = st_ps;
            a.out_cs = C;
        } else {
            a.params = d_params;
            a.step = g;
            a.K = m->cfg.mix_k;
            a.sigma_min = m->cfg.sigma_min;
        }
        const int mode = last ? CONV_HEAD : CONV_RELU;
        if (bf16) {
            a.in16 = reinterpret_cast<const uint16_t*>(a.in);
            a.in = nullptr;
            a.out16 = reinterpret_cast<uint16_t*>(a.out);
            a.out = nullptr;
            HIPCHK(launch_conv_bf16(m->ctx16[S.type][g][l], mode, a, s));
        } else {
            HIPCHK(launch_conv(m->ctx[S.type][g][l], mode, a, s));
        }
        if (!last) in = act[l & 1];
    }
    return WV_OK;
}

extern "C" int wv_ar_params(const wv_model* m, const int16_t* d_q, int N, int H, int W,
                            float* d_params, void* stream) {
    if (!m) return fail(WV_EINVAL, "null model");
    if (!m->cfg.ll_ar) return fail(WV_EUNSUPPORTED, "model has no autoregressive LL model");
    if (!d_q || !d_params) return fail(WV_EINVAL, "null pointer");
    if (N < 1) return fail(WV_ESHAPE, "nplanes must be >= 1");
    std::vector<Sub> lay;
    int rc = layout(m->cfg, H, W, lay);
    if (rc) return rc;
    HIPCHK(launch_ar_params(m->ar, d_q + lay[0].off, (long long)H * W, lay[0].h, lay[0].w, N, d_params,
                            (hipStream_t)stream));
    return WV_OK;
}

extern "C" int wv_ar_decode(const wv_model* m, const uint8_t* d_bytes, const long long* d_offsets,
                            int N, int H, int W, int16_t* d_q, int* d_status, void* stream) {
    if (!m) return fail(WV_EINVAL, "null model");
    if (!m->cfg.ll_ar) return fail(WV_EUNSUPPORTED, "model has no autoregressive LL model");
    if (!d_bytes || !d_offsets || !d_q || !d_status) return fail(WV_EINVAL, "null pointer");
    if (N < 1) return fail(WV_ESHAPE, "nplanes must be >= 1");
    std::vector<Sub> lay;
    int rc = layout(m->cfg, H, W, lay);
    if (rc) return rc;
    if (lay[0].w > 4096) return fail(WV_ESHAPE, "LL subband wider than 4096");
    const int nsym = m->cfg.sym_max - m->cfg.sym_min + 1;
    HIPCHK(launch_ar_decode(m->ar, ArStreams{d_bytes, d_offsets}, d_q + lay[0].off, (long long)H * W,
                            lay[0].h, lay[0].w, N, m->cfg.sym_min, nsym, d_status, (hipStream_t)stream));
    return WV_OK;
}

extern "C" int wv_cdf_tables(const float* d_params, long long n, int K, int dist, int sym_min,
                             int sym_max, int cdf_bits, uint16_t* d_cdf, void* stream) {
    if (n < 0) return fail(WV_ESHAPE, "negative row count");
    if (n > 0 && (!d_params || !d_cdf)) return fail(WV_EINVAL, "null pointer");
    if (K < 1 || K > 4) return fail(WV_EUNSUPPORTED, "mix_k must be 1..4");
    const int nsym = sym_max - sym_min + 1;
    if (nsym < 2 || nsym > 255) return fail(WV_EUNSUPPORTED, "alphabet must have 2..255 symbols");
    if (cdf_bits != 16) return fail(WV_EUNSUPPORTED, "cdf_bits must be 16");
    if (dist != WV_DIST_GAUSS && dist != WV_DIST_LAPLACE) return fail(WV_EINVAL, "bad dist");
    HIPCHK(launch_cdf(d_params, n, K, dist, sym_min, nsym, d_cdf, (hipStream_t)stream));
    return WV_OK;
}

extern "C" int wv_cdf_trim_scratch_bytes(long long n, size_t* bytes) {
    if (n < 0 || !bytes) return fail(WV_EINVAL, "bad argument");
    *bytes = cdf_trim_scratch_bytes(n);
    return WV_OK;
}

extern "C" int wv_cdf_trim(const uint16_t* d_cdf, long long n, int nsym, uint8_t* d_lolen, uint16_t* d_packed,
                           long long packed_cap, void* d_scratch, size_t scratch_bytes, void* stream) {
    if (n < 0) return fail(WV_ESHAPE, "negative row count");
    if (nsym < 2 || nsym > 255) return fail(WV_EUNSUPPORTED, "alphabet must have 2..255 symbols");
    if (n == 0) return WV_OK;
    if (!d_cdf || !d_lolen || !d_packed || !d_scratch) return fail(WV_EINVAL, "null pointer");
    if (packed_cap < n * (long long)(nsym - 1)) return fail(WV_ENOMEM, "packed buffer below n (nsym - 1)");
    if (scratch_bytes < cdf_trim_scratch_bytes(n)) return fail(WV_ENOMEM, "scratch below wv_cdf_trim_scratch_bytes");
    HIPCHK(launch_cdf_trim(d_cdf, n, nsym, d_lolen, d_packed, reinterpret_cast<long long*>(d_scratch),
                           (hipStream_t)stream));
    return WV_OK;
}

extern "C" int wv_cdf_trim_noalloc(const uint16_t* d_cdf, long long n, int nsym, uint8_t* d_lolen,
                                   uint16_t* d_packed, long long packed_cap, void* stream) {
    if (n < 0) return fail(WV_ESHAPE, "negative row count");
    if (nsym < 2 || nsym > 255) return fail(WV_EUNSUPPORTED, "alphabet must have 2..255 symbols");
    if (n == 0) return WV_OK;
    if (!d_cdf || !d_lolen || !d_packed) return fail(WV_EINVAL, "null pointer");
    if (n > TRIM_STATIC_MAX_ROWS)
        return fail(WV_ENOMEM, "wv_cdf_trim_noalloc handles at most %lld rows (got %lld); use wv_cdf_trim",
                    TRIM_STATIC_MAX_ROWS, n);
    if (packed_cap < n * (long long)(nsym - 1)) return fail(WV_ENOMEM, "packed buffer below n (nsym - 1)");
    long long* scratch = nullptr;
    HIPCHK(cdf_trim_static_scratch(&scratch));
    HIPCHK(launch_cdf_trim(d_cdf, n, nsym, d_lolen, d_packed, scratch, (hipStream_t)stream));
    return WV_OK;
}

static int sym_io(const wv_config* cfg, int N, int H, int W, int i, int g, std::vector<Sub>& lay) {
    int rc = check_cfg(cfg);
    if (rc) return rc;
    if (N < 1) return fail(WV_ESHAPE, "nplanes must be >= 1");
    rc = layout(*cfg, H, W, lay);
    if (rc) return rc;
    if (i < 0 || i >= (int)lay.size() || g < 0 || g > 3)
        return fail(WV_EORDER, "subband %d / step %d out of range", i, g);
    return WV_OK;
}

extern "C" int wv_scatter_symbols(const wv_config* cfg, const uint8_t* d_sym, int N, int H, int W,
                                  int i, int g, int16_t* d_q, void* stream) {
    std::vector<Sub> lay;
    int rc = sym_io(cfg, N, H, W, i, g, lay);
    if (rc) return rc;
    if (!d_q || (!d_sym && wv_group_count(lay[i].h, lay[i].w, g) > 0))
        return fail(WV_EINVAL, "null pointer");
    HIPCHK(launch_scatter(d_sym, d_q, N, (long long)H * W, lay[i].off, lay[i].h, lay[i].w, g,
                          cfg->sym_min, (hipStream_t)stream));
    return WV_OK;
}

extern "C" int wv_gather_symbols(const wv_config* cfg, const int16_t* d_q, int N, int H, int W,
                                 int i, int g, uint8_t* d_sym, void* stream) {
    std::vector<Sub> lay;
    int rc = sym_io(cfg, N, H, W, i, g, lay);
    if (rc) return rc;
    if (!d_q || (!d_sym && wv_group_count(lay[i].h, lay[i].w, g) > 0))
        return fail(WV_EINVAL, "null pointer");
    HIPCHK(launch_gather(d_q, d_sym, N, (long long)H * W, lay[i].off, lay[i].h, lay[i].w, g,
                         cfg->sym_min, (hipStream_t)stream));
    return WV_OK;
}

static int thaar(float* f, int T, long long n, int inverse, void* stream) {
    if (T < 1 || T > 32 || (T & (T - 1))) return fail(WV_ESHAPE, "T must be a power of two <= 32");
    if (n < 0) return fail(WV_ESHAPE, "negative size");
    if (!f && n > 0) return fail(WV_EINVAL, "null pointer");
    HIPCHK(launch_thaar(f, nullptr, T, n, inverse, (hipStream_t)stream));
    return WV_OK;
}

extern "C" int wv_temporal_haar_forward(float* f, int T, long long n, void* stream) {
    return thaar(f, T, n, 0, stream);
}
extern "C" int wv_temporal_haar_inverse(float* f, int T, long long n, void* stream) {
    return thaar(f, T, n, 1, stream);
}

// ---------------------------------------------------------------------------
// plans: several plane groups of different sizes, one launch per layer
// ---------------------------------------------------------------------------
namespace {
struct PlanLaunch {
    size_t seg_off;      // byte offset of this launch's segment array in the descriptor buffer
    int nseg, mode, nb, grid;
    long long total;     // work items
    MfmaLayer proto;
    MfmaLayer16 proto16;
    int fused = 0;       // 1: a whole step stack in one launch (StackSeg array); 2: the ConvLSTM (LstmSeg)
    int has_sym = 0;
};

// Compute units of the current device, cached per device: the grid of the persistent fused
// launches, which keep one workgroup per compute unit.
int device_cus() {
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    int n = cache[dev].load(std::memory_order_relaxed);
    if (n == 0) {
        if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1) n = 256;
        cache[dev].store(n, std::memory_order_relaxed);
    }
    return n;
}

// Whether a model's step stacks can run as one fused launch per step (wv_stack_bf16.hip):
// BF16, 64 channels, three ReLU layers and the head, the head's 3K outputs in one
// 16-column block.  WV_FUSED_STACKS=0 keeps the layer-by-layer launches (tests compare
// the two forms).
bool stack_fusable(const wv_model* m) {
    const char* env = getenv("WV_FUSED_STACKS");
    if (env && env[0] == '0') return false;
    return m->precision == WV_BF16 && m->cfg.ctx_arch == 0 && m->cfg.ctx_ch == 64 && m->cfg.ctx_layers == 4 &&
           3 * m->cfg.mix_k <= 16;
}

// Fused step-stack segment of a plane group's subband S at step g: input l_i = hcur
// (BF16 NHWC), symbols of this subband (plane 0) at q_sub with plane stride q_ps.
// Returns the segment's work items (0 for a step with no positions).
long long make_stack_seg(const wv_model* m, int type, int g, const float* hcur, const Sub& S, int nplanes,
                         const int16_t* q_sub, long long q_ps, float* params, long long item0, StackSeg& sg,
                         int cap = 128) {
    const std::vector<MfmaLayer16>& Ls = m->ctx16[type][g];
    sg = StackSeg{};
    for (int l = 0; l < 4; ++l) {
        sg.w16[l] = Ls[l].w;
        sg.bias[l] = Ls[l].bias;
    }
    sg.wsym = g > 0 ? Ls[0].wsym : nullptr;
    sg.in16 = reinterpret_cast<const uint16_t*>(hcur);
    sg.in_ps = (long long)S.h * S.w * m->cfg.ctx_ch;
    sg.sym = g > 0 ? q_sub : nullptr;
    sg.sym_ps = q_ps;
    sg.params = params;
    sg.N = nplanes;
    sg.h = S.h;
    sg.w = S.w;
    sg.step = g;
    sg.K = m->cfg.mix_k;
    sg.sigma_min = m->cfg.sigma_min;
    sg.strips_x = (S.w + STACK_STRIP - 1) / STACK_STRIP;
    sg.seg_rows = stack_seg_rows(S.h, cap);
    sg.segs_y = (S.h + sg.seg_rows - 1) / sg.seg_rows;
    sg.item0 = item0;
    if (wv_group_count(S.h, S.w, g) == 0) {   // a 1-wide subband's empty step
        sg.N = 0;
        return 0;
    }
    return (long long)sg.strips_x * sg.segs_y * nplanes;
}

// Segment of a fused ConvLSTM launch for subband S of a plane group whose ConvLSTM state
// halves start at d_state (SS floats each: h then c), symbols at q (plane stride q_ps);
// Pv is the previous subband (null for the first).  Returns the segment's work items.
long long make_lstm_seg(const wv_model* m, int i, const Sub& S, const Sub* Pv, float* d_state, size_t SS,
                        int nplanes, const int16_t* q, long long q_ps, long long item0, LstmSeg& sg,
                        int cap = 128) {
    const int C = m->cfg.ctx_ch;
    sg = LstmSeg{};
    sg.wt = m->lstm16.w;
    sg.wsym = m->lstm16.wsym;
    sg.bias = m->lstm16.bias;
    float* hcur = d_state + (size_t)(i & 1) * 2 * SS;
    if (Pv) {
        float* hold = d_state + (size_t)((i - 1) & 1) * 2 * SS;
        sg.up = (S.h == 2 * Pv->h) ? 1 : 0;
        sg.in16 = reinterpret_cast<const uint16_t*>(hold);
        sg.in_ps = (long long)Pv->h * Pv->w * C;
        sg.sym = q + Pv->off;
        sg.sym_ps = q_ps;
        sg.c_prev = hold + SS;
        sg.cprev_ps = (long long)Pv->h * Pv->w * C;
    }
    sg.h_out = reinterpret_cast<uint16_t*>(hcur);
    sg.c_out = hcur + SS;
    sg.st_ps = (long long)S.h * S.w * C;
    sg.N = nplanes;
    sg.h = S.h;
    sg.w = S.w;
    sg.strips_x = (S.w + LSTM_STRIP - 1) / LSTM_STRIP;
    sg.seg_rows = stack_seg_rows(S.h, cap);
    sg.segs_y = (S.h + sg.seg_rows - 1) / sg.seg_rows;
    sg.item0 = item0;
    return (long long)sg.strips_x * sg.segs_y * nplanes;
}
}  // namespace

struct wv_plan {
    const wv_model* m;
    std::vector<wv_group> groups;
    std::vector<std::vector<Sub>> lay;            // per group
    std::vector<std::vector<PlanLaunch>> steps;   // [subband * 4 + step] -> launches
    std::vector<std::vector<long long>> row_off;  // [subband * 4 + step] -> per group first row, + total
    char* d_desc;
    float* d_params;
    int last = -1;   // coding-order cursor of the plan's groups (subband * 4 + step)
};

static int plan_build(const wv_model* m, int ng, const wv_group* groups, const int* nb_table,
                      std::vector<char>& host, wv_plan* P) {
    if (!m) return fail(WV_EINVAL, "null model");
    if (ng < 1 || !groups) return fail(WV_EINVAL, "no groups");
    if (m->cfg.ctx_arch != 0) return fail(WV_EUNSUPPORTED, "plans need ctx_arch 0");
    const bool bf16 = m->precision != WV_FP32;   // BF16 or FP8 kernels
    const int C = m->cfg.ctx_ch;
    const int J = m->cfg.levels;
    const int nsub = 3 * J + 1;
    const int th = conv_tile_h(bf16), tw = conv_tile_w(bf16);
    P->m = m;
    P->groups.assign(groups, groups + ng);
    P->lay.resize(ng);
    for (int b = 0; b < ng; ++b) {
        if (groups[b].nplanes < 1) return fail(WV_ESHAPE, "group %d has no planes", b);
        int rc = layout(m->cfg, groups[b].H, groups[b].W, P->lay[b]);
        if (rc) return rc;
    }
    P->steps.assign(nsub * 4, {});
    P->row_off.assign(nsub * 4, {});
    host.clear();
    const int seg_size = bf16 ? (int)sizeof(ConvSeg16) : (int)sizeof(ConvSeg);
    for (int i = 0; i < nsub; ++i) {
        for (int g = 0; g < 4; ++g) {
            std::vector<long long>& ro = P->row_off[i * 4 + g];
            long long rows = 0;
            for (int b = 0; b < ng; ++b) {
                ro.push_back(rows);
                rows += (long long)groups[b].nplanes * wv_group_count(P->lay[b][i].h, P->lay[b][i].w, g);
            }
            ro.push_back(rows);
            const int type = P->lay[0][i].type;
            const int level = P->lay[0][i].level;
            const int nlayers = (int)(bf16 ? m->ctx16[type][g].size() : m->ctx[type][g].size());
            const bool fuse = stack_fusable(m);
            // launch list: LSTM at step 0, then the stack's layers (or the fused ConvLSTM and
            // the fused stack)
            if (fuse && g == 0) {
                PlanLaunch pl{};
                host.resize((host.size() + 255) & ~(size_t)255);
                pl.seg_off = host.size();
                pl.nseg = ng;
                pl.fused = 2;
                std::vector<std::array<int, 3>> shapes;
                for (int b = 0; b < ng; ++b)
                    shapes.push_back({P->lay[b][i].h, P->lay[b][i].w, groups[b].nplanes});
                const int cap = fused_seg_cap(shapes, LSTM_STRIP, 3, device_cus());
                long long item = 0;
                for (int b = 0; b < ng; ++b) {
                    const wv_group& G = groups[b];
                    LstmSeg sg;
                    item += make_lstm_seg(m, i, P->lay[b][i], i > 0 ? &P->lay[b][i - 1] : nullptr, G.d_state,
                                          state_floats(m->cfg, G.nplanes, G.H, G.W), G.nplanes, G.d_q,
                                          (long long)G.H * G.W, item, sg, cap);
                    const size_t at = host.size();
                    host.resize(at + sizeof(LstmSeg));
                    memcpy(host.data() + at, &sg, sizeof sg);
                }
                pl.total = item;
                pl.grid = (int)std::min<long long>(item, device_cus());
                P->steps[i * 4].push_back(pl);
                host.resize((host.size() + 255) & ~(size_t)255);
            }
            for (int l = (g == 0 && !fuse ? -1 : 0); l < (fuse ? 0 : nlayers); ++l) {
                const bool lstm = l < 0;
                const bool last = l == nlayers - 1;
                const int mode = lstm ? CONV_LSTM : (last ? CONV_HEAD : CONV_RELU);
                const MfmaLayer* L32 = bf16 ? nullptr : (lstm ? &m->lstm : &m->ctx[type][g][l]);
                const MfmaLayer16* L16 = bf16 ? (lstm ? &m->lstm16 : &m->ctx16[type][g][l]) : nullptr;
                const int nbt = bf16 ? L16->nbt : L32->nbt;
                long long tiles = 0;
                for (int b = 0; b < ng; ++b) {
                    const Sub& S = P->lay[b][i];
                    tiles += (long long)((S.w + tw - 1) / tw) * ((S.h + th - 1) / th) * groups[b].nplanes;
                }
                int nb = conv_pick_nb(nbt, mode, tiles, bf16);
                if (nb_table && mode == CONV_RELU) {
                    const int want = nb_table[level - 1];
                    if (want == 1 || want == 2 || want == 4) nb = want <= nbt ? want : nbt;
                }
                PlanLaunch pl{};
                pl.seg_off = host.size();
                pl.nseg = ng;
                pl.mode = mode;
                pl.nb = nb;
                if (bf16) pl.proto16 = *L16; else pl.proto = *L32;
                long long item = 0;
                for (int b = 0; b < ng; ++b) {
                    const wv_group& G = groups[b];
                    const Sub& S = P->lay[b][i];
                    const long long HW = (long long)G.H * G.W;
                    const size_t SS = state_floats(m->cfg, G.nplanes, G.H, G.W);
                    float* hcur = G.d_state + (size_t)(i & 1) * 2 * SS;
                    const long long st_ps = (long long)S.h * S.w * C;
                    const Scratch sc = scratch_layout(m->cfg, G.nplanes, G.H, G.W);
                    float* act[2] = {(float*)G.d_scratch + sc.act0, (float*)G.d_scratch + sc.act1};
                    ConvArgs a{};
                    a.N = G.nplanes;
                    a.h = S.h;
                    a.w = S.w;
                    a.tiles_x = (S.w + tw - 1) / tw;
                    a.tiles_y = (S.h + th - 1) / th;
                    if (lstm) {
                        a.sym_step = 4;
                        a.h_out = hcur;
                        a.c_out = hcur + SS;
                        a.st_ps = st_ps;
                        a.C = C;
                        if (i > 0) {
                            const Sub& Pv = P->lay[b][i - 1];
                            const int up = (S.h == 2 * Pv.h) ? 1 : 0;
                            float* hold = G.d_state + (size_t)((i - 1) & 1) * 2 * SS;
                            a.in = hold;
                            a.in_ps = (long long)Pv.h * Pv.w * C;
                            a.in_up = up;
                            a.sym = G.d_q + Pv.off;
                            a.sym_ps = HW;
                            a.sym_up = up;
                            a.c_prev = hold + SS;
                            a.cprev_ps = (long long)Pv.h * Pv.w * C;
                            a.cprev_up = up;
                        }
                        if (bf16) {
                            a.in16 = reinterpret_cast<const uint16_t*>(a.in);
                            a.in = nullptr;
                            a.h16_out = reinterpret_cast<uint16_t*>(hcur);
                            a.h_out = nullptr;
                        }
                    } else {
                        a.in = l == 0 ? hcur : act[(l - 1) & 1];
                        a.in_ps = st_ps;
                        if (l == 0 && g > 0) {
                            a.sym = G.d_q + S.off;
                            a.sym_ps = HW;
                            a.sym_step = g;
                        }
                        if (!last) {
                            a.out = act[l & 1];
                            a.out_ps = st_ps;
                            a.out_cs = C;
                        } else {
                            a.params = P->d_params ? P->d_params + ro[b] * 3 * m->cfg.mix_k : nullptr;
                            a.step = g;
                            a.K = m->cfg.mix_k;
                            a.sigma_min = m->cfg.sigma_min;
                        }
                        if (bf16) {
                            a.in16 = reinterpret_cast<const uint16_t*>(a.in);
                            a.in = nullptr;
                            a.out16 = reinterpret_cast<uint16_t*>(a.out);
                            a.out = nullptr;
                        }
                    }
                    const long long items = (long long)a.tiles_x * a.tiles_y * a.N * (mode == CONV_HEAD ? 1 : nbt / nb);
                    const size_t at = host.size();
                    host.resize(at + seg_size);
                    if (bf16) {
                        ConvSeg16 sg{*L16, a, item};
                        memcpy(host.data() + at, &sg, sizeof sg);
                    } else {
                        ConvSeg sg{*L32, a, item};
                        memcpy(host.data() + at, &sg, sizeof sg);
                    }
                    item += items;
                }
                pl.total = item;
                pl.grid = (int)(item < 1024 ? item : 1024);
                P->steps[i * 4 + g].push_back(pl);
                host.resize((host.size() + 255) & ~(size_t)255);
            }
            if (fuse) {
                PlanLaunch pl{};
                host.resize((host.size() + 255) & ~(size_t)255);
                pl.seg_off = host.size();
                pl.nseg = ng;
                pl.fused = 1;
                pl.has_sym = g > 0;
                std::vector<std::array<int, 3>> shapes;
                for (int b = 0; b < ng; ++b)   // a step with no positions in a group adds no items
                    shapes.push_back({P->lay[b][i].h, P->lay[b][i].w,
                                      wv_group_count(P->lay[b][i].h, P->lay[b][i].w, g) ? groups[b].nplanes : 0});
                const int cap = fused_seg_cap(shapes, STACK_STRIP, 10, device_cus());
                long long item = 0;
                for (int b = 0; b < ng; ++b) {
                    const wv_group& G = groups[b];
                    const Sub& S = P->lay[b][i];
                    const size_t SS = state_floats(m->cfg, G.nplanes, G.H, G.W);
                    const float* hcur = G.d_state + (size_t)(i & 1) * 2 * SS;
                    StackSeg sg;
                    item += make_stack_seg(m, type, g, hcur, S, G.nplanes, G.d_q + S.off, (long long)G.H * G.W,
                                           P->d_params ? P->d_params + ro[b] * 3 * m->cfg.mix_k : nullptr, item, sg,
                                           cap);
                    const size_t at = host.size();
                    host.resize(at + sizeof(StackSeg));
                    memcpy(host.data() + at, &sg, sizeof sg);
                }
                pl.total = item;
                pl.grid = (int)std::min<long long>(item, device_cus());
                P->steps[i * 4 + g].push_back(pl);
                host.resize((host.size() + 255) & ~(size_t)255);
            }
        }
    }
    return WV_OK;
}

extern "C" int wv_plan_bytes(const wv_model* m, int ngroups, const wv_group* groups,
                             const int* nb_table, size_t* desc_bytes, long long* max_rows) {
    wv_plan P{};
    P.d_params = nullptr;
    std::vector<char> host;
    int rc = plan_build(m, ngroups, groups, nb_table, host, &P);
    if (rc) return rc;
    if (desc_bytes) *desc_bytes = host.size();
    if (max_rows) {
        long long mx = 0;
        for (auto& ro : P.row_off) mx = ro.back() > mx ? ro.back() : mx;
        *max_rows = mx;
    }
    return WV_OK;
}

extern "C" int wv_plan_create(const wv_model* m, int ngroups, const wv_group* groups,
                              const int* nb_table, void* d_desc, size_t desc_bytes, float* d_params,
                              void* stream, wv_plan** out) {
    if (!d_desc || !d_params || !out) return fail(WV_EINVAL, "null pointer");
    wv_plan* P = new wv_plan();
    P->d_params = d_params;
    std::vector<char> host;
    int rc = plan_build(m, ngroups, groups, nb_table, host, P);
    if (rc) {
        delete P;
        return rc;
    }
    if (host.size() > desc_bytes) {
        delete P;
        return fail(WV_ENOMEM, "descriptor buffer has %zu bytes, needs %zu", desc_bytes, host.size());
    }
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(d_desc, host.data(), host.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        delete P;
        return fail(WV_EDEVICE, "descriptor upload failed: %s", hipGetErrorString(e));
    }
    P->d_desc = (char*)d_desc;
    *out = P;
    return WV_OK;
}

extern "C" void wv_plan_destroy(wv_plan* p) { delete p; }

extern "C" int wv_plan_rows(const wv_plan* p, int i, int g, long long* rows, long long* group_first) {
    if (!p || !rows) return fail(WV_EINVAL, "null pointer");
    const int nsub = (int)p->lay[0].size();
    if (i < 0 || i >= nsub || g < 0 || g > 3) return fail(WV_EORDER, "subband %d / step %d out of range", i, g);
    const auto& ro = p->row_off[i * 4 + g];
    *rows = ro.back();
    if (group_first)
        for (size_t b = 0; b + 1 < ro.size(); ++b) group_first[b] = ro[b];
    return WV_OK;
}

static int plan_step_launch(const wv_plan* p, int i, int g, void* stream);

extern "C" int wv_plan_context_params(wv_plan* p, int i, int g, void* stream) {
    if (!p) return fail(WV_EINVAL, "null plan");
    const int nsub = (int)p->lay[0].size();
    if (i < 0 || i >= nsub || g < 0 || g > 3) return fail(WV_EORDER, "subband %d / step %d out of range", i, g);
    if (!order_ok(p->last, i, g, p->m->cfg.ll_ar != 0)) {
        if (p->last < 0) return fail(WV_EORDER, "wv_plan_context_params: (subband %d, step %d) before (0, 0)", i, g);
        return fail(WV_EORDER, "wv_plan_context_params: (subband %d, step %d) does not follow (subband %d, step %d)",
                    i, g, p->last >> 2, p->last & 3);
    }
    const int rc = plan_step_launch(p, i, g, stream);
    if (rc == WV_OK) p->last = (i == nsub - 1 && g == 3) ? -1 : i * 4 + g;
    return rc;
}

static int plan_step_launch(const wv_plan* p, int i, int g, void* stream) {
    hipStream_t s = (hipStream_t)stream;
    const bool bf16 = p->m->precision != WV_FP32;   // BF16 or FP8 kernels
    for (const PlanLaunch& pl : p->steps[i * 4 + g]) {
        if (pl.fused == 2) {
            HIPCHK(launch_lstm_bf16(reinterpret_cast<const LstmSeg*>(p->d_desc + pl.seg_off), pl.nseg, pl.total,
                                    pl.grid, s));
            continue;
        }
        if (pl.fused) {
            HIPCHK(launch_stack_bf16(reinterpret_cast<const StackSeg*>(p->d_desc + pl.seg_off), pl.nseg, pl.total,
                                     pl.has_sym, pl.grid, s));
            continue;
        }
        if (bf16)
            HIPCHK(launch_conv_seg_bf16(reinterpret_cast<const ConvSeg16*>(p->d_desc + pl.seg_off), pl.nseg,
                                        pl.total, pl.proto16, pl.mode, pl.nb, pl.grid, s));
        else
            HIPCHK(launch_conv_seg(reinterpret_cast<const ConvSeg*>(p->d_desc + pl.seg_off), pl.nseg, pl.total,
                                   pl.proto, pl.mode, pl.nb, pl.grid, s));
    }
    return WV_OK;
}

extern "C" int wv_plan_scatter(const wv_plan* p, const uint8_t* d_sym, int i, int g, void* stream) {
    if (!p || !d_sym) return fail(WV_EINVAL, "null pointer");
    const int nsub = (int)p->lay[0].size();
    if (i < 0 || i >= nsub || g < 0 || g > 3) return fail(WV_EORDER, "subband %d / step %d out of range", i, g);
    const auto& ro = p->row_off[i * 4 + g];
    for (size_t b = 0; b < p->groups.size(); ++b) {
        const wv_group& G = p->groups[b];
        const Sub& S = p->lay[b][i];
        HIPCHK(launch_scatter(d_sym + ro[b], G.d_q, G.nplanes, (long long)G.H * G.W, S.off, S.h, S.w, g,
                              p->m->cfg.sym_min, (hipStream_t)stream));
    }
    return WV_OK;
}

// ---------------------------------------------------------------------------
// items: plane groups at different (subband, step) positions in one call
// ---------------------------------------------------------------------------
namespace {
struct ItemLaunch {
    std::vector<char> segs;
    int nseg = 0, mode = 0, nb = 1;
    int fused = 0, has_sym = 0;   // 1: fused step stacks (segs holds StackSeg); 2: fused ConvLSTM (LstmSeg)
    long long total = 0;
    long long tiles = 0;
    MfmaLayer proto{};
    MfmaLayer16 proto16{};
};

// Append one segment (an item's layer) to a launch list.
void item_seg(ItemLaunch& Lc, bool bf16, const MfmaLayer* L32, const MfmaLayer16* L16, const ConvArgs& a) {
    const size_t at = Lc.segs.size();
    if (bf16) {
        Lc.segs.resize(at + sizeof(ConvSeg16));
        ConvSeg16 sg{*L16, a, 0};
        memcpy(Lc.segs.data() + at, &sg, sizeof sg);
        Lc.proto16 = *L16;
    } else {
        Lc.segs.resize(at + sizeof(ConvSeg));
        ConvSeg sg{*L32, a, 0};
        memcpy(Lc.segs.data() + at, &sg, sizeof sg);
        Lc.proto = *L32;
    }
    Lc.nseg++;
    Lc.tiles += (long long)a.tiles_x * a.tiles_y * a.N;
}

// Fix NB and item offsets once all segments of a launch are known.
void item_finish(ItemLaunch& Lc, bool bf16) {
    if (!Lc.nseg) return;
    const int nbt = bf16 ? Lc.proto16.nbt : Lc.proto.nbt;
    Lc.nb = conv_pick_nb(nbt, Lc.mode, Lc.tiles, bf16);
    long long item = 0;
    const size_t ss = bf16 ? sizeof(ConvSeg16) : sizeof(ConvSeg);
    for (int k = 0; k < Lc.nseg; ++k) {
        char* p = Lc.segs.data() + k * ss;
        const ConvArgs& a = bf16 ? reinterpret_cast<ConvSeg16*>(p)->a : reinterpret_cast<ConvSeg*>(p)->a;
        const int segnbt = bf16 ? reinterpret_cast<ConvSeg16*>(p)->L.nbt : reinterpret_cast<ConvSeg*>(p)->L.nbt;
        if (bf16) reinterpret_cast<ConvSeg16*>(p)->item0 = item;
        else reinterpret_cast<ConvSeg*>(p)->item0 = item;
        item += (long long)a.tiles_x * a.tiles_y * a.N * (Lc.mode == CONV_HEAD ? 1 : segnbt / Lc.nb);
    }
    Lc.total = item;
}
}  // namespace

extern "C" int wv_context_params_items(const wv_model* m, int n, const wv_step_item* items,
                                       void* h_staging, size_t staging_bytes, void* d_desc,
                                       size_t desc_bytes, size_t* used_bytes, void* stream) {
    if (!m) return fail(WV_EINVAL, "null model");
    if (n < 0 || (n > 0 && !items)) return fail(WV_EINVAL, "bad item list");
    if (m->cfg.ctx_arch != 0) return fail(WV_EUNSUPPORTED, "items need ctx_arch 0");
    const bool bf16 = m->precision != WV_FP32;   // BF16 or FP8 kernels
    const int C = m->cfg.ctx_ch;
    const int Lc = m->cfg.ctx_layers;
    const int th = conv_tile_h(bf16), tw = conv_tile_w(bf16);
    // Launch roles: 0 LSTM, 1 first layer without symbols (step 0), 2 first layer with
    // symbols, 3 + (l - 1) inner layer l, last: the head.
    const bool fuse = stack_fusable(m);
    // fused step stacks (steps 0 and >= 1) after the per-layer roles
    std::vector<ItemLaunch> launches(3 + (Lc - 2) + 1 + 2);
    const int fuse0 = 3 + (Lc - 2) + 1;
    launches[fuse0].fused = 1;
    launches[fuse0 + 1].fused = 1;
    launches[fuse0 + 1].has_sym = 1;
    launches[0].mode = CONV_LSTM;
    if (fuse) launches[0].fused = 2;   // the fused ConvLSTM (LstmSeg array)
    launches[1].mode = CONV_RELU;
    launches[2].mode = CONV_RELU;
    for (int l = 1; l < Lc - 1; ++l) launches[2 + l].mode = CONV_RELU;
    launches[fuse0 - 1].mode = CONV_HEAD;
    // Row-piece caps of the three fused launches, from the shapes of all items (an item the
    // checks below reject is skipped here).
    int cap_lstm = 128, cap_st0 = 128, cap_st1 = 128;
    if (fuse) {
        std::vector<std::array<int, 3>> sh_l, sh_0, sh_1;
        for (int k = 0; k < n; ++k) {
            const wv_step_item& it = items[k];
            std::vector<Sub> lay;
            if (it.nplanes < 1 || layout(m->cfg, it.H, it.W, lay) != WV_OK) continue;
            const int i = it.subband, g = it.step;
            if (i < 0 || i >= (int)lay.size() || g < 0 || g > 3) continue;
            const Sub& S = lay[i];
            if (g == 0) sh_l.push_back({S.h, S.w, it.nplanes});
            if (wv_group_count(S.h, S.w, g) > 0) (g > 0 ? sh_1 : sh_0).push_back({S.h, S.w, it.nplanes});
        }
        const long long cus = device_cus();
        cap_lstm = fused_seg_cap(sh_l, LSTM_STRIP, 3, cus);
        cap_st0 = fused_seg_cap(sh_0, STACK_STRIP, 10, cus);
        cap_st1 = fused_seg_cap(sh_1, STACK_STRIP, 10, cus);
    }
    std::vector<int> nsubs;   // per item, for the coding-order cursor
    for (int k = 0; k < n; ++k) {
        const wv_step_item& it = items[k];
        if (!it.d_q || !it.d_state || !it.d_scratch || it.nplanes < 1)
            return fail(WV_EINVAL, "item %d: bad buffers", k);
        std::vector<Sub> lay;
        int rc = layout(m->cfg, it.H, it.W, lay);
        if (rc) return rc;
        const int i = it.subband, g = it.step;
        if (i < 0 || i >= (int)lay.size() || g < 0 || g > 3)
            return fail(WV_EORDER, "item %d: subband %d / step %d out of range", k, i, g);
        for (int k2 = 0; k2 < k; ++k2)
            if (items[k2].d_state == it.d_state) return fail(WV_EINVAL, "items %d and %d share a state buffer", k2, k);
        if ((rc = order_check(it.d_state, i, g, m->cfg.ll_ar != 0, "wv_context_params_items"))) return rc;
        nsubs.push_back((int)lay.size());
        const Sub& S = lay[i];
        const long long ng = wv_group_count(S.h, S.w, g);
        if (ng > 0 && !it.d_params) return fail(WV_EINVAL, "item %d: null params", k);
        const long long HW = (long long)it.H * it.W;
        const size_t SS = state_floats(m->cfg, it.nplanes, it.H, it.W);
        float* hcur = it.d_state + (size_t)(i & 1) * 2 * SS;
        const long long st_ps = (long long)S.h * S.w * C;
        const Scratch sc = scratch_layout(m->cfg, it.nplanes, it.H, it.W);
        float* act[2] = {(float*)it.d_scratch + sc.act0, (float*)it.d_scratch + sc.act1};
        ConvArgs base{};
        base.N = it.nplanes;
        base.h = S.h;
        base.w = S.w;
        base.tiles_x = (S.w + tw - 1) / tw;
        base.tiles_y = (S.h + th - 1) / th;
        if (g == 0 && fuse) {
            ItemLaunch& Ll = launches[0];
            LstmSeg sg;
            Ll.total += make_lstm_seg(m, i, S, i > 0 ? &lay[i - 1] : nullptr, it.d_state, SS, it.nplanes, it.d_q, HW,
                                      Ll.total, sg, cap_lstm);
            const size_t at = Ll.segs.size();
            Ll.segs.resize(at + sizeof(LstmSeg));
            memcpy(Ll.segs.data() + at, &sg, sizeof sg);
            Ll.nseg++;
        } else if (g == 0) {
            ConvArgs a = base;
            a.sym_step = 4;
            a.h_out = hcur;
            a.c_out = hcur + SS;
            a.st_ps = st_ps;
            a.C = C;
            if (i > 0) {
                const Sub& Pv = lay[i - 1];
                const int up = (S.h == 2 * Pv.h) ? 1 : 0;
                float* hold = it.d_state + (size_t)((i - 1) & 1) * 2 * SS;
                a.in = hold;
                a.in_ps = (long long)Pv.h * Pv.w * C;
                a.in_up = up;
                a.sym = it.d_q + Pv.off;
                a.sym_ps = HW;
                a.sym_up = up;
                a.c_prev = hold + SS;
                a.cprev_ps = (long long)Pv.h * Pv.w * C;
                a.cprev_up = up;
            }
            if (bf16) {
                a.in16 = reinterpret_cast<const uint16_t*>(a.in);
                a.in = nullptr;
                a.h16_out = reinterpret_cast<uint16_t*>(hcur);
                a.h_out = nullptr;
            }
            item_seg(launches[0], bf16, bf16 ? nullptr : &m->lstm, bf16 ? &m->lstm16 : nullptr, a);
        }
        if (ng == 0) continue;
        if (fuse) {
            ItemLaunch& Fl = launches[fuse0 + (g > 0)];
            StackSeg sg;
            Fl.total += make_stack_seg(m, S.type, g, hcur, S, it.nplanes, it.d_q + S.off, HW, it.d_params, Fl.total, sg,
                                       g > 0 ? cap_st1 : cap_st0);
            const size_t at = Fl.segs.size();
            Fl.segs.resize(at + sizeof(StackSeg));
            memcpy(Fl.segs.data() + at, &sg, sizeof sg);
            Fl.nseg++;
            continue;
        }
        for (int l = 0; l < Lc; ++l) {
            const bool last = l == Lc - 1;
            ConvArgs a = base;
            a.in = l == 0 ? hcur : act[(l - 1) & 1];
            a.in_ps = st_ps;
            if (l == 0 && g > 0) {
                a.sym = it.d_q + S.off;
                a.sym_ps = HW;
                a.sym_step = g;
            }
            if (!last) {
                a.out = act[l & 1];
                a.out_ps = st_ps;
                a.out_cs = C;
            } else {
                a.params = it.d_params;
                a.step = g;
                a.K = m->cfg.mix_k;
                a.sigma_min = m->cfg.sigma_min;
            }
            if (bf16) {
                a.in16 = reinterpret_cast<const uint16_t*>(a.in);
                a.in = nullptr;
                a.out16 = reinterpret_cast<uint16_t*>(a.out);
                a.out = nullptr;
            }
            const int role = l == 0 ? (g > 0 ? 2 : 1) : (last ? fuse0 - 1 : 2 + l);
            item_seg(launches[role], bf16, bf16 ? nullptr : &m->ctx[S.type][g][l],
                     bf16 ? &m->ctx16[S.type][g][l] : nullptr, a);
        }
    }
    size_t total = 0;
    for (auto& Lx : launches) {
        if (!Lx.fused) item_finish(Lx, bf16);
        total += (Lx.segs.size() + 255) & ~(size_t)255;
    }
    if (used_bytes) *used_bytes = total;
    if (total == 0) {   // only empty steps: nothing to launch, the items still advance
        for (int k = 0; k < n; ++k) order_commit(items[k].d_state, items[k].subband, items[k].step, nsubs[k]);
        return WV_OK;
    }
    if (!h_staging || !d_desc) return fail(WV_EINVAL, "null staging or descriptor buffer");
    if (total > staging_bytes || total > desc_bytes)
        return fail(WV_ENOMEM, "descriptors need %zu bytes", total);
    size_t off = 0;
    std::vector<size_t> offs;
    for (auto& Lx : launches) {
        offs.push_back(off);
        memcpy((char*)h_staging + off, Lx.segs.data(), Lx.segs.size());
        off += (Lx.segs.size() + 255) & ~(size_t)255;
    }
    hipStream_t s = (hipStream_t)stream;
    HIPCHK(hipMemcpyAsync(d_desc, h_staging, total, hipMemcpyHostToDevice, s));
    for (size_t r = 0; r < launches.size(); ++r) {
        const ItemLaunch& Lx = launches[r];
        if (!Lx.nseg || !Lx.total) continue;
        if (Lx.fused == 2) {
            HIPCHK(launch_lstm_bf16(reinterpret_cast<const LstmSeg*>((char*)d_desc + offs[r]), Lx.nseg, Lx.total,
                                    (int)std::min<long long>(Lx.total, device_cus()), s));
            continue;
        }
        if (Lx.fused) {
            HIPCHK(launch_stack_bf16(reinterpret_cast<const StackSeg*>((char*)d_desc + offs[r]), Lx.nseg, Lx.total,
                                     Lx.has_sym, (int)std::min<long long>(Lx.total, device_cus()), s));
            continue;
        }
        const int grid = (int)(Lx.total < 1024 ? Lx.total : 1024);
        if (bf16)
            HIPCHK(launch_conv_seg_bf16(reinterpret_cast<const ConvSeg16*>((char*)d_desc + offs[r]), Lx.nseg,
                                        Lx.total, Lx.proto16, Lx.mode, Lx.nb, grid, s));
        else
            HIPCHK(launch_conv_seg(reinterpret_cast<const ConvSeg*>((char*)d_desc + offs[r]), Lx.nseg, Lx.total,
                                   Lx.proto, Lx.mode, Lx.nb, grid, s));
    }
    for (int k = 0; k < n; ++k) order_commit(items[k].d_state, items[k].subband, items[k].step, nsubs[k]);
    return WV_OK;
}

// ---------------------------------------------------------------------------
// graphs of library calls, and a zero fill that can be captured
// ---------------------------------------------------------------------------
struct wv_graph {
    hipGraph_t graph;
    hipGraphExec_t exec;
};

extern "C" int wv_zero(void* d, size_t bytes, void* stream) {
    if (!bytes) return WV_OK;
    if (!d) return fail(WV_EINVAL, "null pointer");
    if ((uintptr_t)d & 15) return fail(WV_EINVAL, "wv_zero needs a 16-byte aligned pointer");
    HIPCHK(launch_zero(d, bytes, (hipStream_t)stream));
    return WV_OK;
}

extern "C" int wv_graph_begin(void* stream) {
    if (!stream) return fail(WV_EINVAL, "capture needs a stream other than the default stream");
    HIPCHK(hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeThreadLocal));
    return WV_OK;
}

extern "C" int wv_graph_end(void* stream, wv_graph** out) {
    if (!stream || !out) return fail(WV_EINVAL, "null pointer");
    *out = nullptr;
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture((hipStream_t)stream, &g);
    if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return fail(WV_EDEVICE, "capture failed: %s", hipGetErrorString(e));
    }
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(WV_EDEVICE, "graph instantiation failed: %s", hipGetErrorString(e));
    }
    *out = new wv_graph{g, x};
    return WV_OK;
}

extern "C" int wv_graph_launch(const wv_graph* g, void* stream) {
    if (!g) return fail(WV_EINVAL, "null graph");
    HIPCHK(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return WV_OK;
}

extern "C" void wv_graph_destroy(wv_graph* g) {
    if (!g) return;
    (void)hipGraphExecDestroy(g->exec);
    (void)hipGraphDestroy(g->graph);
    delete g;
}

