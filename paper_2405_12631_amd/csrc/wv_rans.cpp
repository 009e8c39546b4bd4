// Host rANS entropy coder for the per-coefficient CDF tables.
//
// Byte-wise renormalising range-ANS (J. Duda, 2013): 32-bit state in
// [L, 256 L) with L = 2^23, probabilities out of M = 2^16.  Symbols are
// pushed last to first so that the decoder pops them in raster order; the
// encoder writes bytes downwards from the end of the output buffer and
// finally the state, little endian, in front of them.  A valid stream
// decodes back to the initial state L with every byte consumed, which is
// checked to flag corrupt input.
#include <stdint.h>
#include <string.h>

#include "../../include/wv.h"

namespace {

constexpr uint32_t kL = 1u << 23;
constexpr int kProbBits = 16;
constexpr uint32_t kM = 1u << kProbBits;

inline uint32_t row_at(const uint16_t* row, int s, int nsym) {
    return s >= nsym ? kM : row[s];   // entry nsym is stored as 0 (mod 2^16)
}

// Tables as stored by wv_cdf_tables: row i at cdf + i (nsym + 1).
struct FullRows {
    const uint16_t* cdf;
    int nsym;
    const uint16_t* row(long long i, uint16_t*) const { return cdf + (size_t)i * (nsym + 1); }
};

// Trimmed tables (wv_cdf_trim): row i rebuilt from (lo, len) and its F values,
// which start at offset off of packed; false if they do not describe a row.
struct TrimRows {
    const uint8_t* lolen;
    const uint16_t* packed;
    long long count;   // values in packed
    int nsym;
    bool build(long long i, long long off, uint16_t* tmp) const {
        const int lo = lolen[2 * i], len = lolen[2 * i + 1];
        if (lo < 1 || lo + len > nsym || off < 0 || off + len > count) return false;
        const int ftop = (int)kM - nsym - 1;   // F_max - 1: the plateau above the window
        for (int j = 0; j < nsym; ++j) {
            const int F = j < lo ? 0 : j < lo + len ? packed[off + j - lo] : ftop;
            tmp[j] = (uint16_t)(j + F);
        }
        return true;
    }
};

}  // namespace

extern "C" int wv_cdf_untrim(const uint8_t* lolen, const uint16_t* packed, long long packed_count, int nsym,
                             long long n, uint16_t* cdf_out) {
    if (nsym < 2 || nsym > 255 || n < 0 || packed_count < 0 || (n > 0 && (!lolen || !cdf_out)) ||
        (packed_count > 0 && !packed))
        return WV_EINVAL;
    TrimRows T{lolen, packed, packed_count, nsym};
    long long off = 0;
    for (long long i = 0; i < n; ++i) {
        uint16_t* row = cdf_out + (size_t)i * (nsym + 1);
        if (!T.build(i, off, row)) return WV_ECORRUPT;
        row[nsym] = 0;   // 2^16 mod 2^16
        off += lolen[2 * i + 1];
    }
    return off == packed_count ? WV_OK : WV_ECORRUPT;
}

namespace {

// Symbols i = n-1 .. 0; row(i) gives row i's table (entries 0 .. nsym-1).
template <class RowOf>
int encode_rows(RowOf&& rowof, int nsym, const uint8_t* sym, long long n, uint8_t* out, size_t cap, size_t* len) {
    uint8_t* ptr = out + cap;
    uint32_t x = kL;
    for (long long i = n - 1; i >= 0; --i) {
        const uint16_t* row = rowof(i);
        if (!row) return WV_EINVAL;
        const int s = sym[i];
        if (s >= nsym) return WV_EINVAL;
        const uint32_t start = row[s];
        const uint32_t end = row_at(row, s + 1, nsym);
        if (end <= start) return WV_EINVAL;   // zero-frequency symbol: not encodable
        const uint32_t freq = end - start;
        const uint32_t x_max = ((kL >> kProbBits) << 8) * freq;
        while (x >= x_max) {
            if (ptr == out) return WV_ENOMEM;
            *--ptr = (uint8_t)(x & 0xff);
            x >>= 8;
        }
        x = ((x / freq) << kProbBits) + (x % freq) + start;
    }
    if ((size_t)(ptr - out) < 4) return WV_ENOMEM;
    ptr -= 4;
    ptr[0] = (uint8_t)(x);
    ptr[1] = (uint8_t)(x >> 8);
    ptr[2] = (uint8_t)(x >> 16);
    ptr[3] = (uint8_t)(x >> 24);
    const size_t total = (size_t)(out + cap - ptr);
    memmove(out, ptr, total);
    *len = total;
    return WV_OK;
}

// Symbols i = 0 .. n-1; row(i) gives row i's table.
template <class RowOf>
int decode_rows(RowOf&& rowof, int nsym, long long n, const uint8_t* in, size_t len, uint8_t* sym_out) {
    if (len < 4) return WV_ECORRUPT;
    uint32_t x = (uint32_t)in[0] | ((uint32_t)in[1] << 8) | ((uint32_t)in[2] << 16) | ((uint32_t)in[3] << 24);
    size_t pos = 4;
    if (x < kL) return WV_ECORRUPT;
    for (long long i = 0; i < n; ++i) {
        const uint16_t* row = rowof(i);
        if (!row) return WV_ECORRUPT;
        const uint32_t slot = x & (kM - 1);
        // largest s with row[s] <= slot (row[0] = 0, row[nsym] = M)
        int lo = 0, hi = nsym;   // invariant: row[lo] <= slot < row_at(hi)
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (row[mid] <= slot)
                lo = mid;
            else
                hi = mid;
        }
        const uint32_t start = row[lo];
        const uint32_t end = row_at(row, lo + 1, nsym);
        if (end <= start || slot < start) return WV_ECORRUPT;
        x = (end - start) * (x >> kProbBits) + slot - start;
        while (x < kL) {
            if (pos >= len) return WV_ECORRUPT;
            x = (x << 8) | in[pos++];
        }
        sym_out[i] = (uint8_t)lo;
    }
    if (x != kL || pos != len) return WV_ECORRUPT;
    return WV_OK;
}

}  // namespace

extern "C" int wv_rans_encode(const uint16_t* cdf, int nsym, const uint8_t* sym, long long n,
                              uint8_t* out, size_t cap, size_t* len) {
    if (nsym < 2 || nsym > 255 || n < 0 || !len || (n > 0 && (!cdf || !sym)) || !out)
        return WV_EINVAL;
    const FullRows R{cdf, nsym};
    return encode_rows([&](long long i) { return R.row(i, nullptr); }, nsym, sym, n, out, cap, len);
}

extern "C" int wv_rans_decode(const uint16_t* cdf, int nsym, long long n, const uint8_t* in,
                              size_t len, uint8_t* sym_out) {
    if (nsym < 2 || nsym > 255 || n < 0 || (n > 0 && (!cdf || !sym_out)) || (len > 0 && !in))
        return WV_EINVAL;
    const FullRows R{cdf, nsym};
    return decode_rows([&](long long i) { return R.row(i, nullptr); }, nsym, n, in, len, sym_out);
}

extern "C" int wv_rans_encode_trim(const uint8_t* lolen, const uint16_t* packed, long long packed_count, int nsym,
                                   const uint8_t* sym, long long n, uint8_t* out, size_t cap, size_t* len) {
    if (nsym < 2 || nsym > 255 || n < 0 || packed_count < 0 || !len || (n > 0 && (!lolen || !sym)) || !out ||
        (packed_count > 0 && !packed))
        return WV_EINVAL;
    long long total = 0;
    for (long long i = 0; i < n; ++i) total += lolen[2 * i + 1];
    if (total != packed_count) return WV_EINVAL;
    const TrimRows T{lolen, packed, packed_count, nsym};
    uint16_t tmp[256];
    long long end = total;   // rows are visited last to first
    return encode_rows(
        [&](long long i) -> const uint16_t* {
            end -= lolen[2 * i + 1];
            return T.build(i, end, tmp) ? tmp : nullptr;
        },
        nsym, sym, n, out, cap, len);
}

extern "C" int wv_rans_decode_trim(const uint8_t* lolen, const uint16_t* packed, long long packed_count, int nsym,
                                   long long n, const uint8_t* in, size_t len, uint8_t* sym_out) {
    if (nsym < 2 || nsym > 255 || n < 0 || packed_count < 0 || (n > 0 && (!lolen || !sym_out)) ||
        (len > 0 && !in) || (packed_count > 0 && !packed))
        return WV_EINVAL;
    const TrimRows T{lolen, packed, packed_count, nsym};
    uint16_t tmp[256];
    long long off = 0;   // rows are visited first to last
    return decode_rows(
        [&](long long i) -> const uint16_t* {
            const bool ok = T.build(i, off, tmp);
            off += lolen[2 * i + 1];
            return ok ? tmp : nullptr;
        },
        nsym, n, in, len, sym_out);
}
