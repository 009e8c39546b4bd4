"""Reference range-variant asymmetric numeral system (rANS) coder (test infrastructure).

Byte-wise renormalising rANS (J. Duda, "Asymmetric numeral systems", 2013),
with a 32-bit state kept in [L, 256 L), L = 2^23, and frequencies summing to
M = 2^16.  Each symbol has its own CDF row (cdf[s] = start of symbol s,
cdf[N_s] = M).  Symbols are encoded in reverse order so the decoder reads them
in raster order; the final state is written as 4 bytes, little endian, at the
front of the stream.
"""
import numpy as np

_L = 1 << 23
_PROB_BITS = 16
_M = 1 << _PROB_BITS


def _row(cdf_row):
    r = [int(v) for v in cdf_row]
    if r[-1] == 0:           # uint16 storage of the final entry M
        r[-1] = _M
    return r


def rans_encode_ref(cdf, idx):
    """Encode symbol indices idx[n] with rows cdf[n][N_s + 1] -> bytes."""
    cdf = np.asarray(cdf)
    x = _L
    out = bytearray()          # bytes in reverse order
    for n in range(len(idx) - 1, -1, -1):
        r = _row(cdf[n])
        s = int(idx[n])
        start, freq = r[s], r[s + 1] - r[s]
        x_max = ((_L >> _PROB_BITS) << 8) * freq
        while x >= x_max:
            out.append(x & 0xFF)
            x >>= 8
        x = ((x // freq) << _PROB_BITS) + (x % freq) + start
    for _ in range(4):
        out.append(x & 0xFF)
        x >>= 8
    # out holds, in reverse: renormalisation bytes then the state's 4 bytes
    # high byte last; reversing gives the state big-end first, so re-order the
    # state to little endian at the front.
    out.reverse()
    state = bytes(out[:4])[::-1]
    return state + bytes(out[4:])


def rans_decode_ref(cdf, data, n):
    """Decode n symbol indices from `data` with rows cdf[n][N_s + 1]."""
    cdf = np.asarray(cdf)
    data = bytes(data)
    if len(data) < 4:
        raise ValueError("truncated stream")
    x = int.from_bytes(data[:4], "little")
    pos = 4
    out = np.empty(n, np.int64)
    for k in range(n):
        r = _row(cdf[k])
        slot = x & (_M - 1)
        s = 0
        while r[s + 1] <= slot:
            s += 1
        start, freq = r[s], r[s + 1] - r[s]
        x = freq * (x >> _PROB_BITS) + slot - start
        while x < _L:
            if pos >= len(data):
                raise ValueError("truncated stream")
            x = (x << 8) | data[pos]
            pos += 1
        out[k] = s
    return out


class RansDecoderRef:
    """Symbol-at-a-time decoder for streams whose next CDF row depends on the
    symbols decoded so far (the autoregressive LL model)."""

    def __init__(self, data):
        self.data = bytes(data)
        if len(self.data) < 4:
            raise ValueError("truncated stream")
        self.x = int.from_bytes(self.data[:4], "little")
        self.pos = 4

    def next(self, cdf_row):
        r = _row(cdf_row)
        slot = self.x & (_M - 1)
        s = 0
        while r[s + 1] <= slot:
            s += 1
        self.x = (r[s + 1] - r[s]) * (self.x >> _PROB_BITS) + slot - r[s]
        while self.x < _L:
            if self.pos >= len(self.data):
                raise ValueError("truncated stream")
            self.x = (self.x << 8) | self.data[self.pos]
            self.pos += 1
        return s

    def finish(self):
        if self.x != _L or self.pos != len(self.data):
            raise ValueError("stream not fully consumed")
