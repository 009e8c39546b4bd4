"""Python runtime over libwv.so: model upload, workspaces, the encode and
decode drivers, and the bitstream container.

Every arithmetic step of the path runs in the HIP library (or, for the
entropy coder, in its host C++ code); this module only allocates torch
buffers, sequences the calls and moves bytes.  There is no fallback: if the
library is missing the first call raises.
"""
import ctypes
import hashlib
import struct
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import torch

from . import _lib as L

_byref = ctypes.byref


def make_config(cfg):
    """wv_config from a workload dict (wvgen.configs layout)."""
    return L.wv_config(levels=cfg["levels"], lift_ch=cfg["lift_ch"], lift_layers=cfg["lift_layers"],
                       ctx_ch=cfg["ctx_ch"], ctx_layers=cfg["ctx_layers"], mix_k=cfg["mix_k"],
                       sym_min=cfg["sym_min"], sym_max=cfg["sym_max"], cdf_bits=cfg["cdf_bits"],
                       sigma_min=cfg["sigma_min"], lift_int=int(cfg.get("lift_int", 0)),
                       dist=L.DISTS[cfg.get("dist", "gauss")],
                       ctx_arch=1 if cfg.get("ctx_arch", "plain") == "blocks" else 0,
                       ll_ar=int(cfg.get("ll_ar", 0)), ar_ch=int(cfg.get("ar_ch", 32)))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def zero(t):
    """Zero a device tensor with the library's fill kernel (safe inside a captured graph)."""
    L.call("wv_zero", _ptr(t), t.numel() * t.element_size(), _stream())
    return t


class Graph:
    """Library calls captured once (wv_graph_begin / wv_graph_end) and replayed.

    `fn` is run once on a side stream while the library records the work its
    calls enqueue; it must only call device entry points on preallocated buffers.
    replay() relaunches the recorded kernels on the current stream."""

    def __init__(self, fn):
        self.h = None
        cur = torch.cuda.current_stream()
        side = torch.cuda.Stream()
        side.wait_stream(cur)
        with torch.cuda.stream(side):
            s = _stream()
            L.call("wv_graph_begin", s)
            h = ctypes.c_void_p()
            try:
                fn()
            finally:
                rc = L.lib().wv_graph_end(s, _byref(h))
            L.check(rc)
        cur.wait_stream(side)
        self.h = h

    def replay(self):
        L.call("wv_graph_launch", self.h, _stream())

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            try:
                L.lib().wv_graph_destroy(h)
            except Exception:
                pass


class Model:
    """A model handle: weights uploaded and repacked on the current device."""

    def __init__(self, cfg, blob, precision=L.WV_FP32, device="cuda"):
        self.cfg = dict(cfg)
        self.c = make_config(cfg)
        self.precision = precision
        blob = np.ascontiguousarray(blob, np.float32)
        n = ctypes.c_longlong()
        L.call("wv_weights_count", _byref(self.c), _byref(n))
        if n.value != blob.size:
            raise ValueError(f"blob has {blob.size} floats, config needs {n.value}")
        self.blob_sha = hashlib.sha256(blob.tobytes()).digest()
        self.d_blob = torch.from_numpy(blob).to(device)
        nb = ctypes.c_size_t()
        L.call("wv_pack_bytes", _byref(self.c), precision, _byref(nb))
        self.d_pack = torch.empty(nb.value, dtype=torch.uint8, device=device)
        h = ctypes.c_void_p()
        L.call("wv_model_create", _byref(self.c), _ptr(self.d_blob), n.value, precision,
               _ptr(self.d_pack), nb.value, _stream(), _byref(h))
        self.h = h
        self.device = device
        self.nsym = cfg["sym_max"] - cfg["sym_min"] + 1

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            try:
                L.lib().wv_model_destroy(h)
            except Exception:
                pass
            self.h = None

    def layout(self, H, W):
        n = 3 * self.cfg["levels"] + 1
        arr = (L.wv_subband * n)()
        coefs = ctypes.c_longlong()
        L.call("wv_layout", _byref(self.c), H, W, arr, n, _byref(coefs))
        return [dict(h=s.h, w=s.w, level=s.level, type=s.type, offset=s.offset) for s in arr]

    @staticmethod
    def group_count(h, w, g):
        return int(L.lib().wv_group_count(h, w, g))

    def deltas(self):
        d = 1.0 / float(self.cfg["step"])
        return d, d


class Workspace:
    """Device state and scratch for nplanes planes of H x W.  With coder=False the
    buffers of the host-coder path (symbol staging and the trimmed table copies) are
    left out, as in the coder-elided server."""

    def __init__(self, model, N, H, W, coder=True, step_buffers=True):
        self.N, self.H, self.W = N, H, W
        self.lay = model.layout(H, W)
        sizes = Workspace.sizes(model, N, H, W, coder, step_buffers)
        dev = model.device
        self.state = torch.empty(sizes["state"] // 4, dtype=torch.float32, device=dev)
        self.scratch = torch.empty(sizes["scratch"] // 4, dtype=torch.float32, device=dev)
        if step_buffers:
            self.params = torch.empty(sizes["params"] // 4, dtype=torch.float32, device=dev)
            self.cdf = torch.empty(sizes["cdf"] // 2, dtype=torch.int16, device=dev)
        if coder:
            self.sym = torch.empty(sizes["sym"], dtype=torch.uint8, device=dev)
            # trimmed copy of the CDF rows for the host coder (wv_cdf_trim)
            self.lolen = torch.empty(sizes["lolen"], dtype=torch.uint8, device=dev)
            self.packed = torch.empty(sizes["packed"] // 2, dtype=torch.int16, device=dev)
            self.trim_scratch = torch.empty(sizes["trim_scratch"], dtype=torch.uint8, device=dev)

    @staticmethod
    def max_step_rows(model, N, H, W):
        """Rows (coefficients) of the largest coding step of N planes of H x W."""
        return N * max(Model.group_count(s["h"], s["w"], 0) for s in model.layout(H, W))

    @staticmethod
    def sizes(model, N, H, W, coder=True, step_buffers=True):
        """Bytes of every device buffer a Workspace allocates (name -> bytes)."""
        sb, xb = ctypes.c_size_t(), ctypes.c_size_t()
        L.call("wv_workspace_bytes", model.h, N, H, W, _byref(sb), _byref(xb))
        maxg = Workspace.max_step_rows(model, 1, H, W)
        out = dict(state=sb.value // 4 * 4, scratch=xb.value // 4 * 4)
        if step_buffers:
            out.update(params=4 * N * maxg * 3 * model.cfg["mix_k"], cdf=2 * N * maxg * (model.nsym + 1))
        if coder:
            tb = ctypes.c_size_t()
            L.call("wv_cdf_trim_scratch_bytes", N * maxg, _byref(tb))
            out.update(sym=N * maxg, lolen=2 * N * maxg, packed=2 * N * maxg * (model.nsym - 1),
                       trim_scratch=max(tb.value, 8))
        return out


# ---------------------------------------------------------------------------
# single calls
# ---------------------------------------------------------------------------
def analyze(model, x, ws, want_y=False):
    """x: uint8 [N,H,W] or centred float [N,H,W] device tensor -> (q int16 [N,HW], y|None, clips)."""
    N, H, W = x.shape
    q = torch.empty((N, H * W), dtype=torch.int16, device=x.device)
    y = torch.empty((N, H * W), dtype=torch.float32, device=x.device) if want_y else None
    clip = torch.zeros(1, dtype=torch.int32, device=x.device)
    dL, dH = model.deltas()
    x8 = x if x.dtype == torch.uint8 else None
    xf = x if x.dtype == torch.float32 else None
    L.call("wv_analyze", model.h, _ptr(x8), _ptr(xf), N, H, W, dL, dH, _ptr(ws.scratch), _ptr(q),
           _ptr(y), _ptr(clip), _stream())
    return q, y, clip


def context_params(model, q, ws, i, g, out=None):
    """Parameters [N, n_g, 3K] of step g of subband i (q: int16 [N, HW] device)."""
    s = ws.lay[i]
    ng = Model.group_count(s["h"], s["w"], g)
    K = model.cfg["mix_k"]
    if out is None:
        out = ws.params[:ws.N * ng * 3 * K]
    L.call("wv_context_params", model.h, _ptr(q), ws.N, ws.H, ws.W, i, g, _ptr(ws.state),
           _ptr(ws.scratch), _ptr(out), _stream())
    return out.view(ws.N, ng, 3 * K)


def cdf_tables(model, params, out=None):
    """uint16 CDF rows (held in an int16 tensor) [n, nsym+1] for params [.., 3K]."""
    K = model.cfg["mix_k"]
    n = params.numel() // (3 * K)
    if out is None:
        out = torch.empty(n * (model.nsym + 1), dtype=torch.int16, device=params.device)
    L.call("wv_cdf_tables", _ptr(params), n, K, model.c.dist, model.cfg["sym_min"],
           model.cfg["sym_max"], model.cfg["cdf_bits"], _ptr(out), _stream())
    return out[:n * (model.nsym + 1)].view(n, model.nsym + 1)


class Trimmed:
    """Host copy of trimmed CDF rows: lolen uint8 [n, 2], packed uint16 [sum len] and the
    row offsets into packed."""

    def __init__(self, lolen, packed, nsym):
        self.lolen = np.ascontiguousarray(lolen, np.uint8).reshape(-1, 2)
        self.packed = np.ascontiguousarray(packed, np.uint16)
        self.nsym = nsym
        self.off = np.zeros(len(self.lolen) + 1, np.int64)
        np.cumsum(self.lolen[:, 1], out=self.off[1:])

    def rows(self, a, b):
        """Rows a..b-1 as (lolen, packed) slices."""
        return self.lolen[a:b], self.packed[self.off[a]:self.off[b]]

    def full(self):
        n = len(self.lolen)
        out = np.empty((n, self.nsym + 1), np.uint16)
        L.call("wv_cdf_untrim", self.lolen.ctypes.data, self.packed.ctypes.data, self.packed.size, self.nsym, n,
               out.ctypes.data)
        return out


def cdf_trim_to_host(model, cdf, ws):
    """Trim device CDF rows [n, nsym+1] and copy them to the host: 2 n + 2 sum(len) bytes."""
    n = cdf.shape[0]
    L.call("wv_cdf_trim", _ptr(cdf), n, model.nsym, _ptr(ws.lolen), _ptr(ws.packed), ws.packed.numel(),
           _ptr(ws.trim_scratch), ws.trim_scratch.numel(), _stream())
    lolen = ws.lolen[:2 * n].cpu().numpy()
    total = int(lolen[1::2].astype(np.int64).sum())
    packed = ws.packed[:total].cpu().numpy().view(np.uint16)
    return Trimmed(lolen, packed, model.nsym)


def scatter_symbols(model, sym, q, ws, i, g):
    L.call("wv_scatter_symbols", _byref(model.c), _ptr(sym), ws.N, ws.H, ws.W, i, g, _ptr(q),
           _stream())


def gather_symbols(model, q, ws, i, g, out=None):
    s = ws.lay[i]
    ng = Model.group_count(s["h"], s["w"], g)
    if out is None:
        out = torch.empty(ws.N * ng, dtype=torch.uint8, device=q.device)
    L.call("wv_gather_symbols", _byref(model.c), _ptr(q), ws.N, ws.H, ws.W, i, g, _ptr(out),
           _stream())
    return out[:ws.N * ng].view(ws.N, ng)


def synthesize(model, ws, q=None, y=None, xhat=None, want_u8=False, offset=128.0):
    """q int16 [N,HW] (or float packed y) -> (xhat float [N,H,W], u8|None)."""
    N, H, W = ws.N, ws.H, ws.W
    dev = (q if q is not None else y).device
    if xhat is None:
        xhat = torch.empty((N, H, W), dtype=torch.float32, device=dev)
    u8 = torch.empty((N, H, W), dtype=torch.uint8, device=dev) if want_u8 else None
    dL, dH = model.deltas()
    L.call("wv_synthesize", model.h, _ptr(q), _ptr(y), N, H, W, dL, dH, offset, _ptr(ws.scratch),
           _ptr(xhat), _ptr(u8), _stream())
    return xhat, u8


def center_u8(x8, out=None):
    """uint8 device tensor -> float x - 128 (library kernel)."""
    if out is None:
        out = torch.empty(x8.shape, dtype=torch.float32, device=x8.device)
    L.call("wv_center_u8", _ptr(x8), x8.numel(), _ptr(out), _stream())
    return out


def add_offset(x, offset, want_u8=False):
    u8 = torch.empty(x.shape, dtype=torch.uint8, device=x.device) if want_u8 else None
    L.call("wv_add_offset", _ptr(x), x.numel(), offset, _ptr(u8), _stream())
    return x, u8


def impulse_responses(model, q_plane, H, W):
    """Subband impulse responses (Sec. 3.4) of one plane's packed symbols q_plane [H*W]
    -> float [3J+1, S, S] with S = 2^levels."""
    nb = ctypes.c_size_t()
    L.call("wv_impulse_scratch_bytes", model.h, _byref(nb))
    scratch = torch.empty(nb.value // 4 + 64, dtype=torch.float32, device=q_plane.device)
    S = 1 << model.cfg["levels"]
    out = torch.empty((3 * model.cfg["levels"] + 1, S, S), dtype=torch.float32, device=q_plane.device)
    dL, dH = model.deltas()
    L.call("wv_impulse_responses", model.h, _ptr(q_plane), H, W, dL, dH, _ptr(scratch), _ptr(out),
           _stream())
    return out


def temporal_haar(frames, inverse=False):
    """In-place temporal Haar lifting of a float device tensor [T, ...]."""
    T = frames.shape[0]
    n = frames.numel() // T
    L.call("wv_temporal_haar_inverse" if inverse else "wv_temporal_haar_forward", _ptr(frames), T,
           n, _stream())
    return frames


def ar_params(model, q, ws, out=None):
    """Autoregressive LL model, encoder side: [N, h_J * w_J, 3K] in raster order."""
    s = ws.lay[0]
    n0 = s["h"] * s["w"]
    K = model.cfg["mix_k"]
    if out is None:
        out = ws.params[:ws.N * n0 * 3 * K]
    L.call("wv_ar_params", model.h, _ptr(q), ws.N, ws.H, ws.W, _ptr(out), _stream())
    return out.view(ws.N, n0, 3 * K)


def ar_decode(model, q, ws, ll_streams):
    """Decode LL of every plane on the GPU from its raster-order streams (list of bytes)."""
    offs = np.zeros(ws.N + 1, np.int64)
    offs[1:] = np.cumsum([len(b) for b in ll_streams])
    blob = np.frombuffer(b"".join(ll_streams) + b"\0", np.uint8)
    d_bytes = torch.from_numpy(blob.copy()).to(q.device)
    d_offs = torch.from_numpy(offs).to(q.device)
    status = torch.zeros(ws.N, dtype=torch.int32, device=q.device)
    L.call("wv_ar_decode", model.h, _ptr(d_bytes), _ptr(d_offs), ws.N, ws.H, ws.W, _ptr(q),
           _ptr(status), _stream())
    if int(status.sum().item()):
        raise L.WvError(L.WV_ECORRUPT, "corrupt LL stream")


def params_all(model, q, ws):
    """Teacher-forced parameters of every (subband, step): list [i][g] of [N, n_g, 3K] copies.
    With the autoregressive LL model, subband 0 has one raster-order entry."""
    out = []
    for i in range(len(ws.lay)):
        row = []
        for g in range(4):
            row.append(context_params(model, q, ws, i, g).clone())
        if i == 0 and model.cfg.get("ll_ar", 0):
            row = [ar_params(model, q, ws).clone()]
        out.append(row)
    return out


# ---------------------------------------------------------------------------
# host coder
# ---------------------------------------------------------------------------
def rans_encode(cdf_u16, sym_u8, nsym):
    """cdf_u16: numpy uint16 [n, nsym+1]; sym_u8: numpy uint8 [n] -> bytes."""
    cdf_u16 = np.ascontiguousarray(cdf_u16, np.uint16)
    sym_u8 = np.ascontiguousarray(sym_u8, np.uint8)
    n = sym_u8.size
    cap = 16 + 4 * n
    buf = np.empty(cap, np.uint8)
    ln = ctypes.c_size_t()
    L.call("wv_rans_encode", cdf_u16.ctypes.data, nsym, sym_u8.ctypes.data, n, buf.ctypes.data, cap,
           _byref(ln))
    return buf[:ln.value].tobytes()


def rans_encode_trim(tr, a, b, sym_u8):
    """Encode rows a..b-1 of a Trimmed table set."""
    lolen, packed = tr.rows(a, b)
    sym_u8 = np.ascontiguousarray(sym_u8, np.uint8)
    n = sym_u8.size
    cap = 16 + 4 * n
    buf = np.empty(cap, np.uint8)
    ln = ctypes.c_size_t()
    pk = packed if packed.size else np.zeros(1, np.uint16)
    L.call("wv_rans_encode_trim", lolen.ctypes.data, pk.ctypes.data, packed.size, tr.nsym, sym_u8.ctypes.data, n,
           buf.ctypes.data, cap, _byref(ln))
    return buf[:ln.value].tobytes()


def rans_decode_trim(tr, a, b, data):
    lolen, packed = tr.rows(a, b)
    n = b - a
    out = np.empty(n, np.uint8)
    src = np.frombuffer(data, np.uint8) if len(data) else np.zeros(1, np.uint8)
    pk = packed if packed.size else np.zeros(1, np.uint16)
    L.call("wv_rans_decode_trim", lolen.ctypes.data, pk.ctypes.data, packed.size, tr.nsym, n, src.ctypes.data,
           len(data), out.ctypes.data)
    return out


def rans_decode(cdf_u16, data, n, nsym):
    cdf_u16 = np.ascontiguousarray(cdf_u16, np.uint16)
    out = np.empty(n, np.uint8)
    src = np.frombuffer(data, np.uint8) if len(data) else np.zeros(1, np.uint8)
    L.call("wv_rans_decode", cdf_u16.ctypes.data, nsym, n, src.ctypes.data, len(data),
           out.ctypes.data)
    return out


# ---------------------------------------------------------------------------
# bitstream container
# ---------------------------------------------------------------------------
_MAGIC = b"WV01"
_HDR = struct.Struct("<4sHHIIBBHff16sI")


def pack_stream(model, N, H, W, streams):
    """streams: list over planes of list over subbands of 4 byte strings."""
    flat = [s for plane in streams for sub in plane for s in sub]
    dL, dH = model.deltas()
    hdr = _HDR.pack(_MAGIC, 1, N, H, W, model.cfg["levels"], model.precision, 0, dL, dH,
                    model.blob_sha[:16], len(flat))
    return hdr + struct.pack(f"<{len(flat)}I", *[len(s) for s in flat]) + b"".join(flat)


def unpack_stream(model, data):
    """-> (N, H, W, streams[plane][subband][step]); raises WvError(WV_ECORRUPT) on a bad container."""
    def bad(msg):
        return L.WvError(L.WV_ECORRUPT, msg)
    if len(data) < _HDR.size:
        raise bad("truncated header")
    magic, ver, N, H, W, J, prec, _, dL, dH, sha, ns = _HDR.unpack_from(data, 0)
    if magic != _MAGIC or ver != 1:
        raise bad("not a wv bitstream")
    if sha != model.blob_sha[:16] or J != model.cfg["levels"] or prec != model.precision:
        raise bad("bitstream was written by another model")
    nsub = 3 * J + 1
    if ns != N * nsub * 4:
        raise bad("stream count does not match the header")
    off = _HDR.size + 4 * ns
    if len(data) < off:
        raise bad("truncated length table")
    lens = struct.unpack_from(f"<{ns}I", data, _HDR.size)
    if off + sum(lens) != len(data):
        raise bad("stream lengths do not match the payload")
    flat = []
    for ln in lens:
        flat.append(data[off:off + ln])
        off += ln
    streams = [[flat[(n * nsub + i) * 4:(n * nsub + i) * 4 + 4] for i in range(nsub)] for n in range(N)]
    return N, H, W, streams


# ---------------------------------------------------------------------------
# encode / decode drivers
# ---------------------------------------------------------------------------
_pool = ThreadPoolExecutor(max_workers=8)


def encode(model, planes, ws=None):
    """uint8 planes [N,H,W] (numpy or device tensor) -> (bitstream bytes, q device tensor)."""
    x = torch.as_tensor(planes).to(model.device)
    N, H, W = x.shape
    ws = ws or Workspace(model, N, H, W)
    q, _, _ = analyze(model, x, ws)
    streams = [[[None] * 4 for _ in ws.lay] for _ in range(N)]
    for i, s in enumerate(ws.lay):
        if i == 0 and model.cfg.get("ll_ar", 0):
            context_params(model, q, ws, 0, 0)          # advances the long context only
            cdf = cdf_tables(model, ar_params(model, q, ws), out=ws.cdf)
            n0 = s["h"] * s["w"]
            tr = cdf_trim_to_host(model, cdf, ws)
            sym_h = (q[:, :n0].cpu().numpy().astype(np.int32) - model.cfg["sym_min"]).astype(np.uint8)
            for n in range(N):
                streams[n][0] = [rans_encode_trim(tr, n * n0, (n + 1) * n0, sym_h[n]), b"", b"", b""]
            continue
        for g in range(4):
            prm = context_params(model, q, ws, i, g)
            cdf = cdf_tables(model, prm, out=ws.cdf)
            sym = gather_symbols(model, q, ws, i, g, out=ws.sym)
            tr = cdf_trim_to_host(model, cdf, ws)
            sym_h = sym.cpu().numpy()
            ng = sym_h.shape[1]
            futs = [_pool.submit(rans_encode_trim, tr, n * ng, (n + 1) * ng, sym_h[n]) for n in range(N)]
            for n, f in enumerate(futs):
                streams[n][i][g] = f.result()
    return pack_stream(model, N, H, W, streams), q


def decode(model, data, ws=None, want_u8=True):
    """bitstream -> (xhat float [N,H,W], u8 [N,H,W] | None, q int16 [N,HW]) on the device."""
    N, H, W, streams = unpack_stream(model, data)
    ws = ws or Workspace(model, N, H, W)
    q = torch.zeros((N, H * W), dtype=torch.int16, device=model.device)
    for i, s in enumerate(ws.lay):
        if i == 0 and model.cfg.get("ll_ar", 0):
            context_params(model, q, ws, 0, 0)          # advances the long context only
            ar_decode(model, q, ws, [streams[n][0][0] for n in range(N)])
            continue
        for g in range(4):
            prm = context_params(model, q, ws, i, g)
            cdf = cdf_tables(model, prm, out=ws.cdf)
            tr = cdf_trim_to_host(model, cdf, ws)
            ng = Model.group_count(s["h"], s["w"], g)
            futs = [_pool.submit(rans_decode_trim, tr, n * ng, (n + 1) * ng, streams[n][i][g]) for n in range(N)]
            sym_h = np.stack([f.result() for f in futs]) if N else np.zeros((0, ng), np.uint8)
            sym = ws.sym[:N * ng]
            sym.copy_(torch.from_numpy(sym_h.reshape(-1)))
            scatter_symbols(model, sym, q, ws, i, g)
    xhat, u8 = synthesize(model, ws, q=q, want_u8=want_u8)
    return xhat, u8, q


def prepare_elided(model, q_known, ws):
    """Per-step symbol indices of known q, gathered once before a timed coder-elided decode."""
    return [[gather_symbols(model, q_known, ws, i, g).clone() for g in range(4)]
            for i in range(len(ws.lay))]


def decode_elided(model, syms, ws, q, xhat=None):
    """The GPU part of decoding with the entropy coder elided: for every
    (subband, step) the context model, its CDF tables and the scatter of that
    step's symbols (taken from `syms` instead of the host coder), then
    synthesis.  All launches are asynchronous on the current stream."""
    for i in range(len(ws.lay)):
        for g in range(4):
            prm = context_params(model, q, ws, i, g)
            cdf_tables(model, prm, out=ws.cdf)
            scatter_symbols(model, syms[i][g], q, ws, i, g)
    return synthesize(model, ws, q=q, xhat=xhat)[0]
