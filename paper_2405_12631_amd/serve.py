"""Continuous-batching decode server for still images and video GOPs.

Requests arrive over time (Poisson), wait in a FIFO queue and are admitted as
soon as their HBM footprint fits the budget.  Every admitted request owns
device-resident buffers for its plane groups (symbols, ConvLSTM state,
scratch, reconstruction).  Each iteration advances every active request by one
coding step: one wv_context_params_items call runs all of their layers as a
handful of persistent launches whatever their positions and sizes, writing the
parameters of all requests into one shared buffer, so that one wv_cdf_tables
launch builds every row's table; then the step's symbols are scattered, and
requests that finished their last step are synthesised (GOPs: inverse
temporal Haar afterwards) and retired.  New requests join at step (0, 0) while
others are mid-decode.

Symbols come from one of two places:
* coder elided (default): each request refers to a prepared input whose
  per-step symbols are already on the device (they stand in for the host
  coder's output), so the server measures the GPU decode path under load;
* host coder (coder=True): the iteration's tables are trimmed on the device
  (wv_cdf_trim), copied to the host in two transfers, the rANS streams of every
  request are decoded by a thread pool, and the symbols go back in one
  transfer.  The active requests then form two cohorts that alternate: while
  the GPU computes one cohort's step, the host copies and decodes the other's
  tables, so GPU, PCIe and coder work overlap.  The run reports the PCIe bytes
  moved and the coder threads' busy time.
"""
import ctypes
import time
from collections import deque
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import torch

from . import _lib as L
from . import codec

_byref = ctypes.byref


class Prepared:
    """An encoded input: plane groups with their per-step symbols on the device and, with
    coder=True, the rANS streams of each plane (streams[n][subband][step])."""

    def __init__(self, model, kind, data, gop_levels=3, coder=False):
        self.kind = kind
        self.groups = []          # (H, W, nplanes, q_known, syms[i][g], streams | None)
        if kind == "image":
            x = torch.from_numpy(np.ascontiguousarray(data)).to(model.device)
            N, H, W = x.shape
            self.pixels = H * W
            self._add(model, x, H, W, N, coder)
        else:
            luma, chroma = data            # [T][H][W], [T][2][H/2][W/2] uint8
            T, H, W = luma.shape
            self.T, self.gop_levels = T, gop_levels
            self.pixels = T * H * W        # luma pixels x frames
            for planes in (luma, chroma.reshape(T, 2, H // 2, W // 2)):
                f = codec.center_u8(torch.from_numpy(np.ascontiguousarray(planes)).to(model.device))
                codec.temporal_haar(f)                      # temporal subbands, first axis
                f = f.reshape(-1, f.shape[-2], f.shape[-1]).contiguous()
                self._add(model, f, f.shape[1], f.shape[2], f.shape[0], coder)
        torch.cuda.synchronize()

    def _add(self, model, x, H, W, N, coder):
        ws = codec.Workspace(model, N, H, W)
        q, _, _ = codec.analyze(model, x, ws)
        syms = codec.prepare_elided(model, q, ws)
        streams = None
        if coder:
            data, q_enc = codec.encode(model, x, ws=codec.Workspace(model, N, H, W))
            assert torch.equal(q_enc, q)
            streams = codec.unpack_stream(model, data)[3]
        self.groups.append((H, W, N, q, syms, streams))


def _shared_row_bytes(model, coder):
    """Device bytes per row of the server's shared step buffers: 3K float parameters and
    one CDF row (int16 [nsym + 1]); with the host coder also the trimmed copy ((lo, len)
    and at most nsym - 1 values), a symbol byte and the trim's block sums."""
    b = 4 * 3 * model.cfg["mix_k"] + 2 * (model.nsym + 1)
    if coder:
        b += 2 + 2 * (model.nsym - 1) + 1 + 1
    return b


def footprint(model, prep, coder=False):
    """Device bytes a request holds while active: its workspaces (state and scratch), its
    symbols (int16) and reconstruction (float), and its share of the server's step buffers
    (the rows of its largest coding step)."""
    total = 0
    for H, W, N, _, _, _ in prep.groups:
        total += sum(codec.Workspace.sizes(model, N, H, W, coder=False, step_buffers=False).values())
        total += N * H * W * (2 + 4)
        total += codec.Workspace.max_step_rows(model, N, H, W) * _shared_row_bytes(model, coder)
    return total


class Slot:
    def __init__(self, model, req, prep):
        self.req, self.prep = req, prep
        self.i, self.g = 0, 0
        self.ws, self.q, self.xhat = [], [], []
        for H, W, N, _, _, _ in prep.groups:
            ws = codec.Workspace(model, N, H, W, coder=False, step_buffers=False)
            self.ws.append(ws)
            self.q.append(torch.zeros((N, H * W), dtype=torch.int16, device=model.device))
            self.xhat.append(torch.empty((N, H, W), dtype=torch.float32, device=model.device))
        self.nsub = len(self.ws[0].lay)
        self.done_event = None

    def rows(self):
        """Rows of this slot's current step, per group."""
        out = []
        for ws in self.ws:
            s = ws.lay[self.i]
            out.append(ws.N * codec.Model.group_count(s["h"], s["w"], self.g))
        return out

    def advance(self):
        self.g += 1
        if self.g == 4:
            self.i, self.g = self.i + 1, 0
        return self.i == self.nsub

    def finish(self, model):
        offset = 128.0 if self.prep.kind == "image" else 0.0
        for b, ws in enumerate(self.ws):
            codec.synthesize(model, ws, q=self.q[b], xhat=self.xhat[b], offset=offset)
        if self.prep.kind == "gop":
            T = self.prep.T
            for b, x in enumerate(self.xhat):
                v = x.view(T, -1)
                codec.temporal_haar(v, inverse=True)
                codec.add_offset(v, 128.0)
        self.done_event = torch.cuda.Event()
        self.done_event.record(torch.cuda.current_stream())

    def release(self, keep_output):
        """Return the request's device memory once its work has completed."""
        self.ws, self.q = [], []
        if not keep_output:
            self.xhat = []


class _StepBuffers:
    """The step buffers shared by the requests of one iteration (one per cohort with the host
    coder), grown between iterations when needed: parameters, CDF rows and, with the coder,
    the trimmed tables, symbols and their pinned host copies."""

    def __init__(self, model, coder):
        self.model, self.coder, self.cap = model, coder, 0

    def grow(self, rows):
        if rows <= self.cap:
            return
        m, dev = self.model, self.model.device
        cap = max(rows, 2 * self.cap)
        self.params = torch.empty(cap * 3 * m.cfg["mix_k"], dtype=torch.float32, device=dev)
        self.cdf = torch.empty(cap * (m.nsym + 1), dtype=torch.int16, device=dev)
        if self.coder:
            tb = ctypes.c_size_t()
            L.call("wv_cdf_trim_scratch_bytes", cap, _byref(tb))
            self.lolen = torch.empty(2 * cap, dtype=torch.uint8, device=dev)
            self.packed = torch.empty(cap * (m.nsym - 1), dtype=torch.int16, device=dev)
            self.trim_scratch = torch.empty(max(tb.value, 8), dtype=torch.uint8, device=dev)
            self.sym = torch.empty(cap, dtype=torch.uint8, device=dev)
            self.sym_h = torch.empty(cap, dtype=torch.uint8, pin_memory=True)
            self.lolen_h = torch.empty(2 * cap, dtype=torch.uint8, pin_memory=True)
            self.packed_h = torch.empty(cap * (m.nsym - 1), dtype=torch.int16, pin_memory=True)
        self.cap = cap


class Server:
    """FIFO admission by footprint, continuous batching, one coding step per iteration (with the
    host coder: per cohort, the two cohorts alternating)."""

    def __init__(self, model, budget_bytes, staging_bytes=16 << 20, on_params=None, coder=False,
                 coder_threads=16):
        self.model = model
        self.budget = budget_bytes
        self.on_params = on_params      # optional hook(slot, group, subband, step, params) for checks
        self.coder = coder
        self.staging = [torch.empty(staging_bytes, dtype=torch.uint8, pin_memory=True) for _ in range(2)]
        self.desc = [torch.empty(staging_bytes, dtype=torch.uint8, device=model.device) for _ in range(2)]
        self.staging_ev = [None, None]
        self.bufs = [_StepBuffers(model, coder) for _ in range(2 if coder else 1)]
        self.pool = ThreadPoolExecutor(max_workers=coder_threads) if coder else None
        self.copy_stream = torch.cuda.Stream() if coder else None   # table copies to the host
        self.coder_threads = coder_threads
        self.d2h = self.h2d = 0
        self.coder_busy = 0.0

    def _launch(self, slots, k, kb):
        """Context parameters and CDF tables of one coding step of `slots` (GPU, asynchronous),
        with staging buffer k and step buffers kb; with the coder also the device trim.
        Returns the per-slot row offsets and counts."""
        m = self.model
        K = m.cfg["mix_k"]
        bf = self.bufs[kb]
        rows = [s.rows() for s in slots]
        total = sum(sum(r) for r in rows)
        bf.grow(max(total, 1))
        items, first = [], []
        at = 0
        for s, rs in zip(slots, rows):
            fs = []
            for b, ws in enumerate(s.ws):
                items.append(L.wv_step_item(ws.H, ws.W, ws.N, s.q[b].data_ptr(), ws.state.data_ptr(),
                                            ws.scratch.data_ptr(), s.i, s.g,
                                            bf.params.data_ptr() + 4 * at * 3 * K))
                fs.append(at)
                at += rs[b]
            first.append(fs)
        arr = (L.wv_step_item * len(items))(*items)
        if self.staging_ev[k] is not None:
            self.staging_ev[k].synchronize()        # staging k is free once its copy ran
        used = ctypes.c_size_t()
        L.call("wv_context_params_items", m.h, len(items), arr,
               ctypes.c_void_p(self.staging[k].data_ptr()), self.staging[k].numel(),
               ctypes.c_void_p(self.desc[k].data_ptr()), self.desc[k].numel(), _byref(used),
               codec._stream())
        ev = torch.cuda.Event()
        ev.record(torch.cuda.current_stream())
        self.staging_ev[k] = ev
        if self.on_params is not None:
            for s, fs, rs in zip(slots, first, rows):
                for b, ws in enumerate(s.ws):
                    prm = bf.params[fs[b] * 3 * K:(fs[b] + rs[b]) * 3 * K]
                    self.on_params(s, b, s.i, s.g, prm.view(ws.N, rs[b] // ws.N, 3 * K))
        if total:
            codec.cdf_tables(m, bf.params[:total * 3 * K], out=bf.cdf)
        tables = None
        if self.coder and total:
            cdf = bf.cdf[:total * (m.nsym + 1)].view(total, m.nsym + 1)
            L.call("wv_cdf_trim", codec._ptr(cdf), total, m.nsym, codec._ptr(bf.lolen), codec._ptr(bf.packed),
                   bf.packed.numel(), codec._ptr(bf.trim_scratch), bf.trim_scratch.numel(), codec._stream())
            tables = torch.cuda.Event()
            tables.record(torch.cuda.current_stream())
        return dict(slots=slots, first=first, rows=rows, total=total, kb=kb, tables=tables)

    def _complete(self, st):
        """Symbols of a launched step (from the prepared input, or decoded by the host coder
        from its trimmed tables), scattered into each slot's q; advances the slots and returns
        those that finished their last step."""
        m = self.model
        slots, first, rows, total, bf = st["slots"], st["first"], st["rows"], st["total"], self.bufs[st["kb"]]
        if self.coder and total:
            self._decode_symbols(st, bf)
        for s, fs, rs in zip(slots, first, rows):
            for b, ws in enumerate(s.ws):
                if not rs[b]:
                    continue
                sym = bf.sym[fs[b]:fs[b] + rs[b]] if self.coder else s.prep.groups[b][4][s.i][s.g]
                codec.scatter_symbols(m, sym, s.q[b], ws, s.i, s.g)
        return [s for s in slots if s.advance()]

    def step(self, slots, k):
        """One iteration over the active slots using staging buffer k (coder elided)."""
        return self._complete(self._launch(slots, k, 0))

    def _decode_symbols(self, st, bf):
        """Host coder for one launched step: copy the trimmed tables to the host on the copy
        stream once the trim has run (the compute stream meanwhile runs the other cohort),
        decode each request's streams on the thread pool, copy the symbols back on the
        compute stream ahead of the scatter."""
        m = self.model
        slots, first, rows, total = st["slots"], st["first"], st["rows"], st["total"]
        cs = self.copy_stream
        cs.wait_event(st["tables"])
        with torch.cuda.stream(cs):
            bf.lolen_h[:2 * total].copy_(bf.lolen[:2 * total], non_blocking=True)
        cs.synchronize()
        lolen = bf.lolen_h[:2 * total].numpy()
        npk = int(lolen[1::2].astype(np.int64).sum())
        with torch.cuda.stream(cs):
            bf.packed_h[:npk].copy_(bf.packed[:npk], non_blocking=True)
        cs.synchronize()
        packed = bf.packed_h[:npk].numpy().view(np.uint16)
        self.d2h += lolen.nbytes + packed.nbytes
        tr = codec.Trimmed(lolen, packed, m.nsym)
        out = bf.sym_h.numpy()

        def work(a, b, data):
            t0 = time.perf_counter()
            out[a:b] = codec.rans_decode_trim(tr, a, b, data)
            return time.perf_counter() - t0

        futs = []
        for s, fs, rs in zip(slots, first, rows):
            for b, ws in enumerate(s.ws):
                if not rs[b]:
                    continue
                streams = s.prep.groups[b][5]
                per = rs[b] // ws.N
                for n in range(ws.N):
                    a = fs[b] + n * per
                    futs.append(self.pool.submit(work, a, a + per, streams[n][s.i][s.g]))
        self.coder_busy += sum(f.result() for f in futs)
        bf.sym[:total].copy_(bf.sym_h[:total], non_blocking=True)
        self.h2d += total

    def run(self, requests, preps, admit_until=None, max_seconds=120.0, log=None, keep_outputs=False,
            tick=None):
        """requests: list of (arrival_s, prep_id) sorted by time.  Returns (stats, slots);
        finished slots keep their reconstruction only if keep_outputs.  With tick set, time
        is virtual: it advances by `tick` per iteration (and jumps to the next arrival when
        nothing is active), so admissions do not depend on the host's speed (tests)."""
        m = self.model
        pending = deque(requests)
        queue, active, finishing, done = deque(), [], [], []
        used = 0
        t0 = time.perf_counter()
        k = 0
        iters = 0
        rejected = 0
        peak_active = 0
        mid_joins = 0      # admissions while another request was past its first step
        self.d2h = self.h2d = 0
        self.coder_busy = 0.0
        fp = {pid: footprint(m, p, self.coder) for pid, p in preps.items()}
        vclock = 0.0
        inflight = [None, None]   # host coder: the launched, not yet decoded step of each cohort
        turn = 0                  # host coder: the cohort launched in this iteration
        while True:
            now = vclock if tick is not None else time.perf_counter() - t0
            while pending and pending[0][0] <= now and (admit_until is None or pending[0][0] <= admit_until):
                queue.append(pending.popleft())
            if admit_until is not None and now > admit_until:
                pending.clear()
            while queue and fp[queue[0][1]] > self.budget:       # can never fit: refuse
                queue.popleft()
                rejected += 1
            while queue and used + fp[queue[0][1]] <= self.budget:
                t_arr, pid = queue.popleft()
                slot = Slot(m, dict(arrival=t_arr, prep=pid, admitted=now), preps[pid])
                slot.cohort = turn
                mid_joins += any((a.i, a.g) != (0, 0) for a in active)
                used += fp[pid]
                active.append(slot)
            peak_active = max(peak_active, len(active))
            fin = []
            if self.coder:
                # Launch this cohort's step, then decode the other cohort's tables (launched in
                # the previous iteration) while the GPU computes.
                mine = [s_ for s_ in active if s_.cohort == turn]
                if mine:
                    inflight[turn] = self._launch(mine, turn, turn)
                if inflight[1 - turn] is not None:
                    fin = self._complete(inflight[1 - turn])
                    inflight[1 - turn] = None
                if mine or fin:
                    iters += 1
                turn ^= 1
            elif active:
                fin = self.step(active, k)
                k ^= 1
                iters += 1
            for s in fin:
                s.finish(m)
                active.remove(s)
                finishing.append(s)
            for s in list(finishing):
                if tick is not None:
                    s.done_event.synchronize()
                if s.done_event.query():
                    s.req["finished"] = vclock if tick is not None else time.perf_counter() - t0
                    finishing.remove(s)
                    used -= fp[s.req["prep"]]
                    s.release(keep_outputs)
                    done.append(s)
            if not (pending or queue or active or finishing):
                break
            if now > max_seconds:
                break
            if tick is not None:   # monotone: one tick per loop, or a jump to the next arrival
                vclock += tick
                if not active and not finishing and pending:
                    vclock = max(vclock, pending[0][0])
            elif not active and not finishing and queue == deque() and pending:
                time.sleep(max(0.0, min(pending[0][0] - now, 0.01)))
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        lat = np.array([s.req["finished"] - s.req["arrival"] for s in done]) if done else np.zeros(0)
        px = sum(s.prep.pixels for s in done)
        stats = dict(completed=len(done), rejected=rejected, left_queued=len(queue) + len(pending),
                     left_active=len(active), peak_active=peak_active, mid_decode_joins=mid_joins,
                     iterations=iters, wall_s=round(wall, 3), mpx_per_s=round(px / wall / 1e6, 3),
                     p50_ms=round(float(np.percentile(lat, 50)) * 1e3, 2) if len(lat) else None,
                     p99_ms=round(float(np.percentile(lat, 99)) * 1e3, 2) if len(lat) else None)
        if self.coder:
            stats.update(coder_threads=self.coder_threads,
                         coder_utilisation=round(self.coder_busy / (self.coder_threads * wall), 4),
                         pcie_d2h_gb_per_s=round(self.d2h / wall / 1e9, 3),
                         pcie_h2d_gb_per_s=round(self.h2d / wall / 1e9, 4),
                         table_bytes_to_host=self.d2h)
        if log:
            log(f"served {stats}")
        return stats, done
