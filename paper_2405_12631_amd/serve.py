"""Continuous-batching decode server for still images and video GOPs.

Requests arrive over time (Poisson), wait in a FIFO queue and are admitted as
soon as their HBM footprint fits the budget.  Every admitted request owns
device-resident buffers for its plane groups (symbols, ConvLSTM state,
scratch, parameters, CDF tables, reconstruction).  Each iteration advances
every active request by one coding step: one wv_context_params_items call
runs all of their layers as a handful of persistent launches whatever their
positions and sizes, then each request's CDF tables and symbol scatter run,
and requests that finished their last step are synthesised (GOPs: inverse
temporal Haar afterwards) and retired.  New requests join at step (0, 0)
while others are mid-decode.

The entropy coder is elided: each request refers to a prepared input whose
per-step symbols are already on the device (they stand in for the host
coder's output), so the server measures the GPU decode path under load.
"""
import ctypes
import time
from collections import deque

import numpy as np
import torch

from . import _lib as L
from . import codec

_byref = ctypes.byref


class Prepared:
    """An encoded input: plane groups with their per-step symbols on the device."""

    def __init__(self, model, kind, data, gop_levels=3):
        self.kind = kind
        self.groups = []          # (H, W, nplanes, q_known, syms[i][g])
        if kind == "image":
            x = torch.from_numpy(np.ascontiguousarray(data)).to(model.device)
            N, H, W = x.shape
            self.pixels = H * W
            self._add(model, x, H, W, N)
        else:
            luma, chroma = data            # [T][H][W], [T][2][H/2][W/2] uint8
            T, H, W = luma.shape
            self.T, self.gop_levels = T, gop_levels
            self.pixels = T * H * W        # luma pixels x frames
            for planes in (luma, chroma.reshape(T, 2, H // 2, W // 2)):
                f = codec.center_u8(torch.from_numpy(np.ascontiguousarray(planes)).to(model.device))
                codec.temporal_haar(f)                      # temporal subbands, first axis
                f = f.reshape(-1, f.shape[-2], f.shape[-1]).contiguous()
                self._add(model, f, f.shape[1], f.shape[2], f.shape[0])
        torch.cuda.synchronize()

    def _add(self, model, x, H, W, N):
        ws = codec.Workspace(model, N, H, W)
        q, _, _ = codec.analyze(model, x, ws)
        syms = codec.prepare_elided(model, q, ws)
        self.groups.append((H, W, N, q, syms))


def footprint(model, prep):
    """Device bytes a request holds while active: every buffer of its slot's
    workspaces (coder-elided form), its symbols (int16) and its reconstruction (float)."""
    total = 0
    for H, W, N, _, _ in prep.groups:
        total += sum(codec.Workspace.sizes(model, N, H, W, coder=False).values())
        total += N * H * W * (2 + 4)
    return total


class Slot:
    def __init__(self, model, req, prep):
        self.req, self.prep = req, prep
        self.i, self.g = 0, 0
        self.ws, self.q, self.xhat = [], [], []
        for H, W, N, _, _ in prep.groups:
            ws = codec.Workspace(model, N, H, W, coder=False)
            self.ws.append(ws)
            self.q.append(torch.zeros((N, H * W), dtype=torch.int16, device=model.device))
            self.xhat.append(torch.empty((N, H, W), dtype=torch.float32, device=model.device))
        self.nsub = len(self.ws[0].lay)
        self.done_event = None

    def items(self):
        out = []
        for b, ws in enumerate(self.ws):
            out.append(L.wv_step_item(ws.H, ws.W, ws.N, self.q[b].data_ptr(), ws.state.data_ptr(),
                                      ws.scratch.data_ptr(), self.i, self.g, ws.params.data_ptr()))
        return out

    def after_params(self, model):
        for b, ws in enumerate(self.ws):
            s = ws.lay[self.i]
            ng = codec.Model.group_count(s["h"], s["w"], self.g)
            prm = ws.params[:ws.N * ng * 3 * model.cfg["mix_k"]]
            codec.cdf_tables(model, prm, out=ws.cdf)
            codec.scatter_symbols(model, self.prep.groups[b][4][self.i][self.g], self.q[b], ws, self.i, self.g)
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


class Server:
    """FIFO admission by footprint, continuous batching, one coding step per iteration."""

    def __init__(self, model, budget_bytes, staging_bytes=16 << 20, on_params=None):
        self.model = model
        self.budget = budget_bytes
        self.on_params = on_params      # optional hook(slot, group, subband, step, params) for checks
        self.staging = [torch.empty(staging_bytes, dtype=torch.uint8, pin_memory=True) for _ in range(2)]
        self.desc = [torch.empty(staging_bytes, dtype=torch.uint8, device=model.device) for _ in range(2)]
        self.staging_ev = [None, None]

    def step(self, slots, k):
        """One iteration over the active slots using staging buffer k."""
        items = [it for s in slots for it in s.items()]
        arr = (L.wv_step_item * len(items))(*items)
        if self.staging_ev[k] is not None:
            self.staging_ev[k].synchronize()        # staging k is free once its copy ran
        used = ctypes.c_size_t()
        L.call("wv_context_params_items", self.model.h, len(items), arr,
               ctypes.c_void_p(self.staging[k].data_ptr()), self.staging[k].numel(),
               ctypes.c_void_p(self.desc[k].data_ptr()), self.desc[k].numel(), _byref(used),
               codec._stream())
        ev = torch.cuda.Event()
        ev.record(torch.cuda.current_stream())
        self.staging_ev[k] = ev
        if self.on_params is not None:
            for s in slots:
                for b, ws in enumerate(s.ws):
                    lay = ws.lay[s.i]
                    ng = codec.Model.group_count(lay["h"], lay["w"], s.g)
                    K = self.model.cfg["mix_k"]
                    self.on_params(s, b, s.i, s.g, ws.params[:ws.N * ng * 3 * K].view(ws.N, ng, 3 * K))
        return [s for s in slots if s.after_params(self.model)]

    def run(self, requests, preps, admit_until=None, max_seconds=120.0, log=None, keep_outputs=False):
        """requests: list of (arrival_s, prep_id) sorted by time.  Returns (stats, slots);
        finished slots keep their reconstruction only if keep_outputs."""
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
        fp = {pid: footprint(m, p) for pid, p in preps.items()}
        while True:
            now = time.perf_counter() - t0
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
                mid_joins += any((a.i, a.g) != (0, 0) for a in active)
                used += fp[pid]
                active.append(slot)
            peak_active = max(peak_active, len(active))
            if active:
                fin = self.step(active, k)
                k ^= 1
                iters += 1
                for s in fin:
                    s.finish(m)
                    active.remove(s)
                    finishing.append(s)
            for s in list(finishing):
                if s.done_event.query():
                    s.req["finished"] = time.perf_counter() - t0
                    finishing.remove(s)
                    used -= fp[s.req["prep"]]
                    s.release(keep_outputs)
                    done.append(s)
            if not (pending or queue or active or finishing):
                break
            if now > max_seconds:
                break
            if not active and not finishing and queue == deque() and pending:
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
        if log:
            log(f"served {stats}")
        return stats, done
