"""Batched decoding of images of uneven size through a plan (wv_plan_*).

Images are grouped by size; each group's planes share one set of device
buffers.  Every layer of a coding step then runs as one persistent launch
over all groups, the CDF tables of a step as one launch over all groups'
rows.  The whole decode can be captured in a HIP graph of the library's
launches (wv_graph_*) and replayed; `autotune` picks the per-level
output-channel blocking by timing replays (the choice never changes bits).
"""
import ctypes
import time

import numpy as np
import torch

from . import _lib as L
from . import codec

_byref = ctypes.byref


class Batch:
    def __init__(self, model, sizes, planes=3, nb_table=None):
        self.model = model
        self.sizes = [tuple(s) for s in sizes]
        self.planes = planes
        order = sorted(set(self.sizes), key=lambda hw: (hw[0] * hw[1], hw))
        self.group_sizes = order
        # image k -> (group, first plane within the group)
        self.where = []
        counts = {hw: 0 for hw in order}
        for hw in self.sizes:
            self.where.append((order.index(hw), counts[hw] * planes))
            counts[hw] += 1
        self.ws = [codec.Workspace(model, counts[hw] * planes, hw[0], hw[1]) for hw in order]
        self.q = [torch.zeros((w.N, w.H * w.W), dtype=torch.int16, device=model.device) for w in self.ws]
        self.xhat = [torch.empty((w.N, w.H, w.W), dtype=torch.float32, device=model.device) for w in self.ws]
        self.pixels = sum(h * w for h, w in self.sizes)
        self._make_plan(nb_table)

    def _groups(self):
        arr = (L.wv_group * len(self.ws))()
        for b, w in enumerate(self.ws):
            arr[b] = L.wv_group(w.H, w.W, w.N, self.q[b].data_ptr(), w.state.data_ptr(), w.scratch.data_ptr())
        return arr

    def _make_plan(self, nb_table):
        m = self.model
        self.nb_table = list(nb_table) if nb_table is not None else None
        tab = (ctypes.c_int * m.cfg["levels"])(*self.nb_table) if self.nb_table else None
        groups = self._groups()
        desc, rows = ctypes.c_size_t(), ctypes.c_longlong()
        L.call("wv_plan_bytes", m.h, len(self.ws), groups, tab, _byref(desc), _byref(rows))
        K = m.cfg["mix_k"]
        self.max_rows = rows.value
        self.d_desc = torch.empty(desc.value + 256, dtype=torch.uint8, device=m.device)
        self.params = torch.empty(rows.value * 3 * K, dtype=torch.float32, device=m.device)
        self.cdf = torch.empty(rows.value * (m.nsym + 1), dtype=torch.int16, device=m.device)
        h = ctypes.c_void_p()
        L.call("wv_plan_create", m.h, len(self.ws), groups, tab, self.d_desc.data_ptr(), desc.value,
               self.params.data_ptr(), codec._stream(), _byref(h))
        self.h = h
        self.nsub = len(self.ws[0].lay)

    def replan(self, nb_table):
        """Rebuild the plan's launch descriptors (same buffers) with another blocking table."""
        L.lib().wv_plan_destroy(self.h)
        self.h = None
        self._make_plan(nb_table)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            try:
                L.lib().wv_plan_destroy(h)
            except Exception:
                pass

    def rows(self, i, g):
        n = ctypes.c_longlong()
        first = (ctypes.c_longlong * len(self.ws))()
        L.call("wv_plan_rows", self.h, i, g, _byref(n), first)
        return n.value, list(first)

    # -- per-step calls -----------------------------------------------------
    def context_params(self, i, g):
        L.call("wv_plan_context_params", self.h, i, g, codec._stream())
        n, _ = self.rows(i, g)
        return self.params[:n * 3 * self.model.cfg["mix_k"]]

    def cdf_tables(self, prm):
        return codec.cdf_tables(self.model, prm, out=self.cdf)

    def scatter(self, sym, i, g):
        L.call("wv_plan_scatter", self.h, codec._ptr(sym), i, g, codec._stream())

    def synthesize(self):
        for b, w in enumerate(self.ws):
            codec.synthesize(self.model, w, q=self.q[b], xhat=self.xhat[b])
        return self.xhat

    # -- inputs ---------------------------------------------------------------
    def load_images(self, images):
        """uint8 planes per image ([planes][H][W]) -> analyse each group into its symbols."""
        for b, w in enumerate(self.ws):
            x = torch.empty((w.N, w.H, w.W), dtype=torch.uint8, device=self.model.device)
            for k, (gb, p0) in enumerate(self.where):
                if gb == b:
                    x[p0:p0 + self.planes] = torch.from_numpy(np.ascontiguousarray(images[k]))
            q, _, _ = codec.analyze(self.model, x, w)
            self.q[b].copy_(q)

    def known_symbols(self):
        """Per (subband, step): the symbols of all groups laid out like the plan's rows."""
        out = []
        for i in range(self.nsub):
            row = []
            for g in range(4):
                parts = [codec.gather_symbols(self.model, self.q[b], w, i, g).reshape(-1)
                         for b, w in enumerate(self.ws)]
                row.append(torch.cat(parts).contiguous())
            out.append(row)
        return out

    # -- decode -------------------------------------------------------------
    def decode_elided(self, syms):
        """Coder-elided decode of the whole batch: every step's context model, CDF
        tables and symbol scatter, then synthesis; asynchronous on the current stream."""
        for q in self.q:
            codec.zero(q)
        for i in range(self.nsub):
            for g in range(4):
                prm = self.context_params(i, g)
                self.cdf_tables(prm)
                self.scatter(syms[i][g], i, g)
        return self.synthesize()

    def capture(self, syms):
        """Capture decode_elided in a library graph (after one eager warm-up run)."""
        self.decode_elided(syms)
        torch.cuda.synchronize()
        graph = codec.Graph(lambda: self.decode_elided(syms))
        torch.cuda.synchronize()
        return graph


def time_graph(graph, reps=3):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        graph.replay()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def autotune(batch, syms, choices=(1, 2, 4), reps=2, log=None):
    """Coordinate search of the per-level output-channel blocking of `batch`: start from
    the occupancy rule, then for each level try every choice with the others fixed and keep
    the fastest graph replay.  Leaves the batch planned with the best table.
    Returns (nb_table or None for the default rule, seconds per decode)."""
    J = batch.model.cfg["levels"]

    def run(tab):
        batch.replan(tab)
        g = batch.capture(syms)
        t = time_graph(g, reps)
        del g
        return t

    best_tab, best_t = None, run(None)
    if log:
        log(f"autotune: default {best_t * 1e3:.2f} ms")
    seen = set()
    for lev in range(J, 0, -1):          # coarse levels first: fewest tiles
        for c in choices:
            tab = list(best_tab or [4] * J)
            tab[lev - 1] = c
            if tuple(tab) in seen:       # measured already (the table being improved)
                continue
            seen.add(tuple(tab))
            t = run(tab)
            if log:
                log(f"autotune: table {tab} {t * 1e3:.2f} ms")
            if t < best_t:
                best_t, best_tab = t, tab
    batch.replan(best_tab)
    return best_tab, best_t
