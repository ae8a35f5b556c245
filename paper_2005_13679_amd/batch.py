"""Batches of (N, M, h, g) instances: persistent batched H.C, segmented
Lanczos vector operations and a 50-step Lanczos recurrence captured in one
HIP graph.  All arithmetic runs in the library's kernels.

A batch vector is the concatenation of the instances' coefficient vectors in
the order the instances were given (``Batch.offsets``).
"""

from __future__ import annotations

import ctypes
import weakref

import numpy as np
import torch

from . import _lib as L
from . import api


def table_bytes(N: int, M: int, double_jumps: bool, form: str = "paper") -> int:
    """Device bytes of the tables of one instance (mc_tables_bytes: the
    double-jump map, if requested, at its largest tiled size)."""
    return api.tables_bytes(N, M, form, double_jumps)


def choose_double_jumps(shapes, budget_bytes: float, form: str = "paper") -> list[bool]:
    """Which instances keep a double-jump map within `budget_bytes` of
    double-jump tables (mc_choose_double_jumps: smallest maps first, so the
    most instances are served); the rest chain single jumps."""
    return api.choose_double_jumps(shapes, budget_bytes, form)


class Batch:
    """Persistent batched H.C over instances [(tables, h, g), ...] on one device."""

    def __init__(self, instances, schedule: dict | None = None):
        if not instances:
            raise ValueError("empty batch")
        self.device = instances[0][0].device
        self.tables = []
        self._keep = []
        n = len(instances)
        items = (L.BatchItem * n)()
        for i, (tab, h, g) in enumerate(instances):
            if tab.device != self.device:
                raise ValueError("all instances must live on one device")
            M = tab.M
            hd = api._as_dev(h, self.device, (M, M))
            gd = api._as_dev(g, self.device, (M, M, M, M))
            self._keep += [hd, gd]
            self.tables.append(tab)
            items[i].tables = ctypes.pointer(tab.c)
            items[i].h_d = hd.data_ptr()
            items[i].g_d = gd.data_ptr()
        self._items = items
        lib = L.load()
        nbytes = L.c_sz()
        L.check(lib.mc_batch_plan_size(n, items, ctypes.byref(nbytes)), "mc_batch_plan_size")
        self.plan = torch.empty(max(256, nbytes.value), dtype=torch.uint8, device=self.device)
        sched = L.BatchSchedule()
        schedule = dict(schedule or {})
        sched.blocks_per_cu = int(schedule.get("blocks_per_cu", 2))
        sched.order = int(schedule.get("order", 3))
        sched.solo_tiles = int(schedule.get("solo_tiles", 16384))
        self.schedule = {"blocks_per_cu": sched.blocks_per_cu, "order": sched.order,
                         "solo_tiles": sched.solo_tiles}
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            L.check(lib.mc_batch_create(n, items, ctypes.byref(sched), api._ptr(self.plan),
                                        self.plan.numel(), api._stream(self.device),
                                        ctypes.byref(handle)), "mc_batch_create")
        self._h = handle
        # destroy the host handle when the batch is collected (or at exit)
        self._finalizer = weakref.finalize(self, lib.mc_batch_destroy, handle)
        self.count = n
        self.length = int(lib.mc_batch_vector_length(handle))
        dims = [t.dim for t in self.tables]
        self.offsets = np.concatenate([[0], np.cumsum(dims)]).astype(np.int64)

    def vector(self) -> torch.Tensor:
        return torch.empty(self.length, dtype=torch.complex128, device=self.device)

    def segment(self, x: torch.Tensor, i: int) -> torch.Tensor:
        return x[int(self.offsets[i]):int(self.offsets[i + 1])]

    def _chk(self, x, name):
        api._require(x, name, torch.complex128, self.device, numel=self.length)

    def apply_H(self, C: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
        self._chk(C, "C")
        self._chk(out, "out")
        with torch.cuda.device(self.device):
            L.check(L.load().mc_batch_apply_H(self._h, api._ptr(C), api._ptr(out),
                                              api._stream(self.device)), "mc_batch_apply_H")
        return out

    def dot(self, x, y, out):
        self._chk(x, "x")
        self._chk(y, "y")
        api._require(out, "out", torch.complex128, self.device, numel=self.count)
        with torch.cuda.device(self.device):
            L.check(L.load().mc_batch_dot(self._h, api._ptr(x), api._ptr(y), api._ptr(out),
                                          api._stream(self.device)), "mc_batch_dot")
        return out

    def lanczos_orth(self, w, v, vprev, alpha, beta):
        nul = ctypes.c_void_p(None)
        with torch.cuda.device(self.device):
            L.check(L.load().mc_batch_lanczos_orth(
                self._h, api._ptr(w), api._ptr(v), api._ptr(vprev) if vprev is not None else nul,
                api._ptr(alpha), api._ptr(beta) if beta is not None else nul,
                api._stream(self.device)), "mc_batch_lanczos_orth")

    def normalize(self, w, out, beta):
        api._require(beta, "beta", torch.float64, self.device, numel=self.count)
        with torch.cuda.device(self.device):
            L.check(L.load().mc_batch_normalize(self._h, api._ptr(w), api._ptr(out), api._ptr(beta),
                                                api._stream(self.device)), "mc_batch_normalize")


class BatchedLanczos:
    """Fixed-length three-term Lanczos recurrence (no reorthogonalisation) for
    every instance of a batch; ``graph=True`` has the library capture all
    steps into one HIP graph (mc_batch_lanczos_graph) that ``run`` replays."""

    def __init__(self, batch: Batch, steps: int = 50, graph: bool = True):
        self.b, self.steps = batch, int(steps)
        dev = batch.device
        self.v_in = batch.vector()
        self.Vbuf = torch.empty((3, batch.length), dtype=torch.complex128, device=dev)
        self.V = [self.Vbuf[i] for i in range(3)]
        self.w = batch.vector()
        self.alphas = torch.zeros((self.steps, batch.count), dtype=torch.complex128, device=dev)
        self.betas = torch.zeros((self.steps + 1, batch.count), dtype=torch.float64, device=dev)
        self.graph = None
        if graph:
            # warm up outside capture (first launches load code objects)
            self._record()
            torch.cuda.synchronize(dev)
            self.stream = torch.cuda.Stream(device=dev)
            handle = ctypes.c_void_p()
            lib = L.load()
            P = api._ptr
            L.check(lib.mc_batch_lanczos_graph(batch._h, self.steps, P(self.v_in), P(self.Vbuf),
                                               P(self.w), P(self.alphas), P(self.betas),
                                               ctypes.c_void_p(self.stream.cuda_stream),
                                               ctypes.byref(handle)), "mc_batch_lanczos_graph")
            self.graph = handle
            self._finalizer = weakref.finalize(self, lib.mc_graph_destroy, handle)

    def _record(self):
        b, V, w = self.b, self.V, self.w
        b.normalize(self.v_in, V[0], self.betas[self.steps])
        for j in range(self.steps):
            cur, prev, nxt = V[j % 3], V[(j - 1) % 3], V[(j + 1) % 3]
            b.apply_H(cur, w)
            b.dot(cur, w, self.alphas[j])
            b.lanczos_orth(w, cur, prev if j > 0 else None, self.alphas[j],
                           self.betas[j - 1] if j > 0 else None)
            b.normalize(w, nxt, self.betas[j])

    def run(self, v0: torch.Tensor):
        """Runs the recurrence from the batch vector v0; returns (alphas
        [steps, count] real, betas [steps, count]) as host arrays."""
        self.b._chk(v0, "v0")
        dev = self.b.device
        self.v_in.copy_(v0)
        if self.graph is not None:
            cur = torch.cuda.current_stream(dev)
            self.stream.wait_stream(cur)
            L.check(L.load().mc_graph_launch(self.graph, ctypes.c_void_p(self.stream.cuda_stream)),
                    "mc_graph_launch")
            cur.wait_stream(self.stream)
        else:
            self._record()
        torch.cuda.synchronize(dev)
        return (self.alphas.real.cpu().numpy().copy(), self.betas[: self.steps].cpu().numpy().copy())


def plain_lanczos(tables, h, g, v0: torch.Tensor, steps: int = 50):
    """The same recurrence for one instance with the single-instance calls
    (mc_apply_H, mc_zdotc, mc_lanczos_orth, mc_normalize), launched eagerly."""
    dev, D = tables.device, tables.dim
    lib = L.load()
    st = api._stream(dev)
    V = [torch.empty(D, dtype=torch.complex128, device=dev) for _ in range(3)]
    w = torch.empty(D, dtype=torch.complex128, device=dev)
    alphas = torch.zeros(steps, dtype=torch.complex128, device=dev)
    betas = torch.zeros(steps + 1, dtype=torch.float64, device=dev)
    ws = torch.empty((L.MC_DOT_BLOCKS + 2) * 16, dtype=torch.uint8, device=dev)
    P = api._ptr
    M = tables.M
    hd = api._as_dev(h, dev, (M, M))
    gd = api._as_dev(g, dev, (M, M, M, M))
    with torch.cuda.device(dev):
        L.check(lib.mc_normalize(D, P(v0), P(V[0]), P(betas[steps]), P(ws), ws.numel(), st), "norm")
        for j in range(steps):
            cur, prev, nxt = V[j % 3], V[(j - 1) % 3], V[(j + 1) % 3]
            api.apply_H(hd, gd, cur, tables, out=w)
            api.zdotc(cur, w, out=alphas[j])
            L.check(lib.mc_lanczos_orth(D, P(w), P(cur), P(prev) if j > 0 else None, P(alphas[j]),
                                        P(betas[j - 1]) if j > 0 else None, st), "orth")
            L.check(lib.mc_normalize(D, P(w), P(nxt), P(betas[j]), P(ws), ws.numel(), st), "norm")
    return alphas, betas[:steps]


def batched_lanczos(instances, steps: int = 50, v0: torch.Tensor | None = None,
                    schedule: dict | None = None, graph: bool = True, seed: int = 0):
    """``steps`` three-term Lanczos steps for every instance [(tables, h, g),
    ...] at once (one captured graph by default).  v0 is a batch vector (a
    seeded complex-normal start per instance if None).  Returns
    (alphas [steps, count], betas [steps, count]) as host arrays."""
    b = Batch(instances, schedule)
    if v0 is None:
        rng = np.random.default_rng(seed)
        v0 = b.vector()
        for i, (t, _, _) in enumerate(instances):
            x = rng.standard_normal(t.dim) + 1j * rng.standard_normal(t.dim)
            b.segment(v0, i).copy_(torch.from_numpy(x))
    return BatchedLanczos(b, steps, graph=graph).run(v0)
