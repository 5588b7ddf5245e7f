"""Batched form: many cubes of different pixel and band counts in one
pca_batched call (a fixed number of launches for the whole batch), with
preallocated outputs, a resident descriptor array, optional capture of the
call in a HIP graph, and tile shapes from the autotuner."""

from __future__ import annotations

import ctypes

import torch

from . import _lib as L
from .api import DEFAULT_MAX_SWEEPS, DEFAULT_TOL


def _lane_split(bands, lanes):
    """Cube indices per lane: the cubes in decreasing band order, the first
    lane taking the widest ones. A cube's Jacobi runs on one CU for a time
    that grows like bands^3, so the widest cubes set the batch's critical
    path; giving them a lane of their own lets their eigendecompositions
    start after only their own covariance passes, and lets the other lanes'
    passes and eigendecompositions run beside them. Lane sizes grow
    geometrically (1/8, 3/8, 1/2 of the cubes for three lanes)."""
    order = sorted(range(len(bands)), key=lambda i: (-bands[i], i))
    if lanes <= 1 or len(order) < 2 * lanes:
        return [order]
    weights = [2 ** j for j in range(lanes)]
    total = sum(weights)
    out, start = [], 0
    for j, w in enumerate(weights):
        end = len(order) if j == lanes - 1 else start + max(1, round(len(order) * w / total))
        out.append(order[start:end])
        start = end
    return [g for g in out if g]


class BatchedPCA:
    """PCA of a fixed list of device cubes. ``run()`` only enqueues kernels
    (no allocation, no host-to-device copy), so it can be captured.

    With ``lanes`` > 1 the batch is split into that many sub-batches by band
    count (see _lane_split), each one pca_batched call on its own HIP stream
    (forked from and joined back to the caller's stream, so a captured graph
    holds all of them)."""

    def __init__(self, cubes, ks, mode: str = "f32", tol: float = DEFAULT_TOL,
                 max_sweeps: int = DEFAULT_MAX_SWEEPS, fp64_angles: bool = True, tuning=None, lanes: int = 1,
                 layout: str = "bip"):
        """cubes: device tensors [pixels, bands] ("bip") or [bands, pixels]
        ("bsq"), all of one element type and layout."""
        if not cubes:
            raise ValueError("empty batch")
        if isinstance(ks, int):
            ks = [ks] * len(cubes)
        if len(ks) != len(cubes):
            raise ValueError("one k per cube")
        self.layout = layout
        dts = {L._cube(Y, layout)[0] for Y in cubes}
        if len(dts) != 1:
            raise ValueError("all cubes of a batch must have the same element type")
        self.dt = dts.pop()
        self.mode = L.COV_MODES[mode] if isinstance(mode, str) else int(mode)
        self.tol, self.max_sweeps, self.fp64_angles = float(tol), int(max_sweeps), bool(fp64_angles)
        self.cubes = list(cubes)
        self.ks = [int(k) for k in ks]
        dev = self.cubes[0].device
        f32 = dict(dtype=torch.float32, device=dev)
        self.mean, self.eigvals, self.V, self.Q, self.info = [], [], [], [], []
        descs = []
        for i, (Y, k) in enumerate(zip(self.cubes, self.ks)):
            _, n, m, ld = L._cube(Y, layout)
            self.mean.append(torch.empty(m, **f32))
            self.eigvals.append(torch.empty(m, **f32))
            self.V.append(torch.empty(m, m, **f32))
            self.Q.append(torch.empty(n, k, **f32))
            self.info.append(L.new_info(dev))
            descs.append(L.PCACube(Y.data_ptr(), n, ld, m, k, self.mean[i].data_ptr(), self.eigvals[i].data_ptr(),
                                   self.V[i].data_ptr(), self.Q[i].data_ptr(), self.info[i].data_ptr()))
        self.groups = _lane_split([L._cube(Y, layout)[2] for Y in self.cubes], int(lanes))
        self._host, self._dev = [], []
        for g in self.groups:
            arr = (L.PCACube * len(g))(*[descs[i] for i in g])
            self._host.append(arr)
            raw = bytes(memoryview(arr).cast("B"))
            self._dev.append(torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(dev))
        self.streams = [torch.cuda.Stream(device=dev) for _ in self.groups] if len(self.groups) > 1 else []
        self.set_tuning(tuning)

    def set_tuning(self, tuning):
        """tuning: None (defaults), a (cov_chunk, proj_tiles) pair or a dict."""
        if tuning is None:
            self.tuning = None
        elif isinstance(tuning, dict):
            self.tuning = L.PCABatchTuning(int(tuning.get("cov_chunk", 0)), int(tuning.get("proj_tiles", 0)))
        else:
            self.tuning = L.PCABatchTuning(int(tuning[0]), int(tuning[1]))
        dev = self.cubes[0].device
        self.ws = []
        for arr in self._host:
            nbytes = L.pca_batched_workspace_size(ctypes.pointer(arr), len(arr), self.mode, self.max_sweeps,
                                                  self.tuning)
            self.ws.append(L.workspace(nbytes, dev))

    def _call(self, j):
        L.pca_batched(ctypes.pointer(self._host[j]), self._dev[j], len(self._host[j]), self.dt, self.mode, self.tol,
                      self.max_sweeps, self.fp64_angles, self.tuning, self.ws[j])

    def run(self):
        if not self.streams:
            self._call(0)
            return
        cur = torch.cuda.current_stream()
        for j, st in enumerate(self.streams):
            st.wait_stream(cur)
            with torch.cuda.stream(st):
                self._call(j)
        for st in self.streams:
            cur.wait_stream(st)

    def capture(self) -> torch.cuda.CUDAGraph:
        """A graph of one run() (replay with graph.replay())."""
        self.run()                      # warm-up outside the capture
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            self.run()
        return g

    def pixel_bands(self) -> int:
        return sum(int(Y.shape[0]) * int(Y.shape[1]) for Y in self.cubes)
