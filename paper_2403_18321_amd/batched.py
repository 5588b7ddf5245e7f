"""Batched form: many cubes of different pixel and band counts in one
pca_batched call (a fixed number of launches for the whole batch), with
preallocated outputs, a resident descriptor array, optional capture of the
call in a HIP graph, and tile shapes from the autotuner."""

from __future__ import annotations

import ctypes

import torch

from . import _lib as L
from .api import DEFAULT_MAX_SWEEPS, DEFAULT_TOL


class BatchedPCA:
    """PCA of a fixed list of device cubes. ``run()`` only enqueues kernels
    (no allocation, no host-to-device copy), so it can be captured."""

    def __init__(self, cubes, ks, mode: str = "f32", tol: float = DEFAULT_TOL,
                 max_sweeps: int = DEFAULT_MAX_SWEEPS, fp64_angles: bool = True, tuning=None):
        if not cubes:
            raise ValueError("empty batch")
        if isinstance(ks, int):
            ks = [ks] * len(cubes)
        if len(ks) != len(cubes):
            raise ValueError("one k per cube")
        dts = {L._cube(Y)[0] for Y in cubes}
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
        arr = (L.PCACube * len(cubes))()
        for i, (Y, k) in enumerate(zip(self.cubes, self.ks)):
            _, n, m, ld = L._cube(Y)
            self.mean.append(torch.empty(m, **f32))
            self.eigvals.append(torch.empty(m, **f32))
            self.V.append(torch.empty(m, m, **f32))
            self.Q.append(torch.empty(n, k, **f32))
            self.info.append(L.new_info(dev))
            arr[i] = L.PCACube(Y.data_ptr(), n, ld, m, k, self.mean[i].data_ptr(), self.eigvals[i].data_ptr(),
                               self.V[i].data_ptr(), self.Q[i].data_ptr(), self.info[i].data_ptr())
        self._host = arr
        raw = bytes(memoryview(arr).cast("B"))
        self._dev = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(dev)
        self.set_tuning(tuning)

    def set_tuning(self, tuning):
        """tuning: None (defaults), a (cov_chunk, proj_tiles) pair or a dict."""
        if tuning is None:
            self.tuning = None
        elif isinstance(tuning, dict):
            self.tuning = L.PCABatchTuning(int(tuning.get("cov_chunk", 0)), int(tuning.get("proj_tiles", 0)))
        else:
            self.tuning = L.PCABatchTuning(int(tuning[0]), int(tuning[1]))
        nbytes = L.pca_batched_workspace_size(ctypes.pointer(self._host), len(self.cubes), self.mode,
                                              self.max_sweeps, self.tuning)
        self.ws = L.workspace(nbytes, self.cubes[0].device)

    def run(self):
        L.pca_batched(ctypes.pointer(self._host), self._dev, len(self.cubes), self.dt, self.mode, self.tol,
                      self.max_sweeps, self.fp64_angles, self.tuning, self.ws)

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
