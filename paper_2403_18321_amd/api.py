"""High-level driver: the four stages of Algorithm 1 on one cube, through
the C ABI. Buffers come from torch's allocator; all work is in libpca."""

from __future__ import annotations

from dataclasses import dataclass

import torch

from . import _lib as L

DEFAULT_TOL = 1e-6          # relative off-norm stop for the float32 Jacobi
DEFAULT_MAX_SWEEPS = 30


@dataclass
class PCAResult:
    mean: torch.Tensor      # [M] float32
    C: torch.Tensor         # [M, M] float32
    eigvals: torch.Tensor   # [M] float32, descending
    V: torch.Tensor         # [M, M] float32, column j = eigenvector j
    Q: torch.Tensor         # [N, k] float32
    info: torch.Tensor      # device pca_info

    def read_info(self) -> dict:
        return L.read_info(self.info)


class PCAPipeline:
    """Preallocated buffers and workspaces for cubes of one shape; forward()
    only enqueues kernels (no allocation, no synchronisation), so it can be
    captured in a HIP graph."""

    def __init__(self, n_pixels: int, n_bands: int, k: int, mode: str = "f32",
                 tol: float = DEFAULT_TOL, max_sweeps: int = DEFAULT_MAX_SWEEPS,
                 fp64_angles: bool = True, device="cuda", layout: str = "bip", overlap_replay: bool = True,
                 jacobi: str = "auto"):
        """layout: "bip" for [pixels, bands] cubes, "bsq" for [bands, pixels]
        (band-sequential) cubes. overlap_replay: with the one-workgroup
        Jacobi, form the eigenvectors while the sweeps run, on other CUs of
        the same launch (for a cube that has the GPU to itself; a stream of
        cubes leaves those CUs to the other cubes' passes). jacobi: "auto"
        (block-cyclic on many CUs from 96 bands, one workgroup below),
        "block" or "one_cu"."""
        self.n, self.m, self.k = int(n_pixels), int(n_bands), int(k)
        self.layout = layout
        self.mode = L.COV_MODES[mode] if isinstance(mode, str) else int(mode)
        self.tol, self.max_sweeps, self.fp64_angles = float(tol), int(max_sweeps), bool(fp64_angles)
        self.overlap_replay = bool(overlap_replay)
        if jacobi not in L.JACOBI_FORMS:
            raise ValueError(f"jacobi must be one of {sorted(L.JACOBI_FORMS)}")
        self.jacobi = jacobi
        dev = torch.device(device)
        f32 = dict(dtype=torch.float32, device=dev)
        self.mean = torch.empty(self.m, **f32)
        self.C = torch.empty(self.m, self.m, **f32)
        self.eigvals = torch.empty(self.m, **f32)
        self.V = torch.empty(self.m, self.m, **f32)
        self.Q = torch.empty(self.n, self.k, **f32)
        self.info = L.new_info(dev)
        self.ws_cov = L.workspace(L.pca_workspace_size(L.PCA_OP_COVARIANCE, self.n, self.m, mode=self.mode), dev)
        self.ws_jac = L.workspace(L.pca_workspace_size(L.PCA_OP_JACOBI, self.n, self.m,
                                                       max_sweeps=self.max_sweeps), dev)

    def covariance(self, Y):
        L.pca_covariance(Y, self.C, self.mean, self.mode, False, self.ws_cov, layout=self.layout)

    def eigh(self):
        L.pca_jacobi_eigh(self.C, self.eigvals, self.V, self.tol, self.max_sweeps, self.fp64_angles,
                          self.info, self.ws_jac, overlap=self.overlap_replay, form=self.jacobi)

    def project(self, Y):
        L.pca_project(Y, self.mean, self.V, self.k, self.Q, layout=self.layout)

    def shape(self):
        return (self.m, self.n) if self.layout == "bsq" else (self.n, self.m)

    def forward(self, Y) -> PCAResult:
        if tuple(Y.shape) != self.shape():
            raise ValueError(f"cube shape {tuple(Y.shape)} != {self.shape()} ({self.layout})")
        self.covariance(Y)
        self.eigh()
        self.project(Y)
        return PCAResult(self.mean, self.C, self.eigvals, self.V, self.Q, self.info)


class PCAStream:
    """A stream of cubes of one shape with several in flight at once.

    Cube i runs on HIP stream i mod depth with its own buffers and workspaces,
    so the single-CU Jacobi of one cube overlaps the all-CU streaming passes
    (covariance, projection) of the others; every cube still goes through
    the whole pipeline. With `chain` the covariance pass of cube i starts
    only after that of cube i-1 has finished (an event between the streams),
    which keeps the streams out of phase: their HBM-bound passes take turns
    instead of all running at once while every Jacobi waits. submit() only
    enqueues: the result of a submitted cube is valid once its event has
    completed and stays valid until the same slot is reused `depth`
    submissions later. The streams keep the default priority."""

    def __init__(self, n_pixels: int, n_bands: int, k: int, mode: str = "f32", depth: int = 4,
                 tol: float = DEFAULT_TOL, max_sweeps: int = DEFAULT_MAX_SWEEPS,
                 fp64_angles: bool = True, device="cuda", chain: bool = True, overlap_replay: bool = False,
                 jacobi: str = "one_cu"):
        """jacobi: the eigen-solver form of every cube (default the
        one-workgroup form: the block-cyclic form spreads one cube over many
        CUs and waits on all of them at every step, which pays only when the
        cube has the GPU to itself)."""
        if depth < 1:
            raise ValueError("depth must be >= 1")
        self.depth = int(depth)
        self.chain = bool(chain)
        self.pipes = [PCAPipeline(n_pixels, n_bands, k, mode, tol, max_sweeps, fp64_angles, device,
                                  overlap_replay=overlap_replay, jacobi=jacobi) for _ in range(self.depth)]
        self.streams = [torch.cuda.Stream(device=device) for _ in range(self.depth)]
        self.events = [torch.cuda.Event() for _ in range(self.depth)]
        self.cov_done = [torch.cuda.Event() for _ in range(self.depth)]
        self.count = 0

    def submit(self, Y):
        """Enqueue the PCA of cube Y (after the work already queued on the
        caller's current stream); returns (PCAResult, completion event)."""
        s = self.count % self.depth
        st = self.streams[s]
        pipe = self.pipes[s]
        if tuple(Y.shape) != pipe.shape():
            raise ValueError(f"cube shape {tuple(Y.shape)} != {pipe.shape()}")
        st.wait_stream(torch.cuda.current_stream())
        if self.chain and self.count > 0:
            st.wait_event(self.cov_done[(self.count - 1) % self.depth])
        Y.record_stream(st)
        with torch.cuda.stream(st):
            pipe.covariance(Y)
            self.cov_done[s].record(st)
            pipe.eigh()
            pipe.project(Y)
            self.events[s].record(st)
        self.count += 1
        return PCAResult(pipe.mean, pipe.C, pipe.eigvals, pipe.V, pipe.Q, pipe.info), self.events[s]

    def join(self):
        """Make the caller's current stream wait for every submitted cube."""
        cur = torch.cuda.current_stream()
        for st in self.streams:
            cur.wait_stream(st)


def run(Y: torch.Tensor, k: int, mode: str = "f32", tol: float = DEFAULT_TOL,
        max_sweeps: int = DEFAULT_MAX_SWEEPS, fp64_angles: bool = True, layout: str = "bip",
        overlap_replay: bool = True) -> PCAResult:
    """PCA of one device cube Y (float32 or uint16): [pixels, bands], or
    [bands, pixels] with layout="bsq"."""
    n, m = (Y.shape[1], Y.shape[0]) if layout == "bsq" else (Y.shape[0], Y.shape[1])
    pipe = PCAPipeline(n, m, k, mode, tol, max_sweeps, fp64_angles, Y.device, layout=layout,
                       overlap_replay=overlap_replay)
    return pipe.forward(Y)


# Pipelines (and their workspaces) of the autograd Function, reused across
# calls of the same shape and settings. A pipeline's calls go to the current
# stream in order; its result tensors are cloned before they are handed out.
_FN_PIPES = {}
_FN_PIPES_MAX = 8


def _fn_pipeline(n, m, k, mode, tol, max_sweeps, device, layout):
    key = (str(device), n, m, k, mode, float(tol), int(max_sweeps), layout)
    pipe = _FN_PIPES.get(key)
    if pipe is None:
        if len(_FN_PIPES) >= _FN_PIPES_MAX:
            _FN_PIPES.pop(next(iter(_FN_PIPES)))
        pipe = PCAPipeline(n, m, k, mode, tol, max_sweeps, True, device, layout=layout)
        _FN_PIPES[key] = pipe
    return pipe


class PCAFunction(torch.autograd.Function):
    """(Q, eigvals, V[:, :k]) = PCA(Y) with the hand-written adjoint of
    pca_backward as its derivative. Forward: fused centring + covariance,
    Jacobi eigenpairs, projection; backward: one pca_backward call. Y is
    [pixels, bands] ("bip") or [bands, pixels] ("bsq"); its gradient has
    the same layout."""

    @staticmethod
    def forward(ctx, Y, k: int, mode: str = "f32", tol: float = DEFAULT_TOL,
                max_sweeps: int = DEFAULT_MAX_SWEEPS, layout: str = "bip"):
        if Y.dtype != torch.float32:
            raise ValueError("PCAFunction needs a float32 cube")
        Yc = Y.detach()
        n, m = (Yc.shape[1], Yc.shape[0]) if layout == "bsq" else (Yc.shape[0], Yc.shape[1])
        pipe = _fn_pipeline(n, m, k, mode, tol, max_sweeps, Yc.device, layout)
        r = pipe.forward(Yc)
        mean, eigvals, V = r.mean.clone(), r.eigvals.clone(), r.V.clone()
        ctx.save_for_backward(Yc, mean, eigvals, V)
        ctx.k = int(k)
        ctx.layout = layout
        return r.Q.clone(), eigvals.clone(), V[:, :k].contiguous()

    @staticmethod
    def backward(ctx, dQ, dEig, dVk):
        Y, mean, eigvals, V = ctx.saved_tensors
        k = ctx.k
        dY = torch.empty_like(Y)
        prep = lambda t: None if t is None else t.detach().to(torch.float32).contiguous()
        L.pca_backward(Y, mean, eigvals, V, k, dY, prep(dQ), prep(dEig), prep(dVk), layout=ctx.layout)
        return dY, None, None, None, None, None


def pca_autograd(Y: torch.Tensor, k: int, mode: str = "f32", tol: float = DEFAULT_TOL,
                 max_sweeps: int = DEFAULT_MAX_SWEEPS, layout: str = "bip"):
    """Differentiable PCA of a float32 device cube: returns (Q, eigvals, V_k)."""
    return PCAFunction.apply(Y, k, mode, tol, max_sweeps, layout)
