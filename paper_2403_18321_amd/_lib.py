"""ctypes binding of libpca.so (argument marshalling only).

Every function here has the name and argument order of the C entry point in
include/pca.h. Tensors are passed as device pointers; the HIP stream is
torch's current stream. No arithmetic of the method happens in Python: if the
library is missing this module raises instead of falling back.
"""

from __future__ import annotations

import ctypes
import os
import struct

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libpca.so")

PCA_OK, PCA_ERR_ARG, PCA_ERR_UNSUPPORTED, PCA_ERR_WORKSPACE, PCA_ERR_HIP = range(5)
PCA_IN_F32, PCA_IN_U16, PCA_IN_F32_BSQ, PCA_IN_U16_BSQ = 0, 1, 2, 3
PCA_COV_F32, PCA_COV_BF16X3, PCA_COV_BF16X4, PCA_COV_FP16X3 = 0, 1, 2, 3
PCA_JACOBI_FP64_ANGLES, PCA_JACOBI_OVERLAP_REPLAY, PCA_JACOBI_ONE_CU, PCA_JACOBI_BLOCK = 1, 2, 4, 8
JACOBI_FORMS = {"auto": 0, "one_cu": PCA_JACOBI_ONE_CU, "block": PCA_JACOBI_BLOCK}
PCA_OP_CENTER, PCA_OP_COVARIANCE, PCA_OP_JACOBI, PCA_OP_PROJECT, PCA_OP_BACKWARD = range(5)

COV_MODES = {"f32": PCA_COV_F32, "bf16x3": PCA_COV_BF16X3, "bf16x4": PCA_COV_BF16X4, "fp16x3": PCA_COV_FP16X3}

# pca_info: int32 sweeps, converged, nonfinite, floor_hit; double off_rel;
# int64 rotations; int32 steps, n_bands.
INFO_FORMAT = "<iiiidqii"
INFO_BYTES = struct.calcsize(INFO_FORMAT)
INFO_FIELDS = ("sweeps", "converged", "nonfinite", "floor_hit", "off_rel", "rotations", "steps", "n_bands")

EXPORTS = ("pca_status_string", "pca_workspace_size", "pca_center", "pca_covariance",
           "pca_jacobi_eigh", "pca_jacobi_eigh_noalloc", "pca_project", "pca_backward", "pca_batched_workspace_size",
           "pca_batched", "pca_set_wait_shift")


class PCACube(ctypes.Structure):
    """struct pca_cube of include/pca.h."""
    _fields_ = [("Y", ctypes.c_void_p), ("n_pixels", ctypes.c_int64), ("ld_y", ctypes.c_int64),
                ("n_bands", ctypes.c_int32), ("k", ctypes.c_int32), ("mean", ctypes.c_void_p),
                ("eigvals", ctypes.c_void_p), ("V", ctypes.c_void_p), ("Q", ctypes.c_void_p),
                ("info", ctypes.c_void_p)]


class PCABatchTuning(ctypes.Structure):
    """struct pca_batch_tuning of include/pca.h."""
    _fields_ = [("cov_chunk", ctypes.c_int32), ("proj_tiles", ctypes.c_int32)]


class PCAError(RuntimeError):
    """A libpca entry point returned a status other than PCA_OK."""

    def __init__(self, fn: str, status: int):
        self.status = status
        msg = _lib().pca_status_string(status).decode() if _LIB is not None else str(status)
        super().__init__(f"{fn}: {msg}")


_LIB = None
_vp, _i32, _i64, _sz, _f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_double


def _lib() -> ctypes.CDLL:
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run python -m paper_2403_18321_amd.build_lib")
        lib = ctypes.CDLL(LIB_PATH)
        lib.pca_status_string.restype = ctypes.c_char_p
        lib.pca_status_string.argtypes = [ctypes.c_int]
        lib.pca_workspace_size.restype = ctypes.c_int
        lib.pca_workspace_size.argtypes = [ctypes.c_int, _i64, _i32, _i32, _i32, _i32, ctypes.POINTER(_sz)]
        lib.pca_center.restype = ctypes.c_int
        lib.pca_center.argtypes = [_vp, ctypes.c_int, _i64, _i32, _i64, _vp, _vp, _i64, _vp, _sz, _vp]
        lib.pca_covariance.restype = ctypes.c_int
        lib.pca_covariance.argtypes = [_vp, ctypes.c_int, _i64, _i32, _i64, _i32, _vp, ctypes.c_int, _vp, _vp,
                                       _sz, _vp]
        lib.pca_jacobi_eigh.restype = ctypes.c_int
        lib.pca_jacobi_eigh.argtypes = [_vp, _i32, _f64, _i32, _i32, _vp, _vp, _vp, _vp, _sz, _vp]
        lib.pca_jacobi_eigh_noalloc.restype = ctypes.c_int
        lib.pca_jacobi_eigh_noalloc.argtypes = [_vp, _i32, _f64, _i32, _i32, _vp, _vp, _vp, _vp]
        lib.pca_project.restype = ctypes.c_int
        lib.pca_project.argtypes = [_vp, ctypes.c_int, _i64, _i32, _i64, _vp, _vp, _i32, _vp, _vp]
        lib.pca_batched_workspace_size.restype = ctypes.c_int
        lib.pca_batched_workspace_size.argtypes = [_vp, _i32, ctypes.c_int, _i32, _vp, ctypes.POINTER(_sz)]
        lib.pca_set_wait_shift.restype = ctypes.c_int
        lib.pca_set_wait_shift.argtypes = [_i32]
        lib.pca_batched.restype = ctypes.c_int
        lib.pca_batched.argtypes = [_vp, _vp, _i32, ctypes.c_int, ctypes.c_int, _f64, _i32, _i32, _vp, _vp, _sz,
                                    _vp]
        lib.pca_backward.restype = ctypes.c_int
        lib.pca_backward.argtypes = [_vp, _i32, _i64, _i32, _i64, _vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp, _i64, _vp, _sz,
                                     _vp]
        _LIB = lib
    return _LIB


def library() -> ctypes.CDLL:
    """The loaded libpca (raises if it is not built)."""
    return _lib()


def _check(fn: str, status: int):
    if status != PCA_OK:
        raise PCAError(fn, status)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _cube(Y: torch.Tensor, layout: str = "bip"):
    """(dt, n_pixels, n_bands, ld) of a device cube: [pixels, bands] with unit
    band stride ("bip"), or [bands, pixels] with unit pixel stride ("bsq")."""
    if layout not in ("bip", "bsq"):
        raise ValueError(f"layout must be 'bip' or 'bsq', not {layout!r}")
    if Y.dim() != 2 or Y.stride(1) != 1:
        raise ValueError("cube must be a 2-D tensor with unit stride along its second axis "
                         "([pixels, bands] for bip, [bands, pixels] for bsq)")
    if Y.dtype == torch.float32:
        dt = PCA_IN_F32
    elif Y.dtype == torch.uint16:
        dt = PCA_IN_U16
    else:
        raise ValueError(f"unsupported cube dtype {Y.dtype}")
    if not Y.is_cuda:
        raise ValueError("cube must be a device tensor")
    if layout == "bsq":
        return dt + 2, Y.shape[1], Y.shape[0], Y.stride(0)
    return dt, Y.shape[0], Y.shape[1], Y.stride(0)


def pca_workspace_size(op: int, n_pixels: int, n_bands: int, k: int = 1, mode: int = 0,
                       max_sweeps: int = 0) -> int:
    out = _sz(0)
    _check("pca_workspace_size",
           _lib().pca_workspace_size(op, n_pixels, n_bands, k, mode, max_sweeps, ctypes.byref(out)))
    return int(out.value)


def workspace(nbytes: int, device=None) -> torch.Tensor:
    """A zero-filled device byte buffer for a workspace argument (torch
    allocations are at least 256-byte aligned; no call depends on what a
    workspace holds before it)."""
    return torch.zeros(max(int(nbytes), 256), dtype=torch.uint8, device=device or "cuda")


def pca_center(Y, mean, X=None, ws=None, layout: str = "bip"):
    dt, n, m, ld = _cube(Y, layout)
    if ws is None:
        ws = workspace(pca_workspace_size(PCA_OP_CENTER, n, m), Y.device)
    ldx = X.stride(0) if X is not None else 0
    _check("pca_center", _lib().pca_center(_ptr(Y), dt, n, m, ld, _ptr(mean), _ptr(X), ldx, _ptr(ws),
                                           ws.numel(), _stream()))


def pca_covariance(Y, C, mean=None, mode: int = PCA_COV_F32, input_is_centered: bool = False, ws=None,
                   layout: str = "bip"):
    dt, n, m, ld = _cube(Y, layout)
    if ws is None:
        ws = workspace(pca_workspace_size(PCA_OP_COVARIANCE, n, m, mode=mode), Y.device)
    _check("pca_covariance", _lib().pca_covariance(_ptr(Y), dt, n, m, ld, int(bool(input_is_centered)), _ptr(mean),
                                                   int(mode), _ptr(C), _ptr(ws), ws.numel(), _stream()))


def pca_jacobi_eigh(C, eigvals, V, tol: float, max_sweeps: int, fp64_angles: bool = True, info=None, ws=None,
                    overlap: bool = False, form: str = "auto"):
    """overlap: PCA_JACOBI_OVERLAP_REPLAY (one-workgroup form: eigenvectors
    formed while the sweeps run; bitwise the same results). form: "auto"
    (the library's choice by band count), "one_cu" (PCA_JACOBI_ONE_CU) or
    "block" (PCA_JACOBI_BLOCK)."""
    m = C.shape[0]
    if ws is None:
        ws = workspace(pca_workspace_size(PCA_OP_JACOBI, 2, m, max_sweeps=max_sweeps), C.device)
    flags = ((PCA_JACOBI_FP64_ANGLES if fp64_angles else 0) | (PCA_JACOBI_OVERLAP_REPLAY if overlap else 0)
             | JACOBI_FORMS[form])
    _check("pca_jacobi_eigh", _lib().pca_jacobi_eigh(_ptr(C), m, float(tol), int(max_sweeps), flags,
                                                     _ptr(eigvals), _ptr(V), _ptr(info), _ptr(ws), ws.numel(),
                                                     _stream()))


def pca_jacobi_eigh_noalloc(C, eigvals, V, tol: float, max_sweeps: int, fp64_angles: bool = True, info=None,
                            overlap: bool = False, form: str = "auto"):
    """pca_jacobi_eigh with the library's own device scratch array as the
    workspace (no allocation by the library or here)."""
    m = C.shape[0]
    flags = ((PCA_JACOBI_FP64_ANGLES if fp64_angles else 0) | (PCA_JACOBI_OVERLAP_REPLAY if overlap else 0)
             | JACOBI_FORMS[form])
    _check("pca_jacobi_eigh_noalloc",
           _lib().pca_jacobi_eigh_noalloc(_ptr(C), m, float(tol), int(max_sweeps), flags, _ptr(eigvals), _ptr(V),
                                          _ptr(info), _stream()))


def pca_project(Y, mean, V, k: int, Q, layout: str = "bip"):
    dt, n, m, ld = _cube(Y, layout)
    _check("pca_project", _lib().pca_project(_ptr(Y), dt, n, m, ld, _ptr(mean), _ptr(V), int(k), _ptr(Q),
                                             _stream()))


def _f32(name, t, shape):
    """A float32 device tensor of the given shape, contiguous (rows may be
    padded only where the C ABI takes a leading dimension)."""
    if t is None:
        return
    if t.dtype != torch.float32 or not t.is_cuda or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 device tensor of shape {tuple(shape)}")


def pca_backward(Y, mean, eigvals, V, k: int, dY, dQ=None, dEig=None, dVk=None, ws=None, layout: str = "bip"):
    """dY in the layout of Y: [pixels, bands] ("bip") or [bands, pixels] ("bsq")."""
    dt, n, m, ld = _cube(Y, layout)
    if dt not in (PCA_IN_F32, PCA_IN_F32_BSQ):
        raise ValueError("pca_backward needs a float32 cube")
    for name, t, shape in (("mean", mean, (m,)), ("eigvals", eigvals, (m,)), ("V", V, (m, m)),
                           ("dQ", dQ, (n, k)), ("dEig", dEig, (m,)), ("dVk", dVk, (m, k))):
        _f32(name, t, shape)
    want = (m, n) if dt == PCA_IN_F32_BSQ else (n, m)
    if dY.dtype != torch.float32 or dY.dim() != 2 or tuple(dY.shape) != want or dY.stride(1) != 1:
        raise ValueError(f"dY must be a float32 {list(want)} device tensor with unit stride along its second axis")
    if ws is None:
        ws = workspace(pca_workspace_size(PCA_OP_BACKWARD, n, m, k=k), Y.device)
    _check("pca_backward", _lib().pca_backward(_ptr(Y), dt, n, m, ld, _ptr(mean), _ptr(eigvals), _ptr(V), int(k),
                                               _ptr(dQ), _ptr(dEig), _ptr(dVk), _ptr(dY), dY.stride(0), _ptr(ws),
                                               ws.numel(), _stream()))


def pca_batched_workspace_size(cubes_host, n_cubes: int, mode: int, max_sweeps: int, tuning=None) -> int:
    out = _sz(0)
    _check("pca_batched_workspace_size",
           _lib().pca_batched_workspace_size(ctypes.cast(cubes_host, _vp), int(n_cubes), int(mode), int(max_sweeps),
                                             None if tuning is None else ctypes.cast(ctypes.pointer(tuning), _vp),
                                             ctypes.byref(out)))
    return int(out.value)


def pca_batched(cubes_host, cubes_dev, n_cubes: int, dt: int, mode: int, tol: float, max_sweeps: int,
                fp64_angles: bool, tuning, ws):
    _check("pca_batched",
           _lib().pca_batched(ctypes.cast(cubes_host, _vp), _ptr(cubes_dev), int(n_cubes), int(dt), int(mode),
                              float(tol), int(max_sweeps), int(bool(fp64_angles)),
                              None if tuning is None else ctypes.cast(ctypes.pointer(tuning), _vp), _ptr(ws),
                              ws.numel(), _stream()))


def set_wait_shift(shift: int):
    """Divide the bounds of the Jacobi kernels' waits by 2^shift (tests of the
    failure handling; 0 restores the defaults). Synchronises the device."""
    torch.cuda.synchronize()
    _check("pca_set_wait_shift", _lib().pca_set_wait_shift(int(shift)))


def new_info(device=None) -> torch.Tensor:
    """Device buffer for a pca_info (8-byte aligned)."""
    return torch.zeros(INFO_BYTES // 8, dtype=torch.float64, device=device or "cuda")


def read_info(info: torch.Tensor) -> dict:
    """Copy a device pca_info back and decode it (synchronises)."""
    raw = info.detach().cpu().numpy().tobytes()[:INFO_BYTES]
    return dict(zip(INFO_FIELDS, struct.unpack(INFO_FORMAT, raw)))
