"""The C ABI library loads on a machine without a GPU, exports every entry
point that include/pca.h declares, and rejects bad arguments before touching
the device."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pca.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2403_18321_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        from paper_2403_18321_amd import build_lib
        build_lib.build(verbose=False)
    return L


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pca_[a-z0-9_]+)\s*\(", text)))


def test_header_symbols_exported(lib):
    names = declared_functions()
    assert "pca_covariance" in names and "pca_jacobi_eigh" in names
    so = ctypes.CDLL(lib.LIB_PATH)
    for name in names:
        assert hasattr(so, name), f"{name} declared in pca.h but not exported"
    assert set(names) <= set(lib.EXPORTS)
    assert "pca_backward" in names


def test_status_strings(lib):
    so = lib.library()
    for code in range(5):
        assert so.pca_status_string(code).startswith(b"PCA_")


def test_workspace_sizes(lib):
    L = lib
    a = L.pca_workspace_size(L.PCA_OP_COVARIANCE, 1 << 20, 224, mode=L.PCA_COV_BF16X3)
    b = L.pca_workspace_size(L.PCA_OP_COVARIANCE, 1 << 16, 224)
    assert a >= b > 0
    assert L.pca_workspace_size(L.PCA_OP_COVARIANCE, 1 << 20, 224, mode=L.PCA_COV_FP16X3) == a
    j = L.pca_workspace_size(L.PCA_OP_JACOBI, 2, 224, max_sweeps=30)
    assert j >= 30 * 223 * 112 * 8
    assert L.pca_workspace_size(L.PCA_OP_PROJECT, 100, 10) == 0
    g = L.pca_workspace_size(L.PCA_OP_BACKWARD, 1 << 16, 128, k=8)
    assert g >= (128 + 8 + 1) * 128 * 4 + 128 * 8 * 8
    with pytest.raises(L.PCAError):
        L.pca_workspace_size(L.PCA_OP_BACKWARD, 1 << 16, 128, k=129)
    with pytest.raises(L.PCAError):
        L.pca_workspace_size(L.PCA_OP_COVARIANCE, 100, 257)
    with pytest.raises(L.PCAError):
        L.pca_workspace_size(L.PCA_OP_COVARIANCE, 1, 16)


def test_invalid_arguments_rejected_on_host(lib):
    so = lib.library()
    ARG = lib.PCA_ERR_ARG
    null = ctypes.c_void_p(0)
    fake = ctypes.c_void_p(4096)     # never dereferenced: checks fail first
    # NULL cube.
    assert so.pca_covariance(null, 0, 100, 8, 8, 0, null, 0, fake, fake, 1 << 20, null) == ARG
    # Too many bands, too few pixels, ld < bands, bad mode, bad dtype.
    assert so.pca_covariance(fake, 0, 100, 257, 257, 0, null, 0, fake, fake, 1 << 20, null) == ARG
    assert so.pca_covariance(fake, 0, 1, 8, 8, 0, null, 0, fake, fake, 1 << 20, null) == ARG
    assert so.pca_covariance(fake, 0, 100, 8, 7, 0, null, 0, fake, fake, 1 << 20, null) == ARG
    assert so.pca_covariance(fake, 0, 100, 8, 8, 0, null, 7, fake, fake, 1 << 20, null) == ARG
    assert so.pca_covariance(fake, 0, 100, 8, 8, 0, null, lib.PCA_COV_FP16X3 + 1, fake, fake, 1 << 20, null) == ARG
    assert so.pca_covariance(fake, 5, 100, 8, 8, 0, null, 0, fake, fake, 1 << 20, null) == ARG
    # Workspace too small.
    assert so.pca_covariance(fake, 0, 100000, 64, 64, 0, null, 0, fake, fake, 256,
                             null) == lib.PCA_ERR_WORKSPACE
    # Band-sequential: the band stride must cover the pixels (not the bands).
    assert so.pca_covariance(fake, lib.PCA_IN_F32_BSQ, 100, 8, 99, 0, null, 0, fake, fake, 1 << 20, null) == ARG
    assert so.pca_covariance(fake, lib.PCA_IN_U16_BSQ, 100, 8, 8, 0, null, 0, fake, fake, 1 << 20, null) == ARG
    assert so.pca_project(fake, lib.PCA_IN_F32_BSQ, 100, 8, 50, null, fake, 2, fake, null) == ARG
    assert so.pca_center(fake, lib.PCA_IN_F32_BSQ, 100, 8, 100, fake, fake, 8, fake, 1 << 20, null) == ARG
    assert so.pca_covariance(fake, 4, 100, 8, 100, 0, null, 0, fake, fake, 1 << 20, null) == ARG
    # Jacobi: negative tolerance, too many bands, misaligned workspace, an
    # unknown flag bit, both forms at once.
    assert so.pca_jacobi_eigh(fake, 8, -1.0, 10, 1, fake, fake, null, fake, 1 << 20, null) == ARG
    assert so.pca_jacobi_eigh(fake, 8, 1e-6, 10, 16, fake, fake, null, fake, 1 << 20, null) == ARG
    assert so.pca_jacobi_eigh(fake, 8, 1e-6, 10, lib.PCA_JACOBI_ONE_CU | lib.PCA_JACOBI_BLOCK, fake, fake, null,
                              fake, 1 << 20, null) == ARG
    assert so.pca_jacobi_eigh(fake, 8, 1e-6, 10, -1, fake, fake, null, fake, 1 << 20, null) == ARG
    assert so.pca_jacobi_eigh(fake, 300, 1e-6, 10, 1, fake, fake, null, fake, 1 << 20, null) == ARG
    assert so.pca_jacobi_eigh(fake, 8, 1e-6, 10, 1, fake, fake, null, ctypes.c_void_p(4100), 1 << 20,
                              null) == ARG
    # The no-allocation form: a request larger than its fixed device array,
    # and bad sizes, are refused before any device call.
    na = so.pca_jacobi_eigh_noalloc
    na.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    assert na(fake, 256, 1e-6, 100000, 1, fake, fake, null, null) == lib.PCA_ERR_WORKSPACE
    assert na(fake, 300, 1e-6, 10, 1, fake, fake, null, null) == ARG
    assert na(fake, 8, 1e-6, -1, 1, fake, fake, null, null) == ARG
    # Projection: k out of range.
    assert so.pca_project(fake, 0, 100, 8, 8, null, fake, 0, fake, null) == ARG
    assert so.pca_project(fake, 0, 100, 8, 8, null, fake, 9, fake, null) == ARG
    # Wait shift out of range (checked before any device call).
    assert so.pca_set_wait_shift(-1) == ARG and so.pca_set_wait_shift(41) == ARG
    # Backward: k out of range, ld_dy < bands, NULL dY, workspace too small,
    # a uint16 cube, a band-sequential dY stride below the pixel count.
    bw = so.pca_backward
    F32, BSQ = lib.PCA_IN_F32, lib.PCA_IN_F32_BSQ
    assert bw(fake, F32, 100, 8, 8, fake, fake, fake, 0, null, null, null, fake, 8, fake, 1 << 20, null) == ARG
    assert bw(fake, F32, 100, 8, 8, fake, fake, fake, 9, null, null, null, fake, 8, fake, 1 << 20, null) == ARG
    assert bw(fake, F32, 100, 8, 8, fake, fake, fake, 2, null, null, null, fake, 7, fake, 1 << 20, null) == ARG
    assert bw(fake, F32, 100, 8, 8, fake, fake, fake, 2, null, null, null, null, 8, fake, 1 << 20, null) == ARG
    assert bw(fake, F32, 100, 8, 8, fake, fake, fake, 2, fake, null, null, fake, 8, fake, 256,
              null) == lib.PCA_ERR_WORKSPACE
    assert bw(fake, lib.PCA_IN_U16, 100, 8, 8, fake, fake, fake, 2, null, null, null, fake, 8, fake, 1 << 20,
              null) == ARG
    assert bw(fake, BSQ, 100, 8, 100, fake, fake, fake, 2, null, null, null, fake, 99, fake, 1 << 20, null) == ARG


def test_batched_arguments_rejected_on_host(lib):
    so = lib.library()
    ARG = lib.PCA_ERR_ARG
    null = ctypes.c_void_p(0)
    fake = 4096
    arr = (lib.PCACube * 2)()
    arr[0] = lib.PCACube(fake, 1000, 64, 64, 5, fake, fake, fake, fake, 0)
    arr[1] = lib.PCACube(fake, 5000, 37, 37, 3, fake, fake, fake, fake, 0)
    cubes = ctypes.cast(ctypes.pointer(arr), ctypes.c_void_p)
    dev = ctypes.c_void_p(fake)
    ws = ctypes.c_void_p(fake)
    need = lib.pca_batched_workspace_size(ctypes.pointer(arr), 2, 0, 30)
    assert need > 0
    ok = lambda *a: so.pca_batched(*a)
    # No device copy of the descriptors, empty batch, bad mode.
    assert ok(cubes, null, 2, 0, 0, 1e-6, 30, 1, null, ws, need, null) == ARG
    assert ok(cubes, dev, 0, 0, 0, 1e-6, 30, 1, null, ws, need, null) == ARG
    assert ok(cubes, dev, 2, 0, 9, 1e-6, 30, 1, null, ws, need, null) == ARG
    # Workspace too small.
    assert ok(cubes, dev, 2, 0, 0, 1e-6, 30, 1, null, ws, need - 1, null) == lib.PCA_ERR_WORKSPACE
    # A cube with k > bands.
    arr[1].k = 40
    assert ok(cubes, dev, 2, 0, 0, 1e-6, 30, 1, null, ws, need, null) == ARG
    arr[1].k = 3
    # Band-sequential: these cubes' strides (64, 37) are below their pixel
    # counts, so read as band rows they would overlap.
    assert ok(cubes, dev, 2, lib.PCA_IN_F32_BSQ, 0, 1e-6, 30, 1, null, ws, need, null) == ARG
    # Tuning: chunk not a multiple of 32.
    t = lib.PCABatchTuning(100, 4)
    assert so.pca_batched(cubes, dev, 2, 0, 0, 1e-6, 30, 1, ctypes.cast(ctypes.pointer(t), ctypes.c_void_p), ws,
                          need, null) == ARG
