"""The C-ABI library loads and exports every entry point include/lbm.h declares
(no compute calls: runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")
LIB = os.path.join(ROOT, "paper_2208_14870_amd", "liblbm.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2208_14870_amd import build
        build.build(verbose=False)
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared()
    for n in ("lbm_create", "lbm_set_material", "lbm_set_body_force", "lbm_step",
              "lbm_solve_to_tol", "lbm_get_displacement", "lbm_batch_create", "lbm_batch_step"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_workspace_sizes_without_gpu(lib):
    lib.lbm_workspace_bytes.restype = ctypes.c_size_t
    lib.lbm_workspace_bytes.argtypes = [ctypes.c_int] * 4
    assert lib.lbm_workspace_bytes(0, 5, 0, 0) == 0
    assert lib.lbm_workspace_bytes(5, 5, 7, 0) == 0
    n = 1024
    b64 = lib.lbm_workspace_bytes(n, n, 0, 0)
    b32 = lib.lbm_workspace_bytes(n, n, 1, 0)
    b16 = lib.lbm_workspace_bytes(n, n, 2, 0)
    assert b64 > b32 > b16 >= n * n * (2 * 8 * 2 + 2 * 4 + 2 * 8)
    assert lib.lbm_workspace_bytes(n, n, 1, 1) >= b32 + n * n * (2 * 8 * 8 + 2 * 8)


def test_inplace_workspace_holds_one_population_buffer(lib):
    lib.lbm_workspace_bytes.restype = ctypes.c_size_t
    lib.lbm_workspace_bytes.argtypes = [ctypes.c_int] * 4
    lib.lbm_workspace_bytes_inplace.restype = ctypes.c_size_t
    lib.lbm_workspace_bytes_inplace.argtypes = [ctypes.c_int] * 3
    assert lib.lbm_workspace_bytes_inplace(0, 4, 1) == 0
    n = 2048
    for prec, esz in ((0, 8), (1, 4), (2, 2)):
        two = lib.lbm_workspace_bytes(n, n, prec, 0)
        one = lib.lbm_workspace_bytes_inplace(n, n, prec)
        # one buffer of 8 planes (padded) fewer
        assert two - one >= 8 * n * n * esz
        assert two - one <= 8 * (n * n + 2048) * esz + 256


def test_inplace_blocked_workspace_adds_the_halo_copies(lib):
    """The in-place workspace for blocked launches adds copies of 2R ring
    columns per strip and 2k rows per segment (eight planes each): FP32 8192^2
    at eight steps has strips of 112 columns (two per lane, ring 8) and
    segments of 128 rows (74 x 64 waves); FP64 strips of 48 columns and
    segments of 256 rows (171 x 32 waves)."""
    lib.lbm_workspace_bytes_inplace.restype = ctypes.c_size_t
    lib.lbm_workspace_bytes_inplace.argtypes = [ctypes.c_int] * 3
    lib.lbm_workspace_bytes_inplace_blocked.restype = ctypes.c_size_t
    lib.lbm_workspace_bytes_inplace_blocked.argtypes = [ctypes.c_int] * 5
    blocked = lib.lbm_workspace_bytes_inplace_blocked

    def f(nx, ny, prec, k, rows=0):
        return blocked(nx, ny, prec, k, rows)

    assert f(0, 4, 1, 8) == 0 and f(64, 64, 1, 1) == 0 and f(64, 64, 1, 9) == 0
    assert f(64, 64, 1, 8, -1) == 0
    n = 8192
    one = lib.lbm_workspace_bytes_inplace(n, n, 1)
    halo = 8 * (74 * 16 * n + 64 * 16 * n) * 4
    assert 0 <= f(n, n, 1, 8) - one - halo <= 512
    assert halo < 0.27 * 8 * n * n * 4
    # FP64: one column per lane (ring 8 of 64 columns: strips of 48)
    halo64 = 8 * (171 * 16 * n + 32 * 16 * n) * 8
    assert 0 <= f(n, n, 0, 8) - lib.lbm_workspace_bytes_inplace(n, n, 0) - halo64 <= 512
    # segments of 64 rows: twice the row copies
    halo_64rows = 8 * (74 * 16 * n + 128 * 16 * n) * 4
    assert 0 <= f(n, n, 1, 8, 64) - one - halo_64rows <= 512
    for prec in (0, 1, 2):
        sizes = [f(1000, 600, prec, k) for k in range(2, 9)]
        assert sizes == sorted(sizes) and sizes[0] > lib.lbm_workspace_bytes_inplace(1000, 600, prec)


def test_binding_has_no_cpu_fallback():
    """The Python binding raises when no GPU is visible instead of computing."""
    import torch
    from paper_2208_14870_amd import lbm
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(RuntimeError):
        lbm.Solver(8, 8)


def test_binding_fails_loudly_without_the_library(monkeypatch, tmp_path):
    """A missing liblbm.so is an error naming the build step, never a fallback."""
    from paper_2208_14870_amd import lbm
    monkeypatch.setattr(lbm, "_lib", None)
    monkeypatch.setattr(lbm, "LIB_PATH", str(tmp_path / "liblbm.so"))
    with pytest.raises(RuntimeError, match="not built"):
        lbm.load()
    with pytest.raises(RuntimeError, match="not built"):
        lbm.Solver(8, 8)
    with pytest.raises(RuntimeError, match="not built"):
        lbm.Batch(4, 1 << 20)
