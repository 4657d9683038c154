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
