"""CPU-side checks of the boundary: the library loads and exports every symbol
include/msp.h declares; status strings; parameter defaults.  No compute calls
(no GPU here)."""
from __future__ import annotations

import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "msp.h")
LIB = os.path.join(ROOT, "paper_2508_08702_amd", "libmsp.so")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(msp_[a-z_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail(f"{LIB} missing: run `python -m paper_2508_08702_amd.build`")
    return C.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert "msp_enumerate" in names and "msp_reduce" in names
    for name in names:
        assert hasattr(lib, name), name


def test_binding_covers_the_header():
    import paper_2508_08702_amd as M
    assert set(M.EXPORTED) == set(declared_functions())
    for name in M.EXPORTED:
        assert callable(getattr(M, name))


def test_strerror_and_defaults(lib):
    import paper_2508_08702_amd as M
    assert M.msp_strerror(0) == "ok"
    assert "capacity" in M.msp_strerror(M.MSP_E_CAPACITY)
    assert M.msp_strerror(12345) == "unknown status"
    p = M.msp_params_default()
    assert p.N == 1024 and abs(p.delta - 0.99) < 1e-15 and p.eps == 1e-9
    assert p.split_depth == -1 and p.hoelder == 1 and p.onedir == 1
    assert p.disc_budget == -1 and p.bkz_block == 0 and p.bkz_tours == 4
    assert p.restarts == 1 and p.restart_seed == 1


def test_status_codes_match_header():
    import paper_2508_08702_amd as M
    txt = open(HEADER).read()
    for name, val in re.findall(r"(MSP_E_[A-Z_]+)\s*=\s*(-?\d+)", txt):
        assert getattr(M, name) == int(val), name


def test_context_without_gpu_fails_cleanly(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    lib.msp_ctx_create.argtypes = [C.c_int, C.POINTER(C.c_void_p)]
    rc = lib.msp_ctx_create(0, C.byref(h))
    assert rc != 0 and not h.value
