"""CPU-side checks of the C ABI: every declared entry point is exported and
argument errors are rejected on the host before any HIP call."""
import ctypes as C
import re
from pathlib import Path

import numpy as np
import pytest

ROOT = Path(__file__).resolve().parents[1]
HEADER = ROOT / "include" / "cvqkd_recon.h"


def _declared_functions():
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in {"if", "while", "for", "sizeof"}))


@pytest.fixture(scope="module")
def lib():
    from paper_2108_08418_amd import _lib
    if not _lib.LIB_PATH.exists():
        pytest.fail("libcvqkd_recon.so is not built (run __graft_entry__.build())")
    return _lib.load()


def test_header_declares_the_four_hot_path_calls():
    names = _declared_functions()
    for n in ("slice_quantize", "slice_llr", "syndrome_check", "ldpc_decode_batch"):
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2108_08418_amd import _lib
    names = _declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), f"{n} not exported"
        assert n in _lib.SIGNATURES, f"{n} has no ctypes signature in the binding"


def test_version_and_error_text(lib):
    assert lib.cvr_version() >= 100
    assert lib.slice_quantize(None, -1, None, 4, 0, None, None) == -1
    assert b"n < 0" in lib.cvr_last_error()


def test_host_side_argument_checks(lib):
    th = np.array([0.3, 0.2, 0.5], np.float64)                  # not ascending
    assert lib.slice_quantize(None, 10, th.ctypes.data, 2, 0, None, None) == -1
    assert b"ascending" in lib.cvr_last_error()
    th_ok = np.array([-1.0, 0.0, 1.0])
    assert lib.slice_quantize(None, 10, th_ok.ctypes.data, 9, 0, None, None) == -1      # m_bits > 8
    assert lib.slice_quantize(None, 0, th_ok.ctypes.data, 2, 0, None, None) == 0        # n = 0: no-op
    assert lib.slice_llr(None, 10, 0.5, th_ok.ctypes.data, 2, 0, 1, 0b10, None, 1, None, None) == -1
    assert b"already" in lib.cvr_last_error()
    assert lib.slice_llr(None, 10, -1.0, th_ok.ctypes.data, 2, 0, 1, 0, None, 1, None, None) == -1
    assert lib.slice_llr(None, 10, 0.5, th_ok.ctypes.data, 2, 0, 1, 0, None, 7, None, None) == -1
    # soft-prior and binary-symmetric forms
    assert lib.slice_llr_prior(None, 10, 0.5, th_ok.ctypes.data, 2, 0, 1, 0b1, None, 0b1, None, 1, None, None) == -1
    assert b"overlap" in lib.cvr_last_error()
    assert lib.slice_llr_prior(None, 10, 0.5, th_ok.ctypes.data, 2, 0, 1, 0, None, 0b10, None, 1, None, None) == -1
    assert b"slice j" in lib.cvr_last_error()
    assert lib.slice_llr_prior(None, 10, 0.5, th_ok.ctypes.data, 2, 0, 0, 0, None, 0b100, None, 1, None, None) == -1
    assert lib.slice_llr_prior(None, 0, 0.5, th_ok.ctypes.data, 2, 0, 0, 0, None, 0b10, None, 1, None, None) == 0
    assert lib.slice_llr_bsc(None, 10, th_ok.ctypes.data, 2, 0, 0, 0.0, 1, None, None) == -1
    assert b"p must be" in lib.cvr_last_error()
    assert lib.slice_llr_bsc(None, 10, th_ok.ctypes.data, 2, 0, 0, 1.0, 1, None, None) == -1
    assert lib.slice_llr_bsc(None, 10, th_ok.ctypes.data, 2, 0, 2, 0.1, 1, None, None) == -1
    assert lib.slice_llr_bsc(None, 0, th_ok.ctypes.data, 2, 0, 1, 0.1, 1, None, None) == 0
    # one pass for slices j and j + 1
    assert lib.slice_llr_next(None, 10, 0.5, th_ok.ctypes.data, 2, 0, 1, 0, None, 1, None, None, None, None) == -1
    assert b"j + 1 < m_bits" in lib.cvr_last_error()
    assert lib.slice_llr_next(None, 10, 0.5, th_ok.ctypes.data, 2, 0, 0, 0b10, None, 1, None, None, None, None) == -1
    assert lib.slice_llr_next(None, 0, 0.5, th_ok.ctypes.data, 2, 0, 0, 0, None, 1, None, None, None, None) == 0
    assert lib.slice_llr_choose(None, None, None, 5, 1, None, None) == -1
    assert lib.slice_llr_choose(None, None, None, 0, 1, None, None) == 0
    # malformed CSR: columns not ascending / out of range / degree 0
    h = C.c_void_p()
    rp = np.array([0, 2, 4], np.int32)
    ci = np.array([1, 0, 2, 3], np.int32)
    assert lib.cvr_code_create_csr(4, 2, rp.ctypes.data, ci.ctypes.data, None, 1, C.byref(h)) == -1
    ci = np.array([0, 1, 2, 9], np.int32)
    assert lib.cvr_code_create_csr(4, 2, rp.ctypes.data, ci.ctypes.data, None, 1, C.byref(h)) == -1
    rp0 = np.array([0, 0, 4], np.int32)
    assert lib.cvr_code_create_csr(4, 2, rp0.ctypes.data, ci.ctypes.data, None, 1, C.byref(h)) == -1
    sh = np.array([[0, 5]], np.int32)                            # shift >= Z
    assert lib.cvr_code_create_qc(2, 1, 4, sh.ctypes.data, None, 1, C.byref(h)) == -1
    assert lib.syndrome_check(None, 1, None, None, None, None, None) == -1
    assert lib.ldpc_decode_batch(None, None, None, None, None, None, None, None, None, 0, None) == -1


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2108_08418_amd import _lib
    monkeypatch.setattr(_lib, "LIB_PATH", tmp_path / "missing.so")
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        _lib.load()


def test_binding_rejects_weights_that_do_not_match_the_batch():
    """The kernels read weights[t * n_types + type] for every t < T: the binding
    refuses a weight tensor of another size, dtype or layout before any call."""
    import torch
    from paper_2108_08418_amd import api
    ok = torch.zeros(20, 3, dtype=torch.float32)
    for bad, msg in ((torch.zeros(19, 3), "20 x 3"), (torch.zeros(20, 4), "20 x 3"),
                     (torch.zeros(20, 3, dtype=torch.float64), "float32"),
                     (torch.zeros(3, 20).t(), "contiguous"), (ok, "device")):
        with pytest.raises(ValueError, match=msg):
            api._check_weights(bad, 20, 3, "test")
    with pytest.raises(ValueError, match=">= 100"):
        api._check_len(torch.zeros(99, dtype=torch.float32), 100, torch.float32, "llr")
    with pytest.raises(ValueError, match="float32"):
        api._check_len(torch.zeros(100, dtype=torch.float64), 100, torch.float32, "llr")
