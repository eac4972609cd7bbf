"""TEST INFRASTRUCTURE -- ctypes front of the fp64 C oracle (bp_oracle.c)."""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from pathlib import Path

import numpy as np

SP = 0
NMS = 1

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "bp_oracle.c"
_LIB = _HERE / "_bp_oracle.so"
_lib = None


def build(force: bool = True) -> Path:
    """Compile the oracle with gcc (-O2, no fast-math, OpenMP across frames)."""
    if force or not _LIB.exists() or _LIB.stat().st_mtime < _SRC.stat().st_mtime:
        tmp = _LIB.with_suffix(f".so.tmp{os.getpid()}")
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-Wall", "-o", str(tmp), str(_SRC), "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build(force=False)
        lib = C.CDLL(str(_LIB))
        P = C.c_void_p
        i32 = C.c_int32
        d = C.c_double
        lib.orc_syndrome.argtypes = [i32, i32, P, P, i32, P, P, P, P]
        lib.orc_decode.argtypes = [i32, i32, P, P, P, i32, i32, P, P, i32, i32, i32, i32, i32,
                                   d, P, d, P, P, P, P, P, P, P]
        lib.orc_nms_unrolled.argtypes = [i32, i32, P, P, P, i32, i32, P, P, P, i32, P, i32, P, P, P, P]
        lib.orc_flood_step.argtypes = [i32, i32, P, P, P, i32, P, P, i32, i32, i32, i32, d, P, d, P, P, P]
        lib.orc_decode_layered.argtypes = [i32, i32, P, P, P, i32, i32, P, i32, P, P, i32, i32, i32, i32, i32,
                                           d, P, d, P, P, P, P, P, P, P]
        lib.orc_layered_step.argtypes = [i32, i32, P, P, P, i32, i32, P, P, P, i32, i32, i32, i32, d, P, d, P, P]
        lib.orc_round_half.argtypes = [d]
        lib.orc_round_half.restype = d
        _lib = lib
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _code_arrays(code):
    rp = np.ascontiguousarray(code.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(code.col_idx, dtype=np.int32)
    et = np.ascontiguousarray(code.edge_type, dtype=np.uint8)
    return rp, ci, et


def round_half(x: float) -> float:
    return _load().orc_round_half(float(x))


def syndrome(code, bits, s_ref=None):
    """Syndromes [F, m] and unsatisfied-check counts [F] of bits [F, n]."""
    lib = _load()
    bits = np.ascontiguousarray(np.atleast_2d(bits), dtype=np.uint8)
    F = bits.shape[0]
    rp, ci, _ = _code_arrays(code)
    s_out = np.zeros((F, code.m), dtype=np.uint8)
    u = np.zeros(F, dtype=np.int32)
    sr = None if s_ref is None else np.ascontiguousarray(np.atleast_2d(s_ref), dtype=np.uint8)
    lib.orc_syndrome(code.n, code.m, _p(rp), _p(ci), F, _p(bits), _p(sr), _p(s_out), _p(u))
    return s_out, u


def decode(code, llr, syndrome=None, *, algo=SP, max_iter=50, early_stop=True,
           store_half=False, alpha=0.75, weights=None, clamp=50.0, trace=False, prec32=False):
    """Flooding BP over frames llr [F, n] (fp64, or every step rounded to
    binary32 with ``prec32``).  Returns a dict with bits, post, iters, ok and,
    with ``trace``, post_trace/scale_trace [F, T+1, n] and unsat_trace [F, T+1]."""
    lib = _load()
    llr = np.ascontiguousarray(np.atleast_2d(llr), dtype=np.float64)
    F, n = llr.shape
    if n != code.n:
        raise ValueError("llr width != code length")
    rp, ci, et = _code_arrays(code)
    syn = None if syndrome is None else np.ascontiguousarray(np.atleast_2d(syndrome), dtype=np.uint8)
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
    if w is not None and w.shape != (max_iter, code.n_types):
        raise ValueError("weights must be [max_iter, n_types]")
    out = dict(bits=np.zeros((F, n), np.uint8), post=np.zeros((F, n)),
               iters=np.zeros(F, np.int32), ok=np.zeros(F, np.uint8))
    tr = sc = ut = None
    if trace:
        tr = np.full((F, max_iter + 1, n), np.nan)
        sc = np.full((F, max_iter + 1, n), np.nan)
        ut = np.full((F, max_iter + 1), -1, dtype=np.int32)
    rc = lib.orc_decode(code.n, code.m, _p(rp), _p(ci), _p(et), code.n_types, F, _p(llr), _p(syn),
                        int(algo), int(max_iter), int(bool(early_stop)), int(bool(store_half)),
                        int(bool(prec32)), float(alpha), _p(w), float(clamp),
                        _p(out["bits"]), _p(out["post"]), _p(out["iters"]), _p(out["ok"]),
                        _p(tr), _p(sc), _p(ut))
    if rc:
        raise ValueError("oracle decode rejected its arguments")
    if trace:
        out.update(post_trace=tr, scale_trace=sc, unsat_trace=ut)
    return out


def nms_unrolled(code, llr, syndrome, truth, weights, want_dllr=False, prec32=False):
    """Unrolled normalized min-sum: loss, final posteriors, d loss / d weights
    [T, n_types] (and d loss / d llr).  ``prec32``: binary32 forward pass."""
    lib = _load()
    llr = np.ascontiguousarray(np.atleast_2d(llr), dtype=np.float64)
    F, n = llr.shape
    w = np.ascontiguousarray(weights, dtype=np.float64)
    T = w.shape[0]
    rp, ci, et = _code_arrays(code)
    syn = None if syndrome is None else np.ascontiguousarray(np.atleast_2d(syndrome), dtype=np.uint8)
    tb = np.ascontiguousarray(np.atleast_2d(truth), dtype=np.uint8)
    loss = np.zeros(1)
    post = np.zeros((F, n))
    dw = np.zeros_like(w)
    dl = np.zeros((F, n)) if want_dllr else None
    rc = lib.orc_nms_unrolled(code.n, code.m, _p(rp), _p(ci), _p(et), code.n_types, F, _p(llr),
                              _p(syn), _p(tb), T, _p(w), int(bool(prec32)), _p(loss), _p(post), _p(dw), _p(dl))
    if rc:
        raise ValueError("oracle nms_unrolled rejected its arguments")
    res = dict(loss=float(loss[0]), post=post, dw=dw)
    if want_dllr:
        res["dllr"] = dl
    return res


def flood_step(code, llr, syndrome, c2v, t, *, algo=SP, store_half=False, prec32=False, alpha=0.75,
               weights=None, clamp=50.0):
    """One flooding iteration of one frame from the state c2v(t) [E] (CSR edge
    order): returns (c2v(t+1), L_post(t+1)).  ``llr`` [n], ``syndrome`` [m] or None."""
    lib = _load()
    rp, ci, et = _code_arrays(code)
    llr = np.ascontiguousarray(llr, dtype=np.float64).reshape(-1)
    cin = np.ascontiguousarray(c2v, dtype=np.float64).reshape(-1)
    syn = None if syndrome is None else np.ascontiguousarray(syndrome, dtype=np.uint8).reshape(-1)
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
    cout = np.zeros(code.n_edges)
    post = np.zeros(code.n)
    rc = lib.orc_flood_step(code.n, code.m, _p(rp), _p(ci), _p(et), code.n_types, _p(llr), _p(syn), int(algo),
                            int(t), int(bool(store_half)), int(bool(prec32)), float(alpha), _p(w), float(clamp),
                            _p(cin), _p(cout), _p(post))
    if rc:
        raise ValueError("oracle flood_step rejected its arguments")
    return cout, post


def qc_layers(mb: int, Z: int) -> np.ndarray:
    """Layer boundaries of a quasi-cyclic code: layer i = the Z checks of block row i."""
    return (np.arange(mb + 1, dtype=np.int32) * Z).astype(np.int32)


def decode_layered(code, llr, syndrome=None, *, layers, algo=SP, max_iter=50, early_stop=True,
                   store_half=False, alpha=0.75, weights=None, clamp=50.0, trace=False, prec32=False):
    """Layered BP over frames llr [F, n]; ``layers`` = row boundaries [n_layers + 1]
    (rows of one layer share no variable).  Same outputs as :func:`decode`."""
    lib = _load()
    llr = np.ascontiguousarray(np.atleast_2d(llr), dtype=np.float64)
    F, n = llr.shape
    if n != code.n:
        raise ValueError("llr width != code length")
    rp, ci, et = _code_arrays(code)
    lp = np.ascontiguousarray(layers, dtype=np.int32)
    syn = None if syndrome is None else np.ascontiguousarray(np.atleast_2d(syndrome), dtype=np.uint8)
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
    if w is not None and w.shape != (max_iter, code.n_types):
        raise ValueError("weights must be [max_iter, n_types]")
    out = dict(bits=np.zeros((F, n), np.uint8), post=np.zeros((F, n)),
               iters=np.zeros(F, np.int32), ok=np.zeros(F, np.uint8))
    tr = sc = ut = None
    if trace:
        tr = np.full((F, max_iter + 1, n), np.nan)
        sc = np.full((F, max_iter + 1, n), np.nan)
        ut = np.full((F, max_iter + 1), -1, dtype=np.int32)
    rc = lib.orc_decode_layered(code.n, code.m, _p(rp), _p(ci), _p(et), code.n_types, len(lp) - 1, _p(lp), F,
                                _p(llr), _p(syn), int(algo), int(max_iter), int(bool(early_stop)),
                                int(bool(store_half)), int(bool(prec32)), float(alpha), _p(w), float(clamp),
                                _p(out["bits"]), _p(out["post"]), _p(out["iters"]), _p(out["ok"]),
                                _p(tr), _p(sc), _p(ut))
    if rc == -2:
        raise ValueError("two rows of one layer share a variable")
    if rc:
        raise ValueError("oracle decode_layered rejected its arguments")
    if trace:
        out.update(post_trace=tr, scale_trace=sc, unsat_trace=ut)
    return out


def layered_step(code, llr, syndrome, c2v, post, t, *, layers, algo=SP, store_half=False, prec32=False,
                 alpha=0.75, weights=None, clamp=50.0):
    """One layered iteration of one frame from the state (c2v [E], post [n]);
    returns the new (c2v, post).  In fp64 mode ``post`` is only an output."""
    lib = _load()
    rp, ci, et = _code_arrays(code)
    lp = np.ascontiguousarray(layers, dtype=np.int32)
    llr = np.ascontiguousarray(llr, dtype=np.float64).reshape(-1)
    c = np.array(c2v, dtype=np.float64).reshape(-1)
    p = np.array(post, dtype=np.float64).reshape(-1)
    syn = None if syndrome is None else np.ascontiguousarray(syndrome, dtype=np.uint8).reshape(-1)
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.float64)
    rc = lib.orc_layered_step(code.n, code.m, _p(rp), _p(ci), _p(et), code.n_types, len(lp) - 1, _p(lp),
                              _p(llr), _p(syn), int(algo), int(t), int(bool(store_half)), int(bool(prec32)),
                              float(alpha), _p(w), float(clamp), _p(c), _p(p))
    if rc == -2:
        raise ValueError("two rows of one layer share a variable")
    if rc:
        raise ValueError("oracle layered_step rejected its arguments")
    return c, p
