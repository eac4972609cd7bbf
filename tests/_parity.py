"""Shared helpers of the GPU parity tests (comparison rules, not arithmetic of
the method)."""
from __future__ import annotations

import numpy as np


def row_parity_unsat(code, L, s):
    """Per-check flag: parity of the hard decisions of L differs from s."""
    hard = (L < 0).astype(np.int64)
    rows = np.repeat(np.arange(code.m), np.diff(code.row_ptr))
    par = np.zeros(code.m, np.int64)
    np.add.at(par, rows, hard[code.col_idx])
    sref = np.zeros(code.m, np.int64) if s is None else s.astype(np.int64)
    return (par % 2) != sref


def row_all_robust(code, robust):
    rows = np.repeat(np.arange(code.m), np.diff(code.row_ptr))
    bad = np.zeros(code.m, np.int64)
    np.add.at(bad, rows, (~robust[code.col_idx]).astype(np.int64))
    return bad == 0


def has_margin(code, post_trace, scale_trace, t_stop, s, rel):
    """Frame margin: with |L_gpu - L_orc| <= rel * scale at every iteration,
    the GPU must take the same stop decision at every t <= t_stop.  True when
    every t < t_stop has an unsatisfied check whose variables all have
    |L_orc| > rel * scale, and at t_stop every variable does."""
    for t in range(t_stop + 1):
        L = post_trace[t]
        robust = np.abs(L) > rel * scale_trace[t]
        if t == t_stop:
            if not robust.all():
                return False
        else:
            uns = row_parity_unsat(code, L, s)
            if not (uns & row_all_robust(code, robust)).any():
                return False
    return True


def compare_trace(gpu_trace, orc_post_trace, orc_scale_trace, t_last, rel, abs_floor=0.0):
    """Max of |L_gpu - L_orc| / (rel * scale) over iterations 0..t_last (<= 1 passes)."""
    g = gpu_trace[: t_last + 1].astype(np.float64)
    o = orc_post_trace[: t_last + 1]
    sc = orc_scale_trace[: t_last + 1]
    err = np.abs(g - o)
    bound = rel * sc + abs_floor
    with np.errstate(invalid="ignore", divide="ignore"):
        ratio = np.where(bound > 0, err / bound, np.where(err > 0, np.inf, 0.0))
    return float(np.nanmax(ratio)) if ratio.size else 0.0
