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


_U32 = 2.0 ** -24              # unit roundoff of binary32


def _ulp16(y):
    """Spacing of binary16 values at magnitude y (subnormal spacing below 2^-14)."""
    return 2.0 ** (np.floor(np.log2(np.maximum(y, 2.0 ** -14))) - 10)


class LayerIndex:
    """Edges of each layer as a padded [rows, max degree] array (-1 = none)."""

    def __init__(self, code, layer_ptr):
        rp = np.asarray(code.row_ptr, dtype=np.int64)
        self.col = np.asarray(code.col_idx, dtype=np.int64)
        self.n = code.n
        self.layers = []
        for l0, l1 in zip(layer_ptr[:-1], layer_ptr[1:]):
            deg = rp[l0 + 1:l1 + 1] - rp[l0:l1]
            dmax = int(deg.max()) if deg.size else 0
            idx = np.full((l1 - l0, dmax), -1, dtype=np.int64)
            for q in range(dmax):
                has = deg > q
                idx[has, q] = rp[l0:l1][has] + q
            self.layers.append(idx)


def _message_bound(x_o, D, mask, w, c_out, algo):
    """Per edge of padded rows [rows, d]: bound on the difference between the
    binary16 message the binary32 side stores and the fp64 side's c_out, given
    the fp64 side's inputs x_o and bounds D on how far the binary32 side's
    inputs lie from them.
      min-sum: the exclusive min of |x| can only be taken at an input whose
        interval |x_k| +- D_k reaches below the smallest upper end of the
        others, so it moves by at most the largest D_k of those candidates;
        if an input's sign is uncertain (|x_k| <= D_k) the message moves by at
        most twice the min plus that amount; times the weight, plus the
        binary32 product's rounding;
      sum-product: the tanh rule has |d c / d x_k| <= 1 for every input, so the
        message moves by at most the sum of the other D_k, plus the binary32
        evaluation of phi (relative error below 1e-6 per evaluation, at most
        1e-6 * d absolute through the outer phi, whose slope times its argument
        is at most 1);
      then both sides round to binary16: at most one unit at the magnitude."""
    ax = np.abs(x_o)
    pre = np.zeros_like(ax)
    if algo == 1:
        lo = np.where(mask, ax - D, np.inf)
        hi = np.where(mask, ax + D, np.inf)
        amb = mask & (ax <= D)
        for q in range(x_o.shape[1]):
            others = mask.copy()
            others[:, q] = False
            hmin = np.where(others, hi, np.inf).min(axis=1, keepdims=True)
            cand = others & (lo <= hmin)
            dmax = np.where(cand, D, 0.0).max(axis=1)
            xmin = np.where(others, ax, np.inf).min(axis=1)
            xmin = np.where(np.isfinite(xmin), xmin, 0.0)
            sign_unsure = (amb & others).any(axis=1)
            ww = w[:, q]
            pre[:, q] = ww * (dmax + np.where(sign_unsure, 2.0 * xmin, 0.0)) + 2 * _U32 * ww * (xmin + dmax)
    else:
        dsum = np.where(mask, D, 0.0).sum(axis=1, keepdims=True)
        deg = mask.sum(axis=1, keepdims=True)
        pre = (dsum - np.where(mask, D, 0.0)) + 1e-6 * (deg + 1) * (1.0 + np.abs(c_out))
    return pre + _ulp16(np.abs(c_out) * (1 + 2.0 ** -10) + pre)


def layered_half_step_bound(lix, llr, c_in, post_in, c_out, w, algo=1):
    """Bound on how far one layered iteration run in binary32 with binary16
    messages (running posterior L; per edge x = L - c_old, c = the binary16
    rounding of the check rule over x, L = x + c, each step rounded to
    binary32) can lie from the same iteration in fp64 with binary16 messages,
    both starting from the messages c_in; post_in is the binary32 side's
    running posterior.  Forward error analysis, layer by layer, with D_k the
    bound on x_k: a posterior's bound enters every later x of its variable,
    a message's bound is that of _message_bound, and each binary32 operation
    adds its unit roundoff.  c_out are the fp64 side's new messages, w the
    per-edge weights, algo 0 sum-product / 1 min-sum.  Returns (bound per
    variable, bound per edge)."""
    col = lix.col
    post_o = np.asarray(llr, dtype=np.float64).copy()
    np.add.at(post_o, col, c_in)
    E = np.abs(np.asarray(post_in, dtype=np.float64) - post_o) * (1 + 1e-12) + 1e-300
    B = np.zeros(len(c_in))
    for idx in lix.layers:
        mask = idx >= 0
        e = np.where(mask, idx, 0)
        v = col[e]
        x_o = post_o[v] - c_in[e]
        D = E[v] + _U32 * (np.abs(x_o) + E[v])
        co = c_out[e]
        Be = _message_bound(x_o, D, mask, w[e], co, algo)
        newpost = x_o + co
        En = D + Be + _U32 * (np.abs(newpost) + D + Be)
        ee, vv = e[mask], v[mask]
        B[ee] = Be[mask]
        E[vv] = En[mask] * (1 + 1e-12)
        post_o[vv] = newpost[mask]
    return E, B


def layered_nms_half_step_bound(lix, llr, c_in, post_in, c_out, w):
    """layered_half_step_bound for min-sum."""
    return layered_half_step_bound(lix, llr, c_in, post_in, c_out, w, algo=1)


def flood_half_step_bound(allrows, llr, c_in, post_in, c_out, w, algo):
    """The same bound for one flooding iteration run in binary32 with binary16
    messages (x = L_post - c, c = the binary16 check rule over x, then
    L_post = L_ch + sum of the new messages in binary32) against fp64 with
    binary16 messages, from the same messages c_in; post_in is the binary32
    side's L_post before the iteration.  ``allrows`` is a LayerIndex with one
    layer holding every row."""
    col = allrows.col
    llr = np.asarray(llr, dtype=np.float64)
    post_o = llr.copy()
    np.add.at(post_o, col, c_in)
    E = np.abs(np.asarray(post_in, dtype=np.float64) - post_o) * (1 + 1e-12) + 1e-300
    idx = allrows.layers[0]
    mask = idx >= 0
    e = np.where(mask, idx, 0)
    v = col[e]
    x_o = post_o[v] - c_in[e]
    D = E[v] + _U32 * (np.abs(x_o) + E[v])
    B = np.zeros(len(c_in))
    B[e[mask]] = _message_bound(x_o, D, mask, w[e], c_out[e], algo)[mask]
    deg = np.bincount(col, minlength=allrows.n)
    mag = np.abs(llr).copy()
    np.add.at(mag, col, np.abs(c_out) + B)
    Ep = np.zeros(allrows.n)
    np.add.at(Ep, col, B)
    return (Ep + (deg + 1) * _U32 * mag) * (1 + 1e-12) + 1e-300, B
