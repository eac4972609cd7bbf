"""The forward error bounds the GPU parity tests use for decoders with binary16
messages, checked on the CPU: the oracle's binary32 modes (the arithmetic the
decoders run) stay within them of the fp64 modes, step by step, on the
layered and flooding schedules for min-sum and sum-product, and planted
mistakes in the binary32 side do not."""
from __future__ import annotations

import numpy as np

import oracle
from paper_2108_08418_amd import inputs
import pytest

from tests._parity import LayerIndex, _ulp16, flood_half_step_bound, layered_half_step_bound, layered_nms_half_step_bound


def _setup():
    qc = inputs.lambda_half_rate_spec(4096)
    csr = qc.to_csr()
    lay = oracle.qc_layers(qc.mb, qc.Z)
    bits = inputs.random_bits((3, qc.n), seed=61)
    s2 = inputs.sigma2_from_ebn0(np.linspace(1.5, 3.0, 3), 0.5)
    llr = inputs.bpsk_llr(bits, s2, seed=62).astype(np.float32).astype(np.float64)
    syn, _ = oracle.syndrome(csr, bits)
    return qc, csr, lay, llr, syn


def test_binary32_layered_steps_lie_within_the_bound():
    qc, csr, lay, llr, syn = _setup()
    lix = LayerIndex(csr, lay)
    a = float(np.float32(0.8))
    w = np.full(csr.n_edges, a)
    worst_p = worst_c = 0.0
    med = []
    for f in range(3):
        c = np.zeros(csr.n_edges)
        post = llr[f].copy()
        for t in range(10):
            c64, p64 = oracle.layered_step(csr, llr[f], syn[f], c, post, t, layers=lay, algo=oracle.NMS,
                                           store_half=True, alpha=a)
            E, B = layered_nms_half_step_bound(lix, llr[f], c, post, c64, w)
            c, post = oracle.layered_step(csr, llr[f], syn[f], c, post, t, layers=lay, algo=oracle.NMS,
                                          store_half=True, prec32=True, alpha=a)
            worst_p = max(worst_p, float(np.max(np.abs(post - p64) / E)))
            worst_c = max(worst_c, float(np.max(np.abs(c - c64) / B)))
            sc = np.abs(llr[f]).copy()
            np.add.at(sc, csr.col_idx, np.abs(c64))
            med.append(float(np.median(E / _ulp16(sc))))
    assert worst_p <= 1.0 and worst_c <= 1.0, (worst_p, worst_c)
    # the bound stays at the scale of a few binary16 units, so it can catch mistakes
    assert max(med) < 4.0, med


def test_a_planted_mistake_exceeds_the_bound():
    """The binary32 side run with the check rule's weight off by 1 % (a wrong
    constant), and with one message of the state dropped from the running
    posterior (a lost term): both leave the bound."""
    qc, csr, lay, llr, syn = _setup()
    lix = LayerIndex(csr, lay)
    a = float(np.float32(0.8))
    w = np.full(csr.n_edges, a)
    c = np.zeros(csr.n_edges)
    post = llr[0].copy()
    for t in range(3):
        c, post = oracle.layered_step(csr, llr[0], syn[0], c, post, t, layers=lay, algo=oracle.NMS,
                                      store_half=True, prec32=True, alpha=a)
    c64, p64 = oracle.layered_step(csr, llr[0], syn[0], c, post, 3, layers=lay, algo=oracle.NMS,
                                   store_half=True, alpha=a)
    E, B = layered_nms_half_step_bound(lix, llr[0], c, post, c64, w)
    c_bad, p_bad = oracle.layered_step(csr, llr[0], syn[0], c, post, 3, layers=lay, algo=oracle.NMS,
                                       store_half=True, prec32=True, alpha=float(np.float32(0.808)))
    assert np.max(np.abs(p_bad - p64) / E) > 1.0
    post_lost = post.copy()
    post_lost[csr.col_idx[5]] -= c[5]
    c_bad, p_bad = oracle.layered_step(csr, llr[0], syn[0], c, post_lost, 3, layers=lay, algo=oracle.NMS,
                                       store_half=True, prec32=True, alpha=a)
    assert np.max(np.abs(p_bad - p64) / E) > 1.0


@pytest.mark.parametrize("layered,algo", [(False, oracle.SP), (False, oracle.NMS), (True, oracle.NMS)])
def test_binary32_steps_within_the_bound_both_schedules(layered, algo):
    """(Layered sum-product is not bounded this way: the sum of the tanh rule's
    slopes compounds from layer to layer, and the bound loses all use.)"""
    qc, csr, lay, llr, syn = _setup()
    lix = LayerIndex(csr, lay if layered else np.array([0, csr.m], dtype=np.int32))
    a = float(np.float32(0.8))
    w = np.full(csr.n_edges, a)
    worst_p = worst_c = 0.0
    med = []
    for f in range(2):
        c = np.zeros(csr.n_edges)
        post = llr[f].copy()
        for t in range(8):
            kw = dict(algo=algo, store_half=True, alpha=a)
            if layered:
                c64, p64 = oracle.layered_step(csr, llr[f], syn[f], c, post, t, layers=lay, **kw)
                E, B = layered_half_step_bound(lix, llr[f], c, post, c64, w, algo)
                c, post = oracle.layered_step(csr, llr[f], syn[f], c, post, t, layers=lay, prec32=True, **kw)
            else:
                c64, p64 = oracle.flood_step(csr, llr[f], syn[f], c, t, **kw)
                E, B = flood_half_step_bound(lix, llr[f], c, post, c64, w, algo)
                c, post = oracle.flood_step(csr, llr[f], syn[f], c, t, prec32=True, **kw)
            worst_p = max(worst_p, float(np.max(np.abs(post - p64) / E)))
            worst_c = max(worst_c, float(np.max(np.abs(c - c64) / B)))
            sc = np.abs(llr[f]).copy()
            np.add.at(sc, csr.col_idx, np.abs(c64))
            med.append(float(np.median(E / _ulp16(sc))))
    assert worst_p <= 1.0 and worst_c <= 1.0, (worst_p, worst_c)
    assert max(med) < 4.0, med


@pytest.mark.parametrize("algo", [oracle.SP, oracle.NMS])
def test_flooding_planted_mistake_exceeds_the_bound(algo):
    """A flooding step whose binary32 side starts from a posterior missing one
    message (a lost term in the variable sum) leaves the bound."""
    qc, csr, lay, llr, syn = _setup()
    lix = LayerIndex(csr, np.array([0, csr.m], dtype=np.int32))
    a = float(np.float32(0.8))
    w = np.full(csr.n_edges, a)
    c = np.zeros(csr.n_edges)
    post = llr[0].copy()
    for t in range(3):
        c, post = oracle.flood_step(csr, llr[0], syn[0], c, t, algo=algo, store_half=True, prec32=True, alpha=a)
    c64, p64 = oracle.flood_step(csr, llr[0], syn[0], c, 3, algo=algo, store_half=True, alpha=a)
    E, B = flood_half_step_bound(lix, llr[0], c, post, c64, w, algo)
    # the binary32 side with the weight 1 % off (min-sum) or the message clamp
    # at 5 instead of 50 (sum-product): wrong constants
    kw = dict(alpha=float(np.float32(0.808))) if algo == oracle.NMS else dict(alpha=a, clamp=5.0)
    c_bad, p_bad = oracle.flood_step(csr, llr[0], syn[0], c, 3, algo=algo, store_half=True, prec32=True, **kw)
    assert np.max(np.abs(p_bad - p64) / E) > 1.0 or np.max(np.abs(c_bad - c64) / B) > 1.0
