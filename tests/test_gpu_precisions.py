"""GPU decoder precisions against the plain fp64 oracle (no binary32 mirror):
binary16 message storage for min-sum and sum-product, binary64 min-sum, and
the workspace-size error path."""
from __future__ import annotations


import numpy as np
import pytest
import torch

import oracle
from paper_2108_08418_amd import api, inputs
from tests._gpu_state import decoded_for
from tests._parity import LayerIndex, compare_trace, flood_half_step_bound, has_margin, layered_half_step_bound

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def _g(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _frames(qc, F, seed):
    bits = inputs.random_bits((F, qc.n), seed=seed)
    s2 = inputs.sigma2_from_ebn0(np.linspace(1.5, 3.0, F), 1.0 - qc.m / qc.n)
    llr = inputs.bpsk_llr(bits, s2, seed=seed + 1)
    syn, _ = oracle.syndrome(qc.to_csr(), bits)
    return llr, syn


def _decode(code, F, llr, syn, p):
    batch = api.Batch.uniform(code, F)
    mdt = torch.float64 if p.math == api.F64 else torch.float32
    tr = torch.full((p.max_iter + 1, batch.total_n), float("nan"), dtype=mdt, device=DEV)
    out = api.ldpc_decode_batch(batch, p, _g(llr.reshape(-1).astype(np.float64 if p.math == api.F64 else np.float32)),
                                _g(syn.reshape(-1)), trace=tr)
    torch.cuda.synchronize()
    res = {k: v.cpu().numpy() for k, v in out.items()}
    res["trace"] = tr.cpu().numpy().reshape(p.max_iter + 1, F, code.n).transpose(1, 0, 2)
    return res


def _half_units(scale, k):
    """k binary16 units in the last place at the magnitude of the scale."""
    return k * 2.0 ** (np.floor(np.log2(np.maximum(np.abs(scale), 2.0 ** -14))) - 10)


def _one_step_parity(qc, p, llr, syn, layered, T, algo):
    """From the decoder's own state after t iterations (t < T), one iteration of
    the fp64 oracle with binary16 storage emulated: the decoder's posteriors
    and stored messages after t + 1 iterations lie within the forward error
    bound of one binary32 iteration with binary16 messages from that state
    (tests/_parity.py), computed from the oracle's values.  The bound is a few
    binary16 units of the scale at most places: a stored message may round to
    the other binary16 neighbour in one precision, and the binary32 rounding
    of the posterior enters the next check rule; on the layered schedule,
    later layers of the iteration also read what earlier ones wrote."""
    csr = qc.to_csr()
    code = api.Code.from_qc(qc)
    lay = oracle.qc_layers(qc.mb, qc.Z)
    lix = LayerIndex(csr, lay if layered else np.array([0, csr.m], dtype=np.int32))
    kw = dict(algo=algo, store_half=True, alpha=float(np.float32(p.alpha)))
    wedge = np.full(csr.n_edges, float(np.float32(p.alpha)))
    worst_post = worst_msg = 0.0
    tight = []
    for f in range(llr.shape[0]):
        l64 = llr[f].astype(np.float32).astype(np.float64)
        post, c2v = decoded_for(code, qc, p, llr[f], syn[f], 0)
        for t in range(T):
            if layered:
                c_o, p_o = oracle.layered_step(csr, l64, syn[f], c2v, post, t, layers=lay, **kw)
                E, B = layered_half_step_bound(lix, l64, c2v, post, c_o, wedge, algo)
            else:
                c_o, p_o = oracle.flood_step(csr, l64, syn[f], c2v, t, **kw)
                E, B = flood_half_step_bound(lix, l64, c2v, post, c_o, wedge, algo)
            sc = np.abs(l64).copy()
            np.add.at(sc, csr.col_idx, np.abs(c_o))
            tight.append(float(np.median(E / _half_units(sc, 1.0))))
            post, c2v = decoded_for(code, qc, p, llr[f], syn[f], t + 1)
            worst_post = max(worst_post, float(np.max(np.abs(post - p_o) / E)))
            worst_msg = max(worst_msg, float(np.max(np.abs(c2v - c_o) / B)))
    assert worst_post <= 1.0, f"posterior deviation {worst_post:.3g} x its bound"
    assert worst_msg <= 1.0, f"message deviation {worst_msg:.3g} x its bound"
    assert max(tight) < 4.0, f"bound too loose to test anything: median {max(tight):.3g} binary16 units"


def _decisions_on_margin_frames(csr, res, ref, F, syn, rel=2.0 ** -4, min_margin=0.5):
    """Whole decodes: iteration counts, status and decisions equal on the frames
    whose oracle posteriors stay farther than rel x scale from zero where the
    stop decision depends on them (binary16 rounding differences grow over
    iterations, so the margin is wide)."""
    margin = 0
    for f in range(F):
        if has_margin(csr, ref["post_trace"][f], ref["scale_trace"][f], int(ref["iters"][f]), syn[f], rel):
            margin += 1
            assert int(res["iters"][f]) == int(ref["iters"][f]), f"frame {f}"
            assert res["ok"][f] == ref["ok"][f]
            np.testing.assert_array_equal(res["bits"].reshape(F, -1)[f], ref["bits"][f])
    assert margin >= min_margin * F, f"only {margin}/{F} frames with margin"


@pytest.mark.parametrize("sched", [api.SCHED_PERSISTENT, api.SCHED_LAYERED])
def test_nms_f16_against_plain_fp64_oracle(sched):
    """Min-sum with binary16 messages (math fp32) against the fp64 oracle with
    binary16 storage emulated and every other step in fp64 (not the binary32
    mode): one iteration at a time from the decoder's own state, within 2
    binary16 units of the scale (a stored message may round to the other
    binary16 neighbour in one precision: one unit of that message, and the
    messages of a variable sum to at most the scale); whole decodes agree in
    their decisions on frames with margin."""
    print(f"[NMS f16 vs fp64 oracle sched={sched}]", flush=True)
    layered = sched == api.SCHED_LAYERED
    qc = inputs.lambda_half_rate_spec(16384)
    csr = qc.to_csr()
    F = 8
    llr, syn = _frames(qc, F, seed=41)
    p = api.Params(algo=api.NMS, max_iter=30, math=api.F32, store=api.F16, alpha=0.8, schedule=sched)
    _one_step_parity(qc, p, llr[:3], syn[:3], layered, 12, oracle.NMS)
    res = _decode(api.Code.from_qc(qc), F, llr, syn, p)
    kw = dict(algo=oracle.NMS, alpha=float(np.float32(0.8)), max_iter=30, trace=True, store_half=True)
    ref = (oracle.decode_layered(csr, llr, syn, layers=oracle.qc_layers(qc.mb, qc.Z), **kw) if layered
           else oracle.decode(csr, llr, syn, **kw))
    _decisions_on_margin_frames(csr, res, ref, F, syn)


def test_sp_f16_storage_against_fp64_oracle():
    """Sum-product with binary16 messages (math fp32) against the fp64 oracle
    with binary16 storage, as the min-sum test: one iteration at a time within
    2 binary16 units of the scale, decisions of whole decodes on margin frames."""
    print("[SP f16 storage vs fp64 oracle]", flush=True)
    qc = inputs.lambda_half_rate_spec(16384)
    csr = qc.to_csr()
    F = 8
    llr, syn = _frames(qc, F, seed=43)
    p = api.Params(algo=api.SP, max_iter=30, math=api.F32, store=api.F16, schedule=api.SCHED_PERSISTENT)
    _one_step_parity(qc, p, llr[:3], syn[:3], False, 12, oracle.SP)
    res = _decode(api.Code.from_qc(qc), F, llr, syn, p)
    ref = oracle.decode(csr, llr, syn, algo=oracle.SP, max_iter=30, trace=True, store_half=True)
    # over whole decodes the oracle's binary32 mode (the decoder's arithmetic)
    # stays within 2^-9.5 of the scale of the fp64 mode on these frames: a
    # margin of 2^-6 leaves 8x room
    _decisions_on_margin_frames(csr, res, ref, F, syn, rel=2.0 ** -6)


@pytest.mark.parametrize("sched", [api.SCHED_PERSISTENT, api.SCHED_PASSES, api.SCHED_LAYERED])
def test_nms_f64_math_against_fp64_oracle(sched):
    """Min-sum in binary64 (fp64 messages) against the fp64 oracle within 1e-12
    of the scale per iteration; exact decisions on frames with margin."""
    print(f"[NMS f64 sched={sched}]", flush=True)
    qc = inputs.lambda_half_rate_spec(16384)
    csr = qc.to_csr()
    F = 6
    llr, syn = _frames(qc, F, seed=45)
    p = api.Params(algo=api.NMS, max_iter=30, math=api.F64, store=api.F64, alpha=0.8, schedule=sched)
    a32 = float(np.float32(0.8))      # the ABI carries alpha as binary32
    res = _decode(api.Code.from_qc(qc), F, llr, syn, p)
    if sched == api.SCHED_LAYERED:
        ref = oracle.decode_layered(csr, llr, syn, layers=oracle.qc_layers(qc.mb, qc.Z), algo=oracle.NMS,
                                    alpha=a32, max_iter=30, trace=True)
    else:
        ref = oracle.decode(csr, llr, syn, algo=oracle.NMS, alpha=a32, max_iter=30, trace=True)
    margin, worst = 0, 0.0
    for f in range(F):
        t_o, t_g = int(ref["iters"][f]), int(res["iters"][f])
        worst = max(worst, compare_trace(res["trace"][f], ref["post_trace"][f], ref["scale_trace"][f],
                                         min(t_o, t_g), 1e-12))
        if has_margin(csr, ref["post_trace"][f], ref["scale_trace"][f], t_o, syn[f], 1e-12):
            margin += 1
            assert t_g == t_o and res["ok"][f] == ref["ok"][f]
            np.testing.assert_array_equal(res["bits"].reshape(F, -1)[f], ref["bits"][f])
    assert worst <= 1.0, f"posterior deviation {worst:.3g} x tolerance"
    assert margin >= F - 1


def test_undersized_workspace_is_refused():
    """A workspace below cvr_decode_workspace_size returns CVR_ENOMEM before
    anything is enqueued; one of exactly that size decodes."""
    print("[workspace size]", flush=True)
    qc = inputs.lambda_half_rate_spec(4096)
    F = 3
    llr, syn = _frames(qc, F, seed=47)
    code = api.Code.from_qc(qc)
    batch = api.Batch.uniform(code, F)
    p = api.Params(algo=api.NMS, max_iter=20, math=api.F32, store=api.F16)
    need = api.decode_workspace_size(batch, p)
    small = torch.empty(need - 256, dtype=torch.uint8, device=DEV)
    with pytest.raises(api._lib.CvrError, match="CVR_ENOMEM"):
        api.ldpc_decode_batch(batch, p, _g(llr.reshape(-1).astype(np.float32)), _g(syn.reshape(-1)), workspace=small)
    exact = torch.empty(need, dtype=torch.uint8, device=DEV)
    out = api.ldpc_decode_batch(batch, p, _g(llr.reshape(-1).astype(np.float32)), _g(syn.reshape(-1)), workspace=exact)
    torch.cuda.synchronize()
    assert out["ok"].sum().item() >= 1
