"""Parity at the benchmark workloads' full sizes, in the launch configurations
that bench.py times, on sampled outputs the oracle computes one by one, plus
properties checked on every frame.

* 2^27 Gaussian pairs at SNR 3 (16 equiprobable levels, 2048 sub-blocks of
  2^16 per coded slice): the benchmark's two-stage chain (slice 2 decoded,
  slice 3's LLRs picked by the decoded bits, slice 3 decoded) with
  sum-product by the persistent kernel at 1024 threads.
* The uneven batch: 4096 sub-blocks of the rate-0.0625 MET code at SNR 0.16
  (2176 x 4096, 1024 x 16384, 640 x 65536, 256 x 262144 bits), min-sum
  alpha 0.75 with binary16 messages, persistent kernel at 1024 threads.

Each batch is decoded in every shape the autotuner may pick for it: one
workgroup per CU (four rows per body), with and without the LDS posterior
cache, and 8 waves per SIMD.  The shapes must agree bit for bit before the
first one is checked against the oracle.

Rules as in test_gpu_decode: quantiser, syndromes and decisions bit-exact;
slice LLRs within one fp32 ulp of the fp64 oracle; SP posteriors within
1e-4 x (|L_ch| + sum |c2v|) of the fp64 oracle with bits, iteration counts
and ok flags exact on frames with margin; min-sum bit-exact against the
binary32 oracle."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2108_08418_amd import api, inputs
from tests._parity import compare_trace, has_margin

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _g(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _decode_in_shapes(batch, llr, syn, kw, shapes):
    """Decode with the persistent kernel at 1024 threads in each (min_waves,
    lds_cache_kb) shape; all outputs must be identical.  Returns the first."""
    first = None
    for mw, cache in shapes:
        print(f"  shape 1024/{mw}/{cache}", flush=True)
        p = api.Params(schedule=api.SCHED_PERSISTENT, wg_threads=1024, min_waves=mw, lds_cache_kb=cache, **kw)
        out = api.ldpc_decode_batch(batch, p, llr, syn)
        torch.cuda.synchronize()
        out = {k: out[k].clone() for k in ("bits", "post", "iters", "ok")}
        if first is None:
            first = out
            continue
        for k in first:
            assert torch.equal(out[k], first[k]), f"shape 1024/{mw}/{cache}: {k} differs from 1024/{shapes[0][0]}/{shapes[0][1]}"
    return first


def _within_ulp(got, ref):
    """fp32 output within one ulp of the fp64 value."""
    ref32 = ref.astype(np.float32)
    return bool((np.abs(got.astype(np.float64) - ref32) <= np.spacing(np.abs(ref32)).astype(np.float64)).all())


def _check_stage(csr, ref, f, iters, ok, bits, post, syn_f, rel):
    """One sampled sub-block of one stage against the oracle's decode: on a
    frame with margin, iteration count, status and decisions exact and the
    final posteriors within rel x scale.  Returns whether it had margin."""
    t_o = int(ref["iters"][0])
    if not has_margin(csr, ref["post_trace"][0], ref["scale_trace"][0], t_o, syn_f, rel):
        return False
    assert int(iters[f]) == t_o, f"frame {f}: iters {int(iters[f])} oracle {t_o}"
    assert bool(ok[f]) == bool(ref["ok"][0])
    np.testing.assert_array_equal(bits[f], ref["bits"][0])
    worst = compare_trace(post[f][None, :], ref["post_trace"][0][t_o][None, :], ref["scale_trace"][0][t_o][None, :],
                          0, rel)
    assert worst <= 1.0, f"frame {f}: posterior deviation {worst:.3g} x tolerance"
    return True


def test_recon_2p27_two_stage_chain_sampled_against_oracle():
    """The benchmark step at 2^27 pairs, as bench.py runs it: Bob's quantiser
    and the syndromes of slices 2 and 3; Alice's one-pass LLRs of slice 2 and
    of slice 3 for either value of slice 2; slice 2 decoded (sum-product, the
    persistent kernel at 1024 threads, in every shape the autotuner may pick);
    slice 3's LLRs picked by the decoded slice 2 and slice 3 decoded.  16
    sampled sub-blocks are followed through the oracle's own chain from their
    (x, y): slice-3 LLRs conditioned on the oracle's decoded slice 2."""
    print("[full size: 2^27 pairs, slices 2 and 3, SP, persistent 1024 threads]", flush=True)
    snr = 3.0
    sig = math.sqrt(1.0 / snr)
    th = inputs.equiprobable_thresholds(4, 1.0 + 1.0 / snr)
    N, n = 1 << 27, 1 << 16
    F = N // n
    x, y = inputs.gaussian_pairs(N, snr, seed=4242)
    xg, yg = _g(x), _g(y)
    rng = np.random.default_rng(17)
    idx = np.sort(rng.choice(N, 1 << 18, replace=False))
    idx_g = torch.from_numpy(idx).to(DEV)
    # Bob: quantiser and slices, syndromes of the coded slices (all sub-blocks in one call each)
    bob = api.slice_quantize(yg, th, 4)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(bob[:, idx_g].cpu().numpy(), oracle.quantize(y[idx], th, 4))
    qcs = {j: inputs.slice_code_spec(j, n) for j in (2, 3)}
    csrs = {j: qcs[j].to_csr() for j in (2, 3)}
    codes = {j: api.Code.from_qc(qcs[j]) for j in (2, 3)}
    syn = {j: api.syndrome_check(codes[j], bob[j].contiguous(), want_unsat=False)[0].view(-1) for j in (2, 3)}
    # Alice: disclosed slices, one pass for slice 2 and both conditional slice-3 LLRs
    alice = torch.zeros_like(bob)
    alice[0:2].copy_(bob[0:2])
    llr2, n30, n31 = api.slice_llr_next(xg, sig, th, 4, 2, 0b11, alice)
    kw = dict(algo=api.SP, max_iter=100, math=api.F32, store=api.F32)
    shapes = [(0, 0), (0, 150), (8, 0)]
    out2 = _decode_in_shapes(api.Batch.uniform(codes[2], F), llr2, syn[2], kw, shapes)
    alice[2].copy_(out2["bits"])
    llr3 = api.slice_llr_choose(n30, n31, alice[2])
    out3 = _decode_in_shapes(api.Batch.uniform(codes[3], F), llr3, syn[3], kw, shapes)
    alice[3].copy_(out3["bits"])
    # every frame of both stages: ok <=> the decisions satisfy Bob's syndrome
    res = {}
    for j, out in ((2, out2), (3, out3)):
        _, unsat = api.syndrome_check(codes[j], out["bits"], syn[j], want_syndrome=False)
        ok = out["ok"].cpu().numpy().astype(bool)
        iters = out["iters"].cpu().numpy()
        np.testing.assert_array_equal(ok, unsat.cpu().numpy() == 0)
        assert ((iters >= 0) & (iters <= 100)).all() and (iters[~ok] == 100).all()
        assert ok.mean() > 0.99, f"slice {j}: FER {1 - ok.mean():.3%}"
        res[j] = dict(ok=ok, iters=iters, bits=out["bits"].cpu().numpy().reshape(F, n),
                      post=out["post"].cpu().numpy().reshape(F, n), syn=syn[j].cpu().numpy().reshape(F, -1))
    L2 = llr2.cpu().numpy().reshape(F, n)
    L3 = llr3.cpu().numpy().reshape(F, n)
    rel = 1e-4
    frames = sorted({0, 1, F // 2, F - 1} | set(int(v) for v in rng.choice(F, 12, replace=False)))
    margin = {2: 0, 3: 0}
    for f in frames:
        sl = slice(f * n, (f + 1) * n)
        Sf = oracle.quantize(y[sl], th, 4)
        A = Sf.copy()
        A[2:] = 0
        syn_f = {j: oracle.syndrome(csrs[j], Sf[j][None, :])[0] for j in (2, 3)}
        for j in (2, 3):
            np.testing.assert_array_equal(res[j]["syn"][f], syn_f[j][0])
        L2f = oracle.slice_llr(x[sl], sig, th, 4, oracle.GRAY, 2, 0b11, A)
        assert _within_ulp(L2[f], L2f), f"frame {f}: slice-2 LLRs"
        ref2 = oracle.decode(csrs[2], L2f[None, :], syn_f[2], algo=oracle.SP, max_iter=100, trace=True)
        if _check_stage(csrs[2], ref2, f, res[2]["iters"], res[2]["ok"], res[2]["bits"], res[2]["post"],
                        syn_f[2][0], rel):
            margin[2] += 1
        A[2] = ref2["bits"][0]                       # the oracle's own decoded slice 2
        L3f = oracle.slice_llr(x[sl], sig, th, 4, oracle.GRAY, 3, 0b111, A)
        if np.array_equal(res[2]["bits"][f], ref2["bits"][0]):
            assert _within_ulp(L3[f], L3f), f"frame {f}: slice-3 LLRs"
            ref3 = oracle.decode(csrs[3], L3f[None, :], syn_f[3], algo=oracle.SP, max_iter=100, trace=True)
            if _check_stage(csrs[3], ref3, f, res[3]["iters"], res[3]["ok"], res[3]["bits"], res[3]["post"],
                            syn_f[3][0], rel):
                margin[3] += 1
    print(f"  sampled {len(frames)} sub-blocks; margin frames: slice 2 {margin[2]}, slice 3 {margin[3]}", flush=True)
    assert margin[2] >= 0.75 * len(frames) and margin[3] >= 0.75 * len(frames), margin


def test_uneven_met_batch_4096_frames_sampled_against_oracle():
    print("[full size: 4096 uneven MET frames, min-sum f16, persistent 1024 threads]", flush=True)
    sizes, counts = (4096, 16384, 65536, 262144), (2176, 1024, 640, 256)
    rng = np.random.default_rng(2108)
    order = rng.permutation(np.repeat(np.arange(len(sizes)), counts))
    qcs = [inputs.met_low_rate_spec(s) for s in sizes]
    csrs = [q.to_csr() for q in qcs]
    codes = [api.Code.from_qc(q) for q in qcs]
    frames, vo, co = [], 0, 0
    for c in order:
        frames.append((int(c), vo, co))
        vo += sizes[c]
        co += qcs[c].m
    batch = api.Batch(codes, frames)
    bits = inputs.random_bits(vo, seed=31)
    llr = inputs.bpsk_llr(bits, 1.0 / 0.16, seed=32).astype(np.float32)
    bits_g = _g(bits)
    syn = torch.empty(co, dtype=torch.uint8, device=DEV)
    for c, q in enumerate(qcs):
        ids = [i for i, fr in enumerate(frames) if fr[0] == c]
        vidx = torch.cat([torch.arange(frames[i][1], frames[i][1] + q.n, device=DEV) for i in ids])
        cidx = torch.cat([torch.arange(frames[i][2], frames[i][2] + q.m, device=DEV) for i in ids])
        s_c, _ = api.syndrome_check(codes[c], bits_g[vidx].contiguous(), want_unsat=False)
        syn[cidx] = s_c.view(-1)
    out = _decode_in_shapes(batch, _g(llr), syn,
                            dict(algo=api.NMS, max_iter=100, math=api.F32, store=api.F16, alpha=0.75),
                            [(0, 0), (0, 150), (8, -1)])
    syn_np = syn.cpu().numpy()
    ok = out["ok"].cpu().numpy().astype(bool)
    iters = out["iters"].cpu().numpy()
    dec = out["bits"].cpu().numpy()
    post = out["post"].cpu().numpy()
    # every frame: ok <=> its decisions satisfy its syndrome
    for c, q in enumerate(qcs):
        ids = [i for i, fr in enumerate(frames) if fr[0] == c]
        vidx = np.concatenate([np.arange(frames[i][1], frames[i][1] + q.n) for i in ids])
        cidx = np.concatenate([np.arange(frames[i][2], frames[i][2] + q.m) for i in ids])
        _, u = api.syndrome_check(codes[c], _g(dec[vidx]), _g(syn_np[cidx]), want_syndrome=False)
        np.testing.assert_array_equal(ok[ids], u.cpu().numpy() == 0)
    assert (iters[~ok] == 100).all()
    # sampled frames (first and last of each size) bit-exact against the binary32 oracle
    for c in range(len(sizes)):
        ids = np.nonzero(order == c)[0]
        for i in (int(ids[0]), int(ids[-1])):
            _, v0, c0 = frames[i]
            n, m = sizes[c], qcs[c].m
            syn_f, _ = oracle.syndrome(csrs[c], bits[v0:v0 + n][None, :])
            np.testing.assert_array_equal(syn_np[c0:c0 + m], syn_f[0])
            ref = oracle.decode(csrs[c], llr[v0:v0 + n][None, :].astype(np.float64), syn_f,
                                algo=oracle.NMS, alpha=float(np.float32(0.75)), max_iter=100, store_half=True,
                                prec32=True)
            assert int(iters[i]) == int(ref["iters"][0]), (i, n)
            assert int(ok[i]) == int(ref["ok"][0]), (i, n)
            np.testing.assert_array_equal(dec[v0:v0 + n], ref["bits"][0])
            np.testing.assert_array_equal(post[v0:v0 + n].astype(np.float64), ref["post"][0])
