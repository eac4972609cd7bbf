"""Parity at the benchmark workloads' full sizes, in the launch configurations
that bench.py times, on sampled outputs the oracle computes one by one, plus
properties checked on every frame.

* 2^27 Gaussian pairs at SNR 3 (16 equiprobable levels, 2048 sub-blocks of
  2^16 per coded slice), slice 2 decoded with sum-product by the persistent
  kernel at 1024 threads.
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


def test_recon_2p27_pairs_sampled_against_oracle():
    print("[full size: 2^27 pairs, slice 2, SP, persistent 1024 threads]", flush=True)
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
    # quantiser and slices
    S = api.slice_quantize(yg, th, 4)
    torch.cuda.synchronize()
    S_ref = oracle.quantize(y[idx], th, 4)
    np.testing.assert_array_equal(S[:, idx_g].cpu().numpy(), S_ref)
    # Bob's syndromes of slice 2, all 2048 sub-blocks in one call
    qc = inputs.slice_code_spec(2, n)
    csr = qc.to_csr()
    code = api.Code.from_qc(qc)
    syn, _ = api.syndrome_check(code, S[2].contiguous(), want_unsat=False)
    # Alice's LLRs of slice 2 given slices 0 and 1
    known = S.clone()
    known[2:] = 0
    llr = api.slice_llr(xg, sig, th, 4, 2, 0b11, known)
    torch.cuda.synchronize()
    A_ref = S_ref.copy()
    A_ref[2:] = 0

    def within_ulp(got, ref):                     # fp32 output within one ulp of the fp64 value
        ref32 = ref.astype(np.float32)
        return (np.abs(got.astype(np.float64) - ref32) <= np.spacing(np.abs(ref32)).astype(np.float64)).all()

    assert within_ulp(llr[idx_g].cpu().numpy(), oracle.slice_llr(x[idx], sig, th, 4, oracle.GRAY, 2, 0b11, A_ref))
    # the decoder in the benchmark's launch configuration
    batch = api.Batch.uniform(code, F)
    out = _decode_in_shapes(batch, llr, syn.view(-1), dict(algo=api.SP, max_iter=100, math=api.F32, store=api.F32),
                            [(0, 0), (0, 150), (8, 0)])
    # every frame: ok <=> its decisions satisfy Bob's syndrome; iteration counts in range
    _, unsat = api.syndrome_check(code, out["bits"], syn.view(-1), want_syndrome=False)
    ok = out["ok"].cpu().numpy().astype(bool)
    iters = out["iters"].cpu().numpy()
    np.testing.assert_array_equal(ok, unsat.cpu().numpy() == 0)
    assert ((iters >= 0) & (iters <= 100)).all() and (iters[~ok] == 100).all()
    assert ok.mean() > 0.99, f"FER {1 - ok.mean():.3%}"
    # sampled sub-blocks: the oracle's own chain from (x, y) of the sub-block
    syn_np = syn.cpu().numpy()
    L_np = llr.cpu().numpy().reshape(F, n)
    bits = out["bits"].cpu().numpy().reshape(F, n)
    post = out["post"].cpu().numpy().reshape(F, n)
    rel, margin = 1e-4, 0
    frames = [0, 1, F // 2, F - 1]
    for f in frames:
        sl = slice(f * n, (f + 1) * n)
        Sf = oracle.quantize(y[sl], th, 4)
        syn_f, _ = oracle.syndrome(csr, Sf[2][None, :])
        np.testing.assert_array_equal(syn_np[f], syn_f[0])
        Af = Sf.copy()
        Af[2:] = 0
        Lf = oracle.slice_llr(x[sl], sig, th, 4, oracle.GRAY, 2, 0b11, Af)
        assert within_ulp(L_np[f], Lf)
        ref = oracle.decode(csr, Lf[None, :], syn_f, algo=oracle.SP, max_iter=100, trace=True)
        t_o = int(ref["iters"][0])
        if has_margin(csr, ref["post_trace"][0], ref["scale_trace"][0], t_o, syn_f[0], rel):
            margin += 1
            assert int(iters[f]) == t_o
            assert bool(ok[f]) == bool(ref["ok"][0])
            np.testing.assert_array_equal(bits[f], ref["bits"][0])
            worst = compare_trace(post[f][None, :], ref["post_trace"][0][t_o][None, :],
                                  ref["scale_trace"][0][t_o][None, :], 0, rel)
            assert worst <= 1.0, f"frame {f}: posterior deviation {worst:.3g} x tolerance"
    assert margin >= 2, f"only {margin} of {len(frames)} sampled frames with margin"


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
