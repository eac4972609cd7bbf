"""Parity at the benchmark workloads' full sizes, in the launch configurations
that bench.py times, on sampled outputs the oracle computes one by one, plus
properties checked on every frame.

* 2^27 Gaussian pairs at SNR 3 (16 equiprobable levels, 2048 sub-blocks of
  2^16 per coded slice): the benchmark's two-stage chain (slice 2 decoded,
  slice 3's LLRs picked by the decoded bits, slice 3 decoded) with each of
  the benchmark's five decoders: sum-product on the layered schedule (the
  headline), flooding sum-product (persistent kernel at 1024 threads),
  learned min-sum with binary16 messages on the flooding (persistent kernel)
  and on the layered schedule, and learned min-sum on slice 2 with
  sum-product on slice 3 (layered).
* The uneven batch: 4096 sub-blocks of the rate-0.0625 MET code at SNR 0.16
  (2176 x 4096, 1024 x 16384, 640 x 65536, 256 x 262144 bits), min-sum
  alpha 0.75 with binary16 messages, persistent kernel at 1024 threads.

Each batch is decoded in every shape the autotuner may pick for it (workgroup
size, LDS posterior cache, waves per SIMD).  The shapes must agree bit for bit
before the first one is checked against the oracle.

Rules as in test_gpu_decode and test_gpu_layered: quantiser, syndromes and
decisions bit-exact; slice LLRs within one fp32 ulp of the fp64 oracle;
flooding SP posteriors within 1e-4 x (|L_ch| + sum |c2v|) of the fp64 oracle
with bits, iteration counts and ok flags exact on frames with margin; layered
SP exact on frames with a margin of 2^-6 of the scale, and within 1e-4 of the
scale one iteration at a time from the decoder's own state; min-sum bit-exact
against the binary32 oracle."""
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


def _decode_in_shapes(batch, llr, syn, kw, shapes, schedule=None):
    """Decode once per launch shape (dicts of Params launch knobs, by default
    the persistent kernel at 1024 threads with (min_waves, lds_cache_kb));
    all outputs must be identical.  Returns the first."""
    first = None
    for sh in shapes:
        knobs = sh if isinstance(sh, dict) else dict(wg_threads=1024, min_waves=sh[0], lds_cache_kb=sh[1])
        print(f"  shape {knobs}", flush=True)
        p = api.Params(schedule=api.SCHED_PERSISTENT if schedule is None else schedule, **knobs, **kw)
        out = api.ldpc_decode_batch(batch, p, llr, syn)
        torch.cuda.synchronize()
        api.check_abandoned(out)
        out = {k: out[k].clone() for k in ("bits", "post", "iters", "ok")}
        if first is None:
            first = out
            continue
        for k in first:
            assert torch.equal(out[k], first[k]), f"shape {knobs}: {k} differs from {shapes[0]}"
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


def _check_exact(ref, f, iters, ok, bits, post):
    """One sampled sub-block bit-exact against the oracle's binary32 mode."""
    assert int(iters[f]) == int(ref["iters"][0]), f"frame {f}: iters {int(iters[f])} oracle {int(ref['iters'][0])}"
    assert bool(ok[f]) == bool(ref["ok"][0]), f"frame {f}"
    np.testing.assert_array_equal(bits[f], ref["bits"][0])
    np.testing.assert_array_equal(post[f].astype(np.float64), ref["post"][0])
    return True


@pytest.fixture(scope="module")
def recon_2p27():
    """The benchmark step's inputs at 2^27 pairs, SNR 3, 16 equiprobable Gray
    levels, 2048 sub-blocks of 2^16: Bob's slices and the syndromes of slices
    2 and 3 (one call each); Alice's one-pass LLRs of slice 2 and of slice 3
    for either value of slice 2.  Checked here: the quantiser on 2^18 sampled
    pairs and the syndromes of the sampled sub-blocks."""
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
    bob = api.slice_quantize(yg, th, 4)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(bob[:, idx_g].cpu().numpy(), oracle.quantize(y[idx], th, 4))
    qcs = {j: inputs.slice_code_spec(j, n) for j in (2, 3)}
    csrs = {j: qcs[j].to_csr() for j in (2, 3)}
    codes = {j: api.Code.from_qc(qcs[j]) for j in (2, 3)}
    syn = {j: api.syndrome_check(codes[j], bob[j].contiguous(), want_unsat=False)[0].view(-1) for j in (2, 3)}
    alice = torch.zeros_like(bob)
    alice[0:2].copy_(bob[0:2])
    llr2, n30, n31 = api.slice_llr_next(xg, sig, th, 4, 2, 0b11, alice)
    frames = sorted({0, 1, F // 2, F - 1} | set(int(v) for v in rng.choice(F, 12, replace=False)))
    syn_np = {j: syn[j].cpu().numpy().reshape(F, -1) for j in (2, 3)}
    Sf = {}
    for f in frames:
        sl = slice(f * n, (f + 1) * n)
        Sf[f] = oracle.quantize(y[sl], th, 4)
        for j in (2, 3):
            np.testing.assert_array_equal(syn_np[j][f], oracle.syndrome(csrs[j], Sf[f][j][None, :])[0][0])
    del xg, yg
    return dict(snr=snr, sig=sig, th=th, N=N, n=n, F=F, x=x, qcs=qcs, csrs=csrs, codes=codes, syn=syn,
                syn_np=syn_np, bob=bob, alice=alice, llr2=llr2, n30=n30, n31=n31, frames=frames, Sf=Sf)


def _run_chain(R, kw, shapes, schedule=None, kw3=None):
    """Slice 2 decoded in every shape, slice 3's LLRs picked by the decoded
    bits, slice 3 decoded in every shape; every frame of both stages: ok <=>
    the decisions satisfy Bob's syndrome.  Returns per-stage numpy outputs and
    Alice's LLRs of both stages."""
    F, n = R["F"], R["n"]
    alice = R["alice"].clone()
    out2 = _decode_in_shapes(api.Batch.uniform(R["codes"][2], F), R["llr2"], R["syn"][2], kw, shapes, schedule)
    alice[2].copy_(out2["bits"])
    llr3 = api.slice_llr_choose(R["n30"], R["n31"], alice[2])
    out3 = _decode_in_shapes(api.Batch.uniform(R["codes"][3], F), llr3, R["syn"][3], kw if kw3 is None else kw3,
                             shapes, schedule)
    res = {}
    T = {2: kw["max_iter"], 3: (kw if kw3 is None else kw3)["max_iter"]}
    for j, out in ((2, out2), (3, out3)):
        _, unsat = api.syndrome_check(R["codes"][j], out["bits"], R["syn"][j], want_syndrome=False)
        ok = out["ok"].cpu().numpy().astype(bool)
        iters = out["iters"].cpu().numpy()
        np.testing.assert_array_equal(ok, unsat.cpu().numpy() == 0)
        assert ((iters >= 0) & (iters <= T[j])).all() and (iters[~ok] == T[j]).all()
        res[j] = dict(ok=ok, iters=iters, bits=out["bits"].cpu().numpy().reshape(F, n),
                      post=out["post"].cpu().numpy().reshape(F, n))
    res["L2"] = R["llr2"].cpu().numpy().reshape(F, n)
    res["L3"] = llr3.cpu().numpy().reshape(F, n)
    return res


def _follow_sampled(R, res, decode_ref, check):
    """The sampled sub-blocks through the oracle's own chain from (x, y):
    slice-2 LLRs from the disclosed slices, decode_ref(j, csr, L, syn) for
    slice 2, slice-3 LLRs conditioned on the oracle's decoded slice 2 (when
    the decoder's slice 2 equals it), decode_ref for slice 3; each decode
    checked by check(j, csr, ref, f, res_j, syn_f).  Returns the number of
    sampled sub-blocks check accepted per stage."""
    n, sig, th, x = R["n"], R["sig"], R["th"], R["x"]
    counted = {2: 0, 3: 0}
    for f in R["frames"]:
        sl = slice(f * n, (f + 1) * n)
        A = R["Sf"][f].copy()
        A[2:] = 0
        syn_f = {j: R["syn_np"][j][f][None, :] for j in (2, 3)}
        L2f = oracle.slice_llr(x[sl], sig, th, 4, oracle.GRAY, 2, 0b11, A)
        assert _within_ulp(res["L2"][f], L2f), f"frame {f}: slice-2 LLRs"
        ref2 = decode_ref(2, R["csrs"][2], L2f, syn_f[2])
        counted[2] += bool(check(2, R["csrs"][2], ref2, f, res[2], syn_f[2][0]))
        A[2] = ref2["bits"][0]                       # the oracle's own decoded slice 2
        L3f = oracle.slice_llr(x[sl], sig, th, 4, oracle.GRAY, 3, 0b111, A)
        if np.array_equal(res[2]["bits"][f], ref2["bits"][0]):
            assert _within_ulp(res["L3"][f], L3f), f"frame {f}: slice-3 LLRs"
            ref3 = decode_ref(3, R["csrs"][3], L3f, syn_f[3])
            counted[3] += bool(check(3, R["csrs"][3], ref3, f, res[3], syn_f[3][0]))
    print(f"  sampled {len(R['frames'])} sub-blocks; accepted: slice 2 {counted[2]}, slice 3 {counted[3]}", flush=True)
    return counted


def test_recon_2p27_two_stage_chain_sampled_against_oracle(recon_2p27):
    """The benchmark's flooding sum-product step at 2^27 pairs: slice 2 and
    slice 3 decoded by the persistent kernel at 1024 threads in every shape
    the autotuner may pick (fp32 messages, 100 iterations); 16 sampled
    sub-blocks followed through the oracle's fp64 flooding chain, with
    posteriors within 1e-4 of the scale and decisions, iteration counts and
    status exact on frames with margin."""
    print("[full size: 2^27 pairs, slices 2 and 3, SP flooding, persistent 1024 threads]", flush=True)
    R = recon_2p27
    kw = dict(algo=api.SP, max_iter=100, math=api.F32, store=api.F32)
    res = _run_chain(R, kw, [(0, 0), (0, 150), (8, 0)])
    for j in (2, 3):
        assert res[j]["ok"].mean() > 0.99, f"slice {j}: FER {1 - res[j]['ok'].mean():.3%}"
    ref = lambda j, csr, L, s: oracle.decode(csr, L[None, :], s, algo=oracle.SP, max_iter=100, trace=True)
    chk = lambda j, csr, r, f, rj, s: _check_stage(csr, r, f, rj["iters"], rj["ok"], rj["bits"], rj["post"], s, 1e-4)
    margin = _follow_sampled(R, res, ref, chk)
    k = len(R["frames"])
    assert margin[2] >= 0.75 * k and margin[3] >= 0.75 * k, margin


def test_recon_2p27_layered_chain_sampled_against_oracle(recon_2p27):
    """The benchmark's headline decoder at 2^27 pairs: sum-product with fp32
    messages on the layered schedule, in the launch shapes its autotuner picks
    from (256, 512 and 1024 threads per frame; LDS posterior cache automatic,
    full or off), all bit-identical.  16 sampled sub-blocks followed through
    the oracle's fp64 layered chain: decisions, iteration counts and status
    exact on frames whose posteriors stay farther than 2^-6 of the scale from
    zero wherever the stop decision depends on them (over a whole decode the
    binary32 running posterior drifts from the fp64 sums; the per-iteration
    1e-4 bound from the decoder's own state is checked on two of them)."""
    print("[full size: 2^27 pairs, slices 2 and 3, SP layered]", flush=True)
    from tests._gpu_state import decoded_for
    R = recon_2p27
    kw = dict(algo=api.SP, max_iter=100, math=api.F32, store=api.F32)
    shapes = [dict(wg_threads=1024, lds_cache_kb=0), dict(wg_threads=512, lds_cache_kb=0),
              dict(wg_threads=256, lds_cache_kb=-1), dict(wg_threads=512, lds_cache_kb=150)]
    res = _run_chain(R, kw, shapes, schedule=api.SCHED_LAYERED)
    for j in (2, 3):
        assert res[j]["ok"].mean() > 0.99, f"slice {j}: FER {1 - res[j]['ok'].mean():.3%}"
    lay = {j: oracle.qc_layers(R["qcs"][j].mb, R["qcs"][j].Z) for j in (2, 3)}
    ref = lambda j, csr, L, s: oracle.decode_layered(csr, L.astype(np.float32).astype(np.float64)[None, :], s,
                                                     layers=lay[j], algo=oracle.SP, max_iter=100, trace=True)
    stepped = []

    def chk(j, csr, r, f, rj, s):
        t_o = int(r["iters"][0])
        if not has_margin(csr, r["post_trace"][0], r["scale_trace"][0], t_o, s, 2.0 ** -6):
            return False
        assert int(rj["iters"][f]) == t_o, f"slice {j} frame {f}: iters {int(rj['iters'][f])} oracle {t_o}"
        assert bool(rj["ok"][f]) == bool(r["ok"][0])
        np.testing.assert_array_equal(rj["bits"][f], r["bits"][0])
        if len(stepped) < 2:
            stepped.append((j, f))
        return True

    margin = _follow_sampled(R, res, ref, chk)
    k = len(R["frames"])
    assert margin[2] >= 0.75 * k and margin[3] >= 0.75 * k, margin
    # one-iteration parity from the decoder's own state, on two sampled
    # sub-blocks, with the frame decoded alone equal to its place in the batch
    p = api.Params(algo=api.SP, max_iter=100, math=api.F32, store=api.F32, schedule=api.SCHED_LAYERED)
    worst = 0.0
    for j, f in stepped:
        qc, csr, code = R["qcs"][j], R["csrs"][j], R["codes"][j]
        Lf = res[f"L{j}"][f]
        s = R["syn_np"][j][f]
        post_T, _ = decoded_for(code, qc, p, Lf, s, int(res[j]["iters"][f]))
        np.testing.assert_array_equal(post_T, res[j]["post"][f].astype(np.float64))
        l64 = Lf.astype(np.float64)
        for t in sorted({0, 3, int(res[j]["iters"][f]) - 1}):
            post, c2v = decoded_for(code, qc, p, Lf, s, t)
            c_o, p_o = oracle.layered_step(csr, l64, s, c2v, post, t, layers=lay[j], algo=oracle.SP)
            post1, _ = decoded_for(code, qc, p, Lf, s, t + 1)
            sc = np.abs(l64).copy()
            np.add.at(sc, csr.col_idx, np.abs(c_o))
            worst = max(worst, float(np.max(np.abs(post1 - p_o) / (1e-4 * sc))))
    assert worst <= 1.0, f"one-step posterior deviation {worst:.3g} x (1e-4 of the scale)"


def test_recon_2p27_learned_min_sum_chain_bit_exact(recon_2p27):
    """The benchmark's learned min-sum at 2^27 pairs: per-iteration,
    per-edge-type weights of each slice code, binary16 messages, flooding
    schedule, persistent kernel at 1024 threads in every shape the autotuner
    may pick.  16 sampled sub-blocks followed through the oracle's chain with
    its binary32 min-sum (same weights, binary16 storage): iteration counts,
    status, decisions and posteriors bit for bit, on every sampled frame."""
    print("[full size: 2^27 pairs, slices 2 and 3, learned NMS f16, persistent 1024 threads]", flush=True)
    from paper_2108_08418_amd.train import load_weights
    R = recon_2p27
    w = {j: load_weights(f"learned_slice{j}", extend_to=100) for j in (2, 3)}
    kws = {j: dict(algo=api.NMS, max_iter=int(w[j].shape[0]), math=api.F32, store=api.F16, weights=_g(w[j]))
           for j in (2, 3)}
    res = _run_chain(R, kws[2], [(0, 0), (0, 150), (8, 0)], kw3=kws[3])
    ref = lambda j, csr, L, s: oracle.decode(csr, L.astype(np.float32).astype(np.float64)[None, :], s,
                                             algo=oracle.NMS, weights=w[j].astype(np.float64),
                                             max_iter=int(w[j].shape[0]), store_half=True, prec32=True)
    chk = lambda j, csr, r, f, rj, s: _check_exact(r, f, rj["iters"], rj["ok"], rj["bits"], rj["post"])
    exact = _follow_sampled(R, res, ref, chk)
    assert exact[2] == len(R["frames"]) and exact[3] == len(R["frames"]), exact


def test_recon_2p27_learned_min_sum_layered_chain_bit_exact(recon_2p27):
    """The benchmark's learned min-sum on the layered schedule at 2^27 pairs
    (binary16 messages, the per-iteration, per-edge-type weights of each slice
    code), in the launch shapes its autotuner picks from (1024, 512 and 256
    threads per frame; LDS posterior cache automatic, full or off), all
    bit-identical.  16 sampled sub-blocks followed through the oracle's chain
    with its binary32 layered min-sum (same weights, binary16 storage):
    iteration counts, status, decisions and posteriors bit for bit.  The
    weights are the ones the benchmark gives this schedule: layered iteration
    t with the learned weights of flooding iteration 2 t."""
    print("[full size: 2^27 pairs, slices 2 and 3, learned NMS f16, layered]", flush=True)
    from paper_2108_08418_amd.train import layered_weights, load_weights
    R = recon_2p27
    w = {j: layered_weights(load_weights(f"learned_slice{j}", extend_to=100)) for j in (2, 3)}
    kws = {j: dict(algo=api.NMS, max_iter=int(w[j].shape[0]), math=api.F32, store=api.F16, weights=_g(w[j]))
           for j in (2, 3)}
    shapes = [dict(wg_threads=1024, lds_cache_kb=0), dict(wg_threads=512, lds_cache_kb=0),
              dict(wg_threads=256, lds_cache_kb=-1), dict(wg_threads=512, lds_cache_kb=150)]
    res = _run_chain(R, kws[2], shapes, schedule=api.SCHED_LAYERED, kw3=kws[3])
    lay = {j: oracle.qc_layers(R["qcs"][j].mb, R["qcs"][j].Z) for j in (2, 3)}
    ref = lambda j, csr, L, s: oracle.decode_layered(csr, L.astype(np.float32).astype(np.float64)[None, :], s,
                                                     layers=lay[j], algo=oracle.NMS, weights=w[j].astype(np.float64),
                                                     max_iter=int(w[j].shape[0]), store_half=True, prec32=True)
    chk = lambda j, csr, r, f, rj, s: _check_exact(r, f, rj["iters"], rj["ok"], rj["bits"], rj["post"])
    exact = _follow_sampled(R, res, ref, chk)
    assert exact[2] == len(R["frames"]) and exact[3] == len(R["frames"]), exact


def test_recon_2p27_mixed_layered_chain_against_oracle(recon_2p27):
    """The benchmark's per-slice decoder choice at 2^27 pairs, on the layered
    schedule: learned min-sum with binary16 messages on slice 2 (layered
    iteration t with the weights of flooding iteration 2 t), slice 3's LLRs
    picked by its decoded bits, sum-product with fp32 messages on slice 3; two
    launch shapes, bit-identical.  16 sampled sub-blocks followed through the
    oracle's chain: slice 2 bit for bit against its binary32 layered min-sum
    (binary16 storage); slice 3 against its fp64 layered sum-product, with
    decisions, iteration counts and status exact on frames with a margin of
    2^-6 of the scale."""
    print("[full size: 2^27 pairs, learned NMS f16 layered on slice 2, SP layered on slice 3]", flush=True)
    from paper_2108_08418_amd.train import layered_weights, load_weights
    R = recon_2p27
    w2 = layered_weights(load_weights("learned_slice2", extend_to=100))
    kw2 = dict(algo=api.NMS, max_iter=int(w2.shape[0]), math=api.F32, store=api.F16, weights=_g(w2))
    kw3 = dict(algo=api.SP, max_iter=100, math=api.F32, store=api.F32)
    shapes = [dict(wg_threads=1024, lds_cache_kb=0), dict(wg_threads=512, lds_cache_kb=150)]
    res = _run_chain(R, kw2, shapes, schedule=api.SCHED_LAYERED, kw3=kw3)
    for j in (2, 3):
        assert res[j]["ok"].mean() > 0.99, f"slice {j}: FER {1 - res[j]['ok'].mean():.3%}"
    lay = {j: oracle.qc_layers(R["qcs"][j].mb, R["qcs"][j].Z) for j in (2, 3)}

    def ref(j, csr, L, s):
        L32 = L.astype(np.float32).astype(np.float64)[None, :]
        if j == 2:
            return oracle.decode_layered(csr, L32, s, layers=lay[2], algo=oracle.NMS, weights=w2.astype(np.float64),
                                         max_iter=int(w2.shape[0]), store_half=True, prec32=True)
        return oracle.decode_layered(csr, L32, s, layers=lay[3], algo=oracle.SP, max_iter=100, trace=True)

    def chk(j, csr, r, f, rj, s):
        if j == 2:
            return _check_exact(r, f, rj["iters"], rj["ok"], rj["bits"], rj["post"])
        t_o = int(r["iters"][0])
        if not has_margin(csr, r["post_trace"][0], r["scale_trace"][0], t_o, s, 2.0 ** -6):
            return False
        assert int(rj["iters"][f]) == t_o, f"slice 3 frame {f}: iters {int(rj['iters'][f])} oracle {t_o}"
        assert bool(rj["ok"][f]) == bool(r["ok"][0])
        np.testing.assert_array_equal(rj["bits"][f], r["bits"][0])
        return True

    counted = _follow_sampled(R, res, ref, chk)
    k = len(R["frames"])
    assert counted[2] == k and counted[3] >= 0.75 * k, counted


def _sweep_point(R, n, j):
    """Slice j of the 2^27 pairs in sub-blocks of n (the block-size sweep's
    codes at that n): the code, Bob's syndromes of all sub-blocks, and Alice's
    LLRs given Bob's true lower slices (slice 3's picked from the one-pass
    pair by Bob's slice 2)."""
    F = R["N"] // n
    qc = inputs.slice_code_spec(j, n)
    code = api.Code.from_qc(qc)
    syn = api.syndrome_check(code, R["bob"][j].contiguous(), want_unsat=False)[0].view(-1)
    llr = R["llr2"] if j == 2 else api.slice_llr_choose(R["n30"], R["n31"], R["bob"][2].contiguous())
    return qc, code, syn, llr, F


def _sweep_sampled(R, n, j, qc, syn, out, frames, kind):
    """Sampled sub-blocks of one sweep decode against the oracle from (x, y):
    Bob's syndrome, Alice's LLRs (one fp32 ulp), and the decode by the rule of
    ``kind`` (flooding or layered sum-product).  Returns the frames with
    margin."""
    csr = qc.to_csr()
    F = R["N"] // n
    sig, th, x = R["sig"], R["th"], R["x"]
    bob = R["bob"]
    syn_np = syn.cpu().numpy().reshape(F, -1)
    iters = out["iters"].cpu().numpy()
    ok = out["ok"].cpu().numpy()
    margin = 0
    for f in frames:
        sl = slice(f * n, (f + 1) * n)
        S = bob[:, f * n:(f + 1) * n].cpu().numpy()
        np.testing.assert_array_equal(syn_np[f], oracle.syndrome(csr, S[j][None, :])[0][0])
        A = S.copy()
        A[j:] = 0
        Lf = oracle.slice_llr(x[sl], sig, th, 4, oracle.GRAY, j, (1 << j) - 1, A)
        Lg = out["llr"][f * n:(f + 1) * n].cpu().numpy()
        assert _within_ulp(Lg, Lf), f"n {n} slice {j} frame {f}: LLRs"
        bits = out["bits"][f * n:(f + 1) * n].cpu().numpy()[None, :]
        post = out["post"][f * n:(f + 1) * n].cpu().numpy()[None, :]
        if kind == "flooding":
            ref = oracle.decode(csr, Lg.astype(np.float64)[None, :], syn_np[f][None, :], algo=oracle.SP,
                                max_iter=100, trace=True)
            margin += _check_stage(csr, ref, 0, iters[f:f + 1], ok[f:f + 1], bits, post, syn_np[f], 1e-4)
        else:
            ref = oracle.decode_layered(csr, Lg.astype(np.float64)[None, :], syn_np[f][None, :],
                                        layers=oracle.qc_layers(qc.mb, qc.Z), algo=oracle.SP, max_iter=100,
                                        trace=True)
            t_o = int(ref["iters"][0])
            if has_margin(csr, ref["post_trace"][0], ref["scale_trace"][0], t_o, syn_np[f], 2.0 ** -6):
                margin += 1
                assert int(iters[f]) == t_o, f"n {n} slice {j} frame {f}: iters {int(iters[f])} oracle {t_o}"
                assert bool(ok[f]) == bool(ref["ok"][0])
                np.testing.assert_array_equal(bits[0], ref["bits"][0])
        del ref
    return margin


@pytest.mark.parametrize("n,kind", [(1 << 18, "flooding"), (1 << 18, "layered"), (1 << 20, "group"),
                                    (1 << 20, "layered")])
def test_sweep_sub_block_sizes_sampled_against_oracle(recon_2p27, n, kind):
    """The block-size sweep's large sub-blocks over the same 2^27 pairs:
    n_R = 2^18 (512 sub-blocks per slice, Z = 2048) with flooding sum-product
    on the persistent kernel and with layered sum-product, and n_R = 2^20
    (128 sub-blocks, Z = 8192) on the group schedule (fewer sub-blocks than
    CUs: a group of workgroups on one XCD per sub-block) and on the layered
    schedule (its decision bits fill the LDS, Bob's syndrome bits live in the
    workspace).  Each decode runs in
    every shape its autotuner picks from (bit-identical), both coded slices
    (slice 3 given Bob's slice 2); two sampled sub-blocks per slice against
    the oracle."""
    print(f"[sweep point n={n} {kind}]", flush=True)
    R = recon_2p27
    kw = dict(algo=api.SP, max_iter=100, math=api.F32, store=api.F32)
    if kind == "flooding":
        shapes, sched = [(0, 0), (0, 150), (8, 0)], api.SCHED_PERSISTENT
    elif kind == "layered":
        shapes = [dict(wg_threads=1024, lds_cache_kb=0), dict(wg_threads=512, lds_cache_kb=0),
                  dict(wg_threads=256, lds_cache_kb=-1)]
        sched = api.SCHED_LAYERED
    else:
        shapes = [dict(min_waves=0, group_wgs=0), dict(min_waves=8, group_wgs=0), dict(min_waves=0, group_wgs=8)]
        sched = api.SCHED_GROUP
    for j in (2, 3):
        qc, code, syn, llr, F = _sweep_point(R, n, j)
        out = _decode_in_shapes(api.Batch.uniform(code, F), llr, syn, kw, shapes, sched)
        _, unsat = api.syndrome_check(code, out["bits"], syn, want_syndrome=False)
        okv = out["ok"].cpu().numpy().astype(bool)
        np.testing.assert_array_equal(okv, unsat.cpu().numpy() == 0)
        assert okv.mean() > 0.99, f"n {n} slice {j}: FER {1 - okv.mean():.3%}"
        out["llr"] = llr
        frames = [0, F - 1 - 7 * j]
        margin = _sweep_sampled(R, n, j, qc, syn, out, frames, "layered" if kind == "layered" else "flooding")
        print(f"  slice {j}: {margin}/{len(frames)} sampled sub-blocks with margin", flush=True)
        assert margin >= 1, f"n {n} slice {j}: no sampled sub-block with margin"
        del out


@pytest.mark.parametrize("layered", [False, True])
def test_uneven_met_batch_4096_frames_sampled_against_oracle(layered):
    """The uneven batch in one launch, on the flooding schedule (persistent
    kernel at 1024 threads) and on the layered schedule, in the shapes the
    autotuner picks from (bit-identical); every frame: ok <=> its decisions
    satisfy its syndrome; the first and last frame of each size bit-exact
    against the oracle's binary32 min-sum of the same schedule."""
    print(f"[full size: 4096 uneven MET frames, min-sum f16, {'layered' if layered else 'persistent 1024 threads'}]",
          flush=True)
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
    kw = dict(algo=api.NMS, max_iter=100, math=api.F32, store=api.F16, alpha=0.75)
    if layered:
        out = _decode_in_shapes(batch, _g(llr), syn, kw,
                                [dict(wg_threads=1024, lds_cache_kb=0), dict(wg_threads=512, lds_cache_kb=0),
                                 dict(wg_threads=256, lds_cache_kb=-1)], api.SCHED_LAYERED)
    else:
        out = _decode_in_shapes(batch, _g(llr), syn, kw, [(0, 0), (0, 150), (8, -1)])
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
            okw = dict(algo=oracle.NMS, alpha=float(np.float32(0.75)), max_iter=100, store_half=True, prec32=True)
            if layered:
                ref = oracle.decode_layered(csrs[c], llr[v0:v0 + n][None, :].astype(np.float64), syn_f,
                                            layers=oracle.qc_layers(qcs[c].mb, qcs[c].Z), **okw)
            else:
                ref = oracle.decode(csrs[c], llr[v0:v0 + n][None, :].astype(np.float64), syn_f, **okw)
            assert int(iters[i]) == int(ref["iters"][0]), (i, n)
            assert int(ok[i]) == int(ref["ok"][0]), (i, n)
            np.testing.assert_array_equal(dec[v0:v0 + n], ref["bits"][0])
            np.testing.assert_array_equal(post[v0:v0 + n].astype(np.float64), ref["post"][0])
