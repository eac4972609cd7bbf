"""GPU parity of ldpc_decode_batch against the fp64 oracle.

Rules (floating point): per variable and iteration
|L_gpu - L_orc| <= rel * (|L_ch| + sum |c2v|) with rel = 1e-4 for fp32
arithmetic, 2 binary16 ulps (2^-10) for fp16-stored messages and 1e-12 for
fp64; decoded bits, iteration counts and ok flags bit-exact on frames that
have margin (see tests/_parity.py)."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2108_08418_amd import api, inputs
from tests._parity import compare_trace, has_margin

pytestmark = pytest.mark.gpu
DEV = "cuda"
SNR = 3.0
SIG = math.sqrt(1.0 / SNR)
TH4 = inputs.equiprobable_thresholds(4, 1.0 + 1.0 / SNR)


def _g(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _decode_gpu(code_obj, F, llr, syn, params, trace=False):
    batch = api.Batch.uniform(code_obj, F)
    tr = None
    mdt = torch.float64 if params.math == api.F64 else torch.float32
    if trace:
        tr = torch.full(((params.max_iter + 1), batch.total_n), float("nan"), dtype=mdt, device=DEV)
    out = api.ldpc_decode_batch(batch, params, _g(llr.reshape(-1).astype(np.float64 if params.math == api.F64 else np.float32)),
                                None if syn is None else _g(syn.reshape(-1)), trace=tr)
    torch.cuda.synchronize()
    res = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
    if trace:
        res["trace"] = tr.cpu().numpy().reshape(params.max_iter + 1, F, code_obj.n).transpose(1, 0, 2)
    return res


def _check_against_oracle(csr, res, ref, F, n, syn, rel, expect_margin_frac=0.5):
    margin = 0
    worst = 0.0
    for f in range(F):
        t_o, t_g = int(ref["iters"][f]), int(res["iters"][f])
        s = None if syn is None else syn[f]
        t_cmp = min(t_o, t_g)
        if "trace" in res:
            worst = max(worst, compare_trace(res["trace"][f], ref["post_trace"][f], ref["scale_trace"][f], t_cmp, rel))
        if has_margin(csr, ref["post_trace"][f], ref["scale_trace"][f], t_o, s, rel):
            margin += 1
            assert t_g == t_o, f"frame {f}: iters gpu {t_g} oracle {t_o}"
            assert res["ok"][f] == ref["ok"][f]
            np.testing.assert_array_equal(res["bits"].reshape(F, n)[f], ref["bits"][f])
    assert worst <= 1.0, f"posterior deviation {worst:.3g} x tolerance"
    assert margin >= expect_margin_frac * F, f"only {margin}/{F} frames with margin"
    return margin


def test_config0_regular_sp_fp64():
    """(3,6)-regular n=1024, all-zero word, Eb/N0 2.5 dB, SP fp64, 50 iterations, 200 frames."""
    print("[decode cfg0 SP f64]", flush=True)
    csr = inputs.regular_code(1024, 3, 6, seed=1)
    F = 200
    llr = inputs.bpsk_llr(np.zeros((F, 1024), np.uint8), 0.56234, seed=7)
    p = api.Params(algo=api.SP, max_iter=50, math=api.F64, store=api.F64)
    res = _decode_gpu(api.Code.from_csr(csr), F, llr, None, p, trace=True)
    ref = oracle.decode(csr, llr, None, algo=oracle.SP, max_iter=50, trace=True)
    m = _check_against_oracle(csr, res, ref, F, 1024, None, 1e-12, expect_margin_frac=0.95)
    print(f"margin frames {m}/{F}; oracle failures {(ref['ok'] == 0).sum()}")


# Kernel tests with small iteration caps decode the slice-3 family member at
# mb = 71 (R = 0.445), on which these frames converge within the caps; the
# pipeline's slice-3 code (R = 0.492, about 34 sum-product iterations at
# n = 65536) is decoded by the tests of the 2^20- and 2^27-pair stages.
KERNEL_MB3 = 71


def _slice_stage(j, n, F, seed, mb=None):
    x, y = inputs.gaussian_pairs(n * F, SNR, seed=seed)
    S = oracle.quantize(y, TH4, 4)
    L = oracle.slice_llr(x, SIG, TH4, 4, oracle.GRAY, j, (1 << j) - 1, S).reshape(F, n)
    qc = inputs.slice_code_spec(j, n) if mb is None else inputs.slice_code_at(j, n, mb)
    csr = qc.to_csr()
    syn, _ = oracle.syndrome(csr, S[j].reshape(F, n))
    return qc, csr, L, syn, S[j].reshape(F, n)


@pytest.mark.parametrize("j", [2, 3])
def test_slice_stage_sp_fp32_qc(j):
    """One coded slice of the 2^20-pair configuration (16 x 65536), SP fp32, 100 iterations,
    every schedule bit-identical.  All 16 frames against the fp64 oracle:
    - every frame, one iteration at a time from the decoder's own state (t = 0, 1, 5, 10
      and the last): posteriors within 1e-4 of the scale of the fp64 step's;
    - frames with margin (at least half of them): iteration counts, status and decisions
      exact, and the whole binary32 trajectory within 1e-3 of the scale of the fp64 one
      (the per-step differences compound over a decode: up to 1.3e-4 was seen on these
      frames, so the whole-trajectory bound is not the per-step one);
    - every frame reported ok satisfies Bob's syndrome."""
    print(f"[decode slice{j} SP f32 qc]", flush=True)
    n, F = 65536, 16
    qc, csr, L, syn, truth = _slice_stage(j, n, F, seed=12345)
    p = api.Params(algo=api.SP, max_iter=100, math=api.F32, store=api.F32, schedule=api.SCHED_PERSISTENT)
    code = api.Code.from_qc(qc)
    res = _decode_gpu(code, F, L, syn, p, trace=True)
    # 16 frames: the default schedule runs frame groups; every schedule is bit-identical
    for sched in (api.SCHED_AUTO, api.SCHED_PASSES):
        other = _decode_gpu(code, F, L, syn, api.Params(algo=api.SP, max_iter=100, math=api.F32, store=api.F32,
                                                        schedule=sched), trace=True)
        for k in ("bits", "post", "iters", "ok", "trace"):
            np.testing.assert_array_equal(res[k], other[k])
    ref = oracle.decode(csr, L, syn, algo=oracle.SP, max_iter=100, trace=True)
    margin = 0
    for f in range(F):
        t_o = int(ref["iters"][f])
        if has_margin(csr, ref["post_trace"][f], ref["scale_trace"][f], t_o, syn[f], 1e-4):
            margin += 1
            assert int(res["iters"][f]) == t_o, f"frame {f}: iters gpu {int(res['iters'][f])} oracle {t_o}"
            assert res["ok"][f] == ref["ok"][f]
            np.testing.assert_array_equal(res["bits"].reshape(F, n)[f], ref["bits"][f])
            worst = compare_trace(res["trace"][f], ref["post_trace"][f], ref["scale_trace"][f], t_o, 1e-3)
            assert worst <= 1.0, f"frame {f}: trajectory deviation {worst:.3g} x 1e-3 of the scale"
    print(f"  {margin}/{F} frames with margin", flush=True)
    assert margin >= F // 2, f"only {margin}/{F} frames with margin"
    from tests._gpu_state import decoded_for
    worst = 0.0
    for f in range(F):
        l64 = L[f].astype(np.float32).astype(np.float64)
        for t in sorted({0, 1, 5, 10, max(int(res["iters"][f]) - 1, 0)}):
            post, c2v = decoded_for(code, qc, p, L[f], syn[f], t)
            c_o, p_o = oracle.flood_step(csr, l64, syn[f], c2v, t, algo=oracle.SP)
            post1, _ = decoded_for(code, qc, p, L[f], syn[f], t + 1)
            sc = np.abs(l64).copy()
            np.add.at(sc, csr.col_idx, np.abs(c_o))
            worst = max(worst, float(np.max(np.abs(post1 - p_o) / (1e-4 * sc))))
    assert worst <= 1.0, f"one-step posterior deviation {worst:.3g} x (1e-4 of the scale)"
    ok = res["ok"].astype(bool)
    bits = res["bits"].reshape(F, n)
    # every frame reported ok satisfies Bob's syndrome
    s_chk, _ = oracle.syndrome(csr, bits[ok], syn[ok])
    np.testing.assert_array_equal(s_chk, syn[ok])


@pytest.mark.parametrize("sched", [api.SCHED_PERSISTENT, api.SCHED_LAYERED])
def test_sp_check_messages_across_the_phi_forms(sched):
    """The binary32 sum-product check rule (Sec. III-C), message by message, against
    the fp64 oracle, on inputs at and around the points where the device evaluation of
    phi changes form (x = 1/8, and e^-x = 1/8 at x = ln 8) and over 1e-3 ... 40.  After
    one iteration from zero messages every stored c2v is within 5e-6 x (1 + |c2v|) of
    the oracle's (flooding): phi is good to about 1.3e-6 relative per evaluation (3e-6
    at x = 40, from rounding x log2(e)), its exclusive sums add a few binary32 roundings
    and |y phi'(y)| <= 1 carries a relative error of y into an absolute one of phi(y).
    On the layered schedule later layers read posteriors rounded to binary32 after the
    earlier layers' updates; there the bound is 2e-5 x (1 + |c2v|).  Every outer form
    (Laurent quotient, logarithm, series) is hit by hundreds of messages."""
    print(f"[phi forms sched={sched}]", flush=True)
    from tests._gpu_state import decoded_for
    n = 8192
    qc = inputs.slice_code_spec(3, n)
    csr = qc.to_csr()
    code = api.Code.from_qc(qc)
    rng = np.random.default_rng(81)
    ln8 = math.log(8.0)
    edges = [1e-3, 0.01, 0.05, 0.1, 0.124, 0.1249, 0.125, 0.1251, 0.126, 0.2, 0.5, 1.0, 1.5, 2.0, 2.07,
             ln8 - 1e-3, ln8, ln8 + 1e-3, 2.1, 2.5, 3.0]
    large = [4.0, 4.5, 5.0, 6.0, 8.0, 12.0, 16.0, 24.0, 32.0, 40.0]
    mag = np.where(rng.random(n) < 0.3, rng.choice(edges, n), rng.choice(large, n))
    llr = (mag * rng.choice([-1.0, 1.0], n)).astype(np.float32)
    syn = rng.integers(0, 2, qc.m, dtype=np.uint8)
    l64 = llr.astype(np.float64)
    p = api.Params(algo=api.SP, max_iter=1, math=api.F32, store=api.F32, schedule=sched)
    _, c_gpu = decoded_for(code, qc, p, llr, syn, 1)
    zero = np.zeros(csr.n_edges)
    if sched == api.SCHED_LAYERED:
        c_o, _ = oracle.layered_step(csr, l64, syn, zero, l64, 0, layers=oracle.qc_layers(qc.mb, qc.Z),
                                     algo=oracle.SP)
        tol = 2e-5
    else:
        c_o, _ = oracle.flood_step(csr, l64, syn, zero, 0, algo=oracle.SP)
        tol = 5e-6
    a = np.abs(c_o)
    laurent, series = int((a > 2.7726).sum()), int((a < 0.2513).sum())
    middle = a.size - laurent - series
    worst = float(np.max(np.abs(c_gpu - c_o) / (tol * (1.0 + a))))
    print(f"  outer forms: {laurent} Laurent, {middle} log, {series} series; worst {worst:.3g} x bound", flush=True)
    assert min(laurent, middle, series) >= 100
    np.testing.assert_array_equal(np.sign(c_gpu), np.sign(c_o))
    assert worst <= 1.0


def test_layouts_and_schedules_are_bit_identical():
    """Explicit CSR per-pass, QC per-pass and QC persistent decoding sum in the
    same order and must agree bit for bit."""
    print("[decode layouts/schedules]", flush=True)
    n, F = 16384, 6
    qc, csr, L, syn, _ = _slice_stage(3, n, F, seed=99, mb=KERNEL_MB3)
    for base in (dict(algo=api.SP, store=api.F32), dict(algo=api.NMS, store=api.F16, alpha=0.8),
                 dict(algo=api.NMS, store=api.F32, alpha=0.7)):
        runs = []
        # (code, schedule, workgroup, min waves, LDS posterior cache KiB, workgroups per frame)
        for code, sched, wg, mw, lk, gw in ((api.Code.from_qc(qc), api.SCHED_PERSISTENT, 0, 0, 0, 0),
                                            (api.Code.from_qc(qc), api.SCHED_PERSISTENT, 0, 0, -1, 0),
                                            (api.Code.from_qc(qc), api.SCHED_PERSISTENT, 512, 0, 5, 0),
                                            (api.Code.from_qc(qc), api.SCHED_PERSISTENT, 1024, 0, 0, 0),
                                            (api.Code.from_qc(qc), api.SCHED_PERSISTENT, 512, 8, 0, 0),
                                            (api.Code.from_qc(qc), api.SCHED_PERSISTENT, 1024, 8, 0, 0),
                                            (api.Code.from_qc(qc), api.SCHED_PERSISTENT, 1024, 8, 150, 0),
                                            (api.Code.from_qc(qc), api.SCHED_PASSES, 0, 0, 0, 0),
                                            (api.Code.from_qc(qc), api.SCHED_GROUP, 0, 0, 0, 0),
                                            (api.Code.from_qc(qc), api.SCHED_GROUP, 0, 0, 0, 1),
                                            (api.Code.from_qc(qc), api.SCHED_GROUP, 0, 0, 0, 3),
                                            (api.Code.from_qc(qc), api.SCHED_GROUP, 0, 8, 0, 0),
                                            (api.Code.from_csr(csr), api.SCHED_PASSES, 0, 0, 0, 0)):
            p = api.Params(max_iter=40, math=api.F32, schedule=sched, wg_threads=wg, min_waves=mw,
                           lds_cache_kb=lk, group_wgs=gw, **base)
            runs.append(_decode_gpu(code, F, L, syn, p, trace=True))
        for r in runs[1:]:
            for k in ("bits", "post", "iters", "ok", "trace"):
                np.testing.assert_array_equal(np.nan_to_num(runs[0][k], nan=1e30), np.nan_to_num(r[k], nan=1e30))


def test_persistent_schedule_rejects_explicit_codes():
    csr = inputs.regular_code(1024, 3, 6, seed=1)
    p = api.Params(algo=api.SP, max_iter=5, math=api.F32, store=api.F32, schedule=api.SCHED_PERSISTENT)
    with pytest.raises(api._lib.CvrError, match="CVR_EUNSUPPORTED"):
        _decode_gpu(api.Code.from_csr(csr), 2, np.zeros((2, 1024)), None, p)


@pytest.mark.parametrize("sched", [api.SCHED_PERSISTENT, api.SCHED_PASSES, api.SCHED_GROUP])
@pytest.mark.parametrize("store", [api.F32, api.F16])
def test_nms_bit_exact_against_binary32_oracle(store, sched):
    """Min-sum uses only +, -, x, min and the binary16 rounding: with the oracle
    taking every step in binary32 (the kernel's precision) the two agree bit for
    bit at every iteration."""
    print(f"[decode NMS store={store} schedule={sched}]", flush=True)
    qc = inputs.lambda_half_rate_spec(16384)
    csr = qc.to_csr()
    F = 8
    bits = inputs.random_bits((F, qc.n), seed=5)
    s2 = inputs.sigma2_from_ebn0(np.linspace(1.5, 3.0, F), 0.5)
    llr = inputs.bpsk_llr(bits, s2, seed=6)
    syn, _ = oracle.syndrome(csr, bits)
    p = api.Params(algo=api.NMS, max_iter=30, math=api.F32, store=store, alpha=0.8, schedule=sched)
    res = _decode_gpu(api.Code.from_qc(qc), F, llr, syn, p, trace=True)
    ref = oracle.decode(csr, llr, syn, algo=oracle.NMS, alpha=float(np.float32(0.8)), max_iter=30, trace=True,
                        store_half=(store == api.F16), prec32=True)
    np.testing.assert_array_equal(res["iters"], ref["iters"])
    np.testing.assert_array_equal(res["ok"], ref["ok"])
    np.testing.assert_array_equal(res["bits"].reshape(F, -1), ref["bits"])
    np.testing.assert_array_equal(res["post"].reshape(F, -1).astype(np.float64), ref["post"])
    for f in range(F):
        t = int(ref["iters"][f])
        np.testing.assert_array_equal(res["trace"][f, : t + 1].astype(np.float64), ref["post_trace"][f, : t + 1])
    if store == api.F32:
        # and against the fp64 oracle within the fp32 tolerance
        ref64 = oracle.decode(csr, llr, syn, algo=oracle.NMS, alpha=float(np.float32(0.8)), max_iter=30, trace=True)
        _check_against_oracle(csr, res, ref64, F, qc.n, syn, 1e-4, expect_margin_frac=0.5)


def test_nms_uniform_weights_equal_alpha():
    qc = inputs.lambda_half_rate_spec(4096)
    F = 4
    bits = inputs.random_bits((F, qc.n), seed=1)
    llr = inputs.bpsk_llr(bits, 0.6, seed=2)
    syn, _ = oracle.syndrome(qc.to_csr(), bits)
    code = api.Code.from_qc(qc)
    pa = api.Params(algo=api.NMS, max_iter=20, math=api.F32, store=api.F16, alpha=0.8)
    w = torch.full((20, qc.n_types), 0.8, dtype=torch.float32, device=DEV)
    pw = api.Params(algo=api.NMS, max_iter=20, math=api.F32, store=api.F16, weights=w)
    a = _decode_gpu(code, F, llr, syn, pa)
    b = _decode_gpu(code, F, llr, syn, pw)
    for k in ("bits", "post", "iters", "ok"):
        np.testing.assert_array_equal(a[k], b[k])


@pytest.mark.parametrize("gw,mw", [(0, 0), (2, 0), (5, 0), (0, 8), (3, 8)])
def test_group_schedule_frames_from_queue(gw, mw):
    """More frames than groups (37 frames: a ragged count over the 8 XCDs) so
    that each group takes several frames from its XCD's queue: the results
    equal the persistent decoder's bit for bit, trace included."""
    print(f"[decode group queue gw={gw} mw={mw}]", flush=True)
    n, F = 16384, 37                  # Z = 128: two rows (variables) per thread and body
    qc, csr, L, syn, _ = _slice_stage(3, n, F, seed=123, mb=KERNEL_MB3)
    code = api.Code.from_qc(qc)
    for base in (dict(algo=api.SP, store=api.F32), dict(algo=api.NMS, store=api.F16, alpha=0.8)):
        ref = _decode_gpu(code, F, L, syn, api.Params(max_iter=40, math=api.F32, schedule=api.SCHED_PERSISTENT, **base),
                          trace=True)
        got = _decode_gpu(code, F, L, syn, api.Params(max_iter=40, math=api.F32, schedule=api.SCHED_GROUP,
                                                      group_wgs=gw, min_waves=mw, **base), trace=True)
        for k in ("bits", "post", "iters", "ok", "trace"):
            np.testing.assert_array_equal(np.nan_to_num(ref[k], nan=1e30), np.nan_to_num(got[k], nan=1e30))
        assert ref["ok"].any() and ref["iters"].min() > 0


@pytest.mark.parametrize("Z", [384, 512, 768, 1536])
def test_multi_row_bodies_at_non_power_of_two_Z(Z):
    """Two and four rows per body (1024 threads, one workgroup per CU: 4 at
    Z % 256 == 0), with the division path of the index arithmetic at Z = 384,
    768 and 1536: the persistent shapes (1024 and 512 threads) and the group
    schedule equal the per-pass kernels bit for bit."""
    print(f"[decode multi-row Z={Z}]", flush=True)
    n, F = 128 * Z, 3 if Z > 768 else 5
    qc, csr, L, syn, _ = _slice_stage(3, n, F, seed=Z, mb=KERNEL_MB3)
    code = api.Code.from_qc(qc)
    for base in (dict(algo=api.SP, store=api.F32), dict(algo=api.NMS, store=api.F16, alpha=0.8)):
        ref = _decode_gpu(code, F, L, syn, api.Params(max_iter=30, math=api.F32, schedule=api.SCHED_PASSES, **base))
        assert ref["ok"].any()
        for sched, wg, lk in ((api.SCHED_PERSISTENT, 1024, 0), (api.SCHED_PERSISTENT, 1024, -1),
                              (api.SCHED_PERSISTENT, 512, 0), (api.SCHED_PERSISTENT, 512, -1), (api.SCHED_GROUP, 0, 0)):
            got = _decode_gpu(code, F, L, syn, api.Params(max_iter=30, math=api.F32, schedule=sched, wg_threads=wg,
                                                          lds_cache_kb=lk, **base))
            for k in ("bits", "post", "iters", "ok"):
                np.testing.assert_array_equal(ref[k], got[k])


def test_degree_one_variables_all_schedules():
    """A code with degree-1 variables (the MET code: 48 of 64 block columns):
    every schedule and launch shape, with and without a trace and the
    posterior output, with and without the LDS posterior cache, gives the
    per-pass kernels' results bit for bit."""
    print("[decode degree-1 variables]", flush=True)
    qc = inputs.met_low_rate_spec(4096)
    csr = qc.to_csr()
    code = api.Code.from_qc(qc)
    F = 12
    bits = inputs.random_bits((F, qc.n), seed=31)
    llr = inputs.bpsk_llr(bits, 1.0 / 0.16, seed=32).astype(np.float32)      # SNR 0.16
    syn, _ = oracle.syndrome(csr, bits)
    for base in (dict(algo=api.SP, store=api.F32), dict(algo=api.NMS, store=api.F16, alpha=0.75)):
        ref = _decode_gpu(code, F, llr, syn, api.Params(max_iter=40, math=api.F32, schedule=api.SCHED_PASSES, **base),
                          trace=True)
        assert ref["ok"].any() and (ref["iters"] > 0).all()
        for sched, lk, mw in ((api.SCHED_PERSISTENT, -1, 0), (api.SCHED_PERSISTENT, 150, 0),
                              (api.SCHED_PERSISTENT, 0, 8), (api.SCHED_GROUP, 0, 0), (api.SCHED_GROUP, 0, 8)):
            p = api.Params(max_iter=40, math=api.F32, schedule=sched, lds_cache_kb=lk, wg_threads=1024,
                           min_waves=mw, **base)
            # with a trace (plain kernels), with the posteriors, with decisions only
            got = _decode_gpu(code, F, llr, syn, p, trace=True)
            for k in ("bits", "post", "iters", "ok", "trace"):
                np.testing.assert_array_equal(np.nan_to_num(ref[k], nan=1e30), np.nan_to_num(got[k], nan=1e30))
            got = _decode_gpu(code, F, llr, syn, p)
            for k in ("bits", "post", "iters", "ok"):
                np.testing.assert_array_equal(np.nan_to_num(ref[k], nan=1e30), np.nan_to_num(got[k], nan=1e30))
            batch = api.Batch.uniform(code, F)
            out = api.ldpc_decode_batch(batch, p, _g(llr.reshape(-1)), _g(syn.reshape(-1)), want_post=False)
            torch.cuda.synchronize()
            for k in ("bits", "iters", "ok"):
                np.testing.assert_array_equal(ref[k], out[k].cpu().numpy())


@pytest.mark.parametrize("sizes,sched,lds_kb", [
    ((4096, 8192, 4096), api.SCHED_PERSISTENT, 0),        # Z = 32 / 64: lane-varying block rows
    ((8192, 16384, 8192), api.SCHED_PERSISTENT, 0),       # Z % 64 == 0: wave-uniform kernel
    ((8192, 16384, 8192), api.SCHED_PERSISTENT, 20),      # a few cached columns, a different number per code
    ((8192, 16384, 8192), api.SCHED_PERSISTENT, -1),
    ((4096, 8192, 4096), api.SCHED_PASSES, 0),
    ((4096, 8192, 4096), api.SCHED_GROUP, 0),             # lane-varying block rows
    ((8192, 16384, 8192), api.SCHED_GROUP, 0),            # wave-uniform
])
def test_ragged_batch_mixed_codes_and_gaps(sizes, sched, lds_kb):
    """Frames of different codes and lengths at scattered offsets: each frame
    decodes exactly as it does alone (the persistent decoder reloads its LDS
    tables and posterior cache at every change of code)."""
    print(f"[decode ragged sizes={sizes} schedule={sched} lds={lds_kb}]", flush=True)
    specs = [inputs.slice_code_spec(3, sizes[0]), inputs.slice_code_spec(2, sizes[1]),
             inputs.lambda_half_rate_spec(sizes[2])]
    codes = [api.Code.from_qc(q) for q in specs]
    order = [0, 2, 1, 0, 1, 2, 2]
    frames, vo, co = [], 17, 5
    llrs, syns, bitss = [], [], []
    for i, c in enumerate(order):
        q = specs[c]
        b = inputs.random_bits(q.n, seed=100 + i)
        llrs.append(inputs.bpsk_llr(b[None, :], 0.55, seed=200 + i)[0])
        syns.append(oracle.syndrome(q.to_csr(), b[None, :])[0][0])
        frames.append((c, vo, co))
        vo += q.n + 3 * i
        co += q.m + i
    total_n, total_m = vo, co
    L = np.zeros(total_n, np.float32)
    S = np.zeros(total_m, np.uint8)
    for (c, v0, c0), l, s in zip(frames, llrs, syns):
        L[v0:v0 + len(l)] = l
        S[c0:c0 + len(s)] = s
    batch = api.Batch(codes, frames)
    assert batch.total_n <= total_n and batch.F == len(order)
    p = api.Params(algo=api.SP, max_iter=30, math=api.F32, store=api.F32, schedule=sched, lds_cache_kb=lds_kb)
    out = api.ldpc_decode_batch(batch, p, _g(L), _g(S))
    torch.cuda.synchronize()
    solo_p = api.Params(algo=api.SP, max_iter=30, math=api.F32, store=api.F32, schedule=api.SCHED_PASSES)
    for i, (c, v0, c0) in enumerate(frames):
        solo = _decode_gpu(codes[c], 1, llrs[i][None, :], syns[i][None, :], solo_p)
        n = specs[c].n
        np.testing.assert_array_equal(out["bits"][v0:v0 + n].cpu().numpy(), solo["bits"])
        np.testing.assert_array_equal(out["post"][v0:v0 + n].cpu().numpy(), solo["post"])
        assert int(out["iters"][i]) == int(solo["iters"][0])


@pytest.mark.parametrize("sched", [api.SCHED_PERSISTENT, api.SCHED_PASSES, api.SCHED_GROUP])
def test_failure_injection_and_edge_cases(sched):
    print(f"[decode edge cases schedule={sched}]", flush=True)
    qc = inputs.lambda_half_rate_spec(4096)
    csr = qc.to_csr()
    code = api.Code.from_qc(qc)
    F = 5
    bits = inputs.random_bits((F, qc.n), seed=3)
    llr = inputs.bpsk_llr(bits, 0.5, seed=4).astype(np.float32)
    syn, _ = oracle.syndrome(csr, bits)
    llr[1] = inputs.bpsk_llr(bits[1:2], 4.0, seed=5)[0]      # far above capacity: undecodable
    llr[2, 7] = np.nan                                        # a NaN LLR
    llr[3] = (1 - 2 * bits[3].astype(np.float32)) * 30.0      # clean frame: stops at t = 0
    syn_bad = syn.copy()
    syn_bad[4, 11] ^= 1                                       # corrupted syndrome bit
    p = api.Params(algo=api.SP, max_iter=25, math=api.F32, store=api.F32, schedule=sched)
    res = _decode_gpu(code, F, llr, syn_bad, p)
    assert res["ok"][0] == 1
    assert res["ok"][1] == 0 and res["iters"][1] == 25
    assert res["ok"][2] == 0
    assert res["ok"][3] == 1 and res["iters"][3] == 0
    np.testing.assert_array_equal(res["bits"].reshape(F, -1)[3], bits[3])
    # frame 0 is unaffected by its neighbours
    solo = _decode_gpu(code, 1, llr[:1], syn[:1], p)
    np.testing.assert_array_equal(solo["bits"], res["bits"].reshape(F, -1)[0])
    # max_iter = 0: channel decisions, ok iff already a coset member
    p0 = api.Params(algo=api.SP, max_iter=0, math=api.F32, store=api.F32, schedule=sched)
    r0 = _decode_gpu(code, F, llr, syn_bad, p0)
    assert (r0["iters"] == 0).all() and r0["ok"][3] == 1 and r0["ok"][0] == 0
    # no early stop: every frame runs max_iter iterations
    pn = api.Params(algo=api.SP, max_iter=12, math=api.F32, store=api.F32, early_stop=False, schedule=sched)
    rn = _decode_gpu(code, F, llr, syn_bad, pn)
    assert (rn["iters"] == 12).all()
    # empty batch is a no-op
    empty = api.Batch([code], [])
    api.ldpc_decode_batch(empty, p, _g(np.zeros(1, np.float32)))


@pytest.mark.parametrize("sched", [api.SCHED_PERSISTENT, api.SCHED_LAYERED])
@pytest.mark.parametrize("math_", [api.F32, api.F64])
@pytest.mark.parametrize("algo", [api.SP, api.NMS])
def test_signed_zero_llrs_decode_like_the_oracle(algo, math_, sched):
    """Channel LLRs of exactly +0 and -0 (no information, either sign bit): both
    have magnitude 0 in the check rule (Sec. III-C), so a row holding one sends
    zero to its other edges and nothing turns into NaN.  Every frame ends as the
    fp64 oracle's does (status, iterations and decisions)."""
    print(f"[signed zero LLRs algo={algo} math={math_} sched={sched}]", flush=True)
    qc = inputs.lambda_half_rate_spec(4096)
    csr = qc.to_csr()
    code = api.Code.from_qc(qc)
    F = 6
    bits = inputs.random_bits((F, qc.n), seed=31)
    llr = inputs.bpsk_llr(bits, 0.4, seed=32)
    rng = np.random.default_rng(33)
    pick = rng.random(llr.shape)
    llr[pick < 0.02] = -0.0
    llr[(pick >= 0.02) & (pick < 0.04)] = 0.0
    assert np.signbit(llr[llr == 0]).any() and (~np.signbit(llr[llr == 0])).any()
    syn, _ = oracle.syndrome(csr, bits)
    dt = np.float64 if math_ == api.F64 else np.float32
    llr = llr.astype(dt)
    store = {api.F64: api.F64, api.F32: api.F32}[math_]
    p = api.Params(algo=algo, max_iter=50, math=math_, store=store, schedule=sched)
    res = _decode_gpu(code, F, llr, syn, p)
    okw = dict(algo=oracle.SP if algo == api.SP else oracle.NMS, max_iter=50)
    l64 = llr.astype(np.float64)
    ref = (oracle.decode_layered(csr, l64, syn, layers=oracle.qc_layers(qc.mb, qc.Z), **okw)
           if sched == api.SCHED_LAYERED else oracle.decode(csr, l64, syn, **okw))
    assert (ref["ok"] == 1).all()
    np.testing.assert_array_equal(res["ok"], ref["ok"])
    np.testing.assert_array_equal(res["iters"], ref["iters"])
    np.testing.assert_array_equal(res["bits"].reshape(F, -1), ref["bits"])


def test_group_barrier_time_out_reports_every_frame_failed():
    """Forced from the host: with a zero wait bound, a group barrier that is not
    complete when a workgroup arrives gives up at once; the launch still ends and
    every frame of that decode is reported abandoned (iters = -1, ok = 0), which
    the binding turns into an error.  With the default bound restored the next
    decode equals the persistent decoder's."""
    print("[decode group barrier time-out]", flush=True)
    n, F = 16384, 12
    qc, csr, L, syn, _ = _slice_stage(3, n, F, seed=321, mb=KERNEL_MB3)
    code = api.Code.from_qc(qc)
    p = api.Params(algo=api.SP, max_iter=30, early_stop=False, math=api.F32, store=api.F32,
                   schedule=api.SCHED_GROUP)
    try:
        api.debug_group_wait_ticks(0)
        failed = _decode_gpu(code, F, L, syn, p)
    finally:
        api.debug_group_wait_ticks()
    assert (failed["ok"] == 0).all()
    assert (failed["iters"] == -1).all()
    with pytest.raises(api._lib.CvrError, match="abandoned"):
        api.check_abandoned({k: torch.from_numpy(v) for k, v in failed.items()})
    good = _decode_gpu(code, F, L, syn, p)
    assert (good["iters"] >= 0).all()
    ref = _decode_gpu(code, F, L, syn, api.Params(algo=api.SP, max_iter=30, early_stop=False, math=api.F32,
                                                  store=api.F32, schedule=api.SCHED_PERSISTENT))
    for k in ("bits", "post", "iters", "ok"):
        np.testing.assert_array_equal(ref[k], good[k])


def test_repeat_runs_are_bit_identical():
    qc, csr, L, syn, _ = _slice_stage(2, 16384, 4, seed=8)
    p = api.Params(algo=api.SP, max_iter=60, math=api.F32, store=api.F32)
    code = api.Code.from_qc(qc)
    a = _decode_gpu(code, 4, L, syn, p)
    b = _decode_gpu(code, 4, L, syn, p)
    for k in ("bits", "post", "iters", "ok"):
        np.testing.assert_array_equal(a[k], b[k])


@pytest.mark.parametrize("sched", [api.SCHED_PERSISTENT, api.SCHED_PASSES, api.SCHED_GROUP])
def test_graph_capture_replays_match_eager(sched):
    """The decode (queue reset + persistent kernel, or the per-pass launches;
    no memset) captured in a HIP graph: every replay, with unrelated eager work
    in between, equals eager."""
    print(f"[decode graph schedule={sched}]", flush=True)
    qc, csr, L, syn, _ = _slice_stage(2, 16384, 8, seed=21)
    code = api.Code.from_qc(qc)
    batch = api.Batch.uniform(code, 8)
    p = api.Params(algo=api.NMS, max_iter=60, math=api.F32, store=api.F16, alpha=0.75, schedule=sched)
    llr = _g(L.reshape(-1).astype(np.float32))
    sg = _g(syn.reshape(-1))
    ref = api.ldpc_decode_batch(batch, p, llr, sg)
    torch.cuda.synchronize()
    ref = {k: v.clone() for k, v in ref.items()}
    ws = api.alloc_workspace(batch, p)
    out = {k: torch.empty_like(v) for k, v in ref.items()}
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        api.ldpc_decode_batch(batch, p, llr, sg, workspace=ws, out=out)
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        api.ldpc_decode_batch(batch, p, llr, sg, workspace=ws, out=out)
    other = api.Params(algo=api.SP, max_iter=10, math=api.F32, store=api.F32)
    for rep in range(3):
        for v in out.values():
            v.fill_(0x55 if v.dtype == torch.uint8 else 7)
        g.replay()
        torch.cuda.synchronize()
        for k in ref:
            assert torch.equal(out[k], ref[k]), (rep, k)
        api.ldpc_decode_batch(batch, other, llr, sg)     # eager work between replays
        torch.cuda.synchronize()


def test_ragged_low_rate_met_batch_sampled_against_oracle():
    """A scaled-down uneven batch of the low-rate MET code (sizes 4096 ...
    65536) at SNR 0.16, NMS with binary16 messages: sampled frames of each
    size decode bit-exactly as the binary32 oracle."""
    print("[decode ragged MET]", flush=True)
    sizes, counts = (4096, 16384, 65536), (24, 8, 3)
    rng = np.random.default_rng(4)
    order = rng.permutation(np.repeat(np.arange(3), counts))
    qcs = [inputs.met_low_rate_spec(n) for n in sizes]
    codes = [api.Code.from_qc(q) for q in qcs]
    frames, vo, co = [], 0, 0
    for c in order:
        frames.append((int(c), vo, co))
        vo += sizes[c]
        co += qcs[c].m
    bits = inputs.random_bits(vo, seed=5)
    llr = inputs.bpsk_llr(bits, 1 / 0.16, seed=6).astype(np.float32)
    syn = np.zeros(co, np.uint8)
    for (c, v0, c0) in frames:
        syn[c0:c0 + qcs[c].m] = oracle.syndrome(qcs[c].to_csr(), bits[v0:v0 + sizes[c]][None, :])[0][0]
    batch = api.Batch(codes, frames)
    p = api.Params(algo=api.NMS, max_iter=100, math=api.F32, store=api.F16, alpha=0.75,
                   schedule=api.SCHED_PERSISTENT)
    out = api.ldpc_decode_batch(batch, p, _g(llr), _g(syn))
    torch.cuda.synchronize()
    picks = [int(np.nonzero(order == c)[0][0]) for c in range(3)] + [len(frames) - 1]
    for i in picks:
        c, v0, c0 = frames[i]
        n = sizes[c]
        ref = oracle.decode(qcs[c].to_csr(), llr[v0:v0 + n][None, :].astype(np.float64), syn[c0:c0 + qcs[c].m][None, :],
                            algo=oracle.NMS, alpha=float(np.float32(0.75)), max_iter=100, store_half=True, prec32=True)
        assert int(out["iters"][i]) == int(ref["iters"][0])
        assert int(out["ok"][i]) == int(ref["ok"][0])
        np.testing.assert_array_equal(out["bits"][v0:v0 + n].cpu().numpy(), ref["bits"][0])
        np.testing.assert_array_equal(out["post"][v0:v0 + n].cpu().numpy().astype(np.float64), ref["post"][0])


@pytest.mark.parametrize("slice_j", [2, 3])
def test_rate_selection_loop_on_the_gpu(slice_j):
    """The rate-selection loop: rates step down by 0.05 from 0.9 C_j, every
    candidate before the selected one fails its decoding test, the selected one
    decodes every sub-block to Bob's word, and C_j estimated from the LLRs is
    the slice capacity of the oracle's quadrature (0.3153, 0.5469)."""
    from paper_2108_08418_amd import rates
    print(f"[rate selection slice {slice_j}, n = 2^16, 32 sub-blocks]", flush=True)
    res = rates.select_slice_rate(slice_j, 1 << 16, frames=32)
    cap = {2: 0.3153, 3: 0.5469}[slice_j]
    assert abs(res["capacity"] - cap) < 2e-3, res["capacity"]
    trail = res["trail"]
    print(trail, flush=True)
    assert res["selected"] is trail[-1]
    assert all(c["failures"] + c["undetected"] > 0 for c in trail[:-1])
    assert trail[-1]["failures"] == 0 and trail[-1]["undetected"] == 0
    assert trail[0]["target"] == round(0.9 * res["capacity"], 4)
    assert all(abs(a["target"] - b["target"] - 0.05) < 1e-9 for a, b in zip(trail, trail[1:]))
    assert all(c["rate"] <= 0.9 * res["capacity"] + 1 / 256 for c in trail)
    assert trail[-1]["ga_iters"] is not None
