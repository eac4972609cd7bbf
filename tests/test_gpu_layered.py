"""GPU parity of the layered (row-serial) schedule against the oracle's
layered mode (Sec. III-C names belief propagation without a schedule; the
layers are the block rows of the QC codes), through the C ABI."""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

import oracle
from paper_2108_08418_amd import api, inputs
from tests._gpu_state import decoded_for
from tests._parity import LayerIndex, compare_trace, has_margin, layered_nms_half_step_bound

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
SNR = 3.0
SIG = math.sqrt(1.0 / SNR)
TH4 = inputs.equiprobable_thresholds(4, 1.0 + 1.0 / SNR)


def _g(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


# Tests with small iteration caps decode the slice-3 family member at mb = 71
# (R = 0.445); the pipeline's slice-3 code (R = 0.492) is decoded at n = 65536.
KERNEL_MB3 = 71


def _slice_stage(j, n, F, seed, mb=None):
    x, y = inputs.gaussian_pairs(n * F, SNR, seed=seed)
    S = oracle.quantize(y, TH4, 4)
    L = oracle.slice_llr(x, SIG, TH4, 4, oracle.GRAY, j, (1 << j) - 1, S).reshape(F, n)
    qc = inputs.slice_code_spec(j, n) if mb is None else inputs.slice_code_at(j, n, mb)
    csr = qc.to_csr()
    syn, _ = oracle.syndrome(csr, S[j].reshape(F, n))
    return qc, csr, L, syn


def _bpsk(qc, F, seed, ebn0=(1.5, 3.0)):
    bits = inputs.random_bits((F, qc.n), seed=seed)
    s2 = inputs.sigma2_from_ebn0(np.linspace(ebn0[0], ebn0[1], F), 1.0 - qc.m / qc.n)
    llr = inputs.bpsk_llr(bits, s2, seed=seed + 1)
    syn, _ = oracle.syndrome(qc.to_csr(), bits)
    return llr, syn


def _decode(code, F, llr, syn, p, trace=False):
    batch = api.Batch.uniform(code, F)
    mdt = torch.float64 if p.math == api.F64 else torch.float32
    tr = None
    if trace:
        tr = torch.full((p.max_iter + 1, batch.total_n), float("nan"), dtype=mdt, device=DEV)
    out = api.ldpc_decode_batch(batch, p, _g(llr.reshape(-1).astype(np.float64 if p.math == api.F64 else np.float32)),
                                None if syn is None else _g(syn.reshape(-1)), trace=tr)
    torch.cuda.synchronize()
    res = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
    if trace:
        res["trace"] = tr.cpu().numpy().reshape(p.max_iter + 1, F, code.n).transpose(1, 0, 2)
    return res


def _layered(qc, csr, llr, syn, **kw):
    return oracle.decode_layered(csr, llr, syn, layers=oracle.qc_layers(qc.mb, qc.Z), **kw)


def _check_margin_frames(csr, res, ref, F, n, syn, rel, min_margin_frac, abs_tol=None):
    """Per-iteration posteriors within rel x scale (or abs_tol(scale)); on the
    frames with margin, iterations, status and decisions exactly equal."""
    margin = 0
    worst = 0.0
    for f in range(F):
        t_o, t_g = int(ref["iters"][f]), int(res["iters"][f])
        t_cmp = min(t_o, t_g)
        g = res["trace"][f, : t_cmp + 1].astype(np.float64)
        o = ref["post_trace"][f, : t_cmp + 1]
        sc = ref["scale_trace"][f, : t_cmp + 1]
        if abs_tol is None:
            worst = max(worst, compare_trace(res["trace"][f], ref["post_trace"][f], ref["scale_trace"][f], t_cmp, rel))
        else:
            worst = max(worst, float(np.nanmax(np.abs(g - o) / abs_tol(sc))))
        s = None if syn is None else syn[f]
        if has_margin(csr, ref["post_trace"][f], ref["scale_trace"][f], t_o, s, rel):
            margin += 1
            assert t_g == t_o, f"frame {f}: iters gpu {t_g} oracle {t_o}"
            assert res["ok"][f] == ref["ok"][f]
            np.testing.assert_array_equal(res["bits"].reshape(F, n)[f], ref["bits"][f])
    assert worst <= 1.0, f"posterior deviation {worst:.3g} x tolerance"
    assert margin >= min_margin_frac * F, f"only {margin}/{F} frames with margin"
    return margin


@pytest.mark.parametrize("j,n", [(3, 4096), (2, 16384)])
def test_layered_sp_fp64_per_iteration(j, n):
    """Sum-product in fp64: posteriors within 1e-12 of the scale after every
    iteration; Z = 32 (rows of a layer fill half a wavefront) and Z = 128."""
    print(f"[layered SP f64 slice{j} n={n}]", flush=True)
    F = 6
    qc, csr, L, syn = _slice_stage(j, n, F, seed=4000 + j, mb=KERNEL_MB3 if j == 3 else None)
    p = api.Params(algo=api.SP, max_iter=60, math=api.F64, store=api.F64, schedule=api.SCHED_LAYERED)
    res = _decode(api.Code.from_qc(qc), F, L, syn, p, trace=True)
    ref = _layered(qc, csr, L, syn, algo=oracle.SP, max_iter=60, trace=True)
    _check_margin_frames(csr, res, ref, F, n, syn, 1e-12, 0.8)
    assert ref["ok"].sum() >= 3


@pytest.mark.parametrize("j", [2, 3])
def test_layered_sp_fp32_slice_codes(j):
    """Sum-product in fp32 (messages fp32) on the pipeline's slice codes at
    n = 65536 (Z = 512), 100 iterations.  Per iteration: from the decoder's
    own state after t iterations, one fp64 layered iteration of the oracle
    gives posteriors within 1e-4 of the scale of the decoder's after t + 1.
    Whole decodes: iteration counts, status and decisions exact on frames
    whose posteriors stay farther than 2^-6 of the scale from zero wherever
    the stop decision depends on them (over a whole decode the binary32
    running posterior drifts from the fp64 sums and the dynamics amplify it:
    up to 2e-4 of the scale was seen on this code), every frame decoded, and
    fewer iterations than flooding on the same frames."""
    print(f"[layered SP f32 slice{j}]", flush=True)
    n, F = 65536, 4
    qc, csr, L, syn = _slice_stage(j, n, F, seed=5100 + j)
    code = api.Code.from_qc(qc)
    p = api.Params(algo=api.SP, max_iter=100, math=api.F32, store=api.F32, schedule=api.SCHED_LAYERED)
    res = _decode(code, F, L, syn, p, trace=True)
    ref = _layered(qc, csr, L.astype(np.float32).astype(np.float64), syn, algo=oracle.SP, max_iter=100, trace=True)
    assert (ref["ok"] == 1).all()
    margin = 0
    for f in range(F):
        t_o = int(ref["iters"][f])
        if has_margin(csr, ref["post_trace"][f], ref["scale_trace"][f], t_o, syn[f], 2.0 ** -6):
            margin += 1
            assert int(res["iters"][f]) == t_o, f"frame {f}"
            assert res["ok"][f] == ref["ok"][f]
            np.testing.assert_array_equal(res["bits"].reshape(F, n)[f], ref["bits"][f])
    assert margin >= F // 2, f"only {margin}/{F} frames with margin"
    lay = oracle.qc_layers(qc.mb, qc.Z)
    worst = 0.0
    for f in range(2):
        l64 = L[f].astype(np.float32).astype(np.float64)
        for t in sorted({0, 1, 5, 10, int(res["iters"][f]) - 1}):
            post, c2v = decoded_for(code, qc, p, L[f], syn[f], t)
            c_o, p_o = oracle.layered_step(csr, l64, syn[f], c2v, post, t, layers=lay, algo=oracle.SP)
            post1, _ = decoded_for(code, qc, p, L[f], syn[f], t + 1)
            sc = np.abs(l64).copy()
            np.add.at(sc, csr.col_idx, np.abs(c_o))
            worst = max(worst, float(np.max(np.abs(post1 - p_o) / (1e-4 * sc))))
    assert worst <= 1.0, f"one-step posterior deviation {worst:.3g} x (1e-4 of the scale)"
    flood = oracle.decode(csr, L, syn, algo=oracle.SP, max_iter=100)
    assert res["iters"].sum() < flood["iters"].sum()


@pytest.mark.parametrize("store", [api.F32, api.F16])
@pytest.mark.parametrize("wg", [0, 256, 1024])
def test_layered_nms_bit_exact_against_binary32_oracle(store, wg):
    """Min-sum on the layered schedule against the oracle's binary32 layered
    mode (the running posterior rounded to binary32 after every update): bit
    for bit at every iteration, every frame."""
    print(f"[layered NMS store={store} wg={wg}]", flush=True)
    qc = inputs.lambda_half_rate_spec(16384)
    csr = qc.to_csr()
    F = 8
    llr, syn = _bpsk(qc, F, seed=5)
    p = api.Params(algo=api.NMS, max_iter=30, math=api.F32, store=store, alpha=0.8, schedule=api.SCHED_LAYERED,
                   wg_threads=wg)
    res = _decode(api.Code.from_qc(qc), F, llr, syn, p, trace=True)
    ref = _layered(qc, csr, llr, syn, algo=oracle.NMS, alpha=float(np.float32(0.8)), max_iter=30, trace=True,
                   store_half=(store == api.F16), prec32=True)
    np.testing.assert_array_equal(res["iters"], ref["iters"])
    np.testing.assert_array_equal(res["ok"], ref["ok"])
    np.testing.assert_array_equal(res["bits"].reshape(F, -1), ref["bits"])
    np.testing.assert_array_equal(res["post"].reshape(F, -1).astype(np.float64), ref["post"])
    for f in range(F):
        t = int(ref["iters"][f])
        np.testing.assert_array_equal(res["trace"][f, : t + 1].astype(np.float64), ref["post_trace"][f, : t + 1])
    assert ref["ok"].sum() >= F // 2


def test_layered_nms_f16_against_fp64_oracle():
    """Min-sum with binary16 messages against the plain fp64 oracle (layered,
    binary16 storage emulated, no binary32 rounding anywhere).  The first
    iteration starts from the same state on both sides: its posteriors lie
    within the forward error bound of a binary32 layered iteration with
    binary16 messages (rounding flips of stored messages carried into the
    later layers of the same iteration).  Later iterations start from states
    that already differ by such roundings (each step from the decoder's own
    state is compared separately).  Over the whole decode: iteration counts,
    status and decisions exact on frames whose posteriors stay farther than
    2^-4 of the scale from zero wherever the stop decision depends on them."""
    print("[layered NMS f16 vs fp64]", flush=True)
    qc = inputs.lambda_half_rate_spec(16384)
    csr = qc.to_csr()
    F = 8
    llr, syn = _bpsk(qc, F, seed=15)
    a = float(np.float32(0.8))
    p = api.Params(algo=api.NMS, max_iter=30, math=api.F32, store=api.F16, alpha=0.8, schedule=api.SCHED_LAYERED)
    res = _decode(api.Code.from_qc(qc), F, llr, syn, p, trace=True)
    l64 = llr.astype(np.float32).astype(np.float64)
    ref = _layered(qc, csr, l64, syn, algo=oracle.NMS, alpha=a, max_iter=30, trace=True, store_half=True)
    lay = oracle.qc_layers(qc.mb, qc.Z)
    lix = LayerIndex(csr, lay)
    worst = 0.0
    for f in range(F):
        if int(res["iters"][f]) < 1:
            continue
        z = np.zeros(csr.n_edges)
        c1, p1 = oracle.layered_step(csr, l64[f], syn[f], z, l64[f], 0, layers=lay, algo=oracle.NMS,
                                     store_half=True, alpha=a)
        E, _ = layered_nms_half_step_bound(lix, l64[f], z, l64[f], c1, np.full(csr.n_edges, a))
        worst = max(worst, float(np.max(np.abs(res["trace"][f, 1].astype(np.float64) - p1) / E)))
    assert worst <= 1.0, f"first-iteration posterior deviation {worst:.3g} x its error bound"
    margin = 0
    for f in range(F):
        t_o = int(ref["iters"][f])
        if has_margin(csr, ref["post_trace"][f], ref["scale_trace"][f], t_o, syn[f], 2.0 ** -4):
            margin += 1
            assert int(res["iters"][f]) == t_o, f"frame {f}"
            assert res["ok"][f] == ref["ok"][f]
            np.testing.assert_array_equal(res["bits"].reshape(F, -1)[f], ref["bits"][f])
    assert margin >= F // 2, f"only {margin}/{F} frames with margin"


def test_layered_learned_weights_bit_exact():
    """Per-iteration, per-edge-type weights on the layered schedule: bit-exact
    against the binary32 layered oracle with the same weights."""
    print("[layered NMS weights]", flush=True)
    n, F = 16384, 6
    qc, csr, L, syn = _slice_stage(3, n, F, seed=5300, mb=KERNEL_MB3)
    rng = np.random.default_rng(9)
    T = 25
    w = rng.uniform(0.55, 0.95, size=(T, qc.n_types)).astype(np.float32)
    p = api.Params(algo=api.NMS, max_iter=T, math=api.F32, store=api.F16, weights=_g(w),
                   schedule=api.SCHED_LAYERED)
    res = _decode(api.Code.from_qc(qc), F, L.astype(np.float32), syn, p, trace=True)
    ref = _layered(qc, csr, L.astype(np.float32).astype(np.float64), syn, algo=oracle.NMS,
                   weights=w.astype(np.float64), max_iter=T, trace=True, store_half=True, prec32=True)
    np.testing.assert_array_equal(res["iters"], ref["iters"])
    np.testing.assert_array_equal(res["ok"], ref["ok"])
    np.testing.assert_array_equal(res["bits"].reshape(F, -1), ref["bits"])
    np.testing.assert_array_equal(res["post"].reshape(F, -1).astype(np.float64), ref["post"])
    assert ref["ok"].sum() >= 1


@pytest.mark.parametrize("n", [4096, 5120])
def test_layered_wavefronts_spanning_block_rows(n):
    """Z = 32 and Z = 40 (Z % 64 != 0): a wavefront's 64 rows span block rows of
    one layer group, so each lane reads its own table entries (masked body);
    at Z = 40 the syndrome test also runs one row per thread (Z % 32 != 0).
    Min-sum with binary16 messages bit-exact against the binary32 layered
    oracle at every iteration, in every workgroup size; sum-product in fp64
    within 1e-12 of the scale at every iteration."""
    print(f"[layered Z={n // 128}]", flush=True)
    qc = inputs.lambda_half_rate_spec(n)
    csr = qc.to_csr()
    F = 6
    llr, syn = _bpsk(qc, F, seed=n + 3)
    code = api.Code.from_qc(qc)
    ref = _layered(qc, csr, llr.astype(np.float32).astype(np.float64), syn, algo=oracle.NMS,
                   alpha=float(np.float32(0.8)), max_iter=30, trace=True, store_half=True, prec32=True)
    for wg in (0, 256, 1024):
        p = api.Params(algo=api.NMS, max_iter=30, math=api.F32, store=api.F16, alpha=0.8, schedule=api.SCHED_LAYERED,
                       wg_threads=wg)
        res = _decode(code, F, llr, syn, p, trace=True)
        np.testing.assert_array_equal(res["iters"], ref["iters"])
        np.testing.assert_array_equal(res["ok"], ref["ok"])
        np.testing.assert_array_equal(res["bits"].reshape(F, -1), ref["bits"])
        for f in range(F):
            t = int(ref["iters"][f])
            np.testing.assert_array_equal(res["trace"][f, : t + 1].astype(np.float64), ref["post_trace"][f, : t + 1])
    assert ref["ok"].sum() >= F // 2
    p = api.Params(algo=api.SP, max_iter=40, math=api.F64, store=api.F64, schedule=api.SCHED_LAYERED)
    res = _decode(code, F, llr, syn, p, trace=True)
    ref = _layered(qc, csr, llr, syn, algo=oracle.SP, max_iter=40, trace=True)
    _check_margin_frames(csr, res, ref, F, n, syn, 1e-12, 0.8)


@pytest.mark.parametrize("Z", [384, 1536, 2048])
def test_layered_launch_shapes_are_bit_identical(Z):
    """Workgroups of 256, 512 and 1024 threads (one, two or four rows of a
    layer per thread and body), with and without the LDS posterior cache, at
    power-of-two and other Z: identical results, trace included."""
    print(f"[layered shapes Z={Z}]", flush=True)
    n, F = 128 * Z, 3
    qc, csr, L, syn = _slice_stage(3, n, F, seed=Z + 7, mb=KERNEL_MB3)
    code = api.Code.from_qc(qc)
    for base in (dict(algo=api.SP, store=api.F32), dict(algo=api.NMS, store=api.F16, alpha=0.85)):
        runs = [_decode(code, F, L, syn, api.Params(max_iter=30, math=api.F32, schedule=api.SCHED_LAYERED,
                                                    wg_threads=wg, lds_cache_kb=lk, **base), trace=True)
                for wg, lk in ((0, 0), (0, -1), (256, 0), (256, 7), (1024, 0), (1024, -1), (512, 150))]
        for r in runs[1:]:
            for k in ("bits", "post", "iters", "ok", "trace"):
                np.testing.assert_array_equal(np.nan_to_num(runs[0][k], nan=1e30), np.nan_to_num(r[k], nan=1e30))
        assert runs[0]["ok"].any()


def test_layered_ragged_batch_equals_frames_alone():
    """Frames of four lengths and codes (the low-rate multi-edge-type code at
    n = 4096 ... 262144, Z = 64 ... 4096) in one layered launch: each frame's
    result equals its decode alone and the oracle's on sampled frames."""
    print("[layered ragged]", flush=True)
    sizes = (4096, 16384, 65536, 262144)
    qcs = [inputs.met_low_rate_spec(n) for n in sizes]
    codes = [api.Code.from_qc(q) for q in qcs]
    order = [0, 3, 1, 0, 2, 1, 0]
    frames, vo, co = [], 0, 0
    for c in order:
        frames.append((c, vo, co))
        vo += sizes[c]
        co += qcs[c].m
    bits = inputs.random_bits(vo, seed=31)
    llr = inputs.bpsk_llr(bits, 1.0 / 0.16, seed=32).astype(np.float32)
    syn = np.concatenate([oracle.syndrome(qcs[c].to_csr(), bits[fv:fv + sizes[c]][None])[0][0]
                          for c, fv, _ in frames])
    p = api.Params(algo=api.NMS, max_iter=40, math=api.F32, store=api.F16, alpha=0.75, schedule=api.SCHED_LAYERED)
    batch = api.Batch(codes, frames)
    out = api.ldpc_decode_batch(batch, p, _g(llr), _g(syn))
    torch.cuda.synchronize()
    for f, (c, fv, fc) in enumerate(frames):
        alone = _decode(codes[c], 1, llr[fv:fv + sizes[c]], syn[fc:fc + qcs[c].m], p)
        np.testing.assert_array_equal(out["bits"][fv:fv + sizes[c]].cpu().numpy(), alone["bits"])
        np.testing.assert_array_equal(out["post"][fv:fv + sizes[c]].cpu().numpy(), alone["post"])
        assert int(out["iters"][f]) == int(alone["iters"][0])
        if sizes[c] <= 16384:
            q = qcs[c]
            ref = _layered(q, q.to_csr(), llr[fv:fv + sizes[c]].astype(np.float64)[None], syn[fc:fc + q.m][None],
                           algo=oracle.NMS, alpha=float(np.float32(0.75)), max_iter=40, store_half=True, prec32=True)
            assert int(ref["iters"][0]) == int(alone["iters"][0])
            np.testing.assert_array_equal(ref["bits"][0], alone["bits"])


def test_layered_edge_cases():
    """A NaN LLR makes its frame fail (ok = 0 after max_iter) without touching the
    others; max_iter = 0 only tests the channel decisions; an empty batch is a
    no-op; explicit (non-QC) codes are refused."""
    print("[layered edge cases]", flush=True)
    n, F = 16384, 4
    qc, csr, L, syn = _slice_stage(3, n, F, seed=5400, mb=KERNEL_MB3)
    code = api.Code.from_qc(qc)
    Ln = L.copy()
    Ln[1, 77] = np.nan
    p = api.Params(algo=api.SP, max_iter=40, math=api.F32, store=api.F32, schedule=api.SCHED_LAYERED)
    res = _decode(code, F, Ln, syn, p)
    ref = _decode(code, F, L, syn, p)
    assert res["ok"][1] == 0 and res["iters"][1] == 40
    for f in (0, 2, 3):
        assert res["iters"][f] == ref["iters"][f]
        np.testing.assert_array_equal(res["bits"].reshape(F, n)[f], ref["bits"].reshape(F, n)[f])
    p0 = api.Params(algo=api.SP, max_iter=0, math=api.F32, store=api.F32, schedule=api.SCHED_LAYERED)
    z = _decode(code, F, L, syn, p0)
    assert (z["iters"] == 0).all()
    np.testing.assert_array_equal(z["bits"].reshape(F, n), (L.astype(np.float32) < 0).astype(np.uint8))
    o0 = _layered(qc, csr, L.astype(np.float32).astype(np.float64), syn, algo=oracle.SP, max_iter=0)
    np.testing.assert_array_equal(z["ok"], o0["ok"])
    empty = api.Batch([code], [])
    api.ldpc_decode_batch(empty, p, _g(np.zeros(1, np.float32)))
    reg = inputs.regular_code(1024, 3, 6, seed=1)
    with pytest.raises(api._lib.CvrError, match="CVR_EUNSUPPORTED"):
        _decode(api.Code.from_csr(reg), 2, np.zeros((2, 1024)), None, p)


def test_layered_graph_replays_match_eager():
    """The layered decode (queue reset + one kernel) captured in a HIP graph:
    every replay, with other eager work in between, equals the eager result."""
    print("[layered graph]", flush=True)
    n, F = 16384, 8
    qc, csr, L, syn = _slice_stage(2, n, F, seed=5500)
    code = api.Code.from_qc(qc)
    batch = api.Batch.uniform(code, F)
    p = api.Params(algo=api.SP, max_iter=60, math=api.F32, store=api.F32, schedule=api.SCHED_LAYERED)
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
    other = api.Params(algo=api.NMS, max_iter=10, math=api.F32, store=api.F16)
    for rep in range(3):
        for v in out.values():
            v.zero_()
        g.replay()
        torch.cuda.synchronize()
        for k in ref:
            assert torch.equal(ref[k], out[k]), f"replay {rep}: {k} differs"
        api.ldpc_decode_batch(batch, other, llr, sg)
        torch.cuda.synchronize()
