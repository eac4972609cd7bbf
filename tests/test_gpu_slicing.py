"""GPU parity of Bob's quantiser/slicer, Alice's slice LLRs and the syndrome
kernel against the fp64 oracle (bit-exact for integer outputs)."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2108_08418_amd import api, inputs

pytestmark = pytest.mark.gpu

SNR = 3.0
SIG = math.sqrt(1.0 / SNR)
TH4 = inputs.equiprobable_thresholds(4, 1.0 + 1.0 / SNR)
DEV = "cuda"


def _g(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.mark.parametrize("n", [1 << 20, 1003, 4, 1, 0])
def test_quantize_bit_exact(n):
    print(f"[quantize n={n}]", flush=True)
    x, y = inputs.gaussian_pairs(max(n, 1), SNR, seed=300 + n)
    y = y[:n]
    if n > 100:
        y[:15] = TH4          # values exactly on thresholds go up
        y[15] = np.nextafter(TH4[3], -np.inf)
    got = api.slice_quantize(_g(y), TH4, 4)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(got.cpu().numpy(), oracle.quantize(y, TH4, 4))


@pytest.mark.parametrize("m_bits", [1, 3, 5, 8])
@pytest.mark.parametrize("lab", [api.GRAY, api.BINARY])
def test_quantize_other_widths_and_labellings(m_bits, lab):
    print(f"[quantize m={m_bits} lab={lab}]", flush=True)
    _, y = inputs.gaussian_pairs(50_001, SNR, seed=7 + m_bits)
    th = inputs.constant_step_thresholds(m_bits, 3.0 / 2 ** m_bits)
    got = api.slice_quantize(_g(y), th, m_bits, lab)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(got.cpu().numpy(), oracle.quantize(y, th, m_bits, lab))


def test_quantize_unaligned_views():
    _, y = inputs.gaussian_pairs(4097, SNR, seed=5)
    yg = _g(y)[1:]                        # 8-byte aligned, not 32: scalar path
    got = api.slice_quantize(yg, TH4, 4)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(got.cpu().numpy(), oracle.quantize(y[1:], TH4, 4))


@pytest.mark.parametrize("j,mask", [(0, 0), (1, 0b1), (2, 0b11), (3, 0b111), (3, 0), (1, 0b1101)])
def test_slice_llr_fp64_parity(j, mask):
    print(f"[slice_llr j={j} mask={mask:b}]", flush=True)
    N = 1 << 18
    x, y = inputs.gaussian_pairs(N, SNR, seed=40 + j)
    x[:33] = np.linspace(-8, 8, 33)            # far tails
    S = oracle.quantize(y, TH4, 4)
    Lg = api.slice_llr(_g(x), SIG, TH4, 4, j, mask, _g(S), out_dtype=api.F64)
    torch.cuda.synchronize()
    Lo = oracle.slice_llr(x, SIG, TH4, 4, oracle.GRAY, j, mask, S)
    Lg = Lg.cpu().numpy()
    assert np.isfinite(Lg).all()
    err = np.abs(Lg - Lo) / np.maximum(1.0, np.abs(Lo))
    assert err.max() <= 1e-12, (err.max(), int(err.argmax()))


@pytest.mark.parametrize("j,mask", [(2, 0b11), (3, 0b111), (1, 0b1101)])
def test_slice_llr_extreme_inputs_use_the_log_domain(j, mask):
    """Samples so far out that the interval probabilities underflow in linear
    fp64 (|z| up to 1.7e3): the kernel redoes them in the log domain and stays
    finite and within the same bound of the oracle; ordinary samples in the
    same launch are unaffected."""
    rng = np.random.default_rng(7 + j)
    far = np.array([-1000.0, -100.0, -40.0, -25.0, 25.0, 40.0, 100.0, 1000.0])
    x = np.concatenate([far, rng.standard_normal(4096 - far.size)])
    S = rng.integers(0, 2, size=(4, x.size), dtype=np.uint8)
    Lg = api.slice_llr(_g(x), SIG, TH4, 4, j, mask, _g(S), out_dtype=api.F64)
    torch.cuda.synchronize()
    Lo = oracle.slice_llr(x, SIG, TH4, 4, oracle.GRAY, j, mask, S)
    Lg = Lg.cpu().numpy()
    assert np.isfinite(Lg).all() and np.isfinite(Lo).all()
    err = np.abs(Lg - Lo) / np.maximum(1.0, np.abs(Lo))
    assert err.max() <= 1e-12, (err.max(), int(err.argmax()))


def test_slice_llr_fp32_output_is_rounded_fp64():
    N = (1 << 20) + 7
    x, y = inputs.gaussian_pairs(N, SNR, seed=9)
    S = oracle.quantize(y, TH4, 4)
    L32 = api.slice_llr(_g(x), SIG, TH4, 4, 3, 0b111, _g(S), out_dtype=api.F32)
    torch.cuda.synchronize()
    Lo = oracle.slice_llr(x, SIG, TH4, 4, oracle.GRAY, 3, 0b111, S)
    ref = Lo.astype(np.float32)
    got = L32.cpu().numpy()
    ulp = np.spacing(np.abs(ref)).astype(np.float64)
    assert (np.abs(got.astype(np.float64) - ref) <= ulp).all()


def test_slice_llr_one_bit_closed_form():
    xs = np.linspace(-9, 9, 1001)
    Lg = api.slice_llr(_g(xs), 0.7, np.array([0.0]), 1, 0, 0, None, out_dtype=api.F64).cpu().numpy()
    from scipy.special import log_ndtr
    ref = log_ndtr(-xs / 0.7) - log_ndtr(xs / 0.7)
    np.testing.assert_allclose(Lg, ref, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("m_bits", [1, 3, 5, 8])
@pytest.mark.parametrize("lab", [api.GRAY, api.BINARY])
def test_slice_llr_forms_other_widths_and_labellings(m_bits, lab):
    """Constant-step quantisers of 1 ... 8 bits (the paper's m = 5 among them),
    both labellings: the hard, soft-prior and binary-symmetric forms against
    the oracle, for the top slice and a middle one."""
    print(f"[slice_llr forms m={m_bits} lab={lab}]", flush=True)
    N = 20_011
    x, y = inputs.gaussian_pairs(N, SNR, seed=70 + m_bits)
    th = inputs.constant_step_thresholds(m_bits, 3.0 / 2 ** m_bits)
    S = oracle.quantize(y, th, m_bits, lab)
    olab = oracle.GRAY if lab == api.GRAY else oracle.BINARY
    lam = _priors(np.random.default_rng(71 + m_bits), N) if m_bits <= 4 else \
        np.random.default_rng(71).normal(0, 6, size=(m_bits, N)).astype(np.float32)
    xg, Sg, lg = _g(x), _g(S), _g(lam)
    for j in sorted({m_bits - 1, m_bits // 2}):
        known = (1 << j) - 1
        Lg = api.slice_llr(xg, SIG, th, m_bits, j, known, Sg, labelling=lab, out_dtype=api.F64)
        torch.cuda.synchronize()
        _same_nonfinite_then_rel(Lg.cpu().numpy(), oracle.slice_llr(x, SIG, th, m_bits, olab, j, known, S), 1e-12)
        if j >= 1:                                 # lowest known slice moved into the priors
            Lp = api.slice_llr_prior(xg, SIG, th, m_bits, j, known & ~1, Sg, 1, lg, labelling=lab,
                                     out_dtype=api.F64)
            torch.cuda.synchronize()
            ref = oracle.slice_llr_prior(x, SIG, th, m_bits, olab, j, known & ~1, S, 1, lam)
            _same_nonfinite_then_rel(Lp.cpu().numpy(), ref, 1e-12)
        Lb = api.slice_llr_bsc(xg, th, m_bits, j, 0.07, labelling=lab, out_dtype=api.F64)
        torch.cuda.synchronize()
        np.testing.assert_allclose(Lb.cpu().numpy(), oracle.slice_llr_bsc(x, th, m_bits, olab, j, 0.07),
                                   rtol=4.5e-16, atol=0)


@pytest.mark.parametrize("m_bits,lab,j,known", [(4, api.GRAY, 2, 0b11), (4, api.GRAY, 0, 0), (4, api.GRAY, 1, 0b1),
                                                (4, api.GRAY, 1, 0b1000), (5, api.BINARY, 3, 0b111),
                                                (5, api.GRAY, 2, 0b10011)])
@pytest.mark.parametrize("dt", [api.F64, api.F32])
def test_slice_llr_next_equals_slice_llr_bit_for_bit(m_bits, lab, j, known, dt):
    """One pass for slice j and both conditional LLRs of slice j+1 equals
    slice_llr on each, bit for bit, far tails (log-domain pass) included; the
    choice by the decoded bits equals slice_llr with those bits known."""
    print(f"[slice_llr_next m={m_bits} lab={lab} j={j} known={known:b} dt={dt}]", flush=True)
    N = (1 << 18) + 13
    x, y = inputs.gaussian_pairs(N, SNR, seed=80 + j)
    x[:33] = np.linspace(-30, 30, 33)
    th = TH4 if m_bits == 4 else inputs.constant_step_thresholds(m_bits, 3.0 / 2 ** m_bits)
    S = oracle.quantize(y, th, m_bits, oracle.GRAY if lab == api.GRAY else oracle.BINARY)
    xg, Sg = _g(x), _g(S)
    L, N0, N1 = api.slice_llr_next(xg, SIG, th, m_bits, j, known, Sg, labelling=lab, out_dtype=dt)
    ref = api.slice_llr(xg, SIG, th, m_bits, j, known, Sg, labelling=lab, out_dtype=dt)
    torch.cuda.synchronize()
    assert torch.equal(L, ref)
    for b, got in ((0, N0), (1, N1)):
        Sb = S.copy()
        Sb[j] = b
        ref_b = api.slice_llr(xg, SIG, th, m_bits, j + 1, known | (1 << j), _g(Sb), labelling=lab, out_dtype=dt)
        torch.cuda.synchronize()
        assert torch.equal(got, ref_b), b
    # the choice by Bob's (here: the true) bits of slice j
    chosen = api.slice_llr_choose(N0, N1, Sg[j])
    direct = api.slice_llr(xg, SIG, th, m_bits, j + 1, known | (1 << j), Sg, labelling=lab, out_dtype=dt)
    torch.cuda.synchronize()
    assert torch.equal(chosen, direct)
    if dt == api.F64:
        olab = oracle.GRAY if lab == api.GRAY else oracle.BINARY
        Lo = oracle.slice_llr(x, SIG, th, m_bits, olab, j + 1, known | (1 << j), S)
        _same_nonfinite_then_rel(chosen.cpu().numpy(), Lo, 1e-12)


def test_slice_llr_choose_edge_cases():
    for n in (0, 1, 1003):
        a = torch.arange(n, dtype=torch.float32, device=DEV)
        b = -a - 1
        bits = torch.from_numpy(np.random.default_rng(n).integers(0, 2, n).astype(np.uint8)).to(DEV)
        got = api.slice_llr_choose(a, b, bits)
        torch.cuda.synchronize()
        assert torch.equal(got, torch.where(bits.bool(), b, a))


def _same_nonfinite_then_rel(got, ref, rel):
    """Non-finite outputs (+-inf, NaN) at the same places with the same value;
    finite ones within rel * max(1, |ref|)."""
    fin = np.isfinite(ref)
    np.testing.assert_array_equal(np.isfinite(got), fin)
    np.testing.assert_array_equal(got[~fin], ref[~fin])     # NaN == NaN under assert_array_equal
    err = np.abs(got[fin] - ref[fin]) / np.maximum(1.0, np.abs(ref[fin]))
    assert err.size == 0 or err.max() <= rel, (err.max(), int(np.nonzero(fin)[0][err.argmax()]))


def _priors(rng, N):
    """Prior LLR rows [4, N]: decoder-like magnitudes, zeros, values whose
    logistic factor underflows in linear fp64 (|lambda| ~ 1e3) and +-inf."""
    lam = rng.normal(0.0, 8.0, size=(4, N))
    sel = rng.random((4, N))
    lam[sel < 0.05] = 0.0
    big = (sel >= 0.05) & (sel < 0.08)
    lam[big] = np.sign(lam[big]) * rng.uniform(700.0, 3000.0, big.sum())
    inf = (sel >= 0.08) & (sel < 0.09)
    lam[inf] = np.where(rng.random(inf.sum()) < 0.5, np.inf, -np.inf)
    return lam.astype(np.float32)


@pytest.mark.parametrize("j,known,prior", [(3, 0b11, 0b100), (2, 0b1, 0b10), (1, 0, 0b1101), (3, 0, 0b111)])
def test_slice_llr_prior_fp64_parity(j, known, prior):
    print(f"[slice_llr_prior j={j} known={known:b} prior={prior:b}]", flush=True)
    N = (1 << 18) + 13
    x, y = inputs.gaussian_pairs(N, SNR, seed=60 + j)
    x[:33] = np.linspace(-30, 30, 33)           # far tails: the log-domain pass
    S = oracle.quantize(y, TH4, 4)
    lam = _priors(np.random.default_rng(61 + j), N)
    Lg = api.slice_llr_prior(_g(x), SIG, TH4, 4, j, known, _g(S), prior, _g(lam), out_dtype=api.F64)
    torch.cuda.synchronize()
    Lo = oracle.slice_llr_prior(x, SIG, TH4, 4, oracle.GRAY, j, known, S, prior, lam)
    _same_nonfinite_then_rel(Lg.cpu().numpy(), Lo, 1e-12)


def test_slice_llr_prior_chain_fp32_output():
    """The literal chain at SNR 3: slices 0 and 1 disclosed, the soft output
    of slice 2 (here its own LLR, scaled like a converged posterior) as the
    prior of slice 3.  fp32 output is the fp64 value rounded (one ulp)."""
    N = (1 << 20) + 7
    x, y = inputs.gaussian_pairs(N, SNR, seed=62)
    S = oracle.quantize(y, TH4, 4)
    lam = np.zeros((4, N), np.float32)
    lam[2] = (4.0 * oracle.slice_llr(x, SIG, TH4, 4, oracle.GRAY, 2, 0b11, S)).astype(np.float32)
    L32 = api.slice_llr_prior(_g(x), SIG, TH4, 4, 3, 0b11, _g(S), 0b100, _g(lam), out_dtype=api.F32)
    torch.cuda.synchronize()
    ref = oracle.slice_llr_prior(x, SIG, TH4, 4, oracle.GRAY, 3, 0b11, S, 0b100, lam).astype(np.float32)
    got = L32.cpu().numpy()
    assert np.isfinite(ref).all()
    ulp = np.spacing(np.abs(ref)).astype(np.float64)
    assert (np.abs(got.astype(np.float64) - ref) <= ulp).all()


def test_slice_llr_prior_hard_priors_equal_known_slices_on_gpu():
    N = 50_001
    x, y = inputs.gaussian_pairs(N, SNR, seed=63)
    S = oracle.quantize(y, TH4, 4)
    lam = np.where(S == 0, np.inf, -np.inf).astype(np.float32)
    Lp = api.slice_llr_prior(_g(x), SIG, TH4, 4, 3, 0b11, _g(S), 0b100, _g(lam), out_dtype=api.F64)
    Lk = api.slice_llr(_g(x), SIG, TH4, 4, 3, 0b111, _g(S), out_dtype=api.F64)
    torch.cuda.synchronize()
    err = np.abs(Lp.cpu().numpy() - Lk.cpu().numpy()) / np.maximum(1.0, np.abs(Lk.cpu().numpy()))
    assert err.max() <= 1e-13


@pytest.mark.parametrize("n", [(1 << 20) + 5, 1003, 1, 0])
def test_slice_llr_bsc_parity(n):
    print(f"[slice_llr_bsc n={n}]", flush=True)
    x, _ = inputs.gaussian_pairs(max(n, 1), SNR, seed=64)
    x = x[:n].copy()
    if n > 100:
        x[:15] = TH4                            # values on a threshold go up, as in the quantiser
    xg = _g(x)
    for j, p in [(0, 0.31), (1, 0.22), (2, 0.11), (3, 0.013)]:
        L64 = api.slice_llr_bsc(xg, TH4, 4, j, p, out_dtype=api.F64)
        L32 = api.slice_llr_bsc(xg, TH4, 4, j, p, out_dtype=api.F32)
        torch.cuda.synchronize()
        ref = oracle.slice_llr_bsc(x, TH4, 4, oracle.GRAY, j, p)
        g64 = L64.cpu().numpy()
        np.testing.assert_array_equal(np.signbit(g64), np.signbit(ref))
        np.testing.assert_allclose(g64, ref, rtol=4.5e-16, atol=0)
        r32 = ref.astype(np.float32)
        ulp = np.spacing(np.abs(r32)).astype(np.float64)
        assert (np.abs(L32.cpu().numpy().astype(np.float64) - r32) <= ulp).all()


@pytest.mark.parametrize("which", ["regular", "qc2", "qc3", "qc_z96", "qc_z32", "met_z64", "qc_z32_f77"])
def test_syndrome_bit_exact(which):
    """Explicit codes take the gather kernel, QC codes the circulant kernel
    (Z = 512, 96: not a power of two, 32: below a wavefront, 64: MET); 77
    frames take several frames per thread with a ragged last group."""
    print(f"[syndrome {which}]", flush=True)
    if which == "regular":
        csr = inputs.regular_code(1024, 3, 6, seed=1)
        code = api.Code.from_csr(csr)
        F = 200
    else:
        qc = {"qc2": lambda: inputs.slice_code_spec(2, 65536), "qc3": lambda: inputs.slice_code_spec(3, 65536),
              "qc_z96": lambda: inputs.slice_code_spec(2, 128 * 96),
              "qc_z32": lambda: inputs.lambda_half_rate_spec(4096),
              "qc_z32_f77": lambda: inputs.lambda_half_rate_spec(4096),
              "met_z64": lambda: inputs.met_low_rate_spec(4096)}[which]()
        csr = qc.to_csr()
        code = api.Code.from_qc(qc)
        F = 77 if which.endswith("f77") else (16 if qc.Z >= 512 else 7)
    bits = inputs.random_bits((F, csr.n), seed=11)
    ref_s = inputs.random_bits((F, csr.m), seed=12)
    s_g, u_g = api.syndrome_check(code, _g(bits), _g(ref_s))
    torch.cuda.synchronize()
    s_o, u_o = oracle.syndrome(csr, bits, ref_s)
    np.testing.assert_array_equal(s_g.cpu().numpy(), s_o)
    np.testing.assert_array_equal(u_g.cpu().numpy(), u_o)
    # a word's own syndrome is satisfied
    _, u_self = api.syndrome_check(code, _g(bits), s_g.contiguous(), want_syndrome=False)
    assert (u_self.cpu().numpy() == 0).all()
