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
