"""GPU parity of the differentiable unrolled min-sum (forward and adjoint)
against the oracle, plus determinism and the autograd wrapper."""
import numpy as np
import pytest
import torch

import oracle
from paper_2108_08418_amd import api, inputs

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _g(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _setup(n, F, T, seed):
    qc = inputs.lambda_half_rate_spec(n)
    csr = qc.to_csr()
    rng = np.random.default_rng(seed)
    bits = inputs.random_bits((F, n), seed=seed + 1)
    s2 = inputs.sigma2_from_ebn0(rng.uniform(1.5, 3.0, F), 0.5)
    llr = inputs.bpsk_llr(bits, s2, seed=seed + 2).astype(np.float32)
    syn, _ = oracle.syndrome(csr, bits)
    w = rng.uniform(0.6, 0.9, (T, qc.n_types)).astype(np.float32)
    code = api.Code.from_qc(qc)
    batch = api.Batch.uniform(code, F)
    return qc, csr, bits, llr, syn, w, code, batch


@pytest.mark.parametrize("n,F,T,K", [(1024, 6, 20, 5), (16384, 8, 20, 5), (4096, 5, 7, 3), (2048, 3, 4, 1)])
def test_forward_equals_decoder_and_binary32_oracle(n, F, T, K):
    print(f"[unrolled fwd n={n} T={T} K={K}]", flush=True)
    qc, csr, bits, llr, syn, w, code, batch = _setup(n, F, T, seed=n + T)
    post, _ = api.nms_unrolled_fwd(batch, T, K, _g(w), _g(llr.reshape(-1)), _g(syn.reshape(-1)))
    p = api.Params(algo=api.NMS, max_iter=T, early_stop=False, math=api.F32, store=api.F32, weights=_g(w))
    dec = api.ldpc_decode_batch(batch, p, _g(llr.reshape(-1)), _g(syn.reshape(-1)))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(post.cpu().numpy(), dec["post"].cpu().numpy())
    ref = oracle.nms_unrolled(csr, llr.astype(np.float64), syn, bits, w.astype(np.float64), prec32=True)
    np.testing.assert_array_equal(post.cpu().numpy().reshape(F, n).astype(np.float64), ref["post"])


@pytest.mark.parametrize("n,F,T,K", [(256, 4, 20, 5), (1024, 6, 20, 5), (16384, 4, 20, 5), (2048, 3, 9, 4)])
def test_gradient_matches_oracle(n, F, T, K):
    print(f"[unrolled grad n={n} T={T} K={K}]", flush=True)
    qc, csr, bits, llr, syn, w, code, batch = _setup(n, F, T, seed=3 * n + T)
    wg = _g(w).requires_grad_(True)
    lg = _g(llr.reshape(-1)).requires_grad_(True)
    post = api.NMSUnrolled.apply(wg, lg, _g(syn.reshape(-1)), batch, T, K)
    target = _g(bits.reshape(-1).astype(np.float32))
    # BCE of P(bit = 1) = sigmoid(-L) against the true bits, mean over all bits,
    # written as softplus(-(1 - 2b) L) so that its derivative stays accurate
    # for confidently decoded bits
    loss = torch.nn.functional.softplus(-(1 - 2 * target) * post).mean()
    loss.backward()
    torch.cuda.synchronize()
    ref = oracle.nms_unrolled(csr, llr.astype(np.float64), syn, bits, w.astype(np.float64), want_dllr=True, prec32=True)
    assert abs(loss.item() - ref["loss"]) <= 1e-5 * abs(ref["loss"])
    dw = wg.grad.cpu().numpy().astype(np.float64)
    scale = np.abs(ref["dw"]).max()
    np.testing.assert_allclose(dw, ref["dw"], rtol=1e-4, atol=1e-4 * scale)
    dl = lg.grad.cpu().numpy().reshape(F, n).astype(np.float64)
    np.testing.assert_allclose(dl, ref["dllr"], rtol=1e-4, atol=1e-4 * np.abs(ref["dllr"]).max())


def test_backward_is_deterministic():
    qc, csr, bits, llr, syn, w, code, batch = _setup(16384, 16, 20, seed=77)
    post, ck = api.nms_unrolled_fwd(batch, 20, 5, _g(w), _g(llr.reshape(-1)), _g(syn.reshape(-1)))
    g = torch.randn(post.numel(), device=DEV, generator=torch.Generator(device=DEV).manual_seed(1)) * 1e-3
    a, _ = api.nms_unrolled_bwd(batch, 20, 5, _g(w), _g(llr.reshape(-1)), _g(syn.reshape(-1)), ck, g)
    b, _ = api.nms_unrolled_bwd(batch, 20, 5, _g(w), _g(llr.reshape(-1)), _g(syn.reshape(-1)), ck, g)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())


def test_checkpoint_interval_does_not_change_results():
    qc, csr, bits, llr, syn, w, code, batch = _setup(4096, 4, 12, seed=5)
    outs = []
    for K in (1, 3, 5, 12):
        wg = _g(w).requires_grad_(True)
        post = api.NMSUnrolled.apply(wg, _g(llr.reshape(-1)), _g(syn.reshape(-1)), batch, 12, K)
        tb = _g(bits.reshape(-1).astype(np.float32))
        loss = torch.nn.functional.softplus(-(1 - 2 * tb) * post).mean()
        loss.backward()
        outs.append((post.detach().cpu().numpy(), wg.grad.cpu().numpy()))
    for p, gw in outs[1:]:
        np.testing.assert_array_equal(p, outs[0][0])
        np.testing.assert_array_equal(gw, outs[0][1])


def test_training_step_at_full_size_against_oracle():
    """The training workload the benchmark times (256 frames of 16384 bits of
    the rate-1/2 lambda(x) code, Eb/N0 uniform in [1.5, 3] dB, 20 iterations,
    checkpoints every 5, weights at their initial 0.75): forward posteriors
    bit-exact against the oracle's binary32 unrolled min-sum on every frame,
    loss within 1e-5 and the weight gradient (a sum over all 256 frames)
    within 1e-4 of the largest component of the oracle's fp64 reverse pass."""
    print("[unrolled training step at full size: 256 x 16384, T = 20, K = 5]", flush=True)
    from paper_2108_08418_amd.train import BpskFrames
    n, F, T, K = 16384, 256, 20, 5
    qc = inputs.lambda_half_rate_spec(n)
    frames = BpskFrames(qc, F, (1.5, 3.0), 0.5, torch.device(DEV))
    llr, syn, bits = frames.batch(0)
    batch = api.Batch.uniform(frames.code, F)
    w = np.full((T, qc.n_types), 0.75, dtype=np.float32)
    wg = _g(w).requires_grad_(True)
    post = api.NMSUnrolled.apply(wg, llr, syn, batch, T, K)
    sign = 1.0 - 2.0 * bits.to(torch.float32)
    loss = torch.nn.functional.softplus(-sign * post).mean()
    loss.backward()
    torch.cuda.synchronize()
    csr = qc.to_csr()
    ref = oracle.nms_unrolled(csr, llr.cpu().numpy().reshape(F, n).astype(np.float64), syn.cpu().numpy().reshape(F, -1),
                              bits.cpu().numpy().reshape(F, n), w.astype(np.float64), prec32=True)
    np.testing.assert_array_equal(post.detach().cpu().numpy().reshape(F, n).astype(np.float64), ref["post"])
    assert abs(loss.item() - ref["loss"]) <= 1e-5 * abs(ref["loss"])
    dw = wg.grad.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(dw, ref["dw"], rtol=1e-4, atol=1e-4 * np.abs(ref["dw"]).max())
