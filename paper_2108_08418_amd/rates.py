"""Rate selection for the coded slices (Sec. V-B), run on the GPU path.

Start 10 % below the slice capacity C_j (Sec. V-B uses codes about 10 % below
capacity) and step the rate down by 0.05 until a candidate code decodes every
test sub-block with BP.  The test: Bob's slices from seeded Gaussian pairs,
their syndromes, Alice's slice LLRs given the true lower slices, flooding
sum-product with early stop; a candidate passes when no sub-block fails and
none converges to a word other than Bob's.  Each candidate also carries the
Gaussian-approximation iteration count to bit error ratio 1/n (Sec. III-C)
beside the measured mean, and C_j is estimated from the LLRs themselves.

Every step runs through the library (quantiser, syndromes, slice LLRs,
decoder); the host only builds candidate codes and counts.
"""
from __future__ import annotations

import math

import torch

from . import api, ga, inputs

NB = 128          # block columns of the slice-code protograph


def select_slice_rate(slice_j: int, n: int, frames: int = 64, snr: float = 3.0, m_bits: int = 4,
                      start_frac: float = 0.9, step: float = 0.05, max_iter: int = 100,
                      seed: int = 5150, code_seed: int = 2108, device: str = "cuda") -> dict:
    """Returns dict(capacity, trail=[candidate dicts, in test order], selected=the
    passing candidate or None).  A candidate: target rate, mb, rate = 1 - mb/128,
    failures, undetected (converged to a wrong word), mean_iters, ga_iters."""
    if slice_j < 1 or slice_j >= m_bits:
        raise ValueError("slice_j must be a coded slice above the lowest one")
    sig = math.sqrt(1.0 / snr)
    th = inputs.equiprobable_thresholds(m_bits, 1.0 + 1.0 / snr)
    x_np, y_np = inputs.gaussian_pairs(frames * n, snr, seed)
    x = torch.from_numpy(x_np).to(device)
    y = torch.from_numpy(y_np).to(device)
    S = api.slice_quantize(y, th, m_bits)
    llr = api.slice_llr(x, sig, th, m_bits, slice_j, (1 << slice_j) - 1, S)
    bob = S[slice_j].view(frames, n)
    sgn = 1.0 - 2.0 * S[slice_j].to(torch.float64)
    cap = 1.0 - float(torch.nn.functional.softplus(-sgn * llr.to(torch.float64)).mean()) / math.log(2.0)
    m0 = ga.biawgn_mean_for_capacity(cap)
    params = api.Params(algo=api.SP, max_iter=max_iter, math=api.F32, store=api.F32)
    trail = []
    seen = set()
    target = start_frac * cap
    while target > 0.0:
        mb = int(round(NB * (1.0 - target)))
        if mb >= NB:
            break
        if mb not in seen:
            seen.add(mb)
            qc = inputs.slice_code_at(slice_j, n, mb, code_seed)
            code = api.Code.from_qc(qc)
            batch = api.Batch.uniform(code, frames)
            syn, _ = api.syndrome_check(code, bob, want_unsat=False)
            out = api.ldpc_decode_batch(batch, params, llr, syn.view(-1), want_post=False)
            torch.cuda.synchronize()        # code and batch are released when rebound
            api.check_abandoned(out)
            ok = out["ok"].to(torch.bool)
            wrong = (out["bits"].view(frames, n) != bob).any(dim=1)
            csr = qc.to_csr()
            lam, rho = ga.degree_distributions(csr.row_ptr, csr.col_idx, n)
            cand = {"target": round(target, 4), "mb": mb, "rate": 1.0 - mb / NB,
                    "failures": int((~ok).sum().item()), "undetected": int((ok & wrong).sum().item()),
                    "mean_iters": float(out["iters"].to(torch.float64).mean().item()),
                    "ga_iters": ga.iterations_to(1.0 / n, m0, lam, rho)}
            trail.append(cand)
            if cand["failures"] == 0 and cand["undetected"] == 0:
                return {"capacity": cap, "trail": trail, "selected": cand}
        target -= step
    return {"capacity": cap, "trail": trail, "selected": None}
