"""ldpc_decode_batch_noalloc (the decode with the library's static workspace)
against ldpc_decode_batch through the C ABI: identical outputs on two calls
in a row, the second with a smaller batch, on every schedule; an oversized
batch is refused before anything is enqueued."""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

import oracle
from paper_2108_08418_amd import api, inputs

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
SNR = 3.0
TH4 = inputs.equiprobable_thresholds(4, 1.0 + 1.0 / SNR)


def _stage(j, n, F, seed):
    x, y = inputs.gaussian_pairs(n * F, SNR, seed=seed)
    S = oracle.quantize(y, TH4, 4)
    L = oracle.slice_llr(x, math.sqrt(1.0 / SNR), TH4, 4, oracle.GRAY, j, (1 << j) - 1, S)
    qc = inputs.slice_code_at(j, n, 71 if j == 3 else 104)     # converges within 40 iterations
    syn, _ = oracle.syndrome(qc.to_csr(), S[j].reshape(F, n))
    return qc, L.astype(np.float32), syn.reshape(-1)


def _outs(batch, want_post=True):
    return dict(bits=torch.full((batch.total_n,), 7, dtype=torch.uint8, device=DEV),
                post=torch.full((batch.total_n,), float("nan"), dtype=torch.float32, device=DEV) if want_post else None,
                iters=torch.full((batch.F,), -7, dtype=torch.int32, device=DEV),
                ok=torch.full((batch.F,), 7, dtype=torch.uint8, device=DEV))


@pytest.mark.parametrize("sched", [api.SCHED_PERSISTENT, api.SCHED_GROUP, api.SCHED_LAYERED, api.SCHED_PASSES])
def test_noalloc_equals_decode_with_workspace(sched):
    print(f"[noalloc sched={sched}]", flush=True)
    cases = [(3, 16384, 12, 801, api.SP, api.F32), (3, 4096, 5, 802, api.NMS, api.F16)]   # second call smaller
    for j, n, F, seed, algo, store in cases:
        qc, L, syn = _stage(j, n, F, seed)
        code = api.Code.from_qc(qc)
        batch = api.Batch.uniform(code, F)
        p = api.Params(algo=algo, max_iter=40, math=api.F32, store=store, alpha=0.8, schedule=sched)
        assert api.decode_workspace_size(batch, p) <= api.NOALLOC_SCRATCH_BYTES
        llr = torch.from_numpy(L).to(DEV)
        sg = torch.from_numpy(syn).to(DEV)
        ref = api.ldpc_decode_batch(batch, p, llr, sg)
        got = api.ldpc_decode_batch_noalloc(batch, p, llr, sg, _outs(batch))
        torch.cuda.synchronize()
        for k in ("bits", "post", "iters", "ok"):
            assert torch.equal(ref[k], got[k]), f"{k} differs (j={j}, n={n}, F={F})"
        assert int(got["ok"].sum()) >= 1
        # without posteriors
        got2 = api.ldpc_decode_batch_noalloc(batch, p, llr, sg, _outs(batch, want_post=False))
        torch.cuda.synchronize()
        for k in ("bits", "iters", "ok"):
            assert torch.equal(ref[k], got2[k])


def test_noalloc_refuses_a_batch_beyond_its_array():
    print("[noalloc oversize]", flush=True)
    qc = inputs.slice_code_spec(3, 65536)
    code = api.Code.from_qc(qc)
    batch = api.Batch.uniform(code, 64)                  # 64 x 233k fp32 messages > 64 MiB
    p = api.Params(algo=api.SP, max_iter=10, math=api.F32, store=api.F32)
    assert api.decode_workspace_size(batch, p) > api.NOALLOC_SCRATCH_BYTES
    llr = torch.zeros(batch.total_n, dtype=torch.float32, device=DEV)
    out = _outs(batch)
    with pytest.raises(api._lib.CvrError, match="CVR_ENOMEM"):
        api.ldpc_decode_batch_noalloc(batch, p, llr, None, out)
    torch.cuda.synchronize()
    assert int(out["iters"][0]) == -7                     # nothing was written
