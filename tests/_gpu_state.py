"""Reading a decoder's state after exactly t iterations through the C ABI
(test helper: the state a one-step comparison with the oracle starts from)."""
from __future__ import annotations

from dataclasses import replace

import numpy as np
import torch

from paper_2108_08418_amd import api


def state_csr(qc, msg):
    """Messages of one frame from the decoder's [block][k] layout (blocks in
    row-major protograph order) to the CSR edge order of qc.to_csr()."""
    csr = qc.to_csr()
    out = np.zeros(csr.n_edges)
    Z = qc.Z
    k = np.arange(Z)
    q = 0
    for i in range(qc.mb):
        cols = np.nonzero(qc.shift[i] >= 0)[0]
        base = csr.row_ptr[i * Z + k]
        for qq in range(len(cols)):
            out[base + qq] = msg[(q + qq) * Z + k]
        q += len(cols)
    return out


def decoded_for(code, qc, p, llr1, syn1, t, device="cuda"):
    """One frame decoded for exactly t iterations: (posteriors, stored messages
    in CSR order, both as fp64).  The messages are the decoder's state at the
    start of its workspace (zero before the first iteration); the posteriors
    are the flooding decoder's L_post or the layered decoder's running L."""
    batch = api.Batch.uniform(code, 1)
    pt = replace(p, max_iter=t, early_stop=False)
    ws = api.alloc_workspace(batch, pt)
    mdt = np.float64 if p.math == api.F64 else np.float32
    g = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(device)
    out = api.ldpc_decode_batch(batch, pt, g(llr1.astype(mdt)), g(syn1), workspace=ws)
    torch.cuda.synchronize()
    post = out["post"].cpu().numpy().astype(np.float64)
    if t == 0:
        return post, np.zeros(qc.to_csr().n_edges)
    sdt, size = {api.F16: (torch.float16, 2), api.F32: (torch.float32, 4), api.F64: (torch.float64, 8)}[p.store]
    nb_z = int((qc.shift >= 0).sum()) * qc.Z
    msg = ws[: nb_z * size].view(sdt).cpu().numpy().astype(np.float64)
    return post, state_csr(qc, msg)
