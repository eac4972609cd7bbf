"""Learning the per-iteration, per-edge-type scales of normalized min-sum.

The decoder is unrolled for T iterations (no early stop) through
``api.NMSUnrolled``: forward and backward run in the library's kernels; the
loss is the binary cross-entropy of P(bit = 1) = sigmoid(-L_post(T)) against
the transmitted bits, averaged over all bits, and Adam updates the T x
n_types weights.

Two frame sources:
* ``bpsk``  -- random words with their syndromes over BPSK/AWGN, Eb/N0 drawn
  uniformly per frame from a range (the rate-1/2 training workload);
* ``slice`` -- the slice-reconciliation channel of a coded slice: Gaussian
  pairs at the given SNR, Bob's quantiser and syndrome, Alice's slice LLRs
  given the lower slices (all through the library).

Training seeds are disjoint from the evaluation seeds used elsewhere
(offset 10^6).
"""
from __future__ import annotations

import argparse
import json
import math
import time
from pathlib import Path

import numpy as np
import torch

from . import api, inputs

SEED_OFFSET = 1_000_000
WEIGHTS_DIR = Path(__file__).resolve().parent / "weights"


class BpskFrames:
    def __init__(self, qc, F, ebn0_range, rate, dev):
        self.qc, self.F, self.lo, self.hi, self.rate, self.dev = qc, F, ebn0_range[0], ebn0_range[1], rate, dev
        self.code = api.Code.from_qc(qc)

    def batch(self, step):
        seed = SEED_OFFSET + 7919 * step
        rng = np.random.default_rng(seed)
        bits = inputs.random_bits((self.F, self.qc.n), seed=seed + 1)
        s2 = inputs.sigma2_from_ebn0(rng.uniform(self.lo, self.hi, self.F), self.rate)
        llr = inputs.bpsk_llr(bits, s2, seed=seed + 2).astype(np.float32)
        b = torch.from_numpy(bits.reshape(-1)).to(self.dev)
        syn, _ = api.syndrome_check(self.code, b, want_unsat=False)
        return torch.from_numpy(llr.reshape(-1)).to(self.dev), syn.view(-1), b


class SliceFrames:
    def __init__(self, j, n, F, snr, dev, m_bits=4, mb=None):
        self.j, self.n, self.F, self.snr, self.dev, self.m = j, n, F, snr, dev, m_bits
        self.th = inputs.equiprobable_thresholds(m_bits, 1.0 + 1.0 / snr)
        self.sig = math.sqrt(1.0 / snr)
        self.qc = inputs.slice_code_spec(j, n) if mb is None else inputs.slice_code_at(j, n, mb)
        self.code = api.Code.from_qc(self.qc)

    def batch(self, step):
        x, y = inputs.gaussian_pairs(self.F * self.n, self.snr, seed=SEED_OFFSET + 104729 * step + self.j)
        xg = torch.from_numpy(x).to(self.dev)
        yg = torch.from_numpy(y).to(self.dev)
        S = api.slice_quantize(yg, self.th, self.m)
        syn, _ = api.syndrome_check(self.code, S[self.j].contiguous(), want_unsat=False)
        llr = api.slice_llr(xg, self.sig, self.th, self.m, self.j, (1 << self.j) - 1, S)
        return llr, syn.view(-1), S[self.j].contiguous()


def train(frames, T, K=5, steps=200, lr=0.02, init=0.75, log_every=10, log=print):
    dev = frames.dev
    code = frames.code
    batch = api.Batch.uniform(code, frames.F)
    w = torch.full((T, code.n_types), float(init), dtype=torch.float32, device=dev, requires_grad=True)
    opt = torch.optim.Adam([w], lr=lr)
    hist = []
    t0 = time.time()
    for step in range(steps):
        llr, syn, bits = frames.batch(step)
        post = api.NMSUnrolled.apply(w, llr, syn, batch, T, K)
        # BCE of sigmoid(-L) against the bits, as softplus(-(1 - 2b) L)
        loss = torch.nn.functional.softplus(-(1 - 2 * bits.to(torch.float32)) * post).mean()
        opt.zero_grad()
        loss.backward()
        opt.step()
        with torch.no_grad():
            w.clamp_(0.05, 1.5)
        if step % log_every == 0 or step == steps - 1:
            ber = float(((post < 0).to(torch.uint8) != bits).float().mean())
            hist.append(dict(step=step, loss=float(loss), ber=ber, t=time.time() - t0))
            log(f"step {step:4d} loss {float(loss):.5f} ber {ber:.3e} ({time.time() - t0:.1f}s)")
    return w.detach().cpu().numpy(), hist


def save(path, name, weights, meta):
    path = Path(path)
    path.parent.mkdir(parents=True, exist_ok=True)
    path.write_text(json.dumps(dict(name=name, T=int(weights.shape[0]), n_types=int(weights.shape[1]),
                                    weights=np.asarray(weights, dtype=float).round(7).tolist(), **meta), indent=1))


def weights_meta(name: str) -> dict:
    """The stored record of a weight set without its weights (code, mb, training)."""
    d = json.loads((WEIGHTS_DIR / f"{name}.json").read_text())
    d.pop("weights", None)
    return d


def load_weights(name: str, extend_to: int | None = None) -> np.ndarray:
    """Weights [T, n_types] stored under ``weights/<name>.json``; with
    ``extend_to`` > T the last learned row is held for the extra iterations."""
    d = json.loads((WEIGHTS_DIR / f"{name}.json").read_text())
    w = np.asarray(d["weights"], dtype=np.float32)
    if extend_to is not None and extend_to > w.shape[0]:
        w = np.concatenate([w, np.repeat(w[-1:], extend_to - w.shape[0], axis=0)])
    return w


def layered_weights(w: np.ndarray, steps: float = 2) -> np.ndarray:
    """Per-iteration weights for the layered schedule from weights learned
    through the flooding decoder: layered iteration t takes flooding
    iteration ``steps * t`` rounded to the nearest integer (ties to even; the
    last row held beyond), since one layered iteration, which updates every
    check with the newest messages, carries information about as far as two
    flooding iterations.  Same shape as w."""
    if not steps >= 1:
        raise ValueError("steps must be >= 1")
    T = w.shape[0]
    return np.ascontiguousarray(w[np.minimum(np.round(steps * np.arange(T)).astype(np.int64), T - 1)])


def main():
    ap = argparse.ArgumentParser(description="learn normalized min-sum scales")
    ap.add_argument("--source", choices=["bpsk", "slice"], required=True)
    ap.add_argument("--slice", type=int, default=2)
    ap.add_argument("--mb", type=int, default=0, help="block rows of the slice code (0 = the selected rate)")
    ap.add_argument("--n", type=int, default=16384)
    ap.add_argument("--frames", type=int, default=256)
    ap.add_argument("--T", type=int, default=20)
    ap.add_argument("--K", type=int, default=5)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--lr", type=float, default=0.02)
    ap.add_argument("--init", type=float, default=0.75)
    ap.add_argument("--out", required=True)
    ap.add_argument("--name", required=True)
    a = ap.parse_args()
    dev = torch.device("cuda:0")
    if a.source == "bpsk":
        fr = BpskFrames(inputs.lambda_half_rate_spec(a.n), a.frames, (1.5, 3.0), 0.5, dev)
        meta = dict(source="bpsk", code=fr.qc.name, ebn0_db=[1.5, 3.0])
    else:
        fr = SliceFrames(a.slice, a.n, a.frames, 3.0, dev, mb=a.mb or None)
        meta = dict(source="slice", code=fr.qc.name, slice=a.slice, snr=3.0, mb=int(fr.qc.mb), T_train=a.T)
    w, hist = train(fr, a.T, a.K, a.steps, a.lr, a.init, log=lambda s: print(s, flush=True))
    meta.update(frames=a.frames, n=a.n, steps=a.steps, lr=a.lr, init=a.init, ckpt_every=a.K, history=hist)
    save(a.out, a.name, w, meta)
    print(json.dumps(dict(name=a.name, weights=w.round(4).tolist())))


if __name__ == "__main__":
    main()
