"""Benchmark of the slice-reconciliation hot path on one MI355X.

A step is one pass of the whole path over one batch of synthetic pairs:
Bob quantises y into 16 equiprobable Gray intervals (4 slices) and computes
the syndromes of slices 2 and 3; slices 0 and 1 are disclosed; Alice forms
slice-2 LLRs from x and slices 0-1, decodes every sub-block of slice 2, forms
slice-3 LLRs from x and slices 0-2 and decodes slice 3.  Inputs are resident
in HBM before the timed region.

Prints one JSON line.  ``value`` = decoded (coded-slice) bits per second.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

DEFAULT_WORKLOAD = "recon-2^27-nR2^16"
WORKLOADS = {
    # 2^27 pairs at SNR 3 split into sub-blocks of 2^16: the n_R = 2^16 point
    # of the block-size sweep, with the 16-level / 4-slice setup
    "recon-2^27-nR2^16": dict(N=1 << 27, n=1 << 16),
    # 2^20 pairs, 16 sub-blocks of 65536
    "recon-2^20-nR2^16": dict(N=1 << 20, n=1 << 16),
    # other sweep points
    "recon-2^27-nR2^12": dict(N=1 << 27, n=1 << 12),
    "recon-2^27-nR2^14": dict(N=1 << 27, n=1 << 14),
    "recon-2^27-nR2^18": dict(N=1 << 27, n=1 << 18),
    "recon-2^27-nR2^20": dict(N=1 << 27, n=1 << 20),
    # 4096 sub-blocks of mixed length (2176 x 4096, 1024 x 16384, 640 x 65536,
    # 256 x 262144; seeded order) of a low-rate multi-edge-type code, BPSK at
    # SNR 0.16, decoded in one persistent launch
    "ragged-4096-frames": dict(kind="ragged", sizes=(4096, 16384, 65536, 262144), counts=(2176, 1024, 640, 256),
                               snr=0.16),
    # one training step of the differentiable unrolled min-sum: 256 frames of
    # the rate-1/2 code (n = 16384), Eb/N0 uniform in [1.5, 3] dB, 20 iterations,
    # 20 x 3 weights, checkpoints every 5 iterations; forward, BCE loss, adjoint,
    # Adam update
    "train-nms-r12-n16384-T20": dict(kind="train", n=16384, F=256, T=20, K=5),
}
SNR = 3.0
M_BITS = 4
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default=DEFAULT_WORKLOAD, choices=sorted(WORKLOADS))
    ap.add_argument("--decoder", default="both", choices=["both", "sp", "nms"],
                    help="both: layered sum-product (the headline), flooding sum-product and learned min-sum, "
                         "timed one after the other")
    ap.add_argument("--max-iter", type=int, default=100)
    ap.add_argument("--alpha", type=float, default=0.75)
    ap.add_argument("--weights", default="", help="learned min-sum weights: stored set name prefix "
                    "(weights/<prefix>_slice<j>.json per coded slice); iterations past their T reuse "
                    "the last learned row up to --max-iter")
    ap.add_argument("--s-be", type=float, default=None,
                    help="Holevo bound S_BE per pair: adds the experimental key rate K'_exp (Sec. V) of each "
                         "reconciliation step to its line (with --sweep: K'_exp against the sub-block length)")
    ap.add_argument("--layered-weight-steps", type=float, default=2,
                    help="on the layered schedule, iteration t uses the learned (flooding) weights of "
                         "iteration steps * t (1: the same index)")
    ap.add_argument("--schedule", default="auto", choices=["auto", "passes", "persistent", "group", "layered"])
    ap.add_argument("--group-wgs", dest="group_wgs", type=int, default=0,
                    help="workgroups per frame of the group schedule (0 = auto)")
    ap.add_argument("--wg", type=int, default=0, help="persistent decoder workgroup size (0 = default)")
    ap.add_argument("--min-waves", dest="min_waves", type=int, default=0, help="0 or 8 resident waves per SIMD")
    ap.add_argument("--lds-cache", dest="lds_cache_kb", type=int, default=0,
                    help="LDS posterior cache KiB of the persistent decoder (0 = auto, -1 = none)")
    ap.add_argument("--cpu-frames", type=int, default=48, help="sub-blocks per stage in the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-other-workloads", action="store_true",
                    help="with the default workload, skip the uneven-batch and training-step summaries")
    ap.add_argument("--seed", type=int, default=2108)
    ap.add_argument("--graph", action="store_true", help="replay the decode from a captured HIP graph")
    ap.add_argument("--sweep", action="store_true",
                    help="block-size sweep: every recon-2^27 workload with flooding and layered sum-product and "
                         "with learned min-sum (--weights, default 'learned'), flooding and layered; prints one JSON "
                         "line per point")
    ap.add_argument("--no-tune", action="store_true", help="skip the launch-shape autotuner (untimed)")
    ap.add_argument("--no-rate-selection", action="store_true",
                    help="use the stored rate table instead of running the Sec. V-B selection loop (untimed)")
    ap.add_argument("--rate-frames", type=int, default=256, help="test sub-blocks of the rate-selection loop")
    ap.add_argument("--fer-seeds", type=int, default=5,
                    help="input seeds over which frame-error rates are counted (the timed one and more, untimed)")
    ap.add_argument("--llr-forms", action="store_true",
                    help="only time Alice's three LLR forms for slice 3 at 2^27 pairs (hard lower slices, "
                         "slice 2 as a soft prior, binary-symmetric hard LLR) and exit")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run one device-to-device copy of MIB MiB (HBM counter calibration) and exit")
    return ap.parse_args()


# The paper's own measurements (Sec. V), other hardware and codes: context only.
PAPER_CONTEXT = {
    "hardware": "NVIDIA GTX 1060, one decoder per GPU thread",
    "slice_bits_per_s": 1.6e7,
    "edge_updates_per_s": 4.46e7,
    "source": "Sec. V: 310 s to decode the m N = 5e9 slice bits of N = 1e9 at N_R = 1e9; "
              "3.2e-9 s per operation at 7 operations per edge and iteration (Sec. III-C), "
              "i.e. 1 / (7 x 3.2e-9) edge updates per second",
}


def wilson95(k: int, F: int):
    """Wilson score interval (95 %) of a frame-error rate with k failures in F frames."""
    if F <= 0:
        return None
    z, p = 1.959963984540054, k / F
    den = 1.0 + z * z / F
    mid = (p + z * z / (2 * F)) / den
    half = z * math.sqrt(p * (1 - p) / F + z * z / (4 * F * F)) / den
    return [max(0.0, mid - half), min(1.0, mid + half)]


# sources each recorded kernel is built from: the decoders, and the adjoint
# of unrolled min-sum, which adds its own translation unit
DECODER_SOURCES = ("cvr_decode_impl.h", "cvr_internal.h", "cvr_decode.hip", "cvr_codes.hip")
ADJOINT_SOURCES = DECODER_SOURCES + ("cvr_nms_grad.hip",)


def csrc_hash(kernel_name: str = "") -> str:
    """Hash of the sources a kernel is built from (a recorded traffic figure
    is valid while it is unchanged): the adjoint kernel's, or the decoders'."""
    import hashlib
    from pathlib import Path
    names = ADJOINT_SOURCES if "k_nms_bwd" in kernel_name else DECODER_SOURCES
    h = hashlib.sha256()
    csrc = Path(ROOT) / "paper_2108_08418_amd" / "csrc"
    for p in sorted(csrc.glob("*")):
        if p.name in names or p.name.startswith("cvr_dec_"):
            h.update(p.read_bytes())
    return h.hexdigest()[:16]


def recorded_traffic(kernel_name: str, workload: str, decoder: str, weights: str):
    """HBM bytes per launch (calibrated FETCH_SIZE + WRITE_SIZE) recorded under
    profiles/ for this kernel instantiation, workload, decoder and weights, or None when
    no record exists or the decoder sources changed since the counters were
    taken."""
    from pathlib import Path
    sha = csrc_hash(kernel_name)
    for p in sorted((Path(ROOT) / "profiles").glob("*_hbm_traffic.md")):
        text = p.read_text()
        if "```json" not in text:
            continue
        rec = json.loads(text.split("```json", 1)[1].split("```", 1)[0])
        if (rec.get("source_sha") == sha and rec.get("kernel", "").startswith(kernel_name)
                and rec.get("workload") == workload and rec.get("decoder") == decoder
                and rec.get("weights", "") == (weights or "")):
            return rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"], p.name
    return None, None


def recorded_valu(kernel_name: str, workload: str, decoder: str, weights: str):
    """Fraction of the chip's VALU issue slots (plain, and with quarter-rate
    transcendentals counted as four slots) recorded under profiles/ from
    rocprofv3 instruction counters for this kernel, workload, decoder and
    weights, or None when no record exists or the sources changed since."""
    from pathlib import Path
    sha = csrc_hash(kernel_name)
    for p in sorted((Path(ROOT) / "profiles").glob("*_valu_counts.md")):
        text = p.read_text()
        if "```json" not in text:
            continue
        for line in text.split("```json", 1)[1].split("```", 1)[0].strip().splitlines():
            rec = json.loads(line)
            if (rec.get("source_sha") == sha and kernel_name.startswith(rec.get("kernel", "?"))
                    and rec.get("workload") == workload and rec.get("decoder") == decoder
                    and rec.get("weights", "") == (weights or "")):
                return {"issue": rec["valu_issue"], "issue_with_transcendentals": rec["valu_issue_with_transcendentals"],
                        "source": p.name}
    return None


def frame_decode_bytes(iters, n, m, E, s_msg):
    """Algorithmic bytes of a whole decode of frames that stopped at ``iters``:
    per iteration every stored message is read and written once and L_ch,
    L_post are read and L_post written (2 s_msg E + 12 n); per syndrome test
    m syndrome bytes; set-up and output 8 n + n (+ the final test's 4 n)."""
    it = iters.astype(np.int64)
    return float((it * (2 * s_msg * E + 12 * n) + (it + 1) * m + 13 * n).sum())


def layered_decode_bytes(iters, n, m, E, s_msg):
    """Algorithmic bytes of a whole layered decode of frames that stopped at
    ``iters``: per iteration every stored message is read and written once and,
    since a block row updates the running posterior of each of its variables,
    that posterior is read and written once per edge (2 s_msg E + 8 E); per
    syndrome test m syndrome bytes (the decisions live on chip); set-up (L_ch
    read, L written) and output bits 9 n."""
    it = iters.astype(np.int64)
    return float((it * (2 * s_msg * E + 8 * E) + (it + 1) * m + 9 * n).sum())


def stage_bytes(iters, T, n, m, E, s_msg):
    """Algorithmic bytes of the check pass and of a full flooding iteration for
    frames that stopped at ``iters``.

    check pass at t (frame active): posterior gather 4n + syndrome m bytes, and
    for t < T one read (t > 0) and one write of the E stored messages.
    full iteration (per edge-iteration figure 2 s_msg + 12 / d_v): every
    message read and written once, L_ch and L_post read, L_post written.
    """
    it = iters.astype(np.int64)
    upd = np.minimum(it, T - 1) + 1 if T > 0 else np.zeros_like(it)   # passes with t < T
    reads = np.maximum(upd - 1, 0)                                       # of those, t > 0
    check = ((it + 1) * (4 * n + m) + (upd + reads) * s_msg * E).sum()
    full_iter = (it * (2 * s_msg * E + 12 * n)).sum()
    return float(check), float(full_iter)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; --gpus must be 1 "
                          "(sub-blocks shard across GPUs with no exchange; one GPU's share is what it measures)"}))
        sys.exit(2)
    import torch

    from paper_2108_08418_amd import api, inputs

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}))
        sys.exit(2)
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": nbytes, "read_bytes": nbytes, "write_bytes": nbytes}))
        return
    if args.llr_forms:
        print(json.dumps(llr_forms(args, dev)))
        return
    if args.sweep:
        import copy
        for name in sorted(k for k in WORKLOADS if k.startswith("recon-2^27")):
            for dec, wts, sched in (("sp", "", "auto"), ("sp", "", "layered"), ("nms", args.weights or "learned", "auto"),
                                    ("nms", args.weights or "learned", "layered")):
                a = copy.copy(args)
                a.workload, a.decoder, a.weights, a.no_cpu_baseline, a.schedule = name, dec, wts, True, sched
                a.fer_seeds, a.no_rate_selection = 1, True
                a.wg = a.min_waves = a.lds_cache_kb = 0
                try:
                    res = recon(a, WORKLOADS[name], dev)
                except api._lib.CvrError as e:      # a schedule that does not take this sub-block size
                    res = {"workload": name, "decoder": dec, "schedule": sched, "error": str(e)}
                print(json.dumps(res), flush=True)
        return
    wl = WORKLOADS[args.workload]
    if wl.get("kind") == "ragged":
        print(json.dumps(ragged(args, wl, dev)))
        return
    if wl.get("kind") == "train":
        print(json.dumps(train_step(args, wl, dev)))
        return
    res = recon(args, wl, dev)
    if args.workload == DEFAULT_WORKLOAD and not args.no_other_workloads:
        res["other_workloads"] = other_workloads(args, dev)
    print(json.dumps(res))


def other_workloads(args, dev):
    """The uneven MET batch (normalized min-sum, alpha 0.75, binary16
    messages, flooding and layered) and the unrolled min-sum training step,
    each timed by its own routine after the headline step (their own
    warm-up, autotuning and timed steps); the summary of each in the
    headline line."""
    import copy
    out = {}
    runs = (("ragged-4096-frames", "auto", ragged), ("ragged-4096-frames", "layered", ragged),
            ("train-nms-r12-n16384-T20", "auto", train_step))
    for name, sched, fn in runs:
        a = copy.copy(args)
        a.workload, a.decoder, a.weights, a.schedule, a.graph = name, "nms", "", sched, False
        a.wg = a.min_waves = a.lds_cache_kb = a.group_wgs = 0
        r = fn(a, WORKLOADS[name], dev)
        key = name if fn is train_step else f"{name}/{'layered' if sched == 'layered' else 'flooding'}"
        out[key] = {k: r[k] for k in ("metric", "value", "unit", "ms_per_step", "steps", "dtype", "config",
                                      "roofline", "fer", "mean_iters", "forward_ms", "adjoint_ms") if k in r}
        print(f"# {key}: {r['ms_per_step']:.2f} ms/step, {r['value']:.3e} bits/s", file=sys.stderr, flush=True)
    return out


def llr_forms(args, dev):
    """Launch time of Alice's slice-3 LLR in its three forms over 2^27 pairs at
    SNR 3 (16 equiprobable Gray levels):
      hard   - slices 0, 1, 2 held as bits (multistage decoding),
      prior  - slices 0, 1 as bits, slice 2 as a soft prior (a scaled LLR row),
      bsc    - ln((1 - p) / p) with the sign of Alice's own quantised bit;
    and the one-pass pair the benchmark step uses:
      next   - slice 2 and slice 3 for either value of slice 2, one pass,
      choose - slice 3 picked by the decoded slice 2.
    Algorithmic bytes per sample: x (8) + the slice bytes and prior rows read
    + the fp32 output (4)."""
    import torch

    from paper_2108_08418_amd import api, inputs
    N = 1 << 27
    snr = 3.0
    sig = math.sqrt(1.0 / snr)
    th = inputs.equiprobable_thresholds(M_BITS, 1.0 + 1.0 / snr)
    x_np, y_np = inputs.gaussian_pairs(N, snr, seed=args.seed)
    x = torch.from_numpy(x_np).to(dev)
    y = torch.from_numpy(y_np).to(dev)
    del x_np, y_np
    S = api.slice_quantize(y, th, M_BITS)
    prior = torch.zeros((M_BITS, N), dtype=torch.float32, device=dev)
    api.slice_llr(x, sig, th, M_BITS, 2, 0b11, S, out=prior[2])
    prior[2] *= 4.0
    out = torch.empty(N, dtype=torch.float32, device=dev)
    nx0, nx1 = torch.empty_like(out), torch.empty_like(out)
    p3 = 0.15
    forms = {
        "hard": (lambda: api.slice_llr(x, sig, th, M_BITS, 3, 0b111, S, out=out), 8 + 3 + 4),
        "prior": (lambda: api.slice_llr_prior(x, sig, th, M_BITS, 3, 0b11, S, 0b100, prior, out=out), 8 + 2 + 4 + 4),
        "bsc": (lambda: api.slice_llr_bsc(x, th, M_BITS, 3, p3, out=out), 8 + 4),
        # slice 2 and both conditional slice-3 LLRs in one pass (three fp32 outputs)
        "next": (lambda: api.slice_llr_next(x, sig, th, M_BITS, 2, 0b11, S, out=(out, nx0, nx1)), 8 + 2 + 12),
        "choose": (lambda: api.slice_llr_choose(nx0, nx1, S[2], out=out), 4 + 4 + 1 + 4),
    }
    res = {}
    for name, (fn, bps) in forms.items():
        for _ in range(max(1, args.warmup)):
            fn()
        torch.cuda.synchronize()
        api.profile_enable(True)
        api.profile_read(1, reset=True)
        for _ in range(args.steps):
            fn()
        torch.cuda.synchronize()
        api.profile_enable(False)
        ms, launches = api.profile_read(1, reset=True)
        avg = ms / max(launches, 1)
        res[name] = {"ms": round(avg, 4), "samples_per_s": N / (avg * 1e-3),
                     "bytes_per_sample": bps, "GB_s": round(N * bps / (avg * 1e-3) / 1e9, 1),
                     "hbm_frac": round(N * bps / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4), "launches": launches}
        print(f"# {name}: {avg:.3f} ms per launch", file=sys.stderr, flush=True)
    return {"llr_forms": res, "n": N, "slice": 3, "bsc_p": p3, "steps": args.steps, "warmup": args.warmup}


def _decoder_configs(args, api):
    """(key, {coded slice: (algo, store, schedule name, weights prefix)}) of the
    decoders one run times.  --decoder both (default): sum-product on the
    layered schedule (the headline), plain flooding sum-product (the baseline
    the paper's belief propagation names), learned min-sum with binary16
    messages on the flooding and on the layered schedule, on both coded
    slices, and, on the layered schedule, learned min-sum on slice 2 with
    sum-product on slice 3 (each slice's decoder picked by its FER)."""
    sp = (api.SP, api.F32, args.schedule, "")
    nms = (api.NMS, api.F16, args.schedule, args.weights)
    if args.decoder == "both":
        lay = (api.SP, api.F32, "layered", "")
        flood = (api.SP, api.F32, "auto", "")
        learned = (api.NMS, api.F16, "auto", args.weights or "learned")
        learned_lay = (api.NMS, api.F16, "layered", args.weights or "learned")
        return [("sp_layered", {2: lay, 3: lay}), ("sp", {2: flood, 3: flood}), ("nms", {2: learned, 3: learned}),
                ("nms_layered", {2: learned_lay, 3: learned_lay}), ("mixed_layered", {2: learned_lay, 3: lay})]
    if args.decoder == "sp":
        return [("sp", {2: sp, 3: sp})]
    return [("nms", {2: nms, 3: nms})]


def recon(args, wl, dev):
    """The slice-reconciliation step on N pairs in sub-blocks of n; returns the result dict."""
    from dataclasses import replace

    import torch

    from paper_2108_08418_amd import api, inputs

    N, n = wl["N"], wl["n"]
    F = N // n
    sig = math.sqrt(1.0 / SNR)
    th = inputs.equiprobable_thresholds(M_BITS, 1.0 + 1.0 / SNR)
    print(f"# workload {args.workload}: N={N} n={n} F={F} decoder={args.decoder}", file=sys.stderr, flush=True)

    # ---- inputs and codes (untimed) ----
    t0 = time.time()
    rate_sel = None
    if not args.no_rate_selection:
        # the Sec. V-B loop on its own seeded test sub-blocks of 2^16 (untimed);
        # the codes the step decodes are the ones it selects
        from paper_2108_08418_amd import rates
        rate_sel = {}
        for j in (2, 3):
            r = rates.select_slice_rate(j, 1 << 16, frames=args.rate_frames)
            if r["selected"] is None:
                raise SystemExit(f"rate selection found no passing code for slice {j}")
            rate_sel[j] = r
        mbs = {j: rate_sel[j]["selected"]["mb"] for j in (2, 3)}
        print(f"# rate selection: {mbs} ({time.time() - t0:.1f}s)", file=sys.stderr, flush=True)
    else:
        mbs = dict(inputs.SLICE_MB)
    x_np, y_np = inputs.gaussian_pairs(N, SNR, seed=args.seed)
    x = torch.from_numpy(x_np).to(dev)
    y = torch.from_numpy(y_np).to(dev)
    qcs = {j: inputs.slice_code_at(j, n, mbs[j]) for j in (2, 3)}
    codes = {j: api.Code.from_qc(qcs[j]) for j in (2, 3)}
    batches = {j: api.Batch.uniform(codes[j], F) for j in (2, 3)}
    bob = torch.empty((M_BITS, N), dtype=torch.uint8, device=dev)
    alice = torch.empty((M_BITS, N), dtype=torch.uint8, device=dev)
    syn = {j: torch.empty(F * codes[j].m, dtype=torch.uint8, device=dev) for j in (2, 3)}
    llr = torch.empty(N, dtype=torch.float32, device=dev)
    llr3 = (torch.empty(N, dtype=torch.float32, device=dev), torch.empty(N, dtype=torch.float32, device=dev))
    outs = {j: dict(bits=alice[j], post=None, iters=torch.empty(F, dtype=torch.int32, device=dev),
                    ok=torch.empty(F, dtype=torch.uint8, device=dev)) for j in (2, 3)}
    sched_of = {"auto": api.SCHED_AUTO, "passes": api.SCHED_PASSES, "persistent": api.SCHED_PERSISTENT,
                "group": api.SCHED_GROUP, "layered": api.SCHED_LAYERED}
    cus = torch.cuda.get_device_properties(dev).multi_processor_count

    decs = []
    for key, spec in _decoder_configs(args, api):
        stage_params = {}
        for j in (2, 3):
            algo, store, sched_name, wts = spec[j]
            stage_params[j] = api.Params(algo=algo, max_iter=args.max_iter, math=api.F32, store=store,
                                         alpha=args.alpha, schedule=sched_of[sched_name], wg_threads=args.wg,
                                         min_waves=args.min_waves, lds_cache_kb=args.lds_cache_kb,
                                         group_wgs=args.group_wgs)
            if wts:
                from paper_2108_08418_amd.train import layered_weights, load_weights, weights_meta
                meta = weights_meta(f"{wts}_slice{j}")
                if meta.get("mb") not in (None, mbs[j]):
                    raise SystemExit(f"weights {wts}_slice{j} were trained for mb = {meta['mb']}, "
                                     f"the slice-{j} code has mb = {mbs[j]}")
                w = load_weights(f"{wts}_slice{j}", extend_to=args.max_iter)
                if sched_name == "layered":
                    w = layered_weights(w, args.layered_weight_steps)
                stage_params[j] = replace(stage_params[j], max_iter=int(w.shape[0]),
                                          weights=torch.from_numpy(w).to(dev))
        decs.append(dict(key=key, spec=spec, stage_params=stage_params))
    ws_bytes = max(api.decode_workspace_size(batches[j], d["stage_params"][j]) for d in decs for j in (2, 3))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    torch.cuda.synchronize()
    print(f"# inputs ready in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)

    # Bob's syndromes (HBM-bound) run on a second stream of default priority,
    # beside Alice's fp64-bound LLR pass; the decoders wait for both.
    side = torch.cuda.Stream(device=dev)

    def make_step(stage_params, xs, ys):
        def step():
            main = torch.cuda.current_stream()
            api.slice_quantize(ys, th, M_BITS, out=bob)                                   # Bob: M(.) and slices
            side.wait_stream(main)
            for j in (2, 3):                                                               # Bob: syndromes
                api.syndrome_check(codes[j], bob[j], want_unsat=False, out_syndrome=syn[j], stream=side)
            alice[0:2].copy_(bob[0:2])                                                    # disclosed slices
            # Alice: slice 2, and in the same pass slice 3 for either value of slice 2
            api.slice_llr_next(xs, sig, th, M_BITS, 2, 0b11, alice, out=(llr, *llr3))
            main.wait_stream(side)
            api.ldpc_decode_batch(batches[2], stage_params[2], llr, syn[2], workspace=ws, out=outs[2])
            api.slice_llr_choose(llr3[0], llr3[1], alice[2], out=llr)                     # slice 3 given decoded slice 2
            api.ldpc_decode_batch(batches[3], stage_params[3], llr, syn[3], workspace=ws, out=outs[3])
        return step

    def counts():
        """Failures and bit errors of the last step, per coded slice."""
        for j in (2, 3):
            api.check_abandoned(outs[j])
        r = {}
        for j in (2, 3):
            okj = outs[j]["ok"].cpu().numpy()
            r[j] = dict(iters=outs[j]["iters"].cpu().numpy(), ok=okj,
                        bit_errors=int((alice[j] != bob[j]).sum().item()))
        return r

    results = {}
    for d in decs:
        stage_params = d["stage_params"]
        step = make_step(stage_params, x, y)
        sched = stage_params[2].schedule
        layered = sched == api.SCHED_LAYERED
        persistent = sched == api.SCHED_PERSISTENT or (sched == api.SCHED_AUTO and F >= cus)
        group = sched == api.SCHED_GROUP or (sched == api.SCHED_AUTO and F < cus)
        tuned = None
        if not args.no_tune and ((persistent and args.wg == 0) or (layered and args.wg == 0)
                                 or (group and args.min_waves == 0 and args.group_wgs == 0)):
            # pick the launch shape on this workload's own decode (untimed)
            step()
            from paper_2108_08418_amd import tune
            knobs, cands = ((tune.LAYERED_KNOBS, tune.LAYERED_CANDIDATES) if layered else
                            (tune.KNOBS, tune.CANDIDATES) if persistent else (tune.GROUP_KNOBS, tune.GROUP_CANDIDATES))
            # one shape for both coded slices, picked on slice 2 (so that one
            # kernel instance, and its recorded HBM traffic, covers the step)
            api.slice_llr(x, sig, th, M_BITS, 2, 0b11, alice, out=llr)
            best, tim = tune.tune_decode(batches[2], stage_params[2], llr, syn[2], ws, outs[2],
                                         candidates=cands, knobs=knobs)
            for j in (2, 3):
                for k, v in zip(knobs, best):
                    setattr(stage_params[j], k, v)
            tuned = {"/".join(f"{k}={v}" for k, v in zip(knobs, c)): round(t, 3) for c, t in tim.items()}
            print(f"# {d['key']} tuned: {[tuple(getattr(stage_params[j], k) for k in knobs) for j in (2, 3)]}",
                  file=sys.stderr, flush=True)
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        api.profile_enable(True)
        for k in range(8):
            api.profile_read(k, reset=True)
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for _ in range(args.steps):
            step()
        torch.cuda.synchronize()
        t_total = time.perf_counter() - t_start
        api.profile_enable(False)
        prof = {name: api.profile_read(k, reset=True) for k, name in enumerate(
            ["quantize", "slice_llr", "syndrome", "check", "var", "dec_setup", "decode_persistent", "adjoint"])}
        c = counts()
        # each coded slice's decode alone (untimed step; the same inputs: slice 2
        # from the disclosed slices, slice 3 given the decoded slice 2)
        per_slice = {}
        for j in (2, 3):
            api.slice_llr(x, sig, th, M_BITS, j, (1 << j) - 1, alice, out=llr)
            saved = outs[j]["bits"].clone()
            torch.cuda.synchronize()
            api.profile_enable(True)
            api.profile_read(api.PROF_FRAMES, reset=True)
            api.profile_read(api.PROF_CHECK, reset=True)
            api.profile_read(api.PROF_VAR, reset=True)
            for _ in range(3):
                api.ldpc_decode_batch(batches[j], stage_params[j], llr, syn[j], workspace=ws, out=outs[j])
            torch.cuda.synchronize()
            api.profile_enable(False)
            ms = sum(api.profile_read(k, reset=True)[0] for k in (api.PROF_FRAMES, api.PROF_CHECK, api.PROF_VAR))
            per_slice[str(j)] = ms / 3
            outs[j]["bits"].copy_(saved)
        res = summarize(args, d, stage_params, qcs, codes, n, F, N, t_total, prof, c, persistent, group, layered)
        res["decode_ms_per_slice"] = per_slice
        res["autotune_ms_per_decode"] = tuned
        results[d["key"]] = res
        print(f"# {d['key']}: {res['ms_per_step']:.2f} ms/step, {res['value']:.3e} bits/s", file=sys.stderr, flush=True)

    # ---- frame-error rates over more seeds (untimed) ----
    fer = {d["key"]: {j: [0, 0] for j in (2, 3)} for d in decs}
    for d in decs:
        for j in (2, 3):
            okj = results[d["key"]]["_counts"][j]["ok"]
            fer[d["key"]][j] = [int((okj == 0).sum()), int(okj.size)]
    for s in range(1, args.fer_seeds):
        xs_np, ys_np = inputs.gaussian_pairs(N, SNR, seed=args.seed + 7919 * s)
        xs = torch.from_numpy(xs_np).to(dev)
        ys = torch.from_numpy(ys_np).to(dev)
        del xs_np, ys_np
        for d in decs:
            make_step(d["stage_params"], xs, ys)()
            torch.cuda.synchronize()
            c = counts()
            for j in (2, 3):
                fer[d["key"]][j][0] += int((c[j]["ok"] == 0).sum())
                fer[d["key"]][j][1] += int(c[j]["ok"].size)
        del xs, ys
        print(f"# FER seed {s}: {fer}", file=sys.stderr, flush=True)
    for d in decs:
        r = results[d["key"]]
        r.pop("_counts")
        r["fer_frames"] = {str(j): {"failures": fer[d["key"]][j][0], "frames": fer[d["key"]][j][1],
                                    "fer": fer[d["key"]][j][0] / fer[d["key"]][j][1],
                                    "wilson95": wilson95(*fer[d["key"]][j])} for j in (2, 3)}

    head = results[decs[0]["key"]]
    result = dict(head)
    result["config"]["rate_selection"] = (
        {str(j): {"capacity": round(rate_sel[j]["capacity"], 4), "test_sub_blocks": args.rate_frames,
                  "trail": [{k: c[k] for k in ("rate", "mb", "failures", "mean_iters")} for c in rate_sel[j]["trail"]]}
         for j in (2, 3)} if rate_sel else "fixed table (inputs.SLICE_MB)")
    if len(decs) > 1:
        base = results["sp"]
        comp = {}
        for d in decs:
            r = results[d["key"]]
            same = {}
            for j in (2, 3):
                lo, hi = base["fer_frames"][str(j)]["wilson95"]
                same[str(j)] = bool(lo <= r["fer_frames"][str(j)]["fer"] <= hi)
            comp[d["key"]] = {
                **{k: r[k] for k in ("value", "ms_per_step", "dtype", "roofline", "decode_iteration",
                                     "decode_ms_per_slice", "kernel_ms_per_step", "mean_iters", "fer_frames",
                                     "bit_errors_vs_bob", "autotune_ms_per_decode")},
                "config": {k: r["config"][k] for k in ("decoder", "max_iter", "schedule", "launch_shape")},
                "bits_per_s_vs_flooding_sp": r["value"] / base["value"],
                "decoder_speedup_vs_flooding_sp_per_slice": {
                    str(j): base["decode_ms_per_slice"][str(j)] / r["decode_ms_per_slice"][str(j)] for j in (2, 3)},
                "same_fer_as_flooding_sp": same,
            }
        result["decoders"] = comp
        result["decoders_rule"] = (
            "sp_layered: sum-product, layered schedule (the value above); sp: sum-product, flooding schedule "
            "(the baseline); nms: learned normalized min-sum, flooding, binary16 messages; nms_layered: the same "
            f"learned min-sum on the layered schedule, iteration t with the weights of flooding iteration "
            f"{args.layered_weight_steps:g} t; mixed_layered: learned min-sum (binary16, layered) on slice 2, "
            "sum-product (fp32, layered) on slice 3.  same_fer_as_flooding_sp: the FER over fer_frames lies inside "
            "flooding sum-product's 95 % Wilson interval")
    # the Gaussian-approximation iteration count (host model) beside the measured
    # mean: a binary-input AWGN channel carrying the capacity that Alice's LLRs
    # (given Bob's true lower slices) carry about Bob's bits, the code's own
    # degree distributions, target bit error ratio 1/n
    from paper_2108_08418_amd import ga
    ga_pred = {}
    api.slice_quantize(y, th, M_BITS, out=bob)
    for j in (2, 3):
        api.slice_llr(x, sig, th, M_BITS, j, (1 << j) - 1, bob, out=llr)
        sgn = 1.0 - 2.0 * bob[j].to(torch.float64)
        cap = 1.0 - float(torch.nn.functional.softplus(-sgn * llr.to(torch.float64)).mean()) / math.log(2.0)
        csr_j = qcs[j].to_csr()
        lam, rho = ga.degree_distributions(csr_j.row_ptr, csr_j.col_idx, n)
        m0 = ga.biawgn_mean_for_capacity(cap)
        ga_pred[str(j)] = {"capacity": round(cap, 4), "m0": round(m0, 4),
                           "iters_to_ber_1_over_n": ga.iterations_to(1.0 / n, m0, lam, rho)}
    result["ga_iterations"] = ga_pred
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(args, x_np, y_np, qcs, th, sig, n, decs[0])
    return result


def summarize(args, d, stage_params, qcs, codes, n, F, N, t_total, prof, c, persistent, group, layered):
    """Result dict of one decoder's timed steps."""
    from paper_2108_08418_amd import api
    spec = d["spec"]
    algo, store, _, wts = spec[2]
    uniform = spec[2] == spec[3]
    ms_step = 1e3 * t_total / args.steps
    value = 2 * N / (t_total / args.steps)
    iters = {j: c[j]["iters"] for j in (2, 3)}
    ok = {j: c[j]["ok"] for j in (2, 3)}
    chk_bytes = iter_bytes = dec_bytes = 0.0
    edge_updates = 0
    for j in (2, 3):
        s_msg = 4 if spec[j][1] == api.F32 else 2
        cb, ib = stage_bytes(iters[j], stage_params[j].max_iter, n, codes[j].m, codes[j].n_edges, s_msg)
        chk_bytes += cb
        iter_bytes += ib
        dec_bytes += (layered_decode_bytes if layered else frame_decode_bytes)(
            iters[j], n, codes[j].m, codes[j].n_edges, s_msg)
        edge_updates += int(iters[j].astype(np.int64).sum()) * codes[j].n_edges
    chk_ms, chk_n = prof["check"]
    var_ms, var_n = prof["var"]
    per_ms, per_n = prof["decode_persistent"]
    dom = max(("check", "var", "slice_llr", "decode_persistent"), key=lambda k: prof[k][0])
    traffic = traffic_src = valu = None
    shape = {j: (stage_params[j].wg_threads, stage_params[j].min_waves, stage_params[j].lds_cache_kb,
                 stage_params[j].group_wgs) for j in (2, 3)}
    if per_ms > 0 and not uniform:
        roof_kernel = "per coded slice: " + ", ".join(
            f"slice {j} {'sum-product' if spec[j][0] == api.SP else 'min-sum'}" for j in (2, 3))
        achieved = (args.steps * dec_bytes) / (per_ms * 1e-3) / 1e9
        launches, launch_ms, launch_bytes = per_n, per_ms, args.steps * dec_bytes
        iter_gbs = achieved
    elif per_ms > 0:
        wg, mw, lk, _ = shape[2]
        wg = wg or 512
        mt = "float, float" if store == api.F32 else "float, __half"
        a = 0 if algo == api.SP else 1
        if layered:
            inst = f"void cvr::k_layered_qc<{mt}, {a}, 8, {wg}, true>"
        elif persistent:
            inst = (f"void cvr::k_frames_qc<{mt}, {a}, 8, {wg}, true, {8 if mw == 8 else 1}, "
                    f"{'false' if lk < 0 else 'true'}>")
        else:                                   # group schedule (workgroups per frame on one XCD)
            inst = f"void cvr::k_group_qc<{mt}, {a}, 8, 1024, true, {8 if mw == 8 else 1}>"
        roof_kernel = inst
        achieved = (args.steps * dec_bytes) / (per_ms * 1e-3) / 1e9
        launches, launch_ms, launch_bytes = per_n, per_ms, args.steps * dec_bytes
        iter_gbs = achieved
        if shape[2] == shape[3]:
            traffic, traffic_src = recorded_traffic(inst, args.workload, "sp" if algo == api.SP else "nms", wts)
            valu = recorded_valu(inst, args.workload, "sp" if algo == api.SP else "nms", wts)
    else:
        roof_kernel = "decoder check-node pass (k_check_qc)"
        achieved = (args.steps * chk_bytes) / (chk_ms * 1e-3) / 1e9 if chk_ms > 0 else None
        launches, launch_ms, launch_bytes = chk_n, chk_ms, args.steps * chk_bytes
        iter_gbs = (args.steps * iter_bytes) / ((chk_ms + var_ms) * 1e-3) / 1e9 if chk_ms + var_ms > 0 else None
    sched_name = {api.SCHED_AUTO: "auto", api.SCHED_PASSES: "passes", api.SCHED_PERSISTENT: "persistent",
                  api.SCHED_GROUP: "group", api.SCHED_LAYERED: "layered"}[stage_params[2].schedule]
    return {
        "metric": "decoded bits/s (slice reconciliation, coded slices) and HBM GB/s of the decoder at fixed FER; "
                  "learned min-sum vs plain sum-product",
        "value": value,
        "unit": "bits/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("f32" if algo == api.SP else "f32 math / f16 messages") if uniform else
                 "f32 (slice 3) and f32 math / f16 messages (slice 2)",
        "data": "synthetic: seeded Gaussian pairs, SNR 3, seeded QC-LDPC slice codes",
        "config": {
            "workload": args.workload, "pairs": N, "sub_block": n, "sub_blocks_per_slice": F,
            "slices": ("16 equiprobable Gray intervals; slices 0-1 disclosed, "
                       f"2 (R={1 - qcs[2].m / n:.4f}) and 3 (R={1 - qcs[3].m / n:.4f}) decoded"),
            "code_rates": {str(j): 1 - qcs[j].m / n for j in (2, 3)},
            "decoder": {str(j): ("sum-product" if spec[j][0] == api.SP else
                                 (f"learned normalized min-sum ({spec[j][3]}_slice{j})" if spec[j][3] else
                                  f"normalized min-sum alpha={args.alpha}")) for j in (2, 3)},
            "max_iter": {str(j): stage_params[j].max_iter for j in (2, 3)}, "schedule": sched_name,
            "launch_shape": {str(j): dict(zip(("wg_threads", "min_waves", "lds_cache_kb", "group_wgs"), shape[j]))
                             for j in (2, 3)},
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": roof_kernel,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": (achieved / HBM_PEAK_GBS) if achieved else None,
            "traffic": traffic,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "traffic_source": traffic_src,
            "traffic_over_algorithmic": (traffic / (launch_bytes / launches)) if (traffic and launches) else None,
            "avg_launch_us": 1e3 * launch_ms / launches if launches else None,
            "algorithmic_bytes_per_launch": launch_bytes / launches if launches else None,
            "valu_issue_frac": valu["issue"] if valu else None,
            "valu_issue_frac_with_transcendentals": valu["issue_with_transcendentals"] if valu else None,
            "valu_source": valu["source"] if valu else None,
            "note": ("group schedule: the decoder state stays in the L2 / Infinity Cache (HBM traffic far "
                     "below the algorithmic bytes), so an iteration is bound by barrier and pass latency, "
                     "not HBM" if (per_ms > 0 and group and not layered) else
                     "layered schedule: the LDS posterior cache keeps HBM traffic below the algorithmic bytes; "
                     "rocprofv3 instruction counters put the kernel near its VALU issue limit "
                     "(valu_issue_frac), which bounds it before HBM does" if (layered and valu) else None),
        },
        "paper_context": PAPER_CONTEXT,
        "decode_iteration": {
            "algorithmic_GBs": iter_gbs,
            "frac_of_hbm_peak": (iter_gbs / HBM_PEAK_GBS) if iter_gbs else None,
            "edge_updates_per_s": edge_updates / (t_total / args.steps),
            # the paper's figure of merit: seconds per arithmetic operation at 7
            # operations per edge and iteration (Sec. III-C), whole step
            "c_h_equivalent_s": (t_total / args.steps) / (7.0 * edge_updates) if edge_updates else None,
            "decode_ms_per_step": (per_ms + chk_ms + var_ms) / args.steps,
        },
        "kernel_ms_per_step": {k: v[0] / args.steps for k, v in prof.items()},
        "dominant_kernel": dom,
        "mean_iters": {str(j): float(iters[j].mean()) for j in (2, 3)},
        "bit_errors_vs_bob": {str(j): c[j]["bit_errors"] for j in (2, 3)},
        "reconciled_pairs_per_s": N / (t_total / args.steps),
        "key_rate_exp": key_rate_exp(args, N, sum(1 - qcs[j].m / n for j in (2, 3)), t_total / args.steps),
        "reconciliation_efficiency": efficiency([0.0, 0.0] + [1 - qcs[j].m / n for j in (2, 3)]),
        "_counts": c,
    }


def efficiency(rates):
    """beta of Sec. III-B for this setup: Bob's label entropy, the slices'
    rates (disclosed slices 0), I_AB = log2(1 + SNR) / 2; beside it the bound
    the quantiser sets, I(M(Y); X) / I_AB (beta with capacity-achieving codes)."""
    from paper_2108_08418_amd import inputs, keyrate
    th = inputs.equiprobable_thresholds(M_BITS, 1.0 + 1.0 / SNR)
    H, I = keyrate.quantiser_information(th, SNR)
    I_AB = keyrate.capacity(SNR)
    return {"beta": keyrate.efficiency(H, M_BITS, rates, I_AB), "quantiser_bound": I / I_AB,
            "label_entropy_bits": H, "I_AB_bits": I_AB, "rates": rates}


def key_rate_exp(args, N, rate_sum, dt):
    """The experimental key rate of Sec. V for this step (None without --s-be):
    the N pairs reconciled by the coded slices' codes (disclosed slices carry
    rate 0) in the step's time, with the paper's standard failure
    probabilities (eps_EC = eps_PA = eps_PE = 2 eps_s = 2.5e-10) and
    m = 4 slices in Delta_AEP.  S_BE, the Holevo bound, is an input."""
    if args.s_be is None:
        return None
    from paper_2108_08418_amd import keyrate
    eps_s, eps_x = 1.25e-10, 2.5e-10
    d_aep = keyrate.delta_aep(M_BITS, N, eps_s, 3 * eps_x + 2 * eps_s)
    return {"bits_per_s": keyrate.k_exp(N, rate_sum, args.s_be, d_aep, eps_x, dt), "S_BE": args.s_be,
            "code_rate_sum": rate_sum, "pairs": N, "dt_s": dt,
            "note": "Sec. V K'_exp with this step as the measured reconciliation time; the paper's codes meet "
                    "eps_EC, here see fer_frames"}


def ragged(args, wl, dev):
    """Uneven batch: every sub-block of the batch in one decode call."""
    import torch

    from paper_2108_08418_amd import api, inputs

    sizes, counts = wl["sizes"], wl["counts"]
    rng = np.random.default_rng(args.seed)
    order = rng.permutation(np.repeat(np.arange(len(sizes)), counts))
    qcs = [inputs.met_low_rate_spec(n) for n in sizes]
    codes = [api.Code.from_qc(q) for q in qcs]
    frames, vo, co = [], 0, 0
    for c in order:
        frames.append((int(c), vo, co))
        vo += sizes[c]
        co += qcs[c].m
    batch = api.Batch(codes, frames)
    total_n, total_m, F = batch.total_n, batch.total_m, batch.F
    print(f"# workload {args.workload}: F={F} total_n={total_n}", file=sys.stderr, flush=True)
    t0 = time.time()
    bits = inputs.random_bits(total_n, seed=args.seed + 1)
    sigma2 = 1.0 / wl["snr"]
    llr_np = inputs.bpsk_llr(bits, sigma2, seed=args.seed + 2).astype(np.float32)
    bits_g = torch.from_numpy(bits).to(dev)
    llr = torch.from_numpy(llr_np).to(dev)
    syn = torch.empty(total_m, dtype=torch.uint8, device=dev)
    # Bob's syndromes, one syndrome_check per code over that code's frames (input synthesis)
    for c, q in enumerate(qcs):
        idx = [i for i, f in enumerate(frames) if f[0] == c]
        vidx = torch.cat([torch.arange(frames[i][1], frames[i][1] + q.n, device=dev) for i in idx])
        cidx = torch.cat([torch.arange(frames[i][2], frames[i][2] + q.m, device=dev) for i in idx])
        s_c, _ = api.syndrome_check(codes[c], bits_g[vidx].contiguous(), want_unsat=False)
        syn[cidx] = s_c.view(-1)
    algo = api.SP if args.decoder == "sp" else api.NMS
    store = api.F32 if args.decoder == "sp" else api.F16
    layered = args.schedule == "layered"
    params = api.Params(algo=algo, max_iter=args.max_iter, math=api.F32, store=store, alpha=args.alpha,
                        wg_threads=args.wg, min_waves=args.min_waves, lds_cache_kb=args.lds_cache_kb,
                        schedule=api.SCHED_LAYERED if layered else api.SCHED_AUTO)
    ws = api.alloc_workspace(batch, params, dev)
    out = dict(bits=torch.empty(total_n, dtype=torch.uint8, device=dev), post=None,
               iters=torch.empty(F, dtype=torch.int32, device=dev), ok=torch.empty(F, dtype=torch.uint8, device=dev))
    torch.cuda.synchronize()
    print(f"# inputs ready in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)

    def step():
        api.ldpc_decode_batch(batch, params, llr, syn, workspace=ws, out=out)

    tuned = None
    if not args.no_tune and args.wg == 0:
        from paper_2108_08418_amd import tune
        knobs, cands = ((tune.LAYERED_KNOBS, tune.LAYERED_CANDIDATES) if layered else (tune.KNOBS, tune.CANDIDATES))
        best, tim = tune.tune_decode(batch, params, llr, syn, ws, out, candidates=cands, knobs=knobs)
        for k, v in zip(knobs, best):
            setattr(params, k, v)
            setattr(args, {"wg_threads": "wg", "min_waves": "min_waves", "lds_cache_kb": "lds_cache_kb"}[k], v)
        tuned = {"/".join(f"{k}={v}" for k, v in zip(knobs, c)): round(t, 3) for c, t in tim.items()}
        print(f"# tuned: {best} {tuned}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    graph = None
    if args.graph:
        graph = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            step()
        torch.cuda.current_stream().wait_stream(s)
        with torch.cuda.graph(graph):
            step()
    torch.cuda.synchronize()
    api.profile_enable(not args.graph)
    for k in range(8):
        api.profile_read(k, reset=True)
    t_start = time.perf_counter()
    for _ in range(args.steps):
        graph.replay() if graph is not None else step()
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    api.profile_enable(False)
    per_ms, per_n = api.profile_read(6, reset=True)
    api.check_abandoned(out)
    iters = out["iters"].cpu().numpy()
    ok = out["ok"].cpu().numpy()
    err = (out["bits"] != bits_g).cpu().numpy()
    s_msg = 4 if store == api.F32 else 2
    dec_bytes = 0.0
    fer = {}
    for c, q in enumerate(qcs):
        sel = order == c
        dec_bytes += (layered_decode_bytes if layered else frame_decode_bytes)(iters[sel], q.n, q.m, q.n_edges, s_msg)
        fer[str(sizes[c])] = float(1.0 - ok[sel].mean())
    achieved = (args.steps * dec_bytes) / (per_ms * 1e-3) / 1e9 if per_ms > 0 else None
    if achieved is None:                  # graph replay: whole step timed by the host clock
        achieved = (args.steps * dec_bytes) / t_total / 1e9
    wg = args.wg or 512
    mt = "float, float" if store == api.F32 else "float, __half"
    if layered:
        inst = f"void cvr::k_layered_qc<{mt}, {0 if algo == api.SP else 1}, 8, {wg}, true>"
    else:
        inst = (f"void cvr::k_frames_qc<{mt}, {0 if algo == api.SP else 1}, 8, {wg}, true, "
                f"{8 if args.min_waves == 8 else 1}, {'false' if args.lds_cache_kb < 0 else 'true'}>")
    traffic, traffic_src = recorded_traffic(inst, args.workload, args.decoder, args.weights)
    value = total_n / (t_total / args.steps)
    result = {
        "metric": "decoded bits/s of a batch of uneven sub-blocks (one launch)",
        "value": value, "unit": "bits/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * t_total / args.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32" if store == api.F32 else "f32 math / f16 messages",
        "data": "synthetic: seeded random words and BPSK/AWGN at SNR 0.16, seeded MET QC codes",
        "config": {"workload": args.workload, "frames": F, "total_bits": total_n,
                   "sizes": list(sizes), "counts": list(counts), "code_rate": 0.0625,
                   "decoder": ("sum-product" if algo == api.SP else f"normalized min-sum alpha={args.alpha}"),
                   "max_iter": args.max_iter, "graph": bool(args.graph), "schedule": "layered" if layered else "auto",
                   "wg_threads": wg, "lds_cache_kb": args.lds_cache_kb,
                   "min_waves": args.min_waves,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": inst, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS if achieved else None, "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "traffic_source": traffic_src,
                     "traffic_over_algorithmic": traffic / dec_bytes if (traffic and dec_bytes) else None,
                     "avg_launch_us": 1e3 * per_ms / per_n if per_n else None,
                     "algorithmic_bytes_per_launch": dec_bytes},
        "fer": fer,
        "mean_iters": float(iters.mean()),
        "bit_errors": int(err.sum()),
        "autotune_ms_per_decode": tuned,
    }
    return result


def adjoint_bytes(F, E, n, T, K):
    """Algorithmic bytes of the adjoint launch: for each frame, the forward
    iterations recomputed from the checkpoints (T - ceil(T / K); each reads and
    writes every fp32 message once and moves 12 bytes per variable), and T
    reverse iterations, each reading the messages of iteration t and the
    adjoint of the messages and writing the new adjoint (12 bytes per edge)
    plus 12 bytes per variable (channel LLR, posterior)."""
    nseg = -(-T // K)
    return float(F) * ((T - nseg) * (8 * E + 12 * n) + T * (12 * E + 12 * n))


def train_step(args, wl, dev):
    """One training step of the unrolled min-sum: forward with checkpoints,
    loss, adjoint, optimiser update, on inputs already resident in HBM."""
    import torch

    from paper_2108_08418_amd import api, inputs
    from paper_2108_08418_amd.train import BpskFrames

    n, F, T, K = wl["n"], wl["F"], wl["T"], wl["K"]
    qc = inputs.lambda_half_rate_spec(n)
    frames = BpskFrames(qc, F, (1.5, 3.0), 0.5, dev)
    llr, syn, bits = frames.batch(0)
    batch = api.Batch.uniform(frames.code, F)
    sign = 1.0 - 2.0 * bits.to(torch.float32)
    w = torch.full((T, qc.n_types), 0.75, dtype=torch.float32, device=dev, requires_grad=True)
    opt = torch.optim.Adam([w], lr=0.02)
    torch.cuda.synchronize()

    def step():
        post = api.NMSUnrolled.apply(w, llr, syn, batch, T, K)
        loss = torch.nn.functional.softplus(-sign * post).mean()
        opt.zero_grad(set_to_none=False)
        loss.backward()
        opt.step()
        with torch.no_grad():
            w.clamp_(0.05, 1.5)
        return loss

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    api.profile_enable(True)
    for k in range(8):
        api.profile_read(k, reset=True)
    t_start = time.perf_counter()
    for _ in range(args.steps):
        loss = step()
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    api.profile_enable(False)
    fwd_ms, fwd_n = api.profile_read(api.PROF_FRAMES, reset=True)
    adj_ms, adj_n = api.profile_read(api.PROF_ADJOINT, reset=True)
    E = qc.n_edges
    adj_bytes = adjoint_bytes(F, E, n, T, K)
    achieved = adj_bytes * adj_n / (adj_ms * 1e-3) / 1e9 if adj_ms > 0 else None
    adj_kernel = "void cvr::k_nms_bwd_qc<8, true, 1024, true>"   # column sums in LDS at n = 16384
    traffic, traffic_src = recorded_traffic(adj_kernel, args.workload, "adjoint", "")
    step_s = t_total / args.steps
    result = {
        "metric": "unrolled min-sum training: bits/s through forward + adjoint",
        "value": F * n / step_s, "unit": "bits/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * step_s, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic: seeded random words and BPSK/AWGN, Eb/N0 uniform in [1.5, 3] dB",
        "config": {"workload": args.workload, "frames": F, "n": n, "T": T, "ckpt_every": K,
                   "code": qc.name, "n_types": qc.n_types, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": adj_kernel, "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS if achieved else None,
                     "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "traffic_source": traffic_src,
                     "traffic_over_algorithmic": traffic / adj_bytes if traffic else None,
                     "avg_launch_us": 1e3 * adj_ms / adj_n if adj_n else None,
                     "algorithmic_bytes_per_launch": adj_bytes},
        "forward_ms": fwd_ms / max(fwd_n, 1), "adjoint_ms": adj_ms / max(adj_n, 1),
        "edge_iterations_per_s": 2.0 * F * E * T / step_s,
        "loss": float(loss),
    }
    return result


def cpu_baseline(args, x_np, y_np, qcs, th, sig, n, dec):
    """The fp64 oracle on a bounded sample of the same workload (the first
    ``cpu_frames`` sub-blocks of both coded slices) with the headline
    decoder's rule and weights, all host threads."""
    import oracle
    Fs = min(args.cpu_frames, len(x_np) // n)
    Ns = Fs * n
    xs, ys = x_np[:Ns], y_np[:Ns]
    csr = {j: qcs[j].to_csr() for j in (2, 3)}
    from paper_2108_08418_amd import api
    t0 = time.perf_counter()
    edge_updates = 0
    S = oracle.quantize(ys, th, M_BITS)
    syn = {j: oracle.syndrome(csr[j], S[j].reshape(Fs, n))[0] for j in (2, 3)}
    A = np.zeros_like(S)
    A[0:2] = S[0:2]
    for j in (2, 3):
        L = oracle.slice_llr(xs, sig, th, M_BITS, oracle.GRAY, j, (1 << j) - 1, A)
        sp = dec["stage_params"][j]
        algo = oracle.SP if sp.algo == api.SP else oracle.NMS
        w = None if sp.weights is None else sp.weights.cpu().numpy().astype(np.float64)
        kw = dict(algo=algo, max_iter=sp.max_iter, alpha=args.alpha, weights=w, store_half=(algo == oracle.NMS))
        if sp.schedule == api.SCHED_LAYERED:
            r = oracle.decode_layered(csr[j], L.reshape(Fs, n), syn[j], layers=oracle.qc_layers(qcs[j].mb, qcs[j].Z),
                                      **kw)
        else:
            r = oracle.decode(csr[j], L.reshape(Fs, n), syn[j], **kw)
        A[j] = r["bits"].reshape(-1)
        edge_updates += int(np.asarray(r["iters"]).astype(np.int64).sum()) * csr[j].n_edges
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    sched = "layered" if dec["stage_params"][2].schedule == api.SCHED_LAYERED else "flooding"
    rule = sched + " " + " / ".join("sum-product" if dec["stage_params"][j].algo == api.SP else
                                    "min-sum with the same weights and binary16 messages" for j in (2, 3))
    return {"value": 2 * Ns / dt, "unit": "bits/s", "cores": min(cores, os.cpu_count() or cores),
            "kind": "oracle", "seconds": dt, "edge_updates_per_s": edge_updates / dt,
            "sample": f"first {Fs} of the {len(x_np) // n} sub-blocks of {n} bits of both coded slices: fp64 "
                      f"quantiser, syndromes, slice LLRs and {rule} (slice 2 / slice 3); decode threads across sub-blocks"}


if __name__ == "__main__":
    main()
