"""Autotuner of the decoder's launch shape.

Times ``ldpc_decode_batch`` for every candidate on the caller's own batch and
inputs with HIP events on the launch stream (the library's launch timing) and
returns the fastest.  Persistent schedule: (workgroup size, minimum waves per
SIMD, LDS posterior cache); group schedule: (minimum waves per SIMD, which
sets the workgroups per CU, and workgroups per frame); layered schedule
(workgroup size, LDS posterior cache).  The knobs change the
launch configuration only, never the results.
"""
from __future__ import annotations

from . import api

# lds_cache_kb: 0 = as much as keeps the register-limited occupancy, -1 = none,
# 150 = nearly all of a CU's LDS (one workgroup per CU)
CANDIDATES = [(512, 0, 0), (1024, 0, 0), (512, 8, 0), (1024, 8, 0), (1024, 8, -1), (1024, 0, 150)]
KNOBS = ("wg_threads", "min_waves", "lds_cache_kb")
# group_wgs: 0 = the workgroups an XCD holds divided by its frames
GROUP_CANDIDATES = [(0, 0), (8, 0), (0, 8)]
GROUP_KNOBS = ("min_waves", "group_wgs")
# layered schedule: workgroup size (rows of a block row per thread) and LDS cache
LAYERED_CANDIDATES = [(256, 0), (512, 0), (1024, 0), (512, 150), (256, -1)]
LAYERED_KNOBS = ("wg_threads", "lds_cache_kb")


def tune_decode(batch, params, llr, syndrome, workspace, out, repeats: int = 2, candidates=CANDIDATES,
                knobs=KNOBS):
    """Returns (best candidate as a tuple in ``knobs`` order, {candidate: ms per decode})."""
    import torch
    timings = {}
    saved = tuple(getattr(params, k) for k in knobs)
    try:
        for cand in candidates:
            for k, v in zip(knobs, cand):
                setattr(params, k, v)
            api.ldpc_decode_batch(batch, params, llr, syndrome, workspace=workspace, out=out)   # warm
            torch.cuda.synchronize()
            api.profile_enable(True)
            api.profile_read(api.PROF_FRAMES, reset=True)
            for _ in range(repeats):
                api.ldpc_decode_batch(batch, params, llr, syndrome, workspace=workspace, out=out)
            torch.cuda.synchronize()
            api.profile_enable(False)
            ms, cnt = api.profile_read(api.PROF_FRAMES, reset=True)
            timings[tuple(cand)] = ms / max(cnt, 1)
    finally:
        for k, v in zip(knobs, saved):
            setattr(params, k, v)
        api.profile_enable(False)
    best = min(timings, key=timings.get)
    return best, timings
