"""Autotuner of the persistent decoder's launch shape.

Times ``ldpc_decode_batch`` for every (workgroup size, check rows per step)
candidate on the caller's own batch and inputs with HIP events on the launch
stream (the library's launch timing) and returns the fastest.  The knobs
change the launch configuration only, never the results.
"""
from __future__ import annotations

from . import api

CANDIDATES = [(512, 1, 0), (1024, 1, 0), (256, 1, 0), (512, 2, 0), (1024, 2, 0), (512, 1, 8), (1024, 1, 8)]


def tune_decode(batch, params, llr, syndrome, workspace, out, repeats: int = 2, candidates=CANDIDATES):
    """Returns ((wg_threads, rows_per_step, min_waves), {candidate: ms per decode})."""
    import torch
    timings = {}
    saved = (params.wg_threads, params.rows_per_step, params.min_waves)
    try:
        for wg, rows, mw in candidates:
            params.wg_threads, params.rows_per_step, params.min_waves = wg, rows, mw
            api.ldpc_decode_batch(batch, params, llr, syndrome, workspace=workspace, out=out)   # warm
            torch.cuda.synchronize()
            api.profile_enable(True)
            api.profile_read(api.PROF_FRAMES, reset=True)
            for _ in range(repeats):
                api.ldpc_decode_batch(batch, params, llr, syndrome, workspace=workspace, out=out)
            torch.cuda.synchronize()
            api.profile_enable(False)
            ms, cnt = api.profile_read(api.PROF_FRAMES, reset=True)
            timings[(wg, rows, mw)] = ms / max(cnt, 1)
    finally:
        params.wg_threads, params.rows_per_step, params.min_waves = saved
        api.profile_enable(False)
    best = min(timings, key=timings.get)
    return best, timings
