"""TEST INFRASTRUCTURE -- the fp64 CPU oracle of the slice-reconciliation hot path.

Plain, slow, obviously-correct reference used only by ``tests/``, the smoke
check and the benchmark's CPU-baseline leg.  It shares no code with the HIP
library and never imports it.

* :mod:`oracle.slicing` -- quantiser/slicer and slice LLRs (NumPy/SciPy, fp64);
* :mod:`oracle.bp`      -- syndrome, flooding and layered sum-product /
  normalized min-sum (whole decodes and single iterations from a given state),
  unrolled min-sum with its reverse-mode derivative (plain C, fp64, via ctypes).
"""
from .slicing import GRAY, BINARY, quantize, slice_llr, slice_llr_prior, slice_llr_bsc, log_interval_probs  # noqa: F401
from .bp import (syndrome, decode, nms_unrolled, round_half, build, SP, NMS,  # noqa: F401
                 flood_step, decode_layered, layered_step, qc_layers)
