"""MI355X-native slice-reconciliation hot path (arXiv 2108.08418).

The compute path lives in ``libcvqkd_recon.so`` (hand-written HIP for gfx950,
C ABI in ``include/cvqkd_recon.h``); :mod:`paper_2108_08418_amd.api` is the
thin binding with the same entry-point names and
:mod:`paper_2108_08418_amd.inputs` the seeded synthetic inputs.

Importing this package does not load the library; the first call does, and
raises if it has not been built.
"""
__all__ = ["api", "inputs"]
