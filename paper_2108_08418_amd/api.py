"""Thin Python binding of the C ABI (same names as the C entry points).

Only argument marshalling happens here: every step of the path runs in the
HIP kernels of libcvqkd_recon.so.  Tensors must live on the current HIP
device; PyTorch supplies the device memory and the stream.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass
from typing import Sequence

import numpy as np
import torch

from . import _lib
from ._lib import DecodeParams, Frame, check, load

GRAY, BINARY = 0, 1
SP, NMS = 0, 1
F64, F32, F16 = 0, 1, 2
SCHED_AUTO, SCHED_PASSES, SCHED_PERSISTENT, SCHED_GROUP, SCHED_LAYERED = 0, 1, 2, 3, 4

_TORCH_OF = {F64: torch.float64, F32: torch.float32}


def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


def _ptr(t) -> int | None:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _host(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# ---------------------------------------------------------------------------
# codes and batches
# ---------------------------------------------------------------------------
class Code:
    """Owner of a cvr_code_t (device copy of a parity-check matrix)."""

    def __init__(self, handle: int):
        self._h = C.c_void_p(handle)
        n, m, nt, qc = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        E = C.c_int64()
        check(load().cvr_code_info(self._h, C.byref(n), C.byref(m), C.byref(E), C.byref(nt), C.byref(qc)),
              "cvr_code_info")
        self.n, self.m, self.n_edges, self.n_types, self.is_qc = n.value, m.value, E.value, nt.value, bool(qc.value)

    @classmethod
    def from_csr(cls, code) -> "Code":
        rp = _host(code.row_ptr, np.int32)
        ci = _host(code.col_idx, np.int32)
        et = _host(code.edge_type, np.uint8)
        h = C.c_void_p()
        check(load().cvr_code_create_csr(int(code.n), int(code.m), rp.ctypes.data, ci.ctypes.data,
                                         et.ctypes.data, int(code.n_types), C.byref(h)), "cvr_code_create_csr")
        return cls(h.value)

    @classmethod
    def from_qc(cls, code) -> "Code":
        sh = _host(code.shift, np.int32)
        bt = _host(code.block_type, np.uint8)
        h = C.c_void_p()
        check(load().cvr_code_create_qc(int(code.nb), int(code.mb), int(code.Z), sh.ctypes.data, bt.ctypes.data,
                                        int(code.n_types), C.byref(h)), "cvr_code_create_qc")
        return cls(h.value)

    @classmethod
    def create(cls, code) -> "Code":
        return cls.from_qc(code) if hasattr(code, "shift") else cls.from_csr(code)

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h is not None and self._h.value:
            load().cvr_code_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Owner of a cvr_batch_t: a ragged set of frames over one or more codes."""

    def __init__(self, codes: Sequence[Code], frames: Sequence[tuple[int, int, int]]):
        self.codes = list(codes)
        arr = (C.c_void_p * len(self.codes))(*[c.handle.value for c in self.codes])
        fr = (Frame * max(1, len(frames)))()
        for i, (ci, vo, co) in enumerate(frames):
            fr[i].code_idx, fr[i].vn_offset, fr[i].chk_offset = int(ci), int(vo), int(co)
        h = C.c_void_p()
        check(load().cvr_batch_create(arr, len(self.codes), fr, len(frames), C.byref(h)), "cvr_batch_create")
        self._h = h
        F, tn, tm, te = C.c_int32(), C.c_int64(), C.c_int64(), C.c_int64()
        check(load().cvr_batch_info(h, C.byref(F), C.byref(tn), C.byref(tm), C.byref(te)), "cvr_batch_info")
        self.F, self.total_n, self.total_m, self.total_edges = F.value, tn.value, tm.value, te.value
        self.frames = [tuple(int(x) for x in f) for f in frames]
        # per-type weights are indexed [t * n_types + type] with the largest
        # number of edge types among the batch's codes
        self.n_types = max((c.n_types for c in self.codes), default=1)

    @classmethod
    def uniform(cls, code: Code, F: int) -> "Batch":
        """F frames of one code laid out back to back."""
        return cls([code], [(0, f * code.n, f * code.m) for f in range(F)])

    @property
    def handle(self):
        return self._h

    def close(self):
        if self._h is not None and self._h.value:
            load().cvr_batch_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class Params:
    algo: int = SP
    max_iter: int = 50
    early_stop: bool = True
    math: int = F32
    store: int = F32
    alpha: float = 0.75
    msg_clamp: float = 50.0
    weights: torch.Tensor | None = None   # device fp32 [max_iter, n_types]
    schedule: int = SCHED_AUTO
    wg_threads: int = 0
    min_waves: int = 0
    lds_cache_kb: int = 0
    group_wgs: int = 0

    def c_struct(self, trace: torch.Tensor | None = None) -> DecodeParams:
        p = DecodeParams()
        p.algo, p.max_iter, p.early_stop = int(self.algo), int(self.max_iter), int(bool(self.early_stop))
        p.math, p.store, p.alpha, p.msg_clamp = int(self.math), int(self.store), float(self.alpha), float(self.msg_clamp)
        p.schedule = int(self.schedule)
        p.wg_threads = int(self.wg_threads)
        p.min_waves = int(self.min_waves)
        p.lds_cache_kb = int(self.lds_cache_kb)
        p.group_wgs = int(self.group_wgs)
        if self.weights is not None:
            if self.weights.dtype != torch.float32:
                raise ValueError("weights must be float32")
        p.weights = _ptr(self.weights)
        p.trace = _ptr(trace)
        return p


# ---------------------------------------------------------------------------
# entry points
# ---------------------------------------------------------------------------
def slice_quantize(y: torch.Tensor, thresholds, m_bits: int, labelling: int = GRAY,
                   out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Bob's quantiser and slices: uint8 [m_bits, n] (row j = bit j of the label)."""
    if y.dtype != torch.float64:
        raise ValueError("y must be float64")
    n = y.numel()
    if out is None:
        out = torch.empty((m_bits, n), dtype=torch.uint8, device=y.device)
    th = _host(thresholds, np.float64)
    check(load().slice_quantize(_ptr(y), n, th.ctypes.data, int(m_bits), int(labelling), _ptr(out),
                                _stream(stream)), "slice_quantize")
    return out


def slice_llr(x: torch.Tensor, sigma_n: float, thresholds, m_bits: int, j: int, known_mask: int,
              slices: torch.Tensor | None = None, labelling: int = GRAY, out_dtype: int = F32,
              out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Alice's LLRs of Bob's slice j given x and the slices in known_mask."""
    if x.dtype != torch.float64:
        raise ValueError("x must be float64")
    n = x.numel()
    if out is None:
        out = torch.empty(n, dtype=_TORCH_OF[out_dtype], device=x.device)
    th = _host(thresholds, np.float64)
    if slices is not None and slices.dtype != torch.uint8:
        raise ValueError("slices must be uint8")
    check(load().slice_llr(_ptr(x), n, float(sigma_n), th.ctypes.data, int(m_bits), int(labelling), int(j),
                           int(known_mask), _ptr(slices), int(out_dtype), _ptr(out), _stream(stream)), "slice_llr")
    return out


def slice_llr_prior(x: torch.Tensor, sigma_n: float, thresholds, m_bits: int, j: int, known_mask: int,
                    slices: torch.Tensor | None, prior_mask: int, prior_llr: torch.Tensor | None,
                    labelling: int = GRAY, out_dtype: int = F32, out: torch.Tensor | None = None,
                    stream=None) -> torch.Tensor:
    """Alice's LLRs of Bob's slice j given x, the hard slices in known_mask and
    the soft priors (fp32 LLR rows [m_bits, n]) of the slices in prior_mask."""
    if x.dtype != torch.float64:
        raise ValueError("x must be float64")
    n = x.numel()
    if slices is not None and (slices.dtype != torch.uint8 or not slices.is_contiguous()
                               or slices.numel() < m_bits * n):
        raise ValueError("slices must be contiguous uint8 [m_bits, n]")
    if prior_llr is not None and (prior_llr.dtype != torch.float32 or not prior_llr.is_contiguous()
                                  or prior_llr.numel() < m_bits * n):
        raise ValueError("prior_llr must be contiguous float32 [m_bits, n]")
    if out is None:
        out = torch.empty(n, dtype=_TORCH_OF[out_dtype], device=x.device)
    th = _host(thresholds, np.float64)
    check(load().slice_llr_prior(_ptr(x), n, float(sigma_n), th.ctypes.data, int(m_bits), int(labelling), int(j),
                                 int(known_mask), _ptr(slices), int(prior_mask), _ptr(prior_llr), int(out_dtype),
                                 _ptr(out), _stream(stream)), "slice_llr_prior")
    return out


def slice_llr_next(x: torch.Tensor, sigma_n: float, thresholds, m_bits: int, j: int, known_mask: int,
                   slices: torch.Tensor | None = None, labelling: int = GRAY, out_dtype: int = F32,
                   out: tuple | None = None, stream=None):
    """(L_j, L_{j+1} | bit j = 0, L_{j+1} | bit j = 1) in one pass; each equal to
    slice_llr's value with the corresponding bits known."""
    if x.dtype != torch.float64:
        raise ValueError("x must be float64")
    n = x.numel()
    if slices is not None and (slices.dtype != torch.uint8 or not slices.is_contiguous()
                               or slices.numel() < m_bits * n):
        raise ValueError("slices must be contiguous uint8 [m_bits, n]")
    if out is None:
        out = tuple(torch.empty(n, dtype=_TORCH_OF[out_dtype], device=x.device) for _ in range(3))
    th = _host(thresholds, np.float64)
    check(load().slice_llr_next(_ptr(x), n, float(sigma_n), th.ctypes.data, int(m_bits), int(labelling), int(j),
                                int(known_mask), _ptr(slices), int(out_dtype), _ptr(out[0]), _ptr(out[1]),
                                _ptr(out[2]), _stream(stream)), "slice_llr_next")
    return out


def slice_llr_choose(llr_if0: torch.Tensor, llr_if1: torch.Tensor, bits: torch.Tensor,
                     out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Per sample: llr_if1 where bits & 1, else llr_if0."""
    n = llr_if0.numel()
    if llr_if1.dtype != llr_if0.dtype or llr_if1.numel() != n or bits.dtype != torch.uint8 or bits.numel() < n:
        raise ValueError("llr_if0/llr_if1 must match in dtype and size; bits uint8 with >= n entries")
    if llr_if0.dtype == torch.float32:
        dt = F32
    elif llr_if0.dtype == torch.float64:
        dt = F64
    else:
        raise ValueError("LLRs must be float32 or float64")
    if out is None:
        out = torch.empty_like(llr_if0)
    check(load().slice_llr_choose(_ptr(llr_if0), _ptr(llr_if1), _ptr(bits), n, dt, _ptr(out), _stream(stream)),
          "slice_llr_choose")
    return out


def slice_llr_bsc(x: torch.Tensor, thresholds, m_bits: int, j: int, p: float, labelling: int = GRAY,
                  out_dtype: int = F32, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Alice's hard LLRs (1 - 2 a_j) ln((1 - p) / p) from her own quantised bit a_j."""
    if x.dtype != torch.float64:
        raise ValueError("x must be float64")
    n = x.numel()
    if out is None:
        out = torch.empty(n, dtype=_TORCH_OF[out_dtype], device=x.device)
    th = _host(thresholds, np.float64)
    check(load().slice_llr_bsc(_ptr(x), n, th.ctypes.data, int(m_bits), int(labelling), int(j), float(p),
                               int(out_dtype), _ptr(out), _stream(stream)), "slice_llr_bsc")
    return out


def syndrome_check(code: Code, bits: torch.Tensor, syndrome: torch.Tensor | None = None,
                   want_syndrome: bool = True, want_unsat: bool = True, stream=None,
                   out_syndrome: torch.Tensor | None = None, out_unsat: torch.Tensor | None = None):
    """(syndrome_out uint8 [F, m] | None, n_unsat int32 [F] | None) of bits [F, n]."""
    if bits.dtype != torch.uint8:
        raise ValueError("bits must be uint8")
    F = bits.numel() // code.n
    if F * code.n != bits.numel():
        raise ValueError("bits size is not a multiple of n")
    s_out = out_syndrome
    if s_out is None and want_syndrome:
        s_out = torch.empty((F, code.m), dtype=torch.uint8, device=bits.device)
    if s_out is not None and (s_out.dtype != torch.uint8 or s_out.numel() < F * code.m):
        raise ValueError("out_syndrome must be uint8 with F * m entries")
    u = out_unsat
    if u is None and want_unsat:
        u = torch.empty(F, dtype=torch.int32, device=bits.device)
    if u is not None and (u.dtype != torch.int32 or u.numel() < F):
        raise ValueError("out_unsat must be int32 with F entries")
    check(load().syndrome_check(code.handle, F, _ptr(bits), _ptr(syndrome), _ptr(s_out), _ptr(u),
                                _stream(stream)), "syndrome_check")
    return s_out, u


def _check_weights(weights: torch.Tensor, T: int, n_types: int, what: str) -> None:
    """The kernels read weights[t * n_types + type] for every t < T."""
    if not isinstance(weights, torch.Tensor):
        raise ValueError(f"{what}: weights must be a tensor")
    if weights.dtype != torch.float32 or not weights.is_contiguous():
        raise ValueError(f"{what}: weights must be contiguous float32")
    if weights.numel() != T * n_types:
        raise ValueError(f"{what}: weights must hold max_iter x n_types = {T} x {n_types} entries, "
                         f"not {weights.numel()}")
    if not weights.is_cuda:
        raise ValueError(f"{what}: weights must be a device tensor")


def _check_len(t: torch.Tensor, n: int, dtype, what: str) -> None:
    if t.dtype != dtype or not t.is_contiguous() or t.numel() < n:
        raise ValueError(f"{what} must be contiguous {dtype} with >= {n} entries")


def decode_workspace_size(batch: Batch, params: Params) -> int:
    sz = C.c_size_t()
    p = params.c_struct()
    check(load().cvr_decode_workspace_size(batch.handle, C.byref(p), C.byref(sz)), "cvr_decode_workspace_size")
    return sz.value


def alloc_workspace(batch: Batch, params: Params, device=None) -> torch.Tensor:
    nbytes = decode_workspace_size(batch, params)
    # torch's caching allocator returns >= 512-byte aligned blocks
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device or "cuda")


def ldpc_decode_batch(batch: Batch, params: Params, llr: torch.Tensor, syndrome: torch.Tensor | None = None,
                      workspace: torch.Tensor | None = None, want_post: bool = True,
                      trace: torch.Tensor | None = None, out: dict | None = None, stream=None) -> dict:
    """Decodes every frame of ``batch``.  Returns dict(bits, post, iters, ok)."""
    mdt = _TORCH_OF[params.math]
    if llr.dtype != mdt:
        raise ValueError(f"llr must be {mdt}")
    if llr.numel() < batch.total_n:
        raise ValueError("llr is shorter than the batch")
    if syndrome is not None and (syndrome.dtype != torch.uint8 or syndrome.numel() < batch.total_m):
        raise ValueError("syndrome must be uint8 with >= total_m entries")
    dev = llr.device
    if out is None:
        out = dict(bits=torch.empty(batch.total_n, dtype=torch.uint8, device=dev),
                   post=torch.empty(batch.total_n, dtype=mdt, device=dev) if want_post else None,
                   iters=torch.empty(batch.F, dtype=torch.int32, device=dev),
                   ok=torch.empty(batch.F, dtype=torch.uint8, device=dev))
    if workspace is None:
        workspace = alloc_workspace(batch, params, dev)
    if trace is not None and (trace.dtype != mdt or trace.numel() < (params.max_iter + 1) * batch.total_n):
        raise ValueError("trace must have (max_iter + 1) * total_n entries of the math dtype")
    if params.weights is not None:
        _check_weights(params.weights, params.max_iter, batch.n_types, "ldpc_decode_batch")
    p = params.c_struct(trace)
    check(load().ldpc_decode_batch(batch.handle, C.byref(p), _ptr(llr), _ptr(syndrome), _ptr(out["bits"]),
                                   _ptr(out.get("post")), _ptr(out["iters"]), _ptr(out["ok"]),
                                   _ptr(workspace), workspace.numel(), _stream(stream)), "ldpc_decode_batch")
    return out


NOALLOC_SCRATCH_BYTES = 64 << 20      # the library's static decode workspace per GPU


def ldpc_decode_batch_noalloc(batch: Batch, params: Params, llr: torch.Tensor, syndrome: torch.Tensor | None,
                              out: dict, trace: torch.Tensor | None = None, stream=None) -> dict:
    """ldpc_decode_batch with the library's static workspace: the caller passes
    preallocated outputs (dict of bits, post or None, iters, ok) and nothing is
    allocated.  Calls that overlap on one GPU race (they share the array)."""
    mdt = _TORCH_OF[params.math]
    if llr.dtype != mdt or llr.numel() < batch.total_n:
        raise ValueError(f"llr must be {mdt} with >= total_n entries")
    if syndrome is not None and (syndrome.dtype != torch.uint8 or syndrome.numel() < batch.total_m):
        raise ValueError("syndrome must be uint8 with >= total_m entries")
    if out["bits"].dtype != torch.uint8 or out["bits"].numel() < batch.total_n:
        raise ValueError("out['bits'] must be uint8 with >= total_n entries")
    if out.get("post") is not None and (out["post"].dtype != mdt or out["post"].numel() < batch.total_n):
        raise ValueError(f"out['post'] must be {mdt} with >= total_n entries")
    if out["iters"].dtype != torch.int32 or out["iters"].numel() < batch.F:
        raise ValueError("out['iters'] must be int32 with >= F entries")
    if out["ok"].dtype != torch.uint8 or out["ok"].numel() < batch.F:
        raise ValueError("out['ok'] must be uint8 with >= F entries")
    if trace is not None and (trace.dtype != mdt or trace.numel() < (params.max_iter + 1) * batch.total_n):
        raise ValueError("trace must have (max_iter + 1) * total_n entries of the math dtype")
    if params.weights is not None:
        _check_weights(params.weights, params.max_iter, batch.n_types, "ldpc_decode_batch_noalloc")
    p = params.c_struct(trace)
    check(load().ldpc_decode_batch_noalloc(batch.handle, C.byref(p), _ptr(llr), _ptr(syndrome), _ptr(out["bits"]),
                                           _ptr(out.get("post")), _ptr(out["iters"]), _ptr(out["ok"]),
                                           _stream(stream)), "ldpc_decode_batch_noalloc")
    return out


def check_abandoned(out: dict) -> None:
    """Raises CvrError(CVR_EHIP) when the decode that wrote ``out`` was abandoned
    (iters = -1: a barrier of the group schedule gave up because its workgroups
    were not all resident).  Waits for the decode."""
    if out["iters"].numel() and int(out["iters"].min().item()) < 0:
        raise _lib.CvrError(_lib.CVR_EHIP, "ldpc_decode_batch",
                            "the decode was abandoned: a group barrier gave up (frames report iters = -1)")


def version() -> int:
    return int(load().cvr_version())


GROUP_WAIT_TICKS_DEFAULT = 20_000_000


def debug_group_wait_ticks(ticks: int = GROUP_WAIT_TICKS_DEFAULT) -> None:
    """Testing hook: bound of one group-barrier wait in 100 MHz ticks (0: give up at once)."""
    check(load().cvr_debug_group_wait_ticks(int(ticks)), "cvr_debug_group_wait_ticks")


# ---------------------------------------------------------------------------
# launch timing
# ---------------------------------------------------------------------------
PROF_QUANTIZE, PROF_LLR, PROF_SYNDROME, PROF_CHECK, PROF_VAR, PROF_DEC_SETUP, PROF_FRAMES, PROF_ADJOINT = range(8)


def profile_enable(on: bool = True) -> None:
    check(load().cvr_profile_enable(int(bool(on))), "cvr_profile_enable")


def profile_read(kind: int, reset: bool = False) -> tuple[float, int]:
    """(summed milliseconds, number of launches) of one kernel kind."""
    ms = C.c_double()
    cnt = C.c_int64()
    check(load().cvr_profile_read(int(kind), C.byref(ms), C.byref(cnt), int(bool(reset))), "cvr_profile_read")
    return ms.value, cnt.value


# ---------------------------------------------------------------------------
# differentiable unrolled min-sum
# ---------------------------------------------------------------------------
def nms_unrolled_sizes(batch: Batch, T: int, ckpt_every: int) -> tuple[int, int, int]:
    """(checkpoint floats, forward workspace bytes, backward workspace bytes)."""
    ck, fw, bw = C.c_size_t(), C.c_size_t(), C.c_size_t()
    check(load().nms_unrolled_sizes(batch.handle, int(T), int(ckpt_every), C.byref(ck), C.byref(fw), C.byref(bw)),
          "nms_unrolled_sizes")
    return ck.value, fw.value, bw.value


def nms_unrolled_fwd(batch: Batch, T: int, ckpt_every: int, weights: torch.Tensor, llr: torch.Tensor,
                     syndrome: torch.Tensor | None = None, stream=None):
    """Posteriors after T weighted min-sum iterations and the checkpoints."""
    ck, fw, _ = nms_unrolled_sizes(batch, T, ckpt_every)
    _check_weights(weights, T, batch.n_types, "nms_unrolled_fwd")
    _check_len(llr, batch.total_n, torch.float32, "nms_unrolled_fwd: llr")
    if syndrome is not None:
        _check_len(syndrome, batch.total_m, torch.uint8, "nms_unrolled_fwd: syndrome")
    dev = llr.device
    post = torch.empty(batch.total_n, dtype=torch.float32, device=dev)
    ckpt = torch.empty(max(ck, 1), dtype=torch.float32, device=dev)
    ws = torch.empty(max(fw, 256), dtype=torch.uint8, device=dev)
    check(load().nms_unrolled_fwd(batch.handle, int(T), int(ckpt_every), _ptr(weights), _ptr(llr),
                                  _ptr(syndrome), _ptr(post), _ptr(ckpt), _ptr(ws), ws.numel(), _stream(stream)),
          "nms_unrolled_fwd")
    return post, ckpt


def nms_unrolled_bwd(batch: Batch, T: int, ckpt_every: int, weights: torch.Tensor, llr: torch.Tensor,
                     syndrome: torch.Tensor | None, ckpt: torch.Tensor, dloss_dpost: torch.Tensor,
                     want_dllr: bool = False, stream=None):
    """(d loss / d weights [T, n_types], d loss / d llr or None)."""
    _, _, bw = nms_unrolled_sizes(batch, T, ckpt_every)
    _check_weights(weights, T, batch.n_types, "nms_unrolled_bwd")
    _check_len(llr, batch.total_n, torch.float32, "nms_unrolled_bwd: llr")
    _check_len(dloss_dpost, batch.total_n, torch.float32, "nms_unrolled_bwd: dloss_dpost")
    if syndrome is not None:
        _check_len(syndrome, batch.total_m, torch.uint8, "nms_unrolled_bwd: syndrome")
    ck, _, _ = nms_unrolled_sizes(batch, T, ckpt_every)
    _check_len(ckpt, ck, torch.float32, "nms_unrolled_bwd: ckpt")
    dev = llr.device
    dw = torch.empty_like(weights, dtype=torch.float32).contiguous()
    dl = torch.empty(batch.total_n, dtype=torch.float32, device=dev) if want_dllr else None
    ws = torch.empty(max(bw, 256), dtype=torch.uint8, device=dev)
    check(load().nms_unrolled_bwd(batch.handle, int(T), int(ckpt_every), _ptr(weights), _ptr(llr),
                                  _ptr(syndrome), _ptr(ckpt), _ptr(dloss_dpost), _ptr(dw), _ptr(dl),
                                  _ptr(ws), ws.numel(), _stream(stream)), "nms_unrolled_bwd")
    return dw, dl


class NMSUnrolled(torch.autograd.Function):
    """L_post(T) of T-iteration weighted min-sum as a differentiable function of
    the weights [T, n_types] (and of the channel LLRs).  Backward is the
    library's adjoint kernel with checkpointed recomputation."""

    @staticmethod
    def forward(ctx, weights, llr, syndrome, batch, T, ckpt_every):
        w = weights.detach().contiguous()
        l = llr.detach().contiguous()
        post, ckpt = nms_unrolled_fwd(batch, T, ckpt_every, w, l, syndrome)
        ctx.save_for_backward(w, l, ckpt)
        ctx.syndrome = syndrome
        ctx.batch, ctx.T, ctx.K = batch, T, ckpt_every
        return post

    @staticmethod
    def backward(ctx, grad_post):
        w, l, ckpt = ctx.saved_tensors
        dw, dl = nms_unrolled_bwd(ctx.batch, ctx.T, ctx.K, w, l, ctx.syndrome, ckpt, grad_post.contiguous(),
                                  want_dllr=ctx.needs_input_grad[1])
        return dw, dl, None, None, None, None
