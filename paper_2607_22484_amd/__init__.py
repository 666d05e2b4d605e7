"""Singular value soft-thresholding through the polar decomposition, on
AMD MI355X (gfx950).

Thin Python binding over ``libpsvt.so`` (C ABI in ``include/psvt.h``).  The
functions here only marshal arguments: check shapes and dtypes, allocate the
output and workspace with torch on the current HIP device, and pass raw
device pointers and the current stream to the library.  Every step of the
computation runs in the library's kernels.  There is no fallback: without the
built library or a gfx950 device the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpsvt.so")

PSVT_OK = 0
PSVT_EINVAL = -1
PSVT_EWORKSPACE = -2
PSVT_EUNSUPPORTED = -3
PSVT_EHIP = -4

OP_SVT, OP_POLAR, OP_POLAR_SYM, OP_RANK_R = 0, 1, 2, 3
SIDE_AUTO, SIDE_RIGHT, SIDE_LEFT = 0, 1, 2
DTYPE_F32, DTYPE_BF16, DTYPE_FP8, DTYPE_BF16X3 = 0, 1, 2, 3
FLAG_PLAIN_S, FLAG_SPLIT_P, FLAG_PLAIN_P, FLAG_STATUS, FLAG_HFORM = 0x1, 0x2, 0x4, 0x8, 0x10
FLAG_PERSISTENT, FLAG_GRAM = 0x20, 0x40
STATUS_NONFINITE_INPUT, STATUS_NONFINITE_OUTPUT, STATUS_NOT_CONVERGED, STATUS_INVALID = 0x1, 0x2, 0x4, 0x8

EXPORTED = [
    "psvt_workspace_bytes", "psvt_svt", "psvt_svt_noalloc", "psvt_polar", "psvt_polar_sym", "psvt_rank_r", "psvt_gemm_nt", "psvt_convert",
    "psvt_strerror", "psvt_last_error", "psvt_version", "psvt_trace_begin", "psvt_trace_end",
    "psvt_tune_force_tile", "psvt_tune_set", "psvt_tune_load", "psvt_tune_pick", "psvt_tune_persistent_tiles",
    "psvt_tune_spin_limit", "psvt_batched_workspace_bytes", "psvt_batched_check_schedule", "psvt_svt_batched", "psvt_rank_r_batched",
    "psvt_batch_workspace_bytes", "psvt_batch_create", "psvt_batch_run", "psvt_batch_run_graph", "psvt_batch_stats",
    "psvt_batch_destroy", "psvt_server_create", "psvt_server_submit", "psvt_server_poll", "psvt_server_wait",
    "psvt_server_drain", "psvt_server_stats", "psvt_server_set_timeout", "psvt_server_inject_fault",
    "psvt_server_destroy",
]
SERVER_FAKE, SERVER_COHORT, SERVER_EAGER = 0x1, 0x2, 0x4
FAULT_TICK, FAULT_PLAN, FAULT_STALL = 1, 2, 3
RQ_QUEUED, RQ_RUNNING, RQ_DONE, RQ_FAILED = 0, 1, 2, -1
TILE_IDS = {64: 1, 128: 2, 192: 3, 256: 4}
TUNE_TABLE = os.path.join(_HERE, "tune_table.txt")


class PsvtError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__("%s failed (%d): %s" % (where, code, detail))
        self.code = code


class Config(ctypes.Structure):
    """Mirror of ``psvt_config``."""
    _fields_ = [
        ("iters", ctypes.c_int32),
        ("n_fp8", ctypes.c_int32),
        ("n_bf16", ctypes.c_int32),
        ("side", ctypes.c_int32),
        ("coeffs", ctypes.POINTER(ctypes.c_double)),
        ("flags", ctypes.c_uint32),
        ("reserved0", ctypes.c_int32),
        ("norm_safety", ctypes.c_double),
        ("status", ctypes.c_void_p),
        ("status_tol", ctypes.c_double),
        ("warm_pi", ctypes.c_void_p),
        ("pi_out", ctypes.c_void_p),
        ("ld_pi", ctypes.c_int64),
        ("warm_iters", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 3),
    ]


class BatchItem(ctypes.Structure):
    """Mirror of ``psvt_batch_item``."""
    _fields_ = [("A", ctypes.c_void_p), ("Y", ctypes.c_void_p), ("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("lda", ctypes.c_int64), ("ldy", ctypes.c_int64), ("tau", ctypes.c_double),
                ("warm_pi", ctypes.c_void_p), ("pi_out", ctypes.c_void_p), ("ld_pi", ctypes.c_int64)]


class Desc(ctypes.Structure):
    """Mirror of ``psvt_desc`` (one matrix of a device-described batch)."""
    _fields_ = [("A", ctypes.c_void_p), ("Y", ctypes.c_void_p), ("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("lda", ctypes.c_int64), ("ldy", ctypes.c_int64), ("tau", ctypes.c_double),
                ("status", ctypes.c_void_p)]


class ServerCounters(ctypes.Structure):
    """Mirror of ``psvt_server_counters``."""
    _fields_ = [(k, ctypes.c_int64) for k in ("submitted", "completed", "failed", "queued", "active", "ticks",
                                              "launches")] + \
               [(k, ctypes.c_double) for k in ("p50_ms", "p99_ms", "max_ms", "queue_p99_ms", "matrices_per_s")] + \
               [("budget_bytes", ctypes.c_size_t), ("peak_bytes", ctypes.c_size_t), ("timed_out", ctypes.c_int64)]


class TraceStat(ctypes.Structure):
    """Mirror of ``psvt_trace_stat``."""
    _fields_ = [("name", ctypes.c_char_p), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("flops", ctypes.c_double), ("bytes", ctypes.c_double)]


_lib = None


def load(path: Optional[str] = None):
    """Load ``libpsvt.so`` (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError("libpsvt.so is not built (run python -m paper_2607_22484_amd.build)")
    lib = ctypes.CDLL(path)
    i64, vp, f64 = ctypes.c_int64, ctypes.c_void_p, ctypes.c_double
    cfgp = ctypes.POINTER(Config)
    lib.psvt_workspace_bytes.argtypes = [ctypes.c_int, i64, i64, cfgp, ctypes.POINTER(ctypes.c_size_t)]
    lib.psvt_svt.argtypes = [vp, i64, i64, i64, f64, vp, i64, vp, ctypes.c_size_t, cfgp, vp]
    lib.psvt_rank_r.argtypes = [vp, i64, i64, i64, f64, vp, i64, vp, ctypes.c_size_t, cfgp, vp]
    lib.psvt_svt_noalloc.argtypes = [vp, i64, i64, i64, f64, vp, i64, cfgp, vp]
    lib.psvt_svt_noalloc.restype = ctypes.c_int
    lib.psvt_polar.argtypes = [vp, i64, i64, i64, vp, i64, vp, ctypes.c_size_t, cfgp, vp]
    lib.psvt_polar_sym.argtypes = [vp, i64, i64, vp, i64, vp, ctypes.c_size_t, cfgp, vp]
    lib.psvt_gemm_nt.argtypes = [ctypes.c_int, vp, i64, vp, i64, vp, i64, vp, i64, i64, i64, i64, ctypes.c_float,
                                 ctypes.c_float, ctypes.c_int, vp]
    lib.psvt_convert.argtypes = [ctypes.c_int, vp, i64, i64, i64, vp, i64, ctypes.c_float, ctypes.c_int, vp]
    for f in ("psvt_workspace_bytes", "psvt_svt", "psvt_rank_r", "psvt_polar", "psvt_polar_sym", "psvt_gemm_nt",
              "psvt_convert"):
        getattr(lib, f).restype = ctypes.c_int
    lib.psvt_strerror.argtypes = [ctypes.c_int]
    lib.psvt_strerror.restype = ctypes.c_char_p
    lib.psvt_last_error.restype = ctypes.c_char_p
    lib.psvt_version.restype = ctypes.c_char_p
    lib.psvt_tune_force_tile.argtypes = [ctypes.c_int]
    lib.psvt_tune_set.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double]
    lib.psvt_tune_load.argtypes = [ctypes.c_char_p]
    lib.psvt_tune_pick.argtypes = [ctypes.c_int, i64, i64, i64, ctypes.c_int]
    lib.psvt_tune_persistent_tiles.argtypes = [ctypes.c_int]
    lib.psvt_tune_spin_limit.argtypes = [i64]
    for f in ("psvt_tune_force_tile", "psvt_tune_set", "psvt_tune_load", "psvt_tune_pick",
              "psvt_tune_persistent_tiles", "psvt_tune_spin_limit"):
        getattr(lib, f).restype = ctypes.c_int
    items_p = ctypes.POINTER(BatchItem)
    lib.psvt_batch_workspace_bytes.argtypes = [ctypes.c_int, items_p, ctypes.c_int32, cfgp,
                                               ctypes.POINTER(ctypes.c_size_t)]
    lib.psvt_batch_create.argtypes = [ctypes.c_int, items_p, ctypes.c_int32, vp, ctypes.c_size_t, cfgp,
                                      ctypes.POINTER(ctypes.c_void_p)]
    lib.psvt_batch_run.argtypes = [vp, vp]
    lib.psvt_batch_run_graph.argtypes = [vp, vp]
    lib.psvt_batch_stats.argtypes = [vp, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)]
    lib.psvt_batch_destroy.argtypes = [vp]
    for f in ("psvt_batch_workspace_bytes", "psvt_batch_create", "psvt_batch_run", "psvt_batch_run_graph",
              "psvt_batch_stats", "psvt_batch_destroy"):
        getattr(lib, f).restype = ctypes.c_int
    lib.psvt_batched_workspace_bytes.argtypes = [ctypes.c_int, ctypes.c_int32, i64, i64, cfgp,
                                                 ctypes.POINTER(ctypes.c_size_t)]
    for f in ("psvt_svt_batched", "psvt_rank_r_batched"):
        getattr(lib, f).argtypes = [vp, ctypes.c_int32, i64, i64, vp, ctypes.c_size_t, cfgp, vp]
    i64p = ctypes.POINTER(i64)
    lib.psvt_batched_check_schedule.argtypes = [ctypes.c_int, i64p, i64p, ctypes.c_int32, i64, i64, cfgp,
                                                ctypes.c_int32, ctypes.c_uint64, i64p]
    for f in ("psvt_batched_workspace_bytes", "psvt_svt_batched", "psvt_rank_r_batched", "psvt_batched_check_schedule"):
        getattr(lib, f).restype = ctypes.c_int
    srv = ctypes.c_void_p
    lib.psvt_server_create.argtypes = [ctypes.c_size_t, ctypes.c_int32, cfgp, ctypes.c_uint32,
                                       ctypes.POINTER(ctypes.c_void_p)]
    lib.psvt_server_submit.argtypes = [srv, ctypes.c_int, items_p, vp, ctypes.POINTER(ctypes.c_uint64)]
    lib.psvt_server_poll.argtypes = [srv, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int32)]
    lib.psvt_server_wait.argtypes = [srv, ctypes.c_uint64, ctypes.c_double, ctypes.POINTER(ctypes.c_int32)]
    lib.psvt_server_drain.argtypes = [srv, ctypes.c_double]
    lib.psvt_server_stats.argtypes = [srv, ctypes.POINTER(ServerCounters)]
    lib.psvt_server_set_timeout.argtypes = [srv, ctypes.c_double]
    lib.psvt_server_inject_fault.argtypes = [srv, ctypes.c_int, i64]
    lib.psvt_server_destroy.argtypes = [srv]
    for f in ("psvt_server_create", "psvt_server_submit", "psvt_server_poll", "psvt_server_wait",
              "psvt_server_drain", "psvt_server_stats", "psvt_server_set_timeout", "psvt_server_inject_fault",
              "psvt_server_destroy"):
        getattr(lib, f).restype = ctypes.c_int
    lib.psvt_trace_begin.restype = ctypes.c_int
    lib.psvt_trace_end.restype = ctypes.c_int
    lib.psvt_trace_end.argtypes = [ctypes.POINTER(TraceStat), ctypes.c_int, ctypes.POINTER(ctypes.c_int)]
    if os.path.exists(TUNE_TABLE):
        rc = lib.psvt_tune_load(TUNE_TABLE.encode())
        if rc != PSVT_OK:
            raise PsvtError(rc, "psvt_tune_load", lib.psvt_last_error().decode())
    _lib = lib
    return lib


def _check(rc: int, where: str):
    if rc != PSVT_OK:
        lib = load()
        raise PsvtError(rc, where, (lib.psvt_last_error() or b"").decode() or lib.psvt_strerror(rc).decode())


def make_config(iters: int = 20, n_fp8: int = 0, n_bf16: int = 0, side: int = SIDE_AUTO,
                coeffs: Optional[Sequence[float]] = None, flags: int = 0, norm_safety: float = 0.0,
                status=None, status_tol: float = 0.0, warm_pi=None, pi_out=None, warm_iters: int = 0):
    """A ``psvt_config``.  ``status``: a 1-element int32/uint32 GPU tensor
    (or a raw device pointer) that receives the status word; passing it sets
    FLAG_STATUS.  ``warm_pi`` / ``pi_out``: s x s float32 GPU tensors (the
    previous call's and this call's (I + S)/2; s the Gram side)."""
    cfg = Config()
    cfg.iters = int(iters)
    cfg.n_fp8 = int(n_fp8)
    cfg.n_bf16 = int(n_bf16)
    cfg.side = int(side)
    cfg.norm_safety = float(norm_safety)
    cfg.status_tol = float(status_tol)
    cfg.warm_iters = int(warm_iters)
    if status is not None:
        ptr = status if isinstance(status, int) else _status_ptr(status)
        cfg.status = ptr
        flags = int(flags) | FLAG_STATUS
    ld = None
    for t, field in ((warm_pi, "warm_pi"), (pi_out, "pi_out")):
        if t is not None:
            _check_pi(t)
            setattr(cfg, field, t.data_ptr())
            ld = _ld(t)
    if ld is not None:
        cfg.ld_pi = ld
    cfg.flags = int(flags)
    keep = None
    if coeffs is not None:
        keep = (ctypes.c_double * len(coeffs))(*[float(c) for c in coeffs])
        cfg.coeffs = ctypes.cast(keep, ctypes.POINTER(ctypes.c_double))
    return cfg, keep


def _check_pi(t):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.ndim != 2 or t.shape[0] != t.shape[1] or t.dtype != torch.float32 \
            or t.device.type != "cuda" or t.stride(1) != 1:
        raise TypeError("warm_pi / pi_out must be square float32 GPU tensors with unit column stride")


def _status_ptr(t):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.numel() < 1 or t.element_size() != 4:
        raise TypeError("status must be a GPU tensor with at least one 4-byte element")
    return t.data_ptr()


def workspace_bytes(op: int, m: int, n: int, cfg: Optional[Config] = None) -> int:
    out = ctypes.c_size_t(0)
    _check(load().psvt_workspace_bytes(op, m, n, ctypes.byref(cfg) if cfg is not None else None,
                                       ctypes.byref(out)), "psvt_workspace_bytes")
    return int(out.value)


def _torch():
    import torch
    return torch


def _check_input(A, name="A"):
    torch = _torch()
    if not isinstance(A, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if A.ndim != 2:
        raise ValueError("input tensor must be 2D")
    if A.dtype != torch.float32:
        raise TypeError("%s must be float32" % name)
    if A.device.type != "cuda":
        raise TypeError("%s must live on the GPU" % name)
    if A.stride(1) != 1 and A.numel() > 0:
        raise ValueError("%s must be row-major with unit column stride" % name)


def _stream_ptr(A):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(A.device).cuda_stream)


def _workspace(op, m, n, cfg, device, ws=None):
    torch = _torch()
    need = workspace_bytes(op, m, n, cfg)
    if ws is not None:
        if not isinstance(ws, torch.Tensor):
            raise TypeError("ws must be a torch.Tensor")
        if ws.device != device:
            raise ValueError("ws must live on %s (got %s)" % (device, ws.device))
        if not ws.is_contiguous():
            raise ValueError("ws must be contiguous")
        if ws.numel() * ws.element_size() < need:
            raise ValueError("workspace too small: %d < %d bytes" % (ws.numel() * ws.element_size(), need))
        return ws, need
    return torch.empty(max(need, 256), dtype=torch.uint8, device=device), need


def _output(out, shape, device, name="out"):
    """The caller's output buffer, checked before anything is launched: a
    float32 tensor of exactly `shape` on `device` with unit column stride
    (the C ABI only sees a pointer and a row stride)."""
    torch = _torch()
    if out is None:
        return torch.empty(shape, dtype=torch.float32, device=device)
    if not isinstance(out, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if out.dtype != torch.float32:
        raise TypeError("%s must be float32 (got %s)" % (name, out.dtype))
    if tuple(out.shape) != tuple(shape):
        raise ValueError("%s must have shape %s (got %s)" % (name, tuple(shape), tuple(out.shape)))
    if out.device != device:
        raise ValueError("%s must live on %s (got %s)" % (name, device, out.device))
    if out.numel() > 0 and (out.stride(1) != 1 or (out.shape[0] > 1 and out.stride(0) < out.shape[1])):
        raise ValueError("%s must be row-major with unit column stride" % name)
    return out


def _ld(A):
    """Row stride in elements.  A one-row tensor's stride is never stepped
    over, so any value >= the column count is valid; use a multiple of 4."""
    if A.shape[0] > 1:
        return A.stride(0)
    cols = max(A.shape[1], 1)
    return A.stride(0) if A.stride(0) >= cols and A.stride(0) % 4 == 0 else (cols + 3) // 4 * 4


def _ld_any(A):
    """Row stride in elements for any element size; one-row tensors get a
    stride that keeps rows 16-byte aligned."""
    if A.shape[0] > 1:
        return A.stride(0)
    per16 = max(1, 16 // A.element_size())
    cols = max(A.shape[1], 1)
    return A.stride(0) if A.stride(0) >= cols and A.stride(0) % per16 == 0 else (cols + per16 - 1) // per16 * per16


def _method(entry, op, A, tau, out, ws, kwargs, has_tau=True):
    """One call of a method entry point: checks, output, workspace, then the
    C call on the current stream of A's device."""
    _check_input(A)
    torch = _torch()
    m, n = A.shape
    cfg, keep = make_config(**kwargs)
    Y = _output(out, (m, n), A.device)
    if m == 0 or n == 0:
        return Y
    buf, need = _workspace(op, m, n, cfg, A.device, ws)
    args = [A.data_ptr(), m, n, _ld(A)] + ([float(tau)] if has_tau else []) + \
           [Y.data_ptr(), _ld(Y), buf.data_ptr(), need, ctypes.byref(cfg), _stream_ptr(A)]
    with torch.cuda.device(A.device):
        _check(getattr(load(), entry)(*args), entry)
    del keep
    return Y


def svt(A, tau: float, iters: int = 20, n_fp8: int = 0, n_bf16: int = 0, side: int = SIDE_AUTO,
        coeffs=None, out=None, ws=None, flags: int = 0, norm_safety: float = 0.0, status=None,
        status_tol: float = 0.0, warm_pi=None, pi_out=None, warm_iters: int = 0):
    """A_tau = U max(Sigma - tau I, 0) V^T via Proposition 1 (FP32 out).
    ``status``: optional 1-element int32 GPU tensor for the status word.
    ``warm_pi`` / ``pi_out``: warm start of the sign iteration from a
    previous call's (I + S)/2, and this call's (psvt.h)."""
    return _method("psvt_svt", OP_SVT, A, tau, out, ws,
                   dict(iters=iters, n_fp8=n_fp8, n_bf16=n_bf16, side=side, coeffs=coeffs, flags=flags,
                        norm_safety=norm_safety, status=status, status_tol=status_tol, warm_pi=warm_pi,
                        pi_out=pi_out, warm_iters=warm_iters))


def svt_noalloc(A, tau: float, iters: int = 20, n_fp8: int = 0, n_bf16: int = 0, side: int = SIDE_AUTO,
                coeffs=None, out=None, flags: int = 0, norm_safety: float = 0.0, status=None,
                status_tol: float = 0.0):
    """svt through psvt_svt_noalloc: the library's static device scratch
    instead of a workspace (no device allocation by the library; the output
    is allocated here unless ``out`` is given).  Sizes up to the scratch
    capacity (PSVT_NOALLOC_SCRATCH_BYTES, every schedule up to 1024^2)."""
    _check_input(A)
    torch = _torch()
    m, n = A.shape
    cfg, keep = make_config(iters, n_fp8, n_bf16, side, coeffs, flags, norm_safety, status, status_tol)
    Y = _output(out, (m, n), A.device)
    if m == 0 or n == 0:
        return Y
    with torch.cuda.device(A.device):
        _check(load().psvt_svt_noalloc(A.data_ptr(), m, n, _ld(A), float(tau), Y.data_ptr(), _ld(Y),
                                       ctypes.byref(cfg), _stream_ptr(A)), "psvt_svt_noalloc")
    del keep
    return Y


def rank_r(A, tau: float, iters: int = 20, n_fp8: int = 0, n_bf16: int = 0, side: int = SIDE_AUTO,
           coeffs=None, out=None, ws=None, flags: int = 0, norm_safety: float = 0.0, status=None,
           status_tol: float = 0.0, warm_pi=None, pi_out=None, warm_iters: int = 0):
    """Best rank-r approximation (Corollary 1), tau between sigma_{r+1} and sigma_r."""
    return _method("psvt_rank_r", OP_RANK_R, A, tau, out, ws,
                   dict(iters=iters, n_fp8=n_fp8, n_bf16=n_bf16, side=side, coeffs=coeffs, flags=flags,
                        norm_safety=norm_safety, status=status, status_tol=status_tol, warm_pi=warm_pi,
                        pi_out=pi_out, warm_iters=warm_iters))


def polar(A, iters: int = 20, n_fp8: int = 0, n_bf16: int = 0, side: int = SIDE_AUTO, coeffs=None, out=None,
          ws=None, flags: int = 0, norm_safety: float = 0.0, status=None):
    """Polar factor U V^T (section 2)."""
    return _method("psvt_polar", OP_POLAR, A, None, out, ws,
                   dict(iters=iters, n_fp8=n_fp8, n_bf16=n_bf16, side=side, coeffs=coeffs, flags=flags,
                        norm_safety=norm_safety, status=status), has_tau=False)


def polar_sym(G, iters: int = 20, n_fp8: int = 0, n_bf16: int = 0, coeffs=None, out=None, ws=None,
              flags: int = 0, norm_safety: float = 0.0, status=None, status_tol: float = 0.0):
    """Matrix sign of symmetric G (symmetrised on load)."""
    _check_input(G, "G")
    torch = _torch()
    n, n2 = G.shape
    if n != n2:
        raise ValueError("polar_sym needs a square matrix")
    cfg, keep = make_config(iters, n_fp8, n_bf16, SIDE_AUTO, coeffs, flags, norm_safety, status, status_tol)
    S = _output(out, (n, n), G.device)
    if n == 0:
        return S
    buf, need = _workspace(OP_POLAR_SYM, n, n, cfg, G.device, ws)
    with torch.cuda.device(G.device):
        _check(load().psvt_polar_sym(G.data_ptr(), n, _ld(G), S.data_ptr(), _ld(S), buf.data_ptr(), need,
                                     ctypes.byref(cfg), _stream_ptr(G)), "psvt_polar_sym")
    del keep
    return S


_DTYPE_OF = {"float32": DTYPE_F32, "bfloat16": DTYPE_BF16, "uint8": DTYPE_FP8, "float8_e4m3fn": DTYPE_FP8}


def gemm_nt(A, B, D=None, alpha: float = 1.0, beta: float = 0.0, sym: bool = False, out=None, dtype=None):
    """C = alpha A B^T + beta D with the library's MFMA kernel.  A and B hold
    float32, bfloat16, or FP8 e4m3 bytes (uint8 / float8_e4m3fn tensors); with
    dtype=DTYPE_BF16X3 they are split-bf16 pairs of planes as ``convert``
    writes them (the product is hi.hi + hi.lo + lo.hi)."""
    torch = _torch()
    for X, name in ((A, "A"), (B, "B")):
        if not isinstance(X, torch.Tensor) or X.ndim != 2 or X.device.type != "cuda" or X.stride(1) != 1:
            raise TypeError("%s must be a 2-D row-major GPU tensor" % name)
    dt = _DTYPE_OF.get(str(A.dtype).replace("torch.", "")) if dtype is None else dtype
    if dt is None or A.dtype != B.dtype:
        raise TypeError("unsupported operand dtype %s / %s" % (A.dtype, B.dtype))
    M, K = A.shape
    N, K2 = B.shape
    if dt == DTYPE_BF16X3:  # split operands: hi plane rows, then lo plane rows (as convert writes them)
        if M % 2 or N % 2:
            raise ValueError("split bf16 operands hold two planes of equal height")
        M, N = M // 2, N // 2
    if K != K2:
        raise ValueError("inner dimensions differ")
    C = out if out is not None else torch.empty((M, N), dtype=torch.float32, device=A.device)
    dptr, ldd = (D.data_ptr(), _ld(D)) if D is not None else (None, 0)
    with torch.cuda.device(A.device):
        _check(load().psvt_gemm_nt(dt, A.data_ptr(), _ld_any(A), B.data_ptr(), _ld_any(B), dptr, ldd, C.data_ptr(),
                                   _ld(C), M, N, K, float(alpha), float(beta), 1 if sym else 0, _stream_ptr(A)),
               "psvt_gemm_nt")
    return C


def convert(X, dtype: int, scale: float = 1.0, transpose: bool = False, out=None):
    """Round scale * X (float32) into bfloat16 bits (torch.bfloat16) or FP8
    e4m3 bytes (torch.uint8), optionally transposed."""
    torch = _torch()
    _check_input(X, "X")
    rows, cols = X.shape
    shape = (cols, rows) if transpose else (rows, cols)
    tdt = {DTYPE_F32: torch.float32, DTYPE_BF16: torch.bfloat16, DTYPE_FP8: torch.uint8,
           DTYPE_BF16X3: torch.bfloat16}[dtype]
    if dtype == DTYPE_BF16X3:  # hi plane then lo plane
        shape = (2 * shape[0], shape[1])
    Y = out if out is not None else torch.empty(shape, dtype=tdt, device=X.device)
    with torch.cuda.device(X.device):
        _check(load().psvt_convert(int(dtype), X.data_ptr(), rows, cols, _ld(X), Y.data_ptr(), _ld_any(Y),
                                   float(scale), 1 if transpose else 0, _stream_ptr(X)), "psvt_convert")
    return Y


def batched_workspace_bytes(count: int, max_m: int, max_n: int, cfg: Optional[Config] = None,
                            op: int = OP_SVT) -> int:
    out = ctypes.c_size_t(0)
    _check(load().psvt_batched_workspace_bytes(op, count, max_m, max_n, ctypes.byref(cfg) if cfg is not None else None,
                                               ctypes.byref(out)), "psvt_batched_workspace_bytes")
    return int(out.value)


def device_descriptors(As, taus, Ys, statuses=None, device=None):
    """A device array (uint8 tensor) of psvt_desc for the given tensors (the
    binding builds it on the host and copies it once)."""
    torch = _torch()
    arr = (Desc * len(As))()
    for i, (A, tau, Y) in enumerate(zip(As, taus, Ys)):
        st = statuses[i] if statuses is not None else None
        arr[i] = Desc(A.data_ptr(), Y.data_ptr(), A.shape[0], A.shape[1], _ld(A), _ld(Y), float(tau),
                      st.data_ptr() if st is not None else None)
    dev = device if device is not None else As[0].device
    return torch.frombuffer(bytearray(bytes(arr)), dtype=torch.uint8).to(dev)


def svt_batched_raw(d_descs_ptr: int, count: int, max_m: int, max_n: int, ws, cfg: Config, op: int = OP_SVT,
                    stream=None):
    """psvt_svt_batched / psvt_rank_r_batched on a device descriptor array
    (raw pointer) and a workspace tensor, on `stream` (a hipStream_t handle;
    None = the current torch stream of ws's device)."""
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream(ws.device).cuda_stream
    entry = "psvt_svt_batched" if op == OP_SVT else "psvt_rank_r_batched"
    with torch.cuda.device(ws.device):
        _check(getattr(load(), entry)(ctypes.c_void_p(d_descs_ptr), int(count), int(max_m), int(max_n),
                                      ws.data_ptr(), ws.numel() * ws.element_size(), ctypes.byref(cfg),
                                      ctypes.c_void_p(stream)), entry)


def check_persistent_schedule(shapes, max_m: int, max_n: int, iters: int = 20, n_fp8: int = 0, n_bf16: int = 0,
                              flags: int = 0, op: int = OP_SVT, blocks: int = 512, seed: int = 0) -> int:
    """Host replay of the persistent executor's schedule for ``shapes`` (list
    of (m, n)); raises RuntimeError naming a violated check; returns the
    ticket count (psvt_batched_check_schedule)."""
    n = len(shapes)
    ms = (ctypes.c_int64 * max(n, 1))(*[int(m) for m, _ in shapes])
    ns = (ctypes.c_int64 * max(n, 1))(*[int(k) for _, k in shapes])
    cfg, keep = make_config(iters, n_fp8, n_bf16, SIDE_AUTO, None, flags)
    out = ctypes.c_int64(0)
    _check(load().psvt_batched_check_schedule(op, ms, ns, n, int(max_m), int(max_n), ctypes.byref(cfg), int(blocks),
                                              int(seed), ctypes.byref(out)), "psvt_batched_check_schedule")
    del keep
    return int(out.value)


def persistent_aborted(ws) -> bool:
    """After a PSVT_FLAG_PERSISTENT call on ``ws`` (once its stream has
    passed it): whether a dependency wait passed its bound (the word at byte
    4 of the workspace)."""
    return bool(int(ws[4:8].view(_torch().int32).item()))


def svt_batched(As, taus, iters: int = 20, n_fp8: int = 0, n_bf16: int = 0, side: int = SIDE_AUTO, flags: int = 0,
                op: int = OP_SVT, outs=None, statuses=None, max_m=None, max_n=None, persistent: bool = False):
    """Soft-thresholding (or rank_r) of many matrices of uneven shapes in one
    device-described batched call on the current stream; returns the
    outputs (the descriptor array and workspace are kept until the stream
    has passed them).  ``persistent``: one persistent launch
    (PSVT_FLAG_PERSISTENT); raises RuntimeError if its abort flag is set."""
    torch = _torch()
    for A in As:
        _check_input(A)
    if not As:
        return []
    dev = As[0].device
    Ys = list(outs) if outs is not None else [torch.empty_like(A) for A in As]
    max_m = max_m or max(A.shape[0] for A in As)
    max_n = max_n or max(A.shape[1] for A in As)
    if statuses is not None:
        flags |= FLAG_STATUS
    if persistent:
        flags |= FLAG_PERSISTENT
    cfg, keep = make_config(iters, n_fp8, n_bf16, side, None, flags)
    need = batched_workspace_bytes(len(As), max_m, max_n, cfg, op)
    ws = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
    d = device_descriptors(As, taus, Ys, statuses, dev)
    svt_batched_raw(d.data_ptr(), len(As), max_m, max_n, ws, cfg, op)
    torch.cuda.current_stream(dev).synchronize()
    del keep
    if persistent and persistent_aborted(ws):
        raise RuntimeError("persistent batched call aborted: a dependency wait passed its bound")
    return Ys


class Batch:
    """Batched soft-thresholding of many uneven matrices (C ABI psvt_batch_*).

    ``As``: list of 2-D float32 GPU tensors; ``taus``: thresholds.  Outputs
    are allocated here (``Ys``).  ``run()`` enqueues the grouped launches,
    ``run_graph()`` replays the captured graph; both on the current stream."""

    def __init__(self, As, taus, iters: int = 20, n_fp8: int = 0, n_bf16: int = 0, op: int = OP_SVT,
                 flags: int = 0, side: int = SIDE_AUTO):
        torch = _torch()
        if len(As) != len(taus) or not As:
            raise ValueError("need one tau per matrix")
        for A in As:
            _check_input(A)
        self.As = list(As)
        self.Ys = [torch.empty_like(A) for A in As]
        items = (BatchItem * len(As))()
        for i, (A, Y, tau) in enumerate(zip(self.As, self.Ys, taus)):
            items[i] = BatchItem(A.data_ptr(), Y.data_ptr(), A.shape[0], A.shape[1], _ld(A), _ld(Y), float(tau),
                                 None, None, 0)
        self._items = items
        self.cfg, self._keep = make_config(iters, n_fp8, n_bf16, side, None, flags)
        lib = load()
        need = ctypes.c_size_t(0)
        _check(lib.psvt_batch_workspace_bytes(op, items, len(As), ctypes.byref(self.cfg), ctypes.byref(need)),
               "psvt_batch_workspace_bytes")
        dev = As[0].device
        self.ws = torch.empty(max(int(need.value), 256), dtype=torch.uint8, device=dev)
        self.device = dev
        h = ctypes.c_void_p()
        with torch.cuda.device(dev):
            _check(lib.psvt_batch_create(op, items, len(As), self.ws.data_ptr(), int(need.value),
                                         ctypes.byref(self.cfg), ctypes.byref(h)), "psvt_batch_create")
        self._h = h

    def run(self):
        torch = _torch()
        with torch.cuda.device(self.device):
            _check(load().psvt_batch_run(self._h, _stream_ptr(self.As[0])), "psvt_batch_run")
        return self.Ys

    def run_graph(self):
        torch = _torch()
        with torch.cuda.device(self.device):
            _check(load().psvt_batch_run_graph(self._h, _stream_ptr(self.As[0])), "psvt_batch_run_graph")
        return self.Ys

    def stats(self):
        n = ctypes.c_int32(0)
        f = ctypes.c_double(0.0)
        _check(load().psvt_batch_stats(self._h, ctypes.byref(n), ctypes.byref(f)), "psvt_batch_stats")
        return int(n.value), float(f.value)

    def close(self):
        if getattr(self, "_h", None):
            load().psvt_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Serving loop (C ABI psvt_server_*): admission by an HBM budget,
    iteration-level continuous batching, latency statistics."""

    def __init__(self, budget_bytes: int, max_slots: int = 64, iters: int = 20, n_fp8: int = 0, n_bf16: int = 0,
                 flags: int = 0, fake: bool = False, side: int = SIDE_AUTO, cohort: bool = True):
        self.cfg, self._keep = make_config(iters, n_fp8, n_bf16, side, None, flags)
        h = ctypes.c_void_p()
        sflags = (SERVER_FAKE if fake else 0) | (0 if cohort else SERVER_EAGER)
        _check(load().psvt_server_create(int(budget_bytes), int(max_slots), ctypes.byref(self.cfg),
                                         sflags, ctypes.byref(h)), "psvt_server_create")
        self._h = h
        self._pinned = {}

    def submit_ptr(self, A_ptr: int, Y_ptr: int, m: int, n: int, lda: int, ldy: int, tau: float,
                   op: int = OP_SVT, stream=None, warm_pi: int = None, pi_out: int = None, ld_pi: int = 0) -> int:
        """Raw submit; ``stream``: the hipStream_t handle (int) whose pending
        work the request must follow (None = the default stream)."""
        item = BatchItem(A_ptr, Y_ptr, m, n, lda, ldy, float(tau), warm_pi, pi_out, int(ld_pi))
        t = ctypes.c_uint64(0)
        _check(load().psvt_server_submit(self._h, op, ctypes.byref(item), ctypes.c_void_p(stream),
                                         ctypes.byref(t)), "psvt_server_submit")
        return int(t.value)

    def submit(self, A, tau: float, out=None, op: int = OP_SVT, warm_pi=None, pi_out=None):
        """Submit A (float32 GPU tensor); returns (ticket, Y).  The request
        is ordered after the work already queued on A's current stream (which
        may still be producing A).  ``warm_pi`` / ``pi_out``: warm start of
        the sign iteration from a previous request's (I + S)/2 and this
        request's (s x s float32 GPU tensors, s the Gram side).  Keep the
        tensors alive until the ticket is done."""
        torch = _torch()
        _check_input(A)
        Y = _output(out, tuple(A.shape), A.device)
        if A.numel() == 0:
            raise ValueError("empty request")
        ld_pi = 0
        for t_ in (warm_pi, pi_out):
            if t_ is not None:
                _check_pi(t_)
                ld_pi = _ld(t_)
        t = self.submit_ptr(A.data_ptr(), Y.data_ptr(), A.shape[0], A.shape[1], _ld(A), _ld(Y), tau, op,
                            stream=torch.cuda.current_stream(A.device).cuda_stream,
                            warm_pi=warm_pi.data_ptr() if warm_pi is not None else None,
                            pi_out=pi_out.data_ptr() if pi_out is not None else None, ld_pi=ld_pi)
        self._pinned[t] = (A, Y, warm_pi, pi_out)
        return t, Y

    def poll(self, ticket: int) -> int:
        st = ctypes.c_int32(0)
        _check(load().psvt_server_poll(self._h, ticket, ctypes.byref(st)), "psvt_server_poll")
        if st.value in (RQ_DONE, RQ_FAILED):
            self._pinned.pop(ticket, None)
        return int(st.value)

    def wait(self, ticket: int, timeout: float = 60.0) -> int:
        st = ctypes.c_int32(0)
        _check(load().psvt_server_wait(self._h, ticket, float(timeout), ctypes.byref(st)), "psvt_server_wait")
        if st.value in (RQ_DONE, RQ_FAILED):
            self._pinned.pop(ticket, None)
        return int(st.value)

    def drain(self, timeout: float = 600.0):
        _check(load().psvt_server_drain(self._h, float(timeout)), "psvt_server_drain")
        self._pinned.clear()

    def set_timeout(self, seconds: float):
        """Requests not done ``seconds`` after submit fail (0 = none)."""
        _check(load().psvt_server_set_timeout(self._h, float(seconds)), "psvt_server_set_timeout")

    def inject_fault(self, kind: int, n: int):
        """Fake servers: FAULT_TICK fails tick n, FAULT_PLAN the n-th plan,
        FAULT_STALL (n != 0) stops fake ticks from completing."""
        _check(load().psvt_server_inject_fault(self._h, int(kind), int(n)), "psvt_server_inject_fault")

    def stats(self) -> dict:
        c = ServerCounters()
        _check(load().psvt_server_stats(self._h, ctypes.byref(c)), "psvt_server_stats")
        return {k: getattr(c, k) for k, _ in ServerCounters._fields_}

    def close(self):
        if getattr(self, "_h", None):
            load().psvt_server_destroy(self._h)
            self._h = None
            self._pinned.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def trace_begin():
    """Start per-launch event tracing on this thread."""
    _check(load().psvt_trace_begin(), "psvt_trace_begin")


def trace_end(max_entries: int = 64):
    """Stop tracing; returns [{name, launches, total_ms, flops, bytes}] by time."""
    rows = (TraceStat * max_entries)()
    n = ctypes.c_int(0)
    _check(load().psvt_trace_end(rows, max_entries, ctypes.byref(n)), "psvt_trace_end")
    return [dict(name=r.name.decode(), launches=int(r.launches), total_ms=float(r.total_ms), flops=float(r.flops),
                 bytes=float(r.bytes)) for r in rows[:n.value]]


def force_tile(tile: int):
    """Force a tile configuration id (0 = automatic) on this thread."""
    _check(load().psvt_tune_force_tile(int(tile)), "psvt_tune_force_tile")


def persistent_tiles(on: bool):
    """Single calls on this thread pick tiles as the persistent batched
    executor does (for bitwise comparisons with it)."""
    _check(load().psvt_tune_persistent_tiles(1 if on else 0), "psvt_tune_persistent_tiles")


def spin_limit(polls: int):
    """This thread's bound on one dependency wait of the persistent executor
    (polls; 0 = abort on any wait not already satisfied)."""
    _check(load().psvt_tune_spin_limit(int(polls)), "psvt_tune_spin_limit")


def pick_tile(M: int, N: int, K: int, sym: bool = False, dtype: int = 0) -> int:
    rc = load().psvt_tune_pick(int(dtype), M, N, K, 1 if sym else 0)
    if rc < 0:
        _check(rc, "psvt_tune_pick")
    return rc


def version() -> str:
    return load().psvt_version().decode()
