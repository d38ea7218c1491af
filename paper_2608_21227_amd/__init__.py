"""svdv: singular values of dense matrices on an AMD Instinct MI355X.

Thin ctypes binding over the C-ABI library ``libsvdv.so`` (declared in
``include/svdv.h``).  This module only marshals arguments: every step of the
computation runs in the library's HIP kernels.  PyTorch supplies device memory
and the current stream.  If the library has not been built the functions raise
``RuntimeError`` -- there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import asdict, dataclass

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsvdv.so")

SVDV_F32, SVDV_F64 = 0, 1
STATUS = {0: "SVDV_OK", -1: "SVDV_ERR_INVALID_ARG", -2: "SVDV_ERR_UNSUPPORTED", -3: "SVDV_ERR_NO_MEMORY",
          -4: "SVDV_ERR_HIP"}

# Every symbol include/svdv.h declares (checked by the CPU test-suite).
EXPORTS = ["svd_values", "svd_values_ex", "svd_values_noalloc", "svdv_noalloc_capacity", "svd_values_batched",
           "svdv_default_config", "svdv_check_config", "svdv_stage_band", "svdv_stage_bidiag", "svdv_stage_values", "svdv_apply_qt", "svdv_status_string",
           "svdv_last_error", "svdv_release", "svdv_timing", "svdv_last_timing",
           "svdv_last_kernel_stats", "svdv_mlp_work_size", "svdv_mlp_forward", "svdv_mlp_gradient",
           "svdv_mlp_adam_step"]


class SvdvError(RuntimeError):
    def __init__(self, status: int, detail: str):
        super().__init__(f"{STATUS.get(status, status)}: {detail}")
        self.status = status


class Unsupported(SvdvError):
    """The configuration is outside the compiled set (the auto-tuner skips it)."""


class _Config(ctypes.Structure):
    _fields_ = [("tile", ctypes.c_int32), ("threads", ctypes.c_int32), ("inner_block", ctypes.c_int32),
                ("sweep_width", ctypes.c_int32), ("update_precision", ctypes.c_int32)]


@dataclass(frozen=True)
class Config:
    tile: int = 32
    threads: int = 256
    inner_block: int = 2
    sweep_width: int = 4
    update_precision: int = 0

    def _c(self) -> _Config:
        return _Config(self.tile, self.threads, self.inner_block, self.sweep_width, self.update_precision)

    def as_dict(self):
        return asdict(self)


_lib = None


def lib():
    """Load libsvdv.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2608_21227_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        cfgp = ctypes.POINTER(_Config)
        sig = {
            "svd_values": [vp, i64, i64, i64, i32, vp, vp],
            "svd_values_ex": [vp, i64, i64, i64, i32, vp, vp, cfgp],
            "svd_values_noalloc": [vp, i64, i64, i64, i32, vp, vp, cfgp],
            "svd_values_batched": [vp, vp, vp, vp, i64, i32, vp, vp, vp, cfgp],
            "svdv_default_config": [i64, i64, i32, cfgp],
            "svdv_check_config": [i64, i64, i32, cfgp],
            "svdv_stage_band": [vp, i64, i64, i64, i32, vp, i64, vp, cfgp],
            "svdv_stage_bidiag": [vp, i64, i64, i64, vp, vp, vp, cfgp],
            "svdv_stage_values": [vp, vp, i64, i32, vp, vp],
            "svdv_apply_qt": [vp, i64, vp, i64, vp, i64, i64, i64, i64, i32, i32, vp, cfgp],
            "svdv_release": [],
            "svdv_timing": [ctypes.c_int],
            "svdv_last_timing": [ctypes.POINTER(ctypes.c_double), ctypes.c_int],
            "svdv_last_kernel_stats": [ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.c_int],
            "svdv_mlp_forward": [vp, vp, i64, vp, vp],
            "svdv_mlp_gradient": [vp, vp, vp, i64, vp, vp, vp, vp],
            "svdv_mlp_adam_step": [vp, vp, vp, vp, i64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                   ctypes.c_float, vp],
        }
        for name, args in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.svdv_noalloc_capacity.argtypes = []
        L.svdv_noalloc_capacity.restype = i64
        L.svdv_mlp_work_size.argtypes = [i64]
        L.svdv_mlp_work_size.restype = i64
        L.svdv_status_string.argtypes = [ctypes.c_int]
        L.svdv_status_string.restype = ctypes.c_char_p
        L.svdv_last_error.argtypes = []
        L.svdv_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(rc: int):
    if rc != 0:
        detail = lib().svdv_last_error().decode(errors="replace")
        if rc == -2:
            raise Unsupported(rc, detail)
        raise SvdvError(rc, detail)


def _cfg_ptr(cfg):
    if cfg is None:
        return None
    if isinstance(cfg, dict):
        cfg = Config(**cfg)
    return ctypes.byref(cfg._c())


def _torch():
    import torch
    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float32:
        return SVDV_F32
    if t.dtype == torch.float64:
        return SVDV_F64
    raise TypeError(f"unsupported dtype {t.dtype} (float32 or float64)")


def _stream(device):
    torch = _torch()
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _on(device):
    """The tensor's device made current for the call (the library launches on the current device)."""
    return _torch().cuda.device(device)


def _need(t, name: str, dtype=None, dim=None, numel=None, device=None, dense=False):
    """Argument checks done before anything reaches the library, which receives plain
    pointers and cannot tell a short or mistyped buffer from a right one."""
    if not getattr(t, "is_cuda", False):
        raise ValueError(f"{name} must be a tensor on a GPU")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, not {t.dtype}")
    if dim is not None and t.dim() != dim:
        raise ValueError(f"{name} must be {dim}-D, not {t.dim()}-D")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} holds {t.numel()} elements, {numel} needed")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, the other arguments on {device}")
    if dense and not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _as_colmajor(a):
    """(ptr, m, n, lda) of a 2-D tensor as a column-major matrix with the same singular values."""
    m, n = a.shape
    if a.stride(0) == 1 and a.stride(1) >= max(1, m):
        return a, m, n, a.stride(1)
    a = a.contiguous()
    # row-major (m, n) == column-major (n, m) = A^T
    return a, n, m, max(1, n)


def default_config(m: int, n: int, dtype: str = "float32") -> Config:
    c = _Config()
    _check(lib().svdv_default_config(m, n, SVDV_F32 if dtype == "float32" else SVDV_F64, ctypes.byref(c)))
    return Config(c.tile, c.threads, c.inner_block, c.sweep_width, c.update_precision)


def check_config(m: int, n: int, dtype: str, cfg) -> bool:
    """True if cfg is runnable for (m, n, dtype); False if the library reports it unsupported."""
    rc = lib().svdv_check_config(m, n, SVDV_F32 if dtype == "float32" else SVDV_F64, _cfg_ptr(cfg))
    if rc == -2:
        return False
    _check(rc)
    return True


def svd_values(a, config=None, out=None):
    """Singular values (descending) of the 2-D CUDA tensor ``a`` (float32/float64)."""
    torch = _torch()
    _need(a, "a", dim=2)
    dt = _dtype_code(a)
    a2, m, n, lda = _as_colmajor(a)
    k = min(m, n)
    s = out if out is not None else torch.empty(k, dtype=a.dtype, device=a.device)
    _need(s, "out", dtype=a.dtype, numel=k, device=a.device, dense=True)
    with _on(a.device):
        _check(lib().svd_values_ex(ctypes.c_void_p(a2.data_ptr()), m, n, lda, dt, ctypes.c_void_p(s.data_ptr()),
                                   _stream(a.device), _cfg_ptr(config)))
    return s


def svd_values_noalloc(a, out, config=None):
    """svd_values through the allocation-free entry point: the library works in its
    fixed device array (no device allocation); ``out`` (min(m, n) values, a's dtype)
    is supplied by the caller."""
    _need(a, "a", dim=2)
    dt = _dtype_code(a)
    a2, m, n, lda = _as_colmajor(a)
    _need(out, "out", dtype=a.dtype, numel=min(m, n), device=a.device, dense=True)
    with _on(a.device):
        _check(lib().svd_values_noalloc(ctypes.c_void_p(a2.data_ptr()), m, n, lda, dt,
                                        ctypes.c_void_p(out.data_ptr()), _stream(a.device), _cfg_ptr(config)))
    return out


def svd_values_batched(mats, config=None, out=None):
    """Singular values of a list of 2-D CUDA tensors (same dtype, uneven sizes) in one call.

    Returns (packed values, offsets): matrix i's values are packed[offsets[i]:offsets[i]+min(m_i,n_i)].
    Passing the previous result as ``out`` keeps the output address, so a repeated call with the
    same shapes replays the captured graph without refreshing its pointer table."""
    torch = _torch()
    if not mats:
        return None, []
    dt = _dtype_code(mats[0])
    keep, ptrs, ms, ns, ldas, offs = [], [], [], [], [], []
    off = 0
    for i, a in enumerate(mats):
        _need(a, f"mats[{i}]", dtype=mats[0].dtype, dim=2, device=mats[0].device)
        a2, m, n, lda = _as_colmajor(a)
        keep.append(a2)
        ptrs.append(a2.data_ptr())
        ms.append(m)
        ns.append(n)
        ldas.append(lda)
        offs.append(off)
        off += min(m, n)
    s = out if out is not None else torch.empty(max(off, 1), dtype=mats[0].dtype, device=mats[0].device)
    _need(s, "out", dtype=mats[0].dtype, numel=off, device=mats[0].device, dense=True)
    B = len(mats)
    P = (ctypes.c_void_p * B)(*ptrs)
    I64 = ctypes.c_int64 * B
    with _on(mats[0].device):
        _check(lib().svd_values_batched(ctypes.cast(P, ctypes.c_void_p), ctypes.cast(I64(*ms), ctypes.c_void_p),
                                        ctypes.cast(I64(*ns), ctypes.c_void_p),
                                        ctypes.cast(I64(*ldas), ctypes.c_void_p), B, dt,
                                        ctypes.c_void_p(s.data_ptr()), ctypes.cast(I64(*offs), ctypes.c_void_p),
                                        _stream(mats[0].device), _cfg_ptr(config)))
    return s, offs


def stage_band(a, config=None):
    """Stage 1 only: the (k, tile+1) float64 band, row i = B(i, i..i+tile), k = min(m, n)."""
    torch = _torch()
    _need(a, "a", dim=2)
    dt = _dtype_code(a)
    cfg = config if config is not None else default_config(*a.shape, "float32" if dt == SVDV_F32 else "float64")
    if isinstance(cfg, dict):
        cfg = Config(**cfg)
    a2, m, n, lda = _as_colmajor(a)
    k = min(m, n)
    band = torch.zeros((k, cfg.tile + 1), dtype=torch.float64, device=a.device)
    with _on(a.device):
        _check(lib().svdv_stage_band(ctypes.c_void_p(a2.data_ptr()), m, n, lda, dt,
                                     ctypes.c_void_p(band.data_ptr()), cfg.tile + 1, _stream(a.device),
                                     _cfg_ptr(cfg)))
    return band


def stage_bidiag(band, b: int, config=None):
    """Stage 2 only: (d, e) of the bidiagonal from a (n, >= b+1) float64 band tensor."""
    torch = _torch()
    _need(band, "band", dtype=torch.float64, dim=2)
    if band.shape[1] < b + 1:
        raise ValueError(f"band has {band.shape[1]} columns, b + 1 = {b + 1} needed")
    n = band.shape[0]
    band = band.contiguous()
    d = torch.empty(n, dtype=torch.float64, device=band.device)
    e = torch.empty(max(n - 1, 1), dtype=torch.float64, device=band.device)
    with _on(band.device):
        _check(lib().svdv_stage_bidiag(ctypes.c_void_p(band.data_ptr()), n, b, band.shape[1],
                                       ctypes.c_void_p(d.data_ptr()), ctypes.c_void_p(e.data_ptr()),
                                       _stream(band.device), _cfg_ptr(config)))
    return d, e[: max(n - 1, 0)]


def stage_values(d, e, out_dtype=None):
    """Stage 3 only: singular values (descending) of the upper bidiagonal (d, e) (float64 tensors)."""
    torch = _torch()
    out_dtype = out_dtype or torch.float64
    if out_dtype not in (torch.float32, torch.float64):
        raise TypeError(f"out_dtype must be float32 or float64, not {out_dtype}")
    _need(d, "d", dtype=torch.float64, dim=1)
    n = d.shape[0]
    _need(e, "e", dtype=torch.float64, dim=1, numel=max(n - 1, 0), device=d.device)
    s = torch.empty(n, dtype=out_dtype, device=d.device)
    d2 = d.contiguous()
    e2 = e.contiguous() if e.numel() else d2
    with _on(d.device):
        _check(lib().svdv_stage_values(ctypes.c_void_p(d2.data_ptr()), ctypes.c_void_p(e2.data_ptr()), n,
                                       SVDV_F32 if out_dtype == torch.float32 else SVDV_F64,
                                       ctypes.c_void_p(s.data_ptr()), _stream(d.device)))
    return s


def apply_qt(V, T, C, side: int = 0, config=None):
    """The stage-1 trailing-update kernel alone: C <- (I - V T V^T)^T C (side 0) or C (I - V T V^T) (side 1).

    V, T, C are column-major CUDA tensors given as torch views of their transposes is NOT assumed:
    pass tensors whose .T is contiguous (i.e. Fortran order), e.g. ``x.t().contiguous().t()``."""
    dt = _dtype_code(C)

    def ld(name, x):  # leading dimension of a column-major (Fortran-order) 2-D tensor
        _need(x, name, dtype=C.dtype, dim=2, device=C.device)
        if x.shape[1] <= 1:
            return max(1, x.shape[0])
        if (x.stride(0) != 1 and x.shape[0] > 1) or x.stride(1) < x.shape[0]:
            raise ValueError(f"apply_qt expects column-major (Fortran-order) tensors; {name} is not")
        return x.stride(1)

    ldv, ldt, ldc = ld("V", V), ld("T", T), ld("C", C)
    h, w = C.shape
    k = V.shape[1]
    if V.shape[0] != (h if side == 0 else w):
        raise ValueError(f"V has {V.shape[0]} rows, the reflector length is {h if side == 0 else w}")
    if T.shape[0] < k or T.shape[1] < k:
        raise ValueError(f"T is {tuple(T.shape)}, at least {k} x {k} needed")
    with _on(C.device):
        _check(lib().svdv_apply_qt(ctypes.c_void_p(V.data_ptr()), ldv, ctypes.c_void_p(T.data_ptr()), ldt,
                                   ctypes.c_void_p(C.data_ptr()), ldc, h, w, k, dt, side, _stream(C.device),
                                   _cfg_ptr(config)))
    return C


STAGES = ["stage_in", "stage1", "band_pack", "chase", "bisect", "total", "chase_kernel"]


def set_timing(enable, kernels: bool = False):
    """Record per-stage HIP events in later calls on this thread (instrumentation);
    with kernels=True also bracket every stage-1 launch (see last_kernel_stats)."""
    _check(lib().svdv_timing((2 if kernels else 1) if enable else 0))


def last_timing() -> dict:
    """Per-stage milliseconds of the last timed call (waits for its events)."""
    buf = (ctypes.c_double * 7)()
    k = lib().svdv_last_timing(buf, 7)
    if k < 0:
        _check(k)
    return {name: buf[i] for i, name in enumerate(STAGES[:k])}


def last_kernel_stats(kind: str) -> dict:
    """Launch count, summed event time (ms) and algorithmic flops / bytes of one
    kernel class ("update" or "panel") in the last timed call."""
    buf = (ctypes.c_double * 4)()
    _check(min(0, lib().svdv_last_kernel_stats({"update": 0, "panel": 1}[kind], buf, 4)))
    return {"launches": int(buf[0]), "ms": buf[1], "flops": buf[2], "bytes": buf[3]}


def release():
    _check(lib().svdv_release())


# --------------------------------------------------------------------------- learned cost model kernels

MLP_IN, MLP_HIDDEN = 6, 64
MLP_NPARAM = MLP_IN * MLP_HIDDEN + MLP_HIDDEN + MLP_HIDDEN * MLP_HIDDEN + MLP_HIDDEN + MLP_HIDDEN + 1


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def mlp_forward(params, X, out=None):
    """Model outputs for the rows of X (float32 CUDA tensors; params has MLP_NPARAM entries)."""
    torch = _torch()
    _mlp_args(params, X)
    y = out if out is not None else torch.empty(X.shape[0], dtype=torch.float32, device=X.device)
    _need(y, "out", dtype=torch.float32, numel=X.shape[0], device=X.device, dense=True)
    with _on(X.device):
        _check(lib().svdv_mlp_forward(_ptr(params), _ptr(X), X.shape[0], _ptr(y), _stream(X.device)))
    return y


def _mlp_args(params, X):
    torch = _torch()
    _need(params, "params", dtype=torch.float32, numel=MLP_NPARAM, dense=True)
    _need(X, "X", dtype=torch.float32, dim=2, device=params.device, dense=True)
    if X.shape[1] != MLP_IN:
        raise ValueError(f"X must have {MLP_IN} feature columns, not {X.shape[1]}")


def mlp_work(n: int, device):
    torch = _torch()
    return torch.empty(max(1, int(lib().svdv_mlp_work_size(n))), dtype=torch.float32, device=device)


def mlp_gradient(params, X, t, grad, loss=None, work=None):
    """grad <- d/dparams of mean((model(X) - t)^2); loss (1-element tensor) receives the loss."""
    torch = _torch()
    _mlp_args(params, X)
    n = X.shape[0]
    _need(t, "t", dtype=torch.float32, numel=n, device=X.device, dense=True)
    _need(grad, "grad", dtype=torch.float32, numel=MLP_NPARAM, device=X.device, dense=True)
    if loss is not None:
        _need(loss, "loss", dtype=torch.float32, numel=1, device=X.device, dense=True)
    work = work if work is not None else mlp_work(n, X.device)
    _need(work, "work", dtype=torch.float32, numel=int(lib().svdv_mlp_work_size(n)), device=X.device, dense=True)
    with _on(X.device):
        _check(lib().svdv_mlp_gradient(_ptr(params), _ptr(X), _ptr(t), n, _ptr(grad),
                                       _ptr(loss) if loss is not None else None, _ptr(work), _stream(X.device)))
    return grad


def mlp_adam_step(params, grad, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    torch = _torch()
    for name, x in (("params", params), ("grad", grad), ("m", m), ("v", v)):
        _need(x, name, dtype=torch.float32, numel=MLP_NPARAM, device=params.device, dense=True)
    with _on(params.device):
        _check(lib().svdv_mlp_adam_step(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), step, lr, beta1, beta2, eps,
                                        _stream(params.device)))
