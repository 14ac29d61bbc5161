"""Python binding of libspin, the gfx950 Strassen block-recursive inverter.

Argument marshalling only: every step of an inversion runs in the HIP
library (include/spin.h).  Names follow the C ABI without the ``spin_``
prefix.  Tensors are torch tensors on the GPU; the library reads them through
their data pointers and strides:

* a column-major (Fortran-ordered) matrix is passed as is;
* a row-major (C-contiguous) matrix is passed unchanged as well: the library
  then inverts A^T in column-major order, which is A^-1 in row-major order.

The library must be built (``python -m paper_1801_04723_amd.build``);
importing this package without it raises instead of falling back to anything
else.
"""
from __future__ import annotations

import ctypes
import os
import re

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspin.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "spin.h")

FP64 = 0
MIXED_FP32 = 1
MIXED_BF16 = 2
MIXED_BF16X3 = 3
# Flag OR-ed into a mode for invert_mixed, invert_batch, Server and
# server_request_bytes: the recursion runs the symmetric schedule of invert_spd
# (exactly symmetric inputs only).
SYMMETRIC = 16
# Flag OR-ed into a mixed mode of invert_mixed: the refinement's products run
# on INT8 matrix cores (gemm_int8).
REFINE_INT8 = 32
MODES = {"fp64": FP64, "fp32": MIXED_FP32, "mixed_fp32": MIXED_FP32,
         "bf16": MIXED_BF16, "mixed_bf16": MIXED_BF16,
         "bf16x3": MIXED_BF16X3, "mixed_bf16x3": MIXED_BF16X3,
         "fp64_sym": FP64 | SYMMETRIC, "fp32_sym": MIXED_FP32 | SYMMETRIC,
         "bf16_sym": MIXED_BF16 | SYMMETRIC, "bf16x3_sym": MIXED_BF16X3 | SYMMETRIC,
         "fp32_int8": MIXED_FP32 | REFINE_INT8, "bf16x3_int8": MIXED_BF16X3 | REFINE_INT8,
         "bf16_int8": MIXED_BF16 | REFINE_INT8}
NS_DIVERGED = -100
MAX_LEAF = 2048

_i64 = ctypes.c_int64
_vp = ctypes.c_void_p


class Report(ctypes.Structure):
    _fields_ = [
        ("rho_before", ctypes.c_double),
        ("rho_after", ctypes.c_double),
        ("r0_fro", ctypes.c_double),
        ("r_fro", ctypes.c_double * 8),
        ("steps", ctypes.c_int),
        ("status", ctypes.c_int),
    ]

    def as_dict(self) -> dict:
        return {
            "rho_before": self.rho_before,
            "rho_after": self.rho_after,
            "r0_fro": self.r0_fro,
            "r_fro": [self.r_fro[i] for i in range(self.steps)],
            "steps": self.steps,
            "status": self.status,
        }


class PlanOp(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int), ("count", ctypes.c_int), ("level", ctypes.c_int),
        ("flags", ctypes.c_int),
        ("m", _i64 * 2), ("n", _i64 * 2), ("k", _i64 * 2),
        ("a_buf", ctypes.c_int * 2), ("b_buf", ctypes.c_int * 2),
        ("c_buf", ctypes.c_int * 2), ("d_buf", ctypes.c_int * 2),
        ("a_off", _i64 * 2), ("b_off", _i64 * 2), ("c_off", _i64 * 2), ("d_off", _i64 * 2),
        ("a_ld", _i64 * 2), ("b_ld", _i64 * 2), ("c_ld", _i64 * 2), ("d_ld", _i64 * 2),
        ("alpha", ctypes.c_double * 2), ("beta", ctypes.c_double * 2),
        ("leaf_order", _i64), ("col0", _i64),
    ]


class TraceRec(ctypes.Structure):
    _fields_ = [
        ("kernel", ctypes.c_char * 48),
        ("ms", ctypes.c_double),
        ("flops", ctypes.c_double),
        ("bytes", ctypes.c_double),
        ("level", ctypes.c_int),
    ]


class SpinError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} ({code})" if what else f"{strerror(code)} ({code})")


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libspin (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1801_04723_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        L.spin_invert.argtypes = [_vp, _i64, _i64, _vp, _i64, _i64, _vp]
        L.spin_invert.restype = ctypes.c_int
        L.spin_invert_mixed.argtypes = [_vp, _i64, _i64, _vp, _i64, _i64, ctypes.c_int, ctypes.c_int,
                                        ctypes.POINTER(Report), _vp]
        L.spin_invert_mixed.restype = ctypes.c_int
        L.spin_gemm.argtypes = [ctypes.c_int, _i64, _i64, _i64, ctypes.c_double, _vp, _i64, _vp, _i64,
                                ctypes.c_double, _vp, _i64, _vp, _i64, ctypes.c_int, _vp]
        L.spin_gemm.restype = ctypes.c_int
        L.spin_gemm_int8.argtypes = [_i64, _i64, _i64, _vp, _i64, _vp, _i64, ctypes.c_int, _vp, _i64, _vp,
                                     _i64, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp]
        L.spin_gemm_int8.restype = ctypes.c_int
        L.spin_info.argtypes = [_vp]
        L.spin_info.restype = ctypes.c_int
        L.spin_residual.argtypes = [_vp, _i64, _i64, _vp, _i64, ctypes.POINTER(ctypes.c_double), _vp]
        L.spin_residual.restype = ctypes.c_int
        L.spin_workspace_bytes.argtypes = [_i64, _i64, ctypes.c_int]
        L.spin_workspace_bytes.restype = ctypes.c_size_t
        L.spin_strerror.argtypes = [ctypes.c_int]
        L.spin_strerror.restype = ctypes.c_char_p
        L.spin_release.argtypes = []
        L.spin_release.restype = None
        L.spin_plan_describe.argtypes = [_i64, _i64, _i64, _i64, ctypes.POINTER(PlanOp), _i64,
                                         ctypes.POINTER(ctypes.c_double)]
        L.spin_plan_describe.restype = _i64
        L.spin_plan_describe_spd.argtypes = L.spin_plan_describe.argtypes
        L.spin_plan_describe_spd.restype = _i64
        L.spin_plan_describe_lu.argtypes = L.spin_plan_describe.argtypes
        L.spin_plan_describe_lu.restype = _i64
        L.spin_plan_ws_elems_lu.argtypes = [_i64, _i64]
        L.spin_plan_ws_elems_lu.restype = _i64
        L.spin_invert_noalloc.argtypes = [_vp, _i64, _i64, _vp, _i64, _i64, _vp, _vp]
        L.spin_invert_noalloc.restype = ctypes.c_int
        L.spin_invert_lu.argtypes = L.spin_invert.argtypes
        L.spin_invert_lu.restype = ctypes.c_int
        L.spin_invert_spd.argtypes = L.spin_invert.argtypes
        L.spin_invert_spd.restype = ctypes.c_int
        L.spin_plan_ws_elems.argtypes = [_i64, _i64]
        L.spin_plan_ws_elems.restype = _i64
        L.spin_trace_enable.argtypes = [ctypes.c_int]
        L.spin_trace_enable.restype = ctypes.c_int
        L.spin_trace_collect.argtypes = [ctypes.POINTER(TraceRec), _i64]
        L.spin_trace_collect.restype = _i64
        P64 = ctypes.POINTER(_i64)
        L.spin_invert_batch.argtypes = [_i64, ctypes.POINTER(_vp), P64, P64, ctypes.POINTER(_vp), P64,
                                        ctypes.POINTER(ctypes.c_int), _i64, ctypes.c_int,
                                        ctypes.POINTER(ctypes.c_int), _vp]
        L.spin_invert_batch.restype = ctypes.c_int
        L.spin_server_create.argtypes = [ctypes.c_size_t, ctypes.c_int, _i64, ctypes.c_int]
        L.spin_server_create.restype = _vp
        L.spin_server_destroy.argtypes = [_vp]
        L.spin_server_destroy.restype = None
        L.spin_server_submit.argtypes = [_vp, _vp, _i64, _i64, _vp, _i64, ctypes.c_int, _i64]
        L.spin_server_submit.restype = ctypes.c_int
        L.spin_server_admit.argtypes = [_vp]
        L.spin_server_admit.restype = ctypes.c_int
        L.spin_server_tick.argtypes = [_vp, _vp]
        L.spin_server_tick.restype = ctypes.c_int
        L.spin_server_poll.argtypes = [_vp, P64, ctypes.POINTER(ctypes.c_int), _i64]
        L.spin_server_poll.restype = _i64
        L.spin_server_stats.argtypes = [_vp, P64, P64, ctypes.POINTER(ctypes.c_size_t)]
        L.spin_server_stats.restype = ctypes.c_int
        L.spin_server_request_bytes.argtypes = [_i64, _i64, ctypes.c_int]
        L.spin_server_request_bytes.restype = ctypes.c_size_t
        _lib = L
    return _lib


def header_functions() -> list[str]:
    """Names of every function the public header declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(spin_[a-z0-9_]+)\s*\(", text)))


# ----------------------------------------------------------------- host-only
def strerror(code: int) -> str:
    return lib().spin_strerror(int(code)).decode()


def workspace_bytes(n: int, leaf: int, mode: int | str = FP64) -> int:
    return int(lib().spin_workspace_bytes(int(n), int(leaf), _mode(mode)))


def plan_ws_elems(n: int, leaf: int) -> int:
    return int(lib().spin_plan_ws_elems(int(n), int(leaf)))


def plan_ws_elems_lu(n: int, leaf: int) -> int:
    return int(lib().spin_plan_ws_elems_lu(int(n), int(leaf)))


def plan_describe(n: int, leaf: int, lda: int | None = None, ldx: int | None = None,
                  spd: bool = False, lu: bool = False):
    """The recursion schedule (of spin_invert_spd when spd=True, of
    spin_invert_lu when lu=True) as a list of dicts, plus its flop count."""
    lda = n if lda is None else lda
    ldx = n if ldx is None else ldx
    L = lib()
    fn = L.spin_plan_describe_lu if lu else L.spin_plan_describe_spd if spd else L.spin_plan_describe
    fl = ctypes.c_double(0)
    cnt = fn(n, lda, ldx, leaf, None, 0, ctypes.byref(fl))
    if cnt < 0:
        raise SpinError(int(cnt), "spin_plan_describe")
    arr = (PlanOp * max(int(cnt), 1))()
    fn(n, lda, ldx, leaf, arr, cnt, ctypes.byref(fl))
    ops = []
    for o in arr[: int(cnt)]:
        if o.kind == 0:
            prods = []
            for q in range(o.count):
                prods.append(dict(m=o.m[q], n=o.n[q], k=o.k[q],
                                  a=(o.a_buf[q], o.a_off[q], o.a_ld[q]),
                                  b=(o.b_buf[q], o.b_off[q], o.b_ld[q]),
                                  c=(o.c_buf[q], o.c_off[q], o.c_ld[q]),
                                  d=(o.d_buf[q], o.d_off[q], o.d_ld[q]),
                                  alpha=o.alpha[q], beta=o.beta[q], lower=bool(o.flags >> q & 1)))
            ops.append(dict(kind="products", level=o.level, products=prods,
                            folds_next=bool(o.flags & 4)))
        elif o.kind == 4:
            ops.append(dict(kind="lu_leaf", level=o.level, L=o.leaf_order, col0=o.col0,
                            src=(o.a_buf[0], o.a_off[0], o.a_ld[0]),
                            li=(o.d_buf[0], o.d_off[0], o.d_ld[0]),
                            ui=(o.c_buf[0], o.c_off[0], o.c_ld[0])))
        elif o.kind == 5:
            ops.append(dict(kind="fill", level=o.level, m=o.m[0], n=o.n[0],
                            dst=(o.d_buf[0], o.d_off[0], o.d_ld[0])))
        elif o.kind == 3:
            ops.append(dict(kind="mirror", level=o.level, n=o.m[0],
                            dst=(o.d_buf[0], o.d_off[0], o.d_ld[0])))
        elif o.kind == 2:
            ops.append(dict(kind="transpose", level=o.level, m=o.m[0], n=o.n[0],
                            src=(o.a_buf[0], o.a_off[0], o.a_ld[0]),
                            dst=(o.d_buf[0], o.d_off[0], o.d_ld[0])))
        else:
            ops.append(dict(kind="leaf", level=o.level, L=o.leaf_order, col0=o.col0,
                            src=(o.a_buf[0], o.a_off[0], o.a_ld[0]),
                            dst=(o.d_buf[0], o.d_off[0], o.d_ld[0])))
    return ops, float(fl.value)


def _mode(mode) -> int:
    if isinstance(mode, str):
        if mode not in MODES:
            raise ValueError(f"unknown mode {mode!r}")
        return MODES[mode]
    return int(mode)


# ------------------------------------------------------------------ tensors
def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream))


def _layout(t):
    """(leading dimension, order) of a 2-D matrix view: 'F' column-major, 'C' row-major."""
    if t.dim() != 2:
        raise ValueError("expected a 2-D tensor")
    s0, s1 = t.stride()
    r, c = t.shape
    if s0 == 1 and (s1 >= max(r, 1) or c == 1):
        return s1 if c > 1 else max(r, 1), "F"
    if s1 == 1 and (s0 >= max(c, 1) or r == 1):
        return s0 if r > 1 else max(c, 1), "C"
    raise ValueError("matrix must be contiguous in one dimension")


def _empty_like_layout(a, order):
    import torch
    n = a.shape[0]
    if order == "F":
        return torch.empty((n, n), dtype=torch.float64, device=a.device).t().contiguous().t()
    return torch.empty((n, n), dtype=torch.float64, device=a.device)


def _check_square(a):
    import torch
    if a.dtype != torch.float64:
        raise TypeError("inversion input must be float64")
    if not a.is_cuda:
        raise ValueError("inversion input must be a GPU tensor")
    if a.shape[0] != a.shape[1]:
        raise ValueError("matrix must be square")


def invert(a, leaf: int, out=None, stream=None):
    """A^-1 by the FP64 Strassen recursion (asynchronous on `stream`)."""
    _check_square(a)
    lda, order = _layout(a)
    if out is None:
        out = _empty_like_layout(a, order)
    ldx, order_x = _layout(out)
    if order_x != order:
        raise ValueError("output must have the same memory order as the input")
    rc = lib().spin_invert(a.data_ptr(), a.shape[0], lda, out.data_ptr(), ldx, int(leaf), _stream(stream))
    if rc != 0:
        raise SpinError(rc, "spin_invert")
    return out


NOALLOC_SCRATCH_MB = 64  # SPIN_NOALLOC_SCRATCH_MB


def invert_noalloc(a, leaf: int, out, info=None, stream=None):
    """spin_invert_noalloc: spin_invert on the library's fixed scratch, with
    no device allocation by the library.  `out` (same layout as `a`) and the
    optional one-element int32 device tensor `info` are the caller's; the
    status lands in `info` in stream order.  Returns `out`."""
    _check_square(a)
    lda, order = _layout(a)
    ldx, order_x = _layout(out)
    if order != order_x:
        raise ValueError("output must have the same memory order as the input")
    if info is not None and (info.dtype.itemsize != 4 or info.numel() < 1):
        raise ValueError("info must hold at least one 32-bit integer")
    rc = lib().spin_invert_noalloc(a.data_ptr(), a.shape[0], lda, out.data_ptr(), ldx, int(leaf),
                                   None if info is None else info.data_ptr(), _stream(stream))
    if rc != 0:
        raise SpinError(rc, "spin_invert_noalloc")
    return out


def invert_spd(a, leaf: int, out=None, stream=None):
    """A^-1 for an exactly symmetric A by the four-product FP64 recursion
    (asynchronous on `stream`)."""
    _check_square(a)
    lda, order = _layout(a)
    if out is None:
        out = _empty_like_layout(a, order)
    ldx, order_x = _layout(out)
    if order_x != order:
        raise ValueError("output must have the same memory order as the input")
    rc = lib().spin_invert_spd(a.data_ptr(), a.shape[0], lda, out.data_ptr(), ldx, int(leaf),
                               _stream(stream))
    if rc != 0:
        raise SpinError(rc, "spin_invert_spd")
    return out


def invert_lu(a, leaf: int = 128, out=None, stream=None):
    """A^-1 through a block LU factorisation without pivoting (the paper's
    comparison method; leaf <= 128), asynchronous on `stream`."""
    _check_square(a)
    lda, order = _layout(a)
    if out is None:
        out = _empty_like_layout(a, order)
    ldx, order_x = _layout(out)
    if order_x != order:
        raise ValueError("output must have the same memory order as the input")
    rc = lib().spin_invert_lu(a.data_ptr(), a.shape[0], lda, out.data_ptr(), ldx, int(leaf),
                              _stream(stream))
    if rc != 0:
        raise SpinError(rc, "spin_invert_lu")
    return out


def invert_mixed(a, leaf: int, mode="fp32", ns_steps: int = 2, out=None, report: bool = False,
                 stream=None):
    """A^-1 with the block products in `mode` ("fp32", "bf16", "bf16x3"),
    FP64 leaves and `ns_steps` FP64 Newton steps.  With report=True the call
    waits and returns (X, report dict)."""
    _check_square(a)
    lda, order = _layout(a)
    if out is None:
        out = _empty_like_layout(a, order)
    ldx, order_x = _layout(out)
    if order_x != order:
        raise ValueError("output must have the same memory order as the input")
    rep = Report() if report else None
    rc = lib().spin_invert_mixed(a.data_ptr(), a.shape[0], lda, out.data_ptr(), ldx, int(leaf),
                                 _mode(mode), int(ns_steps), ctypes.byref(rep) if rep else None,
                                 _stream(stream))
    if rc != 0:
        raise SpinError(rc, "spin_invert_mixed")
    return (out, rep.as_dict()) if report else out


def gemm_cm(m, n, k, alpha, A, lda, B, ldb, beta, C0, ldc, D, ldd, add_identity=False,
            dtype: int = FP64, stream=None):
    """Raw column-major block product on device pointers (ints) or tensors."""
    def ptr(x):
        if x is None:
            return None
        return x if isinstance(x, int) else x.data_ptr()
    rc = lib().spin_gemm(_mode(dtype), m, n, k, float(alpha), ptr(A), lda, ptr(B), ldb, float(beta),
                         ptr(C0), ldc, ptr(D), ldd, 1 if add_identity else 0, _stream(stream))
    if rc != 0:
        raise SpinError(rc, "spin_gemm")


def gemm_int8(m, n, k, A, lda, B, ldb, epilogue, C0, ldc, D, ldd, moduli: int = 14, beta_a: int = 0,
              beta_b: int = 0, stream=None):
    """spin_gemm_int8 on column-major float64 GPU buffers: D = A B (epilogue 0),
    I - A B (1) or C0 + A B (2), FP64-accurate on INT8 matrix cores."""
    ptr = lambda t: None if t is None else t.data_ptr()  # noqa: E731
    rc = lib().spin_gemm_int8(int(m), int(n), int(k), ptr(A), int(lda), ptr(B), int(ldb), int(epilogue),
                              ptr(C0), int(ldc), ptr(D), int(ldd), int(moduli), int(beta_a), int(beta_b),
                              _stream(stream))
    if rc != 0:
        raise SpinError(rc, "spin_gemm_int8")
    return D


def info(stream=None) -> int:
    """Numerical status of the last inversion on the stream (waits)."""
    return int(lib().spin_info(_stream(stream)))


def residual(a, x, stream=None) -> float:
    """rho = |A X - I|_F / (|A|_F |X|_F), computed by the library in FP64."""
    lda, oa = _layout(a)
    ldx, ox = _layout(x)
    if oa != ox:
        raise ValueError("A and X must share a memory order")
    rho = ctypes.c_double(0)
    if oa == "F":
        rc = lib().spin_residual(a.data_ptr(), a.shape[0], lda, x.data_ptr(), ldx, ctypes.byref(rho),
                                 _stream(stream))
    else:
        # row-major buffers read column-major are A^T and X^T, and
        # X^T A^T - I = (A X - I)^T has the same Frobenius norm as A X - I.
        rc = lib().spin_residual(x.data_ptr(), x.shape[0], ldx, a.data_ptr(), lda, ctypes.byref(rho),
                                 _stream(stream))
    if rc != 0:
        raise SpinError(rc, "spin_residual")
    return float(rho.value)


def release() -> None:
    lib().spin_release()


def trace_enable(on: bool = True) -> None:
    lib().spin_trace_enable(1 if on else 0)


def trace_collect() -> list[dict]:
    L = lib()
    arr = (TraceRec * 65536)()
    cnt = L.spin_trace_collect(arr, 65536)
    return [dict(kernel=r.kernel.decode(), ms=r.ms, flops=r.flops, bytes=r.bytes, level=r.level)
            for r in arr[: min(int(cnt), 65536)]]


# ------------------------------------------------------------ batch / server
def invert_batch(mats, leaf: int, modes=None, ns_steps: int = 2, outs=None, stream=None):
    """Inverts a list of square float64 GPU matrices with cross-request
    batching (spin_invert_batch); waits.  Returns (list of inverses, infos)."""
    count = len(mats)
    modes = [FP64] * count if modes is None else [_mode(m) for m in modes]
    if outs is None:
        outs = [_empty_like_layout(a, _layout(a)[1]) for a in mats]
    ptr_a = (_vp * count)(*[a.data_ptr() for a in mats])
    ptr_x = (_vp * count)(*[x.data_ptr() for x in outs])
    ns = (_i64 * count)(*[a.shape[0] for a in mats])
    lda = (_i64 * count)(*[_layout(a)[0] for a in mats])
    ldx = (_i64 * count)(*[_layout(x)[0] for x in outs])
    md = (ctypes.c_int * count)(*modes)
    info = (ctypes.c_int * count)()
    for a, x in zip(mats, outs):
        _check_square(a)
        if _layout(a)[1] != _layout(x)[1]:
            raise ValueError("output must have the same memory order as the input")
    rc = lib().spin_invert_batch(count, ptr_a, ns, lda, ptr_x, ldx, md, int(leaf), int(ns_steps),
                                 info, _stream(stream))
    if rc != 0:
        raise SpinError(rc, "spin_invert_batch")
    return outs, [int(v) for v in info]


def server_request_bytes(n: int, leaf: int, mode=FP64) -> int:
    return int(lib().spin_server_request_bytes(int(n), int(leaf), _mode(mode)))


class Server:
    """Continuous-batching server over the C ABI (one host thread).

    submit() queues a request (A and its output stay referenced until the
    request is reported by poll()); tick() admits what fits and launches one
    step of every admitted request; poll() returns finished (tag, status)."""

    def __init__(self, pool_bytes: int, max_active: int, leaf: int, ns_steps: int = 2):
        self._h = lib().spin_server_create(int(pool_bytes), int(max_active), int(leaf), int(ns_steps))
        if not self._h:
            raise ValueError("invalid server parameters")
        self._keep = {}

    def submit(self, a, out, mode=FP64, tag: int = 0) -> None:
        lda, oa = _layout(a)
        ldx, ox = _layout(out)
        if oa != ox:
            raise ValueError("output must have the same memory order as the input")
        rc = lib().spin_server_submit(self._h, a.data_ptr(), a.shape[0], lda, out.data_ptr(), ldx,
                                      _mode(mode), int(tag))
        if rc != 0:
            raise SpinError(rc, "spin_server_submit")
        self._keep[int(tag)] = (a, out)

    def admit(self) -> int:
        return int(lib().spin_server_admit(self._h))

    def tick(self, stream=None) -> int:
        rc = lib().spin_server_tick(self._h, _stream(stream))
        if rc < 0:
            raise SpinError(rc, "spin_server_tick")
        return rc

    def poll(self, cap: int = 4096):
        tags = (_i64 * cap)()
        info = (ctypes.c_int * cap)()
        cnt = lib().spin_server_poll(self._h, tags, info, cap)
        if cnt < 0:
            raise SpinError(int(cnt), "spin_server_poll")
        out = [(int(tags[i]), int(info[i])) for i in range(cnt)]
        for t, _ in out:
            self._keep.pop(t, None)
        return out

    def stats(self):
        q, a = _i64(0), _i64(0)
        used = ctypes.c_size_t(0)
        lib().spin_server_stats(self._h, ctypes.byref(q), ctypes.byref(a), ctypes.byref(used))
        return {"queued": q.value, "active": a.value, "pool_used": used.value}

    def close(self) -> None:
        if self._h:
            lib().spin_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
