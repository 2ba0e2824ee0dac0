"""Python binding of libfhtfbp (the C ABI declared in include/fhtfbp.h).

Argument marshalling only: tensors are checked for device, dtype, contiguity and shape, and
their device pointers are handed to the library together with torch's current HIP stream.
Every step of the computation runs in the library's HIP kernels; there is no fallback, and a
missing library raises an error.

Layouts (float32, contiguous, on the GPU):
    linogram [B, 4, N, N]  (class q, slope index t, cyclic shift s)
    image    [B, N, N]
    sinogram [B, P, Nd]    (uniform parallel beam, for the direct-FBP comparator)
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfhtfbp.so")

FBP_OK = 0
FBP_EINVAL = -1
FBP_EUNSTABLE = -2
FBP_ENOMEM = -3
FBP_EDEVICE = -4
FBP_ERANGE = -5

FBP_NO_ROW_SCALE = 1
FBP_INPUT_IS_FHT = 2
FBP_ZERO_WINDOW = 4
FBP_NO_SCRATCH = 8
FBP_NOALLOC_SCRATCH_BYTES = 256 << 20

FIT_DC_ZERO = 1
FIT_FREQUENCY = 2

_lib = None


class FbpError(RuntimeError):
    """A libfhtfbp call returned an error code."""

    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} ({code})")


class _PlanDesc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("max_batch", ctypes.c_int32),
        ("order", ctypes.c_int32),
        ("groups", ctypes.c_int32),
        ("b", ctypes.POINTER(ctypes.c_double)),
        ("a", ctypes.POINTER(ctypes.c_double)),
        ("flags", ctypes.c_uint32),
        ("stream", ctypes.c_void_p),
    ]


def load_library():
    """Load libfhtfbp.so (built in-tree by ``paper_2007_06289_amd._build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2007_06289_amd._build` (or __graft_entry__.build())")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32
    dp = ctypes.POINTER(ctypes.c_double)
    sig = {
        "fbp_plan": ([ctypes.POINTER(_PlanDesc), ctypes.POINTER(vp)], ctypes.c_int),
        "fbp_plan_destroy": ([vp], ctypes.c_int),
        "fbp_plan_set_stream": ([vp, vp], ctypes.c_int),
        "fbp_plan_set_coefficients": ([vp, dp, dp], ctypes.c_int),
        "fbp_plan_passes": ([vp, ctypes.POINTER(i32), i32], ctypes.c_int),
        "fbp_filter": ([vp, vp, vp, i32], ctypes.c_int),
        "fht_backproject": ([vp, vp, vp, i32], ctypes.c_int),
        "fht_forward": ([vp, vp, vp, i32], ctypes.c_int),
        "fbp_reconstruct": ([vp, vp, vp, i32], ctypes.c_int),
        "fbp_reconstruct_noalloc": ([vp, vp, vp, i32], ctypes.c_int),
        "fbp_fit_ramp_iir": ([i32, i32, u32, dp, dp, dp], ctypes.c_int),
        "fbp_direct_parallel": ([vp, vp, vp, i32, i32, i32, i32, vp], ctypes.c_int),
        "fbp_direct_filter": ([vp, vp, i32, i32, i32, vp], ctypes.c_int),
        "fbp_direct_linogram": ([vp, vp, vp, i32, i32, vp], ctypes.c_int),
        "fbp_filter_coef_grad": ([vp, vp, vp, vp, i32], ctypes.c_int),
        "fbp_cnn_pack": ([vp, vp, i32, i32, i32, vp], ctypes.c_int),
        "fbp_cnn_packed_elems": ([i32], ctypes.c_int32),
        "fbp_cnn_conv": ([i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, i32, i32, i32, i32, vp],
                         ctypes.c_int),
        "fbp_cnn_forward": ([vp, vp, vp, vp, vp, vp, vp, vp, i32, i32, i32, vp], ctypes.c_int),
        "fbp_cnn_wgrad_partial_floats": ([i32, i32, i32, i32, i32], ctypes.c_int64),
        "fbp_cnn_wgrad": ([i32, i32, vp, vp, vp, vp, vp, vp, i32, i32, i32, vp], ctypes.c_int),
        "fbp_direct_backproject": ([vp, vp, i32, i32, i32, i32, vp], ctypes.c_int),
        "fbp_strerror": ([ctypes.c_int], ctypes.c_char_p),
        "fbp_plan_profile": ([vp, i32], ctypes.c_int),
        "fbp_plan_profile_read": ([vp, dp, ctypes.POINTER(i32)], ctypes.c_int),
        "fbp_plan_set_schedule": ([vp, ctypes.POINTER(i32), i32, i32], ctypes.c_int),
        "fbp_plan_schedule_info": ([vp, ctypes.POINTER(i32), ctypes.POINTER(i32)],
                                   ctypes.c_int),
        "fbp_plan_filter_info": ([vp, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                  ctypes.POINTER(i32), ctypes.POINTER(i32)], ctypes.c_int),
        "fbp_reconstruct_many": ([ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                                  ctypes.POINTER(i32), i32, vp], ctypes.c_int),
        "fbp_graph_create": ([ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(vp),
                              ctypes.POINTER(i32), i32, ctypes.POINTER(vp)], ctypes.c_int),
        "fbp_graph_launch": ([vp, vp], ctypes.c_int),
        "fbp_resample_sinogram": ([vp, vp, i32, i32, i32, i32, vp], ctypes.c_int),
        "fbp_reconstruct_sinogram": ([vp, vp, vp, vp, i32, i32, i32], ctypes.c_int),
        "fbp_graph_destroy": ([vp], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def strerror(code: int) -> str:
    return load_library().fbp_strerror(int(code)).decode()


def _check(rc: int, what: str):
    if rc != FBP_OK:
        raise FbpError(rc, what)


def _stream_ptr():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_ptr(t: torch.Tensor, name: str, shape=None) -> ctypes.c_void_p:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on the GPU (got {t.device})")
    if t.dtype != torch.float32:
        raise ValueError(f"{name} must be float32 (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


def _coef_arrays(b, a, order=None):
    b = np.ascontiguousarray(np.asarray(b, dtype=np.float64))
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if b.ndim == 1:
        b = b[None]
    if a.ndim == 1:
        a = a[None]
    if b.shape != a.shape:
        raise ValueError(f"b {b.shape} and a {a.shape} must have the same [groups, order] shape")
    if order is not None and b.shape[1] != order:
        raise ValueError(f"coefficients have order {b.shape[1]}, plan has {order}")
    return b, a


class Plan:
    """An fbp_plan handle (owns the library's per-size tables and inter-pass scratch)."""

    def __init__(self, n: int, max_batch: int, b, a, flags: int = 0):
        lib = load_library()
        b, a = _coef_arrays(b, a)
        self.n = int(n)
        self.max_batch = int(max_batch)
        self.groups, self.order = b.shape
        self.flags = int(flags)
        self._b, self._a = b, a
        desc = _PlanDesc(self.n, self.max_batch, self.order, self.groups,
                         b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                         a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                         self.flags, _stream_ptr() if torch.cuda.is_available() else None)
        h = ctypes.c_void_p()
        _check(lib.fbp_plan(ctypes.byref(desc), ctypes.byref(h)), "fbp_plan")
        self._h = h

    @property
    def handle(self):
        if self._h is None:
            raise RuntimeError("plan is closed")
        return self._h

    def bind_stream(self):
        _check(load_library().fbp_plan_set_stream(self.handle, _stream_ptr()),
               "fbp_plan_set_stream")

    def passes(self) -> list[int]:
        buf = (ctypes.c_int32 * 16)()
        p = load_library().fbp_plan_passes(self.handle, buf, 16)
        if p < 0:
            raise FbpError(p, "fbp_plan_passes")
        return [int(buf[i]) for i in range(p)]

    def schedule(self) -> tuple[list[int], int, int]:
        """(levels per back-projection pass, log2 of the column-tile width, most levels the
        first pass can fuse)."""
        w, f = ctypes.c_int32(), ctypes.c_int32()
        _check(load_library().fbp_plan_schedule_info(self.handle, ctypes.byref(w),
                                                     ctypes.byref(f)), "fbp_plan_schedule_info")
        return self.passes(), int(w.value), int(f.value)

    def filter_info(self) -> dict:
        """Chunk length, scan levels of the filter's chunks and of the first pass's 32-sample
        chunks, and whether the numerator's remainder term runs."""
        v = [ctypes.c_int32() for _ in range(4)]
        _check(load_library().fbp_plan_filter_info(self.handle, *[ctypes.byref(x) for x in v]),
               "fbp_plan_filter_info")
        return {"chunk": int(v[0].value), "scan_levels": int(v[1].value),
                "first_levels": int(v[2].value), "remainder": bool(v[3].value)}

    def set_schedule(self, levels, log2w: int = 0):
        """Regroup the butterfly levels into passes (results are unchanged, bit for bit)."""
        lv = (ctypes.c_int32 * len(levels))(*[int(x) for x in levels])
        _check(load_library().fbp_plan_set_schedule(self.handle, lv, len(levels), int(log2w)),
               "fbp_plan_set_schedule")

    KERNEL_KINDS = ("first", "middle", "last_v", "last_h", "forward", "filter", "last")

    def profile(self, enable: bool = True):
        """Start (clearing) or stop recording HIP events around every launch of this plan."""
        _check(load_library().fbp_plan_profile(self.handle, 1 if enable else 0),
               "fbp_plan_profile")

    def profile_read(self) -> dict:
        """{kind: (total_ms, launches)} for the recorded launches (synchronises them)."""
        ms = (ctypes.c_double * len(self.KERNEL_KINDS))()
        n = (ctypes.c_int32 * len(self.KERNEL_KINDS))()
        _check(load_library().fbp_plan_profile_read(self.handle, ms, n), "fbp_plan_profile_read")
        return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(self.KERNEL_KINDS) if n[i]}

    def close(self):
        if getattr(self, "_h", None) is not None:
            load_library().fbp_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def fbp_plan(n: int, max_batch: int, b, a, flags: int = 0) -> Plan:
    """Create a plan (see ``fbp_plan`` in include/fhtfbp.h).  ``b``/``a``: [order] or
    [groups, order] float64 arrays (b_0..b_{K-1}, a_1..a_K)."""
    return Plan(n, max_batch, b, a, flags)


def fbp_plan_set_coefficients(plan: Plan, b, a):
    b, a = _coef_arrays(b, a, plan.order)
    if b.shape[0] != plan.groups:
        raise ValueError(f"expected {plan.groups} coefficient groups, got {b.shape[0]}")
    _check(load_library().fbp_plan_set_coefficients(
        plan.handle, b.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
        a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "fbp_plan_set_coefficients")
    plan._b, plan._a = b, a


def _batch_of(t: torch.Tensor, tail_dims: int, name: str) -> int:
    if t.dim() != tail_dims + 1:
        raise ValueError(f"{name} must have {tail_dims + 1} dimensions, got {tuple(t.shape)}")
    return int(t.shape[0])


def fbp_filter(plan: Plan, lino_in: torch.Tensor, lino_out: torch.Tensor | None = None):
    """Recursive ramp-pair filter of every linogram row; ``lino_out`` may be ``lino_in``."""
    B = _batch_of(lino_in, 3, "lino_in")
    shape = (B, 4, plan.n, plan.n)
    if lino_out is None:
        lino_out = torch.empty(shape, device=lino_in.device, dtype=torch.float32)
    pin, pout = _dev_ptr(lino_in, "lino_in", shape), _dev_ptr(lino_out, "lino_out", shape)
    plan.bind_stream()
    _check(load_library().fbp_filter(plan.handle, pin, pout, B), "fbp_filter")
    return lino_out


def fht_backproject(plan: Plan, lino: torch.Tensor, img: torch.Tensor | None = None):
    """Transposed-FHT back projection of the four classes, summed: [B,4,N,N] -> [B,N,N]."""
    B = _batch_of(lino, 3, "lino")
    if img is None:
        img = torch.empty((B, plan.n, plan.n), device=lino.device, dtype=torch.float32)
    pl = _dev_ptr(lino, "lino", (B, 4, plan.n, plan.n))
    pi = _dev_ptr(img, "img", (B, plan.n, plan.n))
    plan.bind_stream()
    _check(load_library().fht_backproject(plan.handle, pl, pi, B), "fht_backproject")
    return img


def fht_forward(plan: Plan, img: torch.Tensor, lino: torch.Tensor | None = None):
    """Dyadic FHT forward projection on the four classes: [B,N,N] -> [B,4,N,N]."""
    B = _batch_of(img, 2, "img")
    if lino is None:
        lino = torch.empty((B, 4, plan.n, plan.n), device=img.device, dtype=torch.float32)
    pi = _dev_ptr(img, "img", (B, plan.n, plan.n))
    pl = _dev_ptr(lino, "lino", (B, 4, plan.n, plan.n))
    plan.bind_stream()
    _check(load_library().fht_forward(plan.handle, pi, pl, B), "fht_forward")
    return lino


def fbp_reconstruct(plan: Plan, lino: torch.Tensor, img: torch.Tensor | None = None):
    """Filter plus back projection (the method end to end): [B,4,N,N] -> [B,N,N]."""
    B = _batch_of(lino, 3, "lino")
    if img is None:
        img = torch.empty((B, plan.n, plan.n), device=lino.device, dtype=torch.float32)
    pl = _dev_ptr(lino, "lino", (B, 4, plan.n, plan.n))
    pi = _dev_ptr(img, "img", (B, plan.n, plan.n))
    plan.bind_stream()
    _check(load_library().fbp_reconstruct(plan.handle, pl, pi, B), "fbp_reconstruct")
    return img


def fbp_reconstruct_noalloc(plan: Plan, lino: torch.Tensor, img: torch.Tensor):
    """fbp_reconstruct with the library's fixed scratch array: the C call allocates nothing
    (the caller passes the output).  [B,4,N,N] -> [B,N,N]."""
    B = _batch_of(lino, 3, "lino")
    pl = _dev_ptr(lino, "lino", (B, 4, plan.n, plan.n))
    pi = _dev_ptr(img, "img", (B, plan.n, plan.n))
    plan.bind_stream()
    _check(load_library().fbp_reconstruct_noalloc(plan.handle, pl, pi, B),
           "fbp_reconstruct_noalloc")
    return img


def fbp_filter_coef_grad(plan: Plan, lino: torch.Tensor, grad_out: torch.Tensor) -> torch.Tensor:
    """dL/d(b, a) per coefficient group, [groups, 2, order] float64 on the GPU, given the filter
    input and the gradient with respect to the filter output."""
    B = _batch_of(lino, 3, "lino")
    shape = (B, 4, plan.n, plan.n)
    out = torch.empty((plan.groups, 2, plan.order), device=lino.device, dtype=torch.float64)
    if not out.is_contiguous():
        raise ValueError("internal: output not contiguous")
    plan.bind_stream()
    _check(load_library().fbp_filter_coef_grad(plan.handle, _dev_ptr(lino, "lino", shape),
                                               _dev_ptr(grad_out, "grad_out", shape),
                                               ctypes.c_void_p(out.data_ptr()), B),
           "fbp_filter_coef_grad")
    return out


def fbp_fit_ramp_iir(order: int, length: int, dc_zero: bool = True, frequency: bool = False):
    """Fit the recursive ramp pair on the host; returns (b, a, relative error of the fit).
    ``frequency``: fit the frequency response to the ramp in relative error (not the paper's
    time-domain criterion; see fbp_fit_ramp_iir in include/fhtfbp.h)."""
    b = np.zeros(order, dtype=np.float64)
    a = np.zeros(order, dtype=np.float64)
    err = ctypes.c_double()
    dp = ctypes.POINTER(ctypes.c_double)
    flags = (FIT_DC_ZERO if dc_zero else 0) | (FIT_FREQUENCY if frequency else 0)
    _check(load_library().fbp_fit_ramp_iir(int(order), int(length), flags,
                                           b.ctypes.data_as(dp), a.ctypes.data_as(dp),
                                           ctypes.byref(err)), "fbp_fit_ramp_iir")
    return b, a, float(err.value)


def fbp_direct_parallel(sino: torch.Tensor, n: int, img: torch.Tensor | None = None,
                        work: torch.Tensor | None = None):
    """Direct FBP comparator on a uniform parallel-beam sinogram [B, P, Nd] -> [B, n, n]."""
    B, P, Nd = _batch_of(sino, 2, "sino"), sino.shape[1], sino.shape[2]
    if img is None:
        img = torch.empty((B, n, n), device=sino.device, dtype=torch.float32)
    if work is None:
        work = torch.empty((B, P, Nd), device=sino.device, dtype=torch.float32)
    ps = _dev_ptr(sino, "sino")
    pw = _dev_ptr(work, "work", (B, P, Nd))
    pi = _dev_ptr(img, "img", (B, n, n))
    _check(load_library().fbp_direct_parallel(ps, pw, pi, B, int(n), int(P), int(Nd),
                                              _stream_ptr()), "fbp_direct_parallel")
    return img


def fbp_direct_linogram(lino: torch.Tensor, img: torch.Tensor | None = None,
                        work: torch.Tensor | None = None):
    """Direct FBP (exact ramp, exact line positions) of a linogram [B,4,N,N] -> [B,N,N]."""
    B, N = _batch_of(lino, 3, "lino"), lino.shape[-1]
    if img is None:
        img = torch.empty((B, N, N), device=lino.device, dtype=torch.float32)
    if work is None:
        work = torch.empty((B, 4 * N, N), device=lino.device, dtype=torch.float32)
    _check(load_library().fbp_direct_linogram(_dev_ptr(lino, "lino", (B, 4, N, N)),
                                              _dev_ptr(work, "work", (B, 4 * N, N)),
                                              _dev_ptr(img, "img", (B, N, N)), B, int(N),
                                              _stream_ptr()), "fbp_direct_linogram")
    return img


def fbp_direct_filter(sino: torch.Tensor, work: torch.Tensor):
    B, P, Nd = _batch_of(sino, 2, "sino"), sino.shape[1], sino.shape[2]
    _check(load_library().fbp_direct_filter(_dev_ptr(sino, "sino"),
                                            _dev_ptr(work, "work", (B, P, Nd)), B, int(P),
                                            int(Nd), _stream_ptr()), "fbp_direct_filter")
    return work


def fbp_direct_backproject(work: torch.Tensor, n: int, img: torch.Tensor):
    B, P, Nd = _batch_of(work, 2, "work"), work.shape[1], work.shape[2]
    _check(load_library().fbp_direct_backproject(_dev_ptr(work, "work"),
                                                 _dev_ptr(img, "img", (B, n, n)), B, int(n),
                                                 int(P), int(Nd), _stream_ptr()),
           "fbp_direct_backproject")
    return img


# ---- learned residual correction (3x3 convolutions on the matrix cores) ------------------------

def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _check_dev(t, name, dtype, shape=None):
    if t is None:
        return
    if t.device.type != "cuda" or t.dtype != dtype or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous {dtype} tensor on the GPU")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")


def fbp_cnn_pack(w: torch.Tensor, transpose_flip: bool = False) -> torch.Tensor:
    """Pack FP32 weights [cout, cin, 3, 3] into the BF16 matrix-core operand order (int16)."""
    cout, cin = int(w.shape[0]), int(w.shape[1])
    _check_dev(w, "w", torch.float32, (cout, cin, 3, 3))
    lib = load_library()
    n = lib.fbp_cnn_packed_elems(cout if transpose_flip else cin)
    out = torch.empty(n, device=w.device, dtype=torch.int16)
    _check(lib.fbp_cnn_pack(_ptr(w), _ptr(out), cin, cout, 1 if transpose_flip else 0,
                            _stream_ptr()), "fbp_cnn_pack")
    return out


def fbp_cnn_conv(cin: int, cout: int, x: torch.Tensor, wpacked: torch.Tensor,
                 bias: torch.Tensor | None = None, mask: torch.Tensor | None = None,
                 resid: torch.Tensor | None = None, relu: bool = False) -> torch.Tensor:
    """One 3x3 convolution: x is FP32 [B,H,W] (cin 1) or BF16-as-int16 [B,H,W,16] (cin 16);
    returns BF16-as-int16 [B,H,W,16] (cout 16) or FP32 [B,H,W] (cout 1)."""
    B, H, W = int(x.shape[0]), int(x.shape[1]), int(x.shape[2])
    if cin == 1:
        _check_dev(x, "x", torch.float32, (B, H, W))
    else:
        _check_dev(x, "x", torch.int16, (B, H, W, 16))
    _check_dev(mask, "mask", torch.int16, (B, H, W, 16))
    _check_dev(resid, "resid", torch.float32, (B, H, W))
    _check_dev(bias, "bias", torch.float32, (cout,))
    if cout == 16:
        out = torch.empty((B, H, W, 16), device=x.device, dtype=torch.int16)
        o16, o32 = out, None
    else:
        out = torch.empty((B, H, W), device=x.device, dtype=torch.float32)
        o16, o32 = None, out
    _check(load_library().fbp_cnn_conv(cin, cout, _ptr(x) if cin == 1 else None,
                                       _ptr(x) if cin == 16 else None, _ptr(wpacked), _ptr(bias),
                                       _ptr(mask), _ptr(resid), _ptr(o16), _ptr(o32),
                                       1 if relu else 0, B, H, W, _stream_ptr()), "fbp_cnn_conv")
    return out


def fbp_cnn_forward(x: torch.Tensor, p1: torch.Tensor, b1: torch.Tensor, p2: torch.Tensor,
                    b2: torch.Tensor, p3: torch.Tensor, b3: torch.Tensor,
                    out: torch.Tensor | None = None) -> torch.Tensor:
    """The residual network at inference in one launch: [B,H,W] FP32 -> [B,H,W], weights packed
    by fbp_cnn_pack."""
    B, H, W = x.shape
    _check_dev(x, "x", torch.float32)
    if out is None:
        out = torch.empty_like(x)
    _check_dev(out, "out", torch.float32, (B, H, W))
    for t, nm, dt in ((p1, "p1", torch.int16), (p2, "p2", torch.int16), (p3, "p3", torch.int16),
                      (b1, "b1", torch.float32), (b2, "b2", torch.float32),
                      (b3, "b3", torch.float32)):
        _check_dev(t, nm, dt)
    _check(load_library().fbp_cnn_forward(_ptr(x), _ptr(p1), _ptr(b1), _ptr(p2), _ptr(b2),
                                          _ptr(p3), _ptr(b3), _ptr(out), B, H, W,
                                          _stream_ptr()), "fbp_cnn_forward")
    return out


def fbp_cnn_wgrad(cin: int, cout: int, dz: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
    """[cout*cin*9 + cout] FP32: weight gradients then bias gradients."""
    B, H, W = int(dz.shape[0]), int(dz.shape[1]), int(dz.shape[2])
    lib = load_library()
    nparts = lib.fbp_cnn_wgrad_partial_floats(cin, cout, B, H, W)
    if nparts < 0:
        raise FbpError(int(nparts), "fbp_cnn_wgrad_partial_floats")
    partial = torch.empty(int(nparts), device=dz.device, dtype=torch.float32)
    out = torch.empty(cout * cin * 9 + cout, device=dz.device, dtype=torch.float32)
    _check(lib.fbp_cnn_wgrad(cin, cout, _ptr(dz) if cout == 1 else None,
                             _ptr(dz) if cout == 16 else None, _ptr(x) if cin == 1 else None,
                             _ptr(x) if cin == 16 else None, _ptr(partial), _ptr(out), B, H, W,
                             _stream_ptr()), "fbp_cnn_wgrad")
    return out


def _many_args(plans, linos, imgs):
    if not (len(plans) == len(linos) == len(imgs)):
        raise ValueError("plans, linograms and images must have the same length")
    k = len(plans)
    P = (ctypes.c_void_p * max(k, 1))()
    L = (ctypes.c_void_p * max(k, 1))()
    I = (ctypes.c_void_p * max(k, 1))()
    B = (ctypes.c_int32 * max(k, 1))()
    for i, (p, lino, img) in enumerate(zip(plans, linos, imgs)):
        b = _batch_of(lino, 3, f"lino[{i}]")
        P[i] = p.handle.value
        L[i] = _dev_ptr(lino, f"lino[{i}]", (b, 4, p.n, p.n)).value
        I[i] = _dev_ptr(img, f"img[{i}]", (b, p.n, p.n)).value
        B[i] = b
    return P, L, I, B, k


def fbp_reconstruct_many(plans, linos, imgs):
    """Reconstruct a mixed batch: linos[i] [B_i,4,N_i,N_i] -> imgs[i] [B_i,N_i,N_i] with
    plans[i], all on the current stream in one library call."""
    P, L, I, B, k = _many_args(plans, linos, imgs)
    _check(load_library().fbp_reconstruct_many(P, L, I, B, k, _stream_ptr()),
           "fbp_reconstruct_many")
    return imgs


class Graph:
    """A captured mixed-batch reconstruction (fbp_graph_create): ``launch()`` replays every
    kernel with one call.  Keeps the plans and buffers alive while it exists."""

    def __init__(self, plans, linos, imgs):
        P, L, I, B, k = _many_args(plans, linos, imgs)
        h = ctypes.c_void_p()
        _check(load_library().fbp_graph_create(P, L, I, B, k, ctypes.byref(h)),
               "fbp_graph_create")
        self._h = h
        self._keep = (list(plans), list(linos), list(imgs))

    def launch(self):
        if self._h is None:
            raise RuntimeError("graph is destroyed")
        _check(load_library().fbp_graph_launch(self._h, _stream_ptr()), "fbp_graph_launch")

    def close(self):
        if getattr(self, "_h", None) is not None:
            load_library().fbp_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fbp_graph_create(plans, linos, imgs) -> Graph:
    return Graph(plans, linos, imgs)


def fbp_resample_sinogram(sino: torch.Tensor, n: int, lino: torch.Tensor | None = None):
    """Parallel-beam sinogram [B, P, D] -> linogram [B, 4, n, n] (bilinear, Sec. 4.2)."""
    B = _batch_of(sino, 2, "sino")
    P, D = int(sino.shape[1]), int(sino.shape[2])
    if lino is None:
        lino = torch.empty((B, 4, n, n), device=sino.device, dtype=torch.float32)
    ps = _dev_ptr(sino, "sino", (B, P, D))
    pl = _dev_ptr(lino, "lino", (B, 4, n, n))
    _check(load_library().fbp_resample_sinogram(ps, pl, B, int(n), P, D, _stream_ptr()),
           "fbp_resample_sinogram")
    return lino


def fbp_reconstruct_sinogram(plan: Plan, sino: torch.Tensor, img: torch.Tensor | None = None,
                             work: torch.Tensor | None = None):
    """The method from scanner data: resample [B, P, D] onto the linogram, then reconstruct."""
    B = _batch_of(sino, 2, "sino")
    P, D = int(sino.shape[1]), int(sino.shape[2])
    n = plan.n
    if img is None:
        img = torch.empty((B, n, n), device=sino.device, dtype=torch.float32)
    if work is None:
        work = torch.empty((B, 4, n, n), device=sino.device, dtype=torch.float32)
    ps = _dev_ptr(sino, "sino", (B, P, D))
    pw = _dev_ptr(work, "work", (B, 4, n, n))
    pi = _dev_ptr(img, "img", (B, n, n))
    plan.bind_stream()
    _check(load_library().fbp_reconstruct_sinogram(plan.handle, ps, pw, pi, B, P, D),
           "fbp_reconstruct_sinogram")
    return img



def fbp_reconstruct_sinogram_padded(plan2: Plan, sino: torch.Tensor, n: int,
                                    img2: torch.Tensor | None = None,
                                    work: torch.Tensor | None = None) -> torch.Tensor:
    """Objects that reach outside the disc of radius 0.34 n, where the cyclic shift axis of the
    n-shift linogram would fold their projections onto themselves: resample and reconstruct
    on the 2n grid (same pixel size and centre; its 0.34 * 2n disc holds the inscribed circle
    of the n x n image) and return the central n x n part as a view of the 2n image.
    ``plan2`` is a plan for 2n."""
    if plan2.n != 2 * n:
        raise ValueError(f"plan2 is for N={plan2.n}, need 2n = {2 * n}")
    img2 = fbp_reconstruct_sinogram(plan2, sino, img2, work)
    o = n // 2
    return img2[:, o:o + n, o:o + n]
