"""Python binding of the MI355X batched orthonormal 2D DCT library (libdct2d.so).

Argument marshalling only: every transform runs in the HIP kernels behind the C ABI
declared in include/dct2d.h.  PyTorch supplies device memory and streams.  There is
no fallback: if the compiled library is missing, importing the binding's entry
points raises.

Transforms (paper, Section 2.1 eq. 1-2): forward Y = Q_h X Q_w^T, inverse
X = Q_h^T Y Q_w, and the fused round trip inverse(forward(X)).
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "_lib", "libdct2d.so")

FORWARD, INVERSE, ROUNDTRIP, FILTER = 0, 1, 2, 3
FP32, SPLIT_BF16X3, SPLIT_BF16X6, SPLIT_FP16X3, BF16, FP16, FP8_E4M3, AUTO = range(8)
PRECISIONS = {"fp32": FP32, "bf16x3": SPLIT_BF16X3, "bf16x6": SPLIT_BF16X6, "fp16x3": SPLIT_FP16X3,
              "bf16": BF16, "fp16": FP16, "fp8": FP8_E4M3, "auto": AUTO}
# "filter" names the spectral filter's entry of the policy / autotuner (dct2d_filter); the
# transform calls accept the first three only
DIRECTIONS = {"forward": FORWARD, "inverse": INVERSE, "roundtrip": ROUNDTRIP, "filter": FILTER}

EXPORTS = ("dct2d_init", "dct2d_finalize", "dct2d_forward", "dct2d_inverse", "dct2d_roundtrip",
           "dct2d_transform_ex", "dct2d_filter", "dct2d_ragged_plan_create", "dct2d_ragged_execute",
           "dct2d_ragged_plan_destroy", "dct2d_ragged_plan_info", "dct2d_variant_count",
           "dct2d_get_variant", "dct2d_set_variant", "dct2d_tune", "dct2d_status_string", "dct2d_version",
           "dct2d_copy", "dct2d_image_transform", "dct2d_image_transform_noalloc", "dct2d_fma_issue")


class DCT2DError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        super().__init__("%s failed: %s (%d)" % (where, status_string(code), code))


class Block(ctypes.Structure):
    _fields_ = [("offset", ctypes.c_int64), ("rows", ctypes.c_int32), ("cols", ctypes.c_int32)]


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libdct2d.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libdct2d.so not built at %s: run __graft_entry__.build() or "
                          "python paper_2609_28519_amd/build.py" % path)
    lib = ctypes.CDLL(path)
    i64, i32, vp, c_int = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int
    lib.dct2d_init.argtypes = [c_int]
    lib.dct2d_finalize.argtypes = []
    lib.dct2d_finalize.restype = None
    for n in ("dct2d_forward", "dct2d_inverse", "dct2d_roundtrip"):
        getattr(lib, n).argtypes = [vp, i64, i32, i32, i64, vp]
    lib.dct2d_transform_ex.argtypes = [c_int, vp, vp, i64, i32, i32, i64, i64, c_int, vp]
    lib.dct2d_filter.argtypes = [vp, vp, i64, i32, i32, i64, i64, vp, i64, vp]
    lib.dct2d_ragged_plan_create.argtypes = [ctypes.POINTER(Block), i64, c_int, c_int, ctypes.POINTER(vp)]
    lib.dct2d_ragged_execute.argtypes = [vp, vp, vp]
    lib.dct2d_ragged_plan_destroy.argtypes = [vp]
    lib.dct2d_ragged_plan_destroy.restype = None
    lib.dct2d_ragged_plan_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(i32)]
    for n in ("dct2d_variant_count", "dct2d_get_variant"):
        getattr(lib, n).argtypes = [i32, i32, c_int, c_int]
    lib.dct2d_set_variant.argtypes = [i32, i32, c_int, c_int, c_int]
    lib.dct2d_tune.argtypes = [i32, i32, c_int, c_int, i64, vp, ctypes.POINTER(ctypes.c_float)]
    lib.dct2d_copy.argtypes = [vp, vp, i64, vp]
    lib.dct2d_fma_issue.argtypes = [vp, i32, i32, vp]
    for n in ("dct2d_image_transform", "dct2d_image_transform_noalloc"):
        getattr(lib, n).argtypes = [c_int, vp, vp, i64, i32, i32, i64, i64, vp]
    lib.dct2d_status_string.argtypes = [c_int]
    lib.dct2d_status_string.restype = ctypes.c_char_p
    lib.dct2d_version.argtypes = []
    lib.dct2d_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def status_string(code: int) -> str:
    return load().dct2d_status_string(int(code)).decode()


def version() -> str:
    return load().dct2d_version().decode()


def _check(rc: int, where: str) -> None:
    if rc != 0:
        raise DCT2DError(rc, where)


def init(device: int = 0) -> None:
    _check(load().dct2d_init(int(device)), "dct2d_init")


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def _geometry(t, rows, cols, stride, batch=None):
    """(batch, rows, cols, stride) of a float32 CUDA tensor shaped (..., rows, cols), or of a flat
    buffer holding arrays `stride` floats apart (batch defaults to as many as fit)."""
    import torch
    if t.dtype != torch.float32:
        raise TypeError("float32 tensor required")
    if not t.is_cuda:
        raise TypeError("CUDA (HIP) tensor required")
    if rows is None:
        rows, cols = int(t.shape[-2]), int(t.shape[-1])
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous (arrays are addressed from its first element)")
    if stride is None:
        stride = rows * cols
    if batch is None:
        batch = 0 if t.numel() < rows * cols else (t.numel() - rows * cols) // stride + 1
    if batch > 0 and (batch - 1) * stride + rows * cols > t.numel():
        raise ValueError("buffer too small for batch/stride")
    return int(batch), int(rows), int(cols), int(stride)


def _check_out(inp, out):
    """The output must be a contiguous float32 tensor with the input's shape on the input's device:
    the C ABI receives a raw device pointer and cannot tell a host or differently typed buffer apart."""
    import torch
    if out.dtype != torch.float32:
        raise TypeError("out must be float32")
    if not out.is_cuda or out.device != inp.device:
        raise TypeError("out must be a CUDA (HIP) tensor on the input's device")
    if out.shape != inp.shape or not out.is_contiguous():
        raise ValueError("out must be contiguous with the input's shape")


def _inplace(name, t, rows, cols, stride, stream, batch=None):
    batch, rows, cols, stride = _geometry(t, rows, cols, stride, batch)
    fn = getattr(load(), name)
    _check(fn(ctypes.c_void_p(t.data_ptr()), batch, rows, cols, stride, ctypes.c_void_p(_stream(stream))), name)
    return t


def forward_(t, rows=None, cols=None, stride=None, stream=None, batch=None):
    """In-place forward 2D DCT-II of every (rows, cols) array in t (dct2d_forward)."""
    return _inplace("dct2d_forward", t, rows, cols, stride, stream, batch)


def inverse_(t, rows=None, cols=None, stride=None, stream=None, batch=None):
    """In-place inverse 2D DCT (dct2d_inverse)."""
    return _inplace("dct2d_inverse", t, rows, cols, stride, stream, batch)


def roundtrip_(t, rows=None, cols=None, stride=None, stream=None, batch=None):
    """In-place fused round trip inverse(forward(X)) (dct2d_roundtrip)."""
    return _inplace("dct2d_roundtrip", t, rows, cols, stride, stream, batch)


def transform(inp, out=None, direction="forward", precision="auto", stream=None):
    """Out-of-place (or in-place if out is inp) transform with an explicit path (dct2d_transform_ex)."""
    import torch
    if out is None:
        out = torch.empty_like(inp)
    d = DIRECTIONS[direction] if isinstance(direction, str) else int(direction)
    p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    batch, rows, cols, stride = _geometry(inp, None, None, None)
    _check_out(inp, out)
    rc = load().dct2d_transform_ex(d, ctypes.c_void_p(inp.data_ptr()), ctypes.c_void_p(out.data_ptr()), batch,
                                   rows, cols, stride, stride, p, ctypes.c_void_p(_stream(stream)))
    _check(rc, "dct2d_transform_ex")
    return out


def filter(inp, lam, out=None, stream=None):
    """Spectral filter Q_h^T (lam o (Q_h X Q_w^T)) Q_w of every (rows, cols) array of inp
    (dct2d_filter; Prop. 1, eq. 4).  lam: float32 CUDA tensor of shape (rows, cols), one
    operator for all arrays, or inp's shape, one per array.  out may be inp (in place)."""
    import torch
    if out is None:
        out = torch.empty_like(inp)
    batch, rows, cols, stride = _geometry(inp, None, None, None)
    _check_out(inp, out)
    if lam.dtype != torch.float32 or not lam.is_cuda or not lam.is_contiguous() or lam.device != inp.device:
        raise TypeError("lam must be a contiguous float32 CUDA tensor on the input's device")
    if tuple(lam.shape) == (rows, cols):
        lam_stride = 0
    elif lam.shape == inp.shape:
        lam_stride = rows * cols
    else:
        raise ValueError("lam must have shape (rows, cols) or the input's shape")
    rc = load().dct2d_filter(ctypes.c_void_p(inp.data_ptr()), ctypes.c_void_p(out.data_ptr()), batch, rows, cols,
                             stride, stride, ctypes.c_void_p(lam.data_ptr()), lam_stride,
                             ctypes.c_void_p(_stream(stream)))
    _check(rc, "dct2d_filter")
    return out


def image_transform(inp, out=None, direction="forward", stream=None, noalloc=False):
    """Batched transform of whole images of any shape with both axes in [8, 1024] (cols a multiple of
    4), dense Q_n for axes the fast kernels do not cover (dct2d_image_transform); noalloc=True calls
    dct2d_image_transform_noalloc, which allocates nothing (dct2d_init must have run)."""
    import torch
    if out is None:
        out = torch.empty_like(inp)
    d = DIRECTIONS[direction] if isinstance(direction, str) else int(direction)
    batch, rows, cols, stride = _geometry(inp, None, None, None)
    _check_out(inp, out)
    name = "dct2d_image_transform_noalloc" if noalloc else "dct2d_image_transform"
    rc = getattr(load(), name)(d, ctypes.c_void_p(inp.data_ptr()), ctypes.c_void_p(out.data_ptr()), batch, rows, cols,
                               stride, stride, ctypes.c_void_p(_stream(stream)))
    _check(rc, name)
    return out


def copy(inp, out=None, stream=None):
    """Plain device copy through the library's reference streaming kernel (dct2d_copy): the
    practical HBM ceiling of a one-read-one-write kernel.  out may be inp."""
    import torch
    if out is None:
        out = torch.empty_like(inp)
    if inp.dtype != torch.float32 or not inp.is_cuda or not inp.is_contiguous():
        raise TypeError("contiguous float32 CUDA tensor required")
    _check_out(inp, out)
    _check(load().dct2d_copy(ctypes.c_void_p(inp.data_ptr()), ctypes.c_void_p(out.data_ptr()), inp.numel(),
                             ctypes.c_void_p(_stream(stream))), "dct2d_copy")
    return out


def fma_issue(sink, blocks, iters, stream=None):
    """Launches the vector-ALU issue reference (dct2d_fma_issue): `blocks` workgroups of 256
    threads, each lane issuing iters x 16 independent float32 FMAs.  sink: a float32 CUDA tensor
    (never written in practice)."""
    import torch
    if sink.dtype != torch.float32 or not sink.is_cuda:
        raise TypeError("float32 CUDA tensor required")
    _check(load().dct2d_fma_issue(ctypes.c_void_p(sink.data_ptr()), int(blocks), int(iters),
                                  ctypes.c_void_p(_stream(stream))), "dct2d_fma_issue")


def _p(precision):
    return PRECISIONS[precision] if isinstance(precision, str) else int(precision)


def _d(direction):
    return DIRECTIONS[direction] if isinstance(direction, str) else int(direction)


def variant_count(rows, cols, direction="forward", precision="fp32") -> int:
    return load().dct2d_variant_count(rows, cols, _d(direction), _p(precision))


def set_variant(rows, cols, direction, precision, variant) -> None:
    _check(load().dct2d_set_variant(rows, cols, _d(direction), _p(precision), variant), "dct2d_set_variant")


def get_variant(rows, cols, direction="forward", precision="fp32") -> int:
    v = load().dct2d_get_variant(rows, cols, _d(direction), _p(precision))
    if v < 0:
        raise DCT2DError(v, "dct2d_get_variant")
    return v


def tune(rows, cols, direction="forward", precision="fp32", batch=4096, stream=None) -> float:
    ms = ctypes.c_float(0)
    _check(load().dct2d_tune(rows, cols, _d(direction), _p(precision), batch, ctypes.c_void_p(_stream(stream)),
                             ctypes.byref(ms)), "dct2d_tune")
    return ms.value


SIZES = (8, 16, 32, 64, 128, 256)


def policy() -> dict:
    """The frozen per-size policy: variant of every (rows, cols, direction, path) and the
    float32-accurate path chosen for "auto" (the autotune cache, as a JSON-able dict)."""
    out = {}
    for r in SIZES:
        for c in SIZES:
            for dname, d in DIRECTIONS.items():
                key = "%dx%d/%s" % (r, c, dname)
                out[key + "/auto"] = get_variant(r, c, d, AUTO)
                for pname, p in PRECISIONS.items():
                    if p != AUTO and variant_count(r, c, d, p) > 0:
                        out["%s/%s" % (key, pname)] = get_variant(r, c, d, p)
    return out


def save_policy(path: str) -> None:
    import json
    with open(path, "w") as f:
        json.dump(policy(), f, indent=0, sort_keys=True)


def load_policy(path: str) -> None:
    """Freezes a policy written by save_policy (auto paths last, after the variants)."""
    import json
    pol = json.load(open(path))
    for key, v in sorted(pol.items(), key=lambda kv: kv[0].endswith("/auto")):
        shape, dname, pname = key.split("/")
        r, c = (int(x) for x in shape.split("x"))
        set_variant(r, c, dname, pname, int(v))


class RaggedPlan:
    """A ragged batch recorded once as a HIP graph and replayed with one launch."""

    def __init__(self, offsets, rows, cols, direction="forward", precision="fp32"):
        n = len(offsets)
        arr = (Block * n)()
        for i in range(n):
            arr[i].offset, arr[i].rows, arr[i].cols = int(offsets[i]), int(rows[i]), int(cols[i])
        h = ctypes.c_void_p()
        d = DIRECTIONS[direction] if isinstance(direction, str) else int(direction)
        p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self._h = None
        _check(load().dct2d_ragged_plan_create(arr, n, d, p, ctypes.byref(h)), "dct2d_ragged_plan_create")
        self._h = h
        # floats a base buffer must hold: the end of the furthest array of the plan
        self.extent = max(int(offsets[i]) + int(rows[i]) * int(cols[i]) for i in range(n))
        import torch
        self.device = torch.device("cuda", torch.cuda.current_device())

    def execute(self, base, stream=None):
        """Runs the plan in place on the arrays of `base` (a contiguous float32 tensor on the
        plan's device holding at least `extent` floats)."""
        import torch
        if base.dtype != torch.float32 or not base.is_cuda or base.device != self.device:
            raise TypeError("base must be a float32 CUDA tensor on the plan's device (%s)" % self.device)
        if not base.is_contiguous():
            raise ValueError("base must be contiguous (arrays are addressed from its first element)")
        if base.numel() < self.extent:
            raise ValueError("base holds %d floats, the plan addresses %d" % (base.numel(), self.extent))
        _check(load().dct2d_ragged_execute(self._h, ctypes.c_void_p(base.data_ptr()),
                                           ctypes.c_void_p(_stream(stream))), "dct2d_ragged_execute")
        return base

    def info(self):
        items, classes, nodes = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        _check(load().dct2d_ragged_plan_info(self._h, ctypes.byref(items), ctypes.byref(classes),
                                             ctypes.byref(nodes)), "dct2d_ragged_plan_info")
        return {"items": items.value, "classes": classes.value, "graph_nodes": nodes.value}

    def close(self):
        if self._h:
            load().dct2d_ragged_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
