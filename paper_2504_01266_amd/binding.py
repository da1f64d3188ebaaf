"""ctypes binding of libfilter2d.so (the C ABI declared in include/filter2d.h).

Argument marshalling only: torch tensors are described by their data
pointers, shapes and strides, and every call is enqueued on torch's current
HIP stream.  All arithmetic happens in the library's HIP kernels; if the
library is missing this module raises instead of computing anything itself.
"""
import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfilter2d.so")

# status codes
OK, EINVAL, EUNSUPPORTED, EWORKSPACE, EHIP = 0, 1, 2, 3, 4
# element types
U8, I32, F32, BF16 = 0, 1, 2, 3
# border rules, channel modes, epilogues
BORDER_CLAMP, BORDER_ZERO = 0, 1
SHARED, DEPTHWISE, BANK = 0, 1, 2
EPI_NONE, EPI_SUMSQ_PAIRS = 0, 1
# tiling-variant paths
PATH_F32, PATH_U8, PATH_BATCHED = 0, 1, 2

_MODES = {"shared": SHARED, "depthwise": DEPTHWISE, "bank": BANK}
_DTYPES = {torch.uint8: U8, torch.int32: I32, torch.float32: F32, torch.bfloat16: BF16}


class F2dTensor(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("dtype", ctypes.c_int32), ("stride_w", ctypes.c_int32),
                ("n", ctypes.c_int64), ("c", ctypes.c_int64), ("h", ctypes.c_int64),
                ("w", ctypes.c_int64), ("stride_n", ctypes.c_int64), ("stride_c", ctypes.c_int64),
                ("stride_h", ctypes.c_int64)]


class F2dFilter(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("dtype", ctypes.c_int32), ("f_out", ctypes.c_int32),
                ("f_in", ctypes.c_int32), ("k", ctypes.c_int32)]


class F2dOpts(ctypes.Structure):
    _fields_ = [("border", ctypes.c_int32), ("channels", ctypes.c_int32),
                ("epilogue", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("row_begin", ctypes.c_int64), ("row_end", ctypes.c_int64)]


class F2dBatchItem(ctypes.Structure):
    _fields_ = [("image", ctypes.c_void_p), ("out", ctypes.c_void_p), ("filter", ctypes.c_void_p),
                ("c", ctypes.c_int64), ("h", ctypes.c_int64), ("w", ctypes.c_int64),
                ("in_stride_c", ctypes.c_int64), ("in_stride_h", ctypes.c_int64),
                ("out_stride_c", ctypes.c_int64), ("out_stride_h", ctypes.c_int64)]


class F2dError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"filter2d status {status}: {message}")
        self.status = status


_lib = None
_P = ctypes.POINTER


def load():
    """Load the HIP library (never falls back to anything else)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2504_01266_amd.build` "
                           "or __graft_entry__.build() first")
    lib = ctypes.CDLL(LIB_PATH)
    i32, i64, vp, sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t
    sigs = {
        "filter2d_forward": (i32, [_P(F2dTensor), _P(F2dFilter), _P(F2dOpts), _P(F2dTensor), i32, vp]),
        "filter2d_forward_separable": (i32, [_P(F2dTensor), vp, vp, i32, _P(F2dOpts), _P(F2dTensor), vp]),
        "filter2d_upsample_forward": (i32, [_P(F2dTensor), _P(F2dFilter), i32, _P(F2dOpts), _P(F2dTensor), vp]),
        "filter2d_backward_workspace": (sz, [_P(F2dTensor), _P(F2dFilter), _P(F2dOpts)]),
        "filter2d_backward": (i32, [_P(F2dTensor), _P(F2dFilter), _P(F2dTensor), i32, _P(F2dOpts),
                                    _P(F2dTensor), vp, vp, sz, vp]),
        "filter2d_backward_noalloc": (i32, [_P(F2dTensor), _P(F2dFilter), _P(F2dTensor), i32, _P(F2dOpts),
                                            _P(F2dTensor), vp, vp]),
        "filter2d_batched_plan": (i64, [_P(F2dBatchItem), i32, i32, i32, _P(i32), _P(i64)]),
        "filter2d_batched": (i32, [vp, vp, i32, i64, i32, i32, _P(F2dOpts), vp]),
        "filter2d_autotune_forward": (i32, [_P(F2dTensor), _P(F2dFilter), _P(F2dOpts), _P(F2dTensor),
                                            i32, i32, vp, _P(i32)]),
        "filter2d_autotune_batched": (i32, [_P(F2dBatchItem), vp, i32, i32, i32, vp, i32, vp,
                                            _P(i32)]),
        "filter2d_variant_count": (i32, [i32]),
        "filter2d_tune_save": (i32, [ctypes.c_char_p]),
        "filter2d_tune_load": (i32, [ctypes.c_char_p]),
        "filter2d_tune_clear": (None, []),
        "filter2d_status_string": (ctypes.c_char_p, [i32]),
        "filter2d_last_error": (ctypes.c_char_p, []),
        "filter2d_version": (i32, []),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status):
    if status != OK:
        msg = load().filter2d_last_error().decode()
        raise F2dError(status, msg)


def last_error():
    return load().filter2d_last_error().decode()


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def tensor_desc(t, dtype=None):
    """Describe a 4-D [n][c][h][w] tensor.  The column stride goes to
    stride_w (1 for planar tensors; an interleaved [n][h][w][c] tensor viewed
    with permute(0, 3, 1, 2) has stride_c 1 and stride_w c); the library
    decides which paths accept it."""
    if t.dim() != 4:
        raise ValueError("expected a 4-D [n][c][h][w] tensor")
    sw = t.stride(3) if t.size(3) > 1 else 1
    code = _DTYPES[t.dtype] if dtype is None else dtype
    return F2dTensor(t.data_ptr(), code, sw, t.size(0), t.size(1), t.size(2), t.size(3),
                     t.stride(0), t.stride(1), t.stride(2))


def filter_desc(f):
    if f.dim() == 2:
        f = f.view(1, 1, *f.shape)
    if f.dim() != 4 or f.size(2) != f.size(3):
        raise ValueError("expected a [f_out][f_in][k][k] filter")
    if not f.is_contiguous():
        raise ValueError("the filter must be contiguous")
    return F2dFilter(f.data_ptr(), _DTYPES[f.dtype], f.size(0), f.size(1), f.size(2)), f


_BORDERS = {"clamp": BORDER_CLAMP, "zero": BORDER_ZERO}


def make_opts(mode="shared", epilogue=EPI_NONE, rows=None, variant=0, border="clamp"):
    m = _MODES[mode] if isinstance(mode, str) else int(mode)
    r0, r1 = (0, 0) if rows is None else rows
    b = _BORDERS[border] if isinstance(border, str) else int(border)
    return F2dOpts(b, m, epilogue, variant, r0, r1)


def _as4(t):
    if t.dim() == 2:
        return t.view(1, 1, *t.shape)
    if t.dim() == 3:
        return t.unsqueeze(0)
    return t


def out_count(mode, filt_shape, channels, epilogue):
    m = _MODES[mode] if isinstance(mode, str) else int(mode)
    if m == DEPTHWISE:
        return filt_shape[0] // channels + (1 if epilogue == EPI_SUMSQ_PAIRS else 0)
    return 1


def interleaved(t):
    """True for an [n][c][h][w] view of interleaved [n][h][w][c] storage."""
    return t.dim() == 4 and t.size(1) > 1 and t.stride(1) == 1 and t.stride(3) == t.size(1)


def _new_out(image, filt, co, h, w, out_dtype, il):
    if out_dtype is not None:
        odt = out_dtype
    elif image.dtype == torch.uint8:
        odt = torch.int32 if filt.dtype == torch.int32 else torch.float32
    else:
        odt = torch.float32
    n = image.size(0)
    if il:
        return torch.empty((n, h, w, co), dtype=odt, device=image.device).permute(0, 3, 1, 2)
    return torch.empty((n, co, h, w), dtype=odt, device=image.device)


def forward(image, filt, mode="shared", epilogue=EPI_NONE, rows=None, outs=None, variant=0,
            out_dtype=None, border="clamp"):
    """Y = filter(X) on the current stream.  Returns one tensor (SHARED, BANK)
    or the list of DEPTHWISE outputs (one per filter index, plus the SUMSQ one).
    border: "clamp" (clamp-to-edge) or "zero".  u8 images: int32 taps give
    int32 outputs and float taps float32 outputs unless out_dtype (e.g.
    torch.uint8, clamped and rounded) says otherwise; an interleaved image
    (an [n][h][w][c] tensor viewed with permute(0, 3, 1, 2)) gets outputs in
    the same layout."""
    lib = load()
    image = _as4(image)
    fd, filt = filter_desc(filt)
    m = _MODES[mode] if isinstance(mode, str) else int(mode)
    n, c, h, w = image.shape
    r0, r1 = (0, h) if rows is None else rows
    nout = out_count(m, filt.shape, c, epilogue)
    if outs is None:
        co = filt.size(0) if m == BANK else c
        outs = [_new_out(image, filt, co, r1 - r0, w, out_dtype, interleaved(image) and m != BANK)
                for _ in range(nout)]
    descs = (F2dTensor * len(outs))(*[tensor_desc(_as4(o)) for o in outs])
    opts = make_opts(m, epilogue, (r0, r1), variant, border)
    _check(lib.filter2d_forward(ctypes.byref(tensor_desc(image)), ctypes.byref(fd),
                                ctypes.byref(opts), descs, len(outs), _stream()))
    return outs if m == DEPTHWISE else outs[0]


def upsample_forward(image, filt, scale, out=None, out_dtype=None, border="clamp"):
    """filter(nearest_upsample(image, scale)) in one pass (u8 images, SHARED):
    returns [N][C][H*scale][W*scale] in the image's layout."""
    lib = load()
    image = _as4(image)
    fd, filt = filter_desc(filt)
    n, c, h, w = image.shape
    if out is None:
        out = _new_out(image, filt, c, h * scale, w * scale, out_dtype, interleaved(image))
    opts = make_opts("shared", EPI_NONE, None, 0, border)
    _check(lib.filter2d_upsample_forward(ctypes.byref(tensor_desc(image)), ctypes.byref(fd), int(scale),
                                         ctypes.byref(opts), ctypes.byref(tensor_desc(_as4(out))), _stream()))
    return out


def forward_separable(image, a, b, rows=None, out=None):
    """Y = filter(X) for the rank-one filter a b^T (FP32, SHARED), on the
    current stream.  a, b: 1-D device tensors of k float32 taps."""
    lib = load()
    image = _as4(image)
    if a.dim() != 1 or b.dim() != 1 or a.numel() != b.numel():
        raise ValueError("a and b must be 1-D with the same length k")
    if a.dtype != torch.float32 or b.dtype != torch.float32 or not a.is_contiguous() or not b.is_contiguous():
        raise ValueError("a and b must be contiguous float32")
    n, c, h, w = image.shape
    r0, r1 = (0, h) if rows is None else rows
    if out is None:
        out = torch.empty((n, c, r1 - r0, w), dtype=torch.float32, device=image.device)
    opts = make_opts("shared", EPI_NONE, (r0, r1))
    _check(lib.filter2d_forward_separable(ctypes.byref(tensor_desc(image)), ctypes.c_void_p(a.data_ptr()),
                                          ctypes.c_void_p(b.data_ptr()), a.numel(), ctypes.byref(opts),
                                          ctypes.byref(tensor_desc(_as4(out))), _stream()))
    return out


def backward_workspace(image, filt, mode="shared"):
    lib = load()
    image = _as4(image)
    fd, filt = filter_desc(filt)
    opts = make_opts(mode)
    return int(lib.filter2d_backward_workspace(ctypes.byref(tensor_desc(image)), ctypes.byref(fd),
                                               ctypes.byref(opts)))


def backward(image, filt, grad_outs, mode="shared", need_input=True, need_filter=True,
             workspace=None, grad_input=None, grad_filter=None):
    """Adjoints of ``forward``: returns (grad_input [N][C][H][W] f32 or None,
    grad_filter f32 shaped like the filter or None).  grad_input / grad_filter
    may be given as preallocated outputs."""
    lib = load()
    image = _as4(image)
    fd, filt4 = filter_desc(filt)
    if isinstance(grad_outs, torch.Tensor):
        grad_outs = [grad_outs]
    grad_outs = [_as4(g) for g in grad_outs]
    opts = make_opts(mode)
    gi, gf = None, None
    if need_input:
        gi = grad_input if grad_input is not None else \
            torch.empty(image.shape, dtype=torch.float32, device=image.device)
    if need_filter:
        gf = grad_filter if grad_filter is not None else \
            torch.empty(filt4.shape, dtype=torch.float32, device=image.device)
        if gf.numel() != filt4.numel() or gf.dtype != torch.float32 or not gf.is_contiguous():
            raise ValueError("grad_filter must be a contiguous float32 tensor with the filter's size")
    ws_bytes = lib.filter2d_backward_workspace(ctypes.byref(tensor_desc(image)), ctypes.byref(fd),
                                               ctypes.byref(opts))
    if workspace is None or workspace.numel() < ws_bytes:
        workspace = torch.empty(max(int(ws_bytes), 1), dtype=torch.uint8, device=image.device)
    gds = (F2dTensor * len(grad_outs))(*[tensor_desc(g) for g in grad_outs])
    gid = ctypes.byref(tensor_desc(gi)) if gi is not None else None
    _check(lib.filter2d_backward(ctypes.byref(tensor_desc(image)), ctypes.byref(fd), gds,
                                 len(grad_outs), ctypes.byref(opts), gid,
                                 ctypes.c_void_p(gf.data_ptr() if gf is not None else 0),
                                 ctypes.c_void_p(workspace.data_ptr()), ws_bytes, _stream()))
    if gf is not None and filt.dim() == 2:
        gf = gf.view(filt.shape)
    return gi, gf


def backward_noalloc(image, filt, grad_outs, mode="shared", need_input=True, need_filter=True,
                     grad_input=None, grad_filter=None):
    """``backward`` through filter2d_backward_noalloc: no workspace argument,
    the library's static per-device scratch is used instead."""
    lib = load()
    image = _as4(image)
    fd, filt4 = filter_desc(filt)
    if isinstance(grad_outs, torch.Tensor):
        grad_outs = [grad_outs]
    grad_outs = [_as4(g) for g in grad_outs]
    opts = make_opts(mode)
    gi, gf = None, None
    if need_input:
        gi = grad_input if grad_input is not None else \
            torch.empty(image.shape, dtype=torch.float32, device=image.device)
    if need_filter:
        gf = grad_filter if grad_filter is not None else \
            torch.empty(filt4.shape, dtype=torch.float32, device=image.device)
        if gf.numel() != filt4.numel() or gf.dtype != torch.float32 or not gf.is_contiguous():
            raise ValueError("grad_filter must be a contiguous float32 tensor with the filter's size")
    gds = (F2dTensor * len(grad_outs))(*[tensor_desc(g) for g in grad_outs])
    gid = ctypes.byref(tensor_desc(gi)) if gi is not None else None
    _check(lib.filter2d_backward_noalloc(ctypes.byref(tensor_desc(image)), ctypes.byref(fd), gds,
                                         len(grad_outs), ctypes.byref(opts), gid,
                                         ctypes.c_void_p(gf.data_ptr() if gf is not None else 0), _stream()))
    if gf is not None and filt.dim() == 2:
        gf = gf.view(filt.shape)
    return gi, gf


def autotune_forward(image, filt, mode="shared", epilogue=EPI_NONE, rows=None, reps=5):
    """Time every tiling variant for these arguments, record and return the best."""
    lib = load()
    image = _as4(image)
    fd, filt = filter_desc(filt)
    m = _MODES[mode] if isinstance(mode, str) else int(mode)
    n, c, h, w = image.shape
    r0, r1 = (0, h) if rows is None else rows
    odt = torch.int32 if image.dtype == torch.uint8 else torch.float32
    co = filt.size(0) if m == BANK else c
    outs = [torch.empty((n, co, r1 - r0, w), dtype=odt, device=image.device)
            for _ in range(out_count(m, filt.shape, c, epilogue))]
    descs = (F2dTensor * len(outs))(*[tensor_desc(_as4(o)) for o in outs])
    best = ctypes.c_int32(0)
    _check(lib.filter2d_autotune_forward(ctypes.byref(tensor_desc(image)), ctypes.byref(fd),
                                         ctypes.byref(make_opts(m, epilogue, (r0, r1))), descs,
                                         len(outs), reps, _stream(), ctypes.byref(best)))
    return best.value


def variant_count(path):
    return int(load().filter2d_variant_count(path))


def tune_save(path):
    _check(load().filter2d_tune_save(path.encode()))


def tune_load(path):
    _check(load().filter2d_tune_load(path.encode()))


def tune_clear():
    load().filter2d_tune_clear()


class RaggedBatch:
    """Descriptor table + tile plan (prefix sums and tag) for ``filter2d_batched``,
    resident on the device.

    images / outs: lists of [C][H][W] tensors (float32, column stride 1);
    filters: list of [K][K] float32 tensors (one per image)."""

    def __init__(self, images, outs, filters, variant=0, k=3):
        lib = load()
        if not (len(images) == len(outs) == len(filters)):
            raise ValueError("images, outs and filters must have the same length")
        self.k = int(filters[0].shape[-1]) if filters else int(k)
        self.images, self.outs, self.filters = images, outs, filters
        n = len(images)
        items = (F2dBatchItem * max(n, 1))()
        for i, (x, y, f) in enumerate(zip(images, outs, filters)):
            if x.dim() != 3 or y.shape != x.shape or not f.is_contiguous():
                raise ValueError(f"item {i}: expected [C][H][W] images/outs and a contiguous filter")
            items[i] = F2dBatchItem(x.data_ptr(), y.data_ptr(), f.data_ptr(), x.size(0), x.size(1),
                                    x.size(2), x.stride(0), x.stride(1), y.stride(0), y.stride(1))
        self.items_host = items
        self.n = n
        prefix = (ctypes.c_int64 * (n + 2))()  # prefix sums + the plan's tag word
        var = ctypes.c_int32(variant)
        total = lib.filter2d_batched_plan(items, n, F32, self.k, ctypes.byref(var), prefix)
        if total < 0:
            _check(int(-total))
        self.total_tiles = int(total)
        self.variant = var.value
        dev = images[0].device if n else torch.device("cuda")
        raw = bytes(memoryview(items)) if n else b""
        self.items_dev = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(dev) if n else \
            torch.empty(1, dtype=torch.uint8, device=dev)
        self.prefix_host = [prefix[i] for i in range(n + 2)]
        self.prefix_dev = torch.tensor(self.prefix_host, dtype=torch.int64, device=dev)

    def run(self, variant=None, k=None):
        """Launch on the current stream.  variant / k default to the planned
        ones (others are only for testing the device-side plan check)."""
        lib = load()
        opts = make_opts("shared", variant=self.variant if variant is None else variant)
        _check(lib.filter2d_batched(ctypes.c_void_p(self.items_dev.data_ptr()),
                                    ctypes.c_void_p(self.prefix_dev.data_ptr()), self.n,
                                    self.total_tiles, F32, self.k if k is None else k,
                                    ctypes.byref(opts), _stream()))

    def autotune(self, reps=3):
        lib = load()
        best = ctypes.c_int32(0)
        _check(lib.filter2d_autotune_batched(self.items_host, ctypes.c_void_p(self.items_dev.data_ptr()),
                                             self.n, F32, self.k,
                                             ctypes.c_void_p(self.prefix_dev.data_ptr()), reps,
                                             _stream(), ctypes.byref(best)))
        # the plan depends on the tile shape: re-plan with the chosen variant
        self.__init__(self.images, self.outs, self.filters, best.value, self.k)
        return best.value
