"""Plain FP64 / INT64 CPU oracle for the clamp-to-edge K x K 2D filter.

TEST INFRASTRUCTURE ONLY.  Imported by ``tests/``, by the smoke check and by
the benchmark's CPU-baseline leg; the GPU library never imports it and it
imports nothing from the GPU library.

The arithmetic lives in ``oracle.c`` (direct loops, binary64 / int64); this
module only marshals numpy arrays.  What is computed (generalising the paper's
3x3 Laplacian sharpen, Section 4.2.4, and the grayscale weighting of
Section 4.2.5):

* forward:      Y[n][o][y][x] = sum_{i in inputs(o)} sum_{u,v} F[o|i][u][v] *
                                X[n][i][cl_H(y+u-r)][cl_W(x+v-r)]
                (binary64, int64, or binary32 in a stated order; clamp-to-edge
                or zero borders; 8-bit outputs by clamping and rounding)
* upsample:     nearest-neighbour, integer factor (Section 4.2.3)
* grad_input:   the adjoint of the forward map in X, in scatter form
* grad_filter:  the adjoint in F, with Neumaier compensated summation

Channel modes: SHARED (one filter for every channel), DEPTHWISE (filter
[C*m][1][K][K], output channel c*m+j reads channel c), BANK (filter
[C_out][C_in][K][K], output channel o sums over all input channels).
"""
import ctypes
import os

import numpy as np

SHARED, DEPTHWISE, BANK = 0, 1, 2
_MODES = {"shared": SHARED, "depthwise": DEPTHWISE, "bank": BANK}

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64 = ctypes.c_int64
_i32 = ctypes.c_int32
_dp = ctypes.POINTER(ctypes.c_double)
_lp = ctypes.POINTER(ctypes.c_int64)
_fp = ctypes.POINTER(ctypes.c_float)
_bp = ctypes.POINTER(ctypes.c_uint8)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build

        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    lib.oracle_forward_f64.argtypes = [_dp, _i64, _i64, _i64, _i64, _dp, _i64, _i64, _i64, _i32,
                                       _i64, _i64, _dp]
    lib.oracle_forward_zero_f64.argtypes = [_dp, _i64, _i64, _i64, _i64, _dp, _i64, _i64, _i64,
                                            _i32, _i64, _i64, _dp]
    lib.oracle_forward_i64.argtypes = [_lp, _i64, _i64, _i64, _i64, _lp, _i64, _i64, _i64, _i32,
                                       _i64, _i64, _lp]
    lib.oracle_forward_zero_i64.argtypes = [_lp, _i64, _i64, _i64, _i64, _lp, _i64, _i64, _i64, _i32,
                                            _i64, _i64, _lp]
    lib.oracle_forward_f32fma.argtypes = [_fp, _i64, _i64, _i64, _i64, _fp, _i64, _i64, _i64, _i32,
                                          _i32, _fp]
    lib.oracle_u8_from_f32.argtypes = [_fp, _i64, _bp]
    lib.oracle_u8_from_i64.argtypes = [_lp, _i64, _bp]
    lib.oracle_sumsq_i64.argtypes = [_lp, _lp, _i64, _lp]
    lib.oracle_grad_input_f64.argtypes = [_dp, _i64, _i64, _i64, _i64, _dp, _i64, _i64, _i64,
                                          _i32, _dp]
    lib.oracle_grad_filter_f64.argtypes = [_dp, _dp, _i64, _i64, _i64, _i64, _i64, _i64, _i64,
                                           _i32, _dp]
    for name in ("oracle_forward_f64", "oracle_forward_zero_f64", "oracle_forward_i64", "oracle_sumsq_i64",
                 "oracle_forward_zero_i64", "oracle_forward_f32fma", "oracle_u8_from_f32", "oracle_u8_from_i64",
                 "oracle_grad_input_f64", "oracle_grad_filter_f64", "oracle_num_threads"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def num_threads():
    """OpenMP threads the oracle runs on."""
    return int(_load().oracle_num_threads())


def _mode(mode):
    return _MODES[mode] if isinstance(mode, str) else int(mode)


def _as4(a):
    a = np.asarray(a)
    if a.ndim == 2:
        a = a[None, None]
    elif a.ndim == 3:
        a = a[None]
    if a.ndim != 4:
        raise ValueError("expected a [N][C][H][W] array")
    return a


def _filt4(f):
    f = np.asarray(f)
    if f.ndim == 2:
        f = f[None, None]
    if f.ndim != 4 or f.shape[2] != f.shape[3]:
        raise ValueError("expected a [FO][FI][K][K] filter")
    return f


def _out_channels(C, FO, mode):
    return C if mode == SHARED else FO


def forward(x, f, mode="shared", rows=None, border="clamp"):
    """FP64 forward filter.  x: [N][C][H][W] (or [H][W]); f: [FO][FI][K][K] (or [K][K]).
    rows=(y0, y1) restricts the output to rows y0..y1-1 (clamping is still done
    with respect to the whole array).  border="zero": out-of-image neighbours
    contribute nothing (the paper's sharpen, Section 4.2.4).  Returns float64
    [N][C_out][y1-y0][W]."""
    if border not in ("clamp", "zero"):
        raise ValueError("border must be 'clamp' or 'zero'")
    m = _mode(mode)
    x = np.ascontiguousarray(_as4(x), dtype=np.float64)
    f = np.ascontiguousarray(_filt4(f), dtype=np.float64)
    N, C, H, W = x.shape
    FO, FI, K, _ = f.shape
    y0, y1 = (0, H) if rows is None else rows
    out = np.empty((N, _out_channels(C, FO, m), y1 - y0, W), np.float64)
    fn = _load().oracle_forward_f64 if border == "clamp" else _load().oracle_forward_zero_f64
    rc = fn(x.ctypes.data_as(_dp), N, C, H, W, f.ctypes.data_as(_dp), FO, FI, K, m, y0, y1,
            out.ctypes.data_as(_dp))
    if rc != 0:
        raise ValueError("oracle forward: invalid arguments")
    return out


def forward_int(x, f, mode="shared", rows=None, border="clamp"):
    """Exact int64 forward filter (the integer path); border "clamp" or "zero"."""
    if border not in ("clamp", "zero"):
        raise ValueError("border must be 'clamp' or 'zero'")
    m = _mode(mode)
    x = np.ascontiguousarray(_as4(x), dtype=np.int64)
    f = np.ascontiguousarray(_filt4(f), dtype=np.int64)
    N, C, H, W = x.shape
    FO, FI, K, _ = f.shape
    y0, y1 = (0, H) if rows is None else rows
    out = np.empty((N, _out_channels(C, FO, m), y1 - y0, W), np.int64)
    fn = _load().oracle_forward_i64 if border == "clamp" else _load().oracle_forward_zero_i64
    rc = fn(x.ctypes.data_as(_lp), N, C, H, W, f.ctypes.data_as(_lp), FO, FI, K, m, y0, y1,
            out.ctypes.data_as(_lp))
    if rc != 0:
        raise ValueError("oracle integer forward: invalid arguments")
    return out


def forward_f32(x, f, mode="shared", border="clamp"):
    """The forward sum in binary32 in a fixed order (accumulator +0, one fused
    multiply-add per term: input channel, tap row, tap column), the precision
    of the paper's float filter taps (Section 4.2.4).  x is converted to
    float32 (exact for 8-bit values).  Returns float32 [N][C_out][H][W]."""
    if border not in ("clamp", "zero"):
        raise ValueError("border must be 'clamp' or 'zero'")
    m = _mode(mode)
    x = np.ascontiguousarray(_as4(x), dtype=np.float32)
    f = np.ascontiguousarray(_filt4(f), dtype=np.float32)
    N, C, H, W = x.shape
    FO, FI, K, _ = f.shape
    out = np.empty((N, _out_channels(C, FO, m), H, W), np.float32)
    rc = _load().oracle_forward_f32fma(x.ctypes.data_as(_fp), N, C, H, W, f.ctypes.data_as(_fp), FO, FI,
                                       K, m, 1 if border == "zero" else 0, out.ctypes.data_as(_fp))
    if rc != 0:
        raise ValueError("oracle_forward_f32fma: invalid arguments")
    return out


def to_u8(a):
    """8-bit image from sums: float32 sums are clamped to [0, 255] and rounded
    to nearest, ties to even; integer sums are clamped."""
    a = np.asarray(a)
    if a.dtype.kind == "f":
        src = np.ascontiguousarray(a, dtype=np.float32)
        out = np.empty(src.shape, np.uint8)
        _load().oracle_u8_from_f32(src.ctypes.data_as(_fp), src.size, out.ctypes.data_as(_bp))
    else:
        src = np.ascontiguousarray(a, dtype=np.int64)
        out = np.empty(src.shape, np.uint8)
        _load().oracle_u8_from_i64(src.ctypes.data_as(_lp), src.size, out.ctypes.data_as(_bp))
    return out


def upsample_nearest(x, s):
    """Nearest-neighbour upsampling by an integer factor s >= 1 (the paper's
    upsampling, Section 4.2.3): output pixel (Y, X) copies input pixel
    (Y // s, X // s); the output is s times taller and wider."""
    s = int(s)
    if s < 1:
        raise ValueError("scale must be >= 1")
    x = np.asarray(x)
    H, W = x.shape[-2], x.shape[-1]
    ys = np.arange(H * s) // s
    xs = np.arange(W * s) // s
    return x[..., ys[:, None], xs[None, :]]


def sumsq(a, b):
    """Exact int64 a^2 + b^2 (gradient magnitude without the square root)."""
    a = np.ascontiguousarray(a, dtype=np.int64)
    b = np.ascontiguousarray(b, dtype=np.int64)
    if a.shape != b.shape:
        raise ValueError("shape mismatch")
    out = np.empty_like(a)
    _load().oracle_sumsq_i64(a.ctypes.data_as(_lp), b.ctypes.data_as(_lp), a.size,
                             out.ctypes.data_as(_lp))
    return out


def grad_input(g, f, image_shape, mode="shared"):
    """FP64 adjoint of ``forward`` in the image: returns [N][C][H][W]."""
    m = _mode(mode)
    g = np.ascontiguousarray(_as4(g), dtype=np.float64)
    f = np.ascontiguousarray(_filt4(f), dtype=np.float64)
    N, C, H, W = image_shape
    FO, FI, K, _ = f.shape
    if g.shape != (N, _out_channels(C, FO, m), H, W):
        raise ValueError("grad_output shape does not match the forward output")
    gx = np.empty((N, C, H, W), np.float64)
    rc = _load().oracle_grad_input_f64(g.ctypes.data_as(_dp), N, C, H, W, f.ctypes.data_as(_dp),
                                       FO, FI, K, m, gx.ctypes.data_as(_dp))
    if rc != 0:
        raise ValueError("oracle_grad_input_f64: invalid arguments")
    return gx


def grad_filter(x, g, filter_shape, mode="shared"):
    """FP64 adjoint of ``forward`` in the filter (Neumaier summation): [FO][FI][K][K]."""
    m = _mode(mode)
    x = np.ascontiguousarray(_as4(x), dtype=np.float64)
    g = np.ascontiguousarray(_as4(g), dtype=np.float64)
    N, C, H, W = x.shape
    FO, FI, K = filter_shape[0], filter_shape[1], filter_shape[2]
    if g.shape != (N, _out_channels(C, FO, m), H, W):
        raise ValueError("grad_output shape does not match the forward output")
    gf = np.empty((FO, FI, K, K), np.float64)
    rc = _load().oracle_grad_filter_f64(x.ctypes.data_as(_dp), g.ctypes.data_as(_dp), N, C, H, W,
                                        FO, FI, K, m, gf.ctypes.data_as(_dp))
    if rc != 0:
        raise ValueError("oracle_grad_filter_f64: invalid arguments")
    return gf


def rel_l2(a, ref):
    """||a - ref||_2 / ||ref||_2 accumulated in FP64 (the acceptance metric)."""
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = float(np.sqrt(np.sum(ref * ref)))
    num = float(np.sqrt(np.sum((a - ref) ** 2)))
    return num / den if den > 0 else num
