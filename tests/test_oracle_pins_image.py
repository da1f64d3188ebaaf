"""Pins of the oracle's image-path pieces: nearest upsampling (Section 4.2.3),
zero-border integer sums, the binary32 fused multiply-add chain used for the
paper's float taps, and the conversion to 8-bit outputs (the sharpen of
Section 4.2.4 and the grayscale of Section 4.2.5 on 8-bit images).

Each is checked against something other than itself: numpy's repeat, scipy's
zero-padded correlation, exact integer arithmetic, an exactly rounded
brute-force evaluation with rational numbers, closed forms on constant and
impulse images, and hand-worked values.
"""
from fractions import Fraction

import numpy as np
import pytest
import scipy.ndimage as nd

import oracle
from paper_2504_01266_amd import workloads as wl


def _rng(*ids):
    return np.random.default_rng([91, *ids])


# ------------------------------------------------------------ upsampling ----
@pytest.mark.parametrize("s", [1, 2, 3, 5, 20])
@pytest.mark.parametrize("shape", [(1, 1, 1, 1), (1, 3, 4, 5), (2, 2, 3, 7)])
def test_upsample_equals_repeat_along_both_axes(s, shape):
    x = _rng(1, s, *shape).integers(0, 256, shape, dtype=np.uint8)
    want = np.repeat(np.repeat(x, s, axis=2), s, axis=3)
    got = oracle.upsample_nearest(x, s)
    assert got.shape == (shape[0], shape[1], shape[2] * s, shape[3] * s)
    assert got.dtype == x.dtype
    assert np.array_equal(got, want)


def test_upsample_source_is_the_floor_of_the_scaled_coordinate():
    """Output (Y, X) copies input (Y // s, X // s): on an image whose value
    encodes its coordinates, every output decodes to the floored source."""
    h, w, s = 6, 9, 4
    x = (np.arange(h)[:, None] * 100 + np.arange(w)[None, :]).astype(np.int64)
    up = oracle.upsample_nearest(x, s)
    yy, xx = np.meshgrid(np.arange(h * s), np.arange(w * s), indexing="ij")
    assert np.array_equal(up // 100, yy // s)
    assert np.array_equal(up % 100, xx // s)


def test_upsample_rejects_scale_below_one():
    with pytest.raises(ValueError):
        oracle.upsample_nearest(np.zeros((2, 2)), 0)


# ------------------------------------------------ zero-border int64 path ----
def _scipy_zero(x, f, mode):
    n_, c_ = x.shape[:2]
    outs = []
    for n in range(n_):
        planes = []
        if mode == "shared":
            planes = [nd.correlate(x[n, c], f[0, 0], mode="constant", cval=0) for c in range(c_)]
        elif mode == "depthwise":
            m = f.shape[0] // c_
            planes = [nd.correlate(x[n, o // m], f[o, 0], mode="constant", cval=0) for o in range(f.shape[0])]
        else:
            planes = [sum(nd.correlate(x[n, i], f[o, i], mode="constant", cval=0) for i in range(c_))
                      for o in range(f.shape[0])]
        outs.append(np.stack(planes))
    return np.stack(outs)


@pytest.mark.parametrize("mode", ["shared", "depthwise", "bank"])
@pytest.mark.parametrize("k", [1, 3, 5, 7])
def test_zero_border_int_equals_scipy(mode, k):
    r = _rng(2, k)
    x = r.integers(0, 256, (2, 3, 9, 11)).astype(np.int64)
    f = {"shared": r.integers(-9, 10, (1, 1, k, k)), "depthwise": r.integers(-9, 10, (6, 1, k, k)),
         "bank": r.integers(-9, 10, (2, 3, k, k))}[mode].astype(np.int64)
    got = oracle.forward_int(x, f, mode, border="zero")
    assert np.array_equal(got, _scipy_zero(x, f, mode))


# ------------------------------------------------ binary32 FMA chain --------
@pytest.mark.parametrize("border", ["clamp", "zero"])
@pytest.mark.parametrize("mode", ["shared", "depthwise", "bank"])
def test_f32_chain_with_integer_taps_is_exact(border, mode):
    """Integer taps on 8-bit values: every partial sum is an integer below
    2^24, so the binary32 chain is exact in any order and equals int64."""
    r = _rng(3, ["clamp", "zero"].index(border), ["shared", "depthwise", "bank"].index(mode))
    x = r.integers(0, 256, (1, 3, 13, 10), dtype=np.uint8)
    f = {"shared": r.integers(-8, 9, (1, 1, 5, 5)), "depthwise": r.integers(-8, 9, (6, 1, 5, 5)),
         "bank": r.integers(-8, 9, (2, 3, 5, 5))}[mode]
    got = oracle.forward_f32(x, f.astype(np.float32), mode, border=border)
    want = oracle.forward_int(x, f, mode, border=border)
    assert np.array_equal(got.astype(np.int64), want)


@pytest.mark.parametrize("border", ["clamp", "zero"])
def test_f32_chain_is_within_the_error_bound_of_the_exact_sum(border):
    """A recursive sum of n fused products has error <= n u sum|terms|
    (u = 2^-24); a dropped or doubled term would be off by a whole term."""
    r = _rng(4, ["clamp", "zero"].index(border))
    x = r.integers(0, 256, (1, 3, 17, 19), dtype=np.uint8)
    f = (r.standard_normal((2, 3, 5, 5)) * 0.3).astype(np.float32)
    got = oracle.forward_f32(x, f, "bank", border=border).astype(np.float64)
    exact = oracle.forward(x.astype(np.float64), f.astype(np.float64), "bank", border=border)
    mag = oracle.forward(x.astype(np.float64), np.abs(f).astype(np.float64), "bank", border=border)
    n = 3 * 25
    assert np.all(np.abs(got - exact) <= n * 2.0 ** -24 * mag + 1e-30)
    assert np.max(np.abs(got - exact)) > 0  # the sample does exercise rounding


def _round_f32(q):
    """The binary32 value nearest to the rational q, ties to even (brute force
    over the neighbours of numpy's conversion of the nearest double)."""
    c = np.float32(float(q))
    best = None
    for cand in (np.nextafter(c, np.float32(-np.inf)), c, np.nextafter(c, np.float32(np.inf))):
        d = abs(Fraction(float(cand)) - q)
        key = (d, int(cand.view(np.uint32)) & 1)  # ties: even significand first
        if best is None or key < best[0]:
            best = (key, cand)
    return best[1]


def _fma32(a, b, c):
    return _round_f32(Fraction(float(a)) * Fraction(float(b)) + Fraction(float(c)))


def test_f32_chain_is_the_stated_fused_order_brute_force():
    """Tiny cases evaluated exactly with rationals, one correctly rounded
    fused multiply-add per term in the stated order (input channel, tap row,
    tap column), clamp-to-edge and zero borders.  The sample is chosen so that
    separate multiply and add, or another term order, give different values."""
    r = _rng(5)
    h, w, k, c = 3, 4, 3, 2
    x = r.integers(0, 256, (1, c, h, w), dtype=np.uint8)
    f = (r.standard_normal((1, c, k, k)) * np.float32(1.37)).astype(np.float32)
    rr = k // 2
    for border in ("clamp", "zero"):
        got = oracle.forward_f32(x, f, "bank", border=border)
        alt_order = np.zeros_like(got)
        unfused = np.zeros_like(got)
        for y in range(h):
            for xx in range(w):
                acc = np.float32(0.0)
                terms = []
                for i in range(c):
                    for u in range(k):
                        for v in range(k):
                            sy, sx = y + u - rr, xx + v - rr
                            if border == "zero" and not (0 <= sy < h and 0 <= sx < w):
                                continue
                            sy, sx = min(max(sy, 0), h - 1), min(max(sx, 0), w - 1)
                            terms.append((f[0, i, u, v], np.float32(x[0, i, sy, sx])))
                for a, b in terms:
                    acc = _fma32(a, b, acc)
                assert got[0, 0, y, xx] == acc, (border, y, xx)
                acc2 = np.float32(0.0)
                for a, b in reversed(terms):
                    acc2 = _fma32(a, b, acc2)
                alt_order[0, 0, y, xx] = acc2
                acc3 = np.float32(0.0)
                for a, b in terms:
                    acc3 = np.float32(acc3 + np.float32(a * b))
                unfused[0, 0, y, xx] = acc3
        assert not np.array_equal(alt_order, got)
        assert not np.array_equal(unfused, got)


# ------------------------------------------------------- 8-bit outputs ------
def test_u8_conversion_hand_values():
    vals = np.array([0.0, -0.0, -3.0, 0.49999997, 0.5, 1.5, 2.5, 3.5, 254.5, 254.50002,
                     255.0, 255.5, 300.7, 1e30, -1e30], np.float32)
    want = [0, 0, 0, 0, 0, 2, 2, 4, 254, 255, 255, 255, 255, 255, 0]
    assert oracle.to_u8(vals).tolist() == want
    ints = np.array([-5, 0, 7, 255, 256, 2040], np.int64)
    assert oracle.to_u8(ints).tolist() == [0, 0, 7, 255, 255, 255]


@pytest.mark.parametrize("v", [0, 40, 51, 85, 100, 255])
def test_paper_sharpen_on_a_constant_u8_image(v):
    """Section 4.2.4: Laplacian (8 centre, -1 around), out-of-image
    neighbours skipped.  A constant image v gives 0 inside, 8v - 5v = 3v on an
    edge and 8v - 3v = 5v at a corner, saturated to 255."""
    x = np.full((1, 3, 6, 7), v, np.uint8)
    lap = wl.LAPLACIAN_8.astype(np.float32)
    for sums in (oracle.forward_f32(x, lap, border="zero"), oracle.forward_int(x, wl.LAPLACIAN_8, border="zero")):
        y = oracle.to_u8(sums)
        assert np.all(y[:, :, 1:-1, 1:-1] == 0)
        assert np.all(y[:, :, 0, 1:-1] == min(3 * v, 255)) and np.all(y[:, :, 1:-1, -1] == min(3 * v, 255))
        assert np.all(y[:, :, [0, 0, -1, -1], [0, -1, 0, -1]] == min(5 * v, 255))


def test_paper_sharpen_on_an_impulse():
    """One bright pixel p on a background b (interior): the centre gets
    8p - 8b, its eight neighbours 8b - 7b - p = b - p, everything else 0."""
    b, p = 20, 200
    x = np.full((1, 1, 9, 9), b, np.uint8)
    x[0, 0, 4, 4] = p
    s = oracle.forward_f32(x, wl.LAPLACIAN_8.astype(np.float32), border="zero")[0, 0]
    assert s[4, 4] == 8 * p - 8 * b
    ring = s[3:6, 3:6].copy()
    ring[1, 1] = b - p
    assert np.all(ring == b - p)
    y = oracle.to_u8(s)
    assert y[4, 4] == 255 and np.all(y[3:6, 3:6][np.arange(3) != 1]) == 0
    assert np.all(y[1:-1, 1:-1][s[1:-1, 1:-1] == 0] == 0)


def test_paper_grayscale_on_u8_in_binary32():
    """Section 4.2.5's weights (R, G, B) as a 3 -> 1 bank with K = 1: a gray
    pixel (r = g = b = v) maps back to v for every v, and every output is the
    exactly rounded weighted sum except where that sum is within 1e-4 of a
    rounding tie."""
    v = np.arange(256, dtype=np.uint8)
    gray = np.broadcast_to(v[None, None, None, :], (1, 3, 1, 256)).copy()
    wts = wl.GRAY_RGB.astype(np.float32).reshape(1, 3, 1, 1)
    assert np.array_equal(oracle.to_u8(oracle.forward_f32(gray, wts, "bank"))[0, 0, 0], v)
    x = _rng(6).integers(0, 256, (2, 3, 31, 37), dtype=np.uint8)
    s32 = oracle.forward_f32(x, wts, "bank")
    s64 = oracle.forward(x.astype(np.float64), wts.astype(np.float64), "bank")
    assert np.all(np.abs(s32 - s64) <= 3 * 2.0 ** -24 * s64 + 1e-6)
    near_tie = np.abs(s64 - np.floor(s64) - 0.5) < 1e-4
    assert np.array_equal(oracle.to_u8(s32)[~near_tie], np.rint(s64)[~near_tie].astype(np.uint8))
