"""Pins of the CPU oracle against facts fixed by the mathematics and the paper.

None of these re-types the oracle's loops: each checks it against a closed
form, an invariant, a library routine (scipy's clamp-to-edge correlation,
numpy's edge padding, math.fsum) or a brute-force dense matrix, chosen so that
a dropped term, a wrong sign or index, a transposed operand or a wrong border
rule fails at least one of them.
"""
import math

import numpy as np
import pytest
import scipy.ndimage as nd

import oracle
from paper_2504_01266_amd import workloads as wl

SHAPES = [(1, 1, 1, 1), (1, 1, 1, 7), (1, 1, 6, 1), (1, 2, 2, 3), (2, 1, 5, 7), (1, 3, 9, 8)]
KS = [1, 3, 5, 7]


def _rng(*ids):
    return np.random.default_rng([77, *ids])


def _filter(mode, c, k, r, m=2, cout=3):
    if mode == "shared":
        return r.standard_normal((1, 1, k, k))
    if mode == "depthwise":
        return r.standard_normal((c * m, 1, k, k))
    return r.standard_normal((cout, c, k, k))


def _scipy_forward(x, f, mode):
    """The forward map assembled from scipy.ndimage.correlate(mode='nearest'),
    which replicates the edge pixel: the textbook clamp-to-edge correlation."""
    n_, c_, h_, w_ = x.shape
    outs = []
    for n in range(n_):
        planes = []
        if mode == "shared":
            for c in range(c_):
                planes.append(nd.correlate(x[n, c], f[0, 0], mode="nearest"))
        elif mode == "depthwise":
            m = f.shape[0] // c_
            for o in range(f.shape[0]):
                planes.append(nd.correlate(x[n, o // m], f[o, 0], mode="nearest"))
        else:
            for o in range(f.shape[0]):
                planes.append(sum(nd.correlate(x[n, i], f[o, i], mode="nearest")
                                  for i in range(c_)))
        outs.append(np.stack(planes))
    return np.stack(outs)


# ---------------------------------------------------------------- pin: scipy --
@pytest.mark.parametrize("mode", ["shared", "depthwise", "bank"])
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("k", KS)
def test_forward_equals_scipy_nearest_correlation(mode, shape, k):
    r = _rng(1, k, *shape)
    x = r.random(shape)
    f = _filter(mode, shape[1], k, r)
    y = oracle.forward(x, f, mode)
    ref = _scipy_forward(x, f, mode)
    assert y.shape == ref.shape
    np.testing.assert_allclose(y, ref, rtol=1e-13, atol=1e-13)


# ------------------------------------------------------- pin 1: identity ----
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("k", KS)
def test_identity_kernel(shape, k):
    x = _rng(2, k, *shape).random(shape)
    f = np.zeros((k, k))
    f[k // 2, k // 2] = 1.0
    assert np.array_equal(oracle.forward(x, f), x)
    # bank with the identity on the diagonal reproduces every channel
    c = shape[1]
    fb = np.zeros((c, c, k, k))
    for i in range(c):
        fb[i, i, k // 2, k // 2] = 1.0
    assert np.array_equal(oracle.forward(x, fb, "bank"), x)


# ------------------------------------------------ pin 2: constant image ----
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("k", [3, 5, 9])
def test_constant_image_everywhere(shape, k):
    """Clamp-to-edge keeps a constant image constant under any filter, borders
    and corners included: Y = c * sum(F).  Zero padding would fail here."""
    c = 0.375
    f = _rng(3, k).standard_normal((k, k))
    y = oracle.forward(np.full(shape, c), f)
    np.testing.assert_allclose(y, c * f.sum(), rtol=1e-13, atol=1e-14)


# ------------------------------------------------------ pin 3: box count ----
@pytest.mark.parametrize("hw", [(1, 1), (2, 3), (7, 5), (12, 13)])
@pytest.mark.parametrize("k", [1, 3, 5, 9])
def test_box_on_integer_constant_counts_every_tap(hw, k):
    y = oracle.forward(np.full((1, 1) + hw, 3.0), np.ones((k, k)))
    assert np.all(y == 3.0 * k * k)
    yi = oracle.forward_int(np.full((1, 1) + hw, 3), np.ones((k, k), np.int64))
    assert np.all(yi == 3 * k * k)


# ------------------------------------------------------ pin 4: linearity ----
@pytest.mark.parametrize("mode", ["shared", "depthwise", "bank"])
def test_linearity_in_image_and_filter(mode):
    r = _rng(4)
    x, z = r.random((2, 3, 9, 11)), r.random((2, 3, 9, 11))
    f, h = _filter(mode, 3, 5, r), _filter(mode, 3, 5, r)
    a, b = 1.75, -0.5
    lhs = oracle.forward(a * x + b * z, f, mode)
    rhs = a * oracle.forward(x, f, mode) + b * oracle.forward(z, f, mode)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12, atol=1e-12)
    lhs = oracle.forward(x, a * f + b * h, mode)
    rhs = a * oracle.forward(x, f, mode) + b * oracle.forward(x, h, mode)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-12, atol=1e-12)


# ------------------------------------------------------ pin 5: separable ----
def _pass_1d(img, taps, axis):
    """One 1D clamp-to-edge correlation pass built from numpy edge padding."""
    r = (len(taps) - 1) // 2
    pad = [(0, 0)] * img.ndim
    pad[axis] = (r, r)
    p = np.pad(img, pad, mode="edge")
    out = np.zeros_like(img, dtype=np.float64)
    n = img.shape[axis]
    for t, w in enumerate(taps):
        out += w * np.take(p, np.arange(t, t + n), axis=axis)
    return out


@pytest.mark.parametrize("hw", [(1, 1), (3, 2), (16, 9), (33, 40)])
@pytest.mark.parametrize("k", [3, 5, 7])
def test_separable_equals_two_1d_passes(hw, k):
    r = _rng(5, k, *hw)
    a, b = r.standard_normal(k), r.standard_normal(k)
    x = r.random(hw)
    y = oracle.forward(x, np.outer(a, b))[0, 0]
    ref = _pass_1d(_pass_1d(x, b, axis=1), a, axis=0)
    np.testing.assert_allclose(y, ref, rtol=1e-12, atol=1e-12)


def test_plain_gaussian_taps_are_the_separable_gaussian():
    """The 5x5 sigma=1 taps: FP32 rounding of the separable FP64 product."""
    d = np.arange(-2, 3, dtype=np.float64)
    g = np.exp(-d * d / 2.0)
    g /= g.sum()
    t = wl.gaussian_taps(5, 1.0)
    assert t.dtype == np.float32
    np.testing.assert_allclose(t.astype(np.float64), np.outer(g, g), rtol=2 ** -24)
    assert abs(float(t.astype(np.float64).sum()) - 1.0) < 1e-6
    x = _rng(5, 99).random((24, 31))
    y = oracle.forward(x, t.astype(np.float64))[0, 0]
    ref = _pass_1d(_pass_1d(x, g, axis=1), g, axis=0)
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-6)


# -------------------------------------------------------- pin 6: adjoint ----
@pytest.mark.parametrize("mode", ["shared", "depthwise", "bank"])
@pytest.mark.parametrize("shape", SHAPES + [(1, 2, 3, 2)])
@pytest.mark.parametrize("k", [1, 3, 5, 9])
def test_adjoint_identity(mode, shape, k):
    r = _rng(6, k, *shape)
    x = r.standard_normal(shape)
    f = _filter(mode, shape[1], k, r)
    y = oracle.forward(x, f, mode)
    g = r.standard_normal(y.shape)
    lhs = float(np.sum(y * g))
    gx = oracle.grad_input(g, f, shape, mode)
    assert abs(lhs - float(np.sum(x * gx))) <= 1e-13 * max(1.0, np.abs(y * g).sum())
    gf = oracle.grad_filter(x, g, f.shape, mode)
    assert abs(lhs - float(np.sum(f * gf))) <= 1e-13 * max(1.0, np.abs(y * g).sum())


# ------------------------------------------------ pin 7: dense brute force --
def _dense(h, w, f2):
    """A[(y,x),(p,q)] = sum_{u,v} F[u][v] [clip(y+u-r)=p][clip(x+v-r)=q]."""
    k = f2.shape[0]
    r = (k - 1) // 2
    a = np.zeros((h * w, h * w))
    for y in range(h):
        for x in range(w):
            for u in range(k):
                for v in range(k):
                    p = int(np.clip(y + u - r, 0, h - 1))
                    q = int(np.clip(x + v - r, 0, w - 1))
                    a[y * w + x, p * w + q] += f2[u, v]
    return a


@pytest.mark.parametrize("hw", [(1, 1), (1, 4), (4, 1), (2, 2), (3, 5), (6, 6), (5, 3)])
@pytest.mark.parametrize("k", [1, 3, 5])
def test_dense_matrix_brute_force(hw, k):
    h, w = hw
    r = _rng(7, k, h, w)
    f2 = r.integers(-4, 5, (k, k)).astype(np.float64)
    x = r.integers(-9, 10, (h, w)).astype(np.float64)
    g = r.integers(-9, 10, (h, w)).astype(np.float64)
    a = _dense(h, w, f2)
    assert np.array_equal(oracle.forward(x, f2)[0, 0].ravel(), a @ x.ravel())
    assert np.array_equal(oracle.grad_input(g[None, None], f2, (1, 1, h, w))[0, 0].ravel(),
                          a.T @ g.ravel())
    # grad_filter by explicit sums: derivative of <A(F) x, g> in F[u][v]
    gf = oracle.grad_filter(x, g, (1, 1, k, k))[0, 0]
    for u in range(k):
        for v in range(k):
            e = np.zeros((k, k))
            e[u, v] = 1.0
            assert gf[u, v] == g.ravel() @ (_dense(h, w, e) @ x.ravel())


# -------------------------------------------------- pin 8: Sobel closed form --
@pytest.mark.parametrize("hw", [(2, 2), (3, 7), (8, 9), (17, 5)])
def test_sobel_on_a_ramp(hw):
    h, w = hw
    a, b = 2, 3
    yy, xx = np.mgrid[0:h, 0:w]
    img = (a * xx + b * yy).astype(np.int64)
    assert img.max() <= 255
    f = wl.sobel_depthwise(1).astype(np.int64)
    out = oracle.forward_int(img[None, None], f, "depthwise")[0]
    gx, gy = out[0], out[1]
    ex = np.full((h, w), 8 * a)
    ex[:, 0] = ex[:, -1] = 4 * a
    ey = np.full((h, w), 8 * b)
    ey[0, :] = ey[-1, :] = 4 * b
    assert np.array_equal(gx, ex) and np.array_equal(gy, ey)
    m = oracle.sumsq(gx, gy)
    assert np.array_equal(m, ex * ex + ey * ey)
    # constant image -> all zero; transposed image swaps the two responses
    z = oracle.forward_int(np.full((1, 1, h, w), 200), f, "depthwise")
    assert not z.any()
    t = oracle.forward_int(img.T.copy()[None, None], f, "depthwise")[0]
    assert np.array_equal(t[0], gy.T) and np.array_equal(t[1], gx.T)


def test_sobel_matches_scipy_on_random_u8():
    x, f = wl.sobel(h=37, w=53)
    out = oracle.forward_int(x, f, "depthwise")
    for c in range(3):
        for j, s in enumerate((wl.SOBEL_X, wl.SOBEL_Y)):
            ref = nd.correlate(x[0, c].astype(np.int64), s.astype(np.int64), mode="nearest")
            assert np.array_equal(out[0, 2 * c + j], ref)
    assert np.abs(out).max() <= 1020


def test_int_path_equals_exact_float_on_integers():
    r = _rng(8)
    x = r.integers(0, 256, (2, 3, 11, 13))
    f = r.integers(-50, 51, (6, 1, 5, 5))
    assert np.array_equal(oracle.forward_int(x, f, "depthwise"),
                          oracle.forward(x.astype(np.float64), f.astype(np.float64),
                                         "depthwise").astype(np.int64))


# -------------------------------------------------------- pin 9: 1x1 image --
@pytest.mark.parametrize("k", [1, 3, 7])
def test_one_pixel_image(k):
    r = _rng(9, k)
    f = r.standard_normal((k, k))
    xv, gv = 0.8125, -1.25
    s = f.sum()
    assert np.allclose(oracle.forward(np.full((1, 1, 1, 1), xv), f), xv * s, rtol=1e-14)
    gx = oracle.grad_input(np.full((1, 1, 1, 1), gv), f, (1, 1, 1, 1))
    assert np.allclose(gx, gv * s, rtol=1e-14)
    gf = oracle.grad_filter(np.full((1, 1, 1, 1), xv), np.full((1, 1, 1, 1), gv), (1, 1, k, k))
    assert np.all(gf == gv * xv)


# ---------------------------------------------- pin 10: paper's Laplacian ----
def test_paper_laplacian_on_parabola():
    """Section 4.2.4: 8 at the centre, -1 around.  On X = x^2 (x the column),
    every interior response is -6 (the 8 neighbours sum to 8 x^2 + 6);
    a constant image gives 0 everywhere under clamp-to-edge."""
    h, w = 9, 12
    img = (np.arange(w, dtype=np.float64) ** 2)[None, :].repeat(h, 0)
    y = oracle.forward(img, wl.LAPLACIAN_8.astype(np.float64))[0, 0]
    assert np.all(y[1:-1, 1:-1] == -6.0)
    assert not oracle.forward(np.full((h, w), 17.0), wl.LAPLACIAN_8.astype(np.float64)).any()


# ------------------------------------------------------ pin: zero border ----
def _scipy_zero_forward(x, f, mode):
    """The zero-border forward map from scipy.ndimage.correlate(mode='constant',
    cval=0): out-of-image neighbours read as 0."""
    n_, c_, h_, w_ = x.shape
    outs = []
    for n in range(n_):
        planes = []
        if mode == "shared":
            for c in range(c_):
                planes.append(nd.correlate(x[n, c], f[0, 0], mode="constant", cval=0.0))
        elif mode == "depthwise":
            m = f.shape[0] // c_
            for o in range(f.shape[0]):
                planes.append(nd.correlate(x[n, o // m], f[o, 0], mode="constant", cval=0.0))
        else:
            for o in range(f.shape[0]):
                planes.append(sum(nd.correlate(x[n, i], f[o, i], mode="constant", cval=0.0)
                                  for i in range(c_)))
        outs.append(np.stack(planes))
    return np.stack(outs)


@pytest.mark.parametrize("mode", ["shared", "depthwise", "bank"])
@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("k", KS)
def test_zero_border_equals_scipy_constant_correlation(mode, shape, k):
    r = _rng(21, k, *shape)
    x = r.random(shape)
    f = _filter(mode, shape[1], k, r)
    got = oracle.forward(x, f, mode, border="zero")
    want = _scipy_zero_forward(x, f, mode)
    assert got.shape == want.shape
    assert np.allclose(got, want, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("k", [3, 5, 7])
def test_zero_border_counts_in_image_taps_and_matches_clamp_inside(k):
    """All-ones filter on a ones image counts the in-image taps: (r+1)^2 at a
    corner, (r+1)(2r+1) along an edge, K^2 inside, where it also equals the
    clamp-to-edge result of any image."""
    rr = (k - 1) // 2
    h, w = 3 * k, 3 * k + 2
    y = oracle.forward(np.ones((h, w)), np.ones((k, k)), border="zero")[0, 0]
    assert y[0, 0] == (rr + 1) ** 2 and y[-1, -1] == (rr + 1) ** 2
    assert y[0, w // 2] == (rr + 1) * k and y[h // 2, 0] == (rr + 1) * k
    assert y[h // 2, w // 2] == k * k
    x = _rng(22, k).random((h, w))
    f = _rng(23, k).standard_normal((k, k))
    z = oracle.forward(x, f, border="zero")[0, 0]
    c = oracle.forward(x, f)[0, 0]
    assert np.array_equal(z[rr:h - rr, rr:w - rr], c[rr:h - rr, rr:w - rr])
    assert not np.allclose(z[0], c[0])


def test_zero_border_paper_laplacian_on_a_constant_image():
    """Section 4.2.4's sharpen skips out-of-image neighbours: on a constant
    image v the Laplacian (8 at the centre, -1 around) gives 0 inside, 8v - 5v
    at an edge pixel (5 neighbours inside) and 8v - 3v at a corner (3 inside)."""
    v = 10.0
    y = oracle.forward(np.full((6, 7), v), wl.LAPLACIAN_8.astype(np.float64), border="zero")[0, 0]
    assert np.all(y[1:-1, 1:-1] == 0.0)
    assert y[0, 3] == 8 * v - 5 * v and y[3, 0] == 8 * v - 5 * v
    assert y[0, 0] == 8 * v - 3 * v


# ---------------------------------------------- pin 11: paper's grayscale ----
def test_paper_grayscale_is_a_k1_bank():
    """Section 4.2.5: Y = 0.299 R + 0.587 G + 0.114 B, as a 3 -> 1 bank with K = 1."""
    x = _rng(11).random((2, 3, 5, 6))
    f = wl.GRAY_RGB.reshape(1, 3, 1, 1)
    y = oracle.forward(x, f, "bank")
    ref = 0.299 * x[:, 0] + 0.587 * x[:, 1] + 0.114 * x[:, 2]
    np.testing.assert_allclose(y[:, 0], ref, rtol=1e-15, atol=1e-15)


# ----------------------------------------- pin 13: finite differences -------
@pytest.mark.parametrize("mode", ["shared", "depthwise", "bank"])
def test_finite_differences_match_the_adjoints(mode):
    """L(x, F) = <A(x; F), G> is linear in x and in F, so the central difference
    with step 1 is the exact directional derivative up to FP64 rounding."""
    r = _rng(13)
    shape = (1, 2, 7, 6)
    x = r.random(shape)
    f = _filter(mode, 2, 5, r)
    g = r.standard_normal(oracle.forward(x, f, mode).shape)

    def loss(xv, fv):
        return float(np.sum(oracle.forward(xv, fv, mode) * g))

    gx = oracle.grad_input(g, f, shape, mode)
    gf = oracle.grad_filter(x, g, f.shape, mode)
    dirs = [r.standard_normal(shape)]
    for (yy, xx) in [(0, 0), (0, 5), (6, 0), (6, 5), (0, 3), (3, 0), (3, 3), (6, 2)]:
        e = np.zeros(shape)
        e[0, 1, yy, xx] = 1.0
        dirs.append(e)
    for d in dirs:
        fd = (loss(x + d, f) - loss(x - d, f)) / 2.0
        assert abs(fd - float(np.sum(gx * d))) <= 1e-12 * max(1.0, abs(fd))
    for t in range(4):
        d = r.standard_normal(f.shape)
        fd = (loss(x, f + d) - loss(x, f - d)) / 2.0
        assert abs(fd - float(np.sum(gf * d))) <= 1e-12 * max(1.0, abs(fd))


# ------------------------------------- pin 15: reduction accuracy (fsum) ----
def test_grad_filter_summation_is_accurate():
    """Neumaier-compensated F-bar against math.fsum (exactly rounded) of the
    same products, gathered with numpy edge padding, on a cancelling input."""
    r = _rng(15)
    h, w, k = 40, 37, 5
    rr = (k - 1) // 2
    x = r.standard_normal((h, w)) * 1e3 + 1e6
    g = r.standard_normal((h, w))
    g -= g.mean()
    gf = oracle.grad_filter(x, g, (1, 1, k, k))[0, 0]
    p = np.pad(x, rr, mode="edge")
    for u in range(k):
        for v in range(k):
            prods = (g * p[u:u + h, v:v + w]).ravel()
            exact = math.fsum(prods.tolist())
            assert abs(gf[u, v] - exact) <= 1e-12 * np.abs(prods).sum() * 1e-3 + 1e-9 * abs(exact)


# ---------------------------------------------------------- band / errors ----
def test_row_band_equals_rows_of_the_whole():
    x = _rng(16).random((1, 2, 20, 9))
    f = _rng(17).standard_normal((7, 7))
    full = oracle.forward(x, f)
    for y0, y1 in [(0, 3), (5, 12), (17, 20), (0, 20), (4, 4)]:
        assert np.array_equal(oracle.forward(x, f, rows=(y0, y1)), full[:, :, y0:y1])


def test_oracle_rejects_bad_arguments():
    x = np.zeros((1, 2, 4, 4))
    with pytest.raises(ValueError):
        oracle.forward(x, np.zeros((2, 2)))  # even K
    with pytest.raises(ValueError):
        oracle.forward(x, np.zeros((3, 1, 3, 3)), "depthwise")  # FO not a multiple of C
    with pytest.raises(ValueError):
        oracle.forward(x, np.zeros((4, 3, 3, 3)), "bank")  # FI != C
    with pytest.raises(ValueError):
        oracle.forward(x, np.zeros((3, 3)), rows=(3, 2))


def test_golden_constants_match_the_paper_fixtures():
    """The constants used by the pins are the ones the paper states
    (tests/golden: Section 4.2.4 Laplacian, Section 4.2.5 grayscale weights)."""
    import os

    here = os.path.join(os.path.dirname(__file__), "golden")
    lap = np.loadtxt(os.path.join(here, "laplacian_3x3.txt"))
    gray = np.loadtxt(os.path.join(here, "grayscale_weights.txt"))
    assert np.array_equal(lap, wl.LAPLACIAN_8.astype(np.float64))
    assert np.array_equal(gray, wl.GRAY_RGB)


def test_rel_l2_acceptance_metric_hand_values():
    """The acceptance metric ||a - ref|| / ||ref|| against values worked by
    hand: a swapped numerator and denominator, a missing square root or a
    normalisation by ||a|| instead of ||ref|| all fail one of these."""
    ref = np.array([3.0, 4.0])                          # ||ref|| = 5
    assert oracle.rel_l2(np.array([3.0, 4.5]), ref) == pytest.approx(0.1, rel=1e-15)
    assert oracle.rel_l2(np.array([3.0, 14.0]), ref) == pytest.approx(2.0, rel=1e-15)
    ref3 = np.array([[1.0, 2.0, 2.0]])                  # ||ref|| = 3
    assert oracle.rel_l2(np.array([[1.0, 2.0, 2.3]]), ref3) == pytest.approx(0.1, rel=1e-13)
    # normalised by the reference: (3, 4) against (6, 8) is 5 / 10, not 5 / 5
    assert oracle.rel_l2(np.array([3.0, 4.0]), np.array([6.0, 8.0])) == pytest.approx(0.5, rel=1e-15)
    assert oracle.rel_l2(np.array([6.0, 8.0]), np.array([3.0, 4.0])) == pytest.approx(1.0, rel=1e-15)
    # squares, not absolute values: (0, 3) vs (4, 0) differ by (-4, 3), norm 5, over ||(4, 0)|| = 4
    assert oracle.rel_l2(np.array([0.0, 3.0]), np.array([4.0, 0.0])) == pytest.approx(1.25, rel=1e-15)
    assert oracle.rel_l2(ref, ref) == 0.0
    # an all-zero reference falls back to the absolute norm of the difference
    assert oracle.rel_l2(np.array([0.0, 0.3, 0.4]), np.zeros(3)) == pytest.approx(0.5, rel=1e-15)
    # float32 inputs are promoted before squaring (no overflow at 1e30)
    big = np.array([1e30, 1e30], dtype=np.float32)
    assert oracle.rel_l2(big * np.float32(1.5), big) == pytest.approx(0.5, rel=1e-6)
