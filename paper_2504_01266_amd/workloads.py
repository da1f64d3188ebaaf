"""Seeded synthetic inputs for the K x K filter workloads.

This module only draws inputs (images, filters, upstream gradients) and holds
none of the filter's arithmetic; both the GPU tests/benchmark and the CPU
oracle consume exactly the arrays produced here.

Every tensor comes from its own numpy PCG64 stream ``default_rng([seed,
tensor_id, index])`` so that a large batch can be generated one image at a
time and give the same values as a whole-batch draw.

Workloads (the paper's images and signals are not available; these synthetic
inputs stand in for them, with the shapes and value ranges below):

* ``plain``    1 x 1 x 1024 x 1024 f32 uniform [0,1), 5x5 Gaussian sigma=1
* ``sobel``    1 x 3 x 4320 x 7680 u8 uniform [0,255], Sobel-x / Sobel-y per
               channel (int32 taps), outputs gx, gy, gx^2+gy^2
* ``ragged``   64 images, 3 channels, H and W uniform integers in [256, 4096],
               pixels uniform [0,1), one 7x7 filter per image with taps N(0, 1/49)
* ``diff``     16 x 3 x 2048 x 2048 f32 uniform [0,1), shared 9x9 filter N(0,1/81),
               upstream gradient N(0,1)
* ``bank``     32 x 16 x 1024 x 1024 inputs N(0,1), C_out = 64, K in {3, 5},
               weights N(0, 2/(C_in K^2)), upstream gradient N(0,1); BF16
               operands are the round-to-nearest-even images of the FP32 draws.
"""
import numpy as np

# ---------------------------------------------------------------- filters --


def gaussian_taps(k=5, sigma=1.0):
    """Sampled Gaussian g(d) = exp(-d^2 / (2 sigma^2)), d = -r..r; 2D taps
    g(u) g(v) / (sum g)^2 computed in float64 and rounded once to float32."""
    r = (k - 1) // 2
    d = np.arange(-r, r + 1, dtype=np.float64)
    g = np.exp(-(d * d) / (2.0 * sigma * sigma))
    t = np.outer(g, g) / (g.sum() ** 2)
    return t.astype(np.float32)


def gaussian_factor(k=9, sigma=2.0):
    """The 1-D factor g / sum(g) of a normalised sampled Gaussian (float64,
    rounded once to float32): the 2-D filter is its outer product with
    itself."""
    r = (k - 1) // 2
    d = np.arange(-r, r + 1, dtype=np.float64)
    g = np.exp(-(d * d) / (2.0 * sigma * sigma))
    return (g / g.sum()).astype(np.float32)


def separable_factors(seed, k):
    """Random float32 factors a, b with taps N(0, 1/k) (a rank-one filter
    a b^T with taps of variance 1/k^2, like the 7x7 and 9x9 workloads)."""
    r = rng(seed, k, 4242)
    return (r.standard_normal(k) / np.sqrt(k)).astype(np.float32), \
        (r.standard_normal(k) / np.sqrt(k)).astype(np.float32)


SOBEL_X = np.array([[-1, 0, 1], [-2, 0, 2], [-1, 0, 1]], dtype=np.int32)
SOBEL_Y = SOBEL_X.T.copy()

# The paper's sharpen filter: 8 at the centre, -1 on the eight neighbours
# (Section 4.2.4, "Sharpening").
LAPLACIAN_8 = np.array([[-1, -1, -1], [-1, 8, -1], [-1, -1, -1]], dtype=np.float32)

# The paper's grayscale weights for R, G, B (Section 4.2.5, "Grayscaling").
GRAY_RGB = np.array([0.299, 0.587, 0.114], dtype=np.float64)


def sobel_depthwise(channels):
    """Depthwise filter [C*2][1][3][3]: filter 2c is Sobel-x, 2c+1 is Sobel-y."""
    f = np.empty((channels * 2, 1, 3, 3), np.int32)
    f[0::2, 0] = SOBEL_X
    f[1::2, 0] = SOBEL_Y
    return f


# ------------------------------------------------------------- bf16 inputs --


def bf16_round(a):
    """Round float32 values to bfloat16 (round to nearest, ties to even).
    Returns (bits as uint16, the rounded values as float32)."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16).astype(np.uint16)
    nan = np.isnan(a)
    if nan.any():
        r[nan] = 0x7FC0
    back = (r.astype(np.uint32) << 16).view(np.float32)
    return r, back


# ----------------------------------------------------------------- streams --


def rng(seed, *ids):
    return np.random.default_rng([int(seed), *[int(i) for i in ids]])


# --------------------------------------------------------------- workloads --

PLAIN_SEED, SOBEL_SEED, RAGGED_SEED, DIFF_SEED, BANK_SEED = 1, 2, 3, 4, 5


def plain(h=1024, w=1024):
    x = rng(PLAIN_SEED, 1).random((1, 1, h, w), dtype=np.float32)
    return x, gaussian_taps(5, 1.0)


def sobel(h=4320, w=7680, c=3):
    x = rng(SOBEL_SEED, 1).integers(0, 256, (1, c, h, w), dtype=np.uint8)
    return x, sobel_depthwise(c)


def ragged_sizes(n=64, lo=256, hi=4096):
    return rng(RAGGED_SEED, 0).integers(lo, hi + 1, (n, 2))


def ragged_item(i, h, w, c=3, k=7):
    x = rng(RAGGED_SEED, 1, i).random((c, h, w), dtype=np.float32)
    f = (rng(RAGGED_SEED, 2, i).standard_normal((k, k), dtype=np.float32) / np.float32(k))
    return x, f.astype(np.float32)


def sharpen_frame(h=2160, w=3840, c=3):
    """A 4K 3-channel frame with integer values 0..255 stored as float32 (the
    sharpen of Section 4.2.4 on an 8-bit image, in the FP32 path)."""
    return rng(9, 4, h, w).integers(0, 256, (1, c, h, w)).astype(np.float32)


def paper_frame_u8(h=2160, w=3840, c=3, seed=10):
    """A 4K RGB frame as OpenCV delivers it (Sections 4.2.3-4.2.5): 8-bit
    values uniform in [0, 255], interleaved [H][W][C] (pixel after pixel)."""
    return rng(seed, 1, h, w).integers(0, 256, (h, w, c), dtype=np.uint8)


def diff_image(n, c=3, h=2048, w=2048):
    return rng(DIFF_SEED, 1, n).random((c, h, w), dtype=np.float32)


def diff_filter(k=9):
    return (rng(DIFF_SEED, 2).standard_normal((k, k), dtype=np.float32) / np.float32(k))


def diff_grad(n, c=3, h=2048, w=2048):
    return rng(DIFF_SEED, 3, n).standard_normal((c, h, w), dtype=np.float32)


def diff_crop_origins(count=8, h=2048, w=2048, size=64):
    r = rng(DIFF_SEED, 4)
    ys = r.integers(0, h - size + 1, count)
    xs = r.integers(0, w - size + 1, count)
    ys[0], xs[0] = 0, 0
    return list(zip(ys.tolist(), xs.tolist()))


def bank_image(n, cin=16, h=1024, w=1024):
    return rng(BANK_SEED, 1, n).standard_normal((cin, h, w), dtype=np.float32)


def bank_weights(k, cout=64, cin=16):
    s = np.float32(np.sqrt(2.0 / (cin * k * k)))
    return rng(BANK_SEED, 2, k).standard_normal((cout, cin, k, k), dtype=np.float32) * s


def bank_grad(n, cout=64, h=1024, w=1024):
    return rng(BANK_SEED, 3, n).standard_normal((cout, h, w), dtype=np.float32)


# --------------------------------------------------------- small test cases --


def random_case(seed, n, c, h, w, k, fo=1, fi=1, dtype="f32"):
    """A generic seeded case: image, filter [fo][fi][k][k], upstream gradient."""
    r = rng(1000 + seed, n, c, h, w, k)
    if dtype == "u8":
        x = r.integers(0, 256, (n, c, h, w), dtype=np.uint8)
        f = r.integers(-8, 9, (fo, fi, k, k)).astype(np.int32)
    else:
        x = r.random((n, c, h, w), dtype=np.float32)
        f = r.standard_normal((fo, fi, k, k), dtype=np.float32) / np.float32(k)
    return x, f
