"""FP32 forward with zero borders (F2D_BORDER_ZERO) against the CPU oracle.

Zero borders are the rule of the paper's sharpen (out-of-image neighbours
are skipped, Section 4.2.4).  The oracle's zero-border forward is pinned
against scipy's constant-border correlation.  FP32 bar: relative L2 error
<= 1e-5 against the FP64 oracle, over ragged shapes spanning several tiles,
every channel mode, K up to 31 and row bands.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2504_01266_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL = 1e-5


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def rel(gpu, ref):
    return oracle.rel_l2(gpu.double().cpu().numpy(), ref)


SHAPES = [(1, 1, 1, 1), (1, 1, 1, 9), (1, 1, 7, 1), (1, 2, 5, 7), (2, 3, 67, 131), (1, 1, 33, 48)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("k", [1, 3, 5, 9, 15, 31])
def test_zero_border_shared(gpu_lib, shape, k):
    x, f = wl.random_case(71, *shape, k)
    y = gpu_lib.forward(dev(x), dev(f[0, 0]), border="zero")
    ref = oracle.forward(x, f.astype(np.float64), border="zero")
    assert y.shape == ref.shape
    assert rel(y, ref) <= TOL


@pytest.mark.parametrize("k", [3, 7])
def test_zero_border_depthwise_and_bank(gpu_lib, k):
    x, f = wl.random_case(72, 2, 3, 45, 70, k, fo=6, fi=1)
    ys = gpu_lib.forward(dev(x), dev(f), mode="depthwise", border="zero")
    ref = oracle.forward(x, f.astype(np.float64), "depthwise", border="zero")
    got = np.stack([y.double().cpu().numpy() for y in ys], axis=2).reshape(ref.shape)
    assert oracle.rel_l2(got, ref) <= TOL
    xb, fb = wl.random_case(73, 2, 3, 45, 70, k, fo=5, fi=3)
    yb = gpu_lib.forward(dev(xb), dev(fb), mode="bank", border="zero")
    assert rel(yb, oracle.forward(xb, fb.astype(np.float64), "bank", border="zero")) <= TOL


@pytest.mark.parametrize("k", [3, 9])
def test_zero_border_bands(gpu_lib, k):
    x, f = wl.random_case(74, 1, 2, 90, 77, k)
    for rows in [(0, 90), (5, 40), (89, 90), (0, 1)]:
        y = gpu_lib.forward(dev(x), dev(f[0, 0]), rows=rows, border="zero")
        assert rel(y, oracle.forward(x, f.astype(np.float64), rows=rows, border="zero")) <= TOL


def test_zero_border_paper_sharpen(gpu_lib):
    """Section 4.2.4's Laplacian sharpen (8 at the centre, -1 around, skipped
    out-of-image neighbours) on a 3-channel image with values 0..255."""
    r = wl.rng(75)
    x = r.integers(0, 256, (1, 3, 130, 200)).astype(np.float32)
    f = wl.LAPLACIAN_8.astype(np.float32)
    y = gpu_lib.forward(dev(x), dev(f), border="zero")
    ref = oracle.forward(x, f.astype(np.float64), border="zero")
    # integer data and taps: every sum is exact in FP32
    assert np.array_equal(y.double().cpu().numpy(), ref)


@pytest.mark.parametrize("k", [1, 5, 31])
def test_zero_border_identity_is_bitwise(gpu_lib, k):
    x, _ = wl.random_case(76, 1, 2, 40, 50, k)
    f = np.zeros((k, k), np.float32)
    f[k // 2, k // 2] = 1.0
    y = gpu_lib.forward(dev(x), dev(f), border="zero")
    assert torch.equal(y.cpu(), torch.from_numpy(x))


@pytest.mark.slow
def test_zero_border_full_size_sharpen(gpu_lib):
    """The benchmark's launch: 3-channel 4K frame (0..255), 3x3 Laplacian with
    zero borders; row bands at the top, the middle and the bottom against the
    oracle, bit-exact (integer data and taps)."""
    x = wl.sharpen_frame()
    f = wl.LAPLACIAN_8
    y = gpu_lib.forward(dev(x), dev(f), border="zero")
    torch.cuda.synchronize()
    for r0, r1 in [(0, 6), (1077, 1083), (2154, 2160)]:
        ref = oracle.forward(x, f.astype(np.float64), rows=(r0, r1), border="zero")
        assert np.array_equal(y[:, :, r0:r1].double().cpu().numpy(), ref)
