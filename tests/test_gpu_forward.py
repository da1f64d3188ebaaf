"""GPU forward paths against the CPU oracle (through the C ABI).

FP32: relative L2 error <= 1e-5 against the FP64 oracle.  u8 -> int32:
bit-exact.  Sizes span several tiles with ragged right/bottom edges; the
full-size plain-Gaussian and 8K Sobel workloads run in the launch
configuration the benchmark times.
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


F32_SHAPES = [(1, 1, 1, 1), (1, 1, 1, 9), (1, 1, 7, 1), (1, 2, 5, 7), (2, 3, 67, 131),
              (1, 1, 130, 257)]


@pytest.mark.parametrize("shape", F32_SHAPES)
@pytest.mark.parametrize("k", [1, 3, 5, 7, 9, 11, 15])
def test_f32_shared_matches_oracle(gpu_lib, shape, k):
    x, f = wl.random_case(1, *shape, k)
    y = gpu_lib.forward(dev(x), dev(f[0, 0]))
    ref = oracle.forward(x, f.astype(np.float64))
    assert y.shape == ref.shape
    assert rel(y, ref) <= TOL


@pytest.mark.parametrize("variant", [1, 2, 3, 4])
@pytest.mark.parametrize("k", [3, 9])
def test_f32_variants_are_bitwise_identical(gpu_lib, variant, k):
    x, f = wl.random_case(2, 2, 2, 150, 203, k)
    base = gpu_lib.forward(dev(x), dev(f[0, 0]), variant=1)
    y = gpu_lib.forward(dev(x), dev(f[0, 0]), variant=variant)
    assert torch.equal(base, y)
    assert rel(y, oracle.forward(x, f.astype(np.float64))) <= TOL


@pytest.mark.parametrize("k", [1, 3, 5, 9])
def test_identity_kernel_is_bitwise(gpu_lib, k):
    x, _ = wl.random_case(3, 1, 3, 77, 90, k)
    f = np.zeros((k, k), np.float32)
    f[k // 2, k // 2] = 1.0
    y = gpu_lib.forward(dev(x), dev(f))
    assert torch.equal(y.cpu(), torch.from_numpy(x))


def test_constant_image_keeps_borders(gpu_lib):
    k = 7
    f = wl.rng(9, 9).standard_normal((k, k), dtype=np.float32)
    x = np.full((1, 1, 45, 70), 0.625, np.float32)
    y = gpu_lib.forward(dev(x), dev(f)).cpu().numpy()
    expect = 0.625 * f.astype(np.float64).sum()
    assert np.max(np.abs(y - expect)) <= 1e-5 * max(1.0, abs(expect))


@pytest.mark.parametrize("m", [1, 2, 3, 4])
@pytest.mark.parametrize("k", [3, 5, 13])
def test_f32_depthwise(gpu_lib, m, k):
    c = 3
    x, f = wl.random_case(4, 2, c, 40, 70, k, fo=c * m, fi=1)
    outs = gpu_lib.forward(dev(x), dev(f), mode="depthwise")
    ref = oracle.forward(x, f.astype(np.float64), "depthwise")
    assert len(outs) == m
    for j in range(m):
        assert rel(outs[j], ref[:, j::m]) <= TOL


@pytest.mark.parametrize("cout", [1, 3, 4, 6])
@pytest.mark.parametrize("k", [1, 3, 5, 9])
def test_f32_bank(gpu_lib, cout, k):
    cin = 3
    x, f = wl.random_case(5, 2, cin, 37, 66, k, fo=cout, fi=cin)
    y = gpu_lib.forward(dev(x), dev(f), mode="bank")
    assert rel(y, oracle.forward(x, f.astype(np.float64), "bank")) <= TOL


def test_paper_grayscale_as_bank(gpu_lib):
    x = wl.rng(6, 1).random((2, 3, 19, 23), dtype=np.float32)
    f = wl.GRAY_RGB.astype(np.float32).reshape(1, 3, 1, 1)
    y = gpu_lib.forward(dev(x), dev(f), mode="bank").cpu().numpy()[:, 0]
    ref = 0.299 * x[:, 0].astype(np.float64) + 0.587 * x[:, 1] + 0.114 * x[:, 2]
    assert oracle.rel_l2(y, ref) <= TOL


def test_strided_views_and_interleaved_outputs(gpu_lib):
    """Non-contiguous image view (row pitch > W) and DEPTHWISE outputs written
    as strided views into one interleaved [N][C*m] tensor."""
    big = wl.rng(7, 1).random((1, 3, 50, 97), dtype=np.float32)
    xv = dev(big)[:, :, 3:47, 5:90]  # row pitch 97, odd offsets
    x = big[:, :, 3:47, 5:90]
    f = wl.rng(7, 2).standard_normal((6, 1, 5, 5), dtype=np.float32)
    inter = torch.empty((1, 6, 44, 85), device="cuda")
    outs = [inter[:, 0::2], inter[:, 1::2]]
    gpu_lib.forward(xv, dev(f), mode="depthwise", outs=outs)
    ref = oracle.forward(x, f.astype(np.float64), "depthwise")
    assert rel(inter, ref) <= TOL


# ------------------------------------------------------------------- u8 ----

U8_SHAPES = [(1, 1, 1, 1), (1, 1, 1, 5), (1, 1, 6, 1), (1, 3, 9, 13), (2, 3, 70, 517),
             (1, 2, 131, 260)]


@pytest.mark.parametrize("shape", U8_SHAPES)
@pytest.mark.parametrize("k", [1, 3, 5, 7])
def test_u8_shared_bit_exact(gpu_lib, shape, k):
    x, f = wl.random_case(8, *shape, k, dtype="u8")
    y = gpu_lib.forward(dev(x), dev(f[0, 0]))
    ref = oracle.forward_int(x, f)
    assert torch.equal(y.cpu(), torch.from_numpy(ref.astype(np.int32)))


@pytest.mark.parametrize("shape", U8_SHAPES)
def test_sobel_bit_exact(gpu_lib, shape):
    x = wl.random_case(9, *shape, 3, dtype="u8")[0]
    f = wl.sobel_depthwise(shape[1])
    gx, gy, m = gpu_lib.forward(dev(x), dev(f), mode="depthwise", epilogue=gpu_lib.EPI_SUMSQ_PAIRS)
    ref = oracle.forward_int(x, f, "depthwise")
    assert torch.equal(gx.cpu(), torch.from_numpy(ref[:, 0::2].astype(np.int32)))
    assert torch.equal(gy.cpu(), torch.from_numpy(ref[:, 1::2].astype(np.int32)))
    mm = oracle.sumsq(ref[:, 0::2], ref[:, 1::2])
    assert torch.equal(m.cpu(), torch.from_numpy(mm.astype(np.int32)))


@pytest.mark.parametrize("variant", [1, 2, 3, 4, 5, 6, 7])
def test_u8_variants_and_large_taps_wrap(gpu_lib, variant):
    """Taps too large for the 24-bit multiplier take the 32-bit path; the
    int32 results wrap modulo 2^32 exactly like the int64 oracle cast to int32."""
    x = wl.rng(10, 1).integers(0, 256, (1, 2, 75, 300), dtype=np.uint8)
    for f in (wl.sobel_depthwise(2),
              wl.rng(10, 2).integers(-(2 ** 30), 2 ** 30, (4, 1, 3, 3)).astype(np.int32)):
        outs = gpu_lib.forward(dev(x), dev(f), mode="depthwise",
                               epilogue=gpu_lib.EPI_SUMSQ_PAIRS, variant=variant)
        ref = oracle.forward_int(x, f, "depthwise")
        mm = oracle.sumsq(ref[:, 0::2], ref[:, 1::2])
        wrap = lambda a: ((a + 2 ** 31) % 2 ** 32 - 2 ** 31).astype(np.int32)  # noqa: E731
        assert torch.equal(outs[0].cpu(), torch.from_numpy(wrap(ref[:, 0::2])))
        assert torch.equal(outs[1].cpu(), torch.from_numpy(wrap(ref[:, 1::2])))
        assert torch.equal(outs[2].cpu(), torch.from_numpy(wrap(mm)))


@pytest.mark.parametrize("shape", [(1, 1, 1, 1), (1, 2, 9, 13), (2, 3, 70, 517), (1, 2, 131, 260)])
@pytest.mark.parametrize("k", [9, 11, 31])
def test_u8_large_k_bit_exact(gpu_lib, shape, k):
    """K = 9 (templated kernel) and K = 11, 31 (the runtime-K kernel) on the
    exact integer path: SHARED, and DEPTHWISE with two filters per channel
    plus the sum-of-squares output, bit-exact against the int64 oracle."""
    x, f = wl.random_case(30 + k, *shape, k, dtype="u8")
    y = gpu_lib.forward(dev(x), dev(f[0, 0]))
    assert torch.equal(y.cpu(), torch.from_numpy(oracle.forward_int(x, f).astype(np.int32)))
    c = shape[1]
    fd = wl.rng(40 + k, 1).integers(-8, 9, (2 * c, 1, k, k)).astype(np.int32)
    gx, gy, m = gpu_lib.forward(dev(x), dev(fd), mode="depthwise", epilogue=gpu_lib.EPI_SUMSQ_PAIRS)
    ref = oracle.forward_int(x, fd, "depthwise")
    assert torch.equal(gx.cpu(), torch.from_numpy(ref[:, 0::2].astype(np.int32)))
    assert torch.equal(gy.cpu(), torch.from_numpy(ref[:, 1::2].astype(np.int32)))
    mm = oracle.sumsq(ref[:, 0::2], ref[:, 1::2])
    assert torch.equal(m.cpu(), torch.from_numpy(mm.astype(np.int32)))


@pytest.mark.parametrize("k", [9, 13])
def test_u8_large_k_three_filters_per_channel(gpu_lib, k):
    """More than two filters per channel (separate launches per filter in the
    runtime-K kernel)."""
    x = wl.rng(50 + k, 1).integers(0, 256, (1, 2, 45, 140), dtype=np.uint8)
    f = wl.rng(50 + k, 2).integers(-100, 101, (6, 1, k, k)).astype(np.int32)
    outs = gpu_lib.forward(dev(x), dev(f), mode="depthwise")
    ref = oracle.forward_int(x, f, "depthwise")
    for j in range(3):
        assert torch.equal(outs[j].cpu(), torch.from_numpy(ref[:, j::3].astype(np.int32)))


def test_u8_unaligned_rows(gpu_lib):
    """Odd row pitch and offset: the word-load and vector-store fast paths
    must switch off; results stay exact."""
    big = wl.rng(11, 1).integers(0, 256, (1, 1, 40, 103), dtype=np.uint8)
    xv = dev(big)[:, :, 1:39, 3:100]
    f = wl.sobel_depthwise(1)
    outs = gpu_lib.forward(xv, dev(f), mode="depthwise")
    ref = oracle.forward_int(big[:, :, 1:39, 3:100], f, "depthwise")
    assert torch.equal(outs[0].cpu(), torch.from_numpy(ref[:, 0::2].astype(np.int32)))
    assert torch.equal(outs[1].cpu(), torch.from_numpy(ref[:, 1::2].astype(np.int32)))


def test_u8_depthwise_three_filters(gpu_lib):
    x, f = wl.random_case(12, 1, 2, 33, 45, 5, fo=6, fi=1, dtype="u8")
    outs = gpu_lib.forward(dev(x), dev(f), mode="depthwise")
    ref = oracle.forward_int(x, f, "depthwise")
    for j in range(3):
        assert torch.equal(outs[j].cpu(), torch.from_numpy(ref[:, j::3].astype(np.int32)))


# ----------------------------------------------------------------- bands ----

@pytest.mark.parametrize("dtype", ["f32", "u8"])
def test_bands_concatenate_to_the_whole_bitwise(gpu_lib, dtype):
    k = 5 if dtype == "f32" else 3
    r = k // 2
    x, f = wl.random_case(13, 1, 2, 97, 150, k, dtype=dtype)
    xd = dev(x)
    fd = dev(f[0, 0])
    whole = gpu_lib.forward(xd, fd)
    cuts = [0, 1, 20, 57, 96, 97]
    parts = []
    for y0, y1 in zip(cuts[:-1], cuts[1:]):
        lo, hi = max(0, y0 - r), min(97, y1 + r)
        parts.append(gpu_lib.forward(xd[:, :, lo:hi], fd, rows=(y0 - lo, y1 - lo)))
    assert torch.equal(torch.cat(parts, dim=2), whole)


# --------------------------------------------------------------- tuner ----

def test_autotune_records_a_variant(gpu_lib, tmp_path):
    x, f = wl.random_case(14, 1, 1, 512, 512, 5)
    best = gpu_lib.autotune_forward(dev(x), dev(f[0, 0]), reps=2)
    assert 1 <= best <= gpu_lib.variant_count(gpu_lib.PATH_F32)
    p = str(tmp_path / "tune.json")
    gpu_lib.tune_save(p)
    gpu_lib.tune_clear()
    gpu_lib.tune_load(p)
    y = gpu_lib.forward(dev(x), dev(f[0, 0]))  # tuned variant, same bits
    assert torch.equal(y, gpu_lib.forward(dev(x), dev(f[0, 0]), variant=1))
    gpu_lib.tune_clear()


# ------------------------------------------------------------ full size ----

def test_plain_gaussian_full_size(gpu_lib):
    x, f = wl.plain()
    y = gpu_lib.forward(dev(x), dev(f))
    assert rel(y, oracle.forward(x, f.astype(np.float64))) <= TOL


def test_sobel_8k_full_size_bit_exact(gpu_lib):
    x, f = wl.sobel()
    print("sobel 8k: 1x3x4320x7680", flush=True)
    gx, gy, m = gpu_lib.forward(dev(x), dev(f), mode="depthwise", epilogue=gpu_lib.EPI_SUMSQ_PAIRS)
    torch.cuda.synchronize()
    ref = oracle.forward_int(x, f, "depthwise")
    assert np.array_equal(gx.cpu().numpy(), ref[:, 0::2])
    assert np.array_equal(gy.cpu().numpy(), ref[:, 1::2])
    assert np.array_equal(m.cpu().numpy(), oracle.sumsq(ref[:, 0::2], ref[:, 1::2]))
