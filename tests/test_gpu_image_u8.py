"""The paper's image operations on 8-bit images (Sections 4.2.3-4.2.5, the
pipeline of Section 6.6) against the oracle, through the C ABI.

8-bit and binary32 outputs are compared bit for bit: both sides compute the
sum in binary32 with one fused multiply-add per term in the same order and
convert with the same rule.  Interleaved (OpenCV) images are compared with the
oracle's planar result transposed.  Shapes span several 2048-element x
32-row tiles with ragged edges; the full-size pipeline (a 4K RGB frame
upsampled x20 and sharpened, and the 8K grayscale) is checked on sampled row
bands in the launch configuration the benchmark times.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2504_01266_amd import workloads as wl

pytestmark = pytest.mark.gpu

LAP = wl.LAPLACIAN_8.astype(np.float32)
LAP_I = wl.LAPLACIAN_8.astype(np.int32)
GRAY = wl.GRAY_RGB.astype(np.float32).reshape(1, 3, 1, 1)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def hwc_dev(x_hwc):
    """[N][H][W][C] host array -> [N][C][H][W] device view of interleaved storage."""
    t = torch.from_numpy(np.ascontiguousarray(x_hwc)).cuda()
    if t.dim() == 3:
        t = t[None]
    return t.permute(0, 3, 1, 2)


def planar_of(x_hwc):
    x = np.asarray(x_hwc)
    if x.ndim == 3:
        x = x[None]
    return np.ascontiguousarray(x.transpose(0, 3, 1, 2))


def expect(x, f, border, out, mode="shared", scale=1):
    """The oracle's result for the planar image x: upsample, binary32 sum (or
    int64 for integer taps), then the output conversion."""
    if scale > 1:
        x = oracle.upsample_nearest(x, scale)
    if np.asarray(f).dtype.kind == "f":
        s = oracle.forward_f32(x, f, mode, border=border)
        return oracle.to_u8(s) if out == "u8" else s
    s = oracle.forward_int(x, f, mode, border=border)
    return oracle.to_u8(s) if out == "u8" else s.astype(np.int64)


SHAPES = [(1, 1, 1, 1), (1, 2, 1, 9), (1, 1, 7, 1), (2, 3, 33, 70), (1, 2, 70, 2100)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("k", [1, 3, 5, 7])
@pytest.mark.parametrize("border", ["zero", "clamp"])
def test_planar_float_taps_u8_and_f32_outputs(gpu_lib, shape, k, border):
    r = wl.rng(81, k, *shape)
    x = r.integers(0, 256, shape, dtype=np.uint8)
    f = (r.standard_normal((k, k)) * 0.7).astype(np.float32)
    y8 = gpu_lib.forward(dev(x), dev(f), border=border, out_dtype=torch.uint8)
    assert np.array_equal(y8.cpu().numpy(), expect(x, f, border, "u8"))
    y32 = gpu_lib.forward(dev(x), dev(f), border=border)
    assert y32.dtype == torch.float32
    assert np.array_equal(y32.cpu().numpy(), expect(x, f, border, "f32"))


@pytest.mark.parametrize("k", [3, 5])
@pytest.mark.parametrize("border", ["zero", "clamp"])
def test_planar_int_taps(gpu_lib, k, border):
    r = wl.rng(82, k)
    x = r.integers(0, 256, (2, 3, 45, 2060), dtype=np.uint8)
    f = r.integers(-9, 10, (k, k)).astype(np.int32)
    y8 = gpu_lib.forward(dev(x), dev(f), border=border, out_dtype=torch.uint8)
    assert np.array_equal(y8.cpu().numpy(), expect(x, f, border, "u8"))
    if border == "zero":  # int32 outputs with zero borders take the same kernel
        yi = gpu_lib.forward(dev(x), dev(f), border=border)
        assert np.array_equal(yi.cpu().numpy().astype(np.int64), expect(x, f, border, "i32"))


def test_paper_sharpen_u8_laplacian_zero_border(gpu_lib):
    """Section 4.2.4 as written: the float Laplacian, out-of-image neighbours
    skipped, 8-bit result; and its constant-image values (0 / 3v / 5v)."""
    x = wl.rng(83).integers(0, 256, (1, 3, 77, 2300), dtype=np.uint8)
    y = gpu_lib.forward(dev(x), dev(LAP), border="zero", out_dtype=torch.uint8)
    assert np.array_equal(y.cpu().numpy(), expect(x, LAP, "zero", "u8"))
    c = np.full((1, 3, 40, 50), 60, np.uint8)
    yc = gpu_lib.forward(dev(c), dev(LAP), border="zero", out_dtype=torch.uint8).cpu().numpy()
    assert np.all(yc[:, :, 1:-1, 1:-1] == 0) and np.all(yc[:, :, 0, 1:-1] == 180)
    assert np.all(yc[:, :, [0, 0, -1, -1], [0, -1, 0, -1]] == 255)


@pytest.mark.parametrize("c", [3, 4])
@pytest.mark.parametrize("k", [3, 5])
@pytest.mark.parametrize("border", ["zero", "clamp"])
def test_interleaved_matches_planar_oracle(gpu_lib, c, k, border):
    r = wl.rng(84, c, k)
    x = r.integers(0, 256, (2, 35, 733, c), dtype=np.uint8)  # 733*c elements: ragged tiles
    f = (r.standard_normal((k, k)) * 0.5).astype(np.float32)
    xd = hwc_dev(x)
    y = gpu_lib.forward(xd, dev(f), border=border, out_dtype=torch.uint8)
    assert y.stride(1) == 1 and y.stride(3) == c  # output in the image's layout
    got = y.permute(0, 2, 3, 1).cpu().numpy()
    want = expect(planar_of(x), f, border, "u8").transpose(0, 2, 3, 1)
    assert np.array_equal(got, want)


def test_u8_bands_concatenate_to_the_whole(gpu_lib):
    x = wl.rng(85).integers(0, 256, (1, 2, 90, 300), dtype=np.uint8)
    f = (wl.rng(86).standard_normal((5, 5)) * 0.4).astype(np.float32)
    for border in ("zero", "clamp"):
        whole = gpu_lib.forward(dev(x), dev(f), border=border, out_dtype=torch.uint8)
        parts = []
        for y0, y1 in [(0, 13), (13, 50), (50, 90)]:
            lo, hi = max(0, y0 - 2), min(90, y1 + 2)
            parts.append(gpu_lib.forward(dev(x[:, :, lo:hi]), dev(f), border=border,
                                         rows=(y0 - lo, y1 - lo), out_dtype=torch.uint8))
        # a band's buffer holds every row its outputs read (the halo), and its
        # edges are the image's edges where it has no halo, so bands
        # concatenate to the whole image for both border rules
        assert torch.equal(torch.cat(parts, dim=2), whole)


# ------------------------------------------------------ fused upsampling ----
@pytest.mark.parametrize("s", [1, 2, 3, 5, 20])
@pytest.mark.parametrize("k", [3, 5])
@pytest.mark.parametrize("border", ["zero", "clamp"])
def test_upsample_then_filter_matches_oracle(gpu_lib, s, k, border):
    r = wl.rng(87, s, k)
    x = r.integers(0, 256, (1, 2, 23, 117), dtype=np.uint8)
    f = (r.standard_normal((k, k)) * 0.6).astype(np.float32)
    y = gpu_lib.upsample_forward(dev(x), dev(f), s, border=border, out_dtype=torch.uint8)
    assert y.shape == (1, 2, 23 * s, 117 * s)
    assert np.array_equal(y.cpu().numpy(), expect(x, f, border, "u8", scale=s))
    y32 = gpu_lib.upsample_forward(dev(x), dev(f), s, border=border)
    assert np.array_equal(y32.cpu().numpy(), expect(x, f, border, "f32", scale=s))


@pytest.mark.parametrize("s", [2, 7])
def test_upsample_interleaved_int_taps_and_laplacian(gpu_lib, s):
    r = wl.rng(88, s)
    x = r.integers(0, 256, (19, 341, 3), dtype=np.uint8)
    xd = hwc_dev(x)
    yl = gpu_lib.upsample_forward(xd, dev(LAP), s, border="zero", out_dtype=torch.uint8)
    want = expect(planar_of(x), LAP, "zero", "u8", scale=s)
    assert np.array_equal(yl.permute(0, 2, 3, 1).cpu().numpy(), want.transpose(0, 2, 3, 1))
    yi = gpu_lib.upsample_forward(xd, dev(LAP_I), s, border="clamp")
    want_i = expect(planar_of(x), LAP_I, "clamp", "i32", scale=s)
    assert np.array_equal(yi.permute(0, 2, 3, 1).cpu().numpy().astype(np.int64), want_i.transpose(0, 2, 3, 1))


def test_upsample_scale_one_equals_forward(gpu_lib):
    x = wl.rng(89).integers(0, 256, (1, 3, 50, 90), dtype=np.uint8)
    f = (wl.rng(90).standard_normal((3, 3))).astype(np.float32)
    a = gpu_lib.upsample_forward(dev(x), dev(f), 1, border="zero", out_dtype=torch.uint8)
    b = gpu_lib.forward(dev(x), dev(f), border="zero", out_dtype=torch.uint8)
    assert torch.equal(a, b)


def _pipeline_band_ref(x_hwc, s, y0, y1):
    """Oracle rows [y0, y1) of sharpen(upsample(x, s)) with zero borders, from
    the source rows those output rows (and their one-row halo) map to."""
    H = x_hwc.shape[0]
    lo, hi = max(0, y0 - 1), min(H * s, y1 + 1)
    src0, src1 = lo // s, (hi - 1) // s + 1
    up = oracle.upsample_nearest(planar_of(x_hwc[src0:src1]), s)[:, :, lo - src0 * s:hi - src0 * s]
    ref = oracle.to_u8(oracle.forward_f32(up, LAP, border="zero"))
    # the crop's top / bottom rows are true image edges only when lo == 0 / hi == H*s
    return ref[:, :, y0 - lo:y1 - lo]


@pytest.mark.timeout(300)
def test_paper_pipeline_4k_x20_full_size(gpu_lib):
    """Section 6.6's pipeline at its largest scale: a 4K RGB frame (interleaved
    8-bit), nearest upsampling x20 and the float Laplacian sharpen with
    skipped out-of-image neighbours, 8-bit out (43200 x 76800 x 3 = 9.95 GB),
    as the benchmark runs it; the top, a middle and the bottom row bands are
    compared with the oracle element by element (whole rows)."""
    s = 20
    x = wl.paper_frame_u8()
    xd = hwc_dev(x)
    y = gpu_lib.upsample_forward(xd, dev(LAP), s, border="zero", out_dtype=torch.uint8)
    torch.cuda.synchronize()
    H = x.shape[0] * s
    for (y0, y1) in [(0, 45), (21587, 21622), (H - 45, H)]:
        print(f"pipeline x20 rows {y0}..{y1}", flush=True)
        got = y[:, :, y0:y1].permute(0, 2, 3, 1).cpu().numpy().transpose(0, 3, 1, 2)
        assert np.array_equal(got, _pipeline_band_ref(x, s, y0, y1)), (y0, y1)
    del y
    torch.cuda.empty_cache()


# ------------------------------------------------------- channel mixing -----
@pytest.mark.parametrize("layout", ["planar", "interleaved"])
@pytest.mark.parametrize("out", ["u8", "f32"])
def test_paper_grayscale(gpu_lib, layout, out):
    """Section 4.2.5: gray = 0.299 R + 0.587 G + 0.114 B per pixel (BANK,
    K = 1), on planar and interleaved RGB."""
    x = wl.rng(91).integers(0, 256, (2, 37, 1030, 3), dtype=np.uint8)
    xd = hwc_dev(x) if layout == "interleaved" else dev(planar_of(x))
    y = gpu_lib.forward(xd, dev(GRAY), mode="bank", out_dtype=torch.uint8 if out == "u8" else None)
    want = expect(planar_of(x), GRAY, "clamp", out, mode="bank")
    assert np.array_equal(y.cpu().numpy(), want)


@pytest.mark.parametrize("cin,cout", [(1, 1), (2, 3), (4, 4), (3, 2)])
def test_channel_mix_general(gpu_lib, cin, cout):
    r = wl.rng(92, cin, cout)
    x = r.integers(0, 256, (1, 21, 517, cin), dtype=np.uint8)
    w = (r.standard_normal((cout, cin, 1, 1)) * 0.5).astype(np.float32)
    for xd in (dev(planar_of(x)), hwc_dev(x) if cin > 1 else None):
        if xd is None:
            continue
        y = gpu_lib.forward(xd, dev(w), mode="bank", out_dtype=torch.uint8)
        assert np.array_equal(y.cpu().numpy(), expect(planar_of(x), w, "clamp", "u8", mode="bank"))
    wi = r.integers(-3, 4, (cout, cin, 1, 1)).astype(np.int32)
    yi = gpu_lib.forward(dev(planar_of(x)), dev(wi), mode="bank")
    assert np.array_equal(yi.cpu().numpy().astype(np.int64), expect(planar_of(x), wi, "clamp", "i32", mode="bank"))


def test_grayscale_8k_full_size(gpu_lib):
    """An 8K RGB frame (interleaved) to 8-bit gray, as the benchmark runs it;
    sampled row bands element by element."""
    x = wl.paper_frame_u8(4320, 7680)
    y = gpu_lib.forward(hwc_dev(x), dev(GRAY), mode="bank", out_dtype=torch.uint8)
    for (y0, y1) in [(0, 8), (2000, 2016), (4312, 4320)]:
        want = expect(planar_of(x[y0:y1]), GRAY, "clamp", "u8", mode="bank")
        assert np.array_equal(y[:, :, y0:y1].cpu().numpy(), want)
