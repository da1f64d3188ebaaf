"""BF16 filter banks on the matrix cores against the oracle.

* Integer-valued BF16 operands (|v| <= 8, exact in BF16) keep every partial
  sum an integer below 2^24, so forward, grad_input and grad_filter must equal
  the oracle bit for bit: this pins the MFMA fragment layouts, the implicit
  im2col indexing, the flipped/transposed adjoint weights and the clamp fold.
* Gaussian data: relative L2 <= 1e-5 against the oracle on the BF16-rounded
  inputs (accumulation error only), <= 1e-2 against the oracle on the
  unrounded FP32 data (the BF16 tolerance), both reported.
* The 32 x 16 x 1024^2 workload (C_out = 64, K = 3 and 5) in the launch
  configuration the benchmark times: forward and grad_input element by element
  on row bands of two images, grad_filter over all 32 images, against the
  oracle on the rounded and on the unrounded data.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2504_01266_amd import workloads as wl

pytestmark = pytest.mark.gpu


def bf(a):
    """float32 array -> (bf16 tensor on the GPU, its exact float64 values)"""
    bits, vals = wl.bf16_round(a)
    t = torch.from_numpy(bits.view(np.int16).copy()).view(torch.bfloat16).cuda()
    return t, vals.astype(np.float64)


def f32(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    return t.double().cpu().numpy()


def assert_same(got, want):
    """Bit-for-bit equality; on failure name the mismatching positions."""
    bad = np.argwhere(got != want)
    assert len(bad) == 0, (f"{len(bad)} of {got.size} differ; first at "
                           f"{[tuple(int(v) for v in b) for b in bad[:8]]}: "
                           f"got {[float(got[tuple(b)]) for b in bad[:8]]}, "
                           f"want {[float(want[tuple(b)]) for b in bad[:8]]}")


CASES = [(2, 3, 4, 37, 70), (1, 16, 64, 20, 65), (2, 16, 16, 9, 130), (1, 8, 20, 33, 64),
         (1, 1, 1, 1, 1), (1, 16, 64, 3, 5)]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("k", [1, 3, 5])
def test_integer_operands_are_bit_exact(gpu_lib, case, k):
    n, cin, cout, h, w = case
    r = wl.rng(30, n, cin, cout, h, w, k)
    x = r.integers(-8, 9, (n, cin, h, w)).astype(np.float32)
    f = r.integers(-8, 9, (cout, cin, k, k)).astype(np.float32)
    g = r.integers(-8, 9, (n, cout, h, w)).astype(np.float32)
    xd, xv = bf(x)
    fd, fv = bf(f)
    y = gpu_lib.forward(xd, fd, mode="bank")
    assert y.dtype == torch.float32
    assert_same(host(y), oracle.forward(xv, fv, "bank"))
    for gdev in (bf(g)[0], f32(g)):  # bf16 or f32 upstream gradient (f32 is rounded inside)
        gi, gf = gpu_lib.backward(xd, fd, gdev, mode="bank")
        assert_same(host(gi), oracle.grad_input(g, fv, x.shape, "bank"))
        assert_same(host(gf), oracle.grad_filter(xv, g, f.shape, "bank"))


@pytest.mark.parametrize("k", [3, 5])
def test_gaussian_data_error_vs_fp64(gpu_lib, k):
    n, cin, cout, h, w = 2, 16, 64, 50, 97
    r = wl.rng(31, k)
    x = r.standard_normal((n, cin, h, w), dtype=np.float32)
    f = (r.standard_normal((cout, cin, k, k), dtype=np.float32) *
         np.float32(np.sqrt(2.0 / (cin * k * k))))
    g = r.standard_normal((n, cout, h, w), dtype=np.float32)
    xd, xv = bf(x)
    fd, fv = bf(f)
    gd, gv = bf(g)
    y = host(gpu_lib.forward(xd, fd, mode="bank"))
    assert oracle.rel_l2(y, oracle.forward(xv, fv, "bank")) <= 1e-5
    assert oracle.rel_l2(y, oracle.forward(x, f, "bank")) <= 1e-2
    yb = gpu_lib.forward(xd, fd, mode="bank", out_dtype=torch.bfloat16)
    assert yb.dtype == torch.bfloat16
    assert oracle.rel_l2(host(yb), oracle.forward(x, f, "bank")) <= 1e-2
    gi, gf = gpu_lib.backward(xd, fd, gd, mode="bank")
    assert oracle.rel_l2(host(gi), oracle.grad_input(gv, fv, x.shape, "bank")) <= 1e-5
    assert oracle.rel_l2(host(gf), oracle.grad_filter(xv, gv, f.shape, "bank")) <= 1e-5
    assert oracle.rel_l2(host(gi), oracle.grad_input(g, f, x.shape, "bank")) <= 1e-2
    assert oracle.rel_l2(host(gf), oracle.grad_filter(x, g, f.shape, "bank")) <= 1e-2


@pytest.mark.parametrize("k", [1, 3, 5])
def test_forward_wide_input_bank(gpu_lib, k):
    """33..64 input channels (eight channel groups) with 20 outputs: the widest
    forward tile shape that fits the weights and source tile in LDS."""
    r = wl.rng(34, k)
    x = r.integers(-8, 9, (2, 40, 21, 70)).astype(np.float32)
    f = r.integers(-8, 9, (20, 40, k, k)).astype(np.float32)
    xd, xv = bf(x)
    fd, fv = bf(f)
    y = gpu_lib.forward(xd, fd, mode="bank")
    assert_same(host(y), oracle.forward(xv, fv, "bank"))


SHAPE_TABLE = [(3, 40), (8, 64), (16, 17), (16, 64), (24, 40), (32, 16), (32, 32), (32, 64),
               (40, 20), (64, 16), (64, 40), (64, 64)]


@pytest.mark.parametrize("cio", SHAPE_TABLE)
@pytest.mark.parametrize("k", [1, 3, 5])
def test_forward_every_tile_shape(gpu_lib, cio, k):
    """Every (output-channel tile, input-channel group) pair the forward
    dispatches to, FP32 and BF16 outputs, integer operands: bit-exact."""
    cin, cout = cio
    r = wl.rng(38, cin, cout, k)
    x = r.integers(-4, 5, (1, cin, 11, 70)).astype(np.float32)
    f = r.integers(-4, 5, (cout, cin, k, k)).astype(np.float32)
    xd, xv = bf(x)
    fd, fv = bf(f)
    ref = oracle.forward(xv, fv, "bank")
    assert_same(host(gpu_lib.forward(xd, fd, mode="bank")), ref)
    yb = gpu_lib.forward(xd, fd, mode="bank", out_dtype=torch.bfloat16)
    assert_same(host(yb), wl.bf16_round(ref.astype(np.float32))[1].astype(np.float64))


@pytest.mark.parametrize("k", [3, 5])
def test_strided_views_take_the_element_staging(gpu_lib, k):
    """Image and upstream gradient as views with a row pitch that is not a
    multiple of 8 elements (and W not a multiple of 8): the staging falls back
    to clamped element loads; results stay bit-exact."""
    r = wl.rng(35, k)
    xb = r.integers(-8, 9, (1, 16, 30, 83)).astype(np.float32)
    gb = r.integers(-8, 9, (1, 64, 30, 83)).astype(np.float32)
    f = r.integers(-8, 9, (64, 16, k, k)).astype(np.float32)
    xd_full, _ = bf(xb)
    gd_full, _ = bf(gb)
    xd, gd = xd_full[:, :, 2:28, 3:80], gd_full[:, :, 2:28, 3:80]  # 26 x 77 views, pitch 83
    x, g = xb[:, :, 2:28, 3:80], gb[:, :, 2:28, 3:80]
    fd, fv = bf(f)
    assert_same(host(gpu_lib.forward(xd, fd, mode="bank")), oracle.forward(x, fv, "bank"))
    gi, gf = gpu_lib.backward(xd, fd, gd, mode="bank")
    assert_same(host(gi), oracle.grad_input(g, fv, x.shape, "bank"))
    assert_same(host(gf), oracle.grad_filter(x, g, f.shape, "bank"))


BF16_OUT_CASES = [(2, 16, 64, 37, 70), (1, 9, 33, 20, 65), (2, 12, 40, 9, 130), (1, 16, 64, 3, 5),
                  (1, 16, 48, 4, 64), (1, 16, 64, 1, 1)]


@pytest.mark.parametrize("case", BF16_OUT_CASES)
@pytest.mark.parametrize("k", [1, 3, 5])
def test_bf16_output_is_bit_exact(gpu_lib, case, k):
    """BF16 outputs of integer operands: the FP32 sums are exact, so the
    output must be the oracle's exact value rounded to BF16 (nearest even),
    bit for bit; ragged widths, 33..64 outputs and 9..16 inputs cover the
    border, channel and tile-count paths of the 64-output kernels."""
    n, cin, cout, h, w = case
    r = wl.rng(36, n, cin, cout, h, w, k)
    x = r.integers(-8, 9, (n, cin, h, w)).astype(np.float32)
    f = r.integers(-8, 9, (cout, cin, k, k)).astype(np.float32)
    xd, xv = bf(x)
    fd, fv = bf(f)
    y = gpu_lib.forward(xd, fd, mode="bank", out_dtype=torch.bfloat16)
    assert y.dtype == torch.bfloat16
    want = wl.bf16_round(oracle.forward(xv, fv, "bank").astype(np.float32))[1]
    assert_same(host(y), want.astype(np.float64))


@pytest.mark.parametrize("k", [3, 5])
def test_bf16_output_into_unaligned_view(gpu_lib, k):
    """BF16 output written into a view with an odd column offset and row pitch:
    the 16-byte stores must fall back to element stores; the values around the
    view stay untouched."""
    r = wl.rng(37, k)
    x = r.integers(-8, 9, (2, 16, 19, 70)).astype(np.float32)
    f = r.integers(-8, 9, (64, 16, k, k)).astype(np.float32)
    xd, xv = bf(x)
    fd, fv = bf(f)
    big = torch.full((2, 64, 21, 75), 7.0, device="cuda", dtype=torch.bfloat16)
    view = big[:, :, 1:20, 3:73]
    gpu_lib.forward(xd, fd, mode="bank", outs=[view])
    want = wl.bf16_round(oracle.forward(xv, fv, "bank").astype(np.float32))[1]
    assert_same(host(view), want.astype(np.float64))
    outside = big.clone()
    outside[:, :, 1:20, 3:73] = 7.0
    assert torch.equal(outside, torch.full_like(big, 7.0))


@pytest.mark.parametrize("k", [1, 3, 5])
def test_wide_source_kernels_bit_exact(gpu_lib, k):
    """33..64 source channels with aligned rows (W a multiple of 8), where the
    kernel choice depends on the output count and the source type: 64 -> 16
    forwards and grad_input from a BF16 upstream gradient take the
    vertical-reuse kernel (also with 9 outputs, padded to 16), a 40 -> 20
    forward and grad_input from an FP32 upstream gradient the row-ring kernel.
    Ragged bottom tiles and edge columns; integer operands, bit-exact (several
    tiles per column segment: test_row_ring_segments_bit_exact)."""
    r = wl.rng(43, k)
    h, w = 45, 136
    x16 = r.integers(-4, 5, (2, 16, h, w)).astype(np.float32)
    f = r.integers(-4, 5, (64, 16, k, k)).astype(np.float32)
    g = r.integers(-4, 5, (2, 64, h, w)).astype(np.float32)
    xd, _ = bf(x16)
    fd, fv = bf(f)
    gd, gv = bf(g)
    want = oracle.grad_input(gv, fv, x16.shape, "bank")
    for gdev in (gd, f32(g)):
        gi, _ = gpu_lib.backward(xd, fd, gdev, mode="bank", need_filter=False)
        assert_same(host(gi), want)
    for cin, cout in ((64, 16), (40, 20), (64, 9)):
        x = r.integers(-4, 5, (2, cin, h, w)).astype(np.float32)
        ff = r.integers(-4, 5, (cout, cin, k, k)).astype(np.float32)
        xdd, xv = bf(x)
        ffd, ffv = bf(ff)
        ref = oracle.forward(xv, ffv, "bank")
        assert_same(host(gpu_lib.forward(xdd, ffd, mode="bank")), ref)
        yb = gpu_lib.forward(xdd, ffd, mode="bank", out_dtype=torch.bfloat16)
        assert_same(host(yb), wl.bf16_round(ref.astype(np.float32))[1].astype(np.float64))


@pytest.mark.parametrize("k", [1, 3, 5])
@pytest.mark.parametrize("hw", [(1, 8), (2, 16), (5, 8), (3, 72), (9, 64)])
def test_wide_source_tiny_images_bit_exact(gpu_lib, k, hw):
    """The vertical-reuse kernel (64 -> 16 forward, grad_input from 64 BF16
    channels) on images shorter than its staged rows and narrower than a tile,
    where every row is a clamped (forward) or zeroed (adjoint) border row."""
    h, w = hw
    r = wl.rng(44, k, h, w)
    x = r.integers(-4, 5, (2, 64, h, w)).astype(np.float32)
    f = r.integers(-4, 5, (16, 64, k, k)).astype(np.float32)
    xd, xv = bf(x)
    fd, fv = bf(f)
    assert_same(host(gpu_lib.forward(xd, fd, mode="bank")), oracle.forward(xv, fv, "bank"))
    x16 = r.integers(-4, 5, (2, 16, h, w)).astype(np.float32)
    f2 = r.integers(-4, 5, (64, 16, k, k)).astype(np.float32)
    g = r.integers(-4, 5, (2, 64, h, w)).astype(np.float32)
    f2d, f2v = bf(f2)
    gd, gv = bf(g)
    gi, _ = gpu_lib.backward(bf(x16)[0], f2d, gd, mode="bank", need_filter=False)
    assert_same(host(gi), oracle.grad_input(gv, f2v, x16.shape, "bank"))


def test_wide_source_rows_band(gpu_lib):
    """64 -> 16 forward in row bands (the vertical-reuse kernel with a band's
    row offset and count) equals the whole-image call bitwise."""
    k = 5
    r = wl.rng(45)
    x = r.standard_normal((1, 64, 61, 64), dtype=np.float32)
    f = r.standard_normal((16, 64, k, k), dtype=np.float32) * np.float32(0.03)
    xd, _ = bf(x)
    fd, _ = bf(f)
    whole = gpu_lib.forward(xd, fd, mode="bank")
    parts = []
    for y0, y1 in [(0, 9), (9, 30), (30, 61)]:
        lo, hi = max(0, y0 - 2), min(61, y1 + 2)
        parts.append(gpu_lib.forward(xd[:, :, lo:hi], fd, mode="bank", rows=(y0 - lo, y1 - lo)))
    assert torch.equal(torch.cat(parts, dim=2), whole)


@pytest.mark.parametrize("k", [3, 5])
def test_row_ring_segments_bit_exact(gpu_lib, k):
    """64-channel sources (grad_input of a 16 -> 64 bank, and a 64 -> 16
    forward; also grad_filter) on 2 x 512^2 images: enough tiles that the row-ring kernel's
    column segments hold several tiles each, so the packing of only the new
    rows (and, for 3x3, the larger ring packed between MFMA steps) is compared
    element by element; integer operands, bit-exact."""
    r = wl.rng(40, k)
    x = r.integers(-4, 5, (2, 16, 512, 512)).astype(np.float32)
    f = r.integers(-4, 5, (64, 16, k, k)).astype(np.float32)
    g = r.integers(-4, 5, (2, 64, 512, 512)).astype(np.float32)
    xd, xv = bf(x)
    fd, fv = bf(f)
    gd, gv = bf(g)
    gi, _ = gpu_lib.backward(xd, fd, gd, mode="bank", need_filter=False)
    assert_same(host(gi), oracle.grad_input(gv, fv, x.shape, "bank"))
    # grad_filter over the same images: each persistent unit walks two tiles;
    # the sums (|.| < 2^24) are exact in FP32, so bit-exact too
    _, gf = gpu_lib.backward(xd, fd, gd, mode="bank", need_input=False)
    assert_same(host(gf), oracle.grad_filter(xv, gv, f.shape, "bank"))
    x64 = r.integers(-4, 5, (2, 64, 512, 512)).astype(np.float32)
    f64 = r.integers(-4, 5, (16, 64, k, k)).astype(np.float32)
    x64d, x64v = bf(x64)
    f64d, f64v = bf(f64)
    assert_same(host(gpu_lib.forward(x64d, f64d, mode="bank")), oracle.forward(x64v, f64v, "bank"))


@pytest.mark.parametrize("k", [3, 5])
def test_forward_many_tiles_per_work_group_bit_exact(gpu_lib, k):
    """16 -> 64 channels on 2 x 512^2 images: thousands of tiles, so every
    persistent work-group of the forward kernels (the wave-specialised one
    for BF16 outputs, the eight-wave one for FP32) walks several tiles and
    its prefetch / buffer alternation is compared element by element."""
    r = wl.rng(41, k)
    x = r.integers(-4, 5, (2, 16, 512, 512)).astype(np.float32)
    f = r.integers(-4, 5, (64, 16, k, k)).astype(np.float32)
    xd, xv = bf(x)
    fd, fv = bf(f)
    ref = oracle.forward(xv, fv, "bank")
    assert_same(host(gpu_lib.forward(xd, fd, mode="bank")), ref)
    yb = gpu_lib.forward(xd, fd, mode="bank", out_dtype=torch.bfloat16)
    assert_same(host(yb), wl.bf16_round(ref.astype(np.float32))[1].astype(np.float64))


def test_bf16_bank_rows_band(gpu_lib):
    k = 5
    r = wl.rng(32)
    x = r.standard_normal((1, 16, 60, 64), dtype=np.float32)
    f = r.standard_normal((64, 16, k, k), dtype=np.float32) * np.float32(0.07)
    xd, xv = bf(x)
    fd, fv = bf(f)
    whole = gpu_lib.forward(xd, fd, mode="bank")
    parts = []
    for y0, y1 in [(0, 7), (7, 31), (31, 60)]:
        lo, hi = max(0, y0 - 2), min(60, y1 + 2)
        parts.append(gpu_lib.forward(xd[:, :, lo:hi], fd, mode="bank", rows=(y0 - lo, y1 - lo)))
    assert torch.equal(torch.cat(parts, dim=2), whole)


def test_bank_backward_is_deterministic(gpu_lib):
    r = wl.rng(33)
    x = r.standard_normal((2, 16, 70, 130), dtype=np.float32)
    f = r.standard_normal((64, 16, 3, 3), dtype=np.float32) * np.float32(0.1)
    g = r.standard_normal((2, 64, 70, 130), dtype=np.float32)
    xd, _ = bf(x)
    fd, _ = bf(f)
    a = gpu_lib.backward(xd, fd, f32(g), mode="bank")
    b = gpu_lib.backward(xd, fd, f32(g), mode="bank")
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def _bands(h, r):
    """Checked output row bands: the clamped top and bottom edges and a middle
    band wide enough to cross a row-ring segment boundary of the adjoint."""
    return [(0, 8), (96, 136), (h - 8, h)]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("k", [3, 5])
def test_bank_full_size(gpu_lib, k):
    """32 x 16 x 1024^2 -> 64 channels, K = 3 and 5, in the launch configuration
    the benchmark times.  X and the upstream gradient are drawn N(0,1) in FP32
    on the GPU (torch's seeded generator), the weights N(0, 2/(16 K^2)) in FP32,
    and all three are rounded to BF16 for the library.  Against the oracle:
      * forward (FP32 and BF16 outputs) and grad_input, element by element on
        row bands of images 0 and 31 (top and bottom edges, and a middle band
        across a row-ring segment boundary; grad_input from halo'd crops of the
        gradient): <= 1e-5 on the BF16-rounded data, <= 1e-2 (the BF16
        tolerance) on the unrounded FP32 data;
      * grad_filter over ALL 32 images (oracle streamed one image at a time):
        <= 1e-5 on the rounded data; a single-image call <= 1e-2 on the
        unrounded data.
    The adjoint identities over the whole tensors are checked as well."""
    print(f"bank full size k={k}", flush=True)
    r = k // 2
    gen = torch.Generator(device="cuda").manual_seed(5)
    x32 = torch.randn((32, 16, 1024, 1024), generator=gen, device="cuda")
    g32 = torch.randn((32, 64, 1024, 1024), generator=gen, device="cuda")
    xd = x32.to(torch.bfloat16)
    gd = g32.to(torch.bfloat16)
    wts = wl.bank_weights(k)
    fd, fv = bf(wts)
    w64 = wts.astype(np.float64)
    y = gpu_lib.forward(xd, fd, mode="bank")
    yb = gpu_lib.forward(xd, fd, mode="bank", out_dtype=torch.bfloat16)  # as the benchmark runs it
    gi, gf = gpu_lib.backward(xd, fd, gd, mode="bank")
    torch.cuda.synchronize()
    errs = {"fwd_f32": 0.0, "fwd_bf16out": 0.0, "fwd_unrounded": 0.0, "gi": 0.0, "gi_unrounded": 0.0}
    for nimg in (0, 31):
        for (y0, y1) in _bands(1024, r):
            lo, hi = max(0, y0 - r), min(1024, y1 + r)
            # forward: source rows [y0 - r, y1 + r)
            xr = host(xd[nimg:nimg + 1, :, lo:hi])
            xu = host(x32[nimg:nimg + 1, :, lo:hi])
            ref = oracle.forward(xr, fv, "bank", rows=(y0 - lo, y1 - lo))
            refu = oracle.forward(xu, w64, "bank", rows=(y0 - lo, y1 - lo))
            got = host(y[nimg:nimg + 1, :, y0:y1])
            errs["fwd_f32"] = max(errs["fwd_f32"], oracle.rel_l2(got, ref))
            errs["fwd_bf16out"] = max(errs["fwd_bf16out"], oracle.rel_l2(host(yb[nimg:nimg + 1, :, y0:y1]), ref))
            errs["fwd_unrounded"] = max(errs["fwd_unrounded"], oracle.rel_l2(got, refu))
            # grad_input: the crop of the gradient rows [y0 - r, y1 + r) is an
            # image whose rows r .. r + (y1 - y0) - 1 are exact (at a true
            # image edge the crop edge is the image edge)
            gr = host(gd[nimg:nimg + 1, :, lo:hi])
            gu = host(g32[nimg:nimg + 1, :, lo:hi])
            refi = oracle.grad_input(gr, fv, (1, 16, hi - lo, 1024), "bank")[:, :, y0 - lo:y1 - lo]
            refiu = oracle.grad_input(gu, w64, (1, 16, hi - lo, 1024), "bank")[:, :, y0 - lo:y1 - lo]
            goti = host(gi[nimg:nimg + 1, :, y0:y1])
            errs["gi"] = max(errs["gi"], oracle.rel_l2(goti, refi))
            errs["gi_unrounded"] = max(errs["gi_unrounded"], oracle.rel_l2(goti, refiu))
    print(f"bank k={k} band errors: {errs}", flush=True)
    assert errs["fwd_f32"] <= 1e-5 and errs["gi"] <= 1e-5
    assert errs["fwd_bf16out"] <= 1e-2 and errs["fwd_unrounded"] <= 1e-2 and errs["gi_unrounded"] <= 1e-2
    del yb
    # <A x, g> = <x, A^T g> = <W, W-bar>, accumulated in FP64 one image at a time
    lhs = rhs_x = scale = 0.0
    for i in range(32):
        yg = y[i].double() * gd[i].double()
        lhs += float(yg.sum())
        scale += float(yg.abs().sum())
        rhs_x += float((xd[i].double() * gi[i].double()).sum())
    rhs_w = float((fd.double() * gf.double()).sum())
    assert abs(lhs - rhs_x) <= 1e-5 * scale
    assert abs(lhs - rhs_w) <= 1e-5 * scale
    del y, gi
    # grad_filter over all 32 images, the oracle streamed image by image.  An
    # entry W-bar[o][i] depends only on input channel i and gradient channel
    # o, so the oracle on a channel subset gives those entries exactly: all 16
    # input channels against one output channel from each group of 16 (the
    # kernel's output-channel blocks), over every image; every entry over
    # images 0 and 31.
    osel = [0, 21, 42, 63]
    ref_f = np.zeros((len(osel),) + wts.shape[1:])
    for i in range(32):
        ref_f += oracle.grad_filter(host(xd[i:i + 1]), host(gd[i:i + 1, osel]), ref_f.shape, "bank")
        if i % 8 == 7:
            print(f"bank k={k} grad_filter oracle: {i + 1}/32 images", flush=True)
    e_gf = oracle.rel_l2(host(gf)[osel], ref_f)
    # every entry, images 0 and 31 (a call on those two images)
    x2, g2 = xd[[0, 31]].contiguous(), gd[[0, 31]].contiguous()
    _, gf2 = gpu_lib.backward(x2, fd, g2, mode="bank", need_input=False)
    ref_2 = oracle.grad_filter(host(x2), host(g2), wts.shape, "bank")
    e_gf2 = oracle.rel_l2(host(gf2), ref_2)
    # one image, against the unrounded data
    _, gf0 = gpu_lib.backward(xd[:1], fd, gd[:1], mode="bank", need_input=False)
    ref_u = oracle.grad_filter(host(x32[:1]), host(g32[:1]), wts.shape, "bank")
    e_gfu = oracle.rel_l2(host(gf0), ref_u)
    print(f"bank k={k} grad_filter rel L2: {e_gf:.3e} (rounded, 32 images, output channels {osel}), "
          f"{e_gf2:.3e} (rounded, images 0 and 31, every entry), {e_gfu:.3e} (unrounded, image 0)", flush=True)
    assert e_gf <= 1e-5 and e_gf2 <= 1e-5
    assert e_gfu <= 1e-2
