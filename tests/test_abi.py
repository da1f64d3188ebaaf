"""The C-ABI library: it loads, exports every symbol its header declares, and
rejects malformed calls on the host before anything is enqueued.  No call
here reaches a kernel, so these tests run without a GPU."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_2504_01266_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "filter2d.h")

FAKE = 0x100000  # never dereferenced: validation fails before any device access


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(filter2d_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.LIB_PATH):
        pytest.skip("libfilter2d.so not built")
    return B.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 14
    out = subprocess.run(["nm", "-D", "--defined-only", B.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (filter2d_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        assert hasattr(lib, n)


def test_struct_sizes_match_the_header(lib):
    assert ctypes.sizeof(B.F2dTensor) == 72
    assert ctypes.sizeof(B.F2dFilter) == 24
    assert ctypes.sizeof(B.F2dOpts) == 32
    assert ctypes.sizeof(B.F2dBatchItem) == 80


def test_version_and_status_strings(lib):
    assert lib.filter2d_version() >= 100
    assert b"EINVAL" in lib.filter2d_status_string(B.EINVAL)
    assert lib.filter2d_variant_count(B.PATH_F32) >= 1
    assert lib.filter2d_variant_count(B.PATH_U8) >= 1
    assert lib.filter2d_variant_count(99) == 0


def _img(dtype=B.F32, n=1, c=3, h=32, w=40):
    return B.F2dTensor(FAKE, dtype, 0, n, c, h, w, c * h * w, h * w, w)


def _filt(k=3, f_out=1, f_in=1, dtype=B.F32):
    return B.F2dFilter(FAKE, dtype, f_out, f_in, k)


def _fwd(lib, image, filt, opts, outs):
    arr = (B.F2dTensor * max(len(outs), 1))(*outs)
    return lib.filter2d_forward(ctypes.byref(image), ctypes.byref(filt), ctypes.byref(opts), arr,
                                len(outs), None)


CASES = [
    # (description, image, filter, opts, outs, expected status, message fragment)
    ("even K", _img(), _filt(k=4), B.make_opts(), [_img()], B.EINVAL, "odd"),
    ("K too large", _img(), _filt(k=33), B.make_opts(), [_img()], B.EINVAL, "odd"),
    ("shared needs 1x1 filter", _img(), _filt(f_out=2), B.make_opts(), [_img()], B.EINVAL, "SHARED"),
    ("depthwise f_out not multiple of C", _img(c=3), _filt(f_out=4), B.make_opts("depthwise"),
     [_img()], B.EINVAL, "multiple"),
    ("bank f_in != C", _img(c=3), _filt(f_out=4, f_in=2), B.make_opts("bank"), [_img()], B.EINVAL,
     "f_in"),
    ("zero border on bf16", _img(B.BF16), _filt(f_out=4, f_in=3, dtype=B.BF16),
     B.F2dOpts(B.BORDER_ZERO, B.BANK, 0, 0, 0, 0), [_img(c=4)], B.EUNSUPPORTED, "f32 and u8 images only"),
    ("zero border on u8 depthwise", _img(B.U8), _filt(f_out=6, dtype=B.I32),
     B.F2dOpts(B.BORDER_ZERO, B.DEPTHWISE, 0, 0, 0, 0), [_img(B.I32), _img(B.I32)], B.EUNSUPPORTED,
     "DEPTHWISE"),
    ("u8 bank k > 1", _img(B.U8), _filt(f_out=1, f_in=3, dtype=B.F32), B.make_opts("bank"),
     [_img(B.U8, c=1)], B.EUNSUPPORTED, "k = 1"),
    ("u8 bank more than 4 channels", _img(B.U8, c=5), _filt(k=1, f_out=1, f_in=5, dtype=B.F32),
     B.make_opts("bank"), [_img(B.U8, c=1)], B.EUNSUPPORTED, "at most 4"),
    ("u8 shared float taps k > 7", _img(B.U8), _filt(k=9, dtype=B.F32), B.make_opts(), [_img(B.U8)],
     B.EUNSUPPORTED, "k <= 7"),
    ("u8 int taps with f32 outputs", _img(B.U8), _filt(dtype=B.I32), B.make_opts(border="zero"),
     [_img(B.F32)], B.EINVAL, "dtype"),
    ("u8 float taps with i32 outputs", _img(B.U8), _filt(dtype=B.F32), B.make_opts(), [_img(B.I32)],
     B.EINVAL, "dtype"),
    ("interleaved f32 image", B.F2dTensor(FAKE, B.F32, 3, 1, 3, 32, 40, 3840, 1, 120), _filt(),
     B.make_opts(), [_img()], B.EUNSUPPORTED, "u8 images only"),
    ("interleaved u8 in, planar out", B.F2dTensor(FAKE, B.U8, 3, 1, 3, 32, 40, 3840, 1, 120),
     _filt(dtype=B.F32), B.make_opts(), [_img(B.U8)], B.EINVAL, "layout"),
    ("interleaved output channels overlap", B.F2dTensor(FAKE, B.U8, 3, 1, 3, 32, 40, 3840, 1, 120),
     _filt(dtype=B.F32), B.make_opts(), [B.F2dTensor(FAKE, B.U8, 2, 1, 3, 32, 40, 3840, 1, 80)],
     B.EINVAL, "channels overlap"),
    ("unknown border", _img(), _filt(), B.F2dOpts(7, 0, 0, 0, 0, 0), [_img()], B.EINVAL, "border"),
    ("wrong output count", _img(), _filt(), B.make_opts(), [_img(), _img()], B.EINVAL, "expected 1"),
    ("wrong output shape", _img(), _filt(), B.make_opts(), [_img(h=31)], B.EINVAL, "shape"),
    ("band outside image", _img(h=32), _filt(), B.make_opts(rows=(10, 40)), [_img(h=30)], B.EINVAL,
     "outside"),
    ("negative stride", _img(), _filt(), B.make_opts(),
     [B.F2dTensor(FAKE, B.F32, 0, 1, 3, 32, 40, -1, 1280, 40)], B.EINVAL, "stride"),
    ("null output data", _img(), _filt(), B.make_opts(),
     [B.F2dTensor(None, B.F32, 0, 1, 3, 32, 40, 3840, 1280, 40)], B.EINVAL, "NULL"),
    ("overlapping output rows", _img(), _filt(), B.make_opts(),
     [B.F2dTensor(FAKE, B.F32, 0, 1, 3, 32, 40, 3840, 1280, 20)], B.EINVAL, "stride_h"),
    ("u8 needs int32 or float filter", _img(B.U8), _filt(dtype=B.BF16), B.make_opts(), [_img(B.I32)],
     B.EINVAL, "int32 or float"),
    ("u8 output must be int32", _img(B.U8), _filt(dtype=B.I32), B.make_opts(), [_img(B.F32)],
     B.EINVAL, "dtype"),
    ("sumsq needs depthwise m=2", _img(B.U8), _filt(dtype=B.I32),
     B.make_opts("shared", B.EPI_SUMSQ_PAIRS), [_img(B.I32)], B.EINVAL, "SUMSQ"),
    ("bf16 only for banks", _img(B.BF16), _filt(dtype=B.BF16), B.make_opts(), [_img()],
     B.EUNSUPPORTED, "BANK"),
    ("null filter data", _img(), B.F2dFilter(None, B.F32, 1, 1, 3), B.make_opts(), [_img()],
     B.EINVAL, "NULL"),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_forward_rejects_on_the_host(lib, case):
    _, image, filt, opts, outs, status, frag = case
    assert _fwd(lib, image, filt, opts, outs) == status
    assert frag.lower() in B.last_error().lower()


SEP_CASES = [
    # (description, image, a, k, opts, out, expected status, message fragment)
    ("null factor", _img(), None, 3, B.make_opts(), _img(), B.EINVAL, "NULL"),
    ("even K", _img(), FAKE, 4, B.make_opts(), _img(), B.EINVAL, "odd"),
    ("K beyond the built range", _img(), FAKE, 17, B.make_opts(), _img(), B.EUNSUPPORTED, "1..15"),
    ("u8 image", _img(B.U8), FAKE, 3, B.make_opts(), _img(B.I32), B.EUNSUPPORTED, "f32 images only"),
    ("depthwise mode", _img(), FAKE, 3, B.make_opts("depthwise"), _img(), B.EUNSUPPORTED, "SHARED"),
    ("wrong output shape", _img(), FAKE, 3, B.make_opts(), _img(w=39), B.EINVAL, "shape"),
    ("band outside image", _img(h=32), FAKE, 3, B.make_opts(rows=(10, 40)), _img(h=30), B.EINVAL,
     "outside"),
    ("zero border", _img(), FAKE, 3, B.make_opts(border="zero"), _img(), B.EUNSUPPORTED, "clamp"),
]


@pytest.mark.parametrize("case", SEP_CASES, ids=[c[0] for c in SEP_CASES])
def test_forward_separable_rejects_on_the_host(lib, case):
    _, image, a, k, opts, out, status, frag = case
    st = lib.filter2d_forward_separable(ctypes.byref(image), a, FAKE, k, ctypes.byref(opts),
                                        ctypes.byref(out), None)
    assert st == status
    assert frag.lower() in B.last_error().lower()


def test_backward_validation_on_the_host(lib):
    image, filt = _img(), _filt(k=3)
    opts = B.make_opts()
    g = (B.F2dTensor * 1)(_img())
    # u8 images are not differentiable
    st = lib.filter2d_backward(ctypes.byref(_img(B.U8)), ctypes.byref(_filt(dtype=B.I32)), g, 1,
                               ctypes.byref(opts), None, None, None, 0, None)
    assert st == B.EUNSUPPORTED
    # bands are forward-only
    st = lib.filter2d_backward(ctypes.byref(image), ctypes.byref(filt), g, 1,
                               ctypes.byref(B.make_opts(rows=(0, 8))), None, None, None, 0, None)
    assert st == B.EUNSUPPORTED
    # zero borders are forward-only
    zopts = B.make_opts(border="zero")
    st = lib.filter2d_backward(ctypes.byref(image), ctypes.byref(filt), g, 1,
                               ctypes.byref(zopts), None, None, None, 0, None)
    assert st == B.EUNSUPPORTED and "zero" in B.last_error().lower()
    assert lib.filter2d_backward_workspace(ctypes.byref(image), ctypes.byref(filt), ctypes.byref(zopts)) == 0
    # even K
    st = lib.filter2d_backward(ctypes.byref(image), ctypes.byref(_filt(k=2)), g, 1,
                               ctypes.byref(opts), None, None, None, 0, None)
    assert st == B.EINVAL
    assert lib.filter2d_backward_workspace(ctypes.byref(image), ctypes.byref(_filt(k=2)),
                                           ctypes.byref(opts)) == 0


NOALLOC_SCRATCH_BYTES = 96 << 20  # F2D_NOALLOC_SCRATCH_BYTES


def test_header_states_the_noalloc_scratch_size():
    text = open(HEADER).read()
    assert re.search(r"#define F2D_NOALLOC_SCRATCH_BYTES \(\(size_t\)96 << 20\)", text)


def test_backward_noalloc_validation_on_the_host(lib):
    """Invalid calls and calls whose workspace exceeds the static scratch are
    rejected before any device access."""
    image, filt = _img(), _filt(k=3)
    opts = B.make_opts()
    g = (B.F2dTensor * 1)(_img())
    st = lib.filter2d_backward_noalloc(ctypes.byref(_img(B.U8)), ctypes.byref(_filt(dtype=B.I32)), g, 1,
                                       ctypes.byref(opts), None, None, None)
    assert st == B.EUNSUPPORTED
    st = lib.filter2d_backward_noalloc(ctypes.byref(image), ctypes.byref(filt), g, 2,
                                       ctypes.byref(opts), None, None, None)
    assert st == B.EINVAL
    st = lib.filter2d_backward_noalloc(ctypes.byref(image), ctypes.byref(filt), g, 1,
                                       ctypes.byref(B.make_opts(border="zero")), None, None, None)
    assert st == B.EUNSUPPORTED
    # a 256-image 5x5 BF16 bank: its workspace is larger than the static scratch
    n, c, h, w = 256, 16, 1024, 1024
    big = B.F2dTensor(FAKE, B.BF16, 0, n, c, h, w, c * h * w, h * w, w)
    bf = B.F2dFilter(FAKE, B.BF16, 64, 16, 5)
    bopts = B.make_opts("bank")
    need = lib.filter2d_backward_workspace(ctypes.byref(big), ctypes.byref(bf), ctypes.byref(bopts))
    assert need > NOALLOC_SCRATCH_BYTES
    gb = (B.F2dTensor * 1)(B.F2dTensor(FAKE, B.BF16, 0, n, 64, h, w, 64 * h * w, h * w, w))
    gi = B.F2dTensor(FAKE, B.F32, 0, n, c, h, w, c * h * w, h * w, w)
    st = lib.filter2d_backward_noalloc(ctypes.byref(big), ctypes.byref(bf), gb, 1, ctypes.byref(bopts),
                                       ctypes.byref(gi), FAKE, None)
    assert st == B.EWORKSPACE and "scratch" in B.last_error()
    # the 32-image 5x5 bank of the benchmark fits
    big32 = B.F2dTensor(FAKE, B.BF16, 0, 32, c, h, w, c * h * w, h * w, w)
    assert lib.filter2d_backward_workspace(ctypes.byref(big32), ctypes.byref(bf),
                                           ctypes.byref(bopts)) <= NOALLOC_SCRATCH_BYTES


UP_CASES = [
    # (description, image, filter, scale, opts, out, expected status, message fragment)
    ("scale 0", _img(B.U8), _filt(dtype=B.F32), 0, B.make_opts(), _img(B.U8), B.EINVAL, "scale"),
    ("f32 image", _img(), _filt(), 2, B.make_opts(), _img(h=64, w=80), B.EUNSUPPORTED, "u8 images only"),
    ("depthwise", _img(B.U8), _filt(f_out=3, dtype=B.I32), 2, B.make_opts("depthwise"),
     _img(B.U8, h=64, w=80), B.EUNSUPPORTED, "SHARED"),
    ("band", _img(B.U8), _filt(dtype=B.F32), 2, B.make_opts(rows=(0, 16)), _img(B.U8, h=32, w=80),
     B.EUNSUPPORTED, "whole images"),
    ("wrong out shape", _img(B.U8), _filt(dtype=B.F32), 2, B.make_opts(), _img(B.U8, h=64, w=79),
     B.EINVAL, "H*scale"),
    ("wrong out dtype", _img(B.U8), _filt(dtype=B.F32), 2, B.make_opts(), _img(B.I32, h=64, w=80),
     B.EINVAL, "dtype"),
    ("k 9", _img(B.U8), _filt(k=9, dtype=B.F32), 2, B.make_opts(), _img(B.U8, h=64, w=80),
     B.EUNSUPPORTED, "k <= 7"),
]


@pytest.mark.parametrize("case", UP_CASES, ids=[c[0] for c in UP_CASES])
def test_upsample_forward_rejects_on_the_host(lib, case):
    _, image, filt, scale, opts, out, status, frag = case
    st = lib.filter2d_upsample_forward(ctypes.byref(image), ctypes.byref(filt), scale, ctypes.byref(opts),
                                       ctypes.byref(out), None)
    assert st == status
    assert frag.lower() in B.last_error().lower()


def test_batched_plan_validation_on_the_host(lib):
    item = B.F2dBatchItem(FAKE, FAKE, FAKE, 3, 10, 12, 120, 12, 120, 12)
    items = (B.F2dBatchItem * 2)(item, item)
    prefix = (ctypes.c_int64 * 4)()  # n_items + 1 prefix sums, then the plan's tag
    var = ctypes.c_int32(0)
    assert lib.filter2d_batched_plan(items, 2, B.F32, 4, ctypes.byref(var), prefix) == -B.EINVAL
    assert lib.filter2d_batched_plan(items, 2, B.U8, 3, ctypes.byref(var), prefix) == -B.EUNSUPPORTED
    bad = B.F2dBatchItem(FAKE, FAKE, FAKE, 3, -1, 12, 120, 12, 120, 12)
    items2 = (B.F2dBatchItem * 1)(bad)
    assert lib.filter2d_batched_plan(items2, 1, B.F32, 3, ctypes.byref(var), prefix) == -B.EINVAL
    total = lib.filter2d_batched_plan(items, 2, B.F32, 3, ctypes.byref(var), prefix)
    assert total > 0 and var.value >= 1
    assert prefix[0] == 0 and prefix[2] == total and prefix[1] == total // 2
    # extents of 2^31 and more are rejected (the kernels clamp in 32 bits)
    for h, w in ((1 << 31, 12), (10, 1 << 31)):
        huge = B.F2dBatchItem(FAKE, FAKE, FAKE, 1, h, w, h * w, w, h * w, w)
        items3 = (B.F2dBatchItem * 1)(huge)
        assert lib.filter2d_batched_plan(items3, 1, B.F32, 3, ctypes.byref(var), prefix) == -B.EUNSUPPORTED
        assert "2^31" in B.last_error()
    # variants past the last are rejected
    var = ctypes.c_int32(lib.filter2d_variant_count(B.PATH_BATCHED) + 1)
    assert lib.filter2d_batched_plan(items, 2, B.F32, 3, ctypes.byref(var), prefix) == -B.EINVAL


def test_batched_plan_tags_the_table(lib):
    """The plan's last word records the tiling variant and K, so that the
    kernel can recognise a table planned for another tile shape (whose tile
    counts would send tiles past an item's planes) and write nothing."""
    item = B.F2dBatchItem(FAKE, FAKE, FAKE, 3, 100, 300, 30000, 300, 30000, 300)
    items = (B.F2dBatchItem * 1)(item)
    tags, totals = {}, {}
    for v in range(1, lib.filter2d_variant_count(B.PATH_BATCHED) + 1):
        for k in (3, 7):
            prefix = (ctypes.c_int64 * 3)()
            var = ctypes.c_int32(v)
            totals[v, k] = lib.filter2d_batched_plan(items, 1, B.F32, k, ctypes.byref(var), prefix)
            assert var.value == v and prefix[1] == totals[v, k]
            tags[v, k] = prefix[2]
    assert len(set(tags.values())) == len(tags), "every (variant, K) has its own tag"
    assert len(set(totals.values())) > 1, "tile counts depend on the variant"
    assert all(totals[v, 3] == totals[v, 7] for v, _ in totals), "tile counts do not depend on K"
    # an empty batch still carries the tag after its single prefix word
    prefix = (ctypes.c_int64 * 2)()
    var = ctypes.c_int32(1)
    assert lib.filter2d_batched_plan(items, 0, B.F32, 3, ctypes.byref(var), prefix) == 0
    assert prefix[0] == 0 and prefix[1] == tags[1, 3]


def test_bf16_bank_k_contract(lib):
    """BF16 banks are built for K in {1, 3, 5}; K = 7 and 9 are rejected on
    the host with F2D_EUNSUPPORTED (forward, backward and workspace query)."""
    image = _img(B.BF16, c=16)
    opts = B.make_opts("bank")
    for k in (7, 9):
        filt = _filt(k=k, f_out=64, f_in=16, dtype=B.BF16)
        assert _fwd(lib, image, filt, opts, [_img(B.F32, c=64)]) == B.EUNSUPPORTED
        assert "k in {1, 3, 5}" in B.last_error()
        g = (B.F2dTensor * 1)(_img(B.BF16, c=64))
        st = lib.filter2d_backward(ctypes.byref(image), ctypes.byref(filt), g, 1, ctypes.byref(opts),
                                   None, None, None, 0, None)
        assert st == B.EUNSUPPORTED
        assert lib.filter2d_backward_workspace(ctypes.byref(image), ctypes.byref(filt), ctypes.byref(opts)) == 0


def test_tune_table_roundtrip(lib, tmp_path):
    p = tmp_path / "tune.json"
    lib.filter2d_tune_clear()
    assert lib.filter2d_tune_save(str(p).encode()) == B.OK
    assert '"entries"' in p.read_text()
    p.write_text('{"format": "filter2d-tune-1", "entries": [[0, 2, 5, 0, 3, 2], [1, 0, 3, 1, 3, 4]]}')
    assert lib.filter2d_tune_load(str(p).encode()) == B.OK
    q = tmp_path / "tune2.json"
    assert lib.filter2d_tune_save(str(q).encode()) == B.OK
    assert "[0, 2, 5, 0, 3, 2]" in q.read_text() and "[1, 0, 3, 1, 3, 4]" in q.read_text()
    lib.filter2d_tune_clear()
    assert lib.filter2d_tune_load(b"/nonexistent/tune.json") == B.EINVAL

