"""Ragged batches in one persistent launch, against the oracle; the batched
result must also equal, bit for bit, the single-image call on each item
(same tile code, same per-pixel summation order), and a captured hipGraph
replay must equal the eager call."""
import numpy as np
import pytest
import torch

import oracle
from paper_2504_01266_amd import workloads as wl

pytestmark = pytest.mark.gpu

SIZES = [(1, 1, 1), (3, 70, 131), (2, 5, 7), (3, 64, 64), (1, 200, 33), (3, 1, 90), (2, 129, 1)]


def _batch(seed, k, sizes):
    xs, fs = [], []
    for i, (c, h, w) in enumerate(sizes):
        r = wl.rng(2000 + seed, i)
        xs.append(r.random((c, h, w), dtype=np.float32))
        fs.append((r.standard_normal((k, k), dtype=np.float32) / np.float32(k)).astype(np.float32))
    return xs, fs


def _run(B, xs, fs, variant=0):
    xd = [torch.from_numpy(x).cuda() for x in xs]
    fd = [torch.from_numpy(f).cuda() for f in fs]
    yd = [torch.full_like(x, float("nan")) for x in xd]
    batch = B.RaggedBatch(xd, yd, fd, variant=variant)
    batch.run()
    return batch, xd, fd, yd


@pytest.mark.parametrize("k", [1, 3, 7, 9])
def test_ragged_batch_matches_oracle_and_single_calls(gpu_lib, k):
    xs, fs = _batch(1, k, SIZES)
    batch, xd, fd, yd = _run(gpu_lib, xs, fs)
    for x, f, xdi, fdi, y in zip(xs, fs, xd, fd, yd):
        ref = oracle.forward(x[None], f.astype(np.float64))[0]
        assert oracle.rel_l2(y.double().cpu().numpy(), ref) <= 1e-5
        single = gpu_lib.forward(xdi, fdi)[0]
        assert torch.equal(single, y)


@pytest.mark.parametrize("variant", [1, 2, 3, 4, 5, 6, 7, 8])
def test_ragged_variants_bitwise(gpu_lib, variant):
    xs, fs = _batch(2, 7, SIZES)
    _, _, _, y1 = _run(gpu_lib, xs, fs, variant=1)
    batch, _, _, yv = _run(gpu_lib, xs, fs, variant=variant)
    assert batch.variant == variant
    for a, b in zip(y1, yv):
        assert torch.equal(a, b)


# Many items with empty ones between them: enough tiles that every
# work-group of the pipelined (persistent) variants walks several tiles, and
# its runs cross plane and item boundaries.
MANY = [(3, 97, 301), (0, 10, 10), (2, 257, 65), (1, 0, 40), (3, 33, 700), (2, 190, 190), (1, 30, 0),
        (3, 300, 129), (1, 1, 1), (2, 513, 77), (3, 64, 64), (1, 129, 400), (3, 700, 520),
        (2, 1100, 333)] * 6


@pytest.mark.parametrize("k", [3, 9])
@pytest.mark.parametrize("variant", [5, 6, 7, 8])
def test_ragged_pipelined_walks_across_items(gpu_lib, variant, k):
    xs, fs = _batch(6, k, MANY)
    batch, xd, fd, yd = _run(gpu_lib, xs, fs, variant=variant)
    assert batch.variant == variant
    # several tiles per work-group: at most 3 resident work-groups on each of 256 CUs
    assert batch.total_tiles > 3 * 768
    for i, (x, f, xdi, fdi, y) in enumerate(zip(xs, fs, xd, fd, yd)):
        if x.size == 0:
            continue
        single = gpu_lib.forward(xdi, fdi, variant=1)[0]
        assert torch.equal(single, y), i
        if i < len(MANY) // 6:
            ref = oracle.forward(x[None], f.astype(np.float64))[0]
            assert oracle.rel_l2(y.double().cpu().numpy(), ref) <= 1e-5, i


def test_ragged_graph_replay_equals_eager(gpu_lib):
    xs, fs = _batch(3, 7, SIZES)
    batch, xd, fd, yd = _run(gpu_lib, xs, fs)
    eager = [y.clone() for y in yd]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        batch.run()
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        batch.run()
    for rep in range(3):
        for y in yd:
            y.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for a, b in zip(eager, yd):
            assert torch.equal(a, b), f"replay {rep} differs"
        # eager work between replays
        gpu_lib.forward(xd[1], fd[1])
        torch.cuda.synchronize()


def test_ragged_autotune_and_empty(gpu_lib):
    xs, fs = _batch(4, 5, SIZES)
    batch, xd, fd, yd = _run(gpu_lib, xs, fs)
    ref = [y.clone() for y in yd]
    best = batch.autotune(reps=2)
    assert 1 <= best <= gpu_lib.variant_count(gpu_lib.PATH_BATCHED)
    for y in yd:
        y.zero_()
    batch.run()
    for a, b in zip(ref, yd):
        assert torch.equal(a, b)
    gpu_lib.tune_clear()
    # an empty item list is a no-op
    empty = gpu_lib.RaggedBatch([], [], [])
    assert empty.total_tiles == 0
    empty.run()


def test_ragged_table_for_another_variant_writes_nothing(gpu_lib):
    """A launch whose variant or K differs from the plan's (recorded in the
    table's tag) writes nothing: the NaN sentinels survive."""
    xs, fs = _batch(5, 5, SIZES)
    xd = [torch.from_numpy(x).cuda() for x in xs]
    fd = [torch.from_numpy(f).cuda() for f in fs]
    yd = [torch.full_like(x, float("nan")) for x in xd]
    batch = gpu_lib.RaggedBatch(xd, yd, fd, variant=2)
    for variant, k in ((1, 5), (3, 5), (4, 5), (6, 5), (8, 5), (2, 3), (2, 7)):
        batch.run(variant=variant, k=k)
        torch.cuda.synchronize()
        assert all(bool(torch.isnan(y).all()) for y in yd), (variant, k)
    batch.run()  # the planned variant and K
    torch.cuda.synchronize()
    for x, f, y in zip(xs, fs, yd):
        ref = oracle.forward(x[None], f.astype(np.float64))[0]
        assert oracle.rel_l2(y.double().cpu().numpy(), ref) <= 1e-5


def _band_rows(h, k):
    """Output row bands checked per image: the top and bottom 8 rows (the
    clamped edges) and 8 rows in the middle."""
    m = h // 2
    return sorted({(0, min(8, h)), (max(0, m - 4), min(h, m + 4)), (max(0, h - 8), h)})


def test_ragged_full_size(gpu_lib):
    """The 64-image ragged workload (H, W uniform in [256, 4096], 3 channels,
    per-image 7x7 filters): EVERY image against the oracle on row bands that
    include its top and bottom edge rows (all columns, so the left and right
    edge columns too), the smallest and the largest image whole, and every
    image bit-exact against its single-image call."""
    sizes = wl.ragged_sizes()
    print("ragged: 64 images, total px", int((sizes[:, 0] * sizes[:, 1]).sum()), flush=True)
    xs, fs = [], []
    for i, (h, w) in enumerate(sizes):
        x, f = wl.ragged_item(i, int(h), int(w))
        xs.append(x)
        fs.append(f)
    batch, xd, fd, yd = _run(gpu_lib, xs, fs)
    torch.cuda.synchronize()
    area = sizes[:, 0] * sizes[:, 1]
    whole = {int(np.argmin(area)), int(np.argmax(area))}
    worst = 0.0
    for i in range(len(xs)):
        h = xs[i].shape[1]
        f64 = fs[i].astype(np.float64)
        if i in whole:
            bands = [(0, h)]
        else:
            bands = _band_rows(h, 7)
        for y0, y1 in bands:
            # rows [y0, y1) need source rows [y0 - 3, y1 + 3) (clamped to the
            # image: at a true edge the crop edge is the image edge)
            lo, hi = max(0, y0 - 3), min(h, y1 + 3)
            ref = oracle.forward(xs[i][None, :, lo:hi], f64, rows=(y0 - lo, y1 - lo))[0]
            got = yd[i][:, y0:y1].double().cpu().numpy()
            e = oracle.rel_l2(got, ref)
            worst = max(worst, e)
            assert e <= 1e-5, (i, y0, y1, e)
    print(f"ragged: worst per-band rel L2 {worst:.3e} over 64 images", flush=True)
    for i in range(len(xs)):
        single = gpu_lib.forward(xd[i], fd[i])[0]
        assert torch.equal(single, yd[i]), i
