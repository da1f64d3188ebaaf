"""GPU adjoints against the oracle: grad_input (with the clamp fold at the
borders) and grad_filter, FP32, relative L2 <= 1e-5; adjoint identity,
finite differences on crops of the 16 x 3 x 2048^2 workload, determinism,
and the autograd wrapper."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from paper_2504_01266_amd import autograd as AG
from paper_2504_01266_amd import workloads as wl

pytestmark = pytest.mark.gpu

TOL = 1e-5


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def rel(gpu, ref):
    return oracle.rel_l2(gpu.double().cpu().numpy(), ref)


SHAPES = [(1, 1, 1, 1), (1, 1, 1, 9), (1, 1, 7, 1), (1, 2, 5, 7), (1, 1, 3, 3), (2, 3, 67, 131),
          (1, 1, 130, 257)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("k", [1, 3, 5, 9, 11])
def test_shared_backward_matches_oracle(gpu_lib, shape, k):
    x, f = wl.random_case(21, *shape, k)
    g = wl.rng(21, 9, *shape, k).standard_normal(shape, dtype=np.float32)
    gi, gf = gpu_lib.backward(dev(x), dev(f[0, 0]), dev(g))
    assert rel(gi, oracle.grad_input(g, f.astype(np.float64), shape)) <= TOL
    ref_f = oracle.grad_filter(x, g, f.shape)[0, 0]
    assert rel(gf, ref_f) <= TOL


@pytest.mark.parametrize("m", [1, 2, 3])
@pytest.mark.parametrize("k", [3, 5, 13])
def test_depthwise_backward(gpu_lib, m, k):
    c = 3
    shape = (2, c, 37, 70)
    x, f = wl.random_case(22, *shape, k, fo=c * m, fi=1)
    g = wl.rng(22, 9, m, k).standard_normal((2, c * m, 37, 70), dtype=np.float32)
    gs = [dev(g[:, j::m]) for j in range(m)]
    gi, gf = gpu_lib.backward(dev(x), dev(f), gs, mode="depthwise")
    assert rel(gi, oracle.grad_input(g, f.astype(np.float64), shape, "depthwise")) <= TOL
    assert rel(gf, oracle.grad_filter(x, g, f.shape, "depthwise")) <= TOL


@pytest.mark.parametrize("cout", [1, 4])
@pytest.mark.parametrize("k", [1, 3, 5])
def test_bank_backward_f32(gpu_lib, cout, k):
    cin = 3
    shape = (2, cin, 33, 47)
    x, f = wl.random_case(23, *shape, k, fo=cout, fi=cin)
    g = wl.rng(23, 9, cout, k).standard_normal((2, cout, 33, 47), dtype=np.float32)
    gi, gf = gpu_lib.backward(dev(x), dev(f), dev(g), mode="bank")
    assert rel(gi, oracle.grad_input(g, f.astype(np.float64), shape, "bank")) <= TOL
    assert rel(gf, oracle.grad_filter(x, g, f.shape, "bank")) <= TOL


@pytest.mark.parametrize("cio", [(4, 8), (8, 12), (6, 8), (4, 6)])
@pytest.mark.parametrize("k", [1, 3, 5])
def test_bank_backward_f32_channel_groups(gpu_lib, cio, k):
    """FP32 banks whose channel counts the grouped kernels divide: grad_input
    with four image channels per work-group (C_in % 4 == 0, K <= 5) and
    grad_filter with 4 x 2 (K <= 3) or 2 x 2 (K = 5) filter pairs per
    work-group; (6, 8) takes the one-channel grad_input and (4, 6) the
    one-pair grad_filter at K <= 3.  Integer
    values keep every sum exact, so both results are bit-exact; two tile rows
    and columns with ragged edges."""
    cin, cout = cio
    r = wl.rng(24, cin, cout, k)
    shape = (2, cin, 70, 133)
    x = r.integers(-4, 5, shape).astype(np.float32)
    f = r.integers(-4, 5, (cout, cin, k, k)).astype(np.float32)
    g = r.integers(-4, 5, (2, cout, 70, 133)).astype(np.float32)
    gi, gf = gpu_lib.backward(dev(x), dev(f), dev(g), mode="bank")
    want_i = oracle.grad_input(g.astype(np.float64), f.astype(np.float64), shape, "bank")
    want_f = oracle.grad_filter(x.astype(np.float64), g.astype(np.float64), f.shape, "bank")
    assert np.array_equal(gi.double().cpu().numpy(), want_i)
    assert np.array_equal(gf.double().cpu().numpy(), want_f)


@pytest.mark.parametrize("hw", [(1, 1), (2, 3), (6, 5), (40, 33)])
def test_adjoint_identity_on_gpu(gpu_lib, hw):
    k = 7
    x, f = wl.random_case(24, 1, 2, *hw, k)
    g = wl.rng(24, 9, *hw).standard_normal((1, 2) + hw, dtype=np.float32)
    y = gpu_lib.forward(dev(x), dev(f[0, 0])).double().cpu().numpy()
    gi, gf = gpu_lib.backward(dev(x), dev(f[0, 0]), dev(g))
    lhs = float(np.sum(y * g))
    scale = float(np.sum(np.abs(y * g))) + 1e-30
    assert abs(lhs - float(np.sum(x * gi.double().cpu().numpy()))) <= TOL * scale
    assert abs(lhs - float(np.sum(f[0, 0] * gf.double().cpu().numpy()))) <= TOL * scale


def test_backward_is_deterministic(gpu_lib):
    x, f = wl.random_case(25, 2, 3, 300, 257, 9)
    g = wl.rng(25, 9).standard_normal(x.shape, dtype=np.float32)
    a = gpu_lib.backward(dev(x), dev(f[0, 0]), dev(g))
    b = gpu_lib.backward(dev(x), dev(f[0, 0]), dev(g))
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_workspace_too_small_is_rejected(gpu_lib):
    from paper_2504_01266_amd import binding as B

    x, f = wl.random_case(26, 1, 1, 64, 64, 3)
    xd, fd = dev(x), dev(f)
    lib = B.load()
    need = gpu_lib.backward_workspace(xd, fd)
    assert need > 0
    ws = torch.empty(need - 1, dtype=torch.uint8, device="cuda")
    gf = torch.empty((1, 1, 3, 3), device="cuda")
    fdesc, _ = B.filter_desc(fd)
    gd = (B.F2dTensor * 1)(B.tensor_desc(xd))
    st = lib.filter2d_backward(ctypes.byref(B.tensor_desc(xd)), ctypes.byref(fdesc), gd, 1,
                               ctypes.byref(B.make_opts()), None, ctypes.c_void_p(gf.data_ptr()),
                               ctypes.c_void_p(ws.data_ptr()), need - 1, None)
    assert st == B.EWORKSPACE


def test_autograd_wrapper(gpu_lib):
    x, f = wl.random_case(27, 2, 3, 45, 61, 5)
    g = wl.rng(27, 9).standard_normal(x.shape, dtype=np.float32)
    xd = dev(x).requires_grad_(True)
    fd = dev(f[0, 0]).requires_grad_(True)
    y = AG.filter2d(xd, fd)
    (y * dev(g)).sum().backward()
    gi, gf = gpu_lib.backward(dev(x), dev(f[0, 0]), dev(g))
    assert torch.equal(xd.grad, gi) and torch.equal(fd.grad, gf)
    # depthwise: two outputs, two upstream gradients
    fdw = wl.rng(27, 3).standard_normal((6, 1, 3, 3), dtype=np.float32)
    xd2 = dev(x).requires_grad_(True)
    fdw_d = dev(fdw).requires_grad_(True)
    o0, o1 = AG.filter2d(xd2, fdw_d, "depthwise")
    (o0 * dev(g) + 2.0 * o1 * dev(g)).sum().backward()
    gcat = np.empty((2, 6, 45, 61), np.float32)
    gcat[:, 0::2] = g
    gcat[:, 1::2] = 2.0 * g
    assert rel(xd2.grad, oracle.grad_input(gcat, fdw.astype(np.float64), x.shape, "depthwise")) <= TOL
    assert rel(fdw_d.grad, oracle.grad_filter(x, gcat, fdw.shape, "depthwise")) <= TOL


def test_finite_differences_on_diff_crops(gpu_lib):
    """All 8 seeded 64 x 64 crops of the 16 x 3 x 2048^2 workload, each an independent image
    (clamped at the crop's own edges): the FP64 central difference of
    L(x, F) = <filter(x; F), G> (exact for any step since L is linear) along
    random and unit directions against the GPU gradients."""
    f = wl.diff_filter()
    x0 = wl.diff_image(0)
    g0 = wl.diff_grad(0)
    rng = wl.rng(4, 7)
    origins = wl.diff_crop_origins()
    assert len(origins) == 8 and (0, 0) in [tuple(o) for o in origins]
    for (oy, ox) in origins:
        xc = x0[None, :, oy:oy + 64, ox:ox + 64].copy()
        gc = g0[None, :, oy:oy + 64, ox:ox + 64].copy()
        gi, gf = gpu_lib.backward(dev(xc), dev(f), dev(gc))
        gi = gi.double().cpu().numpy()
        gf = gf.double().cpu().numpy()

        def loss(xv, fv):
            return float(np.sum(oracle.forward(xv, fv) * gc))

        f64 = f.astype(np.float64)
        dirs = [rng.standard_normal(xc.shape)]
        for (yy, xx) in [(0, 0), (0, 63), (63, 0), (63, 63), (0, 30), (30, 0), (31, 32)]:
            e = np.zeros(xc.shape)
            e[0, 1, yy, xx] = 1.0
            dirs.append(e)
        for d in dirs:
            fd = (loss(xc + d, f64) - loss(xc - d, f64)) / 2.0
            scale = float(np.sum(np.abs(gi * d))) + 1e-12
            assert abs(fd - float(np.sum(gi * d))) <= 1e-5 * max(scale, abs(fd)), (oy, ox)
        d = rng.standard_normal(f.shape)
        fdv = (loss(xc, f64 + d) - loss(xc, f64 - d)) / 2.0
        assert abs(fdv - float(np.sum(gf * d))) <= 1e-5 * max(abs(fdv), float(np.sum(np.abs(gf * d))))


def test_diff_full_size(gpu_lib):
    """16 x 3 x 2048^2, shared 9x9: forward and grad_input of images 0 and 15
    against the oracle, grad_filter over all 16 images against the oracle."""
    f = wl.diff_filter()
    xs = np.stack([wl.diff_image(i) for i in range(16)])
    gs = np.stack([wl.diff_grad(i) for i in range(16)])
    print("diff: 16x3x2048x2048 9x9 fwd+bwd", flush=True)
    xd, fd, gd = dev(xs), dev(f), dev(gs)
    y = gpu_lib.forward(xd, fd)
    gi, gf = gpu_lib.backward(xd, fd, gd)
    torch.cuda.synchronize()
    f64 = f.astype(np.float64)
    for n in (0, 15):
        assert rel(y[n:n + 1], oracle.forward(xs[n:n + 1], f64)) <= TOL
        assert rel(gi[n:n + 1], oracle.grad_input(gs[n:n + 1], f64, (1, 3, 2048, 2048))) <= TOL
    ref_f = oracle.grad_filter(xs, gs, (1, 1, 9, 9))[0, 0]
    assert rel(gf, ref_f) <= TOL
