#!/usr/bin/env python3
"""Throughput of the K x K filter library on one MI355X.

Headline workload: the BF16 filter bank, 32 images x 16 channels x 1024 x 1024
-> 64 output channels, 5 x 5 filters (inputs N(0,1), weights N(0, 2/(16*25))),
BF16 operands with FP32 accumulation on the matrix cores, clamp-to-edge.  One
step = one forward (FP32 outputs) + grad_input + grad_filter over the whole
batch: the forward call and the two adjoint calls, inputs resident in HBM.

Metric: Mpix*taps/s, where a pixel is one output value of one channel and
taps are the multiply-adds per output value (C_in * K^2 = 400 for the bank);
forward + backward counts three times the forward taps.  The suite adds the
other workloads (8K Sobel, plain FP32 forward by graph replay, FP32
forward+backward, separable, zero-border sharpen, ragged batch against the
single-image calls, the bank at K = 3 and with BF16 outputs, the FP32 bank
path) with their ratio to the plain FP32 forward; every suite repetition is
preceded by a 512 MB write that evicts the caches.

Prints ONE JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import hashlib
import json
import os
import platform
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0           # MI355X HBM3E
FP32_VALU_PEAK_TFLOPS = 78.6    # unpacked FP32 FMA: 256 CU x 64 lanes x 2 FLOP x 2.4 GHz
BF16_MFMA_PEAK_TFLOPS = 2516.6  # dense BF16 matrix cores

BANK_N, BANK_CI, BANK_CO, BANK_HW = 32, 16, 64, 1024
BANK_SRC = ["paper_2504_01266_amd/csrc/bank_mfma.hip"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def sha_of(*paths):
    h = hashlib.sha256()
    for p in paths:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_key, sources):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        table = json.load(f)
    e = table.get(kernel_key)
    if not e or e.get("src_sha") != sha_of(*sources):
        return None
    return e.get("bytes_per_launch")


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


class Timer:
    """HIP events on torch's current stream (the stream every library call is
    enqueued on).  Each repetition is preceded by a 512 MB write, so that no
    input is served from the 256 MB last-level cache; the median repetition
    is reported."""

    def __init__(self, torch, evict_mb=512):
        self.torch = torch
        self.scratch = torch.empty(evict_mb << 18, dtype=torch.float32, device="cuda")

    def evict(self):
        self.scratch.fill_(1.0)

    def per_call_ms(self, fn, reps, warmup=2, calls=1):
        torch = self.torch
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        evs = []
        for _ in range(reps):
            self.evict()
            s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            s.record()
            fn()
            e.record()
            evs.append((s, e))
        torch.cuda.synchronize()
        return float(np.median([s.elapsed_time(e) for s, e in evs])) / calls


def roof(bound, achieved, peak, unit, traffic=None, **extra):
    d = {"bound": bound, "achieved": round(achieved, 2), "peak": peak, "unit": unit,
         "frac": round(achieved / peak, 4), "traffic": traffic}
    d.update(extra)
    return d


# ----------------------------------------------------------------- headline --

def bank_tensors(torch, wl, k, fp32=False):
    """The bank workload on the GPU: FP32 draws (torch's seeded generator for
    the images and upstream gradients, numpy's for the weights) and their BF16
    roundings."""
    gen = torch.Generator(device="cuda").manual_seed(wl.BANK_SEED)
    x32 = torch.randn((BANK_N, BANK_CI, BANK_HW, BANK_HW), generator=gen, device="cuda")
    g32 = torch.randn((BANK_N, BANK_CO, BANK_HW, BANK_HW), generator=gen, device="cuda")
    w32 = torch.from_numpy(wl.bank_weights(k)).cuda()
    t = {"x": x32.to(torch.bfloat16), "g": g32.to(torch.bfloat16), "w": w32.to(torch.bfloat16), "w32": w32}
    if fp32:
        t["x32"], t["g32"] = x32, g32
    else:
        del x32, g32
    return t


def bank_bytes(k):
    px_in = BANK_N * BANK_CI * BANK_HW * BANK_HW
    px_out = BANK_N * BANK_CO * BANK_HW * BANK_HW
    flops = 2.0 * px_out * BANK_CI * k * k
    return {
        "fwd_f32out": px_in * 2 + px_out * 4,     # X bf16 in, Y f32 out
        "fwd_bf16out": px_in * 2 + px_out * 2,
        "dgrad": px_out * 2 + px_in * 4,          # G-bar bf16 in, X-bar f32 out
        "wgrad": px_out * 2 + px_in * 2,          # G-bar and X bf16 in (W-bar is 100 KB)
        "flops": flops,
        "taps": px_out * BANK_CI * k * k,
    }


def headline(torch, B, wl, k, steps, warmup):
    t = bank_tensors(torch, wl, k, fp32=True)
    xb, gb, wb = t["x"], t["g"], t["w"]
    y = torch.empty((BANK_N, BANK_CO, BANK_HW, BANK_HW), device="cuda")
    gi = torch.empty((BANK_N, BANK_CI, BANK_HW, BANK_HW), device="cuda")
    ws = torch.empty(B.backward_workspace(xb, wb, mode="bank"), dtype=torch.uint8, device="cuda")
    calls = [
        ("fwd_f32out", lambda: B.forward(xb, wb, mode="bank", outs=[y])),
        ("dgrad", lambda: B.backward(xb, wb, gb, mode="bank", need_filter=False, workspace=ws, grad_input=gi)),
        ("wgrad", lambda: B.backward(xb, wb, gb, mode="bank", need_input=False, workspace=ws)),
    ]

    def step(evs=None):
        for j, (_, fn) in enumerate(calls):
            if evs is not None:
                evs[j][0].record()
            fn()
            if evs is not None:
                evs[j][1].record()

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev = [[[torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)] for _ in calls]
          for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        step(ev[i])
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1e3
    call_ms = {name: float(np.mean([ev[i][j][0].elapsed_time(ev[i][j][1]) for i in range(steps)]))
               for j, (name, _) in enumerate(calls)}
    ms_per_step = wall_ms / steps
    bb = bank_bytes(k)
    value = 3 * bb["taps"] / (ms_per_step * 1e-3) / 1e6
    kernels = {
        "fwd_f32out": {"kernel": f"bank forward {k}x{k} (FP32 out)", "ms": round(call_ms["fwd_f32out"], 4),
                       **roof("hbm", bb["fwd_f32out"] / (call_ms["fwd_f32out"] * 1e-3) / 1e9, HBM_PEAK_GBS, "GB/s",
                              measured_traffic(f"bank_bf16_k{k}_fwd_f32out", BANK_SRC),
                              algorithmic_bytes_per_launch=bb["fwd_f32out"],
                              mfma_frac=round(bb["flops"] / (call_ms["fwd_f32out"] * 1e-3) / 1e12 /
                                              BF16_MFMA_PEAK_TFLOPS, 4))},
        "dgrad": {"kernel": f"bank grad_input {k}x{k} (adjoint + frame fold)", "ms": round(call_ms["dgrad"], 4),
                  **roof("hbm", bb["dgrad"] / (call_ms["dgrad"] * 1e-3) / 1e9, HBM_PEAK_GBS, "GB/s",
                         measured_traffic(f"bank_bf16_k{k}_dgrad", BANK_SRC),
                         algorithmic_bytes_per_launch=bb["dgrad"],
                         mfma_frac=round(bb["flops"] / (call_ms["dgrad"] * 1e-3) / 1e12 / BF16_MFMA_PEAK_TFLOPS, 4))},
        "wgrad": {"kernel": f"bank grad_filter {k}x{k} (partials + fixed-order reduce)", "ms": round(call_ms["wgrad"], 4),
                  **roof("mfma", bb["flops"] / (call_ms["wgrad"] * 1e-3) / 1e12, BF16_MFMA_PEAK_TFLOPS, "TFLOP/s",
                         measured_traffic(f"bank_bf16_k{k}_wgrad", BANK_SRC),
                         algorithmic_flops_per_launch=bb["flops"],
                         hbm_frac=round(bb["wgrad"] / (call_ms["wgrad"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4))},
    }
    dom = max(kernels, key=lambda n: kernels[n]["ms"])
    return dict(t=t, y=y, gi=gi, ws=ws, k=k, ms_per_step=ms_per_step, value=value, kernels=kernels,
                dominant=dom, pix_taps=3 * bb["taps"])


def parity(torch, B, oracle, hd):
    """Relative L2 error of each result against the FP64 oracle, on the
    BF16-rounded inputs (accumulation error) and on the unrounded FP32 draws
    (the BF16 tolerance 1e-2): output rows 0..7 of image 0 for the forward
    (FP32 and BF16 outputs) and grad_input, and grad_filter of the 16-row crop
    of image 0 (a separate call on that crop)."""
    t, k = hd["t"], hd["k"]
    r = k // 2
    host = lambda a: a.double().cpu().numpy()  # noqa: E731
    wr, wu = host(t["w"]), host(t["w32"])
    rows = 8
    yb = B.forward(t["x"][:1, :, :rows + r], t["w"], mode="bank", out_dtype=torch.bfloat16, rows=(0, rows))
    xr, xu = host(t["x"][:1, :, :rows + r]), host(t["x32"][:1, :, :rows + r])
    ref, refu = oracle.forward(xr, wr, "bank", rows=(0, rows)), oracle.forward(xu, wu, "bank", rows=(0, rows))
    y = host(hd["y"][:1, :, :rows])
    gr, gu = host(t["g"][:1, :, :rows + r]), host(t["g32"][:1, :, :rows + r])
    refi = oracle.grad_input(gr, wr, (1, BANK_CI, rows + r, BANK_HW), "bank")[:, :, :rows]
    refiu = oracle.grad_input(gu, wu, (1, BANK_CI, rows + r, BANK_HW), "bank")[:, :, :rows]
    gi = host(hd["gi"][:1, :, :rows])
    crop = 16
    _, gfc = B.backward(t["x"][:1, :, :crop].contiguous(), t["w"], t["g"][:1, :, :crop].contiguous(),
                        mode="bank", need_input=False)
    reff = oracle.grad_filter(host(t["x"][:1, :, :crop]), host(t["g"][:1, :, :crop]), wr.shape, "bank")
    reffu = oracle.grad_filter(host(t["x32"][:1, :, :crop]), host(t["g32"][:1, :, :crop]), wr.shape, "bank")
    gf = host(gfc)
    e = lambda a, b: float(f"{oracle.rel_l2(a, b):.3e}")  # noqa: E731
    return {
        "sample": f"image 0: forward and grad_input rows 0..{rows - 1}; grad_filter of rows 0..{crop - 1}",
        "rel_l2_rounded_inputs": {"fwd_f32out": e(y, ref), "fwd_bf16out": e(host(yb), ref),
                                  "grad_input": e(gi, refi), "grad_filter": e(gf, reff)},
        "rel_l2_unrounded_fp32": {"fwd_f32out": e(y, refu), "fwd_bf16out": e(host(yb), refu),
                                  "grad_input": e(gi, refiu), "grad_filter": e(gf, reffu)},
        "tolerance": {"rounded_inputs": 1e-5, "unrounded_fp32": 1e-2},
    }


def oracle_bank_sample(oracle, x, w, g, rows):
    """The oracle's forward + grad_input + grad_filter on output rows
    0..rows-1 of m bank images (x: [m][16][rows + r][W], g: [m][64][rows + r][W]);
    returns (seconds, Mpix*taps)."""
    k = w.shape[-1]
    r = k // 2
    t0 = time.perf_counter()
    oracle.forward(x, w, "bank", rows=(0, rows))
    oracle.grad_input(g, w, x.shape, "bank")
    oracle.grad_filter(x[:, :, :rows], g[:, :, :rows], w.shape, "bank")
    dt = time.perf_counter() - t0
    return dt, 3 * x.shape[0] * rows * x.shape[3] * w.shape[0] * w.shape[1] * k * k / 1e6


def cpu_baseline(oracle, wl, k, budget_s):
    """The oracle as it stands on a bounded sample of the headline workload:
    forward, grad_input and grad_filter of the bank on the first output rows
    of one image, or on whole images when one takes well under the budget
    (seeded numpy draws of the same shapes), on all the host's oracle threads
    and, in a child process, on one core."""
    r = k // 2
    w = wl.bank_weights(k).astype(np.float64)
    x_all = wl.bank_image(0)[None].astype(np.float64)
    g_all = wl.bank_grad(0)[None].astype(np.float64)

    def sample(rows):
        return oracle_bank_sample(oracle, x_all[:, :, :rows + r], w, g_all[:, :, :rows + r], rows)

    dt, _ = sample(2)
    rows = int(min(BANK_HW - r, max(2, 2 * budget_s / max(dt, 1e-3))))
    dt, mpt = sample(rows)
    images = 1
    if rows == BANK_HW - r and 2 * dt < budget_s:
        images = int(min(BANK_N, budget_s // dt))
        x_all = np.stack([wl.bank_image(i) for i in range(images)]).astype(np.float64)
        g_all = np.stack([wl.bank_grad(i) for i in range(images)]).astype(np.float64)
        dt, mpt = sample(rows)
    one = None
    try:
        # about a third of the budget on one core (the rate per row scales with the thread count)
        per_row_1 = dt * max(oracle.num_threads(), 1) / (rows * images)
        rows1 = int(min(BANK_HW - r, max(1, budget_s / 3 / per_row_1)))
        env = dict(os.environ, OMP_NUM_THREADS="1")
        out = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-one-core", str(rows1),
                              "--k", str(k)], env=env, capture_output=True, text=True, timeout=600)
        one = json.loads(out.stdout.strip().splitlines()[-1])
    except Exception as exc:  # the one-core figure is informational
        one = {"error": str(exc)[:200]}
    return {"value": round(mpt / dt, 3), "unit": "Mpix*taps/s", "cores": oracle.num_threads(),
            "kind": "oracle", "seconds": round(dt, 2), "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "one_core": one,
            "sample": f"forward + grad_input + grad_filter of the {k}x{k} bank (16 -> 64 channels) on output "
                      f"rows 0..{rows - 1} of {images} 1024x1024 image(s) ({rows * images}/{BANK_HW * BANK_N} "
                      f"image rows of the batch), FP64 direct loops, OpenMP over outer indices"}


def oracle_one_core(rows, k):
    import oracle
    from paper_2504_01266_amd import workloads as wl

    r = k // 2
    w = wl.bank_weights(k).astype(np.float64)
    x = wl.bank_image(0)[None, :, :rows + r].astype(np.float64)
    g = wl.bank_grad(0)[None, :, :rows + r].astype(np.float64)
    dt, mpt = oracle_bank_sample(oracle, x, w, g, rows)
    print(json.dumps({"value": round(mpt / dt, 4), "unit": "Mpix*taps/s", "cores": oracle.num_threads(),
                      "seconds": round(dt, 2), "rows": rows}), flush=True)


# -------------------------------------------------------------------- suite --

def suite(torch, B, wl, reps, only=None):
    t = Timer(torch)
    res = {}

    import re as _re

    def want(name):
        return only is None or _re.search(only, name) is not None

    if want('device_ceilings'):
        # device ceilings: a plain fill and a device copy (torch kernels)
        a = torch.empty(298598400, dtype=torch.int32, device="cuda")  # 1.19 GB, the Sobel outputs
        ms_fill = t.per_call_ms(lambda: a.fill_(7), reps)
        b = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        c = torch.empty_like(b)
        ms_copy = t.per_call_ms(lambda: c.copy_(b), reps)
        res["device_ceilings"] = {"fill_1.19GB_GBs": round(a.numel() * 4 / (ms_fill * 1e-3) / 1e9, 1),
                                  "copy_1GiB_GBs": round(2 * b.numel() * 4 / (ms_copy * 1e-3) / 1e9, 1)}
        del a, b, c
        torch.cuda.empty_cache()

    # plain FP32 forward, 1024^2, 5x5 Gaussian: launch-latency bound, so timed
    # by replaying a graph of 100 launches
    x, f = wl.plain()
    xd, fd = torch.from_numpy(x).cuda(), torch.from_numpy(f).cuda()
    out = torch.empty_like(xd)
    for _ in range(3):
        B.forward(xd, fd, outs=[out])
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        B.forward(xd, fd, outs=[out])
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(100):
            B.forward(xd, fd, outs=[out])
    ms = t.per_call_ms(g.replay, max(reps, 5), calls=100)
    ms_eager = t.per_call_ms(lambda: B.forward(xd, fd, outs=[out]), max(reps, 20))
    pt = x.size * 25
    plain = pt / (ms * 1e-3) / 1e6
    res["plain_f32_fwd"] = {"shape": "1x1x1024x1024 f32, 5x5 (graph replay of 100 launches)",
                            "ms": round(ms, 5), "eager_call_ms": round(ms_eager, 5),
                            "mpix_taps_s": round(plain, 1), "vs_plain_fwd": 1.0,
                            "note": "8.4 MB working set: latency-bound, HBM % not meaningful"}
    del g

    if want('sobel_u8_8k'):
        # 8K Sobel (u8 -> int32 gx, gy, gx^2 + gy^2): HBM bound, 92% writes
        x, f = wl.sobel()
        xd, fd = torch.from_numpy(x).cuda(), torch.from_numpy(f).cuda()
        outs = [torch.empty(x.shape, dtype=torch.int32, device="cuda") for _ in range(3)]
        variant = B.autotune_forward(xd, fd, mode="depthwise", epilogue=B.EPI_SUMSQ_PAIRS, reps=5)
        ms = t.per_call_ms(lambda: B.forward(xd, fd, mode="depthwise", epilogue=B.EPI_SUMSQ_PAIRS, outs=outs), reps)
        pix = x.size
        alg = pix * 1 + 3 * pix * 4
        res["sobel_u8_8k"] = {"shape": "1x3x4320x7680 u8, Sobel-x/y + gx^2+gy^2 (int32)", "ms": round(ms, 4),
                              "variant": variant, "mpix_taps_s": round(pix * 18 / (ms * 1e-3) / 1e6, 1),
                              "vs_plain_fwd": round(pix * 18 / (ms * 1e-3) / 1e6 / plain, 3),
                              "roofline": roof("hbm", alg / (ms * 1e-3) / 1e9, HBM_PEAK_GBS, "GB/s",
                                               measured_traffic("sobel_u8_8k", ["paper_2504_01266_amd/csrc/stencil_u8.hip"]),
                                               algorithmic_bytes_per_launch=alg)}
        del xd, outs
        torch.cuda.empty_cache()

    if want('diff_f32'):
        # FP32 forward 16x3x2048^2, 9x9 (VALU bound without packed FP32)
        xs = np.stack([wl.diff_image(i) for i in range(16)])
        f9 = wl.diff_filter()
        xd, fd = torch.from_numpy(xs).cuda(), torch.from_numpy(f9).cuda()
        out = torch.empty_like(xd)
        ms = t.per_call_ms(lambda: B.forward(xd, fd, outs=[out]), reps)
        pt = xs.size * 81
        res["diff_f32_fwd"] = {"shape": "16x3x2048x2048 f32, 9x9", "ms": round(ms, 4),
                               "mpix_taps_s": round(pt / (ms * 1e-3) / 1e6, 1),
                               "vs_plain_fwd": round(pt / (ms * 1e-3) / 1e6 / plain, 3),
                               "roofline": roof("alu", 2.0 * pt / (ms * 1e-3) / 1e12, FP32_VALU_PEAK_TFLOPS, "TFLOP/s"),
                               "hbm_gbs": round(xs.size * 8 / (ms * 1e-3) / 1e9, 1)}
        gs = np.stack([wl.diff_grad(i) for i in range(16)])
        gd = torch.from_numpy(gs).cuda()
        del gs
        ws = torch.empty(B.backward_workspace(xd, fd), dtype=torch.uint8, device="cuda")

        def fwd_bwd():
            B.forward(xd, fd, outs=[out])
            B.backward(xd, fd, gd, workspace=ws)

        ms_fb = t.per_call_ms(fwd_bwd, reps)
        ms_b = t.per_call_ms(lambda: B.backward(xd, fd, gd, workspace=ws), reps)
        pt3 = 3 * pt
        res["diff_f32_fwd_bwd"] = {"shape": "16x3x2048x2048 f32, 9x9, fwd + grad_input + grad_filter",
                                   "ms": round(ms_fb, 4), "bwd_ms": round(ms_b, 4),
                                   "mpix_taps_s": round(pt3 / (ms_fb * 1e-3) / 1e6, 1),
                                   "vs_plain_fwd": round(pt3 / (ms_fb * 1e-3) / 1e6 / plain, 3),
                                   "roofline": roof("alu", 2.0 * pt3 / (ms_fb * 1e-3) / 1e12, FP32_VALU_PEAK_TFLOPS,
                                                    "TFLOP/s")}
        # separable fast path on the same images: the 9x9 normalised Gaussian
        # (sigma 2) as g g^T, 2K = 18 multiply-adds per output, against the direct
        # K x K path with the same filter
        g9 = wl.gaussian_factor(9, 2.0)
        gk = torch.from_numpy(g9).cuda()
        fgg = torch.from_numpy(np.outer(g9, g9).astype(np.float32)).cuda()
        ms_sep = t.per_call_ms(lambda: B.forward_separable(xd, gk, gk, out=out), reps)
        ms_dir = t.per_call_ms(lambda: B.forward(xd, fgg, outs=[out]), reps)
        ps = xs.size * 18
        res["separable_f32_fwd"] = {"shape": "16x3x2048x2048 f32, 9x9 Gaussian as g g^T (18 taps per output)",
                                    "ms": round(ms_sep, 4), "direct_ms": round(ms_dir, 4),
                                    "speedup_vs_direct": round(ms_dir / ms_sep, 3),
                                    "mpix_taps_s": round(ps / (ms_sep * 1e-3) / 1e6, 1),
                                    "vs_plain_fwd": round(ps / (ms_sep * 1e-3) / 1e6 / plain, 3),
                                    "roofline": roof("hbm", xs.size * 8 / (ms_sep * 1e-3) / 1e9, HBM_PEAK_GBS, "GB/s")}
        del xd, out, gd, ws, gk, fgg
        torch.cuda.empty_cache()

    if want('zero_border_f32_fwd'):
        # zero borders (the paper's sharpen skips out-of-image neighbours): the
        # 3x3 Laplacian on a 3-channel 4K frame, against clamp-to-edge on the same
        xz = torch.from_numpy(wl.sharpen_frame()).cuda()
        lap = torch.from_numpy(wl.LAPLACIAN_8).cuda()
        oz = torch.empty_like(xz)
        ms_z = t.per_call_ms(lambda: B.forward(xz, lap, outs=[oz], border="zero"), reps)
        ms_c = t.per_call_ms(lambda: B.forward(xz, lap, outs=[oz]), reps)
        pz = xz.numel()
        res["zero_border_f32_fwd"] = {"shape": "1x3x2160x3840 f32 (0..255), 3x3 Laplacian sharpen, zero borders",
                                      "ms": round(ms_z, 4), "clamp_ms": round(ms_c, 4),
                                      "mpix_taps_s": round(pz * 9 / (ms_z * 1e-3) / 1e6, 1),
                                      "vs_plain_fwd": round(pz * 9 / (ms_z * 1e-3) / 1e6 / plain, 3),
                                      "roofline": roof("hbm", pz * 8 / (ms_z * 1e-3) / 1e9, HBM_PEAK_GBS, "GB/s")}
        del xz, oz, lap
        torch.cuda.empty_cache()

    if want('paper_u8'):
        # the paper's own image operations on 8-bit RGB (interleaved, as OpenCV
        # delivers it): the float Laplacian sharpen with skipped out-of-image
        # neighbours, 8-bit out (Section 4.2.4); the same after nearest
        # upsampling by 2, 4 and 20 in one pass (Sections 4.2.3, 6.6); the
        # grayscale weights on an 8K frame (Section 4.2.5)
        x4k = wl.paper_frame_u8()
        xd = torch.from_numpy(x4k).cuda()[None].permute(0, 3, 1, 2)
        lap = torch.from_numpy(wl.LAPLACIAN_8).cuda()
        px_in = x4k.size
        for s_up in (1, 2, 4, 20):
            out = torch.empty((1, x4k.shape[0] * s_up, x4k.shape[1] * s_up, 3), dtype=torch.uint8,
                              device="cuda").permute(0, 3, 1, 2)
            if s_up == 1:
                fn = lambda: B.forward(xd, lap, border="zero", outs=[out])  # noqa: E731
            else:
                fn = lambda: B.upsample_forward(xd, lap, s_up, out=out, border="zero")  # noqa: E731
            ms = t.per_call_ms(fn, reps)
            px_out = out.numel()
            res[f"paper_sharpen_u8_x{s_up}"] = {
                "shape": f"4K RGB u8 interleaved (2160x3840x3) -> x{s_up} nearest upsample -> 3x3 Laplacian, "
                         f"zero borders, u8 out ({px_out} values)",
                "ms": round(ms, 4), "mpix_taps_s": round(px_out * 9 / (ms * 1e-3) / 1e6, 1),
                "vs_plain_fwd": round(px_out * 9 / (ms * 1e-3) / 1e6 / plain, 3),
                "roofline": roof("hbm", (px_in + px_out) / (ms * 1e-3) / 1e9, HBM_PEAK_GBS, "GB/s",
                                 algorithmic_bytes_per_launch=px_in + px_out)}
            del out
            torch.cuda.empty_cache()
        del xd
        x8k = wl.paper_frame_u8(4320, 7680)
        xd = torch.from_numpy(x8k).cuda()[None].permute(0, 3, 1, 2)
        gw = torch.from_numpy(wl.GRAY_RGB.astype(np.float32).reshape(1, 3, 1, 1)).cuda()
        gout = torch.empty((1, 1, 4320, 7680), dtype=torch.uint8, device="cuda")
        ms = t.per_call_ms(lambda: B.forward(xd, gw, mode="bank", outs=[gout]), reps)
        alg = x8k.size + gout.numel()
        res["paper_grayscale_u8_8k"] = {
            "shape": "8K RGB u8 interleaved (4320x7680x3) -> gray u8 (0.299, 0.587, 0.114)",
            "ms": round(ms, 4), "mpix_taps_s": round(gout.numel() * 3 / (ms * 1e-3) / 1e6, 1),
            "vs_plain_fwd": round(gout.numel() * 3 / (ms * 1e-3) / 1e6 / plain, 3),
            "roofline": roof("hbm", alg / (ms * 1e-3) / 1e9, HBM_PEAK_GBS, "GB/s", algorithmic_bytes_per_launch=alg)}
        del xd, gout
        torch.cuda.empty_cache()

    if want('ragged_batch_f32'):
        # ragged batch: 64 images, H, W uniform in [256, 4096], 3 channels, 7x7
        # each, one launch; against the 64 single-image calls on the same images
        sizes = wl.ragged_sizes()
        xd, yd, fdl = [], [], []
        for i, (h, w) in enumerate(sizes):
            xi, fi = wl.ragged_item(i, int(h), int(w))
            xd.append(torch.from_numpy(xi).cuda())
            yd.append(torch.empty_like(xd[-1]))
            fdl.append(torch.from_numpy(fi).cuda())
        batch = B.RaggedBatch(xd, yd, fdl)
        variant = batch.autotune(reps=3)
        ms = t.per_call_ms(batch.run, reps)

        def singles():
            for x_, f_, y_ in zip(xd, fdl, yd):
                B.forward(x_, f_, outs=[y_])

        ms_single = t.per_call_ms(singles, max(2, reps // 2))
        px = sum(x.numel() for x in xd)
        pt = px * 49
        res["ragged_batch_f32"] = {"shape": f"64 images, {px} px-channels, 7x7, one launch",
                                   "ms": round(ms, 4), "single_calls_ms": round(ms_single, 4),
                                   "tiles": batch.total_tiles, "variant": variant,
                                   "mpix_taps_s": round(pt / (ms * 1e-3) / 1e6, 1),
                                   "vs_plain_fwd": round(pt / (ms * 1e-3) / 1e6 / plain, 3),
                                   "roofline": roof("alu", 2.0 * pt / (ms * 1e-3) / 1e12, FP32_VALU_PEAK_TFLOPS, "TFLOP/s"),
                                   "hbm_frac": round(px * 8 / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        del xd, yd, fdl, batch
        torch.cuda.empty_cache()

    if want('bank_bf16'):
        # BF16 filter bank, each call on its own, K = 3 and 5
        for k in (3, 5):
            bt = bank_tensors(torch, wl, k)
            xb, gb, wb = bt["x"], bt["g"], bt["w"]
            bb = bank_bytes(k)
            y32 = torch.empty((BANK_N, BANK_CO, BANK_HW, BANK_HW), device="cuda")
            y16 = torch.empty((BANK_N, BANK_CO, BANK_HW, BANK_HW), dtype=torch.bfloat16, device="cuda")
            gi = torch.empty((BANK_N, BANK_CI, BANK_HW, BANK_HW), device="cuda")
            ws = torch.empty(B.backward_workspace(xb, wb, mode="bank"), dtype=torch.uint8, device="cuda")
            entry = {"shape": f"32x16x1024x1024 bf16 -> 64 ch, {k}x{k}"}
            for name, fn, key in (
                    ("fwd_f32out", lambda: B.forward(xb, wb, mode="bank", outs=[y32]), "fwd_f32out"),
                    ("fwd_bf16out", lambda: B.forward(xb, wb, mode="bank", outs=[y16]), "fwd_bf16out"),
                    ("dgrad", lambda: B.backward(xb, wb, gb, mode="bank", need_filter=False, workspace=ws,
                                                 grad_input=gi), "dgrad"),
                    ("wgrad", lambda: B.backward(xb, wb, gb, mode="bank", need_input=False, workspace=ws), "wgrad")):
                ms = t.per_call_ms(fn, reps)
                entry[name] = {"ms": round(ms, 4),
                               "hbm_frac": round(bb[key] / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                               "mfma_frac": round(bb["flops"] / (ms * 1e-3) / 1e12 / BF16_MFMA_PEAK_TFLOPS, 4)}

            def fb():
                B.forward(xb, wb, mode="bank", outs=[y32])
                B.backward(xb, wb, gb, mode="bank", workspace=ws, grad_input=gi)

            ms_fb = t.per_call_ms(fb, reps)
            entry["fwd_bwd_ms"] = round(ms_fb, 4)
            entry["fwd_bwd_mpix_taps_s"] = round(3 * bb["taps"] / (ms_fb * 1e-3) / 1e6, 1)
            entry["vs_plain_fwd"] = round(3 * bb["taps"] / (ms_fb * 1e-3) / 1e6 / plain, 3)
            res[f"bank_bf16_k{k}"] = entry
            del bt, xb, gb, wb, y32, y16, gi, ws
            torch.cuda.empty_cache()

    if want('bank_f32'):
        # the FP32 comparison path (VALU): the same 32-image bank in FP32
        for k in (3, 5):
            bt = bank_tensors(torch, wl, k, fp32=True)
            x32, g32, w32 = bt["x32"], bt["g32"], bt["w32"]
            del bt
            torch.cuda.empty_cache()
            bb = bank_bytes(k)
            y = torch.empty((BANK_N, BANK_CO, BANK_HW, BANK_HW), device="cuda")
            gi = torch.empty_like(x32)
            ws = torch.empty(B.backward_workspace(x32, w32, mode="bank"), dtype=torch.uint8, device="cuda")
            ms_f = t.per_call_ms(lambda: B.forward(x32, w32, mode="bank", outs=[y]), 2, warmup=1)
            ms_b = t.per_call_ms(lambda: B.backward(x32, w32, g32, mode="bank", workspace=ws, grad_input=gi), 2, warmup=1)
            res[f"bank_f32_k{k}"] = {"shape": f"32x16x1024x1024 f32 -> 64 ch f32, {k}x{k} (VALU path)",
                                     "fwd_ms": round(ms_f, 3), "bwd_ms": round(ms_b, 3),
                                     "fwd_mpix_taps_s": round(bb["taps"] / (ms_f * 1e-3) / 1e6, 1),
                                     "fwd_bwd_mpix_taps_s": round(3 * bb["taps"] / ((ms_f + ms_b) * 1e-3) / 1e6, 1),
                                     "fwd_valu_frac": round(bb["flops"] / (ms_f * 1e-3) / 1e12 / FP32_VALU_PEAK_TFLOPS, 4),
                                     "bwd_valu_frac": round(2 * bb["flops"] / (ms_b * 1e-3) / 1e12 / FP32_VALU_PEAK_TFLOPS, 4)}
            del x32, g32, w32, y, gi, ws
            torch.cuda.empty_cache()
    return res


def profile_run(torch, B, wl, steps, k):
    """A short run for rocprofv3: the headline step (bank forward + grad_input
    + grad_filter) `steps` times, then one plain device copy of exactly 1 GiB
    (the calibration kernel that converts counter readings to bytes)."""
    t = bank_tensors(torch, wl, k)
    xb, gb, wb = t["x"], t["g"], t["w"]
    y = torch.empty((BANK_N, BANK_CO, BANK_HW, BANK_HW), device="cuda")
    gi = torch.empty((BANK_N, BANK_CI, BANK_HW, BANK_HW), device="cuda")
    ws = torch.empty(B.backward_workspace(xb, wb, mode="bank"), dtype=torch.uint8, device="cuda")
    for i in range(steps):
        B.forward(xb, wb, mode="bank", outs=[y])
        B.backward(xb, wb, gb, mode="bank", need_filter=False, workspace=ws, grad_input=gi)
        B.backward(xb, wb, gb, mode="bank", need_input=False, workspace=ws)
        torch.cuda.synchronize()
        log(f"profile: step {i + 1}/{steps}")
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"profile": f"bank-bf16-{k}x{k}-fwd-bwd", "steps": steps,
                      "copy_bytes_read": a.numel() * 4, "copy_bytes_written": b.numel() * 4}), flush=True)


def profile_sobel(torch, B, wl, steps):
    """rocprofv3 run of the 8K Sobel kernel (tuned variant) `steps` times,
    then the 1 GiB calibration copy."""
    x, f = wl.sobel()
    xd, fd = torch.from_numpy(x).cuda(), torch.from_numpy(f).cuda()
    outs = [torch.empty(x.shape, dtype=torch.int32, device="cuda") for _ in range(3)]
    variant = B.autotune_forward(xd, fd, mode="depthwise", epilogue=B.EPI_SUMSQ_PAIRS, reps=3)
    for _ in range(steps):
        B.forward(xd, fd, mode="depthwise", epilogue=B.EPI_SUMSQ_PAIRS, outs=outs)
    torch.cuda.synchronize()
    a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"profile": "sobel-8k", "variant": variant, "steps": steps}), flush=True)


TRAFFIC_KERNELS = {
    # key in profiles/traffic.json -> (kernel-name test, algorithmic bytes, sources)
    "bank_bf16_k5_fwd_f32out": (lambda n: "k_bank_conv<" in n, lambda: bank_bytes(5)["fwd_f32out"], BANK_SRC),
    "bank_bf16_k5_dgrad": (lambda n: "k_bank_conv_vr<" in n or "k_bank_conv_ring<" in n,
                           lambda: bank_bytes(5)["dgrad"], BANK_SRC),
    "bank_bf16_k5_wgrad": (lambda n: "k_bank_wgrad" in n, lambda: bank_bytes(5)["wgrad"], BANK_SRC),
    # `--profile-sobel`: 8K RGB u8 in, gx, gy, gx^2+gy^2 int32 out
    "sobel_u8_8k": (lambda n: "k_stencil_u8" in n, lambda: 3 * 4320 * 7680 * (1 + 3 * 4),
                    ["paper_2504_01266_amd/csrc/stencil_u8.hip"]),
}


def traffic_from(fetch_dir, write_dir):
    """HBM bytes per launch of the headline kernels and the 8K Sobel from
    rocprofv3 counter runs of `bench.py --profile` and `--profile-sobel`
    (FETCH_SIZE runs under fetch_dir, WRITE_SIZE runs under write_dir, in KiB
    per dispatch), each scaled by what the same counter reads for the runs'
    final 1 GiB device copy (whose bytes are known); written to
    profiles/traffic.json with the kernel sources' hash."""
    import csv
    import glob
    import re

    def rows(d):
        out = []
        for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(path) as f:
                out.extend(csv.DictReader(f))
        if not out:
            raise SystemExit(f"no counter_collection.csv under {d}")
        return out

    def per_kernel(d, counter):
        vals = {}
        for r in rows(d):
            if r.get("Counter_Name") != counter:
                continue
            vals.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
        return vals

    fetch, write = per_kernel(fetch_dir, "FETCH_SIZE"), per_kernel(write_dir, "WRITE_SIZE")
    copy = [n for n in fetch if re.search(r"copy|Copy", n) and "bank" not in n]
    if not copy:
        raise SystemExit("no device copy kernel in the counter runs")
    gib_kib = float(1 << 20)
    ffac = gib_kib / float(np.median(fetch[copy[-1]]))
    wfac = gib_kib / float(np.median(write[copy[-1]]))
    path = os.path.join(ROOT, "profiles", "traffic.json")
    table = json.load(open(path)) if os.path.exists(path) else {}
    for key, (match, alg, srcs) in TRAFFIC_KERNELS.items():
        names = [n for n in fetch if match(n)]
        if not names:
            continue
        fk = float(np.median(fetch[names[0]]))
        wk = float(np.median(write[names[0]]))
        fb, wb = fk * 1024 * ffac, wk * 1024 * wfac
        table[key] = {"src_sha": sha_of(*srcs), "source": ", ".join(srcs), "kernel": names[0][:160],
                      "bytes_per_launch": int(fb + wb), "fetch_bytes": int(fb), "write_bytes": int(wb),
                      "fetch_kib_raw_median": fk, "write_kib_raw_median": wk,
                      "fetch_factor": round(ffac, 4), "write_factor": round(wfac, 4),
                      "algorithmic_bytes": alg(), "traffic_over_algorithmic": round((fb + wb) / alg(), 4)}
    with open(path, "w") as f:
        json.dump(table, f, indent=1)
    print(json.dumps({k: table[k].get("traffic_over_algorithmic") for k in table}), flush=True)


def write_ceiling(torch, reps):
    """What the device's memory system sustains for plain writes and copies:
    torch's fill kernel over 1.19 GB (the size of the Sobel outputs) and 4.3 GB
    (the BF16 bank output), and a 1 GiB device copy, each timed with HIP
    events after a 512 MB eviction write."""
    t = Timer(torch)
    out = {}
    for n, name in ((298598400, "fill_1.19GB"), (1073741824, "fill_4.29GB")):
        a = torch.empty(n, dtype=torch.int32, device="cuda")
        ms = t.per_call_ms(lambda: a.fill_(3), reps)
        out[name] = {"ms": round(ms, 4), "GBs": round(n * 4 / (ms * 1e-3) / 1e9, 1)}
        del a
    b = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    c = torch.empty_like(b)
    ms = t.per_call_ms(lambda: c.copy_(b), reps)
    out["copy_1GiB"] = {"ms": round(ms, 4), "GBs_read_plus_write": round(2 * b.numel() * 4 / (ms * 1e-3) / 1e9, 1)}
    print(json.dumps({"write_ceiling": out}), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--k", type=int, default=5, help="bank filter size of the headline (3 or 5)")
    ap.add_argument("--no-suite", action="store_true", help="headline workload only")
    ap.add_argument("--suite-reps", type=int, default=5)
    ap.add_argument("--suite-only", default=None, help="regex: run only the suite entries it matches")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="oracle sample budget")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline and parity")
    ap.add_argument("--profile", action="store_true",
                    help="rocprofv3 run: the headline step --steps times + a 1 GiB copy")
    ap.add_argument("--profile-sobel", action="store_true",
                    help="rocprofv3 run: the 8K Sobel kernel --steps times + a 1 GiB copy")
    ap.add_argument("--write-ceiling", action="store_true",
                    help="measure the device's plain-write and copy rates")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/traffic.json from two rocprofv3 --pmc runs of --profile")
    ap.add_argument("--oracle-one-core", type=int, default=0, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.oracle_one_core:
        oracle_one_core(args.oracle_one_core, args.k)
        return
    if args.traffic_from:
        traffic_from(*args.traffic_from)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): the filter runs on one GPU's "
              "share and multi-GPU sharding is not built", file=sys.stderr, flush=True)
        sys.exit(2)

    import torch

    import oracle
    from paper_2504_01266_amd import binding as B
    from paper_2504_01266_amd import workloads as wl

    B.load()
    torch.cuda.set_device(0)
    if args.profile:
        profile_run(torch, B, wl, args.steps, args.k)
        return
    if args.profile_sobel:
        profile_sobel(torch, B, wl, args.steps)
        return
    if args.write_ceiling:
        write_ceiling(torch, max(args.suite_reps, 5))
        return
    log(f"bench: headline bank {args.k}x{args.k} fwd+bwd")
    hd = headline(torch, B, wl, args.k, args.steps, args.warmup)
    log(f"bench: headline {hd['ms_per_step']:.4f} ms/step " +
        " ".join(f"{n}={v['ms']:.3f}" for n, v in hd["kernels"].items()))
    cpu, par = None, None
    if not args.no_cpu:
        log("bench: parity sample")
        par = parity(torch, B, oracle, hd)
        log("bench: cpu baseline (oracle)")
        cpu = cpu_baseline(oracle, wl, args.k, args.cpu_seconds)
    dom = hd["dominant"]
    kernels = hd["kernels"]
    for key in ("t", "y", "gi", "ws"):
        del hd[key]
    torch.cuda.empty_cache()
    sres = None
    if not args.no_suite:
        log("bench: suite")
        sres = suite(torch, B, wl, args.suite_reps, args.suite_only)
    k = args.k
    line = {
        "metric": "Mpix*taps/s (BF16 bank fwd+bwd; suite: other workloads vs plain FP32 fwd); "
                  "% of HBM / VALU / MFMA peak",
        "value": round(hd["value"], 1),
        "unit": "Mpix*taps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(hd["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16-in/f32-acc",
        "data": "synthetic (seeded: torch's generator for images and gradients, numpy PCG64 for weights)",
        "config": {"workload": f"bank: 32x16x1024x1024 -> 64 channels, {k}x{k}, BF16 operands, FP32 "
                               "accumulation and FP32 outputs, clamp-to-edge; step = forward + grad_input + "
                               "grad_filter",
                   "pix_taps_per_step": hd["pix_taps"], "parallelism": "single GPU"},
        "roofline": {**kernels[dom], "which": dom},
        "kernels": kernels,
        "cpu_baseline": cpu,
        "parity": par,
        "suite": sres,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
