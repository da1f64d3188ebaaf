// Forward dispatch: maps a validated filter2d_forward call onto stencil
// launches, plus the forward autotuner.
#include <hip/hip_runtime.h>

#include <cstring>

#include "f2d_host.hpp"
#include "f2d_internal.hpp"

namespace f2d {

namespace {

StencilParams base_params(const Problem& pr) {
  StencilParams p;
  std::memset(&p, 0, sizeof(p));
  const f2d_tensor& im = pr.image;
  for (int t = 0; t < kMaxT; ++t) {
    p.src[t] = im.data;
    p.src_sn[t] = im.stride_n;
    p.src_sc[t] = im.stride_c;
    p.src_sh[t] = im.stride_h;
  }
  p.filt = pr.filter.data;
  p.H = im.h;
  p.W = im.w;
  p.row0 = pr.row_begin;
  p.rows = pr.rows;
  p.k = pr.k;
  return p;
}

void set_dst(StencilParams& p, int slot, const f2d_tensor& t) {
  p.dst[slot] = t.data;
  p.dst_sn[slot] = t.stride_n;
  p.dst_sc[slot] = t.stride_c;
  p.dst_sh[slot] = t.stride_h;
}

f2d_status size_grid(StencilParams& p, int64_t n, TileShape ts) {
  p.tiles_x = static_cast<int32_t>((p.W + ts.tw - 1) / ts.tw);
  p.tiles_y = static_cast<int32_t>((p.rows + ts.th - 1) / ts.th);
  p.n_blocks = n * p.groups * static_cast<int64_t>(p.tiles_x) * p.tiles_y;
  if (p.n_blocks > kMaxBlocks)
    return fail(F2D_EUNSUPPORTED, "%lld tiles exceed one launch (max %lld)",
                static_cast<long long>(p.n_blocks), static_cast<long long>(kMaxBlocks));
  return F2D_OK;
}

bool all_aligned(const f2d_tensor* outs, int32_t n, size_t bytes) {
  for (int32_t j = 0; j < n; ++j)
    if (!row_aligned(outs[j], bytes)) return false;
  return true;
}

constexpr int kMaxTemplK = 9;    // templated f32 kernels exist for K <= 9
constexpr int kMaxTaps = 100;    // NOUT*K*K limit of the templated kernels

// Zero borders (out-of-image neighbours add nothing, as in the paper's
// sharpen): one output plane per work-group tile with zero-border staging,
// the 64 x 64 templated kernel for K <= 9 and the runtime-K kernel above
// (DEPTHWISE: one launch per filter index).
f2d_status forward_f32_zero(const Problem& pr, const f2d_tensor* outs, hipStream_t s) {
  const int variant = pr.k <= kMaxTemplK ? 1 : -1;
  const TileShape tg = f32_tile(variant);
  const int64_t C = pr.image.c;
  const int32_t vecflag = all_aligned(outs, pr.mode == F2D_CH_DEPTHWISE ? pr.m : 1, 16) ? kDstVec : 0;
  auto go = [&](StencilParams& p) -> f2d_status {
    p.flags = kZeroBorder | vecflag;
    if (f2d_status e = size_grid(p, pr.image.n, tg)) return e;
    return hip_status(launch_stencil_f32(p, pr.k, 1, false, variant, s), "forward f32 zero-border launch");
  };
  if (pr.mode == F2D_CH_SHARED) {
    StencilParams p = base_params(pr);
    set_dst(p, 0, outs[0]);
    p.groups = static_cast<int32_t>(C);
    p.nsrc = 1;
    p.sc_g = 1;
    p.dc_g = 1;
    return go(p);
  }
  if (pr.mode == F2D_CH_DEPTHWISE) {
    for (int j = 0; j < pr.m; ++j) {
      StencilParams p = base_params(pr);
      set_dst(p, 0, outs[j]);
      p.groups = static_cast<int32_t>(C);
      p.nsrc = 1;
      p.sc_g = 1;
      p.dc_g = 1;
      p.f0 = j;
      p.fg = pr.m;
      if (f2d_status e = go(p)) return e;
    }
    return ok();
  }
  StencilParams p = base_params(pr);  // BANK: output channel g sums all C sources
  set_dst(p, 0, outs[0]);
  p.groups = static_cast<int32_t>(pr.c_out);
  p.nsrc = static_cast<int32_t>(C);
  p.sc_s = 1;
  p.dc_g = 1;
  p.fg = static_cast<int32_t>(C);
  p.fs = 1;
  return go(p);
}

f2d_status forward_f32(const Problem& pr, const f2d_tensor* outs, int32_t n_outs, hipStream_t s) {
  if (pr.opts.border == F2D_BORDER_ZERO) return forward_f32_zero(pr, outs, s);
  const int K = pr.k;
  const bool templ = K <= kMaxTemplK;
  const int variant =
      templ ? resolve_variant(kPathF32, F2D_F32, K, pr.mode, pr.image.w, pr.opts.variant) : -1;
  const TileShape ts = f32_tile(variant);
  const int32_t vecflag = all_aligned(outs, n_outs, 16) ? kDstVec : 0;
  const int64_t C = pr.image.c;

  if (pr.mode == F2D_CH_SHARED) {
    StencilParams p = base_params(pr);
    set_dst(p, 0, outs[0]);
    p.groups = static_cast<int32_t>(C);
    p.nsrc = 1;
    p.sc_g = 1;
    p.dc_g = 1;
    p.flags = vecflag;
    if (f2d_status e = size_grid(p, pr.image.n, ts)) return e;
    return hip_status(launch_stencil_f32(p, K, 1, false, variant, s), "forward f32 launch");
  }
  if (pr.mode == F2D_CH_DEPTHWISE) {
    const int m = pr.m;
    const bool fused = templ && (m == 2 || m == 4) && m * K * K <= kMaxTaps;
    if (fused) {
      StencilParams p = base_params(pr);
      for (int j = 0; j < m; ++j) set_dst(p, j, outs[j]);
      p.groups = static_cast<int32_t>(C);
      p.nsrc = 1;
      p.sc_g = 1;
      p.dt_j = 1;
      p.dc_g = 1;
      p.fg = m;
      p.fj = 1;
      p.flags = vecflag;
      const TileShape t1 = f32_tile(1);
      if (f2d_status e = size_grid(p, pr.image.n, t1)) return e;
      return hip_status(launch_stencil_f32(p, K, m, false, 1, s), "forward f32 launch");
    }
    for (int j = 0; j < m; ++j) {  // one launch per filter index
      StencilParams p = base_params(pr);
      set_dst(p, 0, outs[j]);
      p.groups = static_cast<int32_t>(C);
      p.nsrc = 1;
      p.sc_g = 1;
      p.dc_g = 1;
      p.f0 = j;
      p.fg = m;
      p.flags = vecflag;
      if (f2d_status e = size_grid(p, pr.image.n, ts)) return e;
      hipError_t err = launch_stencil_f32(p, K, 1, false, variant, s);
      if (err != hipSuccess) return hip_status(err, "forward f32 launch");
    }
    return ok();
  }
  // BANK on the VALU: NOUT output channels share each staged source tile
  const int64_t co = pr.c_out;
  int nout = 1;
  if (templ && co % 4 == 0 && 4 * K * K <= kMaxTaps)
    nout = 4;
  else if (templ && co % 2 == 0 && 2 * K * K <= kMaxTaps)
    nout = 2;
  StencilParams p = base_params(pr);
  set_dst(p, 0, outs[0]);
  p.groups = static_cast<int32_t>(co / nout);
  p.nsrc = static_cast<int32_t>(C);
  p.sc_s = 1;
  p.dc_g = nout;
  p.dc_j = 1;
  p.fg = nout * static_cast<int32_t>(C);
  p.fj = static_cast<int32_t>(C);
  p.fs = 1;
  p.flags = vecflag;
  const int v = nout == 1 ? variant : 1;
  if (f2d_status e = size_grid(p, pr.image.n, f32_tile(v))) return e;
  return hip_status(launch_stencil_f32(p, K, nout, false, v, s), "forward f32 bank launch");
}

f2d_status forward_u8(const Problem& pr, const f2d_tensor* outs, int32_t n_outs, hipStream_t s) {
  const int K = pr.k;
  const bool templ = K <= 9;
  const int variant =
      templ ? resolve_variant(kPathU8, F2D_U8, K, pr.mode, pr.image.w, pr.opts.variant) : -1;
  const TileShape ts = u8_tile(variant);
  int32_t flags = 0;
  if (all_aligned(outs, n_outs, 16)) flags |= kDstVec;
  if (row_aligned(pr.image, 4)) flags |= kSrcVec;
  const int64_t C = pr.image.c;
  const bool sumsq = pr.opts.epilogue == F2D_EPI_SUMSQ_PAIRS;
  const int m = pr.m;

  if (m <= 2) {
    StencilParams p = base_params(pr);
    for (int j = 0; j < n_outs; ++j) set_dst(p, j, outs[j]);
    p.groups = static_cast<int32_t>(C);
    p.nsrc = 1;
    p.sc_g = 1;
    p.dt_j = 1;
    p.dc_g = 1;
    p.fg = pr.mode == F2D_CH_SHARED ? 0 : m;
    p.fj = 1;
    p.flags = flags | (sumsq ? kSumSq : 0);
    if (f2d_status e = size_grid(p, pr.image.n, ts)) return e;
    return hip_status(launch_stencil_u8(p, K, m, sumsq, true, variant, s), "forward u8 launch");
  }
  for (int j = 0; j < m; ++j) {
    StencilParams p = base_params(pr);
    set_dst(p, 0, outs[j]);
    p.groups = static_cast<int32_t>(C);
    p.nsrc = 1;
    p.sc_g = 1;
    p.dc_g = 1;
    p.f0 = j;
    p.fg = m;
    p.flags = flags;
    if (f2d_status e = size_grid(p, pr.image.n, ts)) return e;
    hipError_t err = launch_stencil_u8(p, K, 1, false, true, variant, s);
    if (err != hipSuccess) return hip_status(err, "forward u8 launch");
  }
  return ok();
}

}  // namespace

f2d_status bank_forward_bf16(const Problem& pr, const f2d_tensor* outs, hipStream_t s);

f2d_status run_forward(const Problem& pr, const f2d_tensor* outs, int32_t n_outs, hipStream_t s) {
  if (pr.image.n == 0 || pr.rows == 0 || pr.image.w == 0 || pr.c_out == 0 || pr.image.c == 0)
    return ok();
  switch (pr.image.dtype) {
    case F2D_F32: return forward_f32(pr, outs, n_outs, s);
    case F2D_U8: {
      // the integer Sobel path: int32 taps and outputs, clamp-to-edge, planar
      bool int_path = pr.filter.dtype == F2D_I32 && pr.opts.border == F2D_BORDER_CLAMP &&
                      pr.mode != F2D_CH_BANK && pr.image.stride_w <= 1;
      for (int32_t j = 0; j < n_outs; ++j) int_path = int_path && outs[j].dtype == F2D_I32 && outs[j].stride_w <= 1;
      if (int_path) return forward_u8(pr, outs, n_outs, s);
      return forward_u8_image(pr, outs, n_outs, s);
    }
    case F2D_BF16: return bank_forward_bf16(pr, outs, s);
    default: return fail(F2D_EUNSUPPORTED, "image dtype %d", pr.image.dtype);
  }
}

f2d_status autotune_forward(const Problem& pr, const f2d_tensor* outs, int32_t n_outs, int32_t reps,
                            hipStream_t s, int32_t* best) {
  int path = pr.image.dtype == F2D_U8 ? kPathU8 : (pr.image.dtype == F2D_F32 ? kPathF32 : -1);
  if (path < 0) return fail(F2D_EUNSUPPORTED, "autotune: no tiling variants for this dtype");
  if (reps < 1) return fail(F2D_EINVAL, "autotune: reps must be >= 1");
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(F2D_EHIP, "autotune: hipEventCreate failed");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(F2D_EHIP, "autotune: hipEventCreate failed");
  }
  float best_ms = 0.0f;
  int best_v = 1;
  f2d_status st = F2D_OK;
  for (int v = 1; v <= variant_count(path) && st == F2D_OK; ++v) {
    Problem q = pr;
    q.opts.variant = v;
    st = run_forward(q, outs, n_outs, s);  // warm-up
    if (st) break;
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps && st == F2D_OK; ++r) st = run_forward(q, outs, n_outs, s);
    (void)hipEventRecord(e1, s);
    if (hipEventSynchronize(e1) != hipSuccess) {
      st = fail(F2D_EHIP, "autotune: kernel failed");
      break;
    }
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    if (v == 1 || ms < best_ms) {
      best_ms = ms;
      best_v = v;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) return st;
  record_variant(path, pr.image.dtype, pr.k, pr.mode, pr.image.w, best_v);
  if (best) *best = best_v;
  return ok();
}

}  // namespace f2d
