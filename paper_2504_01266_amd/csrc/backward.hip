// Backward dispatch: validation, workspace sizing and the launch sequence of
// the adjoints (grad_input: adjoint stencil + exact edge fold; grad_filter:
// per-unit partials + fixed-order reduction).
#include <hip/hip_runtime.h>

#include <cstring>

#include "f2d_host.hpp"
#include "f2d_internal.hpp"
#include "grad_internal.hpp"

namespace f2d {

f2d_status bank_backward_bf16(const Problem& pr, const f2d_tensor& gout, const f2d_tensor* grad_input,
                              float* grad_filter, void* ws, size_t ws_bytes, hipStream_t s);
size_t bank_backward_bf16_workspace(const Problem& pr);

size_t round_up(size_t b) { return (b + 255) & ~static_cast<size_t>(255); }

namespace {

struct FilterPlan {
  int64_t nf, nrep, chunks, n_units;
  int32_t tiles_x, tiles_y, tpu;
};

FilterPlan filter_plan(const Problem& pr) {
  const f2d_tensor& im = pr.image;
  FilterPlan fp;
  const int64_t C = im.c;
  if (pr.mode == F2D_CH_SHARED) {
    fp.nf = 1;
    fp.nrep = im.n * C;
  } else if (pr.mode == F2D_CH_DEPTHWISE) {
    fp.nf = C * pr.m;
    fp.nrep = im.n;
  } else {
    fp.nf = pr.c_out * C;
    fp.nrep = im.n;
  }
  const TileShape ts = grad_filter_tile();
  fp.tiles_x = static_cast<int32_t>((im.w + ts.tw - 1) / ts.tw);
  fp.tiles_y = static_cast<int32_t>((im.h + ts.th - 1) / ts.th);
  const int64_t tiles = static_cast<int64_t>(fp.tiles_x) * fp.tiles_y;
  // enough work units to fill the GPU several times, each a run of tiles
  const int64_t all = tiles * fp.nf * fp.nrep;
  int64_t tpu = all / 8192;
  tpu = tpu < 1 ? 1 : (tpu > 16 ? 16 : tpu);
  fp.tpu = static_cast<int32_t>(tpu);
  fp.chunks = (tiles + tpu - 1) / tpu;
  fp.n_units = fp.nrep * fp.nf * fp.chunks;
  return fp;
}

bool whole_image(const Problem& pr) { return pr.row_begin == 0 && pr.row_end == pr.image.h; }

}  // namespace

// frame buffer of the image adjoint (templated kernels only)
size_t frame_bytes(const Problem& pr) {
  if (pr.k > 9) return 0;
  const int64_t r = (pr.k - 1) / 2;
  return round_up(static_cast<size_t>(pr.image.n * pr.image.c) *
                  frame_plane_size(pr.image.h, pr.image.w, r) * sizeof(float));
}

size_t backward_workspace(const Problem& pr) {
  if (pr.image.dtype == F2D_BF16) return bank_backward_bf16_workspace(pr);
  if (pr.image.dtype != F2D_F32) return 0;
  const FilterPlan fp = filter_plan(pr);
  const size_t bytes = static_cast<size_t>(fp.n_units) * pr.k * pr.k * sizeof(float);
  return frame_bytes(pr) + round_up(bytes > 0 ? bytes : 1);
}

f2d_status check_backward(const Problem& pr, const f2d_tensor* grad_outs, int32_t n_grad_outs,
                          const f2d_tensor* grad_input) {
  const f2d_tensor& im = pr.image;
  if (im.dtype == F2D_U8) return fail(F2D_EUNSUPPORTED, "u8 images are not differentiable");
  if (!whole_image(pr))
    return fail(F2D_EUNSUPPORTED, "backward works on whole images: row_begin/row_end must select all rows");
  if (pr.opts.epilogue != F2D_EPI_NONE) return fail(F2D_EINVAL, "backward takes no epilogue");
  const int32_t want = pr.mode == F2D_CH_DEPTHWISE ? pr.m : 1;
  if (n_grad_outs != want) return fail(F2D_EINVAL, "expected %d grad_outs, got %d", want, n_grad_outs);
  if (want > kMaxT) return fail(F2D_EUNSUPPORTED, "DEPTHWISE backward supports at most %d filters per channel", kMaxT);
  if (!grad_outs) return fail(F2D_EINVAL, "grad_outs is NULL");
  // upstream gradients share the image's element type (bf16 banks also take f32)
  const int32_t gdt = im.dtype;
  const int64_t co = pr.mode == F2D_CH_BANK ? pr.c_out : im.c;
  for (int32_t j = 0; j < n_grad_outs; ++j) {
    if (f2d_status e = check_tensor(&grad_outs[j], "grad_outs[j]", false)) return e;
    const f2d_tensor& g = grad_outs[j];
    if (g.n != im.n || g.c != co || g.h != im.h || g.w != im.w)
      return fail(F2D_EINVAL, "grad_outs[%d]: shape does not match the forward output", j);
    const bool ok_dt = g.dtype == gdt || (gdt == F2D_BF16 && g.dtype == F2D_F32);
    if (!ok_dt) return fail(F2D_EINVAL, "grad_outs[%d]: dtype %d does not match the image", j, g.dtype);
  }
  if (grad_input) {
    if (f2d_status e = check_tensor(grad_input, "grad_input", true)) return e;
    if (grad_input->n != im.n || grad_input->c != im.c || grad_input->h != im.h || grad_input->w != im.w)
      return fail(F2D_EINVAL, "grad_input: shape must equal the image's");
    if (grad_input->dtype != F2D_F32) return fail(F2D_EINVAL, "grad_input must be f32");
  }
  return F2D_OK;
}

f2d_status run_backward(const Problem& pr, const f2d_tensor* grad_outs, int32_t n_grad_outs,
                        const f2d_tensor* grad_input, float* grad_filter, void* ws, size_t ws_bytes,
                        hipStream_t s) {
  if (f2d_status e = check_backward(pr, grad_outs, n_grad_outs, grad_input)) return e;
  const f2d_tensor& im = pr.image;
  const int64_t co = pr.mode == F2D_CH_BANK ? pr.c_out : im.c;
  const size_t need = backward_workspace(pr);
  if ((grad_filter || grad_input) && need > 0 && (!ws || ws_bytes < need))
    return fail(F2D_EWORKSPACE, "workspace of %zu bytes needed, got %zu", need, ws ? ws_bytes : 0);
  if (im.dtype == F2D_BF16) return bank_backward_bf16(pr, grad_outs[0], grad_input, grad_filter, ws, ws_bytes, s);

  const int K = pr.k;
  const bool empty = im.n == 0 || im.c == 0 || im.h == 0 || im.w == 0 || co == 0;

  // ---------------------------------------------------------- grad_input --
  if (grad_input && !empty) {
    StencilParams p;
    std::memset(&p, 0, sizeof(p));
    EdgeParams e;
    std::memset(&e, 0, sizeof(e));
    for (int t = 0; t < kMaxT; ++t) {
      const f2d_tensor& g = grad_outs[t < n_grad_outs ? t : 0];
      p.src[t] = e.src[t] = g.data;
      p.src_sn[t] = e.src_sn[t] = g.stride_n;
      p.src_sc[t] = e.src_sc[t] = g.stride_c;
      p.src_sh[t] = e.src_sh[t] = g.stride_h;
    }
    p.dst[0] = grad_input->data;
    p.dst_sn[0] = grad_input->stride_n;
    p.dst_sc[0] = grad_input->stride_c;
    p.dst_sh[0] = grad_input->stride_h;
    p.filt = e.filt = pr.filter.data;
    p.H = e.H = im.h;
    p.W = e.W = im.w;
    p.row0 = 0;
    p.rows = im.h;
    p.k = e.k = K;
    p.groups = e.groups = static_cast<int32_t>(im.c);
    p.dc_g = 1;
    if (pr.mode == F2D_CH_SHARED) {
      p.nsrc = 1;
      p.sc_g = 1;
    } else if (pr.mode == F2D_CH_DEPTHWISE) {
      p.nsrc = pr.m;
      p.st_s = pr.m > 1 ? 1 : 0;
      p.sc_g = 1;
      p.fg = pr.m;
      p.fs = 1;
    } else {
      p.nsrc = static_cast<int32_t>(pr.c_out);
      p.sc_s = 1;
      p.fg = 1;
      p.fs = static_cast<int32_t>(im.c);
    }
    e.nsrc = p.nsrc;
    e.st_s = p.st_s;
    e.sc_g = p.sc_g;
    e.sc_s = p.sc_s;
    e.fg = p.fg;
    e.fs = p.fs;
    e.out = static_cast<float*>(grad_input->data);
    e.out_sn = grad_input->stride_n;
    e.out_sc = grad_input->stride_c;
    e.out_sh = grad_input->stride_h;
    e.planes = im.n * im.c;
    p.flags = row_aligned(*grad_input, 16) ? kDstVec : 0;

    const bool templ = K <= 9;
    const TileShape ts = f32_tile(templ ? 1 : -1);
    const int64_t r = (K - 1) / 2;
    if (templ) {
      // zero-border flipped correlation over the image and its r-wide frame
      p.row0 = -r;
      p.rows = im.h + 2 * r;
      p.col0 = -r;
      p.fr = static_cast<int32_t>(r);
      p.frame = static_cast<float*>(ws);
      p.frame_plane = frame_plane_size(im.h, im.w, r);
    }
    // bank: four image channels per work-group (each staged G-bar tile then
    // serves four outputs instead of one) where the taps fit in registers
    const int nout = templ && pr.mode == F2D_CH_BANK && K <= 5 && im.c % 4 == 0 ? 4 : 1;
    if (nout == 4) {
      p.groups = static_cast<int32_t>(im.c / 4);
      p.fg = 4;
      p.fj = 1;
      p.dc_g = 4;
      p.dc_j = 1;
    }
    const int64_t wext = im.w + (templ ? 2 * r : 0);
    p.tiles_x = static_cast<int32_t>((wext + ts.tw - 1) / ts.tw);
    p.tiles_y = static_cast<int32_t>((p.rows + ts.th - 1) / ts.th);
    p.n_blocks = im.n * p.groups * static_cast<int64_t>(p.tiles_x) * p.tiles_y;
    if (p.n_blocks > kMaxBlocks) return fail(F2D_EUNSUPPORTED, "image too large for one launch");
    if (!templ) p.flags |= kFlip | kZeroBorder;
    hipError_t err = launch_stencil_f32(p, K, nout, true, templ ? 1 : -1, s);
    if (err != hipSuccess) return hip_status(err, "grad_input launch");
    if (templ) {
      FoldParams fo;
      fo.frame = p.frame;
      fo.frame_plane = p.frame_plane;
      fo.out = static_cast<float*>(grad_input->data);
      fo.out_sn = grad_input->stride_n;
      fo.out_sc = grad_input->stride_c;
      fo.out_sh = grad_input->stride_h;
      fo.H = im.h;
      fo.W = im.w;
      fo.r = r;
      fo.planes = im.n * im.c;
      fo.groups = im.c;
      err = launch_fold_frame(fo, s);
    } else {
      err = launch_grad_input_edges(e, kEdgeF32, s);
    }
    if (err != hipSuccess) return hip_status(err, "grad_input edge launch");
  }

  // --------------------------------------------------------- grad_filter --
  if (grad_filter) {
    const FilterPlan fp = filter_plan(pr);
    float* partial = reinterpret_cast<float*>(static_cast<char*>(ws) + frame_bytes(pr));
    if (!empty) {
      GradFilterParams q;
      std::memset(&q, 0, sizeof(q));
      q.x = im.data;
      q.x_sn = im.stride_n;
      q.x_sc = im.stride_c;
      q.x_sh = im.stride_h;
      for (int t = 0; t < kMaxT; ++t) {
        const f2d_tensor& g = grad_outs[t < n_grad_outs ? t : 0];
        q.g[t] = g.data;
        q.g_sn[t] = g.stride_n;
        q.g_sc[t] = g.stride_c;
        q.g_sh[t] = g.stride_h;
      }
      bool gvec = true;
      for (int32_t j = 0; j < n_grad_outs; ++j) gvec = gvec && row_aligned(grad_outs[j], 16);
      q.flags = gvec ? kDstVec : 0;
      q.partial = partial;
      q.H = im.h;
      q.W = im.w;
      q.nf = fp.nf;
      q.nrep = fp.nrep;
      q.chunks = fp.chunks;
      q.n_units = fp.n_units;
      q.mode = pr.mode;
      q.m = pr.m;
      q.C = static_cast<int32_t>(im.c);
      q.tiles_x = fp.tiles_x;
      q.tiles_y = fp.tiles_y;
      q.tiles_per_unit = fp.tpu;
      if (fp.n_units > kMaxBlocks) return fail(F2D_EUNSUPPORTED, "too many grad_filter work units");
      int no = 1, ni = 1;
      hipError_t err;
      if (grad_filter_bank_groups(pr.mode, K, pr.c_out, im.c, &no, &ni)) {
        // filter groups: same partial slots, NO * NI pairs per work-group
        q.n_units = fp.nrep * fp.chunks * (pr.c_out / no) * (im.c / ni);
        err = launch_grad_filter_bank_f32(q, K, s);
      } else {
        err = K <= 9 ? launch_grad_filter_f32(q, K, s) : launch_grad_filter_generic(q, K, s);
      }
      if (err != hipSuccess) return hip_status(err, "grad_filter launch");
    }
    hipError_t err = launch_reduce_partials(partial, grad_filter, fp.nf, K * K, fp.nrep,
                                            empty ? 0 : fp.chunks, s);
    if (err != hipSuccess) return hip_status(err, "grad_filter reduce launch");
  }
  return ok();
}

}  // namespace f2d
