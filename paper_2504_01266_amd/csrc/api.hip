// C-ABI entry points: host-side validation, planning and dispatch.
//
// Every entry point validates all of its arguments on the host before it
// enqueues anything; a failing call returns a status, records a message for
// filter2d_last_error() and leaves the outputs untouched.  Nothing here
// allocates device memory or synchronises, except the explicitly synchronous
// autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "f2d_internal.hpp"
#include "f2d_host.hpp"

namespace f2d {

// ------------------------------------------------------------ errors ----
namespace {
thread_local char g_err[512] = "";
}

f2d_status fail(f2d_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return s;
}

f2d_status ok() {
  g_err[0] = '\0';
  return F2D_OK;
}

f2d_status hip_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return ok();
  return fail(F2D_EHIP, "%s: %s", what, hipGetErrorString(e));
}

const char* last_error() { return g_err; }

// ------------------------------------------------------------ tuning ----
namespace {
using TuneKey = std::tuple<int, int, int, int, int>;  // path, dtype, k, channels, wclass
std::map<TuneKey, int> g_tune;
std::mutex g_tune_mu;
}  // namespace

int width_class(int64_t w) { return w < 256 ? 0 : (w < 1024 ? 1 : (w < 4096 ? 2 : 3)); }

int variant_count(int path) {
  switch (path) {
    case kPathF32: return f32_variant_count();
    case kPathU8: return u8_variant_count();
    case kPathBatched: return batched_variant_count();
    default: return 0;
  }
}

int resolve_variant(int path, int dtype, int k, int channels, int64_t w, int requested) {
  if (requested > 0) return requested;
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(TuneKey(path, dtype, k, channels, width_class(w)));
  return it == g_tune.end() ? 1 : it->second;
}

void record_variant(int path, int dtype, int k, int channels, int64_t w, int variant) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune[TuneKey(path, dtype, k, channels, width_class(w))] = variant;
}

f2d_status tune_save(const char* path) {
  if (!path) return fail(F2D_EINVAL, "tune_save: path is NULL");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  FILE* f = fopen(path, "w");
  if (!f) return fail(F2D_EINVAL, "tune_save: cannot open %s", path);
  fprintf(f, "{\"format\": \"filter2d-tune-1\", \"fields\": [\"path\", \"dtype\", \"k\", "
             "\"channels\", \"wclass\", \"variant\"],\n \"entries\": [");
  bool first = true;
  for (const auto& kv : g_tune) {
    fprintf(f, "%s\n  [%d, %d, %d, %d, %d, %d]", first ? "" : ",", std::get<0>(kv.first),
            std::get<1>(kv.first), std::get<2>(kv.first), std::get<3>(kv.first),
            std::get<4>(kv.first), kv.second);
    first = false;
  }
  fprintf(f, "\n ]}\n");
  fclose(f);
  return ok();
}

f2d_status tune_load(const char* path) {
  if (!path) return fail(F2D_EINVAL, "tune_load: path is NULL");
  FILE* f = fopen(path, "r");
  if (!f) return fail(F2D_EINVAL, "tune_load: cannot open %s", path);
  std::string text;
  char buf[4096];
  size_t got;
  while ((got = fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
  fclose(f);
  size_t pos = text.find("\"entries\"");
  if (pos == std::string::npos) return fail(F2D_EINVAL, "tune_load: no \"entries\" in %s", path);
  std::vector<long> nums;
  for (size_t i = pos; i < text.size(); ++i) {
    if ((text[i] >= '0' && text[i] <= '9') || text[i] == '-') {
      char* end = nullptr;
      nums.push_back(strtol(text.c_str() + i, &end, 10));
      i = static_cast<size_t>(end - text.c_str()) - 1;
    }
  }
  if (nums.size() % 6 != 0) return fail(F2D_EINVAL, "tune_load: malformed entries in %s", path);
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (size_t i = 0; i < nums.size(); i += 6) {
    const int p = static_cast<int>(nums[i]);
    const int v = static_cast<int>(nums[i + 5]);
    if (v < 1 || v > variant_count(p)) continue;
    g_tune[TuneKey(p, static_cast<int>(nums[i + 1]), static_cast<int>(nums[i + 2]),
                   static_cast<int>(nums[i + 3]), static_cast<int>(nums[i + 4]))] = v;
  }
  return ok();
}

void tune_clear() {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
}

// -------------------------------------------------------- validation ----

int64_t numel(const f2d_tensor& t) { return t.n * t.c * t.h * t.w; }

f2d_status check_tensor(const f2d_tensor* t, const char* name, bool is_output) {
  if (!t) return fail(F2D_EINVAL, "%s: descriptor is NULL", name);
  if (t->n < 0 || t->c < 0 || t->h < 0 || t->w < 0)
    return fail(F2D_EINVAL, "%s: negative extent", name);
  if (t->stride_n < 0 || t->stride_c < 0 || t->stride_h < 0 || t->stride_w < 0)
    return fail(F2D_EINVAL, "%s: negative stride", name);
  if (t->dtype < F2D_U8 || t->dtype > F2D_BF16) return fail(F2D_EINVAL, "%s: unknown dtype %d", name, t->dtype);
  if (numel(*t) > 0 && !t->data) return fail(F2D_EINVAL, "%s: data is NULL", name);
  if (is_output && numel(*t) > 0) {
    // outputs must not alias themselves
    const int64_t sw = t->stride_w <= 1 ? 1 : t->stride_w;
    if (sw > 1) {
      // interleaved: channels inside the pixel, pixels inside the row, rows inside the image
      const int64_t pixel = (t->c - 1) * t->stride_c + 1;
      if (t->c > 1 && (t->stride_c < 1 || pixel > sw)) return fail(F2D_EINVAL, "%s: channels overlap", name);
      const int64_t row = (t->w - 1) * sw + pixel;
      if (t->h > 1 && t->stride_h < row) return fail(F2D_EINVAL, "%s: rows overlap", name);
      const int64_t image = (t->h - 1) * t->stride_h + row;
      if (t->n > 1 && t->stride_n < image) return fail(F2D_EINVAL, "%s: images overlap", name);
      return F2D_OK;
    }
    // planar: rows, planes and images disjoint
    if (t->h > 1 && t->stride_h < t->w) return fail(F2D_EINVAL, "%s: stride_h < w", name);
    const int64_t plane = (t->h - 1) * t->stride_h + t->w;
    if (t->c > 1 && t->stride_c < plane) return fail(F2D_EINVAL, "%s: planes overlap", name);
    const int64_t image = (t->c - 1) * t->stride_c + plane;
    if (t->n > 1 && t->stride_n < image) return fail(F2D_EINVAL, "%s: images overlap", name);
  }
  return F2D_OK;
}

size_t dtype_size(int32_t dt) { return dt == F2D_U8 ? 1 : (dt == F2D_BF16 ? 2 : 4); }

bool row_aligned(const f2d_tensor& t, size_t bytes) {
  const size_t es = dtype_size(t.dtype);
  const uintptr_t a = reinterpret_cast<uintptr_t>(t.data);
  auto ok_stride = [&](int64_t s, int64_t extent) { return extent <= 1 || (s * es) % bytes == 0; };
  return a % bytes == 0 && ok_stride(t.stride_h, t.h) && ok_stride(t.stride_c, t.c) &&
         ok_stride(t.stride_n, t.n);
}

f2d_status check_common(const f2d_tensor* image, const f2d_filter* filter, const f2d_opts* opts,
                        Problem* pr) {
  if (!opts) return fail(F2D_EINVAL, "opts is NULL");
  if (!filter) return fail(F2D_EINVAL, "filter is NULL");
  f2d_status s = check_tensor(image, "image", false);
  if (s) return s;
  if (opts->border != F2D_BORDER_CLAMP && opts->border != F2D_BORDER_ZERO)
    return fail(F2D_EINVAL, "unknown border %d", opts->border);
  if (opts->channels < F2D_CH_SHARED || opts->channels > F2D_CH_BANK)
    return fail(F2D_EINVAL, "unknown channel mode %d", opts->channels);
  if (opts->epilogue != F2D_EPI_NONE && opts->epilogue != F2D_EPI_SUMSQ_PAIRS)
    return fail(F2D_EINVAL, "unknown epilogue %d", opts->epilogue);
  if (opts->variant < 0) return fail(F2D_EINVAL, "variant %d < 0", opts->variant);
  const int32_t k = filter->k;
  if (k < 1 || k > 31 || k % 2 == 0) return fail(F2D_EINVAL, "filter k=%d: must be odd, 1..31", k);
  if (filter->f_out < 1 || filter->f_in < 1)
    return fail(F2D_EINVAL, "filter f_out=%d f_in=%d: must be >= 1", filter->f_out, filter->f_in);
  if (!filter->data) return fail(F2D_EINVAL, "filter data is NULL");
  if (filter->dtype < F2D_U8 || filter->dtype > F2D_BF16)
    return fail(F2D_EINVAL, "filter: unknown dtype %d", filter->dtype);

  const int64_t C = image->c;
  pr->mode = opts->channels;
  pr->k = k;
  pr->m = 1;
  switch (opts->channels) {
    case F2D_CH_SHARED:
      if (filter->f_out != 1 || filter->f_in != 1)
        return fail(F2D_EINVAL, "SHARED needs a [1][1][k][k] filter, got [%d][%d]", filter->f_out, filter->f_in);
      pr->c_out = C;
      break;
    case F2D_CH_DEPTHWISE:
      if (filter->f_in != 1) return fail(F2D_EINVAL, "DEPTHWISE needs f_in = 1, got %d", filter->f_in);
      if (C < 1 || filter->f_out % C != 0)
        return fail(F2D_EINVAL, "DEPTHWISE needs f_out (%d) a multiple of C (%lld)", filter->f_out,
                    static_cast<long long>(C));
      pr->m = filter->f_out / static_cast<int32_t>(C);
      pr->c_out = C;
      break;
    default:
      if (filter->f_in != C)
        return fail(F2D_EINVAL, "BANK needs f_in = C (%lld), got %d", static_cast<long long>(C), filter->f_in);
      pr->c_out = filter->f_out;
      break;
  }
  if (opts->epilogue == F2D_EPI_SUMSQ_PAIRS && (opts->channels != F2D_CH_DEPTHWISE || pr->m != 2))
    return fail(F2D_EINVAL, "SUMSQ_PAIRS needs DEPTHWISE with 2 filters per channel");

  pr->row_begin = opts->row_begin;
  pr->row_end = opts->row_end <= 0 ? image->h : opts->row_end;
  if (pr->row_begin < 0 || pr->row_begin > pr->row_end || pr->row_end > image->h)
    return fail(F2D_EINVAL, "rows [%lld, %lld) outside the image (h = %lld)",
                static_cast<long long>(pr->row_begin), static_cast<long long>(pr->row_end),
                static_cast<long long>(image->h));
  pr->rows = pr->row_end - pr->row_begin;

  // element-type combinations
  const int32_t it = image->dtype, ft = filter->dtype;
  if (it == F2D_U8) {
    if (ft != F2D_I32 && ft != F2D_F32) return fail(F2D_EINVAL, "u8 images need an int32 or float filter");
    if (opts->channels == F2D_CH_BANK && k != 1)
      return fail(F2D_EUNSUPPORTED, "u8 images in BANK mode: k = 1 (per-pixel channel mixing) only");
    pr->out_dtype = ft == F2D_I32 ? F2D_I32 : F2D_F32;  // or U8, chosen by the output descriptor
  } else if (it == F2D_F32) {
    if (ft != F2D_F32) return fail(F2D_EINVAL, "f32 images need an f32 filter");
    if (opts->epilogue != F2D_EPI_NONE) return fail(F2D_EUNSUPPORTED, "SUMSQ_PAIRS is implemented for u8 images only");
    pr->out_dtype = F2D_F32;
  } else if (it == F2D_BF16) {
    if (ft != F2D_BF16) return fail(F2D_EINVAL, "bf16 images need a bf16 filter");
    if (opts->channels != F2D_CH_BANK) return fail(F2D_EUNSUPPORTED, "bf16 images: only BANK mode is implemented");
    if (k != 1 && k != 3 && k != 5) return fail(F2D_EUNSUPPORTED, "bf16 banks: k in {1, 3, 5} (got %d)", k);
    pr->out_dtype = F2D_F32;  // or BF16, chosen by the output descriptor
  } else {
    return fail(F2D_EUNSUPPORTED, "image dtype %d is not supported", it);
  }
  if (opts->border == F2D_BORDER_ZERO && it != F2D_F32 && it != F2D_U8)
    return fail(F2D_EUNSUPPORTED, "zero borders are implemented for f32 and u8 images only");
  if (it != F2D_U8 && image->stride_w > 1)
    return fail(F2D_EUNSUPPORTED, "image stride_w %d: interleaved layouts are implemented for u8 images only",
                image->stride_w);
  pr->image = *image;
  pr->filter = *filter;
  pr->opts = *opts;
  return F2D_OK;
}

f2d_status check_outputs(const Problem& pr, const f2d_tensor* outs, int32_t n_outs, const char* what) {
  int32_t want = 1;
  if (pr.mode == F2D_CH_DEPTHWISE) want = pr.m + (pr.opts.epilogue == F2D_EPI_SUMSQ_PAIRS ? 1 : 0);
  if (n_outs != want) return fail(F2D_EINVAL, "%s: expected %d output tensors, got %d", what, want, n_outs);
  if (!outs) return fail(F2D_EINVAL, "%s: output array is NULL", what);
  const int64_t co = pr.mode == F2D_CH_BANK ? pr.c_out : pr.image.c;
  for (int32_t j = 0; j < n_outs; ++j) {
    char name[64];
    snprintf(name, sizeof(name), "%s[%d]", what, j);
    f2d_status s = check_tensor(&outs[j], name, true);
    if (s) return s;
    const f2d_tensor& o = outs[j];
    if (o.n != pr.image.n || o.c != co || o.h != pr.rows || o.w != pr.image.w)
      return fail(F2D_EINVAL, "%s: shape [%lld][%lld][%lld][%lld], expected [%lld][%lld][%lld][%lld]", name,
                  static_cast<long long>(o.n), static_cast<long long>(o.c), static_cast<long long>(o.h),
                  static_cast<long long>(o.w), static_cast<long long>(pr.image.n),
                  static_cast<long long>(co), static_cast<long long>(pr.rows),
                  static_cast<long long>(pr.image.w));
    const bool bf16_ok = pr.image.dtype == F2D_BF16 && o.dtype == F2D_BF16;
    const bool u8_ok = pr.image.dtype == F2D_U8 && o.dtype == F2D_U8;
    if (o.dtype != pr.out_dtype && !bf16_ok && !u8_ok)
      return fail(F2D_EINVAL, "%s: dtype %d, expected %d", name, o.dtype, pr.out_dtype);
    if (pr.image.dtype != F2D_U8 && o.stride_w > 1)
      return fail(F2D_EUNSUPPORTED, "%s: interleaved layouts are implemented for u8 images only", name);
  }
  return F2D_OK;
}

}  // namespace f2d

using namespace f2d;

// ===================================================================== ABI

extern "C" {

f2d_status filter2d_forward(const f2d_tensor* image, const f2d_filter* filter, const f2d_opts* opts,
                            const f2d_tensor* outs, int32_t n_outs, void* stream) {
  Problem pr;
  f2d_status s = check_common(image, filter, opts, &pr);
  if (s) return s;
  s = check_outputs(pr, outs, n_outs, "outs");
  if (s) return s;
  return run_forward(pr, outs, n_outs, static_cast<hipStream_t>(stream));
}

f2d_status filter2d_forward_separable(const f2d_tensor* image, const float* a, const float* b, int32_t k,
                                     const f2d_opts* opts, const f2d_tensor* out, void* stream) {
  if (!a || !b) return fail(F2D_EINVAL, "separable: factor a or b is NULL");
  if (opts && opts->channels != F2D_CH_SHARED)
    return fail(F2D_EUNSUPPORTED, "separable: SHARED channel mode only");
  const f2d_filter filter{a, F2D_F32, 1, 1, k};
  Problem pr;
  f2d_status s = check_common(image, &filter, opts, &pr);
  if (s) return s;
  if (image->dtype != F2D_F32) return fail(F2D_EUNSUPPORTED, "separable: f32 images only");
  if (opts->border != F2D_BORDER_CLAMP) return fail(F2D_EUNSUPPORTED, "separable: clamp-to-edge borders only");
  if (k > 15) return fail(F2D_EUNSUPPORTED, "separable: k=%d (1..15 are built)", k);
  s = check_outputs(pr, out, 1, "out");
  if (s) return s;
  return run_forward_separable(pr, a, b, *out, static_cast<hipStream_t>(stream));
}

size_t filter2d_backward_workspace(const f2d_tensor* image, const f2d_filter* filter,
                                   const f2d_opts* opts) {
  Problem pr;
  if (check_common(image, filter, opts, &pr)) return 0;
  if (opts->border != F2D_BORDER_CLAMP) return 0;
  return backward_workspace(pr);
}

f2d_status filter2d_backward(const f2d_tensor* image, const f2d_filter* filter,
                             const f2d_tensor* grad_outs, int32_t n_grad_outs, const f2d_opts* opts,
                             const f2d_tensor* grad_input, float* grad_filter, void* workspace,
                             size_t workspace_bytes, void* stream) {
  Problem pr;
  f2d_status s = check_common(image, filter, opts, &pr);
  if (s) return s;
  if (opts->border != F2D_BORDER_CLAMP)
    return fail(F2D_EUNSUPPORTED, "backward: clamp-to-edge borders only (zero borders are forward-only)");
  return run_backward(pr, grad_outs, n_grad_outs, grad_input, grad_filter, workspace, workspace_bytes,
                      static_cast<hipStream_t>(stream));
}

f2d_status filter2d_backward_noalloc(const f2d_tensor* image, const f2d_filter* filter,
                                     const f2d_tensor* grad_outs, int32_t n_grad_outs, const f2d_opts* opts,
                                     const f2d_tensor* grad_input, float* grad_filter, void* stream) {
  Problem pr;
  f2d_status s = check_common(image, filter, opts, &pr);
  if (s) return s;
  if (opts->border != F2D_BORDER_CLAMP)
    return fail(F2D_EUNSUPPORTED, "backward: clamp-to-edge borders only (zero borders are forward-only)");
  return run_backward_noalloc(pr, grad_outs, n_grad_outs, grad_input, grad_filter,
                              static_cast<hipStream_t>(stream));
}

f2d_status filter2d_upsample_forward(const f2d_tensor* image, const f2d_filter* filter, int32_t scale,
                                     const f2d_opts* opts, const f2d_tensor* out, void* stream) {
  Problem pr;
  f2d_status s = check_common(image, filter, opts, &pr);
  if (s) return s;
  if (scale < 1 || scale > 4096) return fail(F2D_EINVAL, "upsample: scale %d outside 1..4096", scale);
  if (image->dtype != F2D_U8) return fail(F2D_EUNSUPPORTED, "upsample: u8 images only");
  if (opts->channels != F2D_CH_SHARED) return fail(F2D_EUNSUPPORTED, "upsample: SHARED channel mode only");
  if (opts->epilogue != F2D_EPI_NONE) return fail(F2D_EINVAL, "upsample: no epilogue");
  if (pr.row_begin != 0 || pr.row_end != image->h)
    return fail(F2D_EUNSUPPORTED, "upsample: whole images only (row_begin = 0, row_end = 0 or h)");
  if (!out) return fail(F2D_EINVAL, "upsample: out is NULL");
  s = check_tensor(out, "out", true);
  if (s) return s;
  if (out->n != image->n || out->c != image->c || out->h != image->h * scale || out->w != image->w * scale)
    return fail(F2D_EINVAL, "upsample: out must be [N][C][H*scale][W*scale]");
  if (out->dtype != F2D_U8 && out->dtype != pr.out_dtype)
    return fail(F2D_EINVAL, "upsample: out dtype %d (u8, or int32 for int32 taps, f32 for float taps)", out->dtype);
  return run_upsample_forward(pr, scale, *out, static_cast<hipStream_t>(stream));
}

int64_t filter2d_batched_plan(const f2d_batch_item* items, int32_t n_items, int32_t dtype, int32_t k,
                              int32_t* variant, int64_t* tile_prefix) {
  return batched_plan(items, n_items, dtype, k, variant, tile_prefix);
}

f2d_status filter2d_batched(const f2d_batch_item* items_dev, const int64_t* tile_prefix_dev,
                            int32_t n_items, int64_t total_tiles, int32_t dtype, int32_t k,
                            const f2d_opts* opts, void* stream) {
  return run_batched(items_dev, tile_prefix_dev, n_items, total_tiles, dtype, k, opts,
                     static_cast<hipStream_t>(stream));
}

f2d_status filter2d_autotune_forward(const f2d_tensor* image, const f2d_filter* filter,
                                     const f2d_opts* opts, const f2d_tensor* outs, int32_t n_outs,
                                     int32_t reps, void* stream, int32_t* best_variant) {
  Problem pr;
  f2d_status s = check_common(image, filter, opts, &pr);
  if (s) return s;
  s = check_outputs(pr, outs, n_outs, "outs");
  if (s) return s;
  return autotune_forward(pr, outs, n_outs, reps, static_cast<hipStream_t>(stream), best_variant);
}

f2d_status filter2d_autotune_batched(const f2d_batch_item* items_host, const f2d_batch_item* items_dev,
                                     int32_t n_items, int32_t dtype, int32_t k, int64_t* tile_prefix_dev,
                                     int32_t reps, void* stream, int32_t* best_variant) {
  return autotune_batched(items_host, items_dev, n_items, dtype, k, tile_prefix_dev, reps,
                          static_cast<hipStream_t>(stream), best_variant);
}

int32_t filter2d_variant_count(int32_t path) { return variant_count(path); }

f2d_status filter2d_tune_save(const char* path) { return tune_save(path); }
f2d_status filter2d_tune_load(const char* path) { return tune_load(path); }
void filter2d_tune_clear(void) { tune_clear(); }

const char* filter2d_status_string(f2d_status s) {
  switch (s) {
    case F2D_OK: return "F2D_OK";
    case F2D_EINVAL: return "F2D_EINVAL: invalid argument";
    case F2D_EUNSUPPORTED: return "F2D_EUNSUPPORTED: not implemented for these arguments";
    case F2D_EWORKSPACE: return "F2D_EWORKSPACE: workspace missing or too small";
    case F2D_EHIP: return "F2D_EHIP: HIP runtime error";
    default: return "unknown status";
  }
}

const char* filter2d_last_error(void) { return last_error(); }

int32_t filter2d_version(void) { return 100; }

}  // extern "C"
