// Host-side planning and dispatch shared by the library's C-ABI sources.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "filter2d.h"

namespace f2d {

constexpr int kPathF32 = 0;      // forward, f32 VALU stencils
constexpr int kPathU8 = 1;       // forward, u8 -> int32
constexpr int kPathBatched = 2;  // ragged batch, f32

// A validated filter2d call.
struct Problem {
  f2d_tensor image;
  f2d_filter filter;
  f2d_opts opts;
  int32_t mode;   // F2D_CH_*
  int32_t k;
  int32_t m;      // filters per channel (DEPTHWISE), else 1
  int64_t c_out;  // output channels of the whole map
  int64_t row_begin, row_end, rows;
  int32_t out_dtype;
};

// errors (api.hip)
f2d_status fail(f2d_status s, const char* fmt, ...);
f2d_status ok();
f2d_status hip_status(hipError_t e, const char* what);
f2d_status check_tensor(const f2d_tensor* t, const char* name, bool is_output);
f2d_status check_common(const f2d_tensor* image, const f2d_filter* filter, const f2d_opts* opts,
                        Problem* pr);
bool row_aligned(const f2d_tensor& t, size_t bytes);
int64_t numel(const f2d_tensor& t);

// tuning table (api.hip)
int resolve_variant(int path, int dtype, int k, int channels, int64_t w, int requested);
void record_variant(int path, int dtype, int k, int channels, int64_t w, int variant);
int variant_count(int path);

// forward.hip
f2d_status run_forward(const Problem& pr, const f2d_tensor* outs, int32_t n_outs, hipStream_t s);
f2d_status autotune_forward(const Problem& pr, const f2d_tensor* outs, int32_t n_outs, int32_t reps,
                            hipStream_t s, int32_t* best);

// image_u8.hip: 8-bit images (zero borders, float taps, u8 outputs,
// interleaved layouts, channel mixing, fused nearest upsampling)
f2d_status forward_u8_image(const Problem& pr, const f2d_tensor* outs, int32_t n_outs, hipStream_t s);
f2d_status run_upsample_forward(const Problem& pr, int32_t scale, const f2d_tensor& out, hipStream_t s);

// separable_f32.hip (a, b: device pointers to k floats each)
f2d_status run_forward_separable(const Problem& pr, const float* a, const float* b, const f2d_tensor& out,
                                 hipStream_t s);

// backward.hip
size_t backward_workspace(const Problem& pr);
f2d_status check_backward(const Problem& pr, const f2d_tensor* grad_outs, int32_t n_grad_outs,
                          const f2d_tensor* grad_input);
f2d_status run_backward(const Problem& pr, const f2d_tensor* grad_outs, int32_t n_grad_outs,
                        const f2d_tensor* grad_input, float* grad_filter, void* ws, size_t ws_bytes,
                        hipStream_t s);

// noalloc.hip: run_backward on the library's static per-device scratch
f2d_status run_backward_noalloc(const Problem& pr, const f2d_tensor* grad_outs, int32_t n_grad_outs,
                                const f2d_tensor* grad_input, float* grad_filter, hipStream_t s);

// batched.hip
int64_t batched_plan(const f2d_batch_item* items, int32_t n_items, int32_t dtype, int32_t k,
                     int32_t* variant, int64_t* tile_prefix);
f2d_status run_batched(const f2d_batch_item* items_dev, const int64_t* tile_prefix_dev, int32_t n_items,
                       int64_t total_tiles, int32_t dtype, int32_t k, const f2d_opts* opts,
                       hipStream_t s);
f2d_status autotune_batched(const f2d_batch_item* items_host, const f2d_batch_item* items_dev,
                            int32_t n_items, int32_t dtype, int32_t k, int64_t* tile_prefix_dev,
                            int32_t reps, hipStream_t s, int32_t* best);

// Largest grid (work-groups) of one launch: the x dimension may not exceed
// 2^32 - 1 work-items.
constexpr int64_t kMaxBlocks = (int64_t{1} << 32) / 256 - 1;

}  // namespace f2d
