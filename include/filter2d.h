/*
 * filter2d.h -- C ABI of the MI355X (gfx950) K x K 2D filter library.
 *
 * The operation is the generalisation of the 3x3 Laplacian sharpen of
 * arXiv:2504.01266 (Section 4.2.4, "Sharpening": every output pixel is a
 * weighted sum of its neighbourhood, each colour channel on its own) to
 *
 *   Y[n][o][y][x] = sum_{i in inputs(o)} sum_{u,v=0}^{K-1}
 *                   F[o|i][u][v] * X[n][i][cl_H(y+u-r)][cl_W(x+v-r)]
 *
 * with odd K, r = (K-1)/2, correlation (tap (u,v) weighs the neighbour at
 * offset (u-r, v-r)) and clamp-to-edge borders cl_n(t) = min(max(t,0), n-1)
 * applied to each axis.  The paper's sharpen skips out-of-image neighbours
 * (Section 4.2.4); that rule is F2D_BORDER_ZERO (X reads as 0 outside the
 * image), implemented for the FP32 forward and the 8-bit SHARED forward.
 *
 * Channel modes (F is always a contiguous [f_out][f_in][k][k] array):
 *   F2D_CH_SHARED     f_out = f_in = 1: the same filter on every channel
 *                     (the paper's per-channel loop of Section 4.2.4).
 *   F2D_CH_DEPTHWISE  f_in = 1, f_out = C*m: filter c*m+j is applied to
 *                     channel c (m = 2 with Sobel-x / Sobel-y gives edge maps).
 *   F2D_CH_BANK       f_in = C: output channel o sums the correlations of all
 *                     C input channels i with F[o][i] (a convolution layer;
 *                     K = 1, C = 3, f_out = 1 is the weighted RGB -> gray map
 *                     of Section 4.2.5, "Grayscaling").
 *
 * Conventions for every entry point:
 *   - Data pointers in f2d_tensor / f2d_filter / f2d_batch_item are DEVICE
 *     pointers; every other pointer argument is a HOST pointer unless stated.
 *   - The caller owns every buffer (images, filters, outputs, workspaces,
 *     descriptor tables).  The library allocates no device memory, keeps no
 *     device state between calls and never synchronises the stream, except in
 *     the explicitly synchronous filter2d_autotune_* calls.  The one device
 *     state is the static scratch array of filter2d_backward_noalloc.
 *   - `stream` is a hipStream_t (NULL = the default stream); work is only
 *     enqueued on it, so calls are capturable into a hipGraph.
 *   - Arguments are validated on the host before anything is enqueued: an
 *     invalid call returns a non-zero status, enqueues nothing and leaves the
 *     outputs untouched; filter2d_last_error() then names the argument.
 *   - A launch failure returns F2D_EHIP with the HIP error text.  Faults that
 *     happen while the kernels run are reported by the next synchronising
 *     HIP call, as for any asynchronous launch.
 *   - Strides are in ELEMENTS; the x (column) stride is 1 except for the
 *     interleaved 8-bit layouts (f2d_tensor.stride_w).
 *   - Outputs must not overlap inputs.
 */
#ifndef FILTER2D_H
#define FILTER2D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t f2d_status;
#define F2D_OK 0
#define F2D_EINVAL 1       /* malformed argument (shape, stride, null pointer, even K ...) */
#define F2D_EUNSUPPORTED 2 /* well-formed but not implemented (dtype combination, border ...) */
#define F2D_EWORKSPACE 3   /* workspace missing or smaller than required */
#define F2D_EHIP 4         /* the HIP runtime refused a launch */

/* element types */
#define F2D_U8 0
#define F2D_I32 1
#define F2D_F32 2
#define F2D_BF16 3

/* border rules */
#define F2D_BORDER_CLAMP 0 /* replicate the edge pixel: cl_n(t) = min(max(t,0), n-1) */
#define F2D_BORDER_ZERO 1  /* out-of-image neighbours add nothing (the paper's sharpen,
                              Section 4.2.4): filter2d_forward on FP32 images and
                              on U8 images in SHARED mode, and
                              filter2d_upsample_forward (F2D_EUNSUPPORTED
                              elsewhere) */

/* channel modes */
#define F2D_CH_SHARED 0
#define F2D_CH_DEPTHWISE 1
#define F2D_CH_BANK 2

/* epilogues */
#define F2D_EPI_NONE 0
#define F2D_EPI_SUMSQ_PAIRS 1 /* DEPTHWISE m = 2 only: an extra output o0^2 + o1^2 */

/* A 4-D image [n][c][h][w]. */
typedef struct f2d_tensor {
  void* data;       /* device pointer to element (0,0,0,0) */
  int32_t dtype;    /* F2D_U8 / F2D_I32 / F2D_F32 / F2D_BF16 */
  int32_t stride_w; /* elements between horizontally adjacent pixels; 0 means 1.
                       Planar layouts use 1; interleaved 8-bit images (OpenCV's
                       pixel-after-pixel layout, Sections 4.2.3-4.2.4) use
                       stride_w = c with stride_c = 1.  Only the 8-bit paths that
                       say so accept a value other than 0 / 1. */
  int64_t n, c, h, w;
  int64_t stride_n, stride_c, stride_h; /* elements */
} f2d_tensor;

/* A filter bank [f_out][f_in][k][k], contiguous. */
typedef struct f2d_filter {
  const void* data; /* device pointer */
  int32_t dtype;    /* F2D_I32 (u8 images), F2D_F32, F2D_BF16 */
  int32_t f_out, f_in, k;
} f2d_filter;

typedef struct f2d_opts {
  int32_t border;   /* F2D_BORDER_CLAMP */
  int32_t channels; /* F2D_CH_* */
  int32_t epilogue; /* F2D_EPI_* */
  int32_t variant;  /* 0: tuned / default tiling; > 0 forces a tiling variant */
  /* Output rows [row_begin, row_end) of the INPUT buffer are produced
   * (row_end <= 0 means image->h).  A GPU that owns output rows [y0, y1) of an
   * image of height H passes the input rows [max(0,y0-r), min(H,y1+r)) as the
   * image and selects its own rows here; clamping at the buffer edge then
   * equals clamping at the image edge, so bands concatenate to the whole. */
  int64_t row_begin, row_end;
} f2d_opts;

/*
 * filter2d_forward -- Y = filter(X), the equation at the top of this file.
 *
 *   image   [N][C][H][W]
 *   filter  see the channel modes
 *   outs    n_outs output descriptors, each [N][C_o][rows][W] with
 *           rows = row_end - row_begin:
 *             SHARED     n_outs = 1, C_o = C
 *             DEPTHWISE  n_outs = m (+1 with SUMSQ_PAIRS), C_o = C; outs[j]
 *                        holds the response of filter c*m+j to channel c
 *                        (pass strided views for an interleaved [N][C*m] layout)
 *             BANK       n_outs = 1, C_o = f_out
 *   dtypes  U8 image + I32 filter -> I32 outputs (SHARED, DEPTHWISE): exact
 *           integer sums, wrapping modulo 2^32 if they leave the int32 range;
 *           U8 image + F32 filter (the paper's float taps, Section 4.2.4) ->
 *           F32 outputs: the sum in binary32, accumulator +0 and one fused
 *           multiply-add per term (input channel, tap row, tap column);
 *           U8 image + I32 or F32 filter -> U8 outputs: that sum clamped to
 *           [0, 255] and rounded to nearest, ties to even (int32 sums are
 *           clamped; they must stay inside the int32 range);
 *           F32 + F32 -> F32 (all modes), FP32 accumulation;
 *           BF16 + BF16 -> F32 or BF16 (BANK only), FP32 accumulation on the
 *           matrix cores, output rounded to nearest even for BF16.
 *   border  CLAMP for every dtype; ZERO for F32 images (all channel modes,
 *           bands included: rows outside the buffer read as 0) and for U8
 *           images in SHARED mode.
 *   U8      SHARED: K <= 7 unless the filter is I32 with I32 outputs, CLAMP
 *           and a planar layout (then K <= 31); the image may be interleaved
 *           (stride_c = 1, stride_w = C, C = 3 or 4) with an output in the same
 *           layout.  DEPTHWISE: I32 taps and outputs, CLAMP, planar.  BANK:
 *           K = 1 only (per-pixel channel mixing, e.g. the grayscale weights
 *           of Section 4.2.5), at most 4 input and 4 output channels, planar
 *           or interleaved input and output.
 *   K       odd, 1 <= K <= 31 (F32, U8 as above); K in {1,3,5} for BF16 banks
 *           (other odd K return F2D_EUNSUPPORTED); BF16 banks take at most 64
 *           input channels.
 */
f2d_status filter2d_forward(const f2d_tensor* image, const f2d_filter* filter,
                            const f2d_opts* opts, const f2d_tensor* outs, int32_t n_outs,
                            void* stream);

/*
 * filter2d_forward_separable -- filter2d_forward for a rank-one filter
 * F[u][v] = a[u] * b[v] (the equation at the top of this file with that F),
 * computed as a row pass then a column pass: 2K multiply-adds per output
 * instead of K^2.
 *
 *   image   [N][C][H][W] F32
 *   a, b    DEVICE pointers to k floats each: a weighs the row offset u - r,
 *           b the column offset v - r (a normalised Gaussian is g g^T)
 *   k       odd, 1..15 (F2D_EUNSUPPORTED for larger odd k)
 *   opts    border CLAMP, channels SHARED (one a, b for every channel),
 *           epilogue NONE; variant ignored; row_begin / row_end select a band
 *           of output rows exactly as for filter2d_forward
 *   out     [N][C][rows][W] F32, rows = row_end - row_begin
 * Every output is sum_u a[u] * (sum_v b[v] * X[..]) in FP32 with the clamp
 * applied to the source rows and columns, so it equals filter2d_forward with
 * F = a b^T up to FP32 rounding (not bitwise).  Ownership, validation and
 * errors as for filter2d_forward; other dtypes and channel modes return
 * F2D_EUNSUPPORTED.
 */
f2d_status filter2d_forward_separable(const f2d_tensor* image, const float* a, const float* b, int32_t k,
                                      const f2d_opts* opts, const f2d_tensor* out, void* stream);

/*
 * filter2d_upsample_forward -- the paper's upsample-then-sharpen pipeline
 * (Section 6.6) in one pass: Y = filter(U), where U is X enlarged by nearest-
 * neighbour upsampling by the integer factor `scale` (Section 4.2.3: output
 * pixel (Y, X) copies source pixel (Y / scale, X / scale), integer division)
 * and filter is filter2d_forward's SHARED map on U with opts->border (the
 * border is U's border).  U is never written to memory: each output reads
 * the source pixels its taps map to.
 *
 *   image   [N][C][H][W] U8, planar or interleaved (as filter2d_forward)
 *   filter  [1][1][k][k], odd k <= 7, I32 or F32 taps
 *   scale   1..4096 (1 is filter2d_forward)
 *   opts    channels SHARED, epilogue NONE, whole images (row_begin = 0 and
 *           row_end = 0 or H); border CLAMP or ZERO
 *   out     [N][C][H*scale][W*scale] in the image's layout: U8 (clamped and
 *           rounded as filter2d_forward), or I32 (I32 taps) / F32 (F32 taps)
 * Ownership, validation and errors as for filter2d_forward.
 */
f2d_status filter2d_upsample_forward(const f2d_tensor* image, const f2d_filter* filter, int32_t scale,
                                     const f2d_opts* opts, const f2d_tensor* out, void* stream);

/*
 * Workspace bytes that filter2d_backward needs for these arguments (device
 * memory, caller-allocated, any alignment >= 256 bytes).  Returns 0 for
 * invalid arguments.  The workspace holds the r-wide frame of the image
 * adjoint (folded onto the edge pixels afterwards) and the per-work-unit
 * grad_filter partial sums of the reduction below; the paper's own
 * reductions (Section 4.2.8) combine per-block partials the same way.
 */
size_t filter2d_backward_workspace(const f2d_tensor* image, const f2d_filter* filter,
                                   const f2d_opts* opts);

/*
 * filter2d_backward -- the adjoints of filter2d_forward (whole images only:
 * opts->row_begin/row_end must select all rows).  The paper defines only the
 * forward weighted sum (Section 4.2.4); these are the transposes of that
 * linear map, in the image and in the filter, which gradient-based callers
 * (training a filter bank) need.
 *
 *   grad_outs    n_grad_outs upstream gradients laid out like forward's outs
 *                (no SUMSQ output); F32 (or BF16 for BF16 banks).
 *   grad_input   nullable, [N][C][H][W] F32:  X-bar = A^T G-bar.  At the clamp
 *                borders every edge pixel also receives the gradient of the
 *                neighbours that were clamped onto it.
 *   grad_filter  nullable, device, contiguous F32 [f_out][f_in][k][k]:
 *                F-bar[o][i][u][v] = sum_{n,y,x} G-bar[n][o][y][x] *
 *                X[n][i][cl(y+u-r)][cl(x+v-r)]  (summed over channels too in
 *                SHARED mode), reduced in a fixed order, so repeated calls are
 *                bitwise identical.
 *   workspace    device scratch of filter2d_backward_workspace() bytes.
 * U8 images are not differentiable (F2D_EUNSUPPORTED).
 */
f2d_status filter2d_backward(const f2d_tensor* image, const f2d_filter* filter,
                             const f2d_tensor* grad_outs, int32_t n_grad_outs,
                             const f2d_opts* opts, const f2d_tensor* grad_input,
                             float* grad_filter, void* workspace, size_t workspace_bytes,
                             void* stream);

/*
 * filter2d_backward_noalloc -- filter2d_backward without a caller workspace,
 * for callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc).  The workspace is a
 * static device array of F2D_NOALLOC_SCRATCH_BYTES owned by the library: each
 * device the library runs on holds its own copy from its first use until the
 * process ends.  The call allocates nothing (no hipMalloc / hipFree).
 *
 *   Arguments, results, validation and errors as for filter2d_backward.
 *   Arguments whose filter2d_backward_workspace() exceeds
 *   F2D_NOALLOC_SCRATCH_BYTES return F2D_EWORKSPACE and enqueue nothing.
 *   The stream must belong to the current device.
 *   Calls on the same device share the array: calls that overlap in time on
 *   one device (e.g. on two streams) race and give wrong results.  Nothing in
 *   the array needs clearing between calls (every value the kernels read is
 *   written earlier in the same call).
 */
#define F2D_NOALLOC_SCRATCH_BYTES ((size_t)96 << 20)
f2d_status filter2d_backward_noalloc(const f2d_tensor* image, const f2d_filter* filter,
                                     const f2d_tensor* grad_outs, int32_t n_grad_outs,
                                     const f2d_opts* opts, const f2d_tensor* grad_input,
                                     float* grad_filter, void* stream);

/*
 * Ragged batches: images of different sizes, each with its own filter,
 * filtered in ONE launch (the batch processing the paper lists as missing in
 * Section 5).  SHARED mode, F32, clamp-to-edge; every item uses the same K
 * (odd, 1..9).
 */
typedef struct f2d_batch_item {
  const void* image;  /* device [c][h][w] */
  void* out;          /* device [c][h][w] */
  const void* filter; /* device [k][k] */
  int64_t c, h, w;
  int64_t in_stride_c, in_stride_h, out_stride_c, out_stride_h; /* elements */
} f2d_batch_item;

/*
 * Host-side plan: validates the items (host copies) and writes n_items + 2
 * words to tile_prefix (host array): the tile prefix sum tile_prefix[0..n_items]
 * followed by a tag that records the resolved variant and k.  *variant
 * selects the tiling (0 = tuned / default, replaced by the resolved variant
 * on return); pass the same variant and k to filter2d_batched.  Returns the
 * total number of tiles, or a negative f2d_status on error.
 */
int64_t filter2d_batched_plan(const f2d_batch_item* items, int32_t n_items, int32_t dtype,
                              int32_t k, int32_t* variant, int64_t* tile_prefix);

/*
 * filter2d_batched -- one launch over every tile of every item.  Variants
 * 1..4: one work-group per tile, each finding its item in the prefix table;
 * variants 5..8 (the same four tilings): one work-group per run of 4
 * consecutive tiles, staged in 16-byte chunks.  Items must have h and w
 * below 2^31 (the plan returns F2D_EUNSUPPORTED otherwise).
 * items_dev and tile_prefix_dev (n_items + 2 words) are device copies of the
 * plan's inputs and outputs.  The call reads nothing from them on the host,
 * so it is safe to capture into a hipGraph and replay while the tables stay
 * resident.  The kernel compares the table's tag with opts->variant and k: a
 * table planned for another variant or k is detected on the device and the
 * launch then writes nothing (the host cannot see the device table, so the
 * call still returns F2D_OK).
 */
f2d_status filter2d_batched(const f2d_batch_item* items_dev, const int64_t* tile_prefix_dev,
                            int32_t n_items, int64_t total_tiles, int32_t dtype, int32_t k,
                            const f2d_opts* opts, void* stream);

/*
 * Autotuner: times every tiling variant of the forward (resp. batched) call
 * for these arguments `reps` times with HIP events on `stream`, records the
 * fastest in the process-wide tuning table (keyed by path, dtype, K, channel
 * mode and image-width class) and returns it in *best_variant.  These calls
 * synchronise the stream and overwrite the outputs.
 */
f2d_status filter2d_autotune_forward(const f2d_tensor* image, const f2d_filter* filter,
                                     const f2d_opts* opts, const f2d_tensor* outs,
                                     int32_t n_outs, int32_t reps, void* stream,
                                     int32_t* best_variant);
f2d_status filter2d_autotune_batched(const f2d_batch_item* items_host,
                                     const f2d_batch_item* items_dev, int32_t n_items,
                                     int32_t dtype, int32_t k, int64_t* tile_prefix_dev,
                                     int32_t reps, void* stream, int32_t* best_variant);

/* Number of tiling variants of a path: 0 = forward F32, 1 = forward U8,
 * 2 = batched F32 (variant numbers run 1..count). */
int32_t filter2d_variant_count(int32_t path);

/* Save / load the tuning table as JSON (host file).  Loading merges. */
f2d_status filter2d_tune_save(const char* path);
f2d_status filter2d_tune_load(const char* path);
/* Drop every tuned entry (variant 0 then means the built-in default). */
void filter2d_tune_clear(void);

/*
 * Error reporting.  The paper lists inconsistent and limited error handling
 * as a shortcoming of its API (Section 5); here every entry point returns a
 * status and keeps a message.  filter2d_status_string: a static description
 * of a status code.  filter2d_last_error: the detail of the last non-OK
 * status returned on this thread (host string, valid until the thread's next
 * call into the library).
 */
const char* filter2d_status_string(f2d_status s);
const char* filter2d_last_error(void);
/* Library version as major*10000 + minor*100 + patch. */
int32_t filter2d_version(void);

#ifdef __cplusplus
}
#endif

#endif /* FILTER2D_H */
