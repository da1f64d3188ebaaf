// Ragged batch: every tile of every image of a batch in ONE launch.
//
// The host plan turns the items (images of different sizes, each with its own
// K x K filter) into a prefix sum of per-item tile counts, followed by a tag
// that records the tiling variant and K it was planned for.  The kernel runs
// one work-group per tile of the global tile list (the hardware starts the
// next work-group as soon as one retires); a work-group finds the owning item
// by binary search in the prefix table and runs the same tile code as the
// single-image FP32 path (SHARED mode, clamp-to-edge).  A table planned for
// another variant or K is recognised on the device from its tag and the
// launch then writes nothing.  The grid comes from the plan's tile count and
// nothing is read on the host at launch time, so the call can be captured in
// a hipGraph and replayed.
#include <hip/hip_runtime.h>

#include <cstring>
#include <vector>

#include "f2d_host.hpp"
#include "f2d_internal.hpp"
#include "stencil_tile.hpp"

namespace f2d {
namespace {

using namespace tile;

// Tag word after the prefix sums: the plan's variant and K.
constexpr int64_t kPlanMagic = int64_t{0x46324442} << 32;  // "F2DB"
__host__ __device__ inline int64_t plan_tag(int variant, int k) {
  return kPlanMagic | (static_cast<int64_t>(k) << 8) | static_cast<int64_t>(variant);
}

template <int K, int PX, int PY>
__global__ __launch_bounds__(kThreads) void k_batched_f32(const f2d_batch_item* __restrict__ items,
                                                          const int64_t* __restrict__ prefix,
                                                          int32_t n_items, int64_t total_tiles,
                                                          int64_t tag) {
  using G = Geom<K, PX, PY>;
  // a table planned for another tile shape or K: write nothing (uniform)
  if (prefix[n_items + 1] != tag) return;
  __shared__ float4 lds4[(G::LDS_WORDS + 3) / 4];
  float* lds = reinterpret_cast<float*>(lds4);
  const int tx = threadIdx.x % kTX;
  const int ty = threadIdx.x / kTX;

  // Tiles are taken in increasing order, so the owning item only moves
  // forward: one binary search for the first tile, then a forward step; the
  // item and its taps are reloaded only when it changes.
  int64_t t = blockIdx.x;
  if (t >= total_tiles) return;
  int lo = 0;
  {
    int hi = n_items;  // the last i with prefix[i] <= t
    while (hi - lo > 1) {
      const int mid = (lo + hi) / 2;
      if (prefix[mid] <= t) lo = mid; else hi = mid;
    }
  }
  // the search ran on uniform values; say so, so that the item and its taps
  // are fetched with scalar loads into scalar registers
  lo = __builtin_amdgcn_readfirstlane(lo);
  f2d_batch_item it;
  int64_t next_start;
  float tap[1][K * K];
  int64_t start;
  uint32_t tiles_x, per_plane;  // one item has fewer than 2^32 tiles
  auto load_item = [&]() {
    it = items[lo];
    start = prefix[lo];
    next_start = prefix[lo + 1];
    tiles_x = static_cast<uint32_t>((it.w + G::TW - 1) / G::TW);
    per_plane = tiles_x * static_cast<uint32_t>((it.h + G::TH - 1) / G::TH);
    const float* fp = static_cast<const float*>(it.filter);
#pragma unroll
    for (int e = 0; e < K * K; ++e)
      tap[0][e] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(fp[e])));
  };
  load_item();
  for (; t < total_tiles; t += gridDim.x) {
    if (t >= next_start) {
      while (lo + 1 < n_items && prefix[lo + 1] <= t) ++lo;
      lo = __builtin_amdgcn_readfirstlane(lo);
      load_item();
    }
    const uint32_t local = static_cast<uint32_t>(t - start);
    const uint32_t c = local / per_plane;
    if (c >= it.c) continue;  // uniform; unreachable with a matching plan
    const uint32_t r = local - c * per_plane;
    const uint32_t tile_y = r / tiles_x;
    const uint32_t tile_x = r - tile_y * tiles_x;
    const int64_t oy0 = static_cast<int64_t>(tile_y) * G::TH, ox0 = static_cast<int64_t>(tile_x) * G::TW;

    const float* sp = static_cast<const float*>(it.image) + c * it.in_stride_c;
    stage_tile<K, PX, PY, false>(lds, sp, it.in_stride_h, it.h, it.w, oy0, ox0);
    float acc[1][PY][PX];
#pragma unroll
    for (int jy = 0; jy < PY; ++jy)
#pragma unroll
      for (int px = 0; px < PX; ++px) acc[0][jy][px] = 0.0f;
    __syncthreads();
    accumulate<K, 1, PX, PY>(lds, tap, acc);

    float* dp = static_cast<float*>(it.out) + c * it.out_stride_c;
    const bool vec = (reinterpret_cast<uintptr_t>(it.out) % 16 == 0) && (it.out_stride_h % 4 == 0) &&
                     (it.out_stride_c % 4 == 0);
#pragma unroll
    for (int jy = 0; jy < PY; ++jy) {
      const int64_t oy = oy0 + ty * PY + jy;
      if (oy < it.h) store_row<PX>(dp + oy * it.out_stride_h, ox0 + tx * PX, it.w, vec, acc[0][jy]);
    }
    __syncthreads();  // the next tile overwrites the LDS tile
  }
}

template <int PX, int PY>
struct Shape {
  static constexpr int TH = kTY * PY, TW = kTX * PX;
};

// One work-group per tile (capped at 2^30, the loop takes any remainder): the
// hardware starts a new work-group as soon as one retires, so one tile's
// staging overlaps other tiles' arithmetic; measured faster than a grid that
// only fills the device once.
template <int K, int PX, int PY>
hipError_t launch(const f2d_batch_item* items, const int64_t* prefix, int32_t n, int64_t total, int64_t tag,
                  hipStream_t s) {
  constexpr int64_t kMaxGrid = int64_t{1} << 30;
  const int64_t g = total < kMaxGrid ? total : kMaxGrid;
  hipLaunchKernelGGL((k_batched_f32<K, PX, PY>), dim3(static_cast<uint32_t>(g)), dim3(kThreads), 0, s,
                     items, prefix, n, total, tag);
  return hipGetLastError();
}

template <int K>
hipError_t by_variant(int variant, const f2d_batch_item* items, const int64_t* prefix, int32_t n,
                      int64_t total, hipStream_t s) {
  const int64_t tag = plan_tag(variant, K);
  switch (variant) {
    case 2: return launch<K, 4, 2>(items, prefix, n, total, tag, s);
    case 3: return launch<K, 4, 8>(items, prefix, n, total, tag, s);
    case 4: return launch<K, 8, 2>(items, prefix, n, total, tag, s);
    default: return launch<K, 4, 4>(items, prefix, n, total, tag, s);
  }
}

TileShape batched_tile(int variant) {
  switch (variant) {
    case 2: return {Shape<4, 2>::TH, Shape<4, 2>::TW};
    case 3: return {Shape<4, 8>::TH, Shape<4, 8>::TW};
    case 4: return {Shape<8, 2>::TH, Shape<8, 2>::TW};
    default: return {Shape<4, 4>::TH, Shape<4, 4>::TW};
  }
}

bool k_supported(int32_t k) { return k == 1 || k == 3 || k == 5 || k == 7 || k == 9; }

int64_t max_width(const f2d_batch_item* items, int32_t n) {
  int64_t w = 0;
  for (int32_t i = 0; i < n; ++i) w = items[i].w > w ? items[i].w : w;
  return w;
}

}  // namespace

int64_t batched_plan(const f2d_batch_item* items, int32_t n_items, int32_t dtype, int32_t k,
                     int32_t* variant, int64_t* tile_prefix) {
  if (n_items < 0) return -fail(F2D_EINVAL, "n_items < 0");
  if (n_items > 0 && !items) return -fail(F2D_EINVAL, "items is NULL");
  if (!tile_prefix) return -fail(F2D_EINVAL, "tile_prefix is NULL");
  if (!variant) return -fail(F2D_EINVAL, "variant is NULL");
  if (k < 1 || k > 31 || k % 2 == 0) return -fail(F2D_EINVAL, "k=%d: must be odd, 1..31", k);
  if (dtype != F2D_F32) return -fail(F2D_EUNSUPPORTED, "batched: only f32 images are implemented");
  if (!k_supported(k)) return -fail(F2D_EUNSUPPORTED, "batched: k must be <= 9");
  if (*variant < 0 || *variant > variant_count(kPathBatched))
    return -fail(F2D_EINVAL, "variant %d out of range", *variant);
  for (int32_t i = 0; i < n_items; ++i) {
    const f2d_batch_item& it = items[i];
    if (it.c < 0 || it.h < 0 || it.w < 0) return -fail(F2D_EINVAL, "item %d: negative extent", i);
    if (it.in_stride_c < 0 || it.in_stride_h < 0 || it.out_stride_c < 0 || it.out_stride_h < 0)
      return -fail(F2D_EINVAL, "item %d: negative stride", i);
    if (it.c * it.h * it.w > 0) {
      if (!it.image || !it.out || !it.filter) return -fail(F2D_EINVAL, "item %d: NULL pointer", i);
      if (it.h > 1 && it.out_stride_h < it.w) return -fail(F2D_EINVAL, "item %d: out_stride_h < w", i);
      if (it.c > 1 && it.out_stride_c < (it.h - 1) * it.out_stride_h + it.w)
        return -fail(F2D_EINVAL, "item %d: output planes overlap", i);
    }
  }
  const int v = resolve_variant(kPathBatched, dtype, k, F2D_CH_SHARED, max_width(items, n_items), *variant);
  const TileShape ts = batched_tile(v);
  tile_prefix[0] = 0;
  for (int32_t i = 0; i < n_items; ++i) {
    const f2d_batch_item& it = items[i];
    const int64_t tiles = it.c * ((it.h + ts.th - 1) / ts.th) * ((it.w + ts.tw - 1) / ts.tw);
    tile_prefix[i + 1] = tile_prefix[i] + tiles;
  }
  tile_prefix[n_items + 1] = plan_tag(v, k);
  *variant = v;
  ok();
  return tile_prefix[n_items];
}

f2d_status run_batched(const f2d_batch_item* items_dev, const int64_t* tile_prefix_dev, int32_t n_items,
                       int64_t total_tiles, int32_t dtype, int32_t k, const f2d_opts* opts,
                       hipStream_t s) {
  if (!opts) return fail(F2D_EINVAL, "opts is NULL");
  if (opts->border == F2D_BORDER_ZERO)
    return fail(F2D_EUNSUPPORTED, "ragged batch: clamp-to-edge borders only");
  if (opts->border != F2D_BORDER_CLAMP) return fail(F2D_EINVAL, "unknown border %d", opts->border);
  if (opts->channels != F2D_CH_SHARED) return fail(F2D_EUNSUPPORTED, "batched: SHARED mode only");
  if (k < 1 || k > 31 || k % 2 == 0) return fail(F2D_EINVAL, "k=%d: must be odd, 1..31", k);
  if (dtype != F2D_F32) return fail(F2D_EUNSUPPORTED, "batched: only f32 images are implemented");
  if (!k_supported(k)) return fail(F2D_EUNSUPPORTED, "batched: k must be <= 9");
  if (n_items < 0 || total_tiles < 0) return fail(F2D_EINVAL, "negative n_items or total_tiles");
  if (opts->variant < 1 || opts->variant > variant_count(kPathBatched))
    return fail(F2D_EINVAL, "batched: pass the variant resolved by filter2d_batched_plan (got %d)",
                opts->variant);
  if (total_tiles == 0 || n_items == 0) return ok();
  if (!items_dev || !tile_prefix_dev) return fail(F2D_EINVAL, "items_dev or tile_prefix_dev is NULL");
  hipError_t e;
  switch (k) {
    case 1: e = by_variant<1>(opts->variant, items_dev, tile_prefix_dev, n_items, total_tiles, s); break;
    case 3: e = by_variant<3>(opts->variant, items_dev, tile_prefix_dev, n_items, total_tiles, s); break;
    case 5: e = by_variant<5>(opts->variant, items_dev, tile_prefix_dev, n_items, total_tiles, s); break;
    case 7: e = by_variant<7>(opts->variant, items_dev, tile_prefix_dev, n_items, total_tiles, s); break;
    default: e = by_variant<9>(opts->variant, items_dev, tile_prefix_dev, n_items, total_tiles, s); break;
  }
  return hip_status(e, "batched launch");
}

f2d_status autotune_batched(const f2d_batch_item* items_host, const f2d_batch_item* items_dev,
                            int32_t n_items, int32_t dtype, int32_t k, int64_t* tile_prefix_dev,
                            int32_t reps, hipStream_t s, int32_t* best) {
  if (reps < 1) return fail(F2D_EINVAL, "autotune: reps must be >= 1");
  if (!tile_prefix_dev || (n_items > 0 && !items_dev)) return fail(F2D_EINVAL, "NULL device table");
  std::vector<int64_t> prefix(static_cast<size_t>(n_items) + 2);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(F2D_EHIP, "autotune: hipEventCreate failed");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(F2D_EHIP, "autotune: hipEventCreate failed");
  }
  f2d_status st = F2D_OK;
  float best_ms = 0.0f;
  int best_v = 1;
  auto plan_and_upload = [&](int v, int64_t* total) -> f2d_status {
    int32_t var = v;
    const int64_t t = batched_plan(items_host, n_items, dtype, k, &var, prefix.data());
    if (t < 0) return static_cast<f2d_status>(-t);
    hipError_t e = hipMemcpyAsync(tile_prefix_dev, prefix.data(), prefix.size() * sizeof(int64_t),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_status(e, "autotune: prefix upload");
    *total = t;
    return F2D_OK;
  };
  for (int v = 1; v <= variant_count(kPathBatched); ++v) {
    int64_t total = 0;
    st = plan_and_upload(v, &total);
    if (st) break;
    f2d_opts o{F2D_BORDER_CLAMP, F2D_CH_SHARED, F2D_EPI_NONE, v, 0, 0};
    st = run_batched(items_dev, tile_prefix_dev, n_items, total, dtype, k, &o, s);
    if (st) break;
    (void)hipEventRecord(e0, s);
    for (int r = 0; r < reps && st == F2D_OK; ++r)
      st = run_batched(items_dev, tile_prefix_dev, n_items, total, dtype, k, &o, s);
    (void)hipEventRecord(e1, s);
    if (st) break;
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
  if (st == F2D_OK) {
    int64_t total = 0;
    st = plan_and_upload(best_v, &total);  // leave the tables planned for the winner
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st) return st;
  record_variant(kPathBatched, dtype, k, F2D_CH_SHARED, max_width(items_host, n_items), best_v);
  if (best) *best = best_v;
  return ok();
}

}  // namespace f2d
