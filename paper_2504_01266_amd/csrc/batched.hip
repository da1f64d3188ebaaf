// Ragged batch: every tile of every image of a batch in ONE launch.
//
// The host plan turns the items (images of different sizes, each with its own
// K x K filter) into a prefix sum of per-item tile counts, followed by a tag
// that records the tiling variant and K it was planned for.  The kernel runs
// one work-group per tile of the global tile list (the hardware starts the
// next work-group as soon as one retires); a work-group finds the owning item
// by a 64-way search of the prefix table and runs the same tile code as the
// single-image FP32 path (SHARED mode, clamp-to-edge).  A table planned for
// another variant or K is recognised on the device from its tag and the
// launch then writes nothing.  The grid comes from the plan's tile count and
// nothing is read on the host at launch time, so the call can be captured in
// a hipGraph and replayed.
#include <hip/hip_runtime.h>

#include <cstdint>
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

// Pointers read from the descriptor table are generic; these casts tell the
// compiler which memory they name, so that image and output accesses become
// global loads and stores (a scalar row base plus a 32-bit lane offset, no
// 64-bit address per lane) and the taps, read-only for the whole launch,
// become scalar loads.
template <typename T>
__device__ __forceinline__ __attribute__((address_space(1))) T* global_ptr(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}
__device__ __forceinline__ const __attribute__((address_space(4))) float* const_ptr(const void* p) {
  return (const __attribute__((address_space(4))) float*)p;
}

// The owning item of tile t: the last i with prefix[i] <= t.  Each round
// probes 64 evenly spaced entries of the remaining range, one per lane, and
// counts with a ballot the probes at or below t (the prefix is
// non-decreasing, so they are the first lanes); the range shrinks 64-fold
// per round, so up to 64 items take one dependent load.
__device__ __forceinline__ int find_item(const int64_t* __restrict__ prefix, int32_t n_items, int64_t t) {
  const int lane = static_cast<int>(threadIdx.x % 64);
  int lo = 0, hi = n_items;  // prefix[lo] <= t < prefix[hi]
  while (hi - lo > 1) {
    const int step = (hi - lo + 63) / 64;
    const int64_t idx = lo + static_cast<int64_t>(lane + 1) * step;
    const bool le = idx < hi && prefix[idx] <= t;
    const int cnt = __popcll(__ballot(le));
    lo += cnt * step;
    hi = lo + step < hi ? lo + step : hi;
  }
  return lo;
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

  // One tile per work-group in practice (the grid covers 2^30 tiles); each
  // round of the loop maps its work-groups onto a contiguous run of tiles
  // per XCD, so neighbouring tiles share halo rows in one L2.
  const int64_t grid = gridDim.x;
  for (int64_t t0 = 0; t0 < total_tiles; t0 += grid) {
    const int64_t nb = total_tiles - t0 < grid ? total_tiles - t0 : grid;
    if (blockIdx.x >= nb) break;  // uniform
    const int64_t t = t0 + xcd_remap(blockIdx.x, nb);
    const int lo = find_item(prefix, n_items, t);
    const f2d_batch_item& it = items[lo];
    const uint32_t tiles_x = static_cast<uint32_t>((it.w + G::TW - 1) / G::TW);
    const uint32_t per_plane = tiles_x * static_cast<uint32_t>((it.h + G::TH - 1) / G::TH);
    const uint32_t local = static_cast<uint32_t>(t - prefix[lo]);  // one item has < 2^32 tiles
    const uint32_t c = local / per_plane;
    if (c >= it.c) continue;  // uniform; unreachable with a matching plan
    const uint32_t r = local - c * per_plane;
    const uint32_t tile_y = r / tiles_x;
    const uint32_t tile_x = r - tile_y * tiles_x;
    const int64_t oy0 = static_cast<int64_t>(tile_y) * G::TH, ox0 = static_cast<int64_t>(tile_x) * G::TW;

    float tap[1][K * K];
    const auto* fc = const_ptr(it.filter);
#pragma unroll
    for (int e = 0; e < K * K; ++e) tap[0][e] = fc[e];
    const auto sp = global_ptr(static_cast<const float*>(it.image)) + c * it.in_stride_c;
    stage_tile<K, PX, PY, false>(lds, sp, it.in_stride_h, it.h, it.w, oy0, ox0);
    float acc[1][PY][PX];
#pragma unroll
    for (int jy = 0; jy < PY; ++jy)
#pragma unroll
      for (int px = 0; px < PX; ++px) acc[0][jy][px] = 0.0f;
    __syncthreads();
    accumulate<K, 1, PX, PY>(lds, tap, acc);

    const auto dp = global_ptr(static_cast<float*>(it.out)) + c * it.out_stride_c;
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

// ------------------------------------------------------------ tile runs --
// Variants 5..8 (the tilings of 1..4): each work-group takes a short run of
// consecutive tiles of the global tile list (usually neighbours in one image,
// so their halos are L2 hits), finds the first tile's item once and steps to
// the next tiles without divisions.
//
// Staging moves 16-byte chunks: the LDS tile starts 4 columns left of the
// output tile (so every LDS row is 16-byte aligned and the chunk grid is the
// same for every K <= 9), a row is PITCH / 4 chunks, and the 256 threads take
// the LH * PITCH / 4 chunks of the tile in order, a few each: one 16-byte load
// and one 16-byte LDS write per chunk.  Chunks that reach past the left or
// right image edge pick their columns, clamped, from the nearest 4 inside.
template <int K, int PX, int PY>
struct PGeom {
  static constexpr int R = (K - 1) / 2;
  static_assert(R <= 4, "the chunked staging starts 4 columns left of the tile");
  static constexpr int OFF = 4 - R;  // LDS column of the first tap of output column 0
  static constexpr int TW = kTX * PX;
  static constexpr int TH = kTY * PY;
  static constexpr int LH = TH + K - 1;
  static constexpr int WIN4 = (OFF + PX + K - 1 + 3) / 4 * 4;  // floats a thread reads per row
  static constexpr int NEED = 4 + TW + R;                      // columns the taps reach
  static constexpr int PITCH = ((TW - PX + WIN4) > NEED ? (TW - PX + WIN4) : NEED) + 3 & ~3;
  static constexpr int CPR = PITCH / 4;  // chunks per row
  static constexpr int NCH = LH * CPR;   // chunks per tile
  static constexpr int CPT = (NCH + kThreads - 1) / kThreads;  // chunks per thread
  static constexpr int LDS_WORDS = LH * PITCH;
  static_assert(PX % 4 == 0, "windows are read as float4");
};

typedef float f32x4u_t __attribute__((ext_vector_type(4), aligned(4)));

// Position of a tile in the global tile list (all fields uniform).
struct Cursor {
  int32_t item;
  uint32_t c, ty, tx, tiles_x, tiles_y;
};

template <int TH, int TW>
__device__ __forceinline__ void cursor_dims(const f2d_batch_item& it, Cursor& cu) {
  cu.tiles_x = static_cast<uint32_t>((it.w + TW - 1) / TW);
  cu.tiles_y = static_cast<uint32_t>((it.h + TH - 1) / TH);
}

template <int TH, int TW>
__device__ __forceinline__ Cursor cursor_at(const f2d_batch_item* __restrict__ items,
                                            const int64_t* __restrict__ prefix, int32_t n_items,
                                            int64_t t) {
  Cursor cu;
  cu.item = find_item(prefix, n_items, t);
  cursor_dims<TH, TW>(items[cu.item], cu);
  const uint32_t local = static_cast<uint32_t>(t - prefix[cu.item]);
  const uint32_t per_plane = cu.tiles_x * cu.tiles_y;
  cu.c = local / per_plane;
  const uint32_t r = local - cu.c * per_plane;
  cu.ty = r / cu.tiles_x;
  cu.tx = r - cu.ty * cu.tiles_x;
  return cu;
}

// Advance to the next tile of the list (row-major tiles, then planes, then
// items, skipping items without tiles).  Called only while a next tile exists.
template <int TH, int TW>
__device__ __forceinline__ void cursor_step(const f2d_batch_item* __restrict__ items,
                                            const int64_t* __restrict__ prefix, int32_t n_items,
                                            Cursor& cu) {
  if (++cu.tx < cu.tiles_x) return;
  cu.tx = 0;
  if (++cu.ty < cu.tiles_y) return;
  cu.ty = 0;
  if (++cu.c < static_cast<uint32_t>(items[cu.item].c)) return;
  cu.c = 0;
  do {
    ++cu.item;
  } while (cu.item < n_items - 1 && prefix[cu.item + 1] == prefix[cu.item]);
  cursor_dims<TH, TW>(items[cu.item], cu);
}

// Load this thread's chunks of one tile into registers.  crow / ccol: the
// tile row and first LDS column of each chunk (fixed per thread).  A chunk
// whose columns reach past an image edge is loaded from the 4 columns nearest
// to it inside the image and its elements picked from those, clamped.
__device__ __forceinline__ float pick4(const f32x4_t& t, int j) {
  return j <= 0 ? t.x : (j == 1 ? t.y : (j == 2 ? t.z : t.w));
}

template <int K, int PX, int PY, int N>
__device__ __forceinline__ void load_chunks(f32x4_t (&v)[N], const int32_t (&crow)[N],
                                            const int32_t (&ccol)[N], const f2d_batch_item& it,
                                            const Cursor& cu) {
  using G = PGeom<K, PX, PY>;
  static_assert(N == G::CPT, "one register chunk per staged chunk");
  // extents below 2^31 (checked by the plan): 32-bit clamps
  const int32_t H = static_cast<int32_t>(it.h), W = static_cast<int32_t>(it.w);
  const int64_t sh = it.in_stride_h;
  const int32_t row0 = static_cast<int32_t>(cu.ty) * G::TH - G::R;
  const int32_t col0 = static_cast<int32_t>(cu.tx) * G::TW - 4;
  const auto sp = global_ptr(static_cast<const float*>(it.image)) + cu.c * it.in_stride_c;
  const bool inside = col0 >= 0 && col0 + G::PITCH <= W;  // uniform
  using V = const __attribute__((address_space(1))) f32x4u_t;
#pragma unroll
  for (int i = 0; i < G::CPT; ++i) {
    if (crow[i] >= G::LH) continue;  // past the tile (last chunks only)
    int32_t gy = row0 + crow[i];
    gy = gy < 0 ? 0 : (gy >= H ? H - 1 : gy);
    const auto rp = sp + static_cast<int64_t>(gy) * sh;
    const int32_t gx = col0 + ccol[i];
    if (inside) {
      const f32x4u_t t = *reinterpret_cast<V*>(rp + gx);
      v[i] = f32x4_t{t.x, t.y, t.z, t.w};
    } else if (W >= 4) {
      const int32_t xs = gx < 0 ? 0 : (gx > W - 4 ? W - 4 : gx);
      const f32x4u_t u = *reinterpret_cast<V*>(rp + xs);
      const f32x4_t t{u.x, u.y, u.z, u.w};
      const int d = gx - xs;  // element q is column clamp(gx + q) = xs + clamp(d + q, 0, 3)
      v[i] = f32x4_t{pick4(t, d), pick4(t, d + 1), pick4(t, d + 2), pick4(t, d + 3)};
    } else {
      float e[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) e[q] = rp[gx + q < 0 ? 0 : (gx + q >= W ? W - 1 : gx + q)];
      v[i] = f32x4_t{e[0], e[1], e[2], e[3]};
    }
  }
}

template <int K, int PX, int PY, int N>
__device__ __forceinline__ void write_chunks(float* __restrict__ lds, const f32x4_t (&v)[N],
                                             const int32_t (&crow)[N], const int32_t (&ccol)[N]) {
  using G = PGeom<K, PX, PY>;
#pragma unroll
  for (int i = 0; i < G::CPT; ++i)
    if (crow[i] < G::LH) *reinterpret_cast<f32x4_t*>(lds + crow[i] * G::PITCH + ccol[i]) = v[i];
}

// acc[jy][px] += sum_{u,v} tap[u][v] * tile[ty*PY+jy+u][tx*PX+px+v], the LDS
// tile starting OFF columns left of the first tap (same order as accumulate()).
// Each row is read one row ahead of its arithmetic (left alone, the compiler
// issues every read of the tile up front and needs three times the registers).
template <int K, int PX, int PY>
__device__ __forceinline__ void accumulate_off(const float* __restrict__ lds, const float (&tap)[K * K],
                                               float (&acc)[PY][PX]) {
  using G = PGeom<K, PX, PY>;
  constexpr int NQ = G::WIN4 / 4;
  constexpr int RQ = G::PITCH / 4;  // row pitch in 16-byte words
  const int tx = threadIdx.x % kTX;
  const int ty = threadIdx.x / kTX;
  const f32x4_t* base = reinterpret_cast<const f32x4_t*>(lds + ty * PY * G::PITCH + tx * PX);
  f32x4_t cur[NQ], nxt[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) cur[q] = base[q];
#pragma unroll
  for (int ry = 0; ry < PY + K - 1; ++ry) {
    if (ry + 1 < PY + K - 1) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) nxt[q] = base[(ry + 1) * RQ + q];
    }
    float win[G::WIN4];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      win[4 * q + 0] = cur[q].x;
      win[4 * q + 1] = cur[q].y;
      win[4 * q + 2] = cur[q].z;
      win[4 * q + 3] = cur[q].w;
    }
#pragma unroll
    for (int jy = 0; jy < PY; ++jy) {
      const int u = ry - jy;
      if (u < 0 || u >= K) continue;
#pragma unroll
      for (int v = 0; v < K; ++v)
#pragma unroll
        for (int px = 0; px < PX; ++px)
          acc[jy][px] = __builtin_fmaf(tap[u * K + v], win[px + v + G::OFF], acc[jy][px]);
    }
    // the empty statements order this row's arithmetic before the next
    // row's reads (the arithmetic is otherwise free to sink below them all)
#pragma unroll
    for (int jy = 0; jy < PY; ++jy)
#pragma unroll
      for (int px = 0; px < PX; ++px) asm volatile("" : "+v"(acc[jy][px]));
#pragma unroll
    for (int q = 0; q < NQ; ++q) cur[q] = nxt[q];
  }
}

template <int K, int PX, int PY>
__global__ __launch_bounds__(kThreads) void k_batched_pipe(const f2d_batch_item* __restrict__ items,
                                                           const int64_t* __restrict__ prefix,
                                                           int32_t n_items, int64_t total_tiles,
                                                           int64_t tag, int32_t per_group) {
  using G = PGeom<K, PX, PY>;
  if (prefix[n_items + 1] != tag) return;  // uniform, see k_batched_f32
  __shared__ f32x4_t lds4[G::LDS_WORDS / 4];
  float* lds = reinterpret_cast<float*>(lds4);
  const int tx = threadIdx.x % kTX;
  const int ty = threadIdx.x / kTX;

  // a run of per_group consecutive tiles; neighbouring runs on one XCD
  const int64_t w = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t t0 = w * per_group;
  const int64_t t1 = t0 + per_group < total_tiles ? t0 + per_group : total_tiles;
  if (t0 >= t1) return;  // uniform

  int32_t crow[G::CPT], ccol[G::CPT];
#pragma unroll
  for (int i = 0; i < G::CPT; ++i) {
    const int q = static_cast<int>(threadIdx.x) + kThreads * i;
    crow[i] = q / G::CPR;  // >= LH: no chunk
    ccol[i] = (q - (q / G::CPR) * G::CPR) * 4;
  }

  Cursor cc = cursor_at<G::TH, G::TW>(items, prefix, n_items, t0);
  if (cc.c >= items[cc.item].c) return;  // uniform; unreachable with a matching plan
  int32_t tap_item = -1;
  float tap[K * K];
  for (int64_t t = t0; t < t1; ++t) {
    const f2d_batch_item& it = items[cc.item];
    {
      f32x4_t v[G::CPT];
      load_chunks<K, PX, PY>(v, crow, ccol, it, cc);
      write_chunks<K, PX, PY>(lds, v, crow, ccol);
    }
    if (cc.item != tap_item) {
      tap_item = cc.item;
      const auto* fc = const_ptr(it.filter);
#pragma unroll
      for (int e = 0; e < K * K; ++e) {
        tap[e] = fc[e];
        // 81 taps do not fit the scalar registers next to the cursors: hold
        // them in vector registers (the same value in every lane)
        if constexpr (K * K > 64) asm volatile("" : "+v"(tap[e]));
      }
    }
    float acc[PY][PX];
#pragma unroll
    for (int jy = 0; jy < PY; ++jy)
#pragma unroll
      for (int px = 0; px < PX; ++px) acc[jy][px] = 0.0f;
    __syncthreads();
    accumulate_off<K, PX, PY>(lds, tap, acc);
    const auto dp = global_ptr(static_cast<float*>(it.out)) + cc.c * it.out_stride_c;
    const bool vec = (reinterpret_cast<uintptr_t>(it.out) % 16 == 0) && (it.out_stride_h % 4 == 0) &&
                     (it.out_stride_c % 4 == 0);
    const int64_t oy0 = static_cast<int64_t>(cc.ty) * G::TH, ox0 = static_cast<int64_t>(cc.tx) * G::TW;
#pragma unroll
    for (int jy = 0; jy < PY; ++jy) {
      const int64_t oy = oy0 + ty * PY + jy;
      if (oy < it.h) store_row<PX>(dp + oy * it.out_stride_h, ox0 + tx * PX, it.w, vec, acc[jy]);
    }
    if (t + 1 < t1) {
      cursor_step<G::TH, G::TW>(items, prefix, n_items, cc);
      __syncthreads();  // the next tile overwrites the LDS tile
    }
  }
}

template <int PX, int PY>
struct Shape {
  static constexpr int TH = kTY * PY, TW = kTX * PX;
};

// One work-group per tile (capped at 2^30, the loop takes any remainder): the
// hardware starts a new work-group as soon as one retires, so one tile's
// staging overlaps other tiles' arithmetic.
template <int K, int PX, int PY>
hipError_t launch(const f2d_batch_item* items, const int64_t* prefix, int32_t n, int64_t total, int64_t tag,
                  hipStream_t s) {
  constexpr int64_t kMaxGrid = int64_t{1} << 30;
  const int64_t g = total < kMaxGrid ? total : kMaxGrid;
  hipLaunchKernelGGL((k_batched_f32<K, PX, PY>), dim3(static_cast<uint32_t>(g)), dim3(kThreads), 0, s,
                     items, prefix, n, total, tag);
  return hipGetLastError();
}

// Runs of a few tiles per work-group: the search for the first tile's item
// and the tile decode are paid once per run, and the hardware still hands
// runs to work-groups as they retire (no tail of idle CUs behind a static
// split).
constexpr int32_t kTilesPerGroup = 4;

template <int K, int PX, int PY>
hipError_t launch_pipe(const f2d_batch_item* items, const int64_t* prefix, int32_t n, int64_t total,
                       int64_t tag, hipStream_t s) {
  const int64_t g = (total + kTilesPerGroup - 1) / kTilesPerGroup;
  if (g > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_batched_pipe<K, PX, PY>), dim3(static_cast<uint32_t>(g)), dim3(kThreads), 0, s,
                     items, prefix, n, total, tag, kTilesPerGroup);
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
    case 5: return launch_pipe<K, 4, 4>(items, prefix, n, total, tag, s);
    case 6: return launch_pipe<K, 4, 2>(items, prefix, n, total, tag, s);
    case 7: return launch_pipe<K, 4, 8>(items, prefix, n, total, tag, s);
    case 8: return launch_pipe<K, 8, 2>(items, prefix, n, total, tag, s);
    default: return launch<K, 4, 4>(items, prefix, n, total, tag, s);
  }
}

TileShape batched_tile(int variant) {
  switch (variant > 4 ? variant - 4 : variant) {
    case 2: return {Shape<4, 2>::TH, Shape<4, 2>::TW};
    case 3: return {Shape<4, 8>::TH, Shape<4, 8>::TW};
    case 4: return {Shape<8, 2>::TH, Shape<8, 2>::TW};
    default: return {Shape<4, 4>::TH, Shape<4, 4>::TW};
  }
}

}  // namespace

int batched_variant_count() { return 8; }

namespace {

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
  if (*variant < 0 || *variant > batched_variant_count())
    return -fail(F2D_EINVAL, "variant %d out of range", *variant);
  for (int32_t i = 0; i < n_items; ++i) {
    const f2d_batch_item& it = items[i];
    if (it.c < 0 || it.h < 0 || it.w < 0) return -fail(F2D_EINVAL, "item %d: negative extent", i);
    if (it.in_stride_c < 0 || it.in_stride_h < 0 || it.out_stride_c < 0 || it.out_stride_h < 0)
      return -fail(F2D_EINVAL, "item %d: negative stride", i);
    if (it.h > INT32_MAX || it.w > INT32_MAX)
      return -fail(F2D_EUNSUPPORTED, "item %d: h and w must be below 2^31", i);
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
  if (opts->variant < 1 || opts->variant > batched_variant_count())
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
  for (int v = 1; v <= batched_variant_count(); ++v) {
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
