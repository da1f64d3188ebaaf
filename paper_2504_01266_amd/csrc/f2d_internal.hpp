// Internal declarations shared by the library's kernels and its C-ABI layer.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "filter2d.h"

namespace f2d {

constexpr int kMaxT = 4;  // tensors one stencil launch can read from / write to

// Plane addressing for the VALU stencil kernels.  The grid enumerates
// (n, g, tile) with g < groups; each work-group produces NOUT output planes
// j = 0..NOUT-1 of group g by summing nsrc source planes s:
//   source plane  = src[s*st_s] + n*src_sn + (g*sc_g + s*sc_s)*src_sc
//   filter        = filt + (f0 + g*fg + j*fj + s*fs) * K*K
//   output plane  = dst[j*dt_j] + n*dst_sn + (g*dc_g + j*dc_j)*dst_sc
// This covers SHARED / DEPTHWISE / BANK forward and the image adjoints.
struct StencilParams {
  const void* src[kMaxT];
  int64_t src_sn[kMaxT], src_sc[kMaxT], src_sh[kMaxT];
  void* dst[kMaxT];
  int64_t dst_sn[kMaxT], dst_sc[kMaxT], dst_sh[kMaxT];
  const void* filt;
  int64_t H, W;        // source plane extent (clamp bounds)
  int64_t row0, rows;  // output rows [row0, row0 + rows) of the source frame
  int32_t groups, nsrc;
  int32_t st_s, sc_g, sc_s;
  int32_t dt_j, dc_g, dc_j;
  int32_t f0, fg, fj, fs;
  int32_t tiles_x, tiles_y;
  int64_t n_blocks;  // N * groups * tiles_y * tiles_x
  int32_t k;         // runtime K (generic kernel)
  int32_t flags;     // kFlip | kZeroBorder | kSumSq (generic / u8 kernels)
  // image adjoint only: output columns start at col0 (= -r) and rows at row0
  // (= -r), covering the image plus an r-wide frame; values that fall on the
  // frame go to `frame` (frame_plane floats per output plane, frame_index()).
  int64_t col0;
  float* frame;
  int64_t frame_plane;
  int32_t fr;
};

// Layout of the r-wide frame around an H x W plane: the r rows above and the
// r rows below (each W + 2r wide, corners included), then the left and the
// right r columns of the H image rows.
__host__ __device__ inline int64_t frame_plane_size(int64_t H, int64_t W, int64_t r) {
  return 2 * r * (W + 2 * r) + 2 * r * H;
}
__host__ __device__ inline int64_t frame_index(int64_t iy, int64_t ix, int64_t H, int64_t W, int64_t r) {
  const int64_t we = W + 2 * r;
  if (iy < 0) return (iy + r) * we + (ix + r);
  if (iy >= H) return (r + iy - H) * we + (ix + r);
  if (ix < 0) return 2 * r * we + iy * r + (ix + r);
  return 2 * r * we + H * r + iy * r + (ix - W);
}

constexpr int32_t kFlip = 1;       // use F[K-1-u][K-1-v] (image adjoint)
constexpr int32_t kZeroBorder = 2; // out-of-range source pixels read as 0
constexpr int32_t kSumSq = 4;      // u8 path: extra output o0^2 + o1^2
constexpr int32_t kDstVec = 8;     // every output row is 16-byte aligned (vector stores)
constexpr int32_t kSrcVec = 16;    // every source row is 4-byte aligned (u8 word loads)

// Every launcher returns hipSuccess or the launch error.
hipError_t launch_stencil_f32(const StencilParams& p, int K, int nout, bool adjoint, int variant,
                              hipStream_t stream);
hipError_t launch_stencil_u8(const StencilParams& p, int K, int m, bool sumsq, bool vec,
                             int variant, hipStream_t stream);

// Tile geometry of a variant, used by the host for grid sizing.
struct TileShape {
  int th, tw;
};
TileShape f32_tile(int variant);
TileShape u8_tile(int variant);
int f32_variant_count();
int batched_variant_count();  // ragged batch: 1..4 one tile per work-group, 5..8 pipelined
int u8_variant_count();

// XCD-aware work-group ordering: the hardware hands work-groups to the 8 XCDs
// round-robin; this maps the b-th dispatched group to a logical tile so that
// each XCD processes one contiguous run of tiles (neighbouring tiles share
// halo rows in that XCD's L2).
__device__ inline int64_t xcd_remap(int64_t b, int64_t nb) {
  constexpr int64_t kXcd = 8;
  int64_t q = nb / kXcd, rem = nb % kXcd;
  int64_t x = b % kXcd, k = b / kXcd;
  return x * q + (x < rem ? x : rem) + k;
}

}  // namespace f2d
