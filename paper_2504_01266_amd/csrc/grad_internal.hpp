// Parameter blocks and launchers of the adjoint (backward) kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "f2d_internal.hpp"

namespace f2d {

// Edge pixels of grad_input, recomputed exactly from the clamp preimages.
// Plane addressing as in StencilParams: group g of image n sums sources s,
// source plane = src[s*st_s] + n*src_sn + (g*sc_g + s*sc_s)*src_sc, filter
// (NOT flipped) = filt + (f0 + g*fg + s*fs)*K*K, output plane
// out + n*out_sn + g*out_sc (f32).
struct EdgeParams {
  const void* src[kMaxT];
  int64_t src_sn[kMaxT], src_sc[kMaxT], src_sh[kMaxT];
  float* out;
  int64_t out_sn, out_sc, out_sh;
  const void* filt;
  int64_t H, W;
  int64_t planes;  // N * groups
  int32_t groups, nsrc, st_s, sc_g, sc_s, f0, fg, fs, k;
};

// grad_filter partial sums.  Work unit = ((rep * nf + f) * chunks + chunk):
// filter f (nf of them), replica rep (the (n, c) pairs of SHARED mode, else
// the image n), chunk = a run of tiles_per_unit tiles of the plane.
struct GradFilterParams {
  const void* x;
  int64_t x_sn, x_sc, x_sh;
  const void* g[kMaxT];
  int64_t g_sn[kMaxT], g_sc[kMaxT], g_sh[kMaxT];
  float* partial;  // [n_units][K*K]
  int64_t H, W;
  int64_t nf, nrep, chunks, n_units;
  int32_t mode, m, C;  // C = image channels (input channels of a bank)
  int32_t tiles_x, tiles_y, tiles_per_unit;
  int32_t flags;  // kDstVec: G-bar rows 16-byte aligned
};

// The r-wide frame of the image adjoint, folded onto the edge pixels of out.
struct FoldParams {
  const float* frame;
  int64_t frame_plane;
  float* out;
  int64_t out_sn, out_sc, out_sh;
  int64_t H, W, r;
  int64_t planes, groups;
};
hipError_t launch_fold_frame(const FoldParams& p, hipStream_t s);

// element types of the rectangle-sum edge kernel (runtime-K f32 path)
constexpr int kEdgeF32 = 0;
hipError_t launch_grad_input_edges(const EdgeParams& p, int kind, hipStream_t s);
hipError_t launch_grad_filter_f32(const GradFilterParams& p, int K, hipStream_t s);
hipError_t launch_grad_filter_generic(const GradFilterParams& p, int K, hipStream_t s);
bool grad_filter_bank_groups(int mode, int K, int64_t co, int64_t ci, int* no, int* ni);
hipError_t launch_grad_filter_bank_f32(const GradFilterParams& p, int K, hipStream_t s);
// Sums the partials over items (rep, chunk) in a fixed order; overwrites
// some partial slots with intermediate sums.
hipError_t launch_reduce_partials(float* partial, float* out, int64_t nf, int kk, int64_t nrep,
                                  int64_t chunks, hipStream_t s);
TileShape grad_filter_tile();

}  // namespace f2d
