// FP32 K x K stencil kernels (VALU) for gfx950.
//
// One work-group (256 threads = 4 wave64) produces a TH x TW tile of NOUT
// output planes.  For each source plane it stages the (TH+K-1) x (TW+K-1)
// input tile, halo included, in LDS with coalesced row loads, the border rule
// applied by index arithmetic only (clamp-to-edge for the forward map, zero
// for the image adjoint).  Each thread then owns a PY x PX block of outputs in
// registers and slides down its (PX+K-1)-wide LDS window row by row, so every
// LDS word it reads feeds up to PY*K FMAs.  Filter taps are uniform across the
// work-group and live in scalar registers.
//
// Per output value the taps are accumulated in the order (source s, row u,
// column v), independent of the tiling variant, so all variants give bitwise
// identical results.
#include "f2d_internal.hpp"
#include "stencil_tile.hpp"

namespace f2d {
namespace {

using namespace tile;

// Output plane j (compile-time) of group g: outs[j] when the outputs are
// separate tensors (dt_j = 1), else channel g*dc_g + j*dc_j of outs[0].
template <int J>
__device__ __forceinline__ float* dst_fixed(const StencilParams& p, int64_t n, int64_t ch,
                                            int64_t& sh) {
  const bool sep = J > 0 && p.dt_j != 0;
  void* base = sep ? p.dst[J] : p.dst[0];
  const int64_t sn = sep ? p.dst_sn[J] : p.dst_sn[0];
  const int64_t sc = sep ? p.dst_sc[J] : p.dst_sc[0];
  sh = sep ? p.dst_sh[J] : p.dst_sh[0];
  return static_cast<float*>(base) + n * sn + ch * sc;
}

template <int NOUT, int PX, int PY, int J = 0>
__device__ __forceinline__ void store_outputs(const StencilParams& p, int64_t n, int64_t g,
                                              int64_t oy0, int64_t ox0,
                                              const float (&acc)[NOUT][PY][PX]) {
  if constexpr (J < NOUT) {
    const bool vec = (p.flags & kDstVec) != 0;
    const int tx = threadIdx.x % kTX;
    const int ty = threadIdx.x / kTX;
    int64_t dsh;
    float* dp = dst_fixed<J>(p, n, g * p.dc_g + J * p.dc_j, dsh);
#pragma unroll
    for (int jy = 0; jy < PY; ++jy) {
      const int64_t oy = oy0 + ty * PY + jy;
      if (oy < p.rows) store_row<PX>(dp + oy * dsh, ox0 + tx * PX, p.W, vec, acc[J][jy]);
    }
    store_outputs<NOUT, PX, PY, J + 1>(p, n, g, oy0, ox0, acc);
  }
}

// Image adjoint store: image coordinates (iy, ix) = (row0 + oy, ox); pixels
// inside the image go to the output plane, pixels on the r-wide frame to the
// frame buffer (folded onto the edge pixels afterwards).
// Output j of a group is channel g*dc_g + j*dc_j of groups*dc_g per image.
template <int PX, int PY>
__device__ __forceinline__ void store_adjoint(const StencilParams& p, int64_t n, int64_t g, int j, int64_t oy0,
                                              int64_t ox0, const float (&acc)[PY][PX]) {
  const bool vec = (p.flags & kDstVec) != 0;
  const int tx = threadIdx.x % kTX;
  const int ty = threadIdx.x / kTX;
  int64_t dsh;
  const int64_t ch = g * p.dc_g + j * p.dc_j;
  float* dp = dst_fixed<0>(p, n, ch, dsh);
  float* fp = p.frame + (n * p.groups * p.dc_g + ch) * p.frame_plane;
  const int64_t r = p.fr;
#pragma unroll
  for (int jy = 0; jy < PY; ++jy) {
    const int64_t oy = oy0 + ty * PY + jy;
    if (oy >= p.rows) continue;
    const int64_t iy = p.row0 + oy;
    const int64_t ix0 = ox0 + tx * PX;
    if (iy >= 0 && iy < p.H && ix0 >= 0 && ix0 + PX <= p.W) {
      store_row<PX>(dp + iy * dsh, ix0, p.W, vec, acc[jy]);
    } else {
#pragma unroll
      for (int px = 0; px < PX; ++px) {
        const int64_t ix = ix0 + px;
        if (ix >= p.W + r) continue;
        if (iy >= 0 && iy < p.H && ix >= 0 && ix < p.W)
          dp[iy * dsh + ix] = acc[jy][px];
        else
          fp[frame_index(iy, ix, p.H, p.W, r)] = acc[jy][px];
      }
    }
  }
}

// MT: sources come from several tensors (the depthwise adjoint reads the m
// upstream gradients); otherwise every source plane is in src[0].
// ZB: forward map with zero borders (out-of-image neighbours read as 0).
template <int K, int NOUT, bool ADJ, bool MT, int PX, int PY, bool ZB = false>
__global__ __launch_bounds__(kThreads) void k_stencil_f32(StencilParams p) {
  using G = Geom<K, PX, PY>;
  __shared__ float4 lds4[(G::LDS_WORDS + 3) / 4];
  float* lds = reinterpret_cast<float*>(lds4);

  const int64_t b = xcd_remap(blockIdx.x, p.n_blocks);
  const int64_t tiles = static_cast<int64_t>(p.tiles_x) * p.tiles_y;
  const int64_t plane = b / tiles;
  const int64_t t = b - plane * tiles;
  const int64_t tile_y = t / p.tiles_x;
  const int64_t tile_x = t - tile_y * p.tiles_x;
  const int64_t n = plane / p.groups;
  const int64_t g = plane - n * p.groups;
  const int64_t oy0 = tile_y * G::TH;  // first output row of the tile (band-relative)
  const int64_t ox0 = (ADJ ? p.col0 : 0) + tile_x * G::TW;

  float acc[NOUT][PY][PX];
#pragma unroll
  for (int j = 0; j < NOUT; ++j)
#pragma unroll
    for (int jy = 0; jy < PY; ++jy)
#pragma unroll
      for (int px = 0; px < PX; ++px) acc[j][jy][px] = 0.0f;

  const float* filt = static_cast<const float*>(p.filt);
  for (int s = 0; s < p.nsrc; ++s) {
    int64_t sh;
    const int64_t ch = g * p.sc_g + s * p.sc_s;
    const float* sp;
    if constexpr (MT) {
      sp = src_plane(p, s * p.st_s, n, ch, sh);
    } else {
      sp = static_cast<const float*>(p.src[0]) + n * p.src_sn[0] + ch * p.src_sc[0];
      sh = p.src_sh[0];
    }
    stage_tile<K, PX, PY, ADJ || ZB, NOUT == 1>(lds, sp, sh, p.H, p.W, p.row0 + oy0, ox0);

    // Taps live in scalar registers; more than 64 of them (four outputs at
    // K = 5) no longer fit beside the kernel's other scalars, and spilling
    // them to vector-register lanes costs a lane write and read per tap per
    // tile, so the forward accumulates those outputs in two passes over the
    // window, half the outputs each (the same per-output order, so the same
    // bits; 5x5 bank forward 27.7 -> 26.5 ms).  The adjoint keeps one pass:
    // split, it needs more vector registers (one wave per SIMD fewer) and
    // measured slower (5x5 bank backward 61.9 -> 65.4 ms).
    constexpr int NH = !ADJ && NOUT * K * K > 64 && NOUT % 2 == 0 ? NOUT / 2 : NOUT;
    __syncthreads();
#pragma unroll
    for (int h = 0; h < NOUT / NH; ++h) {
      float tap[NH][K * K];
#pragma unroll
      for (int jj = 0; jj < NH; ++jj) {
        const int j = h * NH + jj;
        const float* fp = filt + static_cast<int64_t>(p.f0 + g * p.fg + j * p.fj + s * p.fs) * (K * K);
#pragma unroll
        for (int e = 0; e < K * K; ++e) tap[jj][e] = fp[ADJ ? (K * K - 1 - e) : e];
      }
      accumulate<K, NH, PX, PY>(lds, tap, *reinterpret_cast<float(*)[NH][PY][PX]>(&acc[h * NH]));
    }
    __syncthreads();
  }

  if constexpr (ADJ) {
#pragma unroll
    for (int j = 0; j < NOUT; ++j) store_adjoint<PX, PY>(p, n, g, j, oy0, ox0, acc[j]);
  } else
    store_outputs<NOUT, PX, PY>(p, n, g, oy0, ox0, acc);
}

// Runtime-K fallback (any odd K <= 31, NOUT = 1): one output per thread on a
// 16 x 16 tile, taps read through the scalar cache.  Same accumulation order.
constexpr int kGenT = 16;
constexpr int kGenMaxK = 31;

__global__ __launch_bounds__(kThreads) void k_stencil_f32_generic(StencilParams p) {
  __shared__ float lds[(kGenT + kGenMaxK - 1) * (kGenT + kGenMaxK - 1)];
  const int K = p.k, R = (K - 1) / 2, L = kGenT + K - 1;
  const bool adj = (p.flags & kFlip) != 0;
  const int64_t b = xcd_remap(blockIdx.x, p.n_blocks);
  const int64_t tiles = static_cast<int64_t>(p.tiles_x) * p.tiles_y;
  const int64_t plane = b / tiles;
  const int64_t t = b - plane * tiles;
  const int64_t tile_y = t / p.tiles_x;
  const int64_t tile_x = t - tile_y * p.tiles_x;
  const int64_t n = plane / p.groups;
  const int64_t g = plane - n * p.groups;
  const int64_t oy0 = tile_y * kGenT, ox0 = tile_x * kGenT;
  const int tx = threadIdx.x % kGenT, ty = threadIdx.x / kGenT;
  const float* filt = static_cast<const float*>(p.filt);

  float acc = 0.0f;
  for (int s = 0; s < p.nsrc; ++s) {
    int64_t sh;
    const float* sp = src_plane(p, s * p.st_s, n, g * p.sc_g + s * p.sc_s, sh);
    for (int idx = threadIdx.x; idx < L * L; idx += kThreads) {
      const int ly = idx / L, lx = idx - (idx / L) * L;
      int64_t gy = p.row0 + oy0 - R + ly, gx = ox0 - R + lx;
      float v;
      if (p.flags & kZeroBorder) {
        v = (gy >= 0 && gy < p.H && gx >= 0 && gx < p.W) ? sp[gy * sh + gx] : 0.0f;
      } else {
        gy = gy < 0 ? 0 : (gy >= p.H ? p.H - 1 : gy);
        gx = gx < 0 ? 0 : (gx >= p.W ? p.W - 1 : gx);
        v = sp[gy * sh + gx];
      }
      lds[ly * L + lx] = v;
    }
    __syncthreads();
    const float* fp = filt + static_cast<int64_t>(p.f0 + g * p.fg + s * p.fs) * (K * K);
    for (int u = 0; u < K; ++u)
      for (int v = 0; v < K; ++v) {
        const int e = adj ? (K * K - 1 - (u * K + v)) : (u * K + v);
        acc = __builtin_fmaf(fp[e], lds[(ty + u) * L + tx + v], acc);
      }
    __syncthreads();
  }
  const int64_t oy = oy0 + ty, ox = ox0 + tx;
  if (oy < p.rows && ox < p.W) {
    int64_t dsh;
    float* dp = dst_plane(p, 0, n, g * p.dc_g, dsh);
    dp[oy * dsh + ox] = acc;
  }
}

// ------------------------------------------------------------- dispatch --

template <int K, int NOUT, bool ADJ, int PX, int PY, bool MT = false>
hipError_t go(const StencilParams& p, hipStream_t stream) {
  hipLaunchKernelGGL((k_stencil_f32<K, NOUT, ADJ, MT, PX, PY>), dim3(static_cast<uint32_t>(p.n_blocks)),
                     dim3(kThreads), 0, stream, p);
  return hipGetLastError();
}

// zero-border forward: one output plane per tile, 64 x 64 tiles
template <int K>
hipError_t go_zero(const StencilParams& p, hipStream_t stream) {
  hipLaunchKernelGGL((k_stencil_f32<K, 1, false, false, 4, 4, true>), dim3(static_cast<uint32_t>(p.n_blocks)),
                     dim3(kThreads), 0, stream, p);
  return hipGetLastError();
}

template <int K, int NOUT, bool ADJ>
hipError_t by_variant(const StencilParams& p, int variant, hipStream_t stream) {
  if constexpr (NOUT == 1 && !ADJ) {
    switch (variant) {
      case 2: return go<K, NOUT, ADJ, 4, 2>(p, stream);
      case 3: return go<K, NOUT, ADJ, 4, 8>(p, stream);
      case 4: return go<K, NOUT, ADJ, 8, 2>(p, stream);
      default: return go<K, NOUT, ADJ, 4, 4>(p, stream);
    }
  } else {
    (void)variant;
    return go<K, NOUT, ADJ, 4, 4>(p, stream);
  }
}

template <int K>
hipError_t by_nout(const StencilParams& p, int nout, bool adj, int variant, hipStream_t stream) {
  if (adj) {
    if (p.st_s != 0) return go<K, 1, true, 4, 4, true>(p, stream);
    if (nout == 4) {  // bank adjoint: four image channels per work-group
      if constexpr (4 * K * K <= kMaxTaps) return by_variant<K, 4, true>(p, 1, stream);
      return hipErrorInvalidValue;
    }
    return by_variant<K, 1, true>(p, 1, stream);
  }
  switch (nout) {
    case 2:
      if constexpr (2 * K * K <= kMaxTaps) return by_variant<K, 2, false>(p, variant, stream);
      return hipErrorInvalidValue;
    case 4:
      if constexpr (4 * K * K <= kMaxTaps) return by_variant<K, 4, false>(p, variant, stream);
      return hipErrorInvalidValue;
    default: return by_variant<K, 1, false>(p, variant, stream);
  }
}

}  // namespace

TileShape f32_tile(int variant) {
  switch (variant) {
    case 2: return {kTY * 2, kTX * 4};
    case 3: return {kTY * 8, kTX * 4};
    case 4: return {kTY * 2, kTX * 8};
    case -1: return {kGenT, kGenT};  // generic kernel
    default: return {kTY * 4, kTX * 4};
  }
}

int f32_variant_count() { return 4; }

// Templated kernels exist for K <= 9 with NOUT*K*K <= 100 (taps in SGPRs);
// everything else runs the generic kernel (the caller sizes the grid with
// f32_tile(-1) in that case and passes nout = 1).
hipError_t launch_stencil_f32(const StencilParams& p, int K, int nout, bool adjoint, int variant,
                              hipStream_t stream) {
  if (p.n_blocks <= 0) return hipSuccess;
  if (variant < 0) {
    hipLaunchKernelGGL(k_stencil_f32_generic, dim3(static_cast<uint32_t>(p.n_blocks)),
                       dim3(kThreads), 0, stream, p);
    return hipGetLastError();
  }
  if (p.flags & kZeroBorder) {  // forward with zero borders (variant 1 tiling)
    if (nout != 1 || adjoint) return hipErrorInvalidValue;
    switch (K) {
      case 1: return go_zero<1>(p, stream);
      case 3: return go_zero<3>(p, stream);
      case 5: return go_zero<5>(p, stream);
      case 7: return go_zero<7>(p, stream);
      case 9: return go_zero<9>(p, stream);
      default: return hipErrorInvalidValue;
    }
  }
  switch (K) {
    case 1: return by_nout<1>(p, nout, adjoint, variant, stream);
    case 3: return by_nout<3>(p, nout, adjoint, variant, stream);
    case 5: return by_nout<5>(p, nout, adjoint, variant, stream);
    case 7: return by_nout<7>(p, nout, adjoint, variant, stream);
    case 9: return by_nout<9>(p, nout, adjoint, variant, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace f2d
