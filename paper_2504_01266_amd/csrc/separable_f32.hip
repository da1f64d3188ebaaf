// FP32 forward for a rank-one filter F[u][v] = a[u] * b[v] (gfx950, VALU).
//
// The correlation with clamp-to-edge borders (the generalised sharpen of
// Section 4.2.4) factors into a row pass and a column pass when F is an outer
// product: Y = sum_u a[u] * H[y+u-r], H[t][x] = sum_v b[v] * X[t][cl(x+v-r)],
// with every source row clamped before the row pass.  That is 2K
// multiply-adds per output instead of K^2.
//
// One work-group (256 threads) owns a 64 x 64 output tile of one plane:
//   1. the (64+K-1) x (64+K-1) source tile, halo included, is staged in LDS
//      with the same coalesced, clamped row loads as the K x K kernels;
//   2. row pass: each thread slides a (4+K-1)-wide window over one staged
//      row at a time and writes 4 row sums to a second LDS buffer
//      ((64+K-1) rows x 64 columns, an 80-float pitch, so that the column
//      pass's 16-byte reads of rows four apart never share a bank slot);
//   3. column pass: each thread owns 4 x 4 outputs and walks its column of
//      row sums from top to bottom, every value feeding up to 4 outputs.
// Taps are uniform and live in scalar registers.  Per output the row sum is
// accumulated in the order v = 0..K-1 and the column sum in u = 0..K-1, so
// the result does not depend on the tile position.
#include "f2d_host.hpp"
#include "f2d_internal.hpp"
#include "stencil_tile.hpp"

namespace f2d {
namespace {

using namespace tile;

struct SepParams {
  const float* src;
  int64_t s_sn, s_sc, s_sh;
  float* dst;
  int64_t d_sn, d_sc, d_sh;
  const float* a;  // K column taps (row offsets u - r)
  const float* b;  // K row taps (column offsets v - r)
  int64_t H, W, row0, rows;
  int64_t C;
  int32_t tiles_x, tiles_y;
  int64_t n_blocks;  // N * C * tiles_y * tiles_x
  int32_t vec;       // every output row 16-byte aligned
};

template <int K>
__global__ __launch_bounds__(kThreads) void k_separable_f32(SepParams p) {
  using G = Geom<K, 4, 4>;
  constexpr int HPITCH = G::TW + 16;  // row-sum buffer pitch (floats)
  __shared__ float4 tile4[(G::LDS_WORDS + 3) / 4];
  __shared__ float4 hsum4[(G::LH * HPITCH) / 4];
  float* tile = reinterpret_cast<float*>(tile4);
  float* hsum = reinterpret_cast<float*>(hsum4);
  float a[K], b[K];
#pragma unroll
  for (int i = 0; i < K; ++i) {
    a[i] = p.a[i];
    b[i] = p.b[i];
  }
  const int tx = threadIdx.x % kTX, ty = threadIdx.x / kTX;
  const int64_t per_plane = static_cast<int64_t>(p.tiles_x) * p.tiles_y;
  const int64_t blk = xcd_remap(blockIdx.x, p.n_blocks);
  const int64_t plane = blk / per_plane, t = blk - plane * per_plane;
  const int64_t n = plane / p.C, c = plane - n * p.C;
  const int64_t oy0 = (t / p.tiles_x) * G::TH, ox0 = (t % p.tiles_x) * G::TW;

  stage_tile<K, 4, 4, false>(tile, p.src + n * p.s_sn + c * p.s_sc, p.s_sh, p.H, p.W, p.row0 + oy0, ox0);
  __syncthreads();

  // row pass over the LH staged rows
  for (int r = ty; r < G::LH; r += kTY) {
    float win[G::WIN4];
    const float4* row = reinterpret_cast<const float4*>(tile + r * G::PITCH + tx * 4);
#pragma unroll
    for (int q = 0; q < G::WIN4 / 4; ++q) {
      const float4 w4 = row[q];
      win[4 * q + 0] = w4.x;
      win[4 * q + 1] = w4.y;
      win[4 * q + 2] = w4.z;
      win[4 * q + 3] = w4.w;
    }
    float h[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int v = 0; v < K; ++v)
#pragma unroll
      for (int px = 0; px < 4; ++px) h[px] = __builtin_fmaf(b[v], win[px + v], h[px]);
    *reinterpret_cast<float4*>(hsum + r * HPITCH + tx * 4) = make_float4(h[0], h[1], h[2], h[3]);
  }
  __syncthreads();

  // column pass: outputs (ty*4 + jy, tx*4 + px) read row sums ty*4 + jy + u
  float acc[4][4] = {};
#pragma unroll
  for (int ry = 0; ry < 4 + K - 1; ++ry) {
    const float4 h4 = *reinterpret_cast<const float4*>(hsum + (ty * 4 + ry) * HPITCH + tx * 4);
    const float h[4] = {h4.x, h4.y, h4.z, h4.w};
#pragma unroll
    for (int jy = 0; jy < 4; ++jy) {
      const int u = ry - jy;
      if (u < 0 || u >= K) continue;
#pragma unroll
      for (int px = 0; px < 4; ++px) acc[jy][px] = __builtin_fmaf(a[u], h[px], acc[jy][px]);
    }
  }
  float* dp = p.dst + n * p.d_sn + c * p.d_sc;
#pragma unroll
  for (int jy = 0; jy < 4; ++jy) {
    const int64_t oy = oy0 + ty * 4 + jy;
    if (oy < p.rows) store_row<4>(dp + oy * p.d_sh, ox0 + tx * 4, p.W, p.vec != 0, acc[jy]);
  }
}

template <int K>
hipError_t launch(const SepParams& p, hipStream_t s) {
  hipLaunchKernelGGL(k_separable_f32<K>, dim3(static_cast<uint32_t>(p.n_blocks)), dim3(kThreads), 0, s, p);
  return hipGetLastError();
}

}  // namespace

f2d_status run_forward_separable(const Problem& pr, const float* a, const float* b, const f2d_tensor& out,
                                 hipStream_t s) {
  const f2d_tensor& im = pr.image;
  if (im.n == 0 || im.c == 0 || pr.rows == 0 || im.w == 0) return ok();
  SepParams p{};
  p.src = static_cast<const float*>(im.data);
  p.s_sn = im.stride_n;
  p.s_sc = im.stride_c;
  p.s_sh = im.stride_h;
  p.dst = static_cast<float*>(out.data);
  p.d_sn = out.stride_n;
  p.d_sc = out.stride_c;
  p.d_sh = out.stride_h;
  p.a = a;
  p.b = b;
  p.H = im.h;
  p.W = im.w;
  p.row0 = pr.row_begin;
  p.rows = pr.rows;
  p.C = im.c;
  p.tiles_x = static_cast<int32_t>((im.w + 63) / 64);
  p.tiles_y = static_cast<int32_t>((pr.rows + 63) / 64);
  p.n_blocks = im.n * im.c * static_cast<int64_t>(p.tiles_x) * p.tiles_y;
  if (p.n_blocks > kMaxBlocks)
    return fail(F2D_EUNSUPPORTED, "%lld tiles exceed one launch", static_cast<long long>(p.n_blocks));
  p.vec = row_aligned(out, 16) ? 1 : 0;
  hipError_t e;
  switch (pr.k) {
    case 1: e = launch<1>(p, s); break;
    case 3: e = launch<3>(p, s); break;
    case 5: e = launch<5>(p, s); break;
    case 7: e = launch<7>(p, s); break;
    case 9: e = launch<9>(p, s); break;
    case 11: e = launch<11>(p, s); break;
    case 13: e = launch<13>(p, s); break;
    case 15: e = launch<15>(p, s); break;
    default: return fail(F2D_EUNSUPPORTED, "separable: k=%d (1..15 are built)", pr.k);
  }
  return hip_status(e, "separable f32 launch");
}

}  // namespace f2d
