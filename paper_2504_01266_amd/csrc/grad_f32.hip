// FP32 adjoint kernels: the clamp-border fold of grad_input and grad_filter.
//
// grad_input.  The forward map reads X at clamped indices, so its adjoint is
// "correlate the zero-padded upstream gradient with the flipped filter, then
// fold the gradient that fell outside the image back onto the edge pixels":
// X-bar[p][q] = sum of Z[a][b] over every (a, b) with cl(a) = p, cl(b) = q,
// where Z is that correlation evaluated on the image and an r-wide frame
// around it.  The VALU stencil kernel (adjoint mode) evaluates Z, writing the
// image part to X-bar and the frame part to a frame buffer; k_fold_frame adds
// each edge pixel's frame values.  The runtime-K path (K > 9) instead
// recomputes each edge pixel from the definition in k_grad_input_edges: for
// every tap (u, v) the outputs whose clamped source is (p, q) form the
// rectangle {y : cl(y+u-r) = p} x {x : cl(x+v-r) = q}.
//
// grad_filter.  F-bar[u][v] sums G-bar[y][x] * X[cl(y+u-r)][cl(x+v-r)] over
// every pixel of every plane pair that the filter touches.  A work-group
// takes a run of 64 x 64 tiles of one (X plane, G-bar plane) pair, stages the
// X tile with its clamped halo in LDS, keeps its 4 x 4 block of G-bar in
// registers and accumulates all K*K tap sums per thread; a fixed butterfly
// across each wave and a fixed-order sum across the 4 waves leave one
// partial per tap, written to the workspace.  The reduction kernels then add
// the partials of each filter tap in a fixed order, so the result is the same
// bits on every run.
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>

#include "f2d_internal.hpp"
#include "grad_internal.hpp"
#include "stencil_tile.hpp"

namespace f2d {
namespace {

using namespace tile;

// ------------------------------------------------------- grad_input edges --

// [lo, hi] = { y in [0, n) : cl_n(y + u - r) = p }, empty when lo > hi
__device__ __forceinline__ void preimage(int64_t p, int64_t n, int u, int r, int64_t& lo,
                                         int64_t& hi) {
  const int64_t tlo = p == 0 ? INT64_MIN / 4 : p;
  const int64_t thi = p == n - 1 ? INT64_MAX / 4 : p;
  lo = tlo - u + r;
  hi = thi - u + r;
  lo = lo < 0 ? 0 : lo;
  hi = hi > n - 1 ? n - 1 : hi;
}

// element reader (the edge kernel serves the f32 runtime-K path)
struct ReadF32 {
  using T = float;
  __device__ static float get(const float* p) { return *p; }
};
template <typename RG, typename RF>
__global__ __launch_bounds__(256) void k_grad_input_edges(EdgeParams p) {
  using TG = typename RG::T;
  using TF = typename RF::T;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  const int64_t H = p.H, W = p.W;
  const int64_t hr = H < 2 ? H : 2, wc = W < 2 ? W : 2;
  const int64_t E = W * hr + (H > 2 ? H - 2 : 0) * wc;  // edge pixels per plane
  if (idx >= E * p.planes) return;
  const int64_t plane = idx / E;
  int64_t e = idx - plane * E;
  const int64_t n = plane / p.groups, g = plane - n * p.groups;
  int64_t py, px;
  if (e < W * hr) {
    py = e < W ? 0 : H - 1;
    px = e < W ? e : e - W;
  } else {
    e -= W * hr;
    py = 1 + e / wc;
    px = (e % wc) == 0 ? 0 : W - 1;
  }
  const int K = p.k, r = (K - 1) / 2;
  float acc = 0.0f;
  for (int s = 0; s < p.nsrc; ++s) {
    const int t = s * p.st_s;
    const TG* gp = static_cast<const TG*>(t == 0 ? p.src[0] : t == 1 ? p.src[1] : t == 2 ? p.src[2] : p.src[3]);
    const int64_t sn = t == 0 ? p.src_sn[0] : t == 1 ? p.src_sn[1] : t == 2 ? p.src_sn[2] : p.src_sn[3];
    const int64_t sc = t == 0 ? p.src_sc[0] : t == 1 ? p.src_sc[1] : t == 2 ? p.src_sc[2] : p.src_sc[3];
    const int64_t sh = t == 0 ? p.src_sh[0] : t == 1 ? p.src_sh[1] : t == 2 ? p.src_sh[2] : p.src_sh[3];
    gp += n * sn + (g * p.sc_g + s * p.sc_s) * sc;
    const TF* fp = static_cast<const TF*>(p.filt) + (p.f0 + g * p.fg + s * p.fs) * static_cast<int64_t>(K * K);
    for (int u = 0; u < K; ++u) {
      int64_t ylo, yhi;
      preimage(py, H, u, r, ylo, yhi);
      if (ylo > yhi) continue;
      for (int v = 0; v < K; ++v) {
        int64_t xlo, xhi;
        preimage(px, W, v, r, xlo, xhi);
        if (xlo > xhi) continue;
        float rect = 0.0f;
        for (int64_t y = ylo; y <= yhi; ++y)
          for (int64_t x = xlo; x <= xhi; ++x) rect += RG::get(gp + y * sh + x);
        acc = __builtin_fmaf(RF::get(fp + u * K + v), rect, acc);
      }
    }
  }
  p.out[n * p.out_sn + g * p.out_sc + py * p.out_sh + px] = acc;
}

// Fold the frame onto the edge pixels: X-bar[p][q] += every frame value
// Z[a][b] with cl(a) = p and cl(b) = q, in a fixed order.
__global__ __launch_bounds__(256) void k_fold_frame(FoldParams p) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  const int64_t H = p.H, W = p.W, r = p.r;
  const int64_t hr = H < 2 ? H : 2, wc = W < 2 ? W : 2;
  const int64_t E = W * hr + (H > 2 ? H - 2 : 0) * wc;
  if (idx >= E * p.planes) return;
  const int64_t plane = idx / E;
  int64_t e = idx - plane * E;
  int64_t py, px;
  if (e < W * hr) {
    py = e < W ? 0 : H - 1;
    px = e < W ? e : e - W;
  } else {
    e -= W * hr;
    py = 1 + e / wc;
    px = (e % wc) == 0 ? 0 : W - 1;
  }
  const int64_t alo = py == 0 ? -r : py, ahi = py == H - 1 ? H - 1 + r : py;
  const int64_t blo = px == 0 ? -r : px, bhi = px == W - 1 ? W - 1 + r : px;
  const float* fr = p.frame + plane * p.frame_plane;
  float s = 0.0f;
  for (int64_t a = alo; a <= ahi; ++a)
    for (int64_t b = blo; b <= bhi; ++b) {
      if (a >= 0 && a < H && b >= 0 && b < W) continue;  // the pixel itself
      s += fr[frame_index(a, b, H, W, r)];
    }
  const int64_t n = plane / p.groups, g = plane - n * p.groups;
  float* o = p.out + n * p.out_sn + g * p.out_sc + py * p.out_sh + px;
  *o = *o + s;
}

// ----------------------------------------------------------- grad_filter --

__device__ __forceinline__ int64_t opaque64(int64_t v) {
  asm volatile("" : "+s"(v));
  return v;
}

// G-bar plane `t` of the selected tensor (compare-and-select on laundered
// kernel arguments keeps the argument block out of scratch).
__device__ __forceinline__ const float* gbar_plane(const GradFilterParams& p, int t, int64_t n,
                                                   int64_t ch, int64_t& sh) {
  int64_t b = opaque64(reinterpret_cast<int64_t>(p.g[0]));
  int64_t a = opaque64(p.g_sn[0]), c = opaque64(p.g_sc[0]), h = opaque64(p.g_sh[0]);
#pragma unroll
  for (int q = 1; q < kMaxT; ++q) {
    const int64_t bq = opaque64(reinterpret_cast<int64_t>(p.g[q]));
    const int64_t aq = opaque64(p.g_sn[q]), cq = opaque64(p.g_sc[q]), hq = opaque64(p.g_sh[q]);
    b = t == q ? bq : b;
    a = t == q ? aq : a;
    c = t == q ? cq : c;
    h = t == q ? hq : h;
  }
  sh = h;
  return reinterpret_cast<const float*>(b) + n * a + ch * c;
}

// acc[u][v] += sum_{jy,px} g[jy][px] * tile[ty*PY+jy+u][tx*PX+px+v]
template <int K, int PX, int PY>
__device__ __forceinline__ void accumulate_taps(const float* __restrict__ lds,
                                                const float (&gv)[PY][PX], float (&acc)[K * K]) {
  using G = Geom<K, PX, PY>;
  const int tx = threadIdx.x % kTX;
  const int ty = threadIdx.x / kTX;
#pragma unroll
  for (int ry = 0; ry < PY + K - 1; ++ry) {
    float win[G::WIN4];
    const float4* row = reinterpret_cast<const float4*>(lds + (ty * PY + ry) * G::PITCH + tx * PX);
#pragma unroll
    for (int q = 0; q < G::WIN4 / 4; ++q) {
      const float4 t = row[q];
      win[4 * q + 0] = t.x;
      win[4 * q + 1] = t.y;
      win[4 * q + 2] = t.z;
      win[4 * q + 3] = t.w;
    }
#pragma unroll
    for (int jy = 0; jy < PY; ++jy) {
      const int u = ry - jy;
      if (u < 0 || u >= K) continue;
#pragma unroll
      for (int v = 0; v < K; ++v)
#pragma unroll
        for (int px = 0; px < PX; ++px)
          acc[u * K + v] = __builtin_fmaf(gv[jy][px], win[px + v], acc[u * K + v]);
    }
  }
}

constexpr int kGfPX = 4, kGfPY = 4;

template <int K>
__global__ __launch_bounds__(kThreads) void k_grad_filter_f32(GradFilterParams p) {
  using G = Geom<K, kGfPX, kGfPY>;
  __shared__ float4 lds4[(G::LDS_WORDS + 3) / 4];
  __shared__ float red[kThreads / 64][K * K];
  float* lds = reinterpret_cast<float*>(lds4);

  const int64_t unit = xcd_remap(blockIdx.x, p.n_units);
  const int64_t chunk = unit % p.chunks;
  const int64_t pf = unit / p.chunks;  // rep * nf + f
  const int64_t f = pf % p.nf;
  const int64_t rep = pf / p.nf;
  // planes of this (X, G-bar) pair
  int64_t n, xc, gc;
  int gt = 0;
  if (p.mode == F2D_CH_SHARED) {
    n = rep / p.C;
    xc = gc = rep - n * p.C;
  } else if (p.mode == F2D_CH_DEPTHWISE) {
    n = rep;
    xc = gc = f / p.m;
    gt = static_cast<int>(f - xc * p.m);
  } else {
    n = rep;
    xc = f % p.C;
    gc = f / p.C;
  }
  const float* xp = static_cast<const float*>(p.x) + n * p.x_sn + xc * p.x_sc;
  int64_t gsh;
  const float* gp = gbar_plane(p, gt, n, gc, gsh);

  float acc[K * K];
#pragma unroll
  for (int e = 0; e < K * K; ++e) acc[e] = 0.0f;
  const int tx = threadIdx.x % kTX, ty = threadIdx.x / kTX;
  const int64_t tiles = static_cast<int64_t>(p.tiles_x) * p.tiles_y;
  for (int tt = 0; tt < p.tiles_per_unit; ++tt) {
    const int64_t tile = chunk * p.tiles_per_unit + tt;
    if (tile >= tiles) break;
    const int64_t oy0 = (tile / p.tiles_x) * G::TH, ox0 = (tile % p.tiles_x) * G::TW;
    stage_tile<K, kGfPX, kGfPY, false>(lds, xp, p.x_sh, p.H, p.W, oy0, ox0);
    float gv[kGfPY][kGfPX];
#pragma unroll
    for (int jy = 0; jy < kGfPY; ++jy) {
      const int64_t y = oy0 + ty * kGfPY + jy;
      const int64_t x = ox0 + tx * kGfPX;
      const float* row = gp + (y < p.H ? y : 0) * gsh;
      if ((p.flags & kDstVec) && y < p.H && x + kGfPX <= p.W) {
        const float4 q = *reinterpret_cast<const float4*>(row + x);
        gv[jy][0] = q.x;
        gv[jy][1] = q.y;
        gv[jy][2] = q.z;
        gv[jy][3] = q.w;
      } else {
#pragma unroll
        for (int px = 0; px < kGfPX; ++px)
          gv[jy][px] = (y < p.H && x + px < p.W) ? row[x + px] : 0.0f;
      }
    }
    __syncthreads();
    accumulate_taps<K, kGfPX, kGfPY>(lds, gv, acc);
    __syncthreads();
  }
  // fixed-order reduction: butterfly within each wave, then waves 0..3
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
#pragma unroll
  for (int e = 0; e < K * K; ++e) {
    float v = acc[e];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    acc[e] = v;
  }
  if (lane == 0) {
#pragma unroll
    for (int e = 0; e < K * K; ++e) red[wave][e] = acc[e];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < K * K; e += kThreads) {
    float s = red[0][e];
#pragma unroll
    for (int w = 1; w < kThreads / 64; ++w) s += red[w][e];
    p.partial[unit * (K * K) + e] = s;
  }
}

// Filter banks: a work-group takes NO G-bar planes (output channels
// NO*og ..) and NI X planes (input channels NI*ig ..) of one image over a run
// of tiles, so that every staged X tile serves NO output channels and every
// G-bar block NI input channels (one plane pair per work-group reads each X
// plane C_out times and each G-bar plane C_in times).  Per filter pair the
// sums run in the same order as in k_grad_filter_f32, and the partials land
// in the same workspace slots, so the results are the same bits.
template <int K, int NO, int NI>
__global__ __launch_bounds__(kThreads) void k_grad_filter_bank_f32(GradFilterParams p) {
  using G = Geom<K, kGfPX, kGfPY>;
  constexpr int KK = K * K;
  __shared__ float4 lds4[NI][(G::LDS_WORDS + 3) / 4];
  __shared__ float red[kThreads / 64][NO * NI * KK];

  const int64_t co = p.nf / p.C;
  const int64_t ngo = co / NO, ngi = p.C / NI;
  // output-channel group fastest: consecutive work-groups (one XCD) share
  // their X tiles, and the G-bar tiles recur every ngo*chunks groups
  int64_t rest = xcd_remap(blockIdx.x, p.n_units);
  const int64_t og = rest % ngo;
  rest /= ngo;
  const int64_t chunk = rest % p.chunks;
  rest /= p.chunks;
  const int64_t ig = rest % ngi;
  const int64_t n = rest / ngi;
  const float* xp[NI];
#pragma unroll
  for (int k = 0; k < NI; ++k)
    xp[k] = static_cast<const float*>(p.x) + n * p.x_sn + (ig * NI + k) * p.x_sc;
  const float* gp[NO];
  int64_t gsh = 0;
#pragma unroll
  for (int j = 0; j < NO; ++j) gp[j] = gbar_plane(p, 0, n, og * NO + j, gsh);

  float acc[NO][NI][KK];
#pragma unroll
  for (int j = 0; j < NO; ++j)
#pragma unroll
    for (int k = 0; k < NI; ++k)
#pragma unroll
      for (int e = 0; e < KK; ++e) acc[j][k][e] = 0.0f;
  const int tx = threadIdx.x % kTX, ty = threadIdx.x / kTX;
  const int64_t tiles = static_cast<int64_t>(p.tiles_x) * p.tiles_y;
  for (int tt = 0; tt < p.tiles_per_unit; ++tt) {
    const int64_t tile = chunk * p.tiles_per_unit + tt;
    if (tile >= tiles) break;
    const int64_t oy0 = (tile / p.tiles_x) * G::TH, ox0 = (tile % p.tiles_x) * G::TW;
#pragma unroll
    for (int k = 0; k < NI; ++k)
      stage_tile<K, kGfPX, kGfPY, false>(reinterpret_cast<float*>(lds4[k]), xp[k], p.x_sh, p.H, p.W, oy0, ox0);
    float gv[NO][kGfPY][kGfPX];
#pragma unroll
    for (int j = 0; j < NO; ++j)
#pragma unroll
      for (int jy = 0; jy < kGfPY; ++jy) {
        const int64_t y = oy0 + ty * kGfPY + jy;
        const int64_t x = ox0 + tx * kGfPX;
        const float* row = gp[j] + (y < p.H ? y : 0) * gsh;
        if ((p.flags & kDstVec) && y < p.H && x + kGfPX <= p.W) {
          const float4 q = *reinterpret_cast<const float4*>(row + x);
          gv[j][jy][0] = q.x;
          gv[j][jy][1] = q.y;
          gv[j][jy][2] = q.z;
          gv[j][jy][3] = q.w;
        } else {
#pragma unroll
          for (int px = 0; px < kGfPX; ++px)
            gv[j][jy][px] = (y < p.H && x + px < p.W) ? row[x + px] : 0.0f;
        }
      }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NI; ++k) {
      const float* lds = reinterpret_cast<const float*>(lds4[k]);
#pragma unroll
      for (int ry = 0; ry < kGfPY + K - 1; ++ry) {
        float win[G::WIN4];
        const float4* rowp = reinterpret_cast<const float4*>(lds + (ty * kGfPY + ry) * G::PITCH + tx * kGfPX);
#pragma unroll
        for (int q = 0; q < G::WIN4 / 4; ++q) {
          const float4 t = rowp[q];
          win[4 * q + 0] = t.x;
          win[4 * q + 1] = t.y;
          win[4 * q + 2] = t.z;
          win[4 * q + 3] = t.w;
        }
#pragma unroll
        for (int j = 0; j < NO; ++j)
#pragma unroll
          for (int jy = 0; jy < kGfPY; ++jy) {
            const int u = ry - jy;
            if (u < 0 || u >= K) continue;
#pragma unroll
            for (int v = 0; v < K; ++v)
#pragma unroll
              for (int px = 0; px < kGfPX; ++px)
                acc[j][k][u * K + v] = __builtin_fmaf(gv[j][jy][px], win[px + v], acc[j][k][u * K + v]);
          }
      }
    }
    __syncthreads();
  }
  // the same fixed-order reduction as k_grad_filter_f32, per filter pair
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
#pragma unroll
  for (int j = 0; j < NO; ++j)
#pragma unroll
    for (int k = 0; k < NI; ++k)
#pragma unroll
      for (int e = 0; e < KK; ++e) {
        float v = acc[j][k][e];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == 0) red[wave][(j * NI + k) * KK + e] = v;
      }
  __syncthreads();
  for (int idx = threadIdx.x; idx < NO * NI * KK; idx += kThreads) {
    float sum = red[0][idx];
#pragma unroll
    for (int w = 1; w < kThreads / 64; ++w) sum += red[w][idx];
    const int jk = idx / KK, e = idx - jk * KK;
    const int64_t f = (og * NO + jk / NI) * p.C + ig * NI + jk % NI;
    p.partial[((n * p.nf + f) * p.chunks + chunk) * KK + e] = sum;
  }
}

// Runtime-K fallback (K > 9): one tap at a time, every thread summing its
// pixels of the unit's tiles straight from memory, then the same fixed-order
// block reduction.
__global__ __launch_bounds__(kThreads) void k_grad_filter_generic(GradFilterParams p, int K) {
  __shared__ float red[kThreads / 64];
  const int64_t unit = blockIdx.x;
  const int64_t chunk = unit % p.chunks;
  const int64_t pf = unit / p.chunks;
  const int64_t f = pf % p.nf;
  const int64_t rep = pf / p.nf;
  int64_t n, xc, gc;
  int gt = 0;
  if (p.mode == F2D_CH_SHARED) {
    n = rep / p.C;
    xc = gc = rep - n * p.C;
  } else if (p.mode == F2D_CH_DEPTHWISE) {
    n = rep;
    xc = gc = f / p.m;
    gt = static_cast<int>(f - xc * p.m);
  } else {
    n = rep;
    xc = f % p.C;
    gc = f / p.C;
  }
  const float* xp = static_cast<const float*>(p.x) + n * p.x_sn + xc * p.x_sc;
  int64_t gsh;
  const float* gp = gbar_plane(p, gt, n, gc, gsh);
  const int r = (K - 1) / 2;
  const TileShape ts{kTY * kGfPY, kTX * kGfPX};
  const int64_t tiles = static_cast<int64_t>(p.tiles_x) * p.tiles_y;
  for (int e = 0; e < K * K; ++e) {
    const int u = e / K, v = e % K;
    float s = 0.0f;
    for (int tt = 0; tt < p.tiles_per_unit; ++tt) {
      const int64_t tile = chunk * p.tiles_per_unit + tt;
      if (tile >= tiles) break;
      const int64_t oy0 = (tile / p.tiles_x) * ts.th, ox0 = (tile % p.tiles_x) * ts.tw;
      for (int i = threadIdx.x; i < ts.th * ts.tw; i += kThreads) {
        const int64_t y = oy0 + i / ts.tw, x = ox0 + i % ts.tw;
        if (y >= p.H || x >= p.W) continue;
        int64_t sy = y + u - r, sx = x + v - r;
        sy = sy < 0 ? 0 : (sy >= p.H ? p.H - 1 : sy);
        sx = sx < 0 ? 0 : (sx >= p.W ? p.W - 1 : sx);
        s = __builtin_fmaf(gp[y * gsh + x], xp[sy * p.x_sh + sx], s);
      }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = s;
    __syncthreads();
    if (threadIdx.x == 0) p.partial[unit * (K * K) + e] = ((red[0] + red[1]) + red[2]) + red[3];
    __syncthreads();
  }
}

// out[f][e] = sum over (rep, chunk) of partial[((rep*nf + f)*chunks + chunk)][e],
// each thread summing a fixed stride of units, then a fixed butterfly.
// Fixed-order reduction of the partial sets, in two passes over the layout
// partial[((rep * nf + f) * chunks + c) * kk + e] (item i = rep * chunks + c):
//  pass 1  thread (j = f*kk + e, segment s) adds items s*L .. s*L+L-1 in
//          order and writes the sum over item s*L (it alone reads that slot);
//  pass 2  adds the segment sums in order: one thread per output when there
//          are many outputs, else one work-group per output (strided
//          threads, then a fixed shuffle tree).
__device__ __forceinline__ int64_t partial_index(int64_t i, int64_t f, int e, int64_t nf, int kk, int64_t chunks) {
  const int64_t rep = i / chunks, c = i - rep * chunks;
  return ((rep * nf + f) * chunks + c) * kk + e;
}

__global__ __launch_bounds__(256) void k_reduce_segments(float* __restrict__ partial, int64_t nf, int kk,
                                                         int64_t chunks, int64_t count, int64_t seg) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (j >= nf * kk) return;
  const int64_t f = j / kk;
  const int e = static_cast<int>(j - f * kk);
  const int64_t i0 = static_cast<int64_t>(blockIdx.y) * seg;
  const int64_t i1 = i0 + seg < count ? i0 + seg : count;
  float s = 0.0f;
  int64_t i = i0;
  for (; i + 4 <= i1; i += 4) {
    const float a0 = partial[partial_index(i, f, e, nf, kk, chunks)];
    const float a1 = partial[partial_index(i + 1, f, e, nf, kk, chunks)];
    const float a2 = partial[partial_index(i + 2, f, e, nf, kk, chunks)];
    const float a3 = partial[partial_index(i + 3, f, e, nf, kk, chunks)];
    s = (((s + a0) + a1) + a2) + a3;
  }
  for (; i < i1; ++i) s += partial[partial_index(i, f, e, nf, kk, chunks)];
  partial[partial_index(i0, f, e, nf, kk, chunks)] = s;
}

__global__ __launch_bounds__(256) void k_reduce_columns(const float* __restrict__ partial, float* __restrict__ out,
                                                        int64_t nf, int kk, int64_t chunks, int64_t nseg,
                                                        int64_t seg) {
  const int64_t j = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (j >= nf * kk) return;
  const int64_t f = j / kk;
  const int e = static_cast<int>(j - f * kk);
  float s = 0.0f;
  for (int64_t g = 0; g < nseg; ++g) s += partial[partial_index(g * seg, f, e, nf, kk, chunks)];
  out[j] = s;
}

__global__ __launch_bounds__(256) void k_reduce_rows(const float* __restrict__ partial, float* __restrict__ out,
                                                     int64_t nf, int kk, int64_t chunks, int64_t nseg, int64_t seg) {
  __shared__ float red[4];
  const int64_t f = blockIdx.x / kk;
  const int e = static_cast<int>(blockIdx.x % kk);
  float s = 0.0f;
  for (int64_t g = threadIdx.x; g < nseg; g += 256) s += partial[partial_index(g * seg, f, e, nf, kk, chunks)];
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[f * kk + e] = ((red[0] + red[1]) + red[2]) + red[3];
}

}  // namespace

hipError_t launch_grad_input_edges(const EdgeParams& p, int kind, hipStream_t s) {
  const int64_t H = p.H, W = p.W;
  const int64_t hr = H < 2 ? H : 2, wc = W < 2 ? W : 2;
  const int64_t E = W * hr + (H > 2 ? H - 2 : 0) * wc;
  const int64_t total = E * p.planes;
  if (total <= 0) return hipSuccess;
  const int64_t blocks = (total + 255) / 256;
  const dim3 grid(static_cast<uint32_t>(blocks)), block(256);
  if (kind != kEdgeF32) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_grad_input_edges<ReadF32, ReadF32>), grid, block, 0, s, p);
  return hipGetLastError();
}

hipError_t launch_fold_frame(const FoldParams& p, hipStream_t s) {
  const int64_t H = p.H, W = p.W;
  const int64_t hr = H < 2 ? H : 2, wc = W < 2 ? W : 2;
  const int64_t total = (W * hr + (H > 2 ? H - 2 : 0) * wc) * p.planes;
  if (total <= 0 || p.r == 0) return hipSuccess;
  hipLaunchKernelGGL(k_fold_frame, dim3(static_cast<uint32_t>((total + 255) / 256)), dim3(256), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_grad_filter_f32(const GradFilterParams& p, int K, hipStream_t s) {
  if (p.n_units <= 0) return hipSuccess;
  const dim3 grid(static_cast<uint32_t>(p.n_units)), block(kThreads);
  switch (K) {
    case 1: hipLaunchKernelGGL(k_grad_filter_f32<1>, grid, block, 0, s, p); break;
    case 3: hipLaunchKernelGGL(k_grad_filter_f32<3>, grid, block, 0, s, p); break;
    case 5: hipLaunchKernelGGL(k_grad_filter_f32<5>, grid, block, 0, s, p); break;
    case 7: hipLaunchKernelGGL(k_grad_filter_f32<7>, grid, block, 0, s, p); break;
    case 9: hipLaunchKernelGGL(k_grad_filter_f32<9>, grid, block, 0, s, p); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Filter pairs per work-group of the grouped bank kernel: NO output x NI
// input channels for K = 1, 3 (4 x 2) and 5 (2 x 2); false where it does not
// apply (other modes or K, or channel counts that the groups do not divide).
// (4 x 4 at K = 3 staged fewer tiles but held 240 registers, two waves per
// SIMD: 4% slower than 4 x 2 at three.)
bool grad_filter_bank_groups(int mode, int K, int64_t co, int64_t ci, int* no, int* ni) {
  *no = K <= 3 ? 4 : 2;
  *ni = 2;
  return mode == F2D_CH_BANK && (K == 1 || K == 3 || K == 5) && co % *no == 0 && ci % *ni == 0;
}

// p.n_units = images * chunks * (C_out / NO) * (C_in / NI)
hipError_t launch_grad_filter_bank_f32(const GradFilterParams& p, int K, hipStream_t s) {
  if (p.n_units <= 0) return hipSuccess;
  const dim3 grid(static_cast<uint32_t>(p.n_units)), block(kThreads);
  switch (K) {
    case 1: hipLaunchKernelGGL((k_grad_filter_bank_f32<1, 4, 2>), grid, block, 0, s, p); break;
    case 3: hipLaunchKernelGGL((k_grad_filter_bank_f32<3, 4, 2>), grid, block, 0, s, p); break;
    case 5: hipLaunchKernelGGL((k_grad_filter_bank_f32<5, 2, 2>), grid, block, 0, s, p); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_grad_filter_generic(const GradFilterParams& p, int K, hipStream_t s) {
  if (p.n_units <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_grad_filter_generic, dim3(static_cast<uint32_t>(p.n_units)), dim3(kThreads), 0, s, p,
                     K);
  return hipGetLastError();
}

hipError_t launch_reduce_partials(float* partial, float* out, int64_t nf, int kk, int64_t nrep, int64_t chunks,
                                  hipStream_t s) {
  const int64_t m = nf * kk;  // outputs
  if (m <= 0) return hipSuccess;
  const int64_t count = nrep * chunks;
  constexpr int64_t kSeg = 32;  // items per first-pass segment
  const int64_t nseg = (count + kSeg - 1) / kSeg;
  const int64_t col_blocks = (m + 255) / 256;
  if (nseg > 0) {
    hipLaunchKernelGGL(k_reduce_segments, dim3(static_cast<uint32_t>(col_blocks), static_cast<uint32_t>(nseg)),
                       dim3(256), 0, s, partial, nf, kk, chunks, count, kSeg);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (m >= 4096 || nseg <= 64)
    hipLaunchKernelGGL(k_reduce_columns, dim3(static_cast<uint32_t>(col_blocks)), dim3(256), 0, s, partial, out,
                       nf, kk, chunks, nseg, kSeg);
  else
    hipLaunchKernelGGL(k_reduce_rows, dim3(static_cast<uint32_t>(m)), dim3(256), 0, s, partial, out, nf, kk,
                       chunks, nseg, kSeg);
  return hipGetLastError();
}

TileShape grad_filter_tile() { return {kTY * kGfPY, kTX * kGfPX}; }

}  // namespace f2d
