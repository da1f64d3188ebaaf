// u8 image -> int32 K x K stencil kernels (exact integer arithmetic).
//
// This path is bound by its int32 writes (4 bytes out per output value for
// 1 byte in), so the kernel is shaped around an uninterrupted store stream.
// A work-group (4 waves) owns a 256-pixel-wide, 4*RS-row tile of one
// channel.  It first stages the tile's source rows, halo included, in LDS
// with aligned word loads (clamped byte loads only at the image edges).  Each
// wave then walks down its RS-row strip: every lane keeps the last K source
// rows of its (4+K-1)-byte window in registers, reading one new row from LDS
// per output row, and writes four consecutive pixels of every output plane
// with one 16-byte store (a wave writes 1 KiB contiguous per instruction).
// Because all global loads happen before the first store, no wait on a load
// ever has to drain the stores queued ahead of it (loads and stores share one
// completion counter on this GPU family).  The M filters applied to the same
// channel (Sobel-x and Sobel-y for M = 2) share the window, and the optional
// epilogue writes o0^2 + o1^2.
//
// Integer sums wrap modulo 2^32 (unsigned arithmetic).  When every filter's
// sum of |taps| is at most 32767 (checked once per work-group, a uniform
// branch), each product and the epilogue squares fit the 24-bit multiplier
// exactly and the kernel uses it; otherwise it uses full 32-bit multiplies.
#include "f2d_internal.hpp"

namespace f2d {
namespace {

constexpr int kThreads = 256;
constexpr int kLanes = 64;  // lanes along x (4 pixels each)
constexpr int kWaves = 4;   // row strips per work-group
constexpr int kTW = kLanes * 4;
constexpr int kPitchWords = kTW / 4 + 2;  // staged source columns x0-4 .. x0+TW+3
constexpr int kMaxR = 4;                  // K <= 9

typedef int v4i __attribute__((ext_vector_type(4)));

template <bool SMALL>
__device__ __forceinline__ uint32_t mul(uint32_t a, uint32_t b) {
  if constexpr (SMALL) return static_cast<uint32_t>(__mul24(static_cast<int>(a), static_cast<int>(b)));
  return a * b;
}

__device__ __forceinline__ void store4(int32_t* __restrict__ dp, int64_t x0, int64_t W, bool vec,
                                       const uint32_t (&v)[4], bool nt) {
  if (vec && x0 + 4 <= W) {
    v4i q;
    q.x = static_cast<int>(v[0]);
    q.y = static_cast<int>(v[1]);
    q.z = static_cast<int>(v[2]);
    q.w = static_cast<int>(v[3]);
    if (nt)
      __builtin_nontemporal_store(q, reinterpret_cast<v4i*>(dp + x0));
    else
      *reinterpret_cast<v4i*>(dp + x0) = q;
  } else {
#pragma unroll
    for (int px = 0; px < 4; ++px)
      if (x0 + px < W) dp[x0 + px] = static_cast<int>(v[px]);
  }
}

// Stage source rows row_base .. row_base+LH-1 (clamped), columns x0-4 ..
// x0+TW+3 (clamped) as little-endian words: LDS word d of a row holds source
// columns x0-4+4d .. x0-1+4d.
template <int LH>
__device__ __forceinline__ void stage(uint32_t* __restrict__ lds, const uint8_t* __restrict__ sp,
                                      int64_t sh, int64_t H, int64_t W, int64_t row_base, int64_t x0,
                                      bool word_ok) {
  // Waves take rows (uniform row address), lanes take words.  Interior tiles
  // (a uniform test) load aligned words; tiles touching the left or right
  // edge, or unaligned rows, assemble each word from clamped byte loads.  All
  // loads of a wave are issued before the first LDS write.
  constexpr int CPL = (kPitchWords + kLanes - 1) / kLanes;
  constexpr int RPW = (LH + kWaves - 1) / kWaves;
  const int lane = threadIdx.x % kLanes;
  const int wave = threadIdx.x / kLanes;
  const bool interior = word_ok && x0 - 4 >= 0 && x0 + 4 * kPitchWords - 4 <= W;
  uint32_t buf[RPW][CPL];
  const uint8_t* rows[RPW];
#pragma unroll
  for (int i = 0; i < RPW; ++i) {
    const int ly = wave + kWaves * i;
    int64_t gy = row_base + (ly < LH ? ly : LH - 1);
    gy = gy < 0 ? 0 : (gy >= H ? H - 1 : gy);
    rows[i] = sp + gy * sh;
  }
  if (interior) {
#pragma unroll
    for (int i = 0; i < RPW; ++i)
#pragma unroll
      for (int j = 0; j < CPL; ++j) {
        const int d = lane + kLanes * j < kPitchWords ? lane + kLanes * j : kPitchWords - 1;
        buf[i][j] = *reinterpret_cast<const uint32_t*>(rows[i] + x0 - 4 + 4 * d);
      }
  } else {
#pragma unroll
    for (int i = 0; i < RPW; ++i)
#pragma unroll
      for (int j = 0; j < CPL; ++j) {
        const int64_t gx = x0 - 4 + 4 * (lane + kLanes * j);
        uint32_t v = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          int64_t c = gx + q;
          c = c < 0 ? 0 : (c >= W ? W - 1 : c);
          v |= static_cast<uint32_t>(rows[i][c]) << (8 * q);
        }
        buf[i][j] = v;
      }
  }
#pragma unroll
  for (int i = 0; i < RPW; ++i) {
    const int ly = wave + kWaves * i;
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
      const int d = lane + kLanes * j;
      if (ly < LH && d < kPitchWords) lds[ly * kPitchWords + d] = buf[i][j];
    }
  }
}

// The lane's window of one staged row: source columns xl-R .. xl+3+R where
// xl = x0 + 4*lane, i.e. bytes 4-R .. 7+R of LDS words lane .. lane+2.
template <int K>
__device__ __forceinline__ void window_row(const uint32_t* __restrict__ ldsrow, int lane,
                                           uint32_t (&dst)[4 + K - 1]) {
  constexpr int R = (K - 1) / 2;
  const uint32_t w0 = ldsrow[lane], w1 = ldsrow[lane + 1], w2 = ldsrow[lane + 2];
#pragma unroll
  for (int c = 0; c < 4 + K - 1; ++c) {
    const int j = 4 - R + c;  // byte index in w0:w1:w2
    const uint32_t w = j < 4 ? w0 : (j < 8 ? w1 : w2);
    dst[c] = (w >> (8 * (j & 3))) & 0xffu;
  }
}

template <int K, int M, bool SUMSQ, int RS, bool NT, bool SMALL>
__device__ __forceinline__ void strip(const uint32_t* __restrict__ lds, int lane, int wave,
                                      int32_t* const (&dp)[M + 1], const int64_t (&dsh)[M + 1],
                                      const uint32_t (&tap)[M][K * K], int64_t xl, int64_t W,
                                      int64_t oy0, int nrows, bool vec) {
  constexpr int WIN = 4 + K - 1;
  uint32_t win[K][WIN];
  const uint32_t* base = lds + wave * RS * kPitchWords;
#pragma unroll
  for (int u = 0; u + 1 < K; ++u) window_row<K>(base + u * kPitchWords, lane, win[u + 1]);
  for (int i = 0; i < nrows; ++i) {
#pragma unroll
    for (int u = 0; u + 1 < K; ++u)
#pragma unroll
      for (int c = 0; c < WIN; ++c) win[u][c] = win[u + 1][c];
    window_row<K>(base + (i + K - 1) * kPitchWords, lane, win[K - 1]);

    uint32_t o[M][4];
#pragma unroll
    for (int j = 0; j < M; ++j) {
#pragma unroll
      for (int px = 0; px < 4; ++px) o[j][px] = 0u;
#pragma unroll
      for (int u = 0; u < K; ++u)
#pragma unroll
        for (int v = 0; v < K; ++v)
#pragma unroll
          for (int px = 0; px < 4; ++px) o[j][px] += mul<SMALL>(win[u][px + v], tap[j][u * K + v]);
    }
    const int64_t oy = oy0 + i;
#pragma unroll
    for (int j = 0; j < M; ++j) store4(dp[j] + oy * dsh[j], xl, W, vec, o[j], NT);
    if constexpr (SUMSQ) {
      uint32_t m2[4];
#pragma unroll
      for (int px = 0; px < 4; ++px)
        m2[px] = mul<SMALL>(o[0][px], o[0][px]) + mul<SMALL>(o[1][px], o[1][px]);
      store4(dp[M] + oy * dsh[M], xl, W, vec, m2, NT);
    }
  }
}

template <int K, int M, bool SUMSQ, int RS, bool NT>
__global__ __launch_bounds__(kThreads) void k_stencil_u8(StencilParams p) {
  constexpr int R = (K - 1) / 2;
  constexpr int TH = kWaves * RS;
  constexpr int LH = TH + K - 1;
  static_assert(R <= kMaxR, "K <= 9");
  __shared__ uint32_t lds[LH * kPitchWords];

  const int64_t b = xcd_remap(blockIdx.x, p.n_blocks);
  const int64_t tiles = static_cast<int64_t>(p.tiles_x) * p.tiles_y;
  const int64_t plane = b / tiles;
  const int64_t t = b - plane * tiles;
  const int64_t tile_y = t / p.tiles_x;
  const int64_t tile_x = t - tile_y * p.tiles_x;
  const int64_t n = plane / p.groups;
  const int64_t g = plane - n * p.groups;
  const int lane = threadIdx.x % kLanes;
  const int wave = threadIdx.x / kLanes;
  const int64_t x0 = tile_x * kTW;
  const int64_t ty0 = tile_y * TH;  // first output row of the tile (band-relative)

  const uint8_t* sp = static_cast<const uint8_t*>(p.src[0]) + n * p.src_sn[0] + g * p.src_sc[0];
  stage<LH>(lds, sp, p.src_sh[0], p.H, p.W, p.row0 + ty0 - R, x0, (p.flags & kSrcVec) != 0);

  int32_t* dp[M + 1];
  int64_t dsh[M + 1];
#pragma unroll
  for (int j = 0; j <= M; ++j) {
    const int jj = j < M ? j : (SUMSQ ? M : 0);
    void* base = jj == 0 ? p.dst[0] : jj == 1 ? p.dst[1] : jj == 2 ? p.dst[2] : p.dst[3];
    int64_t sn = jj == 0 ? p.dst_sn[0] : jj == 1 ? p.dst_sn[1] : jj == 2 ? p.dst_sn[2] : p.dst_sn[3];
    int64_t sc = jj == 0 ? p.dst_sc[0] : jj == 1 ? p.dst_sc[1] : jj == 2 ? p.dst_sc[2] : p.dst_sc[3];
    dsh[j] = jj == 0 ? p.dst_sh[0] : jj == 1 ? p.dst_sh[1] : jj == 2 ? p.dst_sh[2] : p.dst_sh[3];
    dp[j] = static_cast<int32_t*>(base) + n * sn + g * sc;
  }

  uint32_t tap[M][K * K];
  bool small = true;
  const int32_t* filt = static_cast<const int32_t*>(p.filt);
#pragma unroll
  for (int j = 0; j < M; ++j) {
    const int32_t* fp = filt + static_cast<int64_t>(p.f0 + g * p.fg + j * p.fj) * (K * K);
    int64_t l1 = 0;
#pragma unroll
    for (int e = 0; e < K * K; ++e) {
      const int32_t v = fp[e];
      tap[j][e] = static_cast<uint32_t>(v);
      l1 += v < 0 ? -static_cast<int64_t>(v) : v;
    }
    small = small && l1 <= 32767;
  }
  __syncthreads();

  const int64_t xl = x0 + 4 * lane;
  const int64_t oy0 = ty0 + wave * RS;
  if (xl >= p.W || oy0 >= p.rows) return;  // no barriers follow
  const int nrows = static_cast<int>(p.rows - oy0 < RS ? p.rows - oy0 : RS);
  const bool vec = (p.flags & kDstVec) != 0;
  if (small)
    strip<K, M, SUMSQ, RS, NT, true>(lds, lane, wave, dp, dsh, tap, xl, p.W, oy0, nrows, vec);
  else
    strip<K, M, SUMSQ, RS, NT, false>(lds, lane, wave, dp, dsh, tap, xl, p.W, oy0, nrows, vec);
}

// Runtime-K fallback: one output value per thread per filter, source read
// through the caches, same integer semantics (full 32-bit multiplies).
__global__ __launch_bounds__(kThreads) void k_stencil_u8_generic(StencilParams p, int m) {
  const int K = p.k, R = (K - 1) / 2;
  const int64_t b = xcd_remap(blockIdx.x, p.n_blocks);
  const int64_t tiles = static_cast<int64_t>(p.tiles_x) * p.tiles_y;
  const int64_t plane = b / tiles;
  const int64_t t = b - plane * tiles;
  const int64_t tile_y = t / p.tiles_x;
  const int64_t tile_x = t - tile_y * p.tiles_x;
  const int64_t n = plane / p.groups;
  const int64_t g = plane - n * p.groups;
  const int64_t oy = tile_y * 16 + threadIdx.x / 16;
  const int64_t ox = tile_x * 16 + threadIdx.x % 16;
  if (oy >= p.rows || ox >= p.W) return;
  const uint8_t* sp = static_cast<const uint8_t*>(p.src[0]) + n * p.src_sn[0] + g * p.src_sc[0];
  const int32_t* filt = static_cast<const int32_t*>(p.filt);
  uint32_t o0 = 0, o1 = 0;
  for (int j = 0; j < m; ++j) {
    const int32_t* fp = filt + static_cast<int64_t>(p.f0 + g * p.fg + j * p.fj) * K * K;
    uint32_t acc = 0;
    for (int u = 0; u < K; ++u) {
      int64_t y = p.row0 + oy + u - R;
      y = y < 0 ? 0 : (y >= p.H ? p.H - 1 : y);
      for (int v = 0; v < K; ++v) {
        int64_t x = ox + v - R;
        x = x < 0 ? 0 : (x >= p.W ? p.W - 1 : x);
        acc += static_cast<uint32_t>(sp[y * p.src_sh[0] + x]) * static_cast<uint32_t>(fp[u * K + v]);
      }
    }
    void* base = j == 0 ? p.dst[0] : j == 1 ? p.dst[1] : j == 2 ? p.dst[2] : p.dst[3];
    int64_t sn = j == 0 ? p.dst_sn[0] : j == 1 ? p.dst_sn[1] : j == 2 ? p.dst_sn[2] : p.dst_sn[3];
    int64_t sc = j == 0 ? p.dst_sc[0] : j == 1 ? p.dst_sc[1] : j == 2 ? p.dst_sc[2] : p.dst_sc[3];
    int64_t sh = j == 0 ? p.dst_sh[0] : j == 1 ? p.dst_sh[1] : j == 2 ? p.dst_sh[2] : p.dst_sh[3];
    static_cast<int32_t*>(base)[n * sn + g * sc + oy * sh + ox] = static_cast<int32_t>(acc);
    if (j == 0) o0 = acc;
    if (j == 1) o1 = acc;
  }
  if ((p.flags & kSumSq) && m == 2) {
    int32_t* d = static_cast<int32_t*>(p.dst[2]);
    d[n * p.dst_sn[2] + g * p.dst_sc[2] + oy * p.dst_sh[2] + ox] =
        static_cast<int32_t>(o0 * o0 + o1 * o1);
  }
}

template <int K, int M, bool SUMSQ, int RS, bool NT>
hipError_t go(const StencilParams& p, hipStream_t stream) {
  hipLaunchKernelGGL((k_stencil_u8<K, M, SUMSQ, RS, NT>), dim3(static_cast<uint32_t>(p.n_blocks)),
                     dim3(kThreads), 0, stream, p);
  return hipGetLastError();
}

template <int K, int M, bool SUMSQ>
hipError_t by_variant(const StencilParams& p, int variant, hipStream_t stream) {
  switch (variant) {
    case 2: return go<K, M, SUMSQ, 8, false>(p, stream);
    case 3: return go<K, M, SUMSQ, 32, false>(p, stream);
    case 4: return go<K, M, SUMSQ, 16, true>(p, stream);
    case 5: return go<K, M, SUMSQ, 8, true>(p, stream);
    case 6: return go<K, M, SUMSQ, 4, false>(p, stream);
    case 7: return go<K, M, SUMSQ, 4, true>(p, stream);
    default: return go<K, M, SUMSQ, 16, false>(p, stream);
  }
}

template <int K>
hipError_t by_m(const StencilParams& p, int m, bool sumsq, int variant, hipStream_t stream) {
  if (m == 2) {
    if (sumsq) return by_variant<K, 2, true>(p, variant, stream);
    return by_variant<K, 2, false>(p, variant, stream);
  }
  return by_variant<K, 1, false>(p, variant, stream);
}

}  // namespace

TileShape u8_tile(int variant) {
  switch (variant) {
    case 2: case 5: return {kWaves * 8, kTW};
    case 3: return {kWaves * 32, kTW};
    case 6: case 7: return {kWaves * 4, kTW};
    case -1: return {16, 16};  // generic kernel
    default: return {kWaves * 16, kTW};
  }
}

int u8_variant_count() { return 7; }

// m is 1 or 2 for the templated kernels (K <= 9); variant < 0 selects
// the generic kernel, which handles m <= 2 for any odd K <= 31.
hipError_t launch_stencil_u8(const StencilParams& p, int K, int m, bool sumsq, bool vec,
                             int variant, hipStream_t stream) {
  (void)vec;
  if (p.n_blocks <= 0) return hipSuccess;
  if (variant < 0) {
    hipLaunchKernelGGL(k_stencil_u8_generic, dim3(static_cast<uint32_t>(p.n_blocks)),
                       dim3(kThreads), 0, stream, p, m);
    return hipGetLastError();
  }
  switch (K) {
    case 1: return by_m<1>(p, m, sumsq, variant, stream);
    case 3: return by_m<3>(p, m, sumsq, variant, stream);
    case 5: return by_m<5>(p, m, sumsq, variant, stream);
    case 7: return by_m<7>(p, m, sumsq, variant, stream);
    case 9: return by_m<9>(p, m, sumsq, variant, stream);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace f2d
