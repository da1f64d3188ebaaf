// 8-bit image kernels: the paper's own image operations on its own data type.
//
// The paper filters 8-bit images read with OpenCV (interleaved channels, one
// pixel after another) with float taps: a 3x3 Laplacian sharpen that skips
// out-of-image neighbours (Section 4.2.4), run on images enlarged by nearest-
// neighbour upsampling (Section 4.2.3; the pipeline of Section 6.6), and a
// weighted RGB -> gray sum (Section 4.2.5).  Two kernels cover them:
//
//  k_u8_gather  one K x K filter (SHARED mode) on planar or interleaved 8-bit
//               images, clamp-to-edge or zero borders, optionally through a
//               nearest upsample by an integer factor s (output pixel (Y, X)
//               reads source pixel (Y / s, X / s)) that is never materialised.
//               A work-group owns a 32-row x 2048-element output tile (an
//               element is one channel of one pixel: for interleaved images a
//               row is W*s*C elements long and the tap offsets step C
//               elements).  It first stages the source rows the tile needs,
//               already expanded along the row (window element j holds the
//               source byte for output element e0 - rC + j, or 0 outside a
//               zero border) into LDS.  Each lane then walks down the tile's
//               rows producing 8 consecutive elements per row from its window
//               of 8 + 2rC bytes.  Rows whose K source rows are the same as the
//               previous row's (inside an upsampled block when s > 1) reuse
//               the previous values and only store.
//  k_u8_mix     per-pixel channel mixing (BANK mode with K = 1, e.g. the
//               grayscale weights): up to 4 input and 4 output channels,
//               planar or interleaved, four pixels per lane.
//
// Arithmetic.  Float taps: binary32, accumulator +0, one fused multiply-add
// per term in the order input channel, tap row, tap column.  Integer taps:
// int32 sums (wrapping modulo 2^32).  8-bit outputs: the sum is clamped to
// [0, 255] and rounded to nearest, ties to even.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>

#include "f2d_host.hpp"
#include "f2d_internal.hpp"

namespace f2d {
namespace {

constexpr int kOutI32 = 0;
constexpr int kOutF32 = 1;
constexpr int kOutU8 = 2;

constexpr int kGThreads = 256;
// A lane produces E = 8 or 16 consecutive output elements per row (16 for
// 8-bit outputs of an image upsampled by 8 or more: one 16-byte store per
// lane and row);
// a tile row is 256 E elements, a staged row 256 E + 2rC bytes plus slack.
template <int E>
struct GTile {
  static constexpr int TW = kGThreads * E;
  static constexpr int PITCH_WORDS = (TW + 32) / 4;
};

struct GatherParams {
  const uint8_t* src;  // element (n, c, 0, 0): planar planes, or interleaved rows (stride_c 1)
  int64_t s_sn, s_sc, s_sh;
  void* dst;  // same layout as the source, in elements of the output type
  int64_t d_sn, d_sc, d_sh;
  const void* taps;  // K*K int32 or float
  int64_t H, W;      // source image, pixels
  int64_t Hout, Wout;  // H*s, W*s
  int64_t row0, out_rows;  // output rows [row0, row0 + out_rows) of the (upsampled) buffer
  int32_t s;         // nearest-upsample factor
  uint32_t s_magic;  // division by s: q = (t + ((x - t) >> 1)) >> s_shift, t = mulhi(x, s_magic)
  int32_t s_shift;   // (s >= 2; Granlund and Montgomery's method for invariant divisors)
  int32_t zero;      // zero borders (else clamp-to-edge)
  int32_t planes_c;  // planes per image on the grid: C (planar) or 1 (interleaved)
  int32_t th;        // output rows per tile
  int32_t lds_rows;  // staged source rows per tile (at most); one more zero row follows
  int32_t tiles_x, tiles_y;
  int64_t n_blocks;
  int32_t vec;  // output rows aligned for the lanes' vector stores
};

// x / s for 0 <= x < 2^32 with the launch's invariant-divisor constants
__device__ __forceinline__ uint32_t div_s(uint32_t x, const GatherParams& p) {
  if (p.s == 1) return x;
  const uint32_t t = __umulhi(x, p.s_magic);
  return (t + ((x - t) >> 1)) >> p.s_shift;
}

template <int K, int P, bool TF, int OUT, int E>
__global__ __launch_bounds__(kGThreads) void k_u8_gather(GatherParams p) {
  constexpr int kGElems = E;
  constexpr int kGTW = GTile<E>::TW;
  constexpr int kGPitchWords = GTile<E>::PITCH_WORDS;
  constexpr int R = (K - 1) / 2;
  constexpr int RP = R * P;
  constexpr int WIN = kGTW + 2 * RP;          // staged elements per row
  constexpr int WORDS = (WIN + 3) / 4;
  constexpr int NW = (kGElems + 2 * RP + 3) / 4;  // words of a lane's window
  static_assert(WORDS <= kGPitchWords && (E / 4) * (kGThreads - 1) + NW <= kGPitchWords, "staged row too short");
  extern __shared__ uint32_t lds[];
  using Acc = typename std::conditional<TF, float, uint32_t>::type;
  const int zrow = p.lds_rows;                // an all-zero row for zero borders

  const int tid = threadIdx.x;
  const int64_t b = xcd_remap(blockIdx.x, p.n_blocks);
  const int64_t tiles = static_cast<int64_t>(p.tiles_x) * p.tiles_y;
  const int64_t plane = b / tiles;
  const int64_t t_in = b - plane * tiles;
  const int64_t ty = t_in / p.tiles_x;
  const int64_t tx = t_in - ty * p.tiles_x;
  const int64_t n = plane / p.planes_c;
  const int64_t c = plane - n * p.planes_c;
  const uint8_t* sp = p.src + n * p.s_sn + c * p.s_sc;
  const int64_t e0 = tx * kGTW;               // first output element of the tile
  const int64_t y0 = ty * p.th;               // first output row (band-relative)
  const int64_t L = p.Wout * P;               // elements per output row
  const int64_t nrow_out = min(static_cast<int64_t>(p.th), p.out_rows - y0);

  // source rows the tile reads: the upsampled rows t = row0 + y + u - R,
  // clamped to [0, Hout) (zero-border rows outside are the zero row);
  // indices fit in 32 bits (at most 2^30 rows and elements per row)
  auto clamp_out_row = [&](int64_t t) { return t < 0 ? int64_t{0} : (t >= p.Hout ? p.Hout - 1 : t); };
  const int32_t rlo = static_cast<int32_t>(div_s(static_cast<uint32_t>(clamp_out_row(p.row0 + y0 - R)), p));
  const int32_t rhi =
      static_cast<int32_t>(div_s(static_cast<uint32_t>(clamp_out_row(p.row0 + y0 + nrow_out - 1 + R)), p));
  const int nsrc = rhi - rlo + 1;  // <= lds_rows (host sizing)

  // ---- stage: row-expanded source bytes of every source row of the tile.
  // A thread owns window words tid + 256 k (k < NQ); their source offsets
  // are computed once, then the loads of two source rows for all its words
  // are issued before any of them is written, so a tile pays about nsrc / 2
  // load latencies.  Offsets < 0 are zero-border elements.
  constexpr int NQ = (WORDS + kGThreads - 1) / kGThreads;
  const int32_t wout = static_cast<int32_t>(p.Wout);
  int32_t off[NQ][4];
#pragma unroll
  for (int k = 0; k < NQ; ++k)
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int32_t e = static_cast<int32_t>(e0) - RP + 4 * (tid + kGThreads * k) + jj;  // >= -RP
      const int32_t xu = (e + P * 4) / P - 4;                                          // floor(e / P)
      const int32_t ch = e - xu * P;
      int32_t xc = xu;
      bool inside = xu >= 0 && xu < wout;
      if (!inside && !p.zero) {
        xc = xu < 0 ? 0 : wout - 1;
        inside = true;
      }
      off[k][jj] = inside ? static_cast<int32_t>(div_s(static_cast<uint32_t>(xc), p)) * P + ch : -1;
    }
  // A window word whose four source bytes lie inside one 8-byte stretch of
  // the row (everywhere but zeroed border elements and the row's last bytes:
  // consecutive bytes without upsampling, at most two source pixels with it;
  // clamped edge pixels may repeat earlier offsets) is one or two 4-byte
  // loads from its lowest offset and a byte permute, instead of four byte
  // loads.
  const int32_t row_len = static_cast<int32_t>(p.W) * P;  // bytes of a source row
  bool dw[NQ], two_dw[NQ];
  int32_t dbase[NQ];
  uint32_t sel[NQ];
#pragma unroll
  for (int k = 0; k < NQ; ++k) {
    int32_t lo = off[k][0], hi = off[k][0];
#pragma unroll
    for (int jj = 1; jj < 4; ++jj) {
      lo = off[k][jj] < lo ? off[k][jj] : lo;
      hi = off[k][jj] > hi ? off[k][jj] : hi;
    }
    const int32_t span = hi - lo;
    two_dw[k] = span > 3;
    dw[k] = lo >= 0 && span <= 7 && lo + (two_dw[k] ? 7 : 3) < row_len;
    dbase[k] = lo < 0 ? 0 : lo;
    sel[k] = 0;
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) sel[k] |= static_cast<uint32_t>((off[k][jj] - lo) & 7) << (8 * jj);
  }
  typedef uint32_t u32_unaligned __attribute__((aligned(1)));
  for (int ri = 0; ri < nsrc; ri += 2) {
    const bool two = ri + 1 < nsrc;  // uniform
    const uint8_t* rp0 = sp + static_cast<int64_t>(rlo + ri) * p.s_sh;
    const uint8_t* rp1 = two ? rp0 + p.s_sh : rp0;
    uint32_t b[2][NQ][4];
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
      if (dw[k]) {
        b[0][k][0] = *reinterpret_cast<const u32_unaligned*>(rp0 + dbase[k]);
        b[1][k][0] = *reinterpret_cast<const u32_unaligned*>(rp1 + dbase[k]);
        b[0][k][1] = two_dw[k] ? *reinterpret_cast<const u32_unaligned*>(rp0 + dbase[k] + 4) : 0u;
        b[1][k][1] = two_dw[k] ? *reinterpret_cast<const u32_unaligned*>(rp1 + dbase[k] + 4) : 0u;
      } else {
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
          const int32_t o = off[k][jj] < 0 ? 0 : off[k][jj];
          b[0][k][jj] = rp0[o];
          b[1][k][jj] = rp1[o];
        }
      }
    }
#pragma unroll
    for (int k = 0; k < NQ; ++k) {
      const int q = tid + kGThreads * k;
      if (q >= WORDS) continue;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        uint32_t w = 0;
        if (dw[k]) {
          w = __builtin_amdgcn_perm(b[h][k][1], b[h][k][0], sel[k]);  // bytes 0-3: first load, 4-7: second
        } else {
#pragma unroll
          for (int jj = 0; jj < 4; ++jj)
            if (off[k][jj] >= 0) w |= b[h][k][jj] << (8 * jj);
        }
        if (h == 0 || two) lds[(ri + h) * kGPitchWords + q] = w;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < NQ; ++k)
    if (tid + kGThreads * k < WORDS) lds[zrow * kGPitchWords + tid + kGThreads * k] = 0u;
  __syncthreads();

  // ---- taps (uniform)
  Acc tap[K * K];
#pragma unroll
  for (int i = 0; i < K * K; ++i) tap[i] = static_cast<const Acc*>(p.taps)[i];

  // ---- walk the rows.  Tap row u of output row y reads upsampled row
  // t = row0 + y + u - R, i.e. source row q_u with t = q_u s + m_u; (q_u, m_u)
  // advance with y, so no division is needed inside the loop.
  int32_t qd[K], md[K];
#pragma unroll
  for (int u = 0; u < K; ++u) {
    const int64_t t = p.row0 + y0 + u - R;  // >= -R
    const uint32_t tp = static_cast<uint32_t>(t + 4 * p.s);  // shifted to stay non-negative
    qd[u] = static_cast<int32_t>(div_s(tp, p)) - 4;
    md[u] = static_cast<int32_t>(t - static_cast<int64_t>(qd[u]) * p.s);
  }
  const int32_t hlast = static_cast<int32_t>(p.H - 1);
  int32_t prev[K];
#pragma unroll
  for (int u = 0; u < K; ++u) prev[u] = -1;
  uint32_t outw[OUT == kOutU8 ? E / 4 : kGElems];
  const int64_t ebase = e0 + kGElems * tid;
  for (int64_t i = 0; i < nrow_out; ++i) {
    const int64_t y = y0 + i;
    int32_t ridx[K];
    bool same = i > 0;
#pragma unroll
    for (int u = 0; u < K; ++u) {
      const int64_t t = p.row0 + y + u - R;
      int32_t r;
      if (t < 0)
        r = p.zero ? zrow : -rlo;
      else if (t >= p.Hout)
        r = p.zero ? zrow : hlast - rlo;
      else
        r = qd[u] - rlo;
      ridx[u] = r;
      same = same && r == prev[u];
      prev[u] = r;
      if (++md[u] == p.s) {
        md[u] = 0;
        ++qd[u];
      }
    }
    if (!same) {
      Acc acc[kGElems];
#pragma unroll
      for (int j = 0; j < kGElems; ++j) acc[j] = Acc(0);
#pragma unroll
      for (int u = 0; u < K; ++u) {
        const uint32_t* row = lds + ridx[u] * kGPitchWords + (E / 4) * tid;
        uint32_t w[NW];
#pragma unroll
        for (int k2 = 0; k2 < NW; ++k2) w[k2] = row[k2];
#pragma unroll
        for (int v = 0; v < K; ++v)
#pragma unroll
          for (int j = 0; j < kGElems; ++j) {
            const int bi = j + v * P;
            const uint32_t byte = (w[bi >> 2] >> (8 * (bi & 3))) & 0xffu;
            if constexpr (TF)
              acc[j] = __builtin_fmaf(tap[u * K + v], static_cast<float>(byte), acc[j]);
            else
              acc[j] += byte * tap[u * K + v];
          }
      }
      if constexpr (OUT == kOutU8) {
        uint32_t q8[kGElems];
#pragma unroll
        for (int j = 0; j < kGElems; ++j) {
          if constexpr (TF) {
            const float v = __builtin_rintf(__builtin_amdgcn_fmed3f(acc[j], 0.0f, 255.0f));
            q8[j] = static_cast<uint32_t>(v);
          } else {
            const int32_t v = static_cast<int32_t>(acc[j]);
            q8[j] = static_cast<uint32_t>(v < 0 ? 0 : (v > 255 ? 255 : v));
          }
        }
#pragma unroll
        for (int w4 = 0; w4 < E / 4; ++w4)
          outw[w4] = q8[4 * w4] | (q8[4 * w4 + 1] << 8) | (q8[4 * w4 + 2] << 16) | (q8[4 * w4 + 3] << 24);
      } else {
#pragma unroll
        for (int j = 0; j < kGElems; ++j) outw[j] = __builtin_bit_cast(uint32_t, acc[j]);
      }
    }
    // ---- store the lane's 8 elements of row y
    if (ebase < L) {
      if constexpr (OUT == kOutU8) {
        uint8_t* dp = static_cast<uint8_t*>(p.dst) + n * p.d_sn + c * p.d_sc + y * p.d_sh + ebase;
        if (p.vec && ebase + kGElems <= L) {
          if constexpr (E == 16)
            *reinterpret_cast<uint4*>(dp) = make_uint4(outw[0], outw[1], outw[2], outw[3]);
          else
            *reinterpret_cast<uint2*>(dp) = make_uint2(outw[0], outw[1]);
        } else {
#pragma unroll
          for (int j = 0; j < kGElems; ++j)
            if (ebase + j < L) dp[j] = static_cast<uint8_t>(outw[j >> 2] >> (8 * (j & 3)));
        }
      } else {
        uint32_t* dp = static_cast<uint32_t*>(p.dst) + n * p.d_sn + c * p.d_sc + y * p.d_sh + ebase;
        if (p.vec && ebase + kGElems <= L) {
#pragma unroll
          for (int w4 = 0; w4 < E / 4; ++w4)
            reinterpret_cast<uint4*>(dp)[w4] =
                make_uint4(outw[4 * w4], outw[4 * w4 + 1], outw[4 * w4 + 2], outw[4 * w4 + 3]);
        } else {
#pragma unroll
          for (int j = 0; j < kGElems; ++j)
            if (ebase + j < L) dp[j] = outw[j];
        }
      }
    }
  }
}

// ------------------------------------------------------------- channel mix --

struct MixParams {
  const uint8_t* src;
  int64_t s_sn, s_sc, s_sh, s_sw;  // elements; interleaved: s_sc = 1, s_sw = CIN
  void* dst;
  int64_t d_sn, d_sc, d_sh, d_sw;  // elements of the output type
  const void* w;                   // [cout][CIN], int32 or float
  int32_t cout;
  int64_t W, row0, rows;  // output rows [row0, row0 + rows) of the buffer
  int32_t tiles_x;        // 1024-pixel segments per row
  int64_t n_blocks;
  int32_t in_vec;   // source rows word-aligned (planar) / interleaved rows word-aligned
  int32_t out_vec;  // output planes rows aligned for 4-pixel stores (planar output)
};

constexpr int kMixThreads = 256;
constexpr int kMixPx = 16;  // pixels per lane (measured: 8K gray 0.048 ms with 4)

template <int CIN, bool TF, int OUT>
__global__ __launch_bounds__(kMixThreads) void k_u8_mix(MixParams p) {
  using Acc = typename std::conditional<TF, float, uint32_t>::type;
  const int64_t b = xcd_remap(blockIdx.x, p.n_blocks);
  const int64_t per_img = p.rows * p.tiles_x;
  const int64_t n = b / per_img;
  const int64_t rem = b - n * per_img;
  const int64_t y = rem / p.tiles_x;
  const int64_t x0 = (rem - y * p.tiles_x) * (kMixThreads * kMixPx) + kMixPx * threadIdx.x;
  if (x0 >= p.W) return;
  const bool full = x0 + kMixPx <= p.W;
  const uint8_t* rp = p.src + n * p.s_sn + (p.row0 + y) * p.s_sh;

  // x[i][k]: channel i of pixel x0 + k
  uint32_t x[CIN][kMixPx];
  if (p.s_sw == CIN && p.s_sc == 1 && CIN > 1) {  // interleaved
    if (p.in_vec && full) {
      uint32_t wd[CIN * kMixPx / 4];
#pragma unroll
      for (int q = 0; q < CIN * kMixPx / 4; ++q) wd[q] = reinterpret_cast<const uint32_t*>(rp + x0 * CIN)[q];
#pragma unroll
      for (int k = 0; k < kMixPx; ++k)
#pragma unroll
        for (int i = 0; i < CIN; ++i) {
          const int bi = k * CIN + i;
          x[i][k] = (wd[bi >> 2] >> (8 * (bi & 3))) & 0xffu;
        }
    } else {
#pragma unroll
      for (int k = 0; k < kMixPx; ++k)
#pragma unroll
        for (int i = 0; i < CIN; ++i) x[i][k] = x0 + k < p.W ? rp[(x0 + k) * CIN + i] : 0u;
    }
  } else {  // planar
#pragma unroll
    for (int i = 0; i < CIN; ++i) {
      const uint8_t* cp = rp + i * p.s_sc;
      if (p.in_vec && full) {
        uint32_t wd[kMixPx / 4];
#pragma unroll
        for (int q = 0; q < kMixPx / 4; ++q) wd[q] = reinterpret_cast<const uint32_t*>(cp + x0)[q];
#pragma unroll
        for (int k = 0; k < kMixPx; ++k) x[i][k] = (wd[k >> 2] >> (8 * (k & 3))) & 0xffu;
      } else {
#pragma unroll
        for (int k = 0; k < kMixPx; ++k) x[i][k] = x0 + k < p.W ? cp[(x0 + k) * p.s_sw] : 0u;
      }
    }
  }

  const Acc* w = static_cast<const Acc*>(p.w);
#pragma unroll
  for (int o = 0; o < 4; ++o) {
    if (o >= p.cout) break;
    Acc acc[kMixPx];
#pragma unroll
    for (int k = 0; k < kMixPx; ++k) acc[k] = Acc(0);
#pragma unroll
    for (int i = 0; i < CIN; ++i) {
      const Acc wi = w[o * CIN + i];
#pragma unroll
      for (int k = 0; k < kMixPx; ++k) {
        if constexpr (TF)
          acc[k] = __builtin_fmaf(wi, static_cast<float>(x[i][k]), acc[k]);
        else
          acc[k] += x[i][k] * wi;
      }
    }
    const int64_t obase = n * p.d_sn + o * p.d_sc + (y)*p.d_sh;
    if constexpr (OUT == kOutU8) {
      uint32_t q8[kMixPx];
#pragma unroll
      for (int k = 0; k < kMixPx; ++k) {
        if constexpr (TF) {
          q8[k] = static_cast<uint32_t>(__builtin_rintf(__builtin_amdgcn_fmed3f(acc[k], 0.0f, 255.0f)));
        } else {
          const int32_t v = static_cast<int32_t>(acc[k]);
          q8[k] = static_cast<uint32_t>(v < 0 ? 0 : (v > 255 ? 255 : v));
        }
      }
      uint8_t* dp = static_cast<uint8_t*>(p.dst) + obase;
      if (p.out_vec && full && p.d_sw == 1) {
#pragma unroll
        for (int q = 0; q < kMixPx / 4; ++q)
          reinterpret_cast<uint32_t*>(dp + x0)[q] =
              q8[4 * q] | (q8[4 * q + 1] << 8) | (q8[4 * q + 2] << 16) | (q8[4 * q + 3] << 24);
      } else {
#pragma unroll
        for (int k = 0; k < kMixPx; ++k)
          if (x0 + k < p.W) dp[(x0 + k) * p.d_sw] = static_cast<uint8_t>(q8[k]);
      }
    } else {
      uint32_t* dp = static_cast<uint32_t*>(p.dst) + obase;
      if (p.out_vec && full && p.d_sw == 1) {
#pragma unroll
        for (int q = 0; q < kMixPx / 4; ++q)
          reinterpret_cast<uint4*>(dp + x0)[q] =
              make_uint4(__builtin_bit_cast(uint32_t, acc[4 * q]), __builtin_bit_cast(uint32_t, acc[4 * q + 1]),
                         __builtin_bit_cast(uint32_t, acc[4 * q + 2]), __builtin_bit_cast(uint32_t, acc[4 * q + 3]));
      } else {
#pragma unroll
        for (int k = 0; k < kMixPx; ++k)
          if (x0 + k < p.W) dp[(x0 + k) * p.d_sw] = __builtin_bit_cast(uint32_t, acc[k]);
      }
    }
  }
}

// ------------------------------------------------------------------ host ----

int64_t eff_sw(const f2d_tensor& t) { return t.stride_w <= 0 ? 1 : t.stride_w; }

// Interleaved: channels adjacent (stride_c 1) and pixels C apart, C > 1.
bool interleaved(const f2d_tensor& t) { return t.c > 1 && t.stride_c == 1 && eff_sw(t) == t.c; }

// Row starts aligned to `bytes` (base pointer, row and image strides); the
// channel stride is ignored for interleaved tensors, whose channels sit
// inside the pixel.
bool rows_aligned(const f2d_tensor& t, size_t bytes) {
  if (!interleaved(t)) return row_aligned(t, bytes);
  const size_t es = t.dtype == F2D_U8 ? 1 : 4;
  const uintptr_t a = reinterpret_cast<uintptr_t>(t.data);
  return a % bytes == 0 && (t.h <= 1 || (t.stride_h * es) % bytes == 0) &&
         (t.n <= 1 || (t.stride_n * es) % bytes == 0);
}

template <int K, int P, bool TF, int OUT, int E>
hipError_t launch_gather_one(const GatherParams& g, hipStream_t s) {
  const void* kern = reinterpret_cast<const void*>(k_u8_gather<K, P, TF, OUT, E>);
  const size_t lds = static_cast<size_t>(g.lds_rows + 1) * GTile<E>::PITCH_WORDS * 4;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_u8_gather<K, P, TF, OUT, E>), dim3(static_cast<uint32_t>(g.n_blocks)), dim3(kGThreads), lds,
                     s, g);
  return hipGetLastError();
}

// 16 elements per lane for 8-bit outputs of images upsampled by 8 or more, else 8
template <int K, int P>
hipError_t launch_gather_kp(const GatherParams& g, bool tf, int out, int e, hipStream_t s) {
  if (out == kOutU8) {
    if (e == 16)
      return tf ? launch_gather_one<K, P, true, kOutU8, 16>(g, s) : launch_gather_one<K, P, false, kOutU8, 16>(g, s);
    return tf ? launch_gather_one<K, P, true, kOutU8, 8>(g, s) : launch_gather_one<K, P, false, kOutU8, 8>(g, s);
  }
  return tf ? launch_gather_one<K, P, true, kOutF32, 8>(g, s) : launch_gather_one<K, P, false, kOutI32, 8>(g, s);
}

template <int K>
hipError_t launch_gather_k(const GatherParams& g, int P, bool tf, int out, int e, hipStream_t s) {
  switch (P) {
    case 1: return launch_gather_kp<K, 1>(g, tf, out, e, s);
    case 3: return launch_gather_kp<K, 3>(g, tf, out, e, s);
    default: return launch_gather_kp<K, 4>(g, tf, out, e, s);
  }
}

int out_kind(int32_t dtype) { return dtype == F2D_U8 ? kOutU8 : (dtype == F2D_F32 ? kOutF32 : kOutI32); }

// SHARED filter on an 8-bit image, optional nearest upsample by `scale`.
f2d_status gather_forward(const Problem& pr, const f2d_tensor& out, int32_t scale, hipStream_t s) {
  const f2d_tensor& im = pr.image;
  const bool il = interleaved(im);
  if (!il && eff_sw(im) != 1) return fail(F2D_EUNSUPPORTED, "u8 images: planar or interleaved (stride_c 1, stride_w C) layouts");
  const int P = il ? static_cast<int>(im.c) : 1;
  if (il && P != 3 && P != 4) return fail(F2D_EUNSUPPORTED, "interleaved u8 images: 3 or 4 channels");
  if (il != interleaved(out) || (!il && eff_sw(out) != 1))
    return fail(F2D_EINVAL, "the output must have the image's layout (planar, or interleaved with the same channels)");
  if (pr.k > 7) return fail(F2D_EUNSUPPORTED, "u8 zero-border / u8-output / float-tap / upsampled filters: k <= 7 (got %d)", pr.k);
  const bool tf = pr.filter.dtype == F2D_F32;
  const int ok_out = out_kind(out.dtype);
  if ((tf && ok_out == kOutI32) || (!tf && ok_out == kOutF32))
    return fail(F2D_EINVAL, "u8 images: int32 taps give int32 or u8 outputs, float taps give f32 or u8 outputs");
  GatherParams g;
  std::memset(&g, 0, sizeof(g));
  g.src = static_cast<const uint8_t*>(im.data);
  g.s_sn = im.stride_n;
  g.s_sc = il ? 0 : im.stride_c;
  g.s_sh = im.stride_h;
  g.dst = out.data;
  g.d_sn = out.stride_n;
  g.d_sc = il ? 0 : out.stride_c;
  g.d_sh = out.stride_h;
  g.taps = pr.filter.data;
  g.H = im.h;
  g.W = im.w;
  g.s = scale;
  g.Hout = im.h * scale;
  g.Wout = im.w * scale;
  g.row0 = pr.row_begin;
  g.out_rows = scale == 1 ? pr.rows : g.Hout;
  g.zero = pr.opts.border == F2D_BORDER_ZERO ? 1 : 0;
  g.planes_c = il ? 1 : static_cast<int32_t>(im.c);
  const int64_t L = g.Wout * P;
  if (L > (int64_t{1} << 30) || g.Hout > (int64_t{1} << 30))
    return fail(F2D_EUNSUPPORTED, "u8 filter: output rows of at most 2^30 elements and 2^30 rows");
  // Tile height: 16 rows without upsampling; with it, about 8 source rows
  // per tile (rows inside an upsampled block repeat, so the work per tile is
  // set by its source rows), at most 512 rows.  LDS holds the tile's source
  // rows: at most (th + 2r - 1) / s + 2 of them.
  const int R = (pr.k - 1) / 2;
  g.th = scale == 1 ? 16 : static_cast<int32_t>(std::min<int64_t>(512, 8 * static_cast<int64_t>(scale)));
  g.lds_rows = std::min(g.th + 2 * R, (g.th + 2 * R - 1) / scale + 2);
  if (scale > 1) {
    int l = 0;
    while ((int64_t{1} << l) < scale) ++l;
    g.s_shift = l - 1;
    g.s_magic = static_cast<uint32_t>((((uint64_t{1} << 32) * ((uint64_t{1} << l) - scale)) / scale) + 1);
  }
  // 16-byte stores measured faster at x20 (1.93 against 2.28 ms on a 4K frame), 8-byte ones at x2 and x4
  const int elems = ok_out == kOutU8 && scale >= 8 ? 16 : 8;
  const int64_t tw = static_cast<int64_t>(kGThreads) * elems;
  g.tiles_x = static_cast<int32_t>((L + tw - 1) / tw);
  g.tiles_y = static_cast<int32_t>((g.out_rows + g.th - 1) / g.th);
  g.n_blocks = im.n * g.planes_c * static_cast<int64_t>(g.tiles_x) * g.tiles_y;
  if (g.n_blocks > kMaxBlocks) return fail(F2D_EUNSUPPORTED, "u8 filter: too many tiles for one launch");
  g.vec = rows_aligned(out, ok_out == kOutU8 ? static_cast<size_t>(elems) : 16) ? 1 : 0;
  if (g.n_blocks == 0) return ok();
  hipError_t err;
  switch (pr.k) {
    case 1: err = launch_gather_k<1>(g, P, tf, ok_out, elems, s); break;
    case 3: err = launch_gather_k<3>(g, P, tf, ok_out, elems, s); break;
    case 5: err = launch_gather_k<5>(g, P, tf, ok_out, elems, s); break;
    default: err = launch_gather_k<7>(g, P, tf, ok_out, elems, s); break;
  }
  return hip_status(err, "u8 filter launch");
}

template <int CIN>
hipError_t launch_mix_c(const MixParams& m, bool tf, int out, hipStream_t s) {
  const dim3 grid(static_cast<uint32_t>(m.n_blocks)), block(kMixThreads);
  if (tf) {
    if (out == kOutU8) hipLaunchKernelGGL((k_u8_mix<CIN, true, kOutU8>), grid, block, 0, s, m);
    else hipLaunchKernelGGL((k_u8_mix<CIN, true, kOutF32>), grid, block, 0, s, m);
  } else {
    if (out == kOutU8) hipLaunchKernelGGL((k_u8_mix<CIN, false, kOutU8>), grid, block, 0, s, m);
    else hipLaunchKernelGGL((k_u8_mix<CIN, false, kOutI32>), grid, block, 0, s, m);
  }
  return hipGetLastError();
}

// BANK with K = 1 on an 8-bit image: per-pixel channel mixing.
f2d_status mix_forward(const Problem& pr, const f2d_tensor& out, hipStream_t s) {
  const f2d_tensor& im = pr.image;
  if (pr.k != 1) return fail(F2D_EUNSUPPORTED, "u8 images in BANK mode: k = 1 (per-pixel channel mixing) only");
  if (im.c > 4 || pr.c_out > 4) return fail(F2D_EUNSUPPORTED, "u8 channel mixing: at most 4 input and 4 output channels");
  const bool il = interleaved(im);
  if (!il && eff_sw(im) != 1) return fail(F2D_EUNSUPPORTED, "u8 images: planar or interleaved layouts");
  const bool oil = interleaved(out);
  if (!oil && eff_sw(out) != 1) return fail(F2D_EUNSUPPORTED, "u8 channel mixing: planar or interleaved outputs");
  const bool tf = pr.filter.dtype == F2D_F32;
  const int ok_out = out_kind(out.dtype);
  if ((tf && ok_out == kOutI32) || (!tf && ok_out == kOutF32))
    return fail(F2D_EINVAL, "u8 images: int32 weights give int32 or u8 outputs, float weights give f32 or u8 outputs");
  MixParams m;
  std::memset(&m, 0, sizeof(m));
  m.src = static_cast<const uint8_t*>(im.data);
  m.s_sn = im.stride_n;
  m.s_sc = im.stride_c;
  m.s_sh = im.stride_h;
  m.s_sw = eff_sw(im);
  m.dst = out.data;
  m.d_sn = out.stride_n;
  m.d_sc = out.stride_c;
  m.d_sh = out.stride_h;
  m.d_sw = eff_sw(out);
  m.w = pr.filter.data;
  m.cout = static_cast<int32_t>(pr.c_out);
  m.W = im.w;
  m.row0 = pr.row_begin;
  m.rows = pr.rows;
  m.tiles_x = static_cast<int32_t>((im.w + kMixThreads * kMixPx - 1) / (kMixThreads * kMixPx));
  m.n_blocks = im.n * m.rows * m.tiles_x;
  if (m.n_blocks > kMaxBlocks) return fail(F2D_EUNSUPPORTED, "u8 channel mixing: too many tiles for one launch");
  m.in_vec = rows_aligned(im, 4) ? 1 : 0;
  m.out_vec = !oil && row_aligned(out, ok_out == kOutU8 ? 4 : 16) ? 1 : 0;
  if (m.n_blocks == 0) return ok();
  hipError_t e;
  switch (im.c) {
    case 1: e = launch_mix_c<1>(m, tf, ok_out, s); break;
    case 2: e = launch_mix_c<2>(m, tf, ok_out, s); break;
    case 3: e = launch_mix_c<3>(m, tf, ok_out, s); break;
    default: e = launch_mix_c<4>(m, tf, ok_out, s); break;
  }
  return hip_status(e, "u8 channel mixing launch");
}

}  // namespace

// 8-bit images beyond the integer Sobel path: zero borders, float taps, u8
// outputs, interleaved layouts (SHARED), and channel mixing (BANK, K = 1).
f2d_status forward_u8_image(const Problem& pr, const f2d_tensor* outs, int32_t n_outs, hipStream_t s) {
  if (pr.mode == F2D_CH_DEPTHWISE)
    return fail(F2D_EUNSUPPORTED, "u8 DEPTHWISE filters: int32 taps, int32 outputs, clamp borders, planar layout");
  if (n_outs != 1) return fail(F2D_EINVAL, "expected one output");
  if (pr.mode == F2D_CH_BANK) return mix_forward(pr, outs[0], s);
  return gather_forward(pr, outs[0], 1, s);
}

f2d_status run_upsample_forward(const Problem& pr, int32_t scale, const f2d_tensor& out, hipStream_t s) {
  if (pr.image.n == 0 || pr.image.h == 0 || pr.image.w == 0 || pr.image.c == 0) return ok();
  return gather_forward(pr, out, scale, s);
}

}  // namespace f2d
