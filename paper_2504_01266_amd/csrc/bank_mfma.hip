// BF16 filter banks on the gfx950 matrix cores (FP32 accumulation).
//
// A bank Y[n][o] = sum_i corr(X[n][i], W[o][i]) is an implicit GEMM: for
// every output pixel p and output channel o, Y[p][o] = sum_k A[p][k] * B[k][o]
// with the contraction index k = (tap (u,v), input channel i), A = the K*K
// neighbourhood of p (never materialised: it is read from an LDS tile with
// its clamped halo) and B = the weights.  k is ordered tap-major,
// channel-minor, so one 8-element MFMA operand slice is 8 consecutive
// channels of one pixel, i.e. 16 contiguous bytes of the channels-last tile.
//
//  k_bank_conv   v_mfma_f32_16x16x32_bf16.  A persistent work-group keeps
//                the weights of its current output group (all taps x channels
//                of OT*16 output channels) in LDS and walks 4 x (16*PT)-pixel
//                tiles; the next tile's global loads are in flight during the
//                MFMA sweeps and, with two tile buffers, are packed into the
//                idle one between the MFMA groups of the last steps.  Each
//                wave owns a share of one tile row and sweeps k once per
//                32-channel pass.  Forward: clamp-to-edge borders.  Adjoint
//                in the image (dgrad): zero borders and the transposed,
//                flipped weights, evaluated on the image plus an r-wide frame
//                whose values are then folded onto the edge pixels (the exact
//                clamp adjoint).  Upstream gradients given in FP32 are rounded
//                to BF16 (nearest even) while staged.
//  k_bank_conv_ring  the same for 33..64 source channels: a work-group walks
//                down a column segment keeping the staged rows as a ring, so
//                every tile after the first stages only its 4 new rows.
//  k_bank_conv_vr  33..64 source channels into at most 16 outputs (the dgrad
//                of the 16 -> 64 bank): weights in registers, and each pixel
//                operand read from LDS feeds the MFMAs of every tile row it
//                reaches (0.4 operand reads per MFMA at K = 5 against 1.5).
//  k_bank_conv_ws  the forward from 9..16 to 33..64 channels with BF16 outputs,
//                with the memory traffic on separate waves: MFMA waves read LDS only,
//                memory waves stage tiles and store results from LDS.
//  k_bank_wgrad  W-bar[o][i][u][v] = sum_p G[o][p] * X[i][shift_uv(p)]: for
//                every tap a 16(o) x 16(i) block contracted over 32-pixel
//                steps; each staged X row is read once as a window and the
//                K horizontal shifts are built with 16-bit funnel shifts.
//                Per-unit partials go to the workspace and are reduced in a
//                fixed order.
#include <hip/hip_bf16.h>
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>
#include <type_traits>

#include "f2d_host.hpp"
#include "f2d_internal.hpp"
#include "grad_internal.hpp"

namespace f2d {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

constexpr int kThreads = 256;      // wgrad work-group
constexpr int kTH = 4;             // conv tile rows

// f(integral_constant<int, 0>) ... f(integral_constant<int, N-1>), in order
template <int N, int I = 0, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    static_for<N, I + 1>(f);
  }
}

struct BankParams {
  const void* src;  // source planes: X (bf16) or, for the adjoint, G-bar (bf16 or f32)
  int64_t s_sn, s_sc, s_sh;
  void* dst;  // output planes (f32, or bf16 for a bf16 forward output)
  int64_t d_sn, d_sc, d_sh;
  const uint16_t* w;  // forward weights [fo][fi][K][K], bf16 bits
  int64_t H, W, row0, rows;
  int32_t CI, CO;  // channels of the source and of the output of THIS map
  int32_t fo, fi;  // forward weight extents
  int32_t tiles_x, tiles_y, o_groups;
  int64_t n_tiles;  // N * o_groups * tiles_y * tiles_x
  int64_t n_img, cols;  // images, and output columns from col0 to cover (tiles_x from the tile width)
  // row-ring kernel: segments of seg_len tile rows, seg_per_col per tile column
  int64_t n_segs;
  int32_t seg_per_col, seg_len;
  // adjoint: output rows start at row0 = -r and columns at col0 <= -r (4-aligned); values
  // on the r-wide frame go to `frame` (frame_plane floats per output plane)
  int64_t col0;
  float* frame;
  int64_t frame_plane;
  int32_t fr;
  int32_t d_vec;  // output rows and planes 16-byte (f32) / 8-byte (bf16) aligned
  int32_t s_vec;  // source rows and planes 16-byte aligned and W % 8 == 0 (vector staging)
  int32_t s_plan32;  // s_vec, and one image of the source spans < 2^31 elements with H, s_sh < 2^24
};

// FP32 -> BF16, round to nearest even (NaN stays NaN): the gfx950 packed
// conversion instruction, one per pair of values.
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t pack_bf16x2(float lo, float hi) {
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{lo, hi}, bf16x2));
}
__device__ __forceinline__ uint16_t f32_to_bf16_bits(float f) {
  return __builtin_bit_cast(uint16_t, static_cast<__bf16>(f));
}

template <typename TS>
__device__ __forceinline__ uint16_t load_bits(const TS* p);
template <>
__device__ __forceinline__ uint16_t load_bits<uint16_t>(const uint16_t* p) {
  return *p;
}
template <>
__device__ __forceinline__ uint16_t load_bits<float>(const float* p) {
  return f32_to_bf16_bits(*p);
}

// Conv work-group of NW waves (4, 8 or 16) over a kTH x TW tile: NW/kTH
// waves per tile row, each with HP 16-pixel blocks.  Groups of eight or more
// waves may use all of LDS; four-wave groups stay within half of it so that
// two fit on a CU.
template <int K, int OT, int PT, int CG, int NW>
struct ConvGeom {
  static constexpr int THREADS = 64 * NW;
  static constexpr int WPR = NW / kTH;               // waves per tile row
  static constexpr int HP = PT / WPR;                // 16-pixel blocks per wave
  static constexpr int LDS_CAP = NW >= 8 ? 160 * 1024 : 80 * 1024;
  static constexpr int R = (K - 1) / 2;
  static constexpr int CI8 = CG * 8;         // staged channels (padded)
  static constexpr int KG = K * K * CG;      // 8-wide k-groups
  static constexpr int STEPS = (KG + 3) / 4; // 32-wide MFMA steps
  static constexpr int KP = STEPS * 32;
  // LDS strides.  A ds_read_b128 is served in two halves of 32 lanes, each
  // over a 512-byte bank window: the 32 accesses of a half must fall in 32
  // distinct 16-byte slots mod 512 bytes.  MFMA operand reads put 16 rows
  // (weight rows, or pixels) at a fixed stride and two 16-byte k-groups per
  // half; both are conflict-free when the row stride is an odd multiple of
  // 32 bytes (the 16 rows then take every even slot, the second k-group
  // every odd one).  KP*2 bytes is a multiple of 64, so 32 bytes are added.
  static constexpr int WSTR = KP + 16;       // weight row stride (elements)
  static constexpr int TW = 16 * PT;
  static constexpr int LH = kTH + K - 1;
  // staged columns x0-8 .. x0+TW+7: 16-byte aligned 8-column chunks (R <= 8);
  // output pixel px, tap column v reads LDS column px + XOFF + v
  static constexpr int LW = TW + 16;
  static constexpr int XOFF = 8 - R;
  static constexpr int CHUNKS = LW / 8;
  // channels-last pixel stride (elements): an odd multiple of 32 bytes where
  // that keeps two source buffers in LDS (see WSTR; with CG = 1 the four
  // quarters read four taps and no stride avoids every conflict), else the
  // smallest 16-byte-padded stride
  static constexpr int PS_CF = CG == 2 ? 16 : (CG == 1 ? 16 : CI8 + 16);
  static constexpr int PS_MIN = CI8 + 8;
  static constexpr int W_ELEMS = OT * 16 * WSTR;
  static constexpr bool fits2(int ps) { return (W_ELEMS + 2 * LH * LW * ps) * 2 <= LDS_CAP; }
  // 33..64 source channels: one tile, kept as a row ring (k_bank_conv_ring)
  // of LH rows, or of LH + kTH rows where those fit beside the weights (then
  // the next tile's rows are packed while the current one computes)
  static constexpr bool RINGED = CG == 8 && NW == 8;
  static constexpr int PS = RINGED || fits2(PS_CF) || !fits2(PS_MIN) ? PS_CF : PS_MIN;
  static constexpr int NSLOT =
      RINGED && (W_ELEMS + (LH + kTH) * LW * PS) * 2 <= 160 * 1024 ? LH + kTH : LH;
  static constexpr int S_ELEMS = NSLOT * LW * PS;   // one source tile or the ring (16-byte multiple)
  // weights + two source tiles when they fit in the LDS share, else one
  static constexpr int NBUF = !RINGED && fits2(PS) ? 2 : 1;
  static constexpr int LDS_ELEMS = W_ELEMS + NBUF * S_ELEMS;
  // staging units (row, channel group, 8-column chunk), 8 per wave instruction
  static constexpr int UNITS = LH * CG * CHUNKS;
  static constexpr int NT = (UNITS + 8 * NW - 1) / (8 * NW);  // per wave
  static_assert(R <= 8, "K <= 17");
  static_assert(NW % kTH == 0 && PT % WPR == 0, "tile split");
};

// Staging of the source tile, channels-last.  A unit = (row ly, channel
// group cg, 8-column chunk) is handled by the 8 lanes u + 8j of the wave
// (u = lane & 7 picks the unit of the instruction, j = lane >> 3): lane j
// loads the chunk's 8 pixels of channel cg*8 + j (one 16-byte load in the
// interior, clamped element loads at the left and right image edges; the 8
// lanes of one j read 8 neighbouring chunks, 128 contiguous bytes), and after
// an 8 x 8 transpose across the unit's lanes it holds the 8 channels of pixel
// j, which it writes as one 16-byte LDS store.  Loads always use valid addresses; the
// border rule (clamp, or zero for the adjoint) and the channel padding are
// applied to the values.
// SW waves share the staging of NR tile rows; staging_nt: unit rounds per wave
template <typename G, int SW, int NR = G::LH>
constexpr int staging_nt() {
  return (NR * (G::UNITS / G::LH) + 8 * SW - 1) / (8 * SW);
}

template <typename G, int CG, int SW, int NR = G::LH>
__device__ __forceinline__ void unit_pos(int it, int wave, int lane, int& ly, int& cg, int& chunk, bool& act) {
  const int u = (it * SW + wave) * 8 + (lane & 7);
  act = u < NR * (G::UNITS / G::LH);
  const int uu = act ? u : 0;
  chunk = uu % G::CHUNKS;
  const int rest = uu / G::CHUNKS;
  cg = rest % CG;
  ly = rest / CG;
}

// Raw staged values of one tile for this wave: 8 consecutive pixels of one
// channel per unit (bf16 pairs, or f32 rounded to bf16 when packed).  The
// transpose and LDS write happen only in stage_store, after the MFMA loop,
// so interior loads stay in flight while the matrix cores work.
template <typename TS, int NT>
struct Raw;
template <int NT>
struct Raw<uint16_t, NT> {
  u32x4 v[NT];
  __device__ __forceinline__ u32x4 pairs(int it) const { return v[it]; }
};
template <int NT>
struct Raw<float, NT> {
  float v[NT][8];
  __device__ __forceinline__ u32x4 pairs(int it) const {
    u32x4 r;
#pragma unroll
    for (int d = 0; d < 4; ++d)
      r[d] = pack_bf16x2(v[it][2 * d], v[it][2 * d + 1]);
    return r;
  }
};

// 8 consecutive elements from a 16-byte aligned address
__device__ __forceinline__ void load_vec(const uint16_t* a, u32x4& out) { out = *reinterpret_cast<const u32x4*>(a); }
__device__ __forceinline__ void load_vec(const float* a, float (&out)[8]) {
  const float4 x = reinterpret_cast<const float4*>(a)[0];
  const float4 y = reinterpret_cast<const float4*>(a)[1];
  out[0] = x.x;
  out[1] = x.y;
  out[2] = x.z;
  out[3] = x.w;
  out[4] = y.x;
  out[5] = y.y;
  out[6] = y.z;
  out[7] = y.w;
}

// 8 consecutive elements of a row starting at column gx0 from element loads
// at clamped columns (zero outside the row for the adjoint): unaligned rows
// or widths that are not a multiple of 8.
template <bool ADJ>
__device__ __forceinline__ void load_chunk(const uint16_t* row, int64_t gx0, int64_t W, u32x4& out) {
  {
    uint32_t h[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int64_t x = gx0 + e;
      const int64_t cx = x < 0 ? 0 : (x >= W ? W - 1 : x);
      const uint32_t v = row[cx];
      h[e] = (ADJ && (x < 0 || x >= W)) ? 0u : v;
    }
    out = u32x4{h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16)};
  }
}
template <bool ADJ>
__device__ __forceinline__ void load_chunk(const float* row, int64_t gx0, int64_t W, float (&out)[8]) {
  {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int64_t x = gx0 + e;
      const int64_t cx = x < 0 ? 0 : (x >= W ? W - 1 : x);
      const float v = row[cx];
      out[e] = (ADJ && (x < 0 || x >= W)) ? 0.0f : v;
    }
  }
}

// Loads for tile rows ly0 .. ly0+NR-1 (of the LH staged rows) of the tile at
// (oy0, ox0).
template <typename G, int K, int CG, bool ADJ, typename TS, int SW = G::THREADS / 64, int NR = G::LH>
__device__ __forceinline__ void stage_load(const BankParams& p, int64_t n, int64_t oy0, int64_t ox0,
                                           int wave, int lane, Raw<TS, staging_nt<G, SW, NR>()>& st, int ly0 = 0) {
  const TS* sp = static_cast<const TS*>(p.src) + n * p.s_sn;
  const int j = lane >> 3;
  const bool vec = p.s_vec != 0;
#pragma unroll
  for (int it = 0; it < staging_nt<G, SW, NR>(); ++it) {
    int ly, cg, chunk;
    bool act;
    unit_pos<G, CG, SW, NR>(it, wave, lane, ly, cg, chunk, act);
    ly += ly0;
    int64_t gy = p.row0 + oy0 - G::R + ly;
    gy = gy < 0 ? 0 : (gy >= p.H ? p.H - 1 : gy);
    const int c = cg * 8 + j;
    const TS* row = sp + static_cast<int64_t>(c < p.CI ? c : p.CI - 1) * p.s_sc + gy * p.s_sh;
    const int64_t gx0 = ox0 - 8 + 8 * chunk;
    if (vec) {
      // aligned rows, W a multiple of 8: every chunk lies left of, inside or
      // right of the row, so one 16-byte load of the nearest chunk inside it
      // always serves; stage_store fixes up the outside chunks
      const int64_t gxl = gx0 < 0 ? 0 : (gx0 > p.W - 8 ? p.W - 8 : gx0);
      load_vec(row + gxl, st.v[it]);
    } else {
      load_chunk<ADJ>(row, gx0, p.W, st.v[it]);
    }
  }
}

// Value of lane j ^ m (m = 1, 2, 4) by DPP: quad permutations for 1 and 2,
// row shifts by 4 lanes (select by bit 2 of the lane) for 4.
template <int M>
__device__ __forceinline__ uint32_t lane_xor(uint32_t v, int j) {
  const int x = static_cast<int>(v);
  if constexpr (M == 1) {
    return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(x, x, 0xB1, 0xF, 0xF, false));  // [1,0,3,2]
  } else if constexpr (M == 2) {
    return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(x, x, 0x4E, 0xF, 0xF, false));  // [2,3,0,1]
  } else {
    const int up = __builtin_amdgcn_update_dpp(x, x, 0x104, 0xF, 0xF, false);    // row_shl:4 (lane + 4)
    const int down = __builtin_amdgcn_update_dpp(x, x, 0x114, 0xF, 0xF, false);  // row_shr:4 (lane - 4)
    return static_cast<uint32_t>((j & 4) ? down : up);
  }
}

// 8 x 8 transpose of 16-bit values across the 8 lanes u, u+8, ..., u+56 of a
// unit (j = lane >> 3): element i of lane j (pair i/2, low half for even i)
// becomes element j of lane i.  The exchanges with the lanes 32 and 16 apart
// swap whole registers (v_permlane32_swap, v_permlane16_swap); the last one,
// 8 apart, swaps 16-bit halves: a DPP rotate by 8 within the 16-lane row,
// then a byte permute.  Every lane of the wave must take part.
__device__ __forceinline__ u32x4 transpose8(u32x4 d, int j) {
  const auto a = __builtin_amdgcn_permlane32_swap(d[0], d[2], false, false);
  const auto b = __builtin_amdgcn_permlane32_swap(d[1], d[3], false, false);
  const auto c = __builtin_amdgcn_permlane16_swap(a[0], b[0], false, false);
  const auto e = __builtin_amdgcn_permlane16_swap(a[1], b[1], false, false);
  const uint32_t x[4] = {c[0], c[1], e[0], e[1]};
  // low lanes keep their low halves and take the partner's; high lanes the
  // high halves (bytes 0-3 select the second operand, 4-7 the first)
  const uint32_t sel = (j & 1) ? 0x03020706u : 0x05040100u;
  u32x4 r;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint32_t t = static_cast<uint32_t>(
        __builtin_amdgcn_mov_dpp(static_cast<int>(x[k]), 0x128 /* row_ror:8 */, 0xf, 0xf, false));
    r[k] = __builtin_amdgcn_perm(t, x[k], sel);
  }
  return r;
}

// Transpose and LDS write of staging unit `it` of this wave.  With RING the
// LDS holds the rows as a ring of NSLOT rows: tile row ly sits in LDS row
// (slot0 + ly) mod NSLOT.
template <typename G, int K, int CG, bool ADJ, typename TS, int SW = G::THREADS / 64, int NR = G::LH,
          bool RING = false>
__device__ __forceinline__ void stage_store_unit(const BankParams& p, int64_t oy0, int64_t ox0, int wave, int lane,
                                                 const Raw<TS, staging_nt<G, SW, NR>()>& st, uint16_t* __restrict__ sl,
                                                 int it, int ly0 = 0, int slot0 = 0) {
  const int j = lane >> 3;
  {
    int ly, cg, chunk;
    bool act;
    unit_pos<G, CG, SW, NR>(it, wave, lane, ly, cg, chunk, act);
    ly += ly0;
    int lrow = ly;
    if constexpr (RING) {
      lrow = slot0 + ly;
      lrow -= lrow >= G::NSLOT ? G::NSLOT : 0;
    }
    bool keep = cg * 8 + j < p.CI;  // padded channels are zero
    if constexpr (ADJ) {
      const int64_t gy = p.row0 + oy0 - G::R + ly;
      keep = keep && gy >= 0 && gy < p.H;
    }
    u32x4 d = st.pairs(it);
    if (p.s_vec) {  // chunks outside the row: edge value (clamp) or zero (adjoint)
      const int64_t gx0 = ox0 - 8 + 8 * chunk;
      if (gx0 < 0 || gx0 >= p.W) {
        const uint32_t e = gx0 < 0 ? (d[0] & 0xffffu) : (d[3] >> 16);
        const uint32_t b = ADJ ? 0u : (e | (e << 16));
        d = u32x4{b, b, b, b};
      }
    }
    if (!keep) d = u32x4{0u, 0u, 0u, 0u};
    d = transpose8(d, j);  // channels cg*8 .. cg*8+7 of pixel chunk*8 + j
    if (act) *reinterpret_cast<u32x4*>(sl + (lrow * G::LW + chunk * 8 + j) * G::PS + cg * 8) = d;
  }
}

template <typename G, int K, int CG, bool ADJ, typename TS, int SW = G::THREADS / 64, int NR = G::LH,
          bool RING = false>
__device__ __forceinline__ void stage_store(const BankParams& p, int64_t oy0, int64_t ox0, int wave, int lane,
                                            const Raw<TS, staging_nt<G, SW, NR>()>& st, uint16_t* __restrict__ sl,
                                            int ly0 = 0, int slot0 = 0) {
#pragma unroll
  for (int it = 0; it < staging_nt<G, SW, NR>(); ++it)
    stage_store_unit<G, K, CG, ADJ, TS, SW, NR, RING>(p, oy0, ox0, wave, lane, st, sl, it, ly0, slot0);
}

// LDS offset (elements) of tap t in the channels-last tile, relative to the
// lane's pixel: neighbour (u, v) of the output pixel.
template <typename G, int K>
__device__ __forceinline__ constexpr int tap_offset(int t) {
  return ((t / K) * G::LW + t % K) * G::PS;
}

// Step s's B-operand offset for lane quarter q, minus the lane-constant part
// already in the base pointer.  k-group gi = 4s + q covers tap gi / CG and
// channel group gi % CG.  With CG >= 4 the four quarters share one tap (the
// channel group is in the base); with CG = 2 two taps alternate (one select);
// with CG = 1 each quarter has its own tap.  s is a compile-time constant in
// the unrolled step loop, so the taps fold to immediates.
template <typename G, int K, int CG>
__device__ __forceinline__ int b_step_offset(int s, bool hsel, int q) {
  if constexpr (CG >= 4) {
    return tap_offset<G, K>((4 * s) / CG) + ((4 * s) % CG) * 8;
  } else if constexpr (CG == 2) {
    const int t0 = 2 * s, t1 = 2 * s + 1;
    return hsel ? tap_offset<G, K>(t1 < K * K ? t1 : 0) : tap_offset<G, K>(t0 < K * K ? t0 : 0);
  } else {
    const int t0 = 4 * s;
    const int o0 = tap_offset<G, K>(t0 < K * K ? t0 : 0);
    const int o1 = tap_offset<G, K>(t0 + 1 < K * K ? t0 + 1 : 0);
    const int o2 = tap_offset<G, K>(t0 + 2 < K * K ? t0 + 2 : 0);
    const int o3 = tap_offset<G, K>(t0 + 3 < K * K ? t0 + 3 : 0);
    return q == 0 ? o0 : (q == 1 ? o1 : (q == 2 ? o2 : o3));
  }
}

// Weights of output group og into LDS, [co_local][k] with k = (uv*CG + cg)*8 + c
// (zero for padded k-groups, channels and outputs).
template <typename G, int K, int OT, int CG, bool ADJ, int NTHR = G::THREADS>
__device__ __forceinline__ void load_weights(const BankParams& p, int og, int tid, uint16_t* __restrict__ wl) {
  for (int idx = tid; idx < OT * 16 * G::KP; idx += NTHR) {
    const int col = idx / G::KP, k = idx - col * G::KP;
    const int co = og * OT * 16 + col;
    const int gi = k / 8, ci = (gi % CG) * 8 + k % 8, uv = gi / CG;
    uint16_t v = 0;
    if (co < p.CO && gi < G::KG && ci < p.CI) {
      const int u = uv / K, vv = uv % K;
      if constexpr (ADJ)  // Wt[co][ci][u][v] = W[ci][co][K-1-u][K-1-v]
        v = p.w[((static_cast<int64_t>(ci) * p.fi + co) * K + (K - 1 - u)) * K + (K - 1 - vv)];
      else
        v = p.w[((static_cast<int64_t>(co) * p.fi + ci) * K + u) * K + vv];
    }
    wl[col * G::WSTR + k] = v;
  }
}

template <bool OUT_BF16>
__device__ __forceinline__ void store4(void* dst, int64_t o, const f32x4& v) {
  if constexpr (OUT_BF16) {
    const uint32_t lo = pack_bf16x2(v[0], v[1]);
    const uint32_t hi = pack_bf16x2(v[2], v[3]);
    *reinterpret_cast<uint2*>(static_cast<uint16_t*>(dst) + o) = make_uint2(lo, hi);
  } else {
    *reinterpret_cast<float4*>(static_cast<float*>(dst) + o) = make_float4(v[0], v[1], v[2], v[3]);
  }
}
template <bool OUT_BF16>
__device__ __forceinline__ void store1(void* dst, int64_t o, float v) {
  if constexpr (OUT_BF16)
    static_cast<uint16_t*>(dst)[o] = f32_to_bf16_bits(v);
  else
    static_cast<float*>(dst)[o] = v;
}

// Store one lane's 4 consecutive outputs (pixels ox_l .. ox_l+3 of output
// channel co, tile row oy): one vector store inside the image, else element
// stores (adjoint: frame values to the frame buffer, columns outside the
// frame skipped).
template <bool ADJ, bool OUT_BF16>
__device__ __forceinline__ void store_px4(const BankParams& p, int64_t n, int co, int64_t oy, int64_t ox_l,
                                          const f32x4& v) {
  if (oy >= p.rows || co >= p.CO) return;
  const int64_t iy = ADJ ? p.row0 + oy : oy;  // adjoint: image row
  const bool inside = p.d_vec && (!ADJ || (iy >= 0 && iy < p.H && ox_l >= 0)) && ox_l + 4 <= p.W;
  if (inside) {
    store4<OUT_BF16>(p.dst, n * p.d_sn + static_cast<int64_t>(co) * p.d_sc + iy * p.d_sh + ox_l, v);
    return;
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t ox = ox_l + j;
    if constexpr (ADJ) {
      if (ox < -p.fr || ox >= p.W + p.fr) continue;
      if (iy >= 0 && iy < p.H && ox >= 0 && ox < p.W)
        store1<false>(p.dst, n * p.d_sn + co * p.d_sc + iy * p.d_sh + ox, v[j]);
      else
        p.frame[(n * p.CO + co) * p.frame_plane + frame_index(iy, ox, p.H, p.W, p.fr)] = v[j];
    } else {
      if (ox >= p.W) continue;
      store1<OUT_BF16>(p.dst, n * p.d_sn + co * p.d_sc + iy * p.d_sh + ox, v[j]);
    }
  }
}

// A wave's OTP x HP accumulator blocks: output channels co0 + 16a, tile row
// oy, pixels oxw + 16b + 4q .. +3.  When the wave's whole row segment
// oxw .. oxw + 16*HP - 1 is inside the image (one uniform test), every
// channel in range takes one vector store per block; border segments go
// through store_px4's per-lane tests.  (Testing per lane everywhere let the
// compiler keep the per-lane column masks in scalar registers, which it
// then had to spill: 5x5 forward with FP32 outputs -3%.)
template <bool ADJ, bool OUT_BF16, int OTP, int HP>
__device__ __forceinline__ void store_acc(const BankParams& p, int64_t n, int co0, int64_t oy, int64_t oxw, int q,
                                          const f32x4 (&acc)[OTP][HP]) {
  const int64_t iy = ADJ ? p.row0 + oy : oy;
  const bool fast = p.d_vec && oy < p.rows && (!ADJ || (iy >= 0 && iy < p.H && oxw >= 0)) && oxw + 16 * HP <= p.W;
  if (fast) {  // uniform
    const int64_t base = n * p.d_sn + iy * p.d_sh + oxw + 4 * q;
#pragma unroll
    for (int a = 0; a < OTP; ++a) {
      const int co = co0 + 16 * a;
      if (co >= p.CO) continue;
#pragma unroll
      for (int b = 0; b < HP; ++b)
        store4<OUT_BF16>(p.dst, base + static_cast<int64_t>(co) * p.d_sc + 16 * b, acc[a][b]);
    }
    return;
  }
#pragma unroll
  for (int a = 0; a < OTP; ++a)
#pragma unroll
    for (int b = 0; b < HP; ++b)
      store_px4<ADJ, OUT_BF16>(p, n, co0 + 16 * a, oy, oxw + 16 * b + 4 * q, acc[a][b]);
}

// One sweep over k for OTP 16-channel blocks x HP 16-pixel blocks:
// acc[a][b] += X(pixel block b) * W(channel block a).  w_pass: this lane's
// weight row of channel block 0; xsrc(step): this lane's pixel operand of
// step s in LDS (pixel block 0).  The operands of step s+1 are read while the
// MFMAs of step s run (two register sets); the scheduling fences keep the
// compiler from sinking the reads back next to their uses.  hook(step) runs
// after each step's MFMAs.
template <typename G, int K, int CG, int OTP, int HP, typename Src, typename Hook>
__device__ __forceinline__ void mfma_sweep(const uint16_t* w_pass, Src&& xsrc, int q, f32x4 (&acc)[OTP][HP],
                                           Hook&& hook) {
#pragma unroll
  for (int a = 0; a < OTP; ++a)
#pragma unroll
    for (int b = 0; b < HP; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
  // Operand addresses: a per-lane base plus a per-step constant, so that in
  // the unrolled step loop every LDS read carries its step offset as an
  // immediate.  Lane quarter q holds k-group gi = 4s + q of step s.
  bf16x8 wf[2][OTP], xf[2][HP];
  auto fetch = [&](auto step, int set) __attribute__((always_inline)) {
    constexpr int s = decltype(step)::value;
#pragma unroll
    for (int a = 0; a < OTP; ++a)
      wf[set][a] = *reinterpret_cast<const bf16x8*>(w_pass + a * 16 * G::WSTR + 32 * s);
    // quarters holding a padded k-group (past KG, only in the last step)
    // zero their operand in registers
    const uint16_t* bp = xsrc(step);
    const bool pad = 4 * s + 3 >= G::KG && 4 * s + q >= G::KG;
#pragma unroll
    for (int b = 0; b < HP; ++b) {
      xf[set][b] = *reinterpret_cast<const bf16x8*>(bp + b * 16 * G::PS);
      if (pad) xf[set][b] = bf16x8{};
    }
  };
  fetch(std::integral_constant<int, 0>{}, 0);
  static_for<G::STEPS>([&](auto step) __attribute__((always_inline)) {
    constexpr int s = decltype(step)::value;
    if constexpr (s + 1 < G::STEPS) fetch(std::integral_constant<int, s + 1>{}, (s + 1) & 1);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int a = 0; a < OTP; ++a)
#pragma unroll
      for (int b = 0; b < HP; ++b)
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xf[s & 1][b], wf[s & 1][a], acc[a][b], 0, 0, 0);
    hook(step);
    __builtin_amdgcn_sched_barrier(0);
  });
}

// Persistent work-group over (image, output group, kTH x TW tile).  Each wave
// computes OT*16 output channels x HP*16 pixels of one tile row in NP passes
// of OTP*16 channels (one full sweep over k per pass, OTP x HP 16x16
// accumulator blocks).
//
//  * the loads of tile t+1 are issued when tile t starts; with two source
//    buffers, tile t+1 is packed into the idle buffer unit by unit between
//    the MFMA groups of tile t's last sweep, so its VALU and LDS work runs
//    beside the matrix cores of the other waves;
//  * each pass stores its results right after its sweep;
//  * one barrier per tile (plus one before repacking when a single source
//    buffer fits, or before reloading the weights of a new output group).
//
// MFMA operands: A = 16 pixels x 32 k (the source tile), B = 32 k x 16 output
// channels (the weights), so D[pixel 4q + j][channel l16]: each lane holds 4
// consecutive pixels of one output channel and writes them with one store.
template <int K, int OT, int PT, int CG, int NW, bool ADJ, typename TS, bool OUT_BF16>
__global__ __launch_bounds__(64 * NW) void k_bank_conv(BankParams p) {
  using G = ConvGeom<K, OT, PT, CG, NW>;
  constexpr int HP = G::HP;
  constexpr int OTP = OT < 2 ? OT : 2;  // 16-channel blocks per pass
  constexpr int NP = OT / OTP;
  static_assert(OT % OTP == 0, "passes");
  extern __shared__ uint4 smem4[];
  uint16_t* wl = reinterpret_cast<uint16_t*>(smem4);
  uint16_t* sl0 = wl + G::W_ELEMS;
  const int tid = threadIdx.x;
  const int lane = tid % 64;
  const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
  const int wrow = wave % kTH;                      // this wave's tile row
  const int wcol = (wave / kTH) * (G::TW / G::WPR); // and its share of the columns
  const int l16 = lane % 16, q = lane / 16;
  const uint16_t* w_lane = wl + l16 * G::WSTR + q * 8;
  const int b_off = (wrow * G::LW + wcol + l16 + G::XOFF) * G::PS + (CG >= 4 ? q * 8 : (CG == 2 ? (q & 1) * 8 : 0));
  const bool hsel = (q >> 1) != 0;

  const int64_t per_group = static_cast<int64_t>(p.tiles_x) * p.tiles_y;
  // tile t -> (image n, output group og, tile origin); tile counts fit in 32 bits
  const uint32_t pg = static_cast<uint32_t>(per_group), tx = static_cast<uint32_t>(p.tiles_x);
  const uint32_t ngr = static_cast<uint32_t>(p.o_groups);
  auto decode = [&](int64_t t64, int64_t& n, int& og, int64_t& oy0, int64_t& ox0) __attribute__((always_inline)) {
    const uint32_t t = static_cast<uint32_t>(t64);
    const uint32_t ng = t / pg, r = t - ng * pg;
    og = static_cast<int>(ng % ngr);
    n = ng / ngr;
    const uint32_t tile_y = r / tx, tile_x = r - tile_y * tx;
    oy0 = static_cast<int64_t>(tile_y) * kTH;
    ox0 = (ADJ ? p.col0 : 0) + static_cast<int64_t>(tile_x) * G::TW;
  };
  // XCD-aware start: the work-groups resident on one XCD take consecutive
  // tiles, so the halo lines neighbouring tiles share are read once into
  // that XCD's L2 (the stride below keeps every round contiguous)
  int64_t t = xcd_remap(blockIdx.x, gridDim.x);
  if (t >= p.n_tiles) return;
  int64_t n, oy0, ox0;
  int og;
  decode(t, n, og, oy0, ox0);
  Raw<TS, G::NT> st;
  stage_load<G, K, CG, ADJ, TS>(p, n, oy0, ox0, wave, lane, st);
  load_weights<G, K, OT, CG, ADJ>(p, og, tid, wl);
  stage_store<G, K, CG, ADJ, TS>(p, oy0, ox0, wave, lane, st, sl0);
  __syncthreads();

  int cur = 0;
  while (true) {
    const int64_t t_next = t + gridDim.x;
    const bool more = t_next < p.n_tiles;
    // prefetch the next tile (the current one again at the end: the same
    // loads either way, so the register state has a single producer)
    int64_t n2, oy2, ox2;
    int og2;
    decode(more ? t_next : t, n2, og2, oy2, ox2);
    stage_load<G, K, CG, ADJ, TS>(p, n2, oy2, ox2, wave, lane, st);
    __builtin_amdgcn_sched_barrier(0);  // keep every prefetch load ahead of the MFMA loop

    const uint16_t* b_lane = sl0 + cur * G::S_ELEMS + b_off;
    uint16_t* sl_next = sl0 + (cur ^ 1) * G::S_ELEMS;
    static_for<NP>([&](auto pass) __attribute__((always_inline)) {
      constexpr int P = decltype(pass)::value;
      const uint16_t* w_pass = w_lane + P * OTP * 16 * G::WSTR;
      f32x4 acc[OTP][HP];
      // in the last pass, with two source buffers, staging unit S0+u goes
      // after step S0+u (the last step also takes any left over)
      constexpr int S0 = G::STEPS > G::NT ? G::STEPS - G::NT : 0;
      // b_step_offset clamps taps past K*K to tap 0, so every read is of staged pixels
      auto xsrc = [&](auto step) __attribute__((always_inline)) {
        return b_lane + b_step_offset<G, K, CG>(decltype(step)::value, hsel, q);
      };
      mfma_sweep<G, K, CG, OTP, HP>(w_pass, xsrc, q, acc, [&](auto step) __attribute__((always_inline)) {
        constexpr int s = decltype(step)::value;
        if constexpr (P == NP - 1 && G::NBUF == 2) {
          constexpr int u0 = s - S0, u1 = s == G::STEPS - 1 ? G::NT : s - S0 + 1;
#pragma unroll
          for (int u = u0 < 0 ? 0 : u0; u < u1; ++u)
            stage_store_unit<G, K, CG, ADJ, TS>(p, oy2, ox2, wave, lane, st, sl_next, u);
        }
      });
      // acc[a][b][j] = output channel (og*NP + P)*OTP*16 + 16a + l16, pixel
      // ox0 + wcol + 16b + 4q + j of tile row wrow
      const int co0 = (og * NP + P) * OTP * 16 + l16;
      store_acc<ADJ, OUT_BF16, OTP, HP>(p, n, co0, oy0 + wrow, ox0 + wcol, q, acc);
    });

    if (more) {
      // a new output group, or a single source buffer: wait until every wave
      // is done reading (uniform branch)
      if (og2 != og || G::NBUF == 1) __syncthreads();
      if (og2 != og) load_weights<G, K, OT, CG, ADJ>(p, og2, tid, wl);
      if constexpr (G::NBUF == 1) stage_store<G, K, CG, ADJ, TS>(p, oy2, ox2, wave, lane, st, sl0);
    }
    __syncthreads();  // tile t+1 staged; everyone done with buffer cur
    if (!more) break;
    t = t_next;
    n = n2;
    og = og2;
    oy0 = oy2;
    ox0 = ox2;
    if (G::NBUF == 2) cur ^= 1;
  }
}

// ------------------------------------------------------------- row ring --
//
// For 33..64 source channels a source tile is large (for K = 5 the weights
// and one tile fill LDS), and restaging the LH = kTH + K - 1 rows of every
// 4-row tile costs more than the MFMAs.  Here a work-group walks down a segment of one
// tile column and keeps the LH source rows in LDS as a ring: the first tile
// of a segment stages all LH rows, every further tile only its kTH new rows,
// whose loads are issued before the previous tile's MFMAs.  Tile row ly sits
// in ring row (slot + ly) mod NSLOT; the MFMA operands of tap row u come from
// ring row (slot + wrow + u) mod NSLOT.  With NSLOT = LH + kTH the new rows go
// to the kTH free ring rows, packed unit by unit between the MFMA groups of
// the last steps (one barrier per tile); with NSLOT = LH they replace the
// oldest rows once no wave reads them any more: for K > kTH packed between
// the MFMA groups of the last tap rows' steps, after a barrier (two barriers
// per tile), else after the sweep, between two barriers.
// The ring kernel's per-tile staging of the NEW rows, planned once per
// column segment.  Everything about a staging unit that does not change from
// one tile to the next (its channel and clamped chunk column as a 32-bit
// element offset into image n, its LDS offset within a ring row, its row and
// flags) is computed when the segment starts; a tile then only adds its row.
// Used with vector staging when one source image spans < 2^31 elements.
template <int NTN>
struct RingPlan {
  uint32_t soff[NTN];  // element offset of the unit's chunk in image n, row 0
  uint32_t loff[NTN];  // LDS element offset within a ring row
  uint32_t info[NTN];  // row (bits 0-7) | active << 8 | channel kept << 9 | outside (1 left, 2 right) << 10
};

template <typename G, int CG, int NR, int NTN>
__device__ __forceinline__ void ring_plan(const BankParams& p, int64_t ox0, int wave, int lane, RingPlan<NTN>& pl) {
  const int j = lane >> 3;
#pragma unroll
  for (int it = 0; it < NTN; ++it) {
    int ly, cg, chunk;
    bool act;
    unit_pos<G, CG, 8, NR>(it, wave, lane, ly, cg, chunk, act);
    const int c = cg * 8 + j;
    const bool keep = c < p.CI;
    const int64_t cc = keep ? c : p.CI - 1;
    const int64_t gx0 = ox0 - 8 + 8 * chunk;
    const int64_t gxl = gx0 < 0 ? 0 : (gx0 > p.W - 8 ? p.W - 8 : gx0);
    const uint32_t outside = gx0 < 0 ? 1u : (gx0 >= p.W ? 2u : 0u);
    pl.soff[it] = static_cast<uint32_t>(cc * p.s_sc + gxl);
    pl.loff[it] = static_cast<uint32_t>((chunk * 8 + j) * G::PS + cg * 8);
    pl.info[it] = static_cast<uint32_t>(ly) | (act ? 1u << 8 : 0u) | (keep ? 1u << 9 : 0u) | (outside << 10);
  }
}

// Load of planned unit `it` for source rows gy_base + row (clamped), and of
// every planned unit.
template <typename TS, int NTN>
__device__ __forceinline__ void ring_load_unit(const BankParams& p, const TS* __restrict__ sp_n, int64_t gy_base,
                                               const RingPlan<NTN>& pl, Raw<TS, NTN>& st, int it) {
  const int32_t hl = static_cast<int32_t>(p.H) - 1;
  const uint32_t sh = static_cast<uint32_t>(p.s_sh);
  int32_t gy = static_cast<int32_t>(gy_base) + static_cast<int32_t>(pl.info[it] & 0xffu);
  gy = gy < 0 ? 0 : (gy > hl ? hl : gy);
  load_vec(sp_n + (pl.soff[it] + __umul24(static_cast<uint32_t>(gy), sh)), st.v[it]);
}
template <typename TS, int NTN>
__device__ __forceinline__ void ring_load(const BankParams& p, const TS* __restrict__ sp_n, int64_t gy_base,
                                          const RingPlan<NTN>& pl, Raw<TS, NTN>& st) {
#pragma unroll
  for (int it = 0; it < NTN; ++it) ring_load_unit<TS, NTN>(p, sp_n, gy_base, pl, st, it);
}

// Edge fix, padding, transpose and ring write of planned unit `it` (tile row
// LH - NR + row goes to ring row (slot0 + LH - NR + row) mod NSLOT).
template <typename G, bool ADJ, typename TS, int NR, int NTN>
__device__ __forceinline__ void ring_store_unit(const BankParams& p, int64_t gy_base, int lane, const RingPlan<NTN>& pl,
                                                const Raw<TS, NTN>& st, uint16_t* __restrict__ ring, int it, int slot0) {
  const int j = lane >> 3;
  const uint32_t info = pl.info[it];
  const int row = static_cast<int>(info & 0xffu);
  bool keep = (info >> 9) & 1u;
  if constexpr (ADJ) {
    const int64_t gy = gy_base + row;
    keep = keep && gy >= 0 && gy < p.H;
  }
  u32x4 d = st.pairs(it);
  const uint32_t outside = (info >> 10) & 3u;
  if (outside) {  // chunks outside the row: edge value (clamp) or zero (adjoint)
    const uint32_t e = outside == 1u ? (d[0] & 0xffffu) : (d[3] >> 16);
    const uint32_t b = ADJ ? 0u : (e | (e << 16));
    d = u32x4{b, b, b, b};
  }
  if (!keep) d = u32x4{0u, 0u, 0u, 0u};
  d = transpose8(d, j);
  int lrow = slot0 + (G::LH - NR) + row;
  lrow -= lrow >= G::NSLOT ? G::NSLOT : 0;
  if ((info >> 8) & 1u) *reinterpret_cast<u32x4*>(ring + lrow * (G::LW * G::PS) + pl.loff[it]) = d;
}

template <int K, int OT, int PT, int CG, bool ADJ, typename TS, bool OUT_BF16>
__global__ __launch_bounds__(512) void k_bank_conv_ring(BankParams p) {
  using G = ConvGeom<K, OT, PT, CG, 8>;
  static_assert(G::RINGED && G::NBUF == 1, "64-channel sources with one LDS tile");
  constexpr bool OVL = G::NSLOT > G::LH;
  constexpr int HP = G::HP;
  constexpr int OTP = OT < 2 ? OT : 2;
  constexpr int NP = OT / OTP;
  constexpr int NEW = kTH;  // rows packed per tile after a segment's first
  constexpr int ROWE = G::LW * G::PS;  // elements per ring row
  // LH-row ring: steps run tap-row major, 2K per tap row (two per tap).
  // Wave row wrow reads ring row wrow + u for tap row u, so from the first
  // step of tap row kTH on no wave reads the kTH oldest rows; where that
  // step falls inside the sweep (LATE), a barrier there lets the new rows
  // replace them, packed between the MFMA groups of the remaining steps.
  static_assert(CG == 8 && G::STEPS == 2 * K * K, "two steps per tap");
  constexpr int SB = 2 * K * kTH;
  constexpr bool LATE = !OVL && SB < G::STEPS;
  extern __shared__ uint4 smem4[];
  uint16_t* wl = reinterpret_cast<uint16_t*>(smem4);
  uint16_t* ring = wl + G::W_ELEMS;
  const int tid = threadIdx.x;
  const int lane = tid % 64;
  const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
  const int wrow = wave % kTH;
  const int wcol = (wave / kTH) * (G::TW / G::WPR);
  const int l16 = lane % 16, q = lane / 16;
  const uint16_t* w_lane = wl + l16 * G::WSTR + q * 8;
  const int lane_off = (wcol + l16 + G::XOFF) * G::PS + q * 8;

  const uint32_t spc = static_cast<uint32_t>(p.seg_per_col), tx = static_cast<uint32_t>(p.tiles_x);
  const uint32_t ngr = static_cast<uint32_t>(p.o_groups);
  int og_loaded = -1;
  // XCD-aware start (see k_bank_conv): horizontally adjacent column
  // segments run on one XCD at the same time and share their halo lines in L2
  for (int64_t sg = xcd_remap(blockIdx.x, gridDim.x); sg < p.n_segs; sg += gridDim.x) {
    const uint32_t col = static_cast<uint32_t>(sg) / spc, sy = static_cast<uint32_t>(sg) - col * spc;
    const uint32_t tile_x = col % tx, ng = col / tx;
    const int og = static_cast<int>(ng % ngr);
    const int64_t n = ng / ngr;
    const int ty0 = static_cast<int>(sy) * p.seg_len;
    const int ty1 = ty0 + p.seg_len < p.tiles_y ? ty0 + p.seg_len : p.tiles_y;
    const int64_t ox0 = (ADJ ? p.col0 : 0) + static_cast<int64_t>(tile_x) * G::TW;
    __syncthreads();  // every wave is done with the ring (and weights) of the previous segment
    if (og != og_loaded) {  // uniform
      load_weights<G, K, OT, CG, ADJ>(p, og, tid, wl);
      og_loaded = og;
    }
    // Staging positions derive from (wave, lane); passing them through an
    // empty asm here and in the tile loop keeps the compiler from hoisting
    // every unit's addresses out of the loops (which spilled ~50 registers).
    int swave = wave, slane = lane;
    asm volatile("" : "+s"(swave), "+v"(slane));
    {
      Raw<TS, staging_nt<G, 8, G::LH>()> sa;
      const int64_t oy0 = static_cast<int64_t>(ty0) * kTH;
      stage_load<G, K, CG, ADJ, TS, 8, G::LH>(p, n, oy0, ox0, swave, slane, sa, 0);
      stage_store<G, K, CG, ADJ, TS, 8, G::LH, true>(p, oy0, ox0, swave, slane, sa, ring, 0, 0);
    }
    int slot = 0;
    __syncthreads();
    constexpr int NTN = staging_nt<G, 8, NEW>();
    Raw<TS, NTN> st;
    const bool planned = p.s_plan32 != 0;  // uniform
    RingPlan<NTN> pl;
    if (planned) ring_plan<G, CG, NEW, NTN>(p, ox0, wave, lane, pl);
    const TS* sp_n = static_cast<const TS*>(p.src) + n * p.s_sn;
    for (int ty = ty0; ty < ty1; ++ty) {
      const int64_t oy0 = static_cast<int64_t>(ty) * kTH;
      const bool more = ty + 1 < ty1;  // uniform
      // source row of planned row 0 of the next tile's NEW rows
      const int64_t gy_next = p.row0 + oy0 + kTH - G::R + (G::LH - NEW);
      swave = wave;
      slane = lane;
      if (!planned) asm volatile("" : "+s"(swave), "+v"(slane));
      if (more) {
        if (planned)
          ring_load<TS, NTN>(p, sp_n, gy_next, pl, st);
        else
          stage_load<G, K, CG, ADJ, TS, 8, NEW>(p, n, oy0 + kTH, ox0, swave, slane, st, G::LH - NEW);
      }
      __builtin_amdgcn_sched_barrier(0);
      // ring row of this wave's tap row u (uniform), then the lane's pixel
      const uint16_t* ring_lane = ring + lane_off;
      const int rbase = slot + wrow;
      // with the larger ring, the next tile's new rows land in the free rows
      int nslot = slot + NEW;
      nslot -= nslot >= G::NSLOT ? G::NSLOT : 0;
      static_for<NP>([&](auto pass) __attribute__((always_inline)) {
        constexpr int P = decltype(pass)::value;
        f32x4 acc[OTP][HP];
        // step s: tap t = s / 2 (32 of the 64 channels per step), channels (s % 2) * 32 + q * 8
        auto xsrc = [&](auto step) __attribute__((always_inline)) {
          constexpr int st8 = decltype(step)::value, t = (4 * st8) / CG;
          int r = rbase + t / K;
          r -= r >= G::NSLOT ? G::NSLOT : 0;
          return ring_lane + r * ROWE + ((t % K) * G::PS + ((4 * st8) % CG) * 8);
        };
        constexpr int S0 = G::STEPS > NTN ? G::STEPS - NTN : 0;
        mfma_sweep<G, K, CG, OTP, HP>(w_lane + P * OTP * 16 * G::WSTR, xsrc, q, acc,
                                      [&](auto step) __attribute__((always_inline)) {
          constexpr int s8 = decltype(step)::value;
          if constexpr ((OVL || LATE) && P == NP - 1) {
            if (more) {  // uniform
              if constexpr (LATE && s8 == SB - 1) __syncthreads();
              constexpr int SS = OVL ? S0 : (SB > S0 ? SB : S0);
              constexpr int u0 = s8 - SS, u1 = s8 == G::STEPS - 1 ? NTN : s8 - SS + 1;
#pragma unroll
              for (int u = u0 < 0 ? 0 : u0; u < u1; ++u) {
                if (planned)
                  ring_store_unit<G, ADJ, TS, NEW, NTN>(p, gy_next, lane, pl, st, ring, u, nslot);
                else
                  stage_store_unit<G, K, CG, ADJ, TS, 8, NEW, true>(p, oy0 + kTH, ox0, swave, slane, st, ring, u,
                                                                   G::LH - NEW, nslot);
              }
            }
          }
        });
        const int co0 = (og * NP + P) * OTP * 16 + l16;
        store_acc<ADJ, OUT_BF16, OTP, HP>(p, n, co0, oy0 + wrow, ox0 + wcol, q, acc);
      });
      if (more) {
        __syncthreads();  // (OVL, LATE: the new rows are packed; all reads of the oldest rows done)
        if constexpr (!OVL && !LATE) {  // the oldest kTH ring rows become the next tile's new rows
          if (planned) {
#pragma unroll
            for (int u = 0; u < NTN; ++u) ring_store_unit<G, ADJ, TS, NEW, NTN>(p, gy_next, lane, pl, st, ring, u, nslot);
          } else {
            stage_store<G, K, CG, ADJ, TS, 8, NEW, true>(p, oy0 + kTH, ox0, swave, slane, st, ring, G::LH - NEW,
                                                        nslot);
          }
          __syncthreads();
        }
        slot = nslot;
      }
    }
  }
}

// ------------------------------------------------- vertical tap reuse --
//
// 33..64 source channels into at most 16 output channels: the adjoint of the
// 16 -> 64 bank (dgrad) and forwards of that shape.  With a single 16-channel
// output block, a pixel operand that k_bank_conv_ring reads from LDS feeds one
// MFMA, and with the weight reads that is 1.5 LDS reads of 1 KiB per MFMA: the
// LDS read port, not the matrix cores, sets the pace there.  Here the weights
// stay in registers, and a wave walks the staged rows of its tile in source-row
// order: the operand of staged row s and tap column v feeds the MFMAs of every
// tile row y it reaches (tap row s - y), so a tile of kTH rows takes LH*K
// operand reads for kTH*K*K MFMAs per 32 channels (0.4 reads per MFMA at
// K = 5).  A wave keeps the K*K taps of one 32-channel half of the source
// channels for its 16 output channels (4*K*K registers); the two halves of the
// same outputs run in two waves and meet in LDS: each leaves its sums of half
// the tile rows there and completes and stores the other rows (splitting the
// stores measured 5% faster at K = 5 than one half storing all).  Eight waves
// per work-group: two halves x four 16-pixel column blocks, each over all kTH
// rows of a kTH x 64 tile; the staged rows are kept as a ring as in
// k_bank_conv_ring, and every load runs a tile ahead of its packing.
template <int K>
struct VrGeom : ConvGeom<K, 1, 4, 8, 8> {
  using Base = ConvGeom<K, 1, 4, 8, 8>;
  static constexpr int ROWE = Base::LW * Base::PS;  // elements per ring row
  // partial sums handed between the halves: two buffers (alternate tiles)
  // of [column block][tile row][lane][4] floats
  static constexpr int RED_F = 2 * 4 * kTH * 64 * 4;
  static constexpr bool fits(int slots) { return slots * ROWE * 2 + RED_F * 4 <= 160 * 1024; }
  // a ring with room for the next tile's kTH new rows where it fits; else LH
  // rows, the new rows replacing the kTH oldest once every wave is past them
  static constexpr int NSLOT = fits(Base::LH + kTH) ? Base::LH + kTH : Base::LH;
  static constexpr int LDS_B = NSLOT * ROWE * 2 + RED_F * 4;
  static_assert(fits(NSLOT), "ring and sums exceed LDS");
};

template <int K, bool ADJ, typename TS, bool OUT_BF16>
__global__ __launch_bounds__(512) void k_bank_conv_vr(BankParams p) {
  using G = VrGeom<K>;
  constexpr int LH = G::LH, KK = K * K;
  constexpr int NG = LH * K;  // (staged row, tap column) operand groups per tile
  constexpr int NEW = kTH;
  constexpr bool OVL = G::NSLOT > LH;
  // groups that read the kTH oldest rows; without room for the new rows in
  // the ring, a barrier after them frees those rows for the next tile
  constexpr int SB = kTH * K;
  constexpr int NTN = staging_nt<G, 8, NEW>();
  // the next tile's rows are packed unit by unit between the MFMA groups
  // from group PK0 on (late enough that their loads have landed)
  constexpr int PK0 = OVL ? NG / 2 : SB;
  static_assert(LH % NEW == 0 || G::NSLOT >= (LH + NEW - 1) / NEW * NEW, "first rows' last batch inside the ring");
  extern __shared__ uint4 smem4[];
  uint16_t* ring = reinterpret_cast<uint16_t*>(smem4);
  float* red = reinterpret_cast<float*>(ring + G::NSLOT * G::ROWE);
  const int tid = threadIdx.x;
  const int lane = tid % 64;
  const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
  const int half = wave >> 2;  // source channels 32*half .. 32*half+31
  const int cb = wave & 3;     // pixels 16*cb .. 16*cb+15 of the tile
  const int l16 = lane % 16, q = lane / 16;
  const int lane_off = (16 * cb + l16 + G::XOFF) * G::PS + half * 32 + q * 8;
  float* red_lane = red + (cb * kTH * 64 + lane) * 4;

  // B operands: output channel l16, source channels 32*half + 8q .. +7 of tap
  // t, read once from the weights laid out in LDS as k_bank_conv keeps them
  // (the ring's space is free until the first segment is staged)
  static_assert(G::W_ELEMS <= G::NSLOT * G::ROWE, "weights staged in the ring space");
  load_weights<G, K, 1, 8, ADJ, 512>(p, 0, tid, ring);
  __syncthreads();
  bf16x8 wr[KK];
#pragma unroll
  for (int t = 0; t < KK; ++t)
    wr[t] = *reinterpret_cast<const bf16x8*>(ring + l16 * G::WSTR + (t * 8 + half * 4 + q) * 8);

  const uint32_t spc = static_cast<uint32_t>(p.seg_per_col), tx = static_cast<uint32_t>(p.tiles_x);
  uint32_t tcount = 0;
  // XCD-aware start (see k_bank_conv)
  for (int64_t sg = xcd_remap(blockIdx.x, gridDim.x); sg < p.n_segs; sg += gridDim.x) {
    const uint32_t col = static_cast<uint32_t>(sg) / spc, sy = static_cast<uint32_t>(sg) - col * spc;
    const uint32_t tile_x = col % tx;
    const int64_t n = col / tx;  // one output group
    const int ty0 = static_cast<int>(sy) * p.seg_len;
    const int ty1 = ty0 + p.seg_len < p.tiles_y ? ty0 + p.seg_len : p.tiles_y;
    const int64_t ox0 = (ADJ ? p.col0 : 0) + static_cast<int64_t>(tile_x) * G::TW;
    __syncthreads();  // every wave is done with the ring and sums of the previous segment
    const TS* sp_n = static_cast<const TS*>(p.src) + n * p.s_sn;
    Raw<TS, NTN> st;
    RingPlan<NTN> pl;
    ring_plan<G, 8, NEW, NTN>(p, ox0, wave, lane, pl);
    // the segment's first LH rows into ring rows 0 .. LH-1, NEW rows at a
    // time with the tile loop's plan (the weights already hold 4*K*K
    // registers); a last partial batch also fills ring rows past LH, which
    // the first tile's new rows overwrite later
    for (int b = 0; b < (LH + NEW - 1) / NEW; ++b) {
      const int64_t gyb = p.row0 + static_cast<int64_t>(ty0) * kTH - G::R + b * NEW;
      ring_load<TS, NTN>(p, sp_n, gyb, pl, st);
      int s0 = b * NEW - (LH - NEW);
      s0 += s0 < 0 ? G::NSLOT : 0;
#pragma unroll
      for (int u = 0; u < NTN; ++u) ring_store_unit<G, ADJ, TS, NEW, NTN>(p, gyb, lane, pl, st, ring, u, s0);
    }
    int slot = 0;
    // the second tile's new rows, packed during the first tile
    ring_load<TS, NTN>(p, sp_n, p.row0 + static_cast<int64_t>(ty0) * kTH + kTH - G::R + (LH - NEW), pl, st);
    __syncthreads();
    // Loads run a tile ahead of their packing: as soon as a unit of the next
    // tile's rows is packed, its registers are reloaded with the same unit of
    // the rows after them, so every load has a whole tile to land.  Every
    // tile, the last of a segment too, loads and packs (rows clamped to the
    // image, so always valid; the spare ones are never read): with no
    // condition between the loads and their uses, the compiler's wait counts
    // stay exact across iterations.
    for (int ty = ty0; ty < ty1; ++ty) {
      const int64_t oy0 = static_cast<int64_t>(ty) * kTH;
      const int64_t gy_next = p.row0 + oy0 + kTH - G::R + (LH - NEW);
      __builtin_amdgcn_sched_barrier(0);
      int nslot = slot + NEW;
      nslot -= nslot >= G::NSLOT ? G::NSLOT : 0;
      const uint16_t* rl = ring + lane_off;
      auto operand = [&](auto gi) __attribute__((always_inline)) {
        constexpr int g = decltype(gi)::value, s = g / K, dx = g % K;
        int r = slot + s;
        r -= r >= G::NSLOT ? G::NSLOT : 0;
        return *reinterpret_cast<const bf16x8*>(rl + r * G::ROWE + dx * G::PS);
      };
      f32x4 acc[kTH];
#pragma unroll
      for (int y = 0; y < kTH; ++y) acc[y] = f32x4{0.f, 0.f, 0.f, 0.f};
      bf16x8 xf[3];
      xf[0] = operand(std::integral_constant<int, 0>{});
      if constexpr (NG > 1) xf[1] = operand(std::integral_constant<int, 1>{});
      static_for<NG>([&](auto gi) __attribute__((always_inline)) {
        constexpr int g = decltype(gi)::value, s = g / K, dx = g % K;
        if constexpr (g + 2 < NG) xf[(g + 2) % 3] = operand(std::integral_constant<int, g + 2>{});
        __builtin_amdgcn_sched_barrier(0);
        constexpr int y0 = s - (K - 1) > 0 ? s - (K - 1) : 0;
        constexpr int y1 = s < kTH - 1 ? s : kTH - 1;
#pragma unroll
        for (int y = y0; y <= y1; ++y)
          acc[y] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xf[g % 3], wr[(s - y) * K + dx], acc[y], 0, 0, 0);
        if constexpr (!OVL && g == SB - 1) __syncthreads();  // the kTH oldest rows are free
        if constexpr (g >= PK0) {
          constexpr int u0 = ((g - PK0) * NTN + (NG - PK0) - 1) / (NG - PK0);
          constexpr int u1 = ((g - PK0 + 1) * NTN + (NG - PK0) - 1) / (NG - PK0);
#pragma unroll
          for (int u = u0; u < u1; ++u) {
            ring_store_unit<G, ADJ, TS, NEW, NTN>(p, gy_next, lane, pl, st, ring, u, nslot);
            ring_load_unit<TS, NTN>(p, sp_n, gy_next + kTH, pl, st, u);
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      });
      // each half completes and stores half of the tile rows: half 0 rows
      // 0 .. kTH/2-1, half 1 the others; each leaves its sums of the other
      // rows in LDS for the other half
      float* rb = red_lane + (tcount & 1u) * (G::RED_F / 2);
      constexpr int HR = kTH / 2;
      const int mine = half * HR, theirs = HR - mine;
#pragma unroll
      for (int y = 0; y < HR; ++y) *reinterpret_cast<f32x4*>(rb + (theirs + y) * 256) = half ? acc[y] : acc[HR + y];
      __syncthreads();  // partial sums in LDS; the next tile's rows are packed
      {
        f32x4 v[HR];
#pragma unroll
        for (int y = 0; y < HR; ++y) v[y] = (half ? acc[HR + y] : acc[y]) + *reinterpret_cast<const f32x4*>(rb + (mine + y) * 256);
        const int64_t oxw = ox0 + 16 * cb, ya = oy0 + mine, yb = ya + HR - 1;
        const int64_t iya = ADJ ? p.row0 + ya : ya, iyb = ADJ ? p.row0 + yb : yb;
        const bool all_fast = p.d_vec && yb < p.rows && (!ADJ || (iya >= 0 && iyb < p.H && oxw >= 0)) &&
                              oxw + 16 <= p.W;
        if (all_fast) {  // uniform
          if (l16 < p.CO) {
            const int64_t base = n * p.d_sn + static_cast<int64_t>(l16) * p.d_sc + iya * p.d_sh + oxw + 4 * q;
#pragma unroll
            for (int y = 0; y < HR; ++y) store4<OUT_BF16>(p.dst, base + y * p.d_sh, v[y]);
          }
        } else {
#pragma unroll
          for (int y = 0; y < HR; ++y) {
            f32x4 w[1][1];
            w[0][0] = v[y];
            store_acc<ADJ, OUT_BF16, 1, 1>(p, n, l16, ya + y, oxw, q, w);
          }
        }
      }
      ++tcount;
      slot = nslot;
    }
  }
}

// ------------------------------------------------------ specialised waves --
//
// Forward for 64 output channels from 9..16 input channels (the filter-bank
// workload) with BF16 outputs, with the memory traffic taken off the waves
// that feed the matrix cores.  A wave issues in order, so in k_bank_conv a load or store held up
// by the output stream also holds up that wave's MFMAs; here kWsMfma waves
// only read LDS and run MFMAs, and kWsMem memory waves (two per SIMD, two per
// tile row, each storing half of its channels: 8 % faster at K = 3 and 3.5 %
// at K = 5 than one per SIMD) stage the next tile and store the previous
// interval's results, which the MFMA
// waves leave in an LDS result buffer.  An interval is one sweep over k for
// all 64 channels of a tile.  One barrier per interval orders the hand-overs:
//   MFMA waves:   sweep (source buffer c)  ->  results to result buffer r
//   memory waves: results of the previous interval (buffer r^1) to HBM;
//                 in the last interval of a tile also the packing of the
//                 next tile into source buffer c^1 (its loads were issued a
//                 tile earlier) and the loads of the tile after it
// Weights, two source tiles and two result buffers take exactly 160 KiB for
// K = 5.
constexpr int kWsMfma = 8, kWsMem = 8;

template <int K, int CG>
struct WsGeom {
  using G = ConvGeom<K, 4, 4, CG, kWsMfma>;  // 4 x 64 tiles, the k_bank_conv MFMA wave layout
  static constexpr int OTP = 4;                 // 16-channel blocks per interval
  static constexpr int EPC = 8;                 // bf16 elements per 16-byte chunk
  static constexpr int ROW_B = 64;              // one region row: 32 pixels of a channel
  static constexpr int REG_B = OTP * 16 * ROW_B;  // one MFMA wave's results
  // Result regions of MFMA waves w and w+4 (the two halves of tile row w)
  // sit 256 bytes apart mod 512, so that a memory wave reading both halves
  // of a channel row hits every bank once; within a region, row c's 16-byte
  // chunks are permuted (chunk m at m ^ swz(c)) so that the MFMA waves'
  // writes (16 channels x 2 chunk halves per 32 lanes) are conflict-free too.
  static constexpr int PAIR_B = 2 * REG_B + 256;
  static constexpr int RBUF_B = 4 * PAIR_B;
  static constexpr int NTM = staging_nt<G, kWsMem>();
  static constexpr int LDS_B = G::W_ELEMS * 2 + 2 * G::S_ELEMS * 2 + 2 * RBUF_B;
  static_assert(G::NBUF == 2 && G::HP == 2, "layout");
  static_assert(REG_B == 4096, "region size");
  static_assert(LDS_B <= 160 * 1024, "LDS");
  static __device__ __forceinline__ int swz(int c) { return (c >> 2) & 3; }
};

template <int K, int CG>
__global__ __launch_bounds__(64 * (kWsMfma + kWsMem)) void k_bank_conv_ws(BankParams p) {
  using WG = WsGeom<K, CG>;
  using G = typename WG::G;
  constexpr int OT = 4, HP = G::HP, OTP = WG::OTP;
  constexpr int NTHR = 64 * (kWsMfma + kWsMem);
  extern __shared__ uint4 smem4[];
  uint16_t* wl = reinterpret_cast<uint16_t*>(smem4);
  uint16_t* sl0 = wl + G::W_ELEMS;
  char* rb = reinterpret_cast<char*>(sl0 + 2 * G::S_ELEMS);
  const int tid = threadIdx.x;
  const int lane = tid % 64;
  const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
  const bool mem = wave >= kWsMfma;  // uniform per wave
  const int mw = wave - kWsMfma;
  // MFMA waves: as in k_bank_conv
  const int wrow = wave % kTH;
  const int wcol = (wave / kTH) * (G::TW / G::WPR);
  const int l16 = lane % 16, q = lane / 16;
  const uint16_t* w_lane = wl + l16 * G::WSTR + q * 8;
  const int b_off = (wrow * G::LW + wcol + l16 + G::XOFF) * G::PS + (CG >= 4 ? q * 8 : (CG == 2 ? (q & 1) * 8 : 0));
  const bool hsel = (q >> 1) != 0;

  const uint32_t pg = static_cast<uint32_t>(static_cast<int64_t>(p.tiles_x) * p.tiles_y);
  const uint32_t tx = static_cast<uint32_t>(p.tiles_x), ngr = static_cast<uint32_t>(p.o_groups);
  auto decode = [&](int64_t t64, int64_t& n, int& og, int64_t& oy0, int64_t& ox0) __attribute__((always_inline)) {
    const uint32_t t = static_cast<uint32_t>(t64);
    const uint32_t ng = t / pg, r = t - ng * pg;
    og = static_cast<int>(ng % ngr);
    n = ng / ngr;
    const uint32_t tile_y = r / tx, tile_x = r - tile_y * tx;
    oy0 = static_cast<int64_t>(tile_y) * kTH;
    ox0 = static_cast<int64_t>(tile_x) * G::TW;
  };

  // memory wave mw: results of tile row mw % kTH (MFMA waves mw % kTH and
  // mw % kTH + 4), its share of the channels, from result buffer rbuf to the
  // output, one 16-byte chunk per lane and instruction (8 channels x 128 bytes)
  auto store_results = [&](int rbuf, int64_t hn, int hco, int64_t hoy, int64_t hox) __attribute__((always_inline)) {
    constexpr int PARTS = kWsMem / kTH;  // memory waves per tile row
    const int mrow = mw % kTH, part = mw / kTH;
    const char* pair = rb + rbuf * WG::RBUF_B + mrow * WG::PAIR_B;
    const int64_t oy = hoy + mrow;
    if (oy >= p.rows) return;
    constexpr int CPI = 8;  // channels per instruction
    constexpr int NI = OTP * 16 / CPI / PARTS;
    static_assert(kWsMem % kTH == 0 && (OTP * 16 / CPI) % PARTS == 0, "store split");
#pragma unroll
    for (int i = part * NI; i < part * NI + NI; ++i) {
      const int c = CPI * i + lane / (64 / CPI);
      const int mm = lane % (64 / CPI);
      const int h = mm / (32 / WG::EPC), m = mm % (32 / WG::EPC);
      const u32x4 v = *reinterpret_cast<const u32x4*>(pair + h * (WG::REG_B + 256) + c * WG::ROW_B +
                                                      ((m ^ WG::swz(c)) * 16));
      const int co = hco + c;
      const int64_t ox = hox + 32 * h + m * WG::EPC;
      if (co >= p.CO) continue;
      char* dp = static_cast<char*>(p.dst) + (hn * p.d_sn + static_cast<int64_t>(co) * p.d_sc + oy * p.d_sh + ox) * 2;
      if (ox + WG::EPC <= p.W && (reinterpret_cast<uintptr_t>(dp) & 15) == 0) {
        *reinterpret_cast<u32x4*>(dp) = v;
      } else {
#pragma unroll
        for (int e = 0; e < WG::EPC; ++e)
          if (ox + e < p.W) reinterpret_cast<uint16_t*>(dp)[e] = static_cast<uint16_t>(v[e / 2] >> (16 * (e % 2)));
      }
    }
  };

  // Both roles walk the same tiles and pass the same barriers (one per tile,
  // plus one when the output group changes); each role has its own loop, so
  // that its registers are not held across the other role's code.
  // XCD-aware start: the work-groups resident on one XCD take consecutive
  // tiles, so the halo lines neighbouring tiles share are read once into
  // that XCD's L2 (the stride below keeps every round contiguous)
  int64_t t = xcd_remap(blockIdx.x, gridDim.x);
  if (t >= p.n_tiles) return;
  int64_t n, oy0, ox0;
  int og;
  decode(t, n, og, oy0, ox0);
  load_weights<G, K, OT, CG, false, NTHR>(p, og, tid, wl);

  if (!mem) {
    __syncthreads();  // weights and the first tile in LDS
    int cur = 0, ri = 0;
    while (true) {
      const int64_t t_next = t + gridDim.x;
      const bool more = t_next < p.n_tiles;
      int64_t n2, oy2, ox2;
      int og2;
      decode(more ? t_next : t, n2, og2, oy2, ox2);
      {
        f32x4 acc[OTP][HP];
        const uint16_t* b_lane = sl0 + cur * G::S_ELEMS + b_off;
        auto xsrc = [&](auto step) __attribute__((always_inline)) {
          return b_lane + b_step_offset<G, K, CG>(decltype(step)::value, hsel, q);
        };
        mfma_sweep<G, K, CG, OTP, HP>(w_lane, xsrc, q, acc, [](auto) __attribute__((always_inline)) {});
        // acc[a][b][j] = channel 16a + l16 of the interval, pixel 16b + 4q + j
        char* reg = rb + ri * WG::RBUF_B + (wave % 4) * WG::PAIR_B + (wave / 4) * (WG::REG_B + 256);
#pragma unroll
        for (int a = 0; a < OTP; ++a) {
          const int c = 16 * a + l16;
#pragma unroll
          for (int b = 0; b < HP; ++b) {
            const int m = 2 * b + (q >> 1);
            *reinterpret_cast<u32x2*>(reg + c * WG::ROW_B + ((m ^ WG::swz(c)) * 16) + (q & 1) * 8) =
                u32x2{pack_bf16x2(acc[a][b][0], acc[a][b][1]), pack_bf16x2(acc[a][b][2], acc[a][b][3])};
          }
        }
        __syncthreads();  // results in buffer ri; the next tile packed
        ri ^= 1;
      }
      if (!more) break;
      if (og2 != og) __syncthreads();  // the memory waves load the new weights
      t = t_next;
      og = og2;
      cur ^= 1;
    }
    return;
  }

  // memory waves: tile t0 staged now, tile t0+1's loads in flight; the loads
  // of tile t+2 are issued right after tile t+1 is packed, a tile ahead
  Raw<uint16_t, WG::NTM> st;
  stage_load<G, K, CG, false, uint16_t, kWsMem>(p, n, oy0, ox0, mw, lane, st);
  stage_store<G, K, CG, false, uint16_t, kWsMem>(p, oy0, ox0, mw, lane, st, sl0);
  {
    const int64_t t1 = t + gridDim.x < p.n_tiles ? t + gridDim.x : t;
    int64_t n1, oy1, ox1;
    int og1;
    decode(t1, n1, og1, oy1, ox1);
    stage_load<G, K, CG, false, uint16_t, kWsMem>(p, n1, oy1, ox1, mw, lane, st);
  }
  __syncthreads();
  bool have = false;  // the other result buffer holds an interval's results
  int64_t hn = 0, hoy = 0, hox = 0;
  int hco = 0;
  int cur = 0, ri = 0;
  while (true) {
    const int64_t t_next = t + gridDim.x;
    const bool more = t_next < p.n_tiles;
    int64_t n2, oy2, ox2;
    int og2;
    decode(more ? t_next : t, n2, og2, oy2, ox2);
    {
      if (have) store_results(ri ^ 1, hn, hco, hoy, hox);
      // pack tile t+1 (loaded a tile ago; tile t again at the end, harmless)
      // and start the loads of tile t+2
      stage_store<G, K, CG, false, uint16_t, kWsMem>(p, oy2, ox2, mw, lane, st, sl0 + (cur ^ 1) * G::S_ELEMS);
      const int64_t t3 = t_next + gridDim.x < p.n_tiles ? t_next + gridDim.x : (more ? t_next : t);
      int64_t n3, oy3, ox3;
      int og3;
      decode(t3, n3, og3, oy3, ox3);
      stage_load<G, K, CG, false, uint16_t, kWsMem>(p, n3, oy3, ox3, mw, lane, st);
      __syncthreads();
      have = true;
      hn = n;
      hoy = oy0;
      hox = ox0;
      hco = og * OTP * 16;
      ri ^= 1;
    }
    if (!more) break;
    if (og2 != og) {  // every MFMA wave is past its last read of the old weights
      load_weights<G, K, OT, CG, false, 64 * kWsMem>(p, og2, tid - 64 * kWsMfma, wl);
      __syncthreads();
    }
    t = t_next;
    n = n2;
    og = og2;
    oy0 = oy2;
    ox0 = ox2;
    cur ^= 1;
  }
  store_results(ri ^ 1, hn, hco, hoy, hox);
}

// ------------------------------------------------------------------ wgrad --

constexpr int kWgTH = 8;      // rows per wgrad tile
constexpr int kWgTW = 64;     // columns per wgrad tile (two 32-pixel steps)
constexpr int kWgUnits = 512; // persistent work-groups (partial sets) at most

struct WgradParams {
  const uint16_t* x;  // bf16 image
  int64_t x_sn, x_sc, x_sh;
  const void* g;  // upstream gradient (bf16 or f32)
  int64_t g_sn, g_sc, g_sh;
  float* partial;  // [unit][CO][CI][K*K]
  int64_t H, W;
  int32_t CI, CO;
  int32_t tiles_x, tiles_y;
  int32_t x_vec, g_vec;  // rows 16-byte aligned (x) / 16-byte-per-8-elements (g)
  int64_t n_tiles;       // N * tiles_y * tiles_x
  int32_t units;         // grid size: unit u takes tiles u, u + units, ...
};

template <int K>
struct WgGeom {
  static constexpr int R = (K - 1) / 2;
  static constexpr int LH = kWgTH + K - 1;
  static constexpr int LWP = kWgTW + 16;      // columns x0-8 .. x0+TW+7
  static constexpr int PLS = LH * LWP + 8;    // channel-plane stride (elements), staggers banks
  static constexpr int ELEMS = 16 * PLS;
  static constexpr int CHUNKS = LWP / 8;      // 16-byte chunks per staged row
  static constexpr int STAGE = 16 * LH * CHUNKS;  // staging tasks per tile
};

__device__ __forceinline__ uint32_t funnel16(uint32_t hi, uint32_t lo) {
  return __builtin_amdgcn_alignbit(hi, lo, 16);
}

// 8 consecutive bf16 starting at element E (8-R <= E <= 8+R) of the window
// held in w[0..11] (elements 0..23, two bf16 per dword, little endian).
template <int E>
__device__ __forceinline__ bf16x8 window8(const uint32_t (&w)[12]) {
  u32x4 r;
  if constexpr (E % 2 == 0) {
    r = u32x4{w[E / 2], w[E / 2 + 1], w[E / 2 + 2], w[E / 2 + 3]};
  } else {
    constexpr int d = E / 2;
    r = u32x4{funnel16(w[d + 1], w[d]), funnel16(w[d + 2], w[d + 1]), funnel16(w[d + 3], w[d + 2]),
              funnel16(w[d + 4], w[d + 3])};
  }
  return __builtin_bit_cast(bf16x8, r);
}

// eight upstream-gradient values of one row as a bf16 A fragment
__device__ __forceinline__ bf16x8 g_fragment(const uint16_t* src) {
  return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u32x4*>(src));
}
__device__ __forceinline__ bf16x8 g_fragment(const float* src) {
  const float4 a = reinterpret_cast<const float4*>(src)[0];
  const float4 b = reinterpret_cast<const float4*>(src)[1];
  const float f[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
  u32x4 r;
#pragma unroll
  for (int d = 0; d < 4; ++d)
    r[d] = pack_bf16x2(f[2 * d], f[2 * d + 1]);
  return __builtin_bit_cast(bf16x8, r);
}

// A fragments of this lane for one 32-pixel step: G-bar[o][y0 + m][xb .. xb+7]
// for the tile's rows m, zero outside the image or past C_out.
template <typename TG>
__device__ __forceinline__ void load_g(const WgradParams& p, const TG* gp, int o, int64_t y0, int64_t xb,
                                       bool fast, bf16x8 (&ga)[kWgTH]) {
  if (fast && y0 + kWgTH <= p.H) {  // uniform
    // every row inside the image: plain loads with nothing applied to the
    // values (a select on each loaded row here made every load wait for the
    // previous one: 2.84 -> 2.37 ms for the 5x5 bank once removed)
#pragma unroll
    for (int m = 0; m < kWgTH; ++m) ga[m] = g_fragment(gp + o * p.g_sc + (y0 + m) * p.g_sh + xb);
    return;
  }
#pragma unroll
  for (int m = 0; m < kWgTH; ++m) {
    const int64_t y = y0 + m;
    if (fast) {
      // rows past H are zeroed
      const int64_t yc = y < p.H ? y : p.H - 1;
      const bf16x8 v = g_fragment(gp + o * p.g_sc + yc * p.g_sh + xb);
      ga[m] = y < p.H ? v : bf16x8{};
    } else {
      u32x4 r = u32x4{0u, 0u, 0u, 0u};
      if (o < p.CO && y < p.H) {
        const TG* row = gp + o * p.g_sc + y * p.g_sh;
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          uint32_t lo = 0, hi = 0;
          if (xb + 2 * d < p.W) lo = load_bits<TG>(row + xb + 2 * d);
          if (xb + 2 * d + 1 < p.W) hi = load_bits<TG>(row + xb + 2 * d + 1);
          r[d] = lo | (hi << 16);
        }
      }
      ga[m] = __builtin_bit_cast(bf16x8, r);
    }
  }
}

// All taps of X row j of the tile against the resident G-bar rows: row j is
// source row y0 - R + j, which meets G-bar row m = j - u at vertical tap u.
// The K horizontal taps are shifts of one window read from LDS.
template <int K, int J>
__device__ __forceinline__ void wg_row(f32x4 (&acc)[K * K], const bf16x8 (&ga)[kWgTH],
                                       const uint16_t* __restrict__ win) {
  constexpr int R = (K - 1) / 2;
  uint32_t w[12] = {};  // only w[2..9] are read for R <= 4
  const uint32_t* wp = reinterpret_cast<const uint32_t*>(win + J * WgGeom<K>::LWP);
  if constexpr (R > 0) {  // elements 4..7 and 16..19 (R <= 4)
    const uint2 lo = *reinterpret_cast<const uint2*>(wp + 2);
    const uint2 hi = *reinterpret_cast<const uint2*>(wp + 8);
    w[2] = lo.x;
    w[3] = lo.y;
    w[8] = hi.x;
    w[9] = hi.y;
  }
  const u32x4 mid = *reinterpret_cast<const u32x4*>(wp + 4);
  w[4] = mid.x;
  w[5] = mid.y;
  w[6] = mid.z;
  w[7] = mid.w;
#pragma unroll
  for (int u = 0; u < K; ++u) {
    const int m = J - u;
    if (m < 0 || m >= kWgTH) continue;
#pragma unroll
    for (int v = 0; v < K; ++v) {
      bf16x8 b;
      switch (8 + v - R) {  // compile-time after unrolling
        case 4: b = window8<4>(w); break;
        case 5: b = window8<5>(w); break;
        case 6: b = window8<6>(w); break;
        case 7: b = window8<7>(w); break;
        case 9: b = window8<9>(w); break;
        case 10: b = window8<10>(w); break;
        case 11: b = window8<11>(w); break;
        case 12: b = window8<12>(w); break;
        default: b = window8<8>(w); break;
      }
      acc[u * K + v] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ga[m], b, acc[u * K + v], 0, 0, 0);
    }
  }
}

template <int K, int J>
__device__ __forceinline__ void wg_rows(f32x4 (&acc)[K * K], const bf16x8 (&ga)[kWgTH],
                                        const uint16_t* __restrict__ win) {
  if constexpr (J < WgGeom<K>::LH) {
    wg_row<K, J>(acc, ga, win);
    wg_rows<K, J + 1>(acc, ga, win);
  }
}

// Persistent work-group over 8 x 64-pixel tiles of all images.  Wave w owns
// output channels 16w .. 16w+15 against all (<= 16) input channels and all
// K*K taps (acc).  Per tile: stage the clamped X tile in LDS (channel planes,
// 16-byte chunks), then for each 32-pixel step hold the 8 G-bar row
// fragments in registers and sweep the LH source rows once.
template <int K, typename TG>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(2))) void k_bank_wgrad(WgradParams p) {
  using G = WgGeom<K>;
  static_assert(G::R <= 4, "K <= 9");
  __shared__ uint4 xs4[(G::ELEMS + 7) / 8];
  uint16_t* xs = reinterpret_cast<uint16_t*>(xs4);
  const int tid = threadIdx.x, lane = tid % 64;
  const int wave = __builtin_amdgcn_readfirstlane(tid / 64);
  const int l16 = lane % 16, q = lane / 16;
  const int o = wave * 16 + l16;  // A row (output channel) of this lane

  f32x4 acc[K * K];
#pragma unroll
  for (int e = 0; e < K * K; ++e) acc[e] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int64_t per_image = static_cast<int64_t>(p.tiles_x) * p.tiles_y;
  // XCD-aware start: the units on one XCD take consecutive tiles (whole tile
  // rows of one image), whose X halo rows and columns then come from L2
  for (int64_t t = xcd_remap(blockIdx.x, p.units); t < p.n_tiles; t += p.units) {
    const int64_t n = t / per_image, r = t - n * per_image;
    const int64_t y0 = (r / p.tiles_x) * kWgTH, x0 = (r % p.tiles_x) * kWgTW;
    const uint16_t* xp = p.x + n * p.x_sn;
    const TG* gp = static_cast<const TG*>(p.g) + n * p.g_sn;
    // X tile [ci][row][col], clamped; LDS column c <-> source column x0 - 8 + c
    const bool x_fast = p.x_vec && x0 - 8 >= 0 && x0 + kWgTW + 8 <= p.W;
    u32x4 sv[(G::STAGE + kThreads - 1) / kThreads];
#pragma unroll
    for (int it = 0; it < (G::STAGE + kThreads - 1) / kThreads; ++it) {
      const int task = tid + kThreads * it < G::STAGE ? tid + kThreads * it : G::STAGE - 1;
      const int c = task / (G::LH * G::CHUNKS), rest = task - c * (G::LH * G::CHUNKS);
      const int ly = rest / G::CHUNKS, ch = rest - ly * G::CHUNKS;
      int64_t gy = y0 - G::R + ly;
      gy = gy < 0 ? 0 : (gy >= p.H ? p.H - 1 : gy);
      const int ci = c < p.CI ? c : p.CI - 1;
      const uint16_t* row = xp + ci * p.x_sc + gy * p.x_sh;
      const int64_t gx = x0 - 8 + 8 * ch;
      if (x_fast) {
        sv[it] = *reinterpret_cast<const u32x4*>(row + gx);
      } else {
        uint32_t h[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          int64_t cx = gx + e;
          cx = cx < 0 ? 0 : (cx >= p.W ? p.W - 1 : cx);
          h[e] = row[cx];
        }
        sv[it] = u32x4{h[0] | (h[1] << 16), h[2] | (h[3] << 16), h[4] | (h[5] << 16), h[6] | (h[7] << 16)};
      }
    }
    const bool g_fast = p.g_vec && o < p.CO && x0 + kWgTW <= p.W;
    bf16x8 ga[kWgTH];
    load_g<TG>(p, gp, o, y0, x0 + 8 * q, g_fast, ga);
    __syncthreads();  // the previous tile's readers are done with the LDS
#pragma unroll
    for (int it = 0; it < (G::STAGE + kThreads - 1) / kThreads; ++it) {
      const int task = tid + kThreads * it;
      if (task >= G::STAGE) break;
      const int c = task / (G::LH * G::CHUNKS), rest = task - c * (G::LH * G::CHUNKS);
      const int ly = rest / G::CHUNKS, ch = rest - ly * G::CHUNKS;
      const u32x4 v = c < p.CI ? sv[it] : u32x4{0u, 0u, 0u, 0u};
      *reinterpret_cast<u32x4*>(xs + c * G::PLS + ly * G::LWP + 8 * ch) = v;
    }
    __syncthreads();
    // lane window: channel l16, columns 32 ks + 8q + {0..23} of every LDS row
    wg_rows<K, 0>(acc, ga, xs + l16 * G::PLS + 8 * q);
    load_g<TG>(p, gp, o, y0, x0 + 32 + 8 * q, g_fast, ga);
    wg_rows<K, 0>(acc, ga, xs + l16 * G::PLS + 32 + 8 * q);
  }
  // D[o = wave*16 + 4q + j][ci = l16]
  const int ci = l16;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int oo = wave * 16 + 4 * q + j;
    if (oo >= p.CO || ci >= p.CI) continue;
    float* dst = p.partial + ((static_cast<int64_t>(blockIdx.x) * p.CO + oo) * p.CI + ci) * (K * K);
#pragma unroll
    for (int e = 0; e < K * K; ++e) dst[e] = acc[e][j];
  }
}

// ------------------------------------------------------------- dispatch --

// Column segments for the row-ring kernels: at most 32 tile rows, at least
// ~4 per work-group when the columns allow, equal length within a column.
// False when there is nothing to do.
bool plan_segments(BankParams& p, int grid) {
  const int64_t cols = p.n_img * p.o_groups * static_cast<int64_t>(p.tiles_x);
  if (cols <= 0 || p.tiles_y <= 0) return false;
  int64_t spc = (p.tiles_y + 31) / 32;
  const int64_t want = (4 * static_cast<int64_t>(grid) + cols - 1) / cols;
  if (want > spc) spc = want < p.tiles_y ? want : p.tiles_y;
  const int64_t len = (p.tiles_y + spc - 1) / spc;
  p.seg_len = static_cast<int32_t>(len);
  p.seg_per_col = static_cast<int32_t>((p.tiles_y + len - 1) / len);
  p.n_segs = cols * p.seg_per_col;
  return true;
}

// Resident work-groups of `kern` on the current device (cached per device by
// the caller's statics).
hipError_t resident_groups(const void* kern, int threads, size_t lds, int* grid) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
  if (e != hipSuccess) return e;
  int per_cu = 0, cus = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, lds);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  *grid = (per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
  return hipSuccess;
}

// 33..64 source channels into at most 16 outputs: k_bank_conv_vr
template <int K, bool ADJ, typename TS, bool OB>
hipError_t conv_vr_go(const BankParams& pin, hipStream_t s) {
  using G = VrGeom<K>;
  BankParams p = pin;
  if (p.CO > 16 || p.CI > 64 || p.o_groups != 1 || !p.s_plan32) return hipErrorNotSupported;
  p.tiles_x = static_cast<int32_t>((p.cols + G::TW - 1) / G::TW);
  p.n_tiles = p.n_img * static_cast<int64_t>(p.tiles_x) * p.tiles_y;
  const size_t lds = G::LDS_B;
  const void* kern = reinterpret_cast<const void*>(k_bank_conv_vr<K, ADJ, TS, OB>);
  static std::mutex mu;
  static int dev_cached = -1, grid_cached = 0;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  int grid;
  {
    std::lock_guard<std::mutex> lk(mu);
    if (dev_cached != dev) {
      e = resident_groups(kern, 512, lds, &grid_cached);
      if (e != hipSuccess) return e;
      dev_cached = dev;
    }
    grid = grid_cached;
  }
  if (!plan_segments(p, grid)) return hipSuccess;
  const int64_t g = p.n_segs < grid ? p.n_segs : grid;
  hipLaunchKernelGGL((k_bank_conv_vr<K, ADJ, TS, OB>), dim3(static_cast<uint32_t>(g)), dim3(512), lds, s, p);
  return hipGetLastError();
}

template <int K, int OT, int PT, int CG, int NW, bool ADJ, typename TS, bool OB>
hipError_t conv_go(const BankParams& pin, hipStream_t s) {
  using G = ConvGeom<K, OT, PT, CG, NW>;
  BankParams p = pin;
  p.tiles_x = static_cast<int32_t>((p.cols + G::TW - 1) / G::TW);
  p.n_tiles = p.n_img * p.o_groups * static_cast<int64_t>(p.tiles_x) * p.tiles_y;
  constexpr bool RING = G::RINGED;
  static_assert(G::LDS_ELEMS * 2 <= 160 * 1024, "weights and source tiles exceed LDS");
  const size_t lds = static_cast<size_t>(G::LDS_ELEMS) * 2;
  static std::mutex mu;
  static int dev_cached = -1, grid_cached = 0;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  int grid;
  {
    std::lock_guard<std::mutex> lk(mu);
    if (dev_cached != dev) {
      const void* kern;
      if constexpr (RING)
        kern = reinterpret_cast<const void*>(k_bank_conv_ring<K, OT, PT, CG, ADJ, TS, OB>);
      else
        kern = reinterpret_cast<const void*>(k_bank_conv<K, OT, PT, CG, NW, ADJ, TS, OB>);
      e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
      if (e != hipSuccess) return e;
      int per_cu = 0, cus = 0;
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, G::THREADS, lds);
      if (e != hipSuccess) return e;
      e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
      if (e != hipSuccess) return e;
      grid_cached = (per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
      dev_cached = dev;
    }
    grid = grid_cached;
  }
  if constexpr (RING) {
    if (!plan_segments(p, grid)) return hipSuccess;
    const int64_t g = p.n_segs < grid ? p.n_segs : grid;
    hipLaunchKernelGGL((k_bank_conv_ring<K, OT, PT, CG, ADJ, TS, OB>), dim3(static_cast<uint32_t>(g)),
                       dim3(G::THREADS), lds, s, p);
    return hipGetLastError();
  }
  else {
    const int64_t g = p.n_tiles < grid ? p.n_tiles : grid;
    if (g <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_bank_conv<K, OT, PT, CG, NW, ADJ, TS, OB>), dim3(static_cast<uint32_t>(g)),
                       dim3(G::THREADS), lds, s, p);
    return hipGetLastError();
  }
}

template <int K, int CG>
hipError_t conv_ws_go(const BankParams& pin, hipStream_t s) {
  using WG = WsGeom<K, CG>;
  using G = typename WG::G;
  BankParams p = pin;
  p.tiles_x = static_cast<int32_t>((p.cols + G::TW - 1) / G::TW);
  p.n_tiles = p.n_img * p.o_groups * static_cast<int64_t>(p.tiles_x) * p.tiles_y;
  constexpr int threads = 64 * (kWsMfma + kWsMem);
  const size_t lds = WG::LDS_B;
  static std::mutex mu;
  static int dev_cached = -1, grid_cached = 0;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  int grid;
  {
    std::lock_guard<std::mutex> lk(mu);
    if (dev_cached != dev) {
      auto kern = k_bank_conv_ws<K, CG>;
      e = hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                              static_cast<int>(lds));
      if (e != hipSuccess) return e;
      int per_cu = 0, cus = 0;
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, lds);
      if (e != hipSuccess) return e;
      e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
      if (e != hipSuccess) return e;
      grid_cached = (per_cu > 0 ? per_cu : 1) * (cus > 0 ? cus : 1);
      dev_cached = dev;
    }
    grid = grid_cached;
  }
  const int64_t g = p.n_tiles < grid ? p.n_tiles : grid;
  if (g <= 0) return hipSuccess;
  hipLaunchKernelGGL((k_bank_conv_ws<K, CG>), dim3(static_cast<uint32_t>(g)), dim3(threads), lds, s, p);
  return hipGetLastError();
}

// 33..64 source channels, one 16-channel output block per pass: the
// vertical-reuse kernel for at most 16 outputs from BF16 sources with planned
// staging, else the row-ring kernel
template <int K, bool ADJ, typename TS, bool OB>
hipError_t conv_wide_go(const BankParams& p, hipStream_t s) {
  if constexpr (std::is_same<TS, uint16_t>::value) {
    if (p.s_plan32 && p.CO <= 16) return conv_vr_go<K, ADJ, TS, OB>(p, s);
  }
  return conv_go<K, 1, 4, 8, 8, ADJ, TS, OB>(p, s);
}

template <int K, bool ADJ, typename TS, bool OB>
hipError_t conv_by_shape(const BankParams& p, int ot, int cg, hipStream_t s) {
  // instantiated (OT, CG) pairs, eight waves; 64-pixel tile rows (PT = 4),
  // 128 for 64 outputs from 9..16 inputs, where two source tiles of that
  // width still fit beside the weights; the adjoint's outputs are the
  // forward's input channels (<= 16, one tile)
  if constexpr (!ADJ) {
    if (ot == 4 && cg == 2) {
      // BF16 outputs: the wave-specialised kernel (measured 4-5% faster at
      // K = 5); FP32 outputs: the eight-wave kernel on 4 x 128 tiles
      // (the specialised one measured slower there)
      if constexpr (OB) return conv_ws_go<K, 2>(p, s);
      return conv_go<K, 4, 8, 2, 8, ADJ, TS, OB>(p, s);
    }
    if (ot == 4 && cg == 1) return conv_go<K, 4, 4, 1, 8, ADJ, TS, OB>(p, s);
    if constexpr (K < 5) {
      if (ot == 4 && cg == 4) return conv_go<K, 4, 4, 4, 8, ADJ, TS, OB>(p, s);
    }
    if (ot == 2 && cg == 4) return conv_go<K, 2, 4, 4, 8, ADJ, TS, OB>(p, s);
    if (ot == 1 && cg == 4) return conv_go<K, 1, 4, 4, 8, ADJ, TS, OB>(p, s);
    if (ot == 2 && cg == 1) return conv_go<K, 2, 4, 1, 8, ADJ, TS, OB>(p, s);
    if (ot == 2 && cg == 2) return conv_go<K, 2, 4, 2, 8, ADJ, TS, OB>(p, s);
    if constexpr (K < 5) {
      if (ot == 2 && cg == 8) return conv_go<K, 2, 4, 8, 8, ADJ, TS, OB>(p, s);
    }
    if (ot == 1 && cg == 1) return conv_go<K, 1, 4, 1, 8, ADJ, TS, OB>(p, s);
    if (ot == 1 && cg == 2) return conv_go<K, 1, 4, 2, 8, ADJ, TS, OB>(p, s);
    if (ot == 1 && cg == 8) return conv_wide_go<K, ADJ, TS, OB>(p, s);
  } else {
    if (ot == 1 && cg == 8) return conv_wide_go<K, ADJ, TS, OB>(p, s);
    if (ot == 1 && cg == 4) return conv_go<K, 1, 4, 4, 8, ADJ, TS, OB>(p, s);
    if (ot == 1 && cg == 2) return conv_go<K, 1, 4, 2, 8, ADJ, TS, OB>(p, s);
    if (ot == 1 && cg == 1) return conv_go<K, 1, 4, 1, 8, ADJ, TS, OB>(p, s);
  }
  return hipErrorNotSupported;
}

template <bool ADJ, typename TS, bool OB>
hipError_t conv_by_k(const BankParams& p, int K, int ot, int cg, hipStream_t s) {
  switch (K) {
    case 1: return conv_by_shape<1, ADJ, TS, OB>(p, ot, cg, s);
    case 3: return conv_by_shape<3, ADJ, TS, OB>(p, ot, cg, s);
    case 5: return conv_by_shape<5, ADJ, TS, OB>(p, ot, cg, s);
    default: return hipErrorNotSupported;
  }
}

// output-channel tiles per work-group and channel groups of 8 for a map
// with ci source and co output channels
bool conv_shape(int64_t ci, int64_t co, int k, int* ot, int* cg) {
  const int64_t g8 = (ci + 7) / 8;
  if (g8 > 8) return false;
  *cg = g8 <= 1 ? 1 : (g8 <= 2 ? 2 : (g8 <= 4 ? 4 : 8));
  *ot = co <= 16 ? 1 : (co <= 32 ? 2 : 4);
  // keep weights + source tile within LDS
  if (*cg == 8 && *ot == 4) *ot = 2;
  if (*cg == 8 && k == 5) *ot = 1;
  if (*cg == 4 && *ot == 4 && k == 5) *ot = 2;
  return true;
}

// persistent wgrad grid: units work-groups over n_tiles tiles
// One image of a staged source (c channels) spans < 2^31 elements, with H
// and the row stride below 2^24 (the ring kernel's 32-bit staging offsets).
bool plan32_fits(const f2d_tensor& t, int64_t c) {
  const int64_t extent = (c - 1) * t.stride_c + (t.h - 1) * t.stride_h + t.w;
  return extent < (int64_t{1} << 31) && t.h < (int64_t{1} << 24) && t.stride_h < (int64_t{1} << 24);
}

size_t wgrad_bytes(const Problem& pr, int32_t* units, int64_t* n_tiles, int32_t* tx, int32_t* ty) {
  const f2d_tensor& im = pr.image;
  *tx = static_cast<int32_t>((im.w + kWgTW - 1) / kWgTW);
  *ty = static_cast<int32_t>((im.h + kWgTH - 1) / kWgTH);
  *n_tiles = im.n * static_cast<int64_t>(*tx) * *ty;
  *units = static_cast<int32_t>(*n_tiles < kWgUnits ? *n_tiles : kWgUnits);
  return static_cast<size_t>(*units) * pr.c_out * im.c * pr.k * pr.k * sizeof(float);
}

}  // namespace

f2d_status bank_forward_bf16(const Problem& pr, const f2d_tensor* outs, hipStream_t s) {
  const f2d_tensor& im = pr.image;
  const f2d_tensor& out = outs[0];
  int ot, cg;
  if (!conv_shape(im.c, pr.c_out, pr.k, &ot, &cg))
    return fail(F2D_EUNSUPPORTED, "bf16 banks: at most 64 input channels");
  if (pr.k != 1 && pr.k != 3 && pr.k != 5) return fail(F2D_EUNSUPPORTED, "bf16 banks: k in {1, 3, 5}");
  BankParams p;
  std::memset(&p, 0, sizeof(p));
  p.src = im.data;
  p.s_sn = im.stride_n;
  p.s_sc = im.stride_c;
  p.s_sh = im.stride_h;
  p.s_vec = row_aligned(im, 16) && im.w % 8 == 0 ? 1 : 0;
  p.s_plan32 = p.s_vec && plan32_fits(im, im.c) ? 1 : 0;
  p.dst = out.data;
  p.d_sn = out.stride_n;
  p.d_sc = out.stride_c;
  p.d_sh = out.stride_h;
  p.d_vec = row_aligned(out, out.dtype == F2D_BF16 ? 8 : 16) ? 1 : 0;
  p.w = static_cast<const uint16_t*>(pr.filter.data);
  p.H = im.h;
  p.W = im.w;
  p.row0 = pr.row_begin;
  p.rows = pr.rows;
  p.CI = static_cast<int32_t>(im.c);
  p.CO = static_cast<int32_t>(pr.c_out);
  p.fo = pr.filter.f_out;
  p.fi = pr.filter.f_in;
  p.o_groups = static_cast<int32_t>((pr.c_out + ot * 16 - 1) / (ot * 16));
  p.n_img = im.n;
  p.cols = im.w;
  p.tiles_y = static_cast<int32_t>((pr.rows + kTH - 1) / kTH);
  hipError_t e = out.dtype == F2D_BF16 ? conv_by_k<false, uint16_t, true>(p, pr.k, ot, cg, s)
                                       : conv_by_k<false, uint16_t, false>(p, pr.k, ot, cg, s);
  if (e == hipErrorNotSupported) return fail(F2D_EUNSUPPORTED, "bf16 banks: channel counts not supported");
  return hip_status(e, "bf16 bank forward launch");
}

size_t bank_frame_bytes(const Problem& pr) {
  const int64_t r = (pr.k - 1) / 2;
  const size_t b = static_cast<size_t>(pr.image.n * pr.image.c) *
                   frame_plane_size(pr.image.h, pr.image.w, r) * sizeof(float);
  return (b + 255) & ~static_cast<size_t>(255);
}

size_t bank_backward_bf16_workspace(const Problem& pr) {
  int32_t units, tx, ty;
  int64_t n_tiles;
  const size_t b = wgrad_bytes(pr, &units, &n_tiles, &tx, &ty);
  return bank_frame_bytes(pr) + ((b + 255) & ~static_cast<size_t>(255)) + 256;
}

f2d_status bank_backward_bf16(const Problem& pr, const f2d_tensor& gout, const f2d_tensor* grad_input,
                              float* grad_filter, void* ws, size_t ws_bytes, hipStream_t s) {
  (void)ws_bytes;
  const f2d_tensor& im = pr.image;
  if (pr.mode != F2D_CH_BANK) return fail(F2D_EUNSUPPORTED, "bf16 images: only BANK mode");
  if (pr.k != 1 && pr.k != 3 && pr.k != 5) return fail(F2D_EUNSUPPORTED, "bf16 banks: k in {1, 3, 5}");
  if (im.c > 16 || pr.c_out > 64) return fail(F2D_EUNSUPPORTED, "bf16 bank backward: C_in <= 16 and C_out <= 64");
  const bool empty = im.n == 0 || im.c == 0 || im.h == 0 || im.w == 0 || pr.c_out == 0;
  const bool g32 = gout.dtype == F2D_F32;
  if (grad_input && !empty) {
    int ot, cg;
    if (!conv_shape(pr.c_out, im.c, pr.k, &ot, &cg)) return fail(F2D_EUNSUPPORTED, "bf16 bank backward shape");
    BankParams p;
    std::memset(&p, 0, sizeof(p));
    p.src = gout.data;
    p.s_sn = gout.stride_n;
    p.s_sc = gout.stride_c;
    p.s_sh = gout.stride_h;
    p.s_vec = row_aligned(gout, 16) && im.w % 8 == 0 ? 1 : 0;
    p.s_plan32 = p.s_vec && plan32_fits(gout, pr.c_out) ? 1 : 0;
    p.dst = grad_input->data;
    p.d_sn = grad_input->stride_n;
    p.d_sc = grad_input->stride_c;
    p.d_sh = grad_input->stride_h;
    p.d_vec = row_aligned(*grad_input, 16) ? 1 : 0;
    p.w = static_cast<const uint16_t*>(pr.filter.data);
    const int64_t r = (pr.k - 1) / 2;
    p.H = im.h;
    p.W = im.w;
    p.row0 = -r;  // the image and its r-wide frame
    p.rows = im.h + 2 * r;
    // tile columns start 4-aligned left of the frame (columns < -r are skipped)
    p.col0 = -8;  // 8-aligned staging chunks; columns < -r are skipped
    p.fr = static_cast<int32_t>(r);
    p.frame = static_cast<float*>(ws);
    p.frame_plane = frame_plane_size(im.h, im.w, r);
    p.CI = static_cast<int32_t>(pr.c_out);
    p.CO = static_cast<int32_t>(im.c);
    p.fo = pr.filter.f_out;
    p.fi = pr.filter.f_in;
    p.o_groups = static_cast<int32_t>((im.c + ot * 16 - 1) / (ot * 16));
    p.n_img = im.n;
    p.cols = im.w + r - p.col0;
    p.tiles_y = static_cast<int32_t>((p.rows + kTH - 1) / kTH);
    hipError_t e = g32 ? conv_by_k<true, float, false>(p, pr.k, ot, cg, s)
                       : conv_by_k<true, uint16_t, false>(p, pr.k, ot, cg, s);
    if (e != hipSuccess) return hip_status(e, "bf16 bank dgrad launch");
    FoldParams fo;
    fo.frame = p.frame;
    fo.frame_plane = p.frame_plane;
    fo.out = static_cast<float*>(grad_input->data);
    fo.out_sn = grad_input->stride_n;
    fo.out_sc = grad_input->stride_c;
    fo.out_sh = grad_input->stride_h;
    fo.H = im.h;
    fo.W = im.w;
    fo.r = r;
    fo.planes = im.n * im.c;
    fo.groups = im.c;
    e = launch_fold_frame(fo, s);
    if (e != hipSuccess) return hip_status(e, "bf16 bank fold launch");
  }
  if (grad_filter) {
    int32_t units, tx, ty;
    int64_t n_tiles;
    wgrad_bytes(pr, &units, &n_tiles, &tx, &ty);
    const int64_t nf = pr.c_out * im.c;
    if (!empty) {
      WgradParams w;
      std::memset(&w, 0, sizeof(w));
      w.x = static_cast<const uint16_t*>(im.data);
      w.x_sn = im.stride_n;
      w.x_sc = im.stride_c;
      w.x_sh = im.stride_h;
      w.g = gout.data;
      w.g_sn = gout.stride_n;
      w.g_sc = gout.stride_c;
      w.g_sh = gout.stride_h;
      w.partial = reinterpret_cast<float*>(static_cast<char*>(ws) + bank_frame_bytes(pr));
      w.H = im.h;
      w.W = im.w;
      w.CI = static_cast<int32_t>(im.c);
      w.CO = static_cast<int32_t>(pr.c_out);
      w.tiles_x = tx;
      w.tiles_y = ty;
      w.x_vec = row_aligned(im, 16) ? 1 : 0;
      w.g_vec = row_aligned(gout, g32 ? 32 : 16) ? 1 : 0;
      w.n_tiles = n_tiles;
      w.units = units;
      const dim3 grid(static_cast<uint32_t>(units)), block(kThreads);
      switch (pr.k) {
        case 1:
          if (g32) hipLaunchKernelGGL((k_bank_wgrad<1, float>), grid, block, 0, s, w);
          else hipLaunchKernelGGL((k_bank_wgrad<1, uint16_t>), grid, block, 0, s, w);
          break;
        case 3:
          if (g32) hipLaunchKernelGGL((k_bank_wgrad<3, float>), grid, block, 0, s, w);
          else hipLaunchKernelGGL((k_bank_wgrad<3, uint16_t>), grid, block, 0, s, w);
          break;
        default:
          if (g32) hipLaunchKernelGGL((k_bank_wgrad<5, float>), grid, block, 0, s, w);
          else hipLaunchKernelGGL((k_bank_wgrad<5, uint16_t>), grid, block, 0, s, w);
          break;
      }
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return hip_status(e, "bf16 bank wgrad launch");
    }
    // partial layout [unit][f][K*K] == reduce layout with nrep = units, chunks = 1
    hipError_t e = launch_reduce_partials(reinterpret_cast<float*>(static_cast<char*>(ws) + bank_frame_bytes(pr)),
                                          grad_filter, nf, pr.k * pr.k, empty ? 0 : units, 1, s);
    if (e != hipSuccess) return hip_status(e, "bf16 bank reduce launch");
  }
  return ok();
}

}  // namespace f2d
