// Device-side building blocks of the FP32 VALU stencil: tile geometry, LDS
// staging with the border rule, the register-blocked tap accumulation and the
// row stores.  Shared by the single-image kernels and the ragged-batch kernel,
// so both accumulate every output value in the same order.
#pragma once

#include "f2d_internal.hpp"

namespace f2d {
namespace tile {

constexpr int kThreads = 256;
constexpr int kTX = 16;  // threads along x
constexpr int kTY = 16;  // threads along y
constexpr int kMaxTaps = 100;  // NOUT*K*K taps held in scalar registers

template <int K, int PX, int PY>
struct Geom {
  static constexpr int R = (K - 1) / 2;
  static constexpr int TW = kTX * PX;
  static constexpr int TH = kTY * PY;
  static constexpr int LW = TW + K - 1;  // staged columns
  static constexpr int LH = TH + K - 1;  // staged rows
  static constexpr int WIN = PX + K - 1;
  static constexpr int WIN4 = (WIN + 3) / 4 * 4;
  // every thread reads WIN4 words starting at tx*PX: the row pitch must cover
  // the last thread's read; keep rows 16-byte aligned for ds_read_b128.
  static constexpr int PITCH = ((TW - PX + WIN4) > LW ? (TW - PX + WIN4) : LW) + 3 & ~3;
  static constexpr int LDS_WORDS = LH * PITCH;
  static_assert(PX % 4 == 0, "windows are read as float4");
};

// Uniform values passed through an empty asm statement: the optimiser can no
// longer see that they are neighbouring kernel-argument words, so it keeps the
// compare-and-select chains below as selects instead of rewriting them into a
// dynamically indexed load, which would copy the whole argument block to scratch.
__device__ __forceinline__ int64_t opaque(int64_t v) {
  asm volatile("" : "+s"(v));
  return v;
}

template <typename T>
__device__ __forceinline__ T* opaque_ptr(T* v) {
  return reinterpret_cast<T*>(opaque(reinterpret_cast<int64_t>(v)));
}

// Select plane t (< kMaxT) of a pointer/stride table and offset it to (n, ch).
template <typename T>
__device__ __forceinline__ T* pick_plane(T* const (&base)[kMaxT], const int64_t (&sn)[kMaxT],
                                         const int64_t (&sc)[kMaxT], const int64_t (&sh)[kMaxT],
                                         int t, int64_t n, int64_t ch, int64_t& row_stride) {
  T* b = opaque_ptr(base[0]);
  int64_t a = opaque(sn[0]), c = opaque(sc[0]), h = opaque(sh[0]);
#pragma unroll
  for (int q = 1; q < kMaxT; ++q) {
    T* bq = opaque_ptr(base[q]);
    const int64_t aq = opaque(sn[q]), cq = opaque(sc[q]), hq = opaque(sh[q]);
    b = t == q ? bq : b;
    a = t == q ? aq : a;
    c = t == q ? cq : c;
    h = t == q ? hq : h;
  }
  row_stride = h;
  return b + n * a + ch * c;
}

__device__ __forceinline__ const float* src_plane(const StencilParams& p, int t, int64_t n,
                                                  int64_t ch, int64_t& sh) {
  const float* const(&base)[kMaxT] = reinterpret_cast<const float* const(&)[kMaxT]>(p.src);
  return pick_plane(base, p.src_sn, p.src_sc, p.src_sh, t, n, ch, sh);
}

__device__ __forceinline__ float* dst_plane(const StencilParams& p, int t, int64_t n, int64_t ch,
                                            int64_t& sh) {
  float* const(&base)[kMaxT] = reinterpret_cast<float* const(&)[kMaxT]>(p.dst);
  return pick_plane(base, p.dst_sn, p.dst_sc, p.dst_sh, t, n, ch, sh);
}

// Stage one source plane's tile (source rows row_base-R.., columns
// col_base-R..) in LDS.  Waves take whole rows (one row address per wave);
// lanes take columns, and each lane's clamped
// (or zero-masked) column offset is computed once for every row.  All of a
// wave's loads are issued into registers before the first LDS write, so the
// wave waits on memory once per tile instead of once per row.
//
// UNI: take the wave index as uniform, so that row indices, clamps and row
// addresses are scalar and each load is scalar base + 32-bit lane offset.
// This shortens single-output kernels; kernels that stage many source planes
// per tile keep the per-lane form, which measured faster there.
//
// SP is the source pointer type: a plain pointer, or one qualified with the
// global address space where the compiler cannot infer it.
template <int K, int PX, int PY, bool ADJ, bool UNI = true, typename SP = const float*>
__device__ __forceinline__ void stage_tile(float* __restrict__ lds, SP __restrict__ sp,
                                           int64_t sh, int64_t H, int64_t W, int64_t row_base,
                                           int64_t col_base) {
  using G = Geom<K, PX, PY>;
  constexpr int kWaveLanes = 64;
  constexpr int kWaves = kThreads / kWaveLanes;
  constexpr int CPL = (G::LW + kWaveLanes - 1) / kWaveLanes;  // column chunks per lane
  constexpr int RPW = (G::LH + kWaves - 1) / kWaves;          // rows per wave
  const int lane = threadIdx.x % kWaveLanes;
  const int wave = UNI ? __builtin_amdgcn_readfirstlane(threadIdx.x / kWaveLanes)
                       : static_cast<int>(threadIdx.x / kWaveLanes);
  uint32_t coff[CPL];
  bool cval[CPL];
#pragma unroll
  for (int j = 0; j < CPL; ++j) {
    const int lx = lane + kWaveLanes * j;
    const int64_t gx = col_base - G::R + lx;
    if constexpr (ADJ) {
      cval[j] = gx >= 0 && gx < W;
      coff[j] = cval[j] ? static_cast<uint32_t>(gx) : 0u;
    } else {
      cval[j] = true;
      coff[j] = static_cast<uint32_t>(gx < 0 ? 0 : (gx >= W ? W - 1 : gx));
    }
  }
  float buf[RPW][CPL];
  if constexpr (ADJ) {
    // Every load is unconditional (the addresses are always valid) and the
    // zero mask is applied at the LDS write: masking each loaded value had
    // the compiler branch around each load and wait for it in turn.
    bool rval[RPW];
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const int ly = wave + kWaves * i;
      const int64_t gy = row_base - G::R + (ly < G::LH ? ly : G::LH - 1);
      rval[i] = gy >= 0 && gy < H;
      const SP rp = sp + (rval[i] ? gy : 0) * sh;
#pragma unroll
      for (int j = 0; j < CPL; ++j) buf[i][j] = rp[coff[j]];
    }
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const int ly = wave + kWaves * i;
#pragma unroll
      for (int j = 0; j < CPL; ++j) {
        const int lx = lane + kWaveLanes * j;
        const float v = (rval[i] && cval[j]) ? buf[i][j] : 0.0f;
        if (ly < G::LH && lx < G::LW) lds[ly * G::PITCH + lx] = v;
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const int ly = wave + kWaves * i;
      int64_t gy = row_base - G::R + (ly < G::LH ? ly : G::LH - 1);
      gy = gy < 0 ? 0 : (gy >= H ? H - 1 : gy);
      const SP rp = sp + gy * sh;
#pragma unroll
      for (int j = 0; j < CPL; ++j) buf[i][j] = rp[coff[j]];
    }
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const int ly = wave + kWaves * i;
#pragma unroll
      for (int j = 0; j < CPL; ++j) {
        const int lx = lane + kWaveLanes * j;
        if (ly < G::LH && lx < G::LW) lds[ly * G::PITCH + lx] = buf[i][j];
      }
    }
  }
}

// acc[j][jy][px] += sum_{u,v} tap_j[u][v] * tile[ty*PY+jy+u][tx*PX+px+v]
template <int K, int NOUT, int PX, int PY>
__device__ __forceinline__ void accumulate(const float* __restrict__ lds,
                                           const float (&tap)[NOUT][K * K],
                                           float (&acc)[NOUT][PY][PX]) {
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
        for (int j = 0; j < NOUT; ++j)
#pragma unroll
          for (int px = 0; px < PX; ++px)
            acc[j][jy][px] = __builtin_fmaf(tap[j][u * K + v], win[px + v], acc[j][jy][px]);
    }
  }
}

typedef float f32x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ void store4(float* p, f32x4_t v) { *reinterpret_cast<f32x4_t*>(p) = v; }
__device__ __forceinline__ void store4(__attribute__((address_space(1))) float* p, f32x4_t v) {
  *reinterpret_cast<__attribute__((address_space(1))) f32x4_t*>(p) = v;
}

// DP: plain or global-address-space output pointer (see stage_tile).
template <int PX, typename DP = float*>
__device__ __forceinline__ void store_row(DP __restrict__ dp, int64_t x0, int64_t W, bool vec,
                                          const float (&v)[PX]) {
  if (vec && x0 + PX <= W) {
#pragma unroll
    for (int q = 0; q < PX / 4; ++q)
      store4(dp + x0 + 4 * q, f32x4_t{v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]});
  } else {
#pragma unroll
    for (int px = 0; px < PX; ++px)
      if (x0 + px < W) dp[x0 + px] = v[px];
  }
}

}  // namespace tile
}  // namespace f2d
