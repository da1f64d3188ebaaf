/*
 * oracle.c -- plain CPU reference for the clamp-to-edge K x K 2D filter.
 *
 * TEST INFRASTRUCTURE ONLY: called by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the GPU library.  It shares no code,
 * header, table or helper with the GPU path.
 *
 * Every function is the definition written out as direct loops (no tiling,
 * no blocking, no reordering beyond the loop nest of the definition).  The
 * only parallelism is an OpenMP "parallel for" over independent outer loop
 * indices, which does not change any result.
 *
 * The definition generalises the paper's Laplacian sharpen (Section 4.2.4):
 * a weighted sum over a K x K neighbourhood, per channel; the readings taken
 * where the paper is silent are: correlation (not convolution), clamp-to-edge
 * borders per axis, odd K anchored at the centre.
 */
#include "oracle.h"

#include <math.h>
#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* clamp-to-edge index map: cl_n(t) = min(max(t, 0), n - 1) */
static int64_t cl(int64_t t, int64_t n) {
  if (t < 0) return 0;
  if (t > n - 1) return n - 1;
  return t;
}

/* Validate the channel mode and return the number of output channels, or -1. */
static int64_t out_channels(int64_t C, int64_t FO, int64_t FI, int64_t K, int32_t mode) {
  if (K < 1 || (K % 2) == 0) return -1;
  if (mode == ORACLE_SHARED) {
    if (FO != 1 || FI != 1) return -1;
    return C;
  }
  if (mode == ORACLE_DEPTHWISE) {
    if (FI != 1 || C < 1 || FO < C || (FO % C) != 0) return -1;
    return FO;
  }
  if (mode == ORACLE_BANK) {
    if (FI != C || FO < 1) return -1;
    return FO;
  }
  return -1;
}

/* For output channel o, input channel number t (0 <= t < n_inputs(o)):
 * which input channel it reads and which filter [fo][fi] it uses. */
static int64_t n_inputs(int64_t C, int32_t mode) { return mode == ORACLE_BANK ? C : 1; }

static void input_of(int64_t o, int64_t t, int64_t C, int64_t FO, int32_t mode, int64_t* in_ch,
                     int64_t* fo, int64_t* fi) {
  if (mode == ORACLE_SHARED) {
    *in_ch = o;
    *fo = 0;
    *fi = 0;
  } else if (mode == ORACLE_DEPTHWISE) {
    int64_t m = FO / C;
    *in_ch = o / m;
    *fo = o;
    *fi = 0;
  } else {
    *in_ch = t;
    *fo = o;
    *fi = t;
  }
}

int oracle_forward_f64(const double* x, int64_t N, int64_t C, int64_t H, int64_t W,
                       const double* f, int64_t FO, int64_t FI, int64_t K, int32_t mode,
                       int64_t y0, int64_t y1, double* out) {
  int64_t CO = out_channels(C, FO, FI, K, mode);
  if (CO < 0 || N < 0 || H < 0 || W < 0 || y0 < 0 || y1 < y0 || y1 > H) return -1;
  if (N == 0 || H == 0 || W == 0 || y1 == y0) return 0;
  int64_t r = (K - 1) / 2, rows = y1 - y0;
  int64_t planes = N * CO;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t p = 0; p < planes * rows; ++p) {
    int64_t n = (p / rows) / CO, o = (p / rows) % CO, y = y0 + p % rows;
    for (int64_t xx = 0; xx < W; ++xx) {
      double acc = 0.0;
      for (int64_t t = 0; t < n_inputs(C, mode); ++t) {
        int64_t i, fo, fi;
        input_of(o, t, C, FO, mode, &i, &fo, &fi);
        const double* xi = x + (n * C + i) * H * W;
        const double* ff = f + (fo * FI + fi) * K * K;
        for (int64_t u = 0; u < K; ++u)
          for (int64_t v = 0; v < K; ++v)
            acc += ff[u * K + v] * xi[cl(y + u - r, H) * W + cl(xx + v - r, W)];
      }
      out[((n * CO + o) * rows + (y - y0)) * W + xx] = acc;
    }
  }
  return 0;
}

/*
 * Zero border: a neighbour outside the image contributes nothing, which is
 * what the paper's sharpen does when it skips out-of-image neighbours
 * (Section 4.2.4).  Same loop nest as oracle_forward_f64; only the border
 * rule differs.
 */
int oracle_forward_zero_f64(const double* x, int64_t N, int64_t C, int64_t H, int64_t W,
                            const double* f, int64_t FO, int64_t FI, int64_t K, int32_t mode,
                            int64_t y0, int64_t y1, double* out) {
  int64_t CO = out_channels(C, FO, FI, K, mode);
  if (CO < 0 || N < 0 || H < 0 || W < 0 || y0 < 0 || y1 < y0 || y1 > H) return -1;
  if (N == 0 || H == 0 || W == 0 || y1 == y0) return 0;
  int64_t r = (K - 1) / 2, rows = y1 - y0;
  int64_t planes = N * CO;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t p = 0; p < planes * rows; ++p) {
    int64_t n = (p / rows) / CO, o = (p / rows) % CO, y = y0 + p % rows;
    for (int64_t xx = 0; xx < W; ++xx) {
      double acc = 0.0;
      for (int64_t t = 0; t < n_inputs(C, mode); ++t) {
        int64_t i, fo, fi;
        input_of(o, t, C, FO, mode, &i, &fo, &fi);
        const double* xi = x + (n * C + i) * H * W;
        const double* ff = f + (fo * FI + fi) * K * K;
        for (int64_t u = 0; u < K; ++u) {
          int64_t sy = y + u - r;
          if (sy < 0 || sy >= H) continue;
          for (int64_t v = 0; v < K; ++v) {
            int64_t sx = xx + v - r;
            if (sx < 0 || sx >= W) continue;
            acc += ff[u * K + v] * xi[sy * W + sx];
          }
        }
      }
      out[((n * CO + o) * rows + (y - y0)) * W + xx] = acc;
    }
  }
  return 0;
}

int oracle_forward_i64(const int64_t* x, int64_t N, int64_t C, int64_t H, int64_t W,
                       const int64_t* f, int64_t FO, int64_t FI, int64_t K, int32_t mode,
                       int64_t y0, int64_t y1, int64_t* out) {
  int64_t CO = out_channels(C, FO, FI, K, mode);
  if (CO < 0 || N < 0 || H < 0 || W < 0 || y0 < 0 || y1 < y0 || y1 > H) return -1;
  if (N == 0 || H == 0 || W == 0 || y1 == y0) return 0;
  int64_t r = (K - 1) / 2, rows = y1 - y0;
  int64_t planes = N * CO;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t p = 0; p < planes * rows; ++p) {
    int64_t n = (p / rows) / CO, o = (p / rows) % CO, y = y0 + p % rows;
    for (int64_t xx = 0; xx < W; ++xx) {
      int64_t acc = 0;
      for (int64_t t = 0; t < n_inputs(C, mode); ++t) {
        int64_t i, fo, fi;
        input_of(o, t, C, FO, mode, &i, &fo, &fi);
        const int64_t* xi = x + (n * C + i) * H * W;
        const int64_t* ff = f + (fo * FI + fi) * K * K;
        for (int64_t u = 0; u < K; ++u)
          for (int64_t v = 0; v < K; ++v)
            acc += ff[u * K + v] * xi[cl(y + u - r, H) * W + cl(xx + v - r, W)];
      }
      out[((n * CO + o) * rows + (y - y0)) * W + xx] = acc;
    }
  }
  return 0;
}

/* Zero-border int64 forward (out-of-image neighbours add nothing). */
int oracle_forward_zero_i64(const int64_t* x, int64_t N, int64_t C, int64_t H, int64_t W,
                       const int64_t* f, int64_t FO, int64_t FI, int64_t K, int32_t mode,
                       int64_t y0, int64_t y1, int64_t* out) {
  int64_t CO = out_channels(C, FO, FI, K, mode);
  if (CO < 0 || N < 0 || H < 0 || W < 0 || y0 < 0 || y1 < y0 || y1 > H) return -1;
  if (N == 0 || H == 0 || W == 0 || y1 == y0) return 0;
  int64_t r = (K - 1) / 2, rows = y1 - y0;
  int64_t planes = N * CO;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t p = 0; p < planes * rows; ++p) {
    int64_t n = (p / rows) / CO, o = (p / rows) % CO, y = y0 + p % rows;
    for (int64_t xx = 0; xx < W; ++xx) {
      int64_t acc = 0;
      for (int64_t t = 0; t < n_inputs(C, mode); ++t) {
        int64_t i, fo, fi;
        input_of(o, t, C, FO, mode, &i, &fo, &fi);
        const int64_t* xi = x + (n * C + i) * H * W;
        const int64_t* ff = f + (fo * FI + fi) * K * K;
        for (int64_t u = 0; u < K; ++u) {
          int64_t sy = y + u - r;
          if (sy < 0 || sy >= H) continue;
          for (int64_t v = 0; v < K; ++v) {
            int64_t sx = xx + v - r;
            if (sx < 0 || sx >= W) continue;
            acc += ff[u * K + v] * xi[sy * W + sx];
          }
        }
      }
      out[((n * CO + o) * rows + (y - y0)) * W + xx] = acc;
    }
  }
  return 0;
}

/*
 * The forward sum in binary32, as the paper's sharpen computes it (float
 * filter taps times 8-bit pixel values, Section 4.2.4).  Here the order of the
 * sum is fixed, because with u8 outputs the rounding decides an integer: the
 * accumulator starts at +0 and takes one fused multiply-add (a single rounding,
 * C's fmaf) per term, input channels outermost, then tap rows u, then tap
 * columns v.  With zero borders an out-of-image neighbour is skipped (adding
 * F * 0 with a fused multiply-add leaves the accumulator unchanged, so either
 * form gives the same value).  Whole images: out is [N][C_out][H][W].
 */
int oracle_forward_f32fma(const float* x, int64_t N, int64_t C, int64_t H, int64_t W, const float* f,
                          int64_t FO, int64_t FI, int64_t K, int32_t mode, int32_t zero_border,
                          float* out) {
  int64_t CO = out_channels(C, FO, FI, K, mode);
  if (CO < 0 || N < 0 || H < 0 || W < 0) return -1;
  if (N == 0 || H == 0 || W == 0) return 0;
  int64_t r = (K - 1) / 2;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t p = 0; p < N * CO * H; ++p) {
    int64_t n = (p / H) / CO, o = (p / H) % CO, y = p % H;
    for (int64_t xx = 0; xx < W; ++xx) {
      float acc = 0.0f;
      for (int64_t t = 0; t < n_inputs(C, mode); ++t) {
        int64_t i, fo, fi;
        input_of(o, t, C, FO, mode, &i, &fo, &fi);
        const float* xi = x + (n * C + i) * H * W;
        const float* ff = f + (fo * FI + fi) * K * K;
        for (int64_t u = 0; u < K; ++u) {
          int64_t sy = y + u - r;
          if (zero_border && (sy < 0 || sy >= H)) continue;
          for (int64_t v = 0; v < K; ++v) {
            int64_t sx = xx + v - r;
            if (zero_border && (sx < 0 || sx >= W)) continue;
            acc = fmaf(ff[u * K + v], xi[cl(sy, H) * W + cl(sx, W)], acc);
          }
        }
      }
      out[((n * CO + o) * H + y) * W + xx] = acc;
    }
  }
  return 0;
}

/*
 * 8-bit outputs.  The paper stores its float sums in 8-bit images without
 * saying how; the reading here is OpenCV's conversion: clamp to [0, 255] and
 * round to the nearest integer, ties to even (rintf in the default rounding
 * mode).  Integer sums are clamped.
 */
int oracle_u8_from_f32(const float* a, int64_t count, uint8_t* out) {
  if (count < 0) return -1;
  for (int64_t k = 0; k < count; ++k) {
    float v = a[k];
    if (!(v > 0.0f)) v = 0.0f;
    if (v > 255.0f) v = 255.0f;
    out[k] = (uint8_t)rintf(v);
  }
  return 0;
}

int oracle_u8_from_i64(const int64_t* a, int64_t count, uint8_t* out) {
  if (count < 0) return -1;
  for (int64_t k = 0; k < count; ++k) out[k] = (uint8_t)(a[k] < 0 ? 0 : (a[k] > 255 ? 255 : a[k]));
  return 0;
}

int oracle_sumsq_i64(const int64_t* a, const int64_t* b, int64_t count, int64_t* out) {
  if (count < 0) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < count; ++k) out[k] = a[k] * a[k] + b[k] * b[k];
  return 0;
}

int oracle_grad_input_f64(const double* g, int64_t N, int64_t C, int64_t H, int64_t W,
                          const double* f, int64_t FO, int64_t FI, int64_t K, int32_t mode,
                          double* gx) {
  int64_t CO = out_channels(C, FO, FI, K, mode);
  if (CO < 0 || N < 0 || H < 0 || W < 0) return -1;
  if (N == 0 || C == 0 || H == 0 || W == 0) return 0;
  int64_t r = (K - 1) / 2;
  /* One OpenMP task per input plane (n, i): it owns gx[n][i] and scatters into
   * it every term whose source pixel lies in that plane. */
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t p = 0; p < N * C; ++p) {
    int64_t n = p / C, ic = p % C;
    double* gxi = gx + (n * C + ic) * H * W;
    for (int64_t k = 0; k < H * W; ++k) gxi[k] = 0.0;
    for (int64_t o = 0; o < CO; ++o) {
      for (int64_t t = 0; t < n_inputs(C, mode); ++t) {
        int64_t i, fo, fi;
        input_of(o, t, C, FO, mode, &i, &fo, &fi);
        if (i != ic) continue;
        const double* go = g + (n * CO + o) * H * W;
        const double* ff = f + (fo * FI + fi) * K * K;
        for (int64_t y = 0; y < H; ++y)
          for (int64_t xx = 0; xx < W; ++xx)
            for (int64_t u = 0; u < K; ++u)
              for (int64_t v = 0; v < K; ++v)
                gxi[cl(y + u - r, H) * W + cl(xx + v - r, W)] += ff[u * K + v] * go[y * W + xx];
      }
    }
  }
  return 0;
}

/* Neumaier's improved Kahan-Babuska summation (Neumaier, 1974). */
typedef struct {
  double s, c;
} nsum;

static void nsum_add(nsum* a, double t) {
  double s = a->s + t;
  if (fabs(a->s) >= fabs(t))
    a->c += (a->s - s) + t;
  else
    a->c += (t - s) + a->s;
  a->s = s;
}

int oracle_grad_filter_f64(const double* x, const double* g, int64_t N, int64_t C, int64_t H,
                           int64_t W, int64_t FO, int64_t FI, int64_t K, int32_t mode,
                           double* gf) {
  int64_t CO = out_channels(C, FO, FI, K, mode);
  if (CO < 0 || N < 0 || H < 0 || W < 0) return -1;
  int64_t r = (K - 1) / 2;
  int64_t nf = FO * FI * K * K;
  /* One OpenMP task per filter element. */
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t e = 0; e < nf; ++e) {
    int64_t fo = e / (FI * K * K), fi = (e / (K * K)) % FI;
    int64_t u = (e / K) % K, v = e % K;
    nsum acc = {0.0, 0.0};
    for (int64_t n = 0; n < N; ++n) {
      for (int64_t o = 0; o < CO; ++o) {
        for (int64_t t = 0; t < n_inputs(C, mode); ++t) {
          int64_t i, efo, efi;
          input_of(o, t, C, FO, mode, &i, &efo, &efi);
          if (efo != fo || efi != fi) continue;
          const double* go = g + (n * CO + o) * H * W;
          const double* xi = x + (n * C + i) * H * W;
          for (int64_t y = 0; y < H; ++y)
            for (int64_t xx = 0; xx < W; ++xx)
              nsum_add(&acc, go[y * W + xx] * xi[cl(y + u - r, H) * W + cl(xx + v - r, W)]);
        }
      }
    }
    gf[e] = acc.s + acc.c;
  }
  return 0;
}

int oracle_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
