/*
 * oracle.h -- plain CPU reference for the clamp-to-edge K x K 2D filter.
 *
 * TEST INFRASTRUCTURE ONLY.  This header and oracle.c are used by the tests,
 * by the smoke check and by the CPU-baseline leg of the benchmark.  The GPU
 * library never includes, links or calls anything here, and nothing here uses
 * any part of the GPU library.
 *
 * The filter is the generalisation of the paper's 3x3 Laplacian sharpen
 * (Section 4.2.4, "Sharpening": each output pixel is a weighted sum of its
 * 3x3 neighbourhood, colour channels handled independently) to
 *   - any odd K (anchor at the centre, r = (K-1)/2),
 *   - correlation (tap (u,v) weighs the neighbour at offset (u-r, v-r)),
 *   - clamp-to-edge borders, cl_n(t) = min(max(t,0), n-1) per axis,
 *   - three channel modes:
 *       SHARED    : one K x K filter applied to every channel,
 *       DEPTHWISE : filter [C*m][1][K][K]; output channel c*m+j is channel c
 *                   filtered by filter c*m+j,
 *       BANK      : filter [C_out][C_in][K][K]; output channel o sums the
 *                   correlations of every input channel i with F[o][i]
 *                   (with K = 1, C_in = 3, C_out = 1 this is the paper's
 *                   grayscale weighting of Section 4.2.5).
 *
 * Arrays are dense, row-major: images [N][C][H][W], filters [FO][FI][K][K].
 * Floating-point arithmetic is IEEE binary64, except oracle_forward_f32fma
 * (binary32 in a stated order, for 8-bit outputs); the integer path is int64.
 * Every function returns 0 on success and a negative value on bad arguments.
 */
#ifndef FILTER2D_ORACLE_H
#define FILTER2D_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORACLE_SHARED 0
#define ORACLE_DEPTHWISE 1
#define ORACLE_BANK 2

/* Forward filter, fp64.  x: [N][C][H][W]; f: [FO][FI][K][K].
 * Output rows y0..y1-1 of every output plane are written to
 * out: [N][C_out][y1-y0][W] where C_out = C (SHARED), FO (DEPTHWISE, BANK).
 * Clamping is with respect to the H x W array x. */
int oracle_forward_f64(const double* x, int64_t N, int64_t C, int64_t H, int64_t W,
                       const double* f, int64_t FO, int64_t FI, int64_t K, int32_t mode,
                       int64_t y0, int64_t y1, double* out);

/* As oracle_forward_f64 with zero borders: out-of-image neighbours add 0. */
int oracle_forward_zero_f64(const double* x, int64_t N, int64_t C, int64_t H, int64_t W,
                            const double* f, int64_t FO, int64_t FI, int64_t K, int32_t mode,
                            int64_t y0, int64_t y1, double* out);

/* The same definition in exact int64 arithmetic (the u8 / integer-tap path). */
int oracle_forward_i64(const int64_t* x, int64_t N, int64_t C, int64_t H, int64_t W,
                       const int64_t* f, int64_t FO, int64_t FI, int64_t K, int32_t mode,
                       int64_t y0, int64_t y1, int64_t* out);

/* As oracle_forward_i64 with zero borders. */
int oracle_forward_zero_i64(const int64_t* x, int64_t N, int64_t C, int64_t H, int64_t W,
                            const int64_t* f, int64_t FO, int64_t FI, int64_t K, int32_t mode,
                            int64_t y0, int64_t y1, int64_t* out);

/* The forward sum in binary32 with a fixed order: acc = +0, then one fused
 * multiply-add per term (input channel, then tap row u, then tap column v).
 * zero_border != 0: out-of-image neighbours are skipped; else clamp-to-edge.
 * Whole images; out: [N][C_out][H][W]. */
int oracle_forward_f32fma(const float* x, int64_t N, int64_t C, int64_t H, int64_t W, const float* f,
                          int64_t FO, int64_t FI, int64_t K, int32_t mode, int32_t zero_border,
                          float* out);

/* 8-bit conversion: clamp to [0, 255], then round to nearest, ties to even
 * (floats) or keep (integers). */
int oracle_u8_from_f32(const float* a, int64_t count, uint8_t* out);
int oracle_u8_from_i64(const int64_t* a, int64_t count, uint8_t* out);

/* out[k] = a[k]^2 + b[k]^2 (the gradient-magnitude epilogue, no square root). */
int oracle_sumsq_i64(const int64_t* a, const int64_t* b, int64_t count, int64_t* out);

/* Adjoint of the forward map with respect to the image, in scatter form:
 * for every output value g[n][o][y][x] and every tap (u,v) of every filter that
 * produced it, add F * g to gx at the clamped source pixel.
 * g: [N][C_out][H][W]; gx: [N][C][H][W] (overwritten). */
int oracle_grad_input_f64(const double* g, int64_t N, int64_t C, int64_t H, int64_t W,
                          const double* f, int64_t FO, int64_t FI, int64_t K, int32_t mode,
                          double* gx);

/* Adjoint with respect to the filter:
 * gf[o][i][u][v] = sum over n, y, x (and over c in SHARED mode) of
 *                  g[n][o'][y][x] * x[n][i'][cl(y+u-r)][cl(x+v-r)],
 * summed with Neumaier's compensated summation.  gf: [FO][FI][K][K]. */
int oracle_grad_filter_f64(const double* x, const double* g, int64_t N, int64_t C, int64_t H,
                           int64_t W, int64_t FO, int64_t FI, int64_t K, int32_t mode,
                           double* gf);

/* Number of OpenMP threads the oracle uses (1 when built without OpenMP). */
int oracle_num_threads(void);

#ifdef __cplusplus
}
#endif

#endif
