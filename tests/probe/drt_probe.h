/*
 * drt_probe.h -- self-tests of the gfx950 builtins that libdrt's kernels rely on.
 *
 * Each entry point launches one small, in-bounds kernel on the null stream, waits for it
 * and returns DRT_OK or DRT_E_DEVICE.  All pointers are device pointers owned by the
 * caller.  They exist so that the test suite can check the hardware behaviour the ray-sum
 * kernels assume, not to compute anything of the DRT method.
 */
#ifndef DRT_PROBE_H
#define DRT_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* One wave executes v_mfma_f32_16x16x4_f32 with lane l supplying A[l%16][l/16] (A is a
 * 16x4 row-major matrix, 64 floats) and B[l/16][l%16] (B 4x16 row-major, 64 floats),
 * accumulator zero, and writes D[4*(l/16)+v][l%16] from accumulator register v into D
 * (16x16 row-major, 256 floats).  D equals A.B exactly when that is the hardware's lane
 * layout. */
int drt_probe_mfma_f32_16x16x4(const float *A, const float *B, float *D);

/* One wave executes v_mfma_f32_16x16x32_f16 with lane l supplying the 8 half-precision
 * values A[l%16][8*(l/16)+j] (A 16x32 row-major, 512 IEEE binary16 values as uint16) and
 * B[8*(l/16)+j][l%16] (B 32x16 row-major), j = 0..7 in vector order, accumulator zero, and
 * writes D[4*(l/16)+v][l%16] (16x16 row-major floats).  D equals A.B when that is the
 * hardware's lane layout. */
int drt_probe_mfma_f16_16x16x32(const uint16_t *A, const uint16_t *B, float *D);

/* v_mfma_f64_16x16x4_f64 on binary64 operands: lane l supplies A[l%16][l/16] and
 * B[l/16][l%16] (as the binary32 instruction) and writes D[l/16+4*v][l%16] from accumulator
 * element v (the binary64 accumulator interleaves its rows, unlike the binary32 one). */
int drt_probe_mfma_f64_16x16x4(const double *A, const double *B, double *D);

/* s[i] = v_sin_f32(x[i]), c[i] = v_cos_f32(x[i]): the hardware sine and cosine of an
 * angle given in revolutions (sin(2 pi x)).  n >= 0 elements. */
int drt_probe_sincos_rev(const float *x, int32_t n, float *s, float *c);

#ifdef __cplusplus
}
#endif

#endif /* DRT_PROBE_H */
