/*
 * pmfmm_peak.h - measured vector-ALU peak of the device (a measurement aid
 * beside the C ABI of pmfmm.h, not part of the method).
 *
 * The pair kernels' flop rates are reported against the published MI355X
 * vector peaks and against the rate this benchmark measures on the same
 * device: fused multiply-add chains on every compute unit, float64 or
 * float32 without packed FP32 instructions (the form every kernel of the
 * library is compiled in).
 */
#ifndef PMFMM_PEAK_H
#define PMFMM_PEAK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { PMFMM_PEAK_OK = 0, PMFMM_PEAK_EINVAL = -1, PMFMM_PEAK_EDEVICE = -3 };

/* Vector fused multiply-add rate of the current HIP device.
 * precision: 0 = float64 (v_fma_f64), 1 = float32 (v_fma_f32, unpacked).
 * iters: loop trips, 16 .. 2^24; each trip is 64 dependent-chain FMAs per
 * lane (8 independent chains x 8), over 8 workgroups of 256 lanes per
 * compute unit.  One untimed launch of iters / 16 trips warms the device,
 * then one launch is timed with HIP events on the null stream.
 * *tflops receives 2 x FMAs / time in TFLOP/s, *ms (if not NULL) the
 * kernel time.  Allocates and frees a (grid x 256) output buffer and waits
 * for the device.  Errors: PMFMM_PEAK_EINVAL (bad argument),
 * PMFMM_PEAK_EDEVICE (no device, allocation or launch failure); the
 * message is in pmfmm_peak_last_error() on the calling thread. */
int pmfmm_peak_fma(int32_t precision, int32_t iters, double* tflops, double* ms);

/* Message of the last failed pmfmm_peak_fma on this thread ("" if none). */
const char* pmfmm_peak_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PMFMM_PEAK_H */
