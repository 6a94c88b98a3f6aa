/* Device peak probes for MI355X (gfx950): the denominators of the rooflines.
 *
 * The datasheet peaks (FP32 vector 157.3 TFLOP/s packed and 78.6 TFLOP/s
 * single-issue, FP64 vector 78.6 TFLOP/s, HBM3E 8 TB/s, transcendentals at a
 * quarter of the vector rate) are what the energy+force kernels are priced
 * against; these probes measure what the device reaches with code built the
 * same way as the kernels (packed FP32 instructions disabled).
 *
 * Library: libnnp_peaks.so, separate from libnnp.so.  Every entry point only
 * enqueues work on `stream` (a hipStream_t; NULL = the null stream) and returns
 * at once; the caller times the launch with events on the same stream.
 *
 * MFMA datasheet peaks (dense): FP32 157.3 TFLOP/s, FP64 78.6 TFLOP/s, BF16
 * 2.5 PFLOP/s.
 *
 * Return value: 0 on success, -1 for a bad argument (nothing launched), -4 if
 * the launch itself failed (hipGetLastError after the launch).
 */
#ifndef NNP_PEAKS_H
#define NNP_PEAKS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* FP32 fused multiply-add issue rate.  `blocks` workgroups of 256 lanes each
 * run `iters` rounds of 16 independent v_fma_f32 chains, i.e.
 * 2 * 16 * iters * 256 * blocks floating-point operations.  `out` is a device
 * buffer of blocks * 256 floats, written only to keep the chains live.
 * blocks in [1, 2^20], iters in [1, 2^24]. */
int nnp_peak_fma_f32(float* out, int blocks, int iters, void* stream);

/* The same for FP64 (v_fma_f64); `out` holds blocks * 256 doubles. */
int nnp_peak_fma_f64(double* out, int blocks, int iters, void* stream);

/* FP32 base-2 exponential issue rate (v_exp_f32): 16 independent chains of
 * x <- 2^(-x), i.e. 16 * iters * 256 * blocks exponentials.  Same limits. */
int nnp_peak_exp_f32(float* out, int blocks, int iters, void* stream);

/* Matrix-core (MFMA) issue rates, the ceiling of the network kernel: each
 * wave of the `blocks` workgroups (4 waves of 64 lanes each) runs `iters`
 * rounds of 4 independent accumulator chains of one instruction shape:
 *  nnp_peak_mfma_f32   v_mfma_f32_16x16x4f32, 2048 operations each
 *                      (out: blocks * 256 floats);
 *  nnp_peak_mfma_f64   v_mfma_f64_16x16x4f64, 2048 operations each
 *                      (out: blocks * 256 doubles);
 *  nnp_peak_mfma_bf16  v_mfma_f32_16x16x32_bf16, 16384 operations each
 *                      (out: blocks * 256 floats).
 * i.e. 4 * 4 * iters * blocks instructions.  `out` is written only to keep
 * the chains live.  Same limits as the FMA probes. */
int nnp_peak_mfma_f32(float* out, int blocks, int iters, void* stream);
int nnp_peak_mfma_f64(double* out, int blocks, int iters, void* stream);
int nnp_peak_mfma_bf16(float* out, int blocks, int iters, void* stream);

/* Streaming device copy of `bytes` bytes (a multiple of 16; both pointers
 * 16-byte aligned, not overlapping): 2 * bytes of HBM traffic.  Launches a
 * grid-stride kernel of `blocks` workgroups (blocks in [1, 2^20]). */
int nnp_peak_copy(const void* src, void* dst, int64_t bytes, int blocks, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* NNP_PEAKS_H */
