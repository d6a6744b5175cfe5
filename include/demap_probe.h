/*
 * demap_probe.h — measurement utilities of libdemap.so (not part of the demapping path).
 *
 * The exact demapper evaluates one exp2 per (symbol, point) pair, so its throughput bound
 * is the GPU's transcendental issue rate together with the adds of the subset sums.  These
 * calls measure those rates and time the library's own kernels with HIP events, so that a
 * benchmark can report its achieved rate against a measured roofline.
 */
#ifndef DEMAP_PROBE_H
#define DEMAP_PROBE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Measure vector-ALU rates on the current device, synchronously on `stream`.
 *   rates[0]  exp2 evaluations per second (v_exp_f32, all CUs)
 *   rates[1]  FP32 FMA lane-operations per second (non-packed)
 *   rates[2]  (exp2 + 2 FP32 adds) steps per second, the demapper's inner step
 *   rates[3]  number of compute units used
 * Returns 0, -1 (null argument), -3 (HIP error) or -4 (allocation failed).
 */
int dm_probe_valu_rates(double* rates, void* stream);

/*
 * Measure device-scope atomic throughput on the current device, synchronously on `stream`:
 * one lane of each of (compute units x 16) wavefronts issues 32 atomicAdds.
 *   rates[0]  atomics per second when all of them target one 32-bit word
 *   rates[1]  atomics per second when wavefront w targets word (w % 64) of 64 words spaced
 *             256 bytes apart (the layout of the fix-up queue's region counters)
 *   rates[2]  number of words used for rates[1] (64)
 * Returns 0, -1 (null argument), -3 (HIP error) or -4 (allocation failed).
 */
int dm_probe_atomic_rates(double* rates, void* stream);

/*
 * Kernel timing with HIP events recorded on the launch stream around the demapping
 * kernel and around the fix-up kernel of every later dm_demap_llr / dm_gmi_estimate
 * call on this thread.  dm_profile_enable(1) starts (and clears), 0 stops.
 * dm_profile_read waits for the recorded events and returns the summed milliseconds of
 * the demapping kernels (main_ms) and fix-up kernels (fixup_ms) and the launch count;
 * reset != 0 clears the record.  Returns 0 or a negative DM_E* code.
 */
int dm_profile_enable(int on);
int dm_profile_read(double* main_ms, double* fixup_ms, int64_t* launches, int reset);

/*
 * One MFMA product with the lane mapping the demapping kernels assume, for checking it.
 *   dtype 0 = BF16, 1 = FP16 operands; shape 0 = v_mfma_f32_32x32x16 (A 32x16, B 16x32,
 *   D 32x32), shape 1 = v_mfma_f32_16x16x32 (A 16x32, B 32x16, D 16x16).
 *   A, B, D are HOST row-major FP32 arrays (A, B rounded to dtype).  Synchronous.
 * Returns 0, -1 (bad argument), -3 (HIP error), -4 (allocation failed).
 */
int dm_probe_mfma_layout(int dtype, int shape, const float* A, const float* B, float* D);

/*
 * The learned demapper's inference-time GELU, x Phi(x) with the tanh-form Phi (the network's
 * activation; the learned demapper is a project addition, see demap.h), evaluated by the
 * very routine the inference kernel uses: packed FP16 arithmetic on the quarter scale, x / 4
 * converted to FP16 rounding toward zero (saturating at +-65504, i.e. |x| at 262016), the
 * result 4 times an FP16 value, returned as FP32.  x and out are HOST arrays of n floats;
 * 0 <= n <= 2^24.  Synchronous on the null
 * stream.  For checking that evaluation's error over every FP16 input.
 * Returns 0, -1 (bad argument), -3 (HIP error), -4 (allocation failed).
 */
int dm_probe_gelu(const float* x, float* out, int64_t n);

#ifdef __cplusplus
}
#endif

#endif /* DEMAP_PROBE_H */
