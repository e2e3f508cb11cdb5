/* Measured hardware ceilings of the current device, for the roofline of the
 * DG kernels (libdgw_ceilings.so, separate from the solver library).
 *
 * Each call runs one microbenchmark on the current HIP device, synchronously
 * on the null stream, and returns its rate through `out`.  Return value: 0 on
 * success, -1 on a HIP error (out untouched).  Device memory is allocated and
 * freed inside the call.  Not thread safe with other work on the device (it
 * times the whole device).
 */
#ifndef DGW_CEILINGS_H
#define DGW_CEILINGS_H
#ifdef __cplusplus
extern "C" {
#endif

/* LDS read bandwidth in bytes/s summed over the device: every lane reads
 * `access_bytes` per access, lanes `lane_stride_bytes` apart inside a wave.
 * Supported pairs: (8, 8) and (16, 16) contiguous, (8, 48) and (16, 48) the
 * lines of a 6-point FP64 tensor, (8, 56) a padded 7-point row; other pairs
 * return -1. */
int dgw_ceiling_lds_read(int access_bytes, int lane_stride_bytes, double* out);

/* Vector FMA throughput in flop/s (2 per FMA), FP64 (fp64 = 1) or FP32
 * (fp64 = 0; scalar v_fma_f32, no packed instructions). */
int dgw_ceiling_vector_fma(int fp64, double* out);

/* Matrix-core throughput in flop/s of v_mfma_f64_16x16x4_f64 (fp64 = 1) or
 * v_mfma_f32_32x32x2_f32 (fp64 = 0). */
int dgw_ceiling_mfma(int fp64, double* out);

/* The 1D contraction of the k = 5 kernels in FP32 (a 6 x 6 matrix along
 * lines of 6 values held in LDS, one workgroup barrier per pass), in lines
 * per second over the device: one line per lane on the vector FMA units
 * (mfma = 0, 36 FMAs per line) or 16 lines per wave with
 * v_mfma_f32_16x16x4f32 (mfma = 1, two instructions per 16 lines, 6 of 16
 * outputs and 6 of 8 summation terms used). */
int dgw_ceiling_contract6(int mfma, double* out);

/* The largest difference between the two contractions above after three
 * passes on the same tile, relative to the largest value (the check that
 * the matrix-core form computes the same product). */
int dgw_ceiling_contract6_check(double* out);

#ifdef __cplusplus
}
#endif
#endif
