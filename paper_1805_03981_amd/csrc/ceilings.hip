// Microbenchmarks of the device ceilings (LDS bandwidth, vector FMA and
// matrix-core rates) that bound the DG kernels.  Each kernel runs a fixed
// amount of independent work per lane; the rate is work / event time.
#include <hip/hip_runtime.h>

#include "dgw_ceilings.h"

namespace {

constexpr int NT = 256;
constexpr int LDS_WORDS = 16384;  // 64 KiB of LDS per workgroup

// Reads of W dwords per lane, lanes STRIDE dwords apart; every index stays
// below 8192 + 63 * STRIDE + W < LDS_WORDS.
template <int W, int STRIDE>
__global__ void __launch_bounds__(NT) lds_read(unsigned* out, int iters) {
  static_assert(STRIDE % W == 0 && 8192 + 63 * STRIDE + W <= LDS_WORDS, "stride");
  __shared__ unsigned buf[LDS_WORDS];
  for (int i = threadIdx.x; i < LDS_WORDS; i += NT) buf[i] = i * 2654435761u;
  __syncthreads();
  unsigned acc = 0;
  const int lane_off = (threadIdx.x & 63) * STRIDE, wave = threadIdx.x >> 6;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int base = ((it * 8 + k) * 64 * W + wave * 1024) & (LDS_WORDS / 2 - 1) & ~(W - 1);
      const int idx = base + lane_off;
      if constexpr (W == 2) {
        const uint2 v = *reinterpret_cast<const uint2*>(&buf[idx]);
        acc ^= v.x ^ v.y;
      } else {
        const uint4 v = *reinterpret_cast<const uint4*>(&buf[idx]);
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
      }
    }
  }
  out[blockIdx.x * NT + threadIdx.x] = acc;
}

// 8 independent FMA chains per lane
template <typename T>
__global__ void __launch_bounds__(NT) vector_fma(T* out, T a, T b, int iters) {
  T x[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) x[j] = (T)(threadIdx.x + j);
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = fma(x[j], a, b);
  T s = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) s += x[j];
  out[blockIdx.x * NT + threadIdx.x] = s;
}

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));

// 4 independent accumulators per wave
__global__ void __launch_bounds__(NT) mfma_f64(double* out, double a, int iters) {
  d4 acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = d4{0.0, 0.0, 0.0, 0.0};
  const double b = a * (double)(threadIdx.x & 3);
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[j], 0, 0, 0);
  double s = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
  out[blockIdx.x * NT + threadIdx.x] = s;
}

__global__ void __launch_bounds__(NT) mfma_f32(float* out, float a, int iters) {
  f16v acc[2];
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int e = 0; e < 16; ++e) acc[j][e] = 0.0f;
  const float b = a * (float)(threadIdx.x & 3);
  for (int it = 0; it < iters; ++it)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[j] = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc[j], 0, 0, 0);
  float s = 0;
#pragma unroll
  for (int j = 0; j < 2; ++j)
#pragma unroll
    for (int e = 0; e < 16; ++e) s += acc[j][e];
  out[blockIdx.x * NT + threadIdx.x] = s;
}

// The 1D contraction of the DG kernels at k = 5 in FP32: a 6 x 6 matrix
// applied along x-lines of 6 values, lines held in LDS (stride 8 floats, the
// last two zero), two tiles of CLINES lines ping-ponged, one workgroup
// barrier per pass as between the kernels' phases.  Lane-per-line on the
// vector FMA units, or 16 lines per wave on the matrix cores.
constexpr int CLINES = 1024;  // lines per tile: 2 tiles x 1024 x 8 floats = 64 KiB

__device__ __forceinline__ void contract_init(float* t0, float* t1) {
  for (int i = threadIdx.x; i < CLINES * 8; i += NT) {
    const int c = i & 7;
    t0[i] = c < 6 ? 1e-3f * (float)((i * 37) % 101 - 50) : 0.0f;
    t1[i] = 0.0f;
  }
  __syncthreads();
}

// one line per lane, 36 FMAs with the matrix entries uniform over the wave
__global__ void __launch_bounds__(NT) contract6_valu(float* out, const float* __restrict__ M, int iters) {
  __shared__ float tile[2][CLINES * 8];
  contract_init(tile[0], tile[1]);
  float m[36];
#pragma unroll
  for (int e = 0; e < 36; ++e) m[e] = M[e];
  for (int it = 0; it < iters; ++it) {
    const float* src = tile[it & 1];
    float* dst = tile[(it & 1) ^ 1];
    for (int l = threadIdx.x; l < CLINES; l += NT) {
      float x[6];
#pragma unroll
      for (int j = 0; j < 6; ++j) x[j] = src[l * 8 + j];
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        float acc = m[i * 6] * x[0];
#pragma unroll
        for (int j = 1; j < 6; ++j) acc = fmaf(m[i * 6 + j], x[j], acc);
        dst[l * 8 + i] = acc;
      }
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < CLINES * 8; i += NT) out[(size_t)blockIdx.x * CLINES * 8 + i] = tile[iters & 1][i];
}

typedef float f4v __attribute__((ext_vector_type(4)));

// 16 lines per wave and v_mfma_f32_16x16x4f32: A = the lines (16 x 4, lane l
// holds line l % 16, entry 4 kk + l / 16), B = M^T (4 x 16, lane l holds
// entry 4 kk + l / 16 of output l % 16; zero outside 6 x 6), D = 16 x 16
// (lane l holds lines 4 (l / 16) + r, output l % 16); K = 6 takes two
// instructions (the last two entries zero), 6 of 16 outputs are used.
__global__ void __launch_bounds__(NT) contract6_mfma(float* out, const float* __restrict__ M, int iters) {
  __shared__ float tile[2][CLINES * 8];
  contract_init(tile[0], tile[1]);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int r16 = lane & 15, g = lane >> 4;
  float b[2];
#pragma unroll
  for (int kk = 0; kk < 2; ++kk) {
    const int k = 4 * kk + g;
    b[kk] = (k < 6 && r16 < 6) ? M[r16 * 6 + k] : 0.0f;
  }
  for (int it = 0; it < iters; ++it) {
    const float* src = tile[it & 1];
    float* dst = tile[(it & 1) ^ 1];
    for (int blk = wave; blk < CLINES / 16; blk += NT / 64) {
      f4v acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int kk = 0; kk < 2; ++kk) {
        const float a = src[(blk * 16 + r16) * 8 + 4 * kk + g];
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b[kk], acc, 0, 0, 0);
      }
      if (r16 < 8) {
#pragma unroll
        for (int r = 0; r < 4; ++r) dst[(blk * 16 + 4 * g + r) * 8 + r16] = acc[r];
      }
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < CLINES * 8; i += NT) out[(size_t)blockIdx.x * CLINES * 8 + i] = tile[iters & 1][i];
}

int n_cus() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -1;
  return n;
}

// time `launch(iters)` (after one short warm-up launch) in seconds
template <typename F>
int time_launch(F launch, int iters, double* sec) {
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess) return -1;
  if (hipEventCreate(&b) != hipSuccess) return -1;
  launch(2);
  int rc = 0;
  if (hipEventRecord(a, 0) != hipSuccess) rc = -1;
  launch(iters);
  if (hipEventRecord(b, 0) != hipSuccess) rc = -1;
  float ms = 0.f;
  if (rc == 0 && (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess)) rc = -1;
  if (hipGetLastError() != hipSuccess) rc = -1;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  *sec = ms * 1e-3;
  return rc;
}

}  // namespace

extern "C" int dgw_ceiling_lds_read(int access_bytes, int lane_stride_bytes, double* out) {
  if (!out) return -1;
  // supported (access, lane stride) pairs: contiguous, and the 48-byte stride
  // of 6-point FP64 lines (plus a 56-byte padded stride for 8-byte accesses)
  void (*kern)(unsigned*, int) = nullptr;
  if (access_bytes == 8 && lane_stride_bytes == 8) kern = lds_read<2, 2>;
  if (access_bytes == 16 && lane_stride_bytes == 16) kern = lds_read<4, 4>;
  if (access_bytes == 8 && lane_stride_bytes == 48) kern = lds_read<2, 12>;
  if (access_bytes == 16 && lane_stride_bytes == 48) kern = lds_read<4, 12>;
  if (access_bytes == 8 && lane_stride_bytes == 56) kern = lds_read<2, 14>;
  if (!kern) return -1;
  const int ncu = n_cus();
  if (ncu <= 0) return -1;
  const int blocks = ncu * 8, iters = 2000;
  unsigned* buf = nullptr;
  if (hipMalloc(&buf, (size_t)blocks * NT * 4) != hipSuccess) return -1;
  double sec = 0;
  auto launch = [&](int it) { hipLaunchKernelGGL(kern, dim3(blocks), dim3(NT), 0, 0, buf, it); };
  const int rc = time_launch(launch, iters, &sec);
  (void)hipFree(buf);
  if (rc || sec <= 0) return -1;
  *out = (double)blocks * NT * iters * 8 * access_bytes / sec;
  return 0;
}

extern "C" int dgw_ceiling_vector_fma(int fp64, double* out) {
  if (!out) return -1;
  const int ncu = n_cus();
  if (ncu <= 0) return -1;
  const int blocks = ncu * 8, iters = 20000;
  void* buf = nullptr;
  if (hipMalloc(&buf, (size_t)blocks * NT * 8) != hipSuccess) return -1;
  double sec = 0;
  auto launch = [&](int it) {
    if (fp64)
      hipLaunchKernelGGL(vector_fma<double>, dim3(blocks), dim3(NT), 0, 0, (double*)buf, 0.999999, 1e-7, it);
    else
      hipLaunchKernelGGL(vector_fma<float>, dim3(blocks), dim3(NT), 0, 0, (float*)buf, 0.9999f, 1e-4f, it);
  };
  const int rc = time_launch(launch, iters, &sec);
  (void)hipFree(buf);
  if (rc || sec <= 0) return -1;
  *out = 2.0 * 8 * (double)blocks * NT * iters / sec;
  return 0;
}

extern "C" int dgw_ceiling_mfma(int fp64, double* out) {
  if (!out) return -1;
  const int ncu = n_cus();
  if (ncu <= 0) return -1;
  const int blocks = ncu * 8, iters = 4000;
  void* buf = nullptr;
  if (hipMalloc(&buf, (size_t)blocks * NT * 8) != hipSuccess) return -1;
  double sec = 0;
  auto launch = [&](int it) {
    if (fp64)
      hipLaunchKernelGGL(mfma_f64, dim3(blocks), dim3(NT), 0, 0, (double*)buf, 1e-3, it);
    else
      hipLaunchKernelGGL(mfma_f32, dim3(blocks), dim3(NT), 0, 0, (float*)buf, 1e-3f, it);
  };
  const int rc = time_launch(launch, iters, &sec);
  (void)hipFree(buf);
  if (rc || sec <= 0) return -1;
  // per wave instruction: 16x16x4 (f64, 4 accumulators) or 32x32x2 (f32, 2)
  const double flop_per_iter_wave = fp64 ? 4 * 2.0 * 16 * 16 * 4 : 2 * 2.0 * 32 * 32 * 2;
  *out = flop_per_iter_wave * (double)blocks * (NT / 64) * iters / sec;
  return 0;
}

// M: a fixed, well-conditioned 6 x 6 matrix (entries of order 0.3), so that
// repeated passes neither overflow nor vanish
static int contract_setup(float** dM) {
  float hM[36];
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) hM[i * 6 + j] = (i == j ? 0.55f : 0.0f) + 0.05f * (float)((i * 7 + j * 3) % 5 - 2);
  if (hipMalloc(dM, sizeof(hM)) != hipSuccess) return -1;
  if (hipMemcpy(*dM, hM, sizeof(hM), hipMemcpyHostToDevice) != hipSuccess) return -1;
  return 0;
}

extern "C" int dgw_ceiling_contract6(int mfma, double* out) {
  if (!out) return -1;
  const int ncu = n_cus();
  if (ncu <= 0) return -1;
  const int blocks = ncu * 2, iters = 2000;  // 64 KiB of LDS per workgroup: two per CU
  float *dM = nullptr, *buf = nullptr;
  if (contract_setup(&dM)) return -1;
  if (hipMalloc(&buf, (size_t)blocks * CLINES * 8 * sizeof(float)) != hipSuccess) {
    (void)hipFree(dM);
    return -1;
  }
  double sec = 0;
  auto launch = [&](int it) {
    if (mfma)
      hipLaunchKernelGGL(contract6_mfma, dim3(blocks), dim3(NT), 0, 0, buf, dM, it);
    else
      hipLaunchKernelGGL(contract6_valu, dim3(blocks), dim3(NT), 0, 0, buf, dM, it);
  };
  const int rc = time_launch(launch, iters, &sec);
  (void)hipFree(buf);
  (void)hipFree(dM);
  if (rc || sec <= 0) return -1;
  *out = (double)blocks * CLINES * iters / sec;
  return 0;
}

extern "C" int dgw_ceiling_contract6_check(double* out) {
  if (!out) return -1;
  float *dM = nullptr, *b0 = nullptr, *b1 = nullptr;
  if (contract_setup(&dM)) return -1;
  const size_t n = (size_t)CLINES * 8;
  if (hipMalloc(&b0, n * sizeof(float)) != hipSuccess || hipMalloc(&b1, n * sizeof(float)) != hipSuccess) {
    (void)hipFree(dM);
    (void)hipFree(b0);
    return -1;
  }
  hipLaunchKernelGGL(contract6_valu, dim3(1), dim3(NT), 0, 0, b0, dM, 3);
  hipLaunchKernelGGL(contract6_mfma, dim3(1), dim3(NT), 0, 0, b1, dM, 3);
  int rc = hipDeviceSynchronize() == hipSuccess ? 0 : -1;
  float* h = new float[2 * n];
  if (!rc && (hipMemcpy(h, b0, n * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess ||
              hipMemcpy(h + n, b1, n * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess))
    rc = -1;
  if (!rc) {
    double mx = 0, dmax = 0;
    for (size_t i = 0; i < n; ++i) {
      mx = fmax(mx, fabs((double)h[i]));
      dmax = fmax(dmax, fabs((double)h[i] - (double)h[n + i]));
    }
    *out = mx > 0 ? dmax / mx : -1.0;
  }
  delete[] h;
  (void)hipFree(b0);
  (void)hipFree(b1);
  (void)hipFree(dM);
  return rc;
}
