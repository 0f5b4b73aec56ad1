// Hardware ceilings of the GPU the library runs on, measured with kernels of its own: the HBM
// bandwidth a plain streaming read and a streaming copy reach, and the FP64 vector FMA rate.
// The PCG iteration is bandwidth-bound (about 0.19 flop per byte), so its roofline fraction is
// stated against the datasheet peak and against these measured ceilings.  Each entry point
// times `reps` back-to-back launches with HIP events on the given stream and returns the mean
// duration of one launch.
#include <hip/hip_runtime.h>

#include "hipsso_ceiling.h"

namespace {

constexpr int TPB = 256;
typedef double d2 __attribute__((ext_vector_type(2)));   // one 16-byte load or store per lane

// Every lane reads 16-byte pieces at a grid stride; the per-workgroup sum is stored so that the
// loads cannot be dropped.
__global__ void __launch_bounds__(TPB) k_read(int64_t n2, const d2* __restrict__ a,
                                              double* __restrict__ partials) {
  double s0 = 0.0, s1 = 0.0;
  const int64_t stride = (int64_t)gridDim.x * TPB;
  int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x;
  for (; i + 3 * stride < n2; i += 4 * stride) {
    const d2 v0 = __builtin_nontemporal_load(a + i);
    const d2 v1 = __builtin_nontemporal_load(a + i + stride);
    const d2 v2 = __builtin_nontemporal_load(a + i + 2 * stride);
    const d2 v3 = __builtin_nontemporal_load(a + i + 3 * stride);
    s0 += (v0.x + v1.x) + (v2.x + v3.x);
    s1 += (v0.y + v1.y) + (v2.y + v3.y);
  }
  for (; i < n2; i += stride) {
    const d2 v = a[i];
    s0 += v.x;
    s1 += v.y;
  }
  __shared__ double lds[TPB];
  lds[threadIdx.x] = s0 + s1;
  __syncthreads();
  for (int h = TPB / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h) lds[threadIdx.x] += lds[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = lds[0];
}

__global__ void __launch_bounds__(TPB) k_copy(int64_t n2, const d2* __restrict__ a,
                                              d2* __restrict__ b) {
  const int64_t stride = (int64_t)gridDim.x * TPB;
  for (int64_t i = blockIdx.x * (int64_t)TPB + threadIdx.x; i < n2; i += stride)
    __builtin_nontemporal_store(__builtin_nontemporal_load(a + i), b + i);
}

// Eight independent FMA chains per lane, `iters` steps each: 16 flops per lane per step.
__global__ void __launch_bounds__(TPB) k_fma(int iters, double x, double y,
                                             double* __restrict__ out) {
  double a0 = threadIdx.x * 1e-9, a1 = a0 + 1e-3, a2 = a0 + 2e-3, a3 = a0 + 3e-3;
  double a4 = a0 + 4e-3, a5 = a0 + 5e-3, a6 = a0 + 6e-3, a7 = a0 + 7e-3;
  for (int k = 0; k < iters; ++k) {
    a0 = __builtin_fma(a0, x, y); a1 = __builtin_fma(a1, x, y);
    a2 = __builtin_fma(a2, x, y); a3 = __builtin_fma(a3, x, y);
    a4 = __builtin_fma(a4, x, y); a5 = __builtin_fma(a5, x, y);
    a6 = __builtin_fma(a6, x, y); a7 = __builtin_fma(a7, x, y);
  }
  const double s = ((a0 + a1) + (a2 + a3)) + ((a4 + a5) + (a6 + a7));
  if (s == 12345.678) out[blockIdx.x] = s;   // never true for the inputs used; keeps the chains
}

int grid_for(int64_t n2) {
  int64_t g = (n2 + 4 * TPB - 1) / (4 * TPB);
  if (g > 8192) g = 8192;
  return (int)(g < 1 ? 1 : g);
}

template <class F>
int timed(int reps, hipStream_t s, F launch, double* us) {
  if (reps < 1 || !us) return -1;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return -3;
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return -3;
  }
  launch();   // warm-up
  (void)hipEventRecord(e0, s);
  for (int r = 0; r < reps; ++r) launch();
  (void)hipEventRecord(e1, s);
  hipError_t e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e == hipSuccess) e = hipGetLastError();
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return -3;
  *us = 1000.0 * ms / reps;
  return 0;
}

}  // namespace

extern "C" {

int hipsso_ceiling_read(const double* src, int64_t n, double* partials, int reps,
                        hipStream_t stream, double* us_per_launch) {
  if (!src || !partials || n <= 0 || (n & 1)) return -1;
  const int64_t n2 = n / 2;
  const int g = grid_for(n2);
  return timed(reps, stream, [&] {
    hipLaunchKernelGGL(k_read, dim3(g), dim3(TPB), 0, stream, n2,
                       reinterpret_cast<const d2*>(src), partials);
  }, us_per_launch);
}

int hipsso_ceiling_copy(const double* src, double* dst, int64_t n, int reps, hipStream_t stream,
                        double* us_per_launch) {
  if (!src || !dst || n <= 0 || (n & 1)) return -1;
  const int64_t n2 = n / 2;
  const int g = grid_for(n2);
  return timed(reps, stream, [&] {
    hipLaunchKernelGGL(k_copy, dim3(g), dim3(TPB), 0, stream, n2,
                       reinterpret_cast<const d2*>(src), reinterpret_cast<d2*>(dst));
  }, us_per_launch);
}

int hipsso_ceiling_fma(double* out, int workgroups, int iters, int reps, hipStream_t stream,
                       double* us_per_launch) {
  if (!out || workgroups <= 0 || iters <= 0) return -1;
  return timed(reps, stream, [&] {
    hipLaunchKernelGGL(k_fma, dim3(workgroups), dim3(TPB), 0, stream, iters, 0.999999, 1e-7,
                       out);
  }, us_per_launch);
}

}  // extern "C"
