// Achievable-peak microbenchmarks for the roofline of the contact kernels:
// an FP32 / FP64 fused multiply-add loop (the VALU issue rate and the
// cycles one wave64 FMA instruction occupies a SIMD) and a device-to-device
// copy (the HBM bandwidth a streaming kernel reaches).  Built into its own
// library (libpeak.so); the contact library does not use it.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

// kChains independent FMA chains per lane keep the VALU busy without
// waiting on a previous result; the loop body is kChains FMAs.
constexpr int kChains = 16;

// KIND 0: v = v * a + b with a, b uniform (one SGPR operand: VOP3 FMA);
// 1: v = v + a * w with a per lane and w the next chain's value (three VGPR
// operands, accumulating form: VOP2 FMAC); 2: v = v + a (add);
// 3: v = v * a (multiply); 4: v = max(v, w) (as in the bound's support
// functions); 5: v = v * a + b with a, b per lane (three VGPR operands, the
// addend not the destination: VOP3 FMA); 6: v = max(v, w, u) (three-input
// VOP3 max, as in the support functions).
template <typename T, int KIND>
__global__ void __launch_bounds__(256) k_fma_loop(T* out, int iters, T a0, T b0) {
  T v[kChains];
  const T a = KIND == 0 ? a0 : a0 + T(threadIdx.x) * T(1e-9);
  const T b = KIND == 5 ? b0 + T(threadIdx.x) * T(1e-9) : b0;
#pragma unroll
  for (int c = 0; c < kChains; ++c) v[c] = T(threadIdx.x + c);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c) {
      if constexpr (KIND == 0) v[c] = v[c] * a + b;
      else if constexpr (KIND == 1) v[c] = v[c] + a * v[(c + 1) % kChains];
      else if constexpr (KIND == 2) v[c] = v[c] + a;
      else if constexpr (KIND == 3) v[c] = v[c] * a;
      else if constexpr (KIND == 4) v[c] = fmaxf(v[c], v[(c + 1) % kChains]);
      else if constexpr (KIND == 5) v[c] = v[c] * a + b;
      else v[c] = fmaxf(fmaxf(v[c], v[(c + 1) % kChains]), v[(c + 2) % kChains]);
    }
  }
  T s = T(0);
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += v[c];
  // a store the compiler cannot remove (the value is practically never 0)
  if (s == T(0)) out[blockIdx.x * blockDim.x + threadIdx.x] = s;
}

__global__ void __launch_bounds__(256) k_copy(const uint4* __restrict__ src, uint4* __restrict__ dst, size_t n) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

}  // namespace

extern "C" {

// VALU loop: `blocks` x 256 threads, each iters x 16 operations of the
// given kind (see k_fma_loop; FP32 if fp64 == 0, else FP64, kind 0 and 1
// only; kind 0..6).  out: device buffer of blocks x 256 elements of that type (never
// written in practice).  Returns 0 or the HIP error code of the launch.
int peak_fma(int fp64, int kind, int blocks, int iters, void* out, void* stream) {
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (blocks < 1 || iters < 1 || !out || kind < 0 || kind > 6 || (fp64 && kind > 1)) return -1;
  const dim3 g(blocks), b(256);
  if (fp64) {
    double* o = static_cast<double*>(out);
    if (kind == 0) hipLaunchKernelGGL((k_fma_loop<double, 0>), g, b, 0, st, o, iters, 0.999999, 1e-7);
    else hipLaunchKernelGGL((k_fma_loop<double, 1>), g, b, 0, st, o, iters, 1e-9, 0.0);
  } else {
    float* o = static_cast<float*>(out);
    switch (kind) {
      case 0: hipLaunchKernelGGL((k_fma_loop<float, 0>), g, b, 0, st, o, iters, 0.999999f, 1e-7f); break;
      case 1: hipLaunchKernelGGL((k_fma_loop<float, 1>), g, b, 0, st, o, iters, 1e-9f, 0.0f); break;
      case 2: hipLaunchKernelGGL((k_fma_loop<float, 2>), g, b, 0, st, o, iters, 1e-7f, 0.0f); break;
      case 3: hipLaunchKernelGGL((k_fma_loop<float, 3>), g, b, 0, st, o, iters, 0.999999f, 0.0f); break;
      case 4: hipLaunchKernelGGL((k_fma_loop<float, 4>), g, b, 0, st, o, iters, 0.5f, 0.0f); break;
      case 5: hipLaunchKernelGGL((k_fma_loop<float, 5>), g, b, 0, st, o, iters, 0.999999f, 1e-7f); break;
      default: hipLaunchKernelGGL((k_fma_loop<float, 6>), g, b, 0, st, o, iters, 0.5f, 0.0f); break;
    }
  }
  return (int)hipGetLastError();
}

// FMA instructions per lane of one peak_fma call (for the issue-rate figure).
long long peak_fma_per_lane(int iters) { return (long long)iters * kChains; }

// Copy `bytes` (a multiple of 16, both buffers 16-byte aligned) from src to
// dst with `blocks` x 256 threads.
int peak_copy(const void* src, void* dst, size_t bytes, int blocks, void* stream) {
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (!src || !dst || bytes % 16 || blocks < 1) return -1;
  hipLaunchKernelGGL(k_copy, dim3(blocks), dim3(256), 0, st, static_cast<const uint4*>(src),
                     static_cast<uint4*>(dst), bytes / 16);
  return (int)hipGetLastError();
}

}  // extern "C"
