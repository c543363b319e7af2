// Achievable-throughput probes of the GPU the library runs on: long loops of
// independent matrix-core or vector FMA chains over a grid that fills every
// CU.  They give the achievable roofs next to the vendor peaks that the
// kernels' roofline fractions are quoted against; nothing of the transport
// path calls them.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace dlra {
namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d4 __attribute__((ext_vector_type(4)));

// four independent accumulators per wave; operands differ per lane and block
// so nothing folds; the sums are stored so the loop stays
__global__ __launch_bounds__(256) void k_probe_mfma32(int iters, double *out) {
  const float a = 1.0f + 1e-7f * float(threadIdx.x), b = 1e-3f * (1.0f + 1e-6f * blockIdx.x);
  f4 c0 = {0.0f, 0.0f, 0.0f, 0.0f}, c1 = c0, c2 = c0, c3 = c0;
  for (int i = 0; i < iters; ++i) {
    c0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f32_16x16x4f32(b, a, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f32_16x16x4f32(a, a, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f32_16x16x4f32(b, b, c3, 0, 0, 0);
  }
  const f4 s = c0 + c1 + c2 + c3;
  out[size_t(blockIdx.x) * blockDim.x + threadIdx.x] = double(s[0] + s[1] + s[2] + s[3]);
}

__global__ __launch_bounds__(256) void k_probe_mfma64(int iters, double *out) {
  const double a = 1.0 + 1e-9 * threadIdx.x, b = 1e-3 * (1.0 + 1e-9 * blockIdx.x);
  d4 c0 = {0.0, 0.0, 0.0, 0.0}, c1 = c0, c2 = c0, c3 = c0;
  for (int i = 0; i < iters; ++i) {
    c0 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c0, 0, 0, 0);
    c1 = __builtin_amdgcn_mfma_f64_16x16x4f64(b, a, c1, 0, 0, 0);
    c2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, a, c2, 0, 0, 0);
    c3 = __builtin_amdgcn_mfma_f64_16x16x4f64(b, b, c3, 0, 0, 0);
  }
  const d4 s = c0 + c1 + c2 + c3;
  out[size_t(blockIdx.x) * blockDim.x + threadIdx.x] = s[0] + s[1] + s[2] + s[3];
}

// eight independent FMA chains per lane, x <- x a + b with |a| < 1 (bounded)
template <typename T>
__global__ __launch_bounds__(256) void k_probe_fma(int iters, double *out) {
  const T a = T(0.999999), b = T(1e-6) * T(1 + threadIdx.x);
  T x[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) x[j] = T(j + blockIdx.x % 7);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = fma(x[j], a, b);
  }
  T s = T(0);
#pragma unroll
  for (int j = 0; j < 8; ++j) s += x[j];
  out[size_t(blockIdx.x) * blockDim.x + threadIdx.x] = double(s);
}

}  // namespace

double roof_probe_flops(int kind, int iters, int blocks) {
  const double waves = double(blocks) * 4.0, lanes = double(blocks) * 256.0;
  switch (kind) {
    case 0:
    case 1: return waves * iters * 4.0 * 2048.0;   // 16 x 16 x 4 multiply-adds per MFMA
    default: return lanes * iters * 8.0 * 2.0;
  }
}

void launch_roof_probe(int kind, int iters, int blocks, double *out, hipStream_t st) {
  switch (kind) {
    case 0: k_probe_mfma32<<<blocks, 256, 0, st>>>(iters, out); break;
    case 1: k_probe_mfma64<<<blocks, 256, 0, st>>>(iters, out); break;
    case 2: k_probe_fma<float><<<blocks, 256, 0, st>>>(iters, out); break;
    default: k_probe_fma<double><<<blocks, 256, 0, st>>>(iters, out); break;
  }
}

}  // namespace dlra
