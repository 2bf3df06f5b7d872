// FP64 vector FMA probe (gfx950): the rate the roofline of the contraction
// kernels is set against, measured on the device it runs on.
//
// Every thread runs `iters` rounds of 16 independent chains
// a_i <- a_i * b + c (one v_fma_f64 each, 32 flop per round), then writes
// the sum of its chains so that none of the arithmetic can be dropped.
// With 256 threads per workgroup and many workgroups per compute unit, the
// 16 chains per wave and the waves per SIMD cover the FMA latency.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "mhc.h"
#include "mhc_internal.h"

namespace mhc {
namespace kern {

constexpr int kProbeBlock = 256;
constexpr int kProbeChains = 16;

// b arrives as an argument (an SGPR operand): as a literal the compiler
// would use the accumulating form v_fmac_f64 with c in the destination and
// a register copy for every FMA.
__global__ __launch_bounds__(kProbeBlock) void fma64_probe(double* out, int iters, double b) {
  const int tid = blockIdx.x * kProbeBlock + threadIdx.x;
  // b < 1 and c > 0 keep every chain bounded (it tends to c / (1 - b))
  const double c = 0x1p-30 * (double)(1 + (threadIdx.x & 7));
  double a[kProbeChains];
#pragma unroll
  for (int i = 0; i < kProbeChains; ++i) a[i] = 1.0 + 0x1p-10 * i;
  for (int it = 0; it < iters; ++it) {
#pragma unroll
    for (int i = 0; i < kProbeChains; ++i) a[i] = fma(a[i], b, c);
  }
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < kProbeChains; ++i) s += a[i];
  out[tid] = s;
}

// FP64 matrix-core probe: every thread runs `iters` rounds of 4
// independent v_mfma_f64_16x16x4_f64 chains (each MFMA: a 16 x 16 x 4
// product, 2048 flop per wave); with_valu adds the vector probe's 16 FMA
// chains to every round, to see whether the matrix cores add FP64
// throughput beside the vector units.
__global__ __launch_bounds__(kProbeBlock) void mfma64_probe(double* out, int iters, double b,
                                                            int with_valu) {
  typedef double v4d __attribute__((ext_vector_type(4)));
  const int tid = blockIdx.x * kProbeBlock + threadIdx.x;
  const double a_in = 0x1p-12 * (double)(1 + (threadIdx.x & 7));
  v4d acc[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) acc[i] = v4d{0.0, 0.0, 0.0, 0.0};
  const double c = 0x1p-30 * (double)(1 + (threadIdx.x & 7));
  double a[kProbeChains];
#pragma unroll
  for (int i = 0; i < kProbeChains; ++i) a[i] = 1.0 + 0x1p-10 * i;
  if (with_valu) {
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
        acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_in, b, acc[i], 0, 0, 0);
#pragma unroll
      for (int i = 0; i < kProbeChains; ++i) a[i] = fma(a[i], b, c);
    }
  } else {
    for (int it = 0; it < iters; ++it) {
#pragma unroll
      for (int i = 0; i < 4; ++i)
        acc[i] = __builtin_amdgcn_mfma_f64_16x16x4f64(a_in, b, acc[i], 0, 0, 0);
    }
  }
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < 4; ++i) s += acc[i][0] + acc[i][1] + acc[i][2] + acc[i][3];
#pragma unroll
  for (int i = 0; i < kProbeChains; ++i) s += a[i];
  out[tid] = s;
}

}  // namespace kern
}  // namespace mhc

extern "C" mhc_status mhc_probe_mfma64(double* out, int32_t n_blocks, int32_t iters,
                                       int32_t with_valu, void* stream) {
  if (!out || n_blocks < 1 || n_blocks > (1 << 20) || iters < 1 || iters > (1 << 24))
    return mhc::fail(MHC_E_ARG, "mhc_probe_mfma64: NULL out, or n_blocks / iters out of range");
  hipLaunchKernelGGL(mhc::kern::mfma64_probe, dim3(n_blocks), dim3(mhc::kern::kProbeBlock), 0,
                     reinterpret_cast<hipStream_t>(stream), out, iters, 1.0 - 0x1p-20,
                     with_valu ? 1 : 0);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return mhc::fail(MHC_E_DEVICE, hipGetErrorString(e));
  return MHC_OK;
}

extern "C" mhc_status mhc_probe_fma64(double* out, int32_t n_blocks, int32_t iters, void* stream) {
  if (!out || n_blocks < 1 || n_blocks > (1 << 20) || iters < 1 || iters > (1 << 24))
    return mhc::fail(MHC_E_ARG, "mhc_probe_fma64: NULL out, or n_blocks / iters out of range");
  hipLaunchKernelGGL(mhc::kern::fma64_probe, dim3(n_blocks), dim3(mhc::kern::kProbeBlock), 0,
                     reinterpret_cast<hipStream_t>(stream), out, iters, 1.0 - 0x1p-20);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return mhc::fail(MHC_E_DEVICE, hipGetErrorString(e));
  return MHC_OK;
}
