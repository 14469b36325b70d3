// Issue-rate probes of single vector-ALU instructions on the current GPU: the measured peaks of
// the integer-VALU roofline.  Each thread runs eight independent chains of one instruction
// (written in inline asm so that the compiler can neither fold nor replace it), enough waves fill
// every SIMD, and the rate is lane-operations per second over the kernel's event time.  Kind 6
// runs eight independent accumulator chains of the int8 matrix instruction the digit-plane
// select-and-sum uses (through its builtin: a matrix product is not folded away while its result
// is used), counted in int8 operations (2 x 16 x 16 x 64 per wave instruction).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace pepsi {
namespace {

constexpr int PR_TPB = 256, PR_CHAINS = 8, PR_UNROLL = 4;
typedef int v4i __attribute__((ext_vector_type(4)));

template <int KIND>
__global__ void __launch_bounds__(PR_TPB) k_probe_valu(uint32_t iters, uint32_t seed, uint64_t* __restrict__ sink) {
  uint32_t x[PR_CHAINS];
  uint64_t w[PR_CHAINS];
  double d[PR_CHAINS];
  const uint32_t c = seed | 1u, c2 = seed * 3u + 7u;
  const double dc = 1.0000001, dc2 = 1e-7;
#pragma unroll
  for (int i = 0; i < PR_CHAINS; ++i) {
    x[i] = (uint32_t)threadIdx.x * 2654435761u + (uint32_t)i;
    w[i] = x[i];
    d[i] = (double)x[i];
  }
  for (uint32_t it = 0; it < (KIND == 6 ? 0u : iters); ++it) {
#pragma unroll
    for (int r = 0; r < PR_UNROLL; ++r)
#pragma unroll
      for (int i = 0; i < PR_CHAINS; ++i) {
        if constexpr (KIND == 0) asm volatile("v_mad_u64_u32 %0, vcc, %1, %2, %0" : "+v"(w[i]) : "v"(x[i]), "v"(c) : "vcc");
        if constexpr (KIND == 1) asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(x[i]) : "v"(c));
        if constexpr (KIND == 2) asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(x[i]) : "v"(c));
        if constexpr (KIND == 3) asm volatile("v_add_u32 %0, %0, %1" : "+v"(x[i]) : "v"(c));
        if constexpr (KIND == 4) asm volatile("v_mad_u32_u24 %0, %0, %1, %2" : "+v"(x[i]) : "v"(c), "v"(c2));
        if constexpr (KIND == 5) asm volatile("v_fma_f64 %0, %0, %1, %2" : "+v"(d[i]) : "v"(dc), "v"(dc2));
      }
  }
  v4i m[PR_CHAINS];
  if constexpr (KIND == 6) {
    const v4i ma = v4i{(int)x[0], (int)x[1], (int)x[2], (int)x[3]};
    const v4i mb = v4i{(int)x[4], (int)x[5], (int)x[6], (int)c};
#pragma unroll
    for (int i = 0; i < PR_CHAINS; ++i) m[i] = v4i{i, 0, 0, 0};
    for (uint32_t it = 0; it < iters; ++it)
#pragma unroll
      for (int r = 0; r < PR_UNROLL; ++r)
#pragma unroll
        for (int i = 0; i < PR_CHAINS; ++i) m[i] = __builtin_amdgcn_mfma_i32_16x16x64_i8(ma, mb, m[i], 0, 0, 0);
  }
  uint64_t acc = 0;
#pragma unroll
  for (int i = 0; i < PR_CHAINS; ++i) acc += x[i] + w[i] + (uint64_t)d[i];
  if constexpr (KIND == 6) {
#pragma unroll
    for (int i = 0; i < PR_CHAINS; ++i) acc += (uint32_t)(m[i][0] + m[i][1] + m[i][2] + m[i][3]);
  }
  sink[(size_t)blockIdx.x * PR_TPB + threadIdx.x] = acc;
}

}  // namespace

int probe_valu(int kind, double* lane_ops_per_s) {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -7;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -7;
  const int blocks = cus * 4 * 8 * 64 / PR_TPB;         // 8 waves per SIMD, 4 SIMDs per CU
  const uint32_t iters = kind == 6 ? 2048 : 16384;     // a matrix instruction takes 16+ cycles
  uint64_t* sink = nullptr;
  if (hipMalloc(&sink, (size_t)blocks * PR_TPB * 8) != hipSuccess) return -6;
  hipEvent_t a, b;
  (void)hipEventCreate(&a);
  (void)hipEventCreate(&b);
  auto launch = [&](uint32_t n) {
    switch (kind) {
      case 0: hipLaunchKernelGGL(k_probe_valu<0>, dim3(blocks), dim3(PR_TPB), 0, 0, n, 12345u, sink); break;
      case 1: hipLaunchKernelGGL(k_probe_valu<1>, dim3(blocks), dim3(PR_TPB), 0, 0, n, 12345u, sink); break;
      case 2: hipLaunchKernelGGL(k_probe_valu<2>, dim3(blocks), dim3(PR_TPB), 0, 0, n, 12345u, sink); break;
      case 3: hipLaunchKernelGGL(k_probe_valu<3>, dim3(blocks), dim3(PR_TPB), 0, 0, n, 12345u, sink); break;
      case 4: hipLaunchKernelGGL(k_probe_valu<4>, dim3(blocks), dim3(PR_TPB), 0, 0, n, 12345u, sink); break;
      case 5: hipLaunchKernelGGL(k_probe_valu<5>, dim3(blocks), dim3(PR_TPB), 0, 0, n, 12345u, sink); break;
      default: hipLaunchKernelGGL(k_probe_valu<6>, dim3(blocks), dim3(PR_TPB), 0, 0, n, 12345u, sink); break;
    }
  };
  launch(64);                                           // warm-up
  (void)hipEventRecord(a, 0);
  launch(iters);
  (void)hipEventRecord(b, 0);
  const hipError_t e = hipEventSynchronize(b);
  float ms = 0;
  (void)hipEventElapsedTime(&ms, a, b);
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  (void)hipFree(sink);
  if (e != hipSuccess || ms <= 0) return -7;
  const double ops = (double)blocks * PR_TPB * iters * PR_UNROLL * PR_CHAINS * (kind == 6 ? 2 * 16 * 16 * 64 / 64 : 1);
  *lane_ops_per_s = ops / (ms * 1e-3);
  return 0;
}

}  // namespace pepsi
