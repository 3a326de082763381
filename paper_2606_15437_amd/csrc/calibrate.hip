// INT32 VALU calibration microkernel: the device's sustained rate of plain
// 32-bit bitwise vector instructions, the ceiling the census evaluator is
// measured against (the analogue of the paper's uint32 XOR/AND/OR
// calibration in its system-evidence section).
//
// Each lane runs four independent chains of v_xor_b32 / v_and_b32 / v_or_b32
// written in inline assembly, so the instruction count is exact: 12
// instructions per loop iteration per lane, no compiler re-association into
// 3-input forms.
#include <hip/hip_runtime.h>

#include <cstdint>

namespace kripke {

__global__ __launch_bounds__(256) void calib_int32(uint32_t* out, uint32_t iters, uint32_t seed) {
  uint32_t a = threadIdx.x ^ seed, b = a * 2654435761u, c = ~a, d = a ^ 0x5bd1e995u;
  for (uint32_t i = 0; i < iters; ++i) {
    asm volatile(
        "v_xor_b32 %0, %0, %1\n\t"
        "v_xor_b32 %1, %1, %2\n\t"
        "v_xor_b32 %2, %2, %3\n\t"
        "v_xor_b32 %3, %3, %0\n\t"
        "v_and_b32 %0, %0, %2\n\t"
        "v_or_b32 %1, %1, %3\n\t"
        "v_and_b32 %2, %2, %0\n\t"
        "v_or_b32 %3, %3, %1\n\t"
        "v_xor_b32 %0, %0, %3\n\t"
        "v_xor_b32 %1, %1, %0\n\t"
        "v_or_b32 %2, %2, %1\n\t"
        "v_and_b32 %3, %3, %2\n\t"
        : "+v"(a), "+v"(b), "+v"(c), "+v"(d));
  }
  const uint32_t r = a ^ b ^ c ^ d;
  if (r == seed + 1) out[blockIdx.x * blockDim.x + threadIdx.x] = r;  // keep the chain live
}

hipError_t run_calibration(int cus, uint32_t iters, double* lane_ops_per_s, hipStream_t s) {
  const int blocks = cus * 32;  // 8 waves per SIMD
  uint32_t* out = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipMalloc(&out, sizeof(uint32_t) * blocks * 256);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(calib_int32, dim3(blocks), dim3(256), 0, s, out, iters / 8, 1u);  // warm
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e0, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(calib_int32, dim3(blocks), dim3(256), 0, s, out, iters, 2u);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
  if (e == hipSuccess)
    *lane_ops_per_s = 12.0 * iters * (double)blocks * 256.0 / (ms * 1e-3);
  // release what was created; the first failure is the one reported
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (out) (void)hipFree(out);
  return e;
}

}  // namespace kripke
