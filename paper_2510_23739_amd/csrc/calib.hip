// Calibration kernel, kept out of the reconstruction library (it builds as
// libpsoam_calib.so): a loop of dense BF16 matrix-core instructions
// (v_mfma_f32_16x16x32_bf16) with independent accumulators, timed by the
// kernel micro-benchmark to measure the rate the matrix cores of this device
// reach, beside the published dense peak that the roofline figures use.
#include <hip/hip_runtime.h>

#include <cstddef>

namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kChains = 8;  // independent accumulators per wave keep the pipe full

__global__ __launch_bounds__(256) void mfma_loop_bf16(float* __restrict__ out, int iters) {
  const int lane = (int)(threadIdx.x & 63);
  bf16x8 a, b;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    a[j] = (__bf16)(0.001f * (float)(lane + j));
    b[j] = (__bf16)(0.002f * (float)(lane - j));
  }
  // distinct starting values, so that the compiler cannot merge the chains
  // (they share a and b)
  f32x4 acc[kChains];
#pragma unroll
  for (int c = 0; c < kChains; ++c) {
    const float v = (float)(c * 64 + lane);
    acc[c] = f32x4{v, v + 0.25f, v + 0.5f, v + 0.75f};
  }
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < kChains; ++c)
      acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
  }
  float s = 0.0f;
#pragma unroll
  for (int c = 0; c < kChains; ++c) s += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  out[(size_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

// out: device, blocks * 256 floats (written, one per thread).  Flops of one
// launch: blocks * 4 waves * iters * 8 instructions * 16 * 16 * 32 * 2.
// Returns 0, 1 for invalid arguments, 3 if the launch failed.
extern "C" int psoam_calib_mfma_bf16(float* out, int blocks, int iters, void* stream) {
  if (!out || blocks <= 0 || iters <= 0) return 1;
  hipLaunchKernelGGL(mfma_loop_bf16, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream,
                     out, iters);
  return hipGetLastError() == hipSuccess ? 0 : 3;
}
