// Pipelined pass kernels instantiated for precision class 6 (FP8 hi/lo split),
// and the device conversion of its factor images.
#include "fd_pass.inc"
#include "fd_pass2.inc"
#include "fd_pass3.inc"

namespace fdk {
template hipError_t launch3_p<6>(const PassArgs&, int, int, size_t, hipStream_t);

// FP32 image (rows x ld, row-major) -> FP8 split image: 16 bytes per 8
// consecutive entries of a row (their hi bytes, then their lo bytes), the
// same conversion the pass kernels apply to their data.
__global__ void fp8s_image_kernel(const float* __restrict__ src, unsigned char* __restrict__ dst, int64_t chunks) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= chunks) return;
  float v[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) v[j] = src[8 * c + j];
  const fp8s f = fp8s_pack8(v);
  *reinterpret_cast<fp8s*>(dst + 16 * c) = f;
}

hipError_t fp8s_image(const float* src, void* dst, int64_t entries, hipStream_t stream) {
  if (entries % 8 != 0) return hipErrorInvalidValue;
  const int64_t chunks = entries / 8;
  if (chunks == 0) return hipSuccess;
  const int64_t blocks = (chunks + 255) / 256;
  hipLaunchKernelGGL(fp8s_image_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, src,
                     static_cast<unsigned char*>(dst), chunks);
  return hipGetLastError();
}
}  // namespace fdk
