// Device-side warm start: unpacks a predicted (u, v, T) field, given per
// pixel with a row stride, into the three dense planes (u, v, theta) that the
// initialisation kernel reads.
#include <hip/hip_runtime.h>

#include "clb_internal.h"

namespace clb {

__global__ void __launch_bounds__(256) uvT_planes_kernel(const float *__restrict__ src,
                                                         int64_t stride, int64_t n,
                                                         double u_scale, double th_offset,
                                                         float *__restrict__ planes) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float *p = src + i * stride;
  planes[i] = (float)(u_scale * p[0]);
  planes[n + i] = (float)(u_scale * p[1]);
  planes[2 * n + i] = (float)(th_offset + p[2]);
}

hipError_t launch_uvT_planes(const float *src, int64_t stride, int64_t n, double u_scale,
                             double th_offset, float *planes, hipStream_t s) {
  hipLaunchKernelGGL(uvT_planes_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src,
                     stride, n, u_scale, th_offset, planes);
  return hipGetLastError();
}

}  // namespace clb
