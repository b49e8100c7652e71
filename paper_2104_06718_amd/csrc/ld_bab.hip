// Row moves of the branch-and-bound driver: subproblems (their bounds and
// warm-start duals) between the driver's store and the batches it bounds.
#include "ld_internal.h"

namespace ld {

namespace {

// Block (p, a) copies row pairs[p].x of array a (row 0 with `broadcast`) to row
// pairs[p].y of its destination.
__global__ void bab_rows_kernel(IntermPack K, const int2* __restrict__ pairs, int broadcast) {
  const int p = blockIdx.x, a = blockIdx.y;
  const int2 pr = pairs[p];
  const int w = K.width[a];
  const float* __restrict__ src = K.src[a] + (size_t)(broadcast ? 0 : pr.x) * w;
  float* __restrict__ dst = K.dst[a] + (size_t)pr.y * w;
  for (int j = threadIdx.x; j < w; j += blockDim.x) dst[j] = src[j];
}

}  // namespace

hipError_t launch_bab_rows(const IntermPack& K, const int2* pairs, int count, int broadcast, hipStream_t s) {
  if (count == 0 || K.n == 0) return hipSuccess;
  if (K.n > kIntermMaxArrays || count < 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(bab_rows_kernel, dim3((unsigned)count, (unsigned)K.n), dim3(256), 0, s, K, pairs, broadcast);
  return hipGetLastError();
}

}  // namespace ld
