// Kernels of the intermediate-bound workload (Sec. 2.2.3): the bounds on the
// pre-activations of layer j are LD bounds of the sub-network that ends at layer j,
// with the objective +x_j[i] (lower bound) or -x_j[i] (upper bound) for every
// neuron i.  Every (subdomain, neuron, sign) is one problem of the batch, so the
// neurons of a layer are solved simultaneously (Sec. 5.2).
//
// Problem g of the expanded batch is subdomain g / P, neuron (g % P) / 2, sign
// + for even g % P and - for odd, with P = 2 n_j.
#include "ld_device.h"

namespace ld {

// One block per problem of the chunk: copy its subdomain's rows of every per-
// subdomain array and write c = +-e_i.
__global__ __launch_bounds__(256) void interm_expand_kernel(IntermPack K, long long start, int P, int nj) {
  const long long g = start + blockIdx.x;
  const long long b = g / P;
  const int r = (int)(g % P);
  const size_t p = blockIdx.x;
  for (int a = 0; a < K.n; ++a) {
    const int w = K.width[a];
    const float* __restrict__ src = K.src[a] + (size_t)b * w;
    float* __restrict__ dst = K.dst[a] + p * w;
    for (int i = threadIdx.x; i < w; i += 256) dst[i] = src[i];
  }
  float* __restrict__ c = K.c + p * nj;
  const int i0 = r >> 1;
  const float v = (r & 1) ? -1.f : 1.f;
  for (int i = threadIdx.x; i < nj; i += 256) c[i] = i == i0 ? v : 0.f;
}

// bound[p] is a lower bound on c^T x_j for problem p: the lower bound of x_j[i]
// (sign +) or minus the upper bound (sign -), rounded outward to FP32.
__global__ __launch_bounds__(256) void interm_collect_kernel(int C, long long start, int P, int nj,
                                                             const double* __restrict__ bound, float* __restrict__ lo,
                                                             float* __restrict__ hi) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= C) return;
  const long long g = start + p;
  const long long b = g / P;
  const int r = (int)(g % P);
  const size_t idx = (size_t)b * nj + (r >> 1);
  const double v = bound[p];
  if ((r & 1) == 0) {
    float f = (float)v;
    if ((double)f > v) f = nextafterf(f, -INFINITY);
    lo[idx] = f;
  } else {
    const double u = -v;
    float f = (float)u;
    if ((double)f < u) f = nextafterf(f, INFINITY);
    hi[idx] = f;
  }
}

hipError_t launch_interm_expand(const IntermPack& K, int C, long long start, int P, int nj, hipStream_t s) {
  if (C <= 0) return hipSuccess;
  if (K.n < 0 || K.n > kIntermMaxArrays || P <= 0 || nj <= 0 || !K.c) return hipErrorInvalidValue;
  hipLaunchKernelGGL(interm_expand_kernel, dim3(C), dim3(256), 0, s, K, start, P, nj);
  return hipGetLastError();
}

hipError_t launch_interm_collect(int C, long long start, int P, int nj, const double* bound, float* lo, float* hi,
                                 hipStream_t s) {
  if (C <= 0) return hipSuccess;
  if (P <= 0 || nj <= 0 || !bound || !lo || !hi) return hipErrorInvalidValue;
  hipLaunchKernelGGL(interm_collect_kernel, dim3((C + 255) / 256), dim3(256), 0, s, C, start, P, nj, bound, lo, hi);
  return hipGetLastError();
}

}  // namespace ld
