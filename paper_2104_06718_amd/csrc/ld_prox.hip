// Kernels of the proximal solver (Sec. 3.3, Algorithm 2; momentum of App. F).
//
// The method of multipliers keeps, per subdomain, the duals lambda_k (rho_k here),
// the primal iterates xB_k, xA_k and the momentum pi_k.  Its augmented Lagrangian
// (eq:z_updates) is minimised approximately by block-coordinate Frank-Wolfe; the
// block of layer k holds (xB_k, xA_{k+1}).  The gradient of the augmented
// Lagrangian with respect to xB_k is rt_k = rho_k + (xB_k - xA_k) / eta, minus its
// gradient with respect to xA_k; the host keeps rt_k current in memory, since it
// is also the operand of the transposed products W_k^T rt_k.
//
// Per block k the host enqueues
//   the forward product zA_{k+1} = W_{k+1} z_k + b_{k+1} (contraction kernels), then
//   prox_block_kernel: one workgroup per subdomain computes the closed-form step
//   gamma* (eq:optimal-gamma-gauss) from two reductions, moves (xB_k, xA_{k+1})
//   along the Frank-Wolfe segment (eq:fw-update), refreshes rt_k and rt_{k+1},
//   and takes the conditional gradient of the next block: the inner minimisation
//   of P_{k+1} (Sec. 3.2.2) with coefficients rt_{k+1} and g_{k+1} = W_{k+2}^T rt_{k+2}.
// The transposed products g of a sweep only depend on the iterates left by the
// previous sweep (a block never changes the rt that a later block's g reads), so
// they are all formed at the start of the sweep.
#include "ld_device.h"

namespace ld {

// Sum of two doubles over the 256 threads of a block; every thread gets the sums.
__device__ __forceinline__ void block_sum2(double& a, double& b) {
  __shared__ double sa[4], sb[4];
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o, 64);
    b += __shfl_xor(b, o, 64);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sa[w] = a;
    sb[w] = b;
  }
  __syncthreads();
  // fixed order: the same sums on every thread and every run
  a = (sa[0] + sa[1]) + (sa[2] + sa[3]);
  b = (sb[0] + sb[1]) + (sb[2] + sb[3]);
}

__global__ __launch_bounds__(256) void prox_block_kernel(ProxBlockArgs P) {
  const int b = blockIdx.x;
  const size_t ob = (size_t)b * P.nB, oa = (size_t)b * P.nA;
  // 1. directional derivative and curvature of the augmented Lagrangian along the
  //    segment from the iterate to the conditional gradient
  double num = 0.0, den = 0.0;
  for (int i = threadIdx.x; i < P.nB; i += 256) {
    const double d = (double)P.xB[ob + i] - (double)P.zB[ob + i];
    num += (double)P.rtB[ob + i] * d;
    den += d * d;
  }
  for (int i = threadIdx.x; i < P.nA; i += 256) {
    const double e = (double)P.xA[oa + i] - (double)P.zA[oa + i];
    if (P.last) {
      num += (double)P.c[oa + i] * e;       // coefficient of xA_n is c (rt_n = -c)
    } else {
      num -= (double)P.rtA[oa + i] * e;
      den += e * e;
    }
  }
  block_sum2(num, den);
  den *= P.inv_eta_d;
  // zero curvature: the segment is linear, take all of it if it descends
  const double gd = den > 0.0 ? fmin(fmax(num / den, 0.0), 1.0) : (num > 0.0 ? 1.0 : 0.0);
  const float g = (float)gd;
  // 2. Frank-Wolfe step on xB_k and the refreshed coefficient rt_k
  for (int i = threadIdx.x; i < P.nB; i += 256) {
    const float x = P.xB[ob + i];
    const float xn = x + g * (P.zB[ob + i] - x);
    P.xB[ob + i] = xn;
    P.rtB[ob + i] = P.rhoB[ob + i] + (xn - P.xAB[ob + i]) * P.inv_eta;
  }
  // 3. Frank-Wolfe step on xA_{k+1}; rt_{k+1}; conditional gradient of block k+1
  for (int i = threadIdx.x; i < P.nA; i += 256) {
    const float x = P.xA[oa + i];
    const float xn = x + g * (P.zA[oa + i] - x);
    P.xA[oa + i] = xn;
    if (P.last) continue;
    const float r = P.rhoA[oa + i] + (P.xBA[oa + i] - xn) * P.inv_eta;
    P.rtA[oa + i] = r;
    float zb, z, val;
    inner_min<float>(r, P.g[oa + i], P.lo[oa + i], P.hi[oa + i], P.tau, zb, z, val);
    P.zB_out[oa + i] = zb;
    if (P.z_bf16)
      ((bf16_t*)P.z_out)[oa + i] = f2bf(z);
    else
      ((float*)P.z_out)[oa + i] = z;
  }
}

// Dual update with momentum (eq:momentum_updates) and the coefficients rt of the
// next outer iteration; update = 0 only refreshes rt.  blockIdx.y: layer.
__global__ __launch_bounds__(256) void prox_dual_kernel(ProxDualPack P, int update, float inv_eta, float mu,
                                                        float inv_eta_next) {
  const int L = blockIdx.y;
  const size_t n = P.cnt[L];
  float* __restrict__ rho = P.rho[L];
  float* __restrict__ pi = P.pi[L];
  const float* __restrict__ xB = P.xB[L];
  const float* __restrict__ xA = P.xA[L];
  float* __restrict__ rt = P.rt[L];
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const float d = xB[i] - xA[i];
    float r = rho[i];
    if (update) {
      const float p = mu * pi[i] + d * inv_eta;
      pi[i] = p;
      r = r + p;
      rho[i] = r;
    }
    rt[i] = r + d * inv_eta_next;
  }
}

// x = max(xB, 0): the ReLU output at a vertex of the hull (every vertex has
// x = relu(xB)), in the operand precision of the forward product.
__global__ __launch_bounds__(256) void relu_operand_kernel(size_t n, const float* __restrict__ xb, void* out,
                                                           int bf16) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const float x = fmaxf(xb[i], 0.f);
    if (bf16)
      ((bf16_t*)out)[i] = f2bf(x);
    else
      ((float*)out)[i] = x;
  }
}

namespace {
unsigned grid_1d(size_t n) {
  const size_t g = (n + 255) / 256;
  return (unsigned)(g < 4096 ? (g > 0 ? g : 1) : 4096);
}
}  // namespace

hipError_t launch_prox_block(const ProxBlockArgs& a, int B, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  if (a.nA <= 0 || a.nB < 0) return hipErrorInvalidValue;
  if (!a.xA || !a.zA || (a.last ? !a.c : (!a.rtA || !a.rhoA || !a.xBA || !a.g || !a.lo || !a.hi || !a.zB_out ||
                                           !a.z_out)))
    return hipErrorInvalidValue;
  if (a.nB > 0 && (!a.xB || !a.zB || !a.rtB || !a.rhoB || !a.xAB)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(prox_block_kernel, dim3(B), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_prox_dual(const ProxDualPack& p, int update, float inv_eta, float mu, float inv_eta_next,
                            hipStream_t s) {
  if (p.n <= 0) return hipSuccess;
  if (p.n > kProxPackMax) return hipErrorInvalidValue;
  size_t mx = 0;
  for (int i = 0; i < p.n; ++i) mx = p.cnt[i] > mx ? p.cnt[i] : mx;
  hipLaunchKernelGGL(prox_dual_kernel, dim3(grid_1d(mx), p.n), dim3(256), 0, s, p, update, inv_eta, mu,
                     inv_eta_next);
  return hipGetLastError();
}

hipError_t launch_relu_operand(size_t n, const float* xb, void* out, int bf16, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(relu_operand_kernel, dim3(grid_1d(n)), dim3(256), 0, s, n, xb, out, bf16);
  return hipGetLastError();
}

}  // namespace ld
