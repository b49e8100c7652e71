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
//   of P_{k+1} (Sec. 3.2.2) with coefficients rt_{k+1} and g_{k+1} = W_{k+2}^T rt_{k+2};
//   in the last sweep of an outer iteration it also takes layer k's dual step.
// The transposed products g of a sweep only depend on the iterates left by the
// previous sweep (a block never changes the rt that a later block's g reads), so
// they are all formed at the start of the sweep.
#include "ld_device.h"

namespace ld {

constexpr int kProxThreads = 1024;  // 16 waves per subdomain: enough loads in flight per CU

// Sum of two doubles over the threads of a block; every thread gets the sums.
__device__ __forceinline__ void block_sum2(double& a, double& b) {
  constexpr int NW = kProxThreads / 64;
  __shared__ double sa[NW], sb[NW];
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
  a = 0.0;
  b = 0.0;
#pragma unroll
  for (int i = 0; i < NW; ++i) {
    a += sa[i];
    b += sb[i];
  }
}

__device__ __forceinline__ float4 ld4f(const float* p) { return *reinterpret_cast<const float4*>(p); }
__device__ __forceinline__ void st4f(float* p, float a, float b, float c, float d) {
  *reinterpret_cast<float4*>(p) = make_float4(a, b, c, d);
}
__device__ __forceinline__ float f4at(const float4& v, int q) { return q == 0 ? v.x : q == 1 ? v.y : q == 2 ? v.z : v.w; }

// Elements of a row that thread `tid` owns: where the row's width is a multiple
// of 4, the 16-byte groups i = 4*tid + 4*kProxThreads*j, else the single
// elements i = tid + kProxThreads*j.  The first group's iterate and conditional
// gradient stay in registers between the two passes (a whole row of up to
// 4*kProxThreads elements is then read once).
__global__ __launch_bounds__(kProxThreads) void prox_block_kernel(ProxBlockArgs P) {
  const int b = blockIdx.x, tid = threadIdx.x;
  const size_t ob = (size_t)b * P.nB, oa = (size_t)b * P.nA;
  const bool vB = (P.nB & 3) == 0, vA = (P.nA & 3) == 0;
  // 1. directional derivative and curvature of the augmented Lagrangian along the
  //    segment from the iterate to the conditional gradient
  double num = 0.0, den = 0.0;
  const int i0 = 4 * tid;
  float4 cxB = make_float4(0.f, 0.f, 0.f, 0.f), czB = cxB, cxA = cxB, czA = cxB;
  if (vB) {
    for (int i = i0; i < P.nB; i += 4 * kProxThreads) {
      const float4 x = ld4f(P.xB + ob + i), z = ld4f(P.zB + ob + i), r = ld4f(P.rtB + ob + i);
      if (i == i0) {
        cxB = x;
        czB = z;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double d = (double)f4at(x, q) - (double)f4at(z, q);
        num += (double)f4at(r, q) * d;
        den += d * d;
      }
    }
  } else {
    for (int i = tid; i < P.nB; i += kProxThreads) {
      const double d = (double)P.xB[ob + i] - (double)P.zB[ob + i];
      num += (double)P.rtB[ob + i] * d;
      den += d * d;
    }
  }
  // coefficient of xA_{k+1}: -rt_{k+1}; of the objective layer's xA_n: c
  const float* cA = P.last ? P.c : P.rtA;
  const double sgn = P.last ? 1.0 : -1.0;
  const double curv = P.last ? 0.0 : 1.0;
  if (vA) {
    for (int i = i0; i < P.nA; i += 4 * kProxThreads) {
      const float4 x = ld4f(P.xA + oa + i), z = ld4f(P.zA + oa + i), r = ld4f(cA + oa + i);
      if (i == i0) {
        cxA = x;
        czA = z;
      }
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const double e = (double)f4at(x, q) - (double)f4at(z, q);
        num += sgn * (double)f4at(r, q) * e;
        den += curv * e * e;
      }
    }
  } else {
    for (int i = tid; i < P.nA; i += kProxThreads) {
      const double e = (double)P.xA[oa + i] - (double)P.zA[oa + i];
      num += sgn * (double)cA[oa + i] * e;
      den += curv * e * e;
    }
  }
  block_sum2(num, den);
  den *= P.inv_eta_d;
  // zero curvature: the segment is linear, take all of it if it descends
  const double gd = den > 0.0 ? fmin(fmax(num / den, 0.0), 1.0) : (num > 0.0 ? 1.0 : 0.0);
  const float g = (float)gd;
  const float ie = P.inv_eta;
  // 2. Frank-Wolfe step on xB_k and the refreshed coefficient rt_k; in the last
  //    sweep of an outer iteration xB_k and xA_k are final here, so layer k's dual
  //    update (eq:momentum_updates) follows, and rt_k is formed for the next eta
  if (vB) {
    for (int i = i0; i < P.nB; i += 4 * kProxThreads) {
      const float4 x = i == i0 ? cxB : ld4f(P.xB + ob + i), z = i == i0 ? czB : ld4f(P.zB + ob + i);
      const float4 r = ld4f(P.rhoB + ob + i), a = ld4f(P.xAB + ob + i);
      float xn[4], rn[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) xn[q] = f4at(x, q) + g * (f4at(z, q) - f4at(x, q));
      st4f(P.xB + ob + i, xn[0], xn[1], xn[2], xn[3]);
      if (P.dual) {
        const float4 p = ld4f(P.piB + ob + i);
        float pn[4], rh[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float d = xn[q] - f4at(a, q);
          pn[q] = P.mu * f4at(p, q) + d * ie;
          rh[q] = f4at(r, q) + pn[q];
          rn[q] = rh[q] + d * P.inv_eta_next;
        }
        st4f(P.piB + ob + i, pn[0], pn[1], pn[2], pn[3]);
        st4f(const_cast<float*>(P.rhoB) + ob + i, rh[0], rh[1], rh[2], rh[3]);
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) rn[q] = f4at(r, q) + (xn[q] - f4at(a, q)) * ie;
      }
      st4f(P.rtB + ob + i, rn[0], rn[1], rn[2], rn[3]);
    }
  } else {
    for (int i = tid; i < P.nB; i += kProxThreads) {
      const float x = P.xB[ob + i];
      const float xn = x + g * (P.zB[ob + i] - x);
      P.xB[ob + i] = xn;
      const float d = xn - P.xAB[ob + i];
      if (P.dual) {
        const float pn = P.mu * P.piB[ob + i] + d * ie;
        const float rh = P.rhoB[ob + i] + pn;
        P.piB[ob + i] = pn;
        const_cast<float*>(P.rhoB)[ob + i] = rh;
        P.rtB[ob + i] = rh + d * P.inv_eta_next;
      } else {
        P.rtB[ob + i] = P.rhoB[ob + i] + d * ie;
      }
    }
  }
  // 3. Frank-Wolfe step on xA_{k+1}; rt_{k+1}; conditional gradient of block k+1
  if (vA) {
    for (int i = i0; i < P.nA; i += 4 * kProxThreads) {
      const float4 x = i == i0 ? cxA : ld4f(P.xA + oa + i), z = i == i0 ? czA : ld4f(P.zA + oa + i);
      float xn[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) xn[q] = f4at(x, q) + g * (f4at(z, q) - f4at(x, q));
      st4f(P.xA + oa + i, xn[0], xn[1], xn[2], xn[3]);
      if (P.last) continue;
      const float4 r = ld4f(P.rhoA + oa + i), xb = ld4f(P.xBA + oa + i), gg = ld4f(P.g + oa + i);
      const float4 lo = ld4f(P.lo + oa + i), hi = ld4f(P.hi + oa + i);
      float rn[4], zb[4], zz[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        rn[q] = f4at(r, q) + (f4at(xb, q) - xn[q]) * ie;
        float val;
        inner_min<float>(rn[q], f4at(gg, q), f4at(lo, q), f4at(hi, q), P.tau, zb[q], zz[q], val);
      }
      st4f(P.rtA + oa + i, rn[0], rn[1], rn[2], rn[3]);
      st4f(P.zB_out + oa + i, zb[0], zb[1], zb[2], zb[3]);
      if (P.z_bf16) {
        uint2 w;
        w.x = (uint32_t)f2bf(zz[0]) | ((uint32_t)f2bf(zz[1]) << 16);
        w.y = (uint32_t)f2bf(zz[2]) | ((uint32_t)f2bf(zz[3]) << 16);
        *reinterpret_cast<uint2*>((bf16_t*)P.z_out + oa + i) = w;
      } else {
        st4f((float*)P.z_out + oa + i, zz[0], zz[1], zz[2], zz[3]);
      }
    }
  } else {
    for (int i = tid; i < P.nA; i += kProxThreads) {
      const float x = P.xA[oa + i];
      const float xn = x + g * (P.zA[oa + i] - x);
      P.xA[oa + i] = xn;
      if (P.last) continue;
      const float r = P.rhoA[oa + i] + (P.xBA[oa + i] - xn) * ie;
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
}

// Coefficients rt = rho + (xB - xA) * inv_eta of every hidden layer (the start of
// a call).  blockIdx.y: layer.
__global__ __launch_bounds__(256) void prox_coeff_kernel(ProxDualPack P, float inv_eta) {
  const int L = blockIdx.y;
  const size_t n = P.cnt[L];
  const float* __restrict__ rho = P.rho[L];
  const float* __restrict__ xB = P.xB[L];
  const float* __restrict__ xA = P.xA[L];
  float* __restrict__ rt = P.rt[L];
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const size_t n4 = n / 4;  // 16-byte groups (every array starts 256-byte aligned)
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
    const float4 b = ld4f(xB + 4 * i), a = ld4f(xA + 4 * i), r = ld4f(rho + 4 * i);
    *reinterpret_cast<float4*>(rt + 4 * i) = make_float4(r.x + (b.x - a.x) * inv_eta, r.y + (b.y - a.y) * inv_eta,
                                                         r.z + (b.z - a.z) * inv_eta, r.w + (b.w - a.w) * inv_eta);
  }
  for (size_t i = 4 * n4 + (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    rt[i] = rho[i] + (xB[i] - xA[i]) * inv_eta;
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
  if (a.nB > 0 && (!a.xB || !a.zB || !a.rtB || !a.rhoB || !a.xAB || (a.dual && !a.piB))) return hipErrorInvalidValue;
  hipLaunchKernelGGL(prox_block_kernel, dim3(B), dim3(kProxThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_prox_coeff(const ProxDualPack& p, float inv_eta, hipStream_t s) {
  if (p.n <= 0) return hipSuccess;
  if (p.n > kProxPackMax) return hipErrorInvalidValue;
  size_t mx = 0;
  for (int i = 0; i < p.n; ++i) mx = p.cnt[i] > mx ? p.cnt[i] : mx;
  hipLaunchKernelGGL(prox_coeff_kernel, dim3(grid_1d(mx / 4 + 1), p.n), dim3(256), 0, s, p, inv_eta);
  return hipGetLastError();
}

hipError_t launch_relu_operand(size_t n, const float* xb, void* out, int bf16, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(relu_operand_kernel, dim3(grid_1d(n)), dim3(256), 0, s, n, xb, out, bf16);
  return hipGetLastError();
}

}  // namespace ld
