// FP64 engine: the ascent of Algorithm 1 (Adam steps with the linear step decay
// of Sec. 7.2) with every operand, every accumulation and the state (rho, m, v)
// in FP64.  It computes the same iteration as the FP32/BF16 engine:
//   phase A  g_{k-1} = W_k^T rho_k for every hidden layer k, fused with the inner
//            minimisation of P_{k-1} (P_0: eq:box_bounds_sol; P_k: eq:min-pk);
//            the last hidden layer uses the constant g_{n-1} = -W_n^T c;
//   phase B  xhat_A,k = W_k x*_{k-1} + b_k fused with the supergradient
//            s_k = xhat_B,k* - xhat_A,k and the Adam ascent step on rho_k.
// The contractions are direct loops over the layer's weights (one thread per
// output neuron, a quarter of K per wave for fully-connected forward products),
// not MFMA tiles: this engine exists for the precision of the result, and its
// cost is dominated by the same HBM traffic as the FP32 engine's.
//
// Floating-point contraction is off in this translation unit, so every product
// and sum is rounded as written (no fused multiply-adds): the Adam update and the
// inner minimisation round like a plain evaluation of their formulas.
#pragma clang fp contract(off)

#include "ld_device.h"

namespace ld {

namespace {

__device__ __forceinline__ double f64_crown(double g, double l, double u, int wk) {
  if (l >= 0.0) return g;
  if (u <= 0.0) return 0.0;
  if (g > 0.0 || wk) return (u / (u - l)) * g;
  return (u >= -l) ? g : 0.0;
}

// Epilogue of one output value acc of neuron i (flat index idx = b*n + i).
__device__ __forceinline__ void f64_epilogue(const F64Epi& e, int b, int i, size_t idx, double acc) {
  switch (e.kind) {
    case F64_STORE:
      e.out[idx] = e.scale * acc;
      break;
    case F64_P0: {
      // box minimiser of P_0: the upper bound where the coefficient is >= 0
      const double x = acc >= 0.0 ? (double)e.hi[idx] : (double)e.lo[idx];
      e.xs[idx] = x;
      e.val[idx] = -(acc * x);
      break;
    }
    case F64_INNER: {
      const double r = e.rho[idx];
      double xb, x, v;
      inner_min<double>(r, acc, (double)e.lo[idx], (double)e.hi[idx], e.tau, xb, x, v);
      e.xb[idx] = xb;
      e.xs[idx] = x;
      e.val[idx] = v - r * e.bias[i / e.bias_div];
      break;
    }
    case F64_CROWN:
      e.out[idx] = f64_crown(acc, (double)e.lo[idx], (double)e.hi[idx], e.wk);
      break;
    case F64_ADAM: {
      const double xa = acc + e.bias[i / e.bias_div];
      const double s = e.xb_in[idx] - xa;
      const double m = e.beta1 * e.m[idx] + e.omb1 * s;
      const double v = e.beta2 * e.v[idx] + e.omb2 * s * s;
      e.m[idx] = m;
      e.v[idx] = v;
      const double mh = m / e.bc1;
      const double vh = v / e.bc2;
      e.rho_w[idx] = e.rho_w[idx] + e.lr * mh / (sqrt(vh) + e.eps);
      break;
    }
    case F64_SUPERGRAD: {
      const double s = e.xb_in[idx] - (acc + e.bias[i / e.bias_div]);
      if (e.out) e.out[idx] = s;
      if (e.out_f) e.out_f[idx] = (float)s;
      break;
    }
    case F64_RELU_FWD: {
      const double y = acc + e.bias[i / e.bias_div];
      if (!(y >= (double)e.lo[idx] && y <= (double)e.hi[idx])) e.flag[b] = 0;
      e.out[idx] = y > 0.0 ? y : 0.0;
      break;
    }
    case F64_BIAS:
      e.out[idx] = acc + e.bias[i / e.bias_div];
      break;
    default:
      break;
  }
}

// Transposed product g[b][j] = sum_i W[i][j] r[b][i] over the outputs i of the
// layer, j over its inputs; or, with gin, g read from gin (the constant
// coefficient of the last hidden layer).  Grid (ceil(n/256), B).
__global__ void __launch_bounds__(256) f64_transposed_kernel(F64Layer L, const double* __restrict__ r,
                                                             const double* __restrict__ gin, int n, F64Epi e) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  const int b = blockIdx.y;
  if (j >= n) return;
  const size_t idx = (size_t)b * n + j;
  double g = 0.0;
  if (gin != nullptr) {
    g = gin[idx];
  } else if (L.kind == 0) {
    const double* rb = r + (size_t)b * L.n_out;
    for (int i = 0; i < L.n_out; ++i) g += L.W[(size_t)i * L.n_in + j] * rb[i];
  } else {
    const double* rb = r + (size_t)b * L.n_out;
    const int HW = L.H * L.W_;
    const int ci = j / HW, rem = j - ci * HW;
    const int y = rem / L.W_, x = rem - (rem / L.W_) * L.W_;
    // taps with y = oy*stride - pad + ky, i.e. ky = (y + pad) mod stride, stepping by stride
    const int ky0 = (y + L.pad) % L.stride, kx0 = (x + L.pad) % L.stride;
    for (int co = 0; co < L.Co; ++co) {
      const double* wc = L.W + ((size_t)co * L.Ci + ci) * L.kh * L.kw;
      const double* rc = rb + (size_t)co * L.Ho * L.Wo;
      for (int ky = ky0; ky < L.kh; ky += L.stride) {
        const int oy = (y + L.pad - ky) / L.stride;
        if (y + L.pad - ky < 0 || oy >= L.Ho) continue;
        for (int kx = kx0; kx < L.kw; kx += L.stride) {
          const int ox = (x + L.pad - kx) / L.stride;
          if (x + L.pad - kx < 0 || ox >= L.Wo) continue;
          g += wc[ky * L.kw + kx] * rc[oy * L.Wo + ox];
        }
      }
    }
  }
  f64_epilogue(e, b, j, idx, g);
}

// Rounding margin of one coefficient map: for input j of the layer,
// out[b][j] = (gamma * sum_i |W[i][j]| |r[b][i]| + tiny) * xmax[b][j], with xmax the
// largest |x_j| on the feasible set of the minimisation the coefficient enters:
// max(|lo|, |hi|) for the input box (box = 1), max(0, hi) after a ReLU (box = 0).
// The same tap walk as f64_transposed_kernel, on absolute values, in FP64.
// Grid (ceil(n/256), B).
__global__ void __launch_bounds__(256) f64_abs_margin_kernel(F64Layer L, const float* __restrict__ r, int n,
                                                             const float* __restrict__ lo,
                                                             const float* __restrict__ hi, int box, double gamma,
                                                             double tiny, double* __restrict__ out) {
  const int j = blockIdx.x * 256 + threadIdx.x;
  const int b = blockIdx.y;
  if (j >= n) return;
  const size_t idx = (size_t)b * n + j;
  const float* rb = r + (size_t)b * L.n_out;
  double t = 0.0;
  if (L.kind == 0) {
    for (int i = 0; i < L.n_out; ++i) t += fabs(L.W[(size_t)i * L.n_in + j]) * fabs((double)rb[i]);
  } else {
    const int HW = L.H * L.W_;
    const int ci = j / HW, rem = j - ci * HW;
    const int y = rem / L.W_, x = rem - (rem / L.W_) * L.W_;
    const int ky0 = (y + L.pad) % L.stride, kx0 = (x + L.pad) % L.stride;
    for (int co = 0; co < L.Co; ++co) {
      const double* wc = L.W + ((size_t)co * L.Ci + ci) * L.kh * L.kw;
      const float* rc = rb + (size_t)co * L.Ho * L.Wo;
      for (int ky = ky0; ky < L.kh; ky += L.stride) {
        const int oy = (y + L.pad - ky) / L.stride;
        if (y + L.pad - ky < 0 || oy >= L.Ho) continue;
        for (int kx = kx0; kx < L.kw; kx += L.stride) {
          const int ox = (x + L.pad - kx) / L.stride;
          if (x + L.pad - kx < 0 || ox >= L.Wo) continue;
          t += fabs(wc[ky * L.kw + kx]) * fabs((double)rc[oy * L.Wo + ox]);
        }
      }
    }
  }
  const double l = (double)lo[idx], h = (double)hi[idx];
  const double xm = box ? fmax(fabs(l), fabs(h)) : fmax(0.0, h);
  out[idx] = (gamma * t + tiny) * xm;
}

// Forward product of a conv layer: y[b][i] = sum W[co][ci][ky][kx] x[b][ci][iy][ix].
// Grid (ceil(n_out/256), B).
__global__ void __launch_bounds__(256) f64_forward_conv_kernel(F64Layer L, const double* __restrict__ x, F64Epi e) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int b = blockIdx.y;
  if (i >= L.n_out) return;
  const int OHW = L.Ho * L.Wo;
  const int co = i / OHW, rem = i - co * OHW;
  const int oy = rem / L.Wo, ox = rem - (rem / L.Wo) * L.Wo;
  const double* xb = x + (size_t)b * L.n_in;
  double acc = 0.0;
  for (int ci = 0; ci < L.Ci; ++ci) {
    const double* wc = L.W + ((size_t)co * L.Ci + ci) * L.kh * L.kw;
    const double* xc = xb + (size_t)ci * L.H * L.W_;
    for (int ky = 0; ky < L.kh; ++ky) {
      const int iy = oy * L.stride - L.pad + ky;
      if (iy < 0 || iy >= L.H) continue;
      for (int kx = 0; kx < L.kw; ++kx) {
        const int ix = ox * L.stride - L.pad + kx;
        if (ix < 0 || ix >= L.W_) continue;
        acc += wc[ky * L.kw + kx] * xc[iy * L.W_ + ix];
      }
    }
  }
  f64_epilogue(e, b, i, (size_t)b * L.n_out + i, acc);
}

// Forward product of a fully-connected layer: 64 outputs per block (lane = output),
// the 4 waves of the block each sum every fourth input (coalesced rows of W^T), and
// the four partial sums are added in wave order.  Grid (ceil(n_out/64), B).
__global__ void __launch_bounds__(256) f64_forward_fc_kernel(F64Layer L, const double* __restrict__ x, F64Epi e) {
  __shared__ double part[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int i = blockIdx.x * 64 + lane;
  const int b = blockIdx.y;
  const double* xb = x + (size_t)b * L.n_in;
  double acc = 0.0;
  if (i < L.n_out)
    for (int j = w; j < L.n_in; j += 4) acc += L.WT[(size_t)j * L.n_out + i] * xb[j];
  part[w][lane] = acc;
  __syncthreads();
  if (w == 0 && i < L.n_out) {
    const double s = ((part[0][lane] + part[1][lane]) + part[2][lane]) + part[3][lane];
    f64_epilogue(e, b, i, (size_t)b * L.n_out + i, s);
  }
}

__global__ void f64_widen_kernel(size_t n, const float* __restrict__ src, double* __restrict__ dst) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = (double)src[i];
}

__global__ void f64_narrow_kernel(size_t n, const double* __restrict__ src, float* __restrict__ dst) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = (float)src[i];
}

__global__ void f64_copy_kernel(size_t n, const double* __restrict__ src, double* __restrict__ dst) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

// out[b] = sum_j c[b][j] * y[b][j] in FP64, fixed order (lane partials, then a tree).
__global__ void f64_cdot_kernel(int n, const float* __restrict__ c, const double* __restrict__ y,
                                double* __restrict__ out) {
  __shared__ double sh[64];
  const int b = blockIdx.x;
  double s = 0.0;
  for (int j = threadIdx.x; j < n; j += 64) s += (double)c[(size_t)b * n + j] * y[(size_t)b * n + j];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 32; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[b] = sh[0];
}

unsigned grid_1d(size_t n) {
  size_t g = (n + 255) / 256;
  if (g > 16384) g = 16384;
  if (g == 0) g = 1;
  return (unsigned)g;
}

}  // namespace

hipError_t launch_f64_transposed(const F64Layer& L, int B, const double* r, const double* gin, int n,
                                 const F64Epi& e, hipStream_t s) {
  if (B == 0 || n == 0) return hipSuccess;
  if (gin == nullptr && (r == nullptr || n != L.n_in)) return hipErrorInvalidValue;
  if (gin == nullptr && L.kind != 0 && (L.stride < 1 || L.pad < 0)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(f64_transposed_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)B), dim3(256), 0, s, L, r,
                     gin, n, e);
  return hipGetLastError();
}

hipError_t launch_f64_abs_margin(const F64Layer& L, int B, const float* r, int n, const float* lo, const float* hi,
                                 int box, double gamma, double tiny, double* out, hipStream_t s) {
  if (B == 0 || n == 0) return hipSuccess;
  if (r == nullptr || lo == nullptr || hi == nullptr || out == nullptr || n != L.n_in) return hipErrorInvalidValue;
  if (L.kind != 0 && (L.stride < 1 || L.pad < 0)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(f64_abs_margin_kernel, dim3((unsigned)((n + 255) / 256), (unsigned)B), dim3(256), 0, s, L, r, n,
                     lo, hi, box, gamma, tiny, out);
  return hipGetLastError();
}

hipError_t launch_f64_forward(const F64Layer& L, int B, const double* x, const F64Epi& e, hipStream_t s) {
  if (B == 0 || L.n_out == 0) return hipSuccess;
  if (L.kind == 0) {
    hipLaunchKernelGGL(f64_forward_fc_kernel, dim3((unsigned)((L.n_out + 63) / 64), (unsigned)B), dim3(256), 0, s,
                       L, x, e);
  } else {
    hipLaunchKernelGGL(f64_forward_conv_kernel, dim3((unsigned)((L.n_out + 255) / 256), (unsigned)B), dim3(256), 0,
                       s, L, x, e);
  }
  return hipGetLastError();
}

hipError_t launch_f64_widen(size_t n, const float* src, double* dst, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(f64_widen_kernel, dim3(grid_1d(n)), dim3(256), 0, s, n, src, dst);
  return hipGetLastError();
}

hipError_t launch_f64_narrow(size_t n, const double* src, float* dst, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(f64_narrow_kernel, dim3(grid_1d(n)), dim3(256), 0, s, n, src, dst);
  return hipGetLastError();
}

hipError_t launch_f64_copy(size_t n, const double* src, double* dst, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(f64_copy_kernel, dim3(grid_1d(n)), dim3(256), 0, s, n, src, dst);
  return hipGetLastError();
}

hipError_t launch_f64_cdot(int B, int n, const float* c, const double* y, double* out, hipStream_t s) {
  if (B == 0) return hipSuccess;
  hipLaunchKernelGGL(f64_cdot_kernel, dim3((unsigned)B), dim3(64), 0, s, n, c, y, out);
  return hipGetLastError();
}

}  // namespace ld
