// HIP kernels (gfx950) of the Lagrangian-decomposition bounding step.
//
// One implicit-GEMM kernel serves every contraction of the method: the forward
// products W_k x + b_k and the transposed products W_k^T rho_k of fully
// connected and convolutional layers (Sec. 5.2: forward passes and
// backpropagation-like products; convolutions stay kernels).  Transposed
// convolutions are split by output-pixel parity ("stride classes"), so that
// every class is a dense GEMM with no structural zeros.  The per-neuron work of
// the method is fused into the epilogue: the closed-form inner minimisations
// over P_0 and P_k (Sec. 3.2.1, 3.2.2), the supergradient and the Adam step
// (Algorithm 1), the CROWN dual assignment (Prop. 2) and the network forward
// used for the upper bound (Sec. 5.1.3).
#include "ld_internal.h"

#include <type_traits>

namespace ld {

constexpr int kMaxClasses = 9;
struct GemmPack {
  int n;
  GemmGeom g[kMaxClasses];
};

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ bf16_t f2bf(float f) {
  // round to nearest even (inputs are finite)
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// ---------------------------------------------------------------------------
// per-neuron inner minimisation (Sec. 3.2.2): minimise r*xB - g*x over the
// ReLU hull with bounds [l, u]; ties go to the larger xB within a relative band.
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void inner_min(T r, T g, T l, T u, T tau, T& xb, T& x, T& val) {
  const T zero = T(0);
  if (l >= zero) {                       // passing: x = xB, coefficient (r - g)
    T cp = r - g;
    xb = (cp <= tau * (fabs(r) + fabs(g))) ? u : l;
    x = xb;
    T a = cp * l, b = cp * u;
    val = a < b ? a : b;
  } else if (u <= zero) {                // blocking: x = 0, coefficient r
    xb = (r <= zero) ? u : l;
    x = zero;
    T a = r * l, b = r * u;
    val = a < b ? a : b;
  } else {                               // ambiguous: vertices (l,0), (0,0), (u,u)
    T Vl = r * l;
    T Vu = (r - g) * u;
    T m = Vl < Vu ? Vl : Vu;
    m = m < zero ? m : zero;
    T band = tau * (fabs(Vl) + fabs(r * u) + fabs(g * u));
    if (Vu <= m + band) {
      xb = u;
      x = u;
    } else if (zero <= m + band) {
      xb = zero;
      x = zero;
    } else {
      xb = l;
      x = zero;
    }
    val = m;
  }
}

__device__ __forceinline__ void store_xs(const EpiArgs& E, size_t idx, float x) {
  if (E.xs_bf16)
    ((bf16_t*)E.xs)[idx] = f2bf(x);
  else
    ((float*)E.xs)[idx] = x;
}

// CROWN dual of one neuron from g = (W^T rho_next)[i] (eq:salman-assignment with
// the slopes of eq:slopes-biases: chord upper slope, lower slope 1[u >= -l]).
__device__ __forceinline__ float crown_dual(float g, float l, float u) {
  if (l >= 0.f) return g;
  if (u <= 0.f) return 0.f;
  if (g > 0.f) return (u / (u - l)) * g;
  return (u >= -l) ? g : 0.f;
}

__device__ __forceinline__ void adam_step(const EpiArgs& E, size_t idx, float s) {
  const float lr = E.adam[0], ibc1 = E.adam[1], ibc2 = E.adam[2], eps = E.adam[3];
  const float b1 = E.adam[4], b2 = E.adam[5];
  float m = b1 * E.m[idx] + (1.f - b1) * s;
  float v = b2 * E.v[idx] + (1.f - b2) * (s * s);
  E.m[idx] = m;
  E.v[idx] = v;
  float mh = m * ibc1;
  float vh = v * ibc2;
  E.rho_w[idx] = E.rho_w[idx] + lr * mh / (sqrtf(vh) + eps);
}

__device__ __forceinline__ void epilogue(const EpiArgs& E, size_t idx, int b, int col, float acc) {
  switch (E.kind) {
    case EPI_STORE:
      E.out_f[idx] = E.scale * acc;
      break;
    case EPI_P0: {
      const float lo = E.lo[idx], hi = E.hi[idx];
      const float x = (acc >= 0.f) ? hi : lo;
      store_xs(E, idx, x);
      if (E.want_val) E.val[idx] = -(double)acc * (double)x;
    } break;
    case EPI_INNER_MIN: {
      const float r = E.rho[idx], lo = E.lo[idx], hi = E.hi[idx];
      if (E.want_val) {
        double xb, x, val;
        inner_min<double>(r, acc, lo, hi, (double)E.tau, xb, x, val);
        E.val[idx] = val - (double)r * (double)E.bias[col / E.bias_div];
        store_xs(E, idx, (float)x);
        E.xb[idx] = (float)xb;
      } else {
        float xb, x, val;
        inner_min<float>(r, acc, lo, hi, E.tau, xb, x, val);
        store_xs(E, idx, x);
        E.xb[idx] = xb;
      }
    } break;
    case EPI_ADAM: {
      const float s = E.xb_in[idx] - (acc + E.bias[col]);
      adam_step(E, idx, s);
    } break;
    case EPI_SUPERGRAD:
      E.out_f[idx] = E.xb_in[idx] - (acc + E.bias[col]);
      break;
    case EPI_CROWN:
      E.out_f[idx] = crown_dual(acc, E.lo[idx], E.hi[idx]);
      break;
    case EPI_RELU_FWD: {
      const float y = acc + E.bias[col];
      if (!(y >= E.lo[idx] && y <= E.hi[idx])) E.flag[b] = 0;
      E.out_f[idx] = fmaxf(y, 0.f);
    } break;
    case EPI_BIAS_STORE:
      E.out_f[idx] = acc + E.bias[col];
      break;
    default:
      break;
  }
}

// ---------------------------------------------------------------------------
// implicit GEMM: block = 4 waves of 64 lanes; tile BM x BN, K step BK.
// ---------------------------------------------------------------------------
template <int BM, int BN, bool MMA_BF16, bool SRC_BF16>
__global__ __launch_bounds__(256) void gemm_kernel(GemmPack P, const void* __restrict__ src_v, EpiArgs E) {
  const GemmGeom& G = P.g[blockIdx.z];
  constexpr int BK = MMA_BF16 ? 32 : 16;
  constexpr int WM = (BN >= 64) ? 2 : 4;
  constexpr int WN = 4 / WM;
  constexpr int WTM = BM / WM;
  constexpr int WTN = BN / WN;
  constexpr int TM = WTM / 16;
  constexpr int TN = WTN / 16;
  static_assert(TM >= 1 && TN >= 1, "tile too small for the wave layout");
  using AT = typename std::conditional<MMA_BF16, bf16_t, float>::type;
  constexpr int LDA = BK + (MMA_BF16 ? 8 : 1);
  constexpr int LDC = BM + 1;

  __shared__ __attribute__((aligned(16))) AT As[BM * LDA];
  __shared__ __attribute__((aligned(16))) AT Bs[BN * LDA];
  __shared__ float Cs[BN * LDC];
  __shared__ int rowb[BM];
  __shared__ int rowy[BM];
  __shared__ int rowx[BM];

  const int m0 = blockIdx.x * BM;
  const int n0 = blockIdx.y * BN;
  if (m0 >= G.M || n0 >= G.N) return;  // uniform per block (classes differ in M)
  const int tid = threadIdx.x;

  for (int r = tid; r < BM; r += 256) {
    const int m = m0 + r;
    if (m < G.M) {
      const int b = m / G.HWq;
      const int rem = m - b * G.HWq;
      const int yq = rem / G.Wq;
      rowb[r] = b;
      rowy[r] = yq;
      rowx[r] = rem - yq * G.Wq;
    } else {
      rowb[r] = -1;
      rowy[r] = 0;
      rowx[r] = 0;
    }
  }
  __syncthreads();

  f32x4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  const float* srcf = (const float*)src_v;
  const bf16_t* srch = (const bf16_t*)src_v;
  const int wave = tid >> 6;
  const int lane = tid & 63;
  const int wm = wave % WM;
  const int wn = wave / WM;

  for (int k0 = 0; k0 < G.K; k0 += BK) {
    // gathered A tile (zero outside the source plane and beyond K)
    for (int e = tid; e < BM * BK; e += 256) {
      const int r = e / BK;
      const int kk = e - r * BK;
      const int k = k0 + kk;
      const int b = rowb[r];
      AT a = AT(0);
      if (b >= 0 && k < G.K) {
        const int4 t = G.ktab[k];
        const int iy = rowy[r] * G.iy_mul + G.iy_off + t.y;
        const int ix = rowx[r] * G.ix_mul + G.ix_off + t.z;
        if ((unsigned)iy < (unsigned)G.src_H && (unsigned)ix < (unsigned)G.src_W) {
          const size_t off = (size_t)b * G.src_n + t.x + iy * G.src_W + ix;
          if constexpr (SRC_BF16) {
            if constexpr (MMA_BF16)
              a = srch[off];
            else
              a = bf2f(srch[off]);
          } else {
            if constexpr (MMA_BF16)
              a = f2bf(srcf[off]);
            else
              a = srcf[off];
          }
        }
      }
      As[r * LDA + kk] = a;
    }
    // B tile from the packed [Np][Kp] operand (padding is zero)
    for (int e = tid; e < BN * BK; e += 256) {
      const int n = e / BK;
      const int kk = e - n * BK;
      const size_t off = (size_t)(n0 + n) * G.Kp + k0 + kk;
      if constexpr (MMA_BF16)
        Bs[n * LDA + kk] = G.Bh[off];
      else
        Bs[n * LDA + kk] = G.Bf[off];
    }
    __syncthreads();

    if constexpr (MMA_BF16) {
      bf16x8 av[TM], bv[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i)
        av[i] = *reinterpret_cast<const bf16x8*>(&As[(wm * WTM + i * 16 + (lane & 15)) * LDA + 8 * (lane >> 4)]);
#pragma unroll
      for (int j = 0; j < TN; ++j)
        bv[j] = *reinterpret_cast<const bf16x8*>(&Bs[(wn * WTN + j * 16 + (lane & 15)) * LDA + 8 * (lane >> 4)]);
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[i], bv[j], acc[i][j], 0, 0, 0);
    } else {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        float av[TM], bv[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) av[i] = As[(wm * WTM + i * 16 + (lane & 15)) * LDA + kk + (lane >> 4)];
#pragma unroll
        for (int j = 0; j < TN; ++j) bv[j] = Bs[(wn * WTN + j * 16 + (lane & 15)) * LDA + kk + (lane >> 4)];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[j], acc[i][j], 0, 0, 0);
      }
    }
    __syncthreads();
  }

  // stage the accumulators through LDS so that the epilogue walks memory in order
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int row = wm * WTM + i * 16 + 4 * (lane >> 4) + q;
        const int col = wn * WTN + j * 16 + (lane & 15);
        Cs[col * LDC + row] = acc[i][j][q];
      }
  __syncthreads();

  for (int e = tid; e < BM * BN; e += 256) {
    int r, n;
    if (G.m_fast) {
      n = e / BM;
      r = e - n * BM;
    } else {
      r = e / BN;
      n = e - r * BN;
    }
    const int b = rowb[r];
    const int col = n0 + n;
    if (b < 0 || col >= G.N) continue;
    const int j = col * G.dst_HW + (rowy[r] * G.oy_mul + G.oy_off) * G.dst_W + rowx[r] * G.ox_mul + G.ox_off;
    epilogue(E, (size_t)b * G.dst_n + j, b, col, Cs[n * LDC + r]);
  }
}

// ---------------------------------------------------------------------------
// tile dispatch
// ---------------------------------------------------------------------------
template <int BM, int BN>
static hipError_t launch_tile(const GemmPack& P, int max_m, const void* src, int src_bf16, int mma_bf16,
                              const EpiArgs& e, hipStream_t s) {
  dim3 grid((max_m + BM - 1) / BM, (P.g[0].N + BN - 1) / BN, P.n);
  dim3 block(256);
  if (mma_bf16) {
    if (src_bf16)
      hipLaunchKernelGGL((gemm_kernel<BM, BN, true, true>), grid, block, 0, s, P, src, e);
    else
      hipLaunchKernelGGL((gemm_kernel<BM, BN, true, false>), grid, block, 0, s, P, src, e);
  } else {
    if (src_bf16) return hipErrorInvalidValue;
    hipLaunchKernelGGL((gemm_kernel<BM, BN, false, false>), grid, block, 0, s, P, src, e);
  }
  return hipGetLastError();
}

int tile_supported(Tile t, int /*mma_bf16*/) {
  const int bm = t.bm, bn = t.bn;
  if (bn == 16 || bn == 32) return bm == 64 || bm == 128 || bm == 256;
  if (bn == 64 || bn == 128) return bm == 32 || bm == 64 || bm == 128;
  return 0;
}

hipError_t launch_gemm(const GemmGeom& g0, const void* src, int src_bf16, int mma_bf16, const EpiArgs& e,
                       Tile t, int n_classes, const GemmGeom* class_geoms, hipStream_t s) {
  GemmPack P;
  if (n_classes <= 0) {
    P.n = 1;
    P.g[0] = g0;
  } else {
    if (n_classes > kMaxClasses) return hipErrorInvalidValue;
    P.n = n_classes;
    for (int i = 0; i < n_classes; ++i) P.g[i] = class_geoms[i];
  }
  int max_m = 0;
  for (int i = 0; i < P.n; ++i) max_m = P.g[i].M > max_m ? P.g[i].M : max_m;
  if (max_m == 0 || P.g[0].N == 0) return hipSuccess;
#define LD_TILE(BM_, BN_) \
  if (t.bm == BM_ && t.bn == BN_) return launch_tile<BM_, BN_>(P, max_m, src, src_bf16, mma_bf16, e, s);
  LD_TILE(64, 16)
  LD_TILE(128, 16)
  LD_TILE(256, 16)
  LD_TILE(64, 32)
  LD_TILE(128, 32)
  LD_TILE(256, 32)
  LD_TILE(32, 64)
  LD_TILE(64, 64)
  LD_TILE(128, 64)
  LD_TILE(32, 128)
  LD_TILE(64, 128)
  LD_TILE(128, 128)
#undef LD_TILE
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// inner minimisation of the last hidden layer, whose coefficient
// g_{n-1} = W_n^T rho_n = -W_n^T c is constant over the ascent.  In ascent mode
// (t_dev != nullptr) thread 0 also advances the step counter and writes the
// scalars of this iteration's Adam step (Sec. 7.2: linear step decay).
// ---------------------------------------------------------------------------
__global__ void inner_min_const_kernel(int B, int n, const float* __restrict__ g, const float* __restrict__ rho,
                                       const float* __restrict__ lo, const float* __restrict__ hi,
                                       const float* __restrict__ bias, int bias_hw, float tau,
                                       float* __restrict__ xb, double* __restrict__ val, int* t_dev,
                                       float* adam, double lr0, double lr_end, int total, double beta1,
                                       double beta2, double eps) {
  const size_t total_n = (size_t)B * n;
  if (t_dev != nullptr && blockIdx.x == 0 && threadIdx.x == 0) {
    const int t = *t_dev + 1;
    *t_dev = t;
    const double lr = total > 1 ? lr0 + (lr_end - lr0) * (double)(t - 1) / (double)(total - 1) : lr0;
    adam[0] = (float)lr;
    adam[1] = (float)(1.0 / (1.0 - pow(beta1, (double)t)));
    adam[2] = (float)(1.0 / (1.0 - pow(beta2, (double)t)));
    adam[3] = (float)eps;
    adam[4] = (float)beta1;
    adam[5] = (float)beta2;
  }
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total_n; i += (size_t)gridDim.x * blockDim.x) {
    const int j = (int)(i % n);
    if (val != nullptr) {
      double xbd, xd, v;
      const double r = rho[i];
      inner_min<double>(r, g[i], lo[i], hi[i], (double)tau, xbd, xd, v);
      val[i] = v - r * (double)bias[j / bias_hw];
      xb[i] = (float)xbd;
    } else {
      float xbf, xf, v;
      inner_min<float>(rho[i], g[i], lo[i], hi[i], tau, xbf, xf, v);
      xb[i] = xbf;
    }
  }
}

__global__ void crown_const_kernel(int B, int n, const float* __restrict__ g, const float* __restrict__ lo,
                                   const float* __restrict__ hi, float* __restrict__ rho) {
  const size_t total_n = (size_t)B * n;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total_n; i += (size_t)gridDim.x * blockDim.x)
    rho[i] = crown_dual(g[i], lo[i], hi[i]);
}

// q[b] = cb[b] + sum over arrays of sum_j arr[b, j]; fixed summation order (FP64).
struct ReducePack {
  int n;
  const double* a[16];
  int sz[16];
};
__global__ void reduce_q_kernel(ReducePack P, const double* __restrict__ cb, double* __restrict__ q) {
  __shared__ double sh[256];
  const int b = blockIdx.x;
  double s = 0.0;
  for (int a = 0; a < P.n; ++a) {
    const double* p = P.a[a] + (size_t)b * P.sz[a];
    for (int j = threadIdx.x; j < P.sz[a]; j += 256) s += p[j];
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) q[b] = (cb ? cb[b] : 0.0) + sh[0];
}

// out[b] = sum_j c[b, j] * (y ? y[b, j] : bias[j])  (FP64)
__global__ void cdot_kernel(int n, const float* __restrict__ c, const float* __restrict__ y,
                            const float* __restrict__ bias, double* __restrict__ out) {
  __shared__ double sh[64];
  const int b = blockIdx.x;
  double s = 0.0;
  for (int j = threadIdx.x; j < n; j += 64) s += (double)c[(size_t)b * n + j] * (double)(y ? y[(size_t)b * n + j] : bias[j]);
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 32; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[b] = sh[0];
}

__global__ void validate_kernel(size_t total, const float* __restrict__ lo, const float* __restrict__ hi, int* bad) {
  int local = 0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const float a = lo[i], b = hi[i];
    if (!(isfinite(a) && isfinite(b) && a <= b)) local = 1;
  }
  if (local) atomicOr(bad, 1);
}

__global__ void fill_f32_kernel(float* p, size_t n, float v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void fill_i32_kernel(int* p, size_t n, int v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void copy_f32_kernel(float* __restrict__ d, const float* __restrict__ s, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) d[i] = s[i];
}
__global__ void max_f64_kernel(int B, const double* a, const double* b, double* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < B) out[i] = a[i] > b[i] ? a[i] : b[i];
}

static unsigned grid_for(size_t n) {
  size_t g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  if (g == 0) g = 1;
  return (unsigned)g;
}

hipError_t launch_inner_min_const(int B, int n, const float* g, const float* rho, const float* lo,
                                  const float* hi, const float* bias, int bias_hw, float tau, float* xb,
                                  double* val, int* t_dev, float* adam, double lr0, double lr_end, int total,
                                  double beta1, double beta2, double eps, hipStream_t s) {
  hipLaunchKernelGGL(inner_min_const_kernel, dim3(grid_for((size_t)B * n)), dim3(256), 0, s, B, n, g, rho, lo, hi,
                     bias, bias_hw, tau, xb, val, t_dev, adam, lr0, lr_end, total, beta1, beta2, eps);
  return hipGetLastError();
}

hipError_t launch_crown_const(int B, int n, const float* g, const float* lo, const float* hi, float* rho,
                              hipStream_t s) {
  hipLaunchKernelGGL(crown_const_kernel, dim3(grid_for((size_t)B * n)), dim3(256), 0, s, B, n, g, lo, hi, rho);
  return hipGetLastError();
}

hipError_t launch_reduce_q(int B, int n_arrays, const double* const* arrays, const int* sizes, const double* cb,
                           double* q, hipStream_t s) {
  ReducePack P;
  if (n_arrays > 16) return hipErrorInvalidValue;
  P.n = n_arrays;
  for (int i = 0; i < n_arrays; ++i) {
    P.a[i] = arrays[i];
    P.sz[i] = sizes[i];
  }
  hipLaunchKernelGGL(reduce_q_kernel, dim3(B), dim3(256), 0, s, P, cb, q);
  return hipGetLastError();
}

hipError_t launch_cdot(int B, int n, const float* c, const float* y, const float* bias, double* out, hipStream_t s) {
  hipLaunchKernelGGL(cdot_kernel, dim3(B), dim3(64), 0, s, n, c, y, bias, out);
  return hipGetLastError();
}

hipError_t launch_validate(int B, int n, const float* lo, const float* hi, int* bad, hipStream_t s) {
  const size_t total = (size_t)B * n;
  hipLaunchKernelGGL(validate_kernel, dim3(grid_for(total)), dim3(256), 0, s, total, lo, hi, bad);
  return hipGetLastError();
}

hipError_t launch_fill_f32(float* p, size_t n, float v, hipStream_t s) {
  hipLaunchKernelGGL(fill_f32_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_fill_i32(int* p, size_t n, int v, hipStream_t s) {
  hipLaunchKernelGGL(fill_i32_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}
hipError_t launch_copy_f32(float* dst, const float* src, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(copy_f32_kernel, dim3(grid_for(n)), dim3(256), 0, s, dst, src, n);
  return hipGetLastError();
}
hipError_t launch_max_f64(int B, const double* a, const double* b, double* out, hipStream_t s) {
  hipLaunchKernelGGL(max_f64_kernel, dim3((B + 255) / 256), dim3(256), 0, s, B, a, b, out);
  return hipGetLastError();
}

}  // namespace ld
