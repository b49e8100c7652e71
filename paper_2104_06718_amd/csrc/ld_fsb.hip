// Kernels of Filtered Smart Branching (Sec. 4.2).
//
// Scores (eq:fsb-scores, and the backup scores of eq:babsr-scores) come from the
// backward pass lambda_k of the WK dual assignment, formed by the contraction
// kernels; per subdomain and hidden layer the ambiguous ReLU with the largest
// s_FSB and the one with the largest t_SR are the candidates (eq:fsb-prefilter).
// Each candidate has two children (the ReLU fixed active: l := 0, or inactive:
// u := 0); every child is one subdomain of an expanded batch whose CROWN and WK
// bounds (q at the propagation duals, Prop. 2) the contraction kernels compute.
// The split is the candidate whose worse child has the best of the two bounds.
// The children of the chosen splits start from their parent's duals (Sec. 7.3).
//
// Child g of the expanded batch: subdomain g / M with M = 4 (n-1); r = g % M gives
// the hidden layer r / 4 + 1, the candidate (r / 2) % 2 (0: s_FSB, 1: t_SR) and the
// phase r % 2 (0: active, 1: inactive).
#include "ld_device.h"

namespace ld {

struct FsbPack {
  int nh;
  const float* lam[kFsbMaxHidden];
  const float* lo[kFsbMaxHidden];
  const float* hi[kFsbMaxHidden];
  const float* bias[kFsbMaxHidden];
  int bias_div[kFsbMaxHidden];
  int width[kFsbMaxHidden];
};

// keep (v, i) if it beats (bv, bi): larger value, the smaller index on ties
__device__ __forceinline__ void take_best(double v, int i, double& bv, int& bi) {
  if (v > bv || (v == bv && i < bi)) {
    bv = v;
    bi = i;
  }
}

// One block per (subdomain, hidden layer): the two candidates of that layer.
__global__ __launch_bounds__(256) void fsb_scores_kernel(FsbPack P, int* __restrict__ cand) {
  const int b = blockIdx.x, k = blockIdx.y;
  const int w = P.width[k];
  const size_t o = (size_t)b * w;
  double bs = -1.0, bt = -1.0;
  int is = 0x7fffffff, it = 0x7fffffff;
  for (int i = threadIdx.x; i < w; i += 256) {
    const double l = P.lo[k][o + i], u = P.hi[k][o + i];
    if (!(l < 0.0 && u > 0.0)) continue;  // only ambiguous ReLUs are branched on
    const double lam = P.lam[k][o + i];
    const double bias = P.bias[k][i / P.bias_div[k]];
    const double den = u - l;
    const double lb = lam * bias;
    const double lp = lam > 0.0 ? lam : 0.0;
    const double sf = fabs(fmin(0.0, lb) - (u / den) * lb + (u * l / den) * lp);
    const double tr = (-u * l / den) * lp;
    take_best(sf, i, bs, is);
    take_best(tr, i, bt, it);
  }
  __shared__ double sv[2][256];
  __shared__ int si[2][256];
  sv[0][threadIdx.x] = bs;
  si[0][threadIdx.x] = is;
  sv[1][threadIdx.x] = bt;
  si[1][threadIdx.x] = it;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (threadIdx.x < h)
      for (int c = 0; c < 2; ++c) {
        double v = sv[c][threadIdx.x];
        int i = si[c][threadIdx.x];
        take_best(sv[c][threadIdx.x + h], si[c][threadIdx.x + h], v, i);
        sv[c][threadIdx.x] = v;
        si[c][threadIdx.x] = i;
      }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const size_t q = ((size_t)b * P.nh + k) * 2;
    cand[q] = si[0][0] == 0x7fffffff ? -1 : si[0][0];
    cand[q + 1] = si[1][0] == 0x7fffffff ? -1 : si[1][0];
  }
}

struct FsbExpandArgs {
  IntermPack K;  // the parent rows copied into every child (l0, u0, l_k, u_k, c)
  float* lo[kFsbMaxHidden];
  float* hi[kFsbMaxHidden];
  int width[kFsbMaxHidden];
  int nh;
  const int* cand;
};

// One block per child: copy its subdomain's rows, then fix the split ReLU.
__global__ __launch_bounds__(256) void fsb_expand_kernel(FsbExpandArgs A) {
  const size_t g = blockIdx.x;
  const int M = 4 * A.nh;
  const size_t b = g / M;
  const int r = (int)(g % M);
  for (int a = 0; a < A.K.n; ++a) {
    const int w = A.K.width[a];
    const float* __restrict__ src = A.K.src[a] + b * w;
    float* __restrict__ dst = A.K.dst[a] + g * w;
    for (int i = threadIdx.x; i < w; i += 256) dst[i] = src[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int k = r / 4, col = (r / 2) % 2, inactive = r % 2;
    const int i = A.cand[(b * A.nh + k) * 2 + col];
    if (i >= 0) {
      float* dst = inactive ? A.hi[k] : A.lo[k];
      dst[g * A.width[k] + i] = 0.f;
    }
  }
}

struct ChildArgs {
  IntermPack K;  // parent rows copied into both children (l0, u0, l_k, u_k, c, then rho_k)
  float* lo[kFsbMaxHidden];
  float* hi[kFsbMaxHidden];
  int width[kFsbMaxHidden];
  int nh;
  const int* layer;
  const int* index;
};

// One block per child: child 2b (active: l := 0) and 2b+1 (inactive: u := 0) of
// subdomain b, split on ReLU index[b] of hidden layer layer[b] (no split if the
// pair is out of range, e.g. index -1).
__global__ __launch_bounds__(256) void branch_children_kernel(ChildArgs A) {
  const size_t g = blockIdx.x;
  const size_t b = g / 2;
  for (int a = 0; a < A.K.n; ++a) {
    const int w = A.K.width[a];
    const float* __restrict__ src = A.K.src[a] + b * w;
    float* __restrict__ dst = A.K.dst[a] + g * w;
    for (int i = threadIdx.x; i < w; i += 256) dst[i] = src[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    // a split outside the network's hidden layers or widths leaves both children unsplit
    const int k = A.layer[b], i = A.index[b];
    if (k >= 1 && k <= A.nh && i >= 0 && i < A.width[k - 1]) {
      float* dst = (g & 1) ? A.hi[k - 1] : A.lo[k - 1];
      dst[g * A.width[k - 1] + i] = 0.f;
    }
  }
}

hipError_t launch_branch_children(const IntermPack& K, int B, int n_hidden, const int* layer, const int* index,
                                  float* const* lo_child, float* const* hi_child, const int* width, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  if (n_hidden <= 0 || n_hidden > kFsbMaxHidden || K.n > kIntermMaxArrays || !layer || !index)
    return hipErrorInvalidValue;
  ChildArgs A;
  A.K = K;
  A.nh = n_hidden;
  A.layer = layer;
  A.index = index;
  for (int k = 0; k < n_hidden; ++k) {
    A.lo[k] = lo_child[k];
    A.hi[k] = hi_child[k];
    A.width[k] = width[k];
  }
  hipLaunchKernelGGL(branch_children_kernel, dim3((unsigned)(2 * (size_t)B)), dim3(256), 0, s, A);
  return hipGetLastError();
}

// One thread per subdomain: the candidate whose worse child has the best bound.
__global__ void fsb_select_kernel(int B, int nh, const int* __restrict__ cand, const double* __restrict__ qc,
                                  const double* __restrict__ qw, int* layer, int* index, double* value) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const int M = 4 * nh;
  double best = -INFINITY;
  int bl = 0, bi = -1;
  for (int k = 0; k < nh; ++k)
    for (int col = 0; col < 2; ++col) {
      const int i = cand[((size_t)b * nh + k) * 2 + col];
      if (i < 0) continue;
      const size_t g = (size_t)b * M + 4 * k + 2 * col;
      const double va = fmax(qc[g], qw[g]), vi = fmax(qc[g + 1], qw[g + 1]);
      const double v = fmin(va, vi);
      if (v > best) {
        best = v;
        bl = k + 1;
        bi = i;
      }
    }
  layer[b] = bl;
  index[b] = bi;
  value[b] = best;
}

hipError_t launch_fsb_scores(int B, int n_hidden, const float* const* lam, const float* const* lo,
                             const float* const* hi, const float* const* bias, const int* bias_div,
                             const int* width, int* cand, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  if (n_hidden <= 0 || n_hidden > kFsbMaxHidden || !cand) return hipErrorInvalidValue;
  FsbPack P;
  P.nh = n_hidden;
  for (int k = 0; k < n_hidden; ++k) {
    if (!lam[k] || !lo[k] || !hi[k] || !bias[k] || bias_div[k] < 1 || width[k] <= 0) return hipErrorInvalidValue;
    P.lam[k] = lam[k];
    P.lo[k] = lo[k];
    P.hi[k] = hi[k];
    P.bias[k] = bias[k];
    P.bias_div[k] = bias_div[k];
    P.width[k] = width[k];
  }
  hipLaunchKernelGGL(fsb_scores_kernel, dim3(B, n_hidden), dim3(256), 0, s, P, cand);
  return hipGetLastError();
}

hipError_t launch_fsb_expand(const IntermPack& K, int B, int n_hidden, const int* cand, float* const* lo_child,
                             float* const* hi_child, const int* width, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  if (n_hidden <= 0 || n_hidden > kFsbMaxHidden || K.n > kIntermMaxArrays || !cand) return hipErrorInvalidValue;
  FsbExpandArgs A;
  A.K = K;
  A.nh = n_hidden;
  A.cand = cand;
  for (int k = 0; k < n_hidden; ++k) {
    A.lo[k] = lo_child[k];
    A.hi[k] = hi_child[k];
    A.width[k] = width[k];
  }
  hipLaunchKernelGGL(fsb_expand_kernel, dim3((unsigned)((size_t)B * 4 * n_hidden)), dim3(256), 0, s, A);
  return hipGetLastError();
}

hipError_t launch_fsb_select(int B, int n_hidden, const int* cand, const double* q_crown, const double* q_wk,
                             int* layer, int* index, double* value, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  if (n_hidden <= 0 || !cand || !q_crown || !q_wk || !layer || !index || !value) return hipErrorInvalidValue;
  hipLaunchKernelGGL(fsb_select_kernel, dim3((B + 255) / 256), dim3(256), 0, s, B, n_hidden, cand, q_crown, q_wk,
                     layer, index, value);
  return hipGetLastError();
}

}  // namespace ld
