// The P_k inner minimisation for sigmoid activations (App. E): the convex hull of
// sigma on [l, u] and the minimum of rho*xB - g*x over it, per neuron.
//
// Hull (App. E.1): the upper (concave) envelope is the chord when sigma'(u) is at
// least the chord's slope, else the line from (l, sigma(l)) tangent to sigma at
// t_up > max(l, 0) followed by sigma itself (t_up = l when l >= 0); the lower
// (convex) envelope mirrors it with the tangent point t_lo < min(u, 0).  The
// tangent points depend on the bounds only, so they are computed once per
// problem (sigmoid_hull_kernel, bisection on the tangency condition) and read by
// every inner minimisation (sigmoid_inner_min_kernel).
//
// Inner minimisation (eq:siglinopt): x takes the upper envelope where g > 0 and
// the lower where g < 0; on each piece the objective is convex, so its minimum
// is among the interval's ends, the tangent point and the stationary points
// logit((1 +- sqrt(1 - 4 rho/g)) / 2) of the piece where x = sigma(xB)
// (eq:with_sig_subp).  Ties go to the larger xB.  All arithmetic is FP64.
#include "ld_device.h"

namespace ld {

__device__ __forceinline__ double sgm(double x) { return 1.0 / (1.0 + exp(-x)); }
__device__ __forceinline__ double dsgm(double x) {
  const double s = sgm(x);
  return s * (1.0 - s);
}

// halvings of the bracket (width <= u - l <= 2^5 in practice): far below FP32 spacing
constexpr int kHullBisect = 44;

__global__ __launch_bounds__(256) void sigmoid_hull_kernel(long long n, const float* __restrict__ lo,
                                                           const float* __restrict__ hi, float* __restrict__ t_up,
                                                           float* __restrict__ t_lo) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double l = lo[i], u = hi[i];
    const double sl = sgm(l), su = sgm(u);
    const double chord = u > l ? (su - sl) / (u - l) : dsgm(l);
    double tu = u, tl = l;
    if (l >= 0.0) {
      tu = l;
    } else if (dsgm(u) < chord) {
      // F(t) = sigma'(t)(t - l) - (sigma(t) - sigma(l)): >= 0 at 0, < 0 at u
      double a = 0.0, b = u;
      for (int it = 0; it < kHullBisect; ++it) {
        const double m = 0.5 * (a + b);
        const double sm = sgm(m);
        if (sm * (1.0 - sm) * (m - l) - (sm - sl) >= 0.0)
          a = m;
        else
          b = m;
      }
      tu = 0.5 * (a + b);
    }
    if (u <= 0.0) {
      tl = u;
    } else if (dsgm(l) < chord) {
      // G(t) = sigma'(t)(u - t) - (sigma(u) - sigma(t)): >= 0 at 0, < 0 at l
      double a = l, b = 0.0;
      for (int it = 0; it < kHullBisect; ++it) {
        const double m = 0.5 * (a + b);
        const double sm = sgm(m);
        if (sm * (1.0 - sm) * (u - m) - (su - sm) >= 0.0)
          b = m;
        else
          a = m;
      }
      tl = 0.5 * (a + b);
    }
    t_up[i] = (float)tu;
    t_lo[i] = (float)tl;
  }
}

// The envelope x takes (upper for g > 0, lower otherwise) as a line on its linear
// piece and sigma on the other: the line through (x0, s0) with slope k holds for
// x <= t (upper) or x >= t (lower).
struct SigEnv {
  bool up;
  double t, x0, s0, k;
  __device__ double at(double x) const {
    const bool on_line = up ? x <= t : x >= t;
    return on_line ? s0 + k * (x - x0) : sgm(x);
  }
};

__global__ __launch_bounds__(256) void sigmoid_inner_min_kernel(long long n, const float* __restrict__ rho_,
                                                                const float* __restrict__ g_,
                                                                const float* __restrict__ lo,
                                                                const float* __restrict__ hi,
                                                                const float* __restrict__ t_up,
                                                                const float* __restrict__ t_lo,
                                                                float* __restrict__ xb_out, float* __restrict__ x_out,
                                                                double* __restrict__ val_out) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const double rho = rho_[i], g = g_[i], l = lo[i], u = hi[i];
    SigEnv E;
    E.up = g > 0.0;
    E.t = E.up ? (double)t_up[i] : (double)t_lo[i];
    // the line: from (l, sigma(l)) to (t, sigma(t)) above, from (t, sigma(t)) to (u, sigma(u)) below
    const double st = sgm(E.t);
    if (E.up) {
      const double sl = sgm(l);
      E.x0 = l;
      E.s0 = sl;
      E.k = E.t > l ? (st - sl) / (E.t - l) : sl * (1.0 - sl);
    } else {
      const double su = sgm(u);
      E.x0 = E.t;
      E.s0 = st;
      E.k = u > E.t ? (su - st) / (u - E.t) : su * (1.0 - su);
    }
    // candidates and their envelope values (a logit root r has sigma(r) = p)
    double cx[5], cs[5];
    int nc = 0;
    cx[nc] = l;
    cs[nc++] = E.at(l);
    cx[nc] = u;
    cs[nc++] = E.at(u);
    cx[nc] = E.t;
    cs[nc++] = E.at(E.t);
    if (g != 0.0) {
      const double disc = 1.0 - 4.0 * (rho / g);
      if (disc >= 0.0) {
        const double sq = sqrt(disc);
        for (int s = 0; s < 2; ++s) {
          const double p = 0.5 * (1.0 + (s == 0 ? sq : -sq));
          if (!(p > 0.0 && p < 1.0)) continue;
          const double r = log(p / (1.0 - p));
          const bool on_curve = E.up ? r >= E.t : r <= E.t;
          if (on_curve && r >= l && r <= u) {
            cx[nc] = r;
            cs[nc++] = p;
          }
        }
      }
    }
    double bx = cx[0], bs = cs[0], bv = rho * cx[0] - g * cs[0];
    for (int c = 1; c < nc; ++c) {
      const double v = rho * cx[c] - g * cs[c];
      if (v < bv || (v == bv && cx[c] > bx)) {
        bv = v;
        bx = cx[c];
        bs = cs[c];
      }
    }
    xb_out[i] = (float)bx;
    x_out[i] = (float)(g == 0.0 ? sgm(bx) : bs);
    val_out[i] = bv;
  }
}

namespace {
unsigned grid_sig(long long n) {
  const long long g = (n + 255) / 256;
  return (unsigned)(g < 8192 ? (g > 0 ? g : 1) : 8192);
}
}  // namespace

hipError_t launch_sigmoid_hull(long long n, const float* l, const float* u, float* t_up, float* t_lo, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(sigmoid_hull_kernel, dim3(grid_sig(n)), dim3(256), 0, s, n, l, u, t_up, t_lo);
  return hipGetLastError();
}

hipError_t launch_sigmoid_inner_min(long long n, const float* rho, const float* g, const float* l, const float* u,
                                    const float* t_up, const float* t_lo, float* xb, float* x, double* val,
                                    hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(sigmoid_inner_min_kernel, dim3(grid_sig(n)), dim3(256), 0, s, n, rho, g, l, u, t_up, t_lo, xb, x,
                     val);
  return hipGetLastError();
}

}  // namespace ld
