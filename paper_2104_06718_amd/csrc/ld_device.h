// Device helpers shared by the kernel translation units: BF16 conversion, the
// closed-form inner minimisation, the CROWN dual assignment and the MFMA
// fragment conventions.
#pragma once
#include "ld_internal.h"

namespace ld {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ bf16_t f2bf(float f) {
  // round to nearest even (the hardware conversion; inputs are finite)
  return __builtin_bit_cast(bf16_t, (__bf16)f);
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

// CROWN dual of one neuron from g = (W^T rho_next)[i] (eq:salman-assignment with
// the slopes of eq:slopes-biases: chord upper slope, lower slope 1[u >= -l]);
// with wk, the WK slopes (the chord as both the upper and the lower slope, Sec. 4.1).
__device__ __forceinline__ float crown_dual(float g, float l, float u, bool wk = false) {
  if (l >= 0.f) return g;
  if (u <= 0.f) return 0.f;
  if (g > 0.f || wk) return (u / (u - l)) * g;
  return (u >= -l) ? g : 0.f;
}

// ---------------------------------------------------------------------------
// MFMA fragments.  FP32 (v_mfma_f32_16x16x4f32): for a K step of 16, lane l
// (r = l & 15, g = l >> 4) holds A[r][k0+4g+j] and B[k0+4g+j][r], j = 0..3, and
// issues one MFMA per j; the 4 MFMAs sum k0..k0+15 once each (the k order inside
// the step is permuted so both operands are contiguous).  BF16
// (v_mfma_f32_16x16x32_bf16): lane holds A[r][k0+8g..+7], B[k0+8g..+7][r].
// Output: lane holds C[4g+q][r], q = 0..3.
// ---------------------------------------------------------------------------
template <bool MMA_BF16>
struct Mma;
template <>
struct Mma<false> {
  static constexpr int KS = 16, VPL = 4;
  typedef float4 BFrag;
  typedef f32x4 AFrag;  // A operand of one lane for one K step, in operand order
  __device__ static BFrag loadB(const GemmGeom& G, size_t off) { return *reinterpret_cast<const float4*>(G.Bf + off); }
  __device__ static void mma(const float (&a)[4], const BFrag& b, f32x4& c) {
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b.x, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1], b.y, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[2], b.z, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[3], b.w, c, 0, 0, 0);
  }
  __device__ static void mma_frag(const AFrag& a, const BFrag& b, f32x4& c) {
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[0], b.x, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[1], b.y, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[2], b.z, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(a[3], b.w, c, 0, 0, 0);
  }
  // weights as the row operand, activations as the column operand
  __device__ static void mma_wx(const BFrag& w, const float (&x)[4], f32x4& c) {
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(w.x, x[0], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(w.y, x[1], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(w.z, x[2], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x4f32(w.w, x[3], c, 0, 0, 0);
  }
};
template <>
struct Mma<true> {
  static constexpr int KS = 32, VPL = 8;
  typedef bf16x8 BFrag;
  typedef bf16x8 AFrag;
  __device__ static BFrag loadB(const GemmGeom& G, size_t off) { return *reinterpret_cast<const bf16x8*>(G.Bh + off); }
  __device__ static void mma(const float (&a)[8], const BFrag& b, f32x4& c) {
    bf16x8 av;
#pragma unroll
    for (int j = 0; j < 8; ++j) av[j] = (__bf16)a[j];
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b, c, 0, 0, 0);
  }
  __device__ static void mma_frag(const AFrag& a, const BFrag& b, f32x4& c) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  // Compensated product: a and the weights each as a BF16 head plus a BF16
  // remainder (w = bh + bl), c += a_l*bh + a_h*bl + a_h*bh (the a_l*bl term, of
  // relative size 2^-16, is dropped); FP32 accumulation, small terms first.
  __device__ static void split(const float (&a)[8], bf16x8& ah, bf16x8& al) {
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      ah[j] = (__bf16)a[j];
      al[j] = (__bf16)(a[j] - (float)ah[j]);
    }
  }
  // the same three terms with the operand already split (head ah, remainder al)
  __device__ static void mma3_frag(const AFrag& ah, const AFrag& al, const BFrag& bh, const BFrag& bl, f32x4& c) {
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
  }
  __device__ static void mma3(const float (&a)[8], const BFrag& bh, const BFrag& bl, f32x4& c) {
    bf16x8 ah, al;
    split(a, ah, al);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
  }
  __device__ static void mma3_wx(const BFrag& wh, const BFrag& wl, const float (&x)[8], f32x4& c) {
    bf16x8 xh, xl;
    split(x, xh, xl);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh, xl, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wl, xh, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wh, xh, c, 0, 0, 0);
  }
  __device__ static void mma_wx(const BFrag& w, const float (&x)[8], f32x4& c) {
    bf16x8 xv;
#pragma unroll
    for (int j = 0; j < 8; ++j) xv[j] = (__bf16)x[j];
    c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, xv, c, 0, 0, 0);
  }
};

}  // namespace ld
