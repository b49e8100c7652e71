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
#include "ld_device.h"

#include <type_traits>

namespace ld {

constexpr int kMaxClasses = 9;

// f(std::integral_constant<int, i>) for i = 0..N-1, unrolled at compile time (arrays
// indexed by i stay in registers)
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (N > 0) {
    static_for<N - 1>(f);
    f(std::integral_constant<int, N - 1>{});
  }
}
struct GemmPack {
  int n;
  GemmGeom g[kMaxClasses];
};

// One thread per launch advances the step counter and writes the scalars of
// this iteration's Adam step: step size with linear decay (Sec. 7.2) and the
// bias corrections 1/(1-beta^t).
__device__ __forceinline__ void adam_tick(const EpiArgs& E) {
  if (E.t_dev == nullptr || blockIdx.x != 0 || blockIdx.y != 0 || blockIdx.z != 0 || threadIdx.x != 0) return;
  const int t = *E.t_dev + 1;
  *E.t_dev = t;
  const double lr = E.total > 1 ? E.lr0 + (E.lr_end - E.lr0) * (double)(t - 1) / (double)(E.total - 1) : E.lr0;
  E.adam_w[0] = (float)lr;
  E.adam_w[1] = (float)(1.0 / (1.0 - pow(E.beta1, (double)t)));
  E.adam_w[2] = (float)(1.0 / (1.0 - pow(E.beta2, (double)t)));
  E.adam_w[3] = (float)E.eps;
  E.adam_w[4] = (float)E.beta1;
  E.adam_w[5] = (float)E.beta2;
}

// ---------------------------------------------------------------------------
// Batched epilogue: four accumulated values of one output column, at indices
// i0 + q*st (q < nv).  All loads of the four elements are issued before any
// arithmetic; with VEC the four elements are contiguous and 16-byte aligned.
// ---------------------------------------------------------------------------
template <bool VEC>
__device__ __forceinline__ void ld4(const float* __restrict__ p, size_t i0, size_t st, int nv, float (&o)[4]) {
  if (VEC) {
    const float4 v = *reinterpret_cast<const float4*>(p + i0);
    o[0] = v.x;
    o[1] = v.y;
    o[2] = v.z;
    o[3] = v.w;
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q) o[q] = q < nv ? p[i0 + q * st] : 0.f;
  }
}
template <bool VEC>
__device__ __forceinline__ void st4(float* __restrict__ p, size_t i0, size_t st, int nv, const float (&o)[4]) {
  if (VEC) {
    *reinterpret_cast<float4*>(p + i0) = make_float4(o[0], o[1], o[2], o[3]);
  } else {
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (q < nv) p[i0 + q * st] = o[q];
  }
}
template <bool VEC>
__device__ __forceinline__ void st4_xs(const EpiArgs& E, size_t i0, size_t st, int nv, const float (&o)[4]) {
  if (E.xs_bf16) {
    bf16_t* p = (bf16_t*)E.xs;
    if (VEC) {
      // four contiguous BF16 values, 8-byte aligned: one store
      uint2 w;
      w.x = (uint32_t)f2bf(o[0]) | ((uint32_t)f2bf(o[1]) << 16);
      w.y = (uint32_t)f2bf(o[2]) | ((uint32_t)f2bf(o[3]) << 16);
      *reinterpret_cast<uint2*>(p + i0) = w;
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (q < nv) p[i0 + q * st] = f2bf(o[q]);
    }
  } else {
    st4<VEC>((float*)E.xs, i0, st, nv, o);
  }
}

// Operands an epilogue reads from device memory, four elements per array (the
// loads are issued before any arithmetic of the epilogue).
struct EpiIn {
  f32x4 a0, a1, a2, a3, a4, a5;
};

template <bool VEC>
__device__ __forceinline__ f32x4 ld4v(const float* __restrict__ p, size_t i0, size_t st, int nv) {
  float t[4];
  ld4<VEC>(p, i0, st, nv, t);
  return f32x4{t[0], t[1], t[2], t[3]};
}

// Index of element i0 (subdomain i0 / lohi_len) in the bound arrays lo/hi, whose
// rows may be shared by row_div consecutive subdomains.
__device__ __forceinline__ size_t lohi_index(const EpiArgs& E, size_t i0) {
  if (E.row_div <= 1) return i0;
  const size_t n = (size_t)E.lohi_len;
  const size_t b = i0 / n;
  return (b / (size_t)E.row_div) * n + (i0 - b * n);
}

// EK: the epilogue kind of a launch fixed at compile time (-1: read from E.kind);
// with kEkNoVal the per-neuron values are not written (E.want_val == 0).
constexpr int kEkKind = 63, kEkNoVal = 64;

// NA: arrays an epilogue of this launch may read (kinds that read more are not
// launched with NA < 6; the members past NA stay zero). SHIFT: the caller's
// elements lie in one subdomain, whose bound rows sit lohi_shift elements from i0.
template <bool VEC, int NA = 6, bool SHIFT = false, int EK = -1>
__device__ __forceinline__ void epi_load(const EpiArgs& E, size_t i0, size_t st, int nv, EpiIn& in,
                                         ptrdiff_t lohi_shift = 0) {
  const auto lohi_at = [&](size_t i) { return SHIFT ? (size_t)((ptrdiff_t)i + lohi_shift) : lohi_index(E, i); };
  switch (EK >= 0 ? (EK & kEkKind) : E.kind) {
    case EPI_P0:
    case EPI_CROWN:
    case EPI_WK:
    case EPI_RELU_FWD: {
      const size_t il = lohi_at(i0);
      in.a0 = ld4v<VEC>(E.lo, il, st, nv);
      in.a1 = ld4v<VEC>(E.hi, il, st, nv);
    } break;
    case EPI_INNER_MIN: {
      const size_t il = lohi_at(i0);
      in.a0 = ld4v<VEC>(E.rho, i0, st, nv);
      in.a1 = ld4v<VEC>(E.lo, il, st, nv);
      in.a2 = ld4v<VEC>(E.hi, il, st, nv);
    } break;
    case EPI_ADAM:
      if (NA >= 4) {
        in.a0 = ld4v<VEC>(E.rho_w, i0, st, nv);
        in.a1 = ld4v<VEC>(E.m, i0, st, nv);
        in.a2 = ld4v<VEC>(E.v, i0, st, nv);
        in.a3 = ld4v<VEC>(E.xb_in, i0, st, nv);
      }
      break;
    case EPI_ADAM_LAST:
      if (NA >= 6) {
        const size_t il = lohi_at(i0);
        in.a0 = ld4v<VEC>(E.rho_w, i0, st, nv);
        in.a1 = ld4v<VEC>(E.m, i0, st, nv);
        in.a2 = ld4v<VEC>(E.v, i0, st, nv);
        in.a3 = ld4v<VEC>(E.gc, i0, st, nv);
        in.a4 = ld4v<VEC>(E.lo, il, st, nv);
        in.a5 = ld4v<VEC>(E.hi, il, st, nv);
      }
      break;
    case EPI_SUPERGRAD:
      in.a0 = ld4v<VEC>(E.xb_in, i0, st, nv);
      break;
    default:
      break;
  }
}

template <bool VEC, int EK = -1>
__device__ __forceinline__ void epi_finish(const EpiArgs& E, size_t i0, size_t st, int nv, int b0, int bstep, int col,
                                           int cstep, const float (&acc)[4], const EpiIn& in) {
  const int kind = EK >= 0 ? (EK & kEkKind) : E.kind;
  // the values of P0 and P_k are skipped in the ascent (EK carries kEkNoVal)
  const bool want_val = EK >= 0 && (EK & kEkNoVal) ? false : E.want_val != 0;
  switch (kind) {
    case EPI_STORE: {
      float o[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) o[q] = E.scale * acc[q];
      st4<VEC>(E.out_f, i0, st, nv, o);
    } break;
    case EPI_P0: {
      float x[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) x[q] = acc[q] >= 0.f ? in.a1[q] : in.a0[q];
      st4_xs<VEC>(E, i0, st, nv, x);
      if (want_val)
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (VEC || q < nv) E.val[i0 + q * st] = -(double)acc[q] * (double)x[q];
    } break;
    case EPI_INNER_MIN: {
      float xb[4], x[4];
      if (want_val) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          double xbd, xd, val;
          inner_min<double>(in.a0[q], acc[q], in.a1[q], in.a2[q], (double)E.tau, xbd, xd, val);
          xb[q] = (float)xbd;
          x[q] = (float)xd;
          if (VEC || q < nv) {
            const double bias = (double)E.bias[(col + q * cstep) / E.bias_div];
            E.val[i0 + q * st] = val - (double)in.a0[q] * bias;
          }
        }
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          float val;
          inner_min<float>(in.a0[q], acc[q], in.a1[q], in.a2[q], E.tau, xb[q], x[q], val);
        }
      }
      st4_xs<VEC>(E, i0, st, nv, x);
      st4<VEC>(E.xb, i0, st, nv, xb);
    } break;
    case EPI_ADAM:
    case EPI_ADAM_LAST: {
      float xb[4], rho[4], m[4], v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        rho[q] = in.a0[q];
        m[q] = in.a1[q];
        v[q] = in.a2[q];
      }
      if (kind == EPI_ADAM_LAST) {
        // inner minimisation of the last hidden layer from its constant coefficient
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          float x, val;
          inner_min<float>(rho[q], in.a3[q], in.a4[q], in.a5[q], E.tau, xb[q], x, val);
        }
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) xb[q] = in.a3[q];
      }
      const float lr = E.adam[0], ibc1 = E.adam[1], ibc2 = E.adam[2], eps = E.adam[3];
      const float b1 = E.adam[4], b2 = E.adam[5];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float bias = (VEC || q < nv) ? E.bias[col + q * cstep] : 0.f;
        const float s = xb[q] - (acc[q] + bias);
        m[q] = b1 * m[q] + (1.f - b1) * s;
        v[q] = b2 * v[q] + (1.f - b2) * (s * s);
        // hardware square root and reciprocal (1 ulp): the step is a sign-like
        // quantity of size lr, so their rounding is far below the tie band
        rho[q] = rho[q] + lr * (m[q] * ibc1) * __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(v[q] * ibc2) + eps);
      }
      st4<VEC>(E.m, i0, st, nv, m);
      st4<VEC>(E.v, i0, st, nv, v);
      st4<VEC>(E.rho_w, i0, st, nv, rho);
    } break;
    case EPI_SUPERGRAD: {
      float o[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) o[q] = in.a0[q] - (acc[q] + ((VEC || q < nv) ? E.bias[col + q * cstep] : 0.f));
      st4<VEC>(E.out_f, i0, st, nv, o);
    } break;
    case EPI_CROWN:
    case EPI_WK: {
      float o[4];
      const bool wk = E.kind == EPI_WK;
#pragma unroll
      for (int q = 0; q < 4; ++q) o[q] = crown_dual(acc[q], in.a0[q], in.a1[q], wk);
      st4<VEC>(E.out_f, i0, st, nv, o);
    } break;
    case EPI_RELU_FWD: {
      float o[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float y = acc[q] + ((VEC || q < nv) ? E.bias[col + q * cstep] : 0.f);
        if ((VEC || q < nv) && !(y >= in.a0[q] && y <= in.a1[q])) E.flag[b0 + q * bstep] = 0;
        o[q] = fmaxf(y, 0.f);
      }
      st4<VEC>(E.out_f, i0, st, nv, o);
    } break;
    case EPI_BIAS_STORE: {
      float o[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) o[q] = acc[q] + ((VEC || q < nv) ? E.bias[col + q * cstep] : 0.f);
      st4<VEC>(E.out_f, i0, st, nv, o);
    } break;
    default:
      break;
  }
}

template <bool VEC, int EK = -1>
__device__ __forceinline__ void epilogue4(const EpiArgs& E, size_t i0, size_t st, int nv, int b0, int bstep, int col,
                                          int cstep, const float (&acc)[4]) {
  EpiIn in{};
  epi_load<VEC, 6, false, EK>(E, i0, st, nv, in);
  epi_finish<VEC, EK>(E, i0, st, nv, b0, bstep, col, cstep, acc, in);
}

// ---------------------------------------------------------------------------
// Convolution contraction, all stride classes; `parts` blocks per subdomain, block
// `part` owning the band of destination rows [part*H/parts, (part+1)*H/parts) of
// every output channel (a band of a class's rows yq lands on a band of destination
// rows, so the classes of one band are whole tiles of their grids).
//  1. staging, one barrier: the block zeroes the padding border of a channel-last
//     LDS image of the subdomain's source map and fills its interior (all global loads of
//     a thread are issued before its LDS writes); the packed weights of every
//     class and the gather offsets go to LDS as well;
//  2. waves compute 16-pixel x 16-column MFMA tiles of every class over the band,
//     A gathered from the image, B read from the staged weights, and write the
//     results into an LDS copy of the band of the destination map (classes land on
//     their pixels);
//  3. all threads stream the epilogue over the band in memory order (a contiguous
//     run per channel), 16 bytes per access.
// ---------------------------------------------------------------------------
constexpr int kConvWaves = 8;
constexpr int kConvThreads = 64 * kConvWaves;

// e / d for 0 <= e < 2^22 with inv ~ 1/d: float estimate, then one correction
__device__ __forceinline__ int fdiv(int e, int d, float inv) {
  int q = (int)((float)e * inv);
  const int r = e - q * d;
  if (r < 0)
    --q;
  else if (r >= d)
    ++q;
  return q;
}


// MM: operands of the product: 0 FP32, 1 BF16, 2 compensated BF16 (FP32 source)
// The LDS image is channel-last ([LH][LW][CP]) and k runs (tap, channel) with the
// channels padded to a multiple of 4, so every 4 consecutive k of a lane are one
// 16-byte LDS read.
template <int MM, bool SRC_BF16, int TN, int EK = -1>
__global__ __launch_bounds__(kConvThreads) void conv_plane_kernel(GemmPack P, const GemmGeom* __restrict__ geo_dev,
                                                         const void* __restrict__ src_v, EpiArgs E,
                                                         int img_floats, int dst_hw4, int kp_max, int n_eff,
                                                         int bstride, int parts, int out_floats) {
  constexpr bool MMA_BF16 = MM != 0;
  using M = Mma<MMA_BF16>;
  typedef typename M::BFrag BFrag;
  typedef typename std::conditional<MMA_BF16, bf16_t, float>::type WT;
  constexpr int KS = M::KS, VPL = M::VPL, EPV = 16 / (int)sizeof(WT);
  extern __shared__ float lds[];
  const GemmGeom& G0 = P.g[0];
  // the scalars of the staging, loaded together ahead of everything else (the pin
  // emits no instruction)
  asm volatile("" ::"s"(G0.src_n), "s"(G0.src_H), "s"(G0.src_W), "s"(G0.CP), "s"(G0.LW), "s"(G0.LH),
               "s"(G0.pad_t), "s"(G0.pad_l), "s"(G0.dst_HW), "s"(G0.dst_W), "s"(P.n), "s"(src_v));
  const int b = blockIdx.x / parts, part = blockIdx.x - b * parts;
  const int tid = threadIdx.x;
  // destination rows of this block and their run length per channel
  const int dst_H = G0.dst_HW / G0.dst_W;
  const int R0 = part * dst_H / parts, R1 = (part + 1) * dst_H / parts;
  const int band = (R1 - R0) * G0.dst_W;
  // LDS row stride of a channel of the band: 4 floats of padding spread the 16
  // channels an MFMA tile writes at once over distinct banks
  const int bandp = band + 4;
  const int wave = tid >> 6, lane = tid & 63, r = lane & 15, g = lane >> 4;
  const int H = G0.src_H, W = G0.src_W, HW = H * W;
  const int C = G0.src_n / HW;
  // the source map, channel-last [LH][LW][CP]: FP32 (MM == 0), or BF16 heads in the
  // first half of the same area (MM == 1) and BF16 remainders in its second half
  // (MM == 2), split once here instead of at every use in the products
  float* img = lds;
  bf16_t* imgh = reinterpret_cast<bf16_t*>(img);
  bf16_t* imgl = imgh + img_floats;
  const int CP = G0.CP;
  const int Cq = (C + 3) & ~3;  // channels of a pixel that k reads (the ones past C are zero)
  float* outp = img + img_floats;                          // [channels][band]
  int* kofs = reinterpret_cast<int*>(outp + out_floats);   // [n classes][kp_max]
  // per class {first pixel, pixel end, MFMA items, items of the classes before}, 16-byte aligned
  int* ctab = reinterpret_cast<int*>(lds + ((img_floats + out_floats + P.n * kp_max + 3) & ~3));
  WT* wB = reinterpret_cast<WT*>(ctab + 4 * P.n);  // [n classes][n_eff][bstride], 16-byte aligned
  WT* wBl = wB + (size_t)P.n * n_eff * bstride;  // MM == 2: the BF16 remainders, same layout
  auto put = [&](int idx, float v) __attribute__((always_inline)) {
    if constexpr (MM == 0) {
      img[idx] = v;
    } else {
      const __bf16 h = (__bf16)v;
      imgh[idx] = __builtin_bit_cast(bf16_t, h);
      if constexpr (MM == 2) imgl[idx] = __builtin_bit_cast(bf16_t, (__bf16)(v - (float)h));
    }
  };

  // 1. staging.  A thread's first round of global loads (up to U float4 of the
  //    source map, its gather offset and weight vectors of every class) is issued
  //    before any LDS write, so the block waits for one memory latency; larger maps
  //    and weight sets continue in further rounds.
  const size_t sbase = (size_t)b * G0.src_n;
  const float inv_w = 1.0f / (float)W, inv_h = 1.0f / (float)H;
  const bool vec_img = (W & 3) == 0;
  const int n4 = G0.src_n >> 2;
  constexpr int U = 4;
  auto load_img4 = [&](int i, float (&v)[4]) __attribute__((always_inline)) {
    if (SRC_BF16) {
      const uint2 raw = *reinterpret_cast<const uint2*>((const bf16_t*)src_v + sbase + 4 * (size_t)i);
      v[0] = bf2f((bf16_t)(raw.x & 0xffffu));
      v[1] = bf2f((bf16_t)(raw.x >> 16));
      v[2] = bf2f((bf16_t)(raw.y & 0xffffu));
      v[3] = bf2f((bf16_t)(raw.y >> 16));
    } else {
      const float4 f = *reinterpret_cast<const float4*>((const float*)src_v + sbase + 4 * (size_t)i);
      v[0] = f.x;
      v[1] = f.y;
      v[2] = f.z;
      v[3] = f.w;
    }
  };
  auto store_img4 = [&](int i, const float (&v)[4]) __attribute__((always_inline)) {
    const int e = 4 * i;
    const int row = fdiv(e, W, inv_w);  // c*H + y
    const int x = e - row * W;
    const int c = fdiv(row, H, inv_h);
    const int y = row - c * H;
    const int d = ((y + G0.pad_t) * G0.LW + x + G0.pad_l) * CP + c;
#pragma unroll
    for (int q = 0; q < 4; ++q) put(d + q * CP, v[q]);
    if (c == C - 1)  // the padding channels of these pixels
      for (int cc = C; cc < Cq; ++cc)
#pragma unroll
        for (int q = 0; q < 4; ++q) put(d + q * CP + cc - c, 0.f);
  };
  // gather offsets and weight vectors of a group of up to kStageClasses classes;
  // the group's scalars (pointers, lengths) are read first, unconditionally, so
  // their loads from the kernel arguments are issued together
  constexpr int kStageClasses = 4;
  int kv[kStageClasses], kp[kStageClasses];
  const int* kt[kStageClasses];
  const u32x4* wsrc[kStageClasses];
  const u32x4* wlsrc[kStageClasses];
  u32x4 wh[kStageClasses], wl[kStageClasses];
  auto class_scalars = [&](int c0) __attribute__((always_inline)) {
    static_for<kStageClasses>([&](auto ci) __attribute__((always_inline)) {
      constexpr int i = decltype(ci)::value;
      const GemmGeom& G = P.g[min(c0 + i, kMaxClasses - 1)];  // in bounds; unused past P.n
      kp[i] = G.Kp;
      kt[i] = G.ktab_cl;
      wsrc[i] = reinterpret_cast<const u32x4*>(MMA_BF16 ? (const void*)G.Bh : (const void*)G.Bf);
      wlsrc[i] = reinterpret_cast<const u32x4*>(G.Bhl);
      // keep the scalar loads here, ahead of the branches below (no instruction)
      asm volatile("" ::"s"(kp[i]), "s"(kt[i]), "s"(wsrc[i]), "s"(wlsrc[i]));
    });
  };
  auto load_classes = [&](int c0) __attribute__((always_inline)) {
    static_for<kStageClasses>([&](auto ci) __attribute__((always_inline)) {
      constexpr int i = decltype(ci)::value;
      if (c0 + i < P.n) {
        if (tid < kp[i]) kv[i] = kt[i][tid];
        if (tid < n_eff * (kp[i] / EPV)) {
          wh[i] = wsrc[i][tid];
          if (MM == 2) wl[i] = wlsrc[i][tid];
        }
      }
    });
  };
  auto store_classes = [&](int c0) __attribute__((always_inline)) {
    static_for<kStageClasses>([&](auto ci) __attribute__((always_inline)) {
      constexpr int i = decltype(ci)::value;
      const int c = c0 + i;
      if (c < P.n) {
        if (tid < kp[i]) kofs[c * kp_max + tid] = kv[i];
        const int vr = kp[i] / EPV;
        if (tid < n_eff * vr) {
          const int row = tid / vr, v = tid - row * vr;
          const size_t o = ((size_t)c * n_eff + row) * bstride + v * EPV;
          *reinterpret_cast<u32x4*>(wB + o) = wh[i];
          if (MM == 2) *reinterpret_cast<u32x4*>(wBl + o) = wl[i];
        }
      }
    });
  };
  // (a) the first round of loads
  class_scalars(0);
  float v0[U][4];
  if (vec_img) {
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (tid + u * kConvThreads < n4) load_img4(tid + u * kConvThreads, v0[u]);
  }
  load_classes(0);
  adam_tick(E);
  // (b) while the loads are in flight: the zero border of the image (disjoint from
  //     the interior: border pixels, all Cq channels; the CP - Cq floats past them are
  //     never read), and the table of the MFMA items of every class (one thread)
  {
    const float inv_lw = 1.0f / (float)G0.LW;
    const int c4 = Cq >> 2;
    for (int e = tid; e < G0.LH * G0.LW * c4; e += kConvThreads) {
      const int pix = e / c4, q = e - pix * c4;
      const int yy = fdiv(pix, G0.LW, inv_lw), xx = pix - yy * G0.LW;
      if (yy < G0.pad_t || yy >= G0.pad_t + H || xx < G0.pad_l || xx >= G0.pad_l + W) {
        if constexpr (MM == 0) {
          *reinterpret_cast<float4*>(img + pix * CP + 4 * q) = make_float4(0.f, 0.f, 0.f, 0.f);
        } else {
          *reinterpret_cast<uint2*>(imgh + pix * CP + 4 * q) = make_uint2(0u, 0u);
          if constexpr (MM == 2) *reinterpret_cast<uint2*>(imgl + pix * CP + 4 * q) = make_uint2(0u, 0u);
        }
      }
    }
  }
  if (tid == 0) {
    int before = 0;
    for (int cl = 0; cl < P.n; ++cl) {
      const GemmGeom& Gc = P.g[cl];
      // the class rows yq whose destination rows yq*oy_mul + oy_off fall in [R0, R1)
      const int yq_lo = R0 - Gc.oy_off <= 0 ? 0 : (R0 - Gc.oy_off + Gc.oy_mul - 1) / Gc.oy_mul;
      const int yq_hi = min(Gc.HWq / Gc.Wq, R1 - Gc.oy_off <= 0 ? 0 : (R1 - Gc.oy_off + Gc.oy_mul - 1) / Gc.oy_mul);
      const int p_lo = yq_lo * Gc.Wq, p_hi = max(p_lo, yq_hi * Gc.Wq);
      const int ntiles = (p_hi - p_lo + 15) >> 4;
      const int nct = (Gc.N + 16 * TN - 1) / (16 * TN);
      // items: (pair of tiles, column chunk)
      const int total = ((ntiles + 1) >> 1) * nct;
      *reinterpret_cast<int4*>(ctab + 4 * cl) = make_int4(p_lo, p_hi, total, before);
      before += total;
    }
  }
  // (c) the LDS writes of the first round
  if (vec_img) {
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (tid + u * kConvThreads < n4) store_img4(tid + u * kConvThreads, v0[u]);
  }
  store_classes(0);
  // (d) further rounds
  for (int c0 = kStageClasses; c0 < P.n; c0 += kStageClasses) {
    class_scalars(c0);
    load_classes(c0);
    store_classes(c0);
  }
  if (vec_img) {
    for (int i0 = tid + U * kConvThreads; i0 < n4; i0 += U * kConvThreads) {
      float v[U][4];
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (i0 + u * kConvThreads < n4) load_img4(i0 + u * kConvThreads, v[u]);
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (i0 + u * kConvThreads < n4) store_img4(i0 + u * kConvThreads, v[u]);
    }
  } else {
    for (int e = tid; e < G0.src_n; e += kConvThreads) {
      const float v = SRC_BF16 ? bf2f(((const bf16_t*)src_v)[sbase + e]) : ((const float*)src_v)[sbase + e];
      const int row = fdiv(e, W, inv_w);
      const int x = e - row * W;
      const int c = fdiv(row, H, inv_h);
      const int y = row - c * H;
      const int d = ((y + G0.pad_t) * G0.LW + x + G0.pad_l) * CP;
      put(d + c, v);
      if (c == C - 1)
        for (int cc = C; cc < Cq; ++cc) put(d + cc, 0.f);
    }
  }
  for (int c = 0; c < P.n; ++c) {
    const GemmGeom& G = P.g[c];
    for (int k = tid + kConvThreads; k < G.Kp; k += kConvThreads) kofs[c * kp_max + k] = G.ktab_cl[k];
    const int vr = G.Kp / EPV;
    const float inv_vr = 1.0f / (float)vr;
    const uint4* srcw = reinterpret_cast<const uint4*>(MMA_BF16 ? (const void*)G.Bh : (const void*)G.Bf);
    const uint4* srcl = reinterpret_cast<const uint4*>(G.Bhl);
    for (int e = tid + kConvThreads; e < n_eff * vr; e += kConvThreads) {
      const int row = fdiv(e, vr, inv_vr);
      const int v = e - row * vr;
      const size_t o = ((size_t)c * n_eff + row) * bstride + v * EPV;
      const uint4 w = srcw[(size_t)row * vr + v];
      if (MM == 2) {
        const uint4 wlo = srcl[(size_t)row * vr + v];
        *reinterpret_cast<uint4*>(wBl + o) = wlo;
      }
      *reinterpret_cast<uint4*>(wB + o) = w;
    }
  }
  __syncthreads();

  // the operands of the thread's first epilogue group, in flight during the products
  // (the epilogue reads and writes them only in that thread, after the products)
  const size_t base = (size_t)b * G0.dst_n + (size_t)R0 * G0.dst_W;
  const int nch = G0.dst_n / G0.dst_HW;
  const float inv_band = 1.0f / (float)band;
  EpiIn pre{};
  if (dst_hw4 && 4 * tid < nch * band) {
    const int col = fdiv(4 * tid, band, inv_band);
    const int j = 4 * tid - col * band;
    epi_load<true, 6, false, EK>(E, base + (size_t)col * G0.dst_HW + j, 1, 4, pre);
  }
  // 2. MFMA tiles of every class into the LDS destination map; items (pair of tiles,
  //    column chunk) are dealt to the waves continuing the rotation across classes,
  //    and a wave skips the classes that hold none of its items
  for (int cl = 0; cl < P.n; ++cl) {
    const int4 ct = *reinterpret_cast<const int4*>(ctab + 4 * cl);
    const int p_lo = __builtin_amdgcn_readfirstlane(ct.x), p_hi = __builtin_amdgcn_readfirstlane(ct.y);
    const int total = __builtin_amdgcn_readfirstlane(ct.z), tiles_before = __builtin_amdgcn_readfirstlane(ct.w);
    int first = (wave - tiles_before) % kConvWaves;
    if (first < 0) first += kConvWaves;
    if (first >= total) continue;
    // the class geometry from the kernel arguments (uniform: scalar loads)
    const GemmGeom& Gl = P.g[cl];
    struct {
      int HWq, Wq, iy_mul, iy_off, ix_mul, ix_off, pad_t, pad_l, LW, K, N, dst_HW, dst_W, oy_mul, oy_off, ox_mul, ox_off;
    } G;
    G.HWq = Gl.HWq;
    G.Wq = Gl.Wq;
    G.iy_mul = Gl.iy_mul;
    G.iy_off = Gl.iy_off;
    G.ix_mul = Gl.ix_mul;
    G.ix_off = Gl.ix_off;
    G.pad_t = Gl.pad_t;
    G.pad_l = Gl.pad_l;
    G.LW = Gl.LW;
    G.K = Gl.K;
    G.N = Gl.N;
    G.dst_HW = Gl.dst_HW;
    G.dst_W = Gl.dst_W;
    G.oy_mul = Gl.oy_mul;
    G.oy_off = Gl.oy_off;
    G.ox_mul = Gl.ox_mul;
    G.ox_off = Gl.ox_off;
    const int* ko = kofs + cl * kp_max;
    const WT* wc = wB + (size_t)cl * n_eff * bstride;
    const WT* wcl = wBl + (size_t)cl * n_eff * bstride;
    const float inv_wq = 1.0f / (float)G.Wq;
    const int nct = (G.N + 16 * TN - 1) / (16 * TN);
    const int j_band = R0 * G.dst_W;
    // a wave multiplies two 16-pixel tiles against each weight fragment it reads
    // (the second tile of an odd count is empty)
    for (int w = first; w < total; w += kConvWaves) {
      const int pair = w / nct;
      const int nc = (w - pair * nct) * 16 * TN;
      int lb[2];
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        const int p = min(p_lo + (2 * pair + m) * 16 + r, p_hi - 1);
        const int yq = fdiv(p, G.Wq, inv_wq);
        const int xq = p - yq * G.Wq;
        lb[m] = ((yq * G.iy_mul + G.iy_off + G.pad_t) * G.LW + xq * G.ix_mul + G.ix_off + G.pad_l) * CP;
      }
      f32x4 acc[2][TN];
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int t = 0; t < TN; ++t) acc[m][t] = f32x4{0.f, 0.f, 0.f, 0.f};
      for (int k0 = 0; k0 < G.K; k0 += KS) {
        const int kl = k0 + VPL * g;
        // each group of 4 consecutive k is 4 channels of one tap: 16-byte aligned
        // and contiguous (VPL = 8 may span two taps)
        int ofs[VPL / 4];
#pragma unroll
        for (int j = 0; j < VPL; j += 4) ofs[j / 4] = ko[kl + j];
        if constexpr (MM == 0) {
          float a[2][VPL];
#pragma unroll
          for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int j = 0; j < VPL; j += 4) {
              const float4 v = *reinterpret_cast<const float4*>(img + lb[m] + ofs[j / 4]);
              a[m][j] = v.x;
              a[m][j + 1] = v.y;
              a[m][j + 2] = v.z;
              a[m][j + 3] = v.w;
            }
#pragma unroll
          for (int t = 0; t < TN; ++t) {
            const size_t wo = (size_t)(nc + 16 * t + r) * bstride + kl;
            const BFrag bf = *reinterpret_cast<const BFrag*>(wc + wo);
#pragma unroll
            for (int m = 0; m < 2; ++m) M::mma(a[m], bf, acc[m][t]);
          }
        } else {
          // BF16 fragments straight from the split map: two runs of 4 channels
          bf16x8 ah[2], al[2];
#pragma unroll
          for (int m = 0; m < 2; ++m) {
            const uint2 h0 = *reinterpret_cast<const uint2*>(imgh + lb[m] + ofs[0]);
            const uint2 h1 = *reinterpret_cast<const uint2*>(imgh + lb[m] + ofs[1]);
            ah[m] = __builtin_bit_cast(bf16x8, u32x4{h0.x, h0.y, h1.x, h1.y});
            if constexpr (MM == 2) {
              const uint2 l0 = *reinterpret_cast<const uint2*>(imgl + lb[m] + ofs[0]);
              const uint2 l1 = *reinterpret_cast<const uint2*>(imgl + lb[m] + ofs[1]);
              al[m] = __builtin_bit_cast(bf16x8, u32x4{l0.x, l0.y, l1.x, l1.y});
            }
          }
#pragma unroll
          for (int t = 0; t < TN; ++t) {
            const size_t wo = (size_t)(nc + 16 * t + r) * bstride + kl;
            const BFrag bf = *reinterpret_cast<const BFrag*>(wc + wo);
            if constexpr (MM == 2) {
              const BFrag bfl = *reinterpret_cast<const BFrag*>(wcl + wo);
#pragma unroll
              for (int m = 0; m < 2; ++m) M::mma3_frag(ah[m], al[m], bf, bfl, acc[m][t]);
            } else {
#pragma unroll
              for (int m = 0; m < 2; ++m) M::mma_frag(ah[m], bf, acc[m][t]);
            }
          }
        }
      }
      // the lane's four rows of a tile are consecutive pixels of the class grid
#pragma unroll
      for (int m = 0; m < 2; ++m) {
        const int p0 = p_lo + (2 * pair + m) * 16 + 4 * g;
        int yy = fdiv(p0, G.Wq, inv_wq);
        int xx = p0 - yy * G.Wq;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          if (p0 + q < p_hi) {
            const int j0 = (yy * G.oy_mul + G.oy_off) * G.dst_W + xx * G.ox_mul + G.ox_off - j_band;
#pragma unroll
            for (int t = 0; t < TN; ++t) {
              const int col = nc + 16 * t + r;
              if (col < G.N) outp[col * bandp + j0] = acc[m][t][q];
            }
          }
          if (++xx == G.Wq) {
            xx = 0;
            ++yy;
          }
        }
      }
    }
  }
  __syncthreads();

  // 3. epilogue over the band of the destination map in memory order
  if (dst_hw4) {
    for (int e = 4 * tid; e < nch * band; e += 4 * kConvThreads) {
      const int col = fdiv(e, band, inv_band);  // channel (four consecutive neurons share it)
      const int j = e - col * band;
      const float4 o4 = *reinterpret_cast<const float4*>(outp + col * bandp + j);
      float v4[4] = {o4.x, o4.y, o4.z, o4.w};
      const size_t i0 = base + (size_t)col * G0.dst_HW + j;
      EpiIn in = pre;
      if (e != 4 * tid) epi_load<true, 6, false, EK>(E, i0, 1, 4, in);
      epi_finish<true, EK>(E, i0, 1, 4, b, 0, col, 0, v4, in);
    }
  } else {
    for (int e = tid; e < nch * band; e += kConvThreads) {
      const int col = fdiv(e, band, inv_band);
      const int j = e - col * band;
      float v4[4] = {outp[col * bandp + j], 0.f, 0.f, 0.f};
      epilogue4<false, EK>(E, base + (size_t)col * G0.dst_HW + j, 1, 1, b, 0, col, 0, v4);
    }
  }
}

// ---------------------------------------------------------------------------
// Fully-connected contraction, computed transposed: C[neuron][subdomain] =
// sum_k W[neuron][k] X[subdomain][k], with both operands loaded register-direct
// (packed weights as the row operand).  A wave owns 16*TN neurons x 16
// subdomains; a block is wm waves along subdomains times kw waves along K, whose
// partial sums meet in LDS and are added in wave order.  A lane ends with four
// consecutive neurons of one subdomain, so the epilogue moves 16 bytes per
// access.  With splits > 1 (long K) every block writes a partial tile and
// fc_split_reduce adds the partials in split order, then runs the epilogue
// (deterministic, no cross-block synchronisation).
// ---------------------------------------------------------------------------
template <int TN, int MM, bool SRC_BF16, int EK = -1>
__global__ __launch_bounds__(1024) void fc_kernel(GemmGeom G, const void* __restrict__ src_v, EpiArgs E, SplitArgs S,
                                                  int wm, int kw) {
  using M = Mma<(MM != 0)>;
  constexpr int KS = M::KS, VPL = M::VPL;
  extern __shared__ float red[];  // [kw-1][wm waves][TN][4][64]
  adam_tick(E);
  const int split = blockIdx.z;
  const int tid = threadIdx.x;
  const int wv = tid >> 6, lane = tid & 63, r = lane & 15, g = lane >> 4;
  const int wave = wv % wm, wk = wv / wm;         // position along subdomains, along K
  const int mt = 16 * wm;                         // subdomains of a block
  const int b0 = blockIdx.x * mt + wave * 16;     // subdomains of this wave
  const int n0 = blockIdx.y * (16 * TN);        // neurons of this block
  const int ksteps = (G.K + KS - 1) / KS;
  const int per = (ksteps + S.splits - 1) / S.splits;
  const int sbeg = split * per;
  const int send = min(ksteps, (split + 1) * per);
  const int perw = (send - sbeg + kw - 1) / kw;
  const int kbeg = (sbeg + wk * perw) * KS;
  const int kend = min(G.K, min(send, sbeg + (wk + 1) * perw) * KS);

  const int sub = b0 + r;
  const bool svalid = sub < G.M;
  const size_t base = (size_t)(svalid ? sub : 0) * G.src_n;
  const bool vec_out = (G.dst_n & 3) == 0;
  const float* srcf = (const float*)src_v;
  const bf16_t* srch = (const bf16_t*)src_v;
  const bool vec = (G.src_n % (SRC_BF16 ? 8 : 4)) == 0;

  f32x4 acc[TN];
#pragma unroll
  for (int t = 0; t < TN; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
  for (int k0 = kbeg; k0 < kend; k0 += KS) {
    const int kl = k0 + VPL * g;
    float x[VPL];
    if (vec && kl + VPL <= G.K) {
      if (SRC_BF16) {
        const bf16x8 h = *reinterpret_cast<const bf16x8*>(srch + base + kl);
#pragma unroll
        for (int j = 0; j < VPL; ++j) x[j] = (float)h[j];
      } else {
#pragma unroll
        for (int j = 0; j < VPL; j += 4) {
          const float4 v = *reinterpret_cast<const float4*>(srcf + base + kl + j);
          x[j] = v.x;
          x[j + 1] = v.y;
          x[j + 2] = v.z;
          x[j + 3] = v.w;
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < VPL; ++j) {
        const int k = kl + j;
        const size_t off = k < G.K ? base + k : base;
        const float v = SRC_BF16 ? bf2f(srch[off]) : srcf[off];
        x[j] = k < G.K ? v : 0.f;
      }
    }
    if (!svalid) {
#pragma unroll
      for (int j = 0; j < VPL; ++j) x[j] = 0.f;
    }
#pragma unroll
    for (int t = 0; t < TN; ++t) {
      const size_t wo = (size_t)(n0 + 16 * t + r) * G.Kp + kl;
      const typename M::BFrag w = M::loadB(G, wo);
      if constexpr (MM == 2)
        M::mma3_wx(w, *reinterpret_cast<const typename M::BFrag*>(G.Bhl + wo), x, acc[t]);
      else
        M::mma_wx(w, x, acc[t]);
    }
  }
  if (kw > 1) {
    float* mine = red + (size_t)((wk - 1) * wm + wave) * (TN * 4 * 64);
    if (wk > 0) {
#pragma unroll
      for (int t = 0; t < TN; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) mine[(t * 4 + q) * 64 + lane] = acc[t][q];
    }
    __syncthreads();
    if (wk > 0) return;
    for (int w = 1; w < kw; ++w) {
      const float* other = red + (size_t)((w - 1) * wm + wave) * (TN * 4 * 64);
#pragma unroll
      for (int t = 0; t < TN; ++t)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[t][q] += other[(t * 4 + q) * 64 + lane];
    }
  }
  // lane holds neurons n0 + 16t + 4g + q of subdomain b0 + r
  if (S.splits > 1) {
    // partial tile layout [tile][split][16*TN neurons][mt subdomains]
    const size_t tile_id = (size_t)blockIdx.y * gridDim.x + blockIdx.x;
    float* mine = S.partial + (tile_id * S.splits + split) * (size_t)(mt * 16 * TN);
#pragma unroll
    for (int t = 0; t < TN; ++t)
#pragma unroll
      for (int q = 0; q < 4; ++q) mine[(16 * t + 4 * g + q) * mt + wave * 16 + r] = acc[t][q];
    return;
  }
  if (!svalid) return;
#pragma unroll
  for (int t = 0; t < TN; ++t) {
    const int j = n0 + 16 * t + 4 * g;
    const int nv = min(4, G.N - j);
    if (nv <= 0) continue;
    float v4[4] = {acc[t][0], acc[t][1], acc[t][2], acc[t][3]};
    const size_t i0 = (size_t)sub * G.dst_n + j;
    if (vec_out && nv == 4)
      epilogue4<true, EK>(E, i0, 1, 4, sub, 0, j, 1, v4);
    else
      epilogue4<false, EK>(E, i0, 1, nv, sub, 0, j, 1, v4);
  }
}

template <int TN>
__global__ __launch_bounds__(256) void fc_split_reduce(GemmGeom G, EpiArgs E, SplitArgs S, int gx, int mt) {
  // one thread per output element, consecutive threads on consecutive subdomains
  // of one neuron (the partial tiles store subdomains contiguously)
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  const int mp = gx * mt;
  if (e >= (size_t)mp * G.N) return;
  const int j = (int)(e / mp);
  const int sub = (int)(e - (size_t)j * mp);
  if (sub >= G.M) return;
  const int cols = 16 * TN;
  const int bx = sub / mt, by = j / cols;
  const size_t tile_id = (size_t)by * gx + bx;
  const float* pt = S.partial + tile_id * S.splits * (size_t)(mt * cols) + (size_t)(j - by * cols) * mt + (sub - bx * mt);
  EpiIn in{};
  epi_load<false>(E, (size_t)sub * G.dst_n + j, 1, 1, in);
  float v = 0.f;
  for (int sp = 0; sp < S.splits; ++sp) v += pt[(size_t)sp * (mt * cols)];
  float v4[4] = {v, 0.f, 0.f, 0.f};
  epi_finish<false>(E, (size_t)sub * G.dst_n + j, 1, 1, sub, 0, j, 1, v4, in);
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
static int conv_img_floats(const GemmGeom& g) { return g.LH * g.LW * g.CP; }

static int max_kp(const GemmGeom* g, int n) {
  int m = 0;
  for (int i = 0; i < n; ++i) m = g[i].Kp > m ? g[i].Kp : m;
  return m;
}

// weight rows staged per class (the columns rounded up to whole tiles) and their
// LDS row stride (padded by 16 bytes against bank conflicts)
static int conv_n_eff(const GemmGeom& g, int tn) { return (g.N + 16 * tn - 1) / (16 * tn) * 16 * tn; }
static int conv_bstride(const GemmGeom* g, int n, int mma_bf16) { return max_kp(g, n) + (mma_bf16 ? 8 : 4); }

// LDS floats of the destination band of one block (the tallest band of `parts`,
// each channel's row padded by 4 floats)
static int conv_out_floats(const GemmGeom& g, int parts) {
  const int H = g.dst_HW / g.dst_W;
  return g.dst_n / g.dst_HW * (((H + parts - 1) / parts) * g.dst_W + 4);
}

size_t conv_lds_bytes(const GemmGeom* g, int n_classes, int tn, int mma_bf16, int parts) {
  // BF16 weights (mode 1), FP32 (0), or BF16 heads and remainders (2)
  const size_t wbytes = (size_t)n_classes * conv_n_eff(g[0], tn) * conv_bstride(g, n_classes, mma_bf16) * (mma_bf16 == 1 ? 2 : 4);
  return ((((size_t)conv_img_floats(g[0]) + conv_out_floats(g[0], parts) +
            (size_t)n_classes * max_kp(g, n_classes) + 3) & ~(size_t)3) + 4 * (size_t)n_classes) * 4 +
         wbytes;
}

// The kernel of a contraction with its epilogue kind fixed at compile time for the
// kinds of the ascent iteration (the code of the other kinds is left out, which
// keeps the kernel small in the instruction cache), else the general one.
template <int MM, bool SRC, int TN>
static const void* conv_fn(int kind, int want_val) {
  if (kind == EPI_INNER_MIN && !want_val) return (const void*)conv_plane_kernel<MM, SRC, TN, EPI_INNER_MIN | kEkNoVal>;
  if (kind == EPI_ADAM) return (const void*)conv_plane_kernel<MM, SRC, TN, EPI_ADAM>;
  return (const void*)conv_plane_kernel<MM, SRC, TN>;
}

template <int TN>
static hipError_t launch_conv_tn(const GemmPack& P, const GemmGeom* geo_dev, int B, const void* src, int src_bf16,
                                 int mma_bf16, const EpiArgs& e, int parts, hipStream_t s) {
  const GemmGeom& G = P.g[0];
  const int dst_H = G.dst_HW / G.dst_W;
  if (parts < 1 || parts > dst_H) return hipErrorInvalidValue;
  const size_t lds = conv_lds_bytes(P.g, P.n, TN, mma_bf16, parts);
  const int kpm = max_kp(P.g, P.n);
  const int img = conv_img_floats(G);
  const int outf = conv_out_floats(G, parts);
  // 16-byte epilogue: every band starts and ends on a multiple of 4 neurons
  const int hw4 = (G.dst_HW % 4) == 0 && (parts == 1 || G.dst_W % 4 == 0);
  const int neff = conv_n_eff(G, TN), bst = conv_bstride(P.g, P.n, mma_bf16);
  dim3 grid((unsigned)((size_t)B * parts)), block(kConvThreads);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  const void* fn;
  if (mma_bf16 == 1 && src_bf16)
    fn = conv_fn<1, true, TN>(e.kind, e.want_val);
  else if (mma_bf16 == 1)
    fn = conv_fn<1, false, TN>(e.kind, e.want_val);
  else if (mma_bf16 == 2 && !src_bf16)
    fn = conv_fn<2, false, TN>(e.kind, e.want_val);
  else if (mma_bf16 == 0 && !src_bf16)
    fn = conv_fn<0, false, TN>(e.kind, e.want_val);
  else
    return hipErrorInvalidValue;
  // the channel-last map: 16-byte pixels, every channel k reads inside the pixel
  if (G.CP % 4 != 0 || G.CP < (((G.src_n / (G.src_H * G.src_W)) + 3) & ~3) || G.K % 4 != 0)
    return hipErrorInvalidValue;
  if (lds > 64 * 1024) {
    const hipError_t err = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
  }
  GemmPack pa = P;
  const GemmGeom* ga = geo_dev;
  const void* sa = src;
  EpiArgs ea = e;
  ea.lohi_len = G.dst_n;
  int a0 = img, a1 = hw4, a2 = kpm, a3 = neff, a4 = bst, a5 = parts, a6 = outf;
  void* args[] = {(void*)&pa, (void*)&ga, (void*)&sa, (void*)&ea, (void*)&a0, (void*)&a1, (void*)&a2, (void*)&a3,
                  (void*)&a4, (void*)&a5, (void*)&a6};
  return hipLaunchKernel(fn, grid, block, args, lds, s);
}

hipError_t launch_conv(const GemmGeom* geoms, const GemmGeom* geo_dev, int n, int B, const void* src, int src_bf16,
                       int mma_bf16, const EpiArgs& e, int tn, int parts, hipStream_t s) {
  GemmPack P;
  if (n <= 0 || n > kMaxClasses) return hipErrorInvalidValue;
  P.n = n;
  for (int i = 0; i < n; ++i) P.g[i] = geoms[i];
  if (B == 0 || P.g[0].N == 0) return hipSuccess;
  if (tn == 1) return launch_conv_tn<1>(P, geo_dev, B, src, src_bf16, mma_bf16, e, parts, s);
  if (tn == 2) return launch_conv_tn<2>(P, geo_dev, B, src, src_bf16, mma_bf16, e, parts, s);
  if (tn == 4) return launch_conv_tn<4>(P, geo_dev, B, src, src_bf16, mma_bf16, e, parts, s);
  return hipErrorInvalidValue;
}

template <int TN, int MM, bool SRC>
static const void* fc_fn(int kind, int want_val) {
  if (kind == EPI_INNER_MIN && !want_val) return (const void*)fc_kernel<TN, MM, SRC, EPI_INNER_MIN | kEkNoVal>;
  if (kind == EPI_ADAM) return (const void*)fc_kernel<TN, MM, SRC, EPI_ADAM>;
  if (kind == EPI_ADAM_LAST) return (const void*)fc_kernel<TN, MM, SRC, EPI_ADAM_LAST>;
  return (const void*)fc_kernel<TN, MM, SRC>;
}

template <int TN>
static hipError_t launch_fc_tn(const GemmGeom& G, const void* src, int src_bf16, int mma_bf16, const EpiArgs& e_in,
                               const SplitArgs& sp, int wm, int kw, hipStream_t s) {
  EpiArgs e = e_in;
  e.lohi_len = G.dst_n;
  if ((wm != 1 && wm != 2 && wm != 4) || (kw != 1 && kw != 2 && kw != 4 && kw != 8) || wm * kw > 16)
    return hipErrorInvalidValue;
  const int mt = 16 * wm;
  const int gx = (G.M + mt - 1) / mt, gy = (G.N + 16 * TN - 1) / (16 * TN);  // subdomain blocks, neuron blocks
  dim3 grid(gx, gy, sp.splits), block(64 * wm * kw);
  const size_t lds = (size_t)(kw - 1) * wm * TN * 4 * 64 * 4;
  const void* fn;
  if (mma_bf16 == 1)
    fn = src_bf16 ? fc_fn<TN, 1, true>(e.kind, e.want_val) : fc_fn<TN, 1, false>(e.kind, e.want_val);
  else if (mma_bf16 == 2 && !src_bf16)
    fn = fc_fn<TN, 2, false>(e.kind, e.want_val);
  else if (mma_bf16 == 0 && !src_bf16)
    fn = fc_fn<TN, 0, false>(e.kind, e.want_val);
  else
    return hipErrorInvalidValue;
  {
    GemmGeom ga = G;
    const void* sa = src;
    EpiArgs ea = e;
    SplitArgs spa = sp;
    int a0 = wm, a1 = kw;
    void* args[] = {(void*)&ga, (void*)&sa, (void*)&ea, (void*)&spa, (void*)&a0, (void*)&a1};
    const hipError_t le = hipLaunchKernel(fn, grid, block, args, lds, s);
    if (le != hipSuccess) return le;
  }
  hipError_t err = hipGetLastError();
  if (err != hipSuccess || sp.splits <= 1) return err;
  EpiArgs e2 = e;
  e2.t_dev = nullptr;  // the step was already counted by the partial launch
  const size_t outs = (size_t)gx * mt * G.N;
  hipLaunchKernelGGL((fc_split_reduce<TN>), dim3((unsigned)((outs + 255) / 256)), dim3(256), 0, s, G, e2, sp, gx, mt);
  return hipGetLastError();
}

hipError_t launch_fc(const GemmGeom& G, const void* src, int src_bf16, int mma_bf16, const EpiArgs& e, int tn,
                     const SplitArgs& sp, int wm, int kw, hipStream_t s) {
  if (G.M == 0 || G.N == 0) return hipSuccess;
  if (tn == 1) return launch_fc_tn<1>(G, src, src_bf16, mma_bf16, e, sp, wm, kw, s);
  if (tn == 2) return launch_fc_tn<2>(G, src, src_bf16, mma_bf16, e, sp, wm, kw, s);
  if (tn == 4) return launch_fc_tn<4>(G, src, src_bf16, mma_bf16, e, sp, wm, kw, s);
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Transposed strided convolution, one block per subdomain, or with `split` one
// block per (subdomain, chunk of input channels) (see ColGeom):
//  0. staging, one round of loads then one of LDS writes: the subdomain's rho
//     (A operand) in MFMA operand order, [K/VPL][Mp][VPL] (BF16 for the BF16
//     product), zero-padded in K and M; the fragment-ordered weights (B
//     operand); the tap tables;
//  1. per chunk of input channels, waves compute 16x16 MFMA tiles of
//     Y = rho^T W into LDS, while the device-memory operands of each thread's
//     first epilogue group of the chunk are in flight (those of the first
//     chunk are issued before the staging loads);
//  2. every output of the chunk sums its taps from Y and goes through the
//     epilogue, four consecutive neurons per thread, with the operands of the
//     next group loaded before the current one is finished.
// ---------------------------------------------------------------------------
constexpr int kTThreads = 256;

// (the register cap keeps the compiler from spending registers on the staging
// round that would leave one wave per SIMD)
template <bool BF, int TM, int EK = -1>
__global__ __launch_bounds__(kTThreads) __attribute__((amdgpu_waves_per_eu(4))) void convT_kernel(ColGeom G, const float* __restrict__ rho, EpiArgs E, int split) {
  using M = Mma<BF>;
  typedef typename M::BFrag BFrag;
  typedef typename M::AFrag AFrag;
  typedef typename std::conditional<BF, __bf16, float>::type AT;
  constexpr int KS = M::KS, VPL = M::VPL, NW = kTThreads / 64;
  extern __shared__ float lds[];
  const int ks = BF ? G.ksh : G.ksf;
  const int kq_n = ks * (KS / VPL);                    // K rounded up to whole steps, in groups of VPL
  // the block's chunks: all, or (split) chunk blockIdx.x mod nchunks only
  const int b = split ? blockIdx.x / G.nchunks : blockIdx.x;
  const int c_first = split ? blockIdx.x - b * G.nchunks : 0;
  const int c_end = split ? c_first + 1 : G.nchunks;
  const int nfrag = (c_end - c_first) * G.ntc * ks * 64;  // fragments (16 bytes each) staged
  BFrag* Bl = reinterpret_cast<BFrag*>(lds);           // [staged chunks][ntc][ks][64 lanes]
  AT* A = reinterpret_cast<AT*>(lds + 4 * nfrag);      // [kq_n][Mp][VPL]
  float* Y = reinterpret_cast<float*>(A + (size_t)kq_n * G.Mp * VPL);  // [Mp][Ns]
  int* tab = reinterpret_cast<int*>(Y + G.Mp * G.Ns);  // toff_y [H][Tmax], cnt_y [H], toff_x [W][Tmax], cnt_x [W]
  const int* ty = tab;
  const int* cy = ty + G.H * G.Tmax;
  const int* tx = cy + G.H;
  const int* cx = tx + G.W * G.Tmax;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, r = lane & 15, g = lane >> 4;
  const size_t dst_base = (size_t)b * G.Ci * G.HW;
  // the subdomain's bound rows, shared by row_div consecutive subdomains
  const ptrdiff_t lshift = (ptrdiff_t)(b / max(E.row_div, 1) - b) * E.lohi_len;
  constexpr int STEP = 4 * kTThreads;
  const bool vec = (G.HW & 3) == 0;
  // operands of the thread's first epilogue group of a chunk: for the first
  // chunk they are in flight during the staging, for the others during the GEMM
  EpiIn nx{};
  auto prefetch = [&](int e0, int e1) {
    if (vec) {
      if (e0 + 4 * tid < e1) epi_load<true, 3, true, EK>(E, dst_base + e0 + 4 * tid, 1, 4, nx, lshift);
    } else {
      if (e0 + tid < e1) epi_load<false, 3, true, EK>(E, dst_base + e0 + tid, 1, 1, nx, lshift);
    }
  };
  prefetch(c_first * G.Cc * G.HW, min(G.Ci, (c_first + 1) * G.Cc) * G.HW);
  adam_tick(E);
  // 0. staging: K groups holding channels of rho are gathered (every load of a
  // round in flight before the LDS writes; the index is clamped into the map and
  // the value masked), the groups of the K padding are zero-filled
  {
    constexpr int UC = 16 / VPL, UF = 8;  // 16 gathered values per thread and round
    const float* src = rho + (size_t)b * G.Co * G.M;
    const int ncell = kq_n * G.Mp;
    const int ncell_r = min(ncell, ((G.Co + VPL - 1) / VPL) * G.Mp);
    const u32x4* fsrc = reinterpret_cast<const u32x4*>(BF ? (const void*)G.Bh : (const void*)G.Bf) +
                        (size_t)c_first * G.ntc * ks * 64;
    const float inv_mp = 1.0f / (float)G.Mp;
    const int rounds = max((ncell_r + UC * kTThreads - 1) / (UC * kTThreads), (nfrag + UF * kTThreads - 1) / (UF * kTThreads));
    // one round: every load in flight (indexes clamped into the arrays), then the
    // LDS writes (the first round is straight-line code, so no wait carries over
    // from a later round's registers)
    const auto round = [&](const int rd) __attribute__((always_inline)) {
      float v[UC][VPL];
      int kqs[UC], ms[UC];
      u32x4 f[UF];
      int tv = 0;
      static_for<UC>([&](auto uc) __attribute__((always_inline)) {
        constexpr int u = decltype(uc)::value;
        const int cell = min((rd * UC + u) * kTThreads + tid, ncell_r - 1);
        kqs[u] = fdiv(cell, G.Mp, inv_mp);
        ms[u] = cell - kqs[u] * G.Mp;
        const float* s0 = src + (unsigned)min(ms[u], G.M - 1);
#pragma unroll
        for (int j = 0; j < VPL; ++j) v[u][j] = s0[(unsigned)(min(kqs[u] * VPL + j, G.Co - 1) * G.M)];
      });
      static_for<UF>([&](auto uf) __attribute__((always_inline)) {
        constexpr int u = decltype(uf)::value;
        const int i = (rd * UF + u) * kTThreads + tid;
        if (i < nfrag) f[u] = fsrc[i];
      });
      if (rd == 0 && tid < G.ntab) tv = G.tab[tid];
      if (rd == 0)
        for (int i = ncell_r + tid; i < ncell; i += kTThreads) *reinterpret_cast<AFrag*>(A + (size_t)i * VPL) = AFrag{};
      static_for<UC>([&](auto uc) __attribute__((always_inline)) {
        constexpr int u = decltype(uc)::value;
        const int cell = (rd * UC + u) * kTThreads + tid;
        if (cell < ncell_r) {
          AFrag a;
#pragma unroll
          for (int j = 0; j < VPL; ++j) a[j] = (kqs[u] * VPL + j < G.Co && ms[u] < G.M) ? (AT)v[u][j] : (AT)0.f;
          *reinterpret_cast<AFrag*>(A + (size_t)cell * VPL) = a;
        }
      });
      static_for<UF>([&](auto uf) __attribute__((always_inline)) {
        constexpr int u = decltype(uf)::value;
        const int i = (rd * UF + u) * kTThreads + tid;
        if (i < nfrag) reinterpret_cast<u32x4*>(Bl)[i] = f[u];
      });
      if (rd == 0 && tid < G.ntab) tab[tid] = tv;
    };
    round(0);
    for (int rd = 1; rd < rounds; ++rd) round(rd);
    for (int i = tid + kTThreads; i < G.ntab; i += kTThreads) tab[i] = G.tab[i];
  }
  __syncthreads();
  const int mtn = G.Mp >> 4;
  for (int c = c_first; c < c_end; ++c) {
    const int c0 = c * G.Cc, c1 = min(G.Ci, c0 + G.Cc);
    const int e0 = c0 * G.HW, e1 = c1 * G.HW;
    if (c > c_first) prefetch(e0, e1);
    // UT independent tiles per wave at a time (their operand reads overlap)
    constexpr int UT = 4;
    const int items = mtn * G.ntc;
    for (int it0 = wave; it0 < items; it0 += UT * NW) {
      const AFrag* fa[UT];
      const BFrag* fb[UT];
      int yofs[UT];
      f32x4 acc[UT];
#pragma unroll
      for (int u = 0; u < UT; ++u) {
        const int it = min(it0 + u * NW, items - 1);
        const int mt = it / G.ntc;
        const int nt = it - mt * G.ntc;
        fa[u] = reinterpret_cast<const AFrag*>(A) + (size_t)g * G.Mp + mt * 16 + r;
        fb[u] = Bl + (size_t)((c - c_first) * G.ntc + nt) * ks * 64 + lane;
        yofs[u] = (mt * 16 + 4 * g) * G.Ns + nt * 16 + r;
        acc[u] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
      for (int st = 0; st < ks; ++st) {
        AFrag av[UT];
        BFrag bv[UT];
#pragma unroll
        for (int u = 0; u < UT; ++u) {
          av[u] = fa[u][(size_t)st * 4 * G.Mp];
          bv[u] = fb[u][(size_t)st * 64];
        }
#pragma unroll
        for (int u = 0; u < UT; ++u) M::mma_frag(av[u], bv[u], acc[u]);
      }
#pragma unroll
      for (int u = 0; u < UT; ++u)
        if (it0 + u * NW < items)
#pragma unroll
          for (int q = 0; q < 4; ++q) Y[yofs[u] + q * G.Ns] = acc[u][q];
    }
    __syncthreads();
    if (vec) {
      for (int e = e0 + 4 * tid; e < e1; e += STEP) {
        const EpiIn cur = nx;
        if (e + STEP < e1) epi_load<true, 3, true, EK>(E, dst_base + e + STEP, 1, 4, nx, lshift);
        const int ci = fdiv(e, G.HW, G.inv_HW);
        const int rem = e - ci * G.HW;
        int y = fdiv(rem, G.W, G.inv_W);
        int x = rem - y * G.W;
        const int nb = (ci - c0) * G.khkw;
        float v4[4];
        if (TM > 0) {
          // fixed tap loops: table entries past a row's (column's) count hold a
          // valid offset and their products are masked, so every LDS read of
          // the group is issued at once
          int oy[4][TM > 0 ? TM : 1], ox[4][TM > 0 ? TM : 1], ny[4], nxx[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            ny[q] = cy[y];
            nxx[q] = cx[x];
#pragma unroll
            for (int i = 0; i < TM; ++i) {
              oy[q][i] = ty[y * TM + i] + nb;
              ox[q][i] = tx[x * TM + i];
            }
            if (++x == G.W) {
              x = 0;
              ++y;
            }
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            float sum = 0.f;
#pragma unroll
            for (int ia = 0; ia < TM; ++ia)
#pragma unroll
              for (int ib = 0; ib < TM; ++ib) {
                const float t = Y[oy[q][ia] + ox[q][ib]];
                sum += (ia < ny[q] && ib < nxx[q]) ? t : 0.f;
              }
            v4[q] = sum;
          }
        } else {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            float sum = 0.f;
            const int ny = cy[y], nxx = cx[x];
            for (int ia = 0; ia < ny; ++ia) {
              const int oy = ty[y * G.Tmax + ia] + nb;
              for (int ib = 0; ib < nxx; ++ib) sum += Y[oy + tx[x * G.Tmax + ib]];
            }
            v4[q] = sum;
            if (++x == G.W) {
              x = 0;
              ++y;
            }
          }
        }
        epi_finish<true, EK>(E, dst_base + e, 1, 4, b, 0, ci, 0, v4, cur);
      }
    } else {
      for (int e = e0 + tid; e < e1; e += kTThreads) {
        const EpiIn cur = nx;
        if (e + kTThreads < e1) epi_load<false, 3, true, EK>(E, dst_base + e + kTThreads, 1, 1, nx, lshift);
        const int ci = fdiv(e, G.HW, G.inv_HW);
        const int rem = e - ci * G.HW;
        const int y = fdiv(rem, G.W, G.inv_W);
        const int x = rem - y * G.W;
        const int nb = (ci - c0) * G.khkw;
        float sum = 0.f;
        for (int ia = 0; ia < cy[y]; ++ia) {
          const int oy = ty[y * G.Tmax + ia] + nb;
          for (int ib = 0; ib < cx[x]; ++ib) sum += Y[oy + tx[x * G.Tmax + ib]];
        }
        float v4[4] = {sum, 0.f, 0.f, 0.f};
        epi_finish<false, EK>(E, dst_base + e, 1, 1, b, 0, ci, 0, v4, cur);
      }
    }
    __syncthreads();
  }
}

// LDS of convT_kernel for the operand type: weight fragments (of every chunk, or
// of one with split), A, Y, tap tables
static size_t convT_lds_bytes_t(const ColGeom& g, int bf16, int split = 0) {
  const int ks = bf16 ? g.ksh : g.ksf, kp = ks * (bf16 ? 32 : 16);
  const size_t nfrag = (size_t)(split ? 1 : g.nchunks) * g.ntc * ks * 64;
  return 16 * nfrag + (size_t)kp * g.Mp * (bf16 ? 2 : 4) + (size_t)4 * g.Mp * g.Ns + (size_t)4 * g.ntab;
}

size_t convT_lds_bytes(const ColGeom& g, int split) {
  const size_t a = convT_lds_bytes_t(g, 0, split), b = convT_lds_bytes_t(g, 1, split);
  return a > b ? a : b;
}

template <bool BF, int TM>
static const void* convT_fn(int kind, int want_val) {
  if (kind == EPI_P0 && !want_val) return (const void*)convT_kernel<BF, TM, EPI_P0 | kEkNoVal>;
  if (kind == EPI_INNER_MIN && !want_val) return (const void*)convT_kernel<BF, TM, EPI_INNER_MIN | kEkNoVal>;
  return (const void*)convT_kernel<BF, TM>;
}

hipError_t launch_convT(const ColGeom& g, int B, const float* rho, int mma_bf16, const EpiArgs& e, int split,
                        hipStream_t s) {
  if (B == 0) return hipSuccess;
  if (e.kind == EPI_ADAM || e.kind == EPI_ADAM_LAST) return hipErrorInvalidValue;  // reads more than 3 arrays
  if (mma_bf16 != 0 && mma_bf16 != 1) return hipErrorInvalidValue;
  const size_t lds = convT_lds_bytes_t(g, mma_bf16, split);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  // tap loops of fixed length where every row and column takes at most one or two taps
  const void* fn;
  if (g.Tmax == 1)
    fn = mma_bf16 ? convT_fn<true, 1>(e.kind, e.want_val) : convT_fn<false, 1>(e.kind, e.want_val);
  else if (g.Tmax == 2)
    fn = mma_bf16 ? convT_fn<true, 2>(e.kind, e.want_val) : convT_fn<false, 2>(e.kind, e.want_val);
  else
    fn = mma_bf16 ? convT_fn<true, 0>(e.kind, e.want_val) : convT_fn<false, 0>(e.kind, e.want_val);
  if (lds > 64 * 1024) {
    hipError_t err = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (err != hipSuccess) return err;
  }
  ColGeom ga = g;
  const float* ra = rho;
  EpiArgs ea = e;
  ea.lohi_len = g.Ci * g.HW;  // the destination map per subdomain
  int sa = split ? 1 : 0;
  void* args[] = {(void*)&ga, (void*)&ra, (void*)&ea, (void*)&sa};
  return hipLaunchKernel(fn, dim3((unsigned)((size_t)B * (split ? g.nchunks : 1))), dim3(kTThreads), args, lds, s);
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
                                       double beta2, double eps, int row_div) {
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
    const size_t il = row_div > 1 ? (i / n / row_div) * n + j : i;  // the subdomain's bound row
    if (val != nullptr) {
      double xbd, xd, v;
      const double r = rho[i];
      inner_min<double>(r, g[i], lo[il], hi[il], (double)tau, xbd, xd, v);
      val[i] = v - r * (double)bias[j / bias_hw];
      xb[i] = (float)xbd;
    } else {
      float xbf, xf, v;
      inner_min<float>(rho[i], g[i], lo[il], hi[il], tau, xbf, xf, v);
      xb[i] = xbf;
    }
  }
}

__global__ void crown_const_kernel(int B, int n, const float* __restrict__ g, const float* __restrict__ lo,
                                   const float* __restrict__ hi, float* __restrict__ rho, int wk, int row_div) {
  const size_t total_n = (size_t)B * n;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total_n; i += (size_t)gridDim.x * blockDim.x) {
    const size_t il = row_div > 1 ? (i / n / row_div) * n + i % n : i;  // the subdomain's bound row
    rho[i] = crown_dual(g[i], lo[il], hi[il], wk != 0);
  }
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

// out[b] = sum_j c[b, j] * (y ? y[b, j] : bias[j / bias_div])  (FP64; a conv layer's
// bias is per channel, bias_div = H*W)
__global__ void cdot_kernel(int n, const float* __restrict__ c, const float* __restrict__ y,
                            const float* __restrict__ bias, int bias_div, double* __restrict__ out) {
  __shared__ double sh[64];
  const int b = blockIdx.x;
  double s = 0.0;
  for (int j = threadIdx.x; j < n; j += 64)
    s += (double)c[(size_t)b * n + j] * (double)(y ? y[(size_t)b * n + j] : bias[j / bias_div]);
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
__global__ void fill_f64_kernel(double* p, size_t n, double v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void fill_i32_kernel(int* p, size_t n, int v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void copy_f32_kernel(float* __restrict__ d, const float* __restrict__ s, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) d[i] = s[i];
}
// The largest dual value of the tracked steps and its step: q (the value at the
// duals a step starts from) against best_q; *step holds the step's number.
__global__ void best_update_kernel(int B, const double* __restrict__ q, double* __restrict__ best_q,
                                   int* __restrict__ best_t, const int* __restrict__ step) {
  const int b = blockIdx.x * 256 + threadIdx.x;
  if (b >= B) return;
  const double v = q[b];
  if (v > best_q[b]) {
    best_q[b] = v;
    best_t[b] = *step;
  }
}

__global__ void inc_i32_kernel(int* c) { *c += 1; }

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
                                  double beta1, double beta2, double eps, int row_div, hipStream_t s) {
  hipLaunchKernelGGL(inner_min_const_kernel, dim3(grid_for((size_t)B * n)), dim3(256), 0, s, B, n, g, rho, lo, hi,
                     bias, bias_hw, tau, xb, val, t_dev, adam, lr0, lr_end, total, beta1, beta2, eps, row_div);
  return hipGetLastError();
}

hipError_t launch_crown_const(int B, int n, const float* g, const float* lo, const float* hi, float* rho, int wk,
                              int row_div, hipStream_t s) {
  hipLaunchKernelGGL(crown_const_kernel, dim3(grid_for((size_t)B * n)), dim3(256), 0, s, B, n, g, lo, hi, rho, wk,
                     row_div);
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

hipError_t launch_cdot(int B, int n, const float* c, const float* y, const float* bias, int bias_div, double* out,
                       hipStream_t s) {
  if (bias_div < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(cdot_kernel, dim3(B), dim3(64), 0, s, n, c, y, bias, bias_div, out);
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
hipError_t launch_fill_f64(double* p, size_t n, double v, hipStream_t s) {
  hipLaunchKernelGGL(fill_f64_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, n, v);
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
hipError_t launch_best_update(int B, const double* q, double* best_q, int* best_t, const int* step, hipStream_t s) {
  if (B == 0) return hipSuccess;
  hipLaunchKernelGGL(best_update_kernel, dim3((B + 255) / 256), dim3(256), 0, s, B, q, best_q, best_t, step);
  return hipGetLastError();
}

hipError_t launch_inc_i32(int* c, hipStream_t s) {
  hipLaunchKernelGGL(inc_i32_kernel, dim3(1), dim3(1), 0, s, c);
  return hipGetLastError();
}

hipError_t launch_max_f64(int B, const double* a, const double* b, double* out, hipStream_t s) {
  hipLaunchKernelGGL(max_f64_kernel, dim3((B + 255) / 256), dim3(256), 0, s, B, a, b, out);
  return hipGetLastError();
}

}  // namespace ld
