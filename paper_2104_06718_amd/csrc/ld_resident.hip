// Resident ascent kernel (gfx950): the whole supergradient/Adam ascent of
// Algorithm 1 for S subdomains per workgroup, in one launch.
//
// Subdomains are independent (Sec. 5.2: bounding is batched over subproblems),
// so a workgroup owns its subdomains for every iteration of the call and never
// synchronises with another workgroup.  Per iteration it sweeps the layers from
// the top: for k = n-1 .. 1
//   g_{k-1} = W_k^T rho_k                  (transposed product, into LDS)
//   inner minimisation of P_{k-1}          (Sec. 3.2.1 / 3.2.2; x* and xB* into LDS)
//   xhat_A,k = W_k x*_{k-1} + b_k          (forward product, into LDS)
//   s_k = xhat_B,k - xhat_A,k; Adam step   (rho_k, m_k, v_k in device memory)
// Every use of rho_k in an iteration (its transposed product and its own inner
// minimisation) happens before its Adam step, so the sweep performs exactly the
// synchronous iteration.  Only x* of one layer and xB* of two layers are live at
// a time; they never leave LDS.  Device memory sees the algorithmic traffic --
// the bounds and the Adam state, once per iteration -- plus the fully-connected
// weights, which stream from L2.  Conv weights and gather tables of the current
// contraction are staged in LDS, so the MFMA loops read LDS only.
#include "ld_internal.h"
#include "ld_device.h"

namespace ld {

constexpr int kRWaves = 16;
constexpr int kRThreads = 64 * kRWaves;

__device__ __forceinline__ void bsync() { __syncthreads(); }

// Zero-padded LDS image geometry of a map consumed by a conv contraction.
struct Img {
  int C, H, W, LH, LW, pt, pl;
};
__device__ __forceinline__ Img img_of(const GemmGeom& g) {
  Img I;
  I.H = g.src_H;
  I.W = g.src_W;
  I.C = g.src_n / (g.src_H * g.src_W);
  I.LH = g.LH;
  I.LW = g.LW;
  I.pt = g.pad_t;
  I.pl = g.pad_l;
  return I;
}
__device__ __forceinline__ int img_pos(const Img& I, int j) {
  const int HW = I.H * I.W;
  const int c = j / HW;
  const int rem = j - c * HW;
  const int y = rem / I.W;
  const int x = rem - y * I.W;
  return (c * I.LH + y + I.pt) * I.LW + x + I.pl;
}
// zero the padding cells of the images of ns subdomains (interior cells untouched)
__device__ void img_border_zero(const Img& I, float* img, int img_stride, int ns, int tid) {
  const int cells = I.C * I.LH * I.LW;
  for (int e = tid; e < ns * cells; e += kRThreads) {
    const int s = e / cells;
    const int cell = e - s * cells;
    const int row = cell / I.LW;
    const int y = row % I.LH - I.pt;
    const int x = cell - row * I.LW - I.pl;
    if ((unsigned)y >= (unsigned)I.H || (unsigned)x >= (unsigned)I.W) img[s * img_stride + cell] = 0.f;
  }
}

// Stage the packed weights (first n_eff rows of each class, row stride kp_max)
// and the gather offsets of a conv contraction into LDS.
template <bool BF>
__device__ void stage_weights(const GemmGeom* geoms, int ncls, int n_eff, int kp_max, float* wb, int tid) {
  typedef typename Mma<BF>::BFrag BFrag;
  constexpr int EPV = BF ? 8 : 4;  // elements per 16-byte vector
  BFrag* wv = reinterpret_cast<BFrag*>(wb);
  const int vrow = kp_max / EPV;
  int* kofs = reinterpret_cast<int*>(wb + (size_t)ncls * n_eff * kp_max / (BF ? 2 : 1));
  for (int c = 0; c < ncls; ++c) {
    const GemmGeom& G = geoms[c];
    const int vr = G.Kp / EPV;
    const BFrag* src = BF ? reinterpret_cast<const BFrag*>(G.Bh) : reinterpret_cast<const BFrag*>(G.Bf);
    for (int e = tid; e < n_eff * vr; e += kRThreads) {
      const int row = e / vr;
      const int v = e - row * vr;
      wv[((size_t)c * n_eff + row) * vrow + v] = src[(size_t)row * vr + v];
    }
    for (int k = tid; k < G.Kp; k += kRThreads) kofs[c * kp_max + k] = G.ktab_lds[k];
  }
}

// ---------------------------------------------------------------------------
// conv contraction from LDS only: for each subdomain s < ns,
// out_s[col*dst_HW + pixel] = sum_k A_s[pixel][k] B[k][col], A gathered from the
// zero-padded image, B and the gather offsets staged by stage_weights.
// Work items (subdomain, class, 16-pixel tile, column chunk) go round-robin to
// the waves.
// ---------------------------------------------------------------------------
template <bool BF, int TN>
__device__ void r_conv(const GemmGeom* __restrict__ geoms, int ncls, int n_eff, int kp_max, const float* wb,
                       const float* img, int img_stride, float* out, int out_stride, int ns, int wave, int lane) {
  using M = Mma<BF>;
  typedef typename M::BFrag BFrag;
  constexpr int KS = M::KS, VPL = M::VPL;
  const int r = lane & 15, g = lane >> 4;
  const BFrag* wv = reinterpret_cast<const BFrag*>(wb);
  const int vrow = kp_max / VPL;
  const int* kofs = reinterpret_cast<const int*>(wb + (size_t)ncls * n_eff * kp_max / (BF ? 2 : 1));
  int items_before = 0;
  for (int s = 0; s < ns; ++s) {
    const float* im = img + s * img_stride;
    float* o = out + s * out_stride;
    for (int cl = 0; cl < ncls; ++cl) {
      const GemmGeom& G = geoms[cl];
      const int* ko = kofs + cl * kp_max;
      const int ntiles = (G.HWq + 15) >> 4;
      const int nct = (G.N + 16 * TN - 1) / (16 * TN);
      const int total = ntiles * nct;
      int first = (wave - items_before) % kRWaves;
      if (first < 0) first += kRWaves;
      for (int w = first; w < total; w += kRWaves) {
        const int tile = w / nct;
        const int nc = (w - tile * nct) * 16 * TN;
        const int p = min(tile * 16 + r, G.HWq - 1);
        const int yq = p / G.Wq;
        const int xq = p - yq * G.Wq;
        const int lb = (yq * G.iy_mul + G.iy_off + G.pad_t) * G.LW + xq * G.ix_mul + G.ix_off + G.pad_l;
        f32x4 acc[TN];
#pragma unroll
        for (int t = 0; t < TN; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
        for (int k0 = 0; k0 < G.K; k0 += KS) {
          const int kl = k0 + VPL * g;
          float a[VPL];
#pragma unroll
          for (int j = 0; j < VPL; ++j) a[j] = im[lb + ko[kl + j]];
#pragma unroll
          for (int t = 0; t < TN; ++t) {
            const BFrag bf = wv[((size_t)cl * n_eff + nc + 16 * t + r) * vrow + kl / VPL];
            M::mma(a, bf, acc[t]);
          }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int pq = tile * 16 + 4 * g + q;
          if (pq < G.HWq) {
            const int yy = pq / G.Wq;
            const int xx = pq - yy * G.Wq;
            const int j0 = (yy * G.oy_mul + G.oy_off) * G.dst_W + xx * G.ox_mul + G.ox_off;
#pragma unroll
            for (int t = 0; t < TN; ++t) {
              const int col = nc + 16 * t + r;
              if (col < G.N) o[col * G.dst_HW + j0] = acc[t][q];
            }
          }
        }
      }
      items_before += total;
    }
  }
}

template <bool BF>
__device__ void r_conv_tn(int tn, const GemmGeom* geoms, int ncls, int n_eff, int kp_max, const float* wb,
                          const float* img, int img_stride, float* out, int out_stride, int ns, int wave, int lane) {
  if (tn == 1)
    r_conv<BF, 1>(geoms, ncls, n_eff, kp_max, wb, img, img_stride, out, out_stride, ns, wave, lane);
  else if (tn == 2)
    r_conv<BF, 2>(geoms, ncls, n_eff, kp_max, wb, img, img_stride, out, out_stride, ns, wave, lane);
  else
    r_conv<BF, 4>(geoms, ncls, n_eff, kp_max, wb, img, img_stride, out, out_stride, ns, wave, lane);
}

// ---------------------------------------------------------------------------
// fully-connected contraction, transposed orientation: out_s[neuron] =
// sum_k Wp[neuron][k] x_s[k] for s < ns (x_s = xsrc + s*xstride, in LDS or device
// memory; weights stream from L2).  Work items (16-neuron tile, K chunk) go
// round-robin to the waves; each item issues the loads of four K steps before
// their MFMAs.  With kc > 1 the chunk results are added in chunk order
// (deterministic).  Must be called by every thread of the block.
// ---------------------------------------------------------------------------
template <bool BF>
__device__ void r_fc(const GemmGeom& G, int kc, const float* xsrc, size_t xstride, int ns, int S, float* out,
                     int out_stride, float* part, int wave, int lane, int tid) {
  using M = Mma<BF>;
  typedef typename M::BFrag BFrag;
  constexpr int KS = M::KS, VPL = M::VPL, U = 4;
  const int r = lane & 15, g = lane >> 4;
  const int ntile = (G.N + 15) >> 4;
  const int ksteps = (G.K + KS - 1) / KS;
  const int per = (ksteps + kc - 1) / kc;
  const bool sv = r < ns;
  const float* xs = xsrc + (size_t)(sv ? r : 0) * xstride;
  const bool vec = (xstride & 3) == 0;
  for (int item = wave; item < ntile * kc; item += kRWaves) {
    const int tile = item / kc;
    const int c = item - tile * kc;
    const int n0 = tile * 16;
    const int kb = c * per * KS;
    const int ke = min(G.K, (c + 1) * per * KS);
    const BFrag* wrow = reinterpret_cast<const BFrag*>(BF ? (const void*)(G.Bh + (size_t)(n0 + r) * G.Kp)
                                                          : (const void*)(G.Bf + (size_t)(n0 + r) * G.Kp));
    f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = kb; k0 < ke; k0 += U * KS) {
      BFrag w[U];
      float x[U][VPL];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int kl = k0 + u * KS + VPL * g;
        const bool in = k0 + u * KS < ke;
        w[u] = wrow[(in ? kl : kb + VPL * g) / VPL];
        if (in && vec && kl + VPL <= G.K) {
#pragma unroll
          for (int j = 0; j < VPL; j += 4) {
            const float4 v = *reinterpret_cast<const float4*>(xs + kl + j);
            x[u][j] = v.x;
            x[u][j + 1] = v.y;
            x[u][j + 2] = v.z;
            x[u][j + 3] = v.w;
          }
        } else {
#pragma unroll
          for (int j = 0; j < VPL; ++j) {
            const int k = kl + j;
            const bool ok = in && k < G.K;
            const float v = xs[ok ? k : 0];
            x[u][j] = ok ? v : 0.f;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (k0 + u * KS < ke) {
          if (!sv) {
#pragma unroll
            for (int j = 0; j < VPL; ++j) x[u][j] = 0.f;
          }
          M::mma_wx(w[u], x[u], acc);
        }
      }
    }
    if (sv) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int neuron = n0 + 4 * g + q;
        if (neuron < G.N) {
          if (kc > 1)
            part[((size_t)c * S + r) * G.N + neuron] = acc[q];
          else
            out[r * out_stride + neuron] = acc[q];
        }
      }
    }
  }
  if (kc > 1) {
    bsync();
    for (int e = tid; e < ns * G.N; e += kRThreads) {
      const int s = e / G.N;
      const int neuron = e - s * G.N;
      float v = 0.f;
      for (int c = 0; c < kc; ++c) v += part[((size_t)c * S + s) * G.N + neuron];
      out[s * out_stride + neuron] = v;
    }
  }
}

__device__ __forceinline__ float4 ldg4(const float* p) { return *reinterpret_cast<const float4*>(p); }
__device__ __forceinline__ void stg4(float* p, float4 v) { *reinterpret_cast<float4*>(p) = v; }
__device__ __forceinline__ float f4(const float4& v, int i) { return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w)); }

template <bool BF>
__global__ __launch_bounds__(kRThreads) void resident_kernel(RPlan P) {
  extern __shared__ float lds[];
  const int S = P.S;
  const int b0 = blockIdx.x * S;
  const int ns = min(S, P.B - b0);
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int n = P.n;
  float* XB[2] = {lds, lds + P.xb_odd};  // [s * xb_stride + j] for even / odd layers
  float* IMG = lds + S * P.xb_stride;
  float* GX = IMG + S * P.img_stride;
  float* WB = GX + S * P.gx_stride;  // conv weights and gather offsets
  float* PART = WB;                  // FC chunk partials (never live with WB)
  float* adam_s = WB + max(P.wb_floats, (P.part_floats + 3) & ~3);  // lr_t, 1/bc1, 1/bc2

  for (int it = 0; it < P.iters; ++it) {
    if (tid == 0) {
      // step t (1-based over all calls on this state): linear step decay, bias corrections
      const int t = P.t0 + it + 1;
      const double lr =
          P.total > 1 ? (double)P.lr0 + ((double)P.lr_end - (double)P.lr0) * (double)(t - 1) / (double)(P.total - 1)
                      : (double)P.lr0;
      adam_s[0] = (float)lr;
      adam_s[1] = (float)(1.0 / (1.0 - pow((double)P.beta1, (double)t)));
      adam_s[2] = (float)(1.0 / (1.0 - pow((double)P.beta2, (double)t)));
    }
    // inner minimisation of the last hidden layer from the constant coefficient -W_n^T c
    {
      const RLayer& Lt = P.L[n - 2];
      const int nt = Lt.n_out;
      float* xb = XB[(n - 1) & 1];
      for (int e = tid; e < ns * nt; e += kRThreads) {
        const int s = e / nt;
        const int j = e - s * nt;
        const size_t gi = (size_t)(b0 + s) * nt + j;
        float xbv, xv, val;
        inner_min<float>(Lt.rho[gi], P.gconst[gi], Lt.lo[gi], Lt.hi[gi], P.tau, xbv, xv, val);
        xb[s * P.xb_stride + j] = xbv;
      }
    }
    bsync();
    const float lr = adam_s[0], ibc1 = adam_s[1], ibc2 = adam_s[2];

    for (int k = n - 1; k >= 1; --k) {
      const RLayer& L = P.L[k - 1];
      const int nin = L.n_in, nout = L.n_out;
      const float* rho_k = L.rho + (size_t)b0 * nout;
      // (1) g_{k-1} = W_k^T rho_k -> GX
      if (L.kind == 1) {
        const Img I = img_of(*L.tr);
        img_border_zero(I, IMG, P.img_stride, ns, tid);
        for (int e = tid; e < ns * nout; e += kRThreads) {
          const int s = e / nout;
          const int j = e - s * nout;
          IMG[s * P.img_stride + img_pos(I, j)] = rho_k[(size_t)s * nout + j];
        }
        stage_weights<BF>(L.tr, L.n_tr, L.neff_tr, L.kpm_tr, WB, tid);
        bsync();
        r_conv_tn<BF>(L.tn_tr, L.tr, L.n_tr, L.neff_tr, L.kpm_tr, WB, IMG, P.img_stride, GX, P.gx_stride, ns, wave,
                      lane);
      } else {
        r_fc<BF>(*L.tr, L.kc_tr, rho_k, (size_t)nout, ns, S, GX, P.gx_stride, PART, wave, lane, tid);
      }
      bsync();
      // (2) inner minimisation of P_{k-1}: x*_{k-1} into IMG (layout of W_k's forward
      //     input), xB*_{k-1} into XB; conv weights of the forward product staged meanwhile
      {
        const bool conv = L.kind == 1;
        Img I;
        if (conv) {
          I = img_of(*L.fwd);
          img_border_zero(I, IMG, P.img_stride, ns, tid);
          stage_weights<BF>(L.fwd, 1, L.neff_fwd, L.kpm_fwd, WB, tid);
        }
        if (k == 1) {
          if ((nin & 3) == 0) {
            for (int e4 = tid; e4 < (ns * nin) >> 2; e4 += kRThreads) {
              const int e = e4 << 2;
              const int s = e / nin;
              const int j = e - s * nin;
              const size_t gi = (size_t)(b0 + s) * nin + j;
              const float4 l4 = ldg4(P.l0 + gi), u4 = ldg4(P.u0 + gi);
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                const float gv = GX[s * P.gx_stride + j + q];
                IMG[s * P.img_stride + (conv ? img_pos(I, j + q) : j + q)] = gv >= 0.f ? f4(u4, q) : f4(l4, q);
              }
            }
          } else {
            for (int e = tid; e < ns * nin; e += kRThreads) {
              const int s = e / nin;
              const int j = e - s * nin;
              const size_t gi = (size_t)(b0 + s) * nin + j;
              const float gv = GX[s * P.gx_stride + j];
              IMG[s * P.img_stride + (conv ? img_pos(I, j) : j)] = gv >= 0.f ? P.u0[gi] : P.l0[gi];
            }
          }
        } else {
          const RLayer& Lp = P.L[k - 2];
          float* xb = XB[(k - 1) & 1];
          if ((nin & 3) == 0) {
            for (int e4 = tid; e4 < (ns * nin) >> 2; e4 += kRThreads) {
              const int e = e4 << 2;
              const int s = e / nin;
              const int j = e - s * nin;
              const size_t gi = (size_t)(b0 + s) * nin + j;
              const float4 r4 = ldg4(Lp.rho + gi), l4 = ldg4(Lp.lo + gi), u4 = ldg4(Lp.hi + gi);
#pragma unroll
              for (int q = 0; q < 4; ++q) {
                float xbv, xv, val;
                inner_min<float>(f4(r4, q), GX[s * P.gx_stride + j + q], f4(l4, q), f4(u4, q), P.tau, xbv, xv, val);
                xb[s * P.xb_stride + j + q] = xbv;
                IMG[s * P.img_stride + (conv ? img_pos(I, j + q) : j + q)] = xv;
              }
            }
          } else {
            for (int e = tid; e < ns * nin; e += kRThreads) {
              const int s = e / nin;
              const int j = e - s * nin;
              const size_t gi = (size_t)(b0 + s) * nin + j;
              float xbv, xv, val;
              inner_min<float>(Lp.rho[gi], GX[s * P.gx_stride + j], Lp.lo[gi], Lp.hi[gi], P.tau, xbv, xv, val);
              xb[s * P.xb_stride + j] = xbv;
              IMG[s * P.img_stride + (conv ? img_pos(I, j) : j)] = xv;
            }
          }
        }
      }
      bsync();
      // (3) xhat_A,k (without bias) = W_k x*_{k-1} -> GX
      if (L.kind == 1)
        r_conv_tn<BF>(L.tn_fwd, L.fwd, 1, L.neff_fwd, L.kpm_fwd, WB, IMG, P.img_stride, GX, P.gx_stride, ns, wave,
                      lane);
      else
        r_fc<BF>(*L.fwd, L.kc_fwd, IMG, (size_t)P.img_stride, ns, S, GX, P.gx_stride, PART, wave, lane, tid);
      bsync();
      // (4) supergradient and Adam ascent step on rho_k
      {
        const float* xb = XB[k & 1];
        const float b1 = P.beta1, b2 = P.beta2, eps = P.eps;
        if ((nout & 3) == 0) {
          for (int e4 = tid; e4 < (ns * nout) >> 2; e4 += kRThreads) {
            const int e = e4 << 2;
            const int s = e / nout;
            const int j = e - s * nout;
            const size_t gi = (size_t)(b0 + s) * nout + j;
            float4 m4 = ldg4(L.m + gi), v4 = ldg4(L.v + gi), r4 = ldg4(L.rho + gi);
            float mo[4], vo[4], ro[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
              const float sg =
                  xb[s * P.xb_stride + j + q] - (GX[s * P.gx_stride + j + q] + L.bias[(j + q) / L.out_hw]);
              mo[q] = b1 * f4(m4, q) + (1.f - b1) * sg;
              vo[q] = b2 * f4(v4, q) + (1.f - b2) * (sg * sg);
              ro[q] = f4(r4, q) + lr * (mo[q] * ibc1) * __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(vo[q] * ibc2) + eps);
            }
            stg4(L.m + gi, make_float4(mo[0], mo[1], mo[2], mo[3]));
            stg4(L.v + gi, make_float4(vo[0], vo[1], vo[2], vo[3]));
            stg4(L.rho + gi, make_float4(ro[0], ro[1], ro[2], ro[3]));
          }
        } else {
          for (int e = tid; e < ns * nout; e += kRThreads) {
            const int s = e / nout;
            const int j = e - s * nout;
            const size_t gi = (size_t)(b0 + s) * nout + j;
            const float sg = xb[s * P.xb_stride + j] - (GX[s * P.gx_stride + j] + L.bias[j / L.out_hw]);
            const float m = b1 * L.m[gi] + (1.f - b1) * sg;
            const float v = b2 * L.v[gi] + (1.f - b2) * (sg * sg);
            L.m[gi] = m;
            L.v[gi] = v;
            L.rho[gi] = L.rho[gi] + lr * (m * ibc1) * __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(v * ibc2) + eps);
          }
        }
      }
      bsync();
    }
  }
  if (blockIdx.x == 0 && tid == 0 && P.t_dev != nullptr) *P.t_dev = P.t0 + P.iters;
}

hipError_t launch_resident(const RPlan& plan, int grid, size_t lds_bytes, int mma_bf16, hipStream_t s) {
  if (lds_bytes > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(mma_bf16 ? (const void*)resident_kernel<true> : (const void*)resident_kernel<false>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
    if (e != hipSuccess) return e;
  }
  if (mma_bf16)
    hipLaunchKernelGGL(resident_kernel<true>, dim3(grid), dim3(kRThreads), lds_bytes, s, plan);
  else
    hipLaunchKernelGGL(resident_kernel<false>, dim3(grid), dim3(kRThreads), lds_bytes, s, plan);
  return hipGetLastError();
}

}  // namespace ld
