// Internal declarations shared by the kernel and host translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace ld {

typedef uint16_t bf16_t;   // raw bfloat16 bits

// ---------------------------------------------------------------------------
// A contraction  C[m, n] = sum_k A[m, k] * B[k, n]  whose A operand is gathered
// from an activation tensor (implicit GEMM).  Rows m enumerate (subdomain, y', x')
// positions; the source element of (m, k) sits at spatial position
// (y'*iy_mul + iy_off + dky[k], x'*ix_mul + ix_off + dkx[k]) of channel plane
// chan_off[k]; out-of-range positions read as zero (zero padding).  Output
// column n of row m is neuron n*dst_HW + (y'*oy_mul+oy_off)*dst_W + (x'*ox_mul+ox_off)
// of the destination layer.  Fully-connected layers use 1x1 geometry.
// ---------------------------------------------------------------------------
struct GemmGeom {
  int M;               // rows = B * HWq
  int HWq, Wq;         // rows per subdomain, row width
  int iy_mul, iy_off, ix_mul, ix_off;
  int src_H, src_W;    // spatial size of the source plane
  int src_n;           // source elements per subdomain
  int K, Kp;           // reduction length; padded length (multiple of 64)
  const int4* ktab;    // [Kp] (chan_off, dky, dkx, 0)
  int N, Np;           // output columns; padded (multiple of 128)
  const float* Bf;     // [Np][Kp] FP32 operand, column-major in k ("n-major")
  const bf16_t* Bh;    // [Np][Kp] BF16 operand
  const bf16_t* Bhl;   // [Np][Kp] BF16 remainder Bf - Bh (compensated BF16 products)
  int dst_n;           // destination elements per subdomain
  int dst_HW, dst_W;
  int oy_mul, oy_off, ox_mul, ox_off;
  int m_fast;          // 1: epilogue walks rows fastest (conv), 0: columns fastest (FC)
  // zero-padded copy of one subdomain's source map in LDS (conv jobs):
  // [src_n / (src_H*src_W)] x LH x LW with the map at offset (pad_t, pad_l)
  int pad_t, pad_l, LH, LW;
  const int* ktab_lds; // [Kp] offset of each k in the channel-major padded map (c*LH*LW + dky*LW + dkx;
                       // the resident engine's map); 0 for padding channels
  // conv: k is ordered (tap, channel) with the channels padded to a multiple of 4
  // (zero weights); the layer-wise gather kernel keeps the map channel-last,
  // [LH][LW][CP] floats (CP >= the padded channel count), so each 4 consecutive k
  // are contiguous in it
  int CP;
  const int* ktab_cl;  // [Kp] offset of each k in the channel-last map ((dky*LW + dkx)*CP + c)
};

// Epilogue selector (what is done with each accumulated value).
enum EpiKind : int {
  EPI_STORE = 0,        // out_f[idx] = scale * acc
  EPI_P0 = 1,           // box minimiser of P_0 (eq:box_bounds_sol): x0* and its value
  EPI_INNER_MIN = 2,    // ReLU-hull vertex minimiser of P_k (eq:min-pk): x*, xB*, value
  EPI_ADAM = 3,         // supergradient xB - (acc + b) and Adam ascent step on rho
  EPI_SUPERGRAD = 4,    // supergradient xB - (acc + b) stored
  EPI_CROWN = 5,        // CROWN dual: a_up [g]_+ + a_lo [g]_-
  EPI_RELU_FWD = 6,     // y = acc + b, feasibility against [l, u], x = relu(y)
  EPI_BIAS_STORE = 7,   // y = acc + b stored
  EPI_ADAM_LAST = 8,    // as EPI_ADAM for the last hidden layer: xB from the constant g (gc)
  EPI_WK = 9            // WK dual: chord slope times g
};

struct EpiArgs {
  int kind;
  int xs_bf16;          // x* written as BF16 (1) or FP32 (0)
  float scale;
  float tau;            // tie band
  int want_val;         // write FP64 per-neuron values
  float* out_f;         // EPI_STORE / EPI_SUPERGRAD / EPI_CROWN / EPI_WK / EPI_RELU_FWD / EPI_BIAS_STORE
  void* xs;             // x* (float or bf16)
  float* xb;            // xB*
  double* val;          // per-neuron FP64 values
  const float* rho;     // dual of the destination layer
  const float* lo;      // lower bounds (l_k or l_0)
  const float* hi;      // upper bounds
  const float* bias;    // bias of the destination layer, index column / bias_div
  int bias_div;
  const float* xb_in;   // xB* read by the forward epilogues
  float* rho_w;         // Adam: rho, m, v (in/out)
  float* m;
  float* v;
  const float* adam;    // device scalars {lr_t, 1/bc1, 1/bc2, eps, beta1, beta2}
  int* flag;            // feasibility flags [B] (EPI_RELU_FWD)
  const float* gc;      // constant coefficient -W_n^T c of the last hidden layer (EPI_ADAM_LAST)
  // step bookkeeping done by one thread of the launch when t_dev != nullptr:
  // t += 1 and the scalars of that Adam step are written to adam_w
  int* t_dev;
  float* adam_w;
  double lr0, lr_end, beta1, beta2, eps;
  int total;
  // lo/hi rows shared by row_div consecutive subdomains (1: one row per subdomain):
  // the bounds of subdomain b are row b / row_div, rows of lohi_len floats (the
  // destination width, set by the launcher)
  int row_div;
  int lohi_len;
};

// Launch-time configuration of one contraction: tn 16-column MFMA tiles per wave;
// fully-connected: wm waves of a block along subdomains (16 each), K split over
// tm waves of the block and over `splits` blocks; transposed strided convs: the
// form (0: dense GEMM + col2im, 1: stride-class gather).
struct Tile {
  int tm, tn, splits, form, wm;
};

// Scratch of split-K launches: partial tiles and one arrival counter per tile
// (zero before the first launch; the last block of a tile resets it).
struct SplitArgs {
  int splits;
  float* partial;
  int* counters;
};

// ---------------------------------------------------------------------------
// Resident ascent (ld_resident.hip): one block owns S subdomains for a whole
// call of ld_step; intermediates live in LDS, the state streams once per
// iteration, and the layers are swept top-down inside each iteration.
// ---------------------------------------------------------------------------
constexpr int kMaxLayers = 15;

struct RLayer {
  int kind;             // 0 linear, 1 conv
  int n_in, n_out;      // widths of the layer's input and output
  int out_hw;           // output H*W (conv) or 1: bias index = neuron / out_hw
  const float* bias;
  const GemmGeom* fwd;  // device copies of the contraction geometries
  const GemmGeom* tr;
  int n_tr;
  int tn_fwd, tn_tr;    // column tiles (x16) of the conv contractions
  int kc_fwd, kc_tr;    // K chunks of the FC contractions (partials summed in order)
  int neff_fwd, neff_tr;  // weight rows staged in LDS (conv): columns rounded to the tile
  int kpm_fwd, kpm_tr;    // padded K row stride of the staged weights (max over classes)
  // hidden layer k = this index + 1 (k <= n-1): state and bounds of the batch
  float* rho;
  float* m;
  float* v;
  const float* lo;
  const float* hi;
};

struct RPlan {
  int n, B, S, n0;
  const float* l0;
  const float* u0;
  const float* gconst;  // [B, n_{n-1}]
  // LDS regions (floats): per subdomain xB (even layers at 0, odd layers at
  // xb_odd), x* image, contraction output; per block the staged conv weights,
  // aliased with the FC chunk partials
  int xb_stride, xb_odd, img_stride, gx_stride, wb_floats, part_floats;
  int t0, iters, total;
  float lr0, lr_end, beta1, beta2, eps, tau;
  int* t_dev;           // receives t0 + iters at the end of the launch
  RLayer L[kMaxLayers];
};

// ---------------------------------------------------------------------------
// Transposed strided convolution as one dense GEMM followed by a col2im sum:
//   Y[m][n] = sum_co rho[co][m] W[co][n],  m = (oy, ox) position of rho, n = (ci, ky, kx),
//   g[ci][y][x] = sum of Y[(oy, ox)][(ci, ky, kx)] over the taps with oy*s - p + ky = y
//   and ox*s - p + kx = x.
// The reduction is over the Co channels of rho only, every product is a useful one
// (no stride-class padding), and the A operand is read contiguously.  Input
// channels are processed in chunks of Cc so that the Y chunk fits in LDS.
// ---------------------------------------------------------------------------
struct ColGeom {
  int Co, M;              // reduction length (channels of rho); positions of rho (OH*OW)
  int Ci, H, W, HW;       // destination map (the forward layer's input)
  int khkw;               // taps per channel
  int Cc, nchunks, ntc;   // channels per chunk, chunks, 16-column tiles per chunk
  int Ns, Mp;             // LDS row stride of the Y chunk (odd, > 16*ntc); rows (M rounded up to 16)
  int Tmax;               // taps reaching one output row (column) at most
  int ksf, ksh;           // K steps: FP32 (16 deep), BF16 (32 deep)
  float inv_HW, inv_W;    // 1/HW, 1/W for the index split of the epilogue
  const float* Bf;        // FP32 fragments [nchunks][ntc][ksf][64 lanes][4]
  const bf16_t* Bh;       // BF16 fragments [nchunks][ntc][ksh][64 lanes][8]
  // tap tables, one contiguous array of ntab ints:
  //   toff_y [H][Tmax] (oy*OW*Ns + ky*kw), cnt_y [H], toff_x [W][Tmax] (ox*Ns + kx), cnt_x [W]
  const int* tab;
  int ntab;
};
// LDS of one convT block: half a CU (two subdomains resident per CU), a whole CU
constexpr size_t kConvTHalfCU = 80 * 1024, kConvTWholeCU = 160 * 1024;
// split: one block per (subdomain, channel chunk) instead of one per subdomain
hipError_t launch_convT(const ColGeom& g, int B, const float* rho, int mma_bf16, const EpiArgs& e, int split,
                        hipStream_t s);
size_t convT_lds_bytes(const ColGeom& g, int split);

// The plan travels by value in the kernel arguments (no host-device race between calls).
hipError_t launch_resident(const RPlan& plan, int grid, size_t lds_bytes, int mma_bf16, hipStream_t s);

// kernels (ld_kernels.hip)
// convolution contraction, `parts` blocks per subdomain (bands of destination rows)
// geo_dev: device copy of the same class geometries (read into LDS by the kernel)
hipError_t launch_conv(const GemmGeom* geoms, const GemmGeom* geo_dev, int n_classes, int B, const void* src,
                       int src_bf16, int mma_bf16, const EpiArgs& e, int tn, int parts, hipStream_t s);
size_t conv_lds_bytes(const GemmGeom* g, int n_classes, int tn, int mma_bf16, int parts);
// fully-connected contraction (G.M = B rows), optional split-K
hipError_t launch_fc(const GemmGeom& g, const void* src, int src_bf16, int mma_bf16, const EpiArgs& e,
                     int tn, const SplitArgs& sp, int wm, int kw, hipStream_t s);

hipError_t launch_inner_min_const(int B, int n, const float* g, const float* rho, const float* lo,
                                  const float* hi, const float* bias, int bias_hw, float tau, float* xb,
                                  double* val, int* t_dev, float* adam_scalars, double lr0,
                                  double lr_end, int total, double beta1, double beta2, double eps,
                                  int row_div, hipStream_t s);
hipError_t launch_crown_const(int B, int n, const float* g, const float* lo, const float* hi,
                              float* rho, int wk, int row_div, hipStream_t s);
hipError_t launch_reduce_q(int B, int n_arrays, const double* const* arrays, const int* sizes,
                           const double* cb, double* q, hipStream_t s);
hipError_t launch_cdot(int B, int n, const float* c, const float* y, const float* bias, int bias_div, double* out,
                       hipStream_t s);
hipError_t launch_validate(int B, int n, const float* lo, const float* hi, int* bad, hipStream_t s);
hipError_t launch_fill_f32(float* p, size_t n, float v, hipStream_t s);
hipError_t launch_fill_i32(int* p, size_t n, int v, hipStream_t s);
hipError_t launch_fill_f64(double* p, size_t n, double v, hipStream_t s);
hipError_t launch_copy_f32(float* dst, const float* src, size_t n, hipStream_t s);
hipError_t launch_max_f64(int B, const double* a, const double* b, double* out, hipStream_t s);
// best_q[b], best_t[b] <- q[b], *step where q[b] > best_q[b]
hipError_t launch_best_update(int B, const double* q, double* best_q, int* best_t, const int* step, hipStream_t s);
// *c += 1 (one thread)
hipError_t launch_inc_i32(int* c, hipStream_t s);

// proximal solver (ld_prox.hip).  One block of the block-coordinate Frank-Wolfe
// sweep, layer k: B part over layer k (nB = n_k, 0 for k = 0), A part over layer
// k+1 (nA = n_{k+1}); `last` when k+1 = n (the objective layer: coefficient -c,
// no proximal term, no next block).  All arrays are [B, width] row-major.
struct ProxBlockArgs {
  int nB, nA, last, z_bf16;
  float inv_eta, tau;
  double inv_eta_d;
  // last sweep of an outer iteration: layer k's dual update with momentum
  // (piB in/out, rhoB written) and rt_k for the next iteration's eta
  int dual;
  float mu, inv_eta_next;
  float* piB;
  // layer k: iterate xB_k (in/out), conditional gradient zB_k, coefficient rt_k
  // (in/out), dual rho_k, iterate xA_k (already moved by the previous block)
  float* xB;
  const float* zB;
  float* rtB;
  const float* rhoB;
  const float* xAB;
  // layer k+1: iterate xA_{k+1} (in/out), its conditional gradient zA_{k+1};
  // not last: rt_{k+1} (out), rho_{k+1}, xB_{k+1}; last: objective c
  float* xA;
  const float* zA;
  float* rtA;
  const float* rhoA;
  const float* xBA;
  const float* c;
  // conditional gradient of block k+1 (not last): g_{k+1} = W_{k+2}^T rt_{k+2},
  // bounds of layer k+1, outputs zB_{k+1} (FP32) and z_{k+1} (operand precision)
  const float* g;
  const float* lo;
  const float* hi;
  float* zB_out;
  void* z_out;
};
// the hidden layers of one launch computing rt = rho + (xB - xA) / eta
constexpr int kProxPackMax = 16;
struct ProxDualPack {
  int n;
  const float* rho[kProxPackMax];
  const float* xB[kProxPackMax];
  const float* xA[kProxPackMax];
  float* rt[kProxPackMax];
  size_t cnt[kProxPackMax];
};
hipError_t launch_prox_block(const ProxBlockArgs& a, int B, hipStream_t s);
hipError_t launch_prox_coeff(const ProxDualPack& p, float inv_eta, hipStream_t s);
hipError_t launch_relu_operand(size_t n, const float* xb, void* out, int bf16, hipStream_t s);

// intermediate bounds (ld_interm.hip): the per-subdomain arrays copied into the
// expanded batch (l_0, u_0, then l_k, u_k of the sub-network's hidden layers)
constexpr int kIntermMaxArrays = 66;
struct IntermPack {
  int n;
  const float* src[kIntermMaxArrays];
  float* dst[kIntermMaxArrays];
  int width[kIntermMaxArrays];
  float* c;
};
hipError_t launch_interm_expand(const IntermPack& K, int C, long long start, int P, int nj, hipStream_t s);
// sigmoid activations (ld_sigmoid.hip): hull tangent points, inner minimisation
hipError_t launch_sigmoid_hull(long long n, const float* l, const float* u, float* t_up, float* t_lo, hipStream_t s);
hipError_t launch_sigmoid_inner_min(long long n, const float* rho, const float* g, const float* l, const float* u,
                                    const float* t_up, const float* t_lo, float* xb, float* x, double* val,
                                    hipStream_t s);

// branching (ld_fsb.hip); at most kFsbMaxHidden hidden layers
constexpr int kFsbMaxHidden = 16;
hipError_t launch_fsb_scores(int B, int n_hidden, const float* const* lam, const float* const* lo,
                             const float* const* hi, const float* const* bias, const int* bias_div,
                             const int* width, int* cand, hipStream_t s);
hipError_t launch_fsb_expand(const IntermPack& K, int B, int n_hidden, const int* cand, float* const* lo_child,
                             float* const* hi_child, const int* width, hipStream_t s);
hipError_t launch_branch_children(const IntermPack& K, int B, int n_hidden, const int* layer, const int* index,
                                  float* const* lo_child, float* const* hi_child, const int* width, hipStream_t s);
hipError_t launch_fsb_select(int B, int n_hidden, const int* cand, const double* q_crown, const double* q_wk,
                             int* layer, int* index, double* value, hipStream_t s);
hipError_t launch_interm_collect(int C, long long start, int P, int nj, const double* bound, float* lo, float* hi,
                                 hipStream_t s);
// branch and bound (ld_bab.hip): for each of `count` pairs, row pairs[p].x of every
// array of K (row 0 with broadcast) to row pairs[p].y of its destination
hipError_t launch_bab_rows(const IntermPack& K, const int2* pairs, int count, int broadcast, hipStream_t s);

// ---------------------------------------------------------------------------
// FP64 engine (ld_fp64.hip): direct FP64 contractions with fused epilogues.
// ---------------------------------------------------------------------------
struct F64Layer {
  int kind;                        // 0 linear, 1 conv
  int Ci, H, W_, Co, Ho, Wo;       // input and output maps (linear: Ci = n_in, Co = n_out, 1x1)
  int kh, kw, stride, pad;
  int n_in, n_out;
  const double* W;                 // conv [Co][Ci][kh][kw]; linear [n_out][n_in]
  const double* WT;                // linear: [n_in][n_out] (coalesced forward products)
};

enum F64EpiKind : int {
  F64_STORE = 0,      // out = scale * acc
  F64_P0 = 1,         // box minimiser of P_0: xs, val = -(g x0*)
  F64_INNER = 2,      // ReLU-hull minimiser of P_k: xb, xs, val = min - rho*b
  F64_CROWN = 3,      // CROWN (or WK, wk = 1) dual from g
  F64_ADAM = 4,       // supergradient xb_in - (acc + b) and the Adam ascent step
  F64_SUPERGRAD = 5,  // supergradient stored (out and/or out_f)
  F64_RELU_FWD = 6,   // y = acc + b, feasibility of y against [lo, hi], out = relu(y)
  F64_BIAS = 7        // out = acc + b
};

struct F64Epi {
  int kind;
  int wk;
  int bias_div;       // neuron index / bias_div = bias index
  double scale;
  double tau;
  const double* rho;  // dual of the epilogue's layer (F64_INNER)
  const float* lo;    // bounds of the epilogue's layer (l_0, u_0 for F64_P0)
  const float* hi;
  const double* bias;
  double* xb;
  double* xs;
  double* val;
  double* out;
  float* out_f;
  const double* xb_in;
  double* rho_w;
  double* m;
  double* v;
  double lr, bc1, bc2, beta1, beta2, omb1, omb2, eps;  // Adam step (omb = 1 - beta)
  int* flag;
};

// g = W^T r fused with an epilogue over the n = L.n_in inputs of the layer, or the
// epilogue alone on g = gin (n values per subdomain).
hipError_t launch_f64_transposed(const F64Layer& L, int B, const double* r, const double* gin, int n,
                                 const F64Epi& e, hipStream_t s);
hipError_t launch_f64_forward(const F64Layer& L, int B, const double* x, const F64Epi& e, hipStream_t s);
// out[b][j] = (gamma * (|W|^T |r|)[b][j] + tiny) * xmax[b][j]; xmax = max(|lo|, |hi|) (box) or max(0, hi)
hipError_t launch_f64_abs_margin(const F64Layer& L, int B, const float* r, int n, const float* lo, const float* hi,
                                 int box, double gamma, double tiny, double* out, hipStream_t s);
hipError_t launch_f64_widen(size_t n, const float* src, double* dst, hipStream_t s);
hipError_t launch_f64_narrow(size_t n, const double* src, float* dst, hipStream_t s);
hipError_t launch_f64_copy(size_t n, const double* src, double* dst, hipStream_t s);
hipError_t launch_f64_cdot(int B, int n, const float* c, const double* y, double* out, hipStream_t s);

}  // namespace ld
