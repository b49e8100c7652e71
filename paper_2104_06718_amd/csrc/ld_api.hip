// Host side of the C ABI declared in include/ld.h.
//
// Builds the contraction plan of a network (forward and stride-class transposed
// implicit GEMMs per layer, packed FP32/BF16 weight operands), validates
// arguments, owns device workspaces, and sequences the kernels of one ascent
// iteration:
//   phase A  (Algorithm 1, inner minimisation): g_{k-1} = W_k^T rho_k for every
//            hidden layer k, each fused with the P_{k-1} minimisation
//            (P_0: eq:box_bounds_sol; P_k: eq:min-pk); the last hidden layer
//            uses the constant g_{n-1} = -W_n^T c.
//   phase B  (supergradient step): xhat_A,k = W_k x*_{k-1} + b_k fused with
//            s_k = xhat_B,k - xhat_A,k and the Adam ascent step on rho_k.
// The iterations of ld_step are captured once into a HIP graph and replayed.
#include "ld.h"
#include "ld_internal.h"

#include <chrono>
#include <cmath>
#include <cstring>
#include <array>
#include <functional>
#include <map>
#include <queue>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

using namespace ld;

namespace {

thread_local std::string g_err;
thread_local int g_validate = 1;
// Subdomains that share one row of the batch's bounds (l_0, u_0, l_k, u_k): the
// intermediate-bound problems of one subdomain read its rows in place (1: one row
// per subdomain).  Set only around the internal calls of ld_intermediate_bounds.
thread_local int g_row_div = 1;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define LD_HIP(expr)                                                                               \
  do {                                                                                             \
    hipError_t e_ = (expr);                                                                        \
    if (e_ != hipSuccess) return fail(LD_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

#define LD_TRY(expr)          \
  do {                        \
    int rc_ = (expr);         \
    if (rc_ != LD_OK) return rc_; \
  } while (0)

size_t round_up(size_t x, size_t m) { return (x + m - 1) / m * m; }

uint16_t host_f2bf(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
float host_bf2f(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

// One contraction of a layer: one GemmGeom per stride class (M is set per launch).
struct Job {
  std::vector<GemmGeom> geoms;
  const GemmGeom* dev = nullptr;  // device copy of geoms
  bool has_col = false;   // transposed strided conv: dense GEMM + col2im form
  ColGeom col;
  // the same form with more, smaller channel chunks looped in one block (LDS within a
  // quarter of a CU), for the BF16 operands: such a block shares a CU with the
  // compensated products of the phase's other layers
  bool has_col_q = false;
  ColGeom col_q;
  // the same form with one block per (subdomain, channel chunk), for several chunk counts
  std::vector<ColGeom> col_split;
};

struct Layer {
  int kind;
  int in_c, in_h, in_w, out_c, out_h, out_w, kh, kw, stride, pad;
  int n_in, n_out;
  float* bias = nullptr;  // device [out_c]
  Job fwd, tr;
  const GemmGeom* fwd_dev = nullptr;  // device copies of the geometries (resident engine)
  const GemmGeom* tr_dev = nullptr;
  // FP64 engine: the weights as given (and W^T of a linear layer) and the bias, in FP64
  F64Layer f64;
  const double* b64 = nullptr;
};

// Buffers of an FP64 evaluation pipeline for a batch of B subdomains.
struct Workspace64 {
  int B = 0;
  void* base = nullptr;
  std::vector<double*> xs;   // x*_k, k = 0..n-1
  std::vector<double*> xb;   // xB*_k, index k = 1..n-1 (entry 0 unused)
  std::vector<double*> val;  // per-neuron values, k = 0..n-1 (layer k >= 1: minimum - rho_k b_k)
  std::vector<double*> rho;  // duals widened from FP32, hidden layers k = 1..n-1 at k-1
  double* c64 = nullptr;     // c widened [B, n_out]
  double* gconst = nullptr;  // -W_n^T c [B, n_{n-1}]
  double* cb = nullptr;      // c . b_n [B]
  double* act0 = nullptr;    // forward-pass activations [B, max width]
  double* act1 = nullptr;
  double* qtmp = nullptr;    // [B]
  int* flag = nullptr;       // [B]
};

// Buffers of one evaluation pipeline for a batch of B subdomains.
struct Workspace {
  int B = 0;
  void* base = nullptr;
  std::vector<void*> xs;      // x*_k, k = 0..n-2 (FP32-sized; BF16 uses the first half)
  std::vector<float*> xb;     // xB*_k, index k = 1..n-1 (entry 0 unused)
  std::vector<double*> val;   // per-neuron FP64 values, k = 0..n-1
  float* gconst = nullptr;    // -W_n^T c   [B, n_{n-1}]
  double* cb = nullptr;       // c . b_n    [B]
  float* act0 = nullptr;      // forward-pass activations [B, max width]
  float* act1 = nullptr;
  double* qtmp = nullptr;     // [B]
  int* flag = nullptr;        // [B]
  int* bad = nullptr;         // [1]
  float* partial = nullptr;   // split-K partial tiles, kPartialLayer floats per layer
  int* counters = nullptr;    // split-K arrival counters (kept at zero between launches)
};

constexpr size_t kPartialLayer = (size_t)2 << 20;  // split-K partial floats per layer (8 MiB)
constexpr size_t kCounterCap = (size_t)1 << 16;

}  // namespace

struct ld_net {
  int n = 0;
  int n0 = 0;
  int max_width = 0;
  std::vector<Layer> L;
  std::vector<void*> allocs;
  Workspace ws;
  // autotuned launch configurations: (layer, dir, B, mma) -> tile and its time (us)
  std::map<std::tuple<int, int, int, int>, Tile> tiles;
  std::map<std::tuple<int, int, int, int>, double> tile_us;
  // autotuned engine: (B, mma) -> {engine, us per iteration layer-wise (graph replay),
  // resident (0: does not fit)}
  std::map<std::pair<int, int>, std::array<double, 3>> engines;
  int tune_gen = 0;  // bumped whenever a tuned choice changes (part of the graph key)
  std::mutex mu;
  Workspace64 ws64;  // FP64 dual evaluations (ld_dual_eval with LD_FP64, ld_init_duals)
  // buffers of the branching pipeline, kept between calls (grown, never shrunk)
  struct FsbBuffers {
    void* base = nullptr;
    size_t bytes = 0;
    Workspace ws;
    std::mutex mu;  // one branching call on the net at a time
  } fsb;
};

struct ld_state {
  const ld_net* net = nullptr;
  int B = 0;
  void* base = nullptr;
  std::vector<float*> rho, m, v;  // hidden layers k = 1..n-1 at index k-1
  int* t_dev = nullptr;
  float* adam = nullptr;          // 8 floats
  double* q0 = nullptr;
  bool initialized = false;
  Workspace ws;
  // stream on which the graphs are captured (no work is ever enqueued on it)
  hipStream_t cap = nullptr;
  // captured ascents of ld_step: graphs of `chunk` iterations each, keyed by the
  // batch pointers, options and tuned configuration (one for the full chunks of a
  // call, one for its remainder)
  struct Graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<double> key;
  };
  Graph graphs[2];
  int t_host = 0;       // Adam steps enqueued so far (mirrors *t_dev)
  // the ascent's best dual value (ld_state_set_tracking): per subdomain the largest
  // q(rho^{t-1}) of the tracked steps t and that t (device [B])
  bool track = false;
  void* track_base = nullptr;
  double* best_q = nullptr;
  int* best_t = nullptr;
  int* track_step = nullptr;  // the state's step count, advanced by each tracked step
  Workspace tws;              // the tracked values' own evaluation buffers
  // recorded after the last work enqueued on the state's memory and graphs; waited
  // on before a graph is replaced or the state is freed (a graph exec or a
  // buffer must not be released while kernels that use it are in flight)
  hipEvent_t done = nullptr;
  // FP64 engine (allocated by its first call): duals and Adam moments in FP64;
  // `active` when the state was initialised by an FP64 ld_step (its duals are
  // then these, and ld_final_bound evaluates in FP64)
  struct F64 {
    void* base = nullptr;
    std::vector<double*> rho, m, v;  // hidden layers k = 1..n-1 at k-1
    double* q0 = nullptr;
    Workspace64 ws;
    bool active = false;
    int t = 0;
  } f64;
  // proximal solver (allocated by its first call): primal iterates xB_k (k = 1..n-1
  // at k-1), xA_k (k = 1..n at k-1), coefficients rt_k and momentum pi_k (k-1),
  // transposed products g_k (k = 1..n-2 at k), the forward product of the current
  // block zA (widest layer) and the operand z_{n-1} of the objective layer
  struct Prox {
    void* base = nullptr;
    std::vector<float*> xB, xA, rt, pi, g;
    float* zA = nullptr;
    void* zlast = nullptr;
    bool ready = false;  // primal iterates hold a start point (set by the first call)
    int mma = -1;        // operand precision the start point was formed with
    int t = 0;           // outer iterations done
  } px;
};

namespace {

// ---------------------------------------------------------------------------
// plan construction
// ---------------------------------------------------------------------------
int alloc_dev(ld_net* net, void** p, size_t bytes) {
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) return fail(LD_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  net->allocs.push_back(*p);
  return LD_OK;
}

// Pack an [N][K] operand (column n holds the K weights reducing into output n),
// zero padded to [Np][Kp], in FP32 and BF16, plus the gather table.
int finish_geom(ld_net* net, GemmGeom& g, const std::vector<float>& Bnk, const std::vector<int4>& ktab) {
  g.Kp = (int)round_up((size_t)std::max(g.K, 1), 64);
  g.Np = (int)round_up((size_t)std::max(g.N, 1), 128);
  std::vector<float> bf((size_t)g.Np * g.Kp, 0.f);
  std::vector<uint16_t> bh((size_t)g.Np * g.Kp, 0), bl((size_t)g.Np * g.Kp, 0);
  for (int n = 0; n < g.N; ++n)
    for (int k = 0; k < g.K; ++k) {
      const float w = Bnk[(size_t)n * g.K + k];
      const uint16_t h = host_f2bf(w);
      bf[(size_t)n * g.Kp + k] = w;
      bh[(size_t)n * g.Kp + k] = h;
      bl[(size_t)n * g.Kp + k] = host_f2bf(w - host_bf2f(h));  // exact difference, rounded to BF16
    }
  std::vector<int4> kt((size_t)g.Kp, int4{0, 0, 0, 0});
  for (int k = 0; k < g.K; ++k) kt[k] = ktab[k];
  if (g.LH > 0) {
    // offsets into the zero-padded LDS image [C][LH][LW]; padded k read offset 0 (weight is 0)
    std::vector<int> kl((size_t)g.Kp, 0);
    for (int k = 0; k < g.K; ++k) {
      const int c = ktab[k].x / (g.src_H * g.src_W);
      // .w marks a padding channel of the channel-last order (weight 0): offset 0
      kl[k] = ktab[k].w ? 0 : c * g.LH * g.LW + ktab[k].y * g.LW + ktab[k].z;
    }
    void* pl;
    LD_TRY(alloc_dev(net, &pl, kl.size() * 4));
    LD_HIP(hipMemcpy(pl, kl.data(), kl.size() * 4, hipMemcpyHostToDevice));
    g.ktab_lds = (const int*)pl;
    if (g.CP > 0) {
      std::vector<int> kc((size_t)g.Kp, 0);
      for (int k = 0; k < g.K; ++k) {
        const int c = ktab[k].x / (g.src_H * g.src_W);
        kc[k] = (ktab[k].y * g.LW + ktab[k].z) * g.CP + c;
      }
      void* pc;
      LD_TRY(alloc_dev(net, &pc, kc.size() * 4));
      LD_HIP(hipMemcpy(pc, kc.data(), kc.size() * 4, hipMemcpyHostToDevice));
      g.ktab_cl = (const int*)pc;
    }
  }
  void *pf, *ph, *phl, *pk;
  LD_TRY(alloc_dev(net, &pf, bf.size() * 4));
  LD_TRY(alloc_dev(net, &ph, bh.size() * 2));
  LD_TRY(alloc_dev(net, &phl, bl.size() * 2));
  LD_TRY(alloc_dev(net, &pk, kt.size() * sizeof(int4)));
  LD_HIP(hipMemcpy(pf, bf.data(), bf.size() * 4, hipMemcpyHostToDevice));
  LD_HIP(hipMemcpy(ph, bh.data(), bh.size() * 2, hipMemcpyHostToDevice));
  LD_HIP(hipMemcpy(phl, bl.data(), bl.size() * 2, hipMemcpyHostToDevice));
  LD_HIP(hipMemcpy(pk, kt.data(), kt.size() * sizeof(int4), hipMemcpyHostToDevice));
  g.Bf = (const float*)pf;
  g.Bh = (const bf16_t*)ph;
  g.Bhl = (const bf16_t*)phl;
  g.ktab = (const int4*)pk;
  return LD_OK;
}

// Channel-last LDS map of a conv source with C channels: channels padded to a
// multiple of 4 in k, pixel stride CP floats (C + 4 when C is a multiple of 8,
// which spreads a row's pixels over the LDS banks; else the padded count)
int cl_channels(int C) { return (C + 3) / 4 * 4; }
int cl_stride(int C) { return C % 8 == 0 ? C + 4 : cl_channels(C); }

GemmGeom base_geom() {
  GemmGeom g;
  std::memset(&g, 0, sizeof(g));
  g.HWq = 1;
  g.Wq = 1;
  g.src_H = 1;
  g.src_W = 1;
  g.dst_HW = 1;
  g.dst_W = 1;
  return g;
}

int build_linear(ld_net* net, Layer& L, const float* W) {
  const int ni = L.n_in, no = L.n_out;
  // forward: rows = subdomains, columns = output neurons, k = input neuron
  {
    GemmGeom g = base_geom();
    g.src_n = ni;
    g.K = ni;
    g.N = no;
    g.dst_n = no;
    g.m_fast = 0;
    std::vector<float> Bnk((size_t)no * ni);
    std::vector<int4> kt(ni);
    for (int o = 0; o < no; ++o)
      for (int i = 0; i < ni; ++i) Bnk[(size_t)o * ni + i] = W[(size_t)o * ni + i];
    for (int i = 0; i < ni; ++i) kt[i] = int4{i, 0, 0, 0};
    LD_TRY(finish_geom(net, g, Bnk, kt));
    L.fwd.geoms = {g};
  }
  // transposed: columns = input neurons, k = output neuron
  {
    GemmGeom g = base_geom();
    g.src_n = no;
    g.K = no;
    g.N = ni;
    g.dst_n = ni;
    g.m_fast = 0;
    std::vector<float> Bnk((size_t)ni * no);
    std::vector<int4> kt(no);
    for (int i = 0; i < ni; ++i)
      for (int o = 0; o < no; ++o) Bnk[(size_t)i * no + o] = W[(size_t)o * ni + i];
    for (int o = 0; o < no; ++o) kt[o] = int4{o, 0, 0, 0};
    LD_TRY(finish_geom(net, g, Bnk, kt));
    L.tr.geoms = {g};
  }
  return LD_OK;
}

// Transposed product of a strided conv as Y = rho^T W (K = Co) plus a col2im sum
// over the taps (ColGeom).  Stride-1 convs, and maps whose Y chunk would not fit
// a modest LDS budget, keep the gather form.
int build_col(ld_net* net, Layer& L, const float* W) {
  const int Ci = L.in_c, H = L.in_h, Wd = L.in_w, Co = L.out_c, OH = L.out_h, OW = L.out_w;
  const int kh = L.kh, kw = L.kw, s = L.stride, p = L.pad, khkw = kh * kw;
  if (s < 2) return LD_OK;
  if ((long)Ci * H * Wd >= (1L << 22)) return LD_OK;
  ColGeom g;
  std::memset(&g, 0, sizeof(g));
  g.Co = Co;
  g.M = OH * OW;
  g.Ci = Ci;
  g.H = H;
  g.W = Wd;
  g.HW = H * Wd;
  g.khkw = khkw;
  g.Mp = (int)round_up((size_t)g.M, 16);
  g.ksf = (Co + 15) / 16;
  g.ksh = (Co + 31) / 32;
  g.inv_HW = 1.0f / (float)g.HW;
  g.inv_W = 1.0f / (float)Wd;
  // taps reaching each output row / column: k = y + p - s*o for o in [0, OH)
  std::vector<std::vector<std::pair<int, int>>> tyv(H), txv(Wd);
  for (int y = 0; y < H; ++y)
    for (int ky = 0; ky < kh; ++ky) {
      const int t = y + p - ky;
      if (t >= 0 && t % s == 0 && t / s < OH) tyv[y].push_back({ky, t / s});
    }
  for (int x = 0; x < Wd; ++x)
    for (int kx = 0; kx < kw; ++kx) {
      const int t = x + p - kx;
      if (t >= 0 && t % s == 0 && t / s < OW) txv[x].push_back({kx, t / s});
    }
  int Tmax = 1;
  for (auto& v : tyv) Tmax = std::max(Tmax, (int)v.size());
  for (auto& v : txv) Tmax = std::max(Tmax, (int)v.size());
  g.Tmax = Tmax;
  g.ntab = H * Tmax + H + Wd * Tmax + Wd;
  // channel chunks: balanced, and as few as keep the block's LDS within half a
  // CU (two subdomains per CU), else within the whole CU
  auto with_chunks = [&](int nch) {
    ColGeom t = g;
    t.Cc = (Ci + nch - 1) / nch;
    t.nchunks = (Ci + t.Cc - 1) / t.Cc;
    t.ntc = (t.Cc * khkw + 15) / 16;
    t.Ns = 16 * t.ntc + 1;
    return t;
  };
  int pick = 0;
  for (int pass = 0; pass < 2 && !pick; ++pass)
    for (int nch = 1; nch <= Ci && !pick; ++nch) {
      const ColGeom t = with_chunks(nch);
      if (nch > 1 && t.Cc == with_chunks(nch - 1).Cc) continue;
      if (convT_lds_bytes(t, 0) <= (pass == 0 ? kConvTHalfCU : kConvTWholeCU)) pick = nch;
    }
  if (!pick) return LD_OK;  // keep the stride-class form
  // device arrays (weight fragments in chunk order, tap tables) of a chunking
  auto materialise = [&](ColGeom g, ColGeom* out) -> int {
    const int Cc = g.Cc;
    std::vector<int> tab((size_t)g.ntab, 0);
    int* toy = tab.data();
    int* coy = toy + (size_t)H * Tmax;
    int* tox = coy + H;
    int* cox = tox + (size_t)Wd * Tmax;
    for (int y = 0; y < H; ++y) {
      coy[y] = (int)tyv[y].size();
      for (int i = 0; i < coy[y]; ++i) toy[(size_t)y * Tmax + i] = tyv[y][i].second * OW * g.Ns + tyv[y][i].first * kw;
    }
    for (int x = 0; x < Wd; ++x) {
      cox[x] = (int)txv[x].size();
      for (int i = 0; i < cox[x]; ++i) tox[(size_t)x * Tmax + i] = txv[x][i].second * g.Ns + txv[x][i].first;
    }
    // B fragments: lane (r, q) of K step st holds W[k][n] for n = 16*nt + r and
    // k = st*KS + VPL*q + j (the k order inside a step matches the A operand)
    auto wv = [&](int c, int nt, int k, int r) -> float {
      const int nl = nt * 16 + r;
      const int ci = c * Cc + nl / khkw;
      if (nl >= Cc * khkw || ci >= Ci || k >= Co) return 0.f;
      return W[((size_t)k * Ci + ci) * khkw + nl % khkw];
  };
    std::vector<float> bf((size_t)g.nchunks * g.ntc * g.ksf * 64 * 4);
    std::vector<uint16_t> bh((size_t)g.nchunks * g.ntc * g.ksh * 64 * 8);
    for (int c = 0; c < g.nchunks; ++c)
      for (int nt = 0; nt < g.ntc; ++nt)
        for (int l = 0; l < 64; ++l) {
          const int r = l & 15, q = l >> 4;
          for (int st = 0; st < g.ksf; ++st)
            for (int j = 0; j < 4; ++j)
              bf[((((size_t)c * g.ntc + nt) * g.ksf + st) * 64 + l) * 4 + j] = wv(c, nt, st * 16 + 4 * q + j, r);
          for (int st = 0; st < g.ksh; ++st)
            for (int j = 0; j < 8; ++j)
              bh[((((size_t)c * g.ntc + nt) * g.ksh + st) * 64 + l) * 8 + j] = host_f2bf(wv(c, nt, st * 32 + 8 * q + j, r));
        }
    void *pbf, *pbh, *ptab;
    LD_TRY(alloc_dev(net, &pbf, bf.size() * 4));
    LD_TRY(alloc_dev(net, &pbh, bh.size() * 2));
    LD_TRY(alloc_dev(net, &ptab, tab.size() * 4));
    LD_HIP(hipMemcpy(pbf, bf.data(), bf.size() * 4, hipMemcpyHostToDevice));
    LD_HIP(hipMemcpy(pbh, bh.data(), bh.size() * 2, hipMemcpyHostToDevice));
    LD_HIP(hipMemcpy(ptab, tab.data(), tab.size() * 4, hipMemcpyHostToDevice));
    g.Bf = (const float*)pbf;
    g.Bh = (const bf16_t*)pbh;
    g.tab = (const int*)ptab;
    *out = g;
    return LD_OK;
  };
  LD_TRY(materialise(with_chunks(pick), &g));
  L.tr.col = g;
  L.tr.has_col = true;
  for (int nch = pick + 1; nch <= Ci && convT_lds_bytes(g, 0) > kConvTHalfCU / 2; ++nch) {
    const ColGeom t = with_chunks(nch);
    if (t.Cc == with_chunks(nch - 1).Cc || convT_lds_bytes(t, 0) > kConvTHalfCU / 2) continue;
    LD_TRY(materialise(t, &L.tr.col_q));
    L.tr.has_col_q = true;
    break;
  }
  // one block per chunk: 2, 3, 4 and 8 chunks (as the channels allow), each block's
  // LDS within a quarter of a CU
  L.tr.col_split.clear();
  for (int nch : {2, 3, 4, 8}) {
    if (nch > Ci) break;
    const ColGeom t = with_chunks(nch);
    if (t.nchunks <= pick || convT_lds_bytes(t, 1) > kConvTHalfCU / 2) continue;
    bool dup = false;
    for (const ColGeom& v : L.tr.col_split) dup |= v.nchunks == t.nchunks;
    if (dup) continue;
    ColGeom m;
    LD_TRY(materialise(t, &m));
    L.tr.col_split.push_back(m);
  }
  return LD_OK;
}

int build_conv(ld_net* net, Layer& L, const float* W) {
  const int Ci = L.in_c, H = L.in_h, Wd = L.in_w, Co = L.out_c, OH = L.out_h, OW = L.out_w;
  const int kh = L.kh, kw = L.kw, s = L.stride, p = L.pad;
  auto w_at = [&](int co, int ci, int ky, int kx) { return W[(((size_t)co * Ci + ci) * kh + ky) * kw + kx]; };
  // forward: rows (b, oy, ox), columns co, k = (ci, ky, kx)
  {
    GemmGeom g = base_geom();
    g.HWq = OH * OW;
    g.Wq = OW;
    g.iy_mul = s;
    g.iy_off = -p;
    g.ix_mul = s;
    g.ix_off = -p;
    g.src_H = H;
    g.src_W = Wd;
    g.src_n = Ci * H * Wd;
    g.N = Co;
    g.dst_n = Co * OH * OW;
    g.dst_HW = OH * OW;
    g.dst_W = OW;
    g.oy_mul = 1;
    g.ox_mul = 1;
    g.m_fast = 1;
    g.pad_t = p;
    g.pad_l = p;
    g.LH = p + H + std::max(0, (OH - 1) * s - p + kh - H);
    g.LW = p + Wd + std::max(0, (OW - 1) * s - p + kw - Wd);
    // channel-last map, k = (ky, kx, ci) with ci padded to a multiple of 4 (zero weights)
    const int Cq = cl_channels(Ci);
    g.CP = cl_stride(Ci);
    g.K = kh * kw * Cq;
    std::vector<float> Bnk((size_t)Co * g.K, 0.f);
    std::vector<int4> kt(g.K);
    for (int ci = 0; ci < Cq; ++ci)
      for (int ky = 0; ky < kh; ++ky)
        for (int kx = 0; kx < kw; ++kx) {
          const int k = (ky * kw + kx) * Cq + ci;
          kt[k] = int4{ci * H * Wd, ky, kx, ci >= Ci ? 1 : 0};
          if (ci < Ci)
            for (int co = 0; co < Co; ++co) Bnk[(size_t)co * g.K + k] = w_at(co, ci, ky, kx);
        }
    LD_TRY(finish_geom(net, g, Bnk, kt));
    L.fwd.geoms = {g};
  }
  // transposed, one GEMM per output-pixel class (ry, rx): input pixel y = y'*s + ry receives
  // the taps ky = ky0 + s*ty with ky0 = (ry + p) mod s, from output row oy = y' + dy - ty,
  // dy = (ry + p - ky0) / s.
  L.tr.geoms.clear();
  int pt = 0, pb = 0, pl = 0, pr = 0;
  for (int ry = 0; ry < s; ++ry) {
    const int Hq = (H - ry + s - 1) / s;
    const int ky0 = (ry + p) % s, dy = (ry + p - ky0) / s;
    const int Ty = kh > ky0 ? (kh - ky0 + s - 1) / s : 0;
    if (Hq <= 0 || Ty <= 0) continue;
    pt = std::max(pt, Ty - 1 - dy);
    pb = std::max(pb, Hq - 1 + dy - (OH - 1));
  }
  for (int rx = 0; rx < s; ++rx) {
    const int Wq = (Wd - rx + s - 1) / s;
    const int kx0 = (rx + p) % s, dx = (rx + p - kx0) / s;
    const int Tx = kw > kx0 ? (kw - kx0 + s - 1) / s : 0;
    if (Wq <= 0 || Tx <= 0) continue;
    pl = std::max(pl, Tx - 1 - dx);
    pr = std::max(pr, Wq - 1 + dx - (OW - 1));
  }
  for (int ry = 0; ry < s; ++ry)
    for (int rx = 0; rx < s; ++rx) {
      const int Hq = (H - ry + s - 1) / s;
      const int Wq = (Wd - rx + s - 1) / s;
      if (Hq <= 0 || Wq <= 0) continue;
      const int ky0 = (ry + p) % s, kx0 = (rx + p) % s;
      const int dy = (ry + p - ky0) / s, dx = (rx + p - kx0) / s;
      const int Ty = kh > ky0 ? (kh - ky0 + s - 1) / s : 0;
      const int Tx = kw > kx0 ? (kw - kx0 + s - 1) / s : 0;
      GemmGeom g = base_geom();
      g.HWq = Hq * Wq;
      g.Wq = Wq;
      g.iy_mul = 1;
      g.iy_off = dy;
      g.ix_mul = 1;
      g.ix_off = dx;
      g.src_H = OH;
      g.src_W = OW;
      g.src_n = Co * OH * OW;
      const int Cq = cl_channels(Co);  // channel-last map, k = (ty, tx, co), co padded
      g.CP = cl_stride(Co);
      g.K = Cq * Ty * Tx;
      g.N = Ci;
      g.dst_n = Ci * H * Wd;
      g.dst_HW = H * Wd;
      g.dst_W = Wd;
      g.oy_mul = s;
      g.oy_off = ry;
      g.ox_mul = s;
      g.ox_off = rx;
      g.m_fast = 1;
      g.pad_t = pt;
      g.pad_l = pl;
      g.LH = pt + OH + pb;
      g.LW = pl + OW + pr;
      std::vector<float> Bnk((size_t)Ci * std::max(g.K, 1), 0.f);
      std::vector<int4> kt(std::max(g.K, 1), int4{0, 0, 0, 0});
      for (int co = 0; co < Cq; ++co)
        for (int ty = 0; ty < Ty; ++ty)
          for (int tx = 0; tx < Tx; ++tx) {
            const int k = (ty * Tx + tx) * Cq + co;
            kt[k] = int4{co * OH * OW, -ty, -tx, co >= Co ? 1 : 0};
            if (co < Co)
              for (int ci = 0; ci < Ci; ++ci) Bnk[(size_t)ci * g.K + k] = w_at(co, ci, ky0 + s * ty, kx0 + s * tx);
          }
      LD_TRY(finish_geom(net, g, Bnk, kt));
      L.tr.geoms.push_back(g);
    }
  if ((int)L.tr.geoms.size() > 9) return fail(LD_E_UNSUPPORTED, "conv stride above 3 is not supported");
  LD_TRY(build_col(net, L, W));
  if (conv_lds_bytes(L.fwd.geoms.data(), 1, 1, 0, 1) > 160 * 1024 ||
      std::max(conv_lds_bytes(L.tr.geoms.data(), (int)L.tr.geoms.size(), 1, 0, 1),
               conv_lds_bytes(L.tr.geoms.data(), (int)L.tr.geoms.size(), 1, 2, 1)) > 160 * 1024)
    return fail(LD_E_UNSUPPORTED, "conv maps too large for the LDS images of one subdomain");
  return LD_OK;
}

// ---------------------------------------------------------------------------
// workspaces
// ---------------------------------------------------------------------------
int width(const ld_net* net, int k) { return k == 0 ? net->n0 : net->L[k - 1].n_out; }

int ws_alloc(const ld_net* net, Workspace& ws, int B) {
  if (ws.base && ws.B >= B) return LD_OK;
  if (ws.base) {
    // work enqueued earlier (on any stream) may still use the old buffers
    LD_HIP(hipDeviceSynchronize());
    (void)hipFree(ws.base);
    ws.base = nullptr;
  }
  const int n = net->n;
  std::vector<size_t> sizes;
  auto add = [&](size_t bytes) {
    sizes.push_back(round_up(std::max<size_t>(bytes, 1), 256));
    return sizes.size() - 1;
  };
  std::vector<size_t> ixs, ixb, ival;
  for (int k = 0; k <= n - 2; ++k) ixs.push_back(add((size_t)B * width(net, k) * 4));
  for (int k = 0; k <= n - 1; ++k) ixb.push_back(add(k == 0 ? 4 : (size_t)B * width(net, k) * 4));
  for (int k = 0; k <= n - 1; ++k) ival.push_back(add((size_t)B * width(net, k) * 8));
  size_t igc = add((size_t)B * width(net, n - 1) * 4);
  size_t icb = add((size_t)B * 8);
  size_t ia0 = add((size_t)B * net->max_width * 4);
  size_t ia1 = add((size_t)B * net->max_width * 4);
  size_t iq = add((size_t)B * 8);
  size_t ifl = add((size_t)B * 4);
  size_t ibad = add(4);
  size_t ipart = add(kPartialLayer * 4 * n);
  size_t icnt = add(kCounterCap * 4);
  size_t total = 0;
  std::vector<size_t> off;
  for (size_t s : sizes) {
    off.push_back(total);
    total += s;
  }
  void* base = nullptr;
  hipError_t e = hipMalloc(&base, total);
  if (e != hipSuccess) return fail(LD_E_NOMEM, std::string("workspace hipMalloc: ") + hipGetErrorString(e));
  char* c = (char*)base;
  ws.base = base;
  ws.B = B;
  ws.xs.assign(n - 1, nullptr);
  ws.xb.assign(n, nullptr);
  ws.val.assign(n, nullptr);
  for (int k = 0; k <= n - 2; ++k) ws.xs[k] = c + off[ixs[k]];
  for (int k = 1; k <= n - 1; ++k) ws.xb[k] = (float*)(c + off[ixb[k]]);
  for (int k = 0; k <= n - 1; ++k) ws.val[k] = (double*)(c + off[ival[k]]);
  ws.gconst = (float*)(c + off[igc]);
  ws.cb = (double*)(c + off[icb]);
  ws.act0 = (float*)(c + off[ia0]);
  ws.act1 = (float*)(c + off[ia1]);
  ws.qtmp = (double*)(c + off[iq]);
  ws.flag = (int*)(c + off[ifl]);
  ws.bad = (int*)(c + off[ibad]);
  ws.partial = (float*)(c + off[ipart]);
  ws.counters = (int*)(c + off[icnt]);
  e = hipMemset(ws.counters, 0, kCounterCap * 4);
  if (e != hipSuccess) return fail(LD_E_DEVICE, std::string("workspace memset: ") + hipGetErrorString(e));
  return LD_OK;
}

// ---------------------------------------------------------------------------
// tiles
// ---------------------------------------------------------------------------
bool job_is_conv(const Job& J) { return J.geoms[0].LH > 0; }

// Columns per wave tile (x16) of a job.  Conv: cover the columns in one pass.
// FC: the widest tile that still yields >= 1024 blocks (occupancy), else 1.
int job_tn(const Job& J, int B) {
  const int N = J.geoms[0].N;
  if (job_is_conv(J)) return N <= 16 ? 1 : (N <= 32 ? 2 : 4);
  const long gx = (B + 63) / 64;
  for (int tn : {4, 2})
    if (gx * ((N + 16 * tn - 1) / (16 * tn)) >= 1024) return tn;
  return 1;
}

// Split count of a fully-connected job: enough blocks to fill the chip, each
// split at least 128 long, scratch within the workspace's capacity.
int fc_splits(const Job& J, int B, int tn, int want) {
  const GemmGeom& g = J.geoms[0];
  const long gx = (B + 63) / 64, gy = (g.N + 16 * tn - 1) / (16 * tn);
  const long tiles = gx * gy;
  if (want <= 0) {
    want = 1;
    if (tiles < 1024 && g.K >= 256) want = (int)std::min<long>(std::min<long>((1024 + tiles - 1) / tiles, g.K / 128), 32);
  }
  int sp = std::max(1, want);
  while (sp > 1 && (size_t)tiles * sp * 64 * 16 * tn > kPartialLayer) --sp;
  return sp;
}

Tile heuristic_tile(const Job& J, int B) {
  Tile t;
  t.tm = 1;
  t.wm = 4;
  t.form = 0;
  t.tn = job_tn(J, B);
  t.splits = job_is_conv(J) ? 1 : fc_splits(J, B, t.tn, 0);
  return t;
}

// Launch configurations the autotuner times for a contraction: the column tile
// widths that the output width allows, both forms of a transposed strided conv,
// and for fully-connected products every split of K over waves and blocks into
// pieces of >= 64.
std::vector<Tile> tile_candidates(const Job& J, int B) {
  std::vector<Tile> c;
  const int N = J.geoms[0].N, K = J.geoms[0].K;
  std::vector<int> tns = {1};
  if (N > 16) tns.push_back(2);
  if (N > 32) tns.push_back(4);
  if (job_is_conv(J)) {
    // the dense GEMM + col2im form: one block per subdomain, or per (subdomain, chunk)
    if (J.has_col) c.push_back(Tile{1, 1, 1, 0, 1});
    for (const ColGeom& v : J.col_split) c.push_back(Tile{1, 1, v.nchunks, 0, 1});
    // the gather form: column tiles, and the destination rows in 1, 2 or 4 bands
    // (one block per band of a subdomain)
    const GemmGeom& g0 = J.geoms[0];
    const int dst_H = g0.dst_HW / g0.dst_W;
    for (int tn : tns)
      for (int parts : {1, 2, 4})
        if (parts <= dst_H &&
            std::max(conv_lds_bytes(J.geoms.data(), (int)J.geoms.size(), tn, 0, parts),
                     conv_lds_bytes(J.geoms.data(), (int)J.geoms.size(), tn, 2, parts)) <= 160 * 1024)
          c.push_back(Tile{1, tn, parts, J.has_col ? 1 : 0, 1});
  } else {
    // one block along K: every (wm, kw) shape of up to 16 waves; several blocks
    // along K (a second kernel adds the partials): 4 waves along subdomains
    for (int tn : tns)
      for (int wm : {1, 2, 4})
        for (int kw : {1, 2, 4, 8})
          if (wm * kw <= 16 && (kw == 1 || K / kw >= 32)) c.push_back(Tile{kw, tn, 1, 0, wm});
    for (int tn : tns)
      for (int kw : {1, 2, 4})
        for (int sp : {2, 4, 8, 16, 32})
          if (fc_splits(J, B, tn, sp) == sp && K / (sp * kw) >= 64) c.push_back(Tile{kw, tn, sp, 0, 4});
  }
  return c;
}

// Form of the transposed strided convs forced for the current thread's launches
// (-1: as tuned).  The CROWN initialisation of a state that the resident engine
// will iterate uses the stride-class form, whose summation order the resident
// kernel repeats: the duals start exactly on kinks of the dual (Prop. 2), so the
// first iteration must see the very same coefficients as the initialisation.
thread_local int g_form_override = -1;
// Set while a caller's workspace has no split-K scratch (the allocation-free dual
// evaluation): fully-connected products then run unsplit.
thread_local int g_no_split = 0;

Tile pick_tile(const ld_net* net, int layer, int dir, int B, int mma) {
  ld_net* mnet = const_cast<ld_net*>(net);
  std::lock_guard<std::mutex> lk(mnet->mu);
  auto it = mnet->tiles.find(std::make_tuple(layer, dir, B, mma));
  const Layer& L = net->L[layer];
  Tile t = it != mnet->tiles.end() ? it->second : heuristic_tile(dir == 0 ? L.fwd : L.tr, B);
  if (g_form_override >= 0) t.form = g_form_override;
  return t;
}

// slot: layer index 0..n-1; jobs of different layers may run concurrently, so
// each layer has its own split-K scratch.
hipError_t run_job(const Job& J, int B, const void* src, int src_bf16, int mma, const EpiArgs& e, Tile t,
                   const Workspace& ws, int slot, hipStream_t s) {
  GemmGeom g[9];
  const int nc = (int)J.geoms.size();
  for (int i = 0; i < nc; ++i) {
    g[i] = J.geoms[i];
    g[i].M = B * g[i].HWq;
  }
  // the dense GEMM + col2im form has no compensated BF16 product: mode 2 takes the stride-class form
  if (J.has_col && t.form == 0 && mma != 2) {
    if (t.splits > 1)
      for (const ColGeom& v : J.col_split)
        if (v.nchunks == t.splits) return launch_convT(v, B, (const float*)src, mma, e, 1, s);
    return launch_convT(mma == 1 && J.has_col_q ? J.col_q : J.col, B, (const float*)src, mma, e, 0, s);
  }
  if (job_is_conv(J)) {
    // bands of destination rows: a tile of the col2im form counts channel chunks, so
    // when the gather form runs in its place (compensated product, forced form) it
    // takes one band
    const int dst_H = g[0].dst_HW / g[0].dst_W;
    const int parts = (J.has_col && t.form == 0) ? 1 : std::min(std::max(1, t.splits), dst_H);
    return launch_conv(g, J.dev, nc, B, src, src_bf16, mma, e, t.tn, parts, s);
  }
  SplitArgs sp{g_no_split ? 1 : fc_splits(J, B, t.tn, t.splits),
               ws.partial ? ws.partial + (size_t)slot * kPartialLayer : nullptr, ws.counters};
  return launch_fc(g[0], src, src_bf16, mma, e, t.tn, sp, std::max(1, t.wm), t.tm, s);
}

// Operand mode of the transposed product W_k^T rho_k (layer k = 1..n) for a precision
// (0 FP32, 1 BF16): in the BF16 form, the products whose result is the coefficient
// of a ReLU layer's inner minimisation (k >= 2) use the compensated BF16 product
// (mode 2: heads and remainders of both operands); the product into the input box
// (k = 1) uses plain BF16.  The constant -W_n^T c is formed in FP32 (mode 0) by its
// caller.
int tr_mode(int mma, int k) { return mma == 1 && k >= 2 ? 2 : mma; }

EpiArgs epi0() {
  EpiArgs e;
  std::memset(&e, 0, sizeof(e));
  e.scale = 1.f;
  e.bias_div = 1;
  e.row_div = g_row_div;
  return e;
}

// ---------------------------------------------------------------------------
// argument checks
// ---------------------------------------------------------------------------
bool aligned16(const void* p) { return ((uintptr_t)p & 15) == 0; }

int check_batch(const ld_net* net, const ld_batch* bt) {
  if (!net) return fail(LD_E_ARG, "net is NULL");
  if (!bt) return fail(LD_E_ARG, "batch is NULL");
  if (bt->B < 0) return fail(LD_E_ARG, "batch size B < 0");
  if (bt->B == 0) return LD_OK;
  if (!bt->l0 || !bt->u0 || !bt->c) return fail(LD_E_ARG, "batch l0/u0/c is NULL");
  if (!bt->l || !bt->u) return fail(LD_E_ARG, "batch l/u pointer arrays are NULL");
  for (int k = 0; k < net->n - 1; ++k)
    if (!bt->l[k] || !bt->u[k]) return fail(LD_E_ARG, "batch l[k]/u[k] is NULL for k=" + std::to_string(k + 1));
  bool al = aligned16(bt->l0) && aligned16(bt->u0) && aligned16(bt->c);
  for (int k = 0; k < net->n - 1; ++k) al = al && aligned16(bt->l[k]) && aligned16(bt->u[k]);
  if (!al) return fail(LD_E_ARG, "batch arrays must be 16-byte aligned");
  return LD_OK;
}

int validate_values(const ld_net* net, const ld_batch* bt, Workspace& ws, hipStream_t s) {
  if (!g_validate || bt->B == 0) return LD_OK;
  LD_HIP(launch_fill_i32(ws.bad, 1, 0, s));
  LD_HIP(launch_validate(bt->B, net->n0, bt->l0, bt->u0, ws.bad, s));
  for (int k = 1; k <= net->n - 1; ++k) LD_HIP(launch_validate(bt->B, width(net, k), bt->l[k - 1], bt->u[k - 1], ws.bad, s));
  LD_HIP(launch_validate(bt->B, width(net, net->n), bt->c, bt->c, ws.bad, s));
  int bad = 0;
  LD_HIP(hipMemcpyAsync(&bad, ws.bad, 4, hipMemcpyDeviceToHost, s));
  LD_HIP(hipStreamSynchronize(s));
  if (bad) return fail(LD_E_NUMERIC, "batch holds a non-finite value or a lower bound above its upper bound");
  return LD_OK;
}

// ---------------------------------------------------------------------------
// pipelines
// ---------------------------------------------------------------------------
// g_{n-1} = -W_n^T c (the last hidden layer's constant coefficient) and c . b_n.
int prepare_objective(const ld_net* net, const ld_batch* bt, Workspace& ws, int mma, hipStream_t s) {
  const int n = net->n;
  const Layer& Ln = net->L[n - 1];
  EpiArgs e = epi0();
  e.kind = EPI_STORE;
  e.scale = -1.f;
  e.out_f = ws.gconst;
  LD_HIP(run_job(Ln.tr, bt->B, bt->c, 0, 0, e, pick_tile(net, n - 1, 1, bt->B, mma), ws, n - 1, s));
  LD_HIP(launch_cdot(bt->B, Ln.n_out, bt->c, nullptr, Ln.bias, Ln.kind == LD_CONV2D ? Ln.out_h * Ln.out_w : 1,
                     ws.cb, s));
  return LD_OK;
}

int bias_div(const ld_net* net, int k) {
  // divisor turning a neuron index of hidden layer k into its bias index
  const Layer& L = net->L[k - 1];
  return L.kind == LD_CONV2D ? L.out_h * L.out_w : 1;
}

// Phase A: inner minimisations of P_0..P_{n-1} at duals rho (rho[k-1] = rho_k).
// In the ascent (o != nullptr) the first launch also advances the step counter,
// and the last hidden layer's minimisation is left to its Adam epilogue.
EpiArgs epi_phase_a(const ld_net* net, const ld_batch* bt, const float* const* rho, const Workspace& ws, int mma,
                    float tau, int want_val, int* t_dev, float* adam, const ld_opts* o, int k) {
  const Layer& L = net->L[k - 1];
  EpiArgs e = epi0();
  e.tau = tau;
  e.want_val = want_val;
  e.xs_bf16 = mma;
  e.xs = ws.xs[k - 1];
  e.val = ws.val[k - 1];
  if (k == 1 && o != nullptr) {
    e.t_dev = t_dev;
    e.adam_w = adam;
    e.lr0 = o->lr0;
    e.lr_end = o->lr_end;
    e.total = o->total_iters;
    e.beta1 = o->beta1;
    e.beta2 = o->beta2;
    e.eps = o->eps;
  }
  if (k == 1) {
    e.kind = EPI_P0;
    e.lo = bt->l0;
    e.hi = bt->u0;
  } else {
    e.kind = EPI_INNER_MIN;
    e.rho = rho[k - 2];
    e.lo = bt->l[k - 2];
    e.hi = bt->u[k - 2];
    e.bias = net->L[k - 2].bias;
    e.xb = ws.xb[k - 1];
    // a linear layer fed by a flattened conv map has one column per neuron of that map
    e.bias_div = L.kind == LD_LINEAR ? bias_div(net, k - 1) : 1;
  }
  return e;
}

int phase_a(const ld_net* net, const ld_batch* bt, const float* const* rho, Workspace& ws, int mma, float tau,
            int want_val, int* t_dev, float* adam, const ld_opts* o, hipStream_t s) {
  const int n = net->n, B = bt->B;
  for (int k = 1; k <= n - 1; ++k) {
    const Layer& L = net->L[k - 1];
    const EpiArgs e = epi_phase_a(net, bt, rho, ws, mma, tau, want_val, t_dev, adam, o, k);
    LD_HIP(run_job(L.tr, B, rho[k - 1], 0, tr_mode(mma, k), e, pick_tile(net, k - 1, 1, B, mma), ws, k - 1, s));
  }
  if (o != nullptr) return LD_OK;
  // last hidden layer: constant coefficient -W_n^T c
  const int k = n - 1;
  LD_HIP(launch_inner_min_const(B, width(net, k), ws.gconst, rho[k - 1], bt->l[k - 1], bt->u[k - 1],
                                net->L[k - 1].bias, bias_div(net, k), tau, ws.xb[k],
                                want_val ? ws.val[k] : nullptr, nullptr, nullptr, 0, 0, 0, 0, 0, 0, g_row_div, s));
  return LD_OK;
}

int dual_eval_impl(const ld_net* net, const ld_batch* bt, const float* const* rho, Workspace& ws, double* q,
                   float* const* supergrad, int mma, float tau, hipStream_t s) {
  const int n = net->n, B = bt->B;
  LD_TRY(prepare_objective(net, bt, ws, mma, s));
  LD_TRY(phase_a(net, bt, rho, ws, mma, tau, 1, nullptr, nullptr, nullptr, s));
  if (q) {
    std::vector<const double*> arrs;
    std::vector<int> sz;
    for (int k = 0; k <= n - 1; ++k) {
      arrs.push_back(ws.val[k]);
      sz.push_back(width(net, k));
    }
    LD_HIP(launch_reduce_q(B, (int)arrs.size(), arrs.data(), sz.data(), ws.cb, q, s));
  }
  if (supergrad) {
    for (int k = 1; k <= n - 1; ++k) {
      if (!supergrad[k - 1]) continue;
      const Layer& L = net->L[k - 1];
      EpiArgs e = epi0();
      e.kind = EPI_SUPERGRAD;
      e.xb_in = ws.xb[k];
      e.bias = L.bias;
      e.out_f = supergrad[k - 1];
      LD_HIP(run_job(L.fwd, B, ws.xs[k - 1], mma, mma, e, pick_tile(net, k - 1, 0, B, mma), ws, k - 1, s));
    }
  }
  return LD_OK;
}

// CROWN or WK duals (Prop. 2) or zeros into rho (rho[k-1] = rho_k).
int init_impl(const ld_net* net, const ld_batch* bt, int init, int mma, float* const* rho, Workspace& ws,
              hipStream_t s) {
  const int n = net->n, B = bt->B;
  if (init == LD_INIT_ZERO) {
    for (int k = 1; k <= n - 1; ++k) LD_HIP(hipMemsetAsync(rho[k - 1], 0, (size_t)B * width(net, k) * 4, s));
    return LD_OK;
  }
  const int wk = init == LD_INIT_WK ? 1 : 0;
  LD_TRY(prepare_objective(net, bt, ws, mma, s));
  LD_HIP(launch_crown_const(B, width(net, n - 1), ws.gconst, bt->l[n - 2], bt->u[n - 2], rho[n - 2], wk, g_row_div,
                            s));
  for (int k = n - 1; k >= 2; --k) {
    // rho_{k-1} from g_{k-1} = W_k^T rho_k
    const Layer& L = net->L[k - 1];
    EpiArgs e = epi0();
    e.kind = wk ? EPI_WK : EPI_CROWN;
    e.lo = bt->l[k - 2];
    e.hi = bt->u[k - 2];
    e.out_f = rho[k - 2];
    LD_HIP(run_job(L.tr, B, rho[k - 1], 0, tr_mode(mma, k), e, pick_tile(net, k - 1, 1, B, mma), ws, k - 1, s));
  }
  return LD_OK;
}

// One ascent iteration (phase A then phase B) on the state.
EpiArgs epi_phase_b(const ld_net* net, const ld_batch* bt, const ld_state* st, const ld_opts* o, int k) {
  const int n = net->n;
  const Layer& L = net->L[k - 1];
  EpiArgs e = epi0();
  e.kind = EPI_ADAM;
  e.xb_in = st->ws.xb[k];
  if (k == n - 1) {
    e.kind = EPI_ADAM_LAST;
    e.gc = st->ws.gconst;
    e.lo = bt->l[k - 1];
    e.hi = bt->u[k - 1];
    e.tau = o->tie_tau;
  }
  e.bias = L.bias;
  e.rho_w = st->rho[k - 1];
  e.m = st->m[k - 1];
  e.v = st->v[k - 1];
  e.adam = st->adam;
  return e;
}

int iteration(const ld_net* net, const ld_batch* bt, ld_state* st, const ld_opts* o, hipStream_t s) {
  const int n = net->n, B = bt->B;
  const int mma = o->precision == LD_BF16 ? 1 : 0;
  std::vector<const float*> rho(st->rho.begin(), st->rho.end());
  LD_TRY(phase_a(net, bt, rho.data(), st->ws, mma, o->tie_tau, 0, st->t_dev, st->adam, o, s));
  for (int k = 1; k <= n - 1; ++k) {
    const Layer& L = net->L[k - 1];
    const EpiArgs e = epi_phase_b(net, bt, st, o, k);
    LD_HIP(run_job(L.fwd, B, st->ws.xs[k - 1], mma, mma, e, pick_tile(net, k - 1, 0, B, mma), st->ws, k - 1, s));
  }
  return LD_OK;
}

void destroy_graph(ld_state* st, int i) {
  ld_state::Graph& G = st->graphs[i];
  // a graph exec is released only once the whole device is idle (its launches and
  // whatever the runtime still does on their behalf on other streams are over)
  if (G.exec) (void)hipDeviceSynchronize();
  if (G.exec) (void)hipGraphExecDestroy(G.exec);
  if (G.graph) (void)hipGraphDestroy(G.graph);
  G.exec = nullptr;
  G.graph = nullptr;
  G.key.clear();
}

std::vector<double> graph_key(const ld_batch* bt, const ld_opts* o, int n, int chunk, int net_tune_gen) {
  std::vector<double> k;
  auto P = [&](const void* p) { k.push_back((double)(uintptr_t)p); };
  k.push_back(bt->B);
  P(bt->l0);
  P(bt->u0);
  P(bt->c);
  for (int i = 0; i < n - 1; ++i) {
    P(bt->l[i]);
    P(bt->u[i]);
  }
  k.push_back(o->total_iters);
  k.push_back(o->lr0);
  k.push_back(o->lr_end);
  k.push_back(o->beta1);
  k.push_back(o->beta2);
  k.push_back(o->eps);
  k.push_back(o->precision);
  k.push_back(o->tie_tau);
  k.push_back(chunk);
  k.push_back(net_tune_gen);
  k.push_back(g_row_div);
  return k;
}

// ---------------------------------------------------------------------------
// FP64 engine (precision LD_FP64): the same iteration with FP64 operands,
// accumulations and state
// ---------------------------------------------------------------------------
// FP64 copies of a layer's weights (as given, plus W^T of a linear layer) and bias.
int upload_f64(ld_net* net, Layer& L, const ld_layer& s) {
  F64Layer& F = L.f64;
  F.kind = s.kind == LD_CONV2D ? 1 : 0;
  F.Ci = L.in_c;
  F.H = L.in_h;
  F.W_ = L.in_w;
  F.Co = L.out_c;
  F.Ho = L.out_h;
  F.Wo = L.out_w;
  F.kh = L.kh;
  F.kw = L.kw;
  F.stride = L.stride;
  F.pad = L.pad;
  F.n_in = L.n_in;
  F.n_out = L.n_out;
  const size_t nw = s.kind == LD_LINEAR ? (size_t)L.n_out * L.n_in : (size_t)s.out_c * s.in_c * s.kh * s.kw;
  std::vector<double> w(nw), b(s.out_c);
  for (size_t i = 0; i < nw; ++i) w[i] = s.W[i];
  for (int i = 0; i < s.out_c; ++i) b[i] = s.b[i];
  void* pw;
  void* pb;
  LD_TRY(alloc_dev(net, &pw, nw * 8));
  LD_TRY(alloc_dev(net, &pb, (size_t)s.out_c * 8));
  LD_HIP(hipMemcpy(pw, w.data(), nw * 8, hipMemcpyHostToDevice));
  LD_HIP(hipMemcpy(pb, b.data(), (size_t)s.out_c * 8, hipMemcpyHostToDevice));
  F.W = (const double*)pw;
  L.b64 = (const double*)pb;
  F.WT = nullptr;
  if (s.kind == LD_LINEAR) {
    std::vector<double> wt(nw);
    for (int i = 0; i < L.n_out; ++i)
      for (int j = 0; j < L.n_in; ++j) wt[(size_t)j * L.n_out + i] = w[(size_t)i * L.n_in + j];
    void* pt;
    LD_TRY(alloc_dev(net, &pt, nw * 8));
    LD_HIP(hipMemcpy(pt, wt.data(), nw * 8, hipMemcpyHostToDevice));
    F.WT = (const double*)pt;
  }
  return LD_OK;
}

int ws64_alloc(const ld_net* net, Workspace64& ws, int B) {
  if (ws.base && ws.B >= B) return LD_OK;
  if (ws.base) {
    // work enqueued earlier (on any stream) may still use the old buffers
    LD_HIP(hipDeviceSynchronize());
    (void)hipFree(ws.base);
    ws.base = nullptr;
  }
  const int n = net->n;
  std::vector<size_t> sizes;
  auto add = [&](size_t bytes) {
    sizes.push_back(round_up(std::max<size_t>(bytes, 1), 256));
    return sizes.size() - 1;
  };
  std::vector<size_t> ixs, ixb, ival;
  for (int k = 0; k <= n - 1; ++k) ixs.push_back(add((size_t)B * width(net, k) * 8));
  for (int k = 0; k <= n - 1; ++k) ixb.push_back(add(k == 0 ? 8 : (size_t)B * width(net, k) * 8));
  for (int k = 0; k <= n - 1; ++k) ival.push_back(add((size_t)B * width(net, k) * 8));
  std::vector<size_t> irho;
  for (int k = 1; k <= n - 1; ++k) irho.push_back(add((size_t)B * width(net, k) * 8));
  const size_t ic = add((size_t)B * width(net, n) * 8);
  const size_t igc = add((size_t)B * width(net, n - 1) * 8);
  const size_t icb = add((size_t)B * 8);
  const size_t ia0 = add((size_t)B * net->max_width * 8);
  const size_t ia1 = add((size_t)B * net->max_width * 8);
  const size_t iq = add((size_t)B * 8);
  const size_t ifl = add((size_t)B * 4);
  size_t total = 0;
  std::vector<size_t> off;
  for (size_t sz : sizes) {
    off.push_back(total);
    total += sz;
  }
  void* base = nullptr;
  const hipError_t e = hipMalloc(&base, total);
  if (e != hipSuccess) return fail(LD_E_NOMEM, std::string("FP64 workspace hipMalloc: ") + hipGetErrorString(e));
  char* c = (char*)base;
  ws.base = base;
  ws.B = B;
  ws.xs.assign(n, nullptr);
  ws.xb.assign(n, nullptr);
  ws.val.assign(n, nullptr);
  for (int k = 0; k <= n - 1; ++k) ws.xs[k] = (double*)(c + off[ixs[k]]);
  for (int k = 1; k <= n - 1; ++k) ws.xb[k] = (double*)(c + off[ixb[k]]);
  for (int k = 0; k <= n - 1; ++k) ws.val[k] = (double*)(c + off[ival[k]]);
  ws.rho.assign(n - 1, nullptr);
  for (int k = 1; k <= n - 1; ++k) ws.rho[k - 1] = (double*)(c + off[irho[k - 1]]);
  ws.c64 = (double*)(c + off[ic]);
  ws.gconst = (double*)(c + off[igc]);
  ws.cb = (double*)(c + off[icb]);
  ws.act0 = (double*)(c + off[ia0]);
  ws.act1 = (double*)(c + off[ia1]);
  ws.qtmp = (double*)(c + off[iq]);
  ws.flag = (int*)(c + off[ifl]);
  return LD_OK;
}

F64Epi epi64() {
  F64Epi e;
  std::memset(&e, 0, sizeof(e));
  e.bias_div = 1;
  e.scale = 1.0;
  return e;
}

// c widened, g_{n-1} = -W_n^T c and c . b_n.
int f64_prepare_objective(const ld_net* net, const ld_batch* bt, Workspace64& ws, hipStream_t s) {
  const int n = net->n, B = bt->B;
  const Layer& Ln = net->L[n - 1];
  LD_HIP(launch_f64_widen((size_t)B * Ln.n_out, bt->c, ws.c64, s));
  F64Epi e = epi64();
  e.kind = F64_STORE;
  e.scale = -1.0;
  e.out = ws.gconst;
  LD_HIP(launch_f64_transposed(Ln.f64, B, ws.c64, nullptr, Ln.n_in, e, s));
  LD_HIP(launch_cdot(B, Ln.n_out, bt->c, nullptr, Ln.bias, Ln.kind == LD_CONV2D ? Ln.out_h * Ln.out_w : 1, ws.cb, s));
  return LD_OK;
}

// Inner minimisations of P_0..P_{n-1} at the FP64 duals rho (rho[k-1] = rho_k).
int f64_phase_a(const ld_net* net, const ld_batch* bt, const double* const* rho, Workspace64& ws, double tau,
                hipStream_t s) {
  const int n = net->n, B = bt->B;
  for (int k = 1; k <= n; ++k) {
    // g_{k-1} = W_k^T rho_k fused with P_{k-1}; the last hidden layer's g is the constant
    F64Epi e = epi64();
    e.tau = tau;
    e.xs = ws.xs[k - 1];
    e.val = ws.val[k - 1];
    if (k == 1) {
      e.kind = F64_P0;
      e.lo = bt->l0;
      e.hi = bt->u0;
    } else {
      e.kind = F64_INNER;
      e.rho = rho[k - 2];
      e.lo = bt->l[k - 2];
      e.hi = bt->u[k - 2];
      e.bias = net->L[k - 2].b64;
      e.bias_div = bias_div(net, k - 1);
      e.xb = ws.xb[k - 1];
    }
    const Layer& L = net->L[k - 1];
    if (k < n)
      LD_HIP(launch_f64_transposed(L.f64, B, rho[k - 1], nullptr, L.n_in, e, s));
    else
      LD_HIP(launch_f64_transposed(L.f64, B, nullptr, ws.gconst, L.n_in, e, s));
  }
  return LD_OK;
}

int f64_reduce_q(const ld_net* net, int B, Workspace64& ws, double* q, hipStream_t s) {
  std::vector<const double*> arrs;
  std::vector<int> sz;
  for (int k = 0; k <= net->n - 1; ++k) {
    arrs.push_back(ws.val[k]);
    sz.push_back(width(net, k));
  }
  LD_HIP(launch_reduce_q(B, (int)arrs.size(), arrs.data(), sz.data(), ws.cb, q, s));
  return LD_OK;
}

// q(rho) and, if asked, the supergradient (FP64 and/or FP32 outputs per layer).
int f64_dual_eval_impl(const ld_net* net, const ld_batch* bt, const double* const* rho, Workspace64& ws, double* q,
                       double* const* sg64, float* const* sg32, double tau, hipStream_t s) {
  const int n = net->n, B = bt->B;
  LD_TRY(f64_prepare_objective(net, bt, ws, s));
  LD_TRY(f64_phase_a(net, bt, rho, ws, tau, s));
  if (q) LD_TRY(f64_reduce_q(net, B, ws, q, s));
  for (int k = 1; k <= n - 1; ++k) {
    double* o64 = sg64 ? sg64[k - 1] : nullptr;
    float* o32 = sg32 ? sg32[k - 1] : nullptr;
    if (!o64 && !o32) continue;
    const Layer& L = net->L[k - 1];
    F64Epi e = epi64();
    e.kind = F64_SUPERGRAD;
    e.xb_in = ws.xb[k];
    e.bias = L.b64;
    e.bias_div = bias_div(net, k);
    e.out = o64;
    e.out_f = o32;
    LD_HIP(launch_f64_forward(L.f64, B, ws.xs[k - 1], e, s));
  }
  return LD_OK;
}

// CROWN or WK duals (Prop. 2) or zeros, in FP64, into rho (rho[k-1] = rho_k).
int f64_init_impl(const ld_net* net, const ld_batch* bt, int init, double* const* rho, Workspace64& ws,
                  hipStream_t s) {
  const int n = net->n, B = bt->B;
  if (init == LD_INIT_ZERO) {
    for (int k = 1; k <= n - 1; ++k) LD_HIP(hipMemsetAsync(rho[k - 1], 0, (size_t)B * width(net, k) * 8, s));
    return LD_OK;
  }
  LD_TRY(f64_prepare_objective(net, bt, ws, s));
  for (int k = n - 1; k >= 1; --k) {
    // rho_k from g_k = W_{k+1}^T rho_{k+1} (the constant -W_n^T c for k = n-1)
    const Layer& L = net->L[k];
    F64Epi e = epi64();
    e.kind = F64_CROWN;
    e.wk = init == LD_INIT_WK ? 1 : 0;
    e.lo = bt->l[k - 1];
    e.hi = bt->u[k - 1];
    e.out = rho[k - 1];
    if (k == n - 1)
      LD_HIP(launch_f64_transposed(L.f64, B, nullptr, ws.gconst, L.n_in, e, s));
    else
      LD_HIP(launch_f64_transposed(L.f64, B, rho[k], nullptr, L.n_in, e, s));
  }
  return LD_OK;
}

// FP64 duals, Adam moments and q(rho^0) of a state (allocated once).
int f64_state_alloc(const ld_net* net, ld_state* st) {
  ld_state::F64& F = st->f64;
  if (F.base) return LD_OK;
  const int n = net->n, B = st->B;
  size_t total = 0;
  std::vector<size_t> off;
  for (int k = 1; k <= n - 1; ++k)
    for (int j = 0; j < 3; ++j) {
      off.push_back(total);
      total += round_up((size_t)B * width(net, k) * 8, 256);
    }
  const size_t o_q0 = total;
  total += round_up((size_t)B * 8, 256);
  if (hipMalloc(&F.base, total) != hipSuccess) {
    F.base = nullptr;
    return fail(LD_E_NOMEM, "FP64 state hipMalloc failed");
  }
  char* c = (char*)F.base;
  F.rho.clear();
  F.m.clear();
  F.v.clear();
  for (int k = 1; k <= n - 1; ++k) {
    F.rho.push_back((double*)(c + off[3 * (k - 1)]));
    F.m.push_back((double*)(c + off[3 * (k - 1) + 1]));
    F.v.push_back((double*)(c + off[3 * (k - 1) + 2]));
  }
  F.q0 = (double*)(c + o_q0);
  return ws64_alloc(net, F.ws, B);
}

// First FP64 call on a state: duals (CROWN/WK/zero, or the FP32 duals of
// ld_state_set_rho widened), zero moments and q(rho^0).
int f64_ensure_initialised(const ld_net* net, const ld_batch* bt, ld_state* st, const ld_opts* o, hipStream_t s) {
  if (st->initialized) {
    if (!st->f64.active) return fail(LD_E_STATE, "state was initialised in FP32/BF16: reset it to step in FP64");
    return LD_OK;
  }
  LD_TRY(f64_state_alloc(net, st));
  ld_state::F64& F = st->f64;
  const int n = net->n, B = bt->B;
  if (o->init == LD_INIT_GIVEN) {
    for (int k = 1; k <= n - 1; ++k) LD_HIP(launch_f64_widen((size_t)B * width(net, k), st->rho[k - 1], F.rho[k - 1], s));
  } else {
    LD_TRY(f64_init_impl(net, bt, o->init, F.rho.data(), F.ws, s));
  }
  for (int k = 1; k <= n - 1; ++k) {
    const size_t bytes = (size_t)B * width(net, k) * 8;
    LD_HIP(hipMemsetAsync(F.m[k - 1], 0, bytes, s));
    LD_HIP(hipMemsetAsync(F.v[k - 1], 0, bytes, s));
  }
  std::vector<const double*> r(F.rho.begin(), F.rho.end());
  LD_TRY(f64_dual_eval_impl(net, bt, r.data(), F.ws, F.q0, nullptr, nullptr, o->tie_tau, s));
  F.t = 0;
  F.active = true;
  st->initialized = true;
  st->t_host = 0;
  LD_HIP(launch_fill_i32(st->t_dev, 1, 0, s));
  return LD_OK;
}

// One FP64 ascent iteration: phase A at the current duals, then per hidden layer
// the forward product with the supergradient and the Adam step (t -> t+1).
int f64_iteration(const ld_net* net, const ld_batch* bt, ld_state* st, const ld_opts* o, hipStream_t s) {
  ld_state::F64& F = st->f64;
  const int n = net->n, B = bt->B;
  std::vector<const double*> r(F.rho.begin(), F.rho.end());
  LD_TRY(f64_phase_a(net, bt, r.data(), F.ws, o->tie_tau, s));
  const int t = F.t + 1;
  const double lr0 = o->lr0, lr_end = o->lr_end, b1 = o->beta1, b2 = o->beta2;
  const int T = o->total_iters;
  const double lr = T <= 1 ? lr0 : lr0 + (lr_end - lr0) * (double)(t - 1) / (double)(T - 1);
  for (int k = 1; k <= n - 1; ++k) {
    const Layer& L = net->L[k - 1];
    F64Epi e = epi64();
    e.kind = F64_ADAM;
    e.xb_in = F.ws.xb[k];
    e.bias = L.b64;
    e.bias_div = bias_div(net, k);
    e.rho_w = F.rho[k - 1];
    e.m = F.m[k - 1];
    e.v = F.v[k - 1];
    e.lr = lr;
    e.beta1 = b1;
    e.beta2 = b2;
    e.omb1 = 1.0 - b1;
    e.omb2 = 1.0 - b2;
    e.bc1 = 1.0 - std::pow(b1, (double)t);
    e.bc2 = 1.0 - std::pow(b2, (double)t);
    e.eps = o->eps;
    LD_HIP(launch_f64_forward(L.f64, B, F.ws.xs[k - 1], e, s));
  }
  F.t = t;
  return LD_OK;
}

// primal = c^T f(x0*) with f the ReLU network in FP64 and the feasibility flag
// (every pre-activation within [l_k, u_k]), x0* in ws.xs[0].
int f64_primal(const ld_net* net, const ld_batch* bt, Workspace64& ws, double* primal, int* feasible,
               hipStream_t s) {
  const int n = net->n, B = bt->B;
  int* flag = feasible ? feasible : ws.flag;
  LD_HIP(launch_fill_i32(flag, (size_t)B, 1, s));
  const double* x = ws.xs[0];
  double* bufs[2] = {ws.act0, ws.act1};
  for (int k = 1; k <= n; ++k) {
    const Layer& L = net->L[k - 1];
    F64Epi e = epi64();
    e.bias = L.b64;
    e.bias_div = bias_div(net, k);
    e.out = bufs[k & 1];
    if (k < n) {
      e.kind = F64_RELU_FWD;
      e.lo = bt->l[k - 1];
      e.hi = bt->u[k - 1];
      e.flag = flag;
    } else {
      e.kind = F64_BIAS;
    }
    LD_HIP(launch_f64_forward(L.f64, B, x, e, s));
    x = bufs[k & 1];
  }
  if (primal) LD_HIP(launch_f64_cdot(B, net->L[n - 1].n_out, bt->c, x, primal, s));
  return LD_OK;
}

// ---------------------------------------------------------------------------
// resident engine planning
// ---------------------------------------------------------------------------
constexpr size_t kLdsBudget = 160 * 1024;

int conv_img_floats_h(const GemmGeom& g) { return g.src_n / (g.src_H * g.src_W) * g.LH * g.LW; }
int round4(int x) { return (x + 3) & ~3; }

// K chunks of an FC contraction inside the resident kernel (enough work items
// for the block's 8 waves, at least 4 K steps per chunk).
int resident_kc(const GemmGeom& g, int mma) {
  const int KS = mma ? 32 : 16;
  const int ntile = (g.N + 15) / 16;
  const int ksteps = (g.K + KS - 1) / KS;
  int kc = (32 + ntile - 1) / ntile;
  kc = std::min(kc, std::max(1, ksteps / 4));
  return std::max(1, kc);
}

struct ResidentShape {
  int S = 0;
  int xb = 0, xb_odd = 0, img = 0, gx = 0, wb = 0, part = 0;
  size_t lds = 0;
};

// Staged weight rows and row stride of a conv contraction in the resident kernel.
void conv_stage_dims(const Job& J, int B, int* n_eff, int* kp_max) {
  const int tn = job_tn(J, B);
  *n_eff = (J.geoms[0].N + 16 * tn - 1) / (16 * tn) * (16 * tn);
  int kp = 0;
  for (auto& g : J.geoms) kp = std::max(kp, g.Kp);
  *kp_max = kp;
}

int conv_stage_floats(const Job& J, int B, int mma) {
  int ne, kp;
  conv_stage_dims(J, B, &ne, &kp);
  const int ncls = (int)J.geoms.size();
  return round4(ncls * ne * kp / (mma ? 2 : 1) + ncls * kp);
}

// Shape of the resident launch for batch size B, or S = 0 when it does not apply.
ResidentShape resident_shape(const ld_net* net, int B, int mma) {
  ResidentShape R;
  const int n = net->n;
  if (n - 1 > kMaxLayers) return R;
  if (net->L[n - 1].kind != LD_LINEAR) return R;  // the engine's objective layer is fully connected
  int xb_even = 0, xb_odd = 0, img = 0, gx = 0, wb = 0;
  for (int k = 1; k <= n - 1; ++k) {
    const Layer& L = net->L[k - 1];
    if (k & 1)
      xb_odd = std::max(xb_odd, L.n_out);
    else
      xb_even = std::max(xb_even, L.n_out);
    gx = std::max(gx, std::max(L.n_in, L.n_out));
    if (L.kind == LD_CONV2D) {
      img = std::max(img, conv_img_floats_h(L.fwd.geoms[0]));
      img = std::max(img, conv_img_floats_h(L.tr.geoms[0]));
      wb = std::max(wb, conv_stage_floats(L.fwd, B, mma));
      wb = std::max(wb, conv_stage_floats(L.tr, B, mma));
    } else {
      img = std::max(img, L.n_in);
    }
  }
  R.xb_odd = round4(xb_even);
  R.xb = round4(R.xb_odd + xb_odd);
  R.img = round4(img);
  R.gx = round4(gx);
  R.wb = wb;
  for (int S : {4, 2, 1}) {
    if (S > 1 && (B + S - 1) / S < 256) continue;  // keep every CU busy first
    int part = 0;
    for (int k = 1; k <= n - 1; ++k) {
      const Layer& L = net->L[k - 1];
      if (L.kind != LD_LINEAR) continue;
      for (const GemmGeom* g : {&L.fwd.geoms[0], &L.tr.geoms[0]}) {
        const int kc = resident_kc(*g, mma);
        if (kc > 1) part = std::max(part, kc * S * g->N);
      }
    }
    const size_t floats = (size_t)S * (R.xb + R.img + R.gx) + (size_t)std::max(R.wb, round4(part)) + 4;
    if (floats * 4 <= kLdsBudget) {
      R.S = S;
      R.part = part;
      R.lds = floats * 4;
      return R;
    }
  }
  R.S = 0;
  return R;
}

int run_resident(const ld_net* net, const ld_batch* bt, ld_state* st, const ld_opts* o, const ResidentShape& R,
                 hipStream_t s) {
  const int n = net->n;
  const int mma = o->precision == LD_BF16 ? 1 : 0;
  RPlan P;
  std::memset(&P, 0, sizeof(P));
  P.n = n;
  P.B = bt->B;
  P.S = R.S;
  P.n0 = net->n0;
  P.l0 = bt->l0;
  P.u0 = bt->u0;
  P.gconst = st->ws.gconst;
  P.xb_stride = R.xb;
  P.xb_odd = R.xb_odd;
  P.img_stride = R.img;
  P.gx_stride = R.gx;
  P.wb_floats = R.wb;
  P.part_floats = R.part;
  P.t0 = st->t_host;
  P.iters = o->iters;
  P.total = o->total_iters;
  P.lr0 = o->lr0;
  P.lr_end = o->lr_end;
  P.beta1 = o->beta1;
  P.beta2 = o->beta2;
  P.eps = o->eps;
  P.tau = o->tie_tau;
  P.t_dev = st->t_dev;
  for (int k = 1; k <= n - 1; ++k) {
    const Layer& L = net->L[k - 1];
    RLayer& Q = P.L[k - 1];
    Q.kind = L.kind == LD_CONV2D ? 1 : 0;
    Q.n_in = L.n_in;
    Q.n_out = L.n_out;
    Q.out_hw = L.kind == LD_CONV2D ? L.out_h * L.out_w : 1;
    Q.bias = L.bias;
    Q.fwd = L.fwd_dev;
    Q.tr = L.tr_dev;
    Q.n_tr = (int)L.tr.geoms.size();
    Q.tn_fwd = job_tn(L.fwd, bt->B);
    Q.tn_tr = job_tn(L.tr, bt->B);
    Q.kc_fwd = L.kind == LD_LINEAR ? resident_kc(L.fwd.geoms[0], mma) : 1;
    Q.kc_tr = L.kind == LD_LINEAR ? resident_kc(L.tr.geoms[0], mma) : 1;
    if (L.kind == LD_CONV2D) {
      conv_stage_dims(L.fwd, bt->B, &Q.neff_fwd, &Q.kpm_fwd);
      conv_stage_dims(L.tr, bt->B, &Q.neff_tr, &Q.kpm_tr);
    }
    Q.rho = st->rho[k - 1];
    Q.m = st->m[k - 1];
    Q.v = st->v[k - 1];
    Q.lo = bt->l[k - 1];
    Q.hi = bt->u[k - 1];
  }
  const int grid = (bt->B + R.S - 1) / R.S;
  LD_HIP(launch_resident(P, grid, R.lds, mma, s));
  return LD_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// Scratch of the allocation-free dual evaluation: one array per device, held for
// the life of the process.  Host code never uses the array's name as an address:
// its device address comes from hipGetSymbolAddress, once per device.
// ---------------------------------------------------------------------------
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {nullptr};

// The scratch address of the current device (looked up on its first use).
static int scratch_address(void** out) {
  int dev = 0;
  LD_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(LD_E_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return fail(LD_E_DEVICE, std::string("scratch address: ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return LD_OK;
}

// The buffers of a dual evaluation of B subdomains carved from `base` (the layout
// of ws_alloc without the forward-pass activations and the split-K scratch);
// *need receives the bytes the layout takes.
static int ws_carve(const ld_net* net, Workspace& ws, int B, char* base, size_t cap, size_t* need) {
  const int n = net->n;
  size_t total = 0;
  auto take = [&](size_t bytes) {
    const size_t o = total;
    total += round_up(std::max<size_t>(bytes, 1), 256);
    return o;
  };
  std::vector<size_t> oxs, oxb, oval;
  for (int k = 0; k <= n - 2; ++k) oxs.push_back(take((size_t)B * width(net, k) * 4));
  for (int k = 0; k <= n - 1; ++k) oxb.push_back(take(k == 0 ? 4 : (size_t)B * width(net, k) * 4));
  for (int k = 0; k <= n - 1; ++k) oval.push_back(take((size_t)B * width(net, k) * 8));
  const size_t ogc = take((size_t)B * width(net, n - 1) * 4), ocb = take((size_t)B * 8);
  const size_t oq = take((size_t)B * 8), ofl = take((size_t)B * 4), obad = take(4);
  *need = total;
  if (total > cap) return LD_OK;
  ws = Workspace();
  ws.B = B;
  ws.xs.assign(n - 1, nullptr);
  ws.xb.assign(n, nullptr);
  ws.val.assign(n, nullptr);
  for (int k = 0; k <= n - 2; ++k) ws.xs[k] = base + oxs[k];
  for (int k = 1; k <= n - 1; ++k) ws.xb[k] = (float*)(base + oxb[k]);
  for (int k = 0; k <= n - 1; ++k) ws.val[k] = (double*)(base + oval[k]);
  ws.gconst = (float*)(base + ogc);
  ws.cb = (double*)(base + ocb);
  ws.qtmp = (double*)(base + oq);
  ws.flag = (int*)(base + ofl);
  ws.bad = (int*)(base + obad);
  return LD_OK;
}

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* ld_last_error(void) { return g_err.c_str(); }

void ld_set_validation(int on) { g_validate = on ? 1 : 0; }

// Host-only validation of a layer list (no HIP call), so that shape errors are
// reported identically with or without a device.
static int check_layers(const ld_layer* layers, int n_layers) {
  if (n_layers < 2) return fail(LD_E_SHAPE, "a network needs at least one hidden layer (n_layers >= 2)");
  if (n_layers > 15) return fail(LD_E_UNSUPPORTED, "at most 15 layers are supported");
  long prev_out = -1;
  for (int i = 0; i < n_layers; ++i) {
    const ld_layer& s = layers[i];
    const std::string at = " (layer " + std::to_string(i + 1) + ")";
    if (!s.W || !s.b) return fail(LD_E_ARG, "W or b is NULL" + at);
    if (s.in_c <= 0 || s.in_h <= 0 || s.in_w <= 0 || s.out_c <= 0 || s.out_h <= 0 || s.out_w <= 0)
      return fail(LD_E_SHAPE, "non-positive size" + at);
    const long n_in = (long)s.in_c * s.in_h * s.in_w;
    long n_out;
    size_t nw;
    if (s.kind == LD_LINEAR) {
      if (s.out_h != 1 || s.out_w != 1) return fail(LD_E_SHAPE, "linear layer needs out_h = out_w = 1" + at);
      n_out = s.out_c;
      nw = (size_t)n_out * n_in;
    } else if (s.kind == LD_CONV2D) {
      if (s.kh <= 0 || s.kw <= 0 || s.stride <= 0 || s.pad < 0) return fail(LD_E_SHAPE, "bad kernel/stride/pad" + at);
      if (s.stride > 3) return fail(LD_E_UNSUPPORTED, "conv stride above 3" + at);
      if (s.in_h + 2 * s.pad < s.kh || s.in_w + 2 * s.pad < s.kw ||
          (s.in_h + 2 * s.pad - s.kh) / s.stride + 1 != s.out_h || (s.in_w + 2 * s.pad - s.kw) / s.stride + 1 != s.out_w)
        return fail(LD_E_SHAPE, "conv output size does not match (in + 2 pad - k) / stride + 1" + at);
      n_out = (long)s.out_c * s.out_h * s.out_w;
      nw = (size_t)s.out_c * s.in_c * s.kh * s.kw;
      if (i > 0) {
        const ld_layer& P = layers[i - 1];
        if (P.kind != LD_CONV2D || P.out_c != s.in_c || P.out_h != s.in_h || P.out_w != s.in_w)
          return fail(LD_E_SHAPE, "conv input must be the previous conv's (C,H,W) map" + at);
      }
    } else {
      return fail(LD_E_ARG, "unknown layer kind" + at);
    }
    if (n_in > (1L << 28) || n_out > (1L << 28)) return fail(LD_E_UNSUPPORTED, "layer too wide" + at);
    if (i > 0 && n_in != prev_out) return fail(LD_E_SHAPE, "input size differs from previous output" + at);
    for (int j = 0; j < s.out_c; ++j)
      if (!std::isfinite(s.b[j])) return fail(LD_E_NUMERIC, "non-finite bias" + at);
    for (size_t j = 0; j < nw; ++j)
      if (!std::isfinite(s.W[j])) return fail(LD_E_NUMERIC, "non-finite weight" + at);
    prev_out = n_out;
  }
  return LD_OK;
}

int ld_create_net(const ld_layer* layers, int n_layers, ld_net** out) {
  g_err.clear();
  if (!layers || !out) return fail(LD_E_ARG, "layers/out is NULL");
  *out = nullptr;
  LD_TRY(check_layers(layers, n_layers));
  ld_net* net = new (std::nothrow) ld_net();
  if (!net) return fail(LD_E_NOMEM, "host allocation failed");
  net->n = n_layers;
  auto cleanup = [&](int rc) {
    ld_destroy_net(net);
    return rc;
  };
  for (int i = 0; i < n_layers; ++i) {
    const ld_layer& s = layers[i];
    Layer L;
    L.kind = s.kind;
    L.in_c = s.in_c;
    L.in_h = s.in_h;
    L.in_w = s.in_w;
    L.out_c = s.out_c;
    L.out_h = s.out_h;
    L.out_w = s.out_w;
    L.kh = s.kind == LD_CONV2D ? s.kh : 1;
    L.kw = s.kind == LD_CONV2D ? s.kw : 1;
    L.stride = s.kind == LD_CONV2D ? s.stride : 1;
    L.pad = s.kind == LD_CONV2D ? s.pad : 0;
    L.n_in = s.in_c * s.in_h * s.in_w;
    L.n_out = s.kind == LD_LINEAR ? s.out_c : s.out_c * s.out_h * s.out_w;
    void* pb;
    int rc = alloc_dev(net, &pb, (size_t)s.out_c * 4);
    if (rc) return cleanup(rc);
    if (hipMemcpy(pb, s.b, (size_t)s.out_c * 4, hipMemcpyHostToDevice) != hipSuccess)
      return cleanup(fail(LD_E_DEVICE, "bias copy failed"));
    L.bias = (float*)pb;
    rc = s.kind == LD_LINEAR ? build_linear(net, L, s.W) : build_conv(net, L, s.W);
    if (rc) return cleanup(rc);
    rc = upload_f64(net, L, s);
    if (rc) return cleanup(rc);
    {
      void* pg;
      const size_t ng = 1 + L.tr.geoms.size();
      rc = alloc_dev(net, &pg, ng * sizeof(GemmGeom));
      if (rc) return cleanup(rc);
      std::vector<GemmGeom> all;
      all.push_back(L.fwd.geoms[0]);
      for (auto& g : L.tr.geoms) all.push_back(g);
      if (hipMemcpy(pg, all.data(), ng * sizeof(GemmGeom), hipMemcpyHostToDevice) != hipSuccess)
        return cleanup(fail(LD_E_DEVICE, "geometry copy failed"));
      L.fwd_dev = (const GemmGeom*)pg;
      L.tr_dev = (const GemmGeom*)pg + 1;
      L.fwd.dev = L.fwd_dev;
      L.tr.dev = L.tr_dev;
    }
    net->L.push_back(L);
  }
  net->n0 = net->L[0].n_in;
  net->max_width = net->n0;
  for (auto& L : net->L) net->max_width = std::max(net->max_width, L.n_out);
  *out = net;
  return LD_OK;
}

void ld_destroy_net(ld_net* net) {
  if (!net) return;
  for (void* p : net->allocs) (void)hipFree(p);
  if (net->ws.base) (void)hipFree(net->ws.base);
  if (net->ws64.base) (void)hipFree(net->ws64.base);
  if (net->fsb.base) (void)hipFree(net->fsb.base);
  if (net->fsb.ws.base) (void)hipFree(net->fsb.ws.base);
  delete net;
}

int ld_net_num_layers(const ld_net* net, int* n_layers) {
  if (!net || !n_layers) return fail(LD_E_ARG, "NULL argument");
  *n_layers = net->n;
  return LD_OK;
}

int ld_net_layer_width(const ld_net* net, int k, int* w) {
  if (!net || !w) return fail(LD_E_ARG, "NULL argument");
  if (k < 0 || k > net->n) return fail(LD_E_ARG, "layer index out of range");
  *w = width(net, k);
  return LD_OK;
}

int ld_state_create(const ld_net* net, int B, ld_state** out) {
  g_err.clear();
  if (!net || !out) return fail(LD_E_ARG, "NULL argument");
  if (B <= 0) return fail(LD_E_ARG, "B must be positive");
  *out = nullptr;
  ld_state* st = new (std::nothrow) ld_state();
  if (!st) return fail(LD_E_NOMEM, "host allocation failed");
  st->net = net;
  st->B = B;
  const int n = net->n;
  size_t total = 0;
  std::vector<size_t> off;
  for (int k = 1; k <= n - 1; ++k)
    for (int j = 0; j < 3; ++j) {
      off.push_back(total);
      total += round_up((size_t)B * width(net, k) * 4, 256);
    }
  const size_t o_t = total;
  total += 256;
  const size_t o_adam = total;
  total += 256;
  const size_t o_q0 = total;
  total += round_up((size_t)B * 8, 256);
  if (hipMalloc(&st->base, total) != hipSuccess) {
    delete st;
    return fail(LD_E_NOMEM, "state hipMalloc failed");
  }
  (void)hipMemset(st->base, 0, total);
  char* c = (char*)st->base;
  for (int k = 1; k <= n - 1; ++k) {
    st->rho.push_back((float*)(c + off[3 * (k - 1)]));
    st->m.push_back((float*)(c + off[3 * (k - 1) + 1]));
    st->v.push_back((float*)(c + off[3 * (k - 1) + 2]));
  }
  st->t_dev = (int*)(c + o_t);
  st->adam = (float*)(c + o_adam);
  st->q0 = (double*)(c + o_q0);
  int rc = ws_alloc(net, st->ws, B);
  if (rc) {
    ld_state_destroy(st);
    return rc;
  }
  const bool ok = hipStreamCreateWithFlags(&st->cap, hipStreamNonBlocking) == hipSuccess &&
                  hipEventCreateWithFlags(&st->done, hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    ld_state_destroy(st);
    return fail(LD_E_DEVICE, "stream creation failed");
  }
  *out = st;
  return LD_OK;
}

void ld_state_destroy(ld_state* st) {
  if (!st) return;
  if (st->done) (void)hipEventSynchronize(st->done);
  if (st->graphs[0].exec || st->graphs[1].exec) (void)hipDeviceSynchronize();
  destroy_graph(st, 0);
  destroy_graph(st, 1);
  if (st->cap) (void)hipStreamDestroy(st->cap);
  if (st->done) (void)hipEventDestroy(st->done);
  if (st->ws.base) (void)hipFree(st->ws.base);
  if (st->track_base) (void)hipFree(st->track_base);
  if (st->tws.base) (void)hipFree(st->tws.base);
  if (st->px.base) (void)hipFree(st->px.base);
  if (st->f64.base) (void)hipFree(st->f64.base);
  if (st->f64.ws.base) (void)hipFree(st->f64.ws.base);
  if (st->base) (void)hipFree(st->base);
  delete st;
}

int ld_state_set_rho(ld_state* st, const float* const* rho, hipStream_t s) {
  g_err.clear();
  if (!st || !rho) return fail(LD_E_ARG, "NULL argument");
  const ld_net* net = st->net;
  for (int k = 1; k <= net->n - 1; ++k) {
    if (!rho[k - 1]) return fail(LD_E_ARG, "rho[k] is NULL");
    const size_t bytes = (size_t)st->B * width(net, k) * 4;
    LD_HIP(hipMemcpyAsync(st->rho[k - 1], rho[k - 1], bytes, hipMemcpyDeviceToDevice, s));
    LD_HIP(hipMemsetAsync(st->m[k - 1], 0, bytes, s));
    LD_HIP(hipMemsetAsync(st->v[k - 1], 0, bytes, s));
  }
  LD_HIP(hipMemsetAsync(st->t_dev, 0, 4, s));
  st->t_host = 0;
  st->initialized = false;  // q(rho^0) is computed by the next ld_step (init = LD_INIT_GIVEN)
  if (st->track) {  // a new ascent starts a new record
    if (st->B > 0) {
      LD_HIP(launch_fill_f64(st->best_q, (size_t)st->B, -INFINITY, s));
      LD_HIP(launch_fill_i32(st->best_t, (size_t)st->B, 0, s));
    }
    LD_HIP(launch_fill_i32(st->track_step, 1, 0, s));
  }
  st->f64.active = false;
  st->px.ready = false;     // the proximal solver restarts its primal iterates from these duals
  st->px.t = 0;
  LD_HIP(hipEventRecord(st->done, s));
  return LD_OK;
}

int ld_state_get_rho(const ld_state* st, float* const* rho, hipStream_t s) {
  g_err.clear();
  if (!st || !rho) return fail(LD_E_ARG, "NULL argument");
  const ld_net* net = st->net;
  for (int k = 1; k <= net->n - 1; ++k) {
    if (!rho[k - 1]) return fail(LD_E_ARG, "rho[k] is NULL");
    const size_t cnt = (size_t)st->B * width(net, k);
    if (st->f64.active)
      LD_HIP(launch_f64_narrow(cnt, st->f64.rho[k - 1], rho[k - 1], s));
    else
      LD_HIP(hipMemcpyAsync(rho[k - 1], st->rho[k - 1], cnt * 4, hipMemcpyDeviceToDevice, s));
  }
  LD_HIP(hipEventRecord(st->done, s));
  return LD_OK;
}

int ld_state_get_rho_f64(const ld_state* st, double* const* rho, hipStream_t s) {
  g_err.clear();
  if (!st || !rho) return fail(LD_E_ARG, "NULL argument");
  const ld_net* net = st->net;
  for (int k = 1; k <= net->n - 1; ++k) {
    if (!rho[k - 1]) return fail(LD_E_ARG, "rho[k] is NULL");
    const size_t cnt = (size_t)st->B * width(net, k);
    if (st->f64.active)
      LD_HIP(launch_f64_copy(cnt, st->f64.rho[k - 1], rho[k - 1], s));
    else
      LD_HIP(launch_f64_widen(cnt, st->rho[k - 1], rho[k - 1], s));
  }
  LD_HIP(hipEventRecord(st->done, s));
  return LD_OK;
}

int ld_state_get_step(const ld_state* st, hipStream_t s, int* t) {
  g_err.clear();
  if (!st || !t) return fail(LD_E_ARG, "NULL argument");
  LD_HIP(hipMemcpyAsync(t, st->t_dev, 4, hipMemcpyDeviceToHost, s));
  LD_HIP(hipStreamSynchronize(s));
  return LD_OK;
}

int ld_init_duals(const ld_net* net, const ld_batch* bt, int init, int precision, float* const* rho, hipStream_t s) {
  g_err.clear();
  LD_TRY(check_batch(net, bt));
  if (!rho) return fail(LD_E_ARG, "rho is NULL");
  if (init != LD_INIT_CROWN && init != LD_INIT_ZERO && init != LD_INIT_WK)
    return fail(LD_E_ARG, "init must be LD_INIT_CROWN, LD_INIT_ZERO or LD_INIT_WK");
  if (precision != LD_FP32 && precision != LD_BF16 && precision != LD_FP64) return fail(LD_E_ARG, "bad precision");
  if (bt->B == 0) return LD_OK;
  for (int k = 0; k < net->n - 1; ++k) {
    if (!rho[k]) return fail(LD_E_ARG, "rho[k] is NULL");
    if (!aligned16(rho[k])) return fail(LD_E_ARG, "rho[k] must be 16-byte aligned");
  }
  ld_net* mnet = const_cast<ld_net*>(net);
  LD_TRY(ws_alloc(net, mnet->ws, bt->B));
  LD_TRY(validate_values(net, bt, mnet->ws, s));
  if (precision == LD_FP64) {
    // FP64 propagation, rounded to the FP32 outputs
    LD_TRY(ws64_alloc(net, mnet->ws64, bt->B));
    Workspace64& w = mnet->ws64;
    LD_TRY(f64_init_impl(net, bt, init, w.rho.data(), w, s));
    for (int k = 1; k <= net->n - 1; ++k)
      LD_HIP(launch_f64_narrow((size_t)bt->B * width(net, k), w.rho[k - 1], rho[k - 1], s));
    return LD_OK;
  }
  return init_impl(net, bt, init, precision, rho, mnet->ws, s);
}

int ld_dual_eval(const ld_net* net, const ld_batch* bt, const float* const* rho, double* q, float* const* supergrad,
                 int precision, float tie_tau, hipStream_t s) {
  g_err.clear();
  LD_TRY(check_batch(net, bt));
  if (!rho) return fail(LD_E_ARG, "rho is NULL");
  if (precision != LD_FP32 && precision != LD_BF16 && precision != LD_FP64) return fail(LD_E_ARG, "bad precision");
  if (!(tie_tau >= 0.f) || !std::isfinite(tie_tau)) return fail(LD_E_ARG, "tie_tau must be finite and >= 0");
  if (bt->B == 0) return LD_OK;
  for (int k = 0; k < net->n - 1; ++k) {
    if (!rho[k]) return fail(LD_E_ARG, "rho[k] is NULL");
    if (!aligned16(rho[k])) return fail(LD_E_ARG, "rho[k] must be 16-byte aligned");
  }
  ld_net* mnet = const_cast<ld_net*>(net);
  LD_TRY(ws_alloc(net, mnet->ws, bt->B));
  LD_TRY(validate_values(net, bt, mnet->ws, s));
  if (supergrad)
    for (int k = 0; k < net->n - 1; ++k)
      if (supergrad[k] && !aligned16(supergrad[k])) return fail(LD_E_ARG, "supergrad[k] must be 16-byte aligned");
  if (precision == LD_FP64) {
    LD_TRY(ws64_alloc(net, mnet->ws64, bt->B));
    Workspace64& w = mnet->ws64;
    for (int k = 1; k <= net->n - 1; ++k)
      LD_HIP(launch_f64_widen((size_t)bt->B * width(net, k), rho[k - 1], w.rho[k - 1], s));
    std::vector<const double*> r(w.rho.begin(), w.rho.end());
    return f64_dual_eval_impl(net, bt, r.data(), w, q, nullptr, supergrad, tie_tau, s);
  }
  return dual_eval_impl(net, bt, rho, mnet->ws, q, supergrad, precision, tie_tau, s);
}

int ld_dual_eval_noalloc(const ld_net* net, const ld_batch* bt, const float* const* rho, double* q,
                         float* const* supergrad, int precision, float tie_tau, hipStream_t s) {
  g_err.clear();
  LD_TRY(check_batch(net, bt));
  if (!rho) return fail(LD_E_ARG, "rho is NULL");
  if (precision != LD_FP32 && precision != LD_BF16) return fail(LD_E_ARG, "precision must be LD_FP32 or LD_BF16");
  if (!(tie_tau >= 0.f) || !std::isfinite(tie_tau)) return fail(LD_E_ARG, "tie_tau must be finite and >= 0");
  if (bt->B == 0) return LD_OK;
  for (int k = 0; k < net->n - 1; ++k) {
    if (!rho[k]) return fail(LD_E_ARG, "rho[k] is NULL");
    if (!aligned16(rho[k])) return fail(LD_E_ARG, "rho[k] must be 16-byte aligned");
    if (supergrad && supergrad[k] && !aligned16(supergrad[k])) return fail(LD_E_ARG, "supergrad[k] must be 16-byte aligned");
  }
  void* base = nullptr;
  LD_TRY(scratch_address(&base));
  Workspace ws;
  size_t need = 0;
  LD_TRY(ws_carve(net, ws, bt->B, (char*)base, kScratchBytes, &need));
  if (need > kScratchBytes)
    return fail(LD_E_NOMEM, "the batch needs " + std::to_string(need) + " bytes of scratch, more than the " +
                                std::to_string(kScratchBytes) + " the allocation-free dual evaluation holds");
  LD_TRY(validate_values(net, bt, ws, s));
  g_no_split = 1;
  const int rc = dual_eval_impl(net, bt, rho, ws, q, supergrad, precision, tie_tau, s);
  g_no_split = 0;
  return rc;
}

int ld_dual_eval_f64(const ld_net* net, const ld_batch* bt, const double* const* rho, double* q,
                     double* const* supergrad, float tie_tau, hipStream_t s) {
  g_err.clear();
  LD_TRY(check_batch(net, bt));
  if (!rho) return fail(LD_E_ARG, "rho is NULL");
  if (!(tie_tau >= 0.f) || !std::isfinite(tie_tau)) return fail(LD_E_ARG, "tie_tau must be finite and >= 0");
  if (bt->B == 0) return LD_OK;
  for (int k = 0; k < net->n - 1; ++k)
    if (!rho[k]) return fail(LD_E_ARG, "rho[k] is NULL");
  ld_net* mnet = const_cast<ld_net*>(net);
  LD_TRY(ws64_alloc(net, mnet->ws64, bt->B));
  LD_TRY(ws_alloc(net, mnet->ws, bt->B));
  LD_TRY(validate_values(net, bt, mnet->ws, s));
  return f64_dual_eval_impl(net, bt, rho, mnet->ws64, q, supergrad, nullptr, tie_tau, s);
}

int ld_rounding_margin(const ld_net* net, const ld_batch* bt, const float* const* rho, double* margin,
                       hipStream_t s) {
  g_err.clear();
  LD_TRY(check_batch(net, bt));
  if (!rho) return fail(LD_E_ARG, "rho is NULL");
  if (bt->B == 0) return LD_OK;
  if (!margin) return fail(LD_E_ARG, "margin is NULL");
  for (int k = 0; k < net->n - 1; ++k)
    if (!rho[k]) return fail(LD_E_ARG, "rho[k] is NULL");
  ld_net* mnet = const_cast<ld_net*>(net);
  LD_TRY(ws_alloc(net, mnet->ws, bt->B));
  LD_TRY(validate_values(net, bt, mnet->ws, s));
  const int n = net->n, B = bt->B;
  const double u = std::ldexp(1.0, -24);
  std::vector<const double*> arrs;
  std::vector<int> sz;
  for (int k = 1; k <= n; ++k) {
    const Layer& L = net->L[k - 1];
    const F64Layer& F = L.f64;
    // most terms of one coefficient's dot product: the layer's outputs (fully
    // connected); for a conv, per output channel the taps that reach one input
    // position, ceil(kh / stride) x ceil(kw / stride)
    const double K = F.kind == 0 ? (double)F.n_out
                                 : (double)F.Co * ((F.kh + F.stride - 1) / F.stride) * ((F.kw + F.stride - 1) / F.stride);
    if (K * u >= 0.5) return fail(LD_E_UNSUPPORTED, "dot products too long for the rounding bound");
    // (the margin's own FP64 sums of non-negative terms err by far less than 2^-30)
    const double gamma = K * u / (1.0 - K * u) * (1.0 + std::ldexp(1.0, -30));
    const double tiny = 2.0 * K * std::ldexp(1.0, -126);  // flushed subnormal products and sums
    const float* r = k < n ? rho[k - 1] : bt->c;
    const float* lo = k == 1 ? bt->l0 : bt->l[k - 2];
    const float* hi = k == 1 ? bt->u0 : bt->u[k - 2];
    double* out = mnet->ws.val[k - 1];
    LD_HIP(launch_f64_abs_margin(F, B, r, width(net, k - 1), lo, hi, k == 1 ? 1 : 0, gamma, tiny, out, s));
    arrs.push_back(out);
    sz.push_back(width(net, k - 1));
  }
  LD_HIP(launch_reduce_q(B, (int)arrs.size(), arrs.data(), sz.data(), nullptr, margin, s));
  return LD_OK;
}

static int check_step_args(const ld_net* net, const ld_batch* bt, const ld_state* st, const ld_opts* o) {
  LD_TRY(check_batch(net, bt));
  if (!st || !o) return fail(LD_E_ARG, "state/opts is NULL");
  if (st->net != net || st->B != bt->B) return fail(LD_E_STATE, "state was created for another net or batch size");
  if (bt->B == 0) return fail(LD_E_ARG, "empty batch");
  if (o->iters < 0 || o->total_iters < 1) return fail(LD_E_ARG, "iters must be >= 0 and total_iters >= 1");
  if (o->precision != LD_FP32 && o->precision != LD_BF16 && o->precision != LD_FP64)
    return fail(LD_E_ARG, "bad precision");
  if (o->init != LD_INIT_CROWN && o->init != LD_INIT_ZERO && o->init != LD_INIT_GIVEN && o->init != LD_INIT_WK)
    return fail(LD_E_ARG, "bad init");
  if (o->engine != LD_ENGINE_AUTO && o->engine != LD_ENGINE_RESIDENT && o->engine != LD_ENGINE_LAYERWISE)
    return fail(LD_E_ARG, "bad engine");
  if (!std::isfinite(o->lr0) || !std::isfinite(o->lr_end) || !(o->beta1 >= 0.f && o->beta1 < 1.f) ||
      !(o->beta2 >= 0.f && o->beta2 < 1.f) || !(o->eps > 0.f) || !(o->tie_tau >= 0.f) || !std::isfinite(o->tie_tau))
    return fail(LD_E_ARG, "bad Adam constants");
  return LD_OK;
}

// First call on a state: dual initialisation, zeroed moments and q(rho^0).
static int ensure_initialised(const ld_net* net, const ld_batch* bt, ld_state* st, const ld_opts* o, hipStream_t s) {
  if (st->initialized && st->f64.active)
    return fail(LD_E_STATE, "state was initialised in FP64: reset it to step in FP32/BF16");
  const int mma = o->precision == LD_BF16 ? 1 : 0;
  LD_TRY(prepare_objective(net, bt, st->ws, mma, s));
  if (!st->initialized) {
    if (o->init != LD_INIT_GIVEN) {
      std::vector<float*> r(st->rho.begin(), st->rho.end());
      const bool resident = o->engine == LD_ENGINE_RESIDENT && resident_shape(net, bt->B, mma).S > 0;
      g_form_override = resident ? 1 : -1;
      const int rc = init_impl(net, bt, o->init, mma, r.data(), st->ws, s);
      g_form_override = -1;
      LD_TRY(rc);
      for (int k = 1; k <= net->n - 1; ++k) {
        const size_t bytes = (size_t)st->B * width(net, k) * 4;
        LD_HIP(hipMemsetAsync(st->m[k - 1], 0, bytes, s));
        LD_HIP(hipMemsetAsync(st->v[k - 1], 0, bytes, s));
      }
      LD_HIP(hipMemsetAsync(st->t_dev, 0, 4, s));
      st->t_host = 0;
    }
    std::vector<const float*> r(st->rho.begin(), st->rho.end());
    LD_TRY(dual_eval_impl(net, bt, r.data(), st->ws, st->q0, nullptr, LD_FP32, o->tie_tau, s));
    LD_TRY(prepare_objective(net, bt, st->ws, mma, s));
    st->initialized = true;
  }
  return LD_OK;
}

// Graph of `chunk` ascent iterations, built node by node.  Each layer job of a
// phase is captured alone (no stream fork, no event) into a scratch graph, a
// chain of one or two kernel nodes; the parent graph receives copies of those
// kernel nodes for every iteration: per phase, the first node of every job's
// chain depends on the last nodes of all jobs of the previous phase, so the jobs
// of a phase are independent branches and the phases follow one another in the
// order of iteration().
static int build_graph(const ld_net* net, const ld_batch* bt, ld_state* st, const ld_opts* o, int chunk,
                       hipGraph_t* out) {
  const int n = net->n, B = bt->B, mma = o->precision == LD_BF16 ? 1 : 0;
  std::vector<const float*> rho(st->rho.begin(), st->rho.end());
  std::vector<hipGraph_t> job;                          // [phase A jobs][phase B jobs]
  std::vector<std::vector<hipKernelNodeParams>> chain;  // kernel nodes of each job, in order
  hipGraph_t g = nullptr;
  auto release = [&]() {
    for (hipGraph_t c : job)
      if (c) (void)hipGraphDestroy(c);
    if (g) (void)hipGraphDestroy(g);
  };
  auto failed = [&](const char* what, hipError_t e) {
    release();
    return fail(LD_E_DEVICE, std::string(what) + hipGetErrorString(e));
  };
  // phase A: the transposed products (n-1 jobs) and, when the state keeps its best
  // value, one more job: q at the duals the step starts from, with FP32 operands in
  // a workspace of its own, and the record; phase B: forward products and Adam
  const int jobs_a = st->track ? n : n - 1;
  auto jobs_in = [&](int phase) { return phase == 0 ? jobs_a : n - 1; };
  for (int phase = 0; phase < 2; ++phase)
    for (int k = 1; k <= jobs_in(phase); ++k) {
      const Layer& L = net->L[std::min(k, n - 1) - 1];
      hipError_t e = hipStreamBeginCapture(st->cap, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return failed("graph capture: ", e);
      if (phase == 0 && k == n) {
        // as ld_dual_eval with FP32 operands, with the state's constants (-W_n^T c and
        // c . b_n, formed when the state was initialised)
        e = launch_inc_i32(st->track_step, st->cap);
        Workspace& tw = st->tws;
        tw.gconst = st->ws.gconst;
        if (e == hipSuccess &&
            phase_a(net, bt, rho.data(), tw, 0, o->tie_tau, 1, nullptr, nullptr, nullptr, st->cap) != LD_OK)
          e = hipErrorUnknown;
        std::vector<const double*> arrs;
        std::vector<int> sz;
        for (int j = 0; j <= n - 1; ++j) {
          arrs.push_back(tw.val[j]);
          sz.push_back(width(net, j));
        }
        if (e == hipSuccess) e = launch_reduce_q(B, (int)arrs.size(), arrs.data(), sz.data(), st->ws.cb, tw.qtmp, st->cap);
        if (e == hipSuccess) e = launch_best_update(B, tw.qtmp, st->best_q, st->best_t, st->track_step, st->cap);
      } else if (phase == 0) {
        const EpiArgs ea = epi_phase_a(net, bt, rho.data(), st->ws, mma, o->tie_tau, 0, st->t_dev, st->adam, o, k);
        e = run_job(L.tr, B, rho[k - 1], 0, tr_mode(mma, k), ea, pick_tile(net, k - 1, 1, B, mma), st->ws, k - 1,
                    st->cap);
      } else {
        const EpiArgs eb = epi_phase_b(net, bt, st, o, k);
        e = run_job(L.fwd, B, st->ws.xs[k - 1], mma, mma, eb, pick_tile(net, k - 1, 0, B, mma), st->ws, k - 1, st->cap);
      }
      hipGraph_t c = nullptr;
      const hipError_t e2 = hipStreamEndCapture(st->cap, &c);
      job.push_back(c);
      if (e != hipSuccess || e2 != hipSuccess) return failed("graph capture: ", e != hipSuccess ? e : e2);
      // order the job's kernel nodes along their dependencies (a chain)
      size_t nn = 0;
      if ((e = hipGraphGetNodes(c, nullptr, &nn)) != hipSuccess) return failed("graph nodes: ", e);
      std::vector<hipGraphNode_t> nodes(nn);
      if (nn && (e = hipGraphGetNodes(c, nodes.data(), &nn)) != hipSuccess) return failed("graph nodes: ", e);
      std::vector<hipKernelNodeParams> ch;
      hipGraphNode_t prev = nullptr;
      for (size_t step = 0; step < nn; ++step) {
        hipGraphNode_t next = nullptr;
        for (hipGraphNode_t x : nodes) {
          size_t nd = 0;
          if ((e = hipGraphNodeGetDependencies(x, nullptr, &nd)) != hipSuccess) return failed("graph nodes: ", e);
          hipGraphNode_t d = nullptr;
          if (nd == 1 && (e = hipGraphNodeGetDependencies(x, &d, &nd)) != hipSuccess) return failed("graph nodes: ", e);
          if ((prev == nullptr && nd == 0) || (prev != nullptr && nd == 1 && d == prev)) {
            next = x;
            break;
          }
        }
        hipGraphNodeType type;
        if (next == nullptr || hipGraphNodeGetType(next, &type) != hipSuccess || type != hipGraphNodeTypeKernel) {
          release();
          return fail(LD_E_DEVICE, "a layer job did not capture as a chain of kernel nodes");
        }
        hipKernelNodeParams kp;
        if ((e = hipGraphKernelNodeGetParams(next, &kp)) != hipSuccess) return failed("graph nodes: ", e);
        ch.push_back(kp);
        prev = next;
      }
      chain.push_back(ch);
    }
  hipError_t e = hipGraphCreate(&g, 0);
  std::vector<hipGraphNode_t> before, last;  // last nodes of the previous phase's jobs, of this phase's
  for (int it = 0; it < chunk && e == hipSuccess; ++it)
    for (int phase = 0; phase < 2 && e == hipSuccess; ++phase) {
      last.clear();
      const int base = phase == 0 ? 0 : jobs_a;
      for (int j = 0; j < jobs_in(phase) && e == hipSuccess; ++j) {
        std::vector<hipGraphNode_t> deps = before;
        for (const hipKernelNodeParams& kp : chain[base + j]) {
          hipGraphNode_t node = nullptr;
          e = hipGraphAddKernelNode(&node, g, deps.empty() ? nullptr : deps.data(), deps.size(), &kp);
          if (e != hipSuccess) break;
          deps.assign(1, node);
        }
        if (e == hipSuccess && !chain[base + j].empty()) last.push_back(deps[0]);
      }
      before = last;
    }
  if (e != hipSuccess) return failed("graph build: ", e);
  for (hipGraph_t c : job) (void)hipGraphDestroy(c);  // the parent holds its own copies of the nodes
  *out = g;
  return LD_OK;
}

// Iterations per captured graph: an ld_step call of up to this many iterations is
// one graph launch.
constexpr int kGraphIters = 1000;

// The ascent of one ld_step call on an initialised state, engine already chosen.
static int step_impl(const ld_net* net, const ld_batch* bt, ld_state* st, const ld_opts* o, hipStream_t s) {
  if (o->iters == 0) return LD_OK;
  const int mma_sel = o->precision == LD_BF16 ? 1 : 0;
  if (o->engine != LD_ENGINE_LAYERWISE) {
    const ResidentShape R = resident_shape(net, bt->B, mma_sel);
    const bool use = R.S > 0 && o->engine == LD_ENGINE_RESIDENT;
    if (o->engine == LD_ENGINE_RESIDENT && R.S == 0)
      return fail(LD_E_UNSUPPORTED, "the resident engine does not fit this network in LDS");
    if (use) {
      LD_TRY(run_resident(net, bt, st, o, R, s));
      st->t_host += o->iters;
      LD_HIP(hipEventRecord(st->done, s));
      return LD_OK;
    }
  }
  // A call of up to kGraphIters iterations is one graph launch; a longer one
  // replays a graph of kGraphIters iterations and ends with a graph of the rest.
  const int full = o->iters / kGraphIters, rest = o->iters % kGraphIters;
  auto exec_for = [&](int slot, int chunk, hipGraphExec_t* x) -> int {
    ld_state::Graph& G = st->graphs[slot];
    std::vector<double> key = graph_key(bt, o, net->n, chunk, net->tune_gen);
    key.push_back(st->track ? 1.0 : 0.0);
    if (!G.exec || key != G.key) {
      destroy_graph(st, slot);
      hipGraph_t g = nullptr;
      LD_TRY(build_graph(net, bt, st, o, chunk, &g));
      G.graph = g;
      const hipError_t e = hipGraphInstantiate(&G.exec, g, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        destroy_graph(st, slot);
        return fail(LD_E_DEVICE, std::string("graph instantiate: ") + hipGetErrorString(e));
      }
      G.key = key;
    }
    *x = G.exec;
    return LD_OK;
  };
  hipGraphExec_t x = nullptr;
  if (full > 0) {
    LD_TRY(exec_for(0, kGraphIters, &x));
    for (int r = 0; r < full; ++r) LD_HIP(hipGraphLaunch(x, s));
  }
  if (rest > 0) {
    LD_TRY(exec_for(full > 0 ? 1 : 0, rest, &x));
    LD_HIP(hipGraphLaunch(x, s));
  }
  st->t_host += o->iters;
  LD_HIP(hipEventRecord(st->done, s));
  return LD_OK;
}

// Best of three timings of `reps` back-to-back calls of f (after one warm-up call).
static int time_calls(const std::function<int()>& f, hipStream_t s, hipEvent_t e0, hipEvent_t e1, int reps, double* us) {
  LD_TRY(f());
  double best = 1e300;
  for (int trial = 0; trial < 3; ++trial) {
    LD_HIP(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) LD_TRY(f());
    LD_HIP(hipEventRecord(e1, s));
    LD_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    LD_HIP(hipEventElapsedTime(&ms, e0, e1));
    best = std::min(best, 1000.0 * ms / reps);
  }
  *us = best;
  return LD_OK;
}

// Autotuner: on a scratch state of the same batch, time every candidate launch
// configuration of every contraction of the iteration (with its real epilogue)
// and keep the fastest; then time the two engines over a short ascent.
static int autotune_impl(const ld_net* net, const ld_batch* bt, const ld_opts* o, hipStream_t s) {
  const int B = bt->B, n = net->n, mma = o->precision == LD_BF16 ? 1 : 0;
  ld_net* mnet = const_cast<ld_net*>(net);
  if (B == 0) return LD_OK;
  {
    std::lock_guard<std::mutex> lk(mnet->mu);
    for (auto it = mnet->tiles.begin(); it != mnet->tiles.end();)
      if (std::get<2>(it->first) == B && std::get<3>(it->first) == mma) {
        mnet->tile_us.erase(it->first);
        it = mnet->tiles.erase(it);
      } else {
        ++it;
      }
    mnet->engines.erase({B, mma});
    mnet->tune_gen++;
  }
  ld_state* tmp = nullptr;
  LD_TRY(ld_state_create(net, B, &tmp));
  struct StateGuard {
    ld_state* p;
    ~StateGuard() { ld_state_destroy(p); }
  } guard{tmp};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  LD_HIP(hipEventCreate(&e0));
  LD_HIP(hipEventCreate(&e1));
  struct EventGuard {
    hipEvent_t a, b;
    ~EventGuard() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } eguard{e0, e1};
  LD_TRY(validate_values(net, bt, tmp->ws, s));
  ld_opts to = *o;
  to.engine = LD_ENGINE_LAYERWISE;
  to.init = LD_INIT_CROWN;
  to.iters = 1;
  LD_TRY(ensure_initialised(net, bt, tmp, &to, s));
  LD_TRY(iteration(net, bt, tmp, &to, s));  // x* of every layer in the operand precision
  std::vector<const float*> rho(tmp->rho.begin(), tmp->rho.end());
  for (int k = 1; k <= n - 1; ++k)
    for (int dir = 1; dir >= 0; --dir) {
      const Job& J = dir ? net->L[k - 1].tr : net->L[k - 1].fwd;
      double best = 1e300;
      Tile pick = heuristic_tile(J, B);
      for (const Tile& t : tile_candidates(J, B)) {
        auto launch = [&]() -> int {
          if (dir == 1) {
            const EpiArgs e = epi_phase_a(net, bt, rho.data(), tmp->ws, mma, o->tie_tau, 0, nullptr, nullptr, nullptr, k);
            LD_HIP(run_job(J, B, rho[k - 1], 0, tr_mode(mma, k), e, t, tmp->ws, k - 1, s));
          } else {
            const EpiArgs e = epi_phase_b(net, bt, tmp, &to, k);
            LD_HIP(run_job(J, B, tmp->ws.xs[k - 1], mma, mma, e, t, tmp->ws, k - 1, s));
          }
          return LD_OK;
        };
        double us = 0;
        LD_TRY(time_calls(launch, s, e0, e1, 3, &us));
        if (us < best) {
          best = us;
          pick = t;
        }
      }
      std::lock_guard<std::mutex> lk(mnet->mu);
      const auto key = std::make_tuple(k - 1, dir, B, mma);
      mnet->tiles[key] = pick;
      mnet->tile_us[key] = best;
    }
  {
    std::lock_guard<std::mutex> lk(mnet->mu);
    mnet->tune_gen++;
  }
  // engines: a short ascent of each (graph replay for the layer-wise engine)
  const int T = 20;
  to.iters = T;
  to.total_iters = std::max(o->total_iters, 2 * T);
  auto run_engine = [&](int engine) -> int {
    to.engine = engine;
    return step_impl(net, bt, tmp, &to, s);
  };
  double us_lw = 0, us_res = 0;
  LD_TRY(time_calls([&]() { return run_engine(LD_ENGINE_LAYERWISE); }, s, e0, e1, 1, &us_lw));
  LD_HIP(hipEventRecord(tmp->done, s));
  // the resident engine's BF16 form uses plain BF16 transposed products (no
  // compensated product): it is offered to AUTO for FP32 only
  if (mma == 0 && g_row_div == 1 && resident_shape(net, B, mma).S > 0)
    LD_TRY(time_calls([&]() { return run_engine(LD_ENGINE_RESIDENT); }, s, e0, e1, 1, &us_res));
  LD_HIP(hipStreamSynchronize(s));
  const int eng = (us_res > 0 && us_res < us_lw) ? LD_ENGINE_RESIDENT : LD_ENGINE_LAYERWISE;
  std::lock_guard<std::mutex> lk(mnet->mu);
  mnet->engines[{B, mma}] = {(double)eng, us_lw / T, us_res / T};
  return LD_OK;
}

static int tuned_engine(const ld_net* net, int B, int mma) {
  ld_net* mnet = const_cast<ld_net*>(net);
  std::lock_guard<std::mutex> lk(mnet->mu);
  auto it = mnet->engines.find({B, mma});
  return it == mnet->engines.end() ? -1 : (int)it->second[0];
}

// ---------------------------------------------------------------------------
// proximal solver (Sec. 3.3, Algorithm 2)
// ---------------------------------------------------------------------------
static int prox_alloc(const ld_net* net, ld_state* st) {
  ld_state::Prox& P = st->px;
  if (P.base) return LD_OK;
  const int n = net->n, B = st->B;
  int wmax = 0;
  for (int k = 1; k <= n; ++k) wmax = std::max(wmax, width(net, k));
  std::vector<size_t> sizes;
  auto add = [&](size_t floats) {
    sizes.push_back(round_up(std::max<size_t>(floats * 4, 4), 256));
  };
  for (int k = 1; k <= n - 1; ++k) add((size_t)B * width(net, k));  // xB
  for (int k = 1; k <= n; ++k) add((size_t)B * width(net, k));      // xA
  for (int k = 1; k <= n - 1; ++k) add((size_t)B * width(net, k));  // rt
  for (int k = 1; k <= n - 1; ++k) add((size_t)B * width(net, k));  // pi
  for (int k = 1; k <= n - 2; ++k) add((size_t)B * width(net, k));  // g
  add((size_t)B * wmax);                                             // zA
  add((size_t)B * width(net, n - 1));                                // z_{n-1}
  size_t total = 0;
  for (size_t z : sizes) total += z;
  void* base = nullptr;
  if (hipMalloc(&base, total) != hipSuccess) return fail(LD_E_NOMEM, "proximal buffers: hipMalloc failed");
  char* c = (char*)base;
  size_t i = 0, off = 0;
  auto next = [&]() {
    char* p = c + off;
    off += sizes[i++];
    return (float*)p;
  };
  P.base = base;
  for (int k = 1; k <= n - 1; ++k) P.xB.push_back(next());
  for (int k = 1; k <= n; ++k) P.xA.push_back(next());
  for (int k = 1; k <= n - 1; ++k) P.rt.push_back(next());
  for (int k = 1; k <= n - 1; ++k) P.pi.push_back(next());
  P.g.assign(std::max(n - 1, 1), nullptr);
  for (int k = 1; k <= n - 2; ++k) P.g[k] = next();
  P.zA = next();
  P.zlast = next();
  return LD_OK;
}

// eta at outer iteration t (1-based): linear from eta0 (t = 1) to eta_end (t = T).
static double prox_eta(const ld_prox_opts* o, int t) {
  if (o->total_iters <= 1) return o->eta0;
  return (double)o->eta0 + ((double)o->eta_end - (double)o->eta0) * (double)(t - 1) / (double)(o->total_iters - 1);
}

// Operand of the forward product of layer k+1 (k = 0..n-1): z_k.
static const void* prox_operand(const ld_net* net, const ld_state* st, int k) {
  return k <= net->n - 2 ? st->ws.xs[k] : st->px.zlast;
}

// Start of Algorithm 2: a minimiser of the Lagrangian at the current duals (the
// inner minimisations of Sec. 3.2), xA_k = W_k x*_{k-1} + b_k for k = 1..n, pi = 0.
static int prox_start(const ld_net* net, const ld_batch* bt, ld_state* st, int mma, float tau, hipStream_t s) {
  const int n = net->n, B = bt->B;
  ld_state::Prox& P = st->px;
  Workspace& ws = st->ws;
  std::vector<const float*> r(st->rho.begin(), st->rho.end());
  LD_TRY(phase_a(net, bt, r.data(), ws, mma, tau, 0, nullptr, nullptr, nullptr, s));
  LD_HIP(launch_relu_operand((size_t)B * width(net, n - 1), ws.xb[n - 1], P.zlast, mma, s));
  for (int k = 0; k <= n - 1; ++k) {
    const Layer& L = net->L[k];
    EpiArgs e = epi0();
    e.kind = EPI_BIAS_STORE;
    e.bias = L.bias;
    e.out_f = P.xA[k];
    LD_HIP(run_job(L.fwd, B, prox_operand(net, st, k), mma, mma, e, pick_tile(net, k, 0, B, mma), ws, k, s));
  }
  for (int k = 1; k <= n - 1; ++k) {
    const size_t cnt = (size_t)B * width(net, k);
    LD_HIP(launch_copy_f32(P.xB[k - 1], ws.xb[k], cnt, s));
    LD_HIP(launch_fill_f32(P.pi[k - 1], cnt, 0.f, s));
  }
  return LD_OK;
}

// rt = rho + (xB - xA) / eta for every hidden layer.
static int prox_coeff(const ld_net* net, ld_state* st, double eta, hipStream_t s) {
  const int nh = net->n - 1;
  for (int first = 1; first <= nh; first += kProxPackMax) {
    ProxDualPack p;
    std::memset(&p, 0, sizeof(p));
    p.n = std::min(kProxPackMax, nh - first + 1);
    for (int i = 0; i < p.n; ++i) {
      const int k = first + i;  // hidden layer
      p.rho[i] = st->rho[k - 1];
      p.xB[i] = st->px.xB[k - 1];
      p.xA[i] = st->px.xA[k - 1];
      p.rt[i] = st->px.rt[k - 1];
      p.cnt[i] = (size_t)st->B * width(net, k);
    }
    LD_HIP(launch_prox_coeff(p, (float)(1.0 / eta), s));
  }
  return LD_OK;
}

// The launches of one block-coordinate Frank-Wolfe sweep over the blocks
// k = 0..n-1, in order, each with its slot: 100+k the transposed product
// W_k^T rt_k, 300+k the forward product of layer k (block k-1), 400+k the block
// kernel of block k.
using Launch = std::pair<int, std::function<int()>>;
// With `dual` the block kernels also take the dual update of the outer iteration
// (momentum mu, then rt for eta_next).  Everything runs on one stream: forking the
// independent transposed products onto side streams made the solve slower.
static void prox_sweep_launches(const ld_net* net, const ld_batch* bt, ld_state* st, int mma, float tau, double eta,
                                bool dual, double mu, double eta_next, hipStream_t s, std::vector<Launch>& out) {
  const int n = net->n, B = bt->B;
  ld_state::Prox& P = st->px;
  Workspace& ws = st->ws;
  // transposed products g_{k-1} = W_k^T rt_k; the one into the input box is fused
  // with the box rule (the conditional gradient of block 0)
  for (int k = 1; k <= n - 1; ++k) {
    const Layer& L = net->L[k - 1];
    EpiArgs e = epi0();
    if (k == 1) {
      e.kind = EPI_P0;
      e.lo = bt->l0;
      e.hi = bt->u0;
      e.xs = ws.xs[0];
      e.xs_bf16 = mma;
    } else {
      e.kind = EPI_STORE;
      e.out_f = P.g[k - 1];
    }
    const Tile t = pick_tile(net, k - 1, 1, B, mma);
    const float* src = P.rt[k - 1];
    out.push_back({100 + k, [=, &L, &ws]() -> int {
                     LD_HIP(run_job(L.tr, B, src, 0, tr_mode(mma, k), e, t, ws, k - 1, s));
                     return LD_OK;
                   }});
  }
  const double inv_eta = 1.0 / eta;
  for (int k = 0; k <= n - 1; ++k) {
    const Layer& L = net->L[k];
    EpiArgs e = epi0();
    e.kind = EPI_BIAS_STORE;
    e.bias = L.bias;
    e.out_f = P.zA;
    const Tile t = pick_tile(net, k, 0, B, mma);
    const void* src = prox_operand(net, st, k);
    out.push_back({300 + k + 1, [=, &L, &ws]() -> int {
                     LD_HIP(run_job(L.fwd, B, src, mma, mma, e, t, ws, k, s));
                     return LD_OK;
                   }});
    ProxBlockArgs a;
    std::memset(&a, 0, sizeof(a));
    a.nB = k >= 1 ? width(net, k) : 0;
    a.nA = width(net, k + 1);
    a.last = k + 1 == n ? 1 : 0;
    a.z_bf16 = mma;
    a.inv_eta = (float)inv_eta;
    a.inv_eta_d = inv_eta;
    a.tau = tau;
    a.dual = dual && k >= 1 ? 1 : 0;
    a.mu = (float)mu;
    a.inv_eta_next = (float)(1.0 / eta_next);
    if (k >= 1) {
      a.piB = P.pi[k - 1];
      a.xB = P.xB[k - 1];
      a.zB = ws.xb[k];
      a.rtB = P.rt[k - 1];
      a.rhoB = st->rho[k - 1];
      a.xAB = P.xA[k - 1];
    }
    a.xA = P.xA[k];
    a.zA = P.zA;
    if (a.last) {
      a.c = bt->c;
    } else {
      a.rtA = P.rt[k];
      a.rhoA = st->rho[k];
      a.xBA = P.xB[k];
      a.g = k + 1 == n - 1 ? ws.gconst : P.g[k + 1];
      a.lo = bt->l[k];
      a.hi = bt->u[k];
      a.zB_out = ws.xb[k + 1];
      a.z_out = const_cast<void*>(prox_operand(net, st, k + 1));
    }
    out.push_back({400 + k, [=]() -> int {
                     LD_HIP(launch_prox_block(a, B, s));
                     return LD_OK;
                   }});
  }
}

static int prox_sweep(const ld_net* net, const ld_batch* bt, ld_state* st, int mma, float tau, double eta,
                      bool dual, double mu, double eta_next, hipStream_t s) {
  std::vector<Launch> ls;
  prox_sweep_launches(net, bt, st, mma, tau, eta, dual, mu, eta_next, s, ls);
  for (auto& l : ls) LD_TRY(l.second());
  return LD_OK;
}

static int check_prox_args(const ld_net* net, const ld_batch* bt, const ld_state* st, const ld_prox_opts* o) {
  LD_TRY(check_batch(net, bt));
  if (!st || !o) return fail(LD_E_ARG, "state/opts is NULL");
  if (st->net != net || st->B != bt->B) return fail(LD_E_STATE, "state was created for another net or batch size");
  if (bt->B == 0) return fail(LD_E_ARG, "empty batch");
  if (o->iters < 0 || o->total_iters < 1 || o->inner_iters < 1)
    return fail(LD_E_ARG, "iters must be >= 0, total_iters >= 1 and inner_iters >= 1");
  if (!(o->eta0 > 0.f) || !(o->eta_end > 0.f) || !std::isfinite(o->eta0) || !std::isfinite(o->eta_end))
    return fail(LD_E_ARG, "eta0 and eta_end must be finite and > 0");
  if (!(o->mu >= 0.f && o->mu < 1.f)) return fail(LD_E_ARG, "mu must be in [0, 1)");
  if (o->precision == LD_FP64) return fail(LD_E_UNSUPPORTED, "the proximal solver has no FP64 form");
  if (o->precision != LD_FP32 && o->precision != LD_BF16) return fail(LD_E_ARG, "bad precision");
  if (o->init != LD_INIT_CROWN && o->init != LD_INIT_ZERO && o->init != LD_INIT_GIVEN && o->init != LD_INIT_WK)
    return fail(LD_E_ARG, "bad init");
  if (!(o->tie_tau >= 0.f) || !std::isfinite(o->tie_tau)) return fail(LD_E_ARG, "tie_tau must be finite and >= 0");
  if (net->n - 1 > 64) return fail(LD_E_UNSUPPORTED, "more than 64 hidden layers");
  return LD_OK;
}

int ld_prox_step(const ld_net* net, const ld_batch* bt, ld_state* st, const ld_prox_opts* o, hipStream_t s) {
  g_err.clear();
  LD_TRY(check_prox_args(net, bt, st, o));
  LD_TRY(validate_values(net, bt, st->ws, s));
  const int mma = o->precision == LD_BF16 ? 1 : 0;
  ld_opts lo;
  std::memset(&lo, 0, sizeof(lo));
  lo.iters = 0;
  lo.total_iters = 1;
  lo.precision = o->precision;
  lo.init = o->init;
  lo.tie_tau = o->tie_tau;
  lo.engine = LD_ENGINE_LAYERWISE;
  LD_TRY(ensure_initialised(net, bt, st, &lo, s));
  LD_TRY(prox_alloc(net, st));
  ld_state::Prox& P = st->px;
  if (!P.ready || P.mma != mma) {
    LD_TRY(prox_start(net, bt, st, mma, o->tie_tau, s));
    P.ready = true;
    P.mma = mma;
    P.t = 0;
  }
  // coefficients of the next iteration under this call's schedule
  LD_TRY(prox_coeff(net, st, prox_eta(o, P.t + 1), s));
  for (int it = 0; it < o->iters; ++it) {
    const int t = P.t + 1;
    const double eta = prox_eta(o, t);
    // the last sweep's block kernels also take the dual update
    for (int j = 0; j < o->inner_iters; ++j)
      LD_TRY(prox_sweep(net, bt, st, mma, o->tie_tau, eta, j == o->inner_iters - 1, o->mu, prox_eta(o, t + 1), s));
    P.t = t;
  }
  LD_HIP(hipEventRecord(st->done, s));
  return LD_OK;
}

int ld_prox_profile_iteration(const ld_net* net, const ld_batch* bt, ld_state* st, const ld_prox_opts* o, int reps,
                              double* avg_us, int* kinds, int max_slots, int* n_slots, hipStream_t s) {
  g_err.clear();
  LD_TRY(check_prox_args(net, bt, st, o));
  if (reps <= 0 || !avg_us || !kinds || !n_slots || max_slots <= 0) return fail(LD_E_ARG, "bad profile arguments");
  if (!st->px.ready) return fail(LD_E_STATE, "no proximal iteration has run on this state");
  const int mma = o->precision == LD_BF16 ? 1 : 0;
  if (st->px.mma != mma) return fail(LD_E_STATE, "the state's proximal iterates were formed in another precision");
  const double eta = prox_eta(o, st->px.t + 1);
  // the last sweep of an outer iteration (block kernels with the dual update)
  std::vector<Launch> ls;
  prox_sweep_launches(net, bt, st, mma, o->tie_tau, eta, true, o->mu, eta, s, ls);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  LD_HIP(hipEventCreate(&e0));
  LD_HIP(hipEventCreate(&e1));
  struct EventGuard {
    hipEvent_t a, b;
    ~EventGuard() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } eguard{e0, e1};
  int ns = 0;
  for (auto& l : ls) {
    if (ns >= max_slots) break;
    LD_TRY(l.second());  // warm-up
    LD_HIP(hipEventRecord(e0, s));
    for (int r = 0; r < reps; ++r) LD_TRY(l.second());
    LD_HIP(hipEventRecord(e1, s));
    LD_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    LD_HIP(hipEventElapsedTime(&ms, e0, e1));
    avg_us[ns] = 1000.0 * ms / reps;
    kinds[ns] = l.first;
    ++ns;
  }
  *n_slots = ns;
  // the repeated launches moved the iterates: restart them at the next call
  st->px.ready = false;
  LD_HIP(hipEventRecord(st->done, s));
  return LD_OK;
}

int ld_prox_get_step(const ld_state* st, int* t) {
  g_err.clear();
  if (!st || !t) return fail(LD_E_ARG, "NULL argument");
  *t = st->px.ready ? st->px.t : 0;
  return LD_OK;
}

// ---------------------------------------------------------------------------
// intermediate bounds (Sec. 2.2.3; batched over the neurons of a layer, Sec. 5.2)
// ---------------------------------------------------------------------------
int ld_intermediate_bounds(const ld_net* sub, const ld_batch* bt, const ld_opts* o, int max_problems, float* lo,
                           float* hi, hipStream_t s) {
  g_err.clear();
  if (!sub || !bt || !o) return fail(LD_E_ARG, "NULL argument");
  const int n = sub->n, B = bt->B;
  if (B < 0) return fail(LD_E_ARG, "batch size B < 0");
  if (B == 0) return LD_OK;
  if (!lo || !hi) return fail(LD_E_ARG, "NULL output");
  if (!bt->l0 || !bt->u0 || !bt->l || !bt->u) return fail(LD_E_ARG, "batch l0/u0/l/u is NULL");
  for (int k = 1; k <= n - 1; ++k)
    if (!bt->l[k - 1] || !bt->u[k - 1]) return fail(LD_E_ARG, "batch l[k]/u[k] is NULL for k=" + std::to_string(k));
  if (o->init == LD_INIT_GIVEN) return fail(LD_E_ARG, "init must be LD_INIT_CROWN, LD_INIT_ZERO or LD_INIT_WK");
  if (n - 1 > 32) return fail(LD_E_UNSUPPORTED, "more than 32 hidden layers");
  const int nj = width(sub, n);
  const long long P = 2LL * nj;
  const long long total = (long long)B * P;
  const long long cmax = max_problems > 0 ? max_problems : 8192;
  // The 2 n_j problems of a subdomain read its bound rows in place when chunks hold
  // whole subdomains (FP32/BF16 layer-wise engine): each chunk's batch points at the
  // rows of its first subdomain and every kernel maps problem p to row p / P.
  // Otherwise every problem of a chunk gets a copy of its subdomain's rows.
  bool share = o->precision != LD_FP64 && o->engine != LD_ENGINE_RESIDENT && P <= cmax &&
               (max_problems <= 0 || max_problems % P == 0);
  const long long C = std::min<long long>(share ? cmax / P * P : cmax, total);
  // a chunk after the first starts at a subdomain's rows: they must stay 16-byte aligned
  if (share && C < total) {
    bool al = sub->n0 % 4 == 0;
    for (int k = 1; k <= n - 1; ++k) al = al && width(sub, k) % 4 == 0;
    share = al;
  }
  // one chunk's expanded batch (or only its objectives) and its bounds
  std::vector<int> widths = {sub->n0, sub->n0};
  for (int k = 1; k <= n - 1; ++k) {
    widths.push_back(width(sub, k));
    widths.push_back(width(sub, k));
  }
  std::vector<size_t> off;
  size_t total_bytes = 0;
  for (int w : widths) {
    off.push_back(total_bytes);
    total_bytes += share ? 0 : round_up((size_t)C * w * 4, 256);
  }
  const size_t off_c = total_bytes;
  total_bytes += round_up((size_t)C * nj * 4, 256);
  const size_t off_b = total_bytes;
  total_bytes += round_up((size_t)C * 8, 256);
  const size_t off_bad = total_bytes;
  total_bytes += 256;
  void* base = nullptr;
  if (hipMalloc(&base, total_bytes) != hipSuccess) return fail(LD_E_NOMEM, "intermediate bounds: hipMalloc failed");
  char* cb = (char*)base;
  IntermPack K;
  std::memset(&K, 0, sizeof(K));
  K.n = share ? 0 : (int)widths.size();
  std::vector<const float*> srcs = {bt->l0, bt->u0};
  for (int k = 1; k <= n - 1; ++k) {
    srcs.push_back(bt->l[k - 1]);
    srcs.push_back(bt->u[k - 1]);
  }
  for (int a = 0; a < K.n; ++a) {
    K.src[a] = srcs[a];
    K.dst[a] = (float*)(cb + off[a]);
    K.width[a] = widths[a];
  }
  K.c = (float*)(cb + off_c);
  double* bound = (double*)(cb + off_b);
  ld_state* states[2] = {nullptr, nullptr};  // full chunks, the tail chunk
  int rc = LD_OK;
  if (share && g_validate) {
    // the caller's rows are read in place: check them once (the chunks skip it)
    int* bad = (int*)(cb + off_bad);
    hipError_t e = launch_fill_i32(bad, 1, 0, s);
    if (e == hipSuccess) e = launch_validate(B, sub->n0, bt->l0, bt->u0, bad, s);
    for (int k = 1; k <= n - 1 && e == hipSuccess; ++k)
      e = launch_validate(B, width(sub, k), bt->l[k - 1], bt->u[k - 1], bad, s);
    int h = 0;
    if (e == hipSuccess) e = hipMemcpyAsync(&h, bad, 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess)
      rc = fail(LD_E_DEVICE, std::string("intermediate bounds: ") + hipGetErrorString(e));
    else if (h)
      rc = fail(LD_E_NUMERIC, "batch holds a non-finite value or a lower bound above its upper bound");
  }
  // the internal calls read shared rows (and skip the validation done above)
  struct ShareScope {
    int div0, val0;
    ShareScope(bool on, int div) : div0(g_row_div), val0(g_validate) {
      if (on) {
        g_row_div = div;
        g_validate = 0;
      }
    }
    ~ShareScope() {
      g_row_div = div0;
      g_validate = val0;
    }
  } scope(share, (int)P);
  for (long long start = 0; start < total && rc == LD_OK; start += C) {
    const int cc = (int)std::min<long long>(C, total - start);
    hipError_t e = launch_interm_expand(K, cc, start, (int)P, nj, s);
    if (e != hipSuccess) {
      rc = fail(LD_E_DEVICE, std::string("interm_expand: ") + hipGetErrorString(e));
      break;
    }
    std::vector<const float*> dl, du;
    ld_batch cbt;
    cbt.B = cc;
    if (share) {
      const long long b0 = start / P;  // the chunk's first subdomain
      cbt.l0 = bt->l0 + b0 * sub->n0;
      cbt.u0 = bt->u0 + b0 * sub->n0;
      for (int k = 1; k <= n - 1; ++k) {
        dl.push_back(bt->l[k - 1] + b0 * width(sub, k));
        du.push_back(bt->u[k - 1] + b0 * width(sub, k));
      }
    } else {
      cbt.l0 = K.dst[0];
      cbt.u0 = K.dst[1];
      for (int k = 1; k <= n - 1; ++k) {
        dl.push_back(K.dst[2 * k]);
        du.push_back(K.dst[2 * k + 1]);
      }
    }
    cbt.l = dl.data();
    cbt.u = du.data();
    cbt.c = K.c;
    ld_state*& st = states[cc == C ? 0 : 1];
    if (!st && (rc = ld_state_create(sub, cc, &st)) != LD_OK) break;
    if ((rc = ld_state_reset(st, s)) != LD_OK) break;
    if ((rc = ld_step(sub, &cbt, st, o, s)) != LD_OK) break;
    if ((rc = ld_final_bound(sub, &cbt, st, bound, nullptr, nullptr, nullptr, o->tie_tau, s)) != LD_OK) break;
    e = launch_interm_collect(cc, start, (int)P, nj, bound, lo, hi, s);
    if (e != hipSuccess) rc = fail(LD_E_DEVICE, std::string("interm_collect: ") + hipGetErrorString(e));
  }
  const hipError_t es = hipStreamSynchronize(s);
  for (ld_state* st : states) ld_state_destroy(st);
  (void)hipFree(base);
  if (rc == LD_OK && es != hipSuccess) rc = fail(LD_E_DEVICE, std::string("intermediate bounds: ") + hipGetErrorString(es));
  return rc;
}

// ---------------------------------------------------------------------------
// Filtered Smart Branching (Sec. 4.2)
// ---------------------------------------------------------------------------
int ld_fsb_branch(const ld_net* net, const ld_batch* bt, int* layer, int* index, double* value, int* candidates,
                  hipStream_t s) {
  g_err.clear();
  LD_TRY(check_batch(net, bt));
  const int n = net->n, B = bt->B, nh = n - 1;
  if (B == 0) return LD_OK;
  if (!layer || !index || !value) return fail(LD_E_ARG, "NULL output");
  if (nh > 16) return fail(LD_E_UNSUPPORTED, "more than 16 hidden layers");
  const int M = 4 * nh;  // children per subdomain: 2 candidates x 2 phases per hidden layer
  const long long Bc = (long long)B * M;
  if (Bc > (1LL << 30)) return fail(LD_E_UNSUPPORTED, "too many children");
  // device buffers: lambda_k (k = 1..n-2; lambda_{n-1} is the objective constant),
  // candidates, the children's batch, their duals and bounds
  std::vector<size_t> sz;
  auto add = [&](size_t bytes) {
    sz.push_back(round_up(std::max<size_t>(bytes, 4), 256));
    return sz.size() - 1;
  };
  std::vector<size_t> i_lam, i_cl, i_cu, i_rho;
  for (int k = 1; k <= n - 2; ++k) i_lam.push_back(add((size_t)B * width(net, k) * 4));
  const size_t i_cand = add((size_t)B * nh * 2 * 4);
  const size_t i_l0 = add((size_t)Bc * net->n0 * 4), i_u0 = add((size_t)Bc * net->n0 * 4);
  for (int k = 1; k <= nh; ++k) {
    i_cl.push_back(add((size_t)Bc * width(net, k) * 4));
    i_cu.push_back(add((size_t)Bc * width(net, k) * 4));
    i_rho.push_back(add((size_t)Bc * width(net, k) * 4));
  }
  const size_t i_c = add((size_t)Bc * width(net, n) * 4);
  const size_t i_qc = add((size_t)Bc * 8), i_qw = add((size_t)Bc * 8);
  std::vector<size_t> off(sz.size());
  size_t total = 0;
  for (size_t i = 0; i < sz.size(); ++i) {
    off[i] = total;
    total += sz[i];
  }
  ld_net* mnet = const_cast<ld_net*>(net);
  std::lock_guard<std::mutex> lk(mnet->fsb.mu);
  if (mnet->fsb.bytes < total) {
    // work of an earlier call may still use the old buffers (the call ends with a
    // stream synchronisation, so this only waits for other streams)
    LD_HIP(hipDeviceSynchronize());
    if (mnet->fsb.base) (void)hipFree(mnet->fsb.base);
    mnet->fsb.base = nullptr;
    mnet->fsb.bytes = 0;
    if (hipMalloc(&mnet->fsb.base, total) != hipSuccess) return fail(LD_E_NOMEM, "branching buffers: hipMalloc failed");
    mnet->fsb.bytes = total;
  }
  char* cb = (char*)mnet->fsb.base;
  auto F = [&](size_t i) { return (float*)(cb + off[i]); };
  Workspace& ws = mnet->fsb.ws;
  int rc = ws_alloc(net, ws, (int)std::max<long long>(Bc, B));
  if (rc == LD_OK) rc = validate_values(net, bt, ws, s);
  int* cand = candidates ? candidates : (int*)(cb + off[i_cand]);
  std::vector<float*> rho(nh);
  for (int k = 1; k <= nh; ++k) rho[k - 1] = F(i_rho[k - 1]);
  // 1. parent: WK duals and the backward pass lambda_k = W_{k+1}^T rho_{k+1} (eq:babsr-scores)
  if (rc == LD_OK) rc = init_impl(net, bt, LD_INIT_WK, 0, rho.data(), ws, s);
  std::vector<const float*> lam(nh), lo(nh), hi(nh), bias(nh);
  std::vector<int> bdiv(nh), wid(nh);
  for (int k = 1; k <= nh && rc == LD_OK; ++k) {
    if (k <= n - 2) {
      EpiArgs e = epi0();
      e.kind = EPI_STORE;
      e.out_f = F(i_lam[k - 1]);
      const hipError_t he = run_job(net->L[k].tr, B, rho[k], 0, 0, e, pick_tile(net, k, 1, B, 0), ws, k, s);
      if (he != hipSuccess) rc = fail(LD_E_DEVICE, std::string("fsb backward pass: ") + hipGetErrorString(he));
      lam[k - 1] = F(i_lam[k - 1]);
    } else {
      lam[k - 1] = ws.gconst;
    }
    lo[k - 1] = bt->l[k - 1];
    hi[k - 1] = bt->u[k - 1];
    bias[k - 1] = net->L[k - 1].bias;
    bdiv[k - 1] = bias_div(net, k);
    wid[k - 1] = width(net, k);
  }
  // 2. scores and the candidates of eq:fsb-prefilter
  if (rc == LD_OK) {
    const hipError_t he = launch_fsb_scores(B, nh, lam.data(), lo.data(), hi.data(), bias.data(), bdiv.data(),
                                            wid.data(), cand, s);
    if (he != hipSuccess) rc = fail(LD_E_DEVICE, std::string("fsb scores: ") + hipGetErrorString(he));
  }
  // 3. the children: one batch of B*M subdomains, each with one ReLU split
  std::vector<const float*> cl(nh), cu(nh);
  std::vector<float*> clw(nh), cuw(nh);
  for (int k = 1; k <= nh; ++k) {
    clw[k - 1] = F(i_cl[k - 1]);
    cuw[k - 1] = F(i_cu[k - 1]);
    cl[k - 1] = clw[k - 1];
    cu[k - 1] = cuw[k - 1];
  }
  if (rc == LD_OK) {
    IntermPack K;
    std::memset(&K, 0, sizeof(K));
    std::vector<std::pair<const float*, float*>> arr = {{bt->l0, F(i_l0)}, {bt->u0, F(i_u0)}};
    std::vector<int> w = {net->n0, net->n0};
    for (int k = 1; k <= nh; ++k) {
      arr.push_back({bt->l[k - 1], clw[k - 1]});
      w.push_back(width(net, k));
      arr.push_back({bt->u[k - 1], cuw[k - 1]});
      w.push_back(width(net, k));
    }
    arr.push_back({bt->c, F(i_c)});
    w.push_back(width(net, n));
    K.n = (int)arr.size();
    for (int a = 0; a < K.n; ++a) {
      K.src[a] = arr[a].first;
      K.dst[a] = arr[a].second;
      K.width[a] = w[a];
    }
    K.c = nullptr;
    const hipError_t he = launch_fsb_expand(K, B, nh, cand, clw.data(), cuw.data(), wid.data(), s);
    if (he != hipSuccess) rc = fail(LD_E_DEVICE, std::string("fsb expand: ") + hipGetErrorString(he));
  }
  // 4. the children's CROWN and WK bounds (q at the propagation duals, Prop. 2)
  ld_batch cbt;
  cbt.B = (int)Bc;
  cbt.l0 = F(i_l0);
  cbt.u0 = F(i_u0);
  cbt.l = cl.data();
  cbt.u = cu.data();
  cbt.c = F(i_c);
  std::vector<const float*> crho(rho.begin(), rho.end());
  double* qc = (double*)(cb + off[i_qc]);
  double* qw = (double*)(cb + off[i_qw]);
  if (rc == LD_OK) rc = init_impl(net, &cbt, LD_INIT_CROWN, 0, rho.data(), ws, s);
  if (rc == LD_OK) rc = dual_eval_impl(net, &cbt, crho.data(), ws, qc, nullptr, 0, 0.f, s);
  if (rc == LD_OK) rc = init_impl(net, &cbt, LD_INIT_WK, 0, rho.data(), ws, s);
  if (rc == LD_OK) rc = dual_eval_impl(net, &cbt, crho.data(), ws, qw, nullptr, 0, 0.f, s);
  // 5. the candidate whose worse child has the best bound
  if (rc == LD_OK) {
    const hipError_t he = launch_fsb_select(B, nh, cand, qc, qw, layer, index, value, s);
    if (he != hipSuccess) rc = fail(LD_E_DEVICE, std::string("fsb select: ") + hipGetErrorString(he));
  }
  const hipError_t es = hipStreamSynchronize(s);
  if (rc == LD_OK && es != hipSuccess) rc = fail(LD_E_DEVICE, std::string("branching: ") + hipGetErrorString(es));
  return rc;
}

int ld_branch_children(const ld_net* net, const ld_batch* bt, const int* layer, const int* index,
                       const float* const* rho, float* l0_out, float* u0_out, float* const* l_out,
                       float* const* u_out, float* c_out, float* const* rho_out, hipStream_t s) {
  g_err.clear();
  LD_TRY(check_batch(net, bt));
  const int n = net->n, B = bt->B, nh = n - 1;
  if (B == 0) return LD_OK;
  if (!layer || !index || !l0_out || !u0_out || !l_out || !u_out || !c_out) return fail(LD_E_ARG, "NULL argument");
  if ((rho == nullptr) != (rho_out == nullptr)) return fail(LD_E_ARG, "rho and rho_out must both be given or both NULL");
  if (nh > kFsbMaxHidden) return fail(LD_E_UNSUPPORTED, "more than 16 hidden layers");
  for (int k = 0; k < nh; ++k) {
    if (!l_out[k] || !u_out[k]) return fail(LD_E_ARG, "l_out[k]/u_out[k] is NULL");
    if (rho && (!rho[k] || !rho_out[k])) return fail(LD_E_ARG, "rho[k]/rho_out[k] is NULL");
  }
  IntermPack K;
  std::memset(&K, 0, sizeof(K));
  std::vector<std::pair<const float*, float*>> arr = {{bt->l0, l0_out}, {bt->u0, u0_out}};
  std::vector<int> w = {net->n0, net->n0}, wid(nh);
  std::vector<float*> lo(nh), hi(nh);
  for (int k = 1; k <= nh; ++k) {
    arr.push_back({bt->l[k - 1], l_out[k - 1]});
    arr.push_back({bt->u[k - 1], u_out[k - 1]});
    w.push_back(width(net, k));
    w.push_back(width(net, k));
    lo[k - 1] = l_out[k - 1];
    hi[k - 1] = u_out[k - 1];
    wid[k - 1] = width(net, k);
  }
  arr.push_back({bt->c, c_out});
  w.push_back(width(net, n));
  if (rho)
    for (int k = 1; k <= nh; ++k) {
      arr.push_back({rho[k - 1], rho_out[k - 1]});
      w.push_back(width(net, k));
    }
  K.n = (int)arr.size();
  for (int a = 0; a < K.n; ++a) {
    K.src[a] = arr[a].first;
    K.dst[a] = arr[a].second;
    K.width[a] = w[a];
  }
  LD_HIP(launch_branch_children(K, B, nh, layer, index, lo.data(), hi.data(), wid.data(), s));
  return LD_OK;
}

// ---------------------------------------------------------------------------
// branch and bound (Sec. 2.3.1, Sec. 5.2, Sec. 7.3)
// ---------------------------------------------------------------------------
int ld_bab(const ld_net* net, const ld_batch* root, const ld_bab_opts* o, ld_bab_result* res, float* x_best,
           hipStream_t s) {
  g_err.clear();
  LD_TRY(check_batch(net, root));
  if (!o || !res) return fail(LD_E_ARG, "NULL argument");
  if (root->B != 1) return fail(LD_E_ARG, "the root batch must hold one subdomain");
  if (o->batch < 1 || o->root_iters < 0 || o->iters < 0 || o->max_rounds < 0 || o->max_subproblems < 1)
    return fail(LD_E_ARG, "batch, max_subproblems >= 1 and iteration counts >= 0 required");
  if (o->precision != LD_FP32 && o->precision != LD_BF16)
    return fail(LD_E_UNSUPPORTED, "branch and bound bounds with LD_FP32 or LD_BF16");
  if (std::isnan(o->threshold) || !(o->gap >= 0.f)) return fail(LD_E_ARG, "threshold must not be NaN, gap >= 0");
  if (net->n - 1 > kFsbMaxHidden) return fail(LD_E_UNSUPPORTED, "more than 16 hidden layers");
  const int n = net->n, nh = n - 1, B = o->batch, C2 = 2 * B, n0 = net->n0, nout = width(net, n);
  const long long cap = o->max_subproblems;
  // device memory: the store (l_k, u_k, rho_k per slot), the parents' and the
  // children's batches, the branching decisions, the bounds, the row pairs
  std::vector<size_t> sz;
  auto add = [&](size_t bytes) {
    sz.push_back(round_up(std::max<size_t>(bytes, 4), 256));
    return sz.size() - 1;
  };
  std::vector<size_t> i_sl, i_su, i_sr, i_pl, i_pu, i_pr, i_cl, i_cu;
  for (int k = 1; k <= nh; ++k) {
    const size_t w = (size_t)width(net, k) * 4;
    i_sl.push_back(add(cap * w));
    i_su.push_back(add(cap * w));
    i_sr.push_back(add(cap * w));
    i_pl.push_back(add(B * w));
    i_pu.push_back(add(B * w));
    i_pr.push_back(add(B * w));
    i_cl.push_back(add(C2 * w));
    i_cu.push_back(add(C2 * w));
  }
  const size_t i_pl0 = add((size_t)B * n0 * 4), i_pu0 = add((size_t)B * n0 * 4), i_pc = add((size_t)B * nout * 4);
  const size_t i_cl0 = add((size_t)C2 * n0 * 4), i_cu0 = add((size_t)C2 * n0 * 4), i_cc = add((size_t)C2 * nout * 4);
  std::vector<size_t> i_crho;
  for (int k = 1; k <= nh; ++k) i_crho.push_back(add((size_t)C2 * width(net, k) * 4));
  const size_t i_layer = add((size_t)B * 4), i_index = add((size_t)B * 4), i_value = add((size_t)B * 8);
  const size_t i_bound = add((size_t)C2 * 8), i_primal = add((size_t)C2 * 8), i_feas = add((size_t)C2 * 4);
  const size_t i_pairs = add((size_t)C2 * 8);
  std::vector<size_t> off(sz.size());
  size_t total = 0;
  for (size_t i = 0; i < sz.size(); ++i) {
    off[i] = total;
    total += sz[i];
  }
  struct Res {
    void* base = nullptr;
    ld_state* root_st = nullptr;
    ld_state* kid_st = nullptr;
    ~Res() {
      ld_state_destroy(kid_st);
      ld_state_destroy(root_st);
      if (base) (void)hipFree(base);
    }
  } r;
  if (hipMalloc(&r.base, total) != hipSuccess) return fail(LD_E_NOMEM, "branch and bound: hipMalloc of the store failed");
  char* cb = (char*)r.base;
  auto F = [&](size_t i) { return (float*)(cb + off[i]); };
  LD_TRY(ld_state_create(net, 1, &r.root_st));
  LD_TRY(ld_state_create(net, C2, &r.kid_st));
  std::vector<const float*> pl(nh), pu(nh), cl(nh), cu(nh);
  std::vector<float*> plw(nh), puw(nh), prw(nh), clw(nh), cuw(nh), crw(nh);
  for (int k = 0; k < nh; ++k) {
    plw[k] = F(i_pl[k]);
    puw[k] = F(i_pu[k]);
    prw[k] = F(i_pr[k]);
    clw[k] = F(i_cl[k]);
    cuw[k] = F(i_cu[k]);
    crw[k] = F(i_crho[k]);
    pl[k] = plw[k];
    pu[k] = puw[k];
    cl[k] = clw[k];
    cu[k] = cuw[k];
  }
  ld_batch pb{B, F(i_pl0), F(i_pu0), pl.data(), pu.data(), F(i_pc)};
  ld_batch kb{C2, F(i_cl0), F(i_cu0), cl.data(), cu.data(), F(i_cc)};
  int2* pairs = (int2*)(cb + off[i_pairs]);
  int* d_layer = (int*)(cb + off[i_layer]);
  int* d_index = (int*)(cb + off[i_index]);
  double* d_bound = (double*)(cb + off[i_bound]);
  double* d_primal = (double*)(cb + off[i_primal]);
  int* d_feas = (int*)(cb + off[i_feas]);
  // packs of row moves: the store <-> a batch; the root's box and objective to a batch
  auto pack = [&](const std::vector<const float*>& src, const std::vector<float*>& dst, const std::vector<int>& w) {
    IntermPack K;
    std::memset(&K, 0, sizeof(K));
    K.n = (int)src.size();
    for (int a = 0; a < K.n; ++a) {
      K.src[a] = src[a];
      K.dst[a] = dst[a];
      K.width[a] = w[a];
    }
    return K;
  };
  std::vector<int> wst;
  std::vector<const float*> store_src, kid_src;
  std::vector<float*> store_dst, parent_dst;
  for (int k = 0; k < nh; ++k) wst.insert(wst.end(), 3, width(net, k + 1));
  for (int k = 0; k < nh; ++k) {
    store_src.insert(store_src.end(), {F(i_sl[k]), F(i_su[k]), F(i_sr[k])});
    store_dst.insert(store_dst.end(), {F(i_sl[k]), F(i_su[k]), F(i_sr[k])});
    parent_dst.insert(parent_dst.end(), {plw[k], puw[k], prw[k]});
    kid_src.insert(kid_src.end(), {clw[k], cuw[k], r.kid_st->rho[k]});
  }
  const IntermPack gather = pack(store_src, parent_dst, wst);   // store slot -> parent row
  const IntermPack scatter = pack(kid_src, store_dst, wst);     // child row -> store slot
  const IntermPack box = pack({root->l0, root->u0, root->c}, {F(i_pl0), F(i_pu0), F(i_pc)}, {n0, n0, nout});
  std::vector<const float*> root_src;
  for (int k = 0; k < nh; ++k) root_src.insert(root_src.end(), {root->l[k], root->u[k], r.root_st->rho[k]});
  const IntermPack root_in = pack(root_src, store_dst, wst);   // the root to its slot
  // row pairs to the device; synchronous, so that the host array is never read
  // after it changes and the previous moves have finished with the device array
  auto put_pairs = [&](const std::vector<int2>& v) -> int {
    LD_HIP(hipMemcpyAsync(pairs, v.data(), v.size() * sizeof(int2), hipMemcpyHostToDevice, s));
    LD_HIP(hipStreamSynchronize(s));
    return LD_OK;
  };
  ld_opts so;
  std::memset(&so, 0, sizeof(so));
  so.beta1 = o->beta1;
  so.beta2 = o->beta2;
  so.eps = o->eps;
  so.precision = o->precision;
  so.tie_tau = o->tie_tau;
  so.engine = LD_ENGINE_LAYERWISE;
  // ---- the root ----
  so.iters = o->root_iters;
  so.total_iters = std::max(1, o->root_iters);
  so.lr0 = o->root_lr0;
  so.lr_end = o->root_lr_end;
  so.init = LD_INIT_CROWN;
  LD_TRY(ld_step(net, root, r.root_st, &so, s));
  LD_TRY(ld_final_bound(net, root, r.root_st, d_bound, nullptr, d_primal, d_feas, o->tie_tau, s));
  double hb[1], hp[1];
  int hf[1];
  LD_HIP(hipMemcpyAsync(hb, d_bound, 8, hipMemcpyDeviceToHost, s));
  LD_HIP(hipMemcpyAsync(hp, d_primal, 8, hipMemcpyDeviceToHost, s));
  LD_HIP(hipMemcpyAsync(hf, d_feas, 4, hipMemcpyDeviceToHost, s));
  LD_HIP(hipStreamSynchronize(s));
  std::memset(res, 0, sizeof(*res));
  res->incumbent = INFINITY;
  res->bounded = 1;
  std::vector<float> xb_host((size_t)n0);
  bool have_x = false;
  if (hf[0] && hp[0] < res->incumbent) {
    res->incumbent = hp[0];
    LD_HIP(hipMemcpy(xb_host.data(), r.root_st->ws.xs[0], (size_t)n0 * 4, hipMemcpyDeviceToHost));
    have_x = true;
  }
  // ---- the open subproblems: a heap on (bound, creation order) and free slots ----
  struct Open {
    double lb;
    long long seq;
    int slot;
    bool operator<(const Open& q) const { return lb > q.lb || (lb == q.lb && seq > q.seq); }
  };
  std::priority_queue<Open> open;
  std::vector<int> free_slots;
  for (long long i = cap - 1; i >= 0; --i) free_slots.push_back((int)i);
  long long seq = 0;
  double pruned_min = INFINITY, leaf_min = INFINITY;
  bool all_above = true, full = false;
  const bool has_thr = o->threshold > -INFINITY;
  auto keep = [&](double lb) -> bool {
    if (has_thr && lb > o->threshold) {
      pruned_min = std::min(pruned_min, lb);
      return false;
    }
    if (lb >= res->incumbent - o->gap) {
      pruned_min = std::min(pruned_min, lb);
      all_above = false;
      return false;
    }
    return true;
  };
  if (keep(hb[0])) {
    const int slot = free_slots.back();
    free_slots.pop_back();
    LD_TRY(put_pairs({int2{0, slot}}));
    LD_HIP(launch_bab_rows(root_in, pairs, 1, 0, s));
    open.push(Open{hb[0], seq++, slot});
  }
  res->max_open = (long long)open.size();
  std::vector<int> h_layer(B), h_index(B), h_feas(C2);
  std::vector<double> h_bound(C2), h_primal(C2);
  // ---- rounds ----
  while (!open.empty() && res->incumbent > o->threshold && res->rounds < o->max_rounds && !full) {
    res->rounds++;
    std::vector<Open> par;
    while (!open.empty() && (int)par.size() < B) {
      par.push_back(open.top());
      open.pop();
    }
    const int np = (int)par.size();
    // the parents into the batch (rows past np repeat the first parent)
    std::vector<int2> pv(B);
    for (int j = 0; j < B; ++j) pv[j] = int2{par[j < np ? j : 0].slot, j};
    LD_TRY(put_pairs(pv));
    LD_HIP(launch_bab_rows(gather, pairs, B, 0, s));
    LD_HIP(launch_bab_rows(box, pairs, B, 1, s));
    for (const Open& p : par) free_slots.push_back(p.slot);
    // split, children with their parent's duals, bound them
    LD_TRY(ld_fsb_branch(net, &pb, d_layer, d_index, (double*)(cb + off[i_value]), nullptr, s));
    std::vector<const float*> prc(prw.begin(), prw.end());
    LD_TRY(ld_branch_children(net, &pb, d_layer, d_index, prc.data(), F(i_cl0), F(i_cu0), clw.data(), cuw.data(),
                              F(i_cc), crw.data(), s));
    std::vector<const float*> crc(crw.begin(), crw.end());
    LD_TRY(ld_state_set_rho(r.kid_st, crc.data(), s));
    so.iters = o->iters;
    so.total_iters = std::max(1, o->iters);
    so.lr0 = o->lr0;
    so.lr_end = o->lr_end;
    so.init = LD_INIT_GIVEN;
    LD_TRY(ld_step(net, &kb, r.kid_st, &so, s));
    LD_TRY(ld_final_bound(net, &kb, r.kid_st, d_bound, nullptr, d_primal, d_feas, o->tie_tau, s));
    LD_HIP(hipMemcpyAsync(h_index.data(), d_index, (size_t)B * 4, hipMemcpyDeviceToHost, s));
    LD_HIP(hipMemcpyAsync(h_bound.data(), d_bound, (size_t)C2 * 8, hipMemcpyDeviceToHost, s));
    LD_HIP(hipMemcpyAsync(h_primal.data(), d_primal, (size_t)C2 * 8, hipMemcpyDeviceToHost, s));
    LD_HIP(hipMemcpyAsync(h_feas.data(), d_feas, (size_t)C2 * 4, hipMemcpyDeviceToHost, s));
    LD_HIP(hipStreamSynchronize(s));
    // incumbent, then the children that stay open
    int best = -1;
    for (int j = 0; j < np; ++j) {
      if (h_index[j] < 0) continue;
      for (int c = 2 * j; c <= 2 * j + 1; ++c)
        if (h_feas[c] && h_primal[c] < res->incumbent) {
          res->incumbent = h_primal[c];
          best = c;
        }
    }
    if (best >= 0) {
      LD_HIP(hipMemcpy(xb_host.data(), (const float*)r.kid_st->ws.xs[0] + (size_t)best * n0, (size_t)n0 * 4,
                       hipMemcpyDeviceToHost));
      have_x = true;
    }
    std::vector<int2> sv;
    for (int j = 0; j < np; ++j) {
      if (h_index[j] < 0) {  // no ambiguous ReLU left: a leaf
        res->leaves++;
        leaf_min = std::min(leaf_min, par[j].lb);
        continue;
      }
      res->bounded += 2;
      for (int c = 2 * j; c <= 2 * j + 1; ++c) {
        const double lb = std::max(h_bound[c], par[j].lb);
        if (!keep(lb)) continue;
        if (free_slots.empty()) {
          full = true;
          pruned_min = std::min(pruned_min, lb);  // dropped unexplored: still counts in the lower bound
          all_above = false;
          continue;
        }
        const int slot = free_slots.back();
        free_slots.pop_back();
        sv.push_back(int2{c, slot});
        open.push(Open{lb, seq++, slot});
      }
    }
    if (!sv.empty()) {
      LD_TRY(put_pairs(sv));
      LD_HIP(launch_bab_rows(scatter, pairs, (int)sv.size(), 0, s));
    }
    res->max_open = std::max(res->max_open, (long long)open.size());
  }
  double lower = std::min(pruned_min, leaf_min);
  const bool left_open = !open.empty();
  for (; !open.empty(); open.pop()) lower = std::min(lower, open.top().lb);
  res->lower = lower;
  if (res->incumbent <= o->threshold)
    res->status = LD_BAB_FALSIFIED;
  else if (left_open || res->leaves > 0 || full)
    res->status = LD_BAB_LIMIT;
  else
    res->status = all_above ? LD_BAB_VERIFIED : LD_BAB_SOLVED;
  if (x_best && have_x) std::memcpy(x_best, xb_host.data(), (size_t)n0 * 4);
  LD_HIP(hipStreamSynchronize(s));
  return LD_OK;
}

// ---------------------------------------------------------------------------
// sigmoid activations (App. E)
// ---------------------------------------------------------------------------
int ld_sigmoid_hull(long long count, const float* l, const float* u, float* t_up, float* t_lo, hipStream_t s) {
  g_err.clear();
  if (count < 0) return fail(LD_E_ARG, "count < 0");
  if (count == 0) return LD_OK;
  if (!l || !u || !t_up || !t_lo) return fail(LD_E_ARG, "NULL argument");
  LD_HIP(launch_sigmoid_hull(count, l, u, t_up, t_lo, s));
  return LD_OK;
}

int ld_sigmoid_inner_min(long long count, const float* rho, const float* g, const float* l, const float* u,
                         const float* t_up, const float* t_lo, float* xb, float* x, double* val, hipStream_t s) {
  g_err.clear();
  if (count < 0) return fail(LD_E_ARG, "count < 0");
  if (count == 0) return LD_OK;
  if (!rho || !g || !l || !u || !t_up || !t_lo || !xb || !x || !val) return fail(LD_E_ARG, "NULL argument");
  LD_HIP(launch_sigmoid_inner_min(count, rho, g, l, u, t_up, t_lo, xb, x, val, s));
  return LD_OK;
}

int ld_step(const ld_net* net, const ld_batch* bt, ld_state* st, const ld_opts* o, hipStream_t s) {
  g_err.clear();
  LD_TRY(check_step_args(net, bt, st, o));
  if (g_row_div > 1 && (o->precision == LD_FP64 || o->engine == LD_ENGINE_RESIDENT))
    return fail(LD_E_UNSUPPORTED, "shared bound rows need the FP32/BF16 layer-wise engine");
  if (st->track && (o->precision == LD_FP64 || o->engine == LD_ENGINE_RESIDENT))
    return fail(LD_E_UNSUPPORTED, "keeping the best value needs the FP32/BF16 layer-wise engine");
  LD_TRY(validate_values(net, bt, st->ws, s));
  if (o->precision == LD_FP64) {
    LD_TRY(f64_ensure_initialised(net, bt, st, o, s));
    for (int i = 0; i < o->iters; ++i) LD_TRY(f64_iteration(net, bt, st, o, s));
    st->t_host = st->f64.t;
    LD_HIP(launch_fill_i32(st->t_dev, 1, st->f64.t, s));
    LD_HIP(hipEventRecord(st->done, s));
    return LD_OK;
  }
  ld_opts eo = *o;
  const int mma = o->precision == LD_BF16 ? 1 : 0;
  if (eo.engine == LD_ENGINE_AUTO && bt->B > 0) {
    if (tuned_engine(net, bt->B, mma) < 0) LD_TRY(autotune_impl(net, bt, o, s));
    eo.engine = st->track ? LD_ENGINE_LAYERWISE : tuned_engine(net, bt->B, mma);
  }
  LD_TRY(ensure_initialised(net, bt, st, &eo, s));
  const int rc = step_impl(net, bt, st, &eo, s);
  LD_HIP(hipEventRecord(st->done, s));
  return rc;
}

int ld_autotune(const ld_net* net, const ld_batch* bt, const ld_opts* o, hipStream_t s) {
  g_err.clear();
  if (!net || !o) return fail(LD_E_ARG, "NULL argument");
  LD_TRY(check_batch(net, bt));
  if (o->precision != LD_FP32 && o->precision != LD_BF16) return fail(LD_E_ARG, "unknown precision");
  return autotune_impl(net, bt, o, s);
}

static void to_ld_tile(const Tile& t, ld_tile* o) {
  o->tn = t.tn;
  o->mwaves = t.wm;
  o->kwaves = t.tm;
  o->splits = t.splits;
  o->form = t.form;
}

int ld_tuned_config(const ld_net* net, int B, int precision, int k, int dir, ld_tile* tile, double* us) {
  g_err.clear();
  if (!net || !tile || !us) return fail(LD_E_ARG, "NULL argument");
  if (k < 1 || k > net->n - 1 || (dir != 0 && dir != 1)) return fail(LD_E_ARG, "layer or direction out of range");
  ld_net* mnet = const_cast<ld_net*>(net);
  std::lock_guard<std::mutex> lk(mnet->mu);
  const auto key = std::make_tuple(k - 1, dir, B, precision == LD_BF16 ? 1 : 0);
  auto it = mnet->tiles.find(key);
  if (it == mnet->tiles.end()) return fail(LD_E_STATE, "no tuned configuration for this batch size and precision");
  to_ld_tile(it->second, tile);
  *us = mnet->tile_us[key];
  return LD_OK;
}

int ld_tile_candidates(const ld_net* net, int B, int k, int dir, ld_tile* out, int max_count, int* count) {
  g_err.clear();
  if (!net || !count || (max_count > 0 && !out)) return fail(LD_E_ARG, "NULL argument");
  if (k < 1 || k > net->n - 1 || (dir != 0 && dir != 1) || B < 0) return fail(LD_E_ARG, "layer or direction out of range");
  const Job& J = dir ? net->L[k - 1].tr : net->L[k - 1].fwd;
  const std::vector<Tile> c = tile_candidates(J, B);
  *count = (int)c.size();
  for (int i = 0; i < std::min(max_count, (int)c.size()); ++i) to_ld_tile(c[i], out + i);
  return LD_OK;
}

int ld_set_tuned_config(ld_net* net, int B, int precision, int k, int dir, const ld_tile* tile) {
  g_err.clear();
  if (!net || !tile) return fail(LD_E_ARG, "NULL argument");
  if (k < 1 || k > net->n - 1 || (dir != 0 && dir != 1) || B < 0) return fail(LD_E_ARG, "layer or direction out of range");
  const Job& J = dir ? net->L[k - 1].tr : net->L[k - 1].fwd;
  for (const Tile& t : tile_candidates(J, B))
    if (t.tn == tile->tn && t.wm == tile->mwaves && t.tm == tile->kwaves && t.splits == tile->splits &&
        t.form == tile->form) {
      std::lock_guard<std::mutex> lk(net->mu);
      const auto key = std::make_tuple(k - 1, dir, B, precision == LD_BF16 ? 1 : 0);
      net->tiles[key] = t;
      net->tile_us[key] = 0.0;
      net->tune_gen++;
      return LD_OK;
    }
  return fail(LD_E_ARG, "not a candidate configuration of this contraction");
}

int ld_tuned_engine(const ld_net* net, int B, int precision, int* engine, int* concurrent, double* us_layerwise,
                    double* us_resident) {
  g_err.clear();
  if (!net || !engine || !concurrent || !us_layerwise || !us_resident) return fail(LD_E_ARG, "NULL argument");
  ld_net* mnet = const_cast<ld_net*>(net);
  std::lock_guard<std::mutex> lk(mnet->mu);
  auto it = mnet->engines.find({B, precision == LD_BF16 ? 1 : 0});
  if (it == mnet->engines.end()) return fail(LD_E_STATE, "no tuned engine for this batch size and precision");
  *engine = (int)it->second[0];
  *concurrent = 1;  // the layer jobs of a phase are independent branches of the captured graph
  *us_layerwise = it->second[1];
  *us_resident = it->second[2];
  return LD_OK;
}

int ld_state_set_tracking(ld_state* st, int on, hipStream_t s) {
  g_err.clear();
  if (!st) return fail(LD_E_ARG, "state is NULL");
  if (on && !st->track_base) {
    const size_t qb = round_up((size_t)std::max(st->B, 1) * 8, 256);
    const size_t tb = round_up((size_t)std::max(st->B, 1) * 4, 256);
    if (hipMalloc(&st->track_base, qb + tb + 256) != hipSuccess) {
      st->track_base = nullptr;
      return fail(LD_E_NOMEM, "tracking hipMalloc failed");
    }
    st->best_q = (double*)st->track_base;
    st->best_t = (int*)((char*)st->track_base + qb);
    st->track_step = (int*)((char*)st->track_base + qb + tb);
  }
  if (on) {
    LD_TRY(ws_alloc(st->net, st->tws, st->B));
    if (st->B > 0) {
      LD_HIP(launch_fill_f64(st->best_q, (size_t)st->B, -INFINITY, s));
      LD_HIP(launch_fill_i32(st->best_t, (size_t)st->B, 0, s));
    }
    LD_HIP(launch_fill_i32(st->track_step, 1, st->t_host, s));
  }
  st->track = on != 0;
  LD_HIP(hipEventRecord(st->done, s));
  return LD_OK;
}

int ld_state_get_best(const ld_state* st, double* best_q, int* best_t, hipStream_t s) {
  g_err.clear();
  if (!st) return fail(LD_E_ARG, "state is NULL");
  if (!st->track_base) return fail(LD_E_STATE, "the state never kept its best value (ld_state_set_tracking)");
  if (st->B == 0) return LD_OK;
  if (best_q) LD_HIP(hipMemcpyAsync(best_q, st->best_q, (size_t)st->B * 8, hipMemcpyDeviceToDevice, s));
  if (best_t) LD_HIP(hipMemcpyAsync(best_t, st->best_t, (size_t)st->B * 4, hipMemcpyDeviceToDevice, s));
  return LD_OK;
}

int ld_state_reset(ld_state* st, hipStream_t s) {
  g_err.clear();
  if (!st) return fail(LD_E_ARG, "state is NULL");
  LD_HIP(hipMemsetAsync(st->t_dev, 0, 4, s));
  st->t_host = 0;
  st->initialized = false;
  st->f64.active = false;
  if (st->track) {  // a new ascent starts a new record
    if (st->B > 0) {
      LD_HIP(launch_fill_f64(st->best_q, (size_t)st->B, -INFINITY, s));
      LD_HIP(launch_fill_i32(st->best_t, (size_t)st->B, 0, s));
    }
    LD_HIP(launch_fill_i32(st->track_step, 1, 0, s));
  }
  st->px.ready = false;
  st->px.t = 0;
  LD_HIP(hipEventRecord(st->done, s));
  return LD_OK;
}

int ld_profile_iteration(const ld_net* net, const ld_batch* bt, ld_state* st, const ld_opts* o, int reps,
                         double* avg_us, int* kinds, int max_slots, int* n_slots, hipStream_t s) {
  g_err.clear();
  LD_TRY(check_step_args(net, bt, st, o));
  if (reps <= 0 || !avg_us || !kinds || !n_slots || max_slots <= 0) return fail(LD_E_ARG, "bad profile arguments");
  if (o->precision == LD_FP64) return fail(LD_E_UNSUPPORTED, "per-launch profiles cover the FP32 and BF16 engines");
  LD_TRY(ensure_initialised(net, bt, st, o, s));
  const int n = net->n, B = bt->B, mma = o->precision == LD_BF16 ? 1 : 0;
  LD_TRY(iteration(net, bt, st, o, s));  // x* of every layer in the operand precision
  st->t_host += 1;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  LD_HIP(hipEventCreate(&e0));
  LD_HIP(hipEventCreate(&e1));
  struct EventGuard {
    hipEvent_t a, b;
    ~EventGuard() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } eguard{e0, e1};
  std::vector<const float*> rho(st->rho.begin(), st->rho.end());
  int ns = 0;
  for (int dir = 1; dir >= 0; --dir)
    for (int k = 1; k <= n - 1 && ns < max_slots; ++k) {
      const Job& J = dir ? net->L[k - 1].tr : net->L[k - 1].fwd;
      const Tile t = pick_tile(net, k - 1, dir, B, mma);
      auto launch = [&]() -> int {
        if (dir == 1) {
          const EpiArgs e = epi_phase_a(net, bt, rho.data(), st->ws, mma, o->tie_tau, 0, nullptr, nullptr, nullptr, k);
          LD_HIP(run_job(J, B, rho[k - 1], 0, tr_mode(mma, k), e, t, st->ws, k - 1, s));
        } else {
          const EpiArgs e = epi_phase_b(net, bt, st, o, k);
          LD_HIP(run_job(J, B, st->ws.xs[k - 1], mma, mma, e, t, st->ws, k - 1, s));
        }
        return LD_OK;
      };
      LD_TRY(launch());  // warm-up
      LD_HIP(hipEventRecord(e0, s));
      for (int r = 0; r < reps; ++r) LD_TRY(launch());
      LD_HIP(hipEventRecord(e1, s));
      LD_HIP(hipEventSynchronize(e1));
      float ms = 0.f;
      LD_HIP(hipEventElapsedTime(&ms, e0, e1));
      avg_us[ns] = 1000.0 * ms / reps;
      kinds[ns] = (dir ? 100 : 300) + k;
      ++ns;
    }
  *n_slots = ns;
  LD_HIP(hipEventRecord(st->done, s));
  return LD_OK;
}

int ld_final_bound(const ld_net* net, const ld_batch* bt, const ld_state* cst, double* bound, double* q_final,
                   double* primal, int* feasible, float tie_tau, hipStream_t s) {
  g_err.clear();
  LD_TRY(check_batch(net, bt));
  if (!cst) return fail(LD_E_ARG, "state is NULL");
  if (cst->net != net || cst->B != bt->B) return fail(LD_E_STATE, "state was created for another net or batch size");
  if (!cst->initialized) return fail(LD_E_STATE, "state has not been initialised by ld_step");
  if (!(tie_tau >= 0.f) || !std::isfinite(tie_tau)) return fail(LD_E_ARG, "tie_tau must be finite and >= 0");
  ld_state* st = const_cast<ld_state*>(cst);
  const int n = net->n, B = bt->B;
  Workspace& ws = st->ws;
  LD_TRY(validate_values(net, bt, ws, s));
  if (st->f64.active) {
    // FP64 state: q(rho^T) and the primal point in FP64
    Workspace64& w64 = st->f64.ws;
    double* qf64 = q_final ? q_final : w64.qtmp;
    std::vector<const double*> r64(st->f64.rho.begin(), st->f64.rho.end());
    LD_TRY(f64_dual_eval_impl(net, bt, r64.data(), w64, qf64, nullptr, nullptr, tie_tau, s));
    if (bound) LD_HIP(launch_max_f64(B, st->f64.q0, qf64, bound, s));
    if (primal || feasible) LD_TRY(f64_primal(net, bt, w64, primal, feasible, s));
    LD_HIP(hipEventRecord(st->done, s));
    return LD_OK;
  }
  double* qf = q_final ? q_final : ws.qtmp;
  std::vector<const float*> r(st->rho.begin(), st->rho.end());
  LD_TRY(dual_eval_impl(net, bt, r.data(), ws, qf, nullptr, LD_FP32, tie_tau, s));
  if (bound) LD_HIP(launch_max_f64(B, st->q0, qf, bound, s));
  if (primal || feasible) {
    int* flag = feasible ? feasible : ws.flag;
    LD_HIP(launch_fill_i32(flag, (size_t)B, 1, s));
    const float* x = (const float*)ws.xs[0];
    float* bufs[2] = {ws.act0, ws.act1};
    for (int k = 1; k <= n; ++k) {
      const Layer& L = net->L[k - 1];
      EpiArgs e = epi0();
      e.bias = L.bias;
      e.out_f = bufs[k & 1];
      if (k < n) {
        e.kind = EPI_RELU_FWD;
        e.lo = bt->l[k - 1];
        e.hi = bt->u[k - 1];
        e.flag = flag;
      } else {
        e.kind = EPI_BIAS_STORE;
      }
      LD_HIP(run_job(L.fwd, B, x, 0, 0, e, pick_tile(net, k - 1, 0, B, 0), ws, k - 1, s));
      x = bufs[k & 1];
    }
    if (primal) LD_HIP(launch_cdot(B, net->L[n - 1].n_out, bt->c, x, nullptr, 1, primal, s));
  }
  LD_HIP(hipEventRecord(st->done, s));
  return LD_OK;
}

}  // extern "C"
