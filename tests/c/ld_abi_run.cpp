// A host program that uses the library through its C ABI alone (include/ld.h,
// the HIP runtime for device memory, no Python or torch): it reads a network and
// a batch of subdomains from a raw file, runs the supergradient method (CROWN
// initialisation, T Adam steps, Sec. 3.2 and Sec. 7.2) and prints the final bound
// of every subdomain (ld_final_bound).
//
// File layout (little-endian int32 header, then float32 arrays):
//   n_layers B, then per layer kind in_c in_h in_w out_c out_h out_w kh kw stride pad,
//   then per layer W and b, then l0 u0 [B, n_0], l_k u_k [B, n_k] for every hidden
//   layer, c [B, n_out].
// Usage: ld_abi_run FILE T PRECISION(0 FP32, 1 BF16).  Prints "bound <b> <value>".
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "ld.h"

#define CHECK_LD(x)                                                          \
  do {                                                                       \
    const int rc_ = (x);                                                     \
    if (rc_ != LD_OK) {                                                      \
      std::fprintf(stderr, "%s failed (%d): %s\n", #x, rc_, ld_last_error()); \
      return 1;                                                              \
    }                                                                        \
  } while (0)
#define CHECK_HIP(x)                                                                  \
  do {                                                                                \
    const hipError_t e_ = (x);                                                        \
    if (e_ != hipSuccess) {                                                           \
      std::fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));             \
      return 1;                                                                       \
    }                                                                                 \
  } while (0)

static bool read_floats(FILE* f, std::vector<float>& v, size_t n) {
  v.resize(n);
  return std::fread(v.data(), sizeof(float), n, f) == n;
}

int main(int argc, char** argv) {
  if (argc != 4) {
    std::fprintf(stderr, "usage: %s FILE T PRECISION\n", argv[0]);
    return 2;
  }
  const int T = std::atoi(argv[2]);
  const int precision = std::atoi(argv[3]);
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) {
    std::fprintf(stderr, "cannot open %s\n", argv[1]);
    return 2;
  }
  int hdr[2];
  if (std::fread(hdr, sizeof(int), 2, f) != 2) return 2;
  const int n = hdr[0], B = hdr[1];
  if (n < 2 || n > 64 || B < 1) return 2;
  std::vector<ld_layer> layers(n);
  std::vector<std::vector<float>> W(n), bias(n);
  for (int k = 0; k < n; ++k) {
    int s[11];
    if (std::fread(s, sizeof(int), 11, f) != 11) return 2;
    ld_layer& L = layers[k];
    L.kind = s[0];
    L.in_c = s[1];
    L.in_h = s[2];
    L.in_w = s[3];
    L.out_c = s[4];
    L.out_h = s[5];
    L.out_w = s[6];
    L.kh = s[7];
    L.kw = s[8];
    L.stride = s[9];
    L.pad = s[10];
  }
  std::vector<size_t> width(n + 1);
  width[0] = (size_t)layers[0].in_c * layers[0].in_h * layers[0].in_w;
  for (int k = 0; k < n; ++k) {
    const ld_layer& L = layers[k];
    const size_t nw = L.kind == LD_LINEAR ? (size_t)L.out_c * L.in_c * L.in_h * L.in_w
                                          : (size_t)L.out_c * L.in_c * L.kh * L.kw;
    if (!read_floats(f, W[k], nw) || !read_floats(f, bias[k], L.out_c)) return 2;
    layers[k].W = W[k].data();
    layers[k].b = bias[k].data();
    width[k + 1] = (size_t)L.out_c * L.out_h * L.out_w;
  }
  // per-subdomain arrays: l0, u0, then l_k, u_k of the hidden layers, then c
  std::vector<size_t> cnt = {width[0], width[0]};
  for (int k = 1; k < n; ++k) {
    cnt.push_back(width[k]);
    cnt.push_back(width[k]);
  }
  cnt.push_back(width[n]);
  std::vector<float*> dev(cnt.size(), nullptr);
  for (size_t a = 0; a < cnt.size(); ++a) {
    std::vector<float> h;
    if (!read_floats(f, h, (size_t)B * cnt[a])) return 2;
    CHECK_HIP(hipMalloc(&dev[a], h.size() * sizeof(float)));
    CHECK_HIP(hipMemcpy(dev[a], h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice));
  }
  std::fclose(f);

  ld_net* net = nullptr;
  CHECK_LD(ld_create_net(layers.data(), n, &net));
  std::vector<const float*> lk, uk;
  for (int k = 1; k < n; ++k) {
    lk.push_back(dev[2 * k]);
    uk.push_back(dev[2 * k + 1]);
  }
  ld_batch batch;
  batch.B = B;
  batch.l0 = dev[0];
  batch.u0 = dev[1];
  batch.l = lk.data();
  batch.u = uk.data();
  batch.c = dev[cnt.size() - 1];

  ld_state* st = nullptr;
  CHECK_LD(ld_state_create(net, B, &st));
  ld_opts o;
  o.iters = T;
  o.total_iters = T;
  o.lr0 = 1e-2f;
  o.lr_end = 1e-4f;
  o.beta1 = 0.9f;
  o.beta2 = 0.999f;
  o.eps = 1e-8f;
  o.precision = precision;
  o.init = LD_INIT_CROWN;
  o.tie_tau = 1.0f / (1 << 20);
  o.engine = LD_ENGINE_LAYERWISE;
  hipStream_t s = nullptr;
  CHECK_HIP(hipStreamCreate(&s));
  CHECK_LD(ld_step(net, &batch, st, &o, s));
  double* bound = nullptr;
  CHECK_HIP(hipMalloc(&bound, B * sizeof(double)));
  CHECK_LD(ld_final_bound(net, &batch, st, bound, nullptr, nullptr, nullptr, o.tie_tau, s));
  std::vector<double> hb(B);
  CHECK_HIP(hipMemcpyAsync(hb.data(), bound, B * sizeof(double), hipMemcpyDeviceToHost, s));
  CHECK_HIP(hipStreamSynchronize(s));
  for (int b = 0; b < B; ++b) std::printf("bound %d %.17g\n", b, hb[b]);

  ld_state_destroy(st);
  ld_destroy_net(net);
  CHECK_HIP(hipFree(bound));
  for (float* p : dev) CHECK_HIP(hipFree(p));
  CHECK_HIP(hipStreamDestroy(s));
  return 0;
}
