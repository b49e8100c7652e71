/*
 * ld.h -- C ABI of the MI355X (gfx950) Lagrangian-decomposition bounding library.
 *
 * The library computes lower bounds for the neural-network verification problem
 * of De Palma et al., "Improved Branch and Bound for Neural Network Verification
 * via Lagrangian Decomposition":
 *
 *   min  c^T x_n   s.t.  x_0 in [l_0, u_0],
 *                        xhat_k = W_k x_{k-1} + b_k,      k = 1..n
 *                        x_k = max(xhat_k, 0),            k = 1..n-1
 *
 * (Sec. 2.1, eq:noncvx_pb; the property is folded into the objective vector c,
 * which is the paper's canonical form with the dummy output dual rho_n = -c).
 * Each hidden layer k carries intermediate bounds xhat_k in [l_k, u_k]
 * (Sec. 2.2.3).  The bound is the Lagrangian-decomposition dual q(rho)
 * (Sec. 3.1, eq:nonprox_problem), maximised by supergradient ascent with Adam
 * steps (Algorithm 1, Sec. 3.2; Adam and the linear step decay of Sec. 7.2).
 *
 * Conventions shared by every entry point
 *  - A "batch" is B independent subdomains of one network (Sec. 5.2.2: the branch-and-bound
 *    framework bounds a batch of subproblems at once).  Every per-subdomain
 *    array is row-major [B, n] with n the width of that layer; conv activations
 *    are flattened in (C, H, W) order.
 *  - Array arguments marked "device" are device pointers owned by the caller;
 *    they must stay valid until the work enqueued on `stream` has completed.
 *    Arrays marked "host" are read before the call returns.
 *  - Work is enqueued on `stream` (0 = the null stream).  Functions that return
 *    values to the host (status of validation) synchronise `stream` first.
 *  - Every function returns LD_OK (0) or a negative error code; the message of
 *    the last error on the calling thread is returned by ld_last_error().  No
 *    C++ exception crosses this boundary.  Arguments are validated on the host
 *    before anything is enqueued; a failed validation enqueues nothing.
 *    Asynchronous device faults surface as LD_E_DEVICE on a later call.
 *  - Calls that share one ld_net (or one ld_state) must not run concurrently:
 *    the net holds a scratch workspace and the state holds the ascent buffers.
 */
#ifndef LD_H_
#define LD_H_

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------------- */
/* status codes                                                              */
/* ------------------------------------------------------------------------- */
enum {
  LD_OK = 0,
  LD_E_ARG = -1,         /* null pointer, bad enum value, bad size               */
  LD_E_SHAPE = -2,       /* inconsistent layer or batch shapes                   */
  LD_E_NUMERIC = -3,     /* NaN/Inf in an input, or l > u somewhere              */
  LD_E_NOMEM = -4,       /* device or host allocation failed                     */
  LD_E_DEVICE = -5,      /* a HIP call failed (includes asynchronous faults)     */
  LD_E_UNSUPPORTED = -6, /* valid request the library does not implement        */
  LD_E_STATE = -7        /* state used with a different net or batch size        */
};

enum { LD_LINEAR = 0, LD_CONV2D = 1 };          /* layer kinds (Sec. 2.1)          */
/* arithmetic of the ascent: FP32 or BF16 operands of the contractions (FP32
 * state), or FP64 operands, accumulations and state (the FP64 engine) */
enum { LD_FP32 = 0, LD_BF16 = 1, LD_FP64 = 2 };
/* dual initialisation: CROWN's or WK's dual assignment (Prop. 2, Sec. 4.1),
 * zeros, or duals set by the caller */
enum { LD_INIT_CROWN = 0, LD_INIT_ZERO = 1, LD_INIT_GIVEN = 2, LD_INIT_WK = 3 };
enum { LD_ENGINE_AUTO = 0, LD_ENGINE_RESIDENT = 1, LD_ENGINE_LAYERWISE = 2 };

/* ------------------------------------------------------------------------- */
/* network                                                                   */
/* ------------------------------------------------------------------------- */
/* One affine layer xhat_k = W_k x_{k-1} + b_k (Sec. 2.1, fully connected or
 * convolutional; Sec. 5.2 keeps convolutions as kernels, never as dense
 * matrices).
 *  LD_LINEAR: W is host [out_c, in_c*in_h*in_w] row-major, b host [out_c];
 *             out_h = out_w = 1.  The input may be a flattened (C,H,W) map.
 *  LD_CONV2D: W is host [out_c, in_c, kh, kw], b host [out_c] (one bias per
 *             output channel, broadcast over H x W); zero padding `pad` and
 *             `stride` on both axes; out_h = (in_h + 2 pad - kh) / stride + 1.
 * Consecutive layers must agree in size (out of layer k = in of layer k+1).
 * A ReLU follows every layer but the last. */
typedef struct ld_layer {
  int kind;
  int in_c, in_h, in_w;
  int out_c, out_h, out_w;
  int kh, kw, stride, pad;
  const float* W;
  const float* b;
} ld_layer;

typedef struct ld_net ld_net;

/* Validate the layer list (n_layers >= 2, shapes chained, output-size formula
 * for convs; the last layer, whose output the objective c weighs, may be a conv,
 * as in the sub-network of an intermediate bound), copy the weights to the device and
 * repack them into the tile-major FP32 and BF16 operand layouts the kernels
 * use.  Synchronous.  *out receives a handle to free with ld_destroy_net. */
int ld_create_net(const ld_layer* layers, int n_layers, ld_net** out);
void ld_destroy_net(ld_net* net);

/* Sizes: number of layers n, input width n_0, output width n_out, and the
 * width of layer k (k = 1..n; width of layer 0 is n_0). */
int ld_net_layer_width(const ld_net* net, int k, int* width);
int ld_net_num_layers(const ld_net* net, int* n_layers);

/* ------------------------------------------------------------------------- */
/* batch of subdomains                                                       */
/* ------------------------------------------------------------------------- */
/* l0, u0 : device [B, n_0], the input box C = [l0, u0] (Sec. 3.2.1).
 * l, u   : host arrays of n-1 device pointers; l[k-1], u[k-1] are [B, n_k],
 *          the intermediate bounds of hidden layer k (Sec. 2.2.3).  A split
 *          ReLU is expressed by l = 0 (active) or u = 0 (inactive) (Sec. 2.3.2).
 * c      : device [B, n_out], the objective c^T x_n of each subdomain
 *          (e.g. e_t - e_j for a robustness margin, Sec. 7.1).
 * All values must be finite with l <= u (else LD_E_NUMERIC when validation is
 * on).  ReLU status follows Sec. 2.3.2: passing if l >= 0, else blocking if
 * u <= 0, else ambiguous. */
typedef struct ld_batch {
  int B;
  const float* l0;
  const float* u0;
  const float* const* l;
  const float* const* u;
  const float* c;
} ld_batch;

/* Turn the device-side validation of batch values (finite, l <= u) on (1,
 * default) or off (0) for this thread.  Validation costs one extra kernel and
 * one synchronisation of `stream` per call; shapes are always checked. */
void ld_set_validation(int on);

/* ------------------------------------------------------------------------- */
/* ascent state (duals rho_k, Adam moments, step counter)                    */
/* ------------------------------------------------------------------------- */
typedef struct ld_state ld_state;

/* Device state for B subdomains of `net`: rho_k, m_k, v_k (FP32, [B, n_k] for
 * k = 1..n-1), the step counter t, q(rho^0), and the workspace of the ascent.
 * The state must be used with this net and batch size only (LD_E_STATE). */
int ld_state_create(const ld_net* net, int B, ld_state** out);
void ld_state_destroy(ld_state* st);
/* Copy duals in (rho: host array of n-1 device pointers [B, n_k]); resets the
 * Adam moments and t to 0 and marks the state as initialised, so that ld_step
 * with init = LD_INIT_GIVEN continues from these duals (warm start from a
 * parent subdomain, Sec. 8.2). */
int ld_state_set_rho(ld_state* st, const float* const* rho, hipStream_t stream);
/* Copy the current duals out (host array of n-1 device pointers); the duals of
 * a state stepped in LD_FP64 are rounded to FP32. */
int ld_state_get_rho(const ld_state* st, float* const* rho, hipStream_t stream);
/* The current duals in FP64 (host array of n-1 device pointers, double [B, n_k]):
 * the FP64 engine's duals, or the FP32 duals widened. */
int ld_state_get_rho_f64(const ld_state* st, double* const* rho, hipStream_t stream);
/* Number of Adam steps taken so far (synchronises `stream`). */
int ld_state_get_step(const ld_state* st, hipStream_t stream, int* t);
/* Mark the state as fresh: the next ld_step initialises the duals again (per its
 * `init`), zeroes the Adam moments and the step counter and recomputes q(rho^0).
 * Buffers, tuned tiles and the captured graph are kept, so a bounding run can be
 * repeated on new subdomain data of the same shape without allocation. */
int ld_state_reset(ld_state* st, hipStream_t stream);
/* Keep the ascent's best dual value (optional).  Every dual value q(rho^t) is a
 * lower bound of the subdomain's minimum (weak duality, Sec. 3.1); with `on`, each
 * later step t of ld_step (FP32 or BF16, layer-wise engine: LD_ENGINE_AUTO takes
 * it, LD_FP64 and LD_ENGINE_RESIDENT return LD_E_UNSUPPORTED) also evaluates
 * q(rho^{t-1}) at the duals it starts from, as ld_dual_eval does with FP32
 * operands (in buffers of its own, beside the step's transposed products; the
 * ascent itself is unchanged), and keeps per subdomain the largest value and
 * that t.  Turning it on starts an empty record (value -inf, step 0), and so do
 * ld_state_reset and ld_state_set_rho while it is on; `on` = 0 stops it and keeps
 * the record.  Each tracked step costs one more FP32 dual evaluation. */
int ld_state_set_tracking(ld_state* st, int on, hipStream_t stream);
/* The record of ld_state_set_tracking: best_q (device double [B], may be NULL)
 * and best_t (device int [B], may be NULL).  LD_E_STATE if tracking was never on. */
int ld_state_get_best(const ld_state* st, double* best_q, int* best_t, hipStream_t stream);

/* ------------------------------------------------------------------------- */
/* dual initialisation (Prop. 2)                                              */
/* ------------------------------------------------------------------------- */
/* Dual point of the CROWN propagation bound: one backward pass
 * rho_k = a_up [g_k]_+ + a_lo [g_k]_-,  g_k = W_{k+1}^T rho_{k+1}, rho_n = -c
 * (eq:salman-assignment; slopes: chord upper slope u/(u-l), lower slope
 * 1[u >= -l] for ambiguous ReLUs, Sec. 4.2 footnote), at which q equals the
 * CROWN bound (Prop. 2).  init = LD_INIT_WK takes the chord as both slopes (the
 * WK bound's dual point); init = LD_INIT_ZERO writes zeros.  rho: host array of
 * n-1 device pointers [B, n_k] that receive the duals.  precision: operand type
 * of the backward pass (LD_FP64: propagated in FP64, rounded to FP32 on output). */
int ld_init_duals(const ld_net* net, const ld_batch* batch, int init, int precision,
                  float* const* rho, hipStream_t stream);

/* ------------------------------------------------------------------------- */
/* dual evaluation (eq:nonprox_problem)                                       */
/* ------------------------------------------------------------------------- */
/* q(rho) for every subdomain, by the closed-form inner minimisations over P_0
 * (box, eq:box_bounds_sol) and P_k (ReLU hull vertices, eq:min-pk), summed in
 * FP64 (q: device double [B]).  If `supergrad` is not NULL (host array of n-1
 * device pointers [B, n_k]) it receives the supergradient
 * s_k = xhat_B,k* - xhat_A,k* (Algorithm 1).  rho: host array of n-1 device
 * pointers [B, n_k].  `precision` selects the operand type of the
 * contractions (the inner minimisation and the sum are FP32/FP64 regardless);
 * LD_FP64 widens rho and evaluates everything in FP64 (the supergradient is
 * rounded to FP32 on output).
 * Ties of the inner minimisation are broken towards the larger xhat_B within
 * the relative band `tie_tau` (0 = exact argmin); the value is exact.
 * Uses a workspace owned by the net: calls on one net must not overlap on
 * different streams (serialise them, or use one net per stream). */
int ld_dual_eval(const ld_net* net, const ld_batch* batch, const float* const* rho,
                 double* q, float* const* supergrad, int precision, float tie_tau,
                 hipStream_t stream);
/* As ld_dual_eval (LD_FP32 or LD_BF16), for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  It allocates nothing: its workspace is a 64 MiB array of the
 * library in each device's memory, held for the life of the process (the call
 * returns LD_E_NOMEM, with the size it needs, for a batch whose workspace does not
 * fit: about 137 KB per subdomain of the wide conv net).  Every call on a device
 * shares that device's array and leaves its contents behind; calls that overlap
 * on one device (several streams or threads) race.  Fully-connected products run
 * without split-K, so results can differ from ld_dual_eval's in summation order.
 * With validation on (ld_set_validation) the call synchronises `stream`; turn it
 * off to capture the call in a graph. */
int ld_dual_eval_noalloc(const ld_net* net, const ld_batch* batch, const float* const* rho, double* q,
                         float* const* supergrad, int precision, float tie_tau, hipStream_t stream);
/* As ld_dual_eval in FP64 with FP64 duals: rho host array of n-1 device pointers
 * double [B, n_k]; supergrad (optional) double [B, n_k].  Same workspace rules. */
int ld_dual_eval_f64(const ld_net* net, const ld_batch* batch, const double* const* rho, double* q,
                     double* const* supergrad, float tie_tau, hipStream_t stream);

/* Rounding margin of the FP32-operand dual value (ld_dual_eval with LD_FP32, and
 * ld_final_bound): margin[b] (device double [B]) bounds how far the value it
 * returns can sit above the exact q(rho) at the same FP32 duals, so
 * q - margin is a lower bound of q(rho) and, by weak duality (Sec. 3.1), of the
 * subdomain's minimum even with the products' rounding counted.  The paper works
 * in exact arithmetic; every coefficient g_{k-1} = W_k^T rho_k (and the constant
 * -W_n^T c) is a dot product of K terms rounded in single precision, which errs by
 * at most gamma_K |W_k|^T |rho_k| with gamma_K = K u / (1 - K u), u = 2^-24
 * (Higham's bound, any summation order, with or without fused multiply-adds); it
 * enters one inner minimisation (eq:box_bounds_sol, eq:min-pk) multiplied by
 * x_{k-1}, whose feasible |x| is at most max(|l0|, |u0|) on the input box and
 * max(0, u) after a ReLU.  So
 *   margin[b] = sum_k sum_j (gamma_K (|W_k|^T |rho_k|)_j + 2 K 2^-126) max|x_{k-1,j}|
 * with K the layer's outputs (fully connected) or, for a conv, Co ceil(kh/stride)
 * ceil(kw/stride) (the taps that reach one input position), evaluated in
 * FP64 from the FP64 copies of the weights.  The rest of q (inner minimisation
 * values, bias terms, c . b_n) is formed from FP32 values in FP64 and its rounding,
 * below 2^-40 of q's terms, is not counted; the margin's own FP64 sums are
 * covered by widening it by 2^-30.  rho: host array of n-1 device pointers
 * [B, n_k].  With B = 0 it does nothing (margin may be NULL).  Uses the net's
 * workspace, like ld_dual_eval. */
int ld_rounding_margin(const ld_net* net, const ld_batch* batch, const float* const* rho, double* margin,
                       hipStream_t stream);

/* ------------------------------------------------------------------------- */
/* ascent (Algorithm 1 with Adam)                                             */
/* ------------------------------------------------------------------------- */
/* iters       Adam steps to take in this call (>= 0)
 * total_iters length of the step schedule: step t (1-based, counted over all
 *             calls on this state) uses lr0 + (lr_end - lr0) (t-1)/(total_iters-1),
 *             so several calls of k steps equal one call of their sum.
 * beta1, beta2, eps  Adam constants; the update is an ascent step
 *             rho += lr_t * mhat / (sqrt(vhat) + eps) with bias correction.
 * precision   LD_FP32, LD_BF16 or LD_FP64 for the contractions of the ascent.
 *             LD_FP64: the FP64 engine; duals, Adam moments, every product,
 *             sum, square root and division in FP64 (IEEE, no fused
 *             multiply-adds), the Adam constants and step sizes widened from
 *             the float fields below; `engine` is ignored.  A state keeps the
 *             family it was initialised in: an FP64 step on a state initialised
 *             in FP32/BF16 (or the reverse) returns LD_E_STATE until
 *             ld_state_reset or ld_state_set_rho.  LD_BF16:
 *             every contraction runs on BF16 MFMA with FP32 accumulation; the
 *             forward products W_k x and the product W_1^T rho_1 into the input
 *             box take plain BF16 operands, while the products W_k^T rho_k
 *             (k >= 2) whose result decides a ReLU layer's inner minimisation
 *             are compensated: each operand is a BF16 head plus a BF16
 *             remainder and three MFMA terms are summed (head*head + head*rem
 *             + rem*head).  The constant -W_n^T c is formed with FP32 operands
 *             in both precisions.  The resident engine's BF16 form uses plain
 *             BF16 throughout (AUTO picks it for FP32 only).  The bound is
 *             always re-evaluated with FP32 operands and an FP64 sum
 *             (ld_final_bound).
 * init        used on the first call of a state: LD_INIT_CROWN (default of
 *             the paper, Sec. 7.2), LD_INIT_WK, LD_INIT_ZERO, or LD_INIT_GIVEN
 *             (duals set by ld_state_set_rho).  On that call q(rho^0) is stored.
 * tie_tau     relative tie band of the inner minimisation (2^-20 suggested).
 * engine      LD_ENGINE_RESIDENT: one launch runs all `iters` steps, each
 *             workgroup owning S subdomains with their intermediates in LDS
 *             (LD_E_UNSUPPORTED if the layer maps do not fit);
 *             LD_ENGINE_LAYERWISE: one batched launch per contraction and
 *             iteration, all `iters` iterations of the call captured in one
 *             HIP graph (up to 1000 per graph; a longer call replays a graph
 *             of 1000 and ends with one of the rest) and launched once;
 *             LD_ENGINE_AUTO: the engine and the launch configuration of every
 *             contraction picked by the autotuner (ld_autotune) for this
 *             net, batch size and precision; the first AUTO call for a new
 *             (B, precision) runs the tuner (synchronous, a few hundred
 *             launches on a scratch state).
 *             Both engines compute the same iteration. */
typedef struct ld_opts {
  int iters;
  int total_iters;
  float lr0, lr_end;
  float beta1, beta2, eps;
  int precision;
  int init;
  float tie_tau;
  int engine;
} ld_opts;

/* Enqueue `iters` Adam supergradient steps for every subdomain (engine per
 * ld_opts).  The layer-wise engine captures its loop once per (state, batch
 * pointers, options, iteration count, tuned configuration) into a HIP graph and
 * replays it on later calls with the same key. */
int ld_step(const ld_net* net, const ld_batch* batch, ld_state* st, const ld_opts* opts,
            hipStream_t stream);

/* Autotuner (the batched launches of Sec. 5.2 sized for this device).  On a
 * scratch state of `batch` (CROWN duals, one iteration done), time every
 * candidate configuration of every contraction of the ascent iteration with
 * its real epilogue: 16-column tiles per wave (1, 2, 4 as the width allows),
 * for transposed strided convs the dense GEMM + col2im form against the
 * stride-class gather form, for convs 1, 2 or 4 blocks per subdomain (bands of
 * destination rows; channel chunks in the col2im form), for fully-connected products the shape of a block
 * (waves along subdomains and along K) and splits of K over blocks.  The
 * fastest configuration of each contraction is kept for (net, batch->B,
 * opts->precision); then `opts` is used to time a 20-step ascent with each
 * engine and the faster one becomes the choice of LD_ENGINE_AUTO.  Replaces
 * earlier choices for the same (B, precision).
 * Synchronises `stream`; allocates and frees its scratch state.  Only the
 * precision, tie_tau, Adam constants and total_iters of `opts` are used. */
int ld_autotune(const ld_net* net, const ld_batch* batch, const ld_opts* opts, hipStream_t stream);

/* Launch configuration of one contraction (what the autotuner chooses). */
typedef struct ld_tile {
  int tn;      /* 16-column MFMA tiles per wave */
  int mwaves;  /* fully-connected: waves of a block along subdomains (16 each); convs: 1 */
  int kwaves;  /* fully-connected: waves of a block along K (partial sums added in LDS); convs: 1 */
  int splits;  /* fully-connected: blocks along K (partials added by a second kernel); convs:
                  blocks per subdomain (stride-class gather form: bands of destination rows;
                  dense GEMM + col2im form: chunks of input channels) */
  int form;    /* transposed strided convs: 0 dense GEMM + col2im, 1 stride-class gather; else 0 */
} ld_tile;

/* The tuned configuration of the contraction of hidden layer k (1..n-1) in
 * direction dir (0: forward W_k x, 1: transposed W_k^T rho_k) for (B,
 * precision) and its measured time in microseconds (host outputs).
 * LD_E_STATE if nothing was tuned for (B, precision). */
int ld_tuned_config(const ld_net* net, int B, int precision, int k, int dir, ld_tile* tile, double* us);

/* The candidate configurations the autotuner times for the contraction of
 * hidden layer k in direction dir at batch size B: up to max_count entries
 * written to `out` (host array); *count receives the number of candidates. */
int ld_tile_candidates(const ld_net* net, int B, int k, int dir, ld_tile* out, int max_count, int* count);

/* Pin the configuration of one contraction for (B, precision), e.g. to restore
 * a stored tuning; it must be one of ld_tile_candidates (else LD_E_ARG).
 * Not thread-safe against concurrent calls on the same net. */
int ld_set_tuned_config(ld_net* net, int B, int precision, int k, int dir, const ld_tile* tile);

/* The engine chosen by the autotuner for (B, precision), *concurrent = 1 (the
 * independent layer jobs of a phase are separate branches of the layer-wise
 * engine's captured graph, which the runtime may run concurrently), and the
 * measured time per iteration of each engine in microseconds (us_resident = 0
 * when the resident engine does not fit).  LD_E_STATE if nothing was tuned. */
int ld_tuned_engine(const ld_net* net, int B, int precision, int* engine, int* concurrent, double* us_layerwise,
                    double* us_resident);

/* Diagnostic: after one ascent iteration on `st`, time every contraction
 * launch of the iteration (with its fused epilogue and the tuned
 * configuration): one warm-up launch, then `reps` back-to-back launches between
 * a HIP event pair on `stream`.  avg_us (host [max_slots]) receives the average
 * duration in microseconds and kinds (host [max_slots]) the slot: 100+k =
 * transposed product of layer k fused with the inner minimisation of layer k-1
 * (phase A), 300+k = forward product of layer k fused with the supergradient
 * and Adam step (phase B).  The repeated phase-B launches advance the Adam
 * state of `st` (a profile is not an ascent).  *n_slots receives the number of
 * slots.  Synchronises `stream`. */
int ld_profile_iteration(const ld_net* net, const ld_batch* batch, ld_state* st, const ld_opts* opts,
                         int reps, double* avg_us, int* kinds, int max_slots, int* n_slots,
                         hipStream_t stream);

/* ------------------------------------------------------------------------- */
/* sigmoid activations: the P_k inner minimisation over the hull (App. E)    */
/* ------------------------------------------------------------------------- */
/* Tangent points of the convex hull of sigma(x) = 1/(1 + e^-x) on [l, u], per
 * element (App. E.1): t_up, where the upper envelope leaves the line from
 * (l, sigma(l)) for sigma itself (t_up = u: the chord, Case 1; t_up = l when
 * l >= 0), and t_lo, where the lower envelope leaves sigma for the line to
 * (u, sigma(u)) (t_lo = l: the chord; t_lo = u when u <= 0).  Bisection on the
 * tangency condition in FP64.  They depend on the bounds only: compute them once
 * per problem.  All arrays are device arrays of `count` elements, l <= u. */
int ld_sigmoid_hull(long long count, const float* l, const float* u, float* t_up, float* t_lo,
                    hipStream_t stream);
/* Per element, the minimum of rho*xB - g*x over the hull (eq:siglinopt): xB* (xb),
 * x* on the envelope g selects (upper for g > 0, lower for g < 0; sigma(xB*) for
 * g = 0) and the value (FP64, val), from the ends, the tangent point and the logit
 * roots of eq:with_sig_subp; ties go to the larger xB.  Inputs as in P_k: rho the
 * layer's dual, g = (W_{k+1}^T rho_{k+1}), the bounds and the tangent points of
 * ld_sigmoid_hull.  FP64 arithmetic. */
int ld_sigmoid_inner_min(long long count, const float* rho, const float* g, const float* l, const float* u,
                         const float* t_up, const float* t_lo, float* xb, float* x, double* val,
                         hipStream_t stream);

/* ------------------------------------------------------------------------- */
/* branching: Filtered Smart Branching (Sec. 4.2)                             */
/* ------------------------------------------------------------------------- */
/* For every subdomain of `batch`, the ReLU split FSB picks:
 *  - the scores s_FSB (eq:fsb-scores) and t_SR (eq:babsr-scores) of every
 *    ambiguous ReLU, from the backward pass lambda_{n-1} = -W_n^T c,
 *    lambda_{k-1} = W_k^T (a_k lambda_k) with the chord slope a_k (FP32
 *    contractions, FP64 scores);
 *  - per hidden layer the ReLU with the largest s_FSB and the one with the
 *    largest t_SR (eq:fsb-prefilter; the first index on ties);
 *  - for each candidate, its two children (l := 0 active, u := 0 inactive),
 *    each bounded by the better of CROWN and WK (q at their dual assignments,
 *    Prop. 2, FP32 operands, FP64 sum);
 *  - the candidate whose worse child has the best bound (the first in layer,
 *    then s_FSB-before-t_SR order on ties).
 * layer[b] (1..n-1, 0 if no ReLU is ambiguous), index[b] (neuron in (C,H,W)
 * order, -1 if none), value[b] (that worse child's bound, -inf if none): device
 * arrays [B].  candidates: NULL or device int [B, n-1, 2] receiving the
 * prefilter's indices (-1: no ambiguous ReLU in that layer).  Bounds l <= u
 * and the objective c are read from `batch`.  Synchronous; the buffers of the
 * 4 (n-1) B children stay with the net for later calls (grown when B grows,
 * freed by ld_destroy_net), and calls on one net are serialised.  At most 16
 * hidden layers (LD_E_UNSUPPORTED). */
int ld_fsb_branch(const ld_net* net, const ld_batch* batch, int* layer, int* index, double* value,
                  int* candidates, hipStream_t stream);

/* The children of every subdomain for its split (layer[b], index[b]), as
 * ld_fsb_branch returns it: child 2b has the ReLU fixed active (l := 0), child
 * 2b+1 inactive (u := 0); a subdomain whose (layer, index) is out of range
 * (index < 0, layer outside 1..n-1, index >= n_layer) is copied into both.  The
 * outputs are caller-owned device arrays for 2B subdomains: l0_out, u0_out
 * [2B, n_0], l_out[k], u_out[k] [2B, n_k] (host arrays of n-1 device pointers),
 * c_out [2B, n_out].  rho / rho_out (both or neither): the parents' duals [B, n_k]
 * copied to both children, the warm start of Sec. 7.3 (pass rho_out to
 * ld_state_set_rho and step with LD_INIT_GIVEN, or to ld_dual_eval; at the
 * parent's duals a child's q is never below its parent's).  Asynchronous on
 * `stream`.  layer and index are device int arrays [B]. */
int ld_branch_children(const ld_net* net, const ld_batch* batch, const int* layer, const int* index,
                       const float* const* rho, float* l0_out, float* u0_out, float* const* l_out,
                       float* const* u_out, float* c_out, float* const* rho_out, hipStream_t stream);

/* ------------------------------------------------------------------------- */
/* branch and bound (Sec. 2.3.1; batches of Sec. 5.2; warm starts of Sec. 7.3) */
/* ------------------------------------------------------------------------- */
/* Complete verification of one property: is min c^T f(x) over the input box
 * (and within the root's intermediate bounds) above `threshold`?
 *  - The root is bounded by ld_step from CROWN's duals (root_iters steps,
 *    root_lr0 -> root_lr_end) and ld_final_bound.
 *  - Each round takes the `batch` open subproblems with the lowest lower bounds
 *    (ties in creation order).  It splits each on the ReLU ld_fsb_branch picks
 *    (ld_branch_children), then bounds the 2*batch children by ld_step from
 *    their parent's final duals (iters steps, lr0 -> lr_end) and ld_final_bound.
 *    A child's bound is the larger of that and its parent's.
 *  - Upper bounds: the network at each bounding's last P_0 minimiser, when every
 *    pre-activation is within its bounds (Sec. 5.1.3); the smallest is the
 *    incumbent.
 *  - A subproblem is discarded when its bound is above `threshold`, or at least
 *    incumbent - gap.  One with no ambiguous ReLU left is a leaf and stays open,
 *    unsplit.
 * threshold = -INFINITY minimises instead: the result brackets the minimum
 * between `lower` and `incumbent`.  The open subproblems (their bounds and warm-start duals,
 * (2 N_h + N_h) floats each) live in a device store of max_subproblems entries
 * that the call allocates and frees; it stops with LD_BAB_LIMIT when the store is
 * full, after max_rounds rounds, or with leaves left open.  Synchronous. */
enum { LD_BAB_VERIFIED = 0, LD_BAB_FALSIFIED = 1, LD_BAB_SOLVED = 2, LD_BAB_LIMIT = 3 };
typedef struct ld_bab_opts {
  int batch;                 /* subproblems split per round (>= 1) */
  int root_iters, iters;     /* Adam steps at the root and for each child (>= 0) */
  float root_lr0, root_lr_end, lr0, lr_end;
  float beta1, beta2, eps;   /* Adam constants (as ld_opts) */
  float threshold;           /* the property is min > threshold; -INFINITY: minimise */
  float gap;                 /* >= 0: also discard when bound >= incumbent - gap */
  int max_rounds;            /* >= 0 */
  int max_subproblems;       /* capacity of the store of open subproblems (>= 1) */
  int precision;             /* LD_FP32 or LD_BF16 contractions in the ascents */
  float tie_tau;             /* as ld_opts */
} ld_bab_opts;
typedef struct ld_bab_result {
  int status;                /* LD_BAB_* */
  double lower;              /* lower bound on the minimum over every subproblem left */
  double incumbent;          /* smallest network value at a feasible point (+inf if none) */
  int rounds;
  int leaves;                /* subproblems with no ambiguous ReLU left open */
  long long bounded;         /* subproblems bounded, the root included */
  long long max_open;        /* the store's peak occupancy */
} ld_bab_result;
/* root: a batch of one subdomain (B = 1).  result: host.  x_best: NULL or host
 * float[n_0], receives the input of the incumbent (unchanged when none). */
int ld_bab(const ld_net* net, const ld_batch* root, const ld_bab_opts* opts, ld_bab_result* result, float* x_best,
           hipStream_t stream);

/* ------------------------------------------------------------------------- */
/* intermediate bounds (Sec. 2.2.3), batched over neurons (Sec. 5.2)          */
/* ------------------------------------------------------------------------- */
/* LD bounds on the pre-activations of a layer j: `sub` is the network of the
 * first j layers (ld_create_net on them; its last layer, layer j, may be a conv).
 * For every subdomain b of `batch` and neuron i of layer j, the LD step of
 * `opts` (ld_step: init CROWN or ZERO, iters, schedule, precision, engine) runs
 * on the objectives +x_j[i] and -x_j[i]; lo[b, i] receives the lower bound and
 * hi[b, i] the upper bound (the best of q(rho^0) and q(rho^T), Sec. 3.1),
 * rounded outward to FP32.  batch->l0/u0 and l[k]/u[k] (the bounds of the
 * sub-network's hidden layers 1..j-1) are read; batch->c is not.  The
 * 2 B n_j problems run in chunks of at most max_problems (<= 0: 8192) on a
 * state the call creates; lo and hi are device arrays [B, n_j].  Synchronous
 * (the call allocates its chunk buffers and waits for them).  Errors as ld_step;
 * LD_E_ARG for init = LD_INIT_GIVEN. */
int ld_intermediate_bounds(const ld_net* sub, const ld_batch* batch, const ld_opts* opts, int max_problems,
                           float* lo, float* hi, hipStream_t stream);

/* ------------------------------------------------------------------------- */
/* proximal solver (Sec. 3.3, Algorithm 2; momentum of App. F)                */
/* ------------------------------------------------------------------------- */
/* The method of multipliers on the same dual q: each outer iteration runs
 * inner_iters sweeps of block-coordinate Frank-Wolfe on the augmented
 * Lagrangian of eq:z_updates (blocks (xB_k, xA_{k+1}), k = 0..n-1 in order;
 * conditional gradient = the inner minimisation of Sec. 3.2 with the duals
 * replaced by the gradient coefficients; step = the closed form of
 * eq:optimal-gamma-gauss, clipped to [0, 1]), then the dual update
 * pi = mu pi + (xB - xA)/eta, rho += pi (eq:momentum_updates; mu = 0 gives
 * eq:lambda_updates).
 * iters        outer iterations run by this call (>= 0)
 * total_iters  T of the schedule of eta: iteration t (1-based, counted over
 *              all calls on this state) uses eta0 + (eta_end - eta0)(t-1)/(T-1)
 * inner_iters  J, Frank-Wolfe sweeps per outer iteration (>= 1; the paper: 2)
 * eta0, eta_end  weight of the proximal terms (> 0; the paper: 10 -> 500, or
 *              100 fixed inside branch and bound)
 * mu           momentum in [0, 1) (the paper: 0.3, or 0 inside branch and bound)
 * precision    LD_FP32 or LD_BF16 operands of the contractions (as ld_opts;
 *              LD_FP64: LD_E_UNSUPPORTED)
 * init, tie_tau  as ld_opts */
typedef struct ld_prox_opts {
  int iters;
  int total_iters;
  int inner_iters;
  float eta0, eta_end;
  float mu;
  int precision;
  int init;
  float tie_tau;
} ld_prox_opts;

/* Enqueue `iters` outer iterations of the proximal solver on the state's duals.
 * The state is shared with ld_step: its duals (rho), q(rho^0) and
 * ld_final_bound have the same meaning.  On the first call of a state (or
 * after ld_state_set_rho / ld_state_reset, or a change of precision) the duals
 * are initialised as by ld_step and the primal iterates start at a minimiser
 * of the Lagrangian at those duals (Algorithm 2), with zero momentum.  Several
 * calls of k iterations equal one call of their sum.  The library allocates
 * the solver's buffers (about 7 floats per neuron and subdomain) on the first
 * call.  Errors: LD_E_ARG (bad options), LD_E_STATE, LD_E_NUMERIC, LD_E_NOMEM. */
int ld_prox_step(const ld_net* net, const ld_batch* batch, ld_state* st, const ld_prox_opts* opts,
                 hipStream_t stream);
/* Per-launch timing of the last sweep of an outer iteration of the proximal
 * solver (its block kernels also take the dual update), for profiling: each
 * launch is enqueued reps + 1 times back to back on `stream` and timed with HIP
 * events (the first is a warm-up); slots 100+k: W_k^T rt_k; 300+k: forward
 * product of layer k; 400+k: block kernel of block k.  Needs a state on which ld_prox_step has
 * run with the same precision; the repeated launches move the iterates and the
 * duals (a profile is not a solve), and the next ld_prox_step restarts the
 * primal iterates at the state's duals.
 * Synchronises `stream`. */
int ld_prox_profile_iteration(const ld_net* net, const ld_batch* batch, ld_state* st,
                              const ld_prox_opts* opts, int reps, double* avg_us, int* kinds,
                              int max_slots, int* n_slots, hipStream_t stream);
/* Outer iterations of the proximal solver done on this state (0 before the first). */
int ld_prox_get_step(const ld_state* st, int* t);

/* ------------------------------------------------------------------------- */
/* final bound (Algorithm 1's return value; upper bound of Sec. 5.1.3)        */
/* ------------------------------------------------------------------------- */
/* At the state's current duals: q_final = q(rho^T) with FP32 operands and an
 * FP64 cross-layer sum (all in FP64, with the network forward for the primal
 * value, for a state stepped in LD_FP64); bound = max(q(rho^0), q(rho^T)) (both are valid lower
 * bounds by weak duality, Sec. 3.1); primal = c^T f(x_0*) for the true ReLU
 * network at the P_0 minimiser x_0*, an upper bound on the subdomain minimum
 * when feasible = 1 (every pre-activation within [l_k, u_k]).  All outputs are
 * device arrays of length B; any of them may be NULL. */
int ld_final_bound(const ld_net* net, const ld_batch* batch, const ld_state* st, double* bound,
                   double* q_final, double* primal, int* feasible, float tie_tau,
                   hipStream_t stream);

/* Message of the last error returned on this thread ("" if none). */
const char* ld_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LD_H_ */
