"""FP64 CPU oracle for the Lagrangian-decomposition (LD) bounding step.

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow, obviously-correct
reference that the GPU library is checked against.  Only the test-suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the
product path never does.  It shares no code with the GPU library.

Everything follows De Palma et al., "Improved Branch and Bound for Neural
Network Verification via Lagrangian Decomposition":

* the problem (Sec. 2.1, eq:noncvx_pb) with the objective folded as c^T y, i.e.
  the dummy dual of the output layer is rho_n = -c (App. A / App. B use the same
  convention with rho_n = -1 for a scalar output);
* the LD dual q(rho) (Sec. 3.1, eq:nonprox_problem) and its decomposition over
  the subproblems P_0 and P_k (App. A, eq:dual_decomp_vs_dj);
* the inner minimisations: box solution of P_0 (Sec. 3.2.1, eq:box_bounds_sol),
  vertex enumeration for ambiguous ReLUs (Sec. 3.2.2, eq:min-pk) and the box
  solution for passing / blocking ReLUs (Sec. 3.2.2, "Non-ambiguous ReLUs");
* the supergradient x_B* - x_A* (Algorithm 1, eq:subgradient_update) driven by
  Adam with a linearly decaying step (Sec. 3.2 and Sec. 7.2);
* initialisation from a propagation-based dual assignment (Prop. 2,
  eq:salman-assignment) with CROWN slopes (Sec. 7.2; footnote of Sec. 4.2);
* the upper bound from the network output at the last P_0 minimiser (Sec. 5.1.3);
* the proximal solver (Sec. 3.3, Algorithm 2): the method of multipliers on q, its
  augmented Lagrangian (eq:z_updates) minimised approximately by J sweeps of
  block-coordinate Frank-Wolfe with the closed-form step (eq:optimal-gamma-gauss),
  and momentum on the dual update (App. F, eq:momentum_updates);
* intermediate bounds (Sec. 2.2.3): the same LD step on the sub-network ending at
  layer j with the objectives +x_j[i] and -x_j[i], batched over neurons (Sec. 5.2);
* Filtered Smart Branching (Sec. 4.2): the scores of eq:fsb-scores and
  eq:babsr-scores from one backward pass, the candidates of eq:fsb-prefilter and the
  split whose worse child has the best CROWN-or-WK bound;
* branch and bound (Sec. 2.3.1, Sec. 5.2, Sec. 7.3): rounds over the B subproblems
  with the lowest bounds, FSB splits, children warm-started from their parent's
  duals, discarding on the threshold and the incumbent;
* the P_k inner minimisation for sigmoid activations (App. E): the hull's tangent
  points, its envelopes and the minimum over the pieces (eq:siglinopt,
  eq:with_sig_subp);
* a rounding margin for dual values whose coefficients W_k^T rho_k are formed with
  single-precision products (the paper computes exactly): Higham's dot-product bound
  times the largest feasible |x| of each inner minimisation.

Readings where the paper is silent (all listed in the design doc):
* Adam uses beta1=0.9, beta2=0.999, eps=1e-8 with bias correction, as ascent.
* The step decays linearly from lr0 (step 1) to lr_end (step T).
* ReLU status: passing if l >= 0, else blocking if u <= 0, else ambiguous.
* Ties in the inner minimisation are broken towards the larger x_B, within a
  relative band tau (0 gives the pure argmin); the value is always the exact min.
* Proximal: the weight eta grows linearly from eta0 (iteration 1) to eta_end
  (iteration T), the same form as the step decay; a block whose step has zero
  curvature takes gamma = 1 if the segment descends, else 0; the momentum starts at 0.

Parity pins: every function here is checked in tests/test_oracle_pins.py against
closed forms, brute force and the paper's identities (Prop. 1, Prop. 2, weak
duality, Danskin's supergradient), and the proximal solver in
tests/test_oracle_prox_pins.py (exact line search, conditional gradient by
autograd and vertex enumeration, convergence to the Planet LP optimum), and the
intermediate bounds in tests/test_oracle_interm_pins.py (sampled pre-activations,
per-neuron Planet LP optimum), and branching in tests/test_oracle_fsb_pins.py (bias
sensitivity of an independent WK bound, chord gap, brute-force candidate search; the
s_FSB formula itself is "parity unpinned" beyond its support and sign), and the
sigmoid inner minimisation in tests/test_oracle_sigmoid_pins.py (sampled convex
hull, dense search, weak duality), and the rounding margin in
tests/test_oracle_margin_pins.py (dense conv matrices, a hand-worked net, and the
errors of single-precision coefficients computed by torch, which it must cover).  The final
bound after T Adam steps has no value printed in the paper: "parity unpinned"
beyond those inequalities.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Sequence

import torch
import torch.nn.functional as F

DT = torch.float64
TAU_DEFAULT = 2.0 ** -20


# ----------------------------------------------------------------------------
# network
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class OLayer:
    """One affine layer W_k x + b_k (Sec. 2.1: fully connected or convolutional)."""
    kind: str
    W: torch.Tensor            # float64; linear [out, in]; conv [Co, Ci, kh, kw]
    b: torch.Tensor            # float64 [Co]
    in_shape: tuple
    out_shape: tuple
    stride: int = 1
    pad: int = 0

    def n_out(self):
        return int(torch.tensor(self.out_shape).prod())

    def bias_full(self) -> torch.Tensor:
        """Bias of every output neuron in (C, H, W) order."""
        if self.kind == "linear":
            return self.b
        C, H, W = self.out_shape
        return self.b.repeat_interleave(H * W)

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        """x: [B, n_in] -> W x + b: [B, n_out]."""
        if self.kind == "linear":
            return x @ self.W.T + self.b
        C, H, W = self.in_shape
        y = F.conv2d(x.reshape(-1, C, H, W), self.W, self.b, stride=self.stride, padding=self.pad)
        assert tuple(y.shape[1:]) == tuple(self.out_shape)
        return y.reshape(x.shape[0], -1)

    def transposed(self, r: torch.Tensor) -> torch.Tensor:
        """r: [B, n_out] -> W^T r: [B, n_in] (the adjoint of the linear map, no bias)."""
        if self.kind == "linear":
            return r @ self.W
        C, H, W = self.in_shape
        Co, Ho, Wo = self.out_shape
        kh = self.W.shape[2]
        kw = self.W.shape[3]
        # output_padding makes conv_transpose2d return exactly the input shape
        oph = H - ((Ho - 1) * self.stride - 2 * self.pad + kh)
        opw = W - ((Wo - 1) * self.stride - 2 * self.pad + kw)
        g = F.conv_transpose2d(r.reshape(-1, Co, Ho, Wo), self.W, None, stride=self.stride,
                               padding=self.pad, output_padding=(oph, opw))
        assert tuple(g.shape[1:]) == (C, H, W)
        return g.reshape(r.shape[0], -1)


def net_from_specs(specs) -> List[OLayer]:
    """Build oracle layers from generator LayerSpecs (float32 values taken exactly)."""
    out = []
    for s in specs:
        out.append(OLayer(s.kind, torch.from_numpy(s.W).to(DT), torch.from_numpy(s.b).to(DT),
                          tuple(s.in_shape), tuple(s.out_shape), int(s.stride), int(s.pad)))
    return out


@dataclasses.dataclass
class OBatch:
    """Per-subdomain data: input box C = [l0, u0] (Sec. 3.2.1), intermediate
    bounds [l_k, u_k] for k = 1..n-1 (Sec. 2.2.3) and objective vector c."""
    l0: torch.Tensor
    u0: torch.Tensor
    l: List[torch.Tensor]
    u: List[torch.Tensor]
    c: torch.Tensor


def batch_from_instance(inst, idx: Optional[Sequence[int]] = None) -> OBatch:
    def t(a):
        x = torch.from_numpy(a).to(DT)
        return x if idx is None else x[torch.as_tensor(list(idx))]
    return OBatch(t(inst.l0), t(inst.u0), [t(a) for a in inst.l], [t(a) for a in inst.u], t(inst.c))


# ----------------------------------------------------------------------------
# inner minimisation (Sec. 3.2.1, 3.2.2)
# ----------------------------------------------------------------------------
def relu_status(l: torch.Tensor, u: torch.Tensor) -> torch.Tensor:
    """0 = passing (l >= 0), 1 = blocking (u <= 0), 2 = ambiguous (Sec. 2.3.2)."""
    st = torch.full_like(l, 2, dtype=torch.int8)
    st[u <= 0] = 1
    st[l >= 0] = 0
    return st


def inner_min_p0(g0: torch.Tensor, l0: torch.Tensor, u0: torch.Tensor):
    """min over x0 in [l0, u0] of -g0^T x0, with g0 = W_1^T rho_1 (eq:box_bounds_sol).

    The minimiser takes u0 where g0 >= 0 and l0 where g0 < 0.
    Returns (x0*, value per subdomain)."""
    x0 = torch.where(g0 >= 0, u0, l0)
    return x0, -(g0 * x0).sum(dim=1)


def inner_min_pk(rho: torch.Tensor, g: torch.Tensor, l: torch.Tensor, u: torch.Tensor,
                 tau: float = TAU_DEFAULT):
    """Per-neuron minimum of  rho*xB - g*x  over the ReLU hull (eq:min-pk, eq:planet-relu-hull),
    with g = (W_{k+1}^T rho_{k+1}).

    ambiguous: vertices (l,0), (0,0), (u,u)  -> values rho*l, 0, (rho-g)*u
    passing:   x = xB in [l, u]              -> box minimum of (rho-g)*xB
    blocking:  x = 0, xB in [l, u]           -> box minimum of rho*xB
    Returns (xB*, x*, value) elementwise.  Tie rule: the larger xB wins within a
    band tau * (sum of the magnitudes of the terms compared); the value is the exact
    minimum.
    """
    st = relu_status(l, u)
    zero = torch.zeros_like(rho)
    # ambiguous
    Vl = rho * l
    Vu = (rho - g) * u
    m = torch.minimum(torch.minimum(Vl, Vu), zero)
    # the band scales with the terms entering the values (rho*l, rho*u, g*u), so that
    # the rounding of rho*u - g*u cannot hide a tie
    band = tau * (Vl.abs() + (rho * u).abs() + (g * u).abs())
    xb_amb = torch.where(Vu <= m + band, u, torch.where(zero <= m + band, zero, l))
    # passing: coefficient (rho - g) on xB
    cp = rho - g
    xb_pass = torch.where(cp <= tau * (rho.abs() + g.abs()), u, l)
    val_pass = torch.minimum(cp * l, cp * u)
    # blocking: coefficient rho on xB
    xb_blk = torch.where(rho <= 0, u, l)
    val_blk = torch.minimum(rho * l, rho * u)
    xb = torch.where(st == 0, xb_pass, torch.where(st == 1, xb_blk, xb_amb))
    val = torch.where(st == 0, val_pass, torch.where(st == 1, val_blk, m))
    x = torch.where(st == 1, zero, torch.clamp(xb, min=0.0))
    return xb, x, val


# ----------------------------------------------------------------------------
# dual function q(rho) and its supergradient (eq:nonprox_problem, Algorithm 1)
# ----------------------------------------------------------------------------
def dual_eval(net: List[OLayer], batch: OBatch, rho: List[torch.Tensor], tau: float = TAU_DEFAULT,
              need_supergrad: bool = True) -> Dict:
    """q(rho) per subdomain, the inner minimisers and the supergradient.

    rho[k-1] is the dual of hidden layer k (k = 1..n-1); rho_n = -c.
    Decomposition (App. A): q = min_{P0}(-rho_1^T xA_1) + sum_k min_{P_k}(rho_k^T xB_k - rho_{k+1}^T xA_{k+1}),
    with xA_{k+1} = W_{k+1} x_k + b_{k+1}; the bias terms give  -sum_{k=1}^{n} rho_k^T b_k.
    """
    n = len(net)
    assert len(rho) == n - 1
    duals = list(rho) + [-batch.c]                 # rho_1..rho_n
    g = [net[k].transposed(duals[k]) for k in range(n)]   # g[k] = W_{k+1}^T rho_{k+1}, k = 0..n-1
    x0, v0 = inner_min_p0(g[0], batch.l0, batch.u0)
    q = v0.clone()
    xB, xs, vals = [], [], []
    for k in range(1, n):
        xb, x, val = inner_min_pk(duals[k - 1], g[k], batch.l[k - 1], batch.u[k - 1], tau)
        xB.append(xb)
        xs.append(x)
        vals.append(val)
        q = q + val.sum(dim=1)
    for k in range(1, n + 1):
        q = q - (duals[k - 1] * net[k - 1].bias_full()).sum(dim=1)
    out = dict(q=q, x0=x0, xB=xB, x=xs, vals=vals, v0=v0, g=g)
    if need_supergrad:
        prev = [x0] + xs
        xA = [net[k - 1].forward(prev[k - 1]) for k in range(1, n)]   # xA_k, k = 1..n-1
        out["xA"] = xA
        out["s"] = [xB[k] - xA[k] for k in range(n - 1)]
        out["xA_n"] = (batch.c * net[n - 1].forward(prev[n - 1])).sum(dim=1)
    return out


def q_scale(net: List[OLayer], batch: OBatch, rho: List[torch.Tensor], ev: Dict) -> torch.Tensor:
    """Magnitude scale of the terms summed into q (used to state relative tolerances)."""
    n = len(net)
    duals = list(rho) + [-batch.c]
    S = ev["v0"].abs()
    for v in ev["vals"]:
        S = S + v.abs().sum(dim=1)
    for k in range(1, n + 1):
        S = S + (duals[k - 1] * net[k - 1].bias_full()).abs().sum(dim=1)
    return S


# ----------------------------------------------------------------------------
# rounding margin of a dual value whose coefficients are formed with FP32
# products (a reading: the paper's q is exact arithmetic)
# ----------------------------------------------------------------------------
U32 = 2.0 ** -24


def abs_layer(L: OLayer) -> OLayer:
    """The layer with every weight replaced by its magnitude (same shapes)."""
    return OLayer(L.kind, L.W.abs(), L.b, L.in_shape, L.out_shape, L.stride, L.pad)


def dot_terms(L: OLayer) -> int:
    """Most terms of one coefficient's dot product (W^T r)_j: every output (fully
    connected); for a conv, per output channel the taps that can reach one input
    position, ceil(kh / stride) x ceil(kw / stride)."""
    if L.kind == "linear":
        return int(L.W.shape[0])
    s = L.stride
    return int(L.W.shape[0] * (-(-L.W.shape[2] // s)) * (-(-L.W.shape[3] // s)))


def rounding_margin(net: List[OLayer], batch: OBatch, rho: List[torch.Tensor]) -> torch.Tensor:
    """How far q computed from single-precision coefficients g_{k-1} = W_k^T rho_k
    (k = 1..n, rho_n = -c) can sit above the exact q(rho), per subdomain.

    A K-term dot product rounded in single precision errs by at most
    gamma_K |W|^T |r|, gamma_K = K u / (1 - K u), u = 2^-24 (Higham's bound);
    g_{k-1} enters one inner minimisation multiplied by x_{k-1}, and replacing the
    coefficient moves that minimum by at most sum_j |error_j| max|x_{k-1,j}| over
    the feasible set: max(|l0|, |u0|) on the input box (eq:box_bounds_sol), max(0, u)
    after a ReLU (eq:min-pk).  Subnormals flushed to zero add at most 2 K 2^-126 per
    coefficient."""
    n = len(net)
    duals = list(rho) + [-batch.c]
    m = torch.zeros(batch.c.shape[0], dtype=DT)
    for k in range(1, n + 1):
        L = net[k - 1]
        K = dot_terms(L)
        gamma = K * U32 / (1.0 - K * U32)
        t = abs_layer(L).transposed(duals[k - 1].abs())
        if k == 1:
            xm = torch.maximum(batch.l0.abs(), batch.u0.abs())
        else:
            xm = batch.u[k - 2].clamp(min=0.0)
        m = m + ((gamma * t + 2.0 * K * 2.0 ** -126) * xm).sum(dim=1)
    return m


# ----------------------------------------------------------------------------
# initialisation (Prop. 2): dual assignment of a propagation method
# ----------------------------------------------------------------------------
def crown_slopes(l: torch.Tensor, u: torch.Tensor):
    """CROWN relaxation slopes (upper: chord u/(u-l); lower: 1 if u >= -l else 0 for
    ambiguous ReLUs; 1/1 passing; 0/0 blocking)."""
    st = relu_status(l, u)
    den = torch.where(st == 2, u - l, torch.ones_like(u))
    a_up = torch.where(st == 2, u / den, torch.where(st == 0, torch.ones_like(u), torch.zeros_like(u)))
    a_lo = torch.where(st == 2, (u >= -l).to(l.dtype), torch.where(st == 0, torch.ones_like(u), torch.zeros_like(u)))
    return a_up, a_lo


def propagation_duals(net: List[OLayer], batch: OBatch, slopes) -> List[torch.Tensor]:
    """One backward pass (eq:salman-assignment) with the objective folded in:
    lambda_{n-1} = W_n^T (-rho_n) ... written here directly on the LD duals:
    rho_k = a_up [g_k]_+ + a_lo [g_k]_-,  g_k = W_{k+1}^T rho_{k+1},  rho_n = -c."""
    n = len(net)
    rho = [None] * (n - 1)
    cur = -batch.c
    for k in range(n - 1, 0, -1):               # hidden layer k
        gk = net[k].transposed(cur)             # W_{k+1}^T rho_{k+1}
        a_up, a_lo = slopes[k - 1]
        rho[k - 1] = a_up * torch.clamp(gk, min=0) + a_lo * torch.clamp(gk, max=0)
        cur = rho[k - 1]
    return rho


def crown_init(net: List[OLayer], batch: OBatch) -> List[torch.Tensor]:
    slopes = [crown_slopes(l, u) for l, u in zip(batch.l, batch.u)]
    return propagation_duals(net, batch, slopes)


def zero_init(net, batch) -> List[torch.Tensor]:
    return [torch.zeros_like(l) for l in batch.l]


# ----------------------------------------------------------------------------
# Adam supergradient ascent (Algorithm 1 with Adam, Sec. 3.2 / Sec. 7.2)
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class AdamOpts:
    T: int = 500
    lr0: float = 1e-2
    lr_end: float = 1e-4
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    tau: float = TAU_DEFAULT
    init: str = "crown"          # "crown" | "zero" | "given"


def step_size(t: int, T: int, lr0: float, lr_end: float) -> float:
    """Linear decay: step t (1-based) of T goes from lr0 (t=1) to lr_end (t=T)."""
    if T <= 1:
        return lr0
    return lr0 + (lr_end - lr0) * (t - 1) / (T - 1)


def ascent(net: List[OLayer], batch: OBatch, opts: AdamOpts, rho0: Optional[List[torch.Tensor]] = None,
           state: Optional[Dict] = None, iters: Optional[int] = None, record: bool = False) -> Dict:
    """Run `iters` Adam steps (default opts.T) of supergradient ascent on q.

    `state` (rho, m, v, t, q0) lets a run continue where a previous call stopped;
    the step schedule is always taken over opts.T total steps."""
    if state is None:
        if opts.init == "given":
            assert rho0 is not None
            rho = [r.clone() for r in rho0]
        elif opts.init == "crown":
            rho = crown_init(net, batch)
        else:
            rho = zero_init(net, batch)
        q0 = dual_eval(net, batch, rho, opts.tau, need_supergrad=False)["q"]
        state = dict(rho=rho, m=[torch.zeros_like(r) for r in rho], v=[torch.zeros_like(r) for r in rho],
                     t=0, q0=q0)
    else:
        state = dict(rho=[r.clone() for r in state["rho"]], m=[r.clone() for r in state["m"]],
                     v=[r.clone() for r in state["v"]], t=state["t"], q0=state["q0"])
    iters = opts.T if iters is None else iters
    traj = []
    for _ in range(iters):
        ev = dual_eval(net, batch, state["rho"], opts.tau)
        if record:
            traj.append(ev["q"].clone())
        t = state["t"] + 1
        a = step_size(t, opts.T, opts.lr0, opts.lr_end)
        bc1 = 1.0 - opts.beta1 ** t
        bc2 = 1.0 - opts.beta2 ** t
        for k in range(len(state["rho"])):
            s = ev["s"][k]
            state["m"][k] = opts.beta1 * state["m"][k] + (1.0 - opts.beta1) * s
            state["v"][k] = opts.beta2 * state["v"][k] + (1.0 - opts.beta2) * s * s
            mh = state["m"][k] / bc1
            vh = state["v"][k] / bc2
            state["rho"][k] = state["rho"][k] + a * mh / (torch.sqrt(vh) + opts.eps)
        state["t"] = t
    state["traj"] = traj
    return state


def final_bound(net: List[OLayer], batch: OBatch, state: Dict, tau: float = TAU_DEFAULT) -> Dict:
    """Bound returned by the method: q at the final duals (Algorithm 1 returns q(rho^T)),
    the best of q(rho^0) and q(rho^T) (both valid by weak duality), and the network
    value at the final P_0 minimiser (Sec. 5.1.3) with its feasibility flag."""
    ev = dual_eval(net, batch, state["rho"], tau, need_supergrad=False)
    p, feas = primal_value(net, batch, ev["x0"])
    return dict(q_final=ev["q"], bound=torch.maximum(ev["q"], state["q0"]), primal=p, feasible=feas,
                x0=ev["x0"])


def primal_value(net: List[OLayer], batch: OBatch, x0: torch.Tensor):
    """c^T f(x0) for the true ReLU network, and whether every pre-activation lies
    within the subdomain's intermediate bounds (then it upper-bounds the subdomain)."""
    x = x0
    feas = torch.ones(x0.shape[0], dtype=torch.bool)
    for k in range(len(net) - 1):
        xh = net[k].forward(x)
        feas &= ((xh >= batch.l[k]) & (xh <= batch.u[k])).all(dim=1)
        x = torch.clamp(xh, min=0.0)
    y = net[-1].forward(x)
    return (batch.c * y).sum(dim=1), feas


def network_output(net: List[OLayer], x0: torch.Tensor) -> torch.Tensor:
    x = x0
    for k in range(len(net) - 1):
        x = torch.clamp(net[k].forward(x), min=0.0)
    return net[-1].forward(x)


# ----------------------------------------------------------------------------
# proximal solver (Sec. 3.3, Algorithm 2 "Proximal method"; App. F momentum)
# ----------------------------------------------------------------------------
# Primal iterates of the method of multipliers, per subdomain:
#   xB[k-1] = xB_k  (k = 1..n-1), the relaxed pre-activation copy inside P_k;
#   xA[k-1] = xA_k  (k = 1..n),   the image W_k x_{k-1} + b_k leaving P_{k-1}
#   (xA_n is the network output vector; the objective is c^T xA_n).
# Duals: rho[k-1] = lambda_k as in the supergradient method (rho_n = -c).
@dataclasses.dataclass
class ProxOpts:
    T: int = 100                 # outer iterations (dual updates)
    J: int = 2                   # Frank-Wolfe sweeps per outer iteration (Sec. 7.2)
    eta0: float = 1e1            # proximal weight, linear from eta0 (iteration 1) ...
    eta_end: float = 5e2         # ... to eta_end (iteration T) (Sec. 7.2)
    mu: float = 0.3              # momentum on the dual update (App. F); 0 = eq:lambda_updates
    tau: float = TAU_DEFAULT
    init: str = "crown"          # "crown" | "zero" | "given"


def prox_eta(t: int, T: int, eta0: float, eta_end: float) -> float:
    """Weight of the proximal terms at outer iteration t (1-based), linear in t."""
    return step_size(t, T, eta0, eta_end)


def aug_lagrangian(net: List[OLayer], batch: OBatch, rho: List[torch.Tensor], eta: float,
                   xB: List[torch.Tensor], xA: List[torch.Tensor]) -> torch.Tensor:
    """The augmented Lagrangian of eq:z_updates per subdomain, written out:
    c^T xA_n + sum_k lambda_k^T (xB_k - xA_k) + sum_k ||xB_k - xA_k||^2 / (2 eta).
    (The momentum form of App. F adds a term constant in the primal variables.)"""
    L = (batch.c * xA[-1]).sum(dim=1)
    for k in range(len(rho)):
        d = xB[k] - xA[k]
        L = L + (rho[k] * d).sum(dim=1) + (d * d).sum(dim=1) / (2.0 * eta)
    return L


def prox_coeff(rho: List[torch.Tensor], batch: OBatch, eta: float, xB: List[torch.Tensor],
               xA: List[torch.Tensor], k: int) -> torch.Tensor:
    """Gradient of the augmented Lagrangian with respect to xB_k (k = 1..n-1), which is
    minus its gradient with respect to xA_k: lambda_k + (xB_k - xA_k) / eta.  For
    k = n it is -c (the objective's coefficient, eta_n = infinity)."""
    if k == len(rho) + 1:
        return -batch.c
    return rho[k - 1] + (xB[k - 1] - xA[k - 1]) / eta


def prox_primal_init(net: List[OLayer], batch: OBatch, rho: List[torch.Tensor], tau: float = TAU_DEFAULT):
    """Primal start of Algorithm 2: an inner minimiser of q at the initial duals
    (Sec. 3.2.1 / 3.2.2), xA_k = W_k x*_{k-1} + b_k for k = 1..n."""
    ev = dual_eval(net, batch, rho, tau, need_supergrad=False)
    prev = [ev["x0"]] + ev["x"]
    xA = [net[k].forward(prev[k]) for k in range(len(net))]
    return [x.clone() for x in ev["xB"]], xA


def prox_block(net: List[OLayer], batch: OBatch, rho: List[torch.Tensor], eta: float,
               xB: List[torch.Tensor], xA: List[torch.Tensor], k: int, tau: float = TAU_DEFAULT) -> Dict:
    """One block-coordinate Frank-Wolfe step on the block (xB_k, xA_{k+1}), k = 0..n-1
    (Sec. 3.3.2).  Updates xB[k-1] (k >= 1) and xA[k] in place.

    Conditional gradient: the inner minimisation of P_k with the duals replaced by the
    gradient coefficients (eq. of the conditional gradient; for k = 0 the box rule).
    Step: gamma* of eq:optimal-gamma-gauss, clipped to [0, 1]; with a zero curvature the
    segment is linear and gamma is 1 if it descends, else 0."""
    n = len(net)
    r_next = prox_coeff(rho, batch, eta, xB, xA, k + 1)      # coefficient of layer k+1
    g = net[k].transposed(r_next)                            # W_{k+1}^T r_{k+1}
    if k == 0:
        z, _ = inner_min_p0(g, batch.l0, batch.u0)
        num = torch.zeros(g.shape[0], dtype=g.dtype)
        den = torch.zeros_like(num)
        zB = None
    else:
        r_k = prox_coeff(rho, batch, eta, xB, xA, k)
        zB, z, _ = inner_min_pk(r_k, g, batch.l[k - 1], batch.u[k - 1], tau)
        dB = xB[k - 1] - zB
        num = (r_k * dB).sum(dim=1)
        den = (dB * dB).sum(dim=1) / eta
    zA = net[k].forward(z)                                   # W_{k+1} z_k + b_{k+1}
    dA = xA[k] - zA
    # gradient with respect to xA_{k+1} is -r_{k+1}
    num = num - (r_next * dA).sum(dim=1)
    if k + 1 < n:
        den = den + (dA * dA).sum(dim=1) / eta
    ratio = torch.where(den > 0, num / torch.where(den > 0, den, torch.ones_like(den)), torch.zeros_like(num))
    gamma = torch.where(den > 0, torch.clamp(ratio, 0.0, 1.0), (num > 0).to(num.dtype))
    if k >= 1:
        xB[k - 1] = xB[k - 1] + gamma[:, None] * (zB - xB[k - 1])
    xA[k] = xA[k] + gamma[:, None] * (zA - xA[k])
    return dict(gamma=gamma, z=z, zB=zB, zA=zA, num=num, den=den)


def proximal(net: List[OLayer], batch: OBatch, opts: ProxOpts, rho0: Optional[List[torch.Tensor]] = None,
             state: Optional[Dict] = None, iters: Optional[int] = None, record: bool = False) -> Dict:
    """Algorithm 2: `iters` outer iterations (default opts.T) of the method of
    multipliers, each running J block-coordinate Frank-Wolfe sweeps (blocks k = 0..n-1
    in order) on the augmented Lagrangian and then the dual update with momentum
    (eq:momentum_updates; mu = 0 gives eq:lambda_updates).

    `state` (rho, pi, xB, xA, t, q0) continues a previous call; the eta schedule is
    taken over opts.T."""
    n = len(net)
    if state is None:
        if opts.init == "given":
            assert rho0 is not None
            rho = [r.clone() for r in rho0]
        elif opts.init == "crown":
            rho = crown_init(net, batch)
        else:
            rho = zero_init(net, batch)
        q0 = dual_eval(net, batch, rho, opts.tau, need_supergrad=False)["q"]
        xB, xA = prox_primal_init(net, batch, rho, opts.tau)
        state = dict(rho=rho, pi=[torch.zeros_like(r) for r in rho], xB=xB, xA=xA, t=0, q0=q0)
    else:
        state = {key: ([x.clone() for x in val] if isinstance(val, list) else val) for key, val in state.items()}
    iters = opts.T if iters is None else iters
    traj = []
    for _ in range(iters):
        t = state["t"] + 1
        eta = prox_eta(t, opts.T, opts.eta0, opts.eta_end)
        for _j in range(opts.J):
            for k in range(n):
                prox_block(net, batch, state["rho"], eta, state["xB"], state["xA"], k, opts.tau)
        for k in range(n - 1):
            d = (state["xB"][k] - state["xA"][k]) / eta
            state["pi"][k] = opts.mu * state["pi"][k] + d
            state["rho"][k] = state["rho"][k] + state["pi"][k]
        state["t"] = t
        if record:
            traj.append(dual_eval(net, batch, state["rho"], opts.tau, need_supergrad=False)["q"])
    state["traj"] = traj
    return state


# ----------------------------------------------------------------------------
# intermediate bounds (Sec. 2.2.3): LD on the sub-network that ends at layer j
# ----------------------------------------------------------------------------
def neuron_batch(batch: OBatch, j: int, n_j: int) -> OBatch:
    """The 2 B n_j problems bounding the pre-activations of layer j: problem
    (b, i, s) is subdomain b with the bounds of layers 1..j-1 and the objective
    c = e_i (s = 0, lower bound) or c = -e_i (s = 1, minus the upper bound),
    ordered b-major, then i, then s."""
    B = batch.l0.shape[0]
    P = 2 * n_j
    idx = torch.arange(B).repeat_interleave(P)
    r = torch.arange(P).repeat(B)
    c = torch.zeros(B * P, n_j, dtype=DT)
    c[torch.arange(B * P), r // 2] = 1.0 - 2.0 * (r % 2).to(DT)
    return OBatch(batch.l0[idx], batch.u0[idx], [x[idx] for x in batch.l[:j - 1]],
                  [x[idx] for x in batch.u[:j - 1]], c)


def intermediate_bounds(net: List[OLayer], batch: OBatch, j: int, opts: AdamOpts):
    """Lower and upper bounds [B, n_j] on the pre-activations of hidden layer j
    (j >= 2): the bound of the LD step on the network's first j layers with the
    objectives +x_j[i] and -x_j[i] (the returned bound of each, Sec. 3.1)."""
    sub = net[:j]
    n_j = sub[-1].n_out()
    eb = neuron_batch(batch, j, n_j)
    st = ascent(sub, eb, opts)
    b = final_bound(sub, eb, st)["bound"].reshape(-1, n_j, 2)
    return b[:, :, 0], -b[:, :, 1]


# ----------------------------------------------------------------------------
# Filtered Smart Branching (Sec. 4.2, eq:fsb-scores, eq:fsb-prefilter)
# ----------------------------------------------------------------------------
def wk_slopes(l: torch.Tensor, u: torch.Tensor):
    """Slopes of the WK relaxation: the chord [u]_+ / ([u]_+ - [l]_-) as both the upper
    and the (parallel) lower slope: 1 passing, 0 blocking (Sec. 4.1)."""
    st = relu_status(l, u)
    den = torch.where(st == 2, u - l, torch.ones_like(u))
    a = torch.where(st == 2, u / den, torch.where(st == 0, torch.ones_like(u), torch.zeros_like(u)))
    return a, a


def fsb_lambdas(net: List[OLayer], batch: OBatch) -> List[torch.Tensor]:
    """The backward pass of eq:babsr-scores: lambda_{n-1} = -W_n^T c (the objective
    folded as rho_n = -c) and lambda_{k-1} = W_k^T (a_k lambda_k) with the chord slope
    a_k, i.e. the coefficients g_k of the WK dual assignment; k = 1..n-1."""
    rho = propagation_duals(net, batch, [wk_slopes(l, u) for l, u in zip(batch.l, batch.u)])
    duals = list(rho) + [-batch.c]
    return [net[k].transposed(duals[k]) for k in range(1, len(net))]


def fsb_scores(net: List[OLayer], batch: OBatch):
    """s_FSB,k and t_SR,k for every hidden layer (eq:fsb-scores, eq:babsr-scores);
    non-ambiguous neurons score 0."""
    n = len(net)
    lams = fsb_lambdas(net, batch)
    s_out, t_out = [], []
    for k in range(1, n):
        lam = lams[k - 1]
        l, u = batch.l[k - 1], batch.u[k - 1]
        amb = relu_status(l, u) == 2
        den = torch.where(amb, u - l, torch.ones_like(u))
        bias = net[k - 1].bias_full().expand_as(lam)
        lb = lam * bias
        s = (torch.minimum(torch.zeros_like(lb), lb) - (u / den) * lb + (u * l / den) * torch.clamp(lam, min=0)).abs()
        t = (-u * l / den) * torch.clamp(lam, min=0)
        s_out.append(torch.where(amb, s, torch.zeros_like(s)))
        t_out.append(torch.where(amb, t, torch.zeros_like(t)))
    return s_out, t_out


def fsb_candidates(batch: OBatch, s: List[torch.Tensor], t: List[torch.Tensor]):
    """eq:fsb-prefilter: per subdomain and hidden layer k, the ambiguous neuron with the
    largest s_FSB,k and the one with the largest t_SR,k (the first index on ties);
    -1 where layer k has no ambiguous neuron.  Returns int64 [B, n-1, 2]."""
    B = batch.l0.shape[0]
    out = torch.full((B, len(s), 2), -1, dtype=torch.int64)
    for k in range(len(s)):
        amb = relu_status(batch.l[k], batch.u[k]) == 2
        for col, sc in enumerate((s[k], t[k])):
            masked = torch.where(amb, sc, torch.full_like(sc, -1.0))
            best = masked.max(dim=1)
            # first index attaining the maximum
            first = (masked == best.values[:, None]).to(torch.int64).argmax(dim=1)
            out[:, k, col] = torch.where(amb.any(dim=1), first, torch.full_like(first, -1))
    return out


def split_child(batch: OBatch, b: int, k: int, i: int, active: bool) -> OBatch:
    """Subdomain b with ReLU i of hidden layer k split: active (l := 0, passing) or
    inactive (u := 0, blocking)."""
    l = [x[b:b + 1].clone() for x in batch.l]
    u = [x[b:b + 1].clone() for x in batch.u]
    if active:
        l[k - 1][0, i] = 0.0
    else:
        u[k - 1][0, i] = 0.0
    return OBatch(batch.l0[b:b + 1], batch.u0[b:b + 1], l, u, batch.c[b:b + 1])


def propagation_bound(net: List[OLayer], batch: OBatch) -> torch.Tensor:
    """The better of the CROWN and WK bounds: q at their dual assignments (Prop. 2)."""
    q = []
    for slopes in ([crown_slopes(l, u) for l, u in zip(batch.l, batch.u)],
                   [wk_slopes(l, u) for l, u in zip(batch.l, batch.u)]):
        q.append(dual_eval(net, batch, propagation_duals(net, batch, slopes), need_supergrad=False)["q"])
    return torch.maximum(q[0], q[1])


def fsb_branch(net: List[OLayer], batch: OBatch):
    """FSB's decision per subdomain: among the candidates of eq:fsb-prefilter, the one
    whose worse child has the largest bound (best of CROWN and WK); ties go to the
    first candidate in (layer, s then t) order.  Returns (layer [B], index [B],
    value [B]); layer = 0 and value = -inf when no ReLU is ambiguous."""
    s, t = fsb_scores(net, batch)
    cand = fsb_candidates(batch, s, t)
    B = batch.l0.shape[0]
    layer = torch.zeros(B, dtype=torch.int64)
    index = torch.full((B,), -1, dtype=torch.int64)
    value = torch.full((B,), -float("inf"), dtype=DT)
    for b in range(B):
        for k in range(1, len(net)):
            for col in range(2):
                i = int(cand[b, k - 1, col])
                if i < 0:
                    continue
                v = min(propagation_bound(net, split_child(batch, b, k, i, h)).item() for h in (True, False))
                if v > value[b]:
                    layer[b], index[b], value[b] = k, i, v
    return layer, index, value


def branch_children(batch: OBatch, layer: torch.Tensor, index: torch.Tensor) -> OBatch:
    """The two children of every subdomain for its split (layer, index): child 2b has
    the ReLU fixed active (l := 0), child 2b+1 inactive (u := 0); a subdomain with
    no split (index < 0) is copied into both.  A child warm-starts from its parent's
    duals (Sec. 7.3)."""
    kids = []
    for b in range(batch.l0.shape[0]):
        k, i = int(layer[b]), int(index[b])
        for active in (True, False):
            if i < 0:
                kids.append(OBatch(batch.l0[b:b + 1], batch.u0[b:b + 1], [x[b:b + 1] for x in batch.l],
                                   [x[b:b + 1] for x in batch.u], batch.c[b:b + 1]))
            else:
                kids.append(split_child(batch, b, k, i, active))
    cat = lambda xs: torch.cat(xs, dim=0)  # noqa: E731
    nh = len(batch.l)
    return OBatch(cat([c.l0 for c in kids]), cat([c.u0 for c in kids]),
                  [cat([c.l[k] for c in kids]) for k in range(nh)], [cat([c.u[k] for c in kids]) for k in range(nh)],
                  cat([c.c for c in kids]))


# ----------------------------------------------------------------------------
# branch and bound (Sec. 2.3.1 operating principle; Sec. 5.2 batches of the B
# subproblems with the lowest lower bounds; Sec. 7.3 children warm-started from the
# parent's duals; Sec. 5.1.3 upper bound at the last P_0 minimiser)
# ----------------------------------------------------------------------------
@dataclasses.dataclass
class BabOpts:
    batch: int = 4               # B subproblems branched per round
    root_iters: int = 100        # Adam steps at the root, from CROWN's duals
    root_lr0: float = 1e-2
    root_lr_end: float = 1e-4
    iters: int = 50              # Adam steps of each child, from its parent's duals
    lr0: float = 1e-3            # the children's step schedule (Sec. 7.3: 1e-3 -> 1e-4)
    lr_end: float = 1e-4
    threshold: float = 0.0       # the property: is min c^T f > threshold (-inf: no property, minimise)
    gap: float = 0.0             # also discard subproblems with lb >= incumbent - gap
    max_rounds: int = 200
    beta1: float = 0.9
    beta2: float = 0.999
    eps: float = 1e-8
    tau: float = TAU_DEFAULT


def _sub_batch(batch: OBatch, idx) -> OBatch:
    ix = torch.as_tensor(list(idx), dtype=torch.long)
    return OBatch(batch.l0[ix], batch.u0[ix], [x[ix] for x in batch.l], [x[ix] for x in batch.u], batch.c[ix])


def _cat_batches(bs: List[OBatch]) -> OBatch:
    cat = lambda xs: torch.cat(xs, dim=0)  # noqa: E731
    nh = len(bs[0].l)
    return OBatch(cat([b.l0 for b in bs]), cat([b.u0 for b in bs]), [cat([b.l[k] for b in bs]) for k in range(nh)],
                  [cat([b.u[k] for b in bs]) for k in range(nh)], cat([b.c for b in bs]))


def bab(net: List[OLayer], root: OBatch, opts: BabOpts) -> Dict:
    """Branch and bound on one property (root: one subdomain).

    Bounding: the Adam supergradient ascent (CROWN duals at the root, the parent's
    final duals for a child), the returned bound max(q(rho^0), q(rho^T)), and for a
    child the larger of that and its parent's bound (a child's minimum is at least
    its parent's).  Upper bounds: the network at the bounding's last P_0 minimiser
    when it is feasible; the incumbent is the smallest.  Each round takes the B open
    subproblems with the lowest bounds (ties in creation order), splits each on the
    ReLU Filtered Smart Branching picks, and bounds the 2B children.  A subproblem
    is discarded when its bound is above the threshold or at least incumbent - gap.
    A subproblem with no ambiguous ReLU is a leaf: it cannot be split further.

    Status: 'falsified' (a feasible point at or below the threshold), 'verified'
    (every subproblem discarded with its bound above the threshold), 'solved' (every
    subproblem discarded, some by the gap: the minimum lies in [lower, incumbent]),
    'limit' (rounds exhausted, or leaves left open)."""
    def ascend(b, T, lr0, lr_end, rho0):
        o = AdamOpts(T=T, lr0=lr0, lr_end=lr_end, beta1=opts.beta1, beta2=opts.beta2, eps=opts.eps, tau=opts.tau,
                     init="crown" if rho0 is None else "given")
        st = ascent(net, b, o, rho0=rho0)
        return st, final_bound(net, b, st, opts.tau)

    st, fb = ascend(root, opts.root_iters, opts.root_lr0, opts.root_lr_end, None)
    res = dict(incumbent=float("inf"), x_best=None, rounds=0, bounded=1, leaves=0)
    pruned_min = float("inf")
    all_above = True

    def offer(fbr, i):
        if bool(fbr["feasible"][i]) and fbr["primal"][i].item() < res["incumbent"]:
            res["incumbent"] = fbr["primal"][i].item()
            res["x_best"] = fbr["x0"][i].clone()

    offer(fb, 0)
    seq = 0
    open_: List = []
    leaves: List = []

    def place(lb, dom, rho):
        nonlocal seq, pruned_min, all_above
        if opts.threshold > -float("inf") and lb > opts.threshold:
            pruned_min = min(pruned_min, lb)
        elif lb >= res["incumbent"] - opts.gap:
            pruned_min = min(pruned_min, lb)
            all_above = False
        else:
            open_.append((lb, seq, dom, rho))
            seq += 1

    place(fb["bound"][0].item(), root, [r.clone() for r in st["rho"]])
    while open_ and res["incumbent"] > opts.threshold and res["rounds"] < opts.max_rounds:
        res["rounds"] += 1
        open_.sort(key=lambda e: (e[0], e[1]))
        take, open_[:] = open_[:opts.batch], open_[opts.batch:]
        parents = _cat_batches([e[2] for e in take])
        layer, index, _ = fsb_branch(net, parents)
        split = [j for j in range(len(take)) if int(index[j]) >= 0]
        for j in range(len(take)):
            if int(index[j]) < 0:
                leaves.append(take[j])
        if not split:
            continue
        pb = _sub_batch(parents, split)
        kids = branch_children(pb, layer[split], index[split])
        rho0 = [torch.cat([torch.stack([take[j][3][k][0]] * 2) for j in split]) for k in range(len(net) - 1)]
        st, fb = ascend(kids, opts.iters, opts.lr0, opts.lr_end, rho0)
        res["bounded"] += kids.l0.shape[0]
        for c in range(kids.l0.shape[0]):
            offer(fb, c)
        for c in range(kids.l0.shape[0]):
            lb = max(fb["bound"][c].item(), take[split[c // 2]][0])
            place(lb, _sub_batch(kids, [c]), [r[c:c + 1].clone() for r in st["rho"]])
    res["leaves"] = len(leaves)
    lower = min([e[0] for e in open_] + [e[0] for e in leaves] + [pruned_min])
    res["lower"] = lower
    if res["incumbent"] <= opts.threshold:
        res["status"] = "falsified"
    elif open_ or leaves:
        res["status"] = "limit"
    else:
        res["status"] = "verified" if all_above else "solved"
    return res


# ----------------------------------------------------------------------------
# sigmoid activations: the P_k inner minimisation over the sigmoid's convex hull
# (App. E)
# ----------------------------------------------------------------------------
def _sig(x):
    return 1.0 / (1.0 + torch.exp(-x))


def _dsig(x):
    s = _sig(x)
    return s * (1.0 - s)


def _logit(p):
    return torch.log(p / (1.0 - p))


def sigmoid_hull(l: torch.Tensor, u: torch.Tensor, iters: int = 200):
    """Tangent points of the sigmoid's convex hull on [l, u] (App. E.1).

    Upper (concave) envelope phi: the chord if sigma'(u) >= the chord's slope (Case 1,
    returned as t_up = u); else the line from (l, sigma(l)) tangent to sigma at
    t_up > max(l, 0), then sigma on [t_up, u] (Case 2; t_up = l when l >= 0).  The
    lower (convex) envelope psi is the mirror image: sigma on [l, t_lo], then the line
    tangent at t_lo to (u, sigma(u)) (t_lo = u when u <= 0; t_lo = l in Case 1).
    The tangent points are found by bisection on the tangency condition."""
    sl, su = _sig(l), _sig(u)
    width = torch.where(u > l, u - l, torch.ones_like(u))
    chord = torch.where(u > l, (su - sl) / width, _dsig(l))
    # upper: F(t) = sigma'(t)(t - l) - (sigma(t) - sigma(l)), F >= 0 at max(l, 0), < 0 at u
    case2_up = _dsig(u) < chord
    a = torch.clamp(l, min=0.0)
    b = u.clone()
    for _ in range(iters):
        m = 0.5 * (a + b)
        F = _dsig(m) * (m - l) - (_sig(m) - sl)
        a = torch.where(F >= 0, m, a)
        b = torch.where(F >= 0, b, m)
    t_up = torch.where(l >= 0, l, torch.where(case2_up, 0.5 * (a + b), u))
    # lower: G(t) = sigma'(t)(u - t) - (sigma(u) - sigma(t)), G >= 0 at min(u, 0), < 0 at l
    case2_lo = _dsig(l) < chord
    a = l.clone()
    b = torch.clamp(u, max=0.0)
    for _ in range(iters):
        m = 0.5 * (a + b)
        G = _dsig(m) * (u - m) - (su - _sig(m))
        b = torch.where(G >= 0, m, b)
        a = torch.where(G >= 0, a, m)
    t_lo = torch.where(u <= 0, u, torch.where(case2_lo, 0.5 * (a + b), l))
    return t_up, t_lo


def sigmoid_upper(x, l, u, t_up):
    """phi(x): the line from (l, sigma(l)) to (t_up, sigma(t_up)) on [l, t_up], sigma
    beyond (Case 1 is t_up = u: the chord)."""
    st = _sig(t_up)
    slope = torch.where(t_up > l, (st - _sig(l)) / torch.where(t_up > l, t_up - l, torch.ones_like(l)), _dsig(l))
    return torch.where(x <= t_up, _sig(l) + slope * (x - l), _sig(x))


def sigmoid_lower(x, l, u, t_lo):
    """psi(x): sigma on [l, t_lo], then the line from (t_lo, sigma(t_lo)) to (u, sigma(u))."""
    st = _sig(t_lo)
    slope = torch.where(u > t_lo, (_sig(u) - st) / torch.where(u > t_lo, u - t_lo, torch.ones_like(u)), _dsig(u))
    return torch.where(x >= t_lo, st + slope * (x - t_lo), _sig(x))


def inner_min_sigmoid(rho, g, l, u, t_up, t_lo):
    """Per-neuron minimum of rho*xB - g*x over the sigmoid's hull on [l, u]
    (eq:siglinopt): x takes the upper envelope where g > 0 and the lower where g < 0
    (g = 0: x = sigma(xB)); the minimum over xB is taken among the interval's ends,
    the tangent point and the stationary points sigma^{-1}((1 +- sqrt(1 - 4 rho/g))/2)
    of the piece where x = sigma(xB) (eq:with_sig_subp).  Ties go to the larger xB.
    Returns (xB*, x*, value)."""
    up = g > 0
    env = lambda x: torch.where(up, sigmoid_upper(x, l, u, t_up), sigmoid_lower(x, l, u, t_lo))  # noqa: E731
    cands = [l, u, torch.where(up, t_up, t_lo)]
    ratio = torch.where(g != 0, rho / torch.where(g != 0, g, torch.ones_like(g)), torch.zeros_like(g))
    disc = 1.0 - 4.0 * ratio
    ok = (g != 0) & (disc >= 0)
    sq = torch.sqrt(torch.clamp(disc, min=0.0))
    for sgn in (1.0, -1.0):
        p = 0.5 * (1.0 + sgn * sq)
        inside = ok & (p > 0) & (p < 1)
        r = _logit(torch.where(inside, p, torch.full_like(p, 0.5)))
        # the stationary point counts only on the piece where x = sigma(xB)
        on_curve = torch.where(up, r >= t_up, r <= t_lo)
        r = torch.where(inside & on_curve & (r >= l) & (r <= u), r, l)
        cands.append(r)
    best_x = None
    best_v = None
    for c in cands:
        v = rho * c - g * env(c)
        if best_v is None:
            best_x, best_v = c, v
        else:
            take = (v < best_v) | ((v == best_v) & (c > best_x))
            best_x = torch.where(take, c, best_x)
            best_v = torch.where(take, v, best_v)
    x = torch.where(g == 0, _sig(best_x), env(best_x))
    return best_x, x, best_v
