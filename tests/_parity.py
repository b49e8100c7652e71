"""Helpers for the GPU-vs-oracle parity tests (tolerances and stability masks).

Tolerances, per the bar "dual value and supergradient at fixed duals match the
oracle to 1e-5 relative in FP32":
  q : |q_gpu - q_orc| <= 1e-5 * S, with S the sum of the magnitudes of every
      term summed into q (reading of "relative" for a sum that can be near 0).
  s : |s_gpu - s_orc| <= 1e-5 * (|W| |x*| + |b| + |xB|) elementwise, on
      subdomains whose inner minimisation has no near-tie (several argmins are
      correct there; q, which is unique, is compared everywhere).
"""
import numpy as np
import torch

from oracle import ld_oracle as O

REL = 1e-5
TIE_REL = 2e-4   # decisions closer than this (relative to the FP32 error scale) can flip
ULP32 = 8 * 2.0 ** -24


def abs_layer(L):
    return O.OLayer(L.kind, L.W.abs(), L.b.abs(), L.in_shape, L.out_shape, L.stride, L.pad)


def unstable_decisions(net, batch, rho, ev, tau=O.TAU_DEFAULT, tie_rel=TIE_REL, exact_ties_stable=False):
    """Per-layer boolean masks (layer 0 = P_0, then hidden layers 1..n-1): True where
    an inner-minimisation decision of the oracle sits within tie_rel (relative to
    the error scale of the contraction feeding it) of flipping.

    exact_ties_stable: the duals were formed by the GPU from the very contraction it
    repeats (the CROWN point, where rho = a g; zeros).  A hidden-layer decision at an
    exact tie of the oracle's vertex values (a kink of q, Prop. 2) is then an exact
    tie up to FP32 rounding (< 2^-21 of the magnitudes) on the GPU too, inside the
    tie band (2^-20), and both sides take the preferred vertex."""
    TIE_REL = tie_rel  # noqa: N806
    n = len(net)
    duals = list(rho) + [-batch.c]
    absnet = [abs_layer(L) for L in net]
    G = [absnet[k].transposed(duals[k].abs()) for k in range(n)]   # magnitude of the terms of g_k
    masks = [(ev["g"][0].abs() <= TIE_REL * G[0]) & (G[0] > 0)]    # P0: sign of g0
    for k in range(1, n):
        r, g, l, u = duals[k - 1], ev["g"][k], batch.l[k - 1], batch.u[k - 1]
        st = O.relu_status(l, u)
        # passing: the test of cp against its band; the error scale of g is G
        cp = r - g
        e_pass = TIE_REL * G[k] + ULP32 * (r.abs() + g.abs())
        # where the error scale is zero both sides compute the identical exact value
        ok_pass = ((cp - tau * (r.abs() + g.abs())).abs() > e_pass) | (e_pass == 0)
        if exact_ties_stable:
            ok_pass = ok_pass | (cp.abs() <= 1e-12 * (r.abs() + g.abs()))
        # blocking: the sign of rho is an input, identical on both sides
        # ambiguous: a vertex at the minimum is always accepted; any other vertex must
        # not sit near the acceptance threshold m + band
        Vl, Vu = r * l, (r - g) * u
        V0 = torch.zeros_like(Vl)
        m = torch.minimum(torch.minimum(Vl, Vu), V0)
        thr = m + tau * (Vl.abs() + (r * u).abs() + (g * u).abs())
        err = 2 * TIE_REL * G[k] * (l.abs() + u.abs()) + ULP32 * (Vl.abs() + Vu.abs())

        mag = Vl.abs() + (r * u).abs() + (g * u).abs()
        at_min = 1e-12 * mag if exact_ties_stable else torch.zeros_like(mag)

        def far(V):
            return ((V - m).abs() <= at_min) | (V == m) | ((V - thr).abs() > err) | (err == 0)
        ok_amb = far(Vl) & far(V0) & far(Vu)
        ok = torch.where(st == 0, ok_pass, torch.where(st == 1, torch.ones_like(ok_pass), ok_amb))
        masks.append(~ok)
    return masks


def supergrad_masks(net, masks):
    """Entries of s_k that a flipped decision can change: the neuron's own decision,
    or any input of W_k whose decision may flip (receptive field through |W_k|)."""
    out = []
    for k in range(1, len(net)):
        spread = abs_layer(net[k - 1]).forward(masks[k - 1].double()) - abs_layer(net[k - 1]).bias_full()
        out.append(masks[k] | (spread > 0))
    return out


def q_tol(net, batch, rho, ev):
    return REL * O.q_scale(net, batch, rho, ev) + 1e-9


def s_scale(net, ev):
    n = len(net)
    prev = [ev["x0"]] + ev["x"]
    out = []
    for k in range(1, n):
        L = abs_layer(net[k - 1])
        out.append(L.forward(prev[k - 1].abs()) + ev["xB"][k - 1].abs())
    return out


def supergrad_bound(net, batch, masks, scale, rel):
    """Per-entry bound on |s_gpu - s_orc| when the GPU may take a different vertex at
    every decision flagged in ``masks`` (from unstable_decisions):
      rel * scale                     contraction rounding (decisions agree)
    + |W_k| (m_{k-1} * (|l|+|u|))     a flipped x*_{k-1}[j] moves xA_k by |W_k[:, j]| * |dx_j|
    + m_k * (u - l)                   a flipped xB*_k[i] moves by at most u - l
    with dx_j <= u0 - l0 for the input layer and <= |l| + |u| for a hidden neuron."""
    out = []
    n = len(net)
    for k in range(1, n):
        if k == 1:
            dx = masks[0].double() * (batch.u0 - batch.l0)
        else:
            dx = masks[k - 1].double() * (batch.l[k - 2].abs() + batch.u[k - 2].abs())
        L = abs_layer(net[k - 1])
        spread = L.forward(dx) - L.bias_full()
        own = masks[k].double() * (batch.u[k - 1] - batch.l[k - 1])
        out.append(rel * scale[k - 1] + spread + own)
    return out



def first_step_may_differ(net, batch, rho, tau=O.TAU_DEFAULT, exact_ties_stable=False):
    """Duals whose first Adam step from rho (zero moments) may differ between the
    GPU's FP32 evaluation and the oracle's.  That step is lr * s / (|s| + eps) per
    entry, about lr * sign(s): it changes only where s may change sign, i.e. where
    |s| lies within supergrad_bound's bound on |s_gpu - s_orc| (contraction rounding
    plus every decision within rounding of a tie, carried through |W|)."""
    ev = O.dual_eval(net, batch, rho, tau)
    masks = unstable_decisions(net, batch, rho, ev, tau, exact_ties_stable=exact_ties_stable)
    bound = supergrad_bound(net, batch, masks, s_scale(net, ev), REL)
    return [ev["s"][k].abs() <= bound[k] + 1e-7 for k in range(len(net) - 1)]
