"""Pins of the oracle's proximal solver (Sec. 3.3, Algorithm 2, App. F).

None of these re-types the oracle's formulas: the step size is checked against a
direct search along the Frank-Wolfe segment of the augmented Lagrangian written
from its definition; the conditional gradient against the gradient taken by
automatic differentiation and a vertex enumeration of each ReLU hull; the whole
method against the Planet LP optimum (Prop. 1) computed by HiGHS.
"""
import numpy as np
import pytest
import torch

import ldgen
from oracle import ld_oracle as O
from tests import _brute
from tests.test_oracle_pins import _planet_lp


def _setup(name, **kw):
    inst = ldgen.make_instance(name, **kw)
    return inst, O.net_from_specs(inst.layers), O.batch_from_instance(inst)


def _mid_run_state(net, batch, iters=3, **kw):
    """A primal/dual point of a run a few iterations in (not at a vertex)."""
    opts = O.ProxOpts(T=20, **kw)
    return O.proximal(net, batch, opts, iters=iters), opts


def _al(net, batch, rho, eta, xB, xA):
    """Augmented Lagrangian of eq:z_updates from its definition, per subdomain."""
    L = (batch.c * xA[-1]).sum(dim=1)
    for k in range(len(rho)):
        d = xB[k] - xA[k]
        L = L + (rho[k] * d).sum(dim=1) + 0.5 / eta * (d * d).sum(dim=1)
    return L


@pytest.mark.parametrize("name", ["fc_tiny", "tiny_conv2", "tiny_conv3"])
def test_gamma_is_the_exact_line_search(name):
    """eq:optimal-gamma-gauss: gamma* minimises the augmented Lagrangian over the
    Frank-Wolfe segment of the block, clipped to [0, 1]."""
    inst, net, batch = _setup(name)
    st, opts = _mid_run_state(net, batch)
    eta = 37.0
    grid = torch.linspace(0.0, 1.0, 4001, dtype=torch.float64)
    for k in range(len(net)):
        xB = [x.clone() for x in st["xB"]]
        xA = [x.clone() for x in st["xA"]]
        xB0 = [x.clone() for x in xB]
        xA0 = [x.clone() for x in xA]
        out = O.prox_block(net, batch, st["rho"], eta, xB, xA, k)
        gam = out["gamma"]
        assert bool(((gam >= 0) & (gam <= 1)).all())
        L_new = _al(net, batch, st["rho"], eta, xB, xA)
        best = torch.full_like(L_new, float("inf"))
        for g in grid:
            yB = [x.clone() for x in xB0]
            yA = [x.clone() for x in xA0]
            if k >= 1:
                yB[k - 1] = xB0[k - 1] + g * (out["zB"] - xB0[k - 1])
            yA[k] = xA0[k] + g * (out["zA"] - xA0[k])
            best = torch.minimum(best, _al(net, batch, st["rho"], eta, yB, yA))
        scale = 1e-11 * (1 + L_new.abs())
        assert bool((L_new <= best + scale).all()), (k, (L_new - best).max().item())
        assert bool((L_new <= _al(net, batch, st["rho"], eta, xB0, xA0) + scale).all())


@pytest.mark.parametrize("name", ["fc_tiny", "tiny_conv2"])
def test_conditional_gradient_minimises_the_linearisation(name):
    """The conditional gradient of block k minimises the linearised augmented
    Lagrangian over P_k (Sec. 3.3.2): compare with autograd's gradient and a vertex
    enumeration of each ReLU hull (box endpoints for P_0)."""
    inst, net, batch = _setup(name)
    st, opts = _mid_run_state(net, batch)
    eta = 23.0
    mats = [_brute.dense_matrix(s) for s in inst.layers]
    bias = [_brute.dense_bias(s) for s in inst.layers]
    n = len(net)
    for k in range(n):
        xB = [x.clone().requires_grad_(True) for x in st["xB"]]
        xA = [x.clone().requires_grad_(True) for x in st["xA"]]
        _al(net, batch, st["rho"], eta, xB, xA).sum().backward()
        GA = xA[k].grad.detach().numpy()                 # gradient w.r.t. xA_{k+1}
        GB = xB[k - 1].grad.detach().numpy() if k >= 1 else None
        out = O.prox_block(net, batch, st["rho"], eta, [x.detach().clone() for x in xB],
                           [x.detach().clone() for x in xA], k)
        zA = out["zA"].numpy()
        for b in range(inst.B):
            h = mats[k].T @ GA[b]                        # coefficient of x_k (or x_0)
            const = GA[b] @ bias[k]
            if k == 0:
                lo, hi = inst.l0[b].astype(np.float64), inst.u0[b].astype(np.float64)
                brute = const + np.minimum(h * lo, h * hi).sum()
                got = GA[b] @ zA[b]
            else:
                lo = inst.l[k - 1][b].astype(np.float64)
                hi = inst.u[k - 1][b].astype(np.float64)
                brute = const + sum(_brute.hull_min(GB[b, i], -h[i], lo[i], hi[i]) for i in range(len(lo)))
                got = GB[b] @ out["zB"][b].numpy() + GA[b] @ zA[b]
            assert abs(got - brute) <= 1e-9 * (1 + abs(brute)), (k, b, got, brute)


@pytest.mark.parametrize("name", ["fc_tiny", "tiny_conv3"])
def test_block_steps_never_increase_the_augmented_lagrangian(name):
    inst, net, batch = _setup(name)
    st, opts = _mid_run_state(net, batch)
    eta = 50.0
    xB = [x.clone() for x in st["xB"]]
    xA = [x.clone() for x in st["xA"]]
    prev = _al(net, batch, st["rho"], eta, xB, xA)
    for _ in range(15):
        for k in range(len(net)):
            O.prox_block(net, batch, st["rho"], eta, xB, xA, k)
            cur = _al(net, batch, st["rho"], eta, xB, xA)
            assert bool((cur <= prev + 1e-11 * (1 + prev.abs())).all())
            prev = cur


@pytest.mark.parametrize("name", ["fc_tiny", "tiny_conv"])
def test_proximal_approaches_the_lp_optimum(name):
    """Prop. 1: every q is below the Planet LP optimum, and the method of multipliers
    approaches it (Sec. 7.2 settings: J = 2, mu = 0.3, eta 10 -> 500)."""
    inst, net, batch = _setup(name, split_frac=0.0)
    st = O.proximal(net, batch, O.ProxOpts(T=1000), record=True)
    fb = O.final_bound(net, batch, st)
    for b in range(inst.B):
        p = _planet_lp(inst, b)
        assert max(q[b].item() for q in st["traj"]) <= p + 1e-9
        gap0 = p - st["q0"][b].item()
        assert gap0 > 1e-3
        assert p - fb["bound"][b].item() <= 0.01 * gap0, (b, p, st["q0"][b].item(), fb["bound"][b].item())


def test_proximal_resume_equals_single_run():
    inst, net, batch = _setup("tiny_conv2")
    opts = O.ProxOpts(T=12)
    full = O.proximal(net, batch, opts)
    half = O.proximal(net, batch, opts, iters=5)
    rest = O.proximal(net, batch, opts, state=half, iters=7)
    for key in ("rho", "pi", "xB", "xA"):
        for a, b in zip(full[key], rest[key]):
            assert torch.equal(a, b), key


def test_eta_schedule_endpoints():
    assert O.prox_eta(1, 100, 10.0, 500.0) == 10.0
    assert abs(O.prox_eta(100, 100, 10.0, 500.0) - 500.0) < 1e-12
    assert O.prox_eta(7, 100, 100.0, 100.0) == 100.0


def test_initial_primal_is_an_inner_minimiser():
    """Algorithm 2 starts the primal at a minimiser of the Lagrangian at rho^0: its
    Lagrangian value (the augmented one at eta = infinity) equals q(rho^0)."""
    inst, net, batch = _setup("tiny_conv2")
    rho = O.crown_init(net, batch)
    xB, xA = O.prox_primal_init(net, batch, rho)
    L = (batch.c * xA[-1]).sum(dim=1)
    for k in range(len(rho)):
        L = L + (rho[k] * (xB[k] - xA[k])).sum(dim=1)
    q = O.dual_eval(net, batch, rho, need_supergrad=False)["q"]
    assert torch.allclose(L, q, rtol=1e-12, atol=1e-12)
