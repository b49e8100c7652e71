"""Pins of the oracle's Filtered Smart Branching (Sec. 4.2).

The backward pass behind the scores is checked against finite differences of an
independent WK bound (dense matrices, tests/test_oracle_pins.py); the backup score
against the largest gap between the chord and the ReLU found by sampling; the
bounds of the children against that independent propagation bound (the better of
CROWN and WK); the decision against a brute-force search of the candidate set;
s_FSB and t_SR against values worked out by hand on a net of two ambiguous ReLUs
(tests/golden/hand_examples.json, fsb_examples).
"""
import copy
import json
import os
import types

import numpy as np
import pytest
import torch

import ldgen
from oracle import ld_oracle as O
from tests.test_oracle_pins import _propagation_bound


def _setup(name, **kw):
    inst = ldgen.make_instance(name, **kw)
    return inst, O.net_from_specs(inst.layers), O.batch_from_instance(inst)


def _wk_bound(inst, b):
    return _propagation_bound(inst, b, "wk", None)[1]


def _child_inst(inst, b, k, i, active):
    l = [a[b:b + 1].copy() for a in inst.l]
    u = [a[b:b + 1].copy() for a in inst.u]
    if active:
        l[k - 1][0, i] = 0.0
    else:
        u[k - 1][0, i] = 0.0
    return types.SimpleNamespace(layers=inst.layers, l0=inst.l0[b:b + 1], u0=inst.u0[b:b + 1], l=l, u=u,
                                 c=inst.c[b:b + 1])


def _indep_best(inst1):
    return max(_propagation_bound(inst1, 0, kind, None)[1] for kind in ("crown", "wk"))


@pytest.mark.parametrize("name", ["fc_tiny", "tiny_conv", "tiny_conv2"])
def test_backward_pass_is_the_wk_bias_sensitivity(name):
    """The WK bound is affine in the bias b_k with coefficient -a_k * lambda_k per
    neuron (a_k the chord slope), so central differences of the independent WK bound
    in one bias (a channel's, for a conv) pin lambda_k."""
    inst, net, batch = _setup(name)
    lams = O.fsb_lambdas(net, batch)
    h = 1e-3
    for k in range(1, len(net)):
        lam = lams[k - 1]
        l, u = batch.l[k - 1], batch.u[k - 1]
        amb = (l < 0) & (u > 0)
        a = torch.where(amb, u / torch.where(amb, u - l, torch.ones_like(u)), (l >= 0).to(u.dtype))
        coef = -(a * lam)
        spec = inst.layers[k - 1]
        per = 1 if spec.kind == "linear" else spec.out_shape[1] * spec.out_shape[2]
        for ch in range(min(spec.b.size, 4)):
            vals = []
            for sgn in (1, -1):
                mod = copy.deepcopy(inst)
                mod.layers[k - 1].b = mod.layers[k - 1].b.astype(np.float64).copy()
                mod.layers[k - 1].b[ch] += sgn * h
                vals.append(np.array([_wk_bound(mod, b) for b in range(inst.B)]))
            fd = (vals[0] - vals[1]) / (2 * h)
            want = coef[:, ch * per:(ch + 1) * per].sum(dim=1).numpy()
            np.testing.assert_allclose(fd, want, rtol=1e-6, atol=1e-8)


def test_backup_score_is_the_chord_gap():
    """t_SR / [lambda]_+ is the largest vertical gap between the chord and the ReLU on
    [l, u] (the distance the SR backup score weighs)."""
    inst, net, batch = _setup("tiny_conv")
    s, t = O.fsb_scores(net, batch)
    lams = O.fsb_lambdas(net, batch)
    checked = 0
    for k in range(1, len(net)):
        lam = lams[k - 1]
        l, u = batch.l[k - 1], batch.u[k - 1]
        for b in range(inst.B):
            for i in range(l.shape[1]):
                lo, hi, la = l[b, i].item(), u[b, i].item(), lam[b, i].item()
                if not (lo < 0 < hi) or la <= 0:
                    continue
                x = np.linspace(lo, hi, 200001)
                gap = np.max(hi * (x - lo) / (hi - lo) - np.maximum(x, 0))
                assert abs(t[k - 1][b, i].item() / la - gap) <= 1e-4 * (1 + gap)
                checked += 1
    assert checked > 0


@pytest.mark.parametrize("name", ["tiny_conv", "tiny_conv2"])
def test_scores_are_nonnegative_and_only_on_ambiguous_relus(name):
    inst, net, batch = _setup(name)
    s, t = O.fsb_scores(net, batch)
    for k in range(len(s)):
        amb = O.relu_status(batch.l[k], batch.u[k]) == 2
        assert bool((s[k] >= 0).all()) and bool((t[k] >= 0).all())
        assert bool((s[k][~amb] == 0).all()) and bool((t[k][~amb] == 0).all())


@pytest.mark.parametrize("name", ["fc_tiny", "tiny_conv", "tiny_conv2"])
def test_decision_is_the_best_worst_child(name):
    """FSB's value is max over the candidates of the worse child's bound, each child
    bounded independently by the better of CROWN and WK."""
    inst, net, batch = _setup(name)
    layer, index, value = O.fsb_branch(net, batch)
    s, t = O.fsb_scores(net, batch)
    cand = O.fsb_candidates(batch, s, t)
    for b in range(inst.B):
        best = -np.inf
        for k in range(1, len(net)):
            for col in range(2):
                i = int(cand[b, k - 1, col])
                if i < 0:
                    continue
                assert O.relu_status(batch.l[k - 1][b:b + 1, i], batch.u[k - 1][b:b + 1, i]).item() == 2
                v = min(_indep_best(_child_inst(inst, b, k, i, act)) for act in (True, False))
                best = max(best, v)
        assert abs(value[b].item() - best) <= 1e-10 * (1 + abs(best)), (b, value[b].item(), best)
        k, i = int(layer[b]), int(index[b])
        v = min(_indep_best(_child_inst(inst, b, k, i, act)) for act in (True, False))
        assert abs(v - best) <= 1e-10 * (1 + abs(best))


@pytest.mark.parametrize("name", ["fc_tiny", "tiny_conv", "tiny_conv2"])
def test_children_bound_at_parent_duals_is_not_below_the_parent(name):
    """A child's feasible set is a subset of its parent's, so at the parent's duals the
    child's dual value is at least the parent's (the property warm starts rely on)."""
    inst, net, batch = _setup(name)
    layer, index, _ = O.fsb_branch(net, batch)
    kids = O.branch_children(batch, layer, index)
    rng = np.random.default_rng(5)
    for rho in (O.crown_init(net, batch),
                [torch.as_tensor(rng.normal(size=r.shape) * 0.1) for r in O.crown_init(net, batch)]):
        qp = O.dual_eval(net, batch, rho, need_supergrad=False)["q"]
        rk = [r.repeat_interleave(2, dim=0) for r in rho]
        qc = O.dual_eval(net, kids, rk, need_supergrad=False)["q"]
        assert bool((qc >= qp.repeat_interleave(2) - 1e-12).all())
    # the split itself: child 2b active (l = 0), child 2b+1 inactive (u = 0)
    for b in range(inst.B):
        k, i = int(layer[b]), int(index[b])
        assert kids.l[k - 1][2 * b, i] == 0.0 and kids.u[k - 1][2 * b + 1, i] == 0.0
        assert kids.u[k - 1][2 * b, i] == batch.u[k - 1][b, i] and kids.l[k - 1][2 * b + 1, i] == batch.l[k - 1][b, i]


def test_fsb_scores_hand_example():
    """eq:fsb-scores and eq:babsr-scores on a hand-worked net: the min of the FSB score
    (the max of the SR score would give 6/13 for neuron a, not 7/13), the chord slope,
    the lambda of the folded objective, and the prefilter's argmax."""
    data = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "hand_examples.json")))
    for ex in data["fsb_examples"]:
        net, batch = [], None
        n_in = len(ex["l0"])
        for L in ex["layers"]:
            W = torch.tensor(L["W"], dtype=torch.float64)
            net.append(O.OLayer("linear", W, torch.tensor(L["b"], dtype=torch.float64), (n_in, 1, 1),
                                (W.shape[0], 1, 1)))
            n_in = W.shape[0]
        t = lambda a: torch.tensor([a], dtype=torch.float64)  # noqa: E731
        batch = O.OBatch(t(ex["l0"]), t(ex["u0"]), [t(a) for a in ex["l"]], [t(a) for a in ex["u"]], t(ex["c"]))
        s, tt = O.fsb_scores(net, batch)
        for k in range(len(s)):
            np.testing.assert_allclose(s[k].numpy()[0], ex["s_fsb"][k], rtol=1e-14, atol=1e-15)
            np.testing.assert_allclose(tt[k].numpy()[0], ex["t_sr"][k], rtol=1e-14, atol=1e-15)
        cand = O.fsb_candidates(batch, s, tt)
        assert cand[0].tolist() == ex["candidates"]

