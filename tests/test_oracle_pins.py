"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the passage it relies on.  None of them re-types the oracle's
formula: they use brute force, hand-derived closed forms, a different formula
the paper proves equal (Prop. 1, Prop. 2), inequalities (weak duality) or
numerical differentiation (Danskin's theorem).
"""
import json
import os

import numpy as np
import pytest
import torch

import ldgen
from oracle import ld_oracle as O
from tests import _brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _setup(name, **kw):
    inst = ldgen.make_instance(name, **kw)
    return inst, O.net_from_specs(inst.layers), O.batch_from_instance(inst)


def _t(a):
    return torch.as_tensor(np.asarray(a), dtype=torch.float64)


# --------------------------------------------------------------------------
# linear maps: forward against the convolution's definition; transposed product
# against the adjoint identity  <W x, r> = <x, W^T r>
# --------------------------------------------------------------------------
@pytest.mark.parametrize("name", ["tiny_conv", "tiny_conv2", "fc_tiny"])
def test_layer_maps_match_dense_definition(name):
    inst, net, _ = _setup(name)
    rng = np.random.default_rng(0)
    for spec, L in zip(inst.layers, net):
        M = _brute.dense_matrix(spec)
        bias = _brute.dense_bias(spec)
        x = rng.standard_normal((3, M.shape[1]))
        r = rng.standard_normal((3, M.shape[0]))
        np.testing.assert_allclose(L.forward(_t(x)).numpy(), x @ M.T + bias, rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(L.transposed(_t(r)).numpy(), r @ M, rtol=1e-12, atol=1e-12)
        lhs = (L.forward(_t(x)) - L.bias_full()) * _t(r)
        rhs = _t(x) * L.transposed(_t(r))
        np.testing.assert_allclose(lhs.sum(1).numpy(), rhs.sum(1).numpy(), rtol=1e-10)


# --------------------------------------------------------------------------
# P1: the closed-form inner minimum over the ReLU hull (eq:min-pk and the
# non-ambiguous case) against vertex enumeration of the constraint polygon
# (eq:planet-relu-hull plus the box) and against dense sampling
# --------------------------------------------------------------------------
def _pk_cases():
    rng = np.random.default_rng(1)
    cases = []
    for _ in range(400):
        kind = rng.integers(0, 3)
        a, b = sorted(rng.standard_normal(2) * 2)
        if kind == 0:        # passing
            l, u = abs(a), abs(a) + abs(b)
        elif kind == 1:      # blocking
            l, u = -abs(a) - abs(b), -abs(a)
        else:                # ambiguous
            l, u = -abs(a) - 1e-3, abs(b) + 1e-3
        cases.append((rng.standard_normal() * 2, rng.standard_normal() * 2, l, u))
    # boundary / degenerate cases: l = 0, u = 0, l = u, zero duals, exact ties
    cases += [(0.3, -0.2, 0.0, 1.5), (-0.4, 0.7, -2.0, 0.0), (0.5, 0.5, 0.7, 0.7), (0.1, 1.0, -0.5, -0.5),
              (0.0, 0.0, -1.0, 1.0), (0.0, 0.3, -1.0, 2.0), (0.25, 1.0, -1.0, 1.0), (1.0, 1.0, -1.0, 1.0),
              (-0.5, -0.5, -1.0, 1.0), (0.0, -0.5, -1.0, 1.0), (0.0, 0.0, 0.0, 0.0)]
    return cases


def test_inner_min_pk_matches_vertex_enumeration():
    cases = _pk_cases()
    rho, g, l, u = (_t([c[i] for c in cases]) for i in range(4))
    for tau in (0.0, O.TAU_DEFAULT):
        xb, x, val = O.inner_min_pk(rho, g, l, u, tau=tau)
        for i, (r_, g_, l_, u_) in enumerate(cases):
            ref = _brute.hull_min(r_, g_, l_, u_)
            assert abs(val[i].item() - ref) <= 1e-12 * (1 + abs(ref)), (cases[i], val[i].item(), ref)
            # the returned minimiser is feasible and (for tau = 0) attains the minimum
            assert _brute.hull_feasible(xb[i].item(), x[i].item(), l_, u_), cases[i]
            obj = r_ * xb[i].item() - g_ * x[i].item()
            slack = 0.0 if tau == 0.0 else 4 * tau * (abs(r_) + abs(g_)) * (abs(l_) + abs(u_))
            assert obj <= ref + 1e-12 * (1 + abs(ref)) + slack, (cases[i], obj, ref)


def test_inner_min_pk_dense_sampling_never_below():
    rng = np.random.default_rng(2)
    for (r_, g_, l_, u_) in _pk_cases()[:60]:
        ref = O.inner_min_pk(_t([r_]), _t([g_]), _t([l_]), _t([u_]), tau=0.0)[2].item()
        xs = rng.uniform(l_, u_, size=2000)
        if l_ >= 0:
            ys = xs
        elif u_ <= 0:
            ys = np.zeros_like(xs)
        else:
            lo = np.maximum(xs, 0.0)
            hi = u_ * (xs - l_) / (u_ - l_)
            ys = lo + rng.uniform(size=xs.size) * (hi - lo)
        assert (r_ * xs - g_ * ys).min() >= ref - 1e-12


def test_tie_rule_prefers_larger_xb():
    # exact kinks of a CROWN-initialised neuron (derivation in App. B): V_l = V_u when g > 0
    l, u, g = -1.0, 3.0, 2.0
    rho = u / (u - l) * g
    xb, _, _ = O.inner_min_pk(_t([rho]), _t([g]), _t([l]), _t([u]))
    assert xb.item() == u
    # V_0 = V_u with lower slope 1 and g < 0
    xb, _, _ = O.inner_min_pk(_t([-0.5]), _t([-0.5]), _t([l]), _t([u]))
    assert xb.item() == u
    # V_l = V_0 with lower slope 0 and g < 0
    xb, _, _ = O.inner_min_pk(_t([0.0]), _t([-0.5]), _t([l]), _t([u]))
    assert xb.item() == 0.0


# --------------------------------------------------------------------------
# P2: box solution of P_0 (eq:box_bounds_sol) against all 2^n0 corners
# --------------------------------------------------------------------------
def test_inner_min_p0_matches_corner_enumeration():
    rng = np.random.default_rng(3)
    n0 = 9
    corners = np.array(np.meshgrid(*[[0, 1]] * n0, indexing="ij")).reshape(n0, -1).T
    for trial in range(20):
        g0 = rng.standard_normal((1, n0))
        if trial == 0:
            g0[0, :3] = 0.0
        l0 = rng.standard_normal((1, n0))
        u0 = l0 + np.abs(rng.standard_normal((1, n0)))
        pts = np.where(corners == 1, u0, l0)
        ref = (-(pts @ g0[0])).min()
        x0, v = O.inner_min_p0(_t(g0), _t(l0), _t(u0))
        assert abs(v.item() - ref) <= 1e-12 * (1 + abs(ref))
        assert abs(-(x0.numpy()[0] @ g0[0]) - ref) <= 1e-12 * (1 + abs(ref))


# --------------------------------------------------------------------------
# hand-derived closed forms (tests/golden/hand_examples.json)
# --------------------------------------------------------------------------
def _golden_net(ex):
    layers = []
    n_in = len(ex["l0"])
    for L in ex["layers"]:
        W = _t(L["W"])
        layers.append(O.OLayer("linear", W, _t(L["b"]), (n_in, 1, 1), (W.shape[0], 1, 1)))
        n_in = W.shape[0]
    batch = O.OBatch(_t([ex["l0"]]), _t([ex["u0"]]), [_t([a]) for a in ex["l"]],
                     [_t([a]) for a in ex["u"]], _t([ex["c"]]))
    return layers, batch


def test_golden_hand_examples():
    data = json.load(open(os.path.join(GOLDEN, "hand_examples.json")))
    for ex in data["examples"]:
        net, batch = _golden_net(ex)
        for case in ex["cases"]:
            rho = [_t(r)[None, :] if _t(r).dim() == 1 else _t(r) for r in case["rho"]]
            ev = O.dual_eval(net, batch, rho, tau=0.0)
            assert abs(ev["q"].item() - case["q"]) < 1e-12, (ex["name"], case, ev["q"].item())
            if "supergrad" in case:
                for s, ref in zip(ev["s"], case["supergrad"]):
                    np.testing.assert_allclose(s.numpy()[0], ref, atol=1e-12)
        if "lp_optimum" in ex:
            st = O.ascent(net, batch, O.AdamOpts(T=400, lr0=1e-2, lr_end=1e-4, init="zero"))
            fb = O.final_bound(net, batch, st)
            assert fb["bound"].item() <= ex["lp_optimum"] + 1e-12
            assert fb["bound"].item() >= ex["lp_optimum"] - 1e-6


def test_golden_primal_values():
    """Sec. 5.1.3: the upper bound is the network's value at the last P_0 minimiser.
    x0*, c^T f(x0*) and its feasibility against the intermediate bounds, worked out
    by hand (tests/golden/hand_examples.json, primal_cases)."""
    data = json.load(open(os.path.join(GOLDEN, "hand_examples.json")))
    seen = set()
    for ex in data["examples"]:
        net, batch = _golden_net(ex)
        for case in ex.get("primal_cases", []):
            rho = [_t(r)[None, :] for r in case["rho"]]
            ev = O.dual_eval(net, batch, rho, tau=0.0)
            np.testing.assert_array_equal(ev["x0"].numpy()[0], case["x0"])
            p, feas = O.primal_value(net, batch, ev["x0"])
            assert abs(p.item() - case["primal"]) < 1e-12, (ex["name"], case, p.item())
            assert bool(feas.item()) == case["feasible"], (ex["name"], case)
            seen.add(case["feasible"])
    assert seen == {True, False}


@pytest.mark.parametrize("name", ["fc_tiny", "tiny_conv", "tiny_conv2", "tiny_conv3"])
def test_primal_value_matches_dense_forward(name):
    """c^T f(x) and the feasibility flag against the network written as dense matrices
    (built from the convolution's definition, no oracle code): random points of the
    box, the box corners the P_0 rule picks, on split and unsplit subdomains."""
    inst = ldgen.make_instance(name)
    root = ldgen.make_instance(name, split_frac=0.0)
    rng = np.random.default_rng(5)
    Ms = [_brute.dense_matrix(sp) for sp in inst.layers]
    bs = [_brute.dense_bias(sp) for sp in inst.layers]
    net = O.net_from_specs(inst.layers)
    flags = []
    for it in (inst, root):
        batch = O.batch_from_instance(it)
        B = it.B
        for trial in range(4):
            w = rng.uniform(size=it.l0.shape) if trial < 2 else (rng.uniform(size=it.l0.shape) < 0.5) * 1.0
            x0 = it.l0.astype(np.float64) + w * (it.u0.astype(np.float64) - it.l0.astype(np.float64))
            p, feas = O.primal_value(net, batch, _t(x0))
            for b in range(B):
                x = x0[b]
                ok = True
                for k in range(len(Ms) - 1):
                    xh = Ms[k] @ x + bs[k]
                    ok &= bool(np.all(xh >= it.l[k][b].astype(np.float64)) and
                               np.all(xh <= it.u[k][b].astype(np.float64)))
                    x = np.maximum(xh, 0.0)
                y = Ms[-1] @ x + bs[-1]
                ref = float(it.c[b].astype(np.float64) @ y)
                assert abs(p[b].item() - ref) <= 1e-10 * (1.0 + abs(ref)), (b, p[b].item(), ref)
                assert bool(feas[b].item()) == ok, (name, b)
                flags.append(ok)
    # root subdomains: the interval bounds contain every pre-activation of the box
    assert any(flags) and all(flags[-4 * root.B:])


# --------------------------------------------------------------------------
# P3: q(0) equals interval propagation through the c-folded last layer (Sec. 7.2:
# IBP corresponds to all duals set to zero)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("name", ["fc_tiny", "tiny_conv", "tiny_conv2"])
def test_q_of_zero_is_interval_bound(name):
    inst, net, batch = _setup(name)
    ev = O.dual_eval(net, batch, O.zero_init(net, batch), need_supergrad=False)
    Wn = _brute.dense_matrix(inst.layers[-1])
    bn = _brute.dense_bias(inst.layers[-1])
    for b in range(inst.B):
        w = Wn.T @ inst.c[b].astype(np.float64)
        lo = np.maximum(inst.l[-1][b].astype(np.float64), 0)
        hi = np.maximum(inst.u[-1][b].astype(np.float64), 0)
        ref = inst.c[b].astype(np.float64) @ bn + np.minimum(w * lo, w * hi).sum()
        assert abs(ev["q"][b].item() - ref) <= 1e-12 * (1 + abs(ref))


# --------------------------------------------------------------------------
# P4: Prop. 2 -- at the dual point of a propagation method, q equals the
# propagation bound of eq:bounds-propagation, for any lower slope in [0, 1]
# (App. B, eq:slopes-biases).  The propagation side is computed here from
# dense matrices.
# --------------------------------------------------------------------------
def _propagation_bound(inst, b, slope_kind, rng):
    mats = [_brute.dense_matrix(s) for s in inst.layers]
    biases = [_brute.dense_bias(s) for s in inst.layers]
    n = len(mats)
    lam = mats[-1].T @ (-inst.c[b].astype(np.float64))      # lambda_{n-1}
    mus = [None] * (n - 1)
    bbar_terms = 0.0
    for k in range(n - 1, 0, -1):
        l = inst.l[k - 1][b].astype(np.float64)
        u = inst.u[k - 1][b].astype(np.float64)
        amb = (l < 0) & (u > 0)
        pas = l >= 0
        den = np.where(amb, u - l, 1.0)
        a_up = np.where(amb, u / den, np.where(pas, 1.0, 0.0))
        if slope_kind == "crown":
            a_lo = np.where(amb, (u >= -l).astype(float), np.where(pas, 1.0, 0.0))
        elif slope_kind == "wk":
            a_lo = a_up.copy()
        else:
            a_lo = np.where(amb, rng.uniform(size=l.size), np.where(pas, 1.0, 0.0))
        bbar = np.where(amb, -l * u / den, 0.0)
        mu = a_up * np.maximum(lam, 0) + a_lo * np.minimum(lam, 0)
        bbar_terms += np.maximum(lam, 0) @ bbar
        mus[k - 1] = mu
        lam = mats[k - 1].T @ mu
    # lam is now W_1^T mu_1
    l0 = inst.l0[b].astype(np.float64)
    u0 = inst.u0[b].astype(np.float64)
    p0 = -np.maximum(lam * l0, lam * u0).sum()
    bias_terms = sum(mus[k] @ biases[k] for k in range(n - 1))
    dP = p0 + inst.c[b].astype(np.float64) @ biases[-1] - bias_terms - bbar_terms
    return mus, dP


@pytest.mark.parametrize("name", ["fc_tiny", "tiny_conv", "tiny_conv2"])
@pytest.mark.parametrize("slope_kind", ["crown", "wk", "random"])
def test_prop2_q_equals_propagation_bound(name, slope_kind):
    inst, net, batch = _setup(name)
    rng = np.random.default_rng(4)
    for b in range(inst.B):
        mus, dP = _propagation_bound(inst, b, slope_kind, rng)
        sub = O.batch_from_instance(inst, [b])
        q = O.dual_eval(net, sub, [_t(m)[None, :] for m in mus], need_supergrad=False)["q"].item()
        assert abs(q - dP) <= 1e-10 * (1 + abs(dP)), (b, q, dP)
    # the oracle's own CROWN initialisation reaches the same CROWN bound
    if slope_kind == "crown":
        rho = O.crown_init(net, batch)
        q = O.dual_eval(net, batch, rho, need_supergrad=False)["q"]
        for b in range(inst.B):
            _, dP = _propagation_bound(inst, b, "crown", rng)
            assert abs(q[b].item() - dP) <= 1e-10 * (1 + abs(dP))


# --------------------------------------------------------------------------
# P9: the Lagrangian at the inner minimisers equals the decomposed minimum
# (eq:nonprox_problem): q = xA_n + sum_k rho_k^T (xB_k - xA_k)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("name", ["fc_tiny", "tiny_conv", "tiny_conv2"])
def test_lagrangian_identity(name):
    inst, net, batch = _setup(name)
    rho = [_t(r) for r in ldgen.random_duals(inst, seed=5, scale=0.3)]
    ev = O.dual_eval(net, batch, rho, tau=0.0)
    rhs = ev["xA_n"] + sum((r * s).sum(1) for r, s in zip(rho, ev["s"]))
    np.testing.assert_allclose(ev["q"].numpy(), rhs.numpy(), rtol=1e-11, atol=1e-11)


# --------------------------------------------------------------------------
# P7: the supergradient xB* - xA* (Algorithm 1) equals the directional
# derivative of the piecewise-linear q away from kinks (central differences)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("name", ["fc_tiny", "tiny_conv", "tiny_conv2"])
def test_supergradient_matches_finite_differences(name):
    inst, net, batch = _setup(name)
    rng = np.random.default_rng(6)
    h = 1e-4
    checked = 0
    for trial in range(6):
        rho = [_t(r) for r in ldgen.random_duals(inst, seed=100 + trial, scale=0.3)]
        d = [_t(rng.standard_normal(r.shape)) for r in rho]
        ev = O.dual_eval(net, batch, rho, tau=0.0)
        evp = O.dual_eval(net, batch, [r + h * e for r, e in zip(rho, d)], tau=0.0, need_supergrad=False)
        evm = O.dual_eval(net, batch, [r - h * e for r, e in zip(rho, d)], tau=0.0, need_supergrad=False)
        fd = (evp["q"] - evm["q"]) / (2 * h)
        sd = sum((s * e).sum(1) for s, e in zip(ev["s"], d))
        for b in range(inst.B):
            same = all(torch.equal(a[b], p[b]) and torch.equal(a[b], m[b])
                       for a, p, m in zip([ev["x0"]] + ev["xB"], [evp["x0"]] + evp["xB"], [evm["x0"]] + evm["xB"]))
            if same:
                checked += 1
                assert abs(fd[b].item() - sd[b].item()) <= 1e-7 * (1 + abs(sd[b].item()))
    assert checked >= 6


# --------------------------------------------------------------------------
# P5: weak duality (Sec. 3.1): every q(rho) is below the network output at
# every input of the subdomain -- dense samples, box corners and PGD minima
# --------------------------------------------------------------------------
def _feasible_mask(net, batch, b, X):
    x = X
    ok = torch.ones(X.shape[0], dtype=torch.bool)
    for k in range(len(net) - 1):
        xh = net[k].forward(x)
        ok &= ((xh >= batch.l[k][b]) & (xh <= batch.u[k][b])).all(1)
        x = torch.clamp(xh, min=0)
    return ok


def _pgd_min(net, c, l0, u0, steps=200, restarts=8, seed=0):
    g = torch.Generator().manual_seed(seed)
    x = l0 + (u0 - l0) * torch.rand((restarts, l0.numel()), generator=g, dtype=torch.float64)
    best = float("inf")
    lr = (u0 - l0).max().item() * 0.05
    for _ in range(steps):
        x = x.detach().requires_grad_(True)
        val = (O.network_output(net, x) * c).sum(1)
        best = min(best, val.min().item())
        (gr,) = torch.autograd.grad(val.sum(), x)
        x = torch.minimum(torch.maximum(x - lr * gr.sign(), l0), u0)
    return best


@pytest.mark.parametrize("name", ["fc_tiny", "tiny_conv", "tiny_conv2"])
def test_weak_duality(name):
    inst, net, batch = _setup(name, split_frac=0.0)     # root subdomains: the whole box is feasible
    rho_sets = [O.crown_init(net, batch), O.zero_init(net, batch),
                [_t(r) for r in ldgen.random_duals(inst, seed=7, scale=0.3)]]
    st = O.ascent(net, batch, O.AdamOpts(T=60), record=True)
    rho_sets.append(st["rho"])
    qs = [O.dual_eval(net, batch, r, need_supergrad=False)["q"] for r in rho_sets] + st["traj"]
    gen = torch.Generator().manual_seed(8)
    for b in range(inst.B):
        l0, u0, c = batch.l0[b], batch.u0[b], batch.c[b]
        X = l0 + (u0 - l0) * torch.rand((3000, l0.numel()), generator=gen, dtype=torch.float64)
        assert bool(_feasible_mask(net, batch, b, X).all())
        vals = (O.network_output(net, X) * c).sum(1)
        ub = min(vals.min().item(), _pgd_min(net, c, l0, u0, seed=b))
        for q in qs:
            assert q[b].item() <= ub + 1e-9, (b, q[b].item(), ub)


def test_weak_duality_with_splits_on_feasible_samples():
    # splits drawn consistently with the activation pattern of one input, so that
    # the subdomain is non-empty; then feasible samples are found around it
    inst, net, batch = _setup("fc_tiny", split_frac=0.0)
    rng = np.random.default_rng(9)
    xs = batch.l0 + (batch.u0 - batch.l0) * _t(rng.uniform(size=batch.l0.shape))
    x = xs
    for k in range(len(net) - 1):
        xh = net[k].forward(x)
        amb = (batch.l[k] < 0) & (batch.u[k] > 0)
        pick = amb & _t(rng.uniform(size=xh.shape) < 0.3).bool()
        batch.l[k] = torch.where(pick & (xh >= 0), torch.zeros_like(xh), batch.l[k])
        batch.u[k] = torch.where(pick & (xh < 0), torch.zeros_like(xh), batch.u[k])
        x = torch.clamp(xh, min=0)
    rho_sets = [O.crown_init(net, batch), O.ascent(net, batch, O.AdamOpts(T=100))["rho"]]
    gen = torch.Generator().manual_seed(9)
    X = xs + 0.05 * (batch.u0 - batch.l0) * (torch.rand((20000, batch.l0.shape[1]), generator=gen,
                                                         dtype=torch.float64) - 0.5)
    X = torch.minimum(torch.maximum(X, batch.l0), batch.u0)
    X = torch.cat([xs, X])
    ok = _feasible_mask(net, batch, 0, X)
    assert bool(ok[0]) and int(ok.sum()) > 10
    ub = (O.network_output(net, X[ok]) * batch.c[0]).sum(1).min().item()
    for r in rho_sets:
        assert O.dual_eval(net, batch, r, need_supergrad=False)["q"][0].item() <= ub + 1e-9


# --------------------------------------------------------------------------
# P6: Prop. 1 -- max_rho q = optimum of the Planet LP (eq:planet-relax).  Every
# q is below the LP optimum (HiGHS), and the ascent approaches it.
# --------------------------------------------------------------------------
def _planet_lp(inst, b):
    from scipy.optimize import linprog
    mats = [_brute.dense_matrix(s) for s in inst.layers]
    biases = [_brute.dense_bias(s) for s in inst.layers]
    n = len(mats)
    n0 = mats[0].shape[1]
    sizes = [m.shape[0] for m in mats[:-1]]
    # variables: x0, then (xhat_k, x_k) for each hidden layer
    off = [n0]
    for s in sizes:
        off.append(off[-1] + 2 * s)
    nv = off[-1]
    xh = lambda k: slice(off[k - 1], off[k - 1] + sizes[k - 1])          # noqa: E731
    xr = lambda k: slice(off[k - 1] + sizes[k - 1], off[k])                # noqa: E731
    Aeq, beq, Aub, bub = [], [], [], []
    bounds = [(float(inst.l0[b, j]), float(inst.u0[b, j])) for j in range(n0)]
    for k in range(1, n):
        l = inst.l[k - 1][b].astype(np.float64)
        u = inst.u[k - 1][b].astype(np.float64)
        bounds += [(float(l[i]), float(u[i])) for i in range(sizes[k - 1])]
        bounds += [(float(max(l[i], 0)), float(max(u[i], 0))) for i in range(sizes[k - 1])]
        # xhat_k = W_k x_{k-1} + b_k
        for i in range(sizes[k - 1]):
            row = np.zeros(nv)
            row[xh(k)][i] = 1.0
            src = slice(0, n0) if k == 1 else xr(k - 1)
            row[src] -= mats[k - 1][i]
            Aeq.append(row)
            beq.append(biases[k - 1][i])
            r2 = np.zeros(nv)
            if l[i] >= 0:
                r2[xr(k)][i] = 1.0
                r2[xh(k)][i] = -1.0
                Aeq.append(r2)
                beq.append(0.0)
            elif u[i] <= 0:
                r2[xr(k)][i] = 1.0
                Aeq.append(r2)
                beq.append(0.0)
            else:
                r2[xh(k)][i] = 1.0
                r2[xr(k)][i] = -1.0          # xhat - x <= 0
                Aub.append(r2)
                bub.append(0.0)
                r3 = np.zeros(nv)
                r3[xr(k)][i] = 1.0
                r3[xh(k)][i] = -u[i] / (u[i] - l[i])   # x - u/(u-l) xhat <= -u l/(u-l)
                Aub.append(r3)
                bub.append(-u[i] * l[i] / (u[i] - l[i]))
    cvec = inst.c[b].astype(np.float64)
    obj = np.zeros(nv)
    obj[xr(n - 1)] = mats[-1].T @ cvec
    res = linprog(obj, A_ub=np.array(Aub) if Aub else None, b_ub=np.array(bub) if bub else None,
                  A_eq=np.array(Aeq), b_eq=np.array(beq), bounds=bounds, method="highs")
    assert res.status == 0, res.message
    return res.fun + cvec @ biases[-1]


@pytest.mark.parametrize("name", ["fc_tiny", "tiny_conv"])
def test_prop1_lp_optimum_bounds_and_is_approached(name):
    # root subdomains: a random split can empty the LP (the dual is then unbounded)
    inst, net, batch = _setup(name, split_frac=0.0)
    st = O.ascent(net, batch, O.AdamOpts(T=1500, lr0=1e-2, lr_end=1e-5), record=True)
    fb = O.final_bound(net, batch, st)
    for b in range(inst.B):
        p = _planet_lp(inst, b)
        assert st["q0"][b].item() <= p + 1e-9
        assert max(q[b].item() for q in st["traj"]) <= p + 1e-9
        assert fb["q_final"][b].item() <= p + 1e-9
        # the ascent closes most of the gap between the CROWN start and the LP optimum
        gap0 = p - st["q0"][b].item()
        assert p - fb["bound"][b].item() <= 0.2 * gap0 + 1e-6, (b, p, st["q0"][b].item(), fb["bound"][b].item())


# --------------------------------------------------------------------------
# Adam (Sec. 7.2): first step is lr0 * s / (|s| + eps); resume equals one run;
# the returned bound is never below the initial one
# --------------------------------------------------------------------------
def test_adam_first_step_closed_form():
    inst, net, batch = _setup("tiny_conv")
    opts = O.AdamOpts(T=10, lr0=0.01, lr_end=0.001)
    rho0 = O.crown_init(net, batch)
    s0 = O.dual_eval(net, batch, rho0)["s"]
    st = O.ascent(net, batch, opts, iters=1)
    for r1, r0, s in zip(st["rho"], rho0, s0):
        np.testing.assert_allclose((r1 - r0).numpy(), (0.01 * s / (s.abs() + 1e-8)).numpy(), rtol=1e-9, atol=1e-15)


def test_step_schedule_endpoints():
    assert O.step_size(1, 500, 1e-2, 1e-4) == 1e-2
    assert abs(O.step_size(500, 500, 1e-2, 1e-4) - 1e-4) < 1e-18
    assert O.step_size(1, 1, 1e-2, 1e-4) == 1e-2


def test_resume_equals_single_run():
    inst, net, batch = _setup("tiny_conv2")
    opts = O.AdamOpts(T=40)
    full = O.ascent(net, batch, opts)
    half = O.ascent(net, batch, opts, iters=25)
    rest = O.ascent(net, batch, opts, state=half, iters=15)
    for a, b in zip(full["rho"], rest["rho"]):
        assert torch.equal(a, b)


def test_best_bound_not_below_initial():
    inst, net, batch = _setup("tiny_conv")
    st = O.ascent(net, batch, O.AdamOpts(T=50))
    fb = O.final_bound(net, batch, st)
    assert bool((fb["bound"] >= st["q0"]).all())
    assert bool((fb["bound"] >= fb["q_final"]).all())


def test_subdomains_do_not_interact():
    """The ascent of a batch equals each subdomain's ascent alone (the dual of
    eq:nonprox_problem separates over subdomains; the GPU's batching relies on it)."""
    inst, net, batch = _setup("tiny_conv")
    opts = O.AdamOpts(T=30)
    full = O.ascent(net, batch, opts)
    fb = O.final_bound(net, batch, full)
    for b in (0, inst.B // 2, inst.B - 1):
        sub = O.batch_from_instance(inst, [b])
        one = O.ascent(net, sub, opts)
        for a, c in zip(full["rho"], one["rho"]):
            assert torch.allclose(a[b:b + 1], c, rtol=0, atol=1e-9)
        ob = O.final_bound(net, sub, one)
        assert abs(fb["bound"][b].item() - ob["bound"][0].item()) <= 1e-9


def test_given_duals_are_used_as_given():
    """An ascent from caller-given duals equal to the CROWN duals is the CROWN ascent,
    and one from other given duals starts there (q0 is their dual value)."""
    inst, net, batch = _setup("tiny_conv")
    rho0 = O.crown_init(net, batch)
    a = O.ascent(net, batch, O.AdamOpts(T=20))
    g = O.ascent(net, batch, O.AdamOpts(T=20, init="given"), rho0=rho0)
    for x, y in zip(a["rho"], g["rho"]):
        assert torch.equal(x, y)
    other = [0.5 * r for r in rho0]
    h = O.ascent(net, batch, O.AdamOpts(T=20, init="given"), rho0=other, iters=0)
    assert torch.equal(h["q0"], O.dual_eval(net, batch, other, need_supergrad=False)["q"])
    for x, y in zip(h["rho"], other):
        assert torch.equal(x, y)
