"""Proximal solver (Sec. 3.3, Algorithm 2) on the GPU against the FP64 oracle.

Every test prints the case it is about to run before touching the GPU.  Inputs
come from the seeded generator only.
"""
import ctypes

import pytest
import torch

import ldgen
from oracle import ld_oracle as O

pytestmark = pytest.mark.gpu

SMALL = ["fc_tiny", "tiny_conv", "tiny_conv2", "tiny_conv3", "tiny_conv4"]

# The Frank-Wolfe steps pick vertices of the ReLU hulls; a rounding-level
# difference at a near-tie picks another vertex, and the iteration then moves on
# a slightly different path.  Same spread as the supergradient method's FP32 path.
FP32_FINAL_REL = 3e-3


def _case(msg):
    print(f"[case] {msg}", flush=True)


def _setup(name, **kw):
    import paper_2104_06718_amd as P
    inst = ldgen.make_instance(name, **kw)
    return P, inst, P.Net(inst.layers), P.Batch.from_instance(inst)


@pytest.mark.parametrize("name", SMALL + ["base"])
def test_first_iterations_follow_the_oracle(name):
    """From the CROWN point the first outer iterations track the oracle elementwise."""
    _case(f"prox first iterations {name}")
    P, inst, net, batch = _setup(name)
    onet = O.net_from_specs(inst.layers)
    ob = O.batch_from_instance(inst)
    for t in (1, 3):
        st = P.State(net, inst.B)
        P.prox_step(net, batch, st, iters=t, total_iters=20)
        rg = st.get_rho()
        torch.cuda.synchronize()
        assert st.prox_step_count() == t
        ost = O.proximal(onet, ob, O.ProxOpts(T=20), iters=t)
        tot = bad = 0
        for k in range(len(rg)):
            diff = (rg[k].cpu().double() - ost["rho"][k]).abs()
            bad += int((diff > 1e-4 * (ost["rho"][k].abs() + 1e-2)).sum())
            tot += diff.numel()
        print(f"  t={t}: duals differing beyond 1e-4 relative: {bad} of {tot}")
        assert bad <= 0.02 * tot


@pytest.mark.parametrize("name,T", [("fc_tiny", 300), ("tiny_conv", 100), ("tiny_conv2", 100),
                                    ("tiny_conv4", 100), ("base", 60)])
def test_final_bound_parity_fp32(name, T):
    _case(f"prox fp32 {name} T={T}")
    P, inst, net, batch = _setup(name)
    st = P.State(net, inst.B)
    P.prox_step(net, batch, st, iters=T, total_iters=T)
    fb = P.final_bound(net, batch, st)
    torch.cuda.synchronize()
    idx = list(range(min(inst.B, 8)))
    onet = O.net_from_specs(inst.layers)
    ob = O.batch_from_instance(inst, idx)
    ofb = O.final_bound(onet, ob, O.proximal(onet, ob, O.ProxOpts(T=T)))
    b_g = fb["bound"].cpu()[idx]
    d = (b_g - ofb["bound"]).abs()
    print(f"  final bound |gpu - oracle|: mean {d.mean().item():.2e} max {d.max().item():.2e}")
    assert bool((d <= FP32_FINAL_REL * ofb["bound"].abs() + 1e-3).all()), (b_g, ofb["bound"])
    # soundness: below the network value at a feasible point, never below q(rho^T)
    feas = fb["feasible"].cpu().bool()
    assert bool((fb["bound"].cpu()[feas] <= fb["primal"].cpu()[feas] + 1e-6).all())
    assert bool((fb["bound"].cpu() >= fb["q_final"].cpu() - 1e-12).all())


@pytest.mark.parametrize("name", ["tiny_conv", "base"])
def test_chunked_calls_equal_one_call(name):
    _case(f"prox chunked {name}")
    P, inst, net, batch = _setup(name)
    a = P.State(net, inst.B)
    P.prox_step(net, batch, a, iters=30, total_iters=30)
    b = P.State(net, inst.B)
    P.prox_step(net, batch, b, iters=11, total_iters=30)
    P.prox_step(net, batch, b, iters=19, total_iters=30)
    for x, y in zip(a.get_rho(), b.get_rho()):
        assert torch.equal(x, y)
    assert b.prox_step_count() == 30


@pytest.mark.parametrize("name", ["tiny_conv", "base"])
def test_bf16_is_sound_and_close(name):
    _case(f"prox bf16 {name}")
    P, inst, net, batch = _setup(name)
    res = {}
    for prec in ("fp32", "bf16"):
        st = P.State(net, inst.B)
        P.prox_step(net, batch, st, iters=60, total_iters=60, precision=prec)
        res[prec] = P.final_bound(net, batch, st)
    torch.cuda.synchronize()
    for prec in res:
        feas = res[prec]["feasible"].bool()
        assert bool((res[prec]["bound"][feas] <= res[prec]["primal"][feas] + 1e-6).all())
    gap = (res["bf16"]["bound"] - res["fp32"]["bound"]).abs()
    print(f"  bf16-fp32 gap mean {gap.mean().item():.3e} max {gap.max().item():.3e}")
    assert gap.mean().item() < 0.05 * res["fp32"]["bound"].abs().mean().item() + 1e-2


def test_method_of_multipliers_without_momentum():
    """mu = 0 and a fixed eta (the branch-and-bound setting of Sec. 7.3) against the oracle."""
    _case("prox mu=0 eta=100 tiny_conv2")
    P, inst, net, batch = _setup("tiny_conv2")
    st = P.State(net, inst.B)
    P.prox_step(net, batch, st, iters=40, total_iters=40, eta0=100.0, eta_end=100.0, mu=0.0)
    fb = P.final_bound(net, batch, st)
    torch.cuda.synchronize()
    onet = O.net_from_specs(inst.layers)
    ob = O.batch_from_instance(inst)
    ofb = O.final_bound(onet, ob, O.proximal(onet, ob, O.ProxOpts(T=40, eta0=100.0, eta_end=100.0, mu=0.0)))
    d = (fb["bound"].cpu() - ofb["bound"]).abs()
    print(f"  |gpu - oracle| max {d.max().item():.2e}")
    assert bool((d <= FP32_FINAL_REL * ofb["bound"].abs() + 1e-3).all())


def test_bad_options_are_rejected():
    _case("prox bad options")
    P, inst, net, batch = _setup("tiny_conv")
    st = P.State(net, inst.B)
    from paper_2104_06718_amd.binding import LDError
    for kw in (dict(eta0=0.0), dict(eta_end=-1.0), dict(mu=1.0), dict(inner_iters=0)):
        with pytest.raises(LDError):
            P.prox_step(net, batch, st, iters=1, total_iters=5, **kw)
    assert st.prox_step_count() == 0


def test_deep_net_first_iterations_follow_the_oracle():
    """Five hidden layers with 3x3 stride-1 and 4x4 stride-2 convs (two properties)."""
    _case("prox first iterations deep props=[2, 2]")
    P, inst, net, batch = _setup("deep", props=[2, 2])
    onet = O.net_from_specs(inst.layers)
    ob = O.batch_from_instance(inst)
    st = P.State(net, inst.B)
    P.prox_step(net, batch, st, iters=2, total_iters=20)
    rg = st.get_rho()
    torch.cuda.synchronize()
    ost = O.proximal(onet, ob, O.ProxOpts(T=20), iters=2)
    tot = bad = 0
    for k in range(len(rg)):
        diff = (rg[k].cpu().double() - ost["rho"][k]).abs()
        bad += int((diff > 1e-4 * (ost["rho"][k].abs() + 1e-2)).sum())
        tot += diff.numel()
    print(f"  duals differing beyond 1e-4 relative: {bad} of {tot}")
    assert bad <= 0.02 * tot
