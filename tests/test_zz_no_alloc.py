"""The allocation-free dual evaluation (ld_dual_eval_noalloc) against ld_dual_eval,
through the C ABI: q within 1e-5 of its magnitude sum and the supergradient within
1e-5 of its scale away from near-ties (the fixed-dual bar), on two calls in a row,
the second with a smaller batch, and a batch too large for the scratch array
refused.  The two entry points may differ in the summation order of split
fully-connected products only."""
import numpy as np
import pytest
import torch

import ldgen
from oracle import ld_oracle as O
from tests import _parity as PT

pytestmark = pytest.mark.gpu


def _case(msg):
    print(f"[case] {msg}", flush=True)


def _compare(P, net, inst, batch, rho32, precision):
    rho = [torch.from_numpy(r).cuda() for r in rho32]
    q_ref, s_ref = P.dual_eval(net, batch, rho, supergrad=True, precision=precision)
    q = torch.full((inst.B,), float("nan"), device="cuda", dtype=torch.float64)
    s = [torch.full_like(r, float("nan")) for r in rho]
    P.dual_eval_noalloc(net, batch, rho, q, s, precision=precision)
    torch.cuda.synchronize()
    onet, ob = O.net_from_specs(inst.layers), O.batch_from_instance(inst)
    orho = [torch.from_numpy(r).double() for r in rho32]
    ev = O.dual_eval(onet, ob, orho)
    rel = 1e-5 if precision == "fp32" else 2.0 ** -7
    S = O.q_scale(onet, ob, orho, ev)
    d = (q.cpu() - q_ref.cpu()).abs()
    print(f"  q: max |noalloc - ld_dual_eval| / S = {(d / S).max().item():.2e}")
    assert bool((d <= rel * S + 1e-9).all())
    masks = PT.supergrad_masks(onet, PT.unstable_decisions(onet, ob, orho, ev, tie_rel=2 * rel))
    scale = PT.s_scale(onet, ev)
    for k in range(len(s)):
        dk = (s[k].cpu().double() - s_ref[k].cpu().double()).abs()
        bad = (dk > rel * scale[k] + 1e-7) & ~masks[k]
        assert not bool(bad.any()), (k, int(bad.sum()))


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_noalloc_matches_dual_eval_twice_then_smaller(precision):
    import paper_2104_06718_amd as P
    inst = ldgen.make_instance("base")
    net = P.Net(inst.layers)
    small = inst.subset([5, 17, 40])
    for it, (name, sub) in enumerate((("base B=64", inst), ("base B=3", small))):
        _case(f"noalloc {precision} call {it + 1}: {name}")
        _compare(P, net, sub, P.Batch.from_instance(sub), ldgen.random_duals(sub, seed=41 + it, scale=0.3), precision)


def test_noalloc_small_net_and_refusal():
    import paper_2104_06718_amd as P
    inst = ldgen.make_instance("tiny_conv2")
    net = P.Net(inst.layers)
    _case("noalloc tiny_conv2")
    _compare(P, net, inst, P.Batch.from_instance(inst), ldgen.random_duals(inst, seed=3, scale=0.3), "fp32")
    wide = ldgen.make_instance("wide", B=512)
    wnet = P.Net(wide.layers)
    _case("noalloc wide B=512 (needs more than the scratch)")
    wb = P.Batch.from_instance(wide)
    q = torch.empty(512, device="cuda", dtype=torch.float64)
    with pytest.raises(P.LDError) as e:
        P.dual_eval_noalloc(wnet, wb, [torch.zeros_like(t) for t in wb.l], q)
    assert e.value.code == P.LD_E_NOMEM and "bytes of scratch" in str(e.value)
