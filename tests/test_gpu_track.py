"""The ascent keeping its best dual value (ld_state_set_tracking / ld_state_get_best)
through the C ABI.

* The first tracked step records q(rho^0): the same value as ld_dual_eval (FP32
  operands) at the CROWN duals, bitwise, and the oracle's within the FP32 bar.
* Over a stepped ascent the record is the largest of q(rho^0), ..., q(rho^{T-1}),
  each evaluated by ld_dual_eval after the step that produced it, with the step of
  its first occurrence; the duals are those of the same ascent without tracking.
* A BF16 ascent records FP32-operand values: its first tracked step equals
  ld_dual_eval's value at the BF16 run's CROWN duals; the record stays finite and in
  range; stopping it keeps the record.  The FP64 and resident engines refuse it."""
import numpy as np
import pytest
import torch

from oracle import ld_oracle as O
from tests import _parity as PT
from tests.test_gpu_parity import _case, _setup

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["fc_tiny", "tiny_conv", "tiny_conv3", "base"])
def test_first_tracked_step_records_q0(name):
    _case(f"tracking: first step {name}")
    P, inst, net, batch = _setup(name)
    st = P.State(net, inst.B)
    st.set_tracking(True)
    P.step(net, batch, st, iters=1, total_iters=50, precision="fp32", engine="layerwise")
    bq, bt = st.best()
    rho0 = P.init_duals(net, batch, "crown")
    q0, _ = P.dual_eval(net, batch, rho0, supergrad=False, precision="fp32")
    assert bool((bt == 1).all())
    assert torch.equal(bq, q0)
    onet = O.net_from_specs(inst.layers)
    ob = O.batch_from_instance(inst)
    orho = [r.cpu().double() for r in rho0]
    ev = O.dual_eval(onet, ob, orho, need_supergrad=False)
    assert bool(((bq.cpu() - ev["q"]).abs() <= PT.q_tol(onet, ob, orho, ev)).all())


@pytest.mark.parametrize("name", ["tiny_conv", "base"])
def test_record_is_the_largest_value_of_the_ascent(name):
    T = 30
    _case(f"tracking: {T} single steps {name}")
    P, inst, net, batch = _setup(name)
    st = P.State(net, inst.B)
    ref = P.State(net, inst.B)
    st.set_tracking(True)
    vals = []
    for t in range(1, T + 1):
        if t == 1:
            rho0 = P.init_duals(net, batch, "crown")
            vals.append(P.dual_eval(net, batch, rho0, supergrad=False, precision="fp32")[0].cpu())
        P.step(net, batch, st, iters=1, total_iters=T, precision="fp32", engine="layerwise")
        P.step(net, batch, ref, iters=1, total_iters=T, precision="fp32", engine="layerwise")
        if t < T:
            vals.append(P.dual_eval(net, batch, st.get_rho(), supergrad=False, precision="fp32")[0].cpu())
    bq, bt = st.best()
    V = torch.stack(vals)  # [T, B]: q(rho^0) .. q(rho^{T-1})
    want_q, want_i = V.max(dim=0)
    first = torch.tensor([int(np.argmax(V[:, b].numpy() == want_q[b].item())) for b in range(inst.B)])
    assert torch.equal(bq.cpu(), want_q)
    assert torch.equal(bt.cpu().long(), first + 1)
    print(f"  best step per subdomain: {sorted(set((first + 1).tolist()))}")
    for a, b in zip(st.get_rho(), ref.get_rho()):
        assert torch.equal(a, b)


def test_bf16_record_and_stop():
    _case("tracking: BF16 ascent, then stopped")
    P, inst, net, batch = _setup("base")
    st = P.State(net, inst.B)
    st.set_tracking(True)
    P.step(net, batch, st, iters=1, total_iters=80, precision="bf16", engine="auto")
    rho0 = P.init_duals(net, batch, "crown", precision="bf16")
    q0, _ = P.dual_eval(net, batch, rho0, supergrad=False, precision="fp32")
    bq, bt = st.best()
    assert torch.equal(bq, q0) and bool((bt == 1).all())
    P.step(net, batch, st, iters=39, total_iters=80, precision="bf16", engine="auto")
    bq, bt = st.best()
    assert bool(torch.isfinite(bq).all())
    assert bool(((bt >= 1) & (bt <= 40)).all())
    st.set_tracking(False)
    P.step(net, batch, st, iters=40, total_iters=80, precision="bf16", engine="auto")
    bq2, bt2 = st.best()
    assert torch.equal(bq, bq2) and torch.equal(bt, bt2)
    st.set_tracking(True)  # a fresh record
    bq3, bt3 = st.best()
    assert bool(torch.isinf(bq3).all()) and bool((bt3 == 0).all())


def test_tracking_refused_where_unsupported():
    _case("tracking: FP64 engine, resident engine, no record")
    P, inst, net, batch = _setup("tiny_conv")
    st = P.State(net, inst.B)
    with pytest.raises(P.LDError):
        st.best()
    st.set_tracking(True)
    with pytest.raises(P.LDError):
        P.step(net, batch, st, iters=2, total_iters=10, precision="fp64")
    with pytest.raises(P.LDError):
        P.step(net, batch, st, iters=2, total_iters=10, precision="fp32", engine="resident")
