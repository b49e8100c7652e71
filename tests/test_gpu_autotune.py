"""The autotuner: every candidate launch configuration computes the same dual
(checked against the FP64 oracle), and a tuned AUTO ascent matches the oracle."""
import pytest
import torch

import ldgen
from oracle import ld_oracle as O
from tests.test_gpu_parity import _case, _check_dual_eval, _oracle_fp32_spread, _oracle_run, _setup

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["base", "tiny_conv2", "tiny_conv3", "tiny_conv4", "tiny_conv5"])
def test_every_candidate_configuration_matches_oracle(name):
    P, inst, net, batch = _setup(name)
    rho = ldgen.random_duals(inst, seed=17, scale=0.3)
    n_layers = len(inst.layers)
    tried = 0
    for prec in ("fp32", "bf16"):
        for k in range(1, n_layers):
            for d in ("transposed", "forward"):
                for tile in P.tile_candidates(net, inst.B, k, d):
                    _case(f"candidate {name} {prec} layer {k} {d} {tile}")
                    P.set_tuned_config(net, inst.B, prec, k, d, tile)
                    if prec == "fp32":
                        _check_dual_eval(P, inst, net, batch, rho)
                    else:
                        # BF16 operands only enter the ascent; the dual value itself is
                        # evaluated with FP32 operands unless asked otherwise
                        q32, _ = P.dual_eval(net, batch, [torch.from_numpy(r).cuda() for r in rho],
                                             supergrad=False, precision="fp32")
                        q16, _ = P.dual_eval(net, batch, [torch.from_numpy(r).cuda() for r in rho],
                                             supergrad=False, precision="bf16")
                        onet = O.net_from_specs(inst.layers)
                        ob = O.batch_from_instance(inst)
                        orho = [torch.from_numpy(r).double() for r in rho]
                        ev = O.dual_eval(onet, ob, orho, need_supergrad=False)
                        S = O.q_scale(onet, ob, orho, ev)
                        assert bool(((q16.cpu() - ev["q"]).abs() <= 2.0 ** -7 * S).all())
                        assert bool(((q32.cpu() - ev["q"]).abs() <= 1e-5 * S + 1e-9).all())
                    tried += 1
    print(f"  {tried} configurations checked")
    assert tried > 0


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_autotuned_auto_ascent(prec):
    _case(f"autotune base {prec}")
    P, inst, net, batch = _setup("base")
    info = P.autotune(net, batch, total_iters=100, precision=prec)
    print(f"  engine {info['engine']}, us/iter layerwise {info['us_per_iter_layerwise']:.1f} "
          f"resident {info['us_per_iter_resident']:.1f}")
    for e in info["layers"]:
        tile = {f: e[f] for f in ("tn", "mwaves", "kwaves", "splits", "form")}
        print(f"  layer {e['layer']} {e['dir']}: {tile} {e['us']:.1f} us")
        assert tile in P.tile_candidates(net, inst.B, e["layer"], e["dir"])
        assert e["us"] > 0
    assert info["engine"] in ("layerwise", "resident")
    assert len(info["layers"]) == 2 * (len(inst.layers) - 1)
    T = 100
    st = P.State(net, inst.B)
    P.step(net, batch, st, iters=T, total_iters=T, precision=prec, engine="auto")
    fb = P.final_bound(net, batch, st)
    torch.cuda.synchronize()
    feas = fb["feasible"].cpu().bool()
    assert bool((fb["bound"].cpu()[feas] <= fb["primal"].cpu()[feas] + 1e-6).all())
    if prec == "fp32":
        idx = list(range(8))
        ofb, _ = _oracle_run(inst, idx, T)
        d = (fb["bound"].cpu()[idx] - ofb["bound"]).abs()
        ref = _oracle_fp32_spread(inst, idx, T, ofb["bound"])
        print(f"  |gpu - oracle| max {d.max().item():.2e}; oracle in float32: max {ref.max().item():.2e}")
        assert d.mean().item() <= 2 * ref.mean().item() + 1e-4
        assert d.max().item() <= 2 * ref.max().item() + 1e-3
