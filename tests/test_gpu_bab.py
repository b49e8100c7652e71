"""The branch-and-bound driver (ld_bab) on the GPU, against the exact minimum of
small nets (the MILP of tests/_brute.py, itself pinned by pattern enumeration) and
the oracle's branch and bound (Sec. 2.3.1, Sec. 5.2, Sec. 7.3).

FP32 bounds are sound up to the rounding of their FP32 contractions (FP64 sums),
about 1e-6 of the terms here; the checks allow 1e-4."""
import math

import numpy as np
import pytest
import torch

import ldgen
from oracle import ld_oracle as O
from tests import _brute

pytestmark = pytest.mark.gpu
SLACK = 1e-4


def _case(msg):
    print(f"[case] {msg}", flush=True)


def _exact(inst, b):
    return _brute.milp_minimum(inst.layers, inst.l0[b].astype(float), inst.u0[b].astype(float),
                               [a[b].astype(float) for a in inst.l], [a[b].astype(float) for a in inst.u],
                               inst.c[b].astype(float))[0]


def _root(P, inst, b):
    return P.Batch.from_instance(inst.subset([b]))


@pytest.mark.parametrize("name", ["bab_fc", "bab_conv"])
def test_bab_verifies_below_and_never_above_the_minimum(name):
    import paper_2104_06718_amd as P
    inst = ldgen.make_instance(name, split_frac=0.0)
    net = P.Net(inst.layers)
    onet = O.net_from_specs(inst.layers)
    for b in range(inst.B):
        m = _exact(inst, b)
        root = _root(P, inst, b)
        _case(f"bab {name} property {b}: min {m:.5f}, threshold min - 0.05")
        r = P.bab(net, root, threshold=m - 0.05, batch=4, iters=200, max_rounds=400)
        ro = O.bab(onet, O.batch_from_instance(inst, [b]), O.BabOpts(threshold=m - 0.05, max_rounds=400, iters=200))
        print(f"  gpu {r['status']} lower {r['lower']:.5f} rounds {r['rounds']} bounded {r['bounded']}; "
              f"oracle {ro['status']} rounds {ro['rounds']} bounded {ro['bounded']}")
        assert r["status"] == "verified" == ro["status"]
        assert r["lower"] <= m + SLACK and r["incumbent"] >= m - SLACK
        _case(f"bab {name} property {b}: threshold min + 0.02")
        r = P.bab(net, root, threshold=m + 0.02, batch=4, iters=200, max_rounds=100)
        assert r["status"] != "verified"
        if r["status"] == "falsified":
            x = r["x_best"].double()
            ob = O.batch_from_instance(inst, [b])
            assert bool(((x >= ob.l0[0]) & (x <= ob.u0[0])).all())
            p, feas = O.primal_value(onet, ob, x[None, :])
            assert bool(feas[0]) and m - SLACK <= p[0].item() <= m + 0.02 + SLACK
            assert abs(p[0].item() - r["incumbent"]) <= SLACK


@pytest.mark.parametrize("name", ["bab_fc", "bab_conv"])
def test_bab_minimisation_brackets_the_minimum(name):
    import paper_2104_06718_amd as P
    inst = ldgen.make_instance(name, split_frac=0.0)
    net = P.Net(inst.layers)
    for b in range(inst.B):
        m = _exact(inst, b)
        _case(f"bab minimise {name} property {b}")
        r = P.bab(net, _root(P, inst, b), threshold=-math.inf, gap=1e-3, batch=4, iters=200, max_rounds=60)
        print(f"  [{r['lower']:.5f}, {r['incumbent']:.5f}] around {m:.5f}: {r['status']}, {r['leaves']} leaves")
        assert r["lower"] <= m + SLACK and m <= r["incumbent"] + SLACK


def test_bab_base_net_rounds_are_consistent():
    """The base conv net, minimising for 4 rounds of 32 splits: the lower bound never
    drops below the root's and never passes the incumbent, the count of bounded
    subproblems follows the splits, and the incumbent is the network's value at its
    input, which lies in the box."""
    import paper_2104_06718_amd as P
    inst = ldgen.make_instance("base", B=1, split_frac=0.0)
    net = P.Net(inst.layers)
    root = _root(P, inst, 0)
    _case("bab base root only")
    r0 = P.bab(net, root, threshold=-math.inf, batch=32, max_rounds=0)
    _case("bab base 4 rounds")
    r = P.bab(net, root, threshold=-math.inf, batch=32, max_rounds=4)
    print(f"  root lower {r0['lower']:.4f}; after {r['rounds']} rounds {r['lower']:.4f}, status {r['status']}, "
          f"bounded {r['bounded']}, open peak {r['max_open']}, incumbent {r['incumbent']:.4f}")
    assert r["rounds"] == 4
    assert r0["lower"] - 1e-9 <= r["lower"] <= r["incumbent"] + SLACK
    # the root, then two children for every split: 1, 2, 4 and 8 parents while fewer
    # than 32 are open and none is discarded or a leaf
    assert r["bounded"] % 2 == 1 and r["bounded"] <= 1 + 2 * (1 + 2 + 4 + 8)
    x = r["x_best"].double()
    ob = O.batch_from_instance(inst, [0])
    assert bool(((x >= ob.l0[0]) & (x <= ob.u0[0])).all())
    p, _ = O.primal_value(O.net_from_specs(inst.layers), ob, x[None, :])
    assert abs(p[0].item() - r["incumbent"]) <= 1e-3 * (1 + abs(r["incumbent"]))
    with pytest.raises(P.LDError) as e:
        P.bab(net, P.Batch.from_instance(inst.subset([0, 0])), threshold=0.0)
    assert e.value.code == P.LD_E_ARG
