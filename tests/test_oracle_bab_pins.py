"""Pins of the oracle's branch and bound (Sec. 2.3.1, Sec. 5.2, Sec. 7.3) against the
exact minimum of c^T f over the input box, on nets small enough to enumerate:

* the exact minimum from one LP per sign pattern of the ambiguous ReLUs (scipy
  HiGHS) equals the big-M mixed-integer program's (so the MILP can stand in on the
  larger net);
* a threshold below the minimum is verified (the bounds close the gap), and the
  returned lower bound never passes the minimum;
* a threshold above it is never verified; a falsification comes with an input of
  the box, inside every intermediate bound, whose network value is at or below it;
* minimisation brackets the minimum between its lower bound and its incumbent.
Planted mistakes (pruning on the wrong side of the threshold; a child's bound taken
0.1 above its value) each fail at least two of these tests.
"""
import math

import numpy as np
import pytest
import torch

import ldgen
from oracle import ld_oracle as O
from tests import _brute


def _exact(inst, b, how="milp"):
    args = (inst.layers, inst.l0[b].astype(float), inst.u0[b].astype(float), [a[b].astype(float) for a in inst.l],
            [a[b].astype(float) for a in inst.u], inst.c[b].astype(float))
    return _brute.enumerate_minimum(*args)[0] if how == "enum" else _brute.milp_minimum(*args)[0]


def test_milp_matches_pattern_enumeration():
    inst = ldgen.make_instance("bab_fc", split_frac=0.0)
    for b in range(inst.B):
        assert abs(_exact(inst, b, "enum") - _exact(inst, b)) <= 1e-9
    # a subdomain with splits (its bounds are constraints too)
    inst = ldgen.make_instance("bab_conv", split_frac=0.3)
    for b in range(inst.B):
        e, m = _exact(inst, b, "enum"), _exact(inst, b)
        assert (math.isinf(e) and math.isinf(m)) or abs(e - m) <= 1e-9


@pytest.mark.parametrize("name", ["bab_fc", "bab_conv"])
def test_bab_verifies_below_and_never_above_the_minimum(name):
    inst = ldgen.make_instance(name, split_frac=0.0)
    onet = O.net_from_specs(inst.layers)
    for b in range(inst.B):
        m = _exact(inst, b)
        ob = O.batch_from_instance(inst, [b])
        r = O.bab(onet, ob, O.BabOpts(threshold=m - 0.05, max_rounds=400, iters=200))
        assert r["status"] == "verified", (b, m, r["status"], r["lower"])
        assert r["lower"] <= m + 1e-9 and r["incumbent"] >= m - 1e-9
        r = O.bab(onet, ob, O.BabOpts(threshold=m + 0.02, max_rounds=100, iters=200))
        assert r["status"] != "verified"
        if r["status"] == "falsified":
            x = r["x_best"]
            assert bool(((x >= ob.l0[0]) & (x <= ob.u0[0])).all())
            p, feas = O.primal_value(onet, ob, x[None, :])
            assert bool(feas[0]) and p[0].item() <= m + 0.02 + 1e-12 and p[0].item() >= m - 1e-9


@pytest.mark.parametrize("name", ["bab_fc", "bab_conv"])
def test_bab_minimisation_brackets_the_minimum(name):
    inst = ldgen.make_instance(name, split_frac=0.0)
    onet = O.net_from_specs(inst.layers)
    for b in range(inst.B):
        m = _exact(inst, b)
        r = O.bab(onet, O.batch_from_instance(inst, [b]), O.BabOpts(threshold=-math.inf, gap=1e-3, max_rounds=60, iters=200))
        assert r["lower"] <= m + 1e-9 <= r["incumbent"] + 2e-9, (b, r["lower"], m, r["incumbent"])
