"""Pins of the oracle's intermediate bounds (Sec. 2.2.3): LD on the sub-network
ending at layer j with the objectives +-x_j[i].

Soundness against the true pre-activations of sampled inputs (weak duality,
Sec. 3.1) and, per neuron, against the Planet LP optimum of the sub-network
(Prop. 1, HiGHS).
"""
import types

import numpy as np
import pytest
import torch

import ldgen
from oracle import ld_oracle as O
from tests.test_oracle_pins import _planet_lp


def _setup(name, **kw):
    inst = ldgen.make_instance(name, **kw)
    return inst, O.net_from_specs(inst.layers), O.batch_from_instance(inst)


def _preacts(net, x, j):
    """x_j = W_j relu(...) + b_j of the true network."""
    for k in range(j - 1):
        x = torch.clamp(net[k].forward(x), min=0.0)
    return net[j - 1].forward(x)


@pytest.mark.parametrize("name,j", [("fc_tiny", 2), ("tiny_conv", 2), ("tiny_conv", 3), ("tiny_conv3", 2)])
def test_bounds_contain_sampled_preactivations(name, j):
    inst, net, batch = _setup(name, split_frac=0.0)
    lo, hi = O.intermediate_bounds(net, batch, j, O.AdamOpts(T=100))
    assert bool((lo <= hi + 1e-12).all())
    g = torch.Generator().manual_seed(7)
    for b in range(inst.B):
        l0, u0 = batch.l0[b], batch.u0[b]
        X = l0 + (u0 - l0) * torch.rand(4000, l0.numel(), generator=g, dtype=torch.float64)
        X = torch.cat([X, torch.where(torch.rand(500, l0.numel(), generator=g) < 0.5, l0, u0)])
        Y = _preacts(net, X, j)
        assert bool((Y >= lo[b] - 1e-9).all()) and bool((Y <= hi[b] + 1e-9).all())


@pytest.mark.parametrize("name,j", [("fc_tiny", 2), ("tiny_conv3", 2)])
def test_bounds_below_the_lp_optimum_and_close_to_it(name, j):
    """Prop. 1 per neuron: LD's bound never passes the Planet LP optimum of the
    sub-network, and 1500 steps close most of the gap from the CROWN start."""
    inst, net, batch = _setup(name, split_frac=0.0)
    b = 0
    sub = inst.layers[:j]
    n_j = sub[-1].n_out
    one = O.OBatch(batch.l0[:1], batch.u0[:1], [x[:1] for x in batch.l], [x[:1] for x in batch.u], batch.c[:1])
    lo, hi = O.intermediate_bounds(net, one, j, O.AdamOpts(T=1500, lr0=1e-2, lr_end=1e-5))
    crown = O.intermediate_bounds(net, one, j, O.AdamOpts(T=0))
    for i in range(min(n_j, 8)):
        for sgn in (1.0, -1.0):
            c = np.zeros((1, n_j))
            c[0, i] = sgn
            fake = types.SimpleNamespace(layers=sub, l0=inst.l0[b:b + 1], u0=inst.u0[b:b + 1],
                                         l=[a[b:b + 1] for a in inst.l[:j - 1]],
                                         u=[a[b:b + 1] for a in inst.u[:j - 1]], c=c)
            p = _planet_lp(fake, 0)
            got = lo[0, i].item() if sgn > 0 else -hi[0, i].item()
            start = crown[0][0, i].item() if sgn > 0 else -crown[1][0, i].item()
            assert got <= p + 1e-9, (i, sgn, got, p)
            assert start <= got + 1e-12
            assert p - got <= 0.2 * (p - start) + 1e-4, (i, sgn, got, p, start)


def test_neuron_batch_layout():
    inst, net, batch = _setup("tiny_conv")
    eb = O.neuron_batch(batch, 2, 36)
    assert eb.c.shape == (inst.B * 72, 36)
    # problem (b=1, i=5, s=1) sits at 1*72 + 2*5 + 1 and carries -e_5 and subdomain 1's box
    p = 72 + 11
    assert eb.c[p, 5] == -1.0 and eb.c[p].abs().sum() == 1.0
    assert torch.equal(eb.l0[p], batch.l0[1]) and torch.equal(eb.u[0][p], batch.u[0][1])
    assert len(eb.l) == 1
