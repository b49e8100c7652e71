"""Pins of the oracle's rounding margin (oracle.ld_oracle.rounding_margin): the
bound on how far a dual value whose coefficients W_k^T rho_k are formed with
single-precision products can sit above the exact q(rho).

* the magnitudes |W|^T |r| of a conv layer equal the product with the absolute
  dense matrix of the layer (built column by column from the forward map);
* a hand-worked fully connected net gives the margin written out below;
* on small nets and several dual scales, the margin covers the actual error of
  coefficients computed by torch in float32 (every other term in float64)."""
import numpy as np
import pytest
import torch

import ldgen
from oracle import ld_oracle as O

U = 2.0 ** -24


def _dense(L):
    """Dense matrix [n_out, n_in] of the layer's linear part, one column per unit input."""
    n_in = int(np.prod(L.in_shape))
    eye = torch.eye(n_in, dtype=torch.float64)
    return (L.forward(eye) - L.bias_full()).T


@pytest.mark.parametrize("name", ["tiny_conv", "tiny_conv3", "tiny_conv5", "base"])
def test_abs_layer_matches_absolute_dense_matrix(name):
    inst = ldgen.make_instance(name)
    net = O.net_from_specs(inst.layers)
    g = torch.Generator().manual_seed(3)
    for L in net:
        if L.kind != "conv":
            continue
        D = _dense(L)
        r = torch.randn(2, D.shape[0], generator=g, dtype=torch.float64)
        got = O.abs_layer(L).transposed(r.abs())
        want = r.abs() @ D.abs()
        assert torch.allclose(got, want, rtol=1e-12, atol=1e-12)
        # every entry of the dense matrix is one weight (or zero): |D| is the dense
        # matrix of |W|, and the term count bounds each column's nonzeros
        assert int((D != 0).sum(dim=0).max()) <= O.dot_terms(L)


def test_hand_worked_fc_net():
    # FC 2-2-1: W1 = [[1, 2], [3, -4]], W2 = [[1, -1]], c = [1]; box x0 in [-1, 2] x [0, 1];
    # hidden bounds [-1, 3] and [-2, 5]; rho_1 = [0.5, -0.25]
    W1 = torch.tensor([[1.0, 2.0], [3.0, -4.0]], dtype=torch.float64)
    W2 = torch.tensor([[1.0, -1.0]], dtype=torch.float64)
    net = [O.OLayer("linear", W1, torch.zeros(2, dtype=torch.float64), (2, 1, 1), (2, 1, 1)),
           O.OLayer("linear", W2, torch.zeros(1, dtype=torch.float64), (2, 1, 1), (1, 1, 1))]
    t = lambda v: torch.tensor([v], dtype=torch.float64)  # noqa: E731
    batch = O.OBatch(t([-1.0, 0.0]), t([2.0, 1.0]), [t([-1.0, -2.0])], [t([3.0, 5.0])], t([1.0]))
    rho = [t([0.5, -0.25])]
    # layer 1: K = 2 terms; |W1|^T |rho_1| = [1*0.5 + 3*0.25, 2*0.5 + 4*0.25] = [1.25, 2];
    #          max |x0| = [2, 1]  ->  gamma_2 * (1.25*2 + 2*1) = 4.5 gamma_2
    # layer 2: K = 1 term;  |W2|^T |c| = [1, 1];  max(0, u_1) = [3, 5]  ->  8 gamma_1
    # subnormals: 2*2*2^-126 * (2 + 1) + 2*1*2^-126 * (3 + 5) = 28 * 2^-126
    g1 = U / (1 - U)
    g2 = 2 * U / (1 - 2 * U)
    want = 4.5 * g2 + 8.0 * g1 + 28.0 * 2.0 ** -126
    got = O.rounding_margin(net, batch, rho)
    assert got.shape == (1,)
    assert abs(got.item() - want) <= 1e-15 * want


def _q_from_coefficients(net, batch, rho, g):
    """q at rho with the coefficients g[k] = W_{k+1}^T rho_{k+1} given (k = 0..n-1)."""
    n = len(net)
    duals = list(rho) + [-batch.c]
    _, v0 = O.inner_min_p0(g[0], batch.l0, batch.u0)
    q = v0.clone()
    for k in range(1, n):
        _, _, val = O.inner_min_pk(duals[k - 1], g[k], batch.l[k - 1], batch.u[k - 1], 0.0)
        q = q + val.sum(dim=1)
    for k in range(1, n + 1):
        q = q - (duals[k - 1] * net[k - 1].bias_full()).sum(dim=1)
    return q


def _f32_layer(L):
    return O.OLayer(L.kind, L.W.float(), L.b.float(), L.in_shape, L.out_shape, L.stride, L.pad)


@pytest.mark.parametrize("name", ["fc_tiny", "tiny_conv", "tiny_conv3", "tiny_conv5", "base"])
def test_margin_covers_single_precision_coefficients(name):
    inst = ldgen.make_instance(name)
    net = O.net_from_specs(inst.layers)
    batch = O.batch_from_instance(inst)
    cases = [[torch.from_numpy(r).double() for r in ldgen.random_duals(inst, seed=s, scale=sc)]
             for s, sc in ((5, 1e-2), (6, 1.0), (7, 1e2))]
    cases.append([r.float().double() for r in O.crown_init(net, batch)])
    worst = 0.0
    for rho in cases:
        ev = O.dual_eval(net, batch, rho, tau=0.0, need_supergrad=False)
        duals = list(rho) + [-batch.c]
        g32 = [_f32_layer(net[k]).transposed(duals[k].float()).double() for k in range(len(net))]
        q32 = _q_from_coefficients(net, batch, rho, g32)
        m = O.rounding_margin(net, batch, rho)
        err = (q32 - ev["q"]).abs()
        assert bool((err <= m).all()), f"error {err.max().item():.3e} above margin {m.min().item():.3e}"
        # the margin is a small share of the dual value's terms
        assert bool((m <= 1e-4 * O.q_scale(net, batch, rho, ev)).all())
        worst = max(worst, float((err / m).max()))
    print(f"  largest error / margin: {worst:.3f}")
