"""Pins of the oracle's sigmoid inner minimisation (App. E): the hull envelopes
against a monotone-chain convex hull of densely sampled points of the curve, the
minimum against a dense search over that brute-force hull, and weak duality
against points on the curve.  Nothing here uses the tangency condition.
"""
import numpy as np
import pytest
import torch

from oracle import ld_oracle as O


def _sig(x):
    return 1.0 / (1.0 + np.exp(-x))


def _hull_chain(xs, ys, upper):
    """Upper (or lower) hull of points sorted by x (monotone chain)."""
    h = []
    for p in zip(xs, ys):
        while len(h) >= 2:
            (x1, y1), (x2, y2) = h[-2], h[-1]
            cross = (x2 - x1) * (p[1] - y1) - (y2 - y1) * (p[0] - x1)
            if (upper and cross >= 0) or (not upper and cross <= 0):
                h.pop()
            else:
                break
        h.append(p)
    hx, hy = np.array([q[0] for q in h]), np.array([q[1] for q in h])
    return lambda x: np.interp(x, hx, hy)


def _cases():
    rng = np.random.default_rng(11)
    ls, us = [], []
    for _ in range(60):
        a, b = np.sort(rng.uniform(-6, 6, size=2))
        if b - a < 1e-3:
            b = a + 0.5
        ls.append(a)
        us.append(b)
    # fixed shapes: convex region only, concave only, straddling, nearly symmetric
    for a, b in ((-5, -1), (0.5, 4), (-3, 2), (-2, 2.5), (-0.2, 0.1), (-1e-3, 1e-3)):
        ls.append(a)
        us.append(b)
    return np.array(ls), np.array(us)


def test_envelopes_match_the_sampled_hull():
    L, U = _cases()
    tu, tl = O.sigmoid_hull(torch.tensor(L), torch.tensor(U))
    for j, (l, u) in enumerate(zip(L, U)):
        xs = np.linspace(l, u, 20001)
        ys = _sig(xs)
        up = _hull_chain(xs, ys, upper=True)
        lo = _hull_chain(xs, ys, upper=False)
        xt = torch.tensor(xs)
        lj, uj = torch.full_like(xt, l), torch.full_like(xt, u)
        phi = O.sigmoid_upper(xt, lj, uj, torch.full_like(xt, tu[j].item())).numpy()
        psi = O.sigmoid_lower(xt, lj, uj, torch.full_like(xt, tl[j].item())).numpy()
        assert np.max(np.abs(phi - up(xs))) <= 1e-7, (l, u)
        assert np.max(np.abs(psi - lo(xs))) <= 1e-7, (l, u)


def test_tangent_points_in_the_closed_form_cases():
    L = torch.tensor([0.5, 0.0, -4.0, -1.0], dtype=torch.float64)
    U = torch.tensor([3.0, 2.0, -1.0, 0.0], dtype=torch.float64)
    tu, tl = O.sigmoid_hull(L, U)
    # sigma concave on [l, u] with l >= 0: phi = sigma from l on
    assert tu[0] == L[0] and tu[1] == L[1]
    # sigma convex on [l, u] with u <= 0: psi = sigma up to u
    assert tl[2] == U[2] and tl[3] == U[3]


@pytest.mark.parametrize("seed", [0, 1])
def test_inner_min_matches_a_dense_search_over_the_hull(seed):
    rng = np.random.default_rng(seed)
    L, U = _cases()
    n = len(L)
    rho = rng.normal(size=n) * rng.choice([0.05, 0.3, 1.0], size=n)
    g = rng.normal(size=n) * rng.choice([0.1, 1.0, 3.0], size=n)
    g[:3] = 0.0
    T = lambda a: torch.tensor(a, dtype=torch.float64)  # noqa: E731
    tu, tl = O.sigmoid_hull(T(L), T(U))
    xb, x, val = O.inner_min_sigmoid(T(rho), T(g), T(L), T(U), tu, tl)
    for j in range(n):
        xs = np.linspace(L[j], U[j], 10001)
        ys = _sig(xs)
        env = _hull_chain(xs, ys, upper=g[j] > 0)(xs)
        brute = np.min(rho[j] * xs - g[j] * env)
        v = val[j].item()
        assert v <= brute + 1e-9, (j, v, brute)
        assert v >= brute - 1e-6 * (1 + abs(rho[j]) + abs(g[j])), (j, v, brute)
        # the minimiser lies in the hull and attains the value
        lo = _hull_chain(xs, ys, upper=False)(xb[j].item())
        hi = _hull_chain(xs, ys, upper=True)(xb[j].item())
        assert lo - 1e-7 <= x[j].item() <= hi + 1e-7
        assert abs(rho[j] * xb[j].item() - g[j] * x[j].item() - v) <= 1e-12 * (1 + abs(v))
        # weak duality: points on the curve are in the hull
        assert v <= np.min(rho[j] * xs - g[j] * ys) + 1e-12
