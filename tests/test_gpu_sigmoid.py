"""Sigmoid inner minimisation (App. E) on the GPU against the FP64 oracle.

Both sides get the same FP32 inputs; the inner minimisation is compared with the
GPU's tangent points fed to the oracle, so the two steps are checked separately.
Every test prints the case before touching the GPU.
"""
import numpy as np
import pytest
import torch

from oracle import ld_oracle as O

pytestmark = pytest.mark.gpu


def _case(msg):
    print(f"[case] {msg}", flush=True)


def _inputs(n, seed):
    rng = np.random.default_rng(seed)
    a = rng.uniform(-6, 6, size=n)
    w = rng.choice([1e-3, 0.1, 1.0, 4.0], size=n) * rng.uniform(0.0, 1.0, size=n)
    l = a.astype(np.float32)
    u = (a + w).astype(np.float32)
    u = np.maximum(u, l)
    u[:5] = l[:5]                                   # degenerate intervals
    rho = (rng.normal(size=n) * rng.choice([0.0, 0.05, 0.3, 1.0], size=n)).astype(np.float32)
    g = (rng.normal(size=n) * rng.choice([0.0, 0.1, 1.0, 3.0], size=n)).astype(np.float32)
    return [torch.from_numpy(x) for x in (l, u, rho, g)]


@pytest.mark.parametrize("n", [0, 1, 257, 3 * 1024 + 7, 512 * 6244])
def test_hull_and_inner_min_match_the_oracle(n):
    import paper_2104_06718_amd as P
    _case(f"sigmoid n={n}")
    l, u, rho, g = _inputs(n, n)
    tu, tl = P.sigmoid_hull(l.cuda(), u.cuda())
    xb, x, val = P.sigmoid_inner_min(rho.cuda(), g.cuda(), l.cuda(), u.cuda(), tu, tl)
    torch.cuda.synchronize()
    if n == 0:
        return
    # the full-size case is checked on a sample the oracle computes one by one
    idx = torch.arange(n) if n < 100000 else torch.from_numpy(np.random.default_rng(1).choice(n, 20000, False))
    D = lambda t: t.double()[idx]  # noqa: E731
    otu, otl = O.sigmoid_hull(D(l), D(u))
    gtu, gtl = tu.cpu().double()[idx], tl.cpu().double()[idx]
    assert bool(((gtu - otu).abs() <= 1e-6 * (1 + otu.abs())).all()), (gtu - otu).abs().max().item()
    assert bool(((gtl - otl).abs() <= 1e-6 * (1 + otl.abs())).all()), (gtl - otl).abs().max().item()
    oxb, ox, ov = O.inner_min_sigmoid(D(rho), D(g), D(l), D(u), gtu, gtl)
    gv = val.cpu()[idx]
    scale = 1 + D(rho).abs() * (D(l).abs() + D(u).abs()) + D(g).abs()
    assert bool(((gv - ov).abs() <= 1e-10 * scale).all()), (gv - ov).abs().max().item()
    # the GPU's minimiser attains the value (it differs from the oracle's only at ties)
    gxb, gx = xb.cpu().double()[idx], x.cpu().double()[idx]
    same = int((gxb == oxb.float().double()).sum())
    print(f"  minimisers equal to the oracle's: {same} of {len(idx)}")
    att = D(rho) * gxb - D(g) * gx
    assert bool(((att - ov).abs() <= 1e-6 * scale).all()), (att - ov).abs().max().item()
    assert bool(((gxb >= D(l)) & (gxb <= D(u))).all())


def test_bad_arguments():
    import paper_2104_06718_amd as P
    _case("sigmoid bad arguments")
    lib = P.load_library()
    assert lib.ld_sigmoid_hull(-1, None, None, None, None, None) == -1
    assert lib.ld_sigmoid_inner_min(4, None, None, None, None, None, None, None, None, None, None) == -1
