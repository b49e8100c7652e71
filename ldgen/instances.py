"""Seeded instance generator (inputs only; see the package docstring).

Workload recipe (all draws from one ``numpy.random.Generator(PCG64(seed))`` per
configuration, in this fixed order):

1. weights  W_k ~ N(0, 2/fan_in)  (fan_in = C_in*kh*kw for conv, n_in for FC);
2. biases   b_k ~ N(0, 0.1)       (0.1 is the variance);
3. for each property, in order: centre x0 ~ U[0,1]^{n_0}; objective pair (t, j)
   (distinct, uniform in 0..n_out-1; c = e_t - e_j, or c = (1, -1) when the
   network has two outputs); then that property's subdomain splits.

The input box is [x0 - eps, x0 + eps] rounded outward to float32 (no clipping).  Intermediate bounds are
interval bounds propagated from the root box in float64 and rounded outward to
float32.  Each subdomain draws round(0.05 * A) distinct neurons from the A
root-ambiguous ReLUs of its property and fixes each one active (lower bound set
to 0) or inactive (upper bound set to 0) with probability 1/2, without
re-propagating bounds.  Conv layers use (C, H, W) flattening.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

BASE_SEED = 2104067180


@dataclasses.dataclass
class LayerSpec:
    kind: str                      # "linear" or "conv"
    W: np.ndarray                  # float32; linear [out, in], conv [Co, Ci, kh, kw]
    b: np.ndarray                  # float32 [out] (conv: [Co], broadcast over H*W)
    in_shape: Tuple[int, int, int]   # (C, H, W); linear: (n_in, 1, 1)
    out_shape: Tuple[int, int, int]  # (C, H, W); linear: (n_out, 1, 1)
    stride: int = 1
    pad: int = 0

    @property
    def n_in(self) -> int:
        return int(np.prod(self.in_shape))

    @property
    def n_out(self) -> int:
        return int(np.prod(self.out_shape))


@dataclasses.dataclass
class Instance:
    name: str
    layers: List[LayerSpec]
    l0: np.ndarray                 # [B, n0] float32
    u0: np.ndarray                 # [B, n0] float32
    l: List[np.ndarray]            # hidden layers 1..n-1, each [B, n_k] float32
    u: List[np.ndarray]
    c: np.ndarray                  # [B, n_out] float32
    prop: np.ndarray               # [B] int32, property index of each subdomain
    meta: Dict

    @property
    def B(self) -> int:
        return int(self.l0.shape[0])

    @property
    def n_layers(self) -> int:
        return len(self.layers)

    def subset(self, idx: Sequence[int]) -> "Instance":
        idx = np.asarray(idx, dtype=np.int64)
        return Instance(self.name, self.layers, self.l0[idx].copy(), self.u0[idx].copy(),
                        [a[idx].copy() for a in self.l], [a[idx].copy() for a in self.u],
                        self.c[idx].copy(), self.prop[idx].copy(), dict(self.meta))


# ----------------------------------------------------------------------------
# configurations (shapes follow the paper's OVAL networks, Sec. 8.1, table tab:oval-nets)
# ----------------------------------------------------------------------------
def _conv(ci, co, k, s, p, hw):
    ho = (hw + 2 * p - k) // s + 1
    return ("conv", ci, co, k, s, p, hw, ho)


CONFIGS: Dict[str, Dict] = {
    # 10-32-32-2 fully connected, box +-0.1, one subdomain, objective y0 - y1
    "fc_tiny": dict(cfg=1, input=(10, 1, 1), eps=0.1, B=1, props=[1], T=500,
                    arch=[("linear", 10, 32), ("linear", 32, 32), ("linear", 32, 2)]),
    # OVAL "Base": conv 8@4x4/2, conv 16@4x4/2, FC 100, FC 10
    "base": dict(cfg=2, input=(3, 32, 32), eps=2.0 / 255, B=64, props=[64], T=500,
                 arch=[_conv(3, 8, 4, 2, 1, 32), _conv(8, 16, 4, 2, 1, 16),
                       ("linear", 1024, 100), ("linear", 100, 10)]),
    # OVAL "Wide": conv 16@4x4/2, conv 32@4x4/2, FC 100, FC 10
    "wide": dict(cfg=3, input=(3, 32, 32), eps=2.0 / 255, B=512, props=[512], T=500,
                 arch=[_conv(3, 16, 4, 2, 1, 32), _conv(16, 32, 4, 2, 1, 16),
                       ("linear", 2048, 100), ("linear", 100, 10)]),
    # deep conv net, layer order conv 8@3x3/1, 8@4x4/2, 8@3x3/1, 8@4x4/2, FC 100, FC 10;
    # six properties of uneven subdomain counts concatenated along the batch
    "deep": dict(cfg=4, input=(3, 32, 32), eps=2.0 / 255, B=4044,
                 props=[37, 150, 600, 1200, 9, 2048], T=300,
                 arch=[_conv(3, 8, 3, 1, 1, 32), _conv(8, 8, 4, 2, 1, 32),
                       _conv(8, 8, 3, 1, 1, 16), _conv(8, 8, 4, 2, 1, 16),
                       ("linear", 512, 100), ("linear", 100, 10)]),
    # small shapes with odd sizes and ragged tails, used only by the test-suite
    "tiny_conv": dict(cfg=6, input=(2, 6, 6), eps=0.1, B=4, props=[4], T=200,
                      arch=[_conv(2, 3, 4, 2, 1, 6), _conv(3, 4, 3, 1, 1, 3),
                            ("linear", 36, 8), ("linear", 8, 3)]),
    "tiny_conv2": dict(cfg=7, input=(3, 7, 7), eps=0.05, B=3, props=[2, 1], T=200,
                       arch=[_conv(3, 5, 3, 2, 1, 7), _conv(5, 6, 3, 1, 1, 4),
                             _conv(6, 4, 4, 2, 1, 4), ("linear", 16, 7), ("linear", 7, 4)]),
    # transposed strided convs with one tap per row (2x2/2) and three (5x5/2)
    "tiny_conv3": dict(cfg=8, input=(2, 8, 8), eps=0.1, B=5, props=[3, 2], T=200,
                       arch=[_conv(2, 3, 5, 2, 2, 8), _conv(3, 4, 2, 2, 0, 4),
                             ("linear", 16, 6), ("linear", 6, 3)]),
    # channel counts that are multiples of 8 (channel-last gather) on odd map sizes
    "tiny_conv4": dict(cfg=9, input=(8, 5, 5), eps=0.1, B=6, props=[4, 2], T=200,
                       arch=[_conv(8, 8, 3, 1, 1, 5), _conv(8, 16, 4, 2, 1, 5),
                             ("linear", 64, 6), ("linear", 6, 3)]),
    # a transposed strided conv whose operand staging takes several rounds (36 channels,
    # ragged in the BF16 and FP32 K groups, on an 11x11 map: 121 positions)
    "tiny_conv5": dict(cfg=10, input=(2, 22, 22), eps=0.05, B=3, props=[2, 1], T=100,
                       arch=[_conv(2, 36, 4, 2, 1, 22), ("linear", 4356, 8), ("linear", 8, 3)]),
    # small nets whose exact minimum is enumerable (branch-and-bound pins): FC 6-12-8-2
    # (12 root-ambiguous ReLUs) and conv 1->2 3x3/2 on 6x6, FC 6, FC 2 (8 of them);
    # three properties each, objective y0 - y1
    "bab_fc": dict(cfg=11, input=(6, 1, 1), eps=0.15, B=3, props=[1, 1, 1], T=100,
                   arch=[("linear", 6, 12), ("linear", 12, 8), ("linear", 8, 2)]),
    "bab_conv": dict(cfg=12, input=(1, 6, 6), eps=0.1, B=3, props=[1, 1, 1], T=100,
                     arch=[_conv(1, 2, 3, 2, 1, 6), ("linear", 18, 6), ("linear", 6, 2)]),
    # MLP 784-1024x4-10, box +-0.02
    "mlp": dict(cfg=5, input=(784, 1, 1), eps=0.02, B=1024, props=[1024], T=0,
                arch=[("linear", 784, 1024), ("linear", 1024, 1024), ("linear", 1024, 1024),
                      ("linear", 1024, 1024), ("linear", 1024, 10)]),
}


def config_names() -> List[str]:
    return list(CONFIGS)


def _build_layers(arch, in_shape, rng) -> List[LayerSpec]:
    specs = []
    shape = in_shape
    raw = []
    for a in arch:
        if a[0] == "linear":
            _, ni, no = a
            assert int(np.prod(shape)) == ni, (shape, ni)
            W = rng.normal(0.0, np.sqrt(2.0 / ni), size=(no, ni))
            raw.append(("linear", W, shape, (no, 1, 1), 1, 0))
            shape = (no, 1, 1)
        else:
            _, ci, co, k, s, p, hw, ho = a
            assert shape == (ci, hw, hw), (shape, ci, hw)
            W = rng.normal(0.0, np.sqrt(2.0 / (ci * k * k)), size=(co, ci, k, k))
            raw.append(("conv", W, shape, (co, ho, ho), s, p))
            shape = (co, ho, ho)
    for (kind, W, ins, outs, s, p) in raw:
        nb = W.shape[0]
        b = rng.normal(0.0, np.sqrt(0.1), size=(nb,))
        specs.append(LayerSpec(kind, W.astype(np.float32), b.astype(np.float32), ins, outs, s, p))
    return specs


def _round_down_f32(x: np.ndarray) -> np.ndarray:
    y = x.astype(np.float32)
    over = y.astype(np.float64) > x
    y[over] = np.nextafter(y[over], np.float32(-np.inf))
    return y


def _round_up_f32(x: np.ndarray) -> np.ndarray:
    y = x.astype(np.float32)
    under = y.astype(np.float64) < x
    y[under] = np.nextafter(y[under], np.float32(np.inf))
    return y


def _interval_bounds(layers: List[LayerSpec], l0: np.ndarray, u0: np.ndarray):
    """Interval propagation of a box through the hidden layers (float64)."""
    import torch
    import torch.nn.functional as F
    lo = torch.from_numpy(l0.astype(np.float64))
    hi = torch.from_numpy(u0.astype(np.float64))
    out_l, out_u = [], []
    for k, L in enumerate(layers[:-1]):
        mid = (lo + hi) / 2
        rad = (hi - lo) / 2
        W = torch.from_numpy(L.W.astype(np.float64))
        b = torch.from_numpy(L.b.astype(np.float64))
        if L.kind == "linear":
            cm = mid @ W.T + b
            cr = rad @ W.abs().T
        else:
            C, H, Wd = L.in_shape
            m4 = mid.reshape(-1, C, H, Wd)
            r4 = rad.reshape(-1, C, H, Wd)
            cm = F.conv2d(m4, W, b, stride=L.stride, padding=L.pad).reshape(mid.shape[0], -1)
            cr = F.conv2d(r4, W.abs(), None, stride=L.stride, padding=L.pad).reshape(mid.shape[0], -1)
        lk = (cm - cr).numpy()
        uk = (cm + cr).numpy()
        out_l.append(_round_down_f32(lk))
        out_u.append(_round_up_f32(uk))
        lo = torch.from_numpy(np.maximum(out_l[-1].astype(np.float64), 0.0))
        hi = torch.from_numpy(np.maximum(out_u[-1].astype(np.float64), 0.0))
    return out_l, out_u


def make_instance(name: str, B: Optional[int] = None, props: Optional[Sequence[int]] = None,
                  seed: Optional[int] = None, split_frac: float = 0.05) -> Instance:
    """Build a configuration's instance.

    ``B`` (single-property configs) or ``props`` (list of per-property subdomain
    counts) override the batch size; shapes stay those of the configuration.
    """
    cfg = CONFIGS[name]
    if props is None:
        props = [B] if B is not None else list(cfg["props"])
        if B is not None and len(cfg["props"]) > 1:
            raise ValueError("use props= for multi-property configs")
    props = [int(p) for p in props]
    if seed is None:
        seed = BASE_SEED + 10 * cfg["cfg"]
    rng = np.random.Generator(np.random.PCG64(seed))
    in_shape = tuple(cfg["input"])
    layers = _build_layers(cfg["arch"], in_shape, rng)
    n0 = int(np.prod(in_shape))
    n_out = layers[-1].n_out
    eps = cfg["eps"]

    l0s, u0s, ls, us, cs, pidx = [], [], [[] for _ in layers[:-1]], [[] for _ in layers[:-1]], [], []
    for p, nsub in enumerate(props):
        x0 = rng.uniform(0.0, 1.0, size=(n0,))
        if n_out == 2:
            cvec = np.array([1.0, -1.0])
        else:
            t, j = rng.choice(n_out, size=2, replace=False)
            cvec = np.zeros(n_out)
            cvec[t] = 1.0
            cvec[j] = -1.0
        # rounded outward, so that the float32 box contains x0 +- eps
        l0 = _round_down_f32(x0 - eps)[None, :]
        u0 = _round_up_f32(x0 + eps)[None, :]
        lk, uk = _interval_bounds(layers, l0, u0)
        flat_l = np.concatenate([a[0] for a in lk])
        flat_u = np.concatenate([a[0] for a in uk])
        amb = np.nonzero((flat_l < 0) & (flat_u > 0))[0]
        nsplit = int(round(split_frac * amb.size))
        Ls = np.repeat(flat_l[None, :], nsub, axis=0)
        Us = np.repeat(flat_u[None, :], nsub, axis=0)
        for s in range(nsub):
            if nsplit == 0:
                continue
            pick = rng.choice(amb, size=nsplit, replace=False)
            active = rng.uniform(size=nsplit) < 0.5
            Ls[s, pick[active]] = 0.0
            Us[s, pick[~active]] = 0.0
        off = 0
        for k, L in enumerate(layers[:-1]):
            nk = L.n_out
            ls[k].append(Ls[:, off:off + nk])
            us[k].append(Us[:, off:off + nk])
            off += nk
        l0s.append(np.repeat(l0, nsub, axis=0))
        u0s.append(np.repeat(u0, nsub, axis=0))
        cs.append(np.repeat(cvec.astype(np.float32)[None, :], nsub, axis=0))
        pidx.append(np.full(nsub, p, dtype=np.int32))
    inst = Instance(
        name=name, layers=layers,
        l0=np.ascontiguousarray(np.concatenate(l0s)), u0=np.ascontiguousarray(np.concatenate(u0s)),
        l=[np.ascontiguousarray(np.concatenate(a)) for a in ls],
        u=[np.ascontiguousarray(np.concatenate(a)) for a in us],
        c=np.ascontiguousarray(np.concatenate(cs)), prop=np.concatenate(pidx),
        meta=dict(config=name, seed=seed, props=props, eps=eps, split_frac=split_frac,
                  T=cfg["T"]))
    return inst


def random_duals(inst: Instance, seed: int, scale: float = 0.1) -> List[np.ndarray]:
    """Random dual points rho_k ~ N(0, scale^2), float32, one array per hidden layer."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return [(scale * rng.standard_normal(size=a.shape)).astype(np.float32) for a in inst.l]


def instance_to_torch(inst: Instance, device="cpu", dtype=None):
    """Convert the arrays of an instance to torch tensors (no arithmetic)."""
    import torch
    def t(a):
        x = torch.from_numpy(np.ascontiguousarray(a))
        if dtype is not None:
            x = x.to(dtype)
        return x.to(device)
    return dict(l0=t(inst.l0), u0=t(inst.u0), l=[t(a) for a in inst.l], u=[t(a) for a in inst.u],
                c=t(inst.c))
