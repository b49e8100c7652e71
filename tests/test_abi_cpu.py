"""CPU-only checks of the C ABI: the library loads, exports every symbol that
include/ld.h declares, and rejects bad arguments on the host before any
device work (no compute call runs here)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ld.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ld_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    from paper_2104_06718_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_2104_06718_amd import build
        build.build()
    return binding.load_library()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    from paper_2104_06718_amd import binding
    assert sorted(binding.EXPORTED) == names


def _layer(kind, ins, outs, k=1, s=1, p=0, W=None, b=None):
    from paper_2104_06718_amd.binding import ld_layer
    L = ld_layer()
    L.kind = kind
    L.in_c, L.in_h, L.in_w = ins
    L.out_c, L.out_h, L.out_w = outs
    L.kh = L.kw = k
    L.stride, L.pad = s, p
    L.W = W.ctypes.data if W is not None else None
    L.b = b.ctypes.data if b is not None else None
    return L


def _create(lib, layers):
    from paper_2104_06718_amd.binding import ld_layer
    arr = (ld_layer * len(layers))(*layers)
    h = ctypes.c_void_p()
    rc = lib.ld_create_net(arr, len(layers), ctypes.byref(h))
    return rc, lib.ld_last_error().decode()


def test_create_net_rejects_bad_shapes(lib):
    W = np.ones(10000, dtype=np.float32)
    b = np.zeros(100, dtype=np.float32)
    # one layer only
    rc, msg = _create(lib, [_layer(0, (4, 1, 1), (2, 1, 1), W=W, b=b)])
    assert rc == -2 and "hidden" in msg
    # chained sizes differ
    rc, _ = _create(lib, [_layer(0, (4, 1, 1), (3, 1, 1), W=W, b=b), _layer(0, (5, 1, 1), (2, 1, 1), W=W, b=b)])
    assert rc == -2
    # conv output size inconsistent with (in + 2p - k)/s + 1
    rc, msg = _create(lib, [_layer(1, (3, 8, 8), (4, 5, 5), k=4, s=2, p=1, W=W, b=b),
                            _layer(0, (100, 1, 1), (2, 1, 1), W=W, b=b)])
    assert rc == -2 and "conv output size" in msg
    # a conv objective layer (an intermediate bound's sub-network) whose input is not the previous map
    rc, _ = _create(lib, [_layer(1, (3, 8, 8), (4, 4, 4), k=4, s=2, p=1, W=W, b=b),
                          _layer(1, (5, 4, 4), (2, 2, 2), k=4, s=2, p=1, W=W, b=b)])
    assert rc == -2
    # NULL weights
    rc, _ = _create(lib, [_layer(0, (4, 1, 1), (3, 1, 1), W=None, b=b), _layer(0, (3, 1, 1), (2, 1, 1), W=W, b=b)])
    assert rc == -1
    # non-finite weight
    Wn = W.copy()
    Wn[3] = np.nan
    rc, _ = _create(lib, [_layer(0, (4, 1, 1), (3, 1, 1), W=Wn, b=b), _layer(0, (3, 1, 1), (2, 1, 1), W=W, b=b)])
    assert rc == -3
    # unsupported stride
    rc, _ = _create(lib, [_layer(1, (3, 16, 16), (4, 4, 4), k=4, s=4, p=0, W=W, b=b),
                          _layer(0, (64, 1, 1), (2, 1, 1), W=W, b=b)])
    assert rc == -6


def test_null_arguments_rejected(lib):
    from paper_2104_06718_amd.binding import ld_batch, ld_opts
    bt = ld_batch()
    assert lib.ld_dual_eval(None, ctypes.byref(bt), None, None, None, 0, ctypes.c_float(0.0), None) == -1
    assert lib.ld_step(None, None, None, None, None) == -1
    assert lib.ld_final_bound(None, None, None, None, None, None, None, ctypes.c_float(0.0), None) == -1
    assert lib.ld_init_duals(None, None, 0, 0, None, None) == -1
    assert lib.ld_state_create(None, 4, ctypes.byref(ctypes.c_void_p())) == -1
    assert lib.ld_prox_step(None, None, None, None, None) == -1
    assert lib.ld_prox_get_step(None, ctypes.byref(ctypes.c_int())) == -1
    assert lib.ld_rounding_margin(None, None, None, None, None) == -1
    assert "NULL" in lib.ld_last_error().decode()


def test_product_path_has_no_oracle_or_cpu_fallback():
    pkg = os.path.join(ROOT, "paper_2104_06718_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in src.replace("no oracle", ""), f
