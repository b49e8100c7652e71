"""The C ABI used from a host program alone (tests/c/ld_abi_run.cpp: include/ld.h
and the HIP runtime, no Python or torch): net creation, the supergradient method
and the final bound, against the FP64 oracle and the Python binding.

The program is built by __graft_entry__.build() next to its source.  Every test
prints the case before touching the GPU.
"""
import os
import struct
import subprocess

import numpy as np
import pytest
import torch

import ldgen
from oracle import ld_oracle as O

pytestmark = pytest.mark.gpu

PROG = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c", "ld_abi_run")
FP32_FINAL_REL = 3e-3


def _write(inst, path):
    with open(path, "wb") as f:
        f.write(struct.pack("<2i", len(inst.layers), inst.B))
        for L in inst.layers:
            lin = L.kind == "linear"
            kh, kw = (1, 1) if lin else L.W.shape[2:4]
            f.write(struct.pack("<11i", 0 if lin else 1, *L.in_shape, *L.out_shape, kh, kw,
                                1 if lin else int(L.stride), 0 if lin else int(L.pad)))
        for L in inst.layers:
            f.write(np.ascontiguousarray(L.W, dtype="<f4").tobytes())
            f.write(np.ascontiguousarray(L.b, dtype="<f4").tobytes())
        arrays = [inst.l0, inst.u0]
        for lo, hi in zip(inst.l, inst.u):
            arrays += [lo, hi]
        arrays.append(inst.c)
        for a in arrays:
            f.write(np.ascontiguousarray(a, dtype="<f4").tobytes())


@pytest.mark.parametrize("name,T", [("fc_tiny", 200), ("tiny_conv", 100), ("base", 60)])
def test_host_program_matches_the_oracle_and_the_binding(name, T, tmp_path):
    _case = print
    _case(f"[case] C ABI program {name} T={T}", flush=True)
    assert os.path.exists(PROG), "build the library and the ABI program first (__graft_entry__.build())"
    inst = ldgen.make_instance(name)
    path = str(tmp_path / f"{name}.bin")
    _write(inst, path)
    res = subprocess.run([PROG, path, str(T), "0"], capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stderr
    got = np.array([float(l.split()[2]) for l in res.stdout.splitlines() if l.startswith("bound ")])
    assert got.shape == (inst.B,)
    # the same run through the Python binding gives the same bounds (same kernels, same inputs)
    import paper_2104_06718_amd as P
    net = P.Net(inst.layers)
    batch = P.Batch.from_instance(inst)
    st = P.State(net, inst.B)
    P.step(net, batch, st, iters=T, total_iters=T, precision="fp32", engine="layerwise")
    fb = P.final_bound(net, batch, st)
    torch.cuda.synchronize()
    d_bind = np.abs(got - fb["bound"].cpu().numpy())
    print(f"  |program - binding| max {d_bind.max():.2e}")
    assert np.all(d_bind <= 1e-9 * (1 + np.abs(got)))
    idx = list(range(min(inst.B, 8)))
    onet = O.net_from_specs(inst.layers)
    ob = O.batch_from_instance(inst, idx)
    ofb = O.final_bound(onet, ob, O.ascent(onet, ob, O.AdamOpts(T=T)))
    d = np.abs(got[idx] - ofb["bound"].numpy())
    print(f"  |program - oracle| max {d.max():.2e}")
    assert np.all(d <= FP32_FINAL_REL * np.abs(ofb["bound"].numpy()) + 1e-3)


def test_host_program_reports_bad_input(tmp_path):
    """Layer 2's input width differs from layer 1's output: ld_create_net refuses the
    net and the program reports the library's error."""
    print("[case] C ABI program, inconsistent layer sizes", flush=True)
    inst = ldgen.make_instance("fc_tiny")
    L1 = inst.layers[1]
    n_out = L1.W.shape[0]
    L1.in_shape = (L1.in_shape[0] + 1, 1, 1)
    L1.W = np.zeros((n_out, L1.in_shape[0]), dtype=np.float32)
    path = str(tmp_path / "bad.bin")
    _write(inst, path)
    res = subprocess.run([PROG, path, "5", "0"], capture_output=True, text=True, timeout=120)
    assert res.returncode == 1, (res.returncode, res.stderr)
    assert "ld_create_net" in res.stderr and "differs" in res.stderr, res.stderr
