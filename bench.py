#!/usr/bin/env python3
"""Benchmark of the Lagrangian-decomposition bounding step on one MI355X.

One "step" is one complete bounding run over a batch of B subdomains: CROWN dual
initialisation, T Adam supergradient iterations (Algorithm 1 with Adam), and the
final bound re-evaluated with FP32 operands and an FP64 sum plus the primal
upper bound.  The default workload is the wide conv net (conv 16@4x4/2,
conv 32@4x4/2, FC 100, FC 10 on 3x32x32 inputs), B = 512, T = 500, with
synthetic seeded weights and subdomains (see ldgen).  Inputs are resident in
device memory before the timed region starts.

Prints ONE JSON line.  `value` is bounds/sec of the BF16 form (BF16 operands on
MFMA, FP32 accumulation) at the iteration count that reaches the FP32 form's
bound: the criterion is mean over subdomains of (FP32 bound - BF16 bound) <= 1e-3,
i.e. the BF16 form is not looser on average (T, then T+50, T+100, ... until it
holds).  Per-subdomain gaps are reported beside it, with the FP32 form, and the
FP64 form (the FP64 engine) with its error against the oracle.  Launch
configurations and the engine come from the autotuner (run during the warm-up,
outside the timed region).

The roofline of the dominant launch counts, as algorithmic bytes, that launch's
share of the state that one iteration must stream at least once: per hidden
neuron rho, l, u read in phase A (the inner minimisation that needs them) and
m, v read and rho, m, v written in phase B, plus the input box: (8 N_h + 2 n_0)
4-byte words per subdomain.  The intermediates (x*, xB*, g, xA) are avoidable by
fusion and are not counted.
"""
import hashlib
import argparse
import json
import os
import sys
import time
import types

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
PEAK_TFLOPS = {"fp32": 157.3, "bf16": 2500.0}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="wide")
    ap.add_argument("--B", type=int, default=None)
    ap.add_argument("--iters", type=int, default=None, help="Adam iterations per bounding run (default: config T)")
    ap.add_argument("--bf16-iters", type=int, default=None,
                    help="iterations of the BF16 form (default: searched for equal bound)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=512, help="subdomains timed on the host oracle")
    ap.add_argument("--quick", action="store_true", help="skip the equal-bound search (profiling runs)")
    ap.add_argument("--profile-only", choices=["fp32", "bf16"], default=None,
                    help="for rocprofv3: one 1 GiB device copy (counter calibration), then --reps ascent "
                         "iterations launched without the graph; prints the per-launch averages")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--pin-tiles", metavar="FILE", default=None,
                    help="after tuning, pin every contraction to the configuration that the bench line in this "
                         "file (JSON, or a markdown summary with the line in a json block) reports for the "
                         "precision (its 'tuned' entry), so that separate counter runs time the same kernels")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="start with the 1 GiB device copy of --profile-only (counter calibration), so that "
                         "--profile-summary can read counter runs of the bench line itself: its last "
                         "contraction launches are the BF16 per-launch timing of one iteration")
    ap.add_argument("--profile-summary", metavar="DIR", default=None,
                    help="no GPU: read the rocprofv3 outputs of --profile-only runs under DIR (T: --kernel-trace "
                         "--stats; F: --pmc FETCH_SIZE; W: --pmc WRITE_SIZE; M, optional: --pmc SQ_INSTS_VALU_MFMA_MOPS_BF16 "
                         "SQ_INSTS_VALU_MFMA_MOPS_F32 SQ_VALU_MFMA_BUSY_CYCLES SQ_BUSY_CU_CYCLES), print the per-launch markdown summary and, with --write-traffic, store the "
                         "calibrated bytes per launch in profiles/traffic.json")
    ap.add_argument("--write-traffic", action="store_true")
    ap.add_argument("--engine", choices=["auto", "layerwise", "resident"], default="auto")
    ap.add_argument("--solver", choices=["ld", "prox", "interm", "fsb", "sigmoid", "bab"], default="ld",
                    help="ld: Adam supergradient ascent (the headline line); prox: the proximal solver; "
                         "interm: LD intermediate bounds of one layer; fsb: branching decisions; "
                         "sigmoid: the sigmoid inner minimisation; bab: branch-and-bound rounds")
    ap.add_argument("--layer", type=int, default=2, help="interm: layer j whose pre-activations are bounded")
    ap.add_argument("--interm-copy", action="store_true",
                    help="interm: chunks that are not whole subdomains, so every problem gets a copy of its "
                         "subdomain's bound rows (the layout without shared rows, for comparison)")
    return ap.parse_args()


def layer_slot_cost(inst, kind, B, prec):
    """Algorithmic bytes and useful FLOPs of one launch of an iteration slot.

    Bytes are the compulsory traffic of the launch's inputs and outputs, each read
    or written once (weights included):
      phase A (100+k): read rho_k; read the bounds (and rho) of layer k-1; write
                       x*_{k-1} (operand type) and, for k-1 >= 1, xB*_{k-1}
      200+k          : read g_const, rho_k, l_k, u_k; write xB*_k
      phase B (300+k): read x*_{k-1} (operand type); read xB*_k; read and write
                       rho_k, m_k, v_k
    FLOPs count 2 per multiply-add of the contraction (no structural zeros)."""
    layers = inst.layers
    opb = 2 if prec == "bf16" else 4
    ph, k = divmod(kind, 100)
    width = lambda j: layers[0].n_in if j == 0 else layers[j - 1].n_out  # noqa: E731
    def macs(L):
        if L.kind == "linear":
            return L.n_in * L.n_out
        Co, Ho, Wo = L.out_shape
        return Co * Ho * Wo * L.in_shape[0] * L.W.shape[2] * L.W.shape[3]
    def wbytes(L):
        return L.W.size * opb
    if ph == 1:
        L = layers[k - 1]
        nb = width(k) * 4 + (width(0) * (8 + opb) if k == 1 else width(k - 1) * (12 + opb + 4))
        # transposed conv: taps that fall outside the input are not work
        flops = 2 * macs(L)
        return B * nb + wbytes(L), B * flops
    if ph == 2:
        return B * width(k) * 20, 0
    L = layers[k - 1]
    nb = width(k - 1) * opb + width(k) * 28
    return B * nb + wbytes(L), B * 2 * macs(L)


def prox_slot_cost(inst, kind, B, prec):
    """Algorithmic bytes and FLOPs of one launch of a proximal-iteration slot.

      100+k W_k^T rt_k : read rt_k and W_k; write g_{k-1} (k >= 2) or, for k = 1,
                         read l_0, u_0 and write z_0 (operand type)
      300+k forward    : read z_{k-1} (operand type) and W_k; write zA_k
      400+k block k    : layer k (k >= 1): read xB, zB, rt, rho, xA, pi, write xB,
                         rt, rho, pi (the last sweep of an outer iteration, timed
                         here, also takes the dual update);
                         layer k+1: read xA, zA, rt, rho, xB, g, l, u, write xA, rt,
                         zB and z (operand type); the objective layer: read xA, zA,
                         c, write xA"""
    layers = inst.layers
    n = len(layers)
    opb = 2 if prec == "bf16" else 4
    ph, k = divmod(kind, 100)
    width = lambda j: layers[0].n_in if j == 0 else layers[j - 1].n_out  # noqa: E731

    def macs(L):
        if L.kind == "linear":
            return L.n_in * L.n_out
        Co, Ho, Wo = L.out_shape
        return Co * Ho * Wo * L.in_shape[0] * L.W.shape[2] * L.W.shape[3]
    if ph == 1:
        L = layers[k - 1]
        nb = width(k) * 4 + (width(0) * (8 + opb) if k == 1 else width(k - 1) * 4)
        return B * nb + L.W.size * opb, B * 2 * macs(L)
    if ph == 3:
        L = layers[k - 1]
        return B * (width(k - 1) * opb + width(k) * 4) + L.W.size * opb, B * 2 * macs(L)
    nb = width(k) * 40 if k >= 1 else 0
    nb += width(k + 1) * (16 if k + 1 == n else 44 + opb)
    return B * nb, 0


def floor_share(inst, kind, B):
    """Bytes of one launch's share of the per-iteration state floor (8 N_h + 2 n_0
    words per subdomain): slot 100+k reads what the inner minimisation of layer k-1
    needs (the box for k = 1: l_0, u_0; else rho, l, u of layer k-1); slot 300+k
    reads m_k, v_k and writes rho_k, m_k, v_k, and for the last hidden layer (whose
    minimisation its epilogue does) also reads rho, l, u."""
    layers = inst.layers
    n = len(layers)
    width = lambda j: layers[0].n_in if j == 0 else layers[j - 1].n_out  # noqa: E731
    ph, k = divmod(kind, 100)
    if ph == 1:
        return B * (8 * width(0) if k == 1 else 12 * width(k - 1))
    return B * (20 + (12 if k == n - 1 else 0)) * width(k)


def state_floor(inst, B):
    """(8 N_h + 2 n_0) * 4 bytes per subdomain: the state streamed once per iteration."""
    nh = sum(L.n_out for L in inst.layers[:-1])
    return B * (8 * nh + 2 * inst.layers[0].n_in) * 4


def kernel_name(info, kind, inst, prec="fp32"):
    """Name of the kernel launched for an iteration slot under the tuned configuration
    (in the BF16 form, transposed products of layers k >= 2 are compensated products,
    which the stride-class form computes)."""
    ph, k = divmod(kind, 100)
    L = inst.layers[k - 1]
    cfg = None
    if info is not None:
        d = "transposed" if ph == 1 else "forward"
        cfg = next((e for e in info["layers"] if e["layer"] == k and e["dir"] == d), None)
    if L.kind == "linear":
        return "fc_kernel"
    compensated = prec == "bf16" and ph == 1 and k >= 2
    if ph == 1 and L.stride > 1 and (cfg is None or cfg["form"] == 0) and not compensated:
        return "convT_kernel"
    return "conv_plane_kernel"


def run_form(P, net, batch, st, iters, prec, steps, warmup, engine="auto"):
    import torch
    for _ in range(warmup):
        st.reset()
        P.step(net, batch, st, iters=iters, total_iters=iters, precision=prec, engine=engine)
        P.final_bound(net, batch, st)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(s)
    fb = None
    for _ in range(steps):
        st.reset()
        P.step(net, batch, st, iters=iters, total_iters=iters, precision=prec, engine=engine)
        fb = P.final_bound(net, batch, st)
    e1.record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return dict(ms_per_step=e0.elapsed_time(e1) / steps, wall_ms_per_step=1000 * wall / steps, fb=fb)


def pin_tiles(P, net, batch, prec, path):
    """Tune (net, B, prec), then pin each contraction's configuration to the one the
    bench line in `path` reports: a JSON file, or a markdown summary that holds the
    line in a ```json block."""
    with open(path) as fh:
        text = fh.read()
    if "```json" in text:
        text = text.split("```json", 1)[1].split("```", 1)[0]
    d = json.loads(text)
    P.autotune(net, batch, precision=prec)
    for lay in d["tuned"][prec]["layers"]:
        P.set_tuned_config(net, batch.B, prec, lay["layer"], lay["dir"], lay)


def cpu_baseline(inst, T, sample):
    """The FP64 oracle on the first `sample` subdomains (all T iterations, CROWN
    init, final bound), timed on the host; also returns its bounds."""
    import numpy as np
    import torch
    from oracle import ld_oracle as O
    idx = list(range(min(sample, inst.B)))
    onet = O.net_from_specs(inst.layers)
    ob = O.batch_from_instance(inst, idx)
    # the step schedule and Adam constants as the library receives them (float fields)
    f32 = lambda x: float(np.float32(x))  # noqa: E731
    opts = O.AdamOpts(T=T, lr0=f32(1e-2), lr_end=f32(1e-4), beta1=f32(0.9), beta2=f32(0.999), eps=f32(1e-8))
    t0 = time.perf_counter()
    st = O.ascent(onet, ob, opts)
    fb = O.final_bound(onet, ob, st)
    dt = time.perf_counter() - t0
    out = dict(value=len(idx) / dt, unit="bounds/s", cores=torch.get_num_threads(), kind="oracle",
               sample=f"{len(idx)} of {inst.B} subdomains (the first ones), {T} iterations each, "
                      f"FP64 torch-CPU oracle, {dt:.1f} s")
    return out, idx, fb["bound"]


def cpu_baseline_prox(inst, T, sample):
    """The FP64 oracle's proximal solver on the first `sample` subdomains, timed on the host."""
    import torch
    from oracle import ld_oracle as O
    idx = list(range(min(sample, inst.B)))
    onet = O.net_from_specs(inst.layers)
    ob = O.batch_from_instance(inst, idx)
    t0 = time.perf_counter()
    st = O.proximal(onet, ob, O.ProxOpts(T=T))
    fb = O.final_bound(onet, ob, st)
    dt = time.perf_counter() - t0
    out = dict(value=len(idx) / dt, unit="bounds/s", cores=torch.get_num_threads(), kind="oracle",
               sample=f"{len(idx)} of {inst.B} subdomains (the first ones), {T} outer iterations each, "
                      f"FP64 torch-CPU oracle, {dt:.1f} s")
    return out, idx, fb["bound"]


def prox_kernel_name(info, kind, inst, prec):
    ph, k = divmod(kind, 100)
    if ph == 1:
        return kernel_name(info, 100 + k, inst, prec)
    if ph == 3:
        return kernel_name(info, 300 + k, inst, prec)
    return "prox_block_kernel"


def main_prox(a, P, inst, net, batch):
    """Proximal solver (Algorithm 2, Sec. 7.2 settings: J = 2, mu = 0.3, eta 10 -> 500)
    on the same workload: CROWN init, T outer iterations, final bound."""
    import torch
    B = inst.B
    T = a.iters or 100
    kw = dict(total_iters=T, inner_iters=2, eta0=10.0, eta_end=500.0, mu=0.3)
    res = {}
    for prec in ("fp32", "bf16"):
        # launch configurations of the contractions (shared with the supergradient method)
        P.autotune(net, batch, precision=prec)
        st = P.State(net, B)
        for _ in range(a.warmup):
            st.reset()
            P.prox_step(net, batch, st, iters=T, precision=prec, **kw)
            P.final_bound(net, batch, st)
        torch.cuda.synchronize()
        s = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        fb = None
        for _ in range(a.steps):
            st.reset()
            P.prox_step(net, batch, st, iters=T, precision=prec, **kw)
            fb = P.final_bound(net, batch, st)
        e1.record(s)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / a.steps
        # per-launch timing of one outer iteration (HIP events on the launch stream)
        slots = P.prox_profile_iteration(net, batch, st, reps=a.reps, precision=prec, **kw)
        torch.cuda.synchronize()
        res[prec] = dict(ms=ms, fb=fb, slots=slots)
    # the supergradient method's bound on the same batch (context, not timed)
    stl = P.State(net, B)
    P.step(net, batch, stl, iters=500, total_iters=500, precision="fp32")
    b_ld = P.final_bound(net, batch, stl)["bound"]
    torch.cuda.synchronize()

    head = "fp32"
    slots = res[head]["slots"]
    info = P.tuning_info(net, B, head)
    kind, us = max(slots, key=lambda x: x[1])
    nbytes, flops = prox_slot_cost(inst, kind, B, head)
    ridge = PEAK_TFLOPS[head] * 1e12 / (PEAK_HBM_GBS * 1e9)
    if flops / max(nbytes, 1) < ridge:
        roof = dict(bound="hbm", achieved=nbytes / (us * 1e-6) / 1e9, peak=PEAK_HBM_GBS, unit="GB/s")
    else:
        roof = dict(bound="mfma", achieved=flops / (us * 1e-6) / 1e12, peak=PEAK_TFLOPS[head], unit="TFLOP/s")
    roof["frac"] = roof["achieved"] / roof["peak"]
    kname = prox_kernel_name(info, kind, inst, head)
    roof["traffic"] = stored_traffic(kname, kind, a.config + "/prox", B, head)
    roof["kernel"] = f"{kname}: slot {kind}"
    roof["avg_us"] = us
    roof["algorithmic_bytes"] = nbytes
    roof["algorithmic_flops"] = flops
    b32 = res["fp32"]["fb"]["bound"]
    b16 = res["bf16"]["fb"]["bound"]
    value = B / (res[head]["ms"] / 1000.0)
    out = {
        "metric": f"proximal-solver bounds/sec ({T} outer iters, J=2, B={B}, {a.config} conv net)",
        "value": value,
        "unit": "bounds/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": res[head]["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{a.config} conv net 3x32x32, B={B}, proximal T={T}, J=2, mu=0.3, eta 10->500, "
                               f"1 property, 5% random ReLU splits per subdomain", "B": B, "iters": T},
        "fp32": {"value": value, "ms_per_step": res["fp32"]["ms"], "mean_bound": b32.mean().item()},
        "bf16": {"value": B / (res["bf16"]["ms"] / 1000.0), "ms_per_step": res["bf16"]["ms"],
                 "mean_bound": b16.mean().item(), "gap_mean": (b32 - b16).mean().item()},
        "supergradient_500_fp32_mean_bound": b_ld.mean().item(),
        "roofline": roof,
        "per_launch_us": {p: {str(k): round(v, 2) for k, v in res[p]["slots"]} for p in res},
    }
    if not a.no_cpu_baseline:
        cb, idx, ob = cpu_baseline_prox(inst, T, a.cpu_sample)
        out["cpu_baseline"] = cb
        for p in ("fp32", "bf16"):
            d = res[p]["fb"]["bound"].cpu()[idx] - ob
            out[p]["minus_oracle"] = {"mean": d.mean().item(), "max_abs": d.abs().max().item(),
                                      "subdomains": len(idx), "oracle_iters": T}
    print(json.dumps(out), flush=True)


def main_interm(a, P, inst):
    """LD intermediate bounds (Sec. 2.2.3) of layer j for a few subdomains: every
    (subdomain, neuron, sign) is one LD problem on the sub-network of the first j
    layers (CROWN init, T Adam steps, final bound), run in chunks of 8192."""
    import torch
    j = a.layer
    Bs = a.B or 4
    T = a.iters or 100
    layers = inst.layers
    nj = layers[j - 1].n_out
    sub = P.Net(layers[:j])
    t = lambda x: torch.from_numpy(x[:Bs]).cuda()  # noqa: E731
    batch = P.Batch(t(inst.l0), t(inst.u0), [t(x) for x in inst.l[:j - 1]], [t(x) for x in inst.u[:j - 1]],
                    torch.zeros(Bs, nj, device="cuda"))
    nprob = 2 * nj * Bs
    chunk = 8192 - 4 if a.interm_copy else 8192
    res = {}
    for prec in ("fp32", "bf16"):
        for _ in range(a.warmup):  # includes the autotuner's run for the chunk sizes
            P.intermediate_bounds(sub, batch, iters=T, precision=prec, max_problems=chunk)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            lo, hi = P.intermediate_bounds(sub, batch, iters=T, precision=prec, max_problems=chunk)
        torch.cuda.synchronize()
        ms = 1000 * (time.perf_counter() - t0) / a.steps
        res[prec] = dict(ms=ms, lo=lo, hi=hi)
    # per-launch timing of one iteration on a chunk of the expanded batch (problems of
    # subdomain 0 first, as the library orders them)
    C = min(chunk, nprob)
    g = torch.arange(C, device="cuda")
    b = g // (2 * nj)
    r = g % (2 * nj)
    c = torch.zeros(C, nj, device="cuda")
    c[g, r // 2] = 1.0 - 2.0 * (r % 2).float()
    eb = P.Batch(batch.l0[b], batch.u0[b], [x[b] for x in batch.l], [x[b] for x in batch.u], c)
    prof = {}
    for prec in ("fp32", "bf16"):
        stp = P.State(sub, C)
        P.step(sub, eb, stp, iters=2, total_iters=T, precision=prec)
        prof[prec] = P.profile_iteration(sub, eb, stp, reps=a.reps, total_iters=T, precision=prec)
    torch.cuda.synchronize()
    head = "fp32"
    info = P.tuning_info(sub, C, head)
    fake = types.SimpleNamespace(layers=layers[:j])
    kind, us = max(prof[head], key=lambda x: x[1])
    nbytes, flops = layer_slot_cost(fake, kind, C, head)
    ridge = PEAK_TFLOPS[head] * 1e12 / (PEAK_HBM_GBS * 1e9)
    if flops / max(nbytes, 1) < ridge:
        roof = dict(bound="hbm", achieved=nbytes / (us * 1e-6) / 1e9, peak=PEAK_HBM_GBS, unit="GB/s")
    else:
        roof = dict(bound="mfma", achieved=flops / (us * 1e-6) / 1e12, peak=PEAK_TFLOPS[head], unit="TFLOP/s")
    roof["frac"] = roof["achieved"] / roof["peak"]
    kname = kernel_name(info, kind, fake, head)
    roof["traffic"] = stored_traffic(kname, kind, f"{a.config}/interm{j}", C, head)
    roof["kernel"] = f"{kname}: slot {kind} (phase {kind // 100}, layer {kind % 100}) at {C} problems"
    roof["avg_us"] = us
    roof["algorithmic_bytes"] = nbytes
    roof["algorithmic_flops"] = flops
    ibp_w = (torch.from_numpy(inst.u[j - 1][:Bs]) - torch.from_numpy(inst.l[j - 1][:Bs])).double()
    out = {
        "metric": f"LD intermediate bounds/sec (layer {j} of the {a.config} conv net, {T} iters, "
                  f"{nprob} problems)",
        "value": nprob / (res[head]["ms"] / 1000.0),
        "unit": "bounds/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": res[head]["ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{a.config} conv net 3x32x32, pre-activation bounds of layer {j} ({nj} neurons) "
                               f"for {Bs} subdomains: {nprob} LD problems (+-e_i), T={T}, chunks of {chunk}, "
                               f"bound rows {'copied per problem' if a.interm_copy else 'shared per subdomain'}",
                   "subdomains": Bs, "layer": j, "problems": nprob, "iters": T},
        "bf16": {"value": nprob / (res["bf16"]["ms"] / 1000.0), "ms_per_step": res["bf16"]["ms"]},
        "mean_width": {p: (res[p]["hi"] - res[p]["lo"]).double().mean().item() for p in res},
        "ibp_mean_width": ibp_w.mean().item(),
        "roofline": roof,
        "per_launch_us": {p: {str(k): round(v, 2) for k, v in prof[p]} for p in prof},
    }
    if not a.no_cpu_baseline:
        # the oracle on the first neurons of subdomain 0 (both signs)
        from oracle import ld_oracle as O
        nn = min(nj, 1024)
        onet = O.net_from_specs(layers)
        ob = O.batch_from_instance(inst, [0])
        ob = O.OBatch(ob.l0, ob.u0, ob.l, ob.u, ob.c)
        sub_o = onet[:j]
        eb_o = O.neuron_batch(ob, j, nj)
        keep = torch.arange(2 * nn)
        eb_o = O.OBatch(eb_o.l0[keep], eb_o.u0[keep], [x[keep] for x in eb_o.l], [x[keep] for x in eb_o.u],
                        eb_o.c[keep])
        t0 = time.perf_counter()
        st = O.ascent(sub_o, eb_o, O.AdamOpts(T=T))
        fbo = O.final_bound(sub_o, eb_o, st)["bound"].reshape(nn, 2)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = dict(value=2 * nn / dt, unit="bounds/s", cores=torch.get_num_threads(), kind="oracle",
                                   sample=f"{2 * nn} of {nprob} problems (neurons 0..{nn - 1} of subdomain 0, both "
                                          f"signs), {T} iterations each, FP64 torch-CPU oracle, {dt:.1f} s")
        d_lo = res[head]["lo"][0, :nn].cpu().double() - fbo[:, 0]
        d_hi = res[head]["hi"][0, :nn].cpu().double() + fbo[:, 1]
        out["minus_oracle"] = {"lower_max_abs": d_lo.abs().max().item(), "upper_max_abs": d_hi.abs().max().item(),
                               "problems": 2 * nn}
    print(json.dumps(out), flush=True)


def main_fsb(a, P, inst, net, batch):
    """Filtered Smart Branching (Sec. 4.2) for every subdomain of the batch: scores,
    candidates, 4 (n-1) children per subdomain bounded by CROWN and WK, the split."""
    import torch
    B = inst.B
    for _ in range(a.warmup):
        P.fsb_branch(net, batch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        layer, index, value = P.fsb_branch(net, batch)
    torch.cuda.synchronize()
    ms = 1000 * (time.perf_counter() - t0) / a.steps
    out = {
        "metric": f"FSB branching decisions/sec (B={B}, {a.config} conv net)",
        "value": B / (ms / 1000.0),
        "unit": "decisions/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{a.config} conv net 3x32x32, B={B} subdomains, {4 * (len(inst.layers) - 1)} "
                               f"children each bounded by CROWN and WK", "B": B},
        "mean_worse_child_bound": value[torch.isfinite(value)].mean().item(),
        # the call is one synchronous pipeline (allocation included); its kernels are
        # timed by rocprofv3 (profiles/), not per launch here
        "roofline": None,
    }
    if not a.no_cpu_baseline:
        from oracle import ld_oracle as O
        idx = list(range(min(B, 256)))
        onet = O.net_from_specs(inst.layers)
        ob = O.batch_from_instance(inst, idx)
        t0 = time.perf_counter()
        ol, oi, ov = O.fsb_branch(onet, ob)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = dict(value=len(idx) / dt, unit="decisions/s", cores=torch.get_num_threads(),
                                   kind="oracle", sample=f"{len(idx)} of {B} subdomains (the first ones), "
                                                         f"FP64 torch-CPU oracle, {dt:.1f} s")
        same = (layer.cpu().long()[idx] == ol) & (index.cpu().long()[idx] == oi)
        out["equal_to_oracle"] = f"{int(same.sum())} of {len(idx)} splits"
    print(json.dumps(out), flush=True)


def main_sigmoid(a, P, inst):
    """The sigmoid P_k inner minimisation (App. E) over every hidden neuron of the
    batch (B x N_h elements, the wide net's shapes): the hull's tangent points once,
    then the minimisation, each timed with HIP events on the launch stream."""
    import numpy as np
    import torch
    B = inst.B
    l = torch.cat([torch.from_numpy(x) for x in inst.l], dim=1).contiguous().cuda()
    u = torch.cat([torch.from_numpy(x) for x in inst.u], dim=1).contiguous().cuda()
    n = l.numel()
    gen = torch.Generator(device="cuda").manual_seed(5)
    rho = (torch.randn(l.shape, generator=gen, device="cuda") * 0.05).contiguous()
    g = (torch.randn(l.shape, generator=gen, device="cuda") * 0.5).contiguous()
    s = torch.cuda.current_stream()

    def timed(f, reps):
        for _ in range(max(a.warmup, 1)):
            out = f()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            out = f()
        e1.record(s)
        torch.cuda.synchronize()
        return out, 1000.0 * e0.elapsed_time(e1) / reps
    (tu, tl), us_hull = timed(lambda: P.sigmoid_hull(l, u), a.reps)
    (xb, x, val), us_min = timed(lambda: P.sigmoid_inner_min(rho, g, l, u, tu, tl), a.reps)
    nbytes = n * (6 * 4 + 2 * 4 + 8)   # read rho, g, l, u, t_up, t_lo; write xB, x (FP32), value (FP64)
    roof = dict(bound="hbm", achieved=nbytes / (us_min * 1e-6) / 1e9, peak=PEAK_HBM_GBS, unit="GB/s")
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof.update(traffic=None, kernel="sigmoid_inner_min_kernel", avg_us=us_min, algorithmic_bytes=nbytes,
                algorithmic_flops=None)
    out = {
        "metric": f"sigmoid inner minimisations/sec ({n} neurons: B={B} x N_h of the {a.config} net)",
        "value": n / (us_min * 1e-6),
        "unit": "neurons/s",
        "n_gpus": 1, "steps": a.reps, "warmup": a.warmup, "ms_per_step": us_min / 1000.0,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{a.config} net bounds, B={B}: {n} sigmoid neurons, rho ~ N(0, 0.05^2), "
                               f"g ~ N(0, 0.5^2)", "neurons": n},
        "hull_us": us_hull,
        "roofline": roof,
    }
    if not a.no_cpu_baseline:
        from oracle import ld_oracle as O
        m = n
        D = lambda t: t.reshape(-1)[:m].double().cpu()  # noqa: E731
        t0 = time.perf_counter()
        otu, otl = O.sigmoid_hull(D(l), D(u))
        ob = O.inner_min_sigmoid(D(rho), D(g), D(l), D(u), otu, otl)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = dict(value=m / dt, unit="neurons/s", cores=torch.get_num_threads(), kind="oracle",
                                   sample=f"{m} of {n} neurons (hull and minimisation), FP64 torch-CPU oracle, "
                                          f"{dt:.1f} s")
        out["minus_oracle_max_abs"] = (val.reshape(-1)[:m].cpu() - ob[2]).abs().max().item()
    print(json.dumps(out), flush=True)


def main_bab(a, P, inst):
    """Branch and bound on the first property of the workload, minimising for a fixed
    number of rounds (Sec. 7.3 settings: children from their parent's duals, 160 Adam
    steps 1e-3 -> 1e-4; the wide net's batch of 200 splits per round): subproblems
    bounded per second, the whole driver included (branching, children, bounding,
    the store's row moves, the host's queue)."""
    import math
    import torch
    rounds = a.iters or 10
    Bs = a.B or 200
    root = P.Batch.from_instance(inst.subset([0]))
    net = P.Net(inst.layers)
    kw = dict(threshold=-math.inf, batch=Bs, root_iters=500, iters=160, lr0=1e-3, lr_end=1e-4, max_rounds=rounds,
              max_subproblems=1 << 17)
    for _ in range(a.warmup):
        P.bab(net, root, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        r = P.bab(net, root, **kw)
    torch.cuda.synchronize()
    ms = 1000 * (time.perf_counter() - t0) / a.steps
    out = {
        "metric": f"branch-and-bound subproblems bounded/sec ({a.config} conv net, {Bs} splits per round, "
                  f"160 iters per child)",
        "value": r["bounded"] / (ms / 1000.0),
        "unit": "subproblems/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{a.config} conv net 3x32x32, one property, minimisation for {rounds} rounds of "
                               f"{Bs} splits, root 500 steps, children 160 steps", "splits_per_round": Bs,
                   "rounds": rounds},
        "result": {k: v for k, v in r.items() if k != "x_best"},
        "roofline": None,
    }
    print(json.dumps(out), flush=True)


def src_hash():
    """Hash of the HIP sources (a stored counter measurement is valid for these sources only)."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2104_06718_amd", "csrc")
    for f in sorted(os.listdir(d)):
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def stored_traffic(kernel, kind, config, B, prec):
    """HBM bytes per launch of `kernel` from the committed counter measurement
    (profiles/traffic.json: FETCH_SIZE + WRITE_SIZE scaled by a copy-kernel
    calibration), if it was taken on the current sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    key = f"{config}/B={B}/{prec}/{kernel}/slot{kind}"
    e = rec.get("kernels", {}).get(key)
    if e is None or rec.get("src_hash") != src_hash():
        return None
    return e["bytes_per_launch"]


def split_shares(B, props):
    """B subdomains split over properties in proportion to their counts: the floor of
    each exact share (at least one), the rest by largest remainder (ties to the
    earlier property); any excess from the minimum of one comes off the largest."""
    if B < len(props):
        raise ValueError(f"B = {B} is smaller than the number of properties ({len(props)})")
    total = sum(props)
    exact = [B * p / total for p in props]
    share = [max(1, int(e)) for e in exact]
    left = B - sum(share)
    order = sorted(range(len(props)), key=lambda i: (-(exact[i] - int(exact[i])), i))
    for i in order[:max(left, 0)]:
        share[i] += 1
    while sum(share) > B:
        share[share.index(max(share))] -= 1
    return share


def profile_summary(a):
    """Per-launch summary of the counter and trace runs of `bench.py --profile-only`
    (or of the bench line with --calibrate-copy, whose last contraction launches are
    its BF16 per-launch timing): the last 6 x (reps + 1) launches of the library's
    contraction kernels are one iteration's slots (101..103, 301..303 for the
    4-layer nets), each a warm-up and `reps` timed launches; the first of each group
    is dropped.  HBM bytes are FETCH_SIZE and WRITE_SIZE (KiB per dispatch) scaled by
    what the counters read for the 1 GiB device copy the run starts with."""
    import csv
    import collections
    import ldgen
    d = a.profile_summary
    prec = os.path.basename(os.path.normpath(d)).split("_")[-1]
    inst = make_workload(ldgen, a.config, a.B)
    B = inst.B
    n = len(inst.layers)
    slots = [100 + k for k in range(1, n)] + [300 + k for k in range(1, n)]
    per = a.reps + 1
    keep = ("conv_plane", "convT", "fc_kernel", "fc_split")

    def groups(rows, key):
        rows = sorted(rows, key=lambda r: int(r["Dispatch_Id"]))
        rows = [r for r in rows if any(k in r["Kernel_Name"] for k in keep)][-len(slots) * per:]
        out = {}
        for i, sl in enumerate(slots):
            g = rows[i * per + 1:(i + 1) * per]
            out[sl] = (g[0]["Kernel_Name"].split("(")[0].replace("void ld::", ""), [key(r) for r in g])
        return out

    def counters(sub):
        path = os.path.join(d, sub, "run_counter_collection.csv")
        if not os.path.exists(path):
            return None, None
        by = collections.defaultdict(lambda: collections.defaultdict(float))
        meta = {}
        with open(path) as fh:
            for r in csv.DictReader(fh):
                did = int(r["Dispatch_Id"])
                by[did][r["Counter_Name"]] += float(r["Counter_Value"])
                meta[did] = r
        # the calibration: the largest device copy of the run (the 1 GiB copy)
        cps = [i for i in meta if "copyBuffer" in meta[i]["Kernel_Name"] and int(meta[i]["Grid_Size"]) >= (1 << 17)]
        copy = dict(by[max(cps, key=lambda i: int(meta[i]["Grid_Size"]))]) if cps else {}
        rows = [dict(meta[i], **{"_c": by[i]}) for i in meta]
        return groups(rows, lambda r: r["_c"]), copy

    with open(os.path.join(d, "T", "run_kernel_trace.csv")) as fh:
        tr = groups(list(csv.DictReader(fh)), lambda r: (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    F, cf = counters("F")
    W, cw = counters("W")
    M, _ = counters("M")
    # every run must have timed the same kernel in each slot (pin the tiles across runs)
    for nm, X in (("F", F), ("W", W), ("M", M)):
        if X:
            for sl in slots:
                if X[sl][0] != tr[sl][0]:
                    print(f"WARNING: slot {sl}: run {nm} launched {X[sl][0]}, the trace run {tr[sl][0]}")
    gib = 1 << 30
    ff = gib / (cf["FETCH_SIZE"] * 1024) if cf else None
    fw = gib / (cw["WRITE_SIZE"] * 1024) if cw else None
    print(f"Counter calibration (1 GiB device copy): FETCH_SIZE x {ff:.4f}, WRITE_SIZE x {fw:.4f} (x 1024 bytes).\n")
    print("| slot | kernel | trace us/launch | HBM read MB | HBM write MB | floor share MB | frac of HBM (floor share / trace) "
          "| traffic / floor share | MFMA TFLOP/s (algorithmic) | MFMA TFLOP/s (executed) | MFMA busy / CU busy |")
    print("|---|---|---|---|---|---|---|---|---|---|")
    rec = {}
    tot_t = tot_b = tot_f = 0.0
    for sl in slots:
        name, ts = tr[sl]
        us = sum(ts) / len(ts)
        rd = sum(c["FETCH_SIZE"] for c in F[sl][1]) / len(F[sl][1]) * 1024 * ff if F else float("nan")
        wr = sum(c["WRITE_SIZE"] for c in W[sl][1]) / len(W[sl][1]) * 1024 * fw if W else float("nan")
        share = floor_share(inst, sl, B)
        _, flops = layer_slot_cost(inst, sl, B, prec)
        if M:
            # MOPS counters count MFMA work in units of 512 flops
            ex = sum((c.get("SQ_INSTS_VALU_MFMA_MOPS_BF16", 0.0) + c.get("SQ_INSTS_VALU_MFMA_MOPS_F32", 0.0)) * 512
                     for c in M[sl][1]) / len(M[sl][1])
            busy = sum(c.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) for c in M[sl][1]) / max(
                1.0, sum(c.get("SQ_BUSY_CU_CYCLES", 0.0) for c in M[sl][1]))
            ex_s, busy_s = f"{ex / (us * 1e-6) / 1e12:.1f}", f"{busy:.3f}"
        else:
            ex_s = busy_s = "n/a"
        print(f"| {sl} | {name} | {us:.2f} | {rd / 1e6:.2f} | {wr / 1e6:.2f} | {share / 1e6:.2f} | "
              f"{share / (us * 1e-6) / 1e9 / PEAK_HBM_GBS:.3f} | {(rd + wr) / share:.2f} | "
              f"{flops / (us * 1e-6) / 1e12:.1f} | {ex_s} | {busy_s} |")
        tot_t += us
        tot_b += rd + wr
        tot_f += share
        kname = name.split("<")[0]
        rec[f"{a.config}/B={B}/{prec}/{kname}/slot{sl}"] = {"kernel": name, "bytes_per_launch": rd + wr,
                                                              "fetch_bytes": rd, "write_bytes": wr}
    print(f"\nIteration: {tot_t:.1f} us over the {len(slots)} launches, {tot_b / 1e6:.1f} MB of HBM traffic against a "
          f"floor of {tot_f / 1e6:.1f} MB ({tot_b / tot_f:.2f}x); floor / time = "
          f"{tot_f / (tot_t * 1e-6) / 1e9 / PEAK_HBM_GBS:.3f} of HBM.")
    if a.write_traffic:
        path = os.path.join(ROOT, "profiles", "traffic.json")
        old = {}
        if os.path.exists(path):
            with open(path) as fh:
                old = json.load(fh)
        ks = old.get("kernels", {}) if old.get("src_hash") == src_hash() else {}
        ks.update(rec)
        with open(path, "w") as fh:
            json.dump({"src_hash": src_hash(),
                       "note": "bytes per launch = FETCH_SIZE*fetch_factor + WRITE_SIZE*write_factor (KiB -> "
                               "bytes), from the counter runs of bench.py --profile-only; valid for the sources "
                               "with this hash", "kernels": ks}, fh, indent=1)


def make_workload(ldgen, config, B):
    """The configuration's instance; with B, one GPU's share of it: for a config of
    several properties, B subdomains split over the properties in proportion to
    their counts (at least one each)."""
    if not B:
        return ldgen.make_instance(config)
    props = ldgen.CONFIGS[config]["props"]
    if len(props) == 1:
        return ldgen.make_instance(config, B=B)
    return ldgen.make_instance(config, props=split_shares(B, props))


def main():
    a = parse()
    if a.profile_summary:
        profile_summary(a)
        return
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); the subdomain batch would be "
              f"sharded across GPUs with no communication until a final all-gather, which is not built.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import ldgen
    import paper_2104_06718_amd as P

    inst = make_workload(ldgen, a.config, a.B)
    T = a.iters or inst.meta["T"] or 500
    B = inst.B
    net = P.Net(inst.layers)
    batch = P.Batch.from_instance(inst)
    P.set_validation(False)

    if a.solver == "prox" and not a.profile_only:
        main_prox(a, P, inst, net, batch)
        return
    if a.solver == "interm":
        main_interm(a, P, inst)
        return
    if a.solver == "fsb":
        main_fsb(a, P, inst, net, batch)
        return
    if a.solver == "sigmoid":
        main_sigmoid(a, P, inst)
        return
    if a.solver == "bab":
        main_bab(a, P, inst)
        return

    if a.profile_only or a.calibrate_copy:
        # counter calibration: a 1 GiB device copy (far larger than L2 and the MALL)
        x = torch.ones(256 << 20, device="cuda", dtype=torch.float32)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    if a.profile_only:
        stp = P.State(net, B)
        if a.solver == "prox":
            P.autotune(net, batch, precision=a.profile_only)
            Tp = a.iters or 100
            P.prox_step(net, batch, stp, iters=2, total_iters=Tp, precision=a.profile_only)
            slots = P.prox_profile_iteration(net, batch, stp, reps=a.reps, total_iters=Tp, precision=a.profile_only)
            name = lambda info, k: prox_kernel_name(info, k, inst, a.profile_only)  # noqa: E731
        else:
            if a.pin_tiles:
                pin_tiles(P, net, batch, a.profile_only, a.pin_tiles)
            P.step(net, batch, stp, iters=2, total_iters=T, precision=a.profile_only)
            slots = P.profile_iteration(net, batch, stp, reps=a.reps, total_iters=T, precision=a.profile_only)
            name = lambda info, k: kernel_name(info, k, inst, a.profile_only)  # noqa: E731
        torch.cuda.synchronize()
        info = P.tuning_info(net, B, a.profile_only)
        print(json.dumps({"profile_only": a.profile_only, "solver": a.solver, "config": a.config, "B": B,
                          "reps": a.reps, "slots": [[k, name(info, k), round(v, 2)] for k, v in slots],
                          "tuned": info}), flush=True)
        return

    if a.pin_tiles:
        for prec in ("fp32", "bf16"):
            pin_tiles(P, net, batch, prec, a.pin_tiles)
    st = P.State(net, B)
    res32 = run_form(P, net, batch, st, T, "fp32", a.steps, a.warmup, a.engine)
    b32 = res32["fb"]["bound"].clone()
    # rounding margin of the FP32-operand value at rho^T (after the timed runs)
    m32 = P.rounding_margin(net, batch, st.get_rho())
    q32 = res32["fb"]["q_final"]
    margin = {"max": m32.max().item(), "max_over_abs_q": (m32 / q32.abs().clamp(min=1e-30)).max().item()}

    # BF16 form: iterations needed to reach the FP32 form's bound (mean gap <= 1e-3):
    # bracketed upward from T in steps of 50, then bisected down to 5 iterations
    st16 = P.State(net, B)
    T16 = a.bf16_iters or T
    tries = []
    if not a.quick and a.bf16_iters is None:
        def reaches(t):
            st16.reset()
            P.step(net, batch, st16, iters=t, total_iters=t, precision="bf16", engine=a.engine)
            bb = P.final_bound(net, batch, st16)["bound"]
            gap = (b32 - bb).mean().item()
            tries.append((t, round(gap, 6)))
            return gap <= 1e-3
        lo, hi, t = None, None, T
        while t <= 3 * T:
            if reaches(t):
                hi = t
                break
            lo, t = t, t + 50
        if hi is not None and lo is not None:
            while hi - lo > 5:
                mid = (lo + hi) // 2
                if reaches(mid):
                    hi = mid
                else:
                    lo = mid
        T16 = hi if hi is not None else tries[-1][0]
    res16 = run_form(P, net, batch, st16, T16, "bf16", a.steps, a.warmup, a.engine)
    b16 = res16["fb"]["bound"]
    d = (b16 - b32)
    equal = (b32 - b16).mean().item() <= 1e-3

    # FP64 engine: the same run with FP64 operands, accumulations and state
    st64 = P.State(net, B)
    res64 = run_form(P, net, batch, st64, T, "fp64", max(1, min(a.steps, 3)), min(a.warmup, 1), a.engine)

    # per-launch timing of one iteration (HIP events around every launch, same stream)
    stp = P.State(net, B)
    prof = {}
    for prec in ("fp32", "bf16"):
        stp.reset()
        P.step(net, batch, stp, iters=5, total_iters=T, precision=prec)
        prof[prec] = P.profile_iteration(net, batch, stp, reps=20, total_iters=T, precision=prec)
    head = "bf16"
    slots = prof[head]
    kind, us = max(slots, key=lambda x: x[1])
    tuned = {p: P.tuning_info(net, B, p) for p in ("fp32", "bf16")}
    nbytes, flops = layer_slot_cost(inst, kind, B, head)
    share = floor_share(inst, kind, B)
    roof = dict(bound="hbm", achieved=share / (us * 1e-6) / 1e9, peak=PEAK_HBM_GBS, unit="GB/s")
    roof["frac"] = roof["achieved"] / roof["peak"]
    kname = kernel_name(tuned[head], kind, inst, head)
    roof["traffic"] = stored_traffic(kname, kind, a.config, B, head)
    roof["kernel"] = f"{kname}: slot {kind} (phase {kind // 100}, layer {kind % 100})"
    roof["avg_us"] = us
    roof["algorithmic_bytes"] = share
    roof["traffic_over_algorithmic"] = roof["traffic"] / share if roof["traffic"] else None
    # the whole iteration against the same floor: the sum of its launches, and the
    # bounding run's time per iteration (initialisation and final bound included)
    floor = state_floor(inst, B)
    it_us = sum(v for _, v in slots)
    run_it_us = 1000.0 * res16["ms_per_step"] / T16
    roof["iteration"] = {"floor_bytes": floor, "sum_of_launches_us": it_us,
                         "frac_sum_of_launches": floor / (it_us * 1e-6) / 1e9 / PEAK_HBM_GBS,
                         "run_us_per_iteration": run_it_us,
                         "frac_run": floor / (run_it_us * 1e-6) / 1e9 / PEAK_HBM_GBS}
    # the launch's contraction on MFMA (algorithmic FLOPs, BF16 dense peak)
    roof["mfma"] = {"flops": flops, "achieved_tflops": flops / (us * 1e-6) / 1e12,
                    "peak_tflops": PEAK_TFLOPS[head], "frac": flops / (us * 1e-6) / 1e12 / PEAK_TFLOPS[head]}
    roof["bytes_with_intermediates"] = nbytes
    roof["per_slot"] = {str(k): {"us": round(v, 2), "floor_bytes": floor_share(inst, k, B),
                                 "frac": floor_share(inst, k, B) / (v * 1e-6) / 1e9 / PEAK_HBM_GBS}
                        for k, v in slots}

    def pct(x):
        q = torch.quantile(x.double().cpu(), torch.tensor([0.5, 0.9, 0.99], dtype=torch.float64))
        return {"p50": q[0].item(), "p90": q[1].item(), "p99": q[2].item(), "max": x.abs().max().item()}

    value = B / (res16["ms_per_step"] / 1000.0)
    out = {
        "metric": "LD bounds/sec (500 iters, B=512, wide conv net); bf16 vs fp32 at equal bound",
        "value": value,
        "unit": "bounds/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": res16["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": f"{a.config} conv net 3x32x32, B={B}, T={T} (bf16: T={T16}), 1 property, "
                               f"5% random ReLU splits per subdomain", "B": B, "iters": T, "bf16_iters": T16},
        "fp32": {"value": B / (res32["ms_per_step"] / 1000.0), "ms_per_step": res32["ms_per_step"],
                 "mean_bound": b32.mean().item(), "rounding_margin_at_rhoT": margin},
        "bf16": {"value": value, "ms_per_step": res16["ms_per_step"], "mean_bound": b16.mean().item(),
                 "equal_bound": equal,
                 "equal_bound_criterion": "mean over subdomains of (fp32 bound - bf16 bound) <= 1e-3",
                 "gap_mean": d.mean().item(), "abs_gap": pct(d.abs()),
                 "frac_within_1e-3": (d.abs() <= 1e-3).float().mean().item(), "search": tries},
        "fp64": {"value": B / (res64["ms_per_step"] / 1000.0), "ms_per_step": res64["ms_per_step"],
                 "mean_bound": res64["fb"]["bound"].mean().item()},
        "roofline": roof,
        "per_launch_us": {p: {str(k): round(v, 2) for k, v in prof[p]} for p in prof},
        "tuned": tuned,
    }
    if not a.no_cpu_baseline:
        cb, idx, ob = cpu_baseline(inst, T, a.cpu_sample)
        out["cpu_baseline"] = cb
        # the BF16 form may run more iterations: compare it with the oracle at its own count
        ob16 = ob if T16 == T else cpu_baseline(inst, T16, a.cpu_sample)[2]
        for p, r, o, t in (("fp32", res32, ob, T), ("bf16", res16, ob16, T16), ("fp64", res64, ob, T)):
            dd = r["fb"]["bound"].cpu()[idx] - o
            out[p]["minus_oracle"] = {"mean": dd.mean().item(), "abs": pct(dd.abs()),
                                      "subdomains": len(idx), "oracle_iters": t}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
