#!/usr/bin/env python3
"""Single-bond QR+CBE TEBD benchmark on one MI355X.

Workload (the single-bond microbenchmark): a uniform two-site cell with d = 5,
chi = 1024, A and B Gaussian right-isometric [chi, d, chi], random positive
bond weights, the clock-model gate U = expm(-i 0.05 h_bond) (g = 2), and
controlled bond expansion with eta = chi + ceil(chi/10) truncated back to
chi~ = chi.  One step = one bond update (Sec. II/III of the paper), bonds
alternating (A,B), (B,A); consecutive updates are dependent, so throughput is
1 / latency.  Both precisions are timed: complex128 (FP64 throughout) and the
mixed path (complex64 storage, FP32 matrix cores, FP64 panels / eig /
re-orthogonalisation / normalisation).  `value` is the mixed path's rate.

Prints one JSON line (see the keys below).  --gpus above 1 is refused: the
benchmark runs on one GPU.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK = 8.0e12
PEAK = {"c128": 78.6e12, "c64": 157.3e12}   # dense FP64 / FP32 matrix-core peaks (MI355X)
# HBM bytes per launch of the mixed path's contraction GEMM (mean over its five
# launches per update), from rocprofv3 FETCH_SIZE and WRITE_SIZE scaled by the
# same counters read for a plain 256 MiB copy (--copy-calibration); the
# commands and raw figures are in profiles/contract_gemm_hbm_d5_chi1024_mixed.md.
# Only valid for the kernel version those counters were taken on.
CONTRACT_TRAFFIC_C64 = 1.3325e9


def run_precision(lib, torch, prec, chi, d, steps, warmup, sweeps=1):
    ctx = lib.Context(0)
    A, B, lA, lB = inputs_cell(chi, d)
    U = lib.clock_gate(d, 2.0, 0.05)
    eta = chi + -(-chi // 10)
    cdt = torch.complex128 if prec == lib.MPS_C128 else torch.complex64
    dev = lambda a, t=None: torch.from_numpy(np.ascontiguousarray(a).reshape(-1)).to(t or torch.float64).to("cuda")
    bufA = [dev(A, cdt), torch.empty(chi * d * chi, dtype=cdt, device="cuda")]
    bufB = [dev(B, cdt), torch.empty(chi * d * chi, dtype=cdt, device="cuda")]
    lam = {"A": dev(lA), "B": dev(lB)}
    du = dev(U, torch.complex128)
    chi_dev = torch.zeros(1, dtype=torch.int32, device="cuda")
    eps_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    desc = lib.bond_desc(d, chi, chi, chi, eta, chi, 1e-14 if prec == lib.MPS_C128 else 1e-6, True, lib.CBE, prec,
                         sweeps)
    state = {"a": 0, "b": 0}

    def one(k):
        # even k: bond (A, B) with Xi = Lambda_A; odd k: bond (B, A) with Xi = Lambda_B
        if k % 2 == 0:
            src_m, src_n, xi, new_xi = bufA[state["a"]], bufB[state["b"]], lam["A"], lam["B"]
            dst_m, dst_n = bufA[1 - state["a"]], bufB[1 - state["b"]]
        else:
            src_m, src_n, xi, new_xi = bufB[state["b"]], bufA[state["a"]], lam["B"], lam["A"]
            dst_m, dst_n = bufB[1 - state["b"]], bufA[1 - state["a"]]
        lib.mps_bond_update(ctx, desc, xi, src_m, src_n, du, dst_m, new_xi, dst_n, chi_dev, eps_dev)
        state["a"], state["b"] = 1 - state["a"], 1 - state["b"]

    for k in range(warmup):
        one(k)
    ctx.sync()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    ctx.profile_enable(True, 16 * steps + 16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record()
        one(warmup + k)
        ev[k][1].record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    gemm_ms, gemm_flops, launches = ctx.profile_read()
    ctx.profile_enable(False)
    ctx.sync()
    lat = np.array([a.elapsed_time(b) for a, b in ev])
    chi_new = int(chi_dev.item())
    eps = float(eps_dev.item())
    ctx.close()
    return dict(
        updates_per_s=steps / (t1 - t0),
        ms_per_step=1e3 * (t1 - t0) / steps,
        p50_ms=float(np.percentile(lat, 50)),
        p99_ms=float(np.percentile(lat, 99)),
        gemm_ms=gemm_ms, gemm_flops=gemm_flops, gemm_launches=launches,
        chi_new=chi_new, last_eps=eps,
    )


def inputs_cell(chi, d):
    from paper_2212_09782_amd import inputs
    return inputs.microbench_cell(chi, d, seed=0)


def cpu_baseline(chi, d, budget_s):
    """The oracle (numpy, complex128) on this host's cores: a bounded sample of the same workload."""
    from oracle import bond as obond
    from paper_2212_09782_amd import inputs
    from oracle import clock
    A, B, lA, lB = inputs.microbench_cell(chi, d, seed=0)
    U = clock.gate(clock.bond_hamiltonian(d, 2.0), 0.05)
    eta = chi + -(-chi // 10)
    n = 0
    t0 = time.perf_counter()
    while True:
        obond.qr_bond_update(lA, A, B, U, mode=obond.CBE, eta=eta, chi_max=chi)
        n += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": n / dt, "unit": "bond updates/s", "cores": cores, "kind": "oracle",
            "sample": f"{n} QR+CBE update(s) at d={d} chi={chi} eta={eta}, complex128 numpy/LAPACK, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--chi", type=int, default=1024)
    ap.add_argument("--d", type=int, default=5)
    ap.add_argument("--prec", choices=["both", "c128", "mixed"], default="both")
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle time (0: skip)")
    ap.add_argument("--sweeps", type=int, default=1, help="QR/LQ sweeps per update (1: the paper's single sweep)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 256 MiB three times (reference run for the HBM byte counters)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        x = torch.ones(64 * 2**20, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print("copied 3 x 256 MiB", flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU; --gpus {args.gpus} is not supported (the bond update is a "
              "single-GPU kernel pipeline; multi-GPU sharding is a design note only)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2212_09782_amd import lib
    lib.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    res = {}
    if args.prec in ("both", "c128"):
        res["c128"] = run_precision(lib, torch, lib.MPS_C128, args.chi, args.d, args.steps, args.warmup, args.sweeps)
    if args.prec in ("both", "mixed"):
        res["c64"] = run_precision(lib, torch, lib.MPS_MIXED_C64, args.chi, args.d, args.steps, args.warmup,
                                   args.sweeps)
    head = "c64" if "c64" in res else "c128"
    h = res[head]
    achieved = h["gemm_flops"] / (h["gemm_ms"] * 1e-3) if h["gemm_ms"] > 0 else 0.0
    line = {
        "metric": f"bond updates/s at d={args.d} chi={args.chi} (mixed vs FP64) + p50/p99 step latency",
        "value": round(h["updates_per_s"], 4),
        "unit": "bond updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(h["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64" if head == "c64" else "c128",
        "data": "synthetic",
        "config": {"workload": f"single-bond QR+CBE update, uniform two-site cell, d={args.d}, chi={args.chi}, "
                               f"eta={args.chi + -(-args.chi // 10)}, chi~={args.chi}, clock gate g=2 dt=0.05"
                               + (f", {args.sweeps} QR/LQ sweeps" if args.sweeps > 1 else ""),
                   "d": args.d, "chi": args.chi, "eta": args.chi + -(-args.chi // 10), "sweeps": args.sweeps},
        "p50_ms": round(h["p50_ms"], 4),
        "p99_ms": round(h["p99_ms"], 4),
        "per_precision": {k: {kk: (round(vv, 6) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                          for k, v in res.items()},
        "roofline": {
            "kernel": ("contract_gemm_kernel<float, float, float>" if head == "c64" else "contract_gemm_kernel<double, double, double>")
                      + " (the 5 contraction GEMMs of each update)",
            "bound": "mfma",
            "achieved": round(achieved / 1e12, 3),
            "peak": round(PEAK[head] / 1e12, 1),
            "unit": "TFLOP/s",
            "frac": round(achieved / PEAK[head], 4),
            "traffic": CONTRACT_TRAFFIC_C64 if head == "c64" else None,
        },
    }
    if args.cpu_budget > 0:
        line["cpu_baseline"] = cpu_baseline(args.chi, args.d, args.cpu_budget)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
