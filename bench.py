#!/usr/bin/env python3
"""Single-bond QR+CBE TEBD benchmark on one MI355X.

Workload (the single-bond microbenchmark): a uniform two-site cell with d = 5,
A and B Gaussian right-isometric [chi, d, chi], random positive bond weights,
the clock-model gate U = expm(-i 0.05 h_bond) (g = 2), and controlled bond
expansion with eta = chi + ceil(chi/10) truncated back to chi~ = chi.  One
step = one bond update (Sec. II/III of the paper), bonds alternating (A,B),
(B,A); consecutive updates are dependent, so throughput is 1 / latency.

Both precisions are timed at every chi of --chis: complex128 (FP64
throughout, the paper's precision) and the mixed path (complex64 storage,
FP32 matrix cores, FP64 panels / eig / re-orthogonalisation /
normalisation).  `value` is the complex128 rate at the first chi (1024 by
default); the mixed rate, its ratio to complex128 and both precisions'
roofline objects are in `per_precision`, the other chis in `per_chi`.

Prints one JSON line.  --gpus above 1 is refused: the benchmark runs on one
GPU.
"""
import argparse
import collections
import csv
import glob
import hashlib
import json
import math
import os
import re
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"c128": 78.6e12, "c64": 157.3e12}   # dense FP64 / FP32 matrix-core peaks (MI355X)
KERNEL = {"c128": "contract_gemm_kernel<double, double, double>", "c64": "contract_gemm_kernel<float, float, float>"}
GEMM_SOURCES = ["paper_2212_09782_amd/csrc/gemm.hip", "paper_2212_09782_amd/csrc/gemm.h",
                "paper_2212_09782_amd/csrc/common.h"]
# HBM bytes per launch of the contraction GEMM at d=5, chi=1024 (mean over the
# five launches of an update), from rocprofv3 FETCH_SIZE and WRITE_SIZE scaled
# by the same counters read for a plain 256 MiB copy (--copy-calibration); the
# commands and raw figures are in profiles/contract_gemm_hbm_d5_chi1024.md.
# Each figure holds only for the kernel sources it was counted on (sha256 of
# GEMM_SOURCES): after a change to them the bench reports traffic null.
TRAFFIC = {
    "c64": (1.3267e9, "07b071944365dbea"),
    "c128": (2.6850e9, "07b071944365dbea"),
}


def gemm_source_hash():
    h = hashlib.sha256()
    for p in GEMM_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def run_precision(lib, torch, prec, chi, d, steps, warmup, sweeps=1, autotune=None):
    from paper_2212_09782_amd import inputs
    ctx = lib.Context(0, autotune_cache=autotune)
    A, B, lA, lB = inputs.microbench_cell(chi, d, seed=0)
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
    stream = torch.cuda.current_stream()

    def one(k):
        # even k: bond (A, B) with Xi = Lambda_A; odd k: bond (B, A) with Xi = Lambda_B
        if k % 2 == 0:
            src_m, src_n, xi, new_xi = bufA[state["a"]], bufB[state["b"]], lam["A"], lam["B"]
            dst_m, dst_n = bufA[1 - state["a"]], bufB[1 - state["b"]]
        else:
            src_m, src_n, xi, new_xi = bufB[state["b"]], bufA[state["a"]], lam["B"], lam["A"]
            dst_m, dst_n = bufB[1 - state["b"]], bufA[1 - state["a"]]
        lib.mps_bond_update(ctx, desc, xi, src_m, src_n, du, dst_m, new_xi, dst_n, chi_dev, eps_dev, stream)
        state["a"], state["b"] = 1 - state["a"], 1 - state["b"]

    for k in range(warmup):
        one(k)
    ctx.sync()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    ctx.profile_enable(True, 16 * steps + 16)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record(stream)
        one(warmup + k)
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # HIP events the library recorded on `stream` around each contraction launch
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


def chain_contraction_flops(chis, d, chi_max, dchi_min, dchi_frac, order=2):
    """Algorithmic flops (8 per complex MAC) of the five contractions of every
    bond update of one Trotter step on a finite chain with this (saturated)
    profile: C = B B, X = theta~ Y0^dag, Y^dag = theta~^dag Q, B~[n], B~[m]."""
    L = len(chis) - 1
    layers = [0, 1, 0] if order == 2 else [0, 1]
    total = 0.0
    for parity in layers:
        for m in range(parity, L - 1, 2):
            cl, cm, cr = chis[m], chis[m + 1], chis[m + 2]
            ml, mr = d * cl, d * cr
            eta = min(cm + max(dchi_min, math.ceil(dchi_frac * cm)), ml, mr)
            k = min(eta, chi_max)
            total += 8.0 * (ml * mr * cm + 2 * ml * eta * mr + k * mr * eta + ml * k * mr)
    return total


def run_chain(lib, torch, prec, L, d, chi_max, steps, warmup, exec_mode, autotune=None):
    """Steady-state throughput of the batched finite chain: a random
    right-isometric MPS at the saturated profile min(d^b, d^(L-b), chi_max)
    (every bond matrix diagonal, random positive, unit norm), the Z_d clock
    gates (g = 2, dt = 0.05), second-order steps: every even bond in one
    layer, then every odd bond, then the even bonds again."""
    from paper_2212_09782_amd import inputs
    ctx = lib.Context(0, autotune_cache=autotune)
    mps = inputs.random_finite_mps(L, d, chi_max, seed=4)
    st = lib.State(ctx, mps["B"], mps["Xi"], finite=True, chi_cap=chi_max, prec=prec)
    gates = lib.chain_gates(d, 2.0, L, True, 0.05)
    svd_min = 1e-14 if prec == lib.MPS_C128 else 1e-6
    pol = lib.sweep_policy(chi_max, svd_min, 0, 0.1, exec=exec_mode, chunk=max(1, steps))
    stream = torch.cuda.current_stream()
    lib.mps_sweep(ctx, [st], [gates], warmup, 2, pol, stream=stream)
    ctx.sync()
    before = lib.sweep_stats(ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lib.mps_sweep(ctx, [st], [gates], steps, 2, pol, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.sync()
    after = lib.sweep_stats(ctx)
    chis = st.chis()
    st.close()
    ctx.close()
    updates = steps * (2 * ((L - 1 + 1) // 2) + (L - 1) // 2)
    flops = steps * chain_contraction_flops(chis, d, chi_max, 0, 0.1)
    return dict(updates_per_s=updates / (t1 - t0), ms_per_step=1e3 * (t1 - t0) / steps,
                ms_per_layer=1e3 * (t1 - t0) / (3 * steps), contraction_tflops=flops / (t1 - t0) / 1e12,
                chis_saturated=chis == [1] + inputs.chi_profile_finite(L, d, chi_max) + [1],
                stats={k: after[k] - before[k] for k in after})


def run_serve(lib, torch, nreq, rate, nsteps, prec, slots, max_batch, budget_bytes):
    """The serving loop on the Poisson request stream (serve.Engine): requests
    of random d, g, chi_max and geometry, admitted by HBM budget, batched
    across requests, each run for nsteps second-order steps from |0...0>."""
    from paper_2212_09782_amd import inputs, serve
    specs = inputs.serving_requests(n=nreq, rate=rate, seed=5)
    reqs = serve.requests_from_stream(specs, nsteps=nsteps, prec=prec)
    execs = [serve.Executor(0) for _ in range(slots)]
    t0 = time.perf_counter()

    def progress(r, eng):
        print(f"# request {r.rid} done at {time.perf_counter() - t0:.1f} s "
              f"({len(eng.finished)}/{nreq}; d={r.d} chi_max={r.chi_max} L={r.L} "
              f"{'failed: ' + r.result.get('error', '') if r.result and r.result.get('failed') else ''})",
              file=sys.stderr, flush=True)

    eng = serve.Engine(execs, hbm_budget=budget_bytes, max_batch=max_batch, on_finish=progress)
    rep = eng.run(reqs)
    for ex in execs:
        ex.close()
    rep["final_chi_max"] = {str(r.rid): max(r.result["chis"]) for r in reqs if r.result and "chis" in r.result}
    rep["errors"] = eng.errors[:5]
    return rep


def run_quench(lib, torch, prec, d, g, chi_max, steps, dt, dchi_min, exec_mode, autotune=None):
    """Uniform two-site cell quenched from |0...0> (second-order steps):
    <Z + Z^dag> on both sites and both bond energies after every step."""
    ctx = lib.Context(0, autotune_cache=autotune)
    e0 = np.zeros((1, d, 1), np.complex128)
    e0[0, 0, 0] = 1
    st = lib.State(ctx, [e0, e0], [np.ones(1), np.ones(1)], finite=False, chi_cap=chi_max, prec=prec)
    gates = lib.chain_gates(d, g, 2, False, dt)
    pol = lib.sweep_policy(chi_max, 1e-14 if prec == lib.MPS_C128 else 1e-6, dchi_min, 0.1, exec=exec_mode)
    w = np.exp(2j * np.pi * np.arange(d) / d)
    zz = torch.from_numpy((np.diag(w) + np.diag(w.conj())).reshape(-1)).to("cuda")
    hb = torch.from_numpy(lib.clock_hamiltonian(d, g).reshape(-1)).to("cuda")
    site = torch.zeros(4, dtype=torch.float64, device="cuda")
    bond = torch.zeros(4, dtype=torch.float64, device="cuda")
    eps = torch.zeros(1, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    z, e, chis = [], [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        lib.mps_sweep(ctx, [st], [gates], 1, 2, pol, trunc_err=eps, stream=stream)
        lib.mps_measure(ctx, st, op1=zz, op2=hb, site_vals=site, bond_vals=bond, stream=stream)
        ctx.sync(stream)
        z.append(site.cpu().numpy().reshape(2, 2)[:, 0].copy())
        e.append(bond.cpu().numpy().reshape(2, 2)[:, 0].copy())
        chis.append(max(st.chis()))
        if len(z) % 10 == 0:
            print(f"#   step {len(z)}: chi {chis[-1]}, <Z+Z^dag> {z[-1][0]:.6f}, {time.perf_counter() - t0:.1f} s",
                  file=sys.stderr, flush=True)
    t1 = time.perf_counter()
    eps_sum = float(eps.item())
    st.close()
    ctx.close()
    return dict(z=np.array(z), e=np.array(e), chis=chis, eps_sum=eps_sum, seconds=t1 - t0)


def run_sym(lib, torch, prec, chi, d, steps, warmup):
    """The microbenchmark cell with the Z_d block structure (charge basis):
    random symmetric right-isometric A, B with chi split evenly over the d
    charge sectors of both bonds, the clock gate (g = 2, dt = 0.05) in the
    charge basis, every sector expanded by ceil(sec/10) (at least 1), chi_max
    = chi.  Updates alternate between the bonds (A,B) and (B,A) on the evolving
    state; each reads its new sector sizes back (one synchronisation per
    update, inside the timed region)."""
    from paper_2212_09782_amd import inputs
    ctx = lib.Context(0)
    sec = inputs.sym_sectors(chi, d)
    _, A, B = inputs.random_sym_bond(sec, sec, sec, d, seed=0)
    r = inputs.rng(2)
    lam = [np.concatenate([np.sort(r.uniform(0, 1, n))[::-1] for n in sec]) for _ in range(2)]
    lam = [x / np.linalg.norm(x) for x in lam]
    cell = lib.SymCell(ctx, [A, B], lam, [sec, sec], chi_cap=chi + d, prec=prec)
    du = torch.from_numpy(lib.clock_gate_charge(d, 2.0, 0.05).reshape(-1)).to("cuda")
    svd_min = 1e-14 if prec == lib.MPS_C128 else 1e-6
    stream = torch.cuda.current_stream()
    for k in range(warmup):
        cell.update(k % 2, du, 1, 0.1, chi, svd_min, stream)
    lat = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        a = time.perf_counter()
        cell.update((warmup + k) % 2, du, 1, 0.1, chi, svd_min, stream)
        lat.append(time.perf_counter() - a)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    out = dict(updates_per_s=steps / (t1 - t0), ms_per_step=1e3 * (t1 - t0) / steps,
               p50_ms=1e3 * float(np.percentile(lat, 50)), p99_ms=1e3 * float(np.percentile(lat, 99)),
               sectors=cell.secs, chi=cell.chis())
    ctx.close()
    return out


def run_schemes(lib, torch, chi, ds, reps, budget_s):
    """Single-gate time of the four truncation schemes of the paper's
    comparison (Sec. IV) on the GPU, complex128: QR (plain, eta = chi), QR+CBE
    (eta = chi + ceil(chi/10)), EIG and SVD (rocSOLVER heevd / gesvd), on the
    microbenchmark cell at each d; a scheme is skipped at larger d once one
    gate took longer than budget_s."""
    from paper_2212_09782_amd import inputs
    ctx = lib.Context(0)
    out, slow = {}, set()
    for d in ds:
        A, B, lA, _ = inputs.microbench_cell(chi, d, seed=0)
        U = lib.clock_gate(d, 2.0, 0.05)
        dev = lambda a, t=torch.complex128: torch.from_numpy(np.ascontiguousarray(a).reshape(-1)).to(t).to("cuda")
        xi, bm, bn, du = dev(lA, torch.float64), dev(A), dev(B), dev(U)
        row = {}
        for name in ("qr", "qr_cbe", "eig", "svd"):
            if name in slow:
                row[name] = None
                continue
            if name in ("qr", "qr_cbe"):
                eta = chi if name == "qr" else chi + -(-chi // 10)
                desc = lib.bond_desc(d, chi, chi, chi, eta, chi, 1e-14, True, lib.PLAIN if name == "qr" else lib.CBE)
                run = lambda: lib.bond_update(ctx, desc, xi, bm, bn, du)
            else:
                desc = lib.bond_desc(d, chi, chi, chi, 1, chi, 1e-14, True, lib.CBE)
                sch = lib.SCHEME_EIG if name == "eig" else lib.SCHEME_SVD
                run = lambda: lib.reference_update(ctx, desc, sch, xi, bm, bn, du)
            print(f"# schemes chi={chi} d={d} {name}", file=sys.stderr, flush=True)
            run()
            ctx.sync()
            times = []
            for _ in range(reps):
                t0 = time.perf_counter()
                run()
                ctx.sync()
                times.append(time.perf_counter() - t0)
                if times[-1] > budget_s:
                    break
            row[name] = 1e3 * float(np.median(times))
            if times[-1] > budget_s:
                slow.add(name)
        out[str(d)] = row
    ctx.close()
    return out


def roofline(r, key, traffic_ok):
    achieved = r["gemm_flops"] / (r["gemm_ms"] * 1e-3) if r["gemm_ms"] > 0 else 0.0
    tb = TRAFFIC[key][0] if traffic_ok.get(key) else None
    return {
        "kernel": KERNEL[key] + " (the 5 contraction GEMMs of each update)",
        "bound": "mfma",
        "achieved": round(achieved / 1e12, 3),
        "peak": round(PEAK[key] / 1e12, 1),
        "unit": "TFLOP/s",
        "frac": round(achieved / PEAK[key], 4),
        "traffic": tb,
        "avg_launch_us": round(1e3 * r["gemm_ms"] / max(1, r["gemm_launches"]), 2),
        "flops_per_launch": round(r["gemm_flops"] / max(1, r["gemm_launches"])),
    }


def _cpu_model():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        f = dict(re.findall(r"^([^:]+):\s*(.*)$", out, re.M))
        model = f.get("Model name", "?")
        phys = int(f.get("Core(s) per socket", "0")) * int(f.get("Socket(s)", "0"))
        return model, phys or None, int(f.get("CPU(s)", "0")) or None
    except Exception:
        return "?", None, os.cpu_count()


def cpu_baseline(chi, d, budget_s):
    """The oracle (numpy/LAPACK) on this host's cores: bounded samples of the same workload.

    Main leg: complex128 at the benchmark's chi with every BLAS thread (the
    figure in `value`).  Extra legs: the same update with complex64 inputs
    (the oracle computes in the inputs' precision), and complex128 on one
    thread at a quarter of the chi (a full-size update on one core takes tens
    of seconds; the rate is also given scaled by chi^3 to the benchmark's chi).
    """
    from threadpoolctl import threadpool_info, threadpool_limits
    from oracle import bond as obond
    from oracle import clock
    from paper_2212_09782_amd import inputs

    def leg(c, dtype, budget, min_n=1):
        A, B, lA, lB = inputs.microbench_cell(c, d, seed=0)
        U = clock.gate(clock.bond_hamiltonian(d, 2.0), 0.05)
        if dtype == "c64":
            A, B, U, lA = A.astype(np.complex64), B.astype(np.complex64), U.astype(np.complex64), lA.astype(np.float32)
        eta = c + -(-c // 10)
        n, t0 = 0, time.perf_counter()
        while True:
            obond.qr_bond_update(lA, A, B, U, mode=obond.CBE, eta=eta, chi_max=c)
            n += 1
            if n >= min_n and time.perf_counter() - t0 > budget:
                break
        return n, time.perf_counter() - t0, eta

    threads = max([i.get("num_threads", 1) for i in threadpool_info() if i.get("user_api") == "blas"] or [1])
    model, phys, logical = _cpu_model()
    n, dt, eta = leg(chi, "c128", budget_s * 0.5)
    out = {"value": n / dt, "unit": "bond updates/s", "cores": threads, "kind": "oracle",
           "sample": f"{n} QR+CBE update(s) at d={d} chi={chi} eta={eta}, complex128 numpy/LAPACK, "
                     f"{threads} BLAS threads, {dt:.1f} s",
           "cpu_model": model, "physical_cores": phys, "logical_cpus": logical}
    n, dt, _ = leg(chi, "c64", budget_s * 0.3)
    out["c64"] = {"value": n / dt, "threads": threads,
                  "sample": f"{n} update(s) at chi={chi} with complex64 inputs, {dt:.1f} s"}
    c1 = max(16, chi // 4)
    with threadpool_limits(limits=1, user_api="blas"):
        n, dt, _ = leg(c1, "c128", budget_s * 0.2)
    out["one_thread"] = {"value": n / dt, "chi": c1, "value_scaled_to_chi": (n / dt) * (c1 / chi) ** 3,
                         "sample": f"{n} complex128 update(s) at chi={c1} on 1 BLAS thread, {dt:.1f} s"}
    return out


# ---- rocprofv3 CSV summaries (profiles/ holds their output) ----

def _short(name):
    name = name.replace("(anonymous namespace)::", "").replace("qrtebd::", "").replace("void ", "")
    name = re.sub(r"\(.*$", "", name)
    return name

def trace_summary(d, out):
    """Per-kernel table of a rocprofv3 --kernel-trace CSV (the default bench):
    all dispatches, and per update over the 200 timed chi=1024 updates of each
    precision (found from the contraction launches); removes the raw CSV."""
    path = os.path.join(d, "run_kernel_trace.csv")
    rows = list(csv.DictReader(open(path)))
    ks = [k for k in rows[0].keys()]
    nk = "Kernel_Name"
    t0k, t1k = "Start_Timestamp", "End_Timestamp"
    rows.sort(key=lambda r: int(r[t0k]))
    by = collections.defaultdict(list)
    for r in rows:
        by[_short(r[nk])].append((int(r[t0k]), int(r[t1k])))
    lines = []
    tot = sum(b - a for v in by.values() for a, b in v)
    lines.append(f"all dispatches: {len(rows)}, total kernel time {tot/1e6:.2f} ms")
    lines.append("")
    lines.append("| kernel | calls | total ms | avg us |")
    lines.append("|---|--:|--:|--:|")
    for k, v in sorted(by.items(), key=lambda kv: -sum(b - a for a, b in kv[1]))[:25]:
        s = sum(b - a for a, b in v)
        lines.append(f"| `{k}` | {len(v)} | {s/1e6:.3f} | {s/len(v)/1e3:.2f} |")
    # the chi=1024 legs: contract launches 25..1024 of each precision's kernel are the timed updates
    for prec, kname in (("c128", "contract_gemm_kernel<double, double, double>"), ("mixed", "contract_gemm_kernel<float, float, float>")):
        v = by.get(kname, [])
        if len(v) < 1025:
            continue
        timed = v[25:1025]
        avg = sum(b - a for a, b in timed) / len(timed)
        lines.append("")
        lines.append(f"{prec}, chi=1024, timed updates: {kname} average {avg/1e3:.2f} us over {len(timed)} launches "
                     f"(launches 26-1025 of the kernel; the first 25 are the 5 warm-up updates)")
        # window: from the first timed contract launch to the last one, per-kernel time per update
        w0, w1 = timed[0][0], timed[-1][1]
        win = collections.defaultdict(lambda: [0, 0])
        for r in rows:
            a, b = int(r[t0k]), int(r[t1k])
            if a >= w0 and b <= w1:
                e = win[_short(r[nk])]
                e[0] += 1
                e[1] += b - a
        wt = sum(e[1] for e in win.values())
        lines.append(f"window of the 200 timed updates: {(w1 - w0)/1e6:.1f} ms wall, {wt/1e6:.1f} ms kernel time "
                     f"(two streams overlap); per update:")
        lines.append("")
        lines.append("| kernel | launches per update | ms per update | avg us |")
        lines.append("|---|--:|--:|--:|")
        for k, e in sorted(win.items(), key=lambda kv: -kv[1][1])[:16]:
            lines.append(f"| `{k}` | {e[0]/200:.1f} | {e[1]/200/1e6:.3f} | {e[1]/max(1,e[0])/1e3:.2f} |")
    open(out, "w").write("\n".join(lines) + "\n")
    os.remove(path)

def pmc_summary(d, out):
    """Per-kernel means of a rocprofv3 --pmc CSV; removes the raw CSV."""
    path = glob.glob(os.path.join(d, "*counter_collection.csv"))[0]
    rows = list(csv.DictReader(open(path)))
    agg = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in rows:
        agg[_short(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    lines = ["| kernel | counter | dispatches | mean per dispatch | total |", "|---|---|--:|--:|--:|"]
    for k in sorted(agg):
        for c, v in sorted(agg[k].items()):
            lines.append(f"| `{k}` | {c} | {len(v)} | {sum(v)/len(v):.6g} | {sum(v):.6g} |")
    open(out, "w").write("\n".join(lines) + "\n")
    os.remove(path)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--chis", default="1024,512,256", help="bond dimensions; the first is the headline")
    ap.add_argument("--chi", type=int, default=None, help="one bond dimension only (overrides --chis)")
    ap.add_argument("--d", type=int, default=5)
    ap.add_argument("--prec", choices=["both", "c128", "mixed"], default="both")
    ap.add_argument("--cpu-budget", type=float, default=24.0, help="seconds of oracle time (0: skip)")
    ap.add_argument("--sweeps", type=int, default=1, help="QR/LQ sweeps per update (1: the paper's single sweep)")
    ap.add_argument("--workload", choices=["bond", "chain", "serve", "quench", "schemes", "sym"], default="bond",
                    help="bond: the single-bond microbenchmark (default); chain: the batched finite chain "
                         "(L=128, Z_4, chi_max=512 by default), steady state, one JSON line of its own")
    ap.add_argument("--requests", type=int, default=64, help="serve: number of requests")
    ap.add_argument("--rate", type=float, default=4.0, help="serve: Poisson arrival rate (requests/s)")
    ap.add_argument("--serve-steps", type=int, default=50, help="serve: Trotter steps per request")
    ap.add_argument("--slots", type=int, default=4, help="serve: executors (contexts and streams)")
    ap.add_argument("--max-batch", type=int, default=8, help="serve: requests per slot batch")
    ap.add_argument("--hbm-budget-gb", type=float, default=200.0, help="serve: admission budget")
    ap.add_argument("--ds", default="2,3,4,5,6,8,10,12,16,20", help="schemes: physical dimensions")
    ap.add_argument("--L", type=int, default=128)
    ap.add_argument("--g", type=float, default=1.5, help="quench: transverse field")
    ap.add_argument("--dt", type=float, default=0.02, help="quench: Trotter step")
    ap.add_argument("--chi-max", type=int, default=512)
    ap.add_argument("--exec", type=int, default=2, help="chain: mps_sweep execution mode (0 eager, 1 speculative, 2 graph)")
    ap.add_argument("--autotune", default=None,
                    help="autotune cache file passed to mps_ctx_create (tuned during the warm-up)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 256 MiB three times (reference run for the HBM byte counters)")
    ap.add_argument("--rocprof-summary", nargs=3, metavar=("KIND", "DIR", "OUT"),
                    help="summarise rocprofv3 CSV output: KIND trace (kernel trace of this bench) or pmc")
    args = ap.parse_args()
    if args.rocprof_summary:
        kind, d, out = args.rocprof_summary
        (trace_summary if kind == "trace" else pmc_summary)(d, out)
        return
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

    if args.workload == "schemes":
        chi = args.chi or 1024
        ds = [int(x) for x in args.ds.split(",") if x.strip()]
        tab = run_schemes(lib, torch, chi, ds, max(1, min(args.steps, 5)), 20.0)
        ratio = {d: (r["svd"] / r["qr_cbe"] if r.get("svd") and r.get("qr_cbe") else None) for d, r in tab.items()}
        print(json.dumps({
            "metric": "single-gate wall time of the truncation schemes (ms), complex128",
            "unit": "ms per bond update", "n_gpus": 1, "higher_is_better": False, "data": "synthetic",
            "config": {"workload": f"microbenchmark cell chi={chi}, clock gate g=2 dt=0.05, schemes: QR (eta=chi), "
                                   f"QR+CBE (eta=chi+ceil(chi/10)), EIG and SVD (rocSOLVER), median of up to 5"},
            "ms": tab, "svd_over_qr_cbe": ratio}), flush=True)
        return
    if args.workload == "sym":
        chi = args.chi or 1024
        res = {}
        for key, p in (("c128", lib.MPS_C128), ("c64", lib.MPS_MIXED_C64)):
            if args.prec not in ("both", "c128" if key == "c128" else "mixed"):
                continue
            print(f"# sym {key} d={args.d} chi={chi}", file=sys.stderr, flush=True)
            res[key] = run_sym(lib, torch, p, chi, args.d, args.steps, args.warmup)
        first = res.get("c128") or res.get("c64")
        print(json.dumps({
            "metric": "bond updates/s, Z_d block-structured QR+CBE update (charge basis)", "value": first["updates_per_s"],
            "unit": "bond updates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "higher_is_better": True, "data": "synthetic",
            "config": {"workload": f"microbenchmark cell with Z_{args.d} blocks, chi={chi} in {args.d} equal sectors "
                                   f"on both bonds, eta_c = sec + ceil(sec/10), chi_max = chi, clock gate g=2 dt=0.05 "
                                   f"in the charge basis, one sector read-back per update"},
            "per_precision": res}), flush=True)
        return
    if args.workload == "quench":
        d = 10 if args.d == 5 else args.d
        cm = args.chi_max if args.chi_max != 512 else 1024
        res = {}
        legs = [("c128", lib.MPS_C128)] * (args.prec in ("both", "c128")) + \
               [("c64", lib.MPS_MIXED_C64)] * (args.prec in ("both", "mixed"))
        for key, p in legs:
            print(f"# quench {key} d={d} g={args.g} chi_max={cm} {args.steps} steps", file=sys.stderr, flush=True)
            res[key] = run_quench(lib, torch, p, d, args.g, cm, args.steps, args.dt, 100, args.exec, args.autotune)
        if len(res) < 2:
            r = next(iter(res.values()))
            print(json.dumps({"quench": next(iter(res)), "seconds": r["seconds"], "final_chi": r["chis"][-1],
                              "z_last": r["z"][-1].tolist(), "trunc_err_sum": r["eps_sum"]}), flush=True)
            return
        a, b = res["c128"], res["c64"]
        dz = np.abs(a["z"] - b["z"]).max(axis=1)
        de = np.abs(a["e"].mean(axis=1) - b["e"].mean(axis=1))
        pick = sorted(set([0, 9, 24, 49, 99, 149, args.steps - 1]) & set(range(args.steps)))
        print(json.dumps({
            "metric": "mixed vs complex128 error on <Z + Z^dag> and the energy per bond, heavy-d quench",
            "value": float(dz.max()), "unit": "max_t |d<Z + Z^dag>|", "n_gpus": 1, "higher_is_better": False,
            "data": "synthetic", "max_abs_dE": float(de.max()),
            "config": {"workload": f"uniform two-site cell, Z_{d} clock model g={args.g}, quench from |0>, "
                                   f"chi_max={cm}, dt={args.dt}, {args.steps} second-order steps, CBE dchi = "
                                   f"max(100, ceil(chi/10)), svd_min 1e-14 (c128) / 1e-6 (mixed)"},
            "per_step": {str(k + 1): {"dZ": float(dz[k]), "dE": float(de[k]), "z_c128": float(a["z"][k, 0]),
                                      "e_c128": float(a["e"][k].mean()), "chi_c128": a["chis"][k],
                                      "chi_mixed": b["chis"][k]} for k in pick},
            "seconds": {"c128": round(a["seconds"], 2), "c64": round(b["seconds"], 2)},
            "trunc_err_sum": {"c128": a["eps_sum"], "c64": b["eps_sum"]}}), flush=True)
        return
    if args.workload == "serve":
        prec = lib.MPS_C128 if args.prec == "c128" else lib.MPS_MIXED_C64
        rep = run_serve(lib, torch, args.requests, args.rate, args.serve_steps, prec, args.slots, args.max_batch,
                        int(args.hbm_budget_gb * 2**30))
        print(json.dumps({
            "metric": "serving: aggregate bond updates/s + p50/p99 per-request step latency",
            "value": round(rep["bond_updates_per_s"], 3), "unit": "bond updates/s", "n_gpus": 1,
            "higher_is_better": True, "dtype": "c128" if prec == lib.MPS_C128 else "c64", "data": "synthetic",
            "p50_step_ms": round(rep["p50_step_ms"], 3), "p99_step_ms": round(rep["p99_step_ms"], 3),
            "config": {"workload": f"{args.requests} quench requests, Poisson arrivals at {args.rate}/s, d in "
                                   f"{{2,3,4,5,8}}, g in [0.5,3], chi_max in {{64..1024}}, finite L in {{32,64}} or "
                                   f"uniform cell, {args.serve_steps} steps dt=0.05 each, {args.slots} slots, "
                                   f"batch <= {args.max_batch}, HBM budget {args.hbm_budget_gb} GB"},
            "report": rep}), flush=True)
        return
    if args.workload == "chain":
        d = 4 if args.d == 5 else args.d
        res = {}
        for key, p in [("c128", lib.MPS_C128)] * (args.prec in ("both", "c128")) + \
                      [("c64", lib.MPS_MIXED_C64)] * (args.prec in ("both", "mixed")):
            print(f"# chain {key} L={args.L} d={d} chi_max={args.chi_max}", file=sys.stderr, flush=True)
            res[key] = run_chain(lib, torch, p, args.L, d, args.chi_max, args.steps, args.warmup, args.exec,
                                 args.autotune)
        head = "c64" if "c64" in res else "c128"
        h = res[head]
        print(json.dumps({
            "metric": f"bond updates/s, batched finite chain L={args.L} d={d} chi_max={args.chi_max}",
            "value": round(h["updates_per_s"], 3), "unit": "bond updates/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": round(h["ms_per_step"], 3), "higher_is_better": True,
            "dtype": head, "data": "synthetic",
            "config": {"workload": f"finite chain L={args.L}, Z_{d} clock gates g=2 dt=0.05, random right-isometric "
                                   f"MPS at the saturated profile min({d}^b, {d}^(L-b), {args.chi_max}), CBE "
                                   f"eta = chi + ceil(chi/10), second-order steps, exec mode {args.exec}"},
            "per_precision": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                              for k, v in res.items()}}), flush=True)
        return
    chis = [args.chi] if args.chi else [int(c) for c in args.chis.split(",") if c.strip()]
    src = gemm_source_hash()
    traffic_ok = {k: (v[0] is not None and v[1] == src and args.d == 5 and chis[0] == 1024) for k, v in TRAFFIC.items()}
    precs = [("c128", lib.MPS_C128)] * (args.prec in ("both", "c128")) + \
            [("c64", lib.MPS_MIXED_C64)] * (args.prec in ("both", "mixed"))
    per_chi = {}
    for chi in chis:
        res = {}
        for key, p in precs:
            print(f"# timing {key} d={args.d} chi={chi}: {args.warmup} warm-up + {args.steps} updates",
                  file=sys.stderr, flush=True)
            res[key] = run_precision(lib, torch, p, chi, args.d, args.steps, args.warmup, args.sweeps, args.autotune)
            res[key]["roofline"] = roofline(res[key], key, traffic_ok if chi == chis[0] else {})
        if "c128" in res and "c64" in res:
            res["mixed_over_c128"] = res["c64"]["updates_per_s"] / res["c128"]["updates_per_s"]
        per_chi[chi] = res
    chi = chis[0]
    res = per_chi[chi]
    head = "c128" if "c128" in res else "c64"
    h = res[head]
    eta = chi + -(-chi // 10)
    rnd = lambda v: {k: (round(x, 6) if isinstance(x, float) else rnd(x) if isinstance(x, dict) else x)
                     for k, x in v.items()}
    line = {
        "metric": f"bond updates/s at d={args.d} \u03c7={chi} (mixed vs FP64) + p50/p99 step latency",
        "value": round(h["updates_per_s"], 4),
        "unit": "bond updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(h["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head,
        "data": "synthetic",
        "config": {"workload": f"single-bond QR+CBE update, uniform two-site cell, d={args.d}, chi={chi}, "
                               f"eta={eta}, chi~={chi}, clock gate g=2 dt=0.05"
                               + (f", {args.sweeps} QR/LQ sweeps" if args.sweeps > 1 else ""),
                   "d": args.d, "chi": chi, "eta": eta, "sweeps": args.sweeps},
        "p50_ms": round(h["p50_ms"], 4),
        "p99_ms": round(h["p99_ms"], 4),
        "per_precision": {k: (rnd(v) if isinstance(v, dict) else round(v, 4)) for k, v in res.items()},
        "roofline": h["roofline"],
        "per_chi": {str(c): {k: {"updates_per_s": round(v["updates_per_s"], 3), "p50_ms": round(v["p50_ms"], 3),
                                 "p99_ms": round(v["p99_ms"], 3), "contract_frac": v["roofline"]["frac"]}
                             for k, v in r.items() if isinstance(v, dict)}
                    for c, r in per_chi.items() if c != chi},
        "gemm_source": src,
    }
    if args.cpu_budget > 0:
        print("# timing the CPU oracle", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(chi, args.d, args.cpu_budget)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
