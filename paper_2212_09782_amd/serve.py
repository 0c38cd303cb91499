"""Serving loop for quench simulations: continuous batching on one GPU.

Requests (d, g, chi_max, geometry, nsteps, dt) arrive over time.  The engine
keeps every admitted request's MPS resident in HBM and advances requests in
batches: a slot owns a batch of requests and repeatedly calls mps_sweep for
one Trotter step on all of them together (their even layers form one layer,
then their odd layers).  Between steps, finished requests leave the batch
and newly admitted ones join it ("continuous batching").  Several slots run
at once, each with its own library context and HIP stream, so their work
overlaps on the device.  Admission is by an HBM budget: a request is admitted
only when its state buffers plus its share of workspace fit.

Metrics: per-request step latency (gap between consecutive step completions
of one request; the first step counts from admission) with p50/p99, and
aggregate bond updates/s (all bond updates / makespan).

The engine logic is independent of the executor: `Executor` runs the real
library; tests may plug a stub executor in to check admission and batching
on the CPU (never a product path).
"""
import heapq
import math
import threading
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    arrival: float
    d: int
    g: float
    chi_max: int
    finite: bool
    L: int
    nsteps: int = 50
    dt: float = 0.05
    prec: int = 0
    # filled by the engine
    admitted_at: float = None
    step_times: list = field(default_factory=list)
    done_at: float = None
    bond_updates: int = 0
    result: dict = None

    def bonds_per_step(self):
        """Bond updates of one second-order step: even(1/2), odd, even(1/2)."""
        if not self.finite:
            return 3
        nb = self.L - 1
        return 2 * math.ceil(nb / 2) + nb // 2


# Plain-launched QR panels use one block per CU on at most 64 CUs each; with
# this many slots running panels at once they still fit the 256 CUs, so every
# panel's blocks are co-resident (more slots could stall its grid barriers).
MAX_SLOTS = 4


def state_bytes(req):
    es = 16 if req.prec == 0 else 8
    return req.L * (req.chi_max * req.d * req.chi_max * es + req.chi_max * 8)


def saturated_chis(req):
    """Bond dimensions (L + 1 entries, bond left of each site) once chi has
    grown to its cap: min(d^b, d^(L-b), chi_max) on a finite chain, chi_max
    on the uniform cell."""
    if not req.finite:
        return [req.chi_max] * 3
    out = [1]
    for b in range(1, req.L):
        out.append(int(min(req.d ** min(b, 30), req.d ** min(req.L - b, 30), req.chi_max)))
    return out + [1]


def layer_bonds(req, parity):
    """(chi_l, chi_m, chi_r) of the bonds one layer of this request updates."""
    ch = saturated_chis(req)
    if not req.finite:
        return [(ch[0], ch[1], ch[0])]
    return [(ch[m], ch[m + 1], ch[m + 2]) for m in range(parity, req.L - 1, 2)]


# mps_sweep runs a layer's bonds in groups (in order) whose workspaces
# together stay within this many bytes, one group after the other.
LAYER_GROUP_BYTES = 16 << 30


def layer_workspace(bond_bytes):
    """Workspace one layer needs: the largest group of consecutive bonds
    (greedy, as mps_sweep forms them) under LAYER_GROUP_BYTES."""
    best = cur = 0
    for b in bond_bytes:
        b = (b + 255) // 256 * 256
        if cur > 0 and cur + b > LAYER_GROUP_BYTES:
            cur = 0
        cur += b
        best = max(best, cur)
    return best


def eta_of(d, chi_l, chi_m, chi_r, dchi_min=100, dchi_frac=0.1):
    """The sweep's eta rule: min(chi_m + max(dchi_min, ceil(dchi_frac chi_m)), d chi_l, d chi_r)."""
    return min(chi_m + max(dchi_min, math.ceil(dchi_frac * chi_m)), d * chi_l, d * chi_r)


class Executor:
    """Runs requests on the GPU through the C-ABI (one instance per slot)."""

    def __init__(self, device=0):
        import torch
        from . import lib
        self.torch = torch
        self.lib = lib
        self.ctx = lib.Context(device)
        self.stream = torch.cuda.Stream(device=device)
        self.states = {}

    def bond_workspace_bytes(self, req, chi_l, chi_m, chi_r):
        """mps_workspace_query of one bond of this request."""
        import ctypes
        lib = self.lib
        eta = eta_of(req.d, chi_l, chi_m, chi_r)
        desc = lib.bond_desc(req.d, chi_l, chi_m, chi_r, eta, req.chi_max, prec=req.prec)
        n = ctypes.c_size_t()
        lib._check(lib.load().mps_workspace_query(self.ctx.h, ctypes.byref(desc), ctypes.byref(n)))
        return int(n.value)

    def workspace_bytes(self, req):
        """Workspace of this request's larger layer at the saturated chi
        profile (see layer_workspace)."""
        return max(layer_workspace([self.bond_workspace_bytes(req, *b) for b in layer_bonds(req, p)])
                   for p in (0, 1))

    def admit(self, req):
        lib, torch = self.lib, self.torch
        with torch.cuda.stream(self.stream):
            e = np.zeros((1, req.d, 1), np.complex128)
            e[0, 0, 0] = 1
            st = lib.State(self.ctx, [e] * req.L, [np.ones(1)] * req.L, finite=req.finite,
                           chi_cap=req.chi_max, prec=req.prec)
            gates = lib.chain_gates(req.d, req.g, req.L, req.finite, req.dt)
            Z = np.diag(np.exp(2j * np.pi * np.arange(req.d) / req.d))
            zz = torch.from_numpy((Z + Z.conj().T).reshape(-1)).to("cuda")
        self.states[req.rid] = (st, gates, zz)

    def step(self, reqs):
        """One Trotter step of every request in reqs: one mps_sweep call per
        precision (the policy's svd_min depends on it; chi_max is each
        state's own cap)."""
        lib = self.lib
        for prec in sorted({r.prec for r in reqs}):
            group = [r for r in reqs if r.prec == prec]
            sts = [self.states[r.rid][0] for r in group]
            gts = [self.states[r.rid][1] for r in group]
            pol = lib.sweep_policy(max(r.chi_max for r in group), 1e-14 if prec == 0 else 1e-6,
                                   exec=lib.EXEC_SPECULATIVE)
            lib.mps_sweep(self.ctx, sts, gts, 1, 2, pol, stream=self.stream)
        self.stream.synchronize()
        lib._check(lib.load().mps_sync(self.ctx.h, lib._stream(self.stream)))

    def drop(self, req):
        """Release a request's device state without measuring (after a failure)."""
        ent = self.states.pop(req.rid, None)
        if ent is not None:
            ent[0].close()

    def finish(self, req):
        torch, lib = self.torch, self.lib
        st, gates, zz = self.states.pop(req.rid)
        # every device tensor of this executor lives on its stream: a zero fill
        # queued on another stream would be unordered with the measurement
        with torch.cuda.stream(self.stream):
            vals = torch.zeros(2 * req.L, dtype=torch.float64, device="cuda")
            lib.mps_measure(self.ctx, st, op1=zz, site_vals=vals, stream=self.stream)
        self.stream.synchronize()
        req.result = {"zz": vals.cpu().numpy().reshape(req.L, 2)[:, 0].copy(), "chis": st.chis()}
        st.close()

    def close(self):
        self.ctx.close()


class Engine:
    """Continuous-batching scheduler over at most MAX_SLOTS executors and an HBM budget.

    HBM accounting: every admitted request holds its state buffers; every
    slot holds its context's workspace, which grows to the largest layer
    workspace (sum over the layer's bonds of every request in the batch)
    the slot has run and is kept while the slot lives.  A request is
    admitted only if its state plus the growth of its slot's workspace
    fits the budget.
    """

    def __init__(self, executors, hbm_budget, max_batch=8, clock=time.perf_counter, on_finish=None):
        if not 1 <= len(executors) <= MAX_SLOTS:
            raise ValueError(f"1 to {MAX_SLOTS} executors (slots) are supported, got {len(executors)}")
        self.execs = executors
        self.budget = hbm_budget
        self.max_batch = max_batch
        self.clock = clock
        self.lock = threading.Lock()
        self.used = 0              # states of admitted requests + every slot's workspace high-water mark
        self.peak_used = 0
        self.waiting = []          # (arrival, rid, req) heap of arrived, not yet admitted
        self.pending = []          # not yet arrived (sorted by arrival)
        self.batches = [[] for _ in executors]
        self.ws_batch = [0 for _ in executors]   # layer workspace of the slot's current batch
        self.ws_high = [0 for _ in executors]    # the slot context's workspace (grow-only)
        self.finished = []
        self.errors = []
        self.on_finish = on_finish   # callback(request, engine) after each finished / failed request
        self.t0 = None

    def _try_admit(self, slot):
        """Move arrived requests into this slot's batch while budget and batch size allow."""
        ex = self.execs[slot]
        with self.lock:
            now = self.clock() - self.t0
            while self.pending and self.pending[0].arrival <= now:
                r = self.pending.pop(0)
                heapq.heappush(self.waiting, (r.arrival, r.rid, r))
            joined = []
            while self.waiting and len(self.batches[slot]) + len(joined) < self.max_batch:
                _, _, r = self.waiting[0]
                sb, wb = state_bytes(r), ex.workspace_bytes(r)
                grow = max(0, self.ws_batch[slot] + wb - self.ws_high[slot])
                if self.used + sb + grow > self.budget:
                    alone = sb + max(wb, max(self.ws_high))
                    if alone > self.budget:   # never admittable: reject rather than stall
                        heapq.heappop(self.waiting)
                        r.result = {"rejected": True}
                        self.finished.append(r)
                        continue
                    break
                heapq.heappop(self.waiting)
                self.used += sb + grow
                self.ws_high[slot] += grow
                self.ws_batch[slot] += wb
                self.peak_used = max(self.peak_used, self.used)
                r._state_bytes, r._ws_bytes = sb, wb
                r.admitted_at = now
                joined.append(r)
        for r in joined:
            try:
                ex.admit(r)
            except Exception as e:   # noqa: BLE001 - a failed request must not stop the engine
                self._fail(slot, [r], e, admitted=False)
                continue
            self.batches[slot].append(r)

    def _release(self, slot, r):
        with self.lock:
            self.used -= r._state_bytes
            self.ws_batch[slot] -= r._ws_bytes

    def _fail(self, slot, reqs, err, admitted=True):
        """Mark requests failed, free their state and budget, record the error."""
        ex = self.execs[slot]
        for r in reqs:
            if admitted:
                try:
                    ex.drop(r)
                except Exception:   # noqa: BLE001
                    pass
            r.result = {"failed": True, "error": f"{type(err).__name__}: {err}"}
            r.done_at = self.clock() - self.t0
            self._release(slot, r)
            with self.lock:
                self.finished.append(r)
                self.errors.append((r.rid, str(err)))
            if self.on_finish:
                self.on_finish(r, self)

    def _worker(self, slot):
        ex = self.execs[slot]
        while True:
            self._try_admit(slot)
            batch = self.batches[slot]
            if not batch:
                with self.lock:
                    idle = not self.pending and not self.waiting
                if idle:
                    return
                time.sleep(0.002)
                continue
            try:
                ex.step(batch)
            except Exception as e:   # noqa: BLE001 - fail this batch, keep serving the others
                self._fail(slot, batch, e)
                self.batches[slot] = []
                continue
            now = self.clock() - self.t0
            keep = []
            for r in batch:
                r.step_times.append(now)
                r.bond_updates += r.bonds_per_step()
                if len(r.step_times) >= r.nsteps:
                    try:
                        ex.finish(r)
                    except Exception as e:   # noqa: BLE001
                        self._fail(slot, [r], e)
                        continue
                    r.done_at = now
                    self._release(slot, r)
                    with self.lock:
                        self.finished.append(r)
                    if self.on_finish:
                        self.on_finish(r, self)
                else:
                    keep.append(r)
            self.batches[slot] = keep

    def run(self, requests):
        self.pending = sorted(requests, key=lambda r: r.arrival)
        self.t0 = self.clock()
        threads = [threading.Thread(target=self._worker, args=(s,)) for s in range(len(self.execs))]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        makespan = self.clock() - self.t0
        return self.report(makespan)

    def report(self, makespan):
        lat = []
        total = 0
        for r in self.finished:
            if r.result and (r.result.get("rejected") or r.result.get("failed")):
                continue
            prev = r.admitted_at
            for t in r.step_times:
                lat.append(t - prev)
                prev = t
            total += r.bond_updates
        lat = np.array(lat) if lat else np.zeros(1)
        return {
            "requests": len(self.finished),
            "rejected": sum(1 for r in self.finished if r.result and r.result.get("rejected")),
            "failed": sum(1 for r in self.finished if r.result and r.result.get("failed")),
            "makespan_s": makespan,
            "bond_updates": total,
            "bond_updates_per_s": total / makespan if makespan > 0 else 0.0,
            "p50_step_ms": 1e3 * float(np.percentile(lat, 50)),
            "p99_step_ms": 1e3 * float(np.percentile(lat, 99)),
            "peak_hbm_bytes": self.peak_used,
        }


def requests_from_stream(specs, nsteps=50, dt=0.05, prec=0, chi_cap=None, time_scale=1.0):
    """Requests from inputs.serving_requests() dicts (optionally capping chi_max)."""
    out = []
    for k, s in enumerate(specs):
        chi = s["chi_max"] if chi_cap is None else min(s["chi_max"], chi_cap)
        out.append(Request(rid=k, arrival=s["arrival"] * time_scale, d=s["d"], g=s["g"], chi_max=chi,
                           finite=s["finite"], L=s["L"], nsteps=nsteps, dt=dt, prec=prec))
    return out
