"""Host logic of the serving engine, driven by a stub executor on the CPU
(the stub is test-only; the product path is serve.Executor on the GPU)."""
import threading
import time

import numpy as np

from paper_2212_09782_amd import inputs, serve


class StubExecutor:
    def __init__(self, log):
        self.log = log
        self.active = set()

    def workspace_bytes(self, req):
        return 1000 * req.chi_max

    def admit(self, req):
        self.active.add(req.rid)

    def step(self, reqs):
        self.log.append(tuple(sorted(r.rid for r in reqs)))
        time.sleep(0.001)

    def finish(self, req):
        self.active.discard(req.rid)
        req.result = {"zz": np.full(req.L, req.rid, float)}


def test_all_requests_finish_within_budget():
    specs = inputs.serving_requests(n=20, rate=400.0, seed=5)
    reqs = serve.requests_from_stream(specs, nsteps=6, chi_cap=64)
    log = []
    execs = [StubExecutor(log), StubExecutor(log)]
    budget = 3 * max(serve.state_bytes(r) + 1000 * r.chi_max for r in reqs)
    eng = serve.Engine(execs, hbm_budget=budget, max_batch=3)
    rep = eng.run(reqs)
    assert rep["requests"] == 20 and rep["rejected"] == 0
    assert eng.peak_used <= budget
    assert all(len(r.step_times) == 6 for r in reqs)
    assert all(len(b) <= 3 for b in log)
    # continuous batching: some batch changed composition between steps
    assert len(set(log)) > 2
    assert rep["p99_step_ms"] >= rep["p50_step_ms"] > 0
    assert rep["bond_updates"] == sum(6 * r.bonds_per_step() for r in reqs)


def test_never_admittable_request_is_rejected():
    reqs = [serve.Request(rid=0, arrival=0.0, d=2, g=1.0, chi_max=8, finite=True, L=4, nsteps=2),
            serve.Request(rid=1, arrival=0.0, d=8, g=1.0, chi_max=1024, finite=True, L=64, nsteps=2)]
    eng = serve.Engine([StubExecutor([])], hbm_budget=serve.state_bytes(reqs[0]) + 10 ** 6, max_batch=2)
    rep = eng.run(reqs)
    assert rep["rejected"] == 1
    assert reqs[0].result["zz"][0] == 0


def test_bonds_per_step():
    assert serve.Request(0, 0, 2, 1.0, 8, True, 20).bonds_per_step() == 2 * 10 + 9
    assert serve.Request(0, 0, 2, 1.0, 8, False, 2).bonds_per_step() == 3
