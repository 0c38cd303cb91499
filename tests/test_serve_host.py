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

    def drop(self, req):
        self.active.discard(req.rid)


class LayerStubExecutor(StubExecutor):
    """Workspace as the library carves it: one region per bond of a layer."""

    def workspace_bytes(self, req):
        return max(sum(10 * cl * cm * cr for cl, cm, cr in serve.layer_bonds(req, p)) for p in (0, 1))


class FailingExecutor(StubExecutor):
    """Raises on the step of one request (as a latched device error or an
    out-of-memory workspace growth would)."""

    def __init__(self, log, bad_rid, fail_on="step"):
        super().__init__(log)
        self.bad, self.fail_on = bad_rid, fail_on

    def admit(self, req):
        if self.fail_on == "admit" and req.rid == self.bad:
            raise RuntimeError("admit failed")
        super().admit(req)

    def step(self, reqs):
        if self.fail_on == "step" and any(r.rid == self.bad for r in reqs):
            raise RuntimeError("libqrtebd error -5: device reported numeric error bits 0x2")
        super().step(reqs)


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


def test_layer_workspace_charged_and_kept_per_slot():
    """A request is charged the sum of its layer's bond workspaces; a slot's
    workspace stays at its high-water mark after requests leave."""
    reqs = [serve.Request(rid=k, arrival=0.0, d=2, g=1.0, chi_max=16, finite=True, L=12, nsteps=3)
            for k in range(4)]
    ex = LayerStubExecutor([])
    one = ex.workspace_bytes(reqs[0])
    bonds = serve.layer_bonds(reqs[0], 0)
    assert len(bonds) == 6 and one == 10 * sum(a * b * c for a, b, c in bonds)
    sb = serve.state_bytes(reqs[0])
    # room for two requests in one batch: states + the two-request layer workspace
    eng = serve.Engine([ex], hbm_budget=2 * sb + 2 * one + 10, max_batch=4)
    rep = eng.run(reqs)
    assert rep["requests"] == 4 and rep["rejected"] == 0 and rep["failed"] == 0
    assert eng.peak_used == 2 * sb + 2 * one
    assert eng.ws_high[0] == 2 * one          # kept after the batch emptied
    assert eng.used == eng.ws_high[0]         # only the slot's workspace remains charged
    assert eng.ws_batch[0] == 0


def test_failed_step_releases_budget_and_engine_terminates():
    specs = inputs.serving_requests(n=8, rate=1000.0, seed=5)
    reqs = serve.requests_from_stream(specs, nsteps=4, chi_cap=32)
    log = []
    execs = [FailingExecutor(log, bad_rid=2), FailingExecutor(log, bad_rid=2)]
    budget = 2 * max(serve.state_bytes(r) + 1000 * r.chi_max for r in reqs)
    eng = serve.Engine(execs, hbm_budget=budget, max_batch=2)
    done = []
    t = threading.Thread(target=lambda: done.append(eng.run(reqs)))
    t.start()
    t.join(timeout=30)
    assert not t.is_alive(), "engine hung after a failed step"
    rep = done[0]
    assert rep["requests"] == 8 and rep["failed"] >= 1
    assert any(rid == 2 for rid, _ in eng.errors)
    ok = [r for r in reqs if not r.result.get("failed")]
    assert all(len(r.step_times) == 4 for r in ok)
    assert eng.used == sum(eng.ws_high)      # every state released


def test_failed_admit_is_reported():
    reqs = [serve.Request(rid=k, arrival=0.0, d=2, g=1.0, chi_max=8, finite=True, L=4, nsteps=2) for k in range(3)]
    eng = serve.Engine([FailingExecutor([], bad_rid=1, fail_on="admit")], hbm_budget=1 << 30, max_batch=3)
    rep = eng.run(reqs)
    assert rep["failed"] == 1 and reqs[1].result["failed"]
    assert all(len(reqs[k].step_times) == 2 for k in (0, 2))


def test_slot_count_is_capped():
    import pytest
    with pytest.raises(ValueError):
        serve.Engine([StubExecutor([]) for _ in range(serve.MAX_SLOTS + 1)], hbm_budget=1 << 30)


def test_layer_workspace_groups():
    G = serve.LAYER_GROUP_BYTES
    assert serve.layer_workspace([100, 200, 300]) == 256 + 256 + 512
    # bonds that do not fit one group run in consecutive groups sharing one region
    assert serve.layer_workspace([G // 2, G // 2, G // 2]) == G
    assert serve.layer_workspace([2 * G, 10]) == 2 * G
