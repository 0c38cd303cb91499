"""Serving on the GPU: each request's result is the same alone and in the mix.

Requests of different d, chi_max and geometry run (a) one at a time and
(b) together with continuous batching on two slots (streams); the final
<Z + Z^dag> profiles must agree to 1e-12 (bond updates never mix data across
requests and every reduction has a fixed order)."""
import numpy as np
import pytest

from paper_2212_09782_amd import serve

pytestmark = pytest.mark.gpu
pytest.importorskip("torch")


def make_requests():
    spec = [(2, 0.8, 16, True, 8), (3, 2.0, 12, True, 6), (3, 1.5, 16, False, 2), (4, 2.5, 10, True, 5)]
    return [serve.Request(rid=k, arrival=0.002 * k, d=d, g=g, chi_max=c, finite=f, L=L, nsteps=4)
            for k, (d, g, c, f, L) in enumerate(spec)]


def test_alone_equals_mix():
    alone = {}
    for r in make_requests():
        ex = serve.Executor(0)
        eng = serve.Engine([ex], hbm_budget=64 << 30, max_batch=1)
        eng.run([r])
        ex.close()
        alone[r.rid] = r.result["zz"]
    execs = [serve.Executor(0), serve.Executor(0)]
    eng = serve.Engine(execs, hbm_budget=64 << 30, max_batch=2)
    reqs = make_requests()
    rep = eng.run(reqs)
    for ex in execs:
        ex.close()
    assert rep["requests"] == 4 and rep["rejected"] == 0
    for r in reqs:
        print(f"request {r.rid}: alone {np.round(alone[r.rid], 6)} mix {np.round(r.result['zz'], 6)} "
              f"chis {r.result['chis']}", flush=True)
    for r in reqs:
        assert np.max(np.abs(r.result["zz"] - alone[r.rid])) < 1e-12, r.rid
    print(rep)
