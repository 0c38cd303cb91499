"""Layer execution of mps_sweep (Fig. 2a): per-layer read-back, speculative
chunks and hipGraph replay give the same state (the config-4 chain against
the oracle in graph mode is in test_gpu_sweep).

Speculative chunks and step graphs run only while the chi profile is
saturated; a chunk in which some bond keeps fewer Schmidt values than
planned is undone and rerun layer by layer.  The three modes run the same
kernels with the same reduction orders, so their results are compared
bitwise.
"""
import numpy as np
import pytest

from oracle import clock
from paper_2212_09782_amd import inputs, lib

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    c = lib.Context(0)
    yield c
    c.close()


def _run(ctx, B, Xi, finite, d, g, dt, chi_max, calls, steps_per_call, exec_mode, prec=lib.MPS_C128, chunk=0,
         dchi_min=100, svd_min=None):
    L = len(B)
    st = lib.State(ctx, B, Xi, finite=finite, chi_cap=chi_max, prec=prec)
    gates = lib.chain_gates(d, g, L, finite, dt)
    if svd_min is None:
        svd_min = 1e-14 if prec == lib.MPS_C128 else 1e-6
    pol = lib.sweep_policy(chi_max, svd_min, dchi_min, 0.1, exec=exec_mode, chunk=chunk)
    Z, _ = clock.clock_ops(d)
    zz = torch.from_numpy((Z + Z.conj().T).reshape(-1)).to("cuda")
    site = torch.zeros(2 * L, dtype=torch.float64, device="cuda")
    eps = torch.zeros(1, dtype=torch.float64, device="cuda")
    before = lib.sweep_stats(ctx)
    zs, chis = [], []
    for _ in range(calls):
        lib.mps_sweep(ctx, [st], [gates], steps_per_call, 2, pol, trunc_err=eps)
        lib.mps_measure(ctx, st, op1=zz, site_vals=site)
        ctx.sync()
        zs.append(site.cpu().numpy().copy())
        chis.append(st.chis())
    after = lib.sweep_stats(ctx)
    stats = {k: after[k] - before[k] for k in after}
    out = dict(z=np.array(zs), chis=chis, eps=float(eps.item()), tensors=st.to_numpy(), stats=stats)
    st.close()
    return out


def _same(a, b):
    assert a["chis"] == b["chis"]
    assert np.array_equal(a["z"], b["z"])
    assert a["eps"] == b["eps"]
    for x, y in zip(a["tensors"][0], b["tensors"][0]):
        assert np.array_equal(x, y)
    for x, y in zip(a["tensors"][1], b["tensors"][1]):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("prec", [lib.MPS_C128, lib.MPS_MIXED_C64], ids=["c128", "mixed"])
def test_graph_and_speculative_equal_eager(ctx, prec):
    """Quench of the Z_3 chain (L = 20, chi_max = 32, g = 2, dt = 0.05): 20
    steps as 4 calls of 5 steps; the profile saturates early, after which the
    speculative and graph modes issue whole chunks without host reads."""
    d, L = 3, 20
    B = [np.eye(1, d, 0).reshape(1, d, 1).astype(np.complex128) for _ in range(L)]
    Xi = [np.ones(1) for _ in range(L)]
    runs = {}
    for mode in (lib.EXEC_EAGER, lib.EXEC_SPECULATIVE, lib.EXEC_GRAPH):
        runs[mode] = _run(ctx, B, Xi, True, d, 2.0, 0.05, 32, 4, 5, mode, prec=prec)
        print(f"exec {mode}: {runs[mode]['stats']}", flush=True)
    _same(runs[lib.EXEC_EAGER], runs[lib.EXEC_SPECULATIVE])
    _same(runs[lib.EXEC_EAGER], runs[lib.EXEC_GRAPH])
    sg = runs[lib.EXEC_GRAPH]["stats"]
    assert runs[lib.EXEC_SPECULATIVE]["stats"]["chunks"] >= 1
    assert sg["graph_captures"] >= 1 and sg["graph_replays"] >= 2
    # fewer host synchronisations than one per layer
    assert sg["host_syncs"] < runs[lib.EXEC_EAGER]["stats"]["host_syncs"]


def test_speculation_rollback(ctx):
    """A saturated profile whose centre bond matrix has rank one: the first
    update of the centre bond keeps fewer Schmidt values than planned (with
    svd_min = 1e-6 the eigensolver's noise-level values of the rank-deficient
    bond are dropped), the chunk is undone and rerun layer by layer; the
    result equals the eager run."""
    d, L, chi_max = 2, 8, 8
    mps = inputs.random_finite_mps(L, d, chi_max, seed=17)
    Xi = [x.copy() for x in mps["Xi"]]
    Xi[4][:] = 0
    Xi[4][0] = 1.0
    a = _run(ctx, mps["B"], Xi, True, d, 1.0, 0.05, chi_max, 2, 3, lib.EXEC_EAGER, dchi_min=2, svd_min=1e-6)
    b = _run(ctx, mps["B"], Xi, True, d, 1.0, 0.05, chi_max, 2, 3, lib.EXEC_GRAPH, dchi_min=2, svd_min=1e-6)
    print("eager", a["stats"], "graph", b["stats"], "chis", b["chis"], flush=True)
    assert b["stats"]["rollbacks"] >= 1
    _same(a, b)
