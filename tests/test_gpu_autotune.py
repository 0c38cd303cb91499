"""Autotuned launch shapes (the autotune cache of mps_ctx_create).

* Forced cache entries drive the non-default shapes (QR panels of about 32
  blocks, 16 matrix rows per tridiagonalisation block) through a whole bond
  update, compared with the oracle like every other bond update.
* A context with an empty cache times every candidate on its first bond
  update and its first speculative sweep chunk, writes the winners to the
  file, and a second context reads them back without trials; results stay
  within rounding of an untuned run.
"""
import numpy as np
import pytest

from oracle import bond as obond
from paper_2212_09782_amd import inputs, lib

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _bond(ctx, xi, bm, bn, U, eta, chi_max, prec=lib.MPS_C128):
    chiL, d, chiM = bm.shape
    chiR = bn.shape[2]
    desc = lib.bond_desc(d, chiL, chiM, chiR, eta, chi_max, 1e-14 if prec == lib.MPS_C128 else 1e-6, True, lib.CBE,
                         prec)
    cdt = torch.complex128 if prec == lib.MPS_C128 else torch.complex64
    out = lib.bond_update(ctx, desc, torch.from_numpy(xi).to("cuda"), torch.from_numpy(bm.reshape(-1)).to(cdt).to("cuda"),
                          torch.from_numpy(bn.reshape(-1)).to(cdt).to("cuda"),
                          torch.from_numpy(U.reshape(-1)).to("cuda"))
    ctx.sync()
    bm2, xi2, bn2, k = lib.unpack_bond(desc, *out[:4])
    return bm2.astype(np.complex128), xi2, bn2.astype(np.complex128), k, float(out[4].item())


def _bond_key(d, chi, eta, chi_max, prec=lib.MPS_C128):
    return f"bond:{prec}:{lib.CBE}:{d}:{chi}:{chi}:{chi}:{eta}:{chi_max}:1:1"


@pytest.mark.parametrize("panel_blocks,tri_rows", [(32, 16), (48, 16), (64, 16)])
def test_forced_shapes_match_oracle(tmp_path, panel_blocks, tri_rows):
    # m = d chi = 2000 rows: about 32, 42 and 63 blocks per QR panel; the
    # eta = 440 tridiagonalisation takes 16 rows per block
    d, chi, eta, chi_max = 5, 400, 440, 400
    path = tmp_path / "tune.txt"
    path.write_text(f"{_bond_key(d, chi, eta, chi_max)} {panel_blocks} {tri_rows} 1.0\n")
    ctx = lib.Context(0, autotune_cache=str(path))
    xi, bm, bn = inputs.random_bond(chi, chi, chi, d, seed=31)
    U = inputs.near_identity_unitary(d * d, inputs.rng(d), scale=0.1)
    g = _bond(ctx, xi, bm, bn, U, eta, chi_max)
    st = lib.sweep_stats(ctx)
    ctx.close()
    assert st["tune_hits"] == 1 and st["tune_trials"] == 0
    r = obond.qr_bond_update(xi, bm, bn, U, mode=obond.CBE, eta=eta, chi_max=chi_max, svd_min=1e-14)
    bm2, xi2, bn2, k, eps = g
    assert k == r["chi"]
    pr, svr, mr = obond.invariants(r["bm"], r["xi"], r["bn"])
    pg, svg, mg = obond.invariants(bm2, xi2, bn2)
    e_pair = np.linalg.norm(pg - pr) / np.linalg.norm(pr)
    e_sv = np.max(np.abs(svg - svr)) / np.max(svr)
    print(f"panel_blocks {panel_blocks} tri_rows {tri_rows}: pair {e_pair:.2e} sv {e_sv:.2e}", flush=True)
    # the random cell cuts a flat spectrum: the kept subspace moves by ~u/gap
    assert e_pair <= 1e-8 and e_sv <= 1e-10
    assert abs(eps - r["eps"]) <= 1e-10


def test_tuning_writes_and_reuses_cache(tmp_path):
    path = tmp_path / "tune.txt"
    d, chi, eta = 4, 96, 106
    xi, bm, bn = inputs.random_bond(chi, chi, chi, d, seed=5)
    U = lib.clock_gate(d, 2.0, 0.05)
    base = lib.Context(0)
    ref = _bond(base, xi, bm, bn, U, eta, chi)
    base.close()

    ctx = lib.Context(0, autotune_cache=str(path))
    first = _bond(ctx, xi, bm, bn, U, eta, chi)
    st = lib.sweep_stats(ctx)
    assert st["tune_trials"] == 6 and st["tune_hits"] == 0
    # a saturated chain: the first speculative chunk is tuned as well
    L, dc, cm = 24, 4, 16
    mps = inputs.random_finite_mps(L, dc, cm, seed=9)
    state = lib.State(ctx, mps["B"], mps["Xi"], finite=True, chi_cap=cm)
    gates = lib.chain_gates(dc, 2.0, L, True, 0.05)
    pol = lib.sweep_policy(cm, 1e-14, 2, 0.1, exec=lib.EXEC_GRAPH)
    lib.mps_sweep(ctx, [state], [gates], 3, 2, pol)
    ctx.sync()
    st2 = lib.sweep_stats(ctx)
    assert st2["tune_trials"] == 12
    state.close()
    ctx.close()
    lines = [l for l in path.read_text().splitlines() if l and not l.startswith("#")]
    assert len(lines) == 2 and lines[0].startswith("bond:") and lines[1].startswith("sweep:")

    again = lib.Context(0, autotune_cache=str(path))
    second = _bond(again, xi, bm, bn, U, eta, chi)
    st3 = lib.sweep_stats(again)
    again.close()
    assert st3["tune_trials"] == 0 and st3["tune_hits"] == 1
    for g in (first, second):
        assert g[3] == ref[3]
        pa, sa, _ = obond.invariants(*g[:3])
        pr, sr, _ = obond.invariants(*ref[:3])
        assert np.linalg.norm(pa - pr) / np.linalg.norm(pr) <= 1e-8
        assert np.max(np.abs(sa - sr)) / np.max(sr) <= 1e-10
