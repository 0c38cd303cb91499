"""GPU parity of mps_bond_update_sym (the Z_d block-structured CBE update)
against the oracle's block-by-block update (oracle/sym.py), and of a
charge-basis quench of the uniform cell against the oracle's dense quench in
the clock basis.

Compared, as for the dense update: the new sector sizes (exact), the Schmidt
values of every sector, the gauge-invariant pair B~[m] B~[n] and M^dag M, the
truncation error, right-isometry of B~[n], and exact zeros outside the
blocks.  Tolerances: 1e-10 (pair: 1e-8 where a flat random spectrum is cut)
in complex128; the mixed path's stated bounds otherwise.
"""
import numpy as np
import pytest

from oracle import bond as obond
from oracle import clock, mps, sym
from paper_2212_09782_amd import inputs, lib

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    c = lib.Context(0)
    yield c
    c.close()


def _dev(a, dt):
    return torch.from_numpy(np.ascontiguousarray(a).reshape(-1)).to(dt).to("cuda")


def run_sym(ctx, xi, bm, bn, U, sl, sm, sr, dchi_min, dchi_frac, chi_max, svd_min, prec):
    d = bm.shape[1]
    desc = lib.sym_desc(d, sl, sm, sr, dchi_min, dchi_frac, chi_max, svd_min, prec)
    cdt = torch.complex128 if prec == lib.MPS_C128 else torch.complex64
    out = lib.bond_update_sym(ctx, desc, _dev(xi, torch.float64), _dev(bm, cdt), _dev(bn, cdt),
                              _dev(U, torch.complex128))
    ctx.sync()
    bm2, xi2, bn2, sec, k = lib.unpack_sym(desc, *out[:5])
    return bm2.astype(np.complex128), xi2, bn2.astype(np.complex128), sec, k, float(out[5].item())


def check(r, g, sl, sr, d, tol_pair=1e-10, tol_sv=1e-10, tol_iso=1e-13, tol_eps=1e-12):
    bm2, xi2, bn2, sec, k, eps = g
    assert sec == r["sec"], (sec, r["sec"])
    assert k == r["chi"]
    assert np.all(bm2[~sym.allowed(sl, sec, d)] == 0) and np.all(bn2[~sym.allowed(sec, sr, d)] == 0)
    o = sym.offsets(sec)
    e_sv = max(np.max(np.abs(xi2[o[c]:o[c + 1]] - r["xi"][o[c]:o[c + 1]]), initial=0) for c in range(d))
    e_sv /= np.max(r["xi"])
    pr, _, mr = obond.invariants(r["bm"], r["xi"], r["bn"])
    pg, _, mg = obond.invariants(bm2, xi2, bn2)
    e_pair = np.linalg.norm(pg - pr) / np.linalg.norm(pr)
    e_mdm = np.linalg.norm(mg - mr) / np.linalg.norm(mr)
    print(f"  sec {sec}  pair {e_pair:.2e}  M^dag M {e_mdm:.2e}  sv {e_sv:.2e}  eps {eps:.3e} vs {r['eps']:.3e}",
          flush=True)
    assert e_pair <= tol_pair and e_mdm <= tol_pair and e_sv <= tol_sv
    B = bn2.reshape(k, -1)
    assert np.max(np.abs(B @ B.conj().T - np.eye(k))) <= tol_iso
    assert abs(eps - r["eps"]) <= tol_eps + 1e-8 * abs(r["eps"])


CASES = [
    # d, sec_l, sec_m, sec_r, dchi_min, dchi_frac, chi_max
    (2, [3, 2], [2, 3], [3, 3], 1, 0.1, 100),
    (3, [10, 7, 5], [8, 6, 9], [7, 10, 4], 2, 0.1, 100),
    (3, [10, 7, 5], [8, 6, 9], [7, 10, 4], 2, 0.1, 15),          # the cut falls between sectors
    (3, [12, 0, 9], [7, 5, 0], [0, 11, 8], 3, 0.1, 100),         # empty sectors, one expanded from zero
    (3, [12, 0, 9], [7, 5, 0], [0, 11, 8], 0, 0.1, 100),         # an empty sector that stays empty
    (4, [20, 17, 25, 19], [22, 18, 21, 20], [19, 24, 18, 20], 4, 0.1, 70),
    (5, [30, 25, 20, 25, 30], [28, 27, 22, 24, 30], [26, 31, 24, 21, 29], 3, 0.1, 150),
    (5, [64, 60, 66, 58, 62], [61, 65, 59, 63, 60], [60, 62, 64, 61, 63], 7, 0.1, 290),
    (10, [8, 9, 7, 10, 8, 9, 7, 8, 10, 9], [9, 8, 8, 9, 7, 10, 8, 9, 8, 9], [8, 8, 9, 9, 10, 7, 8, 9, 9, 8],
     2, 0.1, 90),
]


@pytest.mark.parametrize("case", CASES, ids=[f"d{c[0]}-chi{sum(c[2])}-k{c[6]}-m{c[4]}" for c in CASES])
def test_sym_update_c128(ctx, case):
    d, sl, sm, sr, dmin, dfrac, chi_max = case
    print("sym c128", case, flush=True)
    xi, bm, bn = inputs.random_sym_bond(sl, sm, sr, d, seed=sum(sm) + d)
    U = inputs.random_charge_gate(d, inputs.rng(d + 3), scale=0.2)
    r = sym.sym_bond_update(xi, bm, bn, U, sl, sm, sr, dmin, dfrac, chi_max, 1e-14)
    g = run_sym(ctx, xi, bm, bn, U, sl, sm, sr, dmin, dfrac, chi_max, 1e-14, lib.MPS_C128)
    # a cut through a flat random spectrum moves the kept subspace by ~u/gap
    check(r, g, sl, sr, d, tol_pair=1e-8 if chi_max < sum(r["eta"]) else 1e-10)


@pytest.mark.parametrize("case", [CASES[1], CASES[5], CASES[6], CASES[8]],
                         ids=["d3", "d4", "d5", "d10"])
def test_sym_update_mixed(ctx, case):
    """complex64 storage, FP32 matrix cores, FP64 eigensolver and
    re-orthogonalisation; bounds as for the dense mixed update: pair 2e-5,
    Schmidt values 1e-5 of the largest, B~[n] isometric to 1e-6, eps 1e-5
    (no global cut in these cases, so the sector sizes are exact)."""
    d, sl, sm, sr, dmin, dfrac, _ = case
    chi_max = 10 ** 4
    xi, bm, bn = inputs.random_sym_bond(sl, sm, sr, d, seed=sum(sm) + 2 * d)
    bm = bm.astype(np.complex64).astype(np.complex128)
    bn = bn.astype(np.complex64).astype(np.complex128)
    U = inputs.random_charge_gate(d, inputs.rng(d + 5), scale=0.2)
    r = sym.sym_bond_update(xi, bm, bn, U, sl, sm, sr, dmin, dfrac, chi_max, 1e-6)
    g = run_sym(ctx, xi, bm, bn, U, sl, sm, sr, dmin, dfrac, chi_max, 1e-6, lib.MPS_MIXED_C64)
    check(r, g, sl, sr, d, tol_pair=2e-5, tol_sv=1e-5, tol_iso=1e-6, tol_eps=1e-5)


def test_sym_full_size_d5_chi1024(ctx):
    """d = 5, chi = 1024 on all three bonds (sectors 205, 205, 205, 205, 204),
    eta_c = sec + 21, chi_max = 1024: the microbenchmark's shape with the
    block structure, complex128, against the oracle."""
    d = 5
    sec = inputs.sym_sectors(1024, d)
    xi, bm, bn = inputs.random_sym_bond(sec, sec, sec, d, seed=1024)
    U = inputs.random_charge_gate(d, inputs.rng(11), scale=0.1)
    r = sym.sym_bond_update(xi, bm, bn, U, sec, sec, sec, 21, 0.1, 1024, 1e-14)
    g = run_sym(ctx, xi, bm, bn, U, sec, sec, sec, 21, 0.1, 1024, 1e-14, lib.MPS_C128)
    check(r, g, sec, sec, d, tol_pair=1e-8, tol_sv=1e-10, tol_iso=1e-12)


def test_sym_product_state_start(ctx):
    """The charge-0 product cell (every bond one sector of size 1): the first
    update populates every middle sector."""
    d = 4
    B, Xi, secs = inputs.charge_product_cell(d)
    U = inputs.random_charge_gate(d, inputs.rng(2), scale=0.5)
    r = sym.sym_bond_update(Xi[0], B[0], B[1], U, secs[0], secs[1], secs[0], 10, 0.1, 100, 1e-14)
    g = run_sym(ctx, Xi[0], B[0], B[1], U, secs[0], secs[1], secs[0], 10, 0.1, 100, 1e-14, lib.MPS_C128)
    assert r["sec"] == [1] * d
    check(r, g, secs[0], secs[0], d)


@pytest.mark.parametrize("prec", [lib.MPS_C128, lib.MPS_MIXED_C64], ids=["c128", "mixed"])
def test_sym_cell_quench_matches_dense_oracle(ctx, prec):
    """Uniform cell of the Z_3 clock model (g = 1, dt = 0.05, 12 second-order
    steps, chi_max = 16, svd_min = 1e-6) from the charge-0 product state: in
    the charge basis through SymCell, in the clock basis (the state |+>|+>...)
    through the oracle's dense CBE sweep with eta at its maximum.  Both keep
    the largest chi_max Schmidt values of every update, so the bond
    dimensions (complex128), <X + X^dag> and the bond energy agree to rounding
    (complex128: 1e-10; mixed: 1e-5)."""
    d, g, dt, steps, chi_max = 3, 1.0, 0.05, 12, 16
    B, Xi, secs = inputs.charge_product_cell(d)
    svd_min = 1e-6
    cell = lib.SymCell(ctx, B, Xi, secs, chi_cap=chi_max, prec=prec)
    uh = _dev(lib.clock_gate_charge(d, g, dt / 2), torch.complex128)
    uf = _dev(lib.clock_gate_charge(d, g, dt), torch.complex128)
    w = np.exp(2j * np.pi * np.arange(d) / d)
    xop = _dev(np.diag(w + w.conj()), torch.complex128)
    hop = _dev(lib.clock_hamiltonian_charge(d, g), torch.complex128)
    site = torch.zeros(4, dtype=torch.float64, device="cuda")
    bond = torch.zeros(4, dtype=torch.float64, device="cuda")
    # oracle: |+> in the clock basis, dense CBE with eta = min(chi + 1000, d chi, d chi)
    plus = np.full((1, d, 1), 1 / np.sqrt(d), np.complex128)
    st = dict(B=[plus, plus.copy()], Xi=[np.ones(1), np.ones(1)], finite=False)
    Zc, Xc = clock.clock_ops(d)
    hb = clock.bond_hamiltonian(d, g)
    gh, gf = [clock.gate(hb, dt / 2)] * 2, [clock.gate(hb, dt)] * 2
    worst = 0.0
    for t in range(steps):
        cell.step(uh, uf, 1000, 0.0, chi_max, svd_min)
        cell.measure(op1=xop, op2=hop, site_vals=site, bond_vals=bond)
        ctx.sync()
        mps.trotter_step(st, gh, gf, dchi_rule=lambda c: 1000, chi_max=chi_max, svd_min=svd_min)
        xr, _ = mps.site_expectation(st, Xc + Xc.conj().T)
        er = mps.bond_expectation(st, [hb, hb])
        xs = site.cpu().numpy().reshape(2, 2)[:, 0]
        es = bond.cpu().numpy().reshape(2, 2)[:, 0]
        dev_ = max(np.max(np.abs(xs - xr.real)), np.max(np.abs(es - er.real)))
        worst = max(worst, dev_)
        print(f"  step {t + 1}: chis sym {cell.chis()} dense {[b.shape[0] for b in st['B']]} "
              f"<X+X^dag> {xs[0]:.10f} vs {xr[0].real:.10f}  dev {dev_:.1e}", flush=True)
    if prec == lib.MPS_C128:
        assert cell.chis() == [b.shape[0] for b in st["B"]] == [chi_max, chi_max]
    assert worst <= (1e-10 if prec == lib.MPS_C128 else 1e-5)
