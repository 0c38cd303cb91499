"""Pins of the oracle's Z_d block-structured update (oracle/sym.py) against
what the mathematics fixes: the closed forms of the clock operators in the
charge basis, charge conservation of the gate, the block structure of the
output, and, where every block keeps its full rank, the singular value
decomposition of the whole two-site matrix (numpy's SVD on the dense matrix,
which knows nothing of the blocks) and the dense CBE update of oracle/bond.py.
"""
import numpy as np
import pytest

from oracle import bond, clock, sym
from paper_2212_09782_amd import inputs

CASES = [
    (2, [3, 2], [2, 3], [3, 3]),
    (3, [4, 3, 2], [3, 4, 3], [2, 4, 3]),
    (3, [5, 0, 2], [3, 4, 0], [2, 4, 3]),     # empty sectors
    (4, [3, 2, 2, 1], [2, 3, 1, 2], [1, 2, 3, 2]),
    (5, [2, 2, 1, 2, 1], [1, 2, 2, 2, 1], [2, 1, 2, 2, 1]),
]


def _gate(d, g=1.5, tau=0.1):
    return sym.to_charge_basis_gate(clock.gate(clock.bond_hamiltonian(d, g), tau), d)


@pytest.mark.parametrize("d", [2, 3, 5, 10])
def test_charge_basis_closed_forms(d):
    """In the charge basis X = diag(w^q) and Z raises the charge by one."""
    Z, X = clock.clock_ops(d)
    w = np.exp(2j * np.pi / d)
    assert np.allclose(sym.to_charge_basis_op(X, d), np.diag(w ** np.arange(d)), atol=1e-14)
    raise_ = np.zeros((d, d))
    for q in range(d):
        raise_[(q + 1) % d, q] = 1
    assert np.allclose(sym.to_charge_basis_op(Z, d), raise_, atol=1e-14)


@pytest.mark.parametrize("d", [2, 3, 5, 10])
def test_charge_gate_conserves_total_charge(d):
    U = _gate(d)
    q = np.arange(d * d)
    tot = (q // d + q % d) % d
    off = tot[:, None] != tot[None, :]
    assert np.max(np.abs(U[off])) < 1e-14
    assert np.allclose(U @ U.conj().T, np.eye(d * d), atol=1e-13)


@pytest.mark.parametrize("d,sl,sm,sr", CASES)
def test_output_keeps_block_structure(d, sl, sm, sr):
    xi, bm, bn = inputs.random_sym_bond(sl, sm, sr, d, seed=7)
    assert np.all(bm[~sym.allowed(sl, sm, d)] == 0) and np.all(bn[~sym.allowed(sm, sr, d)] == 0)
    r = sym.sym_bond_update(xi, bm, bn, _gate(d), sl, sm, sr, 1, 0.1, 100, 1e-14)
    assert sum(r["sec"]) == r["chi"] == r["bm"].shape[2] == r["bn"].shape[0]
    assert np.all(r["bm"][~sym.allowed(sl, r["sec"], d)] == 0)
    assert np.all(r["bn"][~sym.allowed(r["sec"], sr, d)] == 0)
    M = r["bn"].reshape(r["chi"], -1)
    assert np.allclose(M @ M.conj().T, np.eye(r["chi"]), atol=1e-13)
    assert np.all(r["xi"] > 0) and abs(np.linalg.norm(r["xi"]) - 1) < 1e-14
    # inside every sector the new values descend
    o = sym.offsets(r["sec"])
    for c in range(d):
        assert np.all(np.diff(r["xi"][o[c]:o[c + 1]]) <= 0)
    assert abs(r["eps"] - r["eps_id"]) < 1e-12


def _dense_svd_charges(Th, sl, sr, d):
    """Singular values of the dense two-site matrix and, for each, the charge
    of the block its right singular vector lives in."""
    _, S, Vh = np.linalg.svd(Th, full_matrices=False)
    ch = []
    for v in Vh:
        w = [np.linalg.norm(v[sym.block_index(sl, sr, d, c)[1]]) for c in range(d)]
        ch.append(int(np.argmax(w)))
        assert max(w) > 1 - 1e-8
    return S, np.array(ch)


@pytest.mark.parametrize("d,sl,sm,sr", CASES)
def test_full_rank_blocks_reproduce_theta(d, sl, sm, sr):
    """eta_c at the full block size, nothing truncated: the kept values are
    the nonzero singular values of the whole two-site matrix (with their
    charges), and Xi^[m] B~^[m] B~^[n] rebuilds theta~."""
    xi, bm, bn = inputs.random_sym_bond(sl, sm, sr, d, seed=11)
    r = sym.sym_bond_update(xi, bm, bn, _gate(d), sl, sm, sr, 10 ** 6, 0.0, 10 ** 6, 1e-10)
    S, ch = _dense_svd_charges(r["Th"], sl, sr, d)
    nz = S > 1e-10
    xs = r["xi"] * np.sqrt(r["kept2"])
    assert np.allclose(np.sort(xs)[::-1], S[nz], rtol=1e-12, atol=1e-13)
    for c in range(d):
        assert r["sec"][c] == np.count_nonzero(ch[nz] == c)
    chiL, chiR = bm.shape[0], bn.shape[2]
    pair = np.repeat(xi, d)[:, None] * (r["bm"].reshape(chiL * d, -1) @ r["bn"].reshape(-1, d * chiR))
    assert np.allclose(pair, r["Th"], atol=1e-12)
    assert r["eps"] < 1e-24


@pytest.mark.parametrize("d,sl,sm,sr", CASES[1:])
def test_truncation_over_all_blocks_is_the_global_svd_cut(d, sl, sm, sr):
    """Full-size blocks, chi_max below the rank: the kept values are the
    chi_max largest singular values of the whole matrix, the sector sizes
    their charges, the pair B~[m] B~[n] the one of the dense CBE update of
    oracle/bond.py with eta at its maximum."""
    xi, bm, bn = inputs.random_sym_bond(sl, sm, sr, d, seed=13)
    U = _gate(d)
    chi_max = 5
    r = sym.sym_bond_update(xi, bm, bn, U, sl, sm, sr, 10 ** 6, 0.0, chi_max, 1e-14)
    S, ch = _dense_svd_charges(r["Th"], sl, sr, d)
    assert r["chi"] == chi_max
    xs = np.sort(r["xi"] * np.sqrt(r["kept2"]))[::-1]
    assert np.allclose(xs, S[:chi_max], rtol=1e-12)
    for c in range(d):
        assert r["sec"][c] == np.count_nonzero(ch[:chi_max] == c)
    chiL, chiM, chiR = bm.shape[0], bm.shape[2], bn.shape[2]
    dense = bond.qr_bond_update(xi, bm, bn, U, mode=bond.CBE, eta=min(d * chiL, d * chiR), chi_max=chi_max,
                                svd_min=1e-14)
    pd, sd, _ = bond.invariants(dense["bm"], dense["xi"], dense["bn"])
    ps, ss, _ = bond.invariants(r["bm"], r["xi"], r["bn"])
    assert np.allclose(ps, pd, atol=1e-11)
    assert np.allclose(ss, sd, atol=1e-13)
    assert abs(r["eps"] - dense["eps"]) < 1e-12


def test_at_least_one_value_and_ties_go_to_the_lower_charge():
    """svd_min above every value keeps exactly one (the largest); with two
    blocks of identical spectra and chi_max odd, the extra value goes to the
    lower charge."""
    d = 2
    sl, sm, sr = [2, 2], [2, 2], [2, 2]
    xi, bm, bn = inputs.random_sym_bond(sl, sm, sr, d, seed=3)
    r = sym.sym_bond_update(xi, bm, bn, _gate(d), sl, sm, sr, 10, 0.0, 10, svd_min=10.0)
    assert r["chi"] == 1 and abs(r["xi"][0] - 1) < 1e-15
    # tensors invariant under exchanging the two charge sectors of every bond
    # (sector sizes 2, 2; index k <-> k + 2 mod 4) and the identity gate: the
    # blocks of middle charge 0 and 1 are the same matrix, so every value
    # appears once in each block and an odd chi_max splits a pair
    r0 = inputs.rng(5)
    bm = np.zeros((4, 2, 4), np.complex128)
    bn = np.zeros((4, 2, 4), np.complex128)
    for T in (bm, bn):
        for al in range(2):
            for q in range(2):
                for be in range(2):
                    v = r0.standard_normal() + 1j * r0.standard_normal()
                    T[al, q, 2 * q + be] = v                        # left sector 0 -> right sector q
                    T[al + 2, q, (2 * q + be + 2) % 4] = v          # the copy in the other sector
    xi = np.array([0.5, 0.3, 0.5, 0.3])
    U = np.eye(4, dtype=np.complex128)
    sec = [2, 2]
    assert np.all(bm[~sym.allowed(sec, sec, d)] == 0)
    r = sym.sym_bond_update(xi, bm, bn, U, sec, sec, sec, 10, 0.0, 3, 1e-14)
    assert np.allclose(r["S"][0], r["S"][1], rtol=1e-14) and r["S"][0][1] > 1e-3
    assert r["sec"] == [2, 1]


def test_charge_basis_quench_matches_the_dense_clock_basis_quench():
    """The uniform cell of the Z_3 clock model (g = 1, dt = 0.05, 12
    second-order steps, chi_max = 16, eta at its maximum) from the charge-0
    product state: block by block in the charge basis and densely (oracle/
    bond.py through oracle/mps.py) in the clock basis from |+>|+>...  Both
    keep the chi_max largest Schmidt values of every update above svd_min =
    1e-6 (clear of the ~1e-8 |S| rounding floor of S from L^dag L, whose
    count depends on the block sizes), so the bond dimensions, <X + X^dag>
    and the bond energies agree to rounding."""
    from oracle import mps
    d, g, dt, steps, chi_max = 3, 1.0, 0.05, 12, 16
    plus = np.full((1, d, 1), 1 / np.sqrt(d), np.complex128)
    st = dict(B=[plus, plus.copy()], Xi=[np.ones(1), np.ones(1)], finite=False)
    _, Xc = clock.clock_ops(d)
    hb = clock.bond_hamiltonian(d, g)
    gh, gf = [clock.gate(hb, dt / 2)] * 2, [clock.gate(hb, dt)] * 2
    B, Xi, secs = inputs.charge_product_cell(d)
    S = dict(B=list(B), Xi=list(Xi), secs=[list(secs[0]), list(secs[1])], finite=False)
    Uh, Uf = sym.to_charge_basis_gate(gh[0], d), sym.to_charge_basis_gate(gf[0], d)
    hc = sym.to_charge_basis_gate(hb, d)
    w = np.exp(2j * np.pi * np.arange(d) / d)
    for _ in range(steps):
        mps.trotter_step(st, gh, gf, dchi_rule=lambda c: 1000, chi_max=chi_max, svd_min=1e-6)
        for bnd, U in ((0, Uh), (1, Uf), (0, Uh)):
            m, n = bnd, 1 - bnd
            r = sym.sym_bond_update(S["Xi"][m], S["B"][m], S["B"][n], U, S["secs"][m], S["secs"][n], S["secs"][m],
                                    1000, 0.0, chi_max, 1e-6)
            S["B"][m], S["B"][n], S["Xi"][n], S["secs"][n] = r["bm"], r["bn"], r["xi"], r["sec"]
        assert [sum(s) for s in S["secs"]] == [b.shape[0] for b in st["B"]]
        xd, _ = mps.site_expectation(st, Xc + Xc.conj().T)
        xs, _ = mps.site_expectation(S, np.diag(w + w.conj()))
        assert np.max(np.abs(xd - xs)) < 1e-12
        assert np.max(np.abs(mps.bond_expectation(st, [hb, hb]) - mps.bond_expectation(S, [hc, hc]))) < 1e-12
    assert max(b.shape[0] for b in st["B"]) == chi_max   # the cut was reached
