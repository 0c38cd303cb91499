"""GPU parity of mps_bond_update against the oracle (gauge-invariant outputs).

The QR gauge is not unique, so the HIP path and the oracle are compared on
  * chi~ (exact),
  * the singular values of the new bond matrix Xi~,
  * the two-site product B~[m] B~[n] (independent of the gauge of B~[n]),
  * the truncation error eps,
and the new right tensor must be an isometry.  Tolerances: 1e-10 relative
for the complex128 path; the mixed path is held to the bounds stated in
test_mixed_* (complex64 storage, FP32 matrix cores).
"""
import numpy as np
import pytest

from oracle import bond as obond
from paper_2212_09782_amd import inputs, lib

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    c = lib.Context(0)
    yield c
    c.close()


def run_gpu(ctx, xi, bm, bn, U, mode, eta, chi_max, svd_min=1e-14, prec=lib.MPS_C128, sweeps=1):
    chiL, d, chiM = bm.shape
    chiR = bn.shape[2]
    diag = np.ndim(xi) == 1
    desc = lib.bond_desc(d, chiL, chiM, chiR, eta, chi_max, svd_min, diag, mode, prec, sweeps)
    cdt = torch.complex128 if prec == lib.MPS_C128 else torch.complex64
    dxi = torch.from_numpy(np.ascontiguousarray(xi).reshape(-1)).to("cuda")
    if not diag:
        dxi = dxi.to(torch.complex128)
    dbm = torch.from_numpy(bm.reshape(-1)).to(cdt).to("cuda")
    dbn = torch.from_numpy(bn.reshape(-1)).to(cdt).to("cuda")
    du = torch.from_numpy(np.ascontiguousarray(U).reshape(-1)).to("cuda")
    out = lib.bond_update(ctx, desc, dxi, dbm, dbn, du)
    ctx.sync()
    bm2, xi2, bn2, k = lib.unpack_bond(desc, *out[:4])
    eps = float(out[4].item())
    return bm2.astype(np.complex128), xi2, bn2.astype(np.complex128), k, eps


def compare(r, g, tol_pair=1e-10, tol_sv=1e-10, tol_iso=1e-13, tol_eps=1e-12, tol_mdm=None):
    """Gauge-invariant comparison of a GPU update g with the oracle's r.

    pair = B~[m] B~[n] and M^dag M (M = Xi~ B~[n], the right reduced density
    matrix: for plain / grow it is (L Q^[n])^dag (L Q^[n]) / |L|^2 and fixes the
    orientation of L) within tol_pair (tol_mdm) relative, Schmidt values within
    tol_sv of the largest, B~[n] isometric, eps and chi~ equal."""
    bm2, xi2, bn2, k, eps = g
    assert k == r["chi"], (k, r["chi"])
    pr, svr, mr = obond.invariants(r["bm"], r["xi"], r["bn"])
    pg, svg, mg = obond.invariants(bm2, xi2, bn2)
    e_pair = np.linalg.norm(pg - pr) / np.linalg.norm(pr)
    e_mdm = np.linalg.norm(mg - mr) / np.linalg.norm(mr)
    e_sv = np.max(np.abs(svg - svr)) / np.max(svr)
    print(f"  pair {e_pair:.2e}  M^dag M {e_mdm:.2e}  sv {e_sv:.2e}  eps {eps:.3e} vs {r['eps']:.3e}", flush=True)
    assert e_pair <= tol_pair
    assert e_mdm <= (tol_pair if tol_mdm is None else tol_mdm)
    assert e_sv <= tol_sv
    B = bn2.reshape(k, -1)
    assert np.max(np.abs(B @ B.conj().T - np.eye(k))) <= tol_iso
    assert abs(eps - r["eps"]) <= tol_eps + 1e-8 * abs(r["eps"])


CASES = [
    # chiL, chiM, chiR, d, mode, eta, chi_max, diag_xi
    (1, 1, 1, 3, obond.CBE, 3, 100, True),
    (1, 3, 9, 3, obond.CBE, 3, 32, True),
    (4, 4, 4, 2, obond.CBE, 8, 8, True),
    (8, 8, 8, 3, obond.PLAIN, 8, 8, True),
    (8, 8, 8, 3, obond.PLAIN, 8, 8, False),
    (16, 20, 12, 3, obond.GROW, 30, 30, True),
    (16, 16, 16, 5, obond.CBE, 18, 16, True),
    (30, 40, 50, 4, obond.CBE, 44, 40, True),
    (64, 64, 64, 5, obond.CBE, 71, 64, True),
    (100, 90, 80, 3, obond.CBE, 99, 95, True),
    (37, 41, 33, 5, obond.CBE, 45, 200, False),
    (200, 200, 200, 5, obond.CBE, 220, 200, True),
    (130, 130, 130, 4, obond.PLAIN, 130, 130, True),
    # the gate's one-wave groups: all outputs in registers at d = 7, 8, 9 (odd d:
    # groups with fewer outputs), five outputs per pass at d = 12
    (3, 5, 20, 7, obond.CBE, 20, 40, True),
    (6, 7, 70, 8, obond.CBE, 40, 50, True),
    (2, 4, 6, 9, obond.CBE, 18, 20, False),
    (4, 3, 5, 12, obond.CBE, 20, 30, True),
    # large d: the gate stages 16 columns per block (d = 13, 20)
    (3, 4, 5, 13, obond.CBE, 20, 30, True),
    (4, 5, 3, 20, obond.CBE, 30, 40, False),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}x{c[2]}d{c[3]}m{c[4]}e{c[5]}k{c[6]}" for c in CASES])
def test_bond_update_c128(ctx, case):
    chiL, chiM, chiR, d, mode, eta, chi_max, diag = case
    print("bond c128", case, flush=True)
    xi, bm, bn = inputs.random_bond(chiL, chiM, chiR, d, seed=chiL * 31 + chiR, diag_xi=diag)
    U = inputs.near_identity_unitary(d * d, inputs.rng(d), scale=0.1)
    r = obond.qr_bond_update(xi, bm, bn, U, mode=mode, eta=eta, chi_max=chi_max, svd_min=1e-14)
    g = run_gpu(ctx, xi, bm, bn, U, mode, eta, chi_max)
    compare(r, g)


SWEEP_CASES = [
    # chiL, chiM, chiR, d, mode, eta, chi_max, sweeps
    (8, 8, 8, 3, obond.PLAIN, 8, 8, 2),
    (16, 20, 12, 3, obond.GROW, 30, 30, 3),
    (40, 40, 40, 4, obond.CBE, 48, 36, 2),
    (70, 64, 66, 5, obond.CBE, 75, 60, 4),
]


@pytest.mark.parametrize("case", SWEEP_CASES, ids=[f"{c[0]}x{c[1]}x{c[2]}d{c[3]}m{c[4]}s{c[7]}" for c in SWEEP_CASES])
def test_bond_update_sweeps(ctx, case):
    """Iterated QR/LQ sweeps (gate far from the identity) against the oracle's nsweeps."""
    chiL, chiM, chiR, d, mode, eta, chi_max, sweeps = case
    print("bond sweeps", case, flush=True)
    xi, bm, bn = inputs.random_bond(chiL, chiM, chiR, d, seed=chiL * 7 + sweeps)
    U = inputs.near_identity_unitary(d * d, inputs.rng(d + 1), scale=0.6)
    r = obond.qr_bond_update(xi, bm, bn, U, mode=mode, eta=eta, chi_max=chi_max, nsweeps=sweeps)
    r1 = obond.qr_bond_update(xi, bm, bn, U, mode=mode, eta=eta, chi_max=chi_max)
    assert r["eps"] <= r1["eps"] * (1 + 1e-9)
    g = run_gpu(ctx, xi, bm, bn, U, mode, eta, chi_max, sweeps=sweeps)
    compare(r, g)


def test_bond_update_clock_gate(ctx):
    """The library's own clock gate: same result as the oracle's expm gate."""
    d, chi = 5, 48
    xi, bm, bn = inputs.random_bond(chi, chi, chi, d, seed=3)
    Ug = lib.clock_gate(d, 2.0, 0.05)
    from oracle import clock
    Uo = clock.gate(clock.bond_hamiltonian(d, 2.0), 0.05)
    r = obond.qr_bond_update(xi, bm, bn, Uo, mode=obond.CBE, eta=53, chi_max=48)
    g = run_gpu(ctx, xi, bm, bn, Ug, obond.CBE, 53, 48)
    compare(r, g)


def test_bond_update_full_eta_is_svd(ctx):
    """Full eta: the GPU result is the truncated SVD of theta~ (Eckart-Young, via numpy)."""
    d, chiL, chiM, chiR = 3, 12, 14, 10
    xi, bm, bn = inputs.random_bond(chiL, chiM, chiR, d, seed=9)
    U = inputs.random_unitary(9, inputs.rng(4))
    eta = min(d * chiL, d * chiR)
    _, Th = obond.two_site(xi, bm, bn, U)
    s = np.linalg.svd(Th, compute_uv=False)
    bm2, xi2, bn2, k, eps = run_gpu(ctx, xi, bm, bn, U, obond.CBE, eta, 12)
    assert k == 12
    assert np.allclose(xi2, s[:12] / np.linalg.norm(s[:12]), rtol=1e-10, atol=1e-13)
    assert abs(eps - np.sum(s[12:] ** 2) / np.sum(s ** 2)) < 1e-12


@pytest.mark.parametrize("chi", [256, 512])
def test_bond_update_bench_shape(ctx, chi):
    """The single-bond benchmark cell at chi = 256, 512 (d = 5, eta = chi + ceil(chi/10))."""
    d = 5
    print("bench shape", chi, flush=True)
    A, B, lA, lB = inputs.microbench_cell(chi, d, seed=0)
    U = lib.clock_gate(d, 2.0, 0.05)
    eta = chi + -(-chi // 10)
    r = obond.qr_bond_update(lA, A, B, U, mode=obond.CBE, eta=eta, chi_max=chi, svd_min=1e-14)
    g = run_gpu(ctx, lA, A, B, U, obond.CBE, eta, chi)
    # random tensors cut through a flat spectrum: the kept subspace moves by ~u/gap
    compare(r, g, tol_pair=1e-8, tol_sv=1e-10, tol_iso=1e-12)


ORACLE_FULL = [
    # chi, d, precision
    (1024, 5, lib.MPS_C128),          # the headline shape, eta = 1127
    (600, 10, lib.MPS_C128),          # d chi = 6000 rows: QR panels beyond two LDS slabs (column loop)
    (512, 8, lib.MPS_C128),           # the register-resident gate (complex128 from d = 7)
    (256, 10, lib.MPS_MIXED_C64),     # the register-resident gate on complex64 storage (from d = 9)
    (256, 5, lib.MPS_MIXED_C64),
    (512, 5, lib.MPS_MIXED_C64),
    (1024, 5, lib.MPS_MIXED_C64),
]


@pytest.mark.parametrize("chi,d,prec", ORACLE_FULL,
                         ids=[f"chi{c}-d{d}-{'c128' if p == lib.MPS_C128 else 'mixed'}" for c, d, p in ORACLE_FULL])
def test_bond_update_full_size_oracle(ctx, chi, d, prec):
    """The single-bond benchmark cell at full size against the oracle (CBE,
    eta = chi + ceil(chi/10), chi~ = chi): chi~, Schmidt values, eps, the
    two-site product and M^dag M built from the oracle's own tensors.
    complex128: the random cell cuts a flat spectrum (gaps ~1e-3 at the cut),
    so the kept subspace moves by ~u/gap and the product is held to 1e-8.
    Mixed: complex64 inputs (the oracle takes the same rounded tensors in
    complex128) under the mixed path's stated bounds."""
    mixed = prec == lib.MPS_MIXED_C64
    print("full size vs oracle", chi, d, "mixed" if mixed else "c128", flush=True)
    A, B, lA, lB = inputs.microbench_cell(chi, d, seed=0)
    if mixed:
        A = A.astype(np.complex64).astype(np.complex128)
        B = B.astype(np.complex64).astype(np.complex128)
    U = lib.clock_gate(d, 2.0, 0.05)
    eta = chi + -(-chi // 10)
    smin = 1e-6 if mixed else 1e-14
    g = run_gpu(ctx, lA, A, B, U, obond.CBE, eta, chi, smin, prec)
    r = obond.qr_bond_update(lA, A, B, U, mode=obond.CBE, eta=eta, chi_max=chi, svd_min=smin)
    if mixed:
        compare_mixed(r, g)
    else:
        compare(r, g, tol_pair=1e-8, tol_sv=1e-10, tol_iso=1e-11)


FULL = [(5, lib.MPS_C128), (10, lib.MPS_C128), (5, lib.MPS_MIXED_C64), (10, lib.MPS_MIXED_C64)]


@pytest.mark.parametrize("d,prec", FULL, ids=[f"d{d}-{'c128' if p == lib.MPS_C128 else 'mixed'}" for d, p in FULL])
def test_bond_update_full_size_properties(ctx, d, prec):
    """chi = 1024 with d = 5 (the headline shape) and d = 10 (theta~ of 10240 x 10240,
    the largest configuration), checked by properties and sampled rows: B~[n]
    isometric, Xi~ normalised and descending, eps = 1 - sum_kept S^2 (|theta~| = 1),
    and sampled rows of B~[m] equal C~[alpha] B~[n]^dag computed on the host.
    Mixed path: isometry to 1e-6 and rows to 2e-5 (complex64 storage)."""
    chi = 1024
    print("full size", d, prec, flush=True)
    A, B, lA, lB = inputs.microbench_cell(chi, d, seed=0)
    U = lib.clock_gate(d, 2.0, 0.05)
    eta = chi + -(-chi // 10)
    mixed = prec == lib.MPS_MIXED_C64
    bm2, xi2, bn2, k, eps = run_gpu(ctx, lA, A, B, U, obond.CBE, eta, chi, 1e-6 if mixed else 1e-14, prec)
    assert k == chi
    Bn = bn2.reshape(k, -1)
    assert np.max(np.abs(Bn @ Bn.conj().T - np.eye(k))) < (1e-6 if mixed else 1e-11)
    assert abs(np.sum(xi2 ** 2) - 1) < 1e-12 and np.all(np.diff(xi2) <= 1e-15)
    assert 0 <= eps < 1
    for alpha in (0, 511, 1023):
        C = np.tensordot(A[alpha], B, axes=([1], [0]))           # [i', j', delta]
        Ct = (U @ C.reshape(d * d, -1)).reshape(d, d * chi)       # [i, (j delta)]
        ref = Ct @ Bn.conj().T
        assert np.linalg.norm(bm2[alpha] - ref) <= (2e-5 if mixed else 1e-12) * np.linalg.norm(ref)


# ---------------------------------------------------------------- mixed precision

MIXED = [
    (16, 16, 16, 5, obond.CBE, 18, 16),
    (64, 64, 64, 3, obond.CBE, 71, 64),
    (120, 100, 90, 4, obond.CBE, 110, 100),
    (64, 64, 64, 3, obond.PLAIN, 64, 64),
    # the gate on complex64 storage: five outputs per pass (d = 7), all in registers (d = 9)
    (10, 12, 30, 7, obond.CBE, 30, 30),
    (20, 24, 70, 9, obond.CBE, 40, 40),
]


@pytest.mark.parametrize("case", MIXED, ids=[f"{c[0]}x{c[1]}x{c[2]}d{c[3]}m{c[4]}" for c in MIXED])
def test_mixed_bond_update(ctx, case):
    """complex64 storage / FP32 matrix cores with FP64 panels, eig and re-orthogonalisation.

    Bounds (stated): two-site product within 2e-5 relative, Schmidt values
    within 1e-5 of the largest, B~[n] isometric to 1e-6, eps within 1e-5.
    Both sides drop Schmidt values below 1e-6 (the mixed path's noise floor);
    a value within the noise of that threshold may land on either side, so
    chi~ may differ by values below 2e-6, which carry weight < 1e-11."""
    chiL, chiM, chiR, d, mode, eta, chi_max = case
    xi, bm, bn = inputs.random_bond(chiL, chiM, chiR, d, seed=chiL + 5)
    bm = bm.astype(np.complex64).astype(np.complex128)
    bn = bn.astype(np.complex64).astype(np.complex128)
    U = inputs.near_identity_unitary(d * d, inputs.rng(d + 1), scale=0.1)
    r = obond.qr_bond_update(xi, bm, bn, U, mode=mode, eta=eta, chi_max=chi_max, svd_min=1e-6)
    g = run_gpu(ctx, xi, bm, bn, U, mode, eta, chi_max, svd_min=1e-6, prec=lib.MPS_MIXED_C64)
    compare_mixed(r, g)


def compare_mixed(r, g, tol_pair=2e-5, tol_sv=1e-5, tol_iso=1e-6, tol_eps=1e-5):
    k = g[3]
    if k != r["chi"]:
        lo = min(k, r["chi"])
        S = np.asarray(r["S"])
        assert abs(k - r["chi"]) <= 2 and np.all(S[lo:max(k, r["chi"])] < 2e-6), (k, r["chi"])
        assert np.max(np.abs(np.sort(np.abs(g[1]))[::-1][:lo] - np.abs(r["xi"])[:lo])) <= tol_sv
        pr, _, _ = obond.invariants(r["bm"], r["xi"], r["bn"])
        pg, _, _ = obond.invariants(*g[:3])
        assert np.linalg.norm(pg - pr) <= tol_pair * np.linalg.norm(pr)
        return
    compare(r, g, tol_pair=tol_pair, tol_sv=tol_sv, tol_iso=tol_iso, tol_eps=tol_eps)
