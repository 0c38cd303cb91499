"""GPU parity of the building blocks through the C-ABI: complex GEMM on MFMA,
Householder QR, FP64 Hermitian eigensolver.  References: numpy in complex128.
"""
import numpy as np
import pytest

from paper_2212_09782_amd import inputs, lib

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ctx():
    c = lib.Context(0)
    yield c
    c.close()


def to_dev(a, dt):
    cdt = torch.complex128 if dt == lib.DT_C128 else torch.complex64
    return torch.from_numpy(np.ascontiguousarray(a).reshape(-1)).to(cdt).to("cuda")


def op(a, o):
    return a if o == 0 else (a.T if o == 1 else a.conj().T)


GEMM_SHAPES = [(1, 1, 1), (17, 33, 5), (64, 64, 16), (130, 70, 200), (5, 300, 1000), (257, 129, 65),
               (128, 128, 16), (300, 260, 47), (513, 640, 300)]


@pytest.mark.parametrize("dt", [lib.DT_C128, lib.DT_C64])
@pytest.mark.parametrize("opA", [0, 1, 2])
@pytest.mark.parametrize("opB", [0, 1, 2])
@pytest.mark.parametrize("MNK", GEMM_SHAPES)
def test_zgemm(ctx, dt, opA, opB, MNK):
    M, N, K = MNK
    print(f"zgemm dt={dt} op={opA}{opB} MNK={MNK}", flush=True)
    r = inputs.rng(1000 + M + N + K)
    A = inputs.gaussian_complex((M, K) if opA == 0 else (K, M), r)
    B = inputs.gaussian_complex((K, N) if opB == 0 else (N, K), r)
    C0 = inputs.gaussian_complex((M, N), r)
    if dt == lib.DT_C64:
        A, B, C0 = (x.astype(np.complex64).astype(np.complex128) for x in (A, B, C0))
    ref = op(A, opA) @ op(B, opB)
    dA, dB = to_dev(A, dt), to_dev(B, dt)
    dC = to_dev(C0, dt)
    lib.mps_zgemm(ctx, dt, opA, opB, M, N, K, dA, A.shape[1], dB, B.shape[1], dC, N, 1.0, 0.0)
    got = dC.cpu().numpy().reshape(M, N).astype(np.complex128)
    tol = 1e-13 if dt == lib.DT_C128 else 3e-6 * np.sqrt(K)
    assert np.linalg.norm(got - ref) <= tol * np.linalg.norm(ref)
    # C = C0 - op(A) op(B)
    dC = to_dev(C0, dt)
    lib.mps_zgemm(ctx, dt, opA, opB, M, N, K, dA, A.shape[1], dB, B.shape[1], dC, N, -1.0, 1.0)
    got = dC.cpu().numpy().reshape(M, N).astype(np.complex128)
    ref2 = C0 - ref
    assert np.linalg.norm(got - ref2) <= tol * (np.linalg.norm(ref) + np.linalg.norm(C0))


QR_SHAPES = [(1, 1), (5, 3), (40, 40), (100, 33), (300, 70), (1000, 64), (2600, 130), (700, 700)]


def _qr_check(ctx, A, dt, tol_res, tol_orth):
    m, n = A.shape
    dA = to_dev(A, dt)
    dQ = torch.zeros(m * n, dtype=dA.dtype, device="cuda")
    lib.mps_qr(ctx, dt, m, n, dA, dQ)
    ctx.sync()
    Rf = dA.cpu().numpy().reshape(m, n).astype(np.complex128)
    R = np.triu(Rf[:n])
    Q = dQ.cpu().numpy().reshape(m, n).astype(np.complex128)
    assert np.linalg.norm(A - Q @ R) <= tol_res * np.linalg.norm(A)
    assert np.max(np.abs(Q.conj().T @ Q - np.eye(n))) <= tol_orth
    return Q, R


@pytest.mark.parametrize("dt", [lib.DT_C128, lib.DT_C64])
@pytest.mark.parametrize("mn", QR_SHAPES)
def test_qr(ctx, dt, mn):
    m, n = mn
    print(f"qr dt={dt} shape={mn}", flush=True)
    A = inputs.gaussian_complex((m, n), inputs.rng(m * 7 + n))
    if dt == lib.DT_C64:
        A = A.astype(np.complex64).astype(np.complex128)
    tol = (1e-13, 1e-13) if dt == lib.DT_C128 else (2e-5, 2e-5)
    Q, R = _qr_check(ctx, A, dt, *tol)
    # |R_ii| is gauge invariant (numpy's Householder QR)
    Rn = np.linalg.qr(A, mode="r")
    assert np.allclose(np.abs(np.diag(R)), np.abs(np.diag(Rn)), rtol=1e-9 if dt == lib.DT_C128 else 1e-3,
                       atol=1e-12 if dt == lib.DT_C128 else 1e-4)


@pytest.mark.parametrize("mnr", [(200, 64, 5), (1000, 100, 1), (513, 96, 40)])
def test_qr_rank_deficient(ctx, mnr):
    """Rank r < n: Q must still be an exact isometry, and span col(A)."""
    m, n, rk = mnr
    r = inputs.rng(77 + m)
    A = inputs.gaussian_complex((m, rk), r) @ inputs.gaussian_complex((rk, n), r)
    Q, R = _qr_check(ctx, A, lib.DT_C128, 1e-13, 1e-13)
    P = Q @ Q.conj().T
    assert np.linalg.norm(P @ A - A) <= 1e-13 * np.linalg.norm(A)


@pytest.mark.parametrize("dt", [lib.DT_C128, lib.DT_C64])
@pytest.mark.parametrize("mnc", [(1000, 64, 1e10), (2600, 96, 1e6), (5000, 40, 1e13)])
def test_qr_ill_conditioned(ctx, dt, mnc):
    """Full rank with condition number cond (singular vectors mixed on both
    sides): panels whose Gram-matrix Cholesky loses orthogonality fall back to
    the column-by-column Householder loop; Q stays an isometry spanning A."""
    m, n, cond = mnc
    print(f"qr ill-conditioned dt={dt} shape={(m, n)} cond={cond:g}", flush=True)
    r = inputs.rng(91 + m)
    W = np.linalg.qr(inputs.gaussian_complex((m, n), r))[0]
    A = (W * np.logspace(0, -np.log10(cond), n)[None, :]) @ inputs.random_unitary(n, r)
    if dt == lib.DT_C64:
        A = A.astype(np.complex64).astype(np.complex128)
    tol = (1e-13, 1e-13) if dt == lib.DT_C128 else (2e-5, 2e-5)
    Q, R = _qr_check(ctx, A, dt, *tol)
    P = Q @ Q.conj().T
    assert np.linalg.norm(P @ A - A) <= tol[0] * np.linalg.norm(A)


def _herm(n, kind, r):
    if kind == "random":
        G = inputs.gaussian_complex((n, n), r)
        return (G + G.conj().T) / 2
    if kind == "gram":  # L^dag L with a rank deficiency, like CBE step (iv)
        L = np.tril(inputs.gaussian_complex((n, n), r))
        L[:, n // 3:] *= np.logspace(0, -9, n - n // 3)[None, :]
        L[:, -max(1, n // 10):] = 0
        return L.conj().T @ L
    if kind == "degenerate":  # exact pairs, as from a Z_d symmetric spectrum
        w = np.repeat(np.sort(r.uniform(0, 1, (n + 1) // 2))[::-1], 2)[:n]
        U = inputs.random_unitary(n, r)
        return (U * w[None, :]) @ U.conj().T
    if kind == "cluster":  # two large clusters (one at the top, ragged panel tail) among distinct values
        w = np.sort(r.uniform(0.1, 1, n))[::-1]
        c1, c2 = min(97, n // 4), min(300, n // 3)
        w[:c1] = 1.0 + 1e-14 * r.standard_normal(c1)
        w[n // 2:n // 2 + c2] = 0.5 + 1e-15 * r.standard_normal(c2)
        w = np.sort(w)[::-1]
        U = inputs.random_unitary(n, r)
        return (U * w[None, :]) @ U.conj().T
    raise ValueError(kind)


HEIG = [(n, kind, n if n < 10 else (n * 3) // 4) for n in (1, 2, 3, 17, 64, 100, 257, 600)
        for kind in ("random", "gram", "degenerate")]
HEIG += [(1127, "gram", 1024), (1127, "random", 1127), (1536, "gram", 1536), (1536, "degenerate", 1152)]
HEIG += [(200, "cluster", 200), (600, "cluster", 450), (1127, "cluster", 1024), (1536, "cluster", 1536)]


@pytest.mark.parametrize("n,kind,k", HEIG, ids=[f"n{n}-{kind}-k{k}" for n, kind, k in HEIG])
def test_heig(ctx, n, kind, k):
    """Eigenvalues against numpy's eigvalsh, eigenvectors by orthonormality and
    residual; n = 1127, k = 1024 is the eigen-decomposition of the headline
    bond update, n = 1536 the largest eta the library accepts."""
    print(f"heig n={n} kind={kind} k={k}", flush=True)
    r = inputs.rng(n + 11)
    G = _herm(n, kind, r)
    dG = to_dev(G, lib.DT_C128)
    lam = torch.zeros(k, dtype=torch.float64, device="cuda")
    E = torch.zeros(n * k, dtype=torch.complex128, device="cuda")
    lib.mps_heig(ctx, n, k, dG, lam, E)
    ctx.sync()
    lam = lam.cpu().numpy()
    E = E.cpu().numpy().reshape(n, k)
    w = np.linalg.eigvalsh(G)[::-1][:k]
    nrm = max(np.max(np.abs(w)), 1e-300)
    assert np.max(np.abs(lam - w)) <= 1e-12 * nrm
    assert np.max(np.abs(E.conj().T @ E - np.eye(k))) <= 1e-12
    res = G @ E - E * lam[None, :]
    assert np.linalg.norm(res) <= 1e-11 * nrm * np.sqrt(n)
