"""Seeded synthetic inputs for the bond update, the sweeps and the serving loop.

This module only draws random numbers and arranges them into the shapes and
forms the method expects as input; it computes no step of the method (no gate,
no contraction, no truncation).  Both the HIP path and the CPU oracle take
their inputs from here.

All generators use numpy's PCG64 with an explicit seed.
"""
import numpy as np


def rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def gaussian_complex(shape, r):
    """Re and Im i.i.d. N(0, 1), complex128."""
    return r.standard_normal(shape) + 1j * r.standard_normal(shape)


def right_isometric(chi_l, d, chi_r, r):
    """Gaussian tensor [chi_l, d, chi_r] made right-isometric.

    Rows of the chi_l x (d chi_r) matrix are orthonormalised (the Q of a QR of
    the conjugate transpose), so sum_{i,b} B[a,i,b] conj(B[a',i,b]) = delta.
    Requires chi_l <= d chi_r.
    """
    assert chi_l <= d * chi_r
    G = gaussian_complex((chi_l, d * chi_r), r)
    Q, _ = np.linalg.qr(G.conj().T, mode="reduced")
    return np.ascontiguousarray(Q.conj().T.reshape(chi_l, d, chi_r))


def random_lambda(chi, r):
    """Positive bond weights: sorted U(0,1) draws, descending, unit 2-norm."""
    u = np.sort(r.uniform(0.0, 1.0, chi))[::-1].copy()
    return u / np.linalg.norm(u)


def random_unitary(n, r):
    """Haar-like random unitary (QR of a complex Gaussian with phase fix)."""
    G = gaussian_complex((n, n), r)
    Q, R = np.linalg.qr(G)
    ph = np.diag(R) / np.abs(np.diag(R))
    return Q * ph[None, :]


def near_identity_unitary(n, r, scale=0.05):
    """exp(-i s H) for a random Hermitian H of unit spectral scale: a gate close to 1."""
    G = gaussian_complex((n, n), r)
    H = (G + G.conj().T) / (2 * np.sqrt(n))
    w, V = np.linalg.eigh(H)
    return (V * np.exp(-1j * scale * w)[None, :]) @ V.conj().T


def microbench_cell(chi, d, seed=0):
    """Two-site uniform cell of the single-bond microbenchmark.

    A and B: Gaussian, right-isometric, shape [chi, d, chi] (seeds seed, seed+1);
    Lambda_A, Lambda_B: random positive weights (seeds seed+2, seed+3).
    """
    A = right_isometric(chi, d, chi, rng(seed))
    B = right_isometric(chi, d, chi, rng(seed + 1))
    lA = random_lambda(chi, rng(seed + 2))
    lB = random_lambda(chi, rng(seed + 3))
    return A, B, lA, lB


def random_bond(chi_l, chi_m, chi_r, d, seed, diag_xi=True):
    """One bond's inputs: Xi^[m] (chi_l), B^[m] [chi_l,d,chi_m], B^[n] [chi_m,d,chi_r].

    diag_xi False gives a dense lower-triangular Xi with unit Frobenius norm
    (the shape of the bond matrix after a plain QR update).
    """
    r = rng(seed)
    bm = right_isometric(chi_l, d, chi_m, r)
    bn = right_isometric(chi_m, d, chi_r, r)
    if diag_xi:
        xi = random_lambda(chi_l, r)
    else:
        xi = np.tril(gaussian_complex((chi_l, chi_l), r))
        xi = xi / np.linalg.norm(xi)
    return xi, bm, bn


def chi_profile_finite(L, d, chi_max):
    """Bond dimensions of a saturated finite chain: min(d^b, d^(L-b), chi_max), b=1..L-1."""
    out = []
    for b in range(1, L):
        out.append(int(min(d ** min(b, 30), d ** min(L - b, 30), chi_max)))
    return out


def random_finite_mps(L, d, chi_max, seed):
    """Random right-isometric finite MPS on the saturated profile, diagonal Xi on every bond."""
    r = rng(seed)
    chis = [1] + chi_profile_finite(L, d, chi_max) + [1]
    B = [right_isometric(chis[m], d, chis[m + 1], r) for m in range(L)]
    Xi = [np.ones(1)] + [random_lambda(chis[m], r) for m in range(1, L)]
    return dict(B=B, Xi=Xi, finite=True)


def serving_requests(n=64, rate=4.0, seed=5):
    """Poisson request stream: arrival times and per-request parameters.

    Each request draws d in {2,3,4,5,8}, g ~ U[0.5,3], chi_max in
    {64,128,256,512,1024} and a geometry in {finite L=32, finite L=64,
    uniform two-site cell}.
    """
    r = rng(seed)
    gaps = r.exponential(1.0 / rate, n)
    t = np.cumsum(gaps) - gaps[0]
    reqs = []
    for k in range(n):
        q = rng(6 + k)
        geo = int(q.integers(0, 3))
        reqs.append(dict(
            arrival=float(t[k]),
            d=int(q.choice([2, 3, 4, 5, 8])),
            g=float(q.uniform(0.5, 3.0)),
            chi_max=int(q.choice([64, 128, 256, 512, 1024])),
            finite=geo < 2,
            L=[32, 64, 2][geo],
        ))
    return reqs


# ---- Z_d block structure (charge basis: eigenbasis of the clock model's shift X)

def sym_sectors(chi, d):
    """chi split into d charge sectors as evenly as possible (lower charges first)."""
    return [chi // d + (1 if a < chi % d else 0) for a in range(d)]


def sym_offsets(sec):
    return np.concatenate([[0], np.cumsum(sec)]).astype(int)


def random_sym_tensor(sec_l, sec_r, d, r):
    """Right-isometric tensor [chi_l, d, chi_r] with the Z_d block structure.

    Virtual indices run over the charge sectors in order; B[alpha, q, beta] is
    nonzero only where charge(beta) = charge(alpha) + q mod d.  For every left
    sector a the rows restricted to their allowed columns are Gaussian, then
    orthonormalised (Q of a QR of the conjugate transpose); needs
    sec_l[a] <= chi_r.
    """
    oL, oR = sym_offsets(sec_l), sym_offsets(sec_r)
    chiL, chiR = int(oL[-1]), int(oR[-1])
    B = np.zeros((chiL, d, chiR), np.complex128)
    for a in range(d):
        if sec_l[a] == 0:
            continue
        cols = [(q, beta) for q in range(d) for beta in range(oR[(a + q) % d], oR[(a + q) % d + 1])]
        assert sec_l[a] <= len(cols)
        G = gaussian_complex((sec_l[a], len(cols)), r)
        Q, _ = np.linalg.qr(G.conj().T, mode="reduced")
        rows = Q.conj().T
        for k, (q, beta) in enumerate(cols):
            B[oL[a]:oL[a + 1], q, beta] = rows[:, k]
    return B


def random_sym_bond(sec_l, sec_m, sec_r, d, seed):
    """(Xi^[m], B^[m], B^[n]) of one bond with the Z_d block structure: Xi a
    positive diagonal (unit 2-norm, descending inside every sector), B^[m] and
    B^[n] right-isometric block-sparse tensors."""
    r = rng(seed)
    xi = np.concatenate([np.sort(r.uniform(0.0, 1.0, n))[::-1] for n in sec_l])
    xi = xi / np.linalg.norm(xi)
    bm = random_sym_tensor(sec_l, sec_m, d, r)
    bn = random_sym_tensor(sec_m, sec_r, d, r)
    return xi, bm, bn


def charge_product_cell(d):
    """Uniform two-site cell in the product state with charge 0 on every site
    (|q=0> in the charge basis, the uniform superposition of the clock states):
    tensors [1, d, 1] and unit bond weights, one sector of size 1 (charge 0)
    on both bonds."""
    e0 = np.zeros((1, d, 1), np.complex128)
    e0[0, 0, 0] = 1.0
    sec = [1] + [0] * (d - 1)
    return [e0, e0.copy()], [np.ones(1), np.ones(1)], [sec, list(sec)]


def random_charge_gate(d, r, scale=0.1):
    """exp(-i s H) for a random Hermitian two-site H that conserves q_i + q_j
    mod d (block diagonal over the total charge, row index q_i d + q_j): a
    charge-conserving gate close to 1 in the charge basis."""
    H = np.zeros((d * d, d * d), np.complex128)
    for s in range(d):
        idx = [q * d + (s - q) % d for q in range(d)]
        G = gaussian_complex((d, d), r)
        H[np.ix_(idx, idx)] = (G + G.conj().T) / (2 * np.sqrt(d))
    w, V = np.linalg.eigh(H)
    return (V * np.exp(-1j * scale * w)[None, :]) @ V.conj().T
