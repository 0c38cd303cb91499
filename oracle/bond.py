"""One two-site bond update (oracle), complex128.

Test infrastructure only (see the package docstring).

Conventions shared with the tests (not with any GPU code):
  B tensors are arrays [chi_left, d, chi_right] in right-isometric form
  (sum_{i,beta} B[a,i,beta] conj(B[a',i,beta]) = delta_{a a'}, Sec. II).
  Xi (the bond matrix left of site m) is either a 1-D array (diagonal, e.g.
  Schmidt values) or a 2-D chi_left x chi_left matrix (Sec. II).
  The two-site tensor is viewed as the matrix with rows (alpha, i) and columns
  (j, delta), alpha-major / j-major.

Readings taken where the paper leaves a choice (each also listed in the design
notes of the repository):
  * theta uses the bond matrix left of site m, Xi^[m].
  * eta is an input; it must satisfy eta <= min(d chi_L, d chi_R).
  * The eta-slice of controlled bond expansion keeps the first eta rows of
    theta in (alpha, i) order (alpha-major).
  * Truncation keeps Schmidt values S >= svd_min (absolute), at most chi_max,
    at least one; eigenvalues are sorted descending with a stable sort.
  * The new bond matrix is normalised to unit Frobenius norm.
  * The truncation error is the squared relative distance
    ||theta - approx||^2 / ||theta||^2 between theta and its low-rank
    approximation Q Q^dag theta P (end of Sec. IV).
"""
import numpy as np

PLAIN, GROW, CBE = 0, 1, 2


def two_site(xi, bm, bn, U):
    """Sec. II step (i): C = B^[m] B^[n], C~ = U C, theta~ = Xi^[m] C~.

    Returns (Ct, Th) as matrices of shape (chi_L d, d chi_R): Ct is the gated
    pair without the bond matrix (the Hastings form of step (iii)), Th the
    gated two-site wave function.
    """
    chiL, d, chiM = bm.shape
    chiM2, d2, chiR = bn.shape
    assert chiM == chiM2 and d == d2 and U.shape == (d * d, d * d)
    C = np.tensordot(bm, bn, axes=([2], [0]))            # [a, i', j', b]
    C = C.transpose(1, 2, 0, 3).reshape(d * d, chiL * chiR)  # [(i'j'), (a b)]
    Ct = (U @ C).reshape(d, d, chiL, chiR).transpose(2, 0, 1, 3)  # [a, i, j, b]
    if xi.ndim == 1:
        Th = xi[:, None, None, None] * Ct
    else:
        Th = np.tensordot(xi, Ct, axes=([1], [0]))
    return Ct.reshape(chiL * d, d * chiR), Th.reshape(chiL * d, d * chiR)


def lq(Y):
    """LQ decomposition Y = L Q (Q with orthonormal rows) from numpy's QR of Y^dag."""
    Qp, Rp = np.linalg.qr(Y.conj().T, mode="reduced")
    return Rp.conj().T, Qp.conj().T


def als_truncate(Th, Y0, nsweeps):
    """Iterated QR/LQ sweeps on a fixed theta~ (the ALS reading in Sec. II comments).

    Starting from the isometry Y0 (rows orthonormal), each sweep does
    X = theta~ Y^dag, Q = qr(X), Y = Q^dag theta~, (L, Q^[n]) = lq(Y) and
    restarts from Q^[n].  Returns the list of relative errors
    1 - |Y|^2/|theta~|^2 after each sweep.
    """
    n2 = float(np.vdot(Th, Th).real)
    errs = []
    for _ in range(nsweeps):
        Q, _ = np.linalg.qr(Th @ Y0.conj().T, mode="reduced")
        Y = Q.conj().T @ Th
        _, Y0 = lq(Y)
        errs.append(1.0 - float(np.vdot(Y, Y).real) / n2)
    return errs


def select_chi(S, chi_max, svd_min):
    """Number of kept Schmidt values: S >= svd_min, at most chi_max, at least one.

    S must be sorted descending.
    """
    k = int(np.count_nonzero(S >= svd_min))
    if chi_max is not None:
        k = min(k, int(chi_max))
    return max(k, 1)


def qr_bond_update(xi, bm, bn, U, mode=CBE, eta=None, chi_max=None, svd_min=1e-14, nsweeps=1, eig_backward=None):
    """QR-based bond update, Sec. II (plain / grow) and Sec. III (CBE).

    nsweeps > 1 repeats steps (i)-(ii) from Y0 = Q^[n] of the previous sweep
    (the alternating-least-squares reading of the Sec. II comments); the
    truncation then uses the last sweep's factors.

    eig_backward (tests only): None, or (rng, c) to hand the eigensolver of
    step (iv) L^dag L + E instead of L^dag L, with E a random Hermitian matrix
    of spectral norm c sqrt(n) u |L^dag L|_2 (u = 2^-52, n the order of
    L^dag L): the backward error a stable eigensolver is allowed, with the
    sqrt(n) growth that independent rounding errors of the n-term sums of a
    Householder reduction typically show.  Running the update with and
    without it measures how far two correct FP64 implementations may drift
    apart.

    Returns a dict with
      bm, bn   new tensors [chi_L, d, chi~] and [chi~, d, chi_R]
      xi       new bond matrix between m and n: 1-D (CBE) or 2-D (plain/grow)
      chi      chi~, the new bond dimension
      eps      truncation error (relative, squared distance, end of Sec. IV)
      S        Schmidt values of the QR approximation (CBE: all eta of them)
      norm2    ||theta~||_F^2
      Q, L, Qn intermediate factors (for the pins)
    """
    chiL, d, chiM = bm.shape
    chiR = bn.shape[2]
    Ct, Th = two_site(xi, bm, bn, U)
    norm2 = float(np.vdot(Th, Th).real)

    # Step (i): initial guess Y0 for the right isometry.
    if mode == PLAIN:
        Y0 = bn.reshape(chiM, d * chiR)          # Y0 = B^[n]  (Sec. II)
    else:
        assert eta is not None
        Y0 = Th[:eta, :]                          # eta-slice of theta~ (Sec. III (i))
    # X = theta~ Y0^dag, QR -> Q^[m]  (Sec. II step (i))
    X = Th @ Y0.conj().T
    Q, _ = np.linalg.qr(X, mode="reduced")
    # Y = Q^dag theta~, LQ -> L, Q^[n]  (Sec. II step (ii))
    Y = Q.conj().T @ Th
    L, Qn = lq(Y)
    for _ in range(nsweeps - 1):                  # further sweeps from Y0 = Q^[n]
        Q, _ = np.linalg.qr(Th @ Qn.conj().T, mode="reduced")
        Y = Q.conj().T @ Th
        L, Qn = lq(Y)

    out = dict(Q=Q, L=L, Qn=Qn, norm2=norm2, Ct=Ct, Th=Th)
    if mode in (PLAIN, GROW):
        # Sec. II step (iii): Xi~ = L, B~[n] = Q^[n], B~[m] = C~ B~[n]^dag.
        k = L.shape[0]
        xi_new = L / np.linalg.norm(L)
        bn_new = Qn
        S = np.linalg.svd(L, compute_uv=False)
        kept2 = float(np.sum(np.abs(L) ** 2))
    else:
        # Sec. III (iv): L^dag L = V^dag S^2 V;  (v): B~[n] = P V Q^[n], Xi~ = P S P.
        G = L.conj().T @ L
        if eig_backward is not None:
            rng, c = eig_backward
            n = G.shape[0]
            P = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
            P = (P + P.conj().T) / 2
            G = G + P * (c * np.sqrt(n) * 2.0 ** -52 * np.linalg.norm(G, 2) / np.linalg.norm(P, 2))
        w, E = np.linalg.eigh(G)
        order = np.argsort(-w, kind="stable")
        w, E = w[order], E[:, order]
        S = np.sqrt(np.maximum(w, 0.0))
        k = select_chi(S, chi_max, svd_min)
        V = E.conj().T
        bn_new = V[:k, :] @ Qn
        kept2 = float(np.sum(S[:k] ** 2))
        xi_new = S[:k] / np.sqrt(kept2)
    bm_new = Ct @ bn_new.conj().T                  # Hastings form, Sec. II comments
    # Truncation error: distance between theta~ and Q Q^dag theta~ P (Sec. IV).
    approx = Q @ (Y @ (bn_new.conj().T @ bn_new))
    eps = float(np.vdot(Th - approx, Th - approx).real) / norm2
    out.update(bm=bm_new.reshape(chiL, d, k), bn=bn_new.reshape(k, d, chiR),
               xi=xi_new, chi=k, eps=eps, S=S, kept2=kept2)
    return out


def svd_bond_update(xi, bm, bn, U, chi_max=None, svd_min=1e-14):
    """Reference truncation: SVD-TEBD (scheme (i) of Sec. IV) in the same Hastings form.

    theta~ = U S V^dag, keep chi~ values, B~[n] = V^dag_kept, Xi~ = S_kept/|S_kept|,
    B~[m] = C~ V_kept.
    """
    chiL, d, chiM = bm.shape
    chiR = bn.shape[2]
    Ct, Th = two_site(xi, bm, bn, U)
    norm2 = float(np.vdot(Th, Th).real)
    _, S, Vh = np.linalg.svd(Th, full_matrices=False)
    k = select_chi(S, chi_max, svd_min)
    bn_new = Vh[:k]
    kept2 = float(np.sum(S[:k] ** 2))
    bm_new = Ct @ bn_new.conj().T
    eps = max(0.0, norm2 - kept2) / norm2
    return dict(bm=bm_new.reshape(chiL, d, k), bn=bn_new.reshape(k, d, chiR),
                xi=S[:k] / np.sqrt(kept2), chi=k, eps=eps, S=S, norm2=norm2, kept2=kept2)


def eta_cbe(chi_l, chi_m, chi_r, d, dchi):
    """eta = min(chi_M + dchi, d chi_L, d chi_R) (Sec. III: eta = chi + dchi <= d chi)."""
    return int(min(chi_m + dchi, d * chi_l, d * chi_r))


def invariants(bm, xi_n, bn):
    """Gauge-invariant content of an updated bond (used to compare implementations).

    Returns (pair, sv, M^dag M):
      pair   B~[m] B~[n] as a (chi_L d) x (d chi_R) matrix (independent of the
             gauge of B~[n] because B~[m] = C~ B~[n]^dag)
      sv     singular values of Xi~ (descending)
      MdM    M^dag M with M = Xi~ B~[n] as chi~ x (d chi_R)
    """
    chiL, d, k = bm.shape
    chiR = bn.shape[2]
    pair = bm.reshape(chiL * d, k) @ bn.reshape(k, d * chiR)
    X = np.diag(xi_n) if np.ndim(xi_n) == 1 else xi_n
    sv = np.linalg.svd(X, compute_uv=False)
    M = X @ bn.reshape(k, d * chiR)
    return pair, sv, M.conj().T @ M
