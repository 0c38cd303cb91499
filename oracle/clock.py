"""The d-state quantum clock model and its two-site Trotter gates (oracle).

Test infrastructure only (see the package docstring).

Paper, Sec. IV: H = -sum_n (Z_n Z_{n+1}^dag + h.c.) - g sum_n (X_n + X_n^dag),
with Z = diag(1, w, ..., w^{d-1}), w = exp(2 pi i / d), and X the cyclic shift
with ones on the first super-diagonal and in the bottom-left corner.

Bond split (a reading; the paper only gives H as a sum): every on-site term is
shared equally by the two bonds that touch the site, so an interior bond
carries g/2 of each neighbour's transverse field; on a finite chain the first
and last site have one bond only and give it their full weight.  The state is
evolved with U = expm(-i tau h_bond) acting on |i>|j>, row index i*d + j with i
the left site (the matrix form of the gate sum in Sec. II, step (i)).
"""
import numpy as np
import scipy.linalg


def clock_ops(d):
    """Z and X of Sec. IV (the clock and shift matrices), complex128 d x d."""
    w = np.exp(2j * np.pi / d)
    Z = np.diag(w ** np.arange(d)).astype(np.complex128)
    X = np.zeros((d, d), np.complex128)
    for k in range(d):
        X[k, (k + 1) % d] = 1.0
    return Z, X


def bond_hamiltonian(d, g, wl=0.5, wr=0.5):
    """Two-site term h = -(Z x Z^dag + h.c.) - g (wl (X+X^dag) x 1 + wr 1 x (X+X^dag)).

    wl, wr: the share of the left / right site's transverse field carried by
    this bond (1/2 in the bulk, 1 at a finite chain's end).
    """
    Z, X = clock_ops(d)
    I = np.eye(d, dtype=np.complex128)
    zz = np.kron(Z, Z.conj().T)
    xs = X + X.conj().T
    return -(zz + zz.conj().T) - g * (wl * np.kron(xs, I) + wr * np.kron(I, xs))


def gate(h, tau):
    """U = expm(-i tau h), the Trotter gate of one bond for a time step tau."""
    return scipy.linalg.expm(-1j * tau * h)


def bond_weights(L, finite):
    """(wl, wr) for every bond.

    Finite chain of L sites: bond b joins sites b and b+1 (b = 0..L-2).
    Uniform two-site cell (L == 2, finite False): bond 0 joins A,B and bond 1
    joins B,A; both are bulk bonds.
    """
    if not finite:
        return [(0.5, 0.5)] * L
    out = []
    for b in range(L - 1):
        wl = 1.0 if b == 0 else 0.5
        wr = 1.0 if b + 1 == L - 1 else 0.5
        out.append((wl, wr))
    return out


def chain_hamiltonians(d, g, L, finite):
    """Bond Hamiltonians for every bond of the chain (see bond_weights)."""
    return [bond_hamiltonian(d, g, wl, wr) for (wl, wr) in bond_weights(L, finite)]


def full_hamiltonian_dense(d, g, L):
    """Dense H of the open chain of L sites, straight from Sec. IV (no bond split).

    Only for tiny L; used to pin the bond split and the energy bookkeeping.
    """
    Z, X = clock_ops(d)
    I = np.eye(d, dtype=np.complex128)

    def site_op(op, n):
        mats = [I] * L
        mats[n] = op
        out = mats[0]
        for m in mats[1:]:
            out = np.kron(out, m)
        return out

    H = np.zeros((d ** L, d ** L), np.complex128)
    for n in range(L - 1):
        t = site_op(Z, n) @ site_op(Z.conj().T, n + 1)
        H -= t + t.conj().T
    for n in range(L):
        x = site_op(X, n)
        H -= g * (x + x.conj().T)
    return H
