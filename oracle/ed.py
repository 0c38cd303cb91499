"""Exact state-vector evolution of an open clock chain (oracle pins).

Test infrastructure only (see the package docstring).

Two references, both independent of any MPS code:
  trotter_circuit  the same even/odd gate sequence as the TEBD sweep, applied
                   to the full state vector (no truncation, so TEBD with an
                   untruncated bond must reproduce it up to rounding);
  exact_evolve     exp(-i t H) |psi> with H built directly from the paper's
                   Hamiltonian (Sec. IV), via scipy's expm_multiply.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import clock


def product_vector(L, d, k=0):
    psi = np.zeros(d ** L, np.complex128)
    idx = 0
    for _ in range(L):
        idx = idx * d + k
    psi[idx] = 1.0
    return psi


def apply_two_site(psi, U, m, L, d):
    """Apply a d^2 x d^2 gate to sites (m, m+1) of a state vector."""
    t = psi.reshape(d ** m, d * d, d ** (L - m - 2))
    return np.einsum("kl,alb->akb", U, t).reshape(-1)


def apply_one_site(psi, O, m, L, d):
    t = psi.reshape(d ** m, d, d ** (L - m - 1))
    return np.einsum("kl,alb->akb", O, t).reshape(-1)


def trotter_circuit(psi, gates_half, gates_full, L, d, nsteps, order=2):
    """Even/odd Trotter circuit on the state vector (the sequence of Fig. 2a)."""
    even = list(range(0, L - 1, 2))
    odd = list(range(1, L - 1, 2))
    for _ in range(nsteps):
        if order == 2:
            for m in even:
                psi = apply_two_site(psi, gates_half[m], m, L, d)
            for m in odd:
                psi = apply_two_site(psi, gates_full[m], m, L, d)
            for m in even:
                psi = apply_two_site(psi, gates_half[m], m, L, d)
        else:
            for m in even:
                psi = apply_two_site(psi, gates_full[m], m, L, d)
            for m in odd:
                psi = apply_two_site(psi, gates_full[m], m, L, d)
    return psi


def sparse_hamiltonian(d, g, L):
    """Sparse H of the open chain, built term by term from Sec. IV."""
    Z, X = clock.clock_ops(d)
    I = sp.identity(d, dtype=np.complex128, format="csr")

    def site_op(op, n):
        out = sp.identity(1, dtype=np.complex128, format="csr")
        for k in range(L):
            out = sp.kron(out, sp.csr_matrix(op) if k == n else I, format="csr")
        return out

    H = sp.csr_matrix((d ** L, d ** L), dtype=np.complex128)
    for n in range(L - 1):
        t = site_op(Z, n) @ site_op(Z.conj().T, n + 1)
        H = H - (t + t.conj().T)
    for n in range(L):
        x = site_op(X, n)
        H = H - g * (x + x.conj().T)
    return H.tocsr()


def exact_evolve(psi, H, t):
    return spla.expm_multiply(-1j * t * H, psi)


def site_expectations(psi, O, L, d):
    return np.array([np.vdot(psi, apply_one_site(psi, O, m, L, d)) for m in range(L)])


def cut_entropy(psi, m, L, d):
    """Von Neumann entropy -Tr rho ln rho of sites 0..m-1 (Sec. IV, Fig. 4 quantity).

    rho is the reduced density matrix Psi Psi^dag of the state vector viewed
    as the d^m x d^(L-m) matrix Psi, normalised to unit trace; its spectrum
    comes from numpy's Hermitian eigensolver.  This is the definition of the
    bipartite entanglement entropy, independent of any MPS form.
    """
    P = psi.reshape(d ** m, d ** (L - m))
    rho = P @ P.conj().T
    w = np.linalg.eigvalsh(rho / np.trace(rho).real)
    w = w[w > 1e-300]
    return float(-np.sum(w * np.log(w)))


def sequential_circuit(psi, gates_half, L, d, nsteps):
    """The gate order of a second-order sequential sweep on the state vector:
    per step U_b(dt/2) for b = 0 .. L-2, then b = L-2 .. 0."""
    for _ in range(nsteps):
        for m in list(range(L - 1)) + list(range(L - 2, -1, -1)):
            psi = apply_two_site(psi, gates_half[m], m, L, d)
    return psi
