"""Finite and uniform MPS in right-isometric form, TEBD sweep and observables (oracle).

Test infrastructure only (see the package docstring).

State layout (a plain dict, shared with the tests only):
  'B'      list of site tensors [chi_left, d, chi_right], right-isometric (Sec. II)
  'Xi'     list of bond matrices; Xi[m] is the bond left of site m (1-D diagonal
           or 2-D matrix).  Finite chain: Xi[0] = [1] (open end), the last
           site has chi_right = 1, and bond m joins sites m, m+1.  Uniform
           two-site cell: sites A=0, B=1; bond 0 is (A,B), bond 1 is (B,A).
  'finite' bool

Sweep (Fig. 2a): gates act alternately on even and odd bonds.  Second order
(a reading): even(dt/2), odd(dt), even(dt/2) per step, half steps never merged.
"""
import numpy as np

from . import bond as _bond


def product_state(L, d, finite=True, k=0):
    """|k k ... k> as an MPS with every bond dimension 1 (Sec. IV quench start, k=0)."""
    e = np.zeros((1, d, 1), np.complex128)
    e[0, k, 0] = 1.0
    B = [e.copy() for _ in range(L)]
    Xi = [np.ones(1) for _ in range(L)]
    return dict(B=B, Xi=Xi, finite=finite)


def bonds_of_layer(L, finite, parity):
    """Site pairs (m, n) updated in the even (parity 0) or odd (parity 1) layer."""
    if finite:
        return [(m, m + 1) for m in range(parity, L - 1, 2)]
    return [(m, (m + 1) % L) for m in range(parity, L, 2)]


def apply_layer(state, gates, parity, mode, dchi_rule, chi_max, svd_min, scheme="qr", nsweeps=1, log=None,
                eig_backward=None):
    """Update every bond of one layer; gates[b] is the gate of the bond starting at site b.

    dchi_rule(chi_m) gives the expansion dchi used for eta (Sec. III); nsweeps
    QR/LQ sweeps per bond (Sec. II comments).  Returns the list of truncation
    errors.  log (a list, optional) receives per bond the site m, the Schmidt
    values S of the update and the kept number chi~ (bookkeeping for tests
    that need the spectrum at the cut); eig_backward is passed to every
    update (see bond.qr_bond_update).
    """
    B, Xi, finite = state["B"], state["Xi"], state["finite"]
    L = len(B)
    eps = []
    for (m, n) in bonds_of_layer(L, finite, parity):
        bm, bn = B[m], B[n]
        chiL, d, chiM = bm.shape
        chiR = bn.shape[2]
        if scheme == "svd":
            r = _bond.svd_bond_update(Xi[m], bm, bn, gates[m], chi_max=chi_max, svd_min=svd_min)
        else:
            eta = chiM if mode == _bond.PLAIN else _bond.eta_cbe(chiL, chiM, chiR, d, dchi_rule(chiM))
            r = _bond.qr_bond_update(Xi[m], bm, bn, gates[m], mode=mode, eta=eta,
                                     chi_max=chi_max, svd_min=svd_min, nsweeps=nsweeps,
                                     eig_backward=eig_backward)
        B[m], B[n], Xi[n] = r["bm"], r["bn"], r["xi"]
        eps.append(r["eps"])
        if log is not None:
            log.append(dict(m=m, S=np.asarray(r["S"]), chi=r["chi"], eps=r["eps"]))
    return eps


def trotter_step(state, gates_half, gates_full, order=2, mode=_bond.CBE,
                 dchi_rule=lambda c: max(100, -(-c // 10)), chi_max=None,
                 svd_min=1e-14, scheme="qr", nsweeps=1, log=None, eig_backward=None):
    """One Trotter step of length dt (Fig. 2a).

    order 2: even(dt/2) odd(dt) even(dt/2);  order 1: even(dt) odd(dt), where
    gates_half / gates_full are the per-bond gates for dt/2 / dt.
    Returns the summed truncation error of the step (log, eig_backward: see
    apply_layer).
    """
    kw = dict(mode=mode, dchi_rule=dchi_rule, chi_max=chi_max, svd_min=svd_min, scheme=scheme, nsweeps=nsweeps,
              log=log, eig_backward=eig_backward)
    eps = []
    if order == 2:
        eps += apply_layer(state, gates_half, 0, **kw)
        eps += apply_layer(state, gates_full, 1, **kw)
        eps += apply_layer(state, gates_half, 0, **kw)
    else:
        eps += apply_layer(state, gates_full, 0, **kw)
        eps += apply_layer(state, gates_full, 1, **kw)
    return float(np.sum(eps))


def _xiB(xi, b):
    if np.ndim(xi) == 1:
        return xi[:, None, None] * b
    return np.tensordot(xi, b, axes=([1], [0]))


def site_expectation(state, op):
    """<O_m> for every site from M = Xi^[m] B^[m] (Fig. 1c), divided by |M|^2.

    Returns (values complex [L], norms real [L]).
    """
    vals, norms = [], []
    for m, b in enumerate(state["B"]):
        M = _xiB(state["Xi"][m], b)
        OM = np.einsum("ij,ajb->aib", op, M)
        n2 = float(np.vdot(M, M).real)
        vals.append(np.vdot(M, OM) / n2)
        norms.append(n2)
    return np.array(vals), np.array(norms)


def bond_expectation(state, hs):
    """<h_b> for every bond b from theta = Xi^[m] B^[m] B^[n], divided by |theta|^2."""
    B, Xi, finite = state["B"], state["Xi"], state["finite"]
    L = len(B)
    pairs = bonds_of_layer(L, finite, 0) + bonds_of_layer(L, finite, 1)
    pairs.sort()
    vals = []
    for (m, n) in pairs:
        th = np.tensordot(_xiB(Xi[m], B[m]), B[n], axes=([2], [0]))  # [a, i, j, b]
        d = th.shape[1]
        hth = np.einsum("kl,alb->akb", hs[m], th.reshape(th.shape[0], d * d, th.shape[3]))
        vals.append(np.vdot(th.reshape(hth.shape), hth) / np.vdot(th, th).real)
    return np.array(vals)


def bond_entropies(state):
    """Von Neumann entropy -sum p ln p, p = s^2/sum s^2, s = singular values of Xi (Sec. II)."""
    out = []
    for xi in state["Xi"]:
        s = np.abs(xi) if np.ndim(xi) == 1 else np.linalg.svd(xi, compute_uv=False)
        p = s ** 2 / np.sum(s ** 2)
        p = p[p > 0]
        out.append(float(-np.sum(p * np.log(p))))
    return np.array(out)


def to_statevector(state):
    """Full contraction Xi^[0] B^[0] ... B^[L-1] of a finite chain (tiny L only)."""
    assert state["finite"]
    B = state["B"]
    psi = _xiB(state["Xi"][0], B[0])
    for b in B[1:]:
        psi = np.tensordot(psi, b, axes=([psi.ndim - 1], [0]))
    return psi.reshape(-1)


def chi_profile(state):
    return [b.shape[2] for b in state["B"]]


# ---- sequential sweeps in the left-isometric form (Sec. II, comments) ----
#
# The QR truncation hands back the new left tensor in left-isometric form,
# A~^[m] = Q^[m], with the bond matrix L (normalised) between m and n and the
# right-isometric B~^[n] = Q^[n].  Keeping that form instead of Hastings' B~^[m]
# lets the update run on a finite chain sweeping to the right: the next bond
# (n, n+1) sees the bond matrix just produced on its left and right-isometric
# tensors on its right.  Reading taken for the return sweep: it is the same
# update applied to the mirror image of the chain (site order reversed, each
# tensor's two virtual legs exchanged, each gate's two sites exchanged), so a
# step of gates G_b(dt/2) for b = 0 .. L-2 followed by b = L-2 .. 0 is
# symmetric (second order) and returns the chain to right-isometric form with
# the bond matrix [[1]] at its left end.


def reflect_tensor(t):
    """Exchange the two virtual legs: [a, i, b] -> [b, i, a]."""
    return np.ascontiguousarray(t.transpose(2, 1, 0))


def reflect_gate(U, d):
    """The gate with its two sites exchanged: (i j),(i' j') -> (j i),(j' i')."""
    return np.ascontiguousarray(U.reshape(d, d, d, d).transpose(1, 0, 3, 2).reshape(d * d, d * d))


def left_sweep(B, center, gates, mode, eta_rule, chi_max=None):
    """Update bonds 0 .. L-2 in order with A~^[b] = Q^[b] (returns the new
    site list; the last site absorbs the final bond matrix from the left).

    B: right-isometric sites, center: dense bond matrix left of site 0.
    mode PLAIN (eta = chi_m) or GROW (eta = eta_rule(chi_l, chi_m, chi_r)).
    """
    B = list(B)
    L = len(B)
    xi = center
    for b in range(L - 1):
        chiL, d, chiM = B[b].shape
        chiR = B[b + 1].shape[2]
        eta = chiM if mode == _bond.PLAIN else eta_rule(chiL, chiM, chiR, d)
        r = _bond.qr_bond_update(xi, B[b], B[b + 1], gates[b], mode=mode, eta=eta, chi_max=chi_max)
        B[b] = r["Q"].reshape(chiL, d, r["Q"].shape[1])
        B[b + 1] = r["bn"]
        xi = r["xi"]
    B[L - 1] = np.tensordot(xi, B[L - 1], axes=([1], [0]))
    return B


def sequential_step(state, gates_half, mode=_bond.PLAIN, eta_rule=None, chi_max=None):
    """One second-order step of sequential sweeps (see the comment above):
    gates_half[b] = U(dt/2) of bond b.  state: finite chain in right-isometric
    form with Xi[0] the dense bond matrix [[1]] at the left end; updated in
    place (afterwards Xi[0] = [[1]] again, other Xi entries are not kept)."""
    assert state["finite"]
    B = state["B"]
    L = len(B)
    d = B[0].shape[1]
    B = left_sweep(B, np.atleast_2d(state["Xi"][0]).astype(np.complex128), gates_half, mode, eta_rule, chi_max)
    R = [reflect_tensor(t) for t in B[::-1]]
    gr = [reflect_gate(U, d) for U in gates_half[:L - 1][::-1]]
    R = left_sweep(R, np.ones((1, 1), np.complex128), gr, mode, eta_rule, chi_max)
    state["B"] = [reflect_tensor(t) for t in R[::-1]]
    state["Xi"] = [np.ones((1, 1), np.complex128)] + [None] * (L - 1)
    return state
