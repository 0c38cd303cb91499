"""ctypes binding of libqrtebd.so with the C-ABI names (include/qrtebd.h).

Argument marshalling only: torch tensors supply device memory and the HIP
stream, every step of the bond update runs in the library's kernels.  There is
no fallback: load() raises if the library is missing or fails to load.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqrtebd.so")

MPS_OK, MPS_ERR_ARG, MPS_ERR_CAPACITY, MPS_ERR_OOM, MPS_ERR_HIP, MPS_ERR_NUMERIC, MPS_ERR_STATE = 0, -1, -2, -3, -4, -5, -6
MPS_C128, MPS_MIXED_C64 = 0, 1
PLAIN, GROW, CBE = 0, 1, 2
DT_C64, DT_C128 = 0, 1

# every function the header declares, for the export check
EXPORTS = [
    "mps_ctx_create", "mps_ctx_destroy", "mps_last_error", "mps_sync", "mps_bond_capacity",
    "mps_workspace_query", "mps_bond_update", "mps_clock_gate", "mps_state_create",
    "mps_state_destroy", "mps_state_chis", "mps_sweep", "mps_measure", "mps_zgemm", "mps_qr",
    "mps_heig", "mps_profile_enable", "mps_profile_read", "mps_bond_update_noalloc", "mps_sweep_stats",
    "mps_clock_hamiltonian", "mps_bond_update_reference", "mps_sweep_sequential",
    "mps_clock_gate_charge", "mps_clock_hamiltonian_charge", "mps_sym_capacity", "mps_sym_workspace_query",
    "mps_bond_update_sym",
]
MPS_SYM_MAX_D = 16
SCHEME_SVD, SCHEME_EIG = 0, 1


class mps_bond_desc(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("chi_l", ctypes.c_int), ("chi_m", ctypes.c_int),
                ("chi_r", ctypes.c_int), ("eta", ctypes.c_int), ("chi_max", ctypes.c_int),
                ("svd_min", ctypes.c_double), ("xi_is_diag", ctypes.c_int), ("mode", ctypes.c_int),
                ("prec", ctypes.c_int), ("sweeps", ctypes.c_int), ("left_iso", ctypes.c_int)]


class mps_sweep_policy(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("chi_max", ctypes.c_int), ("svd_min", ctypes.c_double),
                ("dchi_min", ctypes.c_int), ("dchi_frac", ctypes.c_double), ("sweeps", ctypes.c_int),
                ("exec", ctypes.c_int), ("chunk", ctypes.c_int)]


EXEC_EAGER, EXEC_SPECULATIVE, EXEC_GRAPH = 0, 1, 2


class mps_sym_desc(ctypes.Structure):
    _fields_ = [("d", ctypes.c_int), ("sec_l", ctypes.c_int * MPS_SYM_MAX_D),
                ("sec_m", ctypes.c_int * MPS_SYM_MAX_D), ("sec_r", ctypes.c_int * MPS_SYM_MAX_D),
                ("dchi_min", ctypes.c_int), ("dchi_frac", ctypes.c_double), ("chi_max", ctypes.c_int),
                ("svd_min", ctypes.c_double), ("prec", ctypes.c_int)]


class QrtebdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libqrtebd error {code}: {msg}")
        self.code = code


_lib = None
P = ctypes.c_void_p
I = ctypes.c_int
D = ctypes.c_double
LL = ctypes.c_longlong


def _declare(lib):
    sig = {
        "mps_ctx_create": (I, [I, ctypes.c_char_p, ctypes.POINTER(P)]),
        "mps_ctx_destroy": (I, [P]),
        "mps_last_error": (ctypes.c_char_p, []),
        "mps_sync": (I, [P, P]),
        "mps_bond_capacity": (I, [ctypes.POINTER(mps_bond_desc)]),
        "mps_workspace_query": (I, [P, ctypes.POINTER(mps_bond_desc), ctypes.POINTER(ctypes.c_size_t)]),
        "mps_bond_update": (I, [P, ctypes.POINTER(mps_bond_desc), P, P, P, P, P, P, P, P, P, P]),
        "mps_bond_update_noalloc": (I, [P, ctypes.POINTER(mps_bond_desc), P, P, P, P, P, P, P, P, P, P]),
        "mps_bond_update_reference": (I, [P, ctypes.POINTER(mps_bond_desc), I, P, P, P, P, P, P, P, P, P, P]),
        "mps_clock_gate": (I, [I, D, D, D, D, P]),
        "mps_clock_hamiltonian": (I, [I, D, D, D, P]),
        "mps_clock_gate_charge": (I, [I, D, D, D, D, P]),
        "mps_clock_hamiltonian_charge": (I, [I, D, D, D, P]),
        "mps_sym_capacity": (I, [ctypes.POINTER(mps_sym_desc)]),
        "mps_sym_workspace_query": (I, [P, ctypes.POINTER(mps_sym_desc), ctypes.POINTER(ctypes.c_size_t)]),
        "mps_bond_update_sym": (I, [P, ctypes.POINTER(mps_sym_desc), P, P, P, P, P, P, P, P, P, P, P]),
        "mps_state_create": (I, [P, I, I, I, I, I, ctypes.POINTER(P), ctypes.POINTER(P),
                                 ctypes.POINTER(I), ctypes.POINTER(P)]),
        "mps_state_destroy": (I, [P]),
        "mps_state_chis": (I, [P, ctypes.POINTER(I)]),
        "mps_sweep": (I, [P, ctypes.POINTER(P), I, ctypes.POINTER(P), I, I,
                          ctypes.POINTER(mps_sweep_policy), P, P]),
        "mps_measure": (I, [P, P, P, P, P, P, P, P, P]),
        "mps_sweep_stats": (I, [P, ctypes.POINTER(ctypes.c_longlong)]),
        "mps_sweep_sequential": (I, [P, I, I, I, I, ctypes.POINTER(P), P, ctypes.POINTER(I), P, I, I, I, P]),
        "mps_zgemm": (I, [P, I, I, I, I, I, I, P, LL, P, LL, P, LL, D, D, P]),
        "mps_qr": (I, [P, I, I, I, P, P, P]),
        "mps_heig": (I, [P, I, I, P, P, P, P]),
        "mps_profile_enable": (I, [P, I, I]),
        "mps_profile_read": (I, [P, ctypes.POINTER(D), ctypes.POINTER(D), ctypes.POINTER(I)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


def load():
    """Load the library (once).  Raises if it is missing: there is no CPU path."""
    global _lib
    if _lib is None:
        # torch first: the library then binds to the HIP runtime torch already
        # loaded, so both share one runtime (and one device context)
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise QrtebdError(MPS_ERR_STATE, f"{LIB_PATH} not built (run paper_2212_09782_amd.build)")
        _lib = _declare(ctypes.CDLL(LIB_PATH))
    return _lib


def _check(rc):
    if rc != MPS_OK:
        raise QrtebdError(rc, load().mps_last_error().decode())
    return rc


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return P(s.cuda_stream)


def _ptr(t):
    return P(t.data_ptr()) if t is not None else P(0)


# ---------------------------------------------------------------- context

class Context:
    """Owns an mps_ctx (device workspace of the library)."""

    def __init__(self, device=0, autotune_cache=None):
        self.lib = load()
        h = P()
        path = os.fsencode(autotune_cache) if autotune_cache else None
        _check(self.lib.mps_ctx_create(device, path, ctypes.byref(h)))
        self.h = h

    def close(self):
        if self.h:
            self.lib.mps_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def sync(self, stream=None):
        _check(self.lib.mps_sync(self.h, _stream(stream)))

    def profile_enable(self, on=True, max_launches=100000):
        _check(self.lib.mps_profile_enable(self.h, int(on), max_launches))

    def profile_read(self):
        """(total_ms, total_flops, launches) of the contraction GEMMs since profile_enable."""
        ms, fl, n = D(), D(), I()
        _check(self.lib.mps_profile_read(self.h, ctypes.byref(ms), ctypes.byref(fl), ctypes.byref(n)))
        return ms.value, fl.value, n.value


def clock_gate(d, g, tau, wl=0.5, wr=0.5):
    """mps_clock_gate: host complex128 (d^2 x d^2) gate of the clock model."""
    out = np.zeros((d * d, d * d), np.complex128)
    _check(load().mps_clock_gate(d, g, tau, wl, wr, out.ctypes.data_as(P)))
    return out


def clock_hamiltonian(d, g, wl=0.5, wr=0.5):
    """mps_clock_hamiltonian: host complex128 (d^2 x d^2) bond Hamiltonian of the clock model."""
    out = np.zeros((d * d, d * d), np.complex128)
    _check(load().mps_clock_hamiltonian(d, g, wl, wr, out.ctypes.data_as(P)))
    return out


def clock_gate_charge(d, g, tau, wl=0.5, wr=0.5):
    """mps_clock_gate_charge: the clock gate in the charge basis (eigenbasis of X)."""
    out = np.zeros((d * d, d * d), np.complex128)
    _check(load().mps_clock_gate_charge(d, g, tau, wl, wr, out.ctypes.data_as(P)))
    return out


def clock_hamiltonian_charge(d, g, wl=0.5, wr=0.5):
    """mps_clock_hamiltonian_charge: the bond Hamiltonian in the charge basis."""
    out = np.zeros((d * d, d * d), np.complex128)
    _check(load().mps_clock_hamiltonian_charge(d, g, wl, wr, out.ctypes.data_as(P)))
    return out


def sym_desc(d, sec_l, sec_m, sec_r, dchi_min, dchi_frac, chi_max, svd_min=1e-14, prec=MPS_C128):
    arr = lambda v: (ctypes.c_int * MPS_SYM_MAX_D)(*(list(v) + [0] * (MPS_SYM_MAX_D - len(v))))
    return mps_sym_desc(d, arr(sec_l), arr(sec_m), arr(sec_r), dchi_min, dchi_frac, chi_max, svd_min, prec)


def sym_capacity(desc):
    return _check_cap(load().mps_sym_capacity(ctypes.byref(desc)))


def _check_cap(v):
    if v < 0:
        raise QrtebdError(v, load().mps_last_error().decode())
    return v


def mps_bond_update_sym(ctx, desc, xi_m, b_m, b_n, u, b_m_out, xi_n_out, b_n_out, sec_out, chi_new, trunc_err,
                        stream=None):
    """Direct C-ABI call; every argument a torch tensor on the GPU."""
    _check(ctx.lib.mps_bond_update_sym(ctx.h, ctypes.byref(desc), _ptr(xi_m), _ptr(b_m), _ptr(b_n), _ptr(u),
                                       _ptr(b_m_out), _ptr(xi_n_out), _ptr(b_n_out), _ptr(sec_out), _ptr(chi_new),
                                       _ptr(trunc_err), _stream(stream)))


def bond_update_sym(ctx, desc, xi_m, b_m, b_n, u, stream=None):
    """Allocate capacity-sized outputs, run mps_bond_update_sym, return device
    tensors (b_m_out, xi_n_out, b_n_out, sec_out, chi_new, trunc_err)."""
    import torch
    dev = b_m.device
    cap = sym_capacity(desc)
    d = desc.d
    chi_l, chi_r = sum(desc.sec_l[:d]), sum(desc.sec_r[:d])
    cdt = torch.complex128 if desc.prec == MPS_C128 else torch.complex64
    b_m_out = torch.empty(chi_l * d * cap, dtype=cdt, device=dev)
    b_n_out = torch.empty(cap * d * chi_r, dtype=cdt, device=dev)
    xi_out = torch.empty(cap, dtype=torch.float64, device=dev)
    sec = torch.zeros(d, dtype=torch.int32, device=dev)
    chi = torch.zeros(1, dtype=torch.int32, device=dev)
    eps = torch.zeros(1, dtype=torch.float64, device=dev)
    mps_bond_update_sym(ctx, desc, xi_m, b_m, b_n, u, b_m_out, xi_out, b_n_out, sec, chi, eps, stream)
    return b_m_out, xi_out, b_n_out, sec, chi, eps


def unpack_sym(desc, b_m_out, xi_out, b_n_out, sec, chi):
    """Host numpy views of a finished symmetric update (synchronises):
    (bm, xi, bn, sector sizes, chi~)."""
    d = desc.d
    chi_l, chi_r = sum(desc.sec_l[:d]), sum(desc.sec_r[:d])
    k = int(chi.item())
    bm = b_m_out[: chi_l * d * k].cpu().numpy().reshape(chi_l, d, k)
    bn = b_n_out[: k * d * chi_r].cpu().numpy().reshape(k, d, chi_r)
    return bm, xi_out[:k].cpu().numpy(), bn, [int(x) for x in sec.cpu().numpy()], k


def bond_desc(d, chi_l, chi_m, chi_r, eta, chi_max, svd_min=1e-14, xi_is_diag=True, mode=CBE, prec=MPS_C128,
              sweeps=1, left_iso=False):
    return mps_bond_desc(d, chi_l, chi_m, chi_r, eta, chi_max, svd_min, int(bool(xi_is_diag)), mode, prec, sweeps,
                         int(bool(left_iso)))


def bond_capacity(desc):
    return load().mps_bond_capacity(ctypes.byref(desc))


def mps_bond_update(ctx, desc, xi_m, b_m, b_n, u, b_m_out, xi_n_out, b_n_out, chi_new, trunc_err, stream=None):
    """Direct C-ABI call; every argument a torch tensor on the GPU."""
    _check(ctx.lib.mps_bond_update(ctx.h, ctypes.byref(desc), _ptr(xi_m), _ptr(b_m), _ptr(b_n), _ptr(u),
                                   _ptr(b_m_out), _ptr(xi_n_out), _ptr(b_n_out), _ptr(chi_new),
                                   _ptr(trunc_err), _stream(stream)))


def mps_bond_update_noalloc(ctx, desc, xi_m, b_m, b_n, u, b_m_out, xi_n_out, b_n_out, chi_new, trunc_err,
                            stream=None):
    """Direct C-ABI call of the allocation-free variant (fixed per-GPU scratch)."""
    _check(ctx.lib.mps_bond_update_noalloc(ctx.h, ctypes.byref(desc), _ptr(xi_m), _ptr(b_m), _ptr(b_n), _ptr(u),
                                           _ptr(b_m_out), _ptr(xi_n_out), _ptr(b_n_out), _ptr(chi_new),
                                           _ptr(trunc_err), _stream(stream)))


def mps_bond_update_reference(ctx, desc, scheme, xi_m, b_m, b_n, u, b_m_out, xi_n_out, b_n_out, chi_new, trunc_err,
                              stream=None):
    """Direct C-ABI call of the SVD / EIG comparison schemes (complex128)."""
    _check(ctx.lib.mps_bond_update_reference(ctx.h, ctypes.byref(desc), scheme, _ptr(xi_m), _ptr(b_m), _ptr(b_n),
                                             _ptr(u), _ptr(b_m_out), _ptr(xi_n_out), _ptr(b_n_out), _ptr(chi_new),
                                             _ptr(trunc_err), _stream(stream)))


def reference_update(ctx, desc, scheme, xi_m, b_m, b_n, u, stream=None):
    """Allocate outputs of capacity min(chi_max, d chi_l, d chi_r) and run a comparison scheme."""
    import torch
    dev = b_m.device
    cap = max(1, min(desc.chi_max, desc.d * desc.chi_l, desc.d * desc.chi_r))
    b_m_out = torch.empty(desc.chi_l * desc.d * cap, dtype=torch.complex128, device=dev)
    b_n_out = torch.empty(cap * desc.d * desc.chi_r, dtype=torch.complex128, device=dev)
    xi_out = torch.empty(cap, dtype=torch.float64, device=dev)
    chi = torch.zeros(1, dtype=torch.int32, device=dev)
    eps = torch.zeros(1, dtype=torch.float64, device=dev)
    mps_bond_update_reference(ctx, desc, scheme, xi_m, b_m, b_n, u, b_m_out, xi_out, b_n_out, chi, eps, stream)
    return b_m_out, xi_out, b_n_out, chi, eps


def bond_update(ctx, desc, xi_m, b_m, b_n, u, stream=None):
    """Allocate capacity-sized outputs, run mps_bond_update, return device tensors.

    Returns (b_m_out, xi_n_out, b_n_out, chi_new, trunc_err) where the first
    three are flat capacity buffers (use unpack_bond for shaped views).
    """
    import torch
    dev = b_m.device
    cap = bond_capacity(desc)
    cdt = torch.complex128 if desc.prec == MPS_C128 else torch.complex64
    b_m_out = torch.empty(desc.chi_l * desc.d * cap, dtype=cdt, device=dev)
    b_n_out = torch.empty(cap * desc.d * desc.chi_r, dtype=cdt, device=dev)
    if desc.mode == CBE:
        xi_out = torch.empty(cap, dtype=torch.float64, device=dev)
    else:
        xi_out = torch.empty(cap * cap, dtype=torch.complex128, device=dev)
    chi = torch.zeros(1, dtype=torch.int32, device=dev)
    eps = torch.zeros(1, dtype=torch.float64, device=dev)
    mps_bond_update(ctx, desc, xi_m, b_m, b_n, u, b_m_out, xi_out, b_n_out, chi, eps, stream)
    return b_m_out, xi_out, b_n_out, chi, eps


def unpack_bond(desc, b_m_out, xi_out, b_n_out, chi):
    """Host numpy views of a finished update with the live chi~ (synchronises)."""
    k = int(chi.item())
    bm = b_m_out[: desc.chi_l * desc.d * k].cpu().numpy().reshape(desc.chi_l, desc.d, k)
    bn = b_n_out[: k * desc.d * desc.chi_r].cpu().numpy().reshape(k, desc.d, desc.chi_r)
    if desc.mode == CBE:
        xi = xi_out[:k].cpu().numpy()
    else:
        xi = xi_out.cpu().numpy().reshape(k, k)
    return bm, xi, bn, k


# ---------------------------------------------------------------- building blocks

def mps_zgemm(ctx, dt, opA, opB, M, N, K, A, lda, B, ldb, C, ldc, alpha=1.0, beta=0.0, stream=None):
    _check(ctx.lib.mps_zgemm(ctx.h, dt, opA, opB, M, N, K, _ptr(A), lda, _ptr(B), ldb, _ptr(C), ldc,
                             alpha, beta, _stream(stream)))


def mps_qr(ctx, dt, m, n, A, Q, stream=None):
    _check(ctx.lib.mps_qr(ctx.h, dt, m, n, _ptr(A), _ptr(Q), _stream(stream)))


def mps_heig(ctx, n, k, G, lam, E, stream=None):
    _check(ctx.lib.mps_heig(ctx.h, n, k, _ptr(G), _ptr(lam), _ptr(E), _stream(stream)))


# ---------------------------------------------------------------- states / sweep / measure

class State:
    """Device-resident MPS (torch buffers) registered with the library."""

    def __init__(self, ctx, B, Xi, finite=True, chi_cap=None, prec=MPS_C128):
        """B: list of numpy [chi_l, d, chi_r]; Xi: list of 1-D numpy (bond left of each site)."""
        import torch
        self.ctx = ctx
        self.L = len(B)
        self.d = B[0].shape[1]
        self.finite = finite
        self.prec = prec
        chis = [b.shape[0] for b in B] + [B[-1].shape[2]]
        self.chi_cap = int(chi_cap or max(chis))
        cdt = torch.complex128 if prec == MPS_C128 else torch.complex64
        self.B = [torch.zeros(self.chi_cap * self.d * self.chi_cap, dtype=cdt, device="cuda") for _ in B]
        self.Xi = [torch.zeros(self.chi_cap, dtype=torch.float64, device="cuda") for _ in B]
        for m in range(self.L):
            flat = torch.from_numpy(np.ascontiguousarray(B[m]).reshape(-1)).to(cdt)
            self.B[m][: flat.numel()].copy_(flat)
            x = torch.from_numpy(np.asarray(Xi[m], dtype=np.float64).reshape(-1))
            self.Xi[m][: x.numel()].copy_(x)
        bp = (P * self.L)(*[P(t.data_ptr()) for t in self.B])
        xp = (P * self.L)(*[P(t.data_ptr()) for t in self.Xi])
        ch = (I * (self.L + 1))(*chis)
        h = P()
        _check(ctx.lib.mps_state_create(ctx.h, 0 if finite else 1, self.L, self.d, self.chi_cap, prec,
                                        bp, xp, ch, ctypes.byref(h)))
        self.h = h

    def chis(self):
        out = (I * (self.L + 1))()
        _check(self.ctx.lib.mps_state_chis(self.h, out))
        return list(out)

    def to_numpy(self):
        """(B list, Xi list) with live dimensions (synchronises)."""
        import torch
        torch.cuda.synchronize()
        ch = self.chis()
        B, Xi = [], []
        for m in range(self.L):
            n = ch[m] * self.d * ch[m + 1]
            B.append(self.B[m][:n].cpu().numpy().astype(np.complex128).reshape(ch[m], self.d, ch[m + 1]))
            Xi.append(self.Xi[m][: ch[m]].cpu().numpy())
        return B, Xi

    def close(self):
        if self.h:
            self.ctx.lib.mps_state_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SymCell:
    """Uniform two-site cell (sites A = 0, B = 1; bond 0 = (A,B), bond 1 =
    (B,A)) with the Z_d block structure, in the charge basis: dense
    charge-ordered device tensors with room for chi_cap, the sector sizes of
    every bond (secs[m]: the bond left of site m) kept on the host and read
    back after every update (one synchronisation per update)."""

    def __init__(self, ctx, B, Xi, secs, chi_cap, prec=MPS_C128):
        import torch
        self.ctx, self.prec, self.chi_cap = ctx, prec, int(chi_cap)
        self.d = B[0].shape[1]
        cdt = torch.complex128 if prec == MPS_C128 else torch.complex64
        self.B = [torch.zeros(self.chi_cap * self.d * self.chi_cap, dtype=cdt, device="cuda") for _ in range(2)]
        self.Xi = [torch.zeros(self.chi_cap, dtype=torch.float64, device="cuda") for _ in range(2)]
        for m in range(2):
            flat = torch.from_numpy(np.ascontiguousarray(B[m]).reshape(-1)).to(cdt)
            self.B[m][: flat.numel()].copy_(flat)
            x = torch.from_numpy(np.asarray(Xi[m], dtype=np.float64).reshape(-1))
            self.Xi[m][: x.numel()].copy_(x)
        self.secs = [list(secs[0]), list(secs[1])]
        self.sec_dev = torch.zeros(self.d, dtype=torch.int32, device="cuda")
        self.chi_dev = torch.zeros(1, dtype=torch.int32, device="cuda")
        self.eps_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
        self.eps_sum = 0.0

    def chis(self):
        return [sum(self.secs[0]), sum(self.secs[1])]

    def update(self, bond, u, dchi_min, dchi_frac, chi_max, svd_min=1e-14, stream=None):
        """mps_bond_update_sym on bond 0 (A,B) or 1 (B,A) with the device gate
        u (charge basis); the new tensors replace the old ones in place."""
        m, n = bond, 1 - bond
        desc = sym_desc(self.d, self.secs[m], self.secs[n], self.secs[m], dchi_min, dchi_frac, chi_max, svd_min,
                        self.prec)
        if sym_capacity(desc) > self.chi_cap:
            raise QrtebdError(MPS_ERR_CAPACITY, f"new bond may reach {sym_capacity(desc)} > chi_cap {self.chi_cap}")
        mps_bond_update_sym(self.ctx, desc, self.Xi[m], self.B[m], self.B[n], u, self.B[m], self.Xi[n], self.B[n],
                            self.sec_dev, self.chi_dev, self.eps_dev, stream)
        self.ctx.sync(stream)
        self.secs[n] = [int(x) for x in self.sec_dev.cpu().numpy()]
        self.eps_sum += float(self.eps_dev.item())

    def step(self, u_half, u_full, dchi_min, dchi_frac, chi_max, svd_min=1e-14, stream=None):
        """Second-order step: (A,B) for dt/2, (B,A) for dt, (A,B) for dt/2."""
        for bond, u in ((0, u_half), (1, u_full), (0, u_half)):
            self.update(bond, u, dchi_min, dchi_frac, chi_max, svd_min, stream)

    def measure(self, op1=None, op2=None, site_vals=None, norms=None, bond_vals=None, entropies=None, stream=None):
        """mps_measure on the cell (operators in the charge basis)."""
        ch = self.chis()
        bp = (P * 2)(*[P(t.data_ptr()) for t in self.B])
        xp = (P * 2)(*[P(t.data_ptr()) for t in self.Xi])
        h = P()
        _check(self.ctx.lib.mps_state_create(self.ctx.h, 1, 2, self.d, self.chi_cap, self.prec, bp, xp,
                                             (I * 3)(ch[0], ch[1], ch[0]), ctypes.byref(h)))
        try:
            _check(self.ctx.lib.mps_measure(self.ctx.h, h, _ptr(op1), _ptr(op2), _ptr(site_vals), _ptr(norms),
                                            _ptr(bond_vals), _ptr(entropies), _stream(stream)))
        finally:
            self.ctx.lib.mps_state_destroy(h)

    def to_numpy(self):
        """(B list, Xi list, secs) with live dimensions (synchronises)."""
        import torch
        torch.cuda.synchronize()
        ch = self.chis()
        B, Xi = [], []
        for m in range(2):
            k = ch[m] * self.d * ch[1 - m]
            B.append(self.B[m][:k].cpu().numpy().astype(np.complex128).reshape(ch[m], self.d, ch[1 - m]))
            Xi.append(self.Xi[m][: ch[m]].cpu().numpy())
        return B, Xi, [list(self.secs[0]), list(self.secs[1])]


def sweep_policy(chi_max, svd_min=1e-14, dchi_min=100, dchi_frac=0.1, mode=CBE, sweeps=1, exec=EXEC_EAGER,
                 chunk=0):
    return mps_sweep_policy(mode, chi_max, svd_min, dchi_min, dchi_frac, sweeps, exec, chunk)


SWEEP_STATS = ("layers_eager", "host_syncs", "chunks", "rollbacks", "graph_captures", "graph_replays",
               "tune_trials", "tune_hits")


def sweep_stats(ctx):
    """Counters of the context (dict with the SWEEP_STATS keys)."""
    out = (ctypes.c_longlong * 8)()
    _check(ctx.lib.mps_sweep_stats(ctx.h, out))
    return dict(zip(SWEEP_STATS, list(out)))


def mps_sweep(ctx, states, gates, nsteps, order, policy, trunc_err=None, stream=None):
    """gates: one device complex128 tensor [nbonds, 2, d^2, d^2] per state."""
    n = len(states)
    sp = (P * n)(*[s.h for s in states])
    gp = (P * n)(*[P(g.data_ptr()) for g in gates])
    _check(ctx.lib.mps_sweep(ctx.h, sp, n, gp, nsteps, order, ctypes.byref(policy), _ptr(trunc_err),
                             _stream(stream)))


def mps_measure(ctx, state, op1=None, op2=None, site_vals=None, norms=None, bond_vals=None, entropies=None,
                stream=None):
    _check(ctx.lib.mps_measure(ctx.h, state.h, _ptr(op1), _ptr(op2), _ptr(site_vals), _ptr(norms),
                               _ptr(bond_vals), _ptr(entropies), _stream(stream)))


def chain_gates(d, g, L, finite, dt):
    """Device tensor [nbonds, 2, d^2, d^2]: the clock gates for tau = dt/2 and dt (library builder)."""
    import torch
    nb = L - 1 if finite else L
    out = np.zeros((max(nb, 1), 2, d * d, d * d), np.complex128)
    for b in range(nb):
        if finite:
            wl = 1.0 if b == 0 else 0.5
            wr = 1.0 if b + 1 == L - 1 else 0.5
        else:
            wl = wr = 0.5
        out[b, 0] = clock_gate(d, g, dt / 2, wl, wr)
        out[b, 1] = clock_gate(d, g, dt, wl, wr)
    return torch.from_numpy(out).to("cuda")


class SequentialState:
    """Finite chain for mps_sweep_sequential: site buffers of capacity
    chi_cap*d*chi_cap and the bond matrix at the left end (torch buffers)."""

    def __init__(self, ctx, B, chi_cap, prec=MPS_C128):
        """B: list of numpy [chi_l, d, chi_r] in right-isometric form."""
        import torch
        self.ctx = ctx
        self.L = len(B)
        self.d = B[0].shape[1]
        self.prec = prec
        self.chi_cap = int(chi_cap)
        cdt = torch.complex128 if prec == MPS_C128 else torch.complex64
        self.sites = [torch.zeros(self.chi_cap * self.d * self.chi_cap, dtype=cdt, device="cuda") for _ in B]
        for m in range(self.L):
            flat = torch.from_numpy(np.ascontiguousarray(B[m]).reshape(-1)).to(cdt)
            self.sites[m][: flat.numel()].copy_(flat)
        self.center = torch.zeros(self.chi_cap * self.chi_cap, dtype=torch.complex128, device="cuda")
        self.center[0] = 1
        self.chi = [b.shape[0] for b in B] + [B[-1].shape[2]]

    def sweep(self, gates_half, nsteps, mode=PLAIN, chi_max=0, stream=None):
        """nsteps second-order sequential steps (gates_half: device [L-1, d^2, d^2] complex128)."""
        sp = (P * self.L)(*[P(t.data_ptr()) for t in self.sites])
        ch = (I * (self.L + 1))(*self.chi)
        _check(self.ctx.lib.mps_sweep_sequential(self.ctx.h, self.L, self.d, self.chi_cap, self.prec, sp,
                                                 _ptr(self.center), ch, _ptr(gates_half), nsteps, mode, chi_max,
                                                 _stream(stream)))
        self.chi = list(ch)

    def to_numpy(self):
        import torch
        torch.cuda.synchronize()
        out = []
        for m in range(self.L):
            n = self.chi[m] * self.d * self.chi[m + 1]
            out.append(self.sites[m][:n].cpu().numpy().astype(np.complex128).reshape(self.chi[m], self.d,
                                                                                     self.chi[m + 1]))
        return out
