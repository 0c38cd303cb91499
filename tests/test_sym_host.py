"""Host-side checks of the Z_d block-structured update's C ABI (CPU only, no
GPU work): the charge-basis gate and Hamiltonian builders against the oracle's
basis change of its own clock-basis operators, the capacity of the new bond,
and descriptor errors."""
import ctypes

import numpy as np
import pytest

from oracle import clock, sym
from paper_2212_09782_amd import lib


@pytest.mark.parametrize("d,g,tau", [(2, 1.0, 0.05), (3, 2.0, 0.1), (5, 1.5, 0.02), (10, 1.5, 0.01)])
def test_charge_gate_matches_oracle(d, g, tau):
    U = lib.clock_gate_charge(d, g, tau, 0.5, 0.5)
    ref = sym.to_charge_basis_gate(clock.gate(clock.bond_hamiltonian(d, g, 0.5, 0.5), tau), d)
    assert np.max(np.abs(U - ref)) < 1e-13
    H = lib.clock_hamiltonian_charge(d, g, 0.5, 0.5)
    refH = sym.to_charge_basis_gate(clock.bond_hamiltonian(d, g, 0.5, 0.5), d)
    assert np.max(np.abs(H - refH)) < 1e-13


def test_sym_capacity_follows_the_expansion_rule():
    # chi_l = chi_r = 9; eta_c = min(sec_m + max(2, ceil(0.1 sec_m)), 9, 9)
    desc = lib.sym_desc(3, [3, 3, 3], [4, 0, 2], [2, 4, 3], 2, 0.1, 100)
    etas = sym.eta_sector([3, 3, 3], [4, 0, 2], [2, 4, 3], 3, 2, 0.1)
    assert etas == [6, 2, 4]
    assert lib.sym_capacity(desc) == sum(etas)
    desc = lib.sym_desc(3, [3, 3, 3], [4, 0, 2], [2, 4, 3], 2, 0.1, 5)
    assert lib.sym_capacity(desc) == 5
    # an empty sector that is not expanded stays empty
    desc = lib.sym_desc(3, [3, 3, 3], [4, 0, 2], [2, 4, 3], 0, 0.1, 100)
    assert lib.sym_capacity(desc) == sum(sym.eta_sector([3, 3, 3], [4, 0, 2], [2, 4, 3], 3, 0, 0.1)) == 5 + 3


@pytest.mark.parametrize("mut,code", [
    (lambda D: setattr(D, "d", 1), lib.MPS_ERR_ARG),
    (lambda D: setattr(D, "d", 17), lib.MPS_ERR_ARG),
    (lambda D: setattr(D, "prec", 3), lib.MPS_ERR_ARG),
    (lambda D: setattr(D, "chi_max", 0), lib.MPS_ERR_ARG),
    (lambda D: D.sec_m.__setitem__(1, -1), lib.MPS_ERR_ARG),
    (lambda D: [D.sec_l.__setitem__(i, 0) for i in range(3)], lib.MPS_ERR_ARG),
    (lambda D: D.sec_l.__setitem__(0, 50000), lib.MPS_ERR_CAPACITY),
    (lambda D: [D.sec_m.__setitem__(0, 1600), D.sec_l.__setitem__(0, 1700), D.sec_r.__setitem__(0, 1700)],
     lib.MPS_ERR_CAPACITY),
])
def test_sym_descriptor_errors(mut, code):
    desc = lib.sym_desc(3, [3, 3, 3], [4, 1, 2], [2, 4, 3], 2, 0.1, 100)
    mut(desc)
    assert lib.load().mps_sym_capacity(ctypes.byref(desc)) == code
    n = ctypes.c_size_t()
    assert lib.load().mps_sym_workspace_query(None, ctypes.byref(desc), ctypes.byref(n)) == code


def test_sym_null_pointers():
    desc = lib.sym_desc(3, [3, 3, 3], [4, 1, 2], [2, 4, 3], 2, 0.1, 100)
    L = lib.load()
    assert L.mps_bond_update_sym(None, ctypes.byref(desc), *([None] * 10), None) == lib.MPS_ERR_ARG
    n = ctypes.c_size_t()
    assert L.mps_sym_workspace_query(None, ctypes.byref(desc), ctypes.byref(n)) == lib.MPS_OK and n.value > 0
