"""Host-side checks of the HIP library (CPU only, no GPU work).

The library must load and export every function its header declares; the
host-side clock-gate builder is compared with the oracle's gate.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import clock
from paper_2212_09782_amd import lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"^\s*(?:int|const char\*)\s+(mps_\w+)\s*\(", txt, re.M))
    return names


def test_library_exports_every_declared_symbol():
    L = lib.load()
    declared = _declared()
    assert declared, "no declarations found"
    assert declared == set(lib.EXPORTS)
    for name in declared:
        assert hasattr(L, name), name


def test_error_text_on_bad_arguments():
    L = lib.load()
    desc = lib.bond_desc(3, 4, 4, 4, eta=99, chi_max=4)
    assert L.mps_bond_update(None, ctypes.byref(desc), *([None] * 9), None) == lib.MPS_ERR_ARG
    assert lib.load().mps_last_error()


@pytest.mark.parametrize("d,g,tau,wl,wr", [(2, 2.0, 0.05, 0.5, 0.5), (3, 2.0, 0.025, 1.0, 0.5),
                                           (5, 2.0, 0.05, 0.5, 1.0), (10, 1.5, 0.02, 0.5, 0.5)])
def test_clock_gate_matches_oracle(d, g, tau, wl, wr):
    U = lib.clock_gate(d, g, tau, wl, wr)
    Uo = clock.gate(clock.bond_hamiltonian(d, g, wl, wr), tau)
    assert np.max(np.abs(U - Uo)) < 1e-13
    assert np.allclose(U @ U.conj().T, np.eye(d * d), atol=1e-13)


def test_bond_capacity():
    assert lib.bond_capacity(lib.bond_desc(5, 64, 64, 64, eta=71, chi_max=64)) == 64
    assert lib.bond_capacity(lib.bond_desc(5, 64, 64, 64, eta=71, chi_max=100)) == 71
    assert lib.bond_capacity(lib.bond_desc(5, 64, 64, 64, eta=64, chi_max=8, mode=lib.PLAIN)) == 64
