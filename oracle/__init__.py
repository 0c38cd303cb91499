"""CPU oracle for the QR-based TEBD bond update (Unfried, Hauschild, Pollmann,
"Fast Time-Evolution of Matrix-Product States using the QR decomposition",
arXiv:2212.09782).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or run
anything in this package: only the tests, the smoke check and the CPU-baseline
leg of the benchmark use it.  It shares no code with the HIP library and never
imports it.

Everything is plain numpy/scipy in complex128, written from the paper:

- ``clock``   the d-state clock model and its Trotter gates (Sec. IV).
- ``bond``    the QR truncation (Sec. II, steps (i)-(iii), Fig. 2), the
              heuristic bond growth (end of Sec. II), controlled bond
              expansion (Sec. III, steps (i)-(v), Fig. 3) and, as the
              reference truncation, SVD-TEBD (scheme (i) of Sec. IV).
- ``mps``     finite and uniform MPS in right-isometric form (Sec. II,
              Eq. (1), Fig. 1), the even/odd Trotter sweep (Fig. 2a) and the
              observables of Fig. 4 (local Z, entanglement entropy, truncation
              error).
- ``ed``      exact state-vector evolution used to pin the above.
- ``sym``     the Z_d block structure of the clock model in its charge basis
              and the CBE update block by block with one truncation over all
              blocks (Sec. III, closing paragraph; Sec. IV).

Parity status of each function is stated in its docstring; a function whose
result no test ties to something outside the oracle says "parity unpinned".
"""
