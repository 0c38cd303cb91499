"""MI355X-native QR-based TEBD bond update (arXiv:2212.09782).

The compute path lives in the HIP library ``libqrtebd.so`` (sources in
``csrc/``, C-ABI in ``include/qrtebd.h`` at the repository root).  The Python
side is argument marshalling only:

- ``lib``     ctypes binding with the C-ABI names (``mps_bond_update``,
              ``mps_sweep``, ``mps_measure`` ...), torch tensors for device
              memory and streams.
- ``inputs``  seeded synthetic inputs (random isometric MPS, product states,
              request streams).  No step of the method is computed there.
- ``build``   compiles the library for gfx950.

Importing this package loads nothing; ``lib.load()`` loads the library and
raises if it is missing.
"""
