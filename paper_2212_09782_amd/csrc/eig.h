// FP64 Hermitian eigensolver for L^dag L (internal interface).
#pragma once
#include "qr.h"

namespace qrtebd {

// Largest matrix the eigensolver takes: the cooperative tridiagonalisation
// keeps every row in LDS (at most 150 KiB per block, one block per CU), so
// ceil(n / floor(150 KiB / (16 n))) blocks must fit the 256 CUs.
constexpr int kEigMaxN = 1536;
constexpr int kNsMaxSteps = 5;

struct EigWork {
  double* d;        // n   diagonal of the tridiagonal matrix
  double* e;        // n   off-diagonal (real, >= 0 up to sign)
  c128* tau;        // n   reflector factors
  double* lu;       // 4 * n * n inverse-iteration factors
  unsigned* sync;   // grid barrier words
  c128* red;        // cross-block partial sums: 2 * (256 + 1) + 2 * n  (p vector + row)
  QrWork qtri;      // reflectors of the tridiagonalisation, (n-1) x (n-1) problem with n work columns
  c128* gz;         // n x n Gram matrix of the eigenvector block (Newton-Schulz polish)
  c128* ztmp;       // n x n copy of the eigenvector block
  c128* tpart;      // split-K partials of V_p^H V_p for every panel p (8 x 32 x 32 each)
  int* ns_live;     // Newton-Schulz step state: [0] live size of Z^H Z (kwant or 0), [1] live rows of the
                    // update (n or 0), [2..3] max |Z^H Z - 1| bits, [4] stopped, [5] n
  int* status;
};

size_t eig_work_bytes(int n);
EigWork eig_work_carve(void* base, int n, int* status);

// Largest kwant eigenpairs of the Hermitian n x n matrix G (row-major, ld n,
// destroyed).  lam: kwant eigenvalues in descending order; E: n x kwant
// (row-major, ld kwant) with the matching orthonormal eigenvectors as columns.
int eig_herm_top(c128* G, int n, int kwant, double* lam, c128* E, const EigWork& w, hipStream_t s);

// The same for several matrices at once (tridiagonalisations share
// cooperative launches, the small kernels and GEMMs are batched).
struct EigJob {
  c128* G;
  int n, kwant;
  double* lam;
  c128* E;
  const EigWork* w;
  int ns_steps = 2;   // Newton-Schulz steps of the eigenvectors always taken (0..2); up to
                      // kNsMaxSteps in all until max |Z^H Z - 1| before a step is below 1e-7
                      // (vectors of close, unclustered eigenvalues overlap more)
};
int eig_herm_top_batch(const EigJob* jobs, int njobs, hipStream_t s);

}  // namespace qrtebd
