// One two-site bond update on the device (internal interface).
#pragma once
#include "eig.h"

namespace qrtebd {

// HIP-event records around the contraction GEMMs of the bond update (the
// dominant kernel class), with the algorithmic flops (8 M N K) of each launch.
struct KernelTimer {
  int on = 0;
  int n = 0;                 // recorded launches
  int cap = 0;
  hipEvent_t* ev = nullptr;  // 2 * cap events
  double* flops = nullptr;   // cap
};

// gemm_one with event records when the timer is on.
int timed_gemm(KernelTimer* t, const GemmProb& p, GemmTypes ty, hipStream_t s);

struct BondShape {
  int d, chi_l, chi_m, chi_r, eta, chi_max;
  double svd_min;
  int xi_is_diag, mode, prec;
  int sweeps = 1;      // QR/LQ sweeps (>= 1)
  int left_iso = 0;    // PLAIN / GROW: b_m_out = Q^[m] (left-isometric) instead of Hastings' B~^[m]
  int pre = 0;         // C~ and theta~ already in the workspace (bond_pre_views): skip step (i) and the gate
  int cap() const;     // capacity of the new bond
};

// One truncation over the blocks of a bond with a Z_d block structure (Sec.
// III, closing paragraph): block k hands over its eigenvalues lam[k] (kw[k]
// of them, descending; kw = 0 for an absent block), and the largest ones over
// all blocks are kept (sqrt(max(lam, 0)) >= svd_min, at most chi_max, at
// least one), ranked by max(lam, 0) with ties to the lower block index.
// Outputs: chi[k] kept per block, offs[0..n] their prefix sums, *chi_tot,
// xi (chi_tot values: block after block, S / |S_kept|), *eps.
constexpr int kSymMaxD = 16;
struct SymSelect {
  int n;
  const double* lam[kSymMaxD];
  int kw[kSymMaxD];
  int* chi;                 // n entries
  int* offs;                // n + 1 entries
  int* chi_tot;
  double* xi;
  const double* norm2;      // |theta~|^2 over all blocks
  double* eps;
  int* status;
  double svd_min;
  int chi_max;
};

// Workspace bytes of one bond update of this shape.
size_t bond_work_bytes(const BondShape& b);

// One bond of a batched update: shape, its own workspace (bond_work_bytes)
// and device pointers.  For CBE the outputs may alias the inputs B^[m],
// B^[n] (they are read only before the outputs are written).
struct BondCall {
  BondShape b;
  void* ws;
  int* status;
  const void* xi_m;
  const void* b_m;
  const void* b_n;
  const c128* u;
  void* b_m_out;
  void* xi_n_out;
  void* b_n_out;
  int* chi_new;
  double* eps;
  const SymSelect* sym = nullptr;   // CBE blocks of one symmetric bond: joint truncation instead of select_kernel
};

// Where a bond of this shape keeps C~ and theta~ (for pre = 1) and, in CBE
// mode, the eigenvalues of step (iv) in its workspace.
void bond_pre_views(const BondShape& b, void* ws, void** C, void** Th, double** lam);
// All bonds of a batch must share the precision; modes and shapes may differ.
// as: optional look-ahead resources for the QR factorisations.
int bond_update_batch(const BondCall* calls, int n, hipStream_t s, KernelTimer* timer = nullptr,
                      const QrAsync* as = nullptr);
int timed_gemm_batch(KernelTimer* t, const GemmProb* p, int n, GemmTypes ty, hipStream_t s);

// Run one update with workspace `ws` (bond_work_bytes(b) bytes).  status:
// device error word.  All pointers are device pointers.
int bond_update_run(const BondShape& b, void* ws, int* status, const void* xi_m, const void* b_m,
                    const void* b_n, const c128* u, void* b_m_out, void* xi_n_out, void* b_n_out,
                    int* chi_new, double* eps, hipStream_t s, KernelTimer* timer = nullptr,
                    const QrAsync* as = nullptr);

// ---- pieces shared with the reference truncation schemes (complex128)
// Sec. II step (i): C~ = U (B^[m] B^[n]) into C, theta~ = Xi^[m] C~ into Th,
// |theta~|^2 into *norm2 (partial: at least 4096 doubles of scratch).
int two_site_c128(const BondShape& b, const void* xi_m, const void* b_m, const void* b_n, const c128* u, c128* C,
                  c128* Th, double* partial, double* norm2, hipStream_t s);
// Truncation from the descending spectrum lam = S^2 (kmax entries): chi~ (S >=
// svd_min, at least one), Xi~ = S_kept / |S_kept|, kept weight and eps.
int select_run(const double* lam, int kmax, double svd_min, const double* norm2, int* chi_new, double* xi,
               double* kept2, double* eps, int* status, hipStream_t s);

// ---- small kernels shared with the measurement path
// out[k] = sum over a partial buffer in a fixed order (one block).
int reduce_partials(const double* part, int n, double* out, hipStream_t s);

}  // namespace qrtebd
