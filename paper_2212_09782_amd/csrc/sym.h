// The bond update with a Z_d block structure (internal interface).
#pragma once
#include "bond.h"
#include "qr.h"

namespace qrtebd {

// Sector sizes of the three bonds of an update (charge order) and the policy.
struct SymShape {
  int d;
  int sec_l[kSymMaxD], sec_m[kSymMaxD], sec_r[kSymMaxD];
  int dchi_min;
  double dchi_frac;
  int chi_max;
  double svd_min;
  int prec;
};

// Index bookkeeping shared by the kernels (passed by value).  Block c of the
// two-site matrix: rows (q, alpha) with alpha in sector c - q, q-major, row
// offset rowoff[c][q]; columns (q', beta) with beta in sector c + q', column
// offset coloff[c][q'].
struct SymDims {
  int d, chiL, chiM, chiR;
  int offL[kSymMaxD + 1], offM[kSymMaxD + 1], offR[kSymMaxD + 1];
  int secM[kSymMaxD];
  int rows[kSymMaxD], cols[kSymMaxD];
  int rowoff[kSymMaxD][kSymMaxD], coloff[kSymMaxD][kSymMaxD];
};

struct SymPlan {
  SymDims D;
  int eta[kSymMaxD];         // 0: absent block
  int cap;                   // capacity of the new bond
  BondShape blk[kSymMaxD];   // the dense problem of every present block
  int prec;
  double svd_min;
  int chi_max;
};

// Validates the shape and fills the plan; 0 or an MPS error code.
int sym_plan(const SymShape& s, SymPlan* p);
size_t sym_work_bytes(const SymPlan& p);

// One update: dense charge-ordered tensors in (xi_m chiL doubles, b_m chiL x d
// x chiM, b_n chiM x d x chiR) and out (b_m_out chiL x d x chi~, xi_out chi~,
// b_n_out chi~ x d x chiR, compact with the live chi~; sec_out d sector sizes,
// chi_new, eps), all device pointers.
int sym_update_run(const SymPlan& p, void* ws, int* status, const double* xi_m, const void* b_m, const void* b_n,
                   const c128* u, void* b_m_out, double* xi_out, void* b_n_out, int* sec_out, int* chi_new,
                   double* eps, hipStream_t s, const QrAsync* as);

}  // namespace qrtebd
