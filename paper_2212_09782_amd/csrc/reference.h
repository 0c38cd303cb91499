// Reference truncation schemes (SVD, EIG) for comparison (internal interface).
#pragma once
#include "bond.h"

namespace qrtebd {

constexpr int MPS_SCHEME_SVD = 0;
constexpr int MPS_SCHEME_EIG = 1;

// Workspace bytes of one reference update (complex128).
size_t reference_work_bytes(const BondShape& b, int scheme);

// One bond update with the SVD (scheme 0) or EIG (scheme 1) truncation of
// theta~, complex128; handle: a rocblas_handle.  Outputs as the CBE update
// with capacity min(chi_max, d chi_l, d chi_r).
int reference_update(const BondShape& b, int scheme, void* ws, int* status, void* handle, const void* xi_m,
                     const void* b_m, const void* b_n, const c128* u, void* b_m_out, void* xi_n_out, void* b_n_out,
                     int* chi_new, double* eps, hipStream_t s);

}  // namespace qrtebd
