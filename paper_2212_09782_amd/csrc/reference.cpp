// Reference truncation schemes of the paper's comparison (Sec. IV, schemes
// (i) and (ii)) on the GPU: the same two-site contraction and Hastings form
// as the QR update, with the truncation taken from
//   SVD: theta~ = U S V^dag (rocSOLVER gesvd), B~[n] = V_kept^dag;
//   EIG: theta~^dag theta~ = V S^2 V^dag (rocSOLVER heevd), B~[n] = V_kept^dag.
// They are baselines for timing and accuracy comparisons, not part of the
// QR path, so they use the vendor solver library.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>

#include "bond.h"
#include "reference.h"

namespace qrtebd {
namespace {

inline size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

__global__ void square_kernel(const double* S, int n, double* lam) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) lam[i] = S[i] * S[i];
}

// lam[k] = D[n-1-k] and row k of Bn = column n-1-k of the column-major
// eigenvector matrix W (stored at W + j n), k < kmax.
__global__ void top_eig_kernel(const double* D, const c128* W, int n, int kmax, double* lam, c128* Bn) {
  const int k = blockIdx.y;
  if (k >= kmax) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) lam[k] = D[n - 1 - k];
  const c128* src = W + (long long)(n - 1 - k) * n;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) Bn[(long long)k * n + i] = src[i];
}

__global__ void info_kernel(const rocblas_int* info, int* status) {
  if (*info != 0) latch_error(status, ERRBIT_NONFINITE);
}

struct RefBufs {
  c128 *C, *Th, *U;
  double *S, *E, *lam, *partial, *norm2, *kept2;
  rocblas_int* info;
  size_t total;
};

RefBufs carve_ref(const BondShape& b, int scheme, void* base) {
  const size_t mL = (size_t)b.d * b.chi_l, mR = (size_t)b.d * b.chi_r, mn = std::min(mL, mR);
  char* p = (char*)base;
  RefBufs r{};
  auto take = [&](size_t bytes) {
    void* q = p;
    p += a256(bytes);
    return q;
  };
  r.C = (c128*)take(mL * mR * 16);
  r.Th = (c128*)take(mL * mR * 16);
  r.U = (c128*)take(scheme == MPS_SCHEME_SVD ? mR * mn * 16 : mR * mR * 16);   // left vectors / Gram and eigenvectors
  r.S = (double*)take((scheme == MPS_SCHEME_SVD ? mn : mR) * 8);
  r.E = (double*)take((scheme == MPS_SCHEME_SVD ? mn : mR) * 8);
  r.lam = (double*)take(mn * 8);
  r.partial = (double*)take(std::max<size_t>((size_t)b.chi_l * ((b.chi_r + 15) / 16), 4096) * 8);
  r.norm2 = (double*)take(8);
  r.kept2 = (double*)take(8);
  r.info = (rocblas_int*)take(sizeof(rocblas_int));
  r.total = (size_t)(p - (char*)base);
  return r;
}

}  // namespace

size_t reference_work_bytes(const BondShape& b, int scheme) { return carve_ref(b, scheme, nullptr).total + 256; }

int reference_update(const BondShape& b, int scheme, void* ws, int* status, void* handle, const void* xi_m,
                     const void* b_m, const void* b_n, const c128* u, void* b_m_out, void* xi_n_out, void* b_n_out,
                     int* chi_new, double* eps, hipStream_t s) {
  int rc;
  rocblas_handle h = (rocblas_handle)handle;
  if (rocblas_set_stream(h, s) != rocblas_status_success) return set_error(-4, "rocblas_set_stream failed");
  const int mL = b.d * b.chi_l, mR = b.d * b.chi_r, mn = std::min(mL, mR);
  const int kmax = std::max(1, std::min(b.chi_max, mn));
  RefBufs w = carve_ref(b, scheme, ws);
  if ((rc = two_site_c128(b, xi_m, b_m, b_n, u, w.C, w.Th, w.partial, w.norm2, s))) return rc;
  rocblas_status st;
  if (scheme == MPS_SCHEME_SVD) {
    // theta~ row-major is theta~^T column-major (mR x mL): its left singular
    // vectors U' satisfy U'[c, k] = conj(V[c, k]) = (V^dag)[k, c], so the first
    // chi~ columns of U' (ld mR) are B~[n] row-major
    st = rocsolver_zgesvd(h, rocblas_svect_singular, rocblas_svect_none, mR, mL, (rocblas_double_complex*)w.Th, mR,
                          w.S, (rocblas_double_complex*)w.U, mR, nullptr, 1, w.E, rocblas_outofplace, w.info);
    if (st != rocblas_status_success) return set_error(-4, "rocsolver_zgesvd failed (%d)", (int)st);
    hipLaunchKernelGGL(square_kernel, dim3((mn + 255) / 256), dim3(256), 0, s, w.S, mn, w.lam);
    QT_HIP_CHECK(hipGetLastError());
    QT_HIP_CHECK(hipMemcpyAsync(b_n_out, w.U, (size_t)kmax * mR * sizeof(c128), hipMemcpyDeviceToDevice, s));
  } else {
    // G = theta~^dag theta~ (mR x mR, row-major, Hermitian); its column-major
    // view is conj(G), whose eigenvectors W = conj(V) read row-major are V^dag
    GemmProb g = gemm_prob(w.Th, mR, OP_C, w.Th, mR, OP_N, w.U, mR, mR, mR, mL);
    g.herm = 1;
    if ((rc = gemm_one(g, GemmTypes{DT_C128, DT_C128}, s))) return rc;
    if ((rc = herm_fill_lower(w.U, mR, mR, s))) return rc;
    st = rocsolver_zheevd(h, rocblas_evect_original, rocblas_fill_upper, mR, (rocblas_double_complex*)w.U, mR, w.S, w.E,
                          w.info);
    if (st != rocblas_status_success) return set_error(-4, "rocsolver_zheevd failed (%d)", (int)st);
    hipLaunchKernelGGL(top_eig_kernel, dim3(std::min(64, (mR + 255) / 256), kmax), dim3(256), 0, s, w.S, w.U, mR,
                       kmax, w.lam, (c128*)b_n_out);
    QT_HIP_CHECK(hipGetLastError());
  }
  hipLaunchKernelGGL(info_kernel, dim3(1), dim3(1), 0, s, w.info, status);
  QT_HIP_CHECK(hipGetLastError());
  if ((rc = select_run(w.lam, kmax, b.svd_min, w.norm2, chi_new, (double*)xi_n_out, w.kept2, eps, status, s)))
    return rc;
  // Hastings' form: B~[m] = C~ B~[n]^dag with the live chi~
  GemmProb gp = gemm_prob(w.C, mR, OP_N, b_n_out, mR, OP_C, b_m_out, kmax, mL, kmax, mR);
  gp.dN = chi_new;
  gp.ldc_live_N = 1;
  return gemm_one(gp, GemmTypes{DT_C128, DT_C128}, s, true);
}

}  // namespace qrtebd
