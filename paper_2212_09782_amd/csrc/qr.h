// Blocked Householder QR of tall matrices (internal interface).
#pragma once
#include "gemm.h"

namespace qrtebd {

constexpr int kQrNb = 32;  // panel width
constexpr int kQrLdv = 2 * kQrNb;   // leading dimension of the stored reflectors

// Element offset of panel p's reflectors (its row 0, column 0) in QrWork::V
// of an m-row factorisation.  Panels 2g and 2g+1 share a 64-column block
// whose rows start at row 64g; panel 2g+1 sits 32 rows and 32 columns in,
// with zeros above it, so the pair is one m' x 64 operand.
__host__ __device__ inline size_t qr_v_offset(int p, int m) {
  return (size_t)(p / 2) * m * kQrLdv + (size_t)(p % 2) * (kQrNb * kQrLdv + kQrNb);
}

// Device workspace of one QR of an m x n matrix (n <= m).
struct QrWork {
  void* V;        // explicit reflectors, ld kQrLdv, panel p at qr_v_offset(p, m)
  c128* T;        // per panel 32 x 32 upper triangular (compact-WY factor)
  c128* Tp;       // per pair of panels 64 x 64: the merged compact-WY factor
  c128* gpart;    // per pair: partial sums of V_even^H V_odd over 64-row chunks
  void* W;        // 64 x n product V^H A (element type of the storage)
  void* Wsplit;   // split-K partials: kMaxSplit x 64 x n in the compute type
  c128* wx;       // panel blocks x 32 x 32: partial products of the previous panel's reflectors
  c128* red;      // panel reductions: 2 x nblk x 32 + 2 x 32
  unsigned* sync; // grid barrier words (>= grid_sync_words(kMaxPanelBlocks))
  int* status;
  int wcols;      // column capacity of W / Wsplit
};

constexpr int kMaxPanelBlocks = 256;
constexpr int kMaxQrRows = kMaxPanelBlocks * 160;   // blocks x rows per block
constexpr int kMaxSplit = 64;

// K split for a product with a small M x N output and a long K: enough
// workgroups to fill the GPU, chunks of at least 64.
int splitk_for(int M, int N, int K);

// Bytes of the QrWork of an m x n problem with element size es whose W can
// hold wcols columns (wcols >= n; qr_apply_q may then act on up to wcols).
size_t qr_work_bytes(int m, int n, int es, int wcols);
// Carve a QrWork out of one device allocation of qr_work_bytes bytes.
QrWork qr_work_carve(void* base, int m, int n, int es, int wcols, int* status);

// In-place factorisation A = Q R (A is m x n, row-major with leading dim lda,
// dt = DT_C128 or DT_C64).  On return the upper triangle of A holds R and the
// reflectors are in the work buffers.
int qr_factor(void* A, long long lda, int m, int n, int dt, const QrWork& w, hipStream_t s);

// Q (m x n, ld ldq) := the first n columns of H_0 H_1 ... (explicit thin Q).
int qr_form_q(void* Q, long long ldq, int m, int n, int dt, const QrWork& w, hipStream_t s);

// Z (rows r0..r0+m-1 of a matrix with nz columns, ld ldz) := H_0 H_1 ... Z,
// using the reflectors of a factorisation of an m x n matrix.
int qr_apply_q(void* Z, long long ldz, int nz, int m, int n, int dt, const QrWork& w, hipStream_t s);

// Batched forms: one job per matrix (all of type dt).  Panels of all jobs
// share cooperative launches and their trailing updates share grouped GEMMs.
//   factor: A (m x n, ld lda) in place;  form_q / apply_q: Z (m x nz, ld ldz).
struct QrJob {
  void* A;
  long long lda;
  int m, n;
  void* Z;
  long long ldz;
  int nz;
  const QrWork* w;
};
// Optional look-ahead: with an auxiliary stream (default priority) and two
// events, the update of the columns beyond the next panel runs on aux while
// the next panel is factored on s; the call returns with s joined to aux.
struct QrAsync {
  hipStream_t aux;
  hipEvent_t ev_panel, ev_trail;
};
int qr_factor_batch(const QrJob* jobs, int njobs, int dt, hipStream_t s, const QrAsync* as = nullptr);
int qr_form_q_batch(const QrJob* jobs, int njobs, int dt, hipStream_t s);
int qr_apply_q_batch(const QrJob* jobs, int njobs, int dt, hipStream_t s);

// Helpers shared by the bond update.
int fill_zero(void* p, size_t bytes, hipStream_t s);
// A region to clear: nrep repetitions (rep_stride bytes apart) of rows rows
// (row_stride bytes apart) of row_bytes bytes each; pointers and sizes are
// multiples of 4 bytes.
struct ZeroSpan {
  void* p;
  long long row_bytes, row_stride, rep_stride;
  int rows, nrep;
};
// Clears every span with one launch per 32 spans.
int zero_spans(const ZeroSpan* spans, int n, hipStream_t s);
int set_identity(void* Q, long long ldq, int m, int n, int dt, hipStream_t s);

}  // namespace qrtebd
