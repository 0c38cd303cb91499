// Grouped complex GEMM on MFMA (internal interface).
#pragma once
#include "common.h"

#include <algorithm>

namespace qrtebd {

enum Op : int { OP_N = 0, OP_T = 1, OP_C = 2 };
enum Dt : int { DT_C64 = 0, DT_C128 = 1 };

// C = alpha * op(A) * op(B) + beta * C, all matrices row-major, interleaved
// complex.  op(A) is M x K: OP_N reads A[m*lda + k], OP_T / OP_C read
// A[k*lda + m] (OP_C conjugated).  Likewise op(B) is K x N.
// M, N, K are capacities: they fix the launch grid.  When dM/dN/dK are set the
// live size is min(capacity, *dX), read on the device, so a graph or a later
// kernel can change it without the host.  ldc_live_N makes the output compact
// with the live N as its leading dimension.
// ksplit > 1 splits K: each split writes raw sums to work ([ksplit][Mcap][Ncap]
// in the compute type), and a reduction kernel forms alpha*sum + beta*C
// unless skip_reduce is set.
struct GemmProb {
  const void* A;
  const void* B;
  void* C;
  long long lda, ldb, ldc;
  int M, N, K;
  const int* dM;
  const int* dN;
  const int* dK;
  int ldc_live_N;
  int opA, opB;
  float alpha, beta;
  int ksplit;
  void* work;
  int skip_reduce;   // ksplit > 1: leave the partials in work (the caller reduces them)
  int herm;          // C = op(A) op(B) is Hermitian (M == N): only the 64 x 64 tiles on or above
                     // the diagonal are formed; the caller fills the lower triangle (herm_fill_lower)
};

constexpr int kGemmMaxProb = 16;

struct GemmBatch {
  int nprob;
  int tile_start[kGemmMaxProb + 1];
  int tiles_m[kGemmMaxProb];
  int tiles_n[kGemmMaxProb];
  GemmProb p[kGemmMaxProb];
};

// Input / output element types: DT_C128 in and out computes on FP64 MFMA,
// DT_C64 in and out on FP32 MFMA, DT_C64 in with DT_C128 out on FP64 MFMA.
struct GemmTypes {
  int tin;
  int tout;
};

// Launch one grouped GEMM (all problems share the types).  Problems with
// ksplit > 1 also launch the reduction.  Returns 0 or a negative status.
// contract = true launches the same kernel under the name
// contract_gemm_kernel (the bond update's contractions, profiled apart).
int gemm_run(const GemmProb* probs, int nprob, GemmTypes ty, hipStream_t stream, bool contract = false);
inline int gemm_one(const GemmProb& p, GemmTypes ty, hipStream_t stream, bool contract = false) {
  return gemm_run(&p, 1, ty, stream, contract);
}

// C[i][j] = conj(C[j][i]) for i > j (n x n complex128, row-major, ld ldc).
int herm_fill_lower(c128* C, long long ldc, int n, hipStream_t stream);

// Split of K for a product whose output has few 64x64 tiles: enough
// workgroups (about 1024) to fill the GPU, chunks of at least 128, and no
// more partials ([ks][M][N] of elem bytes) than work_bytes holds.
inline int splitk_auto(int M, int N, int K, size_t work_bytes, size_t elem, bool herm = false) {
  const long long tm = (M + 63) / 64, tn = (N + 63) / 64;
  const long long tiles = herm ? tm * (tm + 1) / 2 : tm * tn;   // herm: the tiles that do work
  long long ks = (1024 + tiles - 1) / tiles;
  ks = std::min<long long>(ks, std::max(1, K / 128));
  ks = std::min<long long>(ks, (long long)(work_bytes / ((size_t)M * N * elem)));
  ks = std::min<long long>(ks, 64);
  return (int)std::max<long long>(1, ks);
}

// Convenience constructor with static sizes.
inline GemmProb gemm_prob(const void* A, long long lda, int opA, const void* B, long long ldb,
                          int opB, void* C, long long ldc, int M, int N, int K,
                          float alpha = 1.f, float beta = 0.f) {
  GemmProb p{};
  p.A = A; p.B = B; p.C = C;
  p.lda = lda; p.ldb = ldb; p.ldc = ldc;
  p.M = M; p.N = N; p.K = K;
  p.opA = opA; p.opB = opB;
  p.alpha = alpha; p.beta = beta;
  p.ksplit = 1;
  return p;
}

}  // namespace qrtebd
