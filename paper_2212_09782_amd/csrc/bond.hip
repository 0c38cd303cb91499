// The two-site bond update of Sec. II (plain QR truncation, bond growth) and
// Sec. III (controlled bond expansion) on one GPU.
//
// Data flow for a bond (m, n) with theta~ viewed as the (chi_l d) x (d chi_r)
// matrix with rows (alpha, i) and columns (j, delta):
//   C   = B^[m] B^[n]                     GEMM   (step (i))
//   C~  = U C,  theta~ = Xi^[m] C~        gate kernel (diagonal Xi) or GEMM (dense Xi);
//                                         |theta~|^2 accumulated in FP64
//   X   = theta~ Y0^dag                   GEMM, Y0 = B^[n] (plain) or theta~[:eta] (grow / CBE)
//   X   = Q^[m] R                         Householder QR, explicit Q^[m]
//   Y^dag = theta~^dag Q^[m]              GEMM   (step (ii))
//   Y^dag = Q' R'  i.e. Y = L Q^[n] with L = R'^dag, Q^[n] = Q'^dag
//   plain / grow: Xi~ = L/|L|, B~^[n] = Q^[n]                        (step (iii))
//   CBE: L^dag L = R' R'^dag (FP64) = E diag(S^2) E^dag, keep chi~,   (Sec. III (iv), (v))
//        Xi~ = S_kept/|S_kept|, B~^[n] = E_kept^dag Q^[n]
//   B~^[m] = C~ B~^[n]^dag                GEMM (Hastings' form: no Xi inverse)
//   eps = (|theta~|^2 - sum_kept S^2) / |theta~|^2
// In the mixed path B~^[n] gets one FP64-checked re-orthogonalisation step,
// B <- B - (B B^dag - 1) B / 2, with B B^dag accumulated in FP64.
#include "bond.h"

#include <algorithm>
#include <vector>

namespace qrtebd {

int BondShape::cap() const {
  if (mode == 2) return std::max(1, std::min(eta, chi_max));
  return eta;
}

namespace {

inline size_t a256(size_t x) { return (x + 255) & ~size_t(255); }

// Gate and Xi over one row alpha of C and W columns delta: the d^2 inputs
// of every column staged in LDS; 256 threads in R = 256 / W groups, thread
// (column t % W, group t / W) forms the outputs o = group, group + R, ... of
// its column, G of them per pass (G independent FP64 chains per LDS read).
// kWave (W = 64): a group is one wave, so the gate entries a thread reads are
// the same across its wave and come through scalar loads.  Each complex
// product-accumulate is four FP64 FMAs.
template <typename S, bool kWave, int G>
__global__ __launch_bounds__(256) void gate_kernel(cpx<S>* C, cpx<S>* Th, const c128* __restrict__ U,
                                                   const double* xi, int d, int chiR, int Wa, double* partial) {
  extern __shared__ unsigned char gate_lds[];
  __shared__ double scr[4];
  cpx<S>* Cs = reinterpret_cast<cpx<S>*>(gate_lds);  // d^2 x W in storage precision
  const int W = kWave ? 64 : Wa;
  const int d2 = d * d, t = threadIdx.x, R = 256 / W, col = t % W;
  const int grp = kWave ? __builtin_amdgcn_readfirstlane(t >> 6) : t / W;
  const int alpha = blockIdx.y, delta = blockIdx.x * W + col;
  const long long base = (long long)alpha * d2 * chiR;
  const bool live = delta < chiR;
  for (int q = grp; q < d2; q += R) Cs[q * W + col] = live ? C[base + (long long)q * chiR + delta] : mk<S>(0, 0);
  __syncthreads();   // a column's inputs come from R threads
  const double x = xi ? xi[alpha] : 1.0;
  const int nout = (d2 - grp + R - 1) / R;   // outputs o = grp + R j, j < nout
  double nrm = 0;
  if (live) {
    for (int j0 = 0; j0 < nout; j0 += G) {
      c128 acc[G];
      int row[G];
#pragma unroll
      for (int u = 0; u < G; ++u) {
        acc[u] = mk<double>(0, 0);
        row[u] = (grp + R * min(j0 + u, nout - 1)) * d2;  // past the last output: recompute it, not stored
      }
      for (int q = 0; q < d2; ++q) {
        const c128 c = ccast<double>(Cs[q * W + col]);
#pragma unroll
        for (int u = 0; u < G; ++u) {
          const c128 g = U[row[u] + q];
          acc[u].re = fma(g.re, c.re, acc[u].re);
          acc[u].im = fma(g.re, c.im, acc[u].im);
          acc[u].re = fma(-g.im, c.im, acc[u].re);
          acc[u].im = fma(g.im, c.re, acc[u].im);
        }
      }
#pragma unroll
      for (int u = 0; u < G; ++u) {
        if (j0 + u >= nout) break;
        const long long off = base + (long long)(grp + R * (j0 + u)) * chiR + delta;
        C[off] = ccast<S>(acc[u]);
        if (Th) {
          const cpx<S> th = ccast<S>(cscale(acc[u], x));
          Th[off] = th;
          nrm += (double)th.re * th.re + (double)th.im * th.im;
        }
      }
    }
  }
  nrm = block_sum(nrm, scr);
  if (t == 0) partial[(long long)blockIdx.y * gridDim.x + blockIdx.x] = nrm;
}

// The gate at 7 <= d <= 10 (64 columns, one wave per output group): every
// output of a group stays in registers (NP passes of G complex FP64
// accumulators, NP G >= ceil(d^2 / 4)) while the inputs pass through LDS in
// chunks of QC rows, so the staged block is QC x 64 elements (about 48 KiB)
// and three workgroups share a CU.  Inside a chunk the passes run one after
// another, each over the chunk's rows with G gate rows (scalar loads
// streaming along q).  A group with fewer outputs recomputes its last one
// (not stored).  All inputs of the columns are read before the first output
// is written in place.
template <typename S, int NP, int G, int QC>
__global__ __launch_bounds__(256) void gate_regs_kernel(cpx<S>* C, cpx<S>* Th, const c128* __restrict__ U,
                                                        const double* xi, int d, int chiR, double* partial) {
  constexpr int NO = NP * G;
  extern __shared__ unsigned char gate_lds[];
  __shared__ double scr[4];
  cpx<S>* Cs = reinterpret_cast<cpx<S>*>(gate_lds);  // QC x 64 in storage precision
  const int d2 = d * d, t = threadIdx.x, col = t & 63;
  const int grp = __builtin_amdgcn_readfirstlane(t >> 6);
  const int alpha = blockIdx.y, delta = blockIdx.x * 64 + col;
  const long long base = (long long)alpha * d2 * chiR;
  const bool live = delta < chiR;
  const int nout = (d2 - grp + 3) / 4;   // outputs o = grp + 4 j, j < nout
  c128 acc[NO];
#pragma unroll
  for (int j = 0; j < NO; ++j) acc[j] = mk<double>(0, 0);
  for (int q0 = 0; q0 < d2; q0 += QC) {
    const int nq = min(QC, d2 - q0);
    __syncthreads();   // the previous chunk is consumed
    for (int q = grp; q < nq; q += 4) Cs[q * 64 + col] = live ? C[base + (long long)(q0 + q) * chiR + delta] : mk<S>(0, 0);
    __syncthreads();
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const c128* Ur[G];
#pragma unroll
      for (int u = 0; u < G; ++u) Ur[u] = U + (long long)(grp + 4 * min(p * G + u, nout - 1)) * d2 + q0;
      for (int q = 0; q < nq; ++q) {
        const c128 c = ccast<double>(Cs[q * 64 + col]);
#pragma unroll
        for (int u = 0; u < G; ++u) {
          const c128 g = Ur[u][q];
          c128& a = acc[p * G + u];
          a.re = fma(g.re, c.re, a.re);
          a.im = fma(g.re, c.im, a.im);
          a.re = fma(-g.im, c.im, a.re);
          a.im = fma(g.im, c.re, a.im);
        }
      }
    }
  }
  const double x = xi ? xi[alpha] : 1.0;
  double nrm = 0;
  if (live) {
#pragma unroll
    for (int j = 0; j < NO; ++j) {
      if (j < nout) {
        const long long off = base + (long long)(grp + 4 * j) * chiR + delta;
        C[off] = ccast<S>(acc[j]);
        if (Th) {
          const cpx<S> th = ccast<S>(cscale(acc[j], x));
          Th[off] = th;
          nrm += (double)th.re * th.re + (double)th.im * th.im;
        }
      }
    }
  }
  nrm = block_sum(nrm, scr);
  if (t == 0) partial[(long long)blockIdx.y * gridDim.x + blockIdx.x] = nrm;
}

// Dynamic LDS the gate kernel may take (160 KiB less its static block sums).
constexpr int kGateMaxLds = 160 * 1024 - 256;

// Columns per workgroup of the gate kernel for physical dimension d: 64 (one
// wave per output group) whenever the staged block fits the LDS of a CU;
// else 32 or 16, the widest whose block (d^2 W elements) leaves room for
// three workgroups per CU.
inline int gate_width(int d, size_t es) {
  if ((size_t)d * d * 64 * es <= (size_t)kGateMaxLds) return 64;
  int W = 32;
  while (W > 16 && (size_t)d * d * W * es > 48 * 1024) W /= 2;
  return W;
}

// Dynamic LDS limits are set once per instantiation.
template <typename S>
int launch_gate(cpx<S>* C, cpx<S>* Th, const c128* U, const double* xi, int d, int chiL, int chiR, int W,
                double* partial, size_t shm, hipStream_t s) {
  // rows per LDS chunk of the register-resident gate (about 50 KiB, three
  // workgroups per CU; d = 10 in two chunks of complex128, one of complex64)
  constexpr int QC = sizeof(S) == 8 ? 50 : 100;
  static bool attr = false;
  if (!attr) {
    QT_HIP_CHECK(hipFuncSetAttribute((const void*)gate_kernel<S, true, 7>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     kGateMaxLds));
    QT_HIP_CHECK(hipFuncSetAttribute((const void*)gate_kernel<S, true, 5>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     kGateMaxLds));
    QT_HIP_CHECK(hipFuncSetAttribute((const void*)gate_kernel<S, false, 5>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, kGateMaxLds));
    attr = true;
  }
  const dim3 grid((chiR + W - 1) / W, chiL);
  const size_t shq = (size_t)std::min(QC, d * d) * 64 * sizeof(cpx<S>);
  // the register-resident form where the whole staged block would hold a
  // CU to fewer than three workgroups (complex128 from d = 7, complex64
  // storage from d = 9; measured faster there, slower below)
  const bool regs = W == 64 && d <= 10 && d >= (sizeof(S) == 8 ? 7 : 9);
  if (W == 64 && d * d <= 28) {   // at most 7 outputs per group: one pass
    hipLaunchKernelGGL((gate_kernel<S, true, 7>), grid, dim3(256), shm, s, C, Th, U, xi, d, chiR, W, partial);
  } else if (regs) {   // ceil(d^2 / 4) outputs per group, all in registers
#define QT_GATE_REGS(NP, G)                                                                                  \
  hipLaunchKernelGGL((gate_regs_kernel<S, NP, G, QC>), grid, dim3(256), shq, s, C, Th, U, xi, d, chiR, partial)
    switch (d) {
      case 7: QT_GATE_REGS(3, 5); break;
      case 8: QT_GATE_REGS(4, 4); break;
      case 9: QT_GATE_REGS(3, 7); break;
      default: QT_GATE_REGS(5, 5); break;
    }
#undef QT_GATE_REGS
  } else if (W == 64) {
    hipLaunchKernelGGL((gate_kernel<S, true, 5>), grid, dim3(256), shm, s, C, Th, U, xi, d, chiR, W, partial);
  } else {
    hipLaunchKernelGGL((gate_kernel<S, false, 5>), grid, dim3(256), shm, s, C, Th, U, xi, d, chiR, W, partial);
  }
  QT_HIP_CHECK(hipGetLastError());
  return 0;
}

template <typename S>
__global__ __launch_bounds__(256) void sumsq_kernel(const cpx<S>* A, long long n, double* partial) {
  __shared__ double scr[4];
  double s = 0;
  for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    const cpx<S> z = A[i];
    s += (double)z.re * z.re + (double)z.im * z.im;
  }
  s = block_sum(s, scr);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(256) void reduce_kernel(const double* part, int n, double* out) {
  __shared__ double scr[4];
  double s = 0;
  for (int i = threadIdx.x; i < n; i += 256) s += part[i];
  s = block_sum(s, scr);
  if (threadIdx.x == 0) *out = s;
}

// R (upper triangle of the first eta rows of the factored Y^dag) with zeros below.
// (Element loops of these small kernels index with 32 bits: a 64-bit division
// per element would cost more than the element's memory traffic.)
template <typename S>
__global__ void extract_r_kernel(const cpx<S>* YH, int eta, cpx<S>* R) {
  const unsigned n = (unsigned)eta * eta, m = eta;
  for (unsigned idx = blockIdx.x * 256u + threadIdx.x; idx < n; idx += gridDim.x * 256u) {
    const unsigned i = idx / m, j = idx - i * m;
    R[idx] = j >= i ? YH[idx] : mk<S>(0, 0);
  }
}

// plain / grow: Xi~ = L / |L|_F with L = R^dag (complex128 output, eta x eta).
template <typename S>
__global__ void plain_xi_kernel(const cpx<S>* R, int eta, const double* kept2, c128* xi) {
  const double inv = 1.0 / sqrt(*kept2);
  const unsigned n = (unsigned)eta * eta, m = eta;
  for (unsigned idx = blockIdx.x * 256u + threadIdx.x; idx < n; idx += gridDim.x * 256u) {
    const int i = (int)(idx / m), j = (int)(idx - (unsigned)i * m);
    c128 v = mk<double>(0, 0);
    if (j <= i) {
      const cpx<S> r = R[(long long)j * eta + i];
      v = mk<double>((double)r.re * inv, -(double)r.im * inv);
    }
    xi[idx] = v;
  }
}

__global__ void plain_finish_kernel(int eta, const double* norm2, const double* kept2, int* chi_new,
                                    double* eps, int* status) {
  const double n2 = *norm2, k2 = *kept2;
  if (!(n2 > 0) || !isfinite(n2)) latch_error(status, n2 == 0 ? ERRBIT_ZERONORM : ERRBIT_NONFINITE);
  *chi_new = eta;
  *eps = n2 > 0 ? fmax(0.0, n2 - k2) / n2 : 0.0;
}

// CBE step (v): chi~ = number of leading S >= svd_min (at most kmax, at least
// one), Xi~ = S_kept / |S_kept|, eps.
__global__ __launch_bounds__(256) void select_kernel(const double* lam, int kmax, double svd_min,
                                                     const double* norm2, int* chi_new, double* xi,
                                                     double* kept2, double* eps, int* status) {
  __shared__ int first_bad;
  __shared__ double scr[4];
  __shared__ double k2s;
  if (threadIdx.x == 0) first_bad = kmax;
  __syncthreads();
  for (int j = threadIdx.x; j < kmax; j += 256) {
    const double l = lam[j];
    if (!isfinite(l)) latch_error(status, ERRBIT_NONFINITE);
    if (!(sqrt(fmax(l, 0.0)) >= svd_min)) atomicMin(&first_bad, j);
  }
  __syncthreads();
  const int k = max(1, first_bad);
  double s = 0;
  for (int j = threadIdx.x; j < k; j += 256) s += fmax(lam[j], 0.0);
  s = block_sum(s, scr);
  if (threadIdx.x == 0) k2s = s;
  __syncthreads();
  const double inv = k2s > 0 ? 1.0 / sqrt(k2s) : 0.0;
  for (int j = threadIdx.x; j < k; j += 256) xi[j] = sqrt(fmax(lam[j], 0.0)) * inv;
  if (threadIdx.x == 0) {
    const double n2 = *norm2;
    if (!(n2 > 0) || !isfinite(n2)) latch_error(status, n2 == 0 ? ERRBIT_ZERONORM : ERRBIT_NONFINITE);
    *chi_new = k;
    *kept2 = k2s;
    *eps = n2 > 0 ? fmax(0.0, n2 - k2s) / n2 : 0.0;
  }
}

// Entries of a non-increasing list (max(lam, 0)) ranked before value v: those
// above it, and those equal to it when ties go to the list.
__device__ inline int ranked_before(const double* lam, int n, double v, bool ties) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    const double x = fmax(lam[mid], 0.0);
    if (ties ? x >= v : x > v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// One truncation over the blocks of a symmetric bond (see SymSelect).
// Within a block the kept entries form a prefix: ranks grow along a list.
__global__ __launch_bounds__(256) void select_sym_kernel(SymSelect S) {
  __shared__ int first_bad[kSymMaxD];
  __shared__ int offs[kSymMaxD + 1];
  __shared__ double scr[4];
  __shared__ double k2s;
  const int tid = threadIdx.x;
  if (tid < kSymMaxD) first_bad[tid] = tid < S.n ? S.kw[tid] : 0;
  __syncthreads();
  for (int k = 0; k < S.n; ++k)
    for (int j = tid; j < S.kw[k]; j += 256) {
      const double l = S.lam[k][j];
      if (!isfinite(l)) latch_error(S.status, ERRBIT_NONFINITE);
      const double v = fmax(l, 0.0);
      long long rank = j;
      for (int k2 = 0; k2 < S.n; ++k2)
        if (k2 != k && S.kw[k2] > 0) rank += ranked_before(S.lam[k2], S.kw[k2], v, k2 < k);
      if (!(rank < S.chi_max && sqrt(v) >= S.svd_min)) atomicMin(&first_bad[k], j);
    }
  __syncthreads();
  if (tid == 0) {
    int tot = 0;
    for (int k = 0; k < S.n; ++k) tot += first_bad[k];
    if (tot == 0) {   // keep the largest value (lowest block on a tie)
      int best = -1;
      double bv = -1.0;
      for (int k = 0; k < S.n; ++k)
        if (S.kw[k] > 0 && fmax(S.lam[k][0], 0.0) > bv) {
          bv = fmax(S.lam[k][0], 0.0);
          best = k;
        }
      if (best >= 0) first_bad[best] = 1;
    }
    offs[0] = 0;
    for (int k = 0; k < S.n; ++k) offs[k + 1] = offs[k] + first_bad[k];
  }
  __syncthreads();
  const int tot = offs[S.n];
  double s = 0;
  for (int g = tid; g < tot; g += 256) {
    int k = 0;
    while (offs[k + 1] <= g) ++k;
    s += fmax(S.lam[k][g - offs[k]], 0.0);
  }
  s = block_sum(s, scr);
  if (tid == 0) k2s = s;
  __syncthreads();
  const double inv = k2s > 0 ? 1.0 / sqrt(k2s) : 0.0;
  for (int g = tid; g < tot; g += 256) {
    int k = 0;
    while (offs[k + 1] <= g) ++k;
    S.xi[g] = sqrt(fmax(S.lam[k][g - offs[k]], 0.0)) * inv;
  }
  if (tid < S.n) S.chi[tid] = first_bad[tid];
  if (tid <= S.n) S.offs[tid] = offs[tid];
  if (tid == 0) {
    const double n2 = *S.norm2;
    if (!(n2 > 0) || !isfinite(n2)) latch_error(S.status, n2 == 0 ? ERRBIT_ZERONORM : ERRBIT_NONFINITE);
    *S.chi_tot = tot;
    *S.eps = n2 > 0 ? fmax(0.0, n2 - k2s) / n2 : 0.0;
  }
}

// out (cols x rows) = conj(in (rows x cols))^T
template <typename S>
__global__ __launch_bounds__(256) void transpose_conj_kernel(const cpx<S>* in, int rows, int cols, cpx<S>* out) {
  __shared__ cpx<S> tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    const int i = by + r, j = bx + tx;
    if (i < rows && j < cols) tile[r][tx] = in[(long long)i * cols + j];
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int j = bx + r, i = by + tx;
    if (i < rows && j < cols) {
      const cpx<S> z = tile[tx][r];
      out[(long long)j * rows + i] = mk<S>(z.re, -z.im);
    }
  }
}

template <typename D, typename S>
__global__ void cast_kernel(const cpx<S>* in, long long n, cpx<D>* out) {
  for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (long long)gridDim.x * 256) out[i] = ccast<D>(in[i]);
}

// Dc = (G - 1)/2 on the live chi~ x chi~ block (G complex128, Dc complex64, ld cap).
__global__ void reorth_prep_kernel(const c128* G, int cap, const int* chi_new, c64* Dc) {
  const int k = *chi_new;
  const unsigned n = (unsigned)k * k, uk = k;
  for (unsigned idx = blockIdx.x * 256u + threadIdx.x; idx < n; idx += gridDim.x * 256u) {
    const int i = (int)(idx / uk), j = (int)(idx - (unsigned)i * uk);
    // G is Hermitian and only its upper triangle was formed
    const c128 g = i <= j ? G[(long long)i * cap + j] : cconj(G[(long long)j * cap + i]);
    Dc[(long long)i * cap + j] = mk<float>((float)(0.5 * (g.re - (i == j ? 1.0 : 0.0))), (float)(0.5 * g.im));
  }
}

int grid_for(long long n) { return (int)std::max<long long>(1, std::min<long long>((n + 255) / 256, 4096)); }

struct Carve {
  char* p;
  void* take(size_t b) {
    void* r = p;
    p += a256(b);
    return r;
  }
};

struct BondBufs {
  void *C, *Th, *X, *YH, *R, *Ec, *XiC, *Dc, *tmp;
  c128 *G, *E, *G2;
  double *lam, *partial, *norm2, *kept2;
  void* qrw;
  void* eigw;
  size_t total;
};

int kwant_of(const BondShape& b) { return b.cap(); }

BondBufs carve(const BondShape& b, void* base) {
  const size_t es = b.prec == 0 ? 16 : 8;
  const size_t mL = (size_t)b.d * b.chi_l, mR = (size_t)b.d * b.chi_r, eta = b.eta;
  const size_t kw = kwant_of(b), cap = b.cap();
  const bool cbe = b.mode == 2, mixed = b.prec != 0;
  Carve c{(char*)base};
  BondBufs o{};
  o.C = c.take(mL * mR * es);
  o.Th = c.take(mL * mR * es);
  o.X = c.take(mL * eta * es);
  o.YH = c.take(mR * eta * es);
  o.R = c.take(eta * eta * es);
  o.G = (c128*)c.take(cbe ? eta * eta * 16 : 0);
  o.E = (c128*)c.take(cbe ? eta * kw * 16 : 0);
  o.Ec = c.take(cbe && mixed ? eta * kw * es : 0);
  o.lam = (double*)c.take(cbe ? kw * 8 : 0);
  o.XiC = c.take(!b.xi_is_diag && mixed ? (size_t)b.chi_l * b.chi_l * es : 0);
  o.G2 = (c128*)c.take(mixed ? cap * cap * 16 : 0);
  o.Dc = c.take(mixed ? cap * cap * 8 : 0);
  o.tmp = c.take(mixed ? cap * mR * es : 0);
  const size_t npart = std::max<size_t>((size_t)b.chi_l * ((b.chi_r + 15) / 16), 4096);   // gate blocks of >= 16 columns
  o.partial = (double*)c.take(npart * 8);
  o.norm2 = (double*)c.take(8);
  o.kept2 = (double*)c.take(8);
  o.qrw = c.take(qr_work_bytes((int)std::max(mL, mR), (int)eta, (int)es, (int)eta));
  o.eigw = c.take(cbe ? eig_work_bytes((int)eta) : 0);
  o.total = (size_t)(c.p - (char*)base);
  return o;
}

template <typename S>
int run_batch(const BondCall* calls, int nc, hipStream_t s, KernelTimer* tm, const QrAsync* as) {
  const int dt = sizeof(S) == 8 ? DT_C128 : DT_C64;
  const GemmTypes ty{dt, dt};
  const bool mixed = dt == DT_C64;
  int rc;
  std::vector<BondBufs> W(nc);
  std::vector<QrWork> QW(nc);
  std::vector<GemmProb> g;
  for (int i = 0; i < nc; ++i) {
    const BondShape& b = calls[i].b;
    W[i] = carve(b, calls[i].ws);
    QW[i] = qr_work_carve(W[i].qrw, std::max(b.d * b.chi_l, b.d * b.chi_r), b.eta, (int)sizeof(cpx<S>), b.eta,
                          calls[i].status);
  }
  // (i) C = B^[m] B^[n] (bonds whose C~ and theta~ were formed by the caller skip this and the gate)
  g.clear();
  for (int i = 0; i < nc; ++i) {
    const BondShape& b = calls[i].b;
    if (b.pre) continue;
    const int mL = b.d * b.chi_l, mR = b.d * b.chi_r;
    g.push_back(gemm_prob(calls[i].b_m, b.chi_m, OP_N, calls[i].b_n, mR, OP_N, W[i].C, mR, mL, mR, b.chi_m));
  }
  if (!g.empty() && (rc = timed_gemm_batch(tm, g.data(), (int)g.size(), ty, s))) return rc;
  // C~ = U C (in place) and theta~ = Xi C~, |theta~|^2
  for (int i = 0; i < nc; ++i) {
    const BondCall& c = calls[i];
    const BondShape& b = c.b;
    if (b.pre) continue;
    BondBufs& w = W[i];
    const int d = b.d, chiL = b.chi_l, chiR = b.chi_r, mL = d * chiL, mR = d * chiR;
    const int Wc = gate_width(d, sizeof(cpx<S>));
    const dim3 grid((chiR + Wc - 1) / Wc, chiL);
    const size_t shm = (size_t)d * d * Wc * sizeof(cpx<S>);
    const bool diag = b.xi_is_diag != 0;
    if ((rc = launch_gate<S>((cpx<S>*)w.C, diag ? (cpx<S>*)w.Th : nullptr, c.u,
                             diag ? (const double*)c.xi_m : nullptr, d, chiL, chiR, Wc, w.partial, shm, s)))
      return rc;
    if (diag) {
      if ((rc = reduce_partials(w.partial, (int)(grid.x * grid.y), w.norm2, s))) return rc;
    } else {
      const void* xiA = c.xi_m;
      if (mixed) {
        const long long nx = (long long)chiL * chiL;
        hipLaunchKernelGGL((cast_kernel<float, double>), dim3(grid_for(nx)), dim3(256), 0, s, (const c128*)c.xi_m, nx,
                           (c64*)w.XiC);
        QT_HIP_CHECK(hipGetLastError());
        xiA = w.XiC;
      }
      const int ncol = d * mR;   // C~ viewed as chi_l x (d d chi_r)
      if ((rc = gemm_one(gemm_prob(xiA, chiL, OP_N, w.C, ncol, OP_N, w.Th, ncol, chiL, ncol, chiL), ty, s))) return rc;
      const long long n = (long long)mL * mR;
      hipLaunchKernelGGL(sumsq_kernel<S>, dim3(1024), dim3(256), 0, s, (const cpx<S>*)w.Th, n, w.partial);
      QT_HIP_CHECK(hipGetLastError());
      if ((rc = reduce_partials(w.partial, 1024, w.norm2, s))) return rc;
    }
  }
  // X = theta~ Y0^dag
  g.clear();
  for (int i = 0; i < nc; ++i) {
    const BondShape& b = calls[i].b;
    const int mL = b.d * b.chi_l, mR = b.d * b.chi_r, eta = b.eta;
    g.push_back(b.mode == 0 ? gemm_prob(W[i].Th, mR, OP_N, calls[i].b_n, mR, OP_C, W[i].X, eta, mL, eta, mR)
                            : gemm_prob(W[i].Th, mR, OP_N, W[i].Th, mR, OP_C, W[i].X, eta, mL, eta, mR));
  }
  if ((rc = timed_gemm_batch(tm, g.data(), nc, ty, s))) return rc;
  // Q^[m]
  std::vector<QrJob> qj(nc);
  for (int i = 0; i < nc; ++i) {
    const BondShape& b = calls[i].b;
    qj[i] = QrJob{W[i].X, b.eta, b.d * b.chi_l, b.eta, W[i].X, b.eta, b.eta, &QW[i]};
  }
  if ((rc = qr_factor_batch(qj.data(), nc, dt, s, as))) return rc;
  if ((rc = qr_form_q_batch(qj.data(), nc, dt, s))) return rc;
  // Y^dag = theta~^dag Q^[m], then Y^dag = Q' R'
  g.clear();
  for (int i = 0; i < nc; ++i) {
    const BondShape& b = calls[i].b;
    const int mL = b.d * b.chi_l, mR = b.d * b.chi_r, eta = b.eta;
    g.push_back(gemm_prob(W[i].Th, mR, OP_C, W[i].X, eta, OP_N, W[i].YH, eta, mR, eta, mL));
  }
  if ((rc = timed_gemm_batch(tm, g.data(), nc, ty, s))) return rc;
  for (int i = 0; i < nc; ++i) {
    const BondShape& b = calls[i].b;
    qj[i] = QrJob{W[i].YH, b.eta, b.d * b.chi_r, b.eta, W[i].YH, b.eta, b.eta, &QW[i]};
  }
  if ((rc = qr_factor_batch(qj.data(), nc, dt, s, as))) return rc;
  for (int i = 0; i < nc; ++i) {
    const int eta = calls[i].b.eta;
    const long long n = (long long)eta * eta;
    hipLaunchKernelGGL(extract_r_kernel<S>, dim3(grid_for(n)), dim3(256), 0, s, (const cpx<S>*)W[i].YH, eta,
                       (cpx<S>*)W[i].R);
    QT_HIP_CHECK(hipGetLastError());
  }
  // further sweeps (bonds with sweeps > it): X = theta~ Q^[n]^dag = theta~ Q',
  // then steps (i)-(ii) again
  int maxsw = 1;
  bool all_cbe = true;
  for (int i = 0; i < nc; ++i) {
    maxsw = std::max(maxsw, calls[i].b.sweeps);
    all_cbe = all_cbe && calls[i].b.mode == 2;
  }
  // With one sweep and CBE, Q' is next read by the B~^[n] product after the
  // eigen-decomposition (which reads only R'): it is formed on the auxiliary
  // stream, beside the latency-bound eigensolver, and joined before that
  // product.  Its launches are issued after the eigensolver's, so that the
  // host's launch time does not delay the eigensolver.
  const bool q_aside = as && as->aux && maxsw == 1 && all_cbe;
  if (q_aside) {
    QT_HIP_CHECK(hipEventRecord(as->ev_panel, s));
  } else if ((rc = qr_form_q_batch(qj.data(), nc, dt, s))) {
    return rc;
  }
  for (int it = 1; it < maxsw; ++it) {
    std::vector<int> act;
    for (int i = 0; i < nc; ++i)
      if (calls[i].b.sweeps > it) act.push_back(i);
    const int na = (int)act.size();
    std::vector<QrJob> qa(na);
    g.clear();
    for (int i : act) {
      const BondShape& b = calls[i].b;
      const int mL = b.d * b.chi_l, mR = b.d * b.chi_r, eta = b.eta;
      g.push_back(gemm_prob(W[i].Th, mR, OP_N, W[i].YH, eta, OP_N, W[i].X, eta, mL, eta, mR));
    }
    if ((rc = timed_gemm_batch(tm, g.data(), na, ty, s))) return rc;
    for (int a = 0; a < na; ++a) {
      const int i = act[a];
      const BondShape& b = calls[i].b;
      qa[a] = QrJob{W[i].X, b.eta, b.d * b.chi_l, b.eta, W[i].X, b.eta, b.eta, &QW[i]};
    }
    if ((rc = qr_factor_batch(qa.data(), na, dt, s, as))) return rc;
    if ((rc = qr_form_q_batch(qa.data(), na, dt, s))) return rc;
    g.clear();
    for (int i : act) {
      const BondShape& b = calls[i].b;
      const int mL = b.d * b.chi_l, mR = b.d * b.chi_r, eta = b.eta;
      g.push_back(gemm_prob(W[i].Th, mR, OP_C, W[i].X, eta, OP_N, W[i].YH, eta, mR, eta, mL));
    }
    if ((rc = timed_gemm_batch(tm, g.data(), na, ty, s))) return rc;
    for (int a = 0; a < na; ++a) {
      const int i = act[a];
      const BondShape& b = calls[i].b;
      qa[a] = QrJob{W[i].YH, b.eta, b.d * b.chi_r, b.eta, W[i].YH, b.eta, b.eta, &QW[i]};
    }
    if ((rc = qr_factor_batch(qa.data(), na, dt, s, as))) return rc;
    for (int i : act) {
      const int eta = calls[i].b.eta;
      const long long n = (long long)eta * eta;
      hipLaunchKernelGGL(extract_r_kernel<S>, dim3(grid_for(n)), dim3(256), 0, s, (const cpx<S>*)W[i].YH, eta,
                         (cpx<S>*)W[i].R);
      QT_HIP_CHECK(hipGetLastError());
    }
    if ((rc = qr_form_q_batch(qa.data(), na, dt, s))) return rc;
  }

  // CBE: L^dag L = R' R'^dag in FP64, eigen-decomposition, selection
  std::vector<int> cb;
  for (int i = 0; i < nc; ++i)
    if (calls[i].b.mode == 2) cb.push_back(i);
  if (!cb.empty()) {
    g.clear();
    std::vector<EigJob> ej;
    std::vector<EigWork> ew(nc);
    for (int i : cb) {
      const BondShape& b = calls[i].b;
      const int eta = b.eta;
      // theta~ is no longer needed: its buffer holds the split-K partials
      const size_t th_bytes = (size_t)b.d * b.chi_l * b.d * b.chi_r * sizeof(cpx<S>);
      GemmProb gg = gemm_prob(W[i].R, eta, OP_N, W[i].R, eta, OP_C, W[i].G, eta, eta, eta, eta);
      gg.ksplit = splitk_auto(eta, eta, eta, th_bytes, sizeof(c128), true);
      gg.work = W[i].Th;
      gg.herm = 1;
      g.push_back(gg);
      ew[i] = eig_work_carve(W[i].eigw, eta, calls[i].status);
    }
    if ((rc = gemm_run(g.data(), (int)g.size(), GemmTypes{dt, DT_C128}, s))) return rc;
    for (int i : cb)
      if ((rc = herm_fill_lower(W[i].G, calls[i].b.eta, calls[i].b.eta, s))) return rc;
    // the mixed path re-orthogonalises B~[n] in FP64 after the complex64
    // rounding of E, so one Newton-Schulz step on E suffices there
    for (int i : cb)
      ej.push_back(EigJob{W[i].G, calls[i].b.eta, kwant_of(calls[i].b), W[i].lam, W[i].E, &ew[i],
                          calls[i].b.prec == 0 ? 2 : 1});
    if ((rc = eig_herm_top_batch(ej.data(), (int)ej.size(), s))) return rc;
    if (q_aside) {
      QT_HIP_CHECK(hipStreamWaitEvent(as->aux, as->ev_panel, 0));
      if ((rc = qr_form_q_batch(qj.data(), nc, dt, as->aux))) return rc;
      QT_HIP_CHECK(hipEventRecord(as->ev_trail, as->aux));
    }
    g.clear();
    std::vector<const SymSelect*> joint;
    for (int i : cb) {
      const BondCall& c = calls[i];
      const int kw = kwant_of(c.b), eta = c.b.eta, mR = c.b.d * c.b.chi_r;
      if (c.sym) {
        if (std::find(joint.begin(), joint.end(), c.sym) == joint.end()) {
          joint.push_back(c.sym);
          hipLaunchKernelGGL(select_sym_kernel, dim3(1), dim3(256), 0, s, *c.sym);
          QT_HIP_CHECK(hipGetLastError());
        }
      } else {
        hipLaunchKernelGGL(select_kernel, dim3(1), dim3(256), 0, s, W[i].lam, kw, c.b.svd_min, W[i].norm2,
                           c.chi_new, (double*)c.xi_n_out, W[i].kept2, c.eps, c.status);
        QT_HIP_CHECK(hipGetLastError());
      }
      const void* Eu = W[i].E;
      if (mixed) {
        const long long n = (long long)eta * kw;
        hipLaunchKernelGGL((cast_kernel<float, double>), dim3(grid_for(n)), dim3(256), 0, s, W[i].E, n, (c64*)W[i].Ec);
        QT_HIP_CHECK(hipGetLastError());
        Eu = W[i].Ec;
      }
      // B~^[n] = E_kept^dag Q'^dag  (chi~ x d chi_r)
      GemmProb gp = gemm_prob(Eu, kw, OP_C, W[i].YH, eta, OP_C, c.b_n_out, mR, kw, mR, eta);
      gp.dM = c.chi_new;
      g.push_back(gp);
    }
    if (q_aside) QT_HIP_CHECK(hipStreamWaitEvent(s, as->ev_trail, 0));
    if ((rc = timed_gemm_batch(tm, g.data(), (int)g.size(), ty, s))) return rc;
  }
  // plain / grow: Xi~ = L/|L|, B~^[n] = Q'^dag
  for (int i = 0; i < nc; ++i) {
    const BondCall& c = calls[i];
    if (c.b.mode == 2) continue;
    const int eta = c.b.eta, mR = c.b.d * c.b.chi_r;
    const long long n = (long long)eta * eta;
    hipLaunchKernelGGL(sumsq_kernel<S>, dim3(1024), dim3(256), 0, s, (const cpx<S>*)W[i].R, n, W[i].partial);
    QT_HIP_CHECK(hipGetLastError());
    if ((rc = reduce_partials(W[i].partial, 1024, W[i].kept2, s))) return rc;
    hipLaunchKernelGGL(plain_xi_kernel<S>, dim3(grid_for(n)), dim3(256), 0, s, (const cpx<S>*)W[i].R, eta, W[i].kept2,
                       (c128*)c.xi_n_out);
    QT_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(plain_finish_kernel, dim3(1), dim3(1), 0, s, eta, W[i].norm2, W[i].kept2, c.chi_new, c.eps,
                       c.status);
    QT_HIP_CHECK(hipGetLastError());
    const dim3 grid((eta + 31) / 32, (mR + 31) / 32);
    hipLaunchKernelGGL(transpose_conj_kernel<S>, grid, dim3(256), 0, s, (const cpx<S>*)W[i].YH, mR, eta,
                       (cpx<S>*)c.b_n_out);
    QT_HIP_CHECK(hipGetLastError());
  }
  if (mixed) {
    // one re-orthogonalisation step of B~^[n] with B B^dag accumulated in FP64
    g.clear();
    for (int i = 0; i < nc; ++i) {
      const BondCall& c = calls[i];
      const int cap = c.b.cap(), mR = c.b.d * c.b.chi_r;
      GemmProb g2 = gemm_prob(c.b_n_out, mR, OP_N, c.b_n_out, mR, OP_C, W[i].G2, cap, cap, cap, mR);
      g2.dM = c.chi_new;
      g2.dN = c.chi_new;
      g2.ksplit = splitk_auto(cap, cap, mR, (size_t)c.b.d * c.b.chi_l * mR * sizeof(cpx<S>), sizeof(c128), true);
      g2.work = W[i].Th;
      g2.herm = 1;   // reorth_prep_kernel reads the upper triangle only
      g.push_back(g2);
    }
    if ((rc = gemm_run(g.data(), nc, GemmTypes{DT_C64, DT_C128}, s))) return rc;
    g.clear();
    for (int i = 0; i < nc; ++i) {
      const BondCall& c = calls[i];
      const int cap = c.b.cap(), mR = c.b.d * c.b.chi_r;
      hipLaunchKernelGGL(reorth_prep_kernel, dim3(grid_for((long long)cap * cap)), dim3(256), 0, s, W[i].G2, cap,
                         c.chi_new, (c64*)W[i].Dc);
      QT_HIP_CHECK(hipGetLastError());
      QT_HIP_CHECK(hipMemcpyAsync(W[i].tmp, c.b_n_out, (size_t)cap * mR * sizeof(cpx<S>), hipMemcpyDeviceToDevice, s));
      GemmProb g3 = gemm_prob(W[i].Dc, cap, OP_N, W[i].tmp, mR, OP_N, c.b_n_out, mR, cap, mR, cap, -1.f, 1.f);
      g3.dM = c.chi_new;
      g3.dK = c.chi_new;
      g.push_back(g3);
    }
    if ((rc = gemm_run(g.data(), nc, ty, s))) return rc;
  }
  // left-isometric output (Sec. II comments): A~^[m] = Q^[m], the explicit Q
  // of the (last) QR of X, (chi_l d) x eta
  for (int i = 0; i < nc; ++i) {
    const BondCall& c = calls[i];
    if (!c.b.left_iso) continue;
    const size_t bytes = (size_t)c.b.d * c.b.chi_l * c.b.eta * sizeof(cpx<S>);
    QT_HIP_CHECK(hipMemcpyAsync(c.b_m_out, W[i].X, bytes, hipMemcpyDeviceToDevice, s));
  }
  // B~^[m] = C~ B~^[n]^dag  (chi_l d x chi~, compact with the live chi~)
  g.clear();
  for (int i = 0; i < nc; ++i) {
    const BondCall& c = calls[i];
    if (c.b.left_iso) continue;
    const int cap = c.b.cap(), mL = c.b.d * c.b.chi_l, mR = c.b.d * c.b.chi_r;
    GemmProb gp = gemm_prob(W[i].C, mR, OP_N, c.b_n_out, mR, OP_C, c.b_m_out, cap, mL, cap, mR);
    gp.dN = c.chi_new;
    gp.ldc_live_N = 1;
    g.push_back(gp);
  }
  return g.empty() ? 0 : timed_gemm_batch(tm, g.data(), (int)g.size(), ty, s);
}

}  // namespace

int timed_gemm_batch(KernelTimer* t, const GemmProb* p, int n, GemmTypes ty, hipStream_t s) {
  if (!t || !t->on || t->n >= t->cap) return gemm_run(p, n, ty, s, true);
  const int i = t->n++;
  double fl = 0;
  for (int k = 0; k < n; ++k) fl += 8.0 * (double)p[k].M * (double)p[k].N * (double)p[k].K;
  t->flops[i] = fl;
  QT_HIP_CHECK(hipEventRecord(t->ev[2 * i], s));
  int rc = gemm_run(p, n, ty, s, true);
  if (rc) return rc;
  QT_HIP_CHECK(hipEventRecord(t->ev[2 * i + 1], s));
  return 0;
}

int timed_gemm(KernelTimer* t, const GemmProb& p, GemmTypes ty, hipStream_t s) {
  if (!t || !t->on || t->n >= t->cap) return gemm_one(p, ty, s, true);
  const int i = t->n++;
  t->flops[i] = 8.0 * (double)p.M * (double)p.N * (double)p.K;
  QT_HIP_CHECK(hipEventRecord(t->ev[2 * i], s));
  int rc = gemm_one(p, ty, s, true);
  if (rc) return rc;
  QT_HIP_CHECK(hipEventRecord(t->ev[2 * i + 1], s));
  return 0;
}

int two_site_c128(const BondShape& b, const void* xi_m, const void* b_m, const void* b_n, const c128* u, c128* C,
                  c128* Th, double* partial, double* norm2, hipStream_t s) {
  int rc;
  const int d = b.d, chiL = b.chi_l, chiR = b.chi_r, mL = d * chiL, mR = d * chiR;
  if ((rc = gemm_one(gemm_prob(b_m, b.chi_m, OP_N, b_n, mR, OP_N, C, mR, mL, mR, b.chi_m), GemmTypes{DT_C128, DT_C128},
                     s, true)))
    return rc;
  const int Wc = gate_width(d, sizeof(c128));
  const dim3 grid((chiR + Wc - 1) / Wc, chiL);
  const size_t shm = (size_t)d * d * Wc * sizeof(c128);
  const bool diag = b.xi_is_diag != 0;
  if ((rc = launch_gate<double>(C, diag ? Th : nullptr, u, diag ? (const double*)xi_m : nullptr, d, chiL, chiR, Wc,
                                partial, shm, s)))
    return rc;
  if (diag) return reduce_partials(partial, (int)(grid.x * grid.y), norm2, s);
  const int ncol = d * mR;
  if ((rc = gemm_one(gemm_prob(xi_m, chiL, OP_N, C, ncol, OP_N, Th, ncol, chiL, ncol, chiL), GemmTypes{DT_C128, DT_C128},
                     s)))
    return rc;
  const long long n = (long long)mL * mR;
  hipLaunchKernelGGL(sumsq_kernel<double>, dim3(1024), dim3(256), 0, s, (const c128*)Th, n, partial);
  QT_HIP_CHECK(hipGetLastError());
  return reduce_partials(partial, 1024, norm2, s);
}

int select_run(const double* lam, int kmax, double svd_min, const double* norm2, int* chi_new, double* xi,
               double* kept2, double* eps, int* status, hipStream_t s) {
  hipLaunchKernelGGL(select_kernel, dim3(1), dim3(256), 0, s, lam, kmax, svd_min, norm2, chi_new, xi, kept2, eps,
                     status);
  QT_HIP_CHECK(hipGetLastError());
  return 0;
}

int reduce_partials(const double* part, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(256), 0, s, part, n, out);
  QT_HIP_CHECK(hipGetLastError());
  return 0;
}

size_t bond_work_bytes(const BondShape& b) { return carve(b, nullptr).total + 256; }

void bond_pre_views(const BondShape& b, void* ws, void** C, void** Th, double** lam) {
  const BondBufs w = carve(b, ws);
  *C = w.C;
  *Th = w.Th;
  *lam = w.lam;
}

int bond_update_batch(const BondCall* calls, int n, hipStream_t s, KernelTimer* timer, const QrAsync* as) {
  if (n <= 0) return 0;
  const int prec = calls[0].b.prec;
  for (int i = 1; i < n; ++i)
    if (calls[i].b.prec != prec) return set_error(-1, "bond_update_batch: mixed precisions in one batch");
  return prec == 0 ? run_batch<double>(calls, n, s, timer, as) : run_batch<float>(calls, n, s, timer, as);
}

int bond_update_run(const BondShape& b, void* ws, int* status, const void* xi_m, const void* b_m, const void* b_n,
                    const c128* u, void* b_m_out, void* xi_n_out, void* b_n_out, int* chi_new, double* eps,
                    hipStream_t s, KernelTimer* timer, const QrAsync* as) {
  BondCall c{b, ws, status, xi_m, b_m, b_n, u, b_m_out, xi_n_out, b_n_out, chi_new, eps};
  return bond_update_batch(&c, 1, s, timer, as);
}

}  // namespace qrtebd
