// FP64 Hermitian eigensolver for step (iv) of controlled bond expansion
// (Sec. III): L^dag L = V^dag S^2 V.
//
//  1. Householder tridiagonalisation A = Q T Q^H (LAPACK zhetd2 conventions,
//     lower form) in one cooperative kernel.  The matrix rows live in LDS,
//     dealt cyclically to the blocks; the reflector vector, the trailing
//     row and the rank-2 update vector live in registers (column j of a
//     vector belongs to thread j mod 512).  Step k needs one grid barrier:
//     each block publishes its slice of p = tau A v and its part of p^H v,
//     and the current row k+1; after the barrier every block rebuilds row k+1
//     itself and derives the next reflector without further communication.
//     T is real symmetric because every off-diagonal beta is real.
//  2. The wanted (largest) eigenvalues of T by Sturm-count multisection, one
//     wave per eigenvalue (64 points per round).
//  3. Their eigenvectors by inverse iteration on T (tridiagonal LU with
//     partial pivoting, two solves from a fixed pseudo-random start), one
//     thread per vector.
//  4. Re-orthogonalisation inside each cluster of eigenvalues closer than
//     1e-11 |T| (where independent inverse iterations can return nearly
//     parallel vectors): modified Gram-Schmidt (two passes) for clusters of
//     up to 16 vectors; larger ones by blocked Gram-Schmidt in one workgroup,
//     one inverse-iteration step of the whole block with a shift just outside
//     the cluster (which removes the rounding that the first
//     orthogonalisation magnified) and blocked Gram-Schmidt again.  Then Newton-Schulz
//     steps Z <- Z - Z (Z^H Z - 1)/2 on the MFMA GEMM (two, and up to five
//     while the overlaps left by close unclustered eigenvalues remain).  Mixing two vectors by
//     their overlap, which is ~u|T|/gap, moves their residuals by ~u|T|
//     whatever the gap, so the polish keeps the eigenvectors accurate.
//  5. Back-transformation E = Q Z with the compact-WY blocks of step 1 on
//     the MFMA GEMM.
#include "eig.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace qrtebd {
namespace {

constexpr int NB = kQrNb;
constexpr int kMaxN = 2048;         // largest matrix
constexpr int kTriThreads = 512;    // threads of a tridiagonalisation block (two waves per SIMD)
constexpr int QMAX = kMaxN / kTriThreads;   // register slots per thread
constexpr size_t kTriLds = 150 * 1024;
// Eigenvalues closer than this times max |lambda| form a cluster whose
// inverse-iteration vectors are orthogonalised by Gram-Schmidt (below it they
// may come out nearly parallel); wider gaps leave overlaps of about u / rtol
// that the Newton-Schulz steps remove.
constexpr double kClusterRtol = 1e-11;
constexpr int kBigCluster = 16;   // larger clusters take the blocked Gram-Schmidt
constexpr int kPan = 16;          // its panel width
constexpr int kTriChunk = 8;          // rows per pass of register partials of A v
constexpr int kTriRows = 16;          // rows per block at most (two passes)
static_assert(kEigMaxN <= kMaxN, "eigensolver limit above the register layout");
static_assert((kEigMaxN + (int)(kTriLds / (16 * (size_t)kEigMaxN)) - 1) / (int)(kTriLds / (16 * (size_t)kEigMaxN)) <= 256,
              "rows of the largest matrix do not fit one block per CU");

__device__ inline c128 z0() { return mk<double>(0, 0); }

// x - (a conj(b) + c conj(d)), written with explicit fused operations so that
// every block evaluates it identically.
__device__ inline c128 rank2_sub(c128 x, c128 a, c128 b, c128 c, c128 d) {
  double re = fma(a.re, b.re, fma(a.im, b.im, fma(c.re, d.re, c.im * d.im)));
  double im = fma(a.im, b.re, fma(-a.re, b.im, fma(c.im, d.re, -c.re * d.im)));
  return mk<double>(x.re - re, x.im - im);
}

// One matrix of a batched tridiagonalisation launch: its blocks are
// [blk0, blk0 + nblk) of the grid and synchronise among themselves only.
struct TriProb {
  const c128* G;
  double* d;
  double* e;
  c128* tau;
  c128* V;        // QrWork V layout of the (n-1) x (n-1) reflector problem
  c128* pbuf;     // [2][n]
  c128* rowbuf;   // [2][n]
  c128* red;      // [2][nblk]
  unsigned* sync;
  int n, rows_loc, nblk, blk0;
};
constexpr int kMaxTriProbs = 16;
struct TriBatch {
  int nprob;
  int* status;
  TriProb p[kMaxTriProbs];
};

// Fixed-order block sums (every thread gets the result) with one barrier:
// scr (one entry per wave) must not be read by any thread after the block's
// previous barrier, so callers alternate between two buffers from one call
// to the next.
__device__ inline c128 block_sum_c1(c128 v, c128* scr) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v.re = wave_sum(v.re);
  v.im = wave_sum(v.im);
  if (lane == 0) scr[wid] = v;
  __syncthreads();
  c128 s = z0();
  for (int w = 0; w < nw; ++w) s = cadd(s, scr[w]);
  return s;
}
__device__ inline double block_sum1(double v, double* scr) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_sum(v);
  if (lane == 0) scr[wid] = v;
  __syncthreads();
  double s = 0;
  for (int w = 0; w < nw; ++w) s += scr[w];
  return s;
}

// Householder tridiagonalisation of one Hermitian matrix per block group.
// Rows are distributed cyclically (global row blk + r P in local row r, kept
// in LDS); every block also holds the current row k+1 and the vectors v, w
// of the step in registers (element j = tid + 512 q).  Step k: the reflector
// of row k (every block derives it from the same data), p = tau A v over the
// own rows, one grid barrier to exchange p and p^H v, w = p - tau/2 (p^H v) v,
// the rank-2 update A -= v w^H + w v^H.  The update of step k and the product
// A v of step k+1 share one pass over LDS: the reflector of row k+1 is formed
// first from the updated row k+1 (published by its owner before the barrier).
__global__ __launch_bounds__(kTriThreads) void tridiag_kernel(TriBatch batch) {
  extern __shared__ c128 rows[];  // rows_loc x n, local row r = global row blk + r * P
  __shared__ double scratch[2][kTriThreads / 64];   // alternating buffers of the block sums
  __shared__ c128 cscr[2][kTriThreads / 64];
  __shared__ double wred[2][kTriThreads / 64][16];   // alternating by row chunk
  __shared__ c128 vloc[2][kTriRows], wloc[kTriRows];
  __shared__ c128 scal[4];
  __shared__ int flag;

  int pi = 0;
  while (pi + 1 < batch.nprob && (int)blockIdx.x >= batch.p[pi + 1].blk0) ++pi;
  const TriProb& a = batch.p[pi];
  const GridSync gs{a.sync, batch.status};
  const int n = a.n, P = a.nblk, blk = (int)blockIdx.x - a.blk0, tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  const int RL = a.rows_loc;
  const int mqr = n - 1;

  for (int r = 0; r < RL; ++r) {
    const int gi = blk + r * P;
    if (gi < n)
      for (int j = tid; j < n; j += kTriThreads) rows[r * n + j] = a.G[(long long)gi * n + j];
  }
  // own[q]: local row of global row j = tid + 512 q if this block owns it, else -1
  int own[QMAX];
  c128 rk[QMAX], v[QMAX], w[QMAX];
#pragma unroll
  for (int q = 0; q < QMAX; ++q) {
    const int j = tid + kTriThreads * q;
    own[q] = (j < n && j % P == blk) ? j / P : -1;
    rk[q] = j < n ? a.G[j] : z0();
    v[q] = z0();
    w[q] = z0();
  }
  if (tid == 0) flag = 0;
  __syncthreads();
  if (n > 1 && 1 % P == blk) {   // row 1, final for step 0
    const int r = 1 / P;
    for (int j = tid; j < n; j += kTriThreads) pub_store(a.rowbuf + j, rows[r * n + j]);
  }

  // Reflector of row kk (held in rk): tau, the vector v (registers, vloc[vb]
  // for the own rows), d[kk], e[kk], tau[kk] and column kk of the QR layout.
  c128 tau = z0();
  auto reflector = [&](int kk, int vb) {
    double xn2 = 0;
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
      const int j = tid + kTriThreads * q;
      if (j >= kk + 2 && j < n) xn2 += cabs2(rk[q]);
      if (j == kk + 1) scal[0] = cconj(rk[q]);
      if (j == kk) scal[1] = rk[q];
    }
    xn2 = block_sum1(xn2, scratch[kk & 1]);  // its barrier also publishes scal[0], scal[1]
    const c128 alpha = scal[0];
    c128 scale = z0();
    tau = z0();
    double beta = alpha.re;
    if (!(xn2 == 0.0 && alpha.im == 0.0)) {
      beta = -copysign(sqrt(alpha.re * alpha.re + alpha.im * alpha.im + xn2), alpha.re);
      const double ib = rcp_refined(beta);
      tau = mk<double>((beta - alpha.re) * ib, -alpha.im * ib);
      const c128 den = mk<double>(alpha.re - beta, alpha.im);
      const double idd = rcp_refined(cabs2(den));
      scale = mk<double>(den.re * idd, -den.im * idd);
    }
    if (blk == 0 && tid == 0) {
      a.d[kk] = scal[1].re;
      a.e[kk] = beta;
      a.tau[kk] = tau;
      if (!isfinite(beta) || !isfinite(scal[1].re)) latch_error(batch.status, ERRBIT_NONFINITE);
    }
    const int p = kk / NB, c = kk % NB, j0 = p * NB;
    c128* Vp = a.V + qr_v_offset(p, mqr);
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
      const int j = tid + kTriThreads * q;
      v[q] = j == kk + 1 ? mk<double>(1, 0) : (j > kk + 1 && j < n ? cmul(cconj(rk[q]), scale) : z0());
      if (own[q] >= 0) {
        vloc[vb][own[q]] = v[q];
        if (j >= j0 + 1) Vp[(long long)(j - 1 - j0) * kQrLdv + c] = j >= kk + 1 ? v[q] : z0();
      }
    }
  };

  // p = tau A v over the own rows c0 .. c0+7 (i > kk) from the partial sums
  // acc[2(r-c0)], acc[2(r-c0)+1] of this thread: publishes those p and adds
  // their p^H v to `part` (wave 0); the last chunk publishes this block's
  // p^H v (slot sl).  Chunks alternate wred buffers, so one block barrier
  // per chunk suffices.
  c128 part = z0();
  auto publish_p = [&](double (&acc)[16], int kk, int sl, int vb, int c0) {
    const int cb = (c0 / kTriChunk) & 1;
    const double ws = wave_sum16(acc);   // lane l: wave total of acc[l >> 2]
    if ((lane & 3) == 0) wred[cb][wid][lane >> 2] = ws;
    __syncthreads();
    if (wid == 0) {
      if (c0 == 0) part = z0();
      if (lane < kTriChunk && c0 + lane < RL) {
        const int r = c0 + lane, gi = blk + r * P;
        c128 s = z0();
#pragma unroll
        for (int g = 0; g < kTriThreads / 64; ++g)
          s = cadd(s, mk<double>(wred[cb][g][2 * lane], wred[cb][g][2 * lane + 1]));
        if (gi > kk && gi < n) {
          const c128 pv = cmul(tau, s);
          pub_store(a.pbuf + (long long)sl * n + gi, pv);
          part = cadd(part, cmulc(pv, vloc[vb][r]));
        }
      }
      if (c0 + kTriChunk >= RL) {
        c128 t = part;
        t.re = wave_sum(t.re);
        t.im = wave_sum(t.im);
        if (lane == 0) pub_store(a.red + (long long)sl * P + blk, t);
      }
    }
  };

  // ---- step 0: reflector and product from the original rows
  int vb = 0;
  if (n > 1) {
    reflector(0, vb);
    for (int c0 = 0; c0 < RL; c0 += kTriChunk) {
      double acc[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[i] = 0.0;
#pragma unroll
      for (int rr = 0; rr < kTriChunk; ++rr) {
        const int r = c0 + rr;
        if (r < RL) {
          const int gi = blk + r * P;
          if (gi > 0 && gi < n) {
            c128 s = z0();
#pragma unroll
            for (int q = 0; q < QMAX; ++q) {
              const int j = tid + kTriThreads * q;
              if (j > 0 && j < n) s = cadd(s, cmul(rows[r * n + j], v[q]));
            }
            acc[2 * rr] = s.re;
            acc[2 * rr + 1] = s.im;
          }
        }
      }
      publish_p(acc, 0, 0, vb, c0);
    }
    if (!grid_barrier(gs, 1u, blk, P, &flag)) return;
  }

  for (int k = 0; k < n - 1; ++k) {
    const int slot = k & 1;
    // ---- one round of loads: block partials of p^H v, p, and row k+1
    const c128 rv = tid < P ? pub_load(a.red + (long long)slot * P + tid) : z0();
    c128 pv[QMAX], xb[QMAX];
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
      const int j = tid + kTriThreads * q;
      pv[q] = (j > k && j < n) ? pub_load(a.pbuf + (long long)slot * n + j) : z0();
      xb[q] = j < n ? pub_load(a.rowbuf + (long long)slot * n + j) : z0();
    }
    const c128 ptv = block_sum_c1(rv, cscr[k & 1]);   // p^H v
    const c128 alpha2 = cscale(cmul(tau, ptv), -0.5);
    // ---- w = p + alpha2 v
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
      const int j = tid + kTriThreads * q;
      w[q] = (j > k && j < n) ? cadd(pv[q], cmul(alpha2, v[q])) : z0();
      if (j == k + 1) scal[2] = w[q];
      if (own[q] >= 0) wloc[own[q]] = w[q];
    }
    __syncthreads();
    // row k+1 after the update of step k (v_{k+1} = 1)
    const c128 wk1 = scal[2];
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
      const int j = tid + kTriThreads * q;
      rk[q] = j < n ? (j > k ? rank2_sub(xb[q], mk<double>(1, 0), w[q], wk1, v[q]) : xb[q]) : z0();
    }
    if (k + 1 >= n - 1) break;   // no reflector left: rk is the last row

    // ---- reflector k+1 from the updated row k+1; v of step k stays in vk
    c128 vk[QMAX];
#pragma unroll
    for (int q = 0; q < QMAX; ++q) vk[q] = v[q];
    reflector(k + 1, vb ^ 1);   // ends with v = v_{k+1}; its block sum orders the LDS writes above
    // ---- one pass over the own rows i > k+1 (chunks of kTriChunk rows):
    // rank-2 update of step k and the partial sums of A v_{k+1} for step k+1
    vb ^= 1;
    for (int c0 = 0; c0 < RL; c0 += kTriChunk) {
      double acc[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[i] = 0.0;
#pragma unroll
      for (int rr = 0; rr < kTriChunk; ++rr) {
        const int r = c0 + rr;
        if (r < RL) {
          const int gi = blk + r * P;
          if (gi > k + 1 && gi < n) {
            const c128 vi = vloc[vb ^ 1][r], wi = wloc[r];
            c128 s = z0();
#pragma unroll
            for (int q = 0; q < QMAX; ++q) {
              const int j = tid + kTriThreads * q;
              if (j > k && j < n) {
                const c128 x = rank2_sub(rows[r * n + j], vi, w[q], wi, vk[q]);
                rows[r * n + j] = x;
                s = cadd(s, cmul(x, v[q]));
              }
            }
            acc[2 * rr] = s.re;
            acc[2 * rr + 1] = s.im;
          }
        }
      }
      publish_p(acc, k + 1, slot ^ 1, vb, c0);   // its block barrier orders the row writes above
    }
    // row k+2, final for step k+1, from its owner
    if ((k + 2) % P == blk) {
      const int r = (k + 2) / P;
      for (int j = tid; j < n; j += kTriThreads) pub_store(a.rowbuf + (long long)(slot ^ 1) * n + j, rows[r * n + j]);
    }
    if (!grid_barrier(gs, (unsigned)(k + 2), blk, P, &flag)) return;
  }
  // d[n-1] from the thread holding column n-1 of the final row
  if (blk == 0) {
#pragma unroll
    for (int q = 0; q < QMAX; ++q)
      if (tid + kTriThreads * q == n - 1) {
        a.d[n - 1] = rk[q].re;
        a.e[n - 1] = 0.0;
        a.tau[n - 1] = z0();
      }
  }
}

// Gershgorin interval and pivmin of (d, e) held in LDS; every thread gets them.
__device__ inline void gersh(const double* d, const double* e2, int n, double* scr, double& lo, double& hi,
                             double& pivmin) {
  double l = 1e300, h = -1e300, em = 0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double r = (i > 0 ? sqrt(e2[i - 1]) : 0.0) + (i < n - 1 ? sqrt(e2[i]) : 0.0);
    l = fmin(l, d[i] - r);
    h = fmax(h, d[i] + r);
    if (i < n - 1) em = fmax(em, e2[i]);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    l = fmin(l, __shfl_xor(l, o, 64));
    h = fmax(h, __shfl_xor(h, o, 64));
    em = fmax(em, __shfl_xor(em, o, 64));
  }
  const int wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    scr[3 * wid] = l;
    scr[3 * wid + 1] = h;
    scr[3 * wid + 2] = em;
  }
  __syncthreads();
  l = scr[0]; h = scr[1]; em = scr[2];
  for (int w = 1; w < nw; ++w) {
    l = fmin(l, scr[3 * w]);
    h = fmax(h, scr[3 * w + 1]);
    em = fmax(em, scr[3 * w + 2]);
  }
  const double tnorm = fmax(fabs(l), fabs(h));
  pivmin = fmax(2.2250738585072014e-308, 2.2250738585072014e-308 * em);
  lo = l - 2.2e-16 * tnorm - 2 * pivmin;
  hi = h + 2.2e-16 * tnorm + 2 * pivmin;
}

struct SmallJob {
  const double* d;
  const double* e;
  double* lam;
  double* lu;
  unsigned char* swp;
  c128* E;
  c128* V;
  c128* T;
  const c128* tau;
  const c128* tpart;
  double* zr;   // blocked Gram-Schmidt: row-major cluster copies (n x m at n j)
  double* zc;   // column-major cluster copies (n x m at n j)
  double* wb;   // projection coefficients (m x kPan at kPan j)
  int n, kwant;
};
constexpr int kMaxSmallJobs = 24;
struct SmallBatch {
  int njobs;
  SmallJob j[kMaxSmallJobs];
};

// lam[j] = (j+1)-th largest eigenvalue, j < kwant.  Multisection with one
// wave per eigenvalue: each lane evaluates one of the 64 interior points of
// the current interval per round, shrinking it 65-fold; the points whose
// count does not exceed the target index form a prefix, so the new interval
// follows from one ballot.  10 rounds shrink the Gershgorin interval by 2^60,
// past FP64 resolution.
constexpr int kBisectPts = 1;
constexpr int kBisectRounds = 10;

__global__ __launch_bounds__(256) void bisect_kernel(SmallBatch sb) {
  const SmallJob& J = sb.j[blockIdx.y];
  const double* d = J.d;
  const double* e = J.e;
  const int n = J.n, kwant = J.kwant;
  double* lam = J.lam;
  if ((int)blockIdx.x * 4 >= kwant) return;
  __shared__ double sd[kMaxN], se2[kMaxN];
  __shared__ double scr[12];
  for (int i = threadIdx.x; i < n; i += 256) {
    sd[i] = d[i];
    se2[i] = i < n - 1 ? e[i] * e[i] : 0.0;
  }
  __syncthreads();
  double lo, hi, pivmin;
  gersh(sd, se2, n, scr, lo, hi, pivmin);
  const int lane = threadIdx.x & 63;
  const int j = min((int)blockIdx.x * 4 + (int)(threadIdx.x >> 6), kwant - 1);
  const int idx = n - 1 - j;  // ascending index
  constexpr int npts = 64 * kBisectPts;
  constexpr double inv = 1.0 / (npts + 1);
  double a = lo, b = hi;
  for (int it = 0; it < kBisectRounds; ++it) {
    const double w = b - a;
    double x[kBisectPts], q[kBisectPts];
    int cnt[kBisectPts];
#pragma unroll
    for (int c = 0; c < kBisectPts; ++c) {
      x[c] = a + w * (double)(kBisectPts * lane + c + 1) * inv;
      q[c] = sd[0] - x[c];
      if (fabs(q[c]) < pivmin) q[c] = -pivmin;
      cnt[c] = q[c] < 0;
    }
    for (int i = 1; i < n; ++i) {
      const double di = sd[i], ei = se2[i - 1];
#pragma unroll
      for (int c = 0; c < kBisectPts; ++c) {
        // e^2 / q by the hardware reciprocal and one Newton step (within an
        // ulp or two of the division, enough for the sign of the pivot; |q|
        // >= pivmin keeps it finite)
        const double r0 = __builtin_amdgcn_rcp(q[c]);
        const double r1 = fma(r0, fma(-q[c], r0, 1.0), r0);
        double t = di - x[c] - ei * r1;
        if (fabs(t) < pivmin) t = -pivmin;
        q[c] = t;
        cnt[c] += t < 0;
      }
    }
    // f = number of points (in increasing order) whose count is <= idx
    int f = 0;
#pragma unroll
    for (int c = 0; c < kBisectPts; ++c) f += __popcll(~__ballot(cnt[c] > idx));
    const double na = f == 0 ? a : a + w * (double)f * inv;
    const double nb = f == npts ? b : a + w * (double)(f + 1) * inv;
    a = na;
    b = nb;
  }
  if (lane == 0 && (int)blockIdx.x * 4 + (int)(threadIdx.x >> 6) < kwant) lam[j] = 0.5 * (a + b);
}

__device__ inline double hash_uniform(unsigned long long x) {
  x += 0x9e3779b97f4a7c15ULL;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ULL;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebULL;
  x ^= x >> 31;
  return (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// Inverse iteration for eigenvalue lam[j]: E[:, j] (real, stored complex).
// One thread per eigenvalue, G eigenvalues per block, everything in LDS: T =
// (d, e) and, per eigenvalue, the factors of T - lam I with partial pivoting
// and the work vector.  Step k of the factorisation keeps the reciprocal
// pivot R0 = 1/u0, a flag for a row interchange, and Q = the second entry u1
// of the pivot row (no interchange) or the displaced pivot candidate c (the
// multiplier's numerator; an interchanged pivot row is (e[k], d[k+1] - lam,
// e[k+1])), so the multiplier is e[k] R0 or c R0 either way.  Two solves: a
// hashed uniform start vector (eliminated while factoring), then the
// max-normalised first solution; the result has unit 2-norm.
constexpr int kInvitLds = 159 * 1024;
constexpr int kIvChunk = 16;   // steps whose operands are loaded before their recurrence
__host__ __device__ inline size_t invit_lds_bytes(int n, int g) { return ((size_t)2 + 3 * (size_t)g) * n * 8 + (size_t)g * n; }
inline int invit_group(int n) {
  int g = 8;
  while (g > 1 && invit_lds_bytes(n, g) > (size_t)kInvitLds) --g;
  return g;
}

__global__ __launch_bounds__(64) void invit_kernel(SmallBatch sb, int G) {
  extern __shared__ double sm[];
  const SmallJob& J = sb.j[blockIdx.y];
  const int n = J.n, kwant = J.kwant;
  if ((int)blockIdx.x * G >= kwant) return;
  double* __restrict__ sd = sm;
  double* __restrict__ se = sm + n;
  const int g = threadIdx.x;
  double tn = 0;
  for (int i = threadIdx.x; i < n; i += 64) {
    sd[i] = J.d[i];
    se[i] = i < n - 1 ? J.e[i] : 0.0;
    tn = fmax(tn, fabs(J.d[i]) + (i > 0 ? fabs(J.e[i - 1]) : 0.0) + (i < n - 1 ? fabs(J.e[i]) : 0.0));
  }
  const double tnorm = wave_max(tn);
  __syncthreads();
  const int j = blockIdx.x * G + g;
  if (g >= G || j >= kwant) return;
  double* __restrict__ R0 = sm + 2 * (size_t)n + (size_t)g * 3 * n;
  double* __restrict__ Q = R0 + n;
  double* __restrict__ W = Q + n;
  unsigned char* __restrict__ sw = (unsigned char*)(sm + 2 * (size_t)n + (size_t)G * 3 * n) + (size_t)g * n;
  const double l = J.lam[j];
  const double tiny = fmax(tnorm, 1e-300) * 2.2e-16;
  auto start = [&](int i) { return hash_uniform(((unsigned long long)j << 32) ^ (unsigned)i); };
  // factor (row k+1 enters at step k) and eliminate the start vector
  double c0 = sd[0] - l, c1 = n > 1 ? se[0] : 0.0;
  double rc = start(0);
#pragma unroll 4
  for (int k = 0; k < n - 1; ++k) {
    const double n0 = se[k], n1 = sd[k + 1] - l, n2 = se[k + 1];
    const double bk1 = start(k + 1);
    // keep: pivot row (c0, c1, 0), else interchange: pivot row (n0, n1, n2);
    // one path for all lanes (a zero pivot is replaced by tiny; then n0 = 0
    // and the multiplier is 0)
    const bool keep = fabs(c0) >= fabs(n0);
    const double r0 = rcp_refined(keep ? (c0 != 0.0 ? c0 : tiny) : n0);
    const double m = (keep ? n0 : c0) * r0;
    R0[k] = r0;
    Q[k] = keep ? c1 : c0;
    sw[k] = keep ? 0 : 1;
    W[k] = keep ? rc : bk1;
    const double c0n = keep ? n1 - m * c1 : c1 - m * n1;
    c1 = keep ? n2 : -m * n2;
    c0 = c0n;
    rc = keep ? bk1 - m * rc : rc - m * bk1;
  }
  R0[n - 1] = rcp_refined(c0 == 0.0 ? tiny : c0);
  Q[n - 1] = 0.0;
  sw[n - 1] = 0;
  W[n - 1] = rc;

  double scale = 1.0, f = 1.0;
  for (int it = 0; it < 2; ++it) {
    if (it == 1) {   // the factorisation's row operations on the scaled first solution
      double r = W[0] * scale;
      for (int k0 = 0; k0 < n - 1; k0 += kIvChunk) {   // operands of a chunk first, then the recurrence
        int xs[kIvChunk];
        double bb[kIvChunk], mm[kIvChunk];
#pragma unroll
        for (int t = 0; t < kIvChunk; ++t)
          if (k0 + t < n - 1) {
            xs[t] = sw[k0 + t];
            bb[t] = W[k0 + t + 1] * scale;
          }
#pragma unroll
        for (int t = 0; t < kIvChunk; ++t)
          if (k0 + t < n - 1) mm[t] = *(xs[t] ? Q + k0 + t : se + k0 + t) * R0[k0 + t];   // a selected address
#pragma unroll
        for (int t = 0; t < kIvChunk; ++t)
          if (k0 + t < n - 1) {
            const bool keep = xs[t] == 0;
            W[k0 + t] = keep ? r : bb[t];
            r = keep ? bb[t] - mm[t] * r : r - mm[t] * bb[t];
          }
      }
      W[n - 1] = r;
    }
    // back substitution; the first pass's max norm rescales the second, the
    // second accumulates the 2-norm
    double z1 = 0.0, z2 = 0.0, nrm = 0.0, s2 = 0.0;
    for (int i0 = n - 1; i0 >= 0; i0 -= kIvChunk) {
      // operands of a chunk first (loads from selected addresses, no
      // branches): after an interchange the pivot row is (e[i], d[i+1] - lam,
      // e[i+1]), else (u0, Q[i], 0); then the recurrence
      int xs[kIvChunk];
      double bb[kIvChunk], rr[kIvChunk], a1[kIvChunk], a2[kIvChunk];
#pragma unroll
      for (int t = 0; t < kIvChunk; ++t)
        if (i0 - t >= 0) {
          xs[t] = sw[i0 - t];
          bb[t] = W[i0 - t];
          rr[t] = R0[i0 - t];
        }
#pragma unroll
      for (int t = 0; t < kIvChunk; ++t)
        if (i0 - t >= 0) {
          const int i = i0 - t;
          a1[t] = *(xs[t] ? sd + i + 1 : Q + i) - (xs[t] ? l : 0.0);
          a2[t] = se[min(i + 1, n - 1)] * (double)xs[t];
        }
#pragma unroll
      for (int t = 0; t < kIvChunk; ++t)
        if (i0 - t >= 0) {
          const double z = (bb[t] - a1[t] * z1 - a2[t] * z2) * rr[t];
          W[i0 - t] = z;
          z2 = z1;
          z1 = z;
          nrm = fmax(nrm, fabs(z));
          s2 += z * z;
        }
    }
    if (it == 0) {
      scale = nrm > 0 ? 1.0 / nrm : 1.0;
    } else {
      f = s2 > 0 ? 1.0 / sqrt(s2) : 0.0;
      if (nrm > 1e150 || (nrm > 0 && nrm < 1e-150)) {   // sum of squares out of range: rescale by the max
        double t2 = 0.0;
        for (int i = 0; i < n; ++i) {
          const double z = W[i] / nrm;
          t2 += z * z;
        }
        f = 1.0 / (nrm * sqrt(t2));
      }
    }
  }
  c128* E = J.E;
  for (int i = 0; i < n; ++i) E[(size_t)i * kwant + j] = mk<double>(W[i] * f, 0.0);
}

// Split-K parts of the panel Gram products V_p^H V_p (K = rows of the panel).
constexpr int kLarftParts = 8;
__host__ __device__ inline int larft_parts(int K) { return K / 128 < 1 ? 1 : (K / 128 > kLarftParts ? kLarftParts : K / 128); }

// T_p for every panel of the tridiagonalisation reflectors from the Gram
// matrix V_p^H V_p (summed from the split-K partials of the GEMM launched
// before this kernel).
__global__ __launch_bounds__(256) void larft_kernel(SmallBatch sb) {
  __shared__ c128 slab[NB][NB + 1];
  __shared__ c128 Tm[NB][NB + 1];
  const SmallJob& J = sb.j[blockIdx.y];
  c128* T = J.T;
  const c128* tau = J.tau;
  const int m = J.n - 1, nrefl = J.n - 1;
  const int p = blockIdx.x, tid = threadIdx.x;
  if (p * NB >= nrefl) return;
  const int j0 = p * NB, jb = min(NB, nrefl - j0), mp = m - j0;
  const int parts = larft_parts(mp);
  const c128* gp = J.tpart + (size_t)p * kLarftParts * NB * NB;
  c128 g[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    c128 l[kLarftParts];
#pragma unroll
    for (int u = 0; u < kLarftParts; ++u) l[u] = u < parts ? gp[(size_t)u * NB * NB + tid + 256 * q] : z0();
    g[q] = l[0];
#pragma unroll
    for (int u = 1; u < kLarftParts; ++u) g[q] = cadd(g[q], l[u]);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = tid + 256 * q;
    slab[e / NB][e % NB] = g[q];
    Tm[e / NB][e % NB] = z0();
  }
  __syncthreads();
  for (int k = 0; k < jb; ++k) {
    const c128 tk = tau[j0 + k];
    if (tid < k) {
      c128 sacc = z0();
      for (int q = tid; q < k; ++q) sacc = cadd(sacc, cmul(Tm[tid][q], slab[q][k]));
      Tm[tid][k] = cmul(mk<double>(-tk.re, -tk.im), sacc);
    }
    if (tid == k) Tm[k][k] = tk;
    __syncthreads();
  }
  for (int idx = tid; idx < NB * NB; idx += 256) T[(size_t)p * NB * NB + idx] = Tm[idx / NB][idx % NB];
}

// Two-pass modified Gram-Schmidt over each cluster of close eigenvalues
// (lam descending; a cluster starts where the gap to the previous value
// exceeds rtol * max|lam|) of at most kBigCluster columns.  Block b handles
// the cluster starting at column b, if any.
__global__ __launch_bounds__(256) void cluster_mgs_kernel(SmallBatch sb, double rtol) {
  __shared__ double scr[8];
  const SmallJob& J = sb.j[blockIdx.y];
  c128* Z = J.E;
  const double* lam = J.lam;
  const int n = J.n, kw = J.kwant;
  const int j = blockIdx.x;
  if (j >= kw) return;
  const double ctol = rtol * fmax(fabs(lam[0]), fabs(lam[kw - 1]));
  if (j > 0 && lam[j - 1] - lam[j] <= ctol) return;
  int e = j;
  while (e + 1 < kw && lam[e] - lam[e + 1] <= ctol && e - j < kBigCluster) ++e;   // larger: cluster_bcgs_kernel
  if (e == j || e - j + 1 > kBigCluster) return;
  for (int pass = 0; pass < 2; ++pass)
    for (int v = j; v <= e; ++v) {
      for (int u = j; u < v; ++u) {
        double dot = 0;
        for (int i = threadIdx.x; i < n; i += 256) dot += Z[(long long)i * kw + u].re * Z[(long long)i * kw + v].re;
        dot = block_sum(dot, scr);
        for (int i = threadIdx.x; i < n; i += 256) Z[(long long)i * kw + v].re -= dot * Z[(long long)i * kw + u].re;
        __syncthreads();
      }
      double nn = 0;
      for (int i = threadIdx.x; i < n; i += 256) nn += Z[(long long)i * kw + v].re * Z[(long long)i * kw + v].re;
      nn = block_sum(nn, scr);
      const double f = nn > 0 ? 1.0 / sqrt(nn) : 0.0;
      for (int i = threadIdx.x; i < n; i += 256) Z[(long long)i * kw + v].re *= f;
      __syncthreads();
    }
}

// ---- blocked Gram-Schmidt for clusters of more than kBigCluster columns
// (one workgroup per cluster).  The cluster's m columns are copied twice,
// row-major (Zr) and column-major (Zc), so that both products below read
// memory contiguously.  Panels of kPan columns, each taken twice:
//   W = Zr[:, :p0]^T Zr[:, p0:p0+P]     (lanes own columns u, loop over rows)
//   Zc[:, p0:p0+P] -= Zc[:, :p0] W      (lanes own rows, loop over u)
//   classical Gram-Schmidt inside the panel, column by column, and
//   normalisation (the panel lives in registers, one block sum per step).
// Two passes of the whole sequence give every column two projections
// against all earlier columns of the cluster, as the two-pass MGS does.
constexpr int kBcgsThreads = 512;
constexpr int kBcgsRows = 3;    // matrix rows per thread in the row-owned phases
constexpr int kBcgsChunk = 64;  // rows (or u) per LDS chunk
static_assert(kEigMaxN <= kBcgsThreads * kBcgsRows, "blocked Gram-Schmidt row slots");
constexpr int kBcgsLds = 2 * kBcgsChunk * kPan + 4 * kBcgsThreads;
// LU factors of T - sigma: four n-vectors and n interchange flags
constexpr int kFilterLds = 4 * kEigMaxN + kEigMaxN / 8;
// distance of the cluster filter's shift from the cluster, relative to max |lam|
constexpr double kFilterRel = 1e-8;

// Start and size of the g-th cluster of more than kBigCluster columns
// (out[0] = -1 if there is none); lam staged in lds (kw doubles).  Every
// thread looks at its own columns: a cluster start walks to its end (at
// most the cluster's size in steps), a large cluster enters a list, and its
// rank in the list (by column) decides which block takes it.
constexpr int kMaxBigClusters = kEigMaxN / (kBigCluster + 1) + 1;
__device__ inline void find_big_cluster(const double* lam, int kw, double rtol, int g, double* lds, int* out) {
  __shared__ int nbig;
  __shared__ int big[kMaxBigClusters];
  for (int c = threadIdx.x; c < kw; c += blockDim.x) lds[c] = lam[c];
  if (threadIdx.x == 0) {
    nbig = 0;
    out[0] = -1;
    out[1] = 0;
  }
  __syncthreads();
  const double ctol = rtol * fmax(fabs(lds[0]), fabs(lds[kw - 1]));
  for (int c = threadIdx.x; c < kw; c += blockDim.x) {
    if (c > 0 && lds[c - 1] - lds[c] <= ctol) continue;   // not a cluster start
    int e = c;
    while (e + 1 < kw && lds[e] - lds[e + 1] <= ctol) ++e;
    if (e - c + 1 > kBigCluster) big[atomicAdd(&nbig, 1)] = c;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nbig; i += blockDim.x) {
    const int c = big[i];
    int rank = 0;
    for (int k = 0; k < nbig; ++k) rank += big[k] < c;
    if (rank == g) {
      int e = c;
      while (e + 1 < kw && lds[e] - lds[e + 1] <= ctol) ++e;
      out[0] = c;
      out[1] = e - c + 1;
    }
  }
  __syncthreads();
}

// Block sum of 16 values (every thread gets all 16), fixed order; sc holds
// 8 * 16 + 16 doubles and must not be read by any thread since the block's
// previous barrier.
__device__ inline void block_sum16(double (&x)[kPan], double* sc) {
  static_assert(kPan == 16, "block_sum16 reduces 16 values");
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const double t = wave_sum16(x);   // lane l: wave total of x[l >> 2]
  if ((lane & 3) == 0) sc[wid * kPan + (lane >> 2)] = t;
  __syncthreads();
  if (threadIdx.x < kPan) {
    double a = 0;
    for (int w = 0; w < kBcgsThreads / 64; ++w) a += sc[w * kPan + threadIdx.x];
    sc[(kBcgsThreads / 64) * kPan + threadIdx.x] = a;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kPan; ++u) x[u] = sc[(kBcgsThreads / 64) * kPan + u];
}

// W[u][v] = sum_i Zr[i][u] Zr[i][p0 + v] for u < p0, v < kPan (zero for v >= P).
__device__ inline void bcgs_dots(const double* Zr, int n, int m, int p0, int P, double* Wb, double* lds) {
  const int tid = threadIdx.x;
  const int Gp = (((p0 + 3) / 4) + 63) & ~63;   // lanes over u, whole waves
  const int R = kBcgsThreads / Gp;             // row slices (>= 1)
  const int ug = tid % Gp, r = tid / Gp;
  const bool act = r < R;
  double acc[4][kPan];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int v = 0; v < kPan; ++v) acc[k][v] = 0;
  double* pan = lds;   // kBcgsChunk x kPan
  for (int i0 = 0; i0 < n; i0 += kBcgsChunk) {
    const int ie = min(kBcgsChunk, n - i0);
    for (int q = tid; q < kBcgsChunk * kPan; q += kBcgsThreads) {
      const int ii = q / kPan, v = q % kPan;
      pan[q] = (ii < ie && v < P) ? Zr[(size_t)(i0 + ii) * m + p0 + v] : 0.0;
    }
    __syncthreads();
    if (act) {
      for (int ii = r; ii < ie; ii += R) {
        const double* row = Zr + (size_t)(i0 + ii) * m;
        double a[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          const int u = ug + k * Gp;
          a[k] = u < p0 ? row[u] : 0.0;
        }
        const double2* pr = (const double2*)(pan + ii * kPan);
#pragma unroll
        for (int v2 = 0; v2 < kPan / 2; ++v2) {
          const double2 pv = pr[v2];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            acc[k][2 * v2] = fma(a[k], pv.x, acc[k][2 * v2]);
            acc[k][2 * v2 + 1] = fma(a[k], pv.y, acc[k][2 * v2 + 1]);
          }
        }
      }
    }
    __syncthreads();
  }
  // sum over the row slices in slice order, four values a round
  double* red = lds;   // (R - 1) x Gp x 4
#pragma unroll
  for (int q = 0; q < 4 * kPan; q += 4) {
    if (act && r > 0)
#pragma unroll
      for (int t = 0; t < 4; ++t) red[((r - 1) * Gp + ug) * 4 + t] = acc[(q + t) / kPan][(q + t) % kPan];
    __syncthreads();
    if (r == 0) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        double sum = acc[(q + t) / kPan][(q + t) % kPan];
        for (int rr = 1; rr < R; ++rr) sum += red[((rr - 1) * Gp + ug) * 4 + t];
        const int u = ug + ((q + t) / kPan) * Gp;
        if (u < p0) Wb[(size_t)u * kPan + (q + t) % kPan] = sum;
      }
    }
    __syncthreads();
  }
}

// Zc[:, p0 + v] -= sum_{u < p0} Zc[:, u] W[u][v], v < P.
__device__ inline void bcgs_update(double* Zc, int n, int p0, int P, const double* Wb, double* lds) {
  const int tid = threadIdx.x;
  double acc[kBcgsRows][kPan];
#pragma unroll
  for (int q = 0; q < kBcgsRows; ++q)
#pragma unroll
    for (int v = 0; v < kPan; ++v) acc[q][v] = 0;
  double* wch = lds;   // kBcgsChunk x kPan
  for (int u0 = 0; u0 < p0; u0 += kBcgsChunk) {
    const int ue = min(kBcgsChunk, p0 - u0);
    for (int q = tid; q < kBcgsChunk * kPan; q += kBcgsThreads)
      wch[q] = q / kPan < ue ? Wb[(size_t)u0 * kPan + q] : 0.0;
    __syncthreads();
#pragma unroll 2
    for (int uu = 0; uu < ue; ++uu) {
      const double* col = Zc + (size_t)(u0 + uu) * n;
      double z[kBcgsRows];
#pragma unroll
      for (int q = 0; q < kBcgsRows; ++q) {
        const int i = tid + q * kBcgsThreads;
        z[q] = i < n ? col[i] : 0.0;
      }
      const double2* wr = (const double2*)(wch + uu * kPan);
#pragma unroll
      for (int v2 = 0; v2 < kPan / 2; ++v2) {
        const double2 w = wr[v2];
#pragma unroll
        for (int q = 0; q < kBcgsRows; ++q) {
          acc[q][2 * v2] = fma(z[q], w.x, acc[q][2 * v2]);
          acc[q][2 * v2 + 1] = fma(z[q], w.y, acc[q][2 * v2 + 1]);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < kBcgsRows; ++q) {
    const int i = tid + q * kBcgsThreads;
    if (i < n)
#pragma unroll
      for (int v = 0; v < kPan; ++v)
        if (v < P) Zc[(size_t)(p0 + v) * n + i] -= acc[q][v];
  }
}

// Classical Gram-Schmidt and normalisation inside the panel (columns p0 ..
// p0 + P of Zc); the result is written to both copies.
__device__ inline void bcgs_panel(double* Zc, double* Zr, int n, int m, int p0, int P, double* lds) {
  const int tid = threadIdx.x;
  double x[kBcgsRows][kPan];
#pragma unroll
  for (int q = 0; q < kBcgsRows; ++q) {
    const int i = tid + q * kBcgsThreads;
#pragma unroll
    for (int v = 0; v < kPan; ++v) x[q][v] = (i < n && v < P) ? Zc[(size_t)(p0 + v) * n + i] : 0.0;
  }
  int buf = 0;
#pragma unroll
  for (int v = 0; v < kPan; ++v) {
    if (v >= P) continue;   // uniform over the block
    if (v > 0) {
      double dp[kPan];
#pragma unroll
      for (int u = 0; u < kPan; ++u) {
        double a = 0;
        if (u < v)
#pragma unroll
          for (int q = 0; q < kBcgsRows; ++q) a = fma(x[q][u], x[q][v], a);
        dp[u] = a;
      }
      block_sum16(dp, lds + buf * 160);
      buf ^= 1;
#pragma unroll
      for (int q = 0; q < kBcgsRows; ++q) {
        double y = x[q][v];
#pragma unroll
        for (int u = 0; u < kPan; ++u)
          if (u < v) y = fma(-dp[u], x[q][u], y);
        x[q][v] = y;
      }
    }
    double nn = 0;
#pragma unroll
    for (int q = 0; q < kBcgsRows; ++q) nn = fma(x[q][v], x[q][v], nn);
    nn = block_sum1(nn, lds + 320 + buf * 8);
    buf ^= 1;
    const double f = nn > 0 ? 1.0 / sqrt(nn) : 0.0;
#pragma unroll
    for (int q = 0; q < kBcgsRows; ++q) x[q][v] *= f;
  }
#pragma unroll
  for (int q = 0; q < kBcgsRows; ++q) {
    const int i = tid + q * kBcgsThreads;
    if (i < n)
#pragma unroll
      for (int v = 0; v < kPan; ++v)
        if (v < P) {
          Zc[(size_t)(p0 + v) * n + i] = x[q][v];
          Zr[(size_t)i * m + p0 + v] = x[q][v];
        }
  }
  __syncthreads();
}

// Zc = Zr (n x m row-major to column-major) through 32 x 32 LDS tiles.
__device__ inline void rows_to_cols(const double* Zr, int n, int m, double* Zc, double* tile) {
  for (int i0 = 0; i0 < n; i0 += 32)
    for (int c0 = 0; c0 < m; c0 += 32) {
      for (int q = threadIdx.x; q < 1024; q += kBcgsThreads) {
        const int a = q >> 5, b = q & 31, i = i0 + a, c = c0 + b;
        tile[a * 33 + b] = (i < n && c < m) ? Zr[(size_t)i * m + c] : 0.0;
      }
      __syncthreads();
      for (int q = threadIdx.x; q < 1024; q += kBcgsThreads) {
        const int a = q >> 5, b = q & 31, c = c0 + a, i = i0 + b;
        if (i < n && c < m) Zc[(size_t)c * n + i] = tile[b * 33 + a];
      }
      __syncthreads();
    }
}

// Both passes over all panels of the cluster.
__device__ __attribute__((noinline)) void bcgs_all(double* Zr, double* Zc, int n, int m, double* Wb, double* lds) {
  for (int p0 = 0; p0 < m; p0 += kPan) {
    const int P = min(kPan, m - p0);
    for (int pass = 0; pass < 2; ++pass) {
      if (p0 > 0) {
        bcgs_dots(Zr, n, m, p0, P, Wb, lds);
        bcgs_update(Zc, n, p0, P, Wb, lds);
      }
      bcgs_panel(Zc, Zr, n, m, p0, P, lds);
    }
  }
}

// Gaussian elimination with partial pivoting of the tridiagonal T - sigma
// (one thread; LAPACK dgttrf layout): multipliers dl, reciprocal pivots rp,
// first and second superdiagonals du, du2 of U, interchange flags sw.  A
// zero pivot becomes tiny.
__device__ inline void tri_lu(const double* d, const double* e, int n, double sigma, double tiny, double* dl,
                              double* rp, double* du, double* du2, unsigned char* sw) {
  double piv = d[0] - sigma, up = n > 1 ? e[0] : 0.0;
  for (int k = 0; k < n - 1; ++k) {
    const double sub = e[k], dn = d[k + 1] - sigma, upn = k + 1 < n - 1 ? e[k + 1] : 0.0;
    if (fabs(piv) >= fabs(sub)) {   // rows stay: pivot row (piv, up, 0)
      const double p = piv != 0.0 ? piv : tiny;
      const double l = sub / p;
      rp[k] = 1.0 / p;
      du[k] = up;
      du2[k] = 0.0;
      dl[k] = l;
      sw[k] = 0;
      piv = dn - l * up;
      up = upn;
    } else {                        // interchange: pivot row (sub, dn, upn)
      const double l = piv / sub;
      rp[k] = 1.0 / sub;
      du[k] = dn;
      du2[k] = upn;
      dl[k] = l;
      sw[k] = 1;
      piv = up - l * dn;
      up = -l * upn;
    }
  }
  rp[n - 1] = 1.0 / (piv != 0.0 ? piv : tiny);
  du[n - 1] = 0.0;
  du2[n - 1] = 0.0;
  sw[n - 1] = 0;
}

// x <- (T - sigma)^-1 x for column c of the row-major n x m block X (in place).
__device__ inline void tri_solve_col(double* X, int n, int m, int c, const double* dl, const double* rp,
                                     const double* du, const double* du2, const unsigned char* sw) {
  constexpr int CH = 8;
  double* x = X + c;
  double b = x[0];   // running row k of the eliminated right-hand side
  for (int k0 = 0; k0 < n - 1; k0 += CH) {
    double nx[CH], out[CH];
#pragma unroll
    for (int t = 0; t < CH; ++t) nx[t] = k0 + t < n - 1 ? x[(size_t)(k0 + t + 1) * m] : 0.0;
#pragma unroll
    for (int t = 0; t < CH; ++t) {
      const int k = k0 + t;
      if (k < n - 1) {
        const double l = dl[k];
        if (sw[k]) {
          out[t] = nx[t];
          b = b - l * nx[t];
        } else {
          out[t] = b;
          b = nx[t] - l * b;
        }
      }
    }
#pragma unroll
    for (int t = 0; t < CH; ++t)
      if (k0 + t < n - 1) x[(size_t)(k0 + t) * m] = out[t];
  }
  x[(size_t)(n - 1) * m] = b;
  double z1 = 0.0, z2 = 0.0;
  for (int k0 = n - 1; k0 >= 0; k0 -= CH) {
    double bb[CH];
#pragma unroll
    for (int t = 0; t < CH; ++t) bb[t] = k0 - t >= 0 ? x[(size_t)(k0 - t) * m] : 0.0;
#pragma unroll
    for (int t = 0; t < CH; ++t) {
      const int k = k0 - t;
      if (k >= 0) {
        const double z = (bb[t] - du[k] * z1 - du2[k] * z2) * rp[k];
        bb[t] = z;
        z2 = z1;
        z1 = z;
      }
    }
#pragma unroll
    for (int t = 0; t < CH; ++t)
      if (k0 - t >= 0) x[(size_t)(k0 - t) * m] = bb[t];
  }
}

// Block (g, job): the g-th cluster of more than kBigCluster columns of the
// job, if there is one.
//  1. Blocked Gram-Schmidt (two passes) of its inverse-iteration vectors.
//     These come out nearly parallel (every shift lies inside the cluster),
//     so the remainders are small and their rounding, which has components
//     outside the cluster's invariant subspace, is magnified by the
//     normalisation.
//  2. One inverse-iteration step with a single shift sigma just outside the
//     cluster (at c = min(kFilterRel |lam|max, gap / 2) from its edge, on the
//     side of the larger known gap): the cluster's directions are amplified
//     by 1/c to within a factor (c + width) / c of each other, a direction
//     at distance D by 1/D, so the magnified rounding shrinks by c / D while
//     the block stays well conditioned.
//  3. Blocked Gram-Schmidt again; its remainders are no longer small.
__global__ __launch_bounds__(kBcgsThreads) void cluster_bcgs_kernel(SmallBatch sb, double rtol) {
  __shared__ double lds[kBcgsLds > kFilterLds ? kBcgsLds : kFilterLds];
  __shared__ int cl[2];
  __shared__ double red[kBcgsThreads / 64];
  const SmallJob& J = sb.j[blockIdx.y];
  const int n = J.n, kw = J.kwant, tid = threadIdx.x;
  find_big_cluster(J.lam, kw, rtol, blockIdx.x, lds, cl);
  const int j0 = cl[0], m = cl[1];
  if (j0 < 0) return;
  c128* Z = J.E;
  double* Zr = J.zr + (size_t)n * j0;
  double* Zc = J.zc + (size_t)n * j0;
  double* Wb = J.wb + (size_t)kPan * j0;
  for (long long q = tid; q < (long long)n * m; q += kBcgsThreads) {
    const long long i = q / m, c = q % m;
    Zr[q] = Z[i * kw + j0 + c].re;
  }
  __syncthreads();
  rows_to_cols(Zr, n, m, Zc, lds);
  bcgs_all(Zr, Zc, n, m, Wb, lds);
  // 2. the shift
  const double* lam = J.lam;
  const double lmax = fmax(fabs(lam[0]), fabs(lam[kw - 1]));
  double tn = 0;
  for (int i = tid; i < n; i += kBcgsThreads)
    tn = fmax(tn, fabs(J.d[i]) + (i > 0 ? fabs(J.e[i - 1]) : 0.0) + (i < n - 1 ? fabs(J.e[i]) : 0.0));
  tn = wave_max(tn);
  if ((tid & 63) == 0) red[tid >> 6] = tn;
  __syncthreads();
  tn = 0;
  for (int w = 0; w < kBcgsThreads / 64; ++w) tn = fmax(tn, red[w]);
  if (lmax > 0) {
    const double inf = HUGE_VAL;
    const double gap_up = j0 > 0 ? lam[j0 - 1] - lam[j0] : inf;
    // below the wanted eigenvalues the next one is unknown unless all are wanted
    const double gap_dn = j0 + m < kw ? lam[j0 + m - 1] - lam[j0 + m] : (kw == n ? inf : 0.0);
    const bool up = gap_up >= gap_dn;
    const double c = fmin(kFilterRel * lmax, 0.5 * (up ? gap_up : gap_dn));
    const double sigma = up ? lam[j0] + c : lam[j0 + m - 1] - c;
    double* dl = lds;
    double* rp = lds + n;
    double* du = lds + 2 * (size_t)n;
    double* du2 = lds + 3 * (size_t)n;
    unsigned char* sw = (unsigned char*)(lds + 4 * (size_t)n);
    if (tid == 0) tri_lu(J.d, J.e, n, sigma, fmax(tn, 1e-300) * 2.2e-16, dl, rp, du, du2, sw);
    __syncthreads();
    for (int c0 = tid; c0 < m; c0 += kBcgsThreads) tri_solve_col(Zr, n, m, c0, dl, rp, du, du2, sw);
    __syncthreads();
    // 3.
    rows_to_cols(Zr, n, m, Zc, lds);
    bcgs_all(Zr, Zc, n, m, Wb, lds);
  }
  for (long long q = tid; q < (long long)n * m; q += kBcgsThreads) {
    const long long i = q / m, c = q % m;
    Z[i * kw + j0 + c].re = Zr[q];
  }
}

// Adaptive Newton-Schulz steps.  live[0]: live size of the next Z^H Z
// (kwant, or 0 once stopped); live[1]: live rows of this step's update (n, or
// 0 when it is skipped); live[2..3]: bits of max |Z^H Z - 1| of this step
// (non-negative doubles order as their bit patterns); live[4]: stopped;
// live[5]: n.  Every kernel of a step that Z^H Z feeds returns at once when
// live[0] is 0, so a finished job costs only its share of the launches.  The
// small kernels of a step take all jobs of the batch in one launch.
struct NsEntry {
  c128* G;          // Z^H Z (k x k)
  const c128* src;  // operand copy of the update: E ...
  c128* dst;        // ... into this buffer (tot elements)
  long long tot;
  int* live;
  int n, k;
  int flag;         // init: -; fix: form the max; decide: optional step
};
constexpr int kMaxNsJobs = 32;
struct NsBatch {
  int n;
  NsEntry e[kMaxNsJobs];
};

__global__ void ns_init_kernel(NsBatch b) {
  const NsEntry& e = b.e[blockIdx.x];
  e.live[0] = e.k;
  e.live[1] = e.n;
  e.live[4] = 0;
  e.live[5] = e.n;
}

// Z^H Z - 1 from the upper triangle the Hermitian product forms: the lower
// triangle filled by conjugation (32 x 32 blocks read transposed through
// LDS), 1 subtracted on the diagonal, and, with flag, max |Z^H Z - 1| over
// the upper triangle into live[2..3].  Nothing while the step is off.
// blockIdx.z: job.
__global__ __launch_bounds__(256) void ns_gram_fix_kernel(NsBatch b) {
  const NsEntry& e = b.e[blockIdx.z];
  const int k = e.k, bi = blockIdx.y, bj = blockIdx.x;   // destination block (bi >= bj)
  if (bj > bi || bi * 32 >= k || e.live[0] == 0) return;
  __shared__ c128 tile[32][33];
  c128* G = e.G;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  double mx = 0;
  for (int r = ty; r < 32; r += 8) {   // source block (bj, bi): rows bj*32 + r
    const int i = bj * 32 + r, j = bi * 32 + tx;
    if (i < k && j < k) {
      c128 v = G[(long long)i * k + j];
      if (i == j) v.re -= 1.0;
      tile[r][tx] = v;
      if (i <= j) mx = fmax(mx, fmax(fabs(v.re), fabs(v.im)));
    }
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int i = bi * 32 + r, j = bj * 32 + tx;
    if (i < k && j < k && i >= j) {
      const c128 v = tile[tx][r];
      G[(long long)i * k + j] = i == j ? v : cconj(v);
    }
  }
  if (e.flag) {
    mx = wave_max(mx);
    if ((threadIdx.x & 63) == 0)
      atomicMax((unsigned long long*)(e.live + 2), (unsigned long long)__double_as_longlong(mx));
  }
}

// From this step's max |Z^H Z - 1| (measured before its update, which squares
// it): skip the update of an optional step (flag) already orthonormal to
// tol_skip; stop all later steps once the error is below tol_stop (the update
// then leaves about tol_stop^2).  blockIdx.x: job.
__global__ void ns_decide_kernel(NsBatch b, double tol_skip, double tol_stop) {
  int* live = b.e[blockIdx.x].live;
  const double mx = __longlong_as_double((long long)*(unsigned long long*)(live + 2));
  const bool stopped = live[4] != 0;
  live[1] = (stopped || (b.e[blockIdx.x].flag && !(mx >= tol_skip))) ? 0 : live[5];
  if (!(mx >= tol_stop)) {
    live[4] = 1;
    live[0] = 0;
  }
  *(unsigned long long*)(live + 2) = 0ull;
}

// The operand copy of the update, unless the update is skipped.  blockIdx.y:
// job.
__global__ void ns_copy_kernel(NsBatch b) {
  const NsEntry& e = b.e[blockIdx.y];
  if (e.live[1] == 0) return;
  for (long long i = blockIdx.x * 256ll + threadIdx.x; i < e.tot; i += (long long)gridDim.x * 256) e.dst[i] = e.src[i];
}

// launch(batch) for the entries, in groups of kMaxNsJobs.
template <typename Launch>
int ns_launch(const std::vector<NsEntry>& es, Launch&& launch) {
  for (size_t i0 = 0; i0 < es.size(); i0 += kMaxNsJobs) {
    NsBatch b{};
    for (size_t i = i0; i < es.size() && b.n < kMaxNsJobs; ++i) b.e[b.n++] = es[i];
    launch(b);
    QT_HIP_CHECK(hipGetLastError());
  }
  return 0;
}

__global__ void eig1_kernel(const c128* G, double* lam, c128* E) {
  lam[0] = G[0].re;
  E[0] = mk<double>(1, 0);
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Rows per block: the tuned count (8 or 16), as LDS allows.
int tri_rows_loc(int n) {
  const int rl = (int)(kTriLds / (16 * (size_t)n));
  const int want = std::max(1, std::min(kTriRows, tune_params().tri_rows));
  return std::max(1, std::min(std::min(n, want), rl));
}

}  // namespace

size_t eig_work_bytes(int n) {
  size_t b = 0;
  b += 3 * align256((size_t)n * 16);                 // d, e, tau
  b += align256(4 * (size_t)n * n * 8);              // lu
  b += align256((size_t)n * n);                      // swap flags
  b += align256(grid_sync_words(256) * 4);
  b += align256((2 * 257 + 4 * (size_t)n) * 16);     // red + pbuf + rowbuf
  b += align256(qr_work_bytes(std::max(n - 1, 1), std::max(n - 1, 1), 16, n));
  b += 2 * align256((size_t)n * n * 16);
  b += align256((size_t)((n - 1 + NB - 1) / NB + 1) * kLarftParts * NB * NB * 16);
  b += 256;   // ns_live
  return b;
}

EigWork eig_work_carve(void* base, int n, int* status) {
  char* p = (char*)base;
  EigWork w{};
  w.d = (double*)p; p += align256((size_t)n * 16);
  w.e = (double*)p; p += align256((size_t)n * 16);
  w.tau = (c128*)p; p += align256((size_t)n * 16);
  w.lu = (double*)p; p += align256(4 * (size_t)n * n * 8);
  p += align256((size_t)n * n);  // swap flags follow lu (see eig_herm_top)
  w.sync = (unsigned*)p; p += align256(grid_sync_words(256) * 4);
  w.red = (c128*)p; p += align256((2 * 257 + 4 * (size_t)n) * 16);
  w.qtri = qr_work_carve(p, std::max(n - 1, 1), std::max(n - 1, 1), 16, n, status);
  p += align256(qr_work_bytes(std::max(n - 1, 1), std::max(n - 1, 1), 16, n));
  w.gz = (c128*)p; p += align256((size_t)n * n * 16);
  w.ztmp = (c128*)p; p += align256((size_t)n * n * 16);
  w.tpart = (c128*)p; p += align256((size_t)((n - 1 + NB - 1) / NB + 1) * kLarftParts * NB * NB * 16);
  w.ns_live = (int*)p; p += 256;
  w.status = status;
  return w;
}

int eig_herm_top_batch(const EigJob* jobs, int njobs, hipStream_t s) {
  int rc;
  static bool attr = false;
  if (!attr) {
    QT_HIP_CHECK(hipFuncSetAttribute((const void*)tridiag_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)kTriLds));
    QT_HIP_CHECK(hipFuncSetAttribute((const void*)invit_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)kInvitLds));
    attr = true;
  }
  // validation, 1 x 1 problems, barrier words and reflector buffers
  std::vector<int> big;
  std::vector<ZeroSpan> zs;
  for (int j = 0; j < njobs; ++j) {
    const EigJob& J = jobs[j];
    if (J.n < 1 || J.kwant < 1 || J.kwant > J.n) return set_error(-1, "eig: bad sizes n=%d kwant=%d", J.n, J.kwant);
    if (J.n > kEigMaxN) return set_error(-2, "eig: n=%d exceeds the supported %d", J.n, kEigMaxN);
    if (J.n == 1) {
      hipLaunchKernelGGL(eig1_kernel, dim3(1), dim3(1), 0, s, J.G, J.lam, J.E);
      QT_HIP_CHECK(hipGetLastError());
      continue;
    }
    const int RL = tri_rows_loc(J.n), P = (J.n + RL - 1) / RL;
    if (P > 256) return set_error(-2, "eig: n=%d needs %d blocks", J.n, P);
    // cleared before the tridiagonalisation: its barrier words, the Newton-
    // Schulz error word, and the reflector entries it does not write that
    // later products read: the top 32 rows of every odd panel of a pair
    // block, and the whole last pair block (its last panel may be partial)
    zs.push_back(ZeroSpan{J.w->sync, (long long)grid_sync_words(P) * 4, 0, 0, 1, 1});
    zs.push_back(ZeroSpan{J.w->ns_live + 2, 8, 0, 0, 1, 1});
    const int mqr = J.n - 1, npan = (mqr + NB - 1) / NB, npair = (npan + 1) / 2;
    const long long pair_bytes = (long long)mqr * kQrLdv * 16, row_bytes = (long long)kQrLdv * 16;
    char* V = (char*)J.w->qtri.V;
    if (npair > 1) zs.push_back(ZeroSpan{V + NB * 16, NB * 16, row_bytes, pair_bytes, NB, npair - 1});
    zs.push_back(ZeroSpan{V + (npair - 1) * pair_bytes, row_bytes, row_bytes, 0, mqr - 2 * NB * (npair - 1), 1});
    big.push_back(j);
  }
  if (big.empty()) return 0;
  if ((rc = zero_spans(zs.data(), (int)zs.size(), s))) return rc;
  // 1. tridiagonalisations, packed into cooperative launches of <= 256 blocks
  {
    TriBatch tb{};
    int used = 0;
    size_t shmem = 0;
    auto flush = [&]() -> int {
      if (tb.nprob == 0) return 0;
      if (stream_capturing(s)) {
        hipLaunchKernelGGL(tridiag_kernel, dim3(used), dim3(kTriThreads), shmem, s, tb);
        QT_HIP_CHECK(hipGetLastError());
      } else {
        void* args[] = {(void*)&tb};
        QT_HIP_CHECK(hipLaunchCooperativeKernel((const void*)tridiag_kernel, dim3(used), dim3(kTriThreads), args,
                                                (unsigned)shmem, s));
      }
      tb = TriBatch{};
      used = 0;
      shmem = 0;
      return 0;
    };
    for (int j : big) {
      const EigJob& J = jobs[j];
      const int RL = tri_rows_loc(J.n), P = (J.n + RL - 1) / RL;
      if (used + P > 256 || tb.nprob == kMaxTriProbs)
        if ((rc = flush())) return rc;
      TriProb& t = tb.p[tb.nprob++];
      tb.status = J.w->status;
      t.G = J.G;
      t.n = J.n;
      t.rows_loc = RL;
      t.nblk = P;
      t.blk0 = used;
      t.d = J.w->d;
      t.e = J.w->e;
      t.tau = J.w->tau;
      t.V = (c128*)J.w->qtri.V;
      t.red = J.w->red;
      t.pbuf = J.w->red + 2 * 257;
      t.rowbuf = t.pbuf + 2 * (size_t)J.n;
      t.sync = J.w->sync;
      used += P;
      shmem = std::max(shmem, (size_t)RL * J.n * sizeof(c128));
    }
    if ((rc = flush())) return rc;
  }
  // 2-5. larft, bisection, inverse iteration, clustered MGS (batched small kernels)
  std::vector<GemmProb> gram;
  for (size_t j0 = 0; j0 < big.size(); j0 += kMaxSmallJobs) {
    SmallBatch sb{};
    int maxn = 0, maxk = 0;
    for (size_t q = j0; q < std::min(big.size(), j0 + kMaxSmallJobs); ++q) {
      const EigJob& J = jobs[big[q]];
      SmallJob& S = sb.j[sb.njobs++];
      S.d = J.w->d;
      S.e = J.w->e;
      S.lam = J.lam;
      S.lu = J.w->lu;
      S.swp = (unsigned char*)((char*)J.w->lu + align256(4 * (size_t)J.n * J.n * 8));
      S.E = J.E;
      S.V = (c128*)J.w->qtri.V;
      S.T = J.w->qtri.T;
      S.tau = J.w->tau;
      S.tpart = J.w->tpart;
      S.zr = (double*)J.w->gz;
      S.zc = (double*)J.w->ztmp;
      S.wb = J.w->lu;
      S.n = J.n;
      S.kwant = J.kwant;
      maxn = std::max(maxn, J.n);
      maxk = std::max(maxk, J.kwant);
      // V_p^H V_p for every panel p of the reflectors (FP64 matrix cores,
      // split-K partials left for larft_kernel; one part writes them directly)
      const int m = J.n - 1;
      for (int p0 = 0; p0 < m; p0 += NB) {
        const int p = p0 / NB, mp = m - p0;
        const c128* Vp = (const c128*)J.w->qtri.V + qr_v_offset(p, m);
        c128* out = J.w->tpart + (size_t)p * kLarftParts * NB * NB;
        GemmProb q = gemm_prob(Vp, kQrLdv, OP_C, Vp, kQrLdv, OP_N, out, NB, NB, NB, mp);
        q.ksplit = larft_parts(mp);
        q.work = out;
        q.skip_reduce = 1;
        gram.push_back(q);
      }
    }
    if (!gram.empty() && (rc = gemm_run(gram.data(), (int)gram.size(), GemmTypes{DT_C128, DT_C128}, s))) return rc;
    gram.clear();
    const int npan = (maxn - 1 + NB - 1) / NB;
    hipLaunchKernelGGL(larft_kernel, dim3(npan, sb.njobs), dim3(256), 0, s, sb);
    QT_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(bisect_kernel, dim3((maxk + 3) / 4, sb.njobs), dim3(256), 0, s, sb);
    QT_HIP_CHECK(hipGetLastError());
    const int ig = invit_group(maxn);
    hipLaunchKernelGGL(invit_kernel, dim3((maxk + ig - 1) / ig, sb.njobs), dim3(64), invit_lds_bytes(maxn, ig), s, sb,
                       ig);
    QT_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(cluster_mgs_kernel, dim3(maxk, sb.njobs), dim3(256), 0, s, sb, kClusterRtol);
    QT_HIP_CHECK(hipGetLastError());
    if (maxk > kBigCluster) {
      hipLaunchKernelGGL(cluster_bcgs_kernel, dim3(maxk / (kBigCluster + 1), sb.njobs), dim3(kBcgsThreads), 0, s, sb,
                         kClusterRtol);
      QT_HIP_CHECK(hipGetLastError());
    }
  }
  // 6. Newton-Schulz steps Z <- Z - Z (Z^H Z - 1)/2 (each squares the
  // orthogonality error of Z), grouped over the jobs: the job's ns_steps
  // always, then further ones (up to kNsMaxSteps) until max |Z^H Z - 1| before
  // a step is below 1e-7 (that step leaves ~1e-14), decided on the device: a
  // finished job's products run with live size 0 and its other kernels return
  // at once.  Vectors of eigenvalues closer than the cluster tolerance were
  // orthogonalised by Gram-Schmidt above; the rest overlap by at most about
  // u / rtol, which these steps remove.
  const GemmTypes ty{DT_C128, DT_C128};
  std::vector<GemmProb> gs;
  std::vector<NsEntry> ne;
  auto entry = [&](const EigJob& J, int flag) {
    return NsEntry{J.w->gz, J.E, J.w->ztmp, (long long)J.n * J.kwant, J.w->ns_live, J.n, J.kwant, flag};
  };
  for (int j : big) ne.push_back(entry(jobs[j], 0));
  if ((rc = ns_launch(ne, [&](const NsBatch& b) { hipLaunchKernelGGL(ns_init_kernel, dim3(b.n), dim3(1), 0, s, b); })))
    return rc;
  for (int it = 0; it < kNsMaxSteps; ++it) {
    std::vector<int> ns;
    for (int j : big)
      if (jobs[j].ns_steps > 0) ns.push_back(j);
    if (ns.empty()) break;
    gs.clear();
    for (int j : ns) {
      const EigJob& J = jobs[j];
      const bool gated = it >= J.ns_steps;
      // the inverse-iteration factors are dead: their buffer holds split-K partials
      GemmProb g1 = gemm_prob(J.E, J.kwant, OP_C, J.E, J.kwant, OP_N, J.w->gz, J.kwant, J.kwant, J.kwant, J.n);
      g1.ksplit = splitk_auto(J.kwant, J.kwant, J.n, 4 * (size_t)J.n * J.n * 8, sizeof(c128), true);
      g1.work = J.w->lu;
      g1.herm = 1;
      if (gated) g1.dM = g1.dN = J.w->ns_live;
      gs.push_back(g1);
    }
    if ((rc = gemm_run(gs.data(), (int)gs.size(), ty, s))) return rc;
    // fill and shift of Z^H Z (with its max from the last fixed step on), the
    // decision on the optional steps, and the operand copies, each one launch
    std::vector<NsEntry> fix, dec, cpy;
    int maxnb = 0;
    long long maxtot = 0;
    gs.clear();
    for (int j : ns) {
      const EigJob& J = jobs[j];
      const bool gated = it >= J.ns_steps;
      const bool decide = it + 1 >= J.ns_steps;   // from the last fixed step on: decide the optional ones
      fix.push_back(entry(J, decide ? 1 : 0));
      maxnb = std::max(maxnb, (J.kwant + 31) / 32);
      if (decide) dec.push_back(entry(J, gated ? 1 : 0));
      GemmProb g2 = gemm_prob(J.E, J.kwant, OP_N, J.w->gz, J.kwant, OP_N, J.E, J.kwant, J.n, J.kwant, J.kwant,
                              -0.5f, 1.f);
      g2.ksplit = splitk_auto(J.n, J.kwant, J.kwant, 4 * (size_t)J.n * J.n * 8, sizeof(c128));
      g2.work = J.w->lu;
      if (g2.ksplit <= 1) {
        // one pass writes E while other tiles of its rows still read it: the
        // left operand is a copy (split K writes only the partials, and the
        // reduction after the product is the one that updates E)
        cpy.push_back(entry(J, 0));
        maxtot = std::max(maxtot, (long long)J.n * J.kwant);
        g2.A = J.w->ztmp;
      }
      if (gated) g2.dM = J.w->ns_live + 1;
      gs.push_back(g2);
    }
    if ((rc = ns_launch(fix, [&](const NsBatch& b) {
           hipLaunchKernelGGL(ns_gram_fix_kernel, dim3(maxnb, maxnb, b.n), dim3(256), 0, s, b);
         })))
      return rc;
    if ((rc = ns_launch(dec, [&](const NsBatch& b) {
           hipLaunchKernelGGL(ns_decide_kernel, dim3(b.n), dim3(1), 0, s, b, 1e-13, 1e-7);
         })))
      return rc;
    const int cgrid = (int)std::min<long long>(2048, (maxtot + 255) / 256);
    if ((rc = ns_launch(cpy, [&](const NsBatch& b) {
           hipLaunchKernelGGL(ns_copy_kernel, dim3(cgrid, b.n), dim3(256), 0, s, b);
         })))
      return rc;
    if ((rc = gemm_run(gs.data(), (int)gs.size(), ty, s))) return rc;
  }
  // 7. back-transformation E = Q Z (rows 1.. of each E)
  std::vector<QrJob> qj;
  for (int j : big) {
    const EigJob& J = jobs[j];
    qj.push_back(QrJob{nullptr, 0, J.n - 1, J.n - 1, J.E + J.kwant, J.kwant, J.kwant, &J.w->qtri});
  }
  return qr_apply_q_batch(qj.data(), (int)qj.size(), DT_C128, s);
}

int eig_herm_top(c128* G, int n, int kwant, double* lam, c128* E, const EigWork& w, hipStream_t s) {
  EigJob J{G, n, kwant, lam, E, &w};
  return eig_herm_top_batch(&J, 1, s);
}

}  // namespace qrtebd
