// FP64 Hermitian eigensolver for step (iv) of controlled bond expansion
// (Sec. III): L^dag L = V^dag S^2 V.
//
//  1. Householder tridiagonalisation A = Q T Q^H (LAPACK zhetd2 conventions,
//     lower form) in one cooperative kernel.  The matrix rows live in LDS,
//     dealt cyclically to the blocks; the reflector vector, the trailing
//     row and the rank-2 update vector live in registers (column j of a
//     vector belongs to thread j mod 256).  Step k needs one grid barrier:
//     each block publishes its slice of p = tau A v and its part of p^H v,
//     and the current row k+1; after the barrier every block rebuilds row k+1
//     itself and derives the next reflector without further communication.
//     T is real symmetric because every off-diagonal beta is real.
//  2. The wanted (largest) eigenvalues of T by Sturm-count bisection, one
//     thread per eigenvalue.
//  3. Their eigenvectors by inverse iteration on T (tridiagonal LU with
//     partial pivoting, three solves from a fixed pseudo-random start), one
//     thread per vector.
//  4. Re-orthogonalisation: modified Gram-Schmidt (two passes) inside each
//     cluster of eigenvalues closer than 1e-9 |T| (where independent inverse
//     iterations can return nearly parallel vectors), then two Newton-Schulz
//     steps Z <- Z - Z (Z^H Z - 1)/2 on the MFMA GEMM.  Mixing two vectors by
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
constexpr int QMAX = 8;            // register slots per thread: n <= 2048
constexpr int kMaxN = 256 * QMAX;
constexpr size_t kTriLds = 150 * 1024;

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

// Fixed-order block sum of a complex value (every thread gets the result).
__device__ inline c128 block_sum_c(c128 v, c128* scr) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v.re = wave_sum(v.re);
  v.im = wave_sum(v.im);
  __syncthreads();
  if (lane == 0) scr[wid] = v;
  __syncthreads();
  c128 s = z0();
  for (int w = 0; w < nw; ++w) s = cadd(s, scr[w]);
  return s;
}

__global__ __launch_bounds__(256) void tridiag_kernel(TriBatch batch) {
  extern __shared__ c128 rows[];  // rows_loc x n, local row r = global row blk + r * P
  __shared__ double scratch[8];
  __shared__ c128 cscr[8];
  __shared__ c128 wred[4][16];
  __shared__ c128 vloc[16], wloc[16];
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
      for (int j = tid; j < n; j += 256) rows[r * n + j] = a.G[(long long)gi * n + j];
  }
  c128 rk[QMAX], v[QMAX], w[QMAX];
#pragma unroll
  for (int q = 0; q < QMAX; ++q) {
    const int j = tid + 256 * q;
    rk[q] = j < n ? a.G[j] : z0();
    v[q] = z0();
    w[q] = z0();
  }
  if (tid == 0) flag = 0;
  __syncthreads();
  // row k+1 is published by its owner's wave 0 as soon as it is final for
  // step k (here for k = 0), long before step k's barrier
  if (n > 1 && 1 % P == blk) {
    const int r = 1 / P;
    for (int j = tid; j < n; j += 256) pub_store(a.rowbuf + j, rows[r * n + j]);
  }

  for (int k = 0; k < n - 1; ++k) {
    const int slot = k & 1;
    // ---- reflector from column k below the diagonal = conj(row k right of it);
    // every thread derives tau, beta, scale itself from the block sums
    double xn2 = 0;
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
      const int j = tid + 256 * q;
      if (j >= k + 2 && j < n) xn2 += cabs2(rk[q]);
      if (j == k + 1) scal[0] = cconj(rk[q]);
      if (j == k) scal[1] = rk[q];
    }
    xn2 = block_sum(xn2, scratch);  // its barriers also publish scal[0], scal[1]
    const c128 alpha = scal[0];
    c128 tau = z0(), scale = z0();
    double beta = alpha.re;
    if (!(xn2 == 0.0 && alpha.im == 0.0)) {
      beta = -copysign(sqrt(alpha.re * alpha.re + alpha.im * alpha.im + xn2), alpha.re);
      tau = mk<double>((beta - alpha.re) / beta, -alpha.im / beta);
      const c128 den = mk<double>(alpha.re - beta, alpha.im);
      const double dd = cabs2(den);
      scale = mk<double>(den.re / dd, -den.im / dd);
    }
    if (blk == 0 && tid == 0) {
      a.d[k] = scal[1].re;
      a.e[k] = beta;
      a.tau[k] = tau;
      if (!isfinite(beta) || !isfinite(scal[1].re)) latch_error(batch.status, ERRBIT_NONFINITE);
    }
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
      const int j = tid + 256 * q;
      v[q] = j == k + 1 ? mk<double>(1, 0) : (j > k + 1 && j < n ? cmul(cconj(rk[q]), scale) : z0());
    }
    // v_i of this block's rows, for the rank-2 update
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
      const int j = tid + 256 * q;
      if (j < n && j % P == blk) vloc[j / P] = v[q];
    }
    // reflector k into the QR-compatible layout (subproblem row i <-> row i+1):
    // each block writes the rows it owns; read only by later kernels
    {
      const int p = k / NB, c = k % NB, j0 = p * NB;
      c128* Vp = a.V + (size_t)p * mqr * NB;
#pragma unroll
      for (int q = 0; q < QMAX; ++q) {
        const int g = tid + 256 * q;  // global row
        if (g >= j0 + 1 && g < n && g % P == blk) Vp[(long long)(g - 1 - j0) * NB + c] = g >= k + 1 ? v[q] : z0();
      }
    }
    // ---- p_i = tau sum_{j>k} A[i][j] v_j for own rows i > k
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      if (r < RL) {
        const int gi = blk + r * P;
        c128 sacc = z0();
        if (gi > k && gi < n) {
#pragma unroll
          for (int q = 0; q < QMAX; ++q) {
            const int j = tid + 256 * q;
            if (j > k && j < n) sacc = cadd(sacc, cmul(rows[r * n + j], v[q]));
          }
        }
        const double sr = wave_sum(sacc.re), si = wave_sum(sacc.im);
        if (lane == 0) wred[wid][r] = mk<double>(sr, si);
      }
    }
    __syncthreads();
    if (wid == 0) {
      // wave 0 publishes p for its rows, this block's part of p^H v, and the
      // current row k+1 if it owns it
      c128 part = z0();
      if (lane < RL) {
        const int r = lane, gi = blk + r * P;
        c128 sacc = z0();
        for (int ww = 0; ww < 4; ++ww) sacc = cadd(sacc, wred[ww][r]);
        if (gi > k && gi < n) {
          const c128 pi = cmul(tau, sacc);
          pub_store(a.pbuf + (long long)slot * n + gi, pi);
          part = cmulc(pi, vloc[r]);
        }
      }
      part.re = wave_sum(part.re);
      part.im = wave_sum(part.im);
      if (lane == 0) pub_store(a.red + (long long)slot * P + blk, part);
    }
    if (!grid_barrier(gs, (unsigned)(k + 1), blk, P, &flag)) return;
    // ---- one round of loads: block partials, p, and row k+1 as published
    const c128 rv = tid < P ? pub_load(a.red + (long long)slot * P + tid) : z0();
    c128 pv[QMAX], xb[QMAX];
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
      const int j = tid + 256 * q;
      pv[q] = (j > k && j < n) ? pub_load(a.pbuf + (long long)slot * n + j) : z0();
      xb[q] = j < n ? pub_load(a.rowbuf + (long long)slot * n + j) : z0();
    }
    const c128 ptv = block_sum_c(rv, cscr);   // p^H v
    const c128 alpha2 = cscale(cmul(tau, ptv), -0.5);
    // ---- w = p + alpha2 v
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
      const int j = tid + 256 * q;
      w[q] = (j > k && j < n) ? cadd(pv[q], cmul(alpha2, v[q])) : z0();
      if (j == k + 1) scal[2] = w[q];
      if (j < n && j % P == blk) wloc[j / P] = w[q];
    }
    __syncthreads();
    // row k+1 (as published before the update) gets the rank-2 update
    const c128 wk1 = scal[2];
#pragma unroll
    for (int q = 0; q < QMAX; ++q) {
      const int j = tid + 256 * q;
      if (j < n) rk[q] = j > k ? rank2_sub(xb[q], mk<double>(1, 0), w[q], wk1, v[q]) : xb[q];
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      if (r < RL) {
        const int gi = blk + r * P;
        if (gi > k && gi < n) {
          const c128 vi = vloc[r], wi = wloc[r];
#pragma unroll
          for (int q = 0; q < QMAX; ++q) {
            const int j = tid + 256 * q;
            if (j > k && j < n) rows[r * n + j] = rank2_sub(rows[r * n + j], vi, w[q], wi, v[q]);
          }
        }
      }
    }
    __syncthreads();
    // publish row k+2 (final for step k+1) into the other slot
    if (k + 2 < n && (k + 2) % P == blk) {
      const int r = (k + 2) / P;
      for (int j = tid; j < n; j += 256) pub_store(a.rowbuf + (long long)((k + 1) & 1) * n + j, rows[r * n + j]);
    }
  }
  // d[n-1] from the thread holding column n-1 of the final row
  if (blk == 0) {
#pragma unroll
    for (int q = 0; q < QMAX; ++q)
      if (tid + 256 * q == n - 1) {
        a.d[n - 1] = rk[q].re;
        a.e[n - 1] = 0.0;
        a.tau[n - 1] = z0();
      }
  }
}

// Number of eigenvalues of the tridiagonal (d, e^2 in LDS) below x (Sturm sequence).
__device__ inline int sturm_count(const double* d, const double* e2, int n, double x, double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += q < 0;
  for (int i = 1; i < n; ++i) {
    q = d[i] - x - e2[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0;
  }
  return cnt;
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

// lam[j] = (j+1)-th largest eigenvalue, j < kwant.  Multisection: the 8 lanes
// of a group evaluate 8 interior points of the eigenvalue's interval per
// round, shrinking it 9-fold; 22 rounds reach full FP64 resolution.
struct SmallJob {
  const double* d;
  const double* e;
  double* lam;
  double* lu;
  unsigned char* swp;
  c128* E;
  c128* V;
  c128* VT;
  c128* T;
  const c128* tau;
  int n, kwant;
};
constexpr int kMaxSmallJobs = 24;
struct SmallBatch {
  int njobs;
  SmallJob j[kMaxSmallJobs];
};

__global__ __launch_bounds__(256) void bisect_kernel(SmallBatch sb) {
  const SmallJob& J = sb.j[blockIdx.y];
  const double* d = J.d;
  const double* e = J.e;
  const int n = J.n, kwant = J.kwant;
  double* lam = J.lam;
  if ((int)blockIdx.x * 32 >= kwant) return;
  __shared__ double sd[kMaxN], se2[kMaxN];
  __shared__ double scr[12];
  for (int i = threadIdx.x; i < n; i += 256) {
    sd[i] = d[i];
    se2[i] = i < n - 1 ? e[i] * e[i] : 0.0;
  }
  __syncthreads();
  double lo, hi, pivmin;
  gersh(sd, se2, n, scr, lo, hi, pivmin);
  const int lane = threadIdx.x & 63, sub = lane & 7, gbase = lane & ~7;
  const int j = blockIdx.x * 32 + (threadIdx.x >> 3);
  const int idx = n - 1 - min(j, kwant - 1);  // ascending index
  double a = lo, b = hi;
  for (int it = 0; it < 22; ++it) {
    const double x = a + (b - a) * (double)(sub + 1) * (1.0 / 9.0);
    const int c = sturm_count(sd, se2, n, x, pivmin);
    const unsigned long long m = __ballot(c > idx);
    const unsigned bits = (unsigned)((m >> gbase) & 0xffull);
    const int f = bits ? __ffs(bits) - 1 : 8;
    const double xb = __shfl(x, gbase + min(f, 7), 64);
    const double xa = __shfl(x, gbase + max(f - 1, 0), 64);
    const double na = f == 0 ? a : xa;
    const double nb = f == 8 ? b : xb;
    a = na;
    b = nb;
  }
  if (j < kwant && sub == 0) lam[j] = 0.5 * (a + b);
}

__device__ inline double hash_uniform(unsigned long long x) {
  x += 0x9e3779b97f4a7c15ULL;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ULL;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebULL;
  x ^= x >> 31;
  return (double)(x >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// Inverse iteration for eigenvalue lam[j]: E[:, j] (real, stored complex).
// lu: [4][n][kwant] (pivot row entries u0, u1, u2 and the multiplier),
// swp: [n][kwant] row-interchange flags; T = (d, e) staged in LDS.
__global__ __launch_bounds__(64) void invit_kernel(SmallBatch sb) {
  const SmallJob& J = sb.j[blockIdx.y];
  const double* d = J.d;
  const double* e = J.e;
  const int n = J.n, kwant = J.kwant;
  const double* lam = J.lam;
  double* lu = J.lu;
  unsigned char* swp = J.swp;
  c128* E = J.E;
  if ((int)blockIdx.x * 64 >= kwant) return;
  __shared__ double sd[kMaxN], se[kMaxN];
  for (int i = threadIdx.x; i < n; i += 64) {
    sd[i] = d[i];
    se[i] = i < n - 1 ? e[i] : 0.0;
  }
  __syncthreads();
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= kwant) return;
  const double l = lam[j];
  double tnorm = 0;
  for (int i = 0; i < n; ++i) tnorm = fmax(tnorm, fabs(sd[i]) + (i > 0 ? fabs(se[i - 1]) : 0.0) + fabs(se[i]));
  const double tiny = fmax(tnorm, 1e-300) * 2.2e-16;
  double* U0 = lu;
  double* U1 = lu + (size_t)n * kwant;
  double* U2 = lu + 2 * (size_t)n * kwant;
  double* ML = lu + 3 * (size_t)n * kwant;
  auto at = [&](int i) { return (size_t)i * kwant + j; };
  // factor T - l I with partial pivoting
  double c0 = sd[0] - l, c1 = n > 1 ? se[0] : 0.0, c2 = 0.0;
  for (int k = 0; k < n - 1; ++k) {
    const double n0 = se[k], n1 = sd[k + 1] - l, n2 = se[k + 1];
    double u0, u1, u2, m;
    unsigned char sw;
    if (fabs(c0) >= fabs(n0)) {
      m = c0 != 0.0 ? n0 / c0 : 0.0;
      u0 = c0; u1 = c1; u2 = c2; sw = 0;
      c0 = n1 - m * c1; c1 = n2 - m * c2; c2 = 0.0;
    } else {
      m = c0 / n0;
      u0 = n0; u1 = n1; u2 = n2; sw = 1;
      c0 = c1 - m * n1; c1 = c2 - m * n2; c2 = 0.0;
    }
    if (u0 == 0.0) u0 = tiny;
    U0[at(k)] = u0; U1[at(k)] = u1; U2[at(k)] = u2; ML[at(k)] = m; swp[at(k)] = sw;
  }
  U0[at(n - 1)] = c0 == 0.0 ? tiny : c0;
  U1[at(n - 1)] = 0.0;
  U2[at(n - 1)] = 0.0;
  // start vector, stored in E's real parts
  for (int i = 0; i < n; ++i) E[at(i)] = mk<double>(hash_uniform(((unsigned long long)j << 32) ^ (unsigned)i), 0.0);
  double scale = 1.0;
  for (int it = 0; it < 2; ++it) {
    // forward: the row operations of the factorisation applied to b (scaled)
    double rc = E[at(0)].re * scale;
    for (int k = 0; k < n - 1; ++k) {
      const double bk1 = E[at(k + 1)].re * scale, m = ML[at(k)];
      if (swp[at(k)] == 0) {
        E[at(k)].re = rc;
        rc = bk1 - m * rc;
      } else {
        E[at(k)].re = bk1;
        rc = rc - m * bk1;
      }
    }
    E[at(n - 1)].re = rc;
    // back substitution; the max norm rescales the next pass
    double z1 = 0.0, z2 = 0.0, nrm = 0.0, s2 = 0.0;
    for (int i = n - 1; i >= 0; --i) {
      const double z = (E[at(i)].re - U1[at(i)] * z1 - U2[at(i)] * z2) / U0[at(i)];
      E[at(i)].re = z;
      z2 = z1;
      z1 = z;
      nrm = fmax(nrm, fabs(z));
    }
    scale = nrm > 0 ? 1.0 / nrm : 1.0;
    if (it == 1) {
      for (int i = 0; i < n; ++i) {
        const double z = E[at(i)].re * scale;
        s2 += z * z;
      }
      const double f = scale / sqrt(s2);
      for (int i = 0; i < n; ++i) E[at(i)].re *= f;
    }
  }
}

// T_p and V_p T_p for every panel of the tridiagonalisation reflectors;
// V_p is staged through LDS in 64-row slabs.
__global__ __launch_bounds__(256) void larft_kernel(SmallBatch sb) {
  __shared__ c128 slab[64][NB + 1];
  __shared__ c128 Tm[NB][NB + 1];
  const SmallJob& J = sb.j[blockIdx.y];
  c128* V = J.V;
  c128* VT = J.VT;
  c128* T = J.T;
  const c128* tau = J.tau;
  const int m = J.n - 1, nrefl = J.n - 1;
  const int p = blockIdx.x, tid = threadIdx.x;
  if (p * NB >= nrefl) return;
  const int j0 = p * NB, jb = min(NB, nrefl - j0), mp = m - j0;
  const c128* Vp = V + (size_t)p * m * NB;
  c128 g[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) g[q] = z0();
  for (int r0 = 0; r0 < mp; r0 += 64) {
    __syncthreads();
    for (int idx = tid; idx < 64 * NB; idx += 256) {
      const int i = idx / NB, c = idx % NB;
      slab[i][c] = (r0 + i < mp) ? Vp[(long long)(r0 + i) * NB + c] : z0();
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q, aa = e / NB, bb = e % NB;
      c128 s = g[q];
      for (int i = 0; i < 64; ++i) s = cadd(s, cmulc(slab[i][aa], slab[i][bb]));
      g[q] = s;
    }
  }
  __syncthreads();
  // G overwrites the slab storage (NB x NB <= 64 x (NB+1))
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
  c128* VTp = VT + (size_t)p * m * NB;
  for (int idx = tid; idx < mp * NB; idx += 256) {
    const int i = idx / NB, c = idx % NB;
    c128 sacc = z0();
    if (c < jb)
      for (int q = 0; q <= c; ++q) sacc = cadd(sacc, cmul(Vp[(long long)i * NB + q], Tm[q][c]));
    VTp[idx] = sacc;
  }
  for (int idx = tid; idx < NB * NB; idx += 256) T[(size_t)p * NB * NB + idx] = Tm[idx / NB][idx % NB];
}

// Two-pass modified Gram-Schmidt over each cluster of close eigenvalues
// (lam descending; a cluster starts where the gap to the previous value
// exceeds rtol * max|lam|).  Block b handles the cluster starting at column b, if any.
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
  while (e + 1 < kw && lam[e] - lam[e + 1] <= ctol) ++e;
  if (e == j) return;
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

// D = G - 1 on a k x k block (in place).
__global__ void sub_identity_kernel(c128* G, int k) {
  const long long tot = (long long)k * k;
  for (long long idx = blockIdx.x * 256ll + threadIdx.x; idx < tot; idx += (long long)gridDim.x * 256)
    if (idx / k == idx % k) G[idx].re -= 1.0;
}

__global__ void eig1_kernel(const c128* G, double* lam, c128* E) {
  lam[0] = G[0].re;
  E[0] = mk<double>(1, 0);
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

int tri_rows_loc(int n) {
  const int rl = (int)(kTriLds / (16 * (size_t)n));
  return std::max(1, std::min(std::min(n, 16), rl));
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
  w.status = status;
  return w;
}

int eig_herm_top_batch(const EigJob* jobs, int njobs, hipStream_t s) {
  int rc;
  static bool attr = false;
  if (!attr) {
    QT_HIP_CHECK(hipFuncSetAttribute((const void*)tridiag_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)kTriLds));
    attr = true;
  }
  // validation, 1 x 1 problems, barrier words and reflector buffers
  std::vector<int> big;
  for (int j = 0; j < njobs; ++j) {
    const EigJob& J = jobs[j];
    if (J.n < 1 || J.kwant < 1 || J.kwant > J.n) return set_error(-1, "eig: bad sizes n=%d kwant=%d", J.n, J.kwant);
    if (J.n > kMaxN) return set_error(-2, "eig: n=%d exceeds the supported %d", J.n, kMaxN);
    if (J.n == 1) {
      hipLaunchKernelGGL(eig1_kernel, dim3(1), dim3(1), 0, s, J.G, J.lam, J.E);
      QT_HIP_CHECK(hipGetLastError());
      continue;
    }
    const int RL = tri_rows_loc(J.n), P = (J.n + RL - 1) / RL;
    if (P > 256) return set_error(-2, "eig: n=%d needs %d blocks", J.n, P);
    if ((rc = fill_zero(J.w->sync, grid_sync_words(P) * 4, s))) return rc;
    const int mqr = J.n - 1, npan = (mqr + NB - 1) / NB;
    if ((rc = fill_zero(J.w->qtri.V, (size_t)npan * mqr * NB * 16, s))) return rc;
    big.push_back(j);
  }
  if (big.empty()) return 0;
  // 1. tridiagonalisations, packed into cooperative launches of <= 256 blocks
  {
    TriBatch tb{};
    int used = 0;
    size_t shmem = 0;
    auto flush = [&]() -> int {
      if (tb.nprob == 0) return 0;
      void* args[] = {(void*)&tb};
      QT_HIP_CHECK(hipLaunchCooperativeKernel((const void*)tridiag_kernel, dim3(used), dim3(256), args,
                                              (unsigned)shmem, s));
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
      S.VT = (c128*)J.w->qtri.VT;
      S.T = J.w->qtri.T;
      S.tau = J.w->tau;
      S.n = J.n;
      S.kwant = J.kwant;
      maxn = std::max(maxn, J.n);
      maxk = std::max(maxk, J.kwant);
    }
    const int npan = (maxn - 1 + NB - 1) / NB;
    hipLaunchKernelGGL(larft_kernel, dim3(npan, sb.njobs), dim3(256), 0, s, sb);
    QT_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(bisect_kernel, dim3((maxk + 31) / 32, sb.njobs), dim3(256), 0, s, sb);
    QT_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(invit_kernel, dim3((maxk + 63) / 64, sb.njobs), dim3(64), 0, s, sb);
    QT_HIP_CHECK(hipGetLastError());
    hipLaunchKernelGGL(cluster_mgs_kernel, dim3(maxk, sb.njobs), dim3(256), 0, s, sb, 1e-9);
    QT_HIP_CHECK(hipGetLastError());
  }
  // 6. two Newton-Schulz steps Z <- Z - Z (Z^H Z - 1)/2, grouped over the jobs
  const GemmTypes ty{DT_C128, DT_C128};
  std::vector<GemmProb> gs;
  for (int it = 0; it < 2; ++it) {
    gs.clear();
    for (int j : big) {
      const EigJob& J = jobs[j];
      gs.push_back(gemm_prob(J.E, J.kwant, OP_C, J.E, J.kwant, OP_N, J.w->gz, J.kwant, J.kwant, J.kwant, J.n));
    }
    if ((rc = gemm_run(gs.data(), (int)gs.size(), ty, s))) return rc;
    gs.clear();
    for (int j : big) {
      const EigJob& J = jobs[j];
      hipLaunchKernelGGL(sub_identity_kernel, dim3(std::min(4096, (J.kwant * J.kwant + 255) / 256)), dim3(256), 0, s,
                         J.w->gz, J.kwant);
      QT_HIP_CHECK(hipGetLastError());
      QT_HIP_CHECK(hipMemcpyAsync(J.w->ztmp, J.E, (size_t)J.n * J.kwant * sizeof(c128), hipMemcpyDeviceToDevice, s));
      gs.push_back(gemm_prob(J.w->ztmp, J.kwant, OP_N, J.w->gz, J.kwant, OP_N, J.E, J.kwant, J.n, J.kwant, J.kwant,
                             -0.5f, 1.f));
    }
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
