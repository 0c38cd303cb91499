// Blocked Householder QR for the tall matrices of the bond update.
//
// Sec. II of the paper truncates with two QR decompositions (X = Q^[m] R and,
// as the QR of Y^dag, Y = L Q^[n]).  Both are thin, unpivoted Householder
// factorisations here:
//
//  * panel: 32 columns at a time, factored by one cooperative kernel whose
//    blocks each keep a slab of panel rows in LDS (FP64 arithmetic whatever
//    the storage precision).  Column k needs one grid barrier: every block
//    contributes sum_i conj(P[i,k]) P[i,c] over its rows below the diagonal
//    for all c, which yields at once the norm below the diagonal (c = k, no
//    cancellation against the diagonal), the reflector's products with the
//    panel (c > k) and the products with the earlier reflectors that build
//    the compact-WY factor T (c < k).  Reflectors follow LAPACK's zlarfg
//    convention: H = I - tau v v^H, v_k = 1, beta real.
//  * trailing update: A <- (I - V T V^H)^H A as W = V^H A (an MFMA GEMM
//    split over the long dimension), W <- T^H W folded into the reduction of
//    the split partials (FP64), and A -= V W (MFMA GEMM).
//  * explicit Q: backward accumulation of the same blocks onto [I; 0], with
//    T in place of T^H.
#include "qr.h"

#include <algorithm>
#include <vector>

namespace qrtebd {
namespace {

constexpr int NB = kQrNb;
constexpr int LDV = kQrLdv;

// One panel problem of a batched panel launch: its blocks are
// [blk0, blk0 + nblk) of the grid and synchronise among themselves only.
struct PanelProb {
  void* A;
  long long lda;
  void* V;        // this panel's reflectors (ld LDV); odd panels also clear the 32 rows above
  c128* T;
  // reflectors of the previous panel, applied to this panel's columns first
  // (null for the first panel): V from the row 32 above this panel, its T,
  // the 32 rows of A above the panel (entries of R) and the exchange buffer
  const void* Vprev;
  const c128* Tprev;
  void* Atop;
  c128* wx;
  c128* red;
  c128* rowbuf;
  unsigned* sync;
  int m, jb, rows_per_blk, nblk, blk0, gen0, odd;
  int chol;   // Cholesky path (two slabs of LDS)
};
constexpr int kMaxPanelProbs = 24;
// Panel launches of at most this many blocks are plain launches (the CUs
// that the auxiliary stream's mask leaves free hold them all).
constexpr int kPlainPanelBlocks = 64;
struct PanelBatch {
  int nprob;
  int* status;
  PanelProb p[kMaxPanelProbs];
};

__device__ inline c128 cz() { return mk<double>(0, 0); }

constexpr int LDP = NB + 1;   // padded LDS row stride of the panel slab
constexpr int kMaxPanelRows = 160;

constexpr int kPanelThreads = 512;   // 16 row groups x 32 columns: two waves per SIMD (1024: slower)
constexpr int kRowGroups = kPanelThreads / 32;
constexpr int kStage = NB * NB / kPanelThreads;          // elements of a 32 x 32 tile per thread
constexpr int kColLanes = kPanelThreads / NB;            // lanes that share one column's partials

template <typename S>
__global__ __launch_bounds__(kPanelThreads) void qr_panel_kernel(PanelBatch batch) {
  extern __shared__ c128 P[];  // rows_per_blk x LDP
  __shared__ c128 part[kRowGroups][NB];
  __shared__ c128 tsum[NB];
  __shared__ c128 Sk[NB][NB + 1];   // per column k: V[:, j]^dag v_k for j < k (builds T after the loop)
  __shared__ c128 Tm[NB][NB + 1];
  __shared__ c128 taus[NB];
  __shared__ c128 rowk[NB];
  __shared__ int flag;
  __shared__ c128 Xm[NB][NB + 1];   // small factors of the Cholesky path
  __shared__ c128 bc[2][4][NB];      // row / column broadcasts of its sweeps (two steps in flight)
  __shared__ double fscr[kPanelThreads / 64];
  __shared__ double pivs[NB];        // per-step reciprocal pivots of those sweeps

  int pi = 0;
  while (pi + 1 < batch.nprob && (int)blockIdx.x >= batch.p[pi + 1].blk0) ++pi;
  const PanelProb& a = batch.p[pi];
  const GridSync gs{a.sync, batch.status};
  const int tid = threadIdx.x, nblk = a.nblk, blk = (int)blockIdx.x - a.blk0;
  const int r0 = blk * a.rows_per_blk;
  const int nr = max(0, min(a.m, r0 + a.rows_per_blk) - r0);
  const int jb = a.jb;
  cpx<S>* A = (cpx<S>*)a.A;

  for (int idx = tid; idx < nr * NB; idx += kPanelThreads) {
    const int i = idx / NB, c = idx % NB;
    P[i * LDP + c] = c < jb ? ccast<double>(A[(long long)(r0 + i) * a.lda + c]) : cz();
  }
  if (tid == 0) flag = 0;
  __syncthreads();

  if (a.Vprev) {
    // The previous panel's reflectors on this panel's columns (rows from 32
    // above the panel): W = V^H A over all rows (block partials exchanged
    // through one barrier), W <- T^H W, A -= V W on the slab in LDS and, in
    // block 0, on the 32 rows above (written back: they belong to R).
    const cpx<S>* Vp = (const cpx<S>*)a.Vprev;
    cpx<S>* At = (cpx<S>*)a.Atop;
    // This block's share of the rows: the 32 rows above the panel (block 0
    // only: A rows from Atop) and the slab (A rows in LDS).  Share row t is
    // row vrow(t) of Vp.  Both products run on FP64 MFMA (16x16x4 blocks,
    // four real products per complex one); a lane holds A element
    // (lane & 15, lane >> 4), B element (lane >> 4, lane & 15) and output
    // rows (lane >> 4) + 4 r of column lane & 15.
    typedef double v4d __attribute__((ext_vector_type(4)));
    auto mfma = [](double x, double y, v4d acc) { return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, acc, 0, 0, 0); };
    const int top = blk == 0 ? NB : 0, K1 = top + nr;
    auto vrow = [&](int t) -> long long { return t < top ? t : NB + r0 + (t - top); };
    const int wv = tid >> 6, lane = tid & 63, lm = lane & 15, lk = lane >> 4;
    {
      // W_blk = V^H A over the share: wave wv owns output block (qi, ci) =
      // (wv & 1, (wv >> 1) & 1) and every other k step (kh = wv >> 2)
      const int qi = wv & 1, ci = (wv >> 1) & 1, kh = wv >> 2;
      const int nsteps = (K1 + 3) / 4;
      constexpr int kB = 16;   // k steps whose operands are loaded together
      v4d cre = {0, 0, 0, 0}, cim = {0, 0, 0, 0};
      for (int s0 = kh; s0 < nsteps; s0 += 2 * kB) {
        c128 va[kB], xa[kB];
#pragma unroll
        for (int u = 0; u < kB; ++u) {
          const int t = 4 * (s0 + 2 * u) + lk, cx = 16 * ci + lm;
          va[u] = cz();
          xa[u] = cz();
          if (t < K1) {
            va[u] = ccast<double>(Vp[vrow(t) * LDV + 16 * qi + lm]);
            xa[u] = t >= top ? P[(t - top) * LDP + cx] : (cx < jb ? ccast<double>(At[(long long)t * a.lda + cx]) : cz());
          }
        }
#pragma unroll
        for (int u = 0; u < kB; ++u) {   // A = V^H: (Re V, -Im V)
          cre = mfma(va[u].re, xa[u].re, cre);
          cre = mfma(va[u].im, xa[u].im, cre);
          cim = mfma(va[u].re, xa[u].im, cim);
          cim = mfma(-va[u].im, xa[u].re, cim);
        }
      }
      // the two k halves meet in Sk (free until the column loop)
      if (kh == 1)
#pragma unroll
        for (int r = 0; r < 4; ++r) Sk[16 * qi + lk + 4 * r][16 * ci + lm] = mk<double>(cre[r], cim[r]);
      __syncthreads();
      if (kh == 0)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int q = 16 * qi + lk + 4 * r, cx = 16 * ci + lm;
          pub_store(a.wx + ((long long)blk * NB + cx) * NB + q, cadd(mk<double>(cre[r], cim[r]), Sk[q][cx]));
        }
    }
    // V rows of this wave's first row block of the update below, requested
    // while the barrier waits (after its store wait, which would otherwise
    // wait for them too) so that their latency passes during the reduction
    c128 va5[NB / 4];
    auto load_v5 = [&](int ti) {
#pragma unroll
      for (int s4 = 0; s4 < NB / 4; ++s4) {
        const int t = 16 * ti + lm;
        va5[s4] = t < K1 ? ccast<double>(Vp[vrow(t) * LDV + 4 * s4 + lk]) : cz();
      }
    };
    if (!grid_barrier(gs, (unsigned)(a.gen0 + 1), blk, nblk, &flag, [&]() { load_v5(wv); })) return;
    // Block b reduces columns b, b + nblk, ...: W[:, c] = sum of the block
    // partials, then (T^H W)[:, c], published for everyone.
    c128* w2 = a.wx + (long long)nblk * NB * NB;
    __syncthreads();
#pragma unroll
    for (int e = 0; e < kStage; ++e) {
      const int idx = tid + kPanelThreads * e;
      Sk[idx / NB][idx % NB] = a.Tprev[idx];
    }
    const auto rwx = coh_rsrc(a.wx);
    for (int c = blk; c < NB; c += nblk) {
      const int r = tid & 31, g = tid >> 5;   // kRowGroups groups of blocks
      c128 acc = cz();
      for (int b0 = g; b0 < nblk; b0 += 4 * kRowGroups) {
        c128 l[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int b = b0 + kRowGroups * u;
          l[u] = b < nblk ? coh_load(rwx, (b * NB + c) * NB + r) : cz();
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) acc = cadd(acc, l[u]);
      }
      part[g][r] = acc;
      __syncthreads();
      if (tid < NB) {
        c128 wr = cz();
#pragma unroll
        for (int gg = 0; gg < kRowGroups; ++gg) wr = cadd(wr, part[gg][tid]);
        Tm[tid][0] = wr;
      }
      __syncthreads();
      if (tid < NB) {   // (T^H W)[q][c] = sum_r conj(T[r][q]) W[r][c], q = tid
        c128 u4[4] = {cz(), cz(), cz(), cz()};
#pragma unroll
        for (int r0 = 0; r0 < NB; r0 += 4)
#pragma unroll
          for (int u = 0; u < 4; ++u) u4[u] = cadd(u4[u], cmulc(Sk[r0 + u][tid], Tm[r0 + u][0]));
        pub_store(w2 + (long long)tid * NB + c, cadd(cadd(u4[0], u4[1]), cadd(u4[2], u4[3])));
      }
      __syncthreads();
    }
    if (!grid_barrier(gs, (unsigned)(a.gen0 + 2), blk, nblk, &flag)) return;
#pragma unroll
    for (int e = 0; e < kStage; ++e) {
      const int idx = tid + kPanelThreads * e;
      Tm[idx / NB][idx % NB] = coh_load(rwx, nblk * NB * NB + idx);
    }
    __syncthreads();
    // A -= V W over the share: wave wv owns row blocks wv, wv + 8, ..., both
    // column blocks
    for (int ti = wv; ti < (K1 + 15) / 16; ti += 8) {
      if (ti != wv) load_v5(ti);
      const c128* va = va5;
      v4d dre[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}}, dim[2] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
#pragma unroll
      for (int s4 = 0; s4 < NB / 4; ++s4)
#pragma unroll
        for (int cj = 0; cj < 2; ++cj) {
          const c128 w = Tm[4 * s4 + lk][16 * cj + lm];
          dre[cj] = mfma(va[s4].re, w.re, dre[cj]);
          dre[cj] = mfma(-va[s4].im, w.im, dre[cj]);
          dim[cj] = mfma(va[s4].re, w.im, dim[cj]);
          dim[cj] = mfma(va[s4].im, w.re, dim[cj]);
        }
#pragma unroll
      for (int cj = 0; cj < 2; ++cj)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int t = 16 * ti + lk + 4 * r, cx = 16 * cj + lm;
          if (t >= K1) continue;
          const c128 d = mk<double>(dre[cj][r], dim[cj][r]);
          if (t >= top) {
            c128* x = P + (t - top) * LDP + cx;
            *x = csub(*x, d);
          } else if (cx < jb) {
            const long long o = (long long)t * a.lda + cx;
            At[o] = ccast<S>(csub(ccast<double>(At[o]), d));
          }
        }
    }
    __syncthreads();
  }


  // ---- Cholesky path (panels whose blocks hold two slabs in LDS).  QR of
  // the slab stack by CholeskyQR2 (A = Q1 R1, Q1 = Q R2 from the Gram
  // matrices, four barriers), then the compact-WY form of Householder
  // reflectors for the same Q: the LU factorisation of [I; 0] - Q D, with the
  // unit-modulus diagonal D chosen at every step so the pivot is 1 + |q|
  // (Ballard et al., Reconstructing Householder vectors from tall-skinny QR),
  // gives V (unit lower trapezoidal) and U; T = U V1^-H, R = D^H R2 R1.  The
  // Gram matrices reach every block in the same order, so every block takes
  // the same decision: when Cholesky breaks down or Q1 is far from
  // orthonormal (||Q1^H Q1 - I||_F > 1/4), the panel falls back to the
  // Householder column loop below with the slab untouched.
  int gen_loop = 3;   // generation of the column loop's first barrier
  if (a.chol) {
    c128* P2 = P + (size_t)a.rows_per_blk * LDP;   // second slab
    c128* gsum = a.wx + (long long)nblk * NB * NB;  // reduced Gram matrix
    const int i0 = tid >> 5, jc = tid & 31;         // owner of entries (i0, jc), (i0 + 16, jc)

    // FP64 MFMA (16x16x4 blocks, four real products per complex one); lane
    // layout as in the product above: A element (lm, lk), B element (lk, lm),
    // output rows lk + 4 r of column lm
    typedef double f64x4 __attribute__((ext_vector_type(4)));
    auto mf = [](double x, double y, f64x4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c, 0, 0, 0); };
    const int wv = tid >> 6, lm = tid & 15, lk = (tid >> 4) & 3;
    // Gram matrix X^H X of slab X over this block's rows, as a block partial
    // (nblk > 1) or directly into Sk: wave wv forms output block (wv & 1,
    // (wv >> 1) & 1) over every other k step; the halves meet in Tm
    auto gram = [&](const c128* X) {
      const int qi = wv & 1, ci = (wv >> 1) & 1, kh = wv >> 2, nst = (nr + 3) / 4;
      f64x4 cre = {0, 0, 0, 0}, cim = {0, 0, 0, 0};
#pragma unroll 2
      for (int st = kh; st < nst; st += 2) {
        const int t = 4 * st + lk;
        const c128 xa = t < nr ? X[t * LDP + 16 * qi + lm] : cz(), xb = t < nr ? X[t * LDP + 16 * ci + lm] : cz();
        cre = mf(xa.re, xb.re, cre);
        cre = mf(xa.im, xb.im, cre);
        cim = mf(xa.re, xb.im, cim);
        cim = mf(-xa.im, xb.re, cim);
      }
      if (kh == 1)
#pragma unroll
        for (int r = 0; r < 4; ++r) Tm[16 * qi + lk + 4 * r][16 * ci + lm] = mk<double>(cre[r], cim[r]);
      __syncthreads();
      if (kh == 0)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int ca = 16 * qi + lk + 4 * r, cb = 16 * ci + lm;
          const c128 g = cadd(mk<double>(cre[r], cim[r]), Tm[ca][cb]);
          if (nblk > 1) pub_store(a.wx + (long long)blk * NB * NB + ca * NB + cb, g);
          else Sk[ca][cb] = (ca == cb && ca >= jb) ? mk<double>(1, 0) : g;
        }
    };
    // sum of the block partials: block b reduces one share of the entries
    // (barrier gen), then every block gathers the sums (barrier gen + 1);
    // columns past jb are given a unit diagonal
    auto reduce_gram = [&](unsigned gen) -> bool {
      if (nblk == 1) {
        __syncthreads();
        return true;
      }
      if (!grid_barrier(gs, gen, blk, nblk, &flag)) return false;
      const int per = (NB * NB + nblk - 1) / nblk, e0 = blk * per;
      const int cnt = min(per, NB * NB - e0), groups = kPanelThreads / per;
      c128* stage = &part[0][0];
      const auto rwx = coh_rsrc(a.wx);
      {
        const int g = tid / per, el = tid - g * per;
        if (g < groups && el < cnt) {
          c128 acc2 = cz();
          for (int b = g; b < nblk; b += groups) acc2 = cadd(acc2, coh_load(rwx, b * NB * NB + e0 + el));
          stage[g * per + el] = acc2;
        }
      }
      __syncthreads();
      if (tid < cnt) {
        c128 t = cz();
        for (int g = 0; g < groups; ++g) t = cadd(t, stage[g * per + tid]);
        pub_store(gsum + e0 + tid, t);
      }
      if (!grid_barrier(gs, gen + 1, blk, nblk, &flag)) return false;
      const auto rgs = coh_rsrc(gsum);
      for (int e = tid; e < NB * NB; e += kPanelThreads) {
        const int ca = e >> 5, cb = e & 31;
        Sk[ca][cb] = (ca == cb && ca >= jb) ? mk<double>(1, 0) : coh_load(rgs, e);
      }
      __syncthreads();
      return true;
    };
    // Cholesky G = R^H R of the Hermitian matrix in Gm (upper triangle) by
    // row elimination on [G | I] without square roots (rows of D R and of
    // D R^-H, D the pivots), each row scaled by 1/sqrt(pivot) at the end:
    // R into Ro, R^-1 into Rio (both may alias Gm).  True when every pivot
    // is positive.
    auto chol_inv = [&](c128 (*Gm)[NB + 1], c128 (*Ro)[NB + 1], c128 (*Rio)[NB + 1]) -> bool {
      // entries (i0, jc) and (i0 + 16, jc) of the left and right halves
      c128 la = jc >= i0 ? Gm[i0][jc] : cz(), lb = jc >= i0 + 16 ? Gm[i0 + 16][jc] : cz();
      c128 ra = mk<double>(i0 == jc ? 1.0 : 0.0, 0.0), rb = mk<double>(i0 + 16 == jc ? 1.0 : 0.0, 0.0);
      bool ok = true;
      // Two pivots per block barrier: the owners publish rows k and k + 1 (as
      // left after step k - 1; pl, pr are the owner's entries), and every
      // thread forms the entries of row k + 1 after step k that it needs with
      // the owner's own expression.  The two halves of k run as separate
      // loops so the owned entries stay in registers.
      auto step2 = [&](int k, c128 pl, c128 pr) {
        const int b = (k >> 1) & 1;
        if (i0 == (k & 15)) {
          bc[b][0][jc] = pl;
          bc[b][1][jc] = pr;
        }
        if (i0 == ((k + 1) & 15)) {
          bc[b][2][jc] = pl;
          bc[b][3][jc] = pr;
        }
        __syncthreads();
        const double piv0 = bc[b][0][k].re;
        const double ip0 = piv0 > 0.0 ? rcp_refined(piv0) : 0.0;
        const c128 g01 = bc[b][0][k + 1];
        auto row1L = [&](int x) { return csub(bc[b][2][x], cscale(cmulc(g01, bc[b][0][x]), ip0)); };
        auto row1R = [&](int x) { return csub(bc[b][3][x], cscale(cmulc(g01, bc[b][1][x]), ip0)); };
        const double piv1 = row1L(k + 1).re;
        const double ip1 = piv1 > 0.0 ? rcp_refined(piv1) : 0.0;
        ok = ok && piv0 > 0.0 && isfinite(piv0) && piv1 > 0.0 && isfinite(piv1);
        if (tid == 0) {
          pivs[k] = ip0;
          pivs[k + 1] = ip1;
        }
        const c128 l1j = row1L(jc), r1j = row1R(jc);
        auto upd = [&](c128& lv, c128& rv, int r) {
          if (r > k) {
            const c128 gkr = bc[b][0][r];
            if (jc >= r) lv = csub(lv, cscale(cmulc(gkr, bc[b][0][jc]), ip0));
            rv = csub(rv, cscale(cmulc(gkr, bc[b][1][jc]), ip0));
          }
          if (r > k + 1) {
            const c128 g1r = row1L(r);
            if (jc >= r) lv = csub(lv, cscale(cmulc(g1r, l1j), ip1));
            rv = csub(rv, cscale(cmulc(g1r, r1j), ip1));
          }
        };
        upd(la, ra, i0);
        upd(lb, rb, i0 + 16);
      };
#pragma unroll 1
      for (int k = 0; k < 16; k += 2) step2(k, la, ra);
#pragma unroll 1
      for (int k = 16; k < NB; k += 2) step2(k, lb, rb);
      __syncthreads();
      // rows of the LDL^H form scaled by 1/sqrt(pivot)
      {
        const double sa = sqrt(pivs[i0]), sb = sqrt(pivs[i0 + 16]);
        la = cscale(la, sa);
        ra = cscale(ra, sa);
        lb = cscale(lb, sb);
        rb = cscale(rb, sb);
      }
      Ro[i0][jc] = la;
      Ro[i0 + 16][jc] = lb;
      Rio[jc][i0] = cconj(ra);
      Rio[jc][i0 + 16] = cconj(rb);
      __syncthreads();
      return ok;
    };
    // X M over this block's rows (M: 32 x 32, row stride LDP), each
    // product element handed to out(row, col, value); waves take 16 x 16
    // output blocks in turn
    auto slab_mul = [&](const c128* X, const c128* M, auto&& out) {
      const int nrb = (nr + 15) / 16;
      for (int ob = wv; ob < 2 * nrb; ob += kPanelThreads / 64) {
        const int rb = ob >> 1, cb = ob & 1, row = 16 * rb + lm;
        f64x4 cre = {0, 0, 0, 0}, cim = {0, 0, 0, 0};
#pragma unroll 4
        for (int st = 0; st < NB / 4; ++st) {
          const int k = 4 * st + lk;
          const c128 xa = row < nr ? X[row * LDP + k] : cz(), mb = M[k * LDP + 16 * cb + lm];
          cre = mf(xa.re, mb.re, cre);
          cre = mf(-xa.im, mb.im, cre);
          cim = mf(xa.re, mb.im, cim);
          cim = mf(xa.im, mb.re, cim);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int orow = 16 * rb + lk + 4 * r;
          if (orow < nr) out(orow, 16 * cb + lm, mk<double>(cre[r], cim[r]));
        }
      }
      __syncthreads();
    };

    // pass 1: G1 = A^H A, R1 (Xm), R1^-1 (Tm), Q1 = A R1^-1 (P2)
    gram(P);
    if (!reduce_gram((unsigned)(a.gen0 + 3))) return;
    bool ok = chol_inv(Sk, Xm, Tm);
    slab_mul(P, &Tm[0][0], [&](int r, int c, c128 v) { P2[r * LDP + c] = v; });
    // pass 2: G2 = Q1^H Q1, R2 (Sk), R2^-1 (Tm)
    gram(P2);
    if (!reduce_gram((unsigned)(a.gen0 + 5))) return;
    double dev = 0;
    for (int e = tid; e < NB * NB; e += kPanelThreads) {
      const int ca = e >> 5, cb = e & 31;
      if (ca <= cb && cb < jb) {
        const c128 g = Sk[ca][cb];
        dev += ca == cb ? (g.re - 1) * (g.re - 1) + g.im * g.im : 2 * cabs2(g);
      }
    }
    dev = block_sum(dev, fscr);
    ok = ok && dev <= 0.0625 && isfinite(dev);
    if (ok && dev <= 1e-12) {
      // G2 = I + E with ||E||_F <= 1e-6: the Cholesky factor to second order,
      // U1 = upper(E) with half its diagonal, U2 = -upper(U1^H U1) with half
      // its diagonal, R2 = I + U1 + U2, R2^-1 = I - U1 - U2 + U1^2, both
      // exact to O(||E||^3), below the rounding of FP64
      for (int e = tid; e < NB * NB; e += kPanelThreads) {
        const int ca = e >> 5, cb = e & 31;
        const c128 g = Sk[ca][cb];
        Sk[ca][cb] = ca < cb ? g : (ca == cb ? mk<double>(0.5 * (g.re - 1.0), 0.0) : cz());
      }
      __syncthreads();
      c128 r2[2], m2[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int r = i0 + 16 * h;
        c128 s1 = cz(), s2 = cz();
#pragma unroll 4
        for (int l = 0; l < NB; ++l) {
          s1 = cadd(s1, cmulc(Sk[l][r], Sk[l][jc]));   // (U1^H U1)[r][jc]
          s2 = cadd(s2, cmul(Sk[r][l], Sk[l][jc]));    // (U1 U1)[r][jc]
        }
        const c128 u1 = Sk[r][jc];
        const c128 u2 = r < jc ? cscale(s1, -1.0) : (r == jc ? mk<double>(-0.5 * s1.re, 0.0) : cz());
        const double id = r == jc ? 1.0 : 0.0;
        r2[h] = mk<double>(id + u1.re + u2.re, u1.im + u2.im);
        m2[h] = mk<double>(id - u1.re - u2.re + s2.re, -u1.im - u2.im + s2.im);
      }
      __syncthreads();
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        Sk[i0 + 16 * h][jc] = r2[h];
        Tm[i0 + 16 * h][jc] = m2[h];
      }
      __syncthreads();
    } else {
      ok = chol_inv(Sk, Sk, Tm) && ok;
    }
    if (ok) {
      slab_mul(P2, &Tm[0][0], [&](int r, int c, c128 v) { P[r * LDP + c] = v; });   // Q; P2 is free from here on
      c128 rra = cz(), rrb = cz();   // R = R2 R1, entries (i0, jc), (i0 + 16, jc) (block 0)
      if (blk == 0) {
#pragma unroll 4
        for (int l = 0; l < NB; ++l) {
          rra = cadd(rra, cmul(Sk[i0][l], Xm[l][jc]));
          rrb = cadd(rrb, cmul(Sk[i0 + 16][l], Xm[l][jc]));
        }
        __syncthreads();
        // LU of [I; 0] - Q D on the top 32 rows, with [.. | I] alongside:
        // V1 (Sk, strictly lower), d (taus), U (Xm), V1^-1 (Tm)
        c128 qa = i0 < nr ? P[i0 * LDP + jc] : cz(), qb = i0 + 16 < nr ? P[(i0 + 16) * LDP + jc] : cz();
        c128 ea = mk<double>(i0 == jc ? 1.0 : 0.0, 0.0), eb = mk<double>(i0 + 16 == jc ? 1.0 : 0.0, 0.0);
        auto lu_step = [&](int i, c128 pq, c128 pe) {
          const int b = i & 1;
          if (i0 == (i & 15)) {
            bc[b][0][jc] = pq;
            bc[b][1][jc] = pe;
          }
          if (jc == i) {
            bc[b][2][i0] = qa;
            bc[b][2][i0 + 16] = qb;
          }
          __syncthreads();
          const c128 av = bc[b][0][i];
          const double m2 = cabs2(av), rs = m2 > 0.0 ? rsq_refined(m2) : 0.0, mag = m2 * rs;
          const c128 di = m2 > 0.0 ? mk<double>(-av.re * rs, av.im * rs) : mk<double>(1, 0);   // -conj(a)/|a|
          const double iu = rcp_refined(1.0 + mag);
          auto upd = [&](c128& qv, c128& ev, int r) {
            if (r > i) {
              const c128 l = cscale(cmul(bc[b][2][r], di), -iu);
              if (jc == i) Sk[r][i] = l;
              if (jc > i) qv = csub(qv, cmul(l, bc[b][0][jc]));
              ev = csub(ev, cmul(l, bc[b][1][jc]));
            }
          };
          upd(qa, ea, i0);
          upd(qb, eb, i0 + 16);
          if (tid == 0) {
            taus[i] = di;
            rowk[i] = mk<double>(1.0 + mag, 0.0);
            pivs[i] = iu;
          }
        };
        for (int i = 0; i < 16; ++i) lu_step(i, qa, ea);
        for (int i = 16; i < NB; ++i) lu_step(i, qb, eb);
        __syncthreads();
        Xm[i0][jc] = jc > i0 ? cscale(cmul(qa, taus[jc]), -1.0) : (jc == i0 ? rowk[i0] : cz());
        Xm[i0 + 16][jc] = jc > i0 + 16 ? cscale(cmul(qb, taus[jc]), -1.0) : (jc == i0 + 16 ? rowk[i0 + 16] : cz());
        Tm[i0][jc] = ea;
        Tm[i0 + 16][jc] = eb;
        __syncthreads();
        // U^-1 by back substitution on [U | I]
        c128 xa = mk<double>(i0 == jc ? 1.0 : 0.0, 0.0), xb = mk<double>(i0 + 16 == jc ? 1.0 : 0.0, 0.0);
        auto bs_step = [&](int i, c128 px) {
          const int b = i & 1;
          if (i0 == (i & 15)) bc[b][1][jc] = px;
          __syncthreads();
          const double ip = pivs[i];   // 1 / U[i][i]
          auto upd = [&](c128& xv, int r) {
            if (r < i) xv = csub(xv, cmul(cscale(Xm[r][i], ip), bc[b][1][jc]));
            else if (r == i) xv = cscale(xv, ip);
          };
          upd(xa, i0);
          upd(xb, i0 + 16);
        };
        for (int i = NB - 1; i >= 16; --i) bs_step(i, xb);
        for (int i = 15; i >= 0; --i) bs_step(i, xa);
        P2[i0 * LDP + jc] = xa;
        P2[(i0 + 16) * LDP + jc] = xb;
        if (nblk > 1) {
          pub_store(a.wx + i0 * NB + jc, xa);
          pub_store(a.wx + (i0 + 16) * NB + jc, xb);
          if (tid < NB) pub_store(a.wx + NB * NB + tid, taus[tid]);
        }
      }
      if (nblk > 1) {
        if (!grid_barrier(gs, (unsigned)(a.gen0 + 7), blk, nblk, &flag)) return;
        if (blk != 0) {
          const auto rwx = coh_rsrc(a.wx);
          for (int e = tid; e < NB * NB; e += kPanelThreads) P2[(e >> 5) * LDP + (e & 31)] = coh_load(rwx, e);
          if (tid < NB) taus[tid] = coh_load(rwx, NB * NB + tid);
        }
      }
      __syncthreads();
      // write back: rows past jb hold V2 = Q M with M = -D U^-1 (in A below
      // the diagonal and in V); the top rows (block 0) R_h = D^H R above the
      // diagonal and V1 below it
      for (int e = tid; e < NB * NB; e += kPanelThreads) {
        c128* x = P2 + (e >> 5) * LDP + (e & 31);
        *x = cscale(cmul(taus[e >> 5], *x), -1.0);
      }
      __syncthreads();
      cpx<S>* V = (cpx<S>*)a.V;
      slab_mul(P, P2, [&](int r, int c, c128 v) {
        if (r0 + r < jb) return;
        const long long row = r0 + r;
        if (c < jb) A[row * a.lda + c] = ccast<S>(v);
        V[row * LDV + c] = ccast<S>(c < jb ? v : cz());
      });
      if (blk == 0) {
        auto top_row = [&](int r, c128 rv) {
          if (r >= jb) return;
          if (jc < jb) A[(long long)r * a.lda + jc] = ccast<S>(jc >= r ? cmul(cconj(taus[r]), rv) : Sk[r][jc]);
          const c128 vc = jc < jb ? (jc < r ? Sk[r][jc] : (jc == r ? mk<double>(1, 0) : cz())) : cz();
          V[(long long)r * LDV + jc] = ccast<S>(vc);
        };
        top_row(i0, rra);
        top_row(i0 + 16, rrb);
        if (a.odd)
          for (int idx = tid; idx < NB * NB; idx += kPanelThreads)
            V[(long long)(idx / NB - NB) * LDV + idx % NB] = ccast<S>(cz());
        // T = U V1^-H
        for (int r = i0; r < NB; r += 16) {
          c128 t = cz();
          for (int l = r; l <= jc; ++l) t = cadd(t, cmul(Xm[r][l], cconj(Tm[jc][l])));
          a.T[r * NB + jc] = (r < jb && jc < jb) ? t : cz();
        }
      }
      return;
    }
    gen_loop = 7;
  }

  // Thread (rg, c) owns column c of the slab rows rg, rg + 16, ...  Its running
  // partial t_c = sum_i conj(P[i,k]) P[i,c] over its rows strictly below the
  // diagonal is formed for column 0 here and for column k + 1 during the
  // update by reflector k (the new column k + 1 is read back right after the
  // lanes of the same wave wrote it).
  const int rg = tid >> 5, c = tid & 31;
  c128 acc = cz();
  for (int i = rg; i < nr; i += kRowGroups)
    if (r0 + i > 0) acc = cadd(acc, cmulc(P[i * LDP], P[i * LDP + c]));

  // T of the compact-WY form, one column per grid barrier in the waves that
  // do not poll: T[k][k] = tau_k, T[r][k] = -tau_k sum_q T[r][q] S_k[q]
  // (q = r..k-1).  The 8 lanes r*8 .. r*8+7 of waves 1-4 build entry r, each
  // summing every 8th term.
  for (int idx = tid; idx < NB * NB; idx += kPanelThreads) Tm[idx / NB][idx % NB] = cz();
  auto t_column = [&](int kc) {
    const int u = tid - 64;
    if (u >= 0 && u < 8 * NB) {
      const int r = u >> 3, part = u & 7;
      c128 sacc = cz();
      if (r < kc)
        for (int q = r + ((part - r) & 7); q < kc; q += 8) sacc = cadd(sacc, cmul(Tm[r][q], Sk[kc][q]));
      // sum over the 8 lanes of the row (DPP): quad sums, then lanes 4..7 of
      // each 8-lane group add the quad below, so lane 7 holds the total
      sacc.re += dpp_mov<0xb1>(sacc.re);
      sacc.im += dpp_mov<0xb1>(sacc.im);
      sacc.re += dpp_mov<0x4e>(sacc.re);
      sacc.im += dpp_mov<0x4e>(sacc.im);
      sacc.re += dpp_mov<0x114, 0xf, true>(sacc.re);
      sacc.im += dpp_mov<0x114, 0xf, true>(sacc.im);
      if (part == 7 && r < kc) Tm[r][kc] = cmul(mk<double>(-taus[kc].re, -taus[kc].im), sacc);
    }
  };

  for (int k = 0; k < jb; ++k) {
    const int slot = k & 1;
    // block partial over the row groups
    part[rg][c] = acc;
    __syncthreads();
    if (tid < NB) {
      c128 sblk = cz();
#pragma unroll
      for (int g = 0; g < kRowGroups; ++g) sblk = cadd(sblk, part[g][tid]);
      pub_store(a.red + ((long long)slot * nblk + blk) * NB + tid, sblk);
      if (k >= r0 && k < r0 + nr) pub_store(a.rowbuf + slot * NB + tid, P[(k - r0) * LDP + tid]);
    }
    if (!grid_barrier(gs, (unsigned)(a.gen0 + gen_loop + k), blk, nblk, &flag, [&]() {
          if (k >= 2) t_column(k - 1);
        }))
      return;
    {  // one round of loads: 8 lanes per column share the block partials
      const int cl = tid / kColLanes, bg = tid % kColLanes;
      constexpr int kMaxPer = kMaxPanelBlocks / kColLanes;
      c128 v[kMaxPer];
      const auto rred = coh_rsrc(a.red), rrow = coh_rsrc(a.rowbuf);
#pragma unroll
      for (int q = 0; q < kMaxPer; ++q) {
        const int w = bg + kColLanes * q;
        v[q] = w < nblk ? coh_load(rred, (slot * nblk + w) * NB + cl) : cz();
      }
      const c128 rk = tid < NB ? coh_load(rrow, slot * NB + tid) : cz();
      c128 t = cz();
#pragma unroll
      for (int q = 0; q < kMaxPer; ++q) t = cadd(t, v[q]);
      // the kColLanes lanes of column cl: one or two DPP rows; the last lane
      // of the group ends with the total
      t.re = row16_sum(t.re);
      t.im = row16_sum(t.im);
      if (kColLanes == 32) {
        t.re += dpp_mov<0x142, 0xa>(t.re);   // row_bcast:15 into rows 1 and 3
        t.im += dpp_mov<0x142, 0xa>(t.im);
      }
      if (bg == kColLanes - 1) tsum[cl] = t;
      if (tid < NB) rowk[tid] = rk;
    }
    __syncthreads();
    // every thread derives the reflector (LAPACK zlarfg conventions)
    const c128 alpha = rowk[k];
    const double xnorm2 = fmax(tsum[k].re, 0.0);
    c128 tau = cz(), scale = cz();
    double beta = alpha.re;
    if (!(xnorm2 == 0.0 && alpha.im == 0.0)) {
      beta = -copysign(sqrt(alpha.re * alpha.re + alpha.im * alpha.im + xnorm2), alpha.re);
      const double ib = rcp_refined(beta);
      tau = mk<double>((beta - alpha.re) * ib, -alpha.im * ib);
      const c128 den = mk<double>(alpha.re - beta, alpha.im);
      const double idd = rcp_refined(cabs2(den));
      scale = mk<double>(den.re * idd, -den.im * idd);
    }
    if (tid == 0) {
      taus[k] = tau;
      Tm[k][k] = tau;
      if (!isfinite(beta)) latch_error(batch.status, ERRBIT_NONFINITE);
    }
    if (tid < k)  // V[:, j]^dag v_k = conj(V[k, j]) + scale * conj(t_j)
      Sk[k][tid] = cadd(cconj(rowk[tid]), cmul(scale, cconj(tsum[tid])));
    // apply H_k^H to this thread's column: P[i,c] -= conj(tau) v_i (v^H P[:,c])
    const c128 cvh = cmul(cconj(tau), cadd(rowk[c], cmulc(scale, tsum[c])));
    const int kn = k + 1;
    // v^H P[:, k+1] scaled, for the new P[i, k+1] every lane forms itself
    const c128 cvhn = kn < jb ? cmul(cconj(tau), cadd(rowk[kn], cmulc(scale, tsum[kn]))) : cz();
    acc = cz();
    // Every lane reads the old P[i,k] and P[i,k+1] of its row (broadcast) and
    // its own P[i,c] before it writes P[i,c]; rows go in unrolled chunks so
    // their loads are in flight together.
    constexpr int RU = 5;
    for (int i0 = rg; i0 < nr; i0 += kRowGroups * RU) {
      c128 pk[RU], pn[RU], b[RU];
#pragma unroll
      for (int u = 0; u < RU; ++u) {
        const int i = i0 + kRowGroups * u < nr ? i0 + kRowGroups * u : i0;   // past the slab: dummy read of an own row
        const c128* Pi = P + i * LDP;
        pk[u] = Pi[k];
        pn[u] = Pi[kn < NB ? kn : k];
        b[u] = Pi[c];
      }
#pragma unroll
      for (int u = 0; u < RU; ++u) {
        const int i = i0 + kRowGroups * u, gi = r0 + i;
        const bool act = i < nr && gi >= k;
        const c128 v = gi == k ? mk<double>(1, 0) : cmul(pk[u], scale);
        const c128 bn = c > k ? csub(b[u], cmul(v, cvh)) : (c == k ? (gi == k ? mk<double>(beta, 0.0) : v) : b[u]);
        if (act && c >= k) P[i * LDP + c] = bn;
        if (act && kn < jb && gi > kn) acc = cadd(acc, cmulc(csub(pn[u], cmul(v, cvhn)), bn));
      }
    }
  }

  // the last column of T (the earlier ones were built during the barriers)
  __syncthreads();
  if (jb >= 2) t_column(jb - 1);
  __syncthreads();

  // write back R / reflectors in place, the explicit V and (block 0) T
  cpx<S>* V = (cpx<S>*)a.V;
  for (int idx = tid; idx < nr * NB; idx += kPanelThreads) {
    const int i = idx / NB, cc = idx % NB, gi = r0 + i;
    const c128 pv = P[i * LDP + cc];
    if (cc < jb) A[(long long)(r0 + i) * a.lda + cc] = ccast<S>(pv);
    const c128 vc = cc < jb ? (gi > cc ? pv : (gi == cc ? mk<double>(1, 0) : cz())) : cz();
    V[(long long)(r0 + i) * LDV + cc] = ccast<S>(vc);
  }
  if (blk == 0 && a.odd)   // the rows of the pair block above an odd panel
    for (int idx = tid; idx < NB * NB; idx += kPanelThreads)
      V[(long long)(idx / NB - NB) * LDV + idx % NB] = ccast<S>(cz());
  if (blk == 0)
    for (int idx = tid; idx < NB * NB; idx += kPanelThreads) {
      const int r = idx / NB, cc = idx % NB;
      a.T[idx] = (r < jb && cc < jb) ? Tm[r][cc] : cz();
    }
}

__global__ void fill_zero_kernel(unsigned* p, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

template <typename S>
// (32-bit element index: m n < 2^32 for every workspace this library sizes.)
__global__ void set_identity_kernel(cpx<S>* Q, long long ldq, int m, int n) {
  const unsigned total = (unsigned)m * (unsigned)n, un = n;
  for (unsigned idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += gridDim.x * blockDim.x) {
    const unsigned i = idx / un, j = idx - i * un;
    Q[(long long)i * ldq + j] = mk<S>(i == j ? S(1) : S(0), S(0));
  }
}

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Rows per block of a panel with mp rows for about `target` blocks (rows a
// multiple of 16, at least 32; at most kMaxPanelRows, which fits the slab in
// LDS).  target <= 64.
int panel_rows_for(int mp, int target) {
  target = std::max(1, std::min(64, target));
  int r = (mp + target - 1) / target;
  r = (r + 15) / 16 * 16;
  return std::min(kMaxPanelRows, std::max(32, r));
}
int panel_rows(int mp) { return panel_rows_for(mp, tune_params().panel_blocks); }

// Most blocks any panel of an m-row factorisation uses (for any tuned target:
// 64 blocks gives the fewest rows per block).
int panel_blocks_max(int m) {
  int mx = 1;
  for (int mp = m; mp > 0; mp -= NB) mx = std::max(mx, (mp + panel_rows_for(mp, 64) - 1) / panel_rows_for(mp, 64));
  return mx;
}

template <typename S>
int launch_panel(const PanelBatch& pb, int nblk_total, int max_rows, hipStream_t s) {
  const size_t shmem = (size_t)(pb.p[0].chol ? 2 : 1) * max_rows * LDP * sizeof(c128);
  static bool attr_set = false;
  if (!attr_set) {
    QT_HIP_CHECK(hipFuncSetAttribute((const void*)qr_panel_kernel<S>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, kMaxPanelRows * LDP * sizeof(c128)));
    attr_set = true;
  }
  if (nblk_total <= kPlainPanelBlocks || stream_capturing(s)) {
    // A plain launch stays on the stream's own queue (a cooperative launch
    // goes through a separate device queue, two cross-queue hops per panel).
    // Its blocks are co-resident: one block per CU, and the CUs that the
    // context's auxiliary stream leaves free hold them all; other work only
    // delays the last blocks (the spins are bounded).
    hipLaunchKernelGGL(qr_panel_kernel<S>, dim3(nblk_total), dim3(kPanelThreads), shmem, s, pb);
    QT_HIP_CHECK(hipGetLastError());
    return 0;
  }
  void* args[] = {(void*)&pb};
  QT_HIP_CHECK(hipLaunchCooperativeKernel((const void*)qr_panel_kernel<S>, dim3(nblk_total), dim3(kPanelThreads), args,
                                          (unsigned)shmem, s));
  return 0;
}

}  // namespace

int splitk_for(int M, int N, int K) {
  const int tiles = ((M + 63) / 64) * ((N + 63) / 64);
  int ks = (512 + tiles - 1) / tiles;
  ks = std::min(ks, std::max(1, K / 64));
  return std::max(1, std::min(ks, kMaxSplit));
}

constexpr int kMaxZeroSpans = 32;
struct ZeroBatch {
  int n;
  ZeroSpan sp[kMaxZeroSpans];
};
// blockIdx.y: span; the blocks along x share its rows, a thread one word at
// a time.
__global__ void zero_spans_kernel(ZeroBatch b) {
  const ZeroSpan& z = b.sp[blockIdx.y];
  const long long wpr = z.row_bytes / 4, tot = wpr * z.rows * (long long)z.nrep;
  for (long long i = blockIdx.x * 256ll + threadIdx.x; i < tot; i += (long long)gridDim.x * 256) {
    const long long row = i / wpr, w = i - row * wpr, rep = row / z.rows, r = row - rep * z.rows;
    *(unsigned*)((char*)z.p + rep * z.rep_stride + r * z.row_stride + w * 4) = 0u;
  }
}

int zero_spans(const ZeroSpan* spans, int n, hipStream_t s) {
  for (int i0 = 0; i0 < n; i0 += kMaxZeroSpans) {
    ZeroBatch b{};
    long long most = 0;
    for (int i = i0; i < n && b.n < kMaxZeroSpans; ++i) {
      b.sp[b.n++] = spans[i];
      most = std::max(most, spans[i].row_bytes / 4 * spans[i].rows * (long long)spans[i].nrep);
    }
    if (most == 0) continue;
    const int gx = (int)std::min<long long>((most + 255) / 256, 256);
    hipLaunchKernelGGL(zero_spans_kernel, dim3(gx, b.n), dim3(256), 0, s, b);
    QT_HIP_CHECK(hipGetLastError());
  }
  return 0;
}

int fill_zero(void* p, size_t bytes, hipStream_t s) {
  const size_t n = bytes / 4;
  if (n == 0) return 0;
  const int grid = (int)std::min<size_t>((n + 255) / 256, 2048);
  hipLaunchKernelGGL(fill_zero_kernel, dim3(grid), dim3(256), 0, s, (unsigned*)p, n);
  QT_HIP_CHECK(hipGetLastError());
  return 0;
}

int set_identity(void* Q, long long ldq, int m, int n, int dt, hipStream_t s) {
  const long long total = (long long)m * n;
  const int grid = (int)std::min<long long>((total + 255) / 256, 4096);
  if (total == 0) return 0;
  if (dt == DT_C128)
    hipLaunchKernelGGL(set_identity_kernel<double>, dim3(grid), dim3(256), 0, s, (c128*)Q, ldq, m, n);
  else
    hipLaunchKernelGGL(set_identity_kernel<float>, dim3(grid), dim3(256), 0, s, (c64*)Q, ldq, m, n);
  QT_HIP_CHECK(hipGetLastError());
  return 0;
}

size_t qr_work_bytes(int m, int n, int es, int wcols) {
  const size_t np = (size_t)(n + NB - 1) / NB, npair = (np + 1) / 2, nch = (size_t)(m + 63) / 64;
  if (wcols < n) wcols = n;
  size_t b = 0;
  b += align256(npair * (size_t)m * LDV * es);
  b += align256(np * NB * NB * sizeof(c128));
  b += align256(npair * 4 * NB * NB * sizeof(c128));
  b += align256(npair * nch * NB * NB * sizeof(c128));
  b += align256((size_t)2 * NB * wcols * es);
  b += align256((size_t)kMaxSplit * 2 * NB * wcols * sizeof(c128));
  b += align256((size_t)(panel_blocks_max(m) + 1) * NB * NB * sizeof(c128));
  b += align256((2 * (size_t)kMaxPanelBlocks * NB + 2 * NB) * sizeof(c128));
  b += align256(grid_sync_words(kMaxPanelBlocks) * 4);
  return b;
}

QrWork qr_work_carve(void* base, int m, int n, int es, int wcols, int* status) {
  const size_t np = (size_t)(n + NB - 1) / NB, npair = (np + 1) / 2, nch = (size_t)(m + 63) / 64;
  if (wcols < n) wcols = n;
  char* p = (char*)base;
  QrWork w{};
  w.V = p; p += align256(npair * (size_t)m * LDV * es);
  w.T = (c128*)p; p += align256(np * NB * NB * sizeof(c128));
  w.Tp = (c128*)p; p += align256(npair * 4 * NB * NB * sizeof(c128));
  w.gpart = (c128*)p; p += align256(npair * nch * NB * NB * sizeof(c128));
  w.W = p; p += align256((size_t)2 * NB * wcols * es);
  w.Wsplit = p; p += align256((size_t)kMaxSplit * 2 * NB * wcols * sizeof(c128));
  w.wx = (c128*)p; p += align256((size_t)(panel_blocks_max(m) + 1) * NB * NB * sizeof(c128));
  w.red = (c128*)p; p += align256((2 * (size_t)kMaxPanelBlocks * NB + 2 * NB) * sizeof(c128));
  w.sync = (unsigned*)p;
  w.status = status;
  w.wcols = wcols;
  return w;
}

// W := op(T) sum_s src[s] for the jb x nt block products W = V^H X (jb <= 64)
// of a batch of jobs, FP64 arithmetic, in place when the product was not
// split.  op = T (explicit Q, Z := H Z) or T^H (factorisation).
constexpr int kTwRows = 2 * NB;
struct TwJob {
  const void* src;   // ks x jb x nt partials (compute type = storage type here)
  int ks, jb, nt;
  const c128* T;     // jb x jb, leading dimension ldt
  int ldt;
  void* W;           // jb x nt, ld nt
};
constexpr int kMaxTwJobs = 24;
struct TwBatch {
  int n, herm;
  TwJob j[kMaxTwJobs];
};

// Block: 4 columns of one job, one element (row r, column nn) per thread:
// the split partials are summed with eight loads in flight, the sums go to
// LDS and the same elements of op(T) S are formed.
constexpr int kTwCols = 256 / kTwRows;

template <typename S>
__global__ __launch_bounds__(256) void reduce_tw_kernel(TwBatch b) {
  __shared__ c128 Ts[kTwRows][kTwRows + 1];
  __shared__ c128 Sm[kTwRows][kTwCols];
  const TwJob& J = b.j[blockIdx.y];
  const int n0 = blockIdx.x * kTwCols;
  if (n0 >= J.nt) return;
  // op(T): all loads in flight together, stored to LDS after the partial sums
  constexpr int kTe = kTwRows * kTwRows / 256;
  c128 tv[kTe];
#pragma unroll
  for (int e = 0; e < kTe; ++e) {
    const int idx = threadIdx.x + 256 * e, r = idx / kTwRows, q = idx % kTwRows;
    tv[e] = cz();
    if (r < J.jb && q < J.jb) tv[e] = b.herm ? cconj(J.T[q * J.ldt + r]) : J.T[r * J.ldt + q];
  }
  const int r = threadIdx.x / kTwCols, nn = threadIdx.x % kTwCols, n = n0 + nn;
  const cpx<S>* src = (const cpx<S>*)J.src + (long long)r * J.nt + n;
  const long long stride = (long long)J.jb * J.nt;
  c128 acc = cz();
  if (n < J.nt && r < J.jb) {
    int k = 0;
    for (; k + 8 <= J.ks; k += 8) {
      cpx<S> t[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) t[u] = src[(k + u) * stride];
#pragma unroll
      for (int u = 0; u < 8; ++u) acc = cadd(acc, ccast<double>(t[u]));
    }
    for (; k < J.ks; ++k) acc = cadd(acc, ccast<double>(src[k * stride]));
  }
  Sm[r][nn] = acc;
#pragma unroll
  for (int e = 0; e < kTe; ++e) {
    const int idx = threadIdx.x + 256 * e;
    Ts[idx / kTwRows][idx % kTwRows] = tv[e];
  }
  __syncthreads();
  if (n >= J.nt || r >= J.jb) return;
  c128 o = cz();
  for (int q = 0; q < J.jb; ++q) o = cadd(o, cmul(Ts[r][q], Sm[q][nn]));
  ((cpx<S>*)J.W)[(long long)r * J.nt + n] = ccast<S>(o);
}

// Merged compact-WY factor of a pair of panels: for H = H_e H_o with
// H_x = I - V_x T_x V_x^H, T = [[T_e, -T_e (V_e^H V_o) T_o], [0, T_o]].
// G = V_e^H V_o is a split-K GEMM on FP64 matrix cores whose partials stay
// in gpart; tpair_kernel sums them and forms T.
struct PairTask {
  const void* V;     // pair block, ld LDV
  int rows;          // rows of the pair block
  int has_odd;
  const c128* Te;    // 32 x 32
  const c128* To;    // 32 x 32 (has_odd)
  c128* gpart;       // nparts x 32 x 32 partial sums of V_e^H V_o
  int nparts;
  c128* Tp;          // 64 x 64
};
constexpr int kMaxPairTasks = 64;
struct PairBatch {
  int n;
  PairTask t[kMaxPairTasks];
};

__global__ __launch_bounds__(256) void tpair_kernel(PairBatch b) {
  __shared__ c128 G[NB][NB + 1], X[NB][NB + 1], Te[NB][NB + 1], To[NB][NB + 1];
  const PairTask& T = b.t[blockIdx.x];
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    const int q = e / NB, c = e % NB;
    Te[q][c] = T.Te[e];
    To[q][c] = T.has_odd ? T.To[e] : cz();
    c128 g = cz();
    if (T.has_odd) {
      const int nch = T.nparts;
      for (int k0 = 0; k0 < nch; k0 += 8) {   // eight loads in flight
        c128 l[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) l[u] = k0 + u < nch ? T.gpart[(long long)(k0 + u) * NB * NB + e] : cz();
#pragma unroll
        for (int u = 0; u < 8; ++u) g = cadd(g, l[u]);
      }
    }
    G[q][c] = g;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < NB * NB; e += 256) {   // X = G T_o
    const int q = e / NB, c = e % NB;
    c128 x = cz();
    for (int k = 0; k < NB; ++k) x = cadd(x, cmul(G[q][k], To[k][c]));
    X[q][c] = x;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 4 * NB * NB; e += 256) {
    const int r = e / (2 * NB), c = e % (2 * NB);
    c128 t = cz();
    if (r < NB && c < NB) {
      t = Te[r][c];
    } else if (r >= NB && c >= NB) {
      t = To[r - NB][c - NB];
    } else if (r < NB && c >= NB) {   // -T_e X
      for (int k = 0; k < NB; ++k) t = csub(t, cmul(Te[r][k], X[k][c - NB]));
    }
    T.Tp[e] = t;
  }
}

static int launch_tw(const std::vector<TwJob>& jobs, bool herm, int dt, hipStream_t s) {
  for (size_t i0 = 0; i0 < jobs.size(); i0 += kMaxTwJobs) {
    TwBatch b{};
    b.herm = herm ? 1 : 0;
    int maxn = 0;
    for (size_t i = i0; i < jobs.size() && b.n < kMaxTwJobs; ++i) {
      b.j[b.n++] = jobs[i];
      maxn = std::max(maxn, jobs[i].nt);
    }
    const dim3 grid((maxn + kTwCols - 1) / kTwCols, b.n);
    if (dt == DT_C128)
      hipLaunchKernelGGL(reduce_tw_kernel<double>, grid, dim3(256), 0, s, b);
    else
      hipLaunchKernelGGL(reduce_tw_kernel<float>, grid, dim3(256), 0, s, b);
    QT_HIP_CHECK(hipGetLastError());
  }
  return 0;
}

// The cooperative panel kernels of step p for all jobs, packed into launches
// of at most kMaxPanelBlocks blocks.
static int launch_panels(const QrJob* jobs, int njobs, int p, int dt, hipStream_t s) {
  const int es = dt == DT_C128 ? 16 : 8;
  PanelBatch pb{};
  int used = 0, max_rows = 0;
  int rc;
  auto flush = [&]() -> int {
    if (pb.nprob == 0) return 0;
    // the Cholesky path keeps a second slab in LDS
    for (int q = 0; q < pb.nprob; ++q) pb.p[q].chol = 2 * max_rows <= kMaxPanelRows;
    int r = dt == DT_C128 ? launch_panel<double>(pb, used, max_rows, s) : launch_panel<float>(pb, used, max_rows, s);
    pb = PanelBatch{};
    used = 0;
    max_rows = 0;
    return r;
  };
  for (int j = 0; j < njobs; ++j) {
    const QrJob& J = jobs[j];
    const int j0 = p * NB;
    if (j0 >= J.n) continue;
    const int jb = std::min(NB, J.n - j0), mp = J.m - j0;
    const int rows = panel_rows(mp);
    const int nblk = (mp + rows - 1) / rows;
    if (nblk > kMaxPanelBlocks) return set_error(-2, "qr_factor: panel of %d rows too tall", mp);
    if (used + nblk > kMaxPanelBlocks || pb.nprob == kMaxPanelProbs)
      if ((rc = flush())) return rc;
    const QrWork& w = *J.w;
    PanelProb& pp = pb.p[pb.nprob++];
    pb.status = w.status;
    pp.A = (char*)J.A + ((long long)j0 * J.lda + j0) * es;
    pp.lda = J.lda;
    pp.V = (char*)w.V + qr_v_offset(p, J.m) * es;
    pp.odd = p & 1;
    pp.T = w.T + (size_t)p * NB * NB;
    if (p >= 1) {
      pp.Vprev = (const char*)w.V + qr_v_offset(p - 1, J.m) * es;
      pp.Tprev = w.T + (size_t)(p - 1) * NB * NB;
      pp.Atop = (char*)J.A + ((long long)(j0 - NB) * J.lda + j0) * es;
    }
    pp.wx = w.wx;
    pp.red = w.red;
    pp.rowbuf = w.red + 2 * (size_t)kMaxPanelBlocks * NB;
    pp.sync = w.sync;
    pp.m = mp;
    pp.jb = jb;
    pp.rows_per_blk = rows;
    pp.nblk = nblk;
    pp.blk0 = used;
    pp.gen0 = p * (NB + 8);   // two barriers before the columns, up to five of the Cholesky path, one per
                              // column; increasing over the panels
    used += nblk;
    max_rows = std::max(max_rows, rows);
  }
  return flush();
}

// Apply the reflectors of panel p (as H^H) to the column blocks [b0, b1) of
// every job (clipped to its n): W = V^H A (split over the rows), W <- T^H W
// in the reduction of the split partials, A -= V W.
static int update_columns(const QrJob* jobs, int njobs, int p, int dt, int b0, int b1, hipStream_t s) {
  const int es = dt == DT_C128 ? 16 : 8;
  std::vector<GemmProb> g1s, g2s;
  std::vector<TwJob> tw;
  for (int j = 0; j < njobs; ++j) {
    const QrJob& J = jobs[j];
    const int j0 = p * NB;
    if (j0 >= J.n) continue;
    const int jb = std::min(NB, J.n - j0), mp = J.m - j0;
    const int c0 = b0 * NB, c1 = (int)std::min<long long>(J.n, (long long)b1 * NB);
    const int nt = c1 - c0;
    if (nt <= 0) continue;
    const QrWork& w = *J.w;
    const char* Vp = (const char*)w.V + qr_v_offset(p, J.m) * es;
    void* At = (char*)J.A + ((long long)j0 * J.lda + c0) * es;
    void* W = w.W;
    GemmProb g1 = gemm_prob(Vp, LDV, OP_C, At, J.lda, OP_N, W, nt, jb, nt, mp);
    g1.ksplit = splitk_for(jb, nt, mp);
    g1.work = w.Wsplit;
    g1.skip_reduce = 1;
    g1s.push_back(g1);
    tw.push_back(TwJob{g1.ksplit > 1 ? g1.work : W, g1.ksplit, jb, nt, w.T + (size_t)p * NB * NB, NB, W});
    g2s.push_back(gemm_prob(Vp, LDV, OP_N, W, nt, OP_N, At, J.lda, mp, nt, jb, -1.f, 1.f));
  }
  const GemmTypes ty{dt, dt};
  int rc;
  if (!g1s.empty() && (rc = gemm_run(g1s.data(), (int)g1s.size(), ty, s))) return rc;
  if (!tw.empty() && (rc = launch_tw(tw, true, dt, s))) return rc;
  if (!g2s.empty() && (rc = gemm_run(g2s.data(), (int)g2s.size(), ty, s))) return rc;
  return 0;
}

int qr_factor_batch(const QrJob* jobs, int njobs, int dt, hipStream_t s, const QrAsync* as) {
  int maxp = 0, rc;
  std::vector<ZeroSpan> zs;
  for (int j = 0; j < njobs; ++j) {
    const QrJob& J = jobs[j];
    if (J.n > J.m || J.n <= 0) return set_error(-1, "qr_factor: need 0 < n <= m (m=%d n=%d)", J.m, J.n);
    if (J.m > kMaxQrRows) return set_error(-2, "qr_factor: m=%d too large", J.m);
    // barrier words are zeroed once per factorisation; generations increase over its panels
    zs.push_back(ZeroSpan{J.w->sync, (long long)grid_sync_words(kMaxPanelBlocks) * 4, 0, 0, 1, 1});
    maxp = std::max(maxp, (J.n + NB - 1) / NB);
  }
  if ((rc = zero_spans(zs.data(), (int)zs.size(), s))) return rc;
  if (!as || !as->aux) {
    // in order on one stream: panel p (which first applies panel p-1 to its
    // own columns), then the columns from panel p+2 on
    for (int p = 0; p < maxp; ++p) {
      if ((rc = launch_panels(jobs, njobs, p, dt, s))) return rc;
      if ((rc = update_columns(jobs, njobs, p, dt, p + 2, 1 << 20, s))) return rc;
    }
    return 0;
  }
  // Look-ahead: panel p applies panel p-1 to its own columns itself and
  // starts once the trailing update of panel p-2 has reached them; the update
  // of the columns from panel p+1 on by panel p-1 runs on the auxiliary
  // stream meanwhile.  The cooperative panels occupy a fraction of the CUs,
  // so the two overlap.
  for (int p = 0; p <= maxp; ++p) {
    if (p >= 1) {
      QT_HIP_CHECK(hipStreamWaitEvent(as->aux, as->ev_panel, 0));
      if ((rc = update_columns(jobs, njobs, p - 1, dt, p + 1, 1 << 20, as->aux))) return rc;
    }
    if (p < maxp) {
      if (p >= 2) QT_HIP_CHECK(hipStreamWaitEvent(s, as->ev_trail, 0));
      if ((rc = launch_panels(jobs, njobs, p, dt, s))) return rc;
      QT_HIP_CHECK(hipEventRecord(as->ev_panel, s));
    }
    if (p >= 1) QT_HIP_CHECK(hipEventRecord(as->ev_trail, as->aux));
  }
  if (maxp >= 1) QT_HIP_CHECK(hipStreamWaitEvent(s, as->ev_trail, 0));
  return 0;
}


// Merged factors of every pair of panels of every job (two launches per
// batch of tasks).
static int build_pair_factors(const QrJob* jobs, int njobs, int dt, hipStream_t s) {
  const int es = dt == DT_C128 ? 16 : 8;
  std::vector<PairTask> tasks;
  std::vector<GemmProb> gp;
  for (int j = 0; j < njobs; ++j) {
    const QrJob& J = jobs[j];
    const QrWork& w = *J.w;
    const int np = (J.n + NB - 1) / NB, npair = (np + 1) / 2, nch = (J.m + 63) / 64;
    for (int g = 0; g < npair; ++g) {
      PairTask t{};
      t.V = (const char*)w.V + qr_v_offset(2 * g, J.m) * es;
      t.rows = J.m - 2 * NB * g;
      t.has_odd = 2 * g + 1 < np;
      t.Te = w.T + (size_t)(2 * g) * NB * NB;
      t.To = w.T + (size_t)(2 * g + 1) * NB * NB;
      t.gpart = w.gpart + (size_t)g * nch * NB * NB;
      t.Tp = w.Tp + (size_t)g * 4 * NB * NB;
      t.nparts = 0;
      if (t.has_odd) {   // G = V_e^H V_o; one split writes gpart[0] directly
        GemmProb q = gemm_prob(t.V, LDV, OP_C, (const char*)t.V + NB * es, LDV, OP_N, t.gpart, NB, NB, NB, t.rows);
        q.ksplit = splitk_auto(NB, NB, t.rows, (size_t)nch * NB * NB * sizeof(c128), sizeof(c128));
        q.work = t.gpart;
        q.skip_reduce = 1;
        t.nparts = q.ksplit;
        gp.push_back(q);
      }
      tasks.push_back(t);
    }
  }
  int rc;
  if (!gp.empty() && (rc = gemm_run(gp.data(), (int)gp.size(), GemmTypes{dt, DT_C128}, s))) return rc;
  for (size_t i0 = 0; i0 < tasks.size(); i0 += kMaxPairTasks) {
    PairBatch b{};
    for (size_t i = i0; i < tasks.size() && b.n < kMaxPairTasks; ++i) b.t[b.n++] = tasks[i];
    hipLaunchKernelGGL(tpair_kernel, dim3(b.n), dim3(256), 0, s, b);
    QT_HIP_CHECK(hipGetLastError());
  }
  return 0;
}

// Z_j := H_0 H_1 ... Z_j for every job (Z rows from each pair's first row),
// two panels at a time with their merged factor; set_id first overwrites Z_j
// with [I; 0] (explicit Q).
static int apply_batch(const QrJob* jobs, int njobs, int dt, bool set_id, hipStream_t s) {
  const int es = dt == DT_C128 ? 16 : 8;
  const GemmTypes ty{dt, dt};
  int maxg = 0, rc;
  for (int j = 0; j < njobs; ++j) {
    const QrJob& J = jobs[j];
    maxg = std::max(maxg, ((J.n + NB - 1) / NB + 1) / 2);
    if (set_id && (rc = set_identity(J.Z, J.ldz, J.m, J.nz, dt, s))) return rc;
    if (J.nz > J.w->wcols) return set_error(-1, "qr_apply_q: %d columns exceed the work size %d", J.nz, J.w->wcols);
  }
  if ((rc = build_pair_factors(jobs, njobs, dt, s))) return rc;
  std::vector<GemmProb> g1s, g2s;
  std::vector<TwJob> tw;
  for (int g = maxg - 1; g >= 0; --g) {
    g1s.clear();
    g2s.clear();
    tw.clear();
    for (int j = 0; j < njobs; ++j) {
      const QrJob& J = jobs[j];
      const int j0 = 2 * NB * g;
      if (j0 >= J.n) continue;
      const int jbp = std::min(2 * NB, J.n - j0), mp = J.m - j0;
      const int c0 = set_id ? j0 : 0;        // explicit Q: columns < j0 are still e_j
      const int nz = J.nz - c0;
      if (nz <= 0) continue;
      const char* Vg = (const char*)J.w->V + qr_v_offset(2 * g, J.m) * es;
      void* Zs = (char*)J.Z + ((long long)j0 * J.ldz + c0) * es;
      GemmProb g1 = gemm_prob(Vg, LDV, OP_C, Zs, J.ldz, OP_N, J.w->W, nz, jbp, nz, mp);
      g1.ksplit = splitk_for(jbp, nz, mp);
      g1.work = J.w->Wsplit;
      g1.skip_reduce = 1;
      g1s.push_back(g1);
      tw.push_back(TwJob{g1.ksplit > 1 ? g1.work : J.w->W, g1.ksplit, jbp, nz, J.w->Tp + (size_t)g * 4 * NB * NB,
                         2 * NB, J.w->W});
      g2s.push_back(gemm_prob(Vg, LDV, OP_N, J.w->W, nz, OP_N, Zs, J.ldz, mp, nz, jbp, -1.f, 1.f));
    }
    if (!g1s.empty() && (rc = gemm_run(g1s.data(), (int)g1s.size(), ty, s))) return rc;
    if (!tw.empty() && (rc = launch_tw(tw, false, dt, s))) return rc;
    if (!g2s.empty() && (rc = gemm_run(g2s.data(), (int)g2s.size(), ty, s))) return rc;
  }
  return 0;
}

int qr_form_q_batch(const QrJob* jobs, int njobs, int dt, hipStream_t s) { return apply_batch(jobs, njobs, dt, true, s); }
int qr_apply_q_batch(const QrJob* jobs, int njobs, int dt, hipStream_t s) { return apply_batch(jobs, njobs, dt, false, s); }

int qr_factor(void* A, long long lda, int m, int n, int dt, const QrWork& w, hipStream_t s) {
  QrJob J{A, lda, m, n, A, lda, n, &w};
  return qr_factor_batch(&J, 1, dt, s);
}

int qr_apply_q(void* Z, long long ldz, int nz, int m, int n, int dt, const QrWork& w, hipStream_t s) {
  QrJob J{nullptr, 0, m, n, Z, ldz, nz, &w};
  return qr_apply_q_batch(&J, 1, dt, s);
}

int qr_form_q(void* Q, long long ldq, int m, int n, int dt, const QrWork& w, hipStream_t s) {
  QrJob J{nullptr, 0, m, n, Q, ldq, n, &w};
  return qr_form_q_batch(&J, 1, dt, s);
}

}  // namespace qrtebd
