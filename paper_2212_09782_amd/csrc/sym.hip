// The bond update with a Z_d block structure (Sec. III, closing paragraph;
// the clock model's Z_d symmetry of Sec. IV, in the eigenbasis of its shift
// operator, where the bond gate conserves q_i + q_j mod d).
//
// Tensors stay dense and charge-ordered in memory (every bond lists its
// sectors in charge order; entries outside the blocks are zero), so they are
// interchangeable with those of the dense update.  The work runs on blocks:
//   M_g = B^[m] rows (q, alpha in g - q)   x  sector g of the middle bond
//   N_g = sector g of the middle bond      x  B^[n] columns (q', beta in g + q')
//   Theta_g = M_g N_g                      one GEMM per middle sector
//   C~_c, theta~_c                          the gate mixes the middle sectors:
//       C~_c[(q, alpha), (q', beta)] = sum_p U[(q q'), (p, s - p)] Theta_{a+p}[(p, alpha), (s - p, beta)]
//       with a = charge(alpha), s = q + q'; theta~_c = Xi^[m] C~_c
//   every block c: the dense CBE steps (i)-(v) with eta_c (bond.hip, pre-formed
//   C~ and theta~), one truncation over all blocks (select_sym_kernel)
//   outputs scattered back into dense charge-ordered tensors
// For d sectors of chi/d the contractions and factorisations cost about
// 1/d^2 of the dense update's.
#include "sym.h"

#include "../../include/qrtebd.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace qrtebd {
namespace {

inline size_t a256(size_t x) { return (x + 255) & ~size_t(255); }
inline int grid_n(long long n) { return (int)std::max<long long>(1, std::min<long long>((n + 255) / 256, 8192)); }

__device__ inline int sector_of(const int* off, int d, int x) {
  int a = 0;
  while (a < d - 1 && x >= off[a + 1]) ++a;
  return a;
}

struct SymPtrs {
  void* p[kSymMaxD];
};

// M_g[(rowoff[g][q] + alpha_local), mu_local] = B^[m][alpha, q, mu]
template <typename S>
__global__ __launch_bounds__(256) void sym_gather_m_kernel(const cpx<S>* __restrict__ B, SymDims D, SymPtrs M) {
  const long long n = (long long)D.chiL * D.d * D.chiM;
  for (long long e = blockIdx.x * 256ll + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
    const int mu = (int)(e % D.chiM);
    const long long t = e / D.chiM;
    const int q = (int)(t % D.d), al = (int)(t / D.d);
    const int a = sector_of(D.offL, D.d, al), g = sector_of(D.offM, D.d, mu);
    if ((a + q) % D.d != g) continue;
    cpx<S>* Mg = (cpx<S>*)M.p[g];
    Mg[(size_t)(D.rowoff[g][q] + al - D.offL[a]) * D.secM[g] + (mu - D.offM[g])] = B[e];
  }
}

// N_g[mu_local, coloff[g][q] + beta_local] = B^[n][mu, q, beta]
template <typename S>
__global__ __launch_bounds__(256) void sym_gather_n_kernel(const cpx<S>* __restrict__ B, SymDims D, SymPtrs N) {
  const long long n = (long long)D.chiM * D.d * D.chiR;
  for (long long e = blockIdx.x * 256ll + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
    const int be = (int)(e % D.chiR);
    const long long t = e / D.chiR;
    const int q = (int)(t % D.d), mu = (int)(t / D.d);
    const int g = sector_of(D.offM, D.d, mu), b = sector_of(D.offR, D.d, be);
    if ((g + q) % D.d != b) continue;
    cpx<S>* Ng = (cpx<S>*)N.p[g];
    Ng[(size_t)(mu - D.offM[g]) * D.cols[g] + D.coloff[g][q] + (be - D.offR[b])] = B[e];
  }
}

// Gate and Xi on the blocks: one thread per (alpha, beta) of the two outer
// bonds; it reads the d entries Theta_{a+p}[(p, alpha), (s-p, beta)] and
// writes the d entries of C~ and theta~ with the same (alpha, beta), one in
// each block of middle charge a + q.  |theta~|^2 partials per workgroup.
template <typename S>
__global__ __launch_bounds__(256) void sym_gate_kernel(SymDims D, SymPtrs Th0, SymPtrs C, SymPtrs Th,
                                                       const c128* __restrict__ U, const double* __restrict__ xi,
                                                       double* partial) {
  __shared__ double scr[4];
  const int d = D.d, d2 = d * d;
  const int al = blockIdx.y, be = blockIdx.x * 256 + threadIdx.x;
  const int a = sector_of(D.offL, d, al), all = al - D.offL[a];
  double nrm = 0;
  if (be < D.chiR) {
    const int b = sector_of(D.offR, d, be), bel = be - D.offR[b];
    const int s = (b - a + d) % d;
    const double x = xi[al];
    for (int q = 0; q < d; ++q) {
      const int c = (a + q) % d, qq = (s - q + d) % d;
      const c128* Urow = U + (size_t)(q * d + qq) * d2;
      c128 acc = mk<double>(0, 0);
      for (int p = 0; p < d; ++p) {
        const int g = (a + p) % d;
        if (D.secM[g] == 0) continue;
        const int pp = (s - p + d) % d;
        const cpx<S>* T = (const cpx<S>*)Th0.p[g];
        const c128 v = ccast<double>(T[(size_t)(D.rowoff[g][p] + all) * D.cols[g] + D.coloff[g][pp] + bel]);
        acc = cadd(acc, cmul(Urow[p * d + pp], v));
      }
      const cpx<S> th = ccast<S>(cscale(acc, x));
      nrm += (double)th.re * th.re + (double)th.im * th.im;
      if (!C.p[c]) continue;   // a block that stays empty: its weight counts as truncated
      const size_t idx = (size_t)(D.rowoff[c][q] + all) * D.cols[c] + D.coloff[c][qq] + bel;
      ((cpx<S>*)C.p[c])[idx] = ccast<S>(acc);
      ((cpx<S>*)Th.p[c])[idx] = th;
    }
  }
  nrm = block_sum(nrm, scr);
  if (threadIdx.x == 0) partial[(size_t)blockIdx.y * gridDim.x + blockIdx.x] = nrm;
}

// Dense B~^[m] [chiL][d][chi~] from the blocks' (rows_c x chi_c, compact) results.
template <typename S>
__global__ __launch_bounds__(256) void sym_scatter_m_kernel(SymDims D, SymPtrs Bm, const int* __restrict__ chi,
                                                            const int* __restrict__ offs, const int* chi_tot,
                                                            cpx<S>* out) {
  __shared__ int on[kSymMaxD + 1];
  __shared__ int ch[kSymMaxD];
  if (threadIdx.x <= D.d) on[threadIdx.x] = offs[threadIdx.x];
  if (threadIdx.x < D.d) ch[threadIdx.x] = chi[threadIdx.x];
  __syncthreads();
  const int K = *chi_tot, d = D.d;
  const long long n = (long long)D.chiL * d * K;
  for (long long e = blockIdx.x * 256ll + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
    const int mu = (int)(e % K);
    const long long t = e / K;
    const int q = (int)(t % d), al = (int)(t / d);
    const int a = sector_of(D.offL, d, al), c = sector_of(on, d, mu);
    cpx<S> v = mk<S>(0, 0);
    if ((a + q) % d == c) v = ((const cpx<S>*)Bm.p[c])[(size_t)(D.rowoff[c][q] + al - D.offL[a]) * ch[c] + (mu - on[c])];
    out[e] = v;
  }
}

// Dense B~^[n] [chi~][d][chiR] from the blocks' (chi_c x cols_c) results.
template <typename S>
__global__ __launch_bounds__(256) void sym_scatter_n_kernel(SymDims D, SymPtrs Bn, const int* __restrict__ offs,
                                                            const int* chi_tot, cpx<S>* out) {
  __shared__ int on[kSymMaxD + 1];
  if (threadIdx.x <= D.d) on[threadIdx.x] = offs[threadIdx.x];
  __syncthreads();
  const int K = *chi_tot, d = D.d;
  const long long n = (long long)K * d * D.chiR;
  for (long long e = blockIdx.x * 256ll + threadIdx.x; e < n; e += (long long)gridDim.x * 256) {
    const int be = (int)(e % D.chiR);
    const long long t = e / D.chiR;
    const int q = (int)(t % d), mu = (int)(t / d);
    const int c = sector_of(on, d, mu), b = sector_of(D.offR, d, be);
    cpx<S> v = mk<S>(0, 0);
    if ((c + q) % d == b)
      v = ((const cpx<S>*)Bn.p[c])[(size_t)(mu - on[c]) * D.cols[c] + D.coloff[c][q] + (be - D.offR[b])];
    out[e] = v;
  }
}

struct SymBufs {
  void* M[kSymMaxD];
  void* N[kSymMaxD];
  void* T[kSymMaxD];
  void* ws[kSymMaxD];
  void* bmo[kSymMaxD];
  void* bno[kSymMaxD];
  double* partial;
  double* norm2;
  int* offs;
  size_t total;
};

inline int gate_blocks_x(const SymDims& D) { return (D.chiR + 255) / 256; }

SymBufs sym_carve(const SymPlan& p, void* base) {
  const SymDims& D = p.D;
  const size_t es = p.prec == 0 ? 16 : 8;
  char* c = (char*)base;
  auto take = [&](size_t b) {
    void* r = c;
    c += a256(b);
    return r;
  };
  SymBufs o{};
  for (int g = 0; g < D.d; ++g) {
    const bool th = D.secM[g] > 0 && D.rows[g] > 0 && D.cols[g] > 0;
    o.M[g] = take(th ? (size_t)D.rows[g] * D.secM[g] * es : 0);
    o.N[g] = take(th ? (size_t)D.secM[g] * D.cols[g] * es : 0);
    o.T[g] = take(th ? (size_t)D.rows[g] * D.cols[g] * es : 0);
  }
  for (int k = 0; k < D.d; ++k) {
    if (p.eta[k] == 0) continue;
    const size_t cap = p.blk[k].cap();
    o.ws[k] = take(bond_work_bytes(p.blk[k]));
    o.bmo[k] = take((size_t)D.rows[k] * cap * es);
    o.bno[k] = take(cap * D.cols[k] * es);
  }
  o.partial = (double*)take((size_t)gate_blocks_x(D) * std::max(1, D.chiL) * 8);
  o.norm2 = (double*)take(8);
  o.offs = (int*)take((kSymMaxD + 1) * 4);
  o.total = (size_t)(c - (char*)base);
  return o;
}

template <typename S>
int run_sym(const SymPlan& p, void* ws, int* status, const double* xi_m, const void* b_m, const void* b_n,
            const c128* u, void* b_m_out, double* xi_out, void* b_n_out, int* sec_out, int* chi_new, double* eps,
            hipStream_t s, const QrAsync* as) {
  const SymDims& D = p.D;
  const int dt = sizeof(S) == 8 ? DT_C128 : DT_C64;
  const SymBufs w = sym_carve(p, ws);
  int rc;
  SymPtrs Mp{}, Np{}, Tp{}, Cp{}, Hp{}, Bmo{}, Bno{};
  std::vector<GemmProb> g;
  for (int k = 0; k < D.d; ++k) {
    Mp.p[k] = w.M[k];
    Np.p[k] = w.N[k];
    Tp.p[k] = w.T[k];
    Bmo.p[k] = w.bmo[k];
    Bno.p[k] = w.bno[k];
    if (D.secM[k] > 0 && D.rows[k] > 0 && D.cols[k] > 0)
      g.push_back(gemm_prob(w.M[k], D.secM[k], OP_N, w.N[k], D.cols[k], OP_N, w.T[k], D.cols[k], D.rows[k],
                            D.cols[k], D.secM[k]));
  }
  // blocks of B^[m] and B^[n], Theta_g = M_g N_g
  hipLaunchKernelGGL(sym_gather_m_kernel<S>, dim3(grid_n((long long)D.chiL * D.d * D.chiM)), dim3(256), 0, s,
                     (const cpx<S>*)b_m, D, Mp);
  QT_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(sym_gather_n_kernel<S>, dim3(grid_n((long long)D.chiM * D.d * D.chiR)), dim3(256), 0, s,
                     (const cpx<S>*)b_n, D, Np);
  QT_HIP_CHECK(hipGetLastError());
  if (!g.empty() && (rc = gemm_run(g.data(), (int)g.size(), GemmTypes{dt, dt}, s, true))) return rc;
  // gate and Xi into the blocks' workspaces
  SymSelect sel{};
  sel.n = D.d;
  std::vector<BondCall> calls;
  for (int k = 0; k < D.d; ++k) {
    if (p.eta[k] == 0) continue;
    double* lam = nullptr;
    bond_pre_views(p.blk[k], w.ws[k], &Cp.p[k], &Hp.p[k], &lam);
    sel.lam[k] = lam;
    sel.kw[k] = p.blk[k].cap();
    BondCall c{p.blk[k], w.ws[k], status, nullptr, nullptr, nullptr, nullptr, w.bmo[k], nullptr, w.bno[k],
               sec_out + k, eps};
    c.sym = &sel;
    calls.push_back(c);
  }
  if (calls.empty()) return set_error(-1, "sym: no block with rows and columns");
  const dim3 gg(gate_blocks_x(D), D.chiL);
  hipLaunchKernelGGL(sym_gate_kernel<S>, gg, dim3(256), 0, s, D, Tp, Cp, Hp, u, xi_m, w.partial);
  QT_HIP_CHECK(hipGetLastError());
  if ((rc = reduce_partials(w.partial, (int)(gg.x * gg.y), w.norm2, s))) return rc;
  sel.chi = sec_out;
  sel.offs = w.offs;
  sel.chi_tot = chi_new;
  sel.xi = xi_out;
  sel.norm2 = w.norm2;
  sel.eps = eps;
  sel.status = status;
  sel.svd_min = p.svd_min;
  sel.chi_max = p.chi_max;
  // steps (i)-(v) on every block, one truncation over all of them
  if ((rc = bond_update_batch(calls.data(), (int)calls.size(), s, nullptr, as))) return rc;
  // back into dense charge-ordered tensors
  hipLaunchKernelGGL(sym_scatter_m_kernel<S>, dim3(grid_n((long long)D.chiL * D.d * p.cap)), dim3(256), 0, s, D,
                     Bmo, sec_out, w.offs, chi_new, (cpx<S>*)b_m_out);
  QT_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(sym_scatter_n_kernel<S>, dim3(grid_n((long long)p.cap * D.d * D.chiR)), dim3(256), 0, s, D, Bno,
                     w.offs, chi_new, (cpx<S>*)b_n_out);
  QT_HIP_CHECK(hipGetLastError());
  return 0;
}

}  // namespace

int sym_plan(const SymShape& s, SymPlan* out) {
  const int d = s.d;
  if (d < 2 || d > kSymMaxD) return set_error(MPS_ERR_ARG, "sym: d=%d outside [2, %d]", d, kSymMaxD);
  if (s.prec < 0 || s.prec > 1) return set_error(MPS_ERR_ARG, "sym: unknown precision %d", s.prec);
  if (s.chi_max < 1 || !(s.svd_min >= 0) || s.dchi_min < 0 || !(s.dchi_frac >= 0))
    return set_error(MPS_ERR_ARG, "sym: bad policy (chi_max=%d svd_min=%g dchi_min=%d dchi_frac=%g)", s.chi_max,
                     s.svd_min, s.dchi_min, s.dchi_frac);
  SymPlan p{};
  SymDims& D = p.D;
  D.d = d;
  for (int a = 0; a < d; ++a)
    if (s.sec_l[a] < 0 || s.sec_m[a] < 0 || s.sec_r[a] < 0) return set_error(MPS_ERR_ARG, "sym: negative sector size");
  for (int a = 0; a < d; ++a) {
    D.offL[a + 1] = D.offL[a] + s.sec_l[a];
    D.offM[a + 1] = D.offM[a] + s.sec_m[a];
    D.offR[a + 1] = D.offR[a] + s.sec_r[a];
    D.secM[a] = s.sec_m[a];
  }
  D.chiL = D.offL[d];
  D.chiM = D.offM[d];
  D.chiR = D.offR[d];
  if (D.chiL < 1 || D.chiM < 1 || D.chiR < 1) return set_error(MPS_ERR_ARG, "sym: every bond needs a sector");
  int capsum = 0;
  for (int c = 0; c < d; ++c) {
    int r = 0, k = 0;
    for (int q = 0; q < d; ++q) {
      D.rowoff[c][q] = r;
      r += s.sec_l[(c - q + d) % d];
      D.coloff[c][q] = k;
      k += s.sec_r[(c + q) % d];
    }
    D.rows[c] = r;
    D.cols[c] = k;
    if (r == 0 || k == 0) {
      p.eta[c] = 0;
      continue;
    }
    const int grow = std::max(s.dchi_min, (int)std::ceil(s.dchi_frac * s.sec_m[c]));
    p.eta[c] = std::min({s.sec_m[c] + grow, r, k});
    if (p.eta[c] == 0) continue;   // an empty block that is not expanded stays empty
    if (std::max(r, k) > kMaxQrRows) return set_error(MPS_ERR_CAPACITY, "sym: block of %d rows too large", std::max(r, k));
    if (p.eta[c] > kEigMaxN) return set_error(MPS_ERR_CAPACITY, "sym: eta_c=%d > %d", p.eta[c], kEigMaxN);
    BondShape& b = p.blk[c];
    b.d = 1;
    b.chi_l = r;
    b.chi_m = std::max(1, s.sec_m[c]);
    b.chi_r = k;
    b.eta = p.eta[c];
    b.chi_max = s.chi_max;
    b.svd_min = s.svd_min;
    b.xi_is_diag = 1;
    b.mode = 2;
    b.prec = s.prec;
    b.sweeps = 1;
    b.pre = 1;
    capsum += b.cap();
  }
  p.cap = std::max(1, std::min(s.chi_max, capsum));
  p.prec = s.prec;
  p.svd_min = s.svd_min;
  p.chi_max = s.chi_max;
  *out = p;
  return 0;
}

size_t sym_work_bytes(const SymPlan& p) { return sym_carve(p, nullptr).total + 256; }

int sym_update_run(const SymPlan& p, void* ws, int* status, const double* xi_m, const void* b_m, const void* b_n,
                   const c128* u, void* b_m_out, double* xi_out, void* b_n_out, int* sec_out, int* chi_new,
                   double* eps, hipStream_t s, const QrAsync* as) {
  return p.prec == 0 ? run_sym<double>(p, ws, status, xi_m, b_m, b_n, u, b_m_out, xi_out, b_n_out, sec_out, chi_new,
                                       eps, s, as)
                     : run_sym<float>(p, ws, status, xi_m, b_m, b_n, u, b_m_out, xi_out, b_n_out, sec_out, chi_new,
                                      eps, s, as);
}

}  // namespace qrtebd
