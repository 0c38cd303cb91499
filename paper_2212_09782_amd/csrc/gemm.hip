// Grouped complex GEMM on CDNA4 matrix cores.
//
// Every contraction of the bond update (theta, X, Y, L^dag L, the new tensors,
// the compact-WY trailing updates of the Householder QR) is a complex matrix
// product, formed from three real MFMA products (Gauss' form: P1 = Re A Re B,
// P2 = Im A Im B, P3 = (Re A + Im A)(Re B + Im B), Re C = P1 - P2,
// Im C = P3 - P1 - P2) instead of four.  FP64 runs on v_mfma_f64_16x16x4f64,
// FP32 on v_mfma_f32_16x16x4f32, both with their native accumulator.  The
// rounding of the form is that of the four-product one up to a constant
// (|err Im C| <= ~3 u sum |Re A + Im A| |Re B + Im B| per term).
//
// Tiling: a 256-thread workgroup owns a 64x64 output tile, each wave a 32x32
// quadrant (2x2 MFMA blocks, one accumulator set per real product).  Operand
// tiles of depth 16 are staged through LDS as re and im planes, [m][k] rows
// with k contiguous, so that a lane reads the four k values of its MFMA steps
// with one vector read per plane and forms re + im in registers.  LDS is
// double-buffered: the next tile is loaded from global memory into registers
// and stored into the other buffer while the current one is consumed, so each
// K stage needs one workgroup barrier.  Workgroup ids are remapped so that the
// 8 XCDs (which take workgroups round-robin) each work on a contiguous range
// of tiles and share operands in their own L2.
#include "gemm.h"

#include <algorithm>

namespace qrtebd {
namespace {

// Tile order within a launch: columns of kTileGroup-tall groups of tiles, so
// that the workgroups running together on one XCD (which receives a
// contiguous range of tiles) share A row panels and B column panels in its
// L2 instead of streaming all of A once per tile column.
constexpr int kTileGroup = 8;
__device__ inline void grouped_tile(int t, int tm, int tn, int& tile_m, int& tile_n) {
  const int per_group = kTileGroup * tn;
  const int g = t / per_group, first_m = g * kTileGroup;
  const int gsize = min(tm - first_m, kTileGroup);
  const int r = t - g * per_group;
  tile_m = first_m + r % gsize;
  tile_n = r / gsize;
}

template <typename T> struct Mfma;
template <> struct Mfma<double> {
  typedef double v4 __attribute__((ext_vector_type(4)));
  __device__ static inline v4 op(double a, double b, v4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  // output row held by (lane, item r) of a 16x16 block
  __device__ static inline int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <> struct Mfma<float> {
  typedef float v4 __attribute__((ext_vector_type(4)));
  __device__ static inline v4 op(float a, float b, v4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};

constexpr int BM = 64, BN = 64, BK = 16;

template <typename Tin, typename Tout, typename Tc>
__device__ __forceinline__ void gemm_body(const GemmBatch& b) {
  using MF = Mfma<Tc>;
  using v4 = typename MF::v4;
  // Three accumulator sets (P1, P2, P3).  FP64 fits two waves per SIMD with
  // them (205 registers; 80 KiB of LDS per workgroup, two workgroups per CU).
  constexpr int NPL = 3;
  // LDS holds the re and im planes of each operand tile, double-buffered, as
  // [m][k] rows with k contiguous (stride BK + 4), so a lane reads the four k
  // values of its four MFMA steps with one vector read per plane (the steps
  // take k = 4 (lane / 16) + s, the same for A and B); re + im is formed in
  // registers.
  constexpr int KS = BK + 4;
  __shared__ __attribute__((aligned(16))) Tc As[2][2][BM][KS];
  __shared__ __attribute__((aligned(16))) Tc Bs[2][2][BN][KS];

  // XCD-aware remap: hardware workgroup g runs on XCD g % 8; give XCD x the
  // contiguous logical range [start_x, start_x + count_x)
  int bid;
  {
    const int total = b.tile_start[b.nprob];
    const int g = blockIdx.x, x = g & 7, loc = g >> 3;
    const int q = total >> 3, r = total & 7;
    bid = x < r ? x * (q + 1) + loc : r * (q + 1) + (x - r) * q + loc;
  }
  int p = 0;
  while (p + 1 < b.nprob && bid >= b.tile_start[p + 1]) ++p;
  const GemmProb& P = b.p[p];
  int t = bid - b.tile_start[p];
  const int tm = b.tiles_m[p], tn = b.tiles_n[p];
  const int split = t / (tm * tn);
  t -= split * tm * tn;
  int tile_m, tile_n;
  grouped_tile(t, tm, tn, tile_m, tile_n);
  if (P.herm && tile_m > tile_n) return;   // Hermitian output: upper tiles only

  int M = P.M, N = P.N, K = P.K;
  if (P.dM) M = min(M, *P.dM);
  if (P.dN) N = min(N, *P.dN);
  if (P.dK) K = min(K, *P.dK);
  const int m0 = tile_m * BM, n0 = tile_n * BN;
  if (m0 >= M || n0 >= N) return;
  const int ks = P.ksplit > 1 ? P.ksplit : 1;
  const int kchunk = ((K + ks - 1) / ks + BK - 1) / BK * BK;
  const int kbeg = split * kchunk;
  const int kend = min(K, kbeg + kchunk);

  const cpx<Tin>* __restrict__ A = (const cpx<Tin>*)P.A;
  const cpx<Tin>* __restrict__ B = (const cpx<Tin>*)P.B;
  const long long lda = P.lda, ldb = P.ldb;
  const int opA = P.opA, opB = P.opB;
  const Tc sa = opA == OP_C ? Tc(-1) : Tc(1);
  const Tc sb = opB == OP_C ? Tc(-1) : Tc(1);

  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = (wid & 1) * 32, wn = (wid >> 1) * 32;

  v4 acc[NPL][2][2];   // P1, P2, P3
#pragma unroll
  for (int pl = 0; pl < NPL; ++pl)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[pl][i][j] = v4{0, 0, 0, 0};

  // thread -> tile element mapping: each thread stages EPT = 4 consecutive k
  // of one row of each operand per stage.  Operands stored m-major (A as
  // stored, B^T / B^H): 64 rows x BK k.  Operands stored k-major (A^T / A^H,
  // B as stored): lane -> m (or n), wave -> four consecutive k, so the global
  // loads stay coalesced (64 consecutive elements per load) and each lane
  // writes one row segment per plane, the conflict-free pattern of the reads.
  constexpr int EPT = BM * BK / 256;
  static_assert(EPT == 4, "one LDS row segment holds the four k values of a thread");
  cpx<Tin> ra[EPT], rb[EPT];
  const int rowq = tid >> 2, colq = (tid & 3) * (BK / 4);
  const int kml = tid & 63, kmk = 4 * (tid >> 6);

  auto load = [&](int k0) {
#pragma unroll
    for (int e = 0; e < EPT; ++e) {
      cpx<Tin> z = mk<Tin>(0, 0);
      if (opA == OP_N) {
        const int m = m0 + rowq, k = k0 + colq + e;
        if (m < M && k < kend) z = A[(long long)m * lda + k];
      } else {
        const int k = k0 + kmk + e, m = m0 + kml;
        if (m < M && k < kend) z = A[(long long)k * lda + m];
      }
      ra[e] = z;
      cpx<Tin> w = mk<Tin>(0, 0);
      if (opB == OP_N) {
        const int k = k0 + kmk + e, n = n0 + kml;
        if (n < N && k < kend) w = B[(long long)k * ldb + n];
      } else {
        const int n = n0 + rowq, k = k0 + colq + e;
        if (n < N && k < kend) w = B[(long long)n * ldb + k];
      }
      rb[e] = w;
    }
  };
  typedef Tc f4 __attribute__((ext_vector_type(4)));
  auto store = [&](int buf) {
    // four consecutive k of one row: one vector write per plane
    const int ar = opA == OP_N ? rowq : kml, ac = opA == OP_N ? colq : kmk;
    const int br = opB == OP_N ? kml : rowq, bc = opB == OP_N ? kmk : colq;
    *(f4*)&As[buf][0][ar][ac] = f4{(Tc)ra[0].re, (Tc)ra[1].re, (Tc)ra[2].re, (Tc)ra[3].re};
    *(f4*)&As[buf][1][ar][ac] = f4{sa * (Tc)ra[0].im, sa * (Tc)ra[1].im, sa * (Tc)ra[2].im, sa * (Tc)ra[3].im};
    *(f4*)&Bs[buf][0][br][bc] = f4{(Tc)rb[0].re, (Tc)rb[1].re, (Tc)rb[2].re, (Tc)rb[3].re};
    *(f4*)&Bs[buf][1][br][bc] = f4{sb * (Tc)rb[0].im, sb * (Tc)rb[1].im, sb * (Tc)rb[2].im, sb * (Tc)rb[3].im};
  };

  if (kbeg < kend) {
    load(kbeg);
    store(0);
  }
  __syncthreads();
  int buf = 0;
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    const bool more = k0 + BK < kend;
    if (more) load(k0 + BK);     // global -> registers, overlapping the MFMAs below
    {
      const int kq = 4 * (lane >> 4);
      f4 a2[2][2], b2[2][2];   // [re / im][block]: k = kq .. kq + 3
#pragma unroll
      for (int pl = 0; pl < 2; ++pl)
#pragma unroll
        for (int i = 0; i < 2; ++i) {
          a2[pl][i] = *(const f4*)&As[buf][pl][wm + i * 16 + (lane & 15)][kq];
          b2[pl][i] = *(const f4*)&Bs[buf][pl][wn + i * 16 + (lane & 15)][kq];
        }
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) {
            const Tc ar = a2[0][i][s4], ai = a2[1][i][s4], br = b2[0][j][s4], bi = b2[1][j][s4];
            acc[0][i][j] = MF::op(ar, br, acc[0][i][j]);
            acc[1][i][j] = MF::op(ai, bi, acc[1][i][j]);
            acc[2][i][j] = MF::op(ar + ai, br + bi, acc[2][i][j]);
          }
    }
    if (more) store(buf ^ 1);    // the other buffer was released by the previous barrier
    __syncthreads();
    buf ^= 1;
  }

  // epilogue: the real and imaginary parts
  v4 acc_re[2][2], acc_im[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      acc_re[i][j] = acc[0][i][j] - acc[1][i][j];
      acc_im[i][j] = acc[2][i][j] - acc[0][i][j] - acc[1][i][j];
    }
  if (ks > 1) {
    cpx<Tc>* W = (cpx<Tc>*)P.work + (long long)split * P.M * P.N;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = m0 + wm + i * 16 + MF::row(lane, r);
          const int col = n0 + wn + j * 16 + (lane & 15);
          if (row < M && col < N) W[(long long)row * P.N + col] = mk<Tc>(acc_re[i][j][r], acc_im[i][j][r]);
        }
    return;
  }
  cpx<Tout>* C = (cpx<Tout>*)P.C;
  const long long ldc = P.ldc_live_N ? (long long)N : P.ldc;
  const Tc alpha = (Tc)P.alpha, beta = (Tc)P.beta;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm + i * 16 + MF::row(lane, r);
        const int col = n0 + wn + j * 16 + (lane & 15);
        if (row < M && col < N) {
          Tc vr = alpha * acc_re[i][j][r], vi = alpha * acc_im[i][j][r];
          cpx<Tout>* c = C + (long long)row * ldc + col;
          if (beta != Tc(0)) {
            const cpx<Tout> o = *c;
            vr += beta * (Tc)o.re;
            vi += beta * (Tc)o.im;
          }
          *c = mk<Tout>((Tout)vr, (Tout)vi);
        }
      }
}

// Two entry points with the same body: the contractions of the bond update
// (the dominant kernel, reported on its own by profilers) and all other
// products (QR trailing updates, explicit Q, Gram matrices).
// Occupancy floors: FP64 two waves per SIMD, FP32 three (both fit without
// spills; fewer waves left the matrix cores idle during staging).
template <typename Tin, typename Tout, typename Tc>
__global__ __launch_bounds__(256, sizeof(Tc) == 8 ? 2 : 3) void gemm_kernel(GemmBatch b) { gemm_body<Tin, Tout, Tc>(b); }
template <typename Tin, typename Tout, typename Tc>
__global__ __launch_bounds__(256, sizeof(Tc) == 8 ? 2 : 3) void contract_gemm_kernel(GemmBatch b) {
  gemm_body<Tin, Tout, Tc>(b);
}

// C = alpha * sum_s work[s] + beta * C over the live M x N, for every problem
// of a batch at once: problem p owns workgroups [tile_start[p], tile_start[p+1]).
template <typename Tout, typename Tc>
__global__ __launch_bounds__(256) void splitk_reduce_kernel(GemmBatch b) {
  const int bid = blockIdx.x;
  int p = 0;
  while (p + 1 < b.nprob && bid >= b.tile_start[p + 1]) ++p;
  const GemmProb& P = b.p[p];
  const int nblk = b.tile_start[p + 1] - b.tile_start[p];
  int M = P.M, N = P.N;
  if (P.dM) M = min(M, *P.dM);
  if (P.dN) N = min(N, *P.dN);
  // 32-bit element index (M N < 2^31 for every product here): a 64-bit
  // division per element would cost more than its memory traffic
  const unsigned total = (unsigned)M * (unsigned)N, un = N;
  const long long ldc = P.ldc_live_N ? (long long)N : P.ldc;
  const cpx<Tc>* W = (const cpx<Tc>*)P.work;
  cpx<Tout>* C = (cpx<Tout>*)P.C;
  const Tc alpha = (Tc)P.alpha, beta = (Tc)P.beta;
  for (unsigned idx = (bid - b.tile_start[p]) * 256u + threadIdx.x; idx < total; idx += nblk * 256u) {
    const int row = (int)(idx / un), col = (int)(idx - (unsigned)row * un);
    Tc sr = 0, si = 0;
    for (int s = 0; s < P.ksplit; ++s) {
      const cpx<Tc> w = W[((long long)s * P.M + row) * P.N + col];
      sr += w.re;
      si += w.im;
    }
    sr *= alpha;
    si *= alpha;
    cpx<Tout>* c = C + (long long)row * ldc + col;
    if (beta != Tc(0)) {
      const cpx<Tout> o = *c;
      sr += beta * (Tc)o.re;
      si += beta * (Tc)o.im;
    }
    *c = mk<Tout>((Tout)sr, (Tout)si);
  }
}

template <typename Tin, typename Tout, typename Tc>
int launch_typed(const GemmProb* probs, int nprob, hipStream_t stream, bool contract) {
  int i = 0;
  while (i < nprob) {
    GemmBatch b{};
    int total = 0;
    b.nprob = 0;
    while (i < nprob && b.nprob < kGemmMaxProb) {
      const GemmProb& q = probs[i++];
      if (q.M <= 0 || q.N <= 0) continue;
      const int tm = (q.M + BM - 1) / BM, tn = (q.N + BN - 1) / BN;
      const int ks = q.ksplit > 1 ? q.ksplit : 1;
      b.p[b.nprob] = q;
      b.tiles_m[b.nprob] = tm;
      b.tiles_n[b.nprob] = tn;
      b.tile_start[b.nprob] = total;
      total += tm * tn * ks;
      b.nprob++;
    }
    if (b.nprob == 0) continue;
    b.tile_start[b.nprob] = total;
    if (contract)
      hipLaunchKernelGGL((contract_gemm_kernel<Tin, Tout, Tc>), dim3(total), dim3(256), 0, stream, b);
    else
      hipLaunchKernelGGL((gemm_kernel<Tin, Tout, Tc>), dim3(total), dim3(256), 0, stream, b);
    QT_HIP_CHECK(hipGetLastError());
    // one launch reduces the split-K partials of every problem of the batch
    GemmBatch r{};
    int nblk = 0;
    for (int q = 0; q < b.nprob; ++q) {
      const GemmProb& pr = b.p[q];
      if (pr.ksplit > 1 && !pr.skip_reduce) {
        const long long tot = (long long)pr.M * pr.N;
        r.p[r.nprob] = pr;
        r.tile_start[r.nprob++] = nblk;
        nblk += (int)std::min<long long>((tot + 255) / 256, 4096);
      }
    }
    if (r.nprob) {
      r.tile_start[r.nprob] = nblk;
      hipLaunchKernelGGL((splitk_reduce_kernel<Tout, Tc>), dim3(nblk), dim3(256), 0, stream, r);
      QT_HIP_CHECK(hipGetLastError());
    }
  }
  return 0;
}

// Lower triangle from the upper one: 32 x 32 blocks below the diagonal,
// read transposed through LDS.
__global__ __launch_bounds__(256) void herm_fill_kernel(c128* C, long long ldc, int n) {
  __shared__ c128 tile[32][33];
  const int bi = blockIdx.y, bj = blockIdx.x;   // destination block (bi >= bj)
  if (bj > bi) return;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {   // source block (bj, bi): rows bj*32 + r
    const int i = bj * 32 + r, j = bi * 32 + tx;
    if (i < n && j < n) tile[r][tx] = C[(long long)i * ldc + j];
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int i = bi * 32 + r, j = bj * 32 + tx;
    if (i < n && j < n && i > j) C[(long long)i * ldc + j] = cconj(tile[tx][r]);
  }
}

}  // namespace

int herm_fill_lower(c128* C, long long ldc, int n, hipStream_t stream) {
  if (n <= 1) return 0;
  const int nb = (n + 31) / 32;
  hipLaunchKernelGGL(herm_fill_kernel, dim3(nb, nb), dim3(256), 0, stream, C, ldc, n);
  QT_HIP_CHECK(hipGetLastError());
  return 0;
}

int gemm_run(const GemmProb* probs, int nprob, GemmTypes ty, hipStream_t stream, bool contract) {
  if (ty.tin == DT_C128 && ty.tout == DT_C128)
    return launch_typed<double, double, double>(probs, nprob, stream, contract);
  if (ty.tin == DT_C64 && ty.tout == DT_C64) return launch_typed<float, float, float>(probs, nprob, stream, contract);
  if (ty.tin == DT_C64 && ty.tout == DT_C128)
    return launch_typed<float, double, double>(probs, nprob, stream, contract);
  return set_error(-1, "gemm_run: unsupported type combination %d/%d", ty.tin, ty.tout);
}

}  // namespace qrtebd
