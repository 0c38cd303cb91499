// Observables of an MPS in right-isometric form (Fig. 1c of the paper) and
// of the two-site wave functions: <O_m> = sum conj(M) O M / |M|^2 with
// M = Xi^[m] B^[m], bond values of a (d^2 x d^2) operator from
// theta = Xi^[m] B^[m] B^[n], and von Neumann entropies of diagonal Xi.
#include "measure.h"

#include <algorithm>
#include <cmath>

namespace qrtebd {
namespace {

// One block per row alpha and W columns beta of a site tensor [chiL][d][chiR]
// (or of a two-site tensor with d -> d^2): partial sums of
// num = sum conj(M_o) sum_q O[o][q] M_q and den = sum |M_o|^2, M = x_alpha T.
// The dd inputs of every column are staged in LDS; 256 threads in R = 256 / W
// groups, thread (column t % W, group t / W) takes the outputs o = group,
// group + R, ...  W is 64, 32 or 16, the widest whose staged block leaves
// room for three workgroups per CU.
template <typename S>
__global__ __launch_bounds__(256) void expect_kernel(const cpx<S>* T, const double* xi, int chiL, int dd, int chiR,
                                                     int W, const c128* __restrict__ O, double* part) {
  extern __shared__ c128 Ms[];  // dd x W
  __shared__ double scr[4];
  const int t = threadIdx.x, R = 256 / W, col = t % W, grp = t / W;
  const int alpha = blockIdx.y, beta = blockIdx.x * W + col;
  const bool live = beta < chiR;
  const double x = xi ? xi[alpha] : 1.0;
  const long long base = (long long)alpha * dd * chiR;
  double den = 0;
  for (int q = grp; q < dd; q += R) {
    const c128 m = live ? cscale(ccast<double>(T[base + (long long)q * chiR + beta]), x) : mk<double>(0, 0);
    Ms[q * W + col] = m;
    den += cabs2(m);
  }
  __syncthreads();
  c128 num = mk<double>(0, 0);
  if (live)
    for (int o = grp; o < dd; o += R) {
      c128 acc = mk<double>(0, 0);
      for (int q = 0; q < dd; ++q) acc = cadd(acc, cmul(O[o * dd + q], Ms[q * W + col]));
      num = cadd(num, cmulc(Ms[o * W + col], acc));
    }
  num.re = block_sum(num.re, scr);
  num.im = block_sum(num.im, scr);
  den = block_sum(den, scr);
  if (t == 0) {
    const long long b = (long long)blockIdx.y * gridDim.x + blockIdx.x;
    part[3 * b + 0] = num.re;
    part[3 * b + 1] = num.im;
    part[3 * b + 2] = den;
  }
}

constexpr int kExpectMaxLds = 160 * 1024 - 256;   // LDS less the kernel's static block sums
inline int expect_width(int dd) {
  int W = 64;
  while (W > 16 && (size_t)dd * W * sizeof(c128) > 48 * 1024) W /= 2;
  return W;
}

__global__ __launch_bounds__(256) void expect_finish_kernel(const double* part, int nb, double* val, double* norm) {
  __shared__ double scr[4];
  double a = 0, b = 0, c = 0;
  for (int i = threadIdx.x; i < nb; i += 256) {
    a += part[3 * i];
    b += part[3 * i + 1];
    c += part[3 * i + 2];
  }
  a = block_sum(a, scr);
  b = block_sum(b, scr);
  c = block_sum(c, scr);
  if (threadIdx.x == 0) {
    if (val) {
      val[0] = a / c;
      val[1] = b / c;
    }
    if (norm) *norm = c;
  }
}

__global__ __launch_bounds__(256) void entropy_kernel(EntropyArgs a, double* out) {
  __shared__ double scr[4];
  const int m = blockIdx.x;
  const double* x = a.xi[m];
  const int n = a.chi[m];
  double s2 = 0;
  for (int k = threadIdx.x; k < n; k += 256) s2 += x[k] * x[k];
  s2 = block_sum(s2, scr);
  double h = 0;
  for (int k = threadIdx.x; k < n; k += 256) {
    const double p = x[k] * x[k] / s2;
    if (p > 0) h -= p * log(p);
  }
  h = block_sum(h, scr);
  if (threadIdx.x == 0) out[m] = h;
}

}  // namespace

size_t expect_part_doubles(int chiL, int chiR) { return 3 * (size_t)chiL * ((chiR + 15) / 16) + 3; }

int expect_run(const void* T, int prec, const double* xi, int chiL, int dd, int chiR, const c128* O, double* part,
               double* val, double* norm, hipStream_t s) {
  const int W = expect_width(dd);
  const dim3 grid((chiR + W - 1) / W, chiL);
  const size_t shm = (size_t)dd * W * sizeof(c128);
  if (shm > (size_t)kExpectMaxLds) return set_error(-2, "expect: local dimension %d too large", dd);
  static bool attr[2] = {false, false};
  if (!attr[prec ? 1 : 0]) {
    if (prec)
      QT_HIP_CHECK(hipFuncSetAttribute((const void*)expect_kernel<float>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       kExpectMaxLds));
    else
      QT_HIP_CHECK(hipFuncSetAttribute((const void*)expect_kernel<double>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, kExpectMaxLds));
    attr[prec ? 1 : 0] = true;
  }
  if (prec)
    hipLaunchKernelGGL(expect_kernel<float>, grid, dim3(256), shm, s, (const c64*)T, xi, chiL, dd, chiR, W, O, part);
  else
    hipLaunchKernelGGL(expect_kernel<double>, grid, dim3(256), shm, s, (const c128*)T, xi, chiL, dd, chiR, W, O,
                       part);
  QT_HIP_CHECK(hipGetLastError());
  hipLaunchKernelGGL(expect_finish_kernel, dim3(1), dim3(256), 0, s, part, (int)(grid.x * grid.y), val, norm);
  QT_HIP_CHECK(hipGetLastError());
  return 0;
}

int entropy_run(const EntropyArgs& a, int n, double* out, hipStream_t s) {
  if (n <= 0) return 0;
  hipLaunchKernelGGL(entropy_kernel, dim3(n), dim3(256), 0, s, a, out);
  QT_HIP_CHECK(hipGetLastError());
  return 0;
}

}  // namespace qrtebd
