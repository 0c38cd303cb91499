// Shared device/host helpers of the QR-TEBD library (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace qrtebd {

// Interleaved complex scalar, the memory layout of complex64 / complex128.
template <typename T> struct alignas(2 * sizeof(T)) cpx { T re, im; };
using c64 = cpx<float>;
using c128 = cpx<double>;

template <typename T> __host__ __device__ inline cpx<T> mk(T r, T i) { cpx<T> z; z.re = r; z.im = i; return z; }
template <typename T> __host__ __device__ inline cpx<T> cadd(cpx<T> a, cpx<T> b) { return mk(a.re + b.re, a.im + b.im); }
template <typename T> __host__ __device__ inline cpx<T> csub(cpx<T> a, cpx<T> b) { return mk(a.re - b.re, a.im - b.im); }
template <typename T> __host__ __device__ inline cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
// conj(a) * b
template <typename T> __host__ __device__ inline cpx<T> cmulc(cpx<T> a, cpx<T> b) {
  return mk(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re);
}
template <typename T> __host__ __device__ inline cpx<T> cconj(cpx<T> a) { return mk(a.re, -a.im); }
template <typename T> __host__ __device__ inline cpx<T> cscale(cpx<T> a, T s) { return mk(a.re * s, a.im * s); }
template <typename T> __host__ __device__ inline T cabs2(cpx<T> a) { return a.re * a.re + a.im * a.im; }

template <typename D, typename S> __host__ __device__ inline cpx<D> ccast(cpx<S> a) {
  return mk<D>((D)a.re, (D)a.im);
}

// Error bits latched in the device status word.
enum : int {
  ERRBIT_BARRIER = 1,    // a grid barrier spun past its limit
  ERRBIT_NONFINITE = 2,  // NaN / Inf met in a norm or spectrum
  ERRBIT_ZERONORM = 4,   // a two-site wave function of zero norm
  ERRBIT_CAPACITY = 8,   // a live dimension exceeded its capacity
};

__device__ inline void latch_error(int* status, int bit) {
  if (status) atomicOr(status, bit);
}

// 1/x from the hardware reciprocal refined by two Newton steps (within an ulp
// or two of the rounded quotient) for finite, nonzero, normal x.
__device__ inline double rcp_refined(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}

// 1/sqrt(x) for x > 0: the hardware estimate plus two Newton steps
// y <- y (3 - x y^2) / 2.
__device__ inline double rsq_refined(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = y * fma(-0.5 * x * y, y, 1.5);
  return y * fma(-0.5 * x * y, y, 1.5);
}

// ---------------------------------------------------------------- reductions
// Lane moves inside the VALU (DPP), no LDS traffic.  Lanes whose source is
// outside the row, or whose row is masked off, receive 0.
template <int CTRL, int ROW_MASK = 0xf, bool BOUND = false>
__device__ inline double dpp_mov(double x) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(x), CTRL, ROW_MASK, 0xf, BOUND);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(x), CTRL, ROW_MASK, 0xf, BOUND);
  return __hiloint2double(hi, lo);
}
template <int CTRL, int ROW_MASK = 0xf, bool BOUND = false>
__device__ inline float dpp_mov(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, ROW_MASK, 0xf, BOUND));
}
__device__ inline double lane_read(double x, int l) {
  return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(x), l),
                          __builtin_amdgcn_readlane(__double2loint(x), l));
}
__device__ inline float lane_read(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

// Sum over each row of 16 lanes: lane 16 r + 15 ends with row r's total
// (quad swaps, then shifts by 4 and 8 within the row).
template <typename T>
__device__ inline T row16_sum(T v) {
  v += dpp_mov<0xb1>(v);              // quad_perm [1,0,3,2]
  v += dpp_mov<0x4e>(v);              // quad_perm [2,3,0,1]
  v += dpp_mov<0x114, 0xf, true>(v);  // row_shr:4
  v += dpp_mov<0x118, 0xf, true>(v);  // row_shr:8
  return v;
}
// Sum over the wave left in lane 63 (row totals combined by row broadcasts).
template <typename T>
__device__ inline T wave_sum_to63(T v) {
  v = row16_sum(v);
  v += dpp_mov<0x142, 0xa>(v);        // row_bcast:15 into rows 1 and 3
  v += dpp_mov<0x143, 0xc>(v);        // row_bcast:31 into rows 2 and 3
  return v;
}
// Wave sums of 16 values at once by halving: each step pairs two values,
// every lane keeps one of them and adds the partner lane's copy of it
// (v_permlane32_swap: lanes l and l + 32; v_permlane16_swap: rows 2i and
// 2i + 1; DPP row_ror:8; DPP row_half_mirror), then quad sums.  Afterwards
// lane l holds the wave total of x[l >> 2] (fixed order).
__device__ inline double swap_sum32(double x, double y) {
  const auto lo = __builtin_amdgcn_permlane32_swap(__double2loint(x), __double2loint(y), false, false);
  const auto hi = __builtin_amdgcn_permlane32_swap(__double2hiint(x), __double2hiint(y), false, false);
  // first result: x in lanes 0-31, y's lanes 0-31 in lanes 32-63; second: the upper halves
  return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}
__device__ inline double swap_sum16(double x, double y) {
  const auto lo = __builtin_amdgcn_permlane16_swap(__double2loint(x), __double2loint(y), false, false);
  const auto hi = __builtin_amdgcn_permlane16_swap(__double2hiint(x), __double2hiint(y), false, false);
  // first result: rows (x0, y0, x2, y2), second: (x1, y1, x3, y3)
  return __hiloint2double(hi[0], lo[0]) + __hiloint2double(hi[1], lo[1]);
}
__device__ inline double wave_sum16(const double (&x)[16]) {
  const int lane = threadIdx.x & 63;
  double b[8], c[4], d[2];
#pragma unroll
  for (int e = 0; e < 8; ++e) b[e] = swap_sum32(x[e], x[e + 8]);   // half h keeps x[e + 8 h]
#pragma unroll
  for (int e = 0; e < 4; ++e) c[e] = swap_sum16(b[e], b[e + 4]);   // row parity j keeps b[e + 4 j]
  const bool b3 = lane & 8, b2 = lane & 4;
#pragma unroll
  for (int e = 0; e < 2; ++e) {                                   // lane bit 3 keeps c[e + 2 bit3]
    const double keep = b3 ? c[e + 2] : c[e], send = b3 ? c[e] : c[e + 2];
    d[e] = keep + dpp_mov<0x128>(send);                           // row_ror:8 (lane i ^ 8)
  }
  const double keep = b2 ? d[1] : d[0], send = b2 ? d[0] : d[1];  // lane bit 2 keeps d[bit2]
  double f = keep + dpp_mov<0x141>(send);                         // row_half_mirror (i <-> 7 - i)
  f += dpp_mov<0xb1>(f);                                          // quad sums
  f += dpp_mov<0x4e>(f);
  return f;
}

// Wave64 sum, every lane gets it (fixed order).
__device__ inline double wave_sum(double v) { return lane_read(wave_sum_to63(v), 63); }
__device__ inline float wave_sum(float v) { return lane_read(wave_sum_to63(v), 63); }
__device__ inline double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Block-wide sum of one double (all threads get the result).  scratch needs
// blockDim.x/64 doubles of LDS.  Contains two barriers.
__device__ inline double block_sum(double v, double* scratch) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v = wave_sum(v);
  __syncthreads();
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  double s = 0;
  for (int w = 0; w < nw; ++w) s += scratch[w];
  return s;
}

// ---------------------------------------------------------------- grid barrier
// Barrier among the blocks of one group of a cooperative launch, without
// cache write-back / invalidate fences:
//  * data that other blocks read after the barrier is written with
//    pub_store and read with pub_load (device-scope atomic accesses, which
//    bypass the non-coherent caches), from any wave;
//  * every wave waits until its own stores have completed, the block
//    synchronises, thread 0 publishes its arrival generation in its own cache
//    line, and the threads of every block poll all flags of the group.
// Spins are bounded: on timeout the block's smem_flag records the generation,
// the error bit is latched and false is returned so the kernel can leave.
// base holds 16*(nblk+1) words zeroed before the first barrier; generations
// must increase from one barrier to the next (they may continue across
// launches that use the same words).  smem_flag: a block-shared int the
// kernel zeroes once before its first barrier.
struct GridSync {
  unsigned* base;
  int* status;
};

__device__ inline void pub_store(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline double pub_load(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void pub_store(c128* p, c128 v) {
  pub_store(&p->re, v.re);
  pub_store(&p->im, v.im);
}
__device__ inline c128 pub_load(const c128* p) { return mk<double>(pub_load(&p->re), pub_load(&p->im)); }

// Published data read in one 16-byte access with the cache policy of the
// device-scope loads (past the non-coherent caches): a buffer resource over
// base (uniform), addressed by a per-lane element index.  Reads after a
// grid_barrier only: the access is not atomic.
__device__ inline __amdgpu_buffer_rsrc_t coh_rsrc(const void* base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, 0x7fffffff, 0x00020000);
}
__device__ inline c128 coh_load(__amdgpu_buffer_rsrc_t r, int elem) {
  typedef int i4 __attribute__((ext_vector_type(4)));
  typedef double d2 __attribute__((ext_vector_type(2)));
  const d2 x = __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(r, elem * 16, 0, 16));
  return mk<double>(x.x, x.y);
}

struct NoWork {
  __device__ void operator()() const {}
};
// idle: block-local work that every thread runs after its share of the flag
// polling and before the closing block barrier; threads past the polling
// range (threadIdx.x >= nblk) start it at once, so it overlaps the wait.  It
// may read what the block wrote before the call and write what nobody reads
// before the call returns.
template <typename F = NoWork>
__device__ inline bool grid_barrier(GridSync gs, unsigned gen, int blk, int nblk, int* smem_flag, F idle = F{}) {
  constexpr long kSpinLimit = 1L << 22;
  unsigned* flags = gs.base + 16;
  __builtin_amdgcn_s_waitcnt(0);   // this wave's published stores are complete
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(flags + 16 * blk, gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  for (int b = (int)threadIdx.x; b < nblk; b += blockDim.x) {
    long spins = 0;
    while (__hip_atomic_load(flags + 16 * b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < gen) {
      if (++spins > kSpinLimit) { *smem_flag = (int)gen; break; }
    }
  }
  idle();
  __syncthreads();
  const bool ok = *smem_flag != (int)gen;
  if (!ok && threadIdx.x == 0) latch_error(gs.status, ERRBIT_BARRIER);
  return ok;
}

// Words needed by grid_barrier for nblk blocks.
inline size_t grid_sync_words(int nblk) { return 16 * (size_t)(nblk + 1); }

// Launch shapes chosen per workload by the autotuner (the context's tuning
// table); the bond-update entry points set them for the calling thread
// before issuing kernels.
//  panel_blocks  target number of blocks of a QR panel (rows per block =
//                ceil(m / panel_blocks), a multiple of 16); at most 64
//  tri_rows      rows of the matrix per block of the tridiagonalisation (8 or
//                16, as LDS allows): more rows, fewer blocks per matrix, more
//                matrices per launch
struct TuneParams {
  int panel_blocks = 64;
  int tri_rows = 8;
};
TuneParams& tune_params();   // the calling thread's current parameters

// True while s records a graph.  Kernels with grid barriers are then launched
// plainly (a captured sequence runs its kernels one after another, so a
// launch of at most one block per CU has all its blocks resident).
inline bool stream_capturing(hipStream_t s) {
  hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
  return s != nullptr && hipStreamIsCapturing(s, &st) == hipSuccess && st == hipStreamCaptureStatusActive;
}

}  // namespace qrtebd

#define QT_HIP_CHECK(expr)                                                     \
  do {                                                                         \
    hipError_t e_ = (expr);                                                    \
    if (e_ != hipSuccess) return ::qrtebd::set_hip_error(e_, #expr, __FILE__, __LINE__); \
  } while (0)

namespace qrtebd {
int set_hip_error(hipError_t e, const char* expr, const char* file, int line);
int set_error(int code, const char* fmt, ...);
}
