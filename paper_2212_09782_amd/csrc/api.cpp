// C ABI of libqrtebd: contexts, errors, the clock-model gate builder, bond
// updates, device-resident MPS, the even/odd Trotter sweep and measurements.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/qrtebd.h"
#include "bond.h"
#include "gemm.h"
#include "measure.h"
#include "reference.h"
#include "sym.h"

#include <rocblas/rocblas.h>

namespace qrtebd {

static thread_local char g_err[1024] = "";

int set_error(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

static thread_local TuneParams g_tune;
TuneParams& tune_params() { return g_tune; }

int set_hip_error(hipError_t e, const char* expr, const char* file, int line) {
  snprintf(g_err, sizeof g_err, "HIP error %s (%d) in %s at %s:%d", hipGetErrorString(e), (int)e, expr, file, line);
  return MPS_ERR_HIP;
}

}  // namespace qrtebd

using namespace qrtebd;

// Fixed workspace of mps_bond_update_noalloc: one copy per GPU, held until the
// process ends.  Host code uses only the address hipGetSymbolAddress returns
// for the current device (kept per device in g_scratch_dev); the array's name
// itself is not a device address on the host.
constexpr size_t kScratchBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[kMaxDevices] = {};

// Address of this device's scratch array; `device` must be current.
int scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return set_error(MPS_ERR_ARG, "device %d out of range", device);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return set_error(MPS_ERR_HIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", device,
                       hipGetErrorString(e));
    }
    g_scratch_dev[device] = p;
  }
  *out = g_scratch_dev[device];
  return 0;
}

}  // namespace

struct SweepStats {
  long long layers_eager = 0;   // layers run with a chi read-back
  long long host_syncs = 0;     // host synchronisations inside mps_sweep
  long long chunks = 0;         // speculative chunks
  long long rollbacks = 0;      // speculative chunks undone
  long long graph_captures = 0;
  long long graph_replays = 0;
  long long tune_trials = 0;    // timed trial runs of the autotuner
  long long tune_hits = 0;      // workloads whose shapes came from the tuning table
};

struct GraphEntry {
  std::vector<long long> key;
  hipGraphExec_t exec;
};

struct mps_ctx_s {
  int device = 0;
  void* scratch = nullptr;   // this device's scratch array (device address)
  void* ws = nullptr;
  size_t ws_bytes = 0;
  unsigned ws_gen = 0;       // bumped whenever ws is reallocated (captured graphs hold its address)
  void* snap = nullptr;      // state copy of a speculative chunk
  size_t snap_bytes = 0;
  hipStream_t cap = nullptr; // stream the step graphs are captured on
  std::vector<GraphEntry> graphs;
  SweepStats stats;
  // autotuning: launch shapes per workload key, kept in a text file
  bool tune_on = false;
  std::string tune_path;
  std::map<std::string, TuneParams> tune_table;
  rocblas_handle blas = nullptr;   // solver library handle of the reference schemes (created on first use)
  int* status = nullptr;     // device error word
  int* chi_host = nullptr;   // pinned scratch for chi read-back
  double* eps_host = nullptr;
  // per-bond scratch outputs of the sweep (device)
  void* tmp_out = nullptr;
  size_t tmp_bytes = 0;
  KernelTimer timer;
  QrAsync qa{};              // auxiliary stream + events of the QR look-ahead
};

struct mps_state_s {
  mps_ctx ctx = nullptr;
  int geometry = 0, L = 0, d = 0, chi_cap = 0, prec = 0;
  std::vector<void*> B, Xi;
  std::vector<int> chi;  // bond left of site m, m = 0..L (finite: chi[L] = 1)
};

namespace {

int ensure(void** p, size_t* have, size_t need, hipStream_t s) {
  if (*have >= need) return 0;
  QT_HIP_CHECK(hipStreamSynchronize(s));
  if (*p) QT_HIP_CHECK(hipFree(*p));
  *p = nullptr;
  *have = 0;
  const size_t bytes = need + (need >> 3) + (1 << 20);
  if (hipMalloc(p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return set_error(MPS_ERR_OOM, "workspace allocation of %zu bytes failed", bytes);
  }
  *have = bytes;
  return 0;
}

int ensure_ws(mps_ctx c, size_t need, hipStream_t s) {
  const void* before = c->ws;
  const size_t have = c->ws_bytes;
  int rc = ensure(&c->ws, &c->ws_bytes, need, s);
  if (c->ws != before || c->ws_bytes != have) ++c->ws_gen;
  return rc;
}

int check_desc(const mps_bond_desc* D) {
  if (!D) return set_error(MPS_ERR_ARG, "null descriptor");
  if (D->d < 1 || D->chi_l < 1 || D->chi_m < 1 || D->chi_r < 1)
    return set_error(MPS_ERR_ARG, "dimensions must be >= 1 (d=%d chi=%d,%d,%d)", D->d, D->chi_l, D->chi_m, D->chi_r);
  if (D->mode < 0 || D->mode > 2) return set_error(MPS_ERR_ARG, "unknown truncation mode %d", D->mode);
  if (D->prec < 0 || D->prec > 1) return set_error(MPS_ERR_ARG, "unknown precision %d", D->prec);
  const int mL = D->d * D->chi_l, mR = D->d * D->chi_r;
  if (D->mode == MPS_TRUNC_PLAIN && D->eta != D->chi_m)
    return set_error(MPS_ERR_ARG, "plain mode needs eta == chi_m (eta=%d chi_m=%d)", D->eta, D->chi_m);
  if (D->eta < 1 || D->eta > std::min(mL, mR))
    return set_error(MPS_ERR_ARG, "eta=%d outside [1, min(d chi_l, d chi_r)=%d]", D->eta, std::min(mL, mR));
  if (D->mode == MPS_TRUNC_CBE && D->chi_max < 1) return set_error(MPS_ERR_ARG, "chi_max must be >= 1");
  if (D->mode == MPS_TRUNC_CBE && !(D->svd_min >= 0)) return set_error(MPS_ERR_ARG, "svd_min must be >= 0");
  if (D->d > 25) return set_error(MPS_ERR_CAPACITY, "d=%d too large (d <= 25)", D->d);
  if (std::max(mL, mR) > kMaxQrRows)
    return set_error(MPS_ERR_CAPACITY, "d chi=%d too large", std::max(mL, mR));
  if (D->mode == MPS_TRUNC_CBE && D->eta > kEigMaxN)
    return set_error(MPS_ERR_CAPACITY, "eta=%d > %d (CBE eigensolver limit)", D->eta, kEigMaxN);
  if (D->sweeps < 0 || D->sweeps > 16) return set_error(MPS_ERR_ARG, "sweeps=%d outside [0, 16]", D->sweeps);
  if (D->left_iso && D->mode == MPS_TRUNC_CBE)
    return set_error(MPS_ERR_ARG, "left-isometric output needs mode PLAIN or GROW (A~ = Q^[m])");
  return 0;
}

BondShape shape_of(const mps_bond_desc* D) {
  BondShape b{};
  b.d = D->d; b.chi_l = D->chi_l; b.chi_m = D->chi_m; b.chi_r = D->chi_r;
  b.eta = D->eta; b.chi_max = D->chi_max; b.svd_min = D->svd_min;
  b.xi_is_diag = D->xi_is_diag; b.mode = D->mode; b.prec = D->prec;
  b.sweeps = std::max(1, D->sweeps);
  b.left_iso = D->left_iso ? 1 : 0;
  return b;
}


// ---- autotuner: candidate launch shapes, timed on the workload itself
const TuneParams kTuneCandidates[] = {{64, 8}, {48, 8}, {32, 8}, {64, 16}, {48, 16}, {32, 16}};

int tune_load(mps_ctx c) {
  std::ifstream f(c->tune_path);
  if (!f) return 0;   // no cache yet
  std::string line;
  while (std::getline(f, line)) {
    if (line.empty() || line[0] == '#') continue;
    std::istringstream is(line);
    std::string key;
    TuneParams t;
    double ms = 0;
    if (!(is >> key >> t.panel_blocks >> t.tri_rows >> ms)) continue;
    if (t.panel_blocks < 1 || t.panel_blocks > 64 || (t.tri_rows != 8 && t.tri_rows != 16)) continue;
    c->tune_table[key] = t;
  }
  return 0;
}

void tune_store(mps_ctx c, const std::string& key, const TuneParams& t, double ms) {
  c->tune_table[key] = t;
  std::ofstream f(c->tune_path, std::ios::app);
  if (!f) return;   // an unwritable cache only loses the persistence
  f.seekp(0, std::ios::end);
  if (f.tellp() == 0) f << "# qrtebd autotune cache: key panel_blocks tri_rows best_ms\n";
  f << key << ' ' << t.panel_blocks << ' ' << t.tri_rows << ' ' << ms << '\n';
}

std::string bond_tune_key(const BondShape& b) {
  std::ostringstream k;
  k << "bond:" << b.prec << ':' << b.mode << ':' << b.d << ':' << b.chi_l << ':' << b.chi_m << ':' << b.chi_r << ':'
    << b.eta << ':' << b.chi_max << ':' << b.sweeps << ':' << b.xi_is_diag;
  return k.str();
}

// Time one candidate: `run` issues the work on s; returns milliseconds.
template <typename F>
int tune_time(hipStream_t s, F run, double* ms) {
  hipEvent_t e0, e1;
  QT_HIP_CHECK(hipEventCreate(&e0));
  QT_HIP_CHECK(hipEventCreate(&e1));
  QT_HIP_CHECK(hipEventRecord(e0, s));
  int rc = run();
  QT_HIP_CHECK(hipEventRecord(e1, s));
  QT_HIP_CHECK(hipEventSynchronize(e1));
  float f = 0;
  QT_HIP_CHECK(hipEventElapsedTime(&f, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms = f;
  return rc;
}

using cd = std::complex<double>;

// expm by scaling and squaring of a Taylor series (n x n, row-major).
void expm_host(std::vector<cd>& A, int n) {
  double nrm = 0;
  for (int j = 0; j < n; ++j) {
    double c = 0;
    for (int i = 0; i < n; ++i) c += std::abs(A[i * n + j]);
    nrm = std::max(nrm, c);
  }
  int sq = 0;
  while (nrm > 0.25) { nrm *= 0.5; ++sq; }
  const double f = std::ldexp(1.0, -sq);
  for (auto& x : A) x *= f;
  std::vector<cd> E(n * n, 0.0), term(n * n, 0.0), tmp(n * n);
  for (int i = 0; i < n; ++i) E[i * n + i] = term[i * n + i] = 1.0;
  for (int k = 1; k <= 24; ++k) {
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        cd s = 0;
        for (int l = 0; l < n; ++l) s += term[i * n + l] * A[l * n + j];
        tmp[i * n + j] = s / (double)k;
      }
    term.swap(tmp);
    for (int i = 0; i < n * n; ++i) E[i] += term[i];
  }
  for (int r = 0; r < sq; ++r) {
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        cd s = 0;
        for (int l = 0; l < n; ++l) s += E[i * n + l] * E[l * n + j];
        tmp[i * n + j] = s;
      }
    E.swap(tmp);
  }
  A.swap(E);
}

}  // namespace

extern "C" {

const char* mps_last_error(void) { return g_err; }

int mps_ctx_create(int device, const char* autotune_cache, mps_ctx* out) {
  if (!out) return set_error(MPS_ERR_ARG, "null output");
  *out = nullptr;
  QT_HIP_CHECK(hipSetDevice(device));
  mps_ctx c = new mps_ctx_s();
  c->device = device;
  if (int rc = scratch_address(device, &c->scratch)) {
    delete c;
    return rc;
  }
  if (hipMalloc(&c->status, 256) != hipSuccess || hipMemset(c->status, 0, 256) != hipSuccess ||
      hipHostMalloc(&c->chi_host, 4096 * sizeof(int)) != hipSuccess ||
      hipHostMalloc(&c->eps_host, 64 * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    delete c;
    return set_error(MPS_ERR_HIP, "context allocation failed");
  }
  // The auxiliary stream (trailing updates of the QR look-ahead) leaves one
  // CU in four to the panel kernels that run beside it (64 of 256: a whole
  // panel of one QR), so the two really overlap; a plain stream if the
  // masked one is unavailable.
  {
    int ncu = 0;
    (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device);
    std::vector<uint32_t> mask((std::max(ncu, 1) + 31) / 32, 0u);
    for (int cu = 0; cu < ncu; ++cu)
      if (cu % 4 != 0) mask[cu / 32] |= 1u << (cu % 32);
    if (ncu < 64 || hipExtStreamCreateWithCUMask(&c->qa.aux, (uint32_t)mask.size(), mask.data()) != hipSuccess) {
      (void)hipGetLastError();
      c->qa.aux = nullptr;
    }
  }
  if ((!c->qa.aux && hipStreamCreateWithFlags(&c->qa.aux, hipStreamNonBlocking) != hipSuccess) ||
      hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&c->qa.ev_panel, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&c->qa.ev_trail, hipEventDisableTiming) != hipSuccess) {
    (void)hipGetLastError();
    mps_ctx_destroy(c);
    return set_error(MPS_ERR_HIP, "context stream creation failed");
  }
  if (autotune_cache && autotune_cache[0]) {
    c->tune_on = true;
    c->tune_path = autotune_cache;
    tune_load(c);
  }
  *out = c;
  return MPS_OK;
}

int mps_ctx_destroy(mps_ctx c) {
  if (!c) return MPS_OK;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  if (c->blas) (void)rocblas_destroy_handle(c->blas);
  for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.exec);
  c->graphs.clear();
  if (c->ws) (void)hipFree(c->ws);
  if (c->snap) (void)hipFree(c->snap);
  if (c->cap) (void)hipStreamDestroy(c->cap);
  if (c->tmp_out) (void)hipFree(c->tmp_out);
  if (c->status) (void)hipFree(c->status);
  if (c->chi_host) (void)hipHostFree(c->chi_host);
  if (c->eps_host) (void)hipHostFree(c->eps_host);
  if (c->qa.ev_panel) (void)hipEventDestroy(c->qa.ev_panel);
  if (c->qa.ev_trail) (void)hipEventDestroy(c->qa.ev_trail);
  if (c->qa.aux) (void)hipStreamDestroy(c->qa.aux);
  if (c->timer.ev) {
    for (int i = 0; i < 2 * c->timer.cap; ++i) (void)hipEventDestroy(c->timer.ev[i]);
    delete[] c->timer.ev;
    delete[] c->timer.flops;
  }
  delete c;
  return MPS_OK;
}

int mps_sync(mps_ctx c, mps_stream stream) {
  if (!c) return set_error(MPS_ERR_ARG, "null context");
  QT_HIP_CHECK(hipStreamSynchronize((hipStream_t)stream));
  int st = 0;
  QT_HIP_CHECK(hipMemcpy(&st, c->status, sizeof(int), hipMemcpyDeviceToHost));
  if (st) {
    QT_HIP_CHECK(hipMemset(c->status, 0, sizeof(int)));
    return set_error(MPS_ERR_NUMERIC, "device reported numeric error bits 0x%x (1 barrier stall, 2 non-finite, "
                                      "4 zero norm, 8 capacity)", st);
  }
  return MPS_OK;
}

int mps_bond_capacity(const mps_bond_desc* D) {
  if (!D) return set_error(MPS_ERR_ARG, "null descriptor");
  return shape_of(D).cap();
}

int mps_workspace_query(mps_ctx c, const mps_bond_desc* D, size_t* bytes) {
  (void)c;
  int rc = check_desc(D);
  if (rc) return rc;
  if (bytes) *bytes = bond_work_bytes(shape_of(D));
  return MPS_OK;
}

int mps_bond_update(mps_ctx c, const mps_bond_desc* D, const void* xi_m, const void* b_m, const void* b_n,
                    const void* u, void* b_m_out, void* xi_n_out, void* b_n_out, int* chi_new_dev,
                    double* trunc_err_dev, mps_stream stream) {
  if (!c) return set_error(MPS_ERR_ARG, "null context");
  int rc = check_desc(D);
  if (rc) return rc;
  if (!xi_m || !b_m || !b_n || !u || !b_m_out || !xi_n_out || !b_n_out || !chi_new_dev || !trunc_err_dev)
    return set_error(MPS_ERR_ARG, "null tensor pointer");
  const BondShape b = shape_of(D);
  hipStream_t s = (hipStream_t)stream;
  if ((rc = ensure_ws(c, bond_work_bytes(b), s))) return rc;
  auto run = [&]() {
    return bond_update_run(b, c->ws, c->status, xi_m, b_m, b_n, (const c128*)u, b_m_out, xi_n_out, b_n_out,
                           chi_new_dev, trunc_err_dev, s, &c->timer, &c->qa);
  };
  g_tune = TuneParams{};
  if (c->tune_on) {
    const std::string key = bond_tune_key(b);
    auto it = c->tune_table.find(key);
    if (it != c->tune_table.end()) {
      g_tune = it->second;
      c->stats.tune_hits++;
    } else {
      // inputs are read only and outputs do not alias them: every candidate
      // runs the whole update on the real data, the best one runs last
      TuneParams best{};
      double best_ms = 1e300;
      const int saved_timer = c->timer.on;
      c->timer.on = 0;
      for (const TuneParams& t : kTuneCandidates) {
        g_tune = t;
        double ms = 0;
        if ((rc = tune_time(s, run, &ms))) {
          c->timer.on = saved_timer;
          return rc;
        }
        c->stats.tune_trials++;
        if (ms < best_ms) {
          best_ms = ms;
          best = t;
        }
      }
      c->timer.on = saved_timer;
      tune_store(c, key, best, best_ms);
      g_tune = best;
    }
  }
  return run();
}

int mps_bond_update_reference(mps_ctx c, const mps_bond_desc* D, int scheme, const void* xi_m, const void* b_m,
                              const void* b_n, const void* u, void* b_m_out, void* xi_n_out, void* b_n_out,
                              int* chi_new_dev, double* trunc_err_dev, mps_stream stream) {
  if (!c) return set_error(MPS_ERR_ARG, "null context");
  if (scheme != MPS_SCHEME_SVD && scheme != MPS_SCHEME_EIG) return set_error(MPS_ERR_ARG, "scheme must be 0 or 1");
  if (!D) return set_error(MPS_ERR_ARG, "null descriptor");
  if (D->mode != MPS_TRUNC_CBE || D->prec != MPS_C128)
    return set_error(MPS_ERR_ARG, "the reference schemes take mode CBE (chi_max, svd_min) and complex128");
  mps_bond_desc Dr = *D;
  Dr.eta = std::min(D->d * D->chi_l, D->d * D->chi_r);   // eta is not used: the whole of theta~ is decomposed
  Dr.sweeps = 0;
  if (Dr.eta > kEigMaxN) Dr.eta = kEigMaxN;   // only the descriptor check's eigensolver limit; not used here
  int rc = check_desc(&Dr);
  if (rc) return rc;
  if (!xi_m || !b_m || !b_n || !u || !b_m_out || !xi_n_out || !b_n_out || !chi_new_dev || !trunc_err_dev)
    return set_error(MPS_ERR_ARG, "null tensor pointer");
  BondShape b = shape_of(&Dr);
  b.eta = std::min(D->d * D->chi_l, D->d * D->chi_r);
  hipStream_t s = (hipStream_t)stream;
  if (!c->blas && rocblas_create_handle(&c->blas) != rocblas_status_success) {
    c->blas = nullptr;
    return set_error(MPS_ERR_HIP, "rocblas_create_handle failed");
  }
  if ((rc = ensure_ws(c, reference_work_bytes(b, scheme), s))) return rc;
  return reference_update(b, scheme, c->ws, c->status, c->blas, xi_m, b_m, b_n, (const c128*)u, b_m_out, xi_n_out,
                          b_n_out, chi_new_dev, trunc_err_dev, s);
}

int mps_bond_update_noalloc(mps_ctx c, const mps_bond_desc* D, const void* xi_m, const void* b_m,
                            const void* b_n, const void* u, void* b_m_out, void* xi_n_out, void* b_n_out,
                            int* chi_new_dev, double* trunc_err_dev, mps_stream stream) {
  if (!c) return set_error(MPS_ERR_ARG, "null context");
  int rc = check_desc(D);
  if (rc) return rc;
  if (!xi_m || !b_m || !b_n || !u || !b_m_out || !xi_n_out || !b_n_out || !chi_new_dev || !trunc_err_dev)
    return set_error(MPS_ERR_ARG, "null tensor pointer");
  const BondShape b = shape_of(D);
  const size_t need = bond_work_bytes(b);
  if (need > kScratchBytes)
    return set_error(MPS_ERR_CAPACITY, "bond needs %zu bytes of workspace, the fixed scratch holds %zu", need,
                     kScratchBytes);
  if (!c->scratch) return set_error(MPS_ERR_STATE, "context has no scratch address");
  auto it = c->tune_table.find(bond_tune_key(b));
  g_tune = it != c->tune_table.end() ? it->second : TuneParams{};
  return bond_update_run(b, c->scratch, c->status, xi_m, b_m, b_n, (const c128*)u, b_m_out, xi_n_out, b_n_out,
                         chi_new_dev, trunc_err_dev, (hipStream_t)stream, &c->timer, &c->qa);
}

int mps_profile_enable(mps_ctx c, int on, int max_launches) {
  if (!c) return set_error(MPS_ERR_ARG, "null context");
  KernelTimer& t = c->timer;
  if (on && max_launches > t.cap) {
    if (t.ev) {
      for (int i = 0; i < 2 * t.cap; ++i) (void)hipEventDestroy(t.ev[i]);
      delete[] t.ev;
      delete[] t.flops;
    }
    t.ev = new hipEvent_t[2 * (size_t)max_launches];
    t.flops = new double[max_launches];
    t.cap = 0;
    for (int i = 0; i < 2 * max_launches; ++i) QT_HIP_CHECK(hipEventCreate(&t.ev[i]));
    t.cap = max_launches;
  }
  t.on = on ? 1 : 0;
  t.n = 0;
  return MPS_OK;
}

int mps_profile_read(mps_ctx c, double* total_ms, double* total_flops, int* launches) {
  if (!c) return set_error(MPS_ERR_ARG, "null context");
  KernelTimer& t = c->timer;
  double ms = 0, fl = 0;
  for (int i = 0; i < t.n; ++i) {
    QT_HIP_CHECK(hipEventSynchronize(t.ev[2 * i + 1]));
    float e = 0;
    QT_HIP_CHECK(hipEventElapsedTime(&e, t.ev[2 * i], t.ev[2 * i + 1]));
    ms += e;
    fl += t.flops[i];
  }
  if (total_ms) *total_ms = ms;
  if (total_flops) *total_flops = fl;
  if (launches) *launches = t.n;
  return MPS_OK;
}

}  // extern "C"

namespace {

// h = -(Z (x) Z^dag + h.c.) - g (wl (X+X^dag) (x) 1 + wr 1 (x) (X+X^dag)), row i*d+j.
// Bond term of the clock model (Sec. IV).  charge = false: clock basis, Z =
// diag(w^k), X the cyclic shift; charge = true: eigenbasis of X (charge q,
// X|q> = w^q |q>), where X = diag(w^q) and Z raises the charge by one.
std::vector<cd> clock_bond_h(int d, double g, double wl, double wr, bool charge = false) {
  const int n = d * d;
  const cd w = std::exp(cd(0, 2 * M_PI / d));
  std::vector<cd> Z(d * d, 0.0), X(d * d, 0.0), xs(d * d);
  for (int k = 0; k < d; ++k) {
    if (charge) {
      Z[((k + 1) % d) * d + k] = 1.0;
      X[k * d + k] = std::pow(w, k);
    } else {
      Z[k * d + k] = std::pow(w, k);
      X[k * d + (k + 1) % d] = 1.0;
    }
  }
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j) xs[i * d + j] = X[i * d + j] + std::conj(X[j * d + i]);
  std::vector<cd> H(n * n, 0.0);
  for (int i = 0; i < d; ++i)
    for (int j = 0; j < d; ++j)
      for (int k = 0; k < d; ++k)
        for (int l = 0; l < d; ++l) {
          const int r = i * d + j, c = k * d + l;
          // Z (x) Z^dag + h.c.
          const cd zz = Z[i * d + k] * std::conj(Z[l * d + j]);
          const cd zzh = std::conj(Z[k * d + i]) * Z[j * d + l];
          cd h = -(zz + zzh);
          h -= g * (wl * xs[i * d + k] * (j == l ? 1.0 : 0.0) + wr * (i == k ? 1.0 : 0.0) * xs[j * d + l]);
          H[r * n + c] = h;
        }
  return H;
}

}  // namespace

extern "C" {

int mps_clock_hamiltonian(int d, double g, double wl, double wr, double* h_out) {
  if (d < 1 || !h_out) return set_error(MPS_ERR_ARG, "bad Hamiltonian arguments");
  const std::vector<cd> H = clock_bond_h(d, g, wl, wr);
  for (size_t i = 0; i < H.size(); ++i) {
    h_out[2 * i] = H[i].real();
    h_out[2 * i + 1] = H[i].imag();
  }
  return MPS_OK;
}

int mps_clock_gate(int d, double g, double tau, double wl, double wr, double* u_out) {
  if (d < 1 || !u_out) return set_error(MPS_ERR_ARG, "bad gate arguments");
  const int n = d * d;
  std::vector<cd> A = clock_bond_h(d, g, wl, wr);
  for (auto& x : A) x *= cd(0, -tau);
  expm_host(A, n);
  for (int i = 0; i < n * n; ++i) {
    u_out[2 * i] = A[i].real();
    u_out[2 * i + 1] = A[i].imag();
  }
  return MPS_OK;
}

int mps_clock_hamiltonian_charge(int d, double g, double wl, double wr, double* h_out) {
  if (d < 1 || !h_out) return set_error(MPS_ERR_ARG, "bad Hamiltonian arguments");
  const std::vector<cd> H = clock_bond_h(d, g, wl, wr, true);
  for (size_t i = 0; i < H.size(); ++i) {
    h_out[2 * i] = H[i].real();
    h_out[2 * i + 1] = H[i].imag();
  }
  return MPS_OK;
}

int mps_clock_gate_charge(int d, double g, double tau, double wl, double wr, double* u_out) {
  if (d < 1 || !u_out) return set_error(MPS_ERR_ARG, "bad gate arguments");
  const int n = d * d;
  std::vector<cd> A = clock_bond_h(d, g, wl, wr, true);
  for (auto& x : A) x *= cd(0, -tau);
  expm_host(A, n);
  for (int i = 0; i < n * n; ++i) {
    u_out[2 * i] = A[i].real();
    u_out[2 * i + 1] = A[i].imag();
  }
  return MPS_OK;
}

// ---------------------------------------------------------------- Z_d blocks

int sym_plan_of(const mps_sym_desc* D, SymPlan* p) {
  if (!D) return set_error(MPS_ERR_ARG, "null descriptor");
  if (D->d < 2 || D->d > MPS_SYM_MAX_D) return set_error(MPS_ERR_ARG, "d=%d outside [2, %d]", D->d, MPS_SYM_MAX_D);
  SymShape sh{};
  sh.d = D->d;
  for (int a = 0; a < D->d; ++a) {
    sh.sec_l[a] = D->sec_l[a];
    sh.sec_m[a] = D->sec_m[a];
    sh.sec_r[a] = D->sec_r[a];
  }
  sh.dchi_min = D->dchi_min;
  sh.dchi_frac = D->dchi_frac;
  sh.chi_max = D->chi_max;
  sh.svd_min = D->svd_min;
  sh.prec = D->prec;
  return sym_plan(sh, p);
}

int mps_sym_capacity(const mps_sym_desc* D) {
  SymPlan p;
  const int rc = sym_plan_of(D, &p);
  return rc ? rc : p.cap;
}

int mps_sym_workspace_query(mps_ctx c, const mps_sym_desc* D, size_t* bytes) {
  (void)c;
  if (!bytes) return set_error(MPS_ERR_ARG, "null argument");
  SymPlan p;
  const int rc = sym_plan_of(D, &p);
  if (rc) return rc;
  *bytes = sym_work_bytes(p);
  return MPS_OK;
}

int mps_bond_update_sym(mps_ctx c, const mps_sym_desc* D, const double* xi_m, const void* b_m, const void* b_n,
                        const void* u, void* b_m_out, double* xi_n_out, void* b_n_out, int* sec_out_dev,
                        int* chi_new_dev, double* trunc_err_dev, mps_stream stream) {
  if (!c) return set_error(MPS_ERR_ARG, "null context");
  SymPlan p;
  int rc = sym_plan_of(D, &p);
  if (rc) return rc;
  if (!xi_m || !b_m || !b_n || !u || !b_m_out || !xi_n_out || !b_n_out || !sec_out_dev || !chi_new_dev ||
      !trunc_err_dev)
    return set_error(MPS_ERR_ARG, "null pointer");
  hipStream_t s = (hipStream_t)stream;
  if ((rc = ensure_ws(c, sym_work_bytes(p), s))) return rc;
  g_tune = TuneParams{};
  return sym_update_run(p, c->ws, c->status, xi_m, b_m, b_n, (const c128*)u, b_m_out, xi_n_out, b_n_out,
                        sec_out_dev, chi_new_dev, trunc_err_dev, s, &c->qa);
}

// ---------------------------------------------------------------- states

int mps_state_create(mps_ctx c, int geometry, int L, int d, int chi_cap, int prec, void* const* b_ptrs,
                     void* const* xi_ptrs, const int* chi_host, mps_state* out) {
  if (!c || !out || !b_ptrs || !xi_ptrs || !chi_host) return set_error(MPS_ERR_ARG, "null argument");
  if (geometry != 0 && geometry != 1) return set_error(MPS_ERR_ARG, "geometry must be 0 or 1");
  if (geometry == 1 && L != 2) return set_error(MPS_ERR_ARG, "the uniform cell has L = 2");
  if (L < 2 || L > kMaxSites) return set_error(MPS_ERR_ARG, "L=%d outside [2, %d]", L, kMaxSites);
  if (d < 1 || chi_cap < 1 || prec < 0 || prec > 1) return set_error(MPS_ERR_ARG, "bad d / chi_cap / prec");
  mps_state st = new mps_state_s();
  st->ctx = c;
  st->geometry = geometry;
  st->L = L;
  st->d = d;
  st->chi_cap = chi_cap;
  st->prec = prec;
  st->B.assign(b_ptrs, b_ptrs + L);
  st->Xi.assign(xi_ptrs, xi_ptrs + L);
  st->chi.assign(chi_host, chi_host + L + 1);
  for (int m = 0; m <= L; ++m)
    if (st->chi[m] < 1 || st->chi[m] > chi_cap) {
      delete st;
      return set_error(MPS_ERR_ARG, "chi[%d]=%d outside [1, chi_cap]", m, chi_host[m]);
    }
  if (geometry == 0 && (st->chi[0] != 1 || st->chi[L] != 1)) {
    delete st;
    return set_error(MPS_ERR_ARG, "a finite chain has chi = 1 at both ends");
  }
  if (geometry == 1) st->chi[2] = st->chi[0];
  *out = st;
  return MPS_OK;
}

int mps_state_destroy(mps_state st) {
  delete st;
  return MPS_OK;
}

int mps_state_chis(mps_state st, int* chi_out) {
  if (!st || !chi_out) return set_error(MPS_ERR_ARG, "null argument");
  std::copy(st->chi.begin(), st->chi.end(), chi_out);
  return MPS_OK;
}

namespace {

struct BondRef {
  mps_state st;
  int m, n, il, im, ir;  // sites m, n and the chi indices left / middle / right
  const c128* gate;
};

std::vector<BondRef> layer_bonds(mps_state st, int parity, const void* gates, int gate_slot) {
  std::vector<BondRef> out;
  const int L = st->L, d2 = st->d * st->d;
  const c128* g = (const c128*)gates;
  if (st->geometry == 0) {
    for (int m = parity; m < L - 1; m += 2)
      out.push_back(BondRef{st, m, m + 1, m, m + 1, m + 2, g + ((size_t)m * 2 + gate_slot) * d2 * d2});
  } else {
    const int m = parity, n = 1 - parity;
    out.push_back(BondRef{st, m, n, m, n, m, g + ((size_t)m * 2 + gate_slot) * d2 * d2});
  }
  return out;
}

constexpr int kMaxLayerBonds = 512;

struct EpsMap {
  int n;
  int state[kMaxLayerBonds];
};

__global__ void add_eps_batch_kernel(const double* eps, EpsMap map, double* acc) {
  for (int k = 0; k < map.n; ++k) acc[map.state[k]] += eps[k];
}

// Speculative layers: the new chi of every bond must equal the one the host
// planned the following layers with; a mismatch sets *flag.
struct ChiExpect {
  int n;
  int chi[kMaxLayerBonds];
};

__global__ void check_chi_kernel(const int* chi_dev, ChiExpect e, int* flag) {
  for (int k = threadIdx.x; k < e.n; k += blockDim.x)
    if (chi_dev[k] != e.chi[k]) atomicOr(flag, 1);
}

// One layer: every bond of every state, shapes from the host copy of chi.
// Bonds of a layer run in groups, in bond order, whose workspaces together
// stay within this many bytes (a bond larger than that forms its own group);
// the groups share one workspace region one after another.
constexpr size_t kLayerGroupBytes = size_t(16) << 30;

struct LayerPlan {
  std::vector<BondRef> bonds;
  std::vector<int> state_index;
  std::vector<BondShape> shapes;
  std::vector<size_t> off;
  std::vector<int> group;   // group of each bond (groups run one after another)
  int ngroups = 0;
  size_t total = 0;
};

int plan_layer(mps_state* states, int nstates, const void* const* gates, int parity, int slot,
               const mps_sweep_policy* pol, LayerPlan& lp) {
  int rc;
  lp = LayerPlan{};
  for (int si = 0; si < nstates; ++si)
    for (auto& x : layer_bonds(states[si], parity, gates[si], slot)) {
      lp.bonds.push_back(x);
      lp.state_index.push_back(si);
    }
  const int nb = (int)lp.bonds.size();
  if (nb > kMaxLayerBonds) return set_error(MPS_ERR_CAPACITY, "a layer of %d bonds exceeds %d", nb, kMaxLayerBonds);
  lp.shapes.resize(nb);
  lp.off.resize(nb);
  lp.group.resize(nb);
  const size_t header = ((size_t)nb * (sizeof(int) + sizeof(double)) + 4096 + 255) & ~size_t(255);
  size_t gbytes = 0, gmax = 0;
  for (int k = 0; k < nb; ++k) {
    const BondRef& br = lp.bonds[k];
    mps_state st = br.st;
    const int d = st->d;
    const int chiL = st->chi[br.il], chiM = st->chi[br.im], chiR = st->chi[br.ir];
    mps_bond_desc D{};
    D.d = d;
    D.chi_l = chiL;
    D.chi_m = chiM;
    D.chi_r = chiR;
    const int dchi = std::max(pol->dchi_min, (int)std::ceil(pol->dchi_frac * chiM));
    D.eta = std::min(std::min(chiM + dchi, d * chiL), d * chiR);
    D.chi_max = std::min(pol->chi_max, st->chi_cap);
    D.svd_min = pol->svd_min;
    D.xi_is_diag = 1;
    D.mode = MPS_TRUNC_CBE;
    D.prec = st->prec;
    D.sweeps = pol->sweeps;
    if ((rc = check_desc(&D))) return rc;
    lp.shapes[k] = shape_of(&D);
    const size_t wb = (bond_work_bytes(lp.shapes[k]) + 255) & ~size_t(255);
    if (k == 0 || (gbytes > 0 && gbytes + wb > kLayerGroupBytes)) {
      ++lp.ngroups;
      gbytes = 0;
    }
    lp.group[k] = lp.ngroups - 1;
    lp.off[k] = header + gbytes;
    gbytes += wb;
    gmax = std::max(gmax, gbytes);
  }
  lp.total = header + gmax;
  return 0;
}

// Issue a planned layer on s (no host synchronisation).  The workspace must
// hold lp.total bytes.  expect: if set, the planned chi of the middle bond of
// every update is checked on the device (speculative layers).
int launch_layer(mps_ctx c, const LayerPlan& lp, double* eps_acc_base, hipStream_t s, bool helpers,
                 int* spec_flag) {
  int rc;
  const int nb = (int)lp.bonds.size();
  if (nb == 0) return 0;
  char* base = (char*)c->ws;
  int* chi_dev = (int*)base;
  double* eps_dev = (double*)(base + (((size_t)nb * sizeof(int) + 255) & ~size_t(255)));
  for (int g = 0; g < lp.ngroups; ++g) {
    std::vector<BondCall> calls[2];
    for (int k = 0; k < nb; ++k) {
      if (lp.group[k] != g) continue;
      const BondRef& br = lp.bonds[k];
      mps_state st = br.st;
      BondCall bc{lp.shapes[k], base + lp.off[k], c->status, st->Xi[br.m], st->B[br.m], st->B[br.n], br.gate,
                  st->B[br.m], st->Xi[br.n], st->B[br.n], chi_dev + k, eps_dev + k};
      calls[st->prec].push_back(bc);
    }
    for (int p = 0; p < 2; ++p)
      if (!calls[p].empty() &&
          (rc = bond_update_batch(calls[p].data(), (int)calls[p].size(), s, helpers ? &c->timer : nullptr,
                                  helpers ? &c->qa : nullptr)))
        return rc;
  }
  if (eps_acc_base) {
    EpsMap map{};
    map.n = nb;
    for (int k = 0; k < nb; ++k) map.state[k] = lp.state_index[k];
    hipLaunchKernelGGL(add_eps_batch_kernel, dim3(1), dim3(1), 0, s, eps_dev, map, eps_acc_base);
    QT_HIP_CHECK(hipGetLastError());
  }
  if (spec_flag) {
    ChiExpect e{};
    e.n = nb;
    for (int k = 0; k < nb; ++k) e.chi[k] = lp.bonds[k].st->chi[lp.bonds[k].im];
    hipLaunchKernelGGL(check_chi_kernel, dim3(1), dim3(256), 0, s, chi_dev, e, spec_flag);
    QT_HIP_CHECK(hipGetLastError());
  }
  return 0;
}

// Eager layer: issue it, read the new chis back (one host synchronisation)
// and update the host copies.
int run_layer_sync(mps_ctx c, LayerPlan& lp, double* eps_acc_base, hipStream_t s) {
  int rc;
  const int nb = (int)lp.bonds.size();
  if (nb == 0) return 0;
  if ((rc = ensure_ws(c, lp.total, s))) return rc;
  if ((rc = launch_layer(c, lp, eps_acc_base, s, true, nullptr))) return rc;
  QT_HIP_CHECK(hipMemcpyAsync(c->chi_host, c->ws, (size_t)nb * sizeof(int), hipMemcpyDeviceToHost, s));
  QT_HIP_CHECK(hipStreamSynchronize(s));
  c->stats.layers_eager++;
  c->stats.host_syncs++;
  for (int k = 0; k < nb; ++k) {
    BondRef& br = lp.bonds[k];
    const int chiN = c->chi_host[k];
    if (chiN < 1 || chiN > lp.shapes[k].cap())
      return set_error(MPS_ERR_NUMERIC, "device returned chi=%d (cap %d)", chiN, lp.shapes[k].cap());
    br.st->chi[br.im] = chiN;
    if (br.st->geometry == 1 && br.im == 0) br.st->chi[2] = chiN;
  }
  return 0;
}

struct Layer {
  int parity, slot;
};

std::vector<Layer> step_layers(int order) {
  if (order == 2) return {{0, 0}, {1, 1}, {0, 0}};
  return {{0, 1}, {1, 1}};
}

// A profile is saturated when no bond update can raise its middle chi:
// chi_m == min(eta, chi_max) for every bond, with eta = min(chi_m + dchi,
// d chi_l, d chi_r).  Then the only possible change is a smaller chi~ (fewer
// Schmidt values above svd_min), which the device checks.
bool saturated(mps_state* states, int nstates, const mps_sweep_policy* pol) {
  for (int si = 0; si < nstates; ++si) {
    mps_state st = states[si];
    for (int parity = 0; parity < 2; ++parity)
      for (const BondRef& br : layer_bonds(st, parity, nullptr, 0)) {
        const int d = st->d, chiL = st->chi[br.il], chiM = st->chi[br.im], chiR = st->chi[br.ir];
        const int dchi = std::max(pol->dchi_min, (int)std::ceil(pol->dchi_frac * chiM));
        const int eta = std::min(std::min(chiM + dchi, d * chiL), d * chiR);
        const int cap = std::max(1, std::min(eta, std::min(pol->chi_max, st->chi_cap)));
        if (cap != chiM) return false;
      }
  }
  return true;
}

int step_eager(mps_ctx c, mps_state* states, int nstates, const void* const* gates, int order,
               const mps_sweep_policy* pol, double* eps_acc, hipStream_t s) {
  int rc;
  g_tune = TuneParams{};   // a growing profile changes shape every step: default launch shapes
  for (const Layer& ly : step_layers(order)) {
    LayerPlan lp;
    if ((rc = plan_layer(states, nstates, gates, ly.parity, ly.slot, pol, lp))) return rc;
    if ((rc = run_layer_sync(c, lp, eps_acc, s))) return rc;
  }
  return 0;
}

// Live bytes of every site tensor and bond vector of every state, and of the
// truncation-error accumulators: what a speculative chunk may overwrite.
struct SnapItem {
  void* dev;
  size_t bytes;
};

std::vector<SnapItem> snapshot_items(mps_state* states, int nstates, double* eps_acc) {
  std::vector<SnapItem> v;
  for (int si = 0; si < nstates; ++si) {
    mps_state st = states[si];
    const size_t es = st->prec ? 8 : 16;
    for (int m = 0; m < st->L; ++m) {
      const int chiR = st->geometry == 0 ? st->chi[m + 1] : st->chi[1 - m];
      v.push_back(SnapItem{st->B[m], (size_t)st->chi[m] * st->d * chiR * es});
      v.push_back(SnapItem{st->Xi[m], (size_t)st->chi[m] * sizeof(double)});
    }
  }
  if (eps_acc) v.push_back(SnapItem{eps_acc, (size_t)nstates * sizeof(double)});
  return v;
}

int snapshot_copy(mps_ctx c, const std::vector<SnapItem>& items, bool save, hipStream_t s) {
  size_t need = 0;
  for (const SnapItem& it : items) need += (it.bytes + 255) & ~size_t(255);
  int rc;
  if (save && (rc = ensure(&c->snap, &c->snap_bytes, need, s))) return rc;
  char* p = (char*)c->snap;
  for (const SnapItem& it : items) {
    if (save) QT_HIP_CHECK(hipMemcpyAsync(p, it.dev, it.bytes, hipMemcpyDeviceToDevice, s));
    else QT_HIP_CHECK(hipMemcpyAsync(it.dev, p, it.bytes, hipMemcpyDeviceToDevice, s));
    p += (it.bytes + 255) & ~size_t(255);
  }
  return 0;
}

// Tuning key of a step: the shapes of every bond of its layers.
std::string sweep_tune_key(const std::vector<LayerPlan>& plans) {
  unsigned long long h = 1469598103934665603ull;   // FNV-1a over the shape fields
  int nb = 0, chimax = 0, precs = 0;
  auto mix = [&](long long v) {
    for (int i = 0; i < 8; ++i) {
      h ^= (unsigned long long)((v >> (8 * i)) & 0xff);
      h *= 1099511628211ull;
    }
  };
  for (const LayerPlan& lp : plans)
    for (const BondShape& b : lp.shapes) {
      mix(b.d); mix(b.chi_l); mix(b.chi_m); mix(b.chi_r); mix(b.eta); mix(b.chi_max); mix(b.prec); mix(b.sweeps);
      ++nb;
      chimax = std::max(chimax, b.chi_m);
      precs |= 1 << b.prec;
    }
  std::ostringstream k;
  k << "sweep:" << precs << ':' << nb << ':' << chimax << ':' << std::hex << h;
  return k.str();
}

// Cache key of a captured step: everything the captured launches depend on.
std::vector<long long> graph_key(mps_ctx c, mps_state* states, int nstates, const void* const* gates, int order,
                                 const mps_sweep_policy* pol, double* eps_acc) {
  std::vector<long long> k;
  k.push_back(nstates);
  k.push_back(order);
  k.push_back((long long)(uintptr_t)eps_acc);
  k.push_back((long long)(uintptr_t)c->ws);
  k.push_back((long long)c->ws_gen);
  k.push_back(pol->chi_max);
  k.push_back(pol->dchi_min);
  k.push_back(pol->sweeps);
  k.push_back(g_tune.panel_blocks);
  k.push_back(g_tune.tri_rows);
  long long f;
  std::memcpy(&f, &pol->dchi_frac, sizeof f);
  k.push_back(f);
  std::memcpy(&f, &pol->svd_min, sizeof f);
  k.push_back(f);
  for (int si = 0; si < nstates; ++si) {
    mps_state st = states[si];
    k.push_back((long long)(uintptr_t)st);
    k.push_back((long long)(uintptr_t)gates[si]);
    k.push_back(st->prec);
    k.push_back(st->chi_cap);
    for (int x : st->chi) k.push_back(x);
    for (void* b : st->B) k.push_back((long long)(uintptr_t)b);
    for (void* x : st->Xi) k.push_back((long long)(uintptr_t)x);
  }
  return k;
}

// One Trotter step of every state captured as a hipGraph on the context's
// capture stream (QR look-ahead stream and event timing are left out of the
// capture; cooperative kernels are launched plainly inside it).
int capture_step(mps_ctx c, const std::vector<LayerPlan>& plans, double* eps_acc, int* spec_flag,
                 hipGraphExec_t* out) {
  hipStream_t cs = c->cap;
  QT_HIP_CHECK(hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed));
  int rc = 0;
  for (const LayerPlan& lp : plans)
    if ((rc = launch_layer(c, lp, eps_acc, cs, false, spec_flag))) break;
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(cs, &g);
  if (rc) {
    if (g) (void)hipGraphDestroy(g);
    return rc;
  }
  if (e != hipSuccess) return set_hip_error(e, "hipStreamEndCapture", __FILE__, __LINE__);
  const hipError_t e2 = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e2 != hipSuccess) return set_hip_error(e2, "hipGraphInstantiate", __FILE__, __LINE__);
  c->stats.graph_captures++;
  return 0;
}

}  // namespace

int mps_sweep(mps_ctx c, mps_state* states, int nstates, const void* const* gates, int nsteps, int order,
              const mps_sweep_policy* pol, double* trunc_err_dev, mps_stream stream) {
  if (!c || !states || !gates || !pol || nstates < 1) return set_error(MPS_ERR_ARG, "null argument");
  if (order != 1 && order != 2) return set_error(MPS_ERR_ARG, "order must be 1 or 2");
  if (pol->mode != MPS_TRUNC_CBE)
    return set_error(MPS_ERR_ARG, "mps_sweep keeps diagonal bond matrices: mode must be MPS_TRUNC_CBE");
  if (pol->exec < 0 || pol->exec > 2) return set_error(MPS_ERR_ARG, "exec must be 0, 1 or 2");
  for (int si = 0; si < nstates; ++si)
    if (!states[si] || states[si]->ctx != c) return set_error(MPS_ERR_ARG, "state %d missing or of another context", si);
  hipStream_t s = (hipStream_t)stream;
  int rc;
  const int chunk_max = pol->chunk > 0 ? pol->chunk : 8;
  int chunk = chunk_max;
  int* spec_flag = c->status + 16;
  int step = 0;
  while (step < nsteps) {
    if (pol->exec == 0 || !saturated(states, nstates, pol)) {
      if ((rc = step_eager(c, states, nstates, gates, order, pol, trunc_err_dev, s))) return rc;
      ++step;
      continue;
    }
    // Speculative chunk: the profile cannot grow, so every layer is planned
    // with the current chis and issued without reading them back; the device
    // flags any smaller chi~, and then the chunk is undone and run eagerly.
    const int K = std::min(chunk, nsteps - step);
    std::vector<LayerPlan> plans;
    size_t need = 0;
    for (const Layer& ly : step_layers(order)) {
      plans.emplace_back();
      if ((rc = plan_layer(states, nstates, gates, ly.parity, ly.slot, pol, plans.back()))) return rc;
      need = std::max(need, plans.back().total);
    }
    if ((rc = ensure_ws(c, need, s))) return rc;
    std::vector<SnapItem> items = snapshot_items(states, nstates, trunc_err_dev);
    // the error word too: a mis-planned layer may latch errors the eager rerun would not
    items.push_back(SnapItem{c->status, sizeof(int)});
    if ((rc = snapshot_copy(c, items, true, s))) return rc;
    g_tune = TuneParams{};
    if (c->tune_on) {
      const std::string key = sweep_tune_key(plans);
      auto it = c->tune_table.find(key);
      if (it != c->tune_table.end()) {
        g_tune = it->second;
        c->stats.tune_hits++;
      } else {
        // time one step per candidate, each from the saved state
        TuneParams best{};
        double best_ms = 1e300;
        for (const TuneParams& t : kTuneCandidates) {
          g_tune = t;
          double ms = 0;
          auto run = [&]() {
            for (const LayerPlan& lp : plans)
              if (int r = launch_layer(c, lp, trunc_err_dev, s, false, nullptr)) return r;
            return 0;
          };
          if ((rc = tune_time(s, run, &ms))) return rc;
          if ((rc = snapshot_copy(c, items, false, s))) return rc;
          c->stats.tune_trials++;
          if (ms < best_ms) {
            best_ms = ms;
            best = t;
          }
        }
        tune_store(c, key, best, best_ms);
        g_tune = best;
      }
    }
    if ((rc = fill_zero(spec_flag, sizeof(int), s))) return rc;
    hipGraphExec_t gx = nullptr;
    if (pol->exec == 2) {
      const std::vector<long long> key = graph_key(c, states, nstates, gates, order, pol, trunc_err_dev);
      for (auto& g : c->graphs)
        if (g.key == key) gx = g.exec;
      if (!gx) {
        if ((rc = capture_step(c, plans, trunc_err_dev, spec_flag, &gx))) return rc;
        if (c->graphs.size() >= 8) {
          (void)hipGraphExecDestroy(c->graphs.front().exec);
          c->graphs.erase(c->graphs.begin());
        }
        c->graphs.push_back(GraphEntry{key, gx});
      }
    }
    for (int k = 0; k < K; ++k) {
      if (gx) {
        QT_HIP_CHECK(hipGraphLaunch(gx, s));
        c->stats.graph_replays++;
      } else {
        for (const LayerPlan& lp : plans)
          if ((rc = launch_layer(c, lp, trunc_err_dev, s, true, spec_flag))) return rc;
      }
    }
    int flag = 0;
    QT_HIP_CHECK(hipMemcpyAsync(&c->chi_host[kMaxLayerBonds], spec_flag, sizeof(int), hipMemcpyDeviceToHost, s));
    QT_HIP_CHECK(hipStreamSynchronize(s));
    flag = c->chi_host[kMaxLayerBonds];
    c->stats.host_syncs++;
    c->stats.chunks++;
    if (!flag) {
      step += K;
      chunk = std::min(chunk_max, 2 * chunk);
      continue;
    }
    // a bond kept fewer Schmidt values than planned: undo the chunk
    if ((rc = snapshot_copy(c, items, false, s))) return rc;
    c->stats.rollbacks++;
    chunk = std::max(1, chunk / 2);
    if ((rc = step_eager(c, states, nstates, gates, order, pol, trunc_err_dev, s))) return rc;
    ++step;
  }
  return MPS_OK;
}

}  // extern "C"

namespace {

// out[b][i][a] = in[a][i][b]
template <typename S>
__global__ void reflect_site_kernel(const cpx<S>* in, int na, int d, int nb, cpx<S>* out) {
  const long long n = (long long)na * d * nb;
  for (long long idx = blockIdx.x * 256ll + threadIdx.x; idx < n; idx += (long long)gridDim.x * 256) {
    const long long ia = idx / ((long long)d * nb), r = idx % ((long long)d * nb);
    const int i = (int)(r / nb), ib = (int)(r % nb);
    out[((long long)ib * d + i) * na + ia] = in[idx];
  }
}

// out[k] = in[nb - 1 - k] with the gate's two sites exchanged:
// out[(j i), (j' i')] = in[(i j), (i' j')]
__global__ void reflect_gates_kernel(const c128* in, int nb, int d, c128* out) {
  const int d2 = d * d;
  const long long per = (long long)d2 * d2, n = per * nb;
  for (long long idx = blockIdx.x * 256ll + threadIdx.x; idx < n; idx += (long long)gridDim.x * 256) {
    const int k = (int)(idx / per);
    const int r = (int)(idx % per), row = r / d2, col = r % d2;
    const int i = row / d, j = row % d, ip = col / d, jp = col % d;
    out[idx] = in[(long long)(nb - 1 - k) * per + (long long)(j * d + i) * d2 + (jp * d + ip)];
  }
}

__global__ void unit_center_kernel(c128* center) { center[0] = mk<double>(1, 0); }

template <typename D>
__global__ void cast_center_kernel(const c128* in, long long n, cpx<D>* out) {
  for (long long i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (long long)gridDim.x * 256) out[i] = ccast<D>(in[i]);
}

inline int grid_of(long long n) { return (int)std::max<long long>(1, std::min<long long>((n + 255) / 256, 4096)); }

}  // namespace

extern "C" {

int mps_sweep_sequential(mps_ctx c, int L, int d, int chi_cap, int prec, void* const* sites, void* center, int* chi,
                         const void* gates_half, int nsteps, int mode, int chi_max, mps_stream stream) {
  if (!c || !sites || !center || !chi || !gates_half) return set_error(MPS_ERR_ARG, "null argument");
  if (L < 2 || L > kMaxSites || d < 1 || chi_cap < 1 || (prec != MPS_C128 && prec != MPS_MIXED_C64))
    return set_error(MPS_ERR_ARG, "bad L / d / chi_cap / prec");
  if (mode != MPS_TRUNC_PLAIN && mode != MPS_TRUNC_GROW) return set_error(MPS_ERR_ARG, "mode must be PLAIN or GROW");
  if (mode == MPS_TRUNC_GROW && chi_max < 1) return set_error(MPS_ERR_ARG, "chi_max must be >= 1");
  if (chi[0] != 1 || chi[L] != 1) return set_error(MPS_ERR_ARG, "a finite chain has chi = 1 at both ends");
  for (int m = 0; m <= L; ++m)
    if (chi[m] < 1 || chi[m] > chi_cap) return set_error(MPS_ERR_ARG, "chi[%d]=%d outside [1, chi_cap]", m, chi[m]);
  hipStream_t s = (hipStream_t)stream;
  const size_t es = prec == MPS_C128 ? 16 : 8;
  const int nb = L - 1;
  // workspace: one bond update at capacity shape, a site-sized buffer, the
  // mirrored gates and the bond matrix in storage precision, chi and eps words
  mps_bond_desc Dc{};
  Dc.d = d;
  Dc.chi_l = Dc.chi_m = Dc.chi_r = chi_cap;
  Dc.eta = mode == MPS_TRUNC_PLAIN ? chi_cap : std::min(std::min(chi_max, chi_cap), d * chi_cap);
  Dc.chi_max = Dc.eta;
  Dc.xi_is_diag = 0;
  Dc.mode = mode;
  Dc.prec = prec;
  Dc.left_iso = 1;
  int rc = check_desc(&Dc);
  if (rc) return rc;
  auto a256 = [](size_t x) { return (x + 255) & ~size_t(255); };
  const size_t bond_ws = a256(bond_work_bytes(shape_of(&Dc)));
  const size_t site_bytes = a256((size_t)chi_cap * d * chi_cap * es);
  const size_t gate_bytes = a256((size_t)nb * d * d * d * d * 16);
  const size_t cen_bytes = a256((size_t)chi_cap * chi_cap * 16);
  if ((rc = ensure_ws(c, bond_ws + site_bytes + gate_bytes + cen_bytes + 512, s))) return rc;
  char* p = (char*)c->ws;
  void* bws = p;
  void* tmp = p + bond_ws;
  c128* rgates = (c128*)(p + bond_ws + site_bytes);
  void* cen_s = p + bond_ws + site_bytes + gate_bytes;
  int* chi_dev = (int*)(p + bond_ws + site_bytes + gate_bytes + cen_bytes);
  double* eps_dev = (double*)(chi_dev + 64);
  hipLaunchKernelGGL(reflect_gates_kernel, dim3(grid_of((long long)nb * d * d * d * d)), dim3(256), 0, s,
                     (const c128*)gates_half, nb, d, rgates);
  QT_HIP_CHECK(hipGetLastError());
  g_tune = TuneParams{};
  std::vector<void*> site(sites, sites + L);
  std::vector<int> ch(chi, chi + L + 1);
  const GemmTypes ty{prec == MPS_C128 ? DT_C128 : DT_C64, prec == MPS_C128 ? DT_C128 : DT_C64};
  for (int step = 0; step < nsteps; ++step)
    for (int half = 0; half < 2; ++half) {
      const c128* g = half == 0 ? (const c128*)gates_half : rgates;
      // sweep to the right: bond b -> A~^[b] = Q^[b], bond matrix L / |L|, B~^[b+1]
      // (outputs overwrite inputs: each input is read before its output is written)
      for (int b = 0; b < nb; ++b) {
        mps_bond_desc D = Dc;
        D.chi_l = ch[b];
        D.chi_m = ch[b + 1];
        D.chi_r = ch[b + 2];
        D.eta = mode == MPS_TRUNC_PLAIN ? ch[b + 1]
                                        : std::min(std::min(chi_max, chi_cap), std::min(d * ch[b], d * ch[b + 2]));
        D.chi_max = D.eta;
        if ((rc = check_desc(&D))) return rc;
        const BondShape bs = shape_of(&D);
        if ((rc = bond_update_run(bs, bws, c->status, center, site[b], site[b + 1], g + (size_t)b * d * d * d * d,
                                  site[b], center, site[b + 1], chi_dev, eps_dev, s, nullptr, &c->qa)))
          return rc;
        ch[b + 1] = D.eta;
      }
      // the last site absorbs the bond matrix: M = Xi B^[L-1]
      const int cl = ch[L - 1];
      const void* xiA = center;
      if (prec != MPS_C128) {
        hipLaunchKernelGGL(cast_center_kernel<float>, dim3(grid_of((long long)cl * cl)), dim3(256), 0, s,
                           (const c128*)center, (long long)cl * cl, (c64*)cen_s);
        QT_HIP_CHECK(hipGetLastError());
        xiA = cen_s;
      }
      const int ncol = d * ch[L];
      if ((rc = gemm_one(gemm_prob(xiA, cl, OP_N, site[L - 1], ncol, OP_N, tmp, ncol, cl, ncol, cl), ty, s))) return rc;
      QT_HIP_CHECK(hipMemcpyAsync(site[L - 1], tmp, (size_t)cl * ncol * es, hipMemcpyDeviceToDevice, s));
      hipLaunchKernelGGL(unit_center_kernel, dim3(1), dim3(1), 0, s, (c128*)center);
      QT_HIP_CHECK(hipGetLastError());
      // mirror the chain: site m <- reflect(site L-1-m), chi reversed
      for (int m = 0; m <= (L - 1) / 2; ++m) {
        const int k = L - 1 - m;
        const long long nm = (long long)ch[m] * d * ch[m + 1], nk = (long long)ch[k] * d * ch[k + 1];
        if (prec == MPS_C128) {
          hipLaunchKernelGGL(reflect_site_kernel<double>, dim3(grid_of(nk)), dim3(256), 0, s, (const c128*)site[k],
                             ch[k], d, ch[k + 1], (c128*)tmp);
          if (k != m)
            hipLaunchKernelGGL(reflect_site_kernel<double>, dim3(grid_of(nm)), dim3(256), 0, s, (const c128*)site[m],
                               ch[m], d, ch[m + 1], (c128*)site[k]);
        } else {
          hipLaunchKernelGGL(reflect_site_kernel<float>, dim3(grid_of(nk)), dim3(256), 0, s, (const c64*)site[k],
                             ch[k], d, ch[k + 1], (c64*)tmp);
          if (k != m)
            hipLaunchKernelGGL(reflect_site_kernel<float>, dim3(grid_of(nm)), dim3(256), 0, s, (const c64*)site[m],
                               ch[m], d, ch[m + 1], (c64*)site[k]);
        }
        QT_HIP_CHECK(hipGetLastError());
        QT_HIP_CHECK(hipMemcpyAsync(site[m], tmp, (size_t)nk * es, hipMemcpyDeviceToDevice, s));
      }
      std::reverse(ch.begin(), ch.end());
    }
  std::copy(ch.begin(), ch.end(), chi);
  return MPS_OK;
}

int mps_sweep_stats(mps_ctx c, long long* out) {
  if (!c || !out) return set_error(MPS_ERR_ARG, "null argument");
  out[0] = c->stats.layers_eager;
  out[1] = c->stats.host_syncs;
  out[2] = c->stats.chunks;
  out[3] = c->stats.rollbacks;
  out[4] = c->stats.graph_captures;
  out[5] = c->stats.graph_replays;
  out[6] = c->stats.tune_trials;
  out[7] = c->stats.tune_hits;
  return MPS_OK;
}

int mps_measure(mps_ctx c, mps_state st, const void* op1, const void* op2, double* site_vals, double* norms,
                double* bond_vals, double* entropies, mps_stream stream) {
  if (!c || !st) return set_error(MPS_ERR_ARG, "null argument");
  hipStream_t s = (hipStream_t)stream;
  const int L = st->L, d = st->d;
  const size_t es = st->prec ? 8 : 16;
  int rc;
  if (op1 && (site_vals || norms)) {
    for (int m = 0; m < L; ++m) {
      const int chiL = st->chi[m], chiR = st->chi[m + 1];
      const size_t need = expect_part_doubles(chiL, chiR) * 8 + 256;
      if ((rc = ensure_ws(c, need, s))) return rc;
      if ((rc = expect_run(st->B[m], st->prec, (const double*)st->Xi[m], chiL, d, chiR, (const c128*)op1,
                           (double*)c->ws, site_vals ? site_vals + 2 * m : nullptr, norms ? norms + m : nullptr, s)))
        return rc;
    }
  }
  if (op2 && bond_vals) {
    const int nb = st->geometry == 0 ? L - 1 : 2;
    for (int b = 0; b < nb; ++b) {
      const int m = b, n = st->geometry == 0 ? b + 1 : 1 - b;
      const int chiL = st->chi[m], chiM = st->chi[n], chiR = st->geometry == 0 ? st->chi[n + 1] : st->chi[m];
      const size_t tb = (size_t)chiL * d * d * chiR * es;
      const size_t need = ((tb + 255) & ~size_t(255)) + expect_part_doubles(chiL, chiR) * 8 + 256;
      if ((rc = ensure_ws(c, need, s))) return rc;
      void* th = c->ws;
      double* part = (double*)((char*)c->ws + ((tb + 255) & ~size_t(255)));
      const int dt = st->prec ? DT_C64 : DT_C128;
      GemmProb g = gemm_prob(st->B[m], chiM, OP_N, st->B[n], d * chiR, OP_N, th, d * chiR, chiL * d, d * chiR, chiM);
      if ((rc = gemm_one(g, GemmTypes{dt, dt}, s))) return rc;
      if ((rc = expect_run(th, st->prec, (const double*)st->Xi[m], chiL, d * d, chiR, (const c128*)op2, part,
                           bond_vals + 2 * b, nullptr, s)))
        return rc;
    }
  }
  if (entropies) {
    EntropyArgs ea{};
    for (int m = 0; m < L; ++m) {
      ea.xi[m] = (const double*)st->Xi[m];
      ea.chi[m] = st->chi[m];
    }
    if ((rc = entropy_run(ea, L, entropies, s))) return rc;
  }
  return MPS_OK;
}

int mps_zgemm(mps_ctx c, int dt, int opA, int opB, int M, int N, int K, const void* A, long long lda, const void* B,
              long long ldb, void* C, long long ldc, double alpha, double beta, mps_stream stream) {
  if (!c || !A || !B || !C) return set_error(MPS_ERR_ARG, "null argument");
  if (dt != DT_C64 && dt != DT_C128) return set_error(MPS_ERR_ARG, "dt must be 0 or 1");
  if (opA < 0 || opA > 2 || opB < 0 || opB > 2) return set_error(MPS_ERR_ARG, "op must be 0, 1 or 2");
  if (M < 0 || N < 0 || K < 0) return set_error(MPS_ERR_ARG, "negative size");
  if (beta != 0.0 && beta != 1.0) return set_error(MPS_ERR_ARG, "beta must be 0 or 1");
  GemmProb g = gemm_prob(A, lda, opA, B, ldb, opB, C, ldc, M, N, K, (float)alpha, (float)beta);
  return gemm_one(g, GemmTypes{dt, dt}, (hipStream_t)stream);
}

int mps_qr(mps_ctx c, int dt, int m, int n, void* A, void* Q, mps_stream stream) {
  if (!c || !A || !Q) return set_error(MPS_ERR_ARG, "null argument");
  if (dt != DT_C64 && dt != DT_C128) return set_error(MPS_ERR_ARG, "dt must be 0 or 1");
  if (n < 1 || n > m) return set_error(MPS_ERR_ARG, "need 1 <= n <= m");
  if (m > kMaxQrRows) return set_error(MPS_ERR_CAPACITY, "m=%d too large", m);
  const int es = dt == DT_C128 ? 16 : 8;
  hipStream_t s = (hipStream_t)stream;
  int rc;
  if ((rc = ensure_ws(c, qr_work_bytes(m, n, es, n), s))) return rc;
  QrWork w = qr_work_carve(c->ws, m, n, es, n, c->status);
  g_tune = TuneParams{};
  QrJob J{A, n, m, n, A, n, n, &w};
  if ((rc = qr_factor_batch(&J, 1, dt, s, &c->qa))) return rc;
  return qr_form_q(Q, n, m, n, dt, w, s);
}

int mps_heig(mps_ctx c, int n, int k, void* G, double* lam, void* E, mps_stream stream) {
  if (!c || !G || !lam || !E) return set_error(MPS_ERR_ARG, "null argument");
  if (n < 1 || k < 1 || k > n) return set_error(MPS_ERR_ARG, "need 1 <= k <= n");
  if (n > kEigMaxN) return set_error(MPS_ERR_CAPACITY, "n=%d > %d", n, kEigMaxN);
  hipStream_t s = (hipStream_t)stream;
  int rc;
  if ((rc = ensure_ws(c, eig_work_bytes(n), s))) return rc;
  EigWork w = eig_work_carve(c->ws, n, c->status);
  g_tune = TuneParams{};
  return eig_herm_top((c128*)G, n, k, lam, (c128*)E, w, s);
}

}  // extern "C"
