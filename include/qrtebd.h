/*
 * qrtebd.h -- C ABI of the MI355X QR-TEBD bond-update library (libqrtebd.so).
 *
 * Implements the QR-based truncation of a two-site TEBD update from
 * J. Unfried, J. Hauschild, F. Pollmann, "Fast Time-Evolution of
 * Matrix-Product States using the QR decomposition" (arXiv:2212.09782):
 * Sec. II steps (i)-(iii) (plain QR truncation and Hastings' form of the new
 * left tensor), the heuristic bond growth at the end of Sec. II, and
 * controlled bond expansion, Sec. III steps (i)-(v).
 *
 * Conventions
 *  - Every tensor argument is a device pointer to contiguous row-major,
 *    interleaved complex data (complex128 = 2 doubles, complex64 = 2 floats).
 *    The caller allocates all of them; the library allocates only its own
 *    workspace inside an mps_ctx.
 *  - Site tensor B[chi_l][d][chi_r] in right-isometric form
 *    (sum_{i,b} B[a][i][b] conj(B[a'][i][b]) = delta(a,a'), Sec. II).
 *  - Bond matrix Xi^[m] (the bond LEFT of site m, Sec. II): either a real
 *    vector of chi_l doubles (diagonal, e.g. Schmidt values) or a dense
 *    chi_l x chi_l complex128 matrix.  Xi is always FP64.
 *  - Two-site gate U: (d*d) x (d*d) complex128 acting on |i>|j>, row index
 *    i*d + j with i the left site (the gate sum of Sec. II step (i)).
 *  - Precision: MPS_C128 keeps site tensors in complex128 and computes in
 *    FP64; MPS_MIXED_C64 keeps them in complex64, runs the contractions and
 *    trailing updates on FP32 matrix cores and keeps FP64 for Householder
 *    panel arithmetic, the eigen-decomposition, the re-orthogonalisation of
 *    the new right tensor and the normalisation of Xi.
 *  - All calls are asynchronous on the given HIP stream (hipStream_t passed
 *    as mps_stream).  Outputs are valid once the stream is synchronised.
 *  - Return value: MPS_OK (0) or a negative status; mps_last_error() gives a
 *    thread-local message.  Argument errors are found on the host before any
 *    launch.  Numeric trouble found on the device (non-finite norms, a zero
 *    wave function, a stalled grid barrier) is latched in the context and
 *    reported by the next mps_sync().
 *  - One mps_ctx per host thread; a context is not thread-safe.
 */
#ifndef QRTEBD_H
#define QRTEBD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ihipStream_t* mps_stream; /* a hipStream_t; NULL = default stream */

enum {
  MPS_OK = 0,
  MPS_ERR_ARG = -1,      /* bad argument (shape, mode, null pointer) */
  MPS_ERR_CAPACITY = -2, /* a size exceeds what the kernels support */
  MPS_ERR_OOM = -3,      /* workspace allocation failed */
  MPS_ERR_HIP = -4,      /* a HIP runtime call failed */
  MPS_ERR_NUMERIC = -5,  /* latched device-side numeric error (see mps_sync) */
  MPS_ERR_STATE = -6     /* object used in a wrong state */
};

typedef enum { MPS_C128 = 0, MPS_MIXED_C64 = 1 } mps_precision;

/* Truncation scheme.  PLAIN: Sec. II with Y0 = B^[n] (eta = chi_m, no
 * truncation beyond the QR projection).  GROW: Sec. II bond growth, Y0 = the
 * first eta rows of theta~.  CBE: Sec. III, Y0 = the first eta rows of
 * theta~, then the eigen-decomposition of L^dag L and truncation. */
typedef enum { MPS_TRUNC_PLAIN = 0, MPS_TRUNC_GROW = 1, MPS_TRUNC_CBE = 2 } mps_trunc;

typedef struct mps_ctx_s* mps_ctx;

/* One bond update (m, n = m+1).
 *  d               physical dimension
 *  chi_l, chi_m, chi_r  dimensions of the bond left of m, between m and n,
 *                  right of n
 *  eta             dimension of the QR / LQ step: PLAIN requires
 *                  eta == chi_m; GROW and CBE require
 *                  1 <= eta <= min(d chi_l, d chi_r) (Sec. III: eta = chi + dchi);
 *                  CBE also needs eta <= 1536 (the eigensolver's limit,
 *                  MPS_ERR_CAPACITY beyond)
 *  chi_max         CBE only: keep at most chi_max Schmidt values
 *  svd_min         CBE only: drop Schmidt values below svd_min (absolute;
 *                  the paper uses 1e-14); at least one value is kept
 *  xi_is_diag      1: xi_m is a real vector of chi_l doubles; 0: dense
 *  mode, prec      see above
 *  sweeps          QR/LQ sweeps on theta~ (0 or 1: one, as in Sec. II);
 *                  more repeat steps (i)-(ii) from Y0 = Q^[n] of the
 *                  previous sweep, the alternating-least-squares reading of
 *                  the Sec. II comments (for gates far from the identity);
 *                  at most 16.  Appended field: a zero-initialised
 *                  descriptor keeps the single sweep. */
typedef struct {
  int d, chi_l, chi_m, chi_r;
  int eta;
  int chi_max;
  double svd_min;
  int xi_is_diag;
  int mode;
  int prec;
  int sweeps;
  int left_iso;   /* PLAIN / GROW only (appended field, zero: Hastings' form):
                     b_m_out receives the left-isometric A~^[m] = Q^[m],
                     [chi_l][d][eta], instead of B~^[m] (Sec. II comments) */
} mps_bond_desc;

/* Create / destroy a context on HIP device `device`.  Workspace grows on
 * demand and is kept until destruction.
 * autotune_cache: NULL (or "") keeps the default launch shapes.  Otherwise
 * the path of a text file of tuned launch shapes (QR panel blocks, rows per
 * block of the tridiagonalisation) per workload, read at creation (a missing
 * file is an empty cache) and appended to: the first mps_bond_update of a
 * bond shape, and the first speculative chunk of an mps_sweep step shape,
 * that the cache does not hold times each candidate on the workload itself
 * (a sweep step is undone after each trial) and keeps the fastest.  Several
 * contexts may share a file; results depend on the shapes chosen only at
 * rounding level.  The precision is not a context property: every bond
 * descriptor and state carries its own, so one context serves both. */
int mps_ctx_create(int device, const char* autotune_cache, mps_ctx* out);
int mps_ctx_destroy(mps_ctx ctx);

/* Thread-local text of the last error. */
const char* mps_last_error(void);

/* Wait for `stream` and report (then clear) latched device errors:
 * MPS_ERR_NUMERIC if any kernel latched one since the last call. */
int mps_sync(mps_ctx ctx, mps_stream stream);

/* Capacity of the new bond: eta for PLAIN / GROW, min(eta, chi_max) for CBE.
 * Output buffers of mps_bond_update must hold this many columns / rows. */
int mps_bond_capacity(const mps_bond_desc* desc);

/* Bytes of workspace a bond of this shape needs (for budgeting). */
int mps_workspace_query(mps_ctx ctx, const mps_bond_desc* desc, size_t* bytes);

/* The two-site update of Sec. II / III: from Xi^[m], B^[m], B^[n] and U
 * compute B~^[m], Xi~^[n] (the new bond between m and n) and B~^[n].
 *  xi_m      chi_l doubles (diag) or chi_l x chi_l complex128
 *  b_m, b_n  [chi_l][d][chi_m], [chi_m][d][chi_r]  (complex128 or complex64)
 *  u         (d*d) x (d*d) complex128
 *  b_m_out   [chi_l][d][chi~]   written compactly with the live chi~
 *  xi_n_out  CBE: chi~ doubles (normalised Schmidt values, descending);
 *            PLAIN / GROW: eta x eta complex128 lower-triangular L / |L|_F
 *  b_n_out   [chi~][d][chi_r]
 *  chi_new_dev  device int: chi~ (== eta for PLAIN / GROW)
 *  trunc_err_dev device double: |theta~ - approx|^2 / |theta~|^2 (end of Sec. IV)
 * Inputs are read only; outputs must not alias inputs.  Output buffers must
 * hold mps_bond_capacity(desc) along the new bond. */
int mps_bond_update(mps_ctx ctx, const mps_bond_desc* desc, const void* xi_m, const void* b_m,
                    const void* b_n, const void* u, void* b_m_out, void* xi_n_out, void* b_n_out,
                    int* chi_new_dev, double* trunc_err_dev, mps_stream stream);

/* The comparison schemes of Sec. IV on the GPU, complex128 only: the same
 * two-site contraction, gate and Hastings form as mps_bond_update, with the
 * truncation of theta~ taken from its SVD (scheme 0: theta~ = U S V^dag,
 * B~^[n] = V_kept^dag) or from the eigen-decomposition of theta~^dag theta~
 * (scheme 1, EIG).  Both use the rocSOLVER library (gesvd / heevd): they are
 * baselines for the QR schemes, not part of them.  desc: mode CBE (chi_max,
 * svd_min as there), prec MPS_C128; eta and sweeps are ignored.  Outputs as
 * for CBE with capacity min(chi_max, d chi_l, d chi_r).  MPS_ERR_HIP if the
 * solver library fails; a failed decomposition (info != 0) is latched. */
int mps_bond_update_reference(mps_ctx ctx, const mps_bond_desc* desc, int scheme, const void* xi_m, const void* b_m,
                              const void* b_n, const void* u, void* b_m_out, void* xi_n_out, void* b_n_out,
                              int* chi_new_dev, double* trunc_err_dev, mps_stream stream);

/* mps_bond_update without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid hipMalloc).  Same arguments, outputs and errors as
 * mps_bond_update; the workspace is a fixed 128 MiB device array per GPU
 * (allocated when the library is loaded, kept until the process ends), so
 * the call makes no hipMalloc / hipFree.  Bonds whose workspace
 * (mps_workspace_query) exceeds 128 MiB return MPS_ERR_CAPACITY (d = 5:
 * chi up to about 256 with eta = chi + chi/10, either precision).  Every call
 * on one GPU, from any context, shares that array: calls that overlap on one
 * GPU (other streams, other threads) race and must be serialised by the
 * caller.  Each call zeroes what it needs zeroed. */
int mps_bond_update_noalloc(mps_ctx ctx, const mps_bond_desc* desc, const void* xi_m, const void* b_m,
                            const void* b_n, const void* u, void* b_m_out, void* xi_n_out, void* b_n_out,
                            int* chi_new_dev, double* trunc_err_dev, mps_stream stream);

/* Two-site Trotter gate of the d-state clock model (Sec. IV):
 * U = expm(-i tau h), h = -(Z (x) Z^dag + h.c.) - g (wl (X+X^dag) (x) 1 +
 * wr 1 (x) (X+X^dag)), Z = diag(w^k), w = exp(2 pi i/d), X the cyclic shift.
 * wl / wr: share of each site's transverse field carried by this bond.
 * Host computation (FP64); u_out: host array of (d*d)^2 complex128. */
int mps_clock_gate(int d, double g, double tau, double wl, double wr, double* u_out);

/* The bond Hamiltonian h of mps_clock_gate itself (Sec. IV), for energy
 * measurements with mps_measure; h_out: host array of (d*d)^2 complex128. */
int mps_clock_hamiltonian(int d, double g, double wl, double wr, double* h_out);

/* ---- Z_d block structure (Sec. III, closing paragraph; Sec. IV) -----------
 * The clock model conserves the Z_d charge generated by prod_i X_i.  In the
 * eigenbasis of X (charge basis: |q> = d^-1/2 sum_k w^(q k) |k>, X|q> = w^q |q>,
 * Z|q> = |q+1>) the bond gate conserves q_i + q_j mod d and an MPS of definite
 * charge is block sparse: every bond splits into d charge sectors, and
 * B[alpha, q, beta] vanishes unless charge(beta) = charge(alpha) + q mod d.
 * Controlled bond expansion then sets the sector sizes dynamically: each
 * block is expanded and one truncation over all blocks keeps the largest
 * Schmidt values. */

/* The gate and bond Hamiltonian of mps_clock_gate / mps_clock_hamiltonian in
 * the charge basis (same arguments; host arrays of (d*d)^2 complex128). */
int mps_clock_gate_charge(int d, double g, double tau, double wl, double wr, double* u_out);
int mps_clock_hamiltonian_charge(int d, double g, double wl, double wr, double* h_out);

#define MPS_SYM_MAX_D 16
/* One bond (m, n) with the block structure.  sec_l / sec_m / sec_r: sector
 * sizes (charge 0 .. d-1) of the bond left of m, of the bond (m, n) and of
 * the bond right of n; each bond's index runs over its sectors in charge
 * order.  Sector c of the bond (m, n) is expanded to
 *   eta_c = min(sec_m[c] + max(dchi_min, ceil(dchi_frac sec_m[c])), chi_l, chi_r)
 * (chi_l, chi_r: the outer bonds' total sizes, which bound every block; a
 * sector with eta_c = 0 stays empty); the update then keeps the Schmidt
 * values S >= svd_min, at most chi_max of them over all sectors, at least
 * one, ranked by S^2 with ties to the lower charge. */
typedef struct {
  int d;                      /* 2 .. MPS_SYM_MAX_D */
  int sec_l[MPS_SYM_MAX_D];
  int sec_m[MPS_SYM_MAX_D];
  int sec_r[MPS_SYM_MAX_D];
  int dchi_min;
  double dchi_frac;
  int chi_max;
  double svd_min;
  int prec;                   /* mps_precision */
} mps_sym_desc;

/* Capacity of the new bond: min(chi_max, sum_c min(eta_c, chi_max)) (>= 1),
 * or a negative error code for an invalid descriptor. */
int mps_sym_capacity(const mps_sym_desc* desc);
/* Workspace the library allocates (and keeps in the context) for this update. */
int mps_sym_workspace_query(mps_ctx ctx, const mps_sym_desc* desc, size_t* bytes);

/* The CBE update (Sec. III, steps (i)-(v)) block by block: theta~ splits into
 * d blocks of middle charge c (rows (q, alpha) with charge(alpha) = c - q,
 * columns (q', beta) with charge(beta) = c + q'); each block takes steps
 * (i)-(iv) with the first eta_c of its rows as the slice of step (i); one
 * truncation over all blocks, then step (v) and Hastings' B~^[m] = C~ B~^[n]^dag
 * per block.  Tensors are dense and charge-ordered, as in mps_bond_update:
 *   xi_m      chi_l doubles: the (diagonal) bond matrix left of m
 *   b_m       [chi_l][d][chi_m], b_n [chi_m][d][chi_r] (storage precision
 *             per prec), zero outside the blocks
 *   u         (d*d)^2 complex128 gate in the charge basis (entries that
 *             change q_i + q_j are not read)
 *   b_m_out   [chi_l][d][chi~], b_n_out [chi~][d][chi_r], xi_n_out chi~
 *             doubles (unit 2-norm): compact with the new chi~, the new bond
 *             in charge order (inside a sector by descending S); capacity
 *             mps_sym_capacity elements along the new bond.  They may alias
 *             b_m / b_n (the inputs are read into blocks first).
 *   sec_out   d ints: the new sector sizes; chi_new: their sum; trunc_err:
 *             (|theta~|^2 - sum_kept S^2) / |theta~|^2
 * All pointers are device pointers owned by the caller; the call is
 * asynchronous on stream.  MPS_ERR_ARG for an invalid descriptor or a null
 * pointer, MPS_ERR_CAPACITY when a block exceeds the dense update's limits
 * (eta_c <= 1536), MPS_ERR_OOM if the workspace cannot be allocated. */
int mps_bond_update_sym(mps_ctx ctx, const mps_sym_desc* desc, const double* xi_m, const void* b_m, const void* b_n,
                        const void* u, void* b_m_out, double* xi_n_out, void* b_n_out, int* sec_out, int* chi_new,
                        double* trunc_err, mps_stream stream);

/* ---- device-resident MPS and the even/odd sweep (Fig. 2a) ---------------- */

typedef struct mps_state_s* mps_state;

/* geometry: 0 finite chain of L sites (bond b joins sites b, b+1; Xi^[0] = 1),
 *           1 uniform cell of L = 2 sites (bonds (A,B) and (B,A)).
 * b_ptrs[m]: device buffer of site m with room for chi_cap*d*chi_cap elements;
 * xi_ptrs[m]: device buffer of the bond left of site m, chi_cap doubles.
 * chi_host[m]: current dimension of the bond left of site m (chi_host[L] is
 * the right end of a finite chain, 1).  The state starts in CBE form (every
 * Xi diagonal).  Buffers stay owned by the caller and are updated in place. */
int mps_state_create(mps_ctx ctx, int geometry, int L, int d, int chi_cap, int prec,
                     void* const* b_ptrs, void* const* xi_ptrs, const int* chi_host, mps_state* out);
int mps_state_destroy(mps_state st);
/* Current bond dimensions (L + 1 entries, host copy kept by the library). */
int mps_state_chis(mps_state st, int* chi_out);

/* Sweep policy shared by all states of one call. */
typedef struct {
  int mode;         /* must be MPS_TRUNC_CBE: the states keep diagonal bond
                       matrices (plain / grow updates, whose Xi~ is a dense L,
                       run through mps_bond_update) */
  int chi_max;
  double svd_min;
  int dchi_min;     /* eta = min(chi + max(dchi_min, ceil(dchi_frac*chi)), d chi_l, d chi_r) */
  double dchi_frac;
  int sweeps;       /* QR/LQ sweeps per bond update, as in mps_bond_desc (0 or 1: one) */
  int exec;         /* 0: every layer reads the new chis back (one host
                       synchronisation per layer); 1: speculative: while the
                       chi profile is saturated (no bond update can raise any
                       chi: chi_m == min(eta, chi_max) on every bond) up to
                       `chunk` steps are issued with no host synchronisation,
                       the device checks that every chi~ equals the planned
                       one, and a chunk with a smaller chi~ is undone (state
                       restored from a copy) and rerun layer by layer; 2: as 1,
                       with each step captured once as a hipGraph (keyed by
                       the chi profile, the buffers and the policy) and
                       replayed.  Results are the same in all three modes.
                       Appended field: zero keeps mode 0. */
  int chunk;        /* steps per speculative chunk (0: 8) */
} mps_sweep_policy;

/* nsteps Trotter steps on every state.  gates[s] points to the device gates
 * of state s: [nbonds][2][(d*d)^2] complex128, index 0 for tau = dt/2 and 1
 * for tau = dt, bond b = the bond starting at site b.  order 2: even(dt/2)
 * odd(dt) even(dt/2); order 1: even(dt) odd(dt).  All even bonds of all states
 * form one batch, then all odd bonds; a batch runs in groups of bonds (in
 * order) whose workspaces together stay within 16 GiB, one group after the
 * other (a larger bond forms its own group).  trunc_err_dev (nullable): per
 * state, the summed truncation error is added to trunc_err_dev[s]. */
int mps_sweep(mps_ctx ctx, mps_state* states, int nstates, const void* const* gates, int nsteps,
              int order, const mps_sweep_policy* policy, double* trunc_err_dev, mps_stream stream);

/* Sequential sweeps on a finite chain in the left-isometric form (Sec. II
 * comments): the QR update hands back A~^[m] = Q^[m] left-isometric, so a
 * sweep to the right updates bond 0, 1, ..., L-2 in turn, each seeing the bond
 * matrix the previous update produced.  One second-order step applies the
 * gates U_b(dt/2) for b = 0 .. L-2 and then for b = L-2 .. 0; the return
 * sweep is the same update on the mirror image of the chain (site order
 * reversed, the two virtual legs of every tensor and the two sites of every
 * gate exchanged), done by transposing the tensors in place.
 *  sites[m]   device buffer of site m, [chi[m]][d][chi[m+1]], capacity
 *             chi_cap*d*chi_cap elements (complex128 or complex64 per prec);
 *             right-isometric on entry and on return
 *  center     device buffer of chi_cap*chi_cap complex128: the bond matrix
 *             left of site 0, [[1]] on entry and on return (the norm is kept
 *             in the sites)
 *  chi        host array of L+1 bond dimensions (chi[0] = chi[L] = 1), in/out
 *  gates_half device [L-1][(d*d)^2] complex128: U_b(dt/2) of bond b
 *  mode       MPS_TRUNC_PLAIN (eta = chi_m: dimensions fixed) or
 *             MPS_TRUNC_GROW (eta = min(chi_max, chi_cap, d chi_l, d chi_r))
 * Each bond's new matrix is L / |L|_F.  Bonds run one after another (each
 * depends on the previous one); no host synchronisation. */
int mps_sweep_sequential(mps_ctx ctx, int L, int d, int chi_cap, int prec, void* const* sites, void* center,
                         int* chi, const void* gates_half, int nsteps, int mode, int chi_max, mps_stream stream);

/* Counters of the context since its creation (8 entries): layers run with a
 * chi read-back, host synchronisations inside mps_sweep, speculative chunks,
 * chunks undone, step graphs captured, step graphs replayed, autotuner trial
 * runs, workloads whose launch shapes came from the autotune cache. */
int mps_sweep_stats(mps_ctx ctx, long long* out8);

/* Observables from the isometric form (Fig. 1c):
 *  site_vals  [L][2] doubles: <op1> at every site from M = Xi^[m] B^[m],
 *             as complex (re, im), divided by |M|^2
 *  norms      [L] doubles: |M|^2 (1 for an exact right-isometric state)
 *  bond_vals  [nbonds][2] doubles: <op2> on every bond from theta = Xi B B,
 *             divided by |theta|^2 (op2 (d*d)^2 complex128, nullable)
 *  entropies  [L] doubles: von Neumann entropy of every bond left of a site
 *             from Xi (-sum p ln p, p = s^2 / sum s^2)
 * op1, op2 are device complex128 matrices; outputs are device buffers
 * (each nullable).  For a finite chain nbonds = L-1, for the cell 2. */
int mps_measure(mps_ctx ctx, mps_state st, const void* op1, const void* op2, double* site_vals,
                double* norms, double* bond_vals, double* entropies, mps_stream stream);

/* ---- profiling ------------------------------------------------------------
 * When enabled, the context records a HIP event pair on the call's stream
 * around every launch of the contraction GEMMs of the bond update (C = B B,
 * X, Y^dag, B~[n], B~[m]; the dominant kernel class) together with its
 * algorithmic flop count 8 M N K, for up to max_launches launches.
 * mps_profile_read waits for the recorded events and returns the summed
 * kernel time (ms), the summed flops and the number of launches since the
 * last mps_profile_enable. */
int mps_profile_enable(mps_ctx ctx, int on, int max_launches);
int mps_profile_read(mps_ctx ctx, double* total_ms, double* total_flops, int* launches);

/* ---- building blocks of the update, exported for checking and reuse ------
 * dt: 0 complex64, 1 complex128.  All matrices row-major device buffers. */

/* C = alpha op(A) op(B) + beta C (op: 0 none, 1 transpose, 2 conjugate
 * transpose; op(A) M x K, op(B) K x N) on the matrix cores; alpha, beta real. */
int mps_zgemm(mps_ctx ctx, int dt, int opA, int opB, int M, int N, int K, const void* A, long long lda,
              const void* B, long long ldb, void* C, long long ldc, double alpha, double beta, mps_stream stream);

/* Thin Householder QR of the m x n matrix A (n <= m, ld n): on return A
 * holds R in its upper triangle (below it: the reflectors) and Q (m x n,
 * ld n) the explicit orthonormal factor, A_in = Q R.  Used for both QR steps
 * of Sec. II (the LQ of Y is the QR of Y^dag). */
int mps_qr(mps_ctx ctx, int dt, int m, int n, void* A, void* Q, mps_stream stream);

/* The k largest eigenpairs of the Hermitian n x n complex128 matrix G
 * (destroyed; 1 <= k <= n <= 1536, MPS_ERR_CAPACITY for larger n): lam (k doubles, descending) and E (n x k complex128, ld k,
 * orthonormal columns).  The FP64 eigensolver of Sec. III step (iv). */
int mps_heig(mps_ctx ctx, int n, int k, void* G, double* lam, void* E, mps_stream stream);

#ifdef __cplusplus
}
#endif

#endif /* QRTEBD_H */
