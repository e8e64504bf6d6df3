/*
 * dgtns.h -- C-ABI of libdgtns: the discrete Gabor transform on a
 * nonseparable lattice by the shear method, on AMD Instinct MI355X (gfx950).
 *
 * Transform (eq. (DGT), Section 2.1).  For a signal f and a window g of
 * length L, time step a, M channels (frequency step b = L/M) and lattice
 * offset lambda = lambda1/lambda2, the coefficients are
 *
 *     c(m, n) = sum_{l in Z_L} f(l) conj(g(l - n a)) exp(-2 pi i l (m + w(n)) / M),
 *     w(n)    = (n lambda1 mod lambda2) / lambda2,   m in Z_M, n in Z_N, N = L/a.
 *
 * (The paper's window argument "l - an + 1" is read as the 0-based l - n a.)
 * The library computes this with the shear algorithm (Alg. 1): a time shear
 * and, when needed, a frequency shear (Thm. 2) applied as chirp
 * multiplications (Lemma 1), a separable DGT by window factorisation
 * (the full-window algorithm of Section 4), and a phase/index correction
 * (Prop. 7).
 *
 * Conventions for every call:
 *   - Complex data is interleaved (re, im).  DGTNS_C64 plans use float,
 *     DGTNS_C128 plans double, for signals, coefficients and windows given to
 *     the hot-path calls; windows given to dgtns_set_window,
 *     dgtns_dual_window and dgtns_tight_window are always complex128.
 *   - Signal layout f[B][L] (contiguous), coefficient layout c[B][N][M]:
 *     coefficient (m, n) of signal k at c[(k N + n) M + m] (channel fastest).
 *   - All pointers named *_dev are device pointers on the current HIP device.
 *     The caller owns all memory: the library never allocates device memory.
 *     Persistent plan memory is handed over once with dgtns_plan_bind, and
 *     each call takes a caller-provided workspace whose size is given by
 *     dgtns_workspace_bytes.
 *   - Device work is enqueued asynchronously on `stream` (a hipStream_t; NULL
 *     means the default stream).  Calls return after enqueueing.
 *   - Argument, state and size errors (DGTNS_EINVAL, DGTNS_ESTATE,
 *     DGTNS_EWORKSPACE, DGTNS_EUNSUPPORTED) are detected synchronously before
 *     any work of the call is enqueued: every call first checks each of its
 *     launches (LDS request, transform sizes) without enqueueing, and
 *     dgtns_check_op runs the same checks on the host alone.  Outputs are then
 *     left untouched.  Launch failures return DGTNS_EDEVICE.  No call throws
 *     across the ABI.  A message for the last error of the calling thread is
 *     available from dgtns_last_error().
 *   - Between two dgtns_set_window calls a plan is immutable: calls on one plan
 *     may run concurrently on different streams if each uses its own
 *     workspace.  dgtns_set_window rewrites the plan's window tables and must
 *     not overlap other calls on the plan.
 */
#ifndef DGTNS_H
#define DGTNS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dgtns_plan_s* dgtns_plan;

enum dgtns_status {
  DGTNS_OK = 0,
  DGTNS_EINVAL = 1,       /* bad argument (null pointer, non-positive size, bad dtype, ...) */
  DGTNS_ELATTICE = 2,     /* (L, a, M, lambda) is not a lattice of Z_L^2 (Prop. 1, Prop. 8) */
  DGTNS_ENOTFRAME = 3,    /* the frame operator is singular (dual window does not exist) */
  DGTNS_EUNSUPPORTED = 4, /* valid lattice outside the implemented sizes (see message) */
  DGTNS_EDEVICE = 5,      /* a HIP call or kernel launch failed */
  DGTNS_EWORKSPACE = 6,   /* workspace too small, or persistent memory too small */
  DGTNS_ESTATE = 7        /* plan not bound, or window not set */
};

enum dgtns_dtype { DGTNS_C64 = 0, DGTNS_C128 = 1 };

enum dgtns_branch {
  DGTNS_SEPARABLE = 0,  /* lambda = 0: no shear */
  DGTNS_TIME_SHEAR = 1, /* s0 = 0: time shear only (Alg. 1, first branch) */
  DGTNS_FREQ_SHEAR = 2, /* s0 != 0: frequency and time shear (Alg. 1, second branch) */
  DGTNS_MULTIWINDOW = 3, /* multiwindow algorithm: lambda2 coset windows (Prop. 4, Prop. 5) */
  DGTNS_FIR = 4,         /* FIR-window algorithm (dgtns_plan_create_fir) */
  DGTNS_SHEAR_OLA = 5    /* shear algorithm on overlap-added blocks (dgtns_plan_create_ola) */
};

/* Algorithm of a plan (dgtns_plan_create_alg). */
enum dgtns_algorithm {
  DGTNS_ALG_SHEAR = 0,      /* shear algorithm, Alg. 1 (dgtns_plan_create) */
  DGTNS_ALG_MULTIWINDOW = 1, /* multiwindow algorithm, Section 3.1 (Prop. 4, Prop. 5) */
  DGTNS_ALG_FIR = 2,         /* FIR-window algorithm: use dgtns_plan_create_fir */
  DGTNS_ALG_SHEAR_OLA = 3,   /* shear-OLA algorithm: use dgtns_plan_create_ola */
  DGTNS_ALG_AUTO = 4         /* shear or multiwindow, chosen by the plan (dgtns_plan_create_alg) */
};

enum dgtns_op {
  DGTNS_OP_FORWARD = 0,
  DGTNS_OP_ADJOINT = 1,
  DGTNS_OP_WINDOW_GRAD = 2,
  DGTNS_OP_SET_WINDOW = 3,
  DGTNS_OP_DUAL = 4
};

typedef struct {
  int64_t L, a, M, lambda1, lambda2;
  int64_t b;        /* frequency step L/M */
  int64_t N;        /* number of time positions L/a */
  int64_t s;        /* absolute shear of the normal form, b lambda1 / lambda2 (Section 2.1) */
  int64_t s0, s1;   /* frequency shear and time shear, A = U_{s0,s1} D V (Thm. 2) */
  int64_t b_r;      /* frequency step of the sheared separable lattice (Alg. 1) */
  int32_t branch;   /* enum dgtns_branch */
  int32_t dtype;    /* enum dgtns_dtype */
  /* separable lattice the factorised DGT runs on, and its constants c, d, p, q
     (eq. (cd), eq. (pq)): time step inner_a, inner_M channels */
  int64_t inner_a, inner_M, c, d, p, q;
  int64_t max_batch;
  size_t persistent_bytes; /* device bytes dgtns_plan_bind needs */
  int64_t windows;         /* windows of the separable lattice: 1, or lambda2 (multiwindow) */
  /* shear-OLA plans: block length L_b and the length L_x of the DGT each
     zero-extended block runs (0 for other plans) */
  int64_t block, block_dgt_length;
  /* real-signal layout (dgtns_forward_real): values per group of lambda2
     time positions; a signal's coefficients are (N / lambda2) real_row values */
  int64_t real_row;
} dgtns_plan_info_t;

/* Human-readable name of a status code (static storage). */
const char* dgtns_status_string(int status);

/* Message of the last error raised on the calling thread ("" if none). */
const char* dgtns_last_error(void);

/*
 * Create a plan (host only; no device work).  Validates the lattice (a | L,
 * M | L, 0 <= lambda1 < lambda2 coprime, lambda = 0 written 0/1, and L a
 * multiple of lambda2 lcm(a, M), Prop. 8), finds the shear factorisation
 * (Thm. 2; a time shear alone when a | s + k b, Prop. 9) and builds all
 * tables on the host.  dtype is enum dgtns_dtype; max_batch bounds B in later
 * calls.  Errors: DGTNS_EINVAL, DGTNS_ELATTICE, DGTNS_EUNSUPPORTED (transform
 * lengths that are not 7-smooth or exceed the in-LDS limit, L > 2^30).
 * On success *plan owns host memory released by dgtns_plan_destroy.
 */
int dgtns_plan_create(dgtns_plan* plan, int64_t L, int64_t a, int64_t M, int64_t lambda1,
                      int64_t lambda2, int dtype, int64_t max_batch);

/*
 * Create a plan for a chosen algorithm (enum dgtns_algorithm).
 * DGTNS_ALG_SHEAR is dgtns_plan_create.  DGTNS_ALG_MULTIWINDOW computes the
 * same coefficients by the multiwindow decomposition (Section 3.1): the
 * lattice is the union of lambda2 cosets of the separable lattice
 * (lambda2 a, M) (Prop. 4), and with n = nt lambda2 + mu
 *     c(m, n) = exp(-2 pi i nt lambda2 a sigma_mu / L) c_mu(m, nt),
 * c_mu the separable DGT with window g_mu(l) = exp(2 pi i l sigma_mu / L)
 * g(l - mu a), sigma_mu = (mu s) mod b (Prop. 5).  The lambda2 windows share
 * one column transform of the signal.  Such a plan runs dgtns_forward,
 * dgtns_forward_batch and dgtns_adjoint; dgtns_window_grad returns
 * DGTNS_EUNSUPPORTED.  DGTNS_ALG_FIR is refused here (DGTNS_EINVAL): it needs the
 * window support of dgtns_plan_create_fir.  dgtns_plan_info reports branch DGTNS_MULTIWINDOW,
 * s0 = s1 = 0, inner_a = lambda2 a, q per window and windows = lambda2; the
 * persistent memory holds lambda2 window tables.  Errors as for
 * dgtns_plan_create, plus DGTNS_EINVAL for an unknown algorithm.
 * DGTNS_ALG_AUTO chooses between the two (Section 4.4: the multiwindow
 * algorithm is the fast one for simple lattices, the shear algorithm for
 * complex ones): the shear plan, unless its factorisation needs a frequency
 * shear (s0 != 0) and the multiwindow lattice (lambda2 a, M) has
 * p = lambda2 a / gcd(lambda2 a, M) <= 15, in which case the multiwindow plan
 * (when the multiwindow kernels cover the lattice).  dgtns_plan_info's
 * branch tells which was chosen.
 */
int dgtns_plan_create_alg(dgtns_plan* plan, int64_t L, int64_t a, int64_t M, int64_t lambda1,
                          int64_t lambda2, int dtype, int64_t max_batch, int algorithm);

/*
 * Create a plan for a window of short support (the FIR-window algorithm of
 * Section 4, the weighted overlap-add DGT; Table 1's multiwindow FIR row on
 * a nonseparable lattice).  The window is taken to be zero outside the g_len
 * samples g_start, ..., g_start + g_len - 1 (mod L): dgtns_set_window keeps
 * only those samples, and the coefficients are eq. (DGT) for that truncated
 * window.  Per time position n the windowed samples f(l) conj(g(l - n a)) are
 * modulated by exp(-2 pi i l w(n) / M), folded modulo M and transformed by
 * one M-point DFT: no intermediate array, about 8 L g_len / a + 4 N M log2 M
 * flops.  M must be 7-smooth and at most 4096; any lattice of
 * dgtns_plan_create.  Such a plan runs dgtns_forward, dgtns_forward_batch
 * and dgtns_adjoint (workspace: M N values per signal);
 * dgtns_window_grad, dgtns_dual_window and dgtns_tight_window return
 * DGTNS_EUNSUPPORTED.  dgtns_plan_info reports branch DGTNS_FIR and c = d =
 * p = q = 0.  Errors as for dgtns_plan_create, plus DGTNS_EINVAL for g_len
 * outside [1, L].
 */
int dgtns_plan_create_fir(dgtns_plan* plan, int64_t L, int64_t a, int64_t M, int64_t lambda1,
                          int64_t lambda2, int dtype, int64_t max_batch, int64_t g_start, int64_t g_len);

/*
 * Create a plan for the shear-OLA algorithm (Section 4): the shear algorithm
 * applied to blocks of the signal, combined by overlap-add, for a window of
 * short support g_start, ..., g_start + g_len - 1 (mod L) as in
 * dgtns_plan_create_fir.  The signal is cut into L / block blocks of block
 * samples; each block, zero-extended, is transformed on the same lattice at
 * a length L_x of about block + g_len (the least feasible one, reported as
 * block_dgt_length), so the sheared window spans L_x samples instead of L.
 * The block transform is the automatic plan of dgtns_plan_create_alg
 * (DGTNS_ALG_AUTO): the shear algorithm, or the multiwindow algorithm where
 * the shear algorithm would need a frequency shear;
 * dgtns_plan_create_ola_alg selects it.  The coefficients of each block are multiplied
 * by the exact phase of its position and added into eq. (DGT)'s
 * coefficients; the result equals eq. (DGT) with the truncated window.  The
 * work grows by the factor rho = L_x / block (eq. (OLA-eff)).  block must
 * divide L and be a multiple of lambda2 a, and max_batch * L / block must not
 * exceed 65535.  Such a plan runs dgtns_forward and dgtns_adjoint (and
 * their real-signal variants); the adjoint takes each stage's adjoint in
 * reverse order: every block receives the global coefficients of its
 * positions times the conjugate position phases, the inner plan synthesises
 * all blocks as one batch, and each block's own samples form the signal.
 * dgtns_forward_batch, dgtns_window_grad, dgtns_dual_window and
 * dgtns_tight_window return DGTNS_EUNSUPPORTED.  dgtns_plan_info reports branch
 * DGTNS_SHEAR_OLA with the inner plan's s0, s1, b_r, c, d, p, q and windows.  Errors as
 * for dgtns_plan_create_fir, plus DGTNS_EINVAL for a bad block length and
 * DGTNS_EUNSUPPORTED when no feasible block length below L exists.
 */
int dgtns_plan_create_ola(dgtns_plan* plan, int64_t L, int64_t a, int64_t M, int64_t lambda1,
                          int64_t lambda2, int dtype, int64_t max_batch, int64_t g_start, int64_t g_len,
                          int64_t block);

/*
 * dgtns_plan_create_ola with the algorithm of the block transform:
 * DGTNS_ALG_SHEAR (Alg. 1 on every block, Section 4's shear-OLA as stated),
 * DGTNS_ALG_MULTIWINDOW or DGTNS_ALG_AUTO (as dgtns_plan_create_ola).
 * DGTNS_EINVAL for another algorithm.
 */
int dgtns_plan_create_ola_alg(dgtns_plan* plan, int64_t L, int64_t a, int64_t M, int64_t lambda1,
                              int64_t lambda2, int dtype, int64_t max_batch, int64_t g_start, int64_t g_len,
                              int64_t block, int inner_algorithm);

/* Fill *info (host only). */
int dgtns_plan_info(dgtns_plan plan, dgtns_plan_info_t* info);

/*
 * Hand the plan its persistent device memory (persistent_bytes from
 * dgtns_plan_info, 256-byte aligned) and upload the tables on `stream`.
 * Blocks until the upload has finished.  The memory stays owned by the
 * caller and must outlive every call on the plan.  Errors: DGTNS_EINVAL,
 * DGTNS_EWORKSPACE (bytes too small), DGTNS_EDEVICE.
 */
int dgtns_plan_bind(dgtns_plan plan, void* persistent_dev, size_t bytes, void* stream);

/* Workspace bytes needed by operation `op` (enum dgtns_op) for a batch of B. */
int dgtns_workspace_bytes(dgtns_plan plan, int op, int64_t B, size_t* bytes);

/*
 * Set the analysis window g_dev (complex128, length L) on `stream`: applies
 * the time-shear chirp, the frequency shear when s0 != 0 (Alg. 1: chirp,
 * length-L DFT, second chirp, division by L) and the factorisation (Zak)
 * transform, all in FP64, and stores the result in the plan's precision.
 * Needs the plan bound.  Workspace: dgtns_workspace_bytes(DGTNS_OP_SET_WINDOW).
 */
int dgtns_set_window(dgtns_plan plan, const void* g_dev, void* ws, size_t ws_bytes, void* stream);

/*
 * Forward transform (Alg. 1): c_dev[B][N][M] = DGT of f_dev[B][L].  If
 * real_input != 0, f_dev holds real samples (float or double by the plan
 * dtype) and is read as complex with zero imaginary part.  Needs the window
 * set.  Workspace: dgtns_workspace_bytes(DGTNS_OP_FORWARD, B).
 */
int dgtns_forward(dgtns_plan plan, const void* f_dev, int real_input, void* c_dev, int64_t B,
                  void* ws, size_t ws_bytes, void* stream);

/*
 * Real-signal variant (Section 4.4 names a real-signal entry point beside the
 * complex one without specifying it; this is the reading).  For a real
 * signal and a real window, conjugating eq. (DGT) gives the coefficient of
 * the negated frequency at the same time position; it lies on column n
 * exactly when e(n) = 2 w(n) is an integer (w(n) in {0, 1/2}), so then
 *     c((-m - e(n)) mod M, n) = conj(c(m, n))
 * and channels 0 .. floor(M/2) determine the column.  The other columns are
 * not redundant.  w(n) depends on n mod lambda2: the half columns are
 * n = 0 and, for even lambda2, n = lambda2/2 (mod lambda2).
 *
 * Layout of a signal's coefficients (real_row = S from dgtns_plan_info):
 * (N / lambda2) rows of S values; column n = j lambda2 + k starts at
 * j S + off(k) and holds cnt(k) channels 0 .. cnt(k)-1, with
 * cnt(k) = floor(M/2) + 1 for the half columns and M for the others, and
 * off(k) = sum of cnt(k') over k' < k.  For lambda2 <= 2 this is an
 * N x (floor(M/2) + 1) array.  c_dev is [B][N/lambda2][S] (plan dtype,
 * complex); f_dev holds B real signals of length L (float or double by the
 * plan dtype).
 *
 * dgtns_forward_real writes those channels of eq. (DGT) of the real signals
 * (any window; the omitted channels are the conjugates of stored ones only
 * when the window is real).  Workspace: DGTNS_OP_FORWARD.  Every algorithm.
 * dgtns_adjoint_real expands c_dev to the full array (an omitted channel m
 * of a half column is conj(c((-m - e(n)) mod M, n))) and writes the real
 * part of its synthesis (the adjoint of eq. (DGT)) to f_dev; with the
 * canonical dual window it inverts dgtns_forward_real.  Workspace:
 * DGTNS_OP_ADJOINT.  Every algorithm with an adjoint (not shear-OLA).
 */
int dgtns_forward_real(dgtns_plan plan, const void* f_dev, void* c_dev, int64_t B, void* ws, size_t ws_bytes,
                       void* stream);
int dgtns_adjoint_real(dgtns_plan plan, const void* c_dev, void* f_dev, int64_t B, void* ws, size_t ws_bytes,
                       void* stream);

/*
 * dgtns_forward for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * same arguments, layouts and results, without a workspace argument.  The
 * workspace lives in a static device array of DGTNS_NOALLOC_SCRATCH_BYTES
 * bytes, one per device, held from the first call on a device until the
 * process ends.  The call allocates nothing (no hipMalloc, no stream or event
 * is created; the opt-in two-stream chunk pipeline is not used).  Returns
 * DGTNS_EWORKSPACE, before enqueueing anything, if the batch needs more
 * scratch than that (dgtns_workspace_bytes(DGTNS_OP_FORWARD, B)), and
 * DGTNS_EINVAL if `stream` belongs to another device than the current one.
 * Every call on a device shares that device's array, which keeps the last
 * call's contents (the forward writes every scratch value before reading
 * it): calls that overlap on one device race, so serialise them (one stream,
 * or events between streams).
 */
#define DGTNS_NOALLOC_SCRATCH_BYTES (64ull << 20)
int dgtns_forward_noalloc(dgtns_plan plan, const void* f_dev, int real_input, void* c_dev, int64_t B,
                          void* stream);

/*
 * Forward transform of B signals that live in separate buffers (batching of
 * independent requests without staging copies): f_list and c_list are HOST
 * arrays of B device pointers, signal k read from f_list[k] (length L) and
 * its coefficients written to c_list[k] (N x M).  B <= DGTNS_MAX_LIST_BATCH.
 * Otherwise as dgtns_forward (same workspace size for the same B).
 */
#define DGTNS_MAX_LIST_BATCH 16
int dgtns_forward_batch(dgtns_plan plan, const void* const* f_list, int real_input, void* const* c_list, int64_t B,
                        void* ws, size_t ws_bytes, void* stream);

/*
 * Adjoint (synthesis) transform, the adjoint of eq. (DGT):
 * f_dev[B][L](l) = sum_{m,n} c(m, n) g(l - n a) exp(2 pi i l (m + w(n)) / M).
 * Computed as the adjoint of every stage of Alg. 1 in reverse order.
 * Workspace: dgtns_workspace_bytes(DGTNS_OP_ADJOINT, B).
 */
int dgtns_adjoint(dgtns_plan plan, const void* c_dev, void* f_dev, int64_t B, void* ws,
                  size_t ws_bytes, void* stream);

/*
 * Gradient of a real loss with respect to the window, summed over the batch.
 * Given signals f_dev[B][L] and the loss gradient gc_dev[B][N][M] with
 * respect to the coefficients (convention dLoss/dRe + i dLoss/dIm), writes
 * gg_dev[L] (plan dtype) with gg(j) = sum_k sum_n f_k(j + n a) conj(y_{k,n}(j + n a)),
 * y_{k,n}(l) = sum_m gc_k(m, n) exp(2 pi i l (m + w(n)) / M).
 * Deterministic (no atomics).  Implemented for shear-algorithm plans (any p,
 * long columns d = d1 d2 included; DGTNS_EUNSUPPORTED otherwise).
 * Workspace: DGTNS_OP_WINDOW_GRAD.
 */
int dgtns_window_grad(dgtns_plan plan, const void* f_dev, const void* gc_dev, void* gg_dev,
                      int64_t B, void* ws, size_t ws_bytes, void* stream);

/*
 * Canonical dual window S^{-1} g of the Gabor frame of g_dev (complex128,
 * length L) on the plan's lattice (Section 2.1, eq. (frameop); computed by
 * shearing as in Alg. 2, with the time shear undone at the end), in FP64.
 * gd_dev: complex128[L].  bounds_dev: 2 doubles on the device receiving the
 * optimal frame bounds (A, B); A == 0 means the system is not a frame and
 * gd_dev is then undefined (asynchronous calls cannot report
 * DGTNS_ENOTFRAME; callers check A).  Implemented for p <= 64 of the sheared
 * lattice (p x p blocks of the frame operator in the Zak domain) and
 * shear-algorithm plans (DGTNS_EUNSUPPORTED otherwise); long columns
 * (d = d1 d2) take the window Zak and its inverse in two passes.
 * Does not change the plan's window.  Workspace: DGTNS_OP_DUAL.
 */
int dgtns_dual_window(dgtns_plan plan, const void* g_dev, void* gd_dev, double* bounds_dev,
                      void* ws, size_t ws_bytes, void* stream);

/*
 * Canonical tight window S^{-1/2} g (Section 4.2): the window whose Gabor
 * system on the plan's lattice is a tight frame with bound 1, so that
 * f = C*_{gt} C_{gt} f.  Same steps, arguments, bounds output, workspace
 * (DGTNS_OP_DUAL) and restrictions as dgtns_dual_window, with the inverse
 * square root of the Zak-domain frame operator in place of its inverse.
 * gt_dev: complex128[L].
 */
int dgtns_tight_window(dgtns_plan plan, const void* g_dev, void* gt_dev, double* bounds_dev,
                       void* ws, size_t ws_bytes, void* stream);

/*
 * Host-only check (no device work, the plan need not be bound): returns
 * DGTNS_OK if operation `op` (enum dgtns_op; DGTNS_OP_DUAL covers both
 * dgtns_dual_window and dgtns_tight_window) on a batch of B is implemented for
 * the plan, else the status the call itself would return before enqueueing
 * anything (DGTNS_EUNSUPPORTED for an algorithm or size the kernels do not
 * cover, with the reason in dgtns_last_error(); DGTNS_EINVAL for a bad op or
 * B outside [1, max_batch]).  It runs the same per-launch checks every device
 * call runs first.
 */
int dgtns_check_op(dgtns_plan plan, int op, int64_t B);

/*
 * Kernel timing for profiling and benchmarks.  While enabled (process-wide),
 * every kernel the library launches is bracketed by two HIP events recorded
 * on its launch stream.  dgtns_timing_collect() waits for all recorded events,
 * adds their durations to per-kernel totals and returns the number of
 * distinct kernels; dgtns_timing_entry(i, ...) reads entry i (name, number of
 * launches, total milliseconds); dgtns_timing_reset() clears the totals.
 */
int dgtns_timing_enable(int on);
int dgtns_timing_collect(void);
int dgtns_timing_entry(int i, char* name, size_t name_bytes, int64_t* launches, double* total_ms);
int dgtns_timing_reset(void);

/* Release host memory of the plan (device memory stays with the caller). */
int dgtns_plan_destroy(dgtns_plan plan);

/*
 * Host-only planner queries used by tests: the shear factorisation for a
 * lattice without creating a plan.  out[0..2] = s0, s1, b_r.
 */
int dgtns_shearfind(int64_t L, int64_t a, int64_t M, int64_t lambda1, int64_t lambda2, int64_t* out);

/*
 * Smallest multiplier of L_min = lambda2 lcm(a, M) for which a time shear
 * alone suffices, L = n L_min c / c1 (Prop. 9): returns c / c1 in *out.
 */
int dgtns_noshear_factor(int64_t a, int64_t M, int64_t lambda1, int64_t lambda2, int64_t* out);

#ifdef __cplusplus
}
#endif

#endif /* DGTNS_H */
