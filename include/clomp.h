/*
 * clomp.h -- C ABI of the MI355X (gfx950) CLOMP hot-path library.
 *
 * CLOMP (coefficients-learning OMP, arXiv 2501.11592) reconstructs a sparse
 * coefficient vector x from measurements y = A x + noise (Methods, Eq. (1));
 * the ABI writes the paper's s as x.  Reconstruction seeks the fewest non-zeros
 * with ||A x - y||_2 small (Eq. (2)); a batch of signals may share one A
 * (Eq. (3)).  Like OMP, CLOMP takes y and A and returns x (Methods, end of
 * "Coefficients learning on OMP (CLOMP)").
 *
 * Conventions for every entry point
 *  - Pointers are DEVICE pointers unless marked (host).  Arrays are owned by
 *    the caller; the library never frees them and keeps no reference after
 *    the call returns, except that device work queued on `hip_stream` reads
 *    and writes them until that work completes.
 *  - A is stored column-major: column (atom) j occupies A[j*lda .. j*lda+m),
 *    entries [m, lda) of each column are ignored.  A must hold n*lda elements,
 *    lda must be a multiple of 4 (F32) or 8 (BF16) and A must be 16-byte
 *    aligned.  BF16 values are raw bfloat16 bit patterns (uint16).
 *  - Calls are asynchronous and stream-ordered on `hip_stream` (NULL: the
 *    default stream); outputs are valid once that stream has been
 *    synchronised.  A handle must not be used by two host threads at once.
 *  - Every entry point returns a clomp_status_t synchronously for argument,
 *    allocation and launch errors; no exception crosses the ABI.  A
 *    human-readable message for the last failure is kept per handle
 *    (clomp_last_error).  Numerical events are reported per instance through
 *    the CLOMP_ST_* bits, never through the return code.
 */
#ifndef CLOMP_H_
#define CLOMP_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct clomp_ctx* clomp_handle_t;

typedef enum {
  CLOMP_OK = 0,
  CLOMP_INVALID_ARGUMENT = 1,  /* null pointer, bad size, layout or alignment */
  CLOMP_OUT_OF_MEMORY = 2,     /* workspace allocation failed */
  CLOMP_DEVICE_ERROR = 3,      /* a HIP call failed (message in last_error) */
  CLOMP_NOT_SUPPORTED = 4      /* valid request the library does not serve */
} clomp_status_t;

typedef enum { CLOMP_F32 = 0, CLOMP_BF16 = 1, CLOMP_F64 = 2 } clomp_dtype_t;

typedef enum {
  CLOMP_METHOD_CLOMP = 0,  /* Adam steps on the masked coefficients */
  CLOMP_METHOD_OMP = 1,    /* plain OMP: least squares on the support */
  CLOMP_METHOD_IHT = 2,    /* normalised iterative hard thresholding to K =
                              k_eff atoms (the experiments' comparison method) */
  CLOMP_METHOD_PAPER = 3   /* CLOMP as the experiments run it: every iteration
                              selects all unselected atoms with |c_j| >=
                              select_threshold * max|c| and takes one Adam
                              step; inner_steps iterations */
} clomp_method_t;

/* Per-instance status bits (written to clomp_instance_t.status). */
#define CLOMP_ST_NAN 1u              /* a non-finite correlation was selected */
#define CLOMP_ST_K_CAPPED 2u         /* k > min(m, n): k_eff = min(k, m, n)   */
#define CLOMP_ST_ZERO_Y 4u           /* y == 0: empty support, x = 0          */
#define CLOMP_ST_REFINE_INACCURATE 8u/* refinement stopped above tolerance    */
#define CLOMP_ST_WATCHDOG 32u        /* a bounded device wait timed out       */

/* Solver flags (clomp_params_t.flags). */
#define CLOMP_FLAG_GRAPH 1u          /* capture the launch sequence of a batch
                                        shape into a HIP graph and replay it on
                                        later calls with the same shape (on a
                                        created stream; calls on the default
                                        stream launch eagerly)                 */
#define CLOMP_FLAG_NO_FUSED_SMALL 2u /* never use the fused small-signal
                                        loop (one workgroup runs a signal's
                                        whole greedy loop with its dictionary
                                        in LDS when k_eff <= 64 and it fits);
                                        for testing the iterated kernels      */
#define CLOMP_FLAG_AUTOTUNE 4u       /* time the scan-kernel candidates on the
                                        first call for each size class         */
#define CLOMP_FLAG_PROFILE 8u        /* record HIP events around every phase
                                        launch (ignored while capturing graphs);
                                        read with clomp_profile_read           */
#define CLOMP_FLAG_RESIDUAL_FLOW 16u /* always use the residual schedule      */
#define CLOMP_FLAG_CORR_FLOW 32u     /* use the correlation-update schedule
                                        (the default whenever H of the
                                        iterated signals fits in 16 GB and the
                                        staged vector in LDS; the flag only
                                        documents the choice)                 */
#define CLOMP_FLAG_NO_SHARED_GRAM 64u/* when every iterated signal of a batch
                                        has the same A (pointer, layout and
                                        master), the library by default forms
                                        the full Gram matrix A^T A and every
                                        c0 = A^T y once (n^2 floats, up to
                                        4 GB) and iterates without passes over
                                        A; this flag keeps the per-signal
                                        passes                                 */

#define CLOMP_FLAG_NO_REFINE 128u    /* CLOMP and OMP: x receives the
                                        coefficients the greedy loop reached
                                        (CLOMP: the Adam iterate on the bulk
                                        matrix; OMP: its least squares on the
                                        bulk matrix) instead of the least-
                                        squares refinement on A_master;
                                        resid_norm is that x's residual on
                                        A_master.  Exposes the learned
                                        coefficients before refinement       */

#define CLOMP_FLAG_IMAGE 256u       /* CLOMP on the columns of one image: the
                                        call's instances, in call order, are
                                        the columns 0 .. count-1 of an n x
                                        count image (x_c = D s_c, D the
                                        orthonormal DCT-II synthesis basis),
                                        all measured with the same A (same
                                        pointer, n, m, lda, master) and with
                                        the same k.  prior_tv then weighs the
                                        2-D total variation of Eq. (6) (the
                                        within-column term of the 1-D prior
                                        plus the term between neighbouring
                                        columns) and prior_lv the local
                                        variation of Eq. (7) (sample standard
                                        deviation over every 3 x 3 window of
                                        the image, step 1).  Every iteration
                                        each column selects its atom, then the
                                        inner_steps Adam steps are taken on
                                        all columns together (the priors
                                        couple them).  x receives the learned
                                        coefficients (no least-squares
                                        refinement: the local variation is not
                                        quadratic) and resid_norm their FP64
                                        residual on A_master.  Requires the
                                        CLOMP method, n <= 4096, k_eff <= 1024
                                        and the shared-dictionary schedule
                                        (not CLOMP_FLAG_NO_SHARED_GRAM or
                                        CLOMP_FLAG_RESIDUAL_FLOW); otherwise
                                        NOT_SUPPORTED                          */

/*
 * Solver parameters.  The paper states the optimiser only as automatic
 * differentiation and back-propagation on learnable s (Methods, "Coefficients
 * learning on OMP"); everything below is this library's fixed reading, the
 * same values the reference oracle uses:
 *   method       CLOMP (default), plain OMP, IHT, or paper-mode CLOMP
 *   inner_steps  CLOMP: T, Adam steps per selected atom (default 32);
 *                IHT and paper mode: the number of iterations R (the
 *                experiments use 200)
 *   lr_rel       learning rate of iteration t: lr_t = lr_rel * |c_j|, the
 *                correlation of the atom selected at t (paper mode: lr_rel *
 *                max_j |c_j| of the iteration) (default 0.05)
 *   beta1/beta2  Adam moment decays (0.9 / 0.999); eps = eps_rel * sigma with
 *                sigma = max_j |a_j^T y| (eps_rel default 1e-8)
 *   resid_tol    must be 0 (early stopping on ||r|| is not served)
 *   refine_iters maximum CGLS iterations of the final refinement for supports
 *                too large for the in-LDS QR (0: library default)
 *   refine_tol   relative CGLS stopping tolerance on ||A_S^T r|| (0: 1e-6)
 *   select_threshold
 *                paper mode: the normalised cut-off threshold T_h in (0, 1]
 *                (default 0.7, the experiments' value; Results, synthetic
 *                data); a batch that would take the support beyond k_eff is
 *                refused whole and sets CLOMP_ST_K_CAPPED.  The support is
 *                returned in increasing index order.  A non-finite
 *                correlation (CLOMP_ST_NAN) or max|c| = 0 ends the loop; the
 *                support reached so far is refined.
 *   prior_tv     CLOMP only: weight w >= 0 of the total-variation prior of
 *                Eq. (4)-(5) on the signal x = D (mask*s), D the orthonormal
 *                DCT-II synthesis basis (atom j of A = M D carries frequency
 *                j).  The loss becomes 1/2 ||y - A(mask*s)||^2 + w TV(x) with
 *                TV(x) = (1/n) sum_j (x_j - x_{j+1})^2, which equals (1/n)
 *                sum_j 4 sin^2(pi j / (2n)) s_j^2; the Adam steps and the
 *                final refinement (least squares with that penalty) use it,
 *                the selection does not.  Served where the refinement runs
 *                as the in-LDS QR ((m + k_eff) * k_eff within about 24K
 *                floats), else clomp_solve_batch returns NOT_SUPPORTED.
 *                0 (default): no prior.  With CLOMP_FLAG_IMAGE: the weight of
 *                the 2-D total variation of Eq. (6).
 *   prior_lv     CLOMP_FLAG_IMAGE only: weight >= 0 of the local variation of
 *                Eq. (7) on the image (0 default: none).
 */
typedef struct {
  int32_t method;
  int32_t inner_steps;
  float lr_rel;
  float beta1;
  float beta2;
  float eps_rel;
  float resid_tol;
  int32_t refine_iters;
  float refine_tol;
  uint32_t flags;
  float select_threshold;
  float prior_tv;
  float prior_lv;
} clomp_params_t;

/*
 * One signal of a batch (all pointers device pointers).
 *   n, m, k      atoms, measurements, requested sparsity; k_eff = min(k, m, n)
 *   A, lda       bulk matrix (dtype given to clomp_solve_batch), column-major
 *   A_master     FP32 master copy used for the final refinement and the FP64
 *                residual check; NULL means A (the bulk dtype must be F32)
 *   lda_master   leading dimension of A_master (0: lda)
 *   y            [m] FP32 measurements
 *   x            [n] FP32 out: coefficients, zero off the support
 *   support      [k] int32 out: selected atoms in selection order, -1 beyond
 *                the number selected
 *   n_selected   [1] int32 out
 *   resid_norm   [1] float64 out: ||y - A_master[:, S] x_S||_2 accumulated in
 *                FP64 (the residual of Eq. (2))
 *   status       [1] uint32 out: CLOMP_ST_* bits
 */
typedef struct {
  int32_t n, m, k;
  int32_t reserved;
  int64_t lda;
  int64_t lda_master;
  const void* A;
  const float* A_master;
  const float* y;
  float* x;
  int32_t* support;
  int32_t* n_selected;
  double* resid_norm;
  uint32_t* status;
} clomp_instance_t;

/* Fill *p (host) with the defaults listed above. */
void clomp_default_params(clomp_params_t* p);

/*
 * Create a handle bound to HIP device `device` with parameters *params (host;
 * NULL: defaults).  The handle owns its device workspace (grown on demand,
 * freed by clomp_destroy) and any captured HIP graphs.
 * Errors: INVALID_ARGUMENT (out == NULL, bad params), DEVICE_ERROR (no such
 * device / HIP failure).
 */
clomp_status_t clomp_create(clomp_handle_t* out, int device,
                            const clomp_params_t* params);

/* Replace the handle's parameters (host pointer, validated as in create). */
clomp_status_t clomp_set_params(clomp_handle_t h, const clomp_params_t* params);

/*
 * Solve `count` independent signals (the batched model of Eq. (3)/(4) with
 * per-signal A, or one shared A when every instance names the same A, n, m and
 * lda).  For each instance, k_eff = min(k, m, n) iterations of
 *   c = A^T r                               (residual injection)
 *   j = argmax over unselected atoms of |c_j|, lowest index on ties
 *   mask[j] = 1                             (mask update by OR)
 *   CLOMP: inner_steps Adam steps on the masked coefficients fitting
 *          1/2 ||A(mask*x) - y||^2;  OMP: least squares on the support
 *   r = y - A(mask*x)
 * run on the bulk A, followed by a least-squares refinement of x on the
 * selected support from A_master and the FP64 residual norm.
 *   inst    (host) array of `count` descriptors, read during the call only
 *   a_dtype CLOMP_F32 or CLOMP_BF16 (the bulk dtype of every instance)
 * Errors: INVALID_ARGUMENT (null pointers, n/m/k <= 0, lda < m, misaligned A,
 * BF16 without A_master, count < 0), NOT_SUPPORTED (F64 bulk, resid_tol != 0),
 * OUT_OF_MEMORY, DEVICE_ERROR.  count == 0 is a no-op returning CLOMP_OK.
 */
clomp_status_t clomp_solve_batch(clomp_handle_t h, const clomp_instance_t* inst,
                                 int32_t count, int32_t a_dtype,
                                 void* hip_stream);

/*
 * Host-only validation of a batch (no HIP call): returns what
 * clomp_solve_batch would return for the arguments alone.  `h` may be NULL;
 * messages then go nowhere.
 */
clomp_status_t clomp_check_batch(clomp_handle_t h, const clomp_instance_t* inst,
                                 int32_t count, int32_t a_dtype);

/*
 * Loss and gradient of the coefficient fit (the residual loss of the
 * coefficients-learning framework with the masked fully connected layer
 * y' = A(mask*x); Methods, "General idea of coefficients learning" and
 * "Coefficients learning on OMP"):
 *   u      = A(mask*x) - y                         ([m], optional output)
 *   loss   = 1/2 ||u||^2                           (scalar output)
 *   grad_x = mask * A^T u * g                      ([n] output)
 * where g = *grad_out (device scalar) or 1 when grad_out is NULL.
 *   dtype  CLOMP_F32 or CLOMP_F64: the type of A, x, y, grad_out, grad_x,
 *          resid_out and loss (F64 exists for gradient checking)
 *   mask   [n] uint8, non-zero = on the support
 * Deterministic: the same inputs give bit-identical outputs.
 * Errors: INVALID_ARGUMENT (null required pointer, n/m <= 0, lda < m,
 * misaligned A), NOT_SUPPORTED (BF16), DEVICE_ERROR.
 */
clomp_status_t clomp_grad(clomp_handle_t h, int32_t n, int32_t m, int64_t lda,
                          int32_t dtype, const void* A, const void* x,
                          const uint8_t* mask, const void* y,
                          const void* grad_out, void* grad_x, void* resid_out,
                          void* loss, void* hip_stream);

/*
 * Allocation-free variant of clomp_grad, for callers that cannot allocate
 * device memory during the call: code under HIP graph capture, tight serving
 * loops, hosts that forbid allocation after start-up.  Same arguments, same
 * kernels and the same results, bit for bit, as clomp_grad; its scratch (the
 * forward partial sums and, when resid_out is NULL, the residual) is a
 * device-resident array of 16 MiB per device, resolved once by clomp_create
 * on the handle's device and held until the process ends.  The call allocates
 * nothing and records no event.
 *   Limit: es * (ceil(n / 256) * m + m + ceil(m / 256)) <= 16 MiB, es = 4
 *   (F32) or 8 (F64); e.g. n = 65536 with m <= 16320 (F32).
 *   Races: every call on one device shares that device's scratch; calls whose
 *   work can overlap on one device (two streams, two host threads, two
 *   handles) must be ordered by the caller.  Nothing in the scratch needs to
 *   start at zero, and the previous call's contents are overwritten.
 * Errors: as clomp_grad, plus INVALID_ARGUMENT when the call needs more
 * scratch than the limit (nothing is launched), DEVICE_ERROR when the scratch
 * address of the handle's device is unknown.
 */
clomp_status_t clomp_grad_noalloc(clomp_handle_t h, int32_t n, int32_t m, int64_t lda,
                                  int32_t dtype, const void* A, const void* x,
                                  const uint8_t* mask, const void* y,
                                  const void* grad_out, void* grad_x, void* resid_out,
                                  void* loss, void* hip_stream);

/*
 * Schedules.  Signals with k_eff <= 64 whose dictionary fits in LDS run the
 * fused small-signal loop (one launch for the whole greedy loop of all of
 * them).  The others are iterated, one launch sequence per iteration: the
 * correlation-update schedule (default whenever it fits) uses
 * c = A^T y - H s with H[:, l] = A^T a_{S_l}: each iteration's pass over A
 * computes the new column of H and runs in the same launch as the
 * coefficient update, and a scan of H gives the next argmax; the residual
 * schedule runs, per iteration, a scan c = A^T r with the argmax, the Gram
 * column, the coefficient update and r = y - A_S s.  All compute the same
 * correlations.
 *
 * Phase timings gathered under CLOMP_FLAG_PROFILE, accumulated over every
 * solve since the last clomp_profile_reset.  Phases: 0 scan (residual
 * schedule: c = A^T r and argmax; correlation schedule: c = A^T y or
 * c0 - H s and argmax), 1 gram (selection record and new Gram column),
 * 2 coef (Adam or the OMP update; in the correlation schedule the launches
 * that carry only coefficient workgroups), 3 resid (r = y - A_S s), 4 refine
 * (QR or CGLS), 5 norm (FP64 residual norm and output scatter), 6 init, 7 pass
 * (correlation schedule: the launches of the pass over A, with the coefficient
 * update when it shares the launch), 8 fused (the whole greedy loop of the signals served by the fused
 * small-signal kernel).
 *   ms[p]        summed device time between HIP events recorded on the launch
 *                stream immediately before and after each launch of phase p
 *   launches[p]  number of launches of phase p
 *   scan_bytes   algorithmic bytes of phase-0 launches: per active instance,
 *                m*n*elem + 4m + n/8 for a scan of A, or 4*n*(t+1) + n/8 for
 *                a scan of H at iteration t
 *   pass_bytes   algorithmic bytes of phase-7 launches: m*n*elem + 4n per
 *                active instance (the bulk columns and the new column of H)
 *   fused_bytes  algorithmic bytes of phase-8 launches: m*n*elem + 4m per
 *                signal (its dictionary and y, each read once)
 * Synchronises on the recorded events.  Errors: INVALID_ARGUMENT, DEVICE_ERROR.
 */
typedef struct {
  double ms[12];        /* phases 0..8; 9..11 reserved (zero) */
  int64_t launches[12];
  double scan_bytes;
  double pass_bytes;
  double fused_bytes;
} clomp_profile_t;

clomp_status_t clomp_profile_read(clomp_handle_t h, clomp_profile_t* out /*host*/);
clomp_status_t clomp_profile_reset(clomp_handle_t h);

/*
 * Launch-shape tuning of a handle (host struct).  In every field 0 keeps the
 * current value and -1 restores the default; other values must lie in
 * [1, 65536] (spin_limit: >= 1).  The tile fields are the number of
 * bulk-matrix kilobytes one workgroup streams in the corresponding kernel.
 * Autotuning (CLOMP_FLAG_AUTOTUNE) writes the same
 * table: on the first solve of a batch whose size class it has not seen, it
 * times candidate values on the batch's own first pass over A and keeps the
 * fastest per (bulk dtype, schedule, size class).
 *   scan_tile_kb   residual-schedule scan workgroups (default 128)
 *   pass_tile_kb   correlation-schedule pass workgroups (default 256)
 *   team_min_rows  correlation schedule: iterations whose support exceeds
 *                  this many atoms update the coefficients with a team of
 *                  ceil((t+1)/16) workgroups per signal (at most 128, and
 *                  only while the teams of all active signals fit on the
 *                  device at once and the occupancy query for the launch's
 *                  shape and LDS admits a member on every CU); smaller
 *                  supports use one workgroup (default 256; a value >= k
 *                  disables teams).  Members wait for one another's
 *                  published coefficients; each wait is bounded (spin_limit)
 *   rscan_min_t    shared-dictionary batches: from the iteration whose
 *                  support has this many atoms on, the correlation scan is
 *                  one contraction C = A^T R over the batch's residuals
 *                  (argmax fused); before it, c = c0 - Gf[:, S] s per signal
 *                  (default 1: always contract; a value >= k never)
 *   shared_min_tiles  IHT and paper mode on a shared dictionary: the batch's
 *                  gradient is one contraction A^T R only when that
 *                  contraction has at least this many 128 x 128 output tiles
 *                  (atoms x signals); smaller batches scan per signal, which
 *                  keeps more of the device busy (default: half the compute
 *                  units; 1 always contracts)
 *   spin_limit     polls of a coefficient-team wait before it gives up: the
 *                  signal then carries CLOMP_ST_WATCHDOG, its coefficients
 *                  are unspecified, and every kernel still finishes (default
 *                  2^20; a small value forces that path, for testing it)
 * clomp_get_tuning returns the values in use for the last solve.
 * Errors: INVALID_ARGUMENT (NULL, or a value outside the ranges above).
 */
typedef struct {
  int32_t scan_tile_kb;
  int32_t pass_tile_kb;
  int32_t team_min_rows;
  int32_t rscan_min_t;
  int32_t shared_min_tiles;
  int32_t spin_limit;
  int32_t reserved[2];
} clomp_tuning_t;

clomp_status_t clomp_set_tuning(clomp_handle_t h, const clomp_tuning_t* t /*host*/);
clomp_status_t clomp_get_tuning(clomp_handle_t h, clomp_tuning_t* t /*host*/);

/*
 * The process-wide autotune table (host only; no handle, no device call).
 * Under CLOMP_FLAG_AUTOTUNE a solve looks up its size class first in its
 * handle's own table, then here, and times the candidates only when neither
 * has it; every timed choice is written to both.  The table outlives handles,
 * and these three calls move it across processes as text:
 *
 *   clomp-tuning 1
 *   <key> <tile KB>
 *   ...
 *
 * One entry per line ('\n', optionally '\r\n'); blank lines and lines that
 * start with '#' are ignored.  A key names a size class as
 * arch/dtype/method/schedule/m<o>/n<o>/c<o> (for example
 * gfx950/bf16/clomp/corr/m12/n13/c12: device architecture, bulk dtype,
 * method, correlation-update or residual schedule, and the octaves
 * floor(log2 v) of the largest m, the largest n and the number of iterated
 * signals); at most 127 characters from [A-Za-z0-9_./:+-].  The value is the
 * tile size in KB that the schedule's tile field takes (pass_tile_kb for
 * "corr", scan_tile_kb for "resid"), 1 .. 65536.
 *
 * clomp_tuning_table_import merges `text` (NUL-terminated) into the table: an
 * imported entry replaces one with the same key.  All or nothing: a missing
 * header, a malformed line, a value out of range or a key given twice leaves
 * the table unchanged and returns INVALID_ARGUMENT.  *n_entries (may be NULL)
 * receives the number of entries imported.
 * clomp_tuning_table_export writes the whole table, NUL-terminated, keys in
 * byte order.  *len receives its length without the NUL; with buf NULL only
 * the length is returned; a `cap` below len + 1 returns INVALID_ARGUMENT and
 * writes nothing to buf.
 * clomp_tuning_table_clear empties the table (handles keep their own).
 * Failures of these calls are reported by clomp_last_error(NULL) on the
 * calling thread.  The table is guarded by a lock: any thread may call them.
 * (A tuning aid, not an operation of the method: a saved table lets later
 * runs of the same size classes skip the candidate timing.)
 */
clomp_status_t clomp_tuning_table_import(const char* text /*host*/, int32_t* n_entries /*host*/);
clomp_status_t clomp_tuning_table_export(char* buf /*host*/, size_t cap, size_t* len /*host*/);
clomp_status_t clomp_tuning_table_clear(void);

/* Free the handle, its workspace and graphs (synchronises its device). */
clomp_status_t clomp_destroy(clomp_handle_t h);

/* Static string naming a status code. */
const char* clomp_status_string(clomp_status_t s);

/* Message of the last failure on `h` ("" if none).  With h NULL: the message
 * of the calling thread's last failed handle-free call (the tuning table),
 * else a static text. */
const char* clomp_last_error(clomp_handle_t h);

#ifdef __cplusplus
}
#endif

#endif /* CLOMP_H_ */
