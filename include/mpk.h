/*
 * mpk.h -- C ABI of the MI355X level-blocked matrix power kernel.
 *
 * The operation (Lacey et al., "Cache Blocking of Distributed-Memory Parallel
 * Matrix Power Kernels", Sec. "RACE Applied to the Matrix Power Kernel"):
 * for a square sparse matrix A in CSR and a dense block x, compute every power
 * y_k = A^k x, k = 1..p, and store all p results.  The level-blocked variant
 * (LB-MPK, executed inside Alg. 2 as localLBMPK) returns exactly the same
 * products as p back-to-back SpMVs (Alg. 1 without halo exchange); it only
 * reorders them in time so that matrix rows are reused from cache across
 * powers.  A three-term-recurrence form covers Chebyshev polynomial filters,
 * Eq. (anderson_spmv).
 *
 * Conventions shared by every call:
 *   - Indices are 0-based; row pointers and column indices are int32.
 *   - Dense blocks are row-major with the right-hand side fastest:
 *       x[i*nrhs + r],   Y[(k-1)*n*nrhs + i*nrhs + r] = (y_k)_{i,r}.
 *     Y holds y_1..y_p (x itself is not copied into Y).
 *   - x and Y are DEVICE pointers (HIP device memory of the plan's device);
 *     they must not overlap.  The caller owns them.
 *   - Calls that take a stream are asynchronous on that stream (NULL = the
 *     null stream).  Argument errors are reported synchronously through the
 *     return code; a device-side failure (a dependency wait that exceeded its
 *     time limit) is reported by mpk_plan_sync.
 *   - No C++ exception crosses this interface.  On any status other than
 *     MPK_OK, mpk_last_error() returns a thread-local message.
 *   - A plan is safe to use from several host threads and streams at once;
 *     concurrent runs on one plan draw separate dependency workspaces.
 */
#ifndef MPK_H
#define MPK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MPK_OK = 0,
    MPK_EINVAL = 1,        /* bad argument (NULL pointer, p < 1, ...)            */
    MPK_EBADCSR = 2,       /* CSR not valid: rowptr not monotone, col out of range */
    MPK_ENOMEM = 3,        /* host or device allocation failed                   */
    MPK_EHIP = 4,          /* a HIP runtime call failed                          */
    MPK_EUNSUPPORTED = 5,  /* valid but unsupported (nrhs > 16, nnz >= 2^31, ...) */
    MPK_ETIMEOUT = 6,      /* device dependency wait exceeded its limit          */
    MPK_ENODEVICE = 7      /* run requested on a host-only plan                  */
} mpk_status_t;

/* Row order of the vectors passed to the run calls. */
enum {
    MPK_ORDER_ORIGINAL = 0, /* x and Y use the caller's row numbering (default)   */
    MPK_ORDER_PLAN = 1      /* x and Y use the plan's (BFS) numbering; see mpk_permute */
};

/* Symmetric reordering applied by the planner. */
enum {
    MPK_REORDER_BFS = 0,    /* BFS level order from the root (the paper's choice) */
    MPK_REORDER_NONE = 1,   /* keep the caller's order (levels derived from it)   */
    MPK_REORDER_SUBLEVELS = 2 /* BFS levels, each ordered by sub-level: the
                               distance from a second root (opts.sublevel_root),
                               so that every edge joins equal or adjacent
                               sub-levels; an XCD's part of each level is then
                               a run of sub-levels (a reading of the paper's
                               recursion that breaks bulky levels, s_m in Sec.
                               "Experimental Setup")                          */
};

/* Traversal order of the (chunk, power) tasks. */
enum {
    MPK_SCHED_STEPS = 0,    /* level groups walked along the diagonals
                               g + 2(k-1) = const; the tasks of one diagonal are
                               independent and run as one kernel launch, the
                               launch boundary orders consecutive diagonals    */
    MPK_SCHED_WAVE = 1,     /* default: one persistent kernel, skewed chunk wavefront with
                               per-chunk completion flags                      */
    MPK_SCHED_DIAG = 2,     /* one persistent kernel, the paper's Lp-diagram
                               diagonals g + k = const over level groups        */
    MPK_SCHED_POWERS = 3,   /* one persistent kernel, power by power            */
    MPK_SCHED_XCD = 4       /* one persistent kernel; each level is split into
                               one part per XCD and every XCD walks its parts in
                               a skewed wavefront from its own queue (exact
                               dependency lists), so most inputs were produced
                               on the same XCD                                 */
};

#define MPK_DEVICE_CURRENT (-1)
#define MPK_DEVICE_NONE (-2)   /* host-only plan: levels and schedules, no device data */
#define MPK_MAX_RHS 16

/* Host CSR handed to mpk_plan.  The plan copies it; the caller may free its
 * arrays when mpk_plan returns.  val may be NULL for a host-only plan. */
typedef struct {
    int64_t n;               /* rows = columns                                 */
    int64_t nnz;             /* rowptr[n]                                      */
    const int32_t *rowptr;   /* n+1 entries, rowptr[0] = 0, non-decreasing     */
    const int32_t *col;      /* nnz entries, 0 <= col < n (duplicates allowed) */
    const double *val;       /* nnz entries                                    */
} mpk_csr_t;

/* opts.root: a pseudo-peripheral row of row 0's component, found by the
 * George-Liu iteration (repeated BFS from a least-degree vertex of the
 * previous search's last level while the eccentricity grows).  The paper
 * roots the levels at row 0 as a rule; a peripheral root gives as many and
 * as thin levels as the heuristic finds.  Costs a few extra BFS sweeps. */
#define MPK_ROOT_PERIPHERAL (-1)

typedef struct {
    int value_bits;          /* 64 (default) or 32: values stored as float,
                                promoted to double before each product        */
    int reorder;             /* MPK_REORDER_BFS (default), MPK_REORDER_NONE or
                                MPK_REORDER_SUBLEVELS                           */
    int order;               /* MPK_ORDER_ORIGINAL (default) or MPK_ORDER_PLAN  */
    int root;                /* BFS root row (default 0), or
                                MPK_ROOT_PERIPHERAL                           */
    int device;              /* HIP device, MPK_DEVICE_CURRENT or MPK_DEVICE_NONE */
    int64_t l2_bytes;        /* per-XCD L2 budget of the XCD schedule's window
                                (0 = 4 MiB, the MI355X L2 per XCD)              */
    int64_t mall_bytes;      /* the plan's initial blocking budget C
                                (tune.cache_bytes; 0 = 64 MiB, the measured
                                fast-read plateau of the Infinity Cache)        */
    int min_group_rows;      /* level groups of the STEPS and DIAG schedules
                                hold at least this many rows (0 = no minimum):
                                enough rows per diagonal to fill the device     */
    int sublevel_root;       /* MPK_REORDER_SUBLEVELS: the second root, or
                                MPK_ROOT_AUTO (default): the vertex of the
                                widest level farthest from that level's
                                smallest vertex                                */
} mpk_plan_opts_t;

#define MPK_ROOT_AUTO (-1)

/* Run-time tuning of a plan (mpk_plan_tune).  None of these changes a result
 * bit: every kernel sums each row sequentially in stored order. */
typedef struct {
    int schedule;            /* MPK_SCHED_WAVE (default), _STEPS, _DIAG,
                                _POWERS, _XCD                                   */
    int64_t cache_bytes;     /* blocking budget C in bytes (default 64 MiB:
                                the measured fast-read plateau of the MI355X
                                Infinity Cache)                                 */
    double cache_safety;     /* fraction of C the window may use (default 1.0) */
    int chunk_nnz;           /* target nonzeros per chunk = per workgroup task
                                (default 32768; capped at nnz / (2 x running
                                workgroups), at least 1024, so that small
                                matrices still fill the device; WAVE and POWERS
                                cut chunks on multiples of 256 rows)            */
    int lag;                 /* WAVE, XCD: slack in chunks; 0 = from the budget
                                and the running workgroups                      */
    int workgroups;          /* persistent schedules: workgroups; 0 = as many as
                                fit, at most two per compute unit (four with the
                                sliced layout)                                  */
    int64_t spin_limit_us;   /* dependency-wait limit in microseconds, 0 = 2 s  */
    int seg_powers;          /* powers blocked together per launch (1..64);
                                p is run as ceil(p / seg_powers) segments that
                                each read the matrix once; 0 = 64 (at most)    */
    int skip_ahead;          /* WAVE, DIAG, POWERS: tasks a workgroup may park
                                while their inputs are not ready, taking newer
                                tickets meanwhile (0..8; 0 = wait in order)     */
    int acquire_always;      /* persistent schedules: 1 = every task invalidates
                                its XCD's caches before reading its inputs;
                                0 (default) = only where a cache line of an
                                output could have been read before it was
                                complete (see mpk_run)                          */
    int dynamic_tickets;     /* WAVE, POWERS: 1 = workgroups take tasks from a
                                shared counter; 0 (default) = workgroup b takes
                                tasks b, b + W, b + 2W, ... (W workgroups) where
                                the launch can hold the device alone: outside
                                graph capture, without skip-ahead, with every
                                workgroup resident; such launches (and XCD
                                launches) of this process wait for each other
                                on a device (another process's persistent
                                kernels are not ordered: a wait they block
                                ends at spin_limit_us with MPK_ETIMEOUT).
                                Other kernels running at the same time hold
                                compute units that the fixed order waits
                                for, so runs made beside other work (several
                                streams, serving) should set 1: with the
                                counter a task waits only on tasks that
                                running workgroups hold                         */
} mpk_tune_t;

typedef struct {
    int64_t n, nnz;
    int32_t n_levels;        /* BFS levels (or order-derived levels)           */
    int32_t max_level_rows;
    int32_t value_bits, reorder, order;
    int64_t matrix_bytes;    /* device CSR bytes: 4(n+1) + (4 + value bytes) nnz */
    double plan_ms;          /* host preprocessing time                         */
    int32_t device;
    int32_t sliced_layout;   /* 1: the kernels read the matrix in slices of 64
                                rows stored slot by slot (one coalesced access
                                per slot for the 64 rows); 0: CSR rows staged
                                through LDS (chosen when padding every slice
                                to its longest row would add more than 25%)  */
    int64_t sliced_entries;  /* stored slots of the sliced layout (0 if none)  */
    int32_t sublevel_root;   /* MPK_REORDER_SUBLEVELS: the second root (plan's
                                caller numbering), else -1                     */
    int32_t max_sublevels;   /* MPK_REORDER_SUBLEVELS: most sub-levels in one
                                level, else 0                                  */
    int64_t l2_bytes, mall_bytes;
    int32_t min_group_rows;
    int32_t sliced_col_bits; /* columns as the sliced layout's kernels read
                                them: 16 = offsets col - row taken modulo n
                                into [-n/2, n/2) (every entry within 32767 of
                                its row that way), 32 = columns, 0 = no
                                sliced layout                                  */
    uint64_t fingerprint;    /* hash of the shape, the ordering and blocking
                                options, the row pointers and a sample of the
                                columns: the matrix part of the autotuner's
                                cache key (values and their precision are not
                                in it); equal for plans of the same matrix
                                from host or device arrays                      */
} mpk_plan_info_t;

typedef struct {
    int32_t p;               /* the schedule's power count                      */
    int32_t n_chunks, n_groups, n_tasks;
    int32_t n_steps;         /* kernel launches per segment (STEPS), else 1     */
    int32_t lag;             /* effective wavefront slack                       */
    int32_t max_reach;       /* max over chunks of dhi - c (in chunks)          */
    double window_bytes;     /* estimated matrix bytes touched by one window    */
    double build_ms;
    int32_t n_queues;        /* XCD: task queues (one per XCD), else 1          */
    int32_t n_deps;          /* XCD: length of the exact dependency lists, else 0 */
} mpk_sched_info_t;

typedef struct mpk_plan_s *mpk_plan_t;

/* Fill *opts / *tune with the defaults documented above. */
void mpk_plan_opts_default(mpk_plan_opts_t *opts);
void mpk_tune_default(mpk_tune_t *tune);

/*
 * Build a plan (host preprocessing + device upload): validate the CSR,
 * symmetrise its pattern for the level construction, split the graph into BFS
 * levels from opts->root with ascending original index inside each level,
 * permute rows and columns symmetrically by level (in-row entry order is
 * preserved), and upload the matrix.  (Sec. "RACE Applied to the Matrix Power
 * Kernel": level equation, BFS reordering, and the endnote on non-symmetric
 * patterns.)  Disconnected graphs restart a new level at the lowest unvisited
 * row.  A device plan in BFS order uploads the CSR as given and builds the
 * levels and the permutation on the GPU (the same result; graphs with more
 * than 16384 levels or 64 components, and MPK_ROOT_PERIPHERAL, are handled
 * on the host); host-only plans always use the host planner.
 * Errors: MPK_EINVAL (NULL, bad opts), MPK_EBADCSR, MPK_EUNSUPPORTED
 * (nnz >= 2^31 or n >= 2^31), MPK_ENOMEM, MPK_EHIP.
 */
mpk_status_t mpk_plan(const mpk_csr_t *A, const mpk_plan_opts_t *opts, mpk_plan_t *out);

/*
 * The same plan from a CSR whose rowptr, col and val are DEVICE pointers (on
 * opts->device, or the current device when MPK_DEVICE_CURRENT).  Validation,
 * the levels and the permutation run on the device, so no matrix crosses the
 * host link.  The pseudo-peripheral root and graphs beyond the device level
 * search (more than 16384 levels or 64 components) are copied to the host
 * and planned as by mpk_plan.  The result, including the autotuner's
 * fingerprint, equals mpk_plan's for the same matrix and options.  The plan
 * copies the matrix: the caller may free its arrays when the call returns.
 * Errors: as mpk_plan; MPK_EINVAL for opts->device == MPK_DEVICE_NONE.
 */
mpk_status_t mpk_plan_device(const mpk_csr_t *A, const mpk_plan_opts_t *opts, mpk_plan_t *out);

/* Release the plan and all device memory it owns (waits for its runs). */
void mpk_plan_destroy(mpk_plan_t plan);

/* Set the tuning used by later runs of this plan (NULL = defaults). */
mpk_status_t mpk_plan_tune(mpk_plan_t plan, const mpk_tune_t *tune);

/*
 * The plan's shape: the level structure of Sec. "RACE Applied to the Matrix
 * Power Kernel" (the level equation's sets after the BFS reordering, or the
 * order-derived levels), the stored matrix and the planner inputs.
 * Errors: MPK_EINVAL (NULL).
 */
mpk_status_t mpk_plan_info(mpk_plan_t plan, mpk_plan_info_t *info);

/* Copy out the level pointer (n_levels+1 entries) and the permutation
 * perm[new] = old (n entries); either pointer may be NULL. */
mpk_status_t mpk_plan_levels(mpk_plan_t plan, int32_t *level_ptr, int32_t *perm);

/*
 * Build (or fetch from the plan's cache) the schedule for p powers with the
 * current tuning and describe it.  Arrays are host memory and may be NULL:
 * chunk_ptr[n_chunks+1] (row ranges in plan order), chunk_group[n_chunks],
 * dep_lo/dep_hi[n_chunks] (inclusive chunk range a chunk's rows read),
 * tasks[2*n_tasks] = (chunk, power) pairs in issue order, and for STEPS
 * step_ptr[n_steps+1] (task ranges of the launches).
 */
mpk_status_t mpk_plan_schedule(mpk_plan_t plan, int p, mpk_sched_info_t *info,
                               int32_t *chunk_ptr, int32_t *chunk_group, int32_t *dep_lo,
                               int32_t *dep_hi, int32_t *tasks, int32_t *step_ptr);

/*
 * The extra arrays of an MPK_SCHED_XCD schedule (MPK_EINVAL for the other
 * schedules).  Host memory, each may be NULL: dep_ptr[n_chunks+1] and
 * dep_idx[n_deps] list, for every chunk, the chunks its rows read (itself
 * included, ascending); chunk_xcd[n_chunks] the owning queue; remote_out
 * [n_chunks] = 1 when a chunk is read by a chunk of another queue; qptr
 * [n_queues+1] splits tasks[] into the per-queue lists, each in dependency
 * order.  Host-only plans assume the 8 XCDs of the MI355X.
 */
mpk_status_t mpk_plan_schedule_xcd(mpk_plan_t plan, int p, int32_t *dep_ptr, int32_t *dep_idx,
                                   int32_t *chunk_xcd, int32_t *remote_out, int32_t *qptr);

/*
 * Level-blocked matrix power kernel: Y = [A x, A^2 x, ..., A^p x].
 * The (chunk, power) tasks run in the schedule's order; a task starts once
 * the chunks its rows read are done at the previous power (the Lp-diagram
 * dependency of Sec. "RACE Applied to the Matrix Power Kernel": level i at
 * power k needs levels i-1..i+1 at power k-1).  STEPS orders tasks by kernel
 * launches; the persistent schedules by per-chunk completion flags.
 * x: n*nrhs doubles; Y: p*n*nrhs doubles (device).  1 <= nrhs <= 16.
 * Errors: MPK_EINVAL (p < 1, NULL), MPK_EUNSUPPORTED (nrhs), MPK_ENODEVICE.
 */
mpk_status_t mpk_run(mpk_plan_t plan, const double *x, int p, int nrhs, double *Y,
                     void *hip_stream);

/*
 * mpk_run for callers that cannot allocate (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the same
 * level-blocked run with the same results, whose dependency workspace is a
 * file-scope device array of the library (1 MiB per GPU, held until the
 * process ends) instead of a workspace from the plan's pool.  The call
 * allocates nothing, builds nothing and records no event: the schedule, slice
 * tables and workgroup count for (p, nrhs) must exist, so call
 * mpk_plan_prepare(plan, p, nrhs) (or run mpk_run once with them) first.
 * status: device or pinned host int32, or NULL; set to 0 when the run starts
 * on the stream and to 1 if a dependency wait hits tune.spin_limit_us (the
 * outputs are then invalid).  Not reported by mpk_plan_sync or
 * mpk_run_status.
 * Every call on one GPU shares that array, which keeps the last call's
 * contents (each run clears what it uses): calls that overlap on one GPU
 * race and give wrong results, so issue them on one stream or order them.
 * Errors: as mpk_run; MPK_EINVAL when (p, nrhs) was not prepared;
 * MPK_EUNSUPPORTED when the schedule has more than 262126 chunks (raise
 * tune.chunk_nnz).
 */
mpk_status_t mpk_run_noalloc(mpk_plan_t plan, const double *x, int p, int nrhs, double *Y,
                             int32_t *status, void *hip_stream);

/*
 * Three-term recurrence, Eq. (anderson_spmv) generalised:
 *   y_1     = alpha[0] A x   + beta[0] x
 *   y_{j+1} = alpha[j] A y_j + beta[j] y_j + gamma[j] y_{j-1},  j = 1..p-1
 * (y_0 = x; gamma[0] is ignored).  Chebyshev: alpha = (1,2,2,...), beta = 0,
 * gamma = (0,-1,-1,...).  alpha, beta, gamma are HOST arrays of p doubles,
 * captured at call time.  Same layouts and errors as mpk_run.
 */
mpk_status_t mpk_run_recur(mpk_plan_t plan, const double *x, int p, int nrhs,
                           const double *alpha, const double *beta, const double *gamma,
                           double *Y, void *hip_stream);

/*
 * Baseline: p back-to-back CSR SpMVs, one kernel launch per power (Alg. 1
 * without halo exchange), on the plan's matrix.  Every kernel of this
 * library forms each entry of y_k as the plain CSR sum: products rounded one
 * by one, added left to right in stored order from 0.0 (no fused
 * multiply-add), so baseline and level-blocked results are bit-identical.
 */
mpk_status_t mpk_run_baseline(mpk_plan_t plan, const double *x, int p, int nrhs, double *Y,
                              void *hip_stream);
mpk_status_t mpk_run_baseline_recur(mpk_plan_t plan, const double *x, int p, int nrhs,
                                    const double *alpha, const double *beta,
                                    const double *gamma, double *Y, void *hip_stream);

/*
 * Weighted sums of the powers: the polynomial that one step of the
 * Chebyshev time propagation evaluates (Sec. "Application: Chebyshev Time
 * Propagation": the new state is a weighted sum of v_0 .. v_M):
 *   acc_a = sum_{k=0..p} wa[k] y_k,   acc_b = sum_{k=0..p} wb[k] y_k,
 * y_0 = x, y_1..y_p from the recurrence of mpk_run_recur (alpha, beta and
 * gamma all NULL: plain powers y_k = A^k x).  The sequence itself is not
 * kept: y_k lives in the ring `work` at work + ((k-1) mod 2)*n*nrhs, so on
 * return work holds y_p and (p >= 2) y_{p-1}.
 * The sums are formed in the kernels' epilogues, in increasing k: a sum's
 * first term with a nonzero weight sets it to w[k]*y_k, each later one adds
 * w[k]*y_k (no fused multiply-add), a weight that is exactly zero omits its
 * term, and a sum whose weights are all zero is written as zeros.  The task
 * that computes y_m holds y_{m-2} and y_{m-1} as well, so up to three
 * consecutive terms are added in one read-modify-write of the sum (the
 * Chebyshev weights touch each sum every fourth power).  The results are therefore the
 * same bit for bit as mpk_run_baseline_poly, and as forming these sums
 * from the output of mpk_run_recur.
 * alpha, beta, gamma: HOST arrays of p doubles (or all NULL); wa, wb: HOST
 * arrays of p + 1 doubles (wb may be NULL: no acc_b), read at call time.
 * acc: device, n*nrhs doubles, or 2*n*nrhs with wb (acc_b at acc + n*nrhs);
 * work: device, 2*n*nrhs doubles.  x, work and acc must not overlap.
 * A ring slot is rewritten only after every task that reads its old value
 * has finished; the schedules' dependencies guarantee that when the
 * pattern is structurally symmetric (every stored (i, j) has a stored
 * (j, i)), which is checked once per plan.  Other patterns give
 * MPK_EUNSUPPORTED here; mpk_run_baseline_poly accepts them.
 * Errors: as mpk_run_recur; MPK_EINVAL (NULL wa / acc / work, overlap).
 */
mpk_status_t mpk_run_poly(mpk_plan_t plan, const double *x, int p, int nrhs, const double *alpha,
                          const double *beta, const double *gamma, const double *wa,
                          const double *wb, double *acc, double *work, void *hip_stream);

/* The same sums with one p x SpMV launch per power (any pattern). */
mpk_status_t mpk_run_baseline_poly(mpk_plan_t plan, const double *x, int p, int nrhs,
                                   const double *alpha, const double *beta, const double *gamma,
                                   const double *wa, const double *wb, double *acc, double *work,
                                   void *hip_stream);

/*
 * Build and upload, ahead of time, what runs with p powers and nrhs
 * right-hand sides fetch from the plan's caches on first use: the
 * schedule of every segment (Sec. "RACE Applied to the Matrix Power
 * Kernel": the (level group, power) tasks of the Lp diagram), its row
 * slices for nrhs, an idle dependency workspace, and the p x SpMV slices
 * for nrhs.  No kernel runs.  Later calls of mpk_run, mpk_run_recur,
 * mpk_run_poly and the baseline forms with the same p and nrhs then do no
 * host planning and allocate nothing on the plan's side, so that their
 * first call does not pay for it, and so that the caller may capture them
 * into its own HIP graph (stream capture) without a run beforehand; a
 * captured level-blocked run keeps its workspace until the plan is destroyed.
 * Slice tables depend only on whether nrhs
 * is 1, 2, 3 or at least 4, so preparing every nrhs costs four tables per
 * schedule.  Valid until mpk_plan_tune changes the tuning.
 * Errors: MPK_EINVAL (p < 1, NULL plan), MPK_EUNSUPPORTED (nrhs outside
 * [1, 16]), MPK_ENODEVICE (host-only plan), MPK_ENOMEM.
 */
mpk_status_t mpk_plan_prepare(mpk_plan_t plan, int p, int nrhs);

/*
 * Coefficients of one Chebyshev time step (Sec. "Application: Chebyshev
 * Time Propagation"): exp(-i dt H) psi is approximated by
 * J_0(dt) v_0 + 2 sum_{k=1..M} (-i)^k J_k(dt) v_k with v_0 = psi,
 * v_1 = H psi, v_{k+1} = 2 H v_k - v_{k-1}, for H with its spectrum in
 * [-1, 1] (scale and shift H first).  Writes alpha, beta, gamma (M doubles
 * each: that recurrence for mpk_run_poly) and wa, wb (M + 1 doubles: real
 * and imaginary parts of the weights; a weight is real for even k and
 * imaginary for odd k, the other part exactly 0).  J_k(dt) comes from
 * Miller's backward recurrence, normalised by J_0 + 2 sum_k J_2k = 1.
 * Host only; all arrays are HOST memory owned by the caller.
 * Errors: MPK_EINVAL (M outside [1, 100000], dt not finite or |dt| > 1e4,
 * NULL array).
 */
mpk_status_t mpk_cheb_time_coefficients(int M, double dt, double *alpha, double *beta,
                                        double *gamma, double *wa, double *wb);

/*
 * Complex states from the two sums of mpk_run_poly (same Section): with
 * column 2j of each vector the real and 2j+1 the imaginary part of state j,
 * complex weights wa + i wb and a real matrix,
 *   out[i][2j]   = acc_a[i][2j]   - acc_b[i][2j+1]
 *   out[i][2j+1] = acc_a[i][2j+1] + acc_b[i][2j].
 * acc: device, 2*n*nrhs doubles (acc_b at acc + n*nrhs); out: device,
 * n*nrhs doubles, not overlapping acc; both 16-byte aligned.  nrhs even,
 * 2..16.  Asynchronous on hip_stream.
 * Errors: MPK_EINVAL (odd nrhs, NULL, alignment, overlap), MPK_ENODEVICE.
 */
mpk_status_t mpk_combine_complex(mpk_plan_t plan, const double *acc, int nrhs, double *out,
                                 void *hip_stream);

/*
 * Convert nvec blocks of n*nrhs doubles between the caller's numbering and
 * the plan's, i.e. apply the symmetric BFS permutation of Sec. "RACE
 * Applied to the Matrix Power Kernel" (rows sorted by level) or its inverse
 * to vectors: to_plan != 0 gives out[new] = in[perm[new]], else
 * out[perm[new]] = in[new].  The paper permutes once and runs many times;
 * with MPK_ORDER_PLAN this call is that one permutation.  Device pointers,
 * must not overlap.  Asynchronous on hip_stream.
 * Errors: MPK_EINVAL (NULL, overlap, nvec < 0, bad nrhs), MPK_ENODEVICE.
 */
mpk_status_t mpk_permute(mpk_plan_t plan, int to_plan, const double *in, double *out, int nvec,
                         int nrhs, void *hip_stream);

/* Wait for every run issued on this plan (all streams it was given) and
 * report device-side failures: MPK_ETIMEOUT when a dependency wait of any
 * run since the previous call hit its limit (the results of that run are
 * invalid), and clear the report.  A failure affects only its own run: every
 * run starts with its abort flag cleared. */
mpk_status_t mpk_plan_sync(mpk_plan_t plan);

/*
 * Per-run failure status without a host synchronisation: enqueue on
 * hip_stream a copy into *status of the failure word of this plan's runs
 * issued on that stream since the previous mpk_run_status call for it
 * (0 = every one completed, 1 = a dependency wait hit its limit, so the
 * outputs of a run among them are invalid), and clear the word.  status is
 * device memory or pinned host memory (e.g. hipHostMalloc); it holds the
 * value once the stream has reached this point, so a caller that records an
 * event after this call can read it as soon as the event has completed, and
 * must not hand out that stream's outputs before.  The kernel abandons a
 * run whose wait hits tune.spin_limit_us (Alg. 2's dependencies cannot
 * deadlock; the limit guards against a stalled device).  p x SpMV and STEPS
 * runs never fail this way.  Plans keep 256 words; beyond 256 streams,
 * streams share words (a failure then shows on each of them).
 * Errors: MPK_EINVAL (NULL), MPK_ENODEVICE, MPK_EHIP.
 */
mpk_status_t mpk_run_status(mpk_plan_t plan, void *hip_stream, int32_t *status);

/*
 * Autotuner (the counterpart of the paper's parameter study over the cache
 * size C and the RACE safety factor, Sec. "Parameter Study"): times the
 * level-blocked run for p powers and nrhs right-hand sides under a fixed list
 * of candidate tunings (schedule x cache budget x chunk size, and for the
 * persistent schedules one or two workgroups per compute unit, p split into
 * two segments, skip-ahead parking), keeps the fastest and sets it on the
 * plan.  Each candidate runs once untimed, then
 * `reps` timed runs on `stream` (mean); the three fastest then run as many
 * times again and are compared on the mean of all their timed runs.  A plan whose tuning has
 * dynamic_tickets = 1 when the call starts keeps the shared counter in every
 * candidate.  Results are cached per (matrix fingerprint, value precision,
 * p, nrhs, recur, that dynamic_tickets): a later call with the same key
 * applies the cached tuning (the plan's spin_limit_us kept) without timing
 * unless force != 0.
 * recur: 0 = time mpk_run, 1 = mpk_run_recur, 2 = the weighted sums of
 * mpk_run_poly (p >= 4; their kernels differ from the plain run's).
 * x: n*nrhs doubles, Y: p*n*nrhs doubles (device scratch; overwritten).
 * best / best_ms may be NULL.  The call synchronizes `stream`.
 * Errors: as mpk_run; MPK_ETIMEOUT if a candidate's waits hit their limit.
 */
mpk_status_t mpk_plan_autotune(mpk_plan_t plan, const double *x, int p, int nrhs, double *Y,
                               int reps, int force, int recur, void *hip_stream,
                               mpk_tune_t *best, double *best_ms);

/*
 * Capture one level-blocked run (mpk_run, or mpk_run_recur when alpha is not
 * NULL) into a HIP graph for repeated launches with the same pointers, p and
 * nrhs.  The plan's current tuning is used; the graph owns a dependency
 * workspace reserved for it.  Launches of one graph must not overlap (launch
 * it on one stream, or synchronize between streams); the graph must be
 * destroyed before its plan.  The capture itself runs on a private stream.
 * A graph that holds a static-order or XCD-queue launch (mpk_tune_t
 * dynamic_tickets) is ordered by mpk_graph_launch after every such launch
 * issued before it on the device, like the eager runs.
 */
typedef struct mpk_graph_s *mpk_graph_t;
mpk_status_t mpk_graph_capture(mpk_plan_t plan, const double *x, int p, int nrhs,
                               const double *alpha, const double *beta, const double *gamma,
                               double *Y, mpk_graph_t *out);

/*
 * Capture one Chebyshev time step (Sec. "Application: Chebyshev Time
 * Propagation"): the weights of mpk_cheb_time_coefficients(M, dt), the
 * weighted sums of mpk_run_poly (baseline != 0: mpk_run_baseline_poly) and
 * mpk_combine_complex into out, as one graph for repeated launches.
 * psi, out: device, n*nrhs doubles (nrhs even, 2..16: real and imaginary
 * columns); acc, work: device scratch, 2*n*nrhs doubles each.  out must not
 * overlap psi, acc or work; acc and out are 16-byte aligned.  A propagation
 * loop captures two graphs (psi -> out and out -> psi) and alternates them.
 * The graph keeps these pointers and the plan's tuning at capture time.
 * Errors: as mpk_run_poly and mpk_graph_capture; MPK_EINVAL (odd nrhs, M,
 * dt, NULL, overlap, alignment).
 */
mpk_status_t mpk_graph_capture_time_step(mpk_plan_t plan, const double *psi, int nrhs, double dt,
                                         int M, int baseline, double *out, double *acc,
                                         double *work, mpk_graph_t *graph);
mpk_status_t mpk_graph_launch(mpk_graph_t graph, void *hip_stream);
void mpk_graph_destroy(mpk_graph_t graph);

/*
 * Load-only bandwidth probe (the MI355X counterpart of the paper's
 * load-bandwidth measurement, Fig. "All Bandwidths"): `workgroups` x 256
 * threads read the device buffer buf[n] (n even) `passes` times with 16-byte
 * loads and write one double per workgroup to sink[workgroups] (device).
 * The caller times the call (e.g. with events on the stream).
 */
mpk_status_t mpk_probe_load(const double *buf, int64_t n, int passes, int workgroups,
                            double *sink, void *hip_stream);

/*
 * XCD-local form of the same probe: buf[n] is cut into `regions` equal parts
 * (n a multiple of 2 x regions) and each workgroup reads, `passes` times, the
 * part of the XCD it runs on (hardware XCC_ID mod regions), so that the
 * working set of each XCD's L2 is n/regions doubles.  sink[workgroups] as
 * above; xcc[workgroups] (device int32) receives the XCC_ID of each
 * workgroup, to check the placement the probe assumes (workgroup b on XCD
 * b mod regions).  regions in [1, 16].
 * Errors: MPK_EINVAL (NULL, n or regions out of range), MPK_EHIP.
 */
mpk_status_t mpk_probe_load_xcd(const double *buf, int64_t n, int regions, int passes,
                                int workgroups, double *sink, int32_t *xcc, void *hip_stream);

/* Device allocator used for plan data (NULL, NULL restores hipMalloc/hipFree). */
mpk_status_t mpk_set_allocator(void *(*alloc_fn)(size_t bytes, void *ctx),
                               void (*free_fn)(void *ptr, void *ctx), void *ctx);

/* Message for the last non-OK status on this thread ("" if none). */
const char *mpk_last_error(void);

/* Library version string. */
const char *mpk_version(void);

#ifdef __cplusplus
}
#endif

#endif /* MPK_H */
