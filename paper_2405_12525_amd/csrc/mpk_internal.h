// Internal interfaces between the host planner, the C ABI and the HIP kernels.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "mpk.h"

namespace mpk {

// ------------------------------------------------------------------ planner

// Result of the level construction on G(A): levels in plan order plus the
// symmetric permutation perm[new] = old, iperm[old] = new.
struct Levels {
    std::vector<int32_t> level_ptr;  // n_levels + 1, plan-order row ranges
    std::vector<int32_t> perm, iperm;
};

// Validates a host CSR; returns MPK_OK or MPK_EBADCSR / MPK_EUNSUPPORTED / MPK_EINVAL.
mpk_status_t validate_csr(const mpk_csr_t *A, bool need_values, std::string &err);

// BFS levels from `root` on the symmetrised pattern, self-loops ignored,
// ascending original index inside a level, restart at the lowest unvisited
// row when the frontier empties.
Levels bfs_levels(int64_t n, const int32_t *rowptr, const int32_t *col, int32_t root);

// Levels broken into sub-levels: rows of each level of `lv` (BFS levels,
// ascending original index inside a level) reordered by (d2, original index)
// with d2 the BFS distance from root2 (the same level construction from
// another root); root2 < 0: the vertex of the widest level (the first among
// equals) farthest from that level's smallest vertex, ties to the smaller
// index.  Both distances change by at most one along any edge, so every
// edge joins equal or adjacent sub-levels.  Returns root2 through *root_out
// and the most sub-levels of one level through *max_sub.
Levels sublevel_order(int64_t n, const int32_t *rowptr, const int32_t *col, const Levels &lv,
                      int32_t root2, int32_t *root_out, int32_t *max_sub);

// Identity permutation with levels derived from the given order: level j+1
// ends just past the farthest neighbour of level j, so every row's
// neighbours lie in its own or an adjacent level.
Levels order_levels(int64_t n, const int32_t *rowptr, const int32_t *col);

// The matrix in plan row order.  `col` holds plan-numbered columns when
// plan_cols is true, else the caller's numbering; row_lo / row_hi are each
// row's smallest / largest column in PLAN numbering (the dependency extent).
struct PermutedCSR {
    std::vector<int32_t> rowptr, col, row_lo, row_hi;
    std::vector<double> val;   // col and val are empty when identity: the
    bool identity = false;     // caller's arrays are in plan order already
};
void permute_csr(int64_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                 const Levels &lv, bool plan_cols, PermutedCSR &out);

// Levels and the permuted CSR computed on the device (gpu_plan.hip): the
// same result as bfs_levels + permute_csr.  rowptr / col / val are the
// caller's CSR on the device in its own order; out_rowptr (n + 1), out_col
// (nnz) and out_val (nnz doubles or floats, by value_bits) receive the
// permuted matrix; `res` the host copies the scheduler needs.  Returns a
// hipError_t (0 on success), or kTooManyLevels when the graph has more
// levels or components than a level-by-level device search handles well
// (the caller then uses the host planner).
constexpr int kTooManyLevels = -1;
struct GpuLevels {
    std::vector<int32_t> level_ptr, perm, iperm, rowptr, row_lo, row_hi;
};
int gpu_levels_permute(int64_t n, int64_t nnz, const int32_t *rowptr, const int32_t *col,
                       const double *val, int32_t root, bool plan_cols, int value_bits,
                       int32_t *out_rowptr, int32_t *out_col, void *out_val, GpuLevels &res);

// Helpers for plans built from a device CSR (gpu_plan.hip; hipError_t
// results).  gpu_validate: flags for a decreasing row pointer and for a
// column out of range, and rowptr[0], rowptr[n].  gpu_order_far: far[i] of
// the order-derived levels (the largest row joined to row i).
// gpu_copy_in_place_order: the plan's copy of a CSR kept in the caller's
// order (values converted for FP32) plus the host row pointer and row
// extents.  gpu_sample_cols: col[k * step] for k < count.
int gpu_validate(int64_t n, int64_t nnz, const int32_t *rowptr, const int32_t *col,
                 int *bad_rows, int *bad_cols, int32_t *first_last);
int gpu_order_far(int64_t n, const int32_t *rowptr, const int32_t *col, std::vector<int32_t> &far);
int gpu_copy_in_place_order(int64_t n, int64_t nnz, const int32_t *rowptr, const int32_t *col,
                            const double *val, int value_bits, int32_t *out_rowptr,
                            int32_t *out_col, void *out_val, std::vector<int32_t> &h_rowptr,
                            std::vector<int32_t> &row_lo, std::vector<int32_t> &row_hi);
int gpu_sample_cols(const int32_t *col, int64_t step, int64_t count, std::vector<int32_t> &out);

// Sliced layout of the plan's matrix (the kernels' row routine for plain
// rows): rows in slices of kSellRows; slice s holds width[s] slots (its
// longest row) stored slot-major, entry j of row r at soff[r / 64] + j * 64 +
// r % 64, so that the 64 rows of a slice read slot j with one coalesced
// access.  Slots past a row's length are padding and never read.
constexpr int kSellRows = 64;
// Row alignment of the persistent schedules' chunks: four slices, one pass
// of a 256-thread workgroup over a chunk of one right-hand side.
constexpr int kChunkRows = 4 * kSellRows;
// gpu_sell_widths: width of every slice (host copy).  gpu_sell_fill: rlen[n]
// and the slotted columns and values (value_bits 64 or 32, like val) into
// buffers of `entries` = soff[n_slices] slots, and when sdel is not null the
// slotted column offsets as 16-bit integers (col - row taken modulo n into
// [-n/2, n/2)) with the largest |offset| in *max_offset: the offsets are
// valid only if it is at most 32767.
int gpu_sell_widths(int64_t n, const int32_t *rowptr, std::vector<int32_t> &width);
int gpu_sell_fill(int64_t n, const int32_t *rowptr, const int32_t *col, const void *val,
                  int value_bits, const int64_t *soff, int64_t entries, int32_t *rlen,
                  int32_t *scol, int16_t *sdel, void *sval, int32_t *max_offset);
// Levels from far[] (order_levels' rule): level 0 = row 0, level j+1 ends
// just past the farthest neighbour of level j.
Levels levels_from_far(int64_t n, const std::vector<int32_t> &far);

// Schedule of (chunk, power) tasks for p powers.
struct Schedule {
    int p = 0;
    std::vector<int32_t> chunk_ptr;    // n_chunks + 1 plan rows
    std::vector<int32_t> chunk_group;  // n_chunks
    std::vector<int32_t> dep_lo, dep_hi;
    std::vector<int32_t> tasks;        // 2 * n_tasks: (chunk, power)
    std::vector<int32_t> step_ptr;     // STEPS: n_steps + 1 task ranges, else empty
    // XCD schedule: exact dependency lists, owning XCD, write-back flags and
    // per-XCD task queues (tasks holds the queues one after the other)
    std::vector<int32_t> dep_ptr, dep_idx;
    std::vector<int32_t> chunk_xcd;
    std::vector<int32_t> remote_out;   // XCD: chunk read by another XCD (reported only)
    std::vector<int32_t> qptr;
    int32_t n_queues = 0;
    int32_t n_groups = 0, lag = 0, max_reach = 0;
    double window_bytes = 0.0, build_ms = 0.0;
    // Every chunk boundary except n is a multiple of kLineRows: a 128-byte
    // line of an output vector (128-byte aligned, n*R a multiple of 16) then
    // holds rows of one chunk only.  Tasks read rows of done chunks only, so
    // no cache can hold a copy of an output line from before the line was
    // complete, and tasks need no cache invalidation before their reads.
    bool line_closed = false;
    int32_t n_chunks() const { return (int32_t)chunk_group.size(); }
    int32_t n_tasks() const { return (int32_t)(tasks.size() / 2); }
    int32_t n_steps() const { return step_ptr.empty() ? 1 : (int32_t)step_ptr.size() - 1; }
};

struct PlanShape {
    int64_t n, nnz;
    int value_bytes;
    const std::vector<int32_t> *level_ptr;
    const std::vector<int32_t> *rowptr;  // plan order
    const std::vector<int32_t> *row_lo, *row_hi;
    const std::vector<int32_t> *pcol;    // plan-numbered columns (XCD schedule)
    int n_xcd;                           // XCDs that own parts of each level (>= 1)
    bool xcd_local;                      // tasks of one queue run on one XCD only
    int64_t l2_bytes = 4 << 20;          // per-XCD window budget (XCD schedule)
    int32_t min_group_rows = 0;          // smallest level group (STEPS, DIAG)
};

mpk_status_t build_schedule(const PlanShape &sh, int p, const mpk_tune_t &tune,
                            int default_workgroups, Schedule &out, std::string &err);

// Checks that the task list covers every (chunk, power) once and that each
// task's dependencies are issued before it (in an earlier step for STEPS).
bool validate_schedule(const Schedule &s, std::string &err);

// ------------------------------------------------------------------ device side

struct DevMatrix {
    const int32_t *rowptr;
    const int32_t *col;
    const void *val;          // double or float
    const int32_t *out_row;   // nullptr: output row = plan row
    int32_t n;
    int32_t value_bits;
    // the sliced layout (null when the plan has none: too much padding)
    const int64_t *soff;      // n_slices + 1 slot offsets
    const int32_t *rlen;      // n row lengths
    const int32_t *scol;      // slotted columns
    const int16_t *sdel;      // slotted column offsets (col - row modulo n, in
                              // [-n/2, n/2)) where they all fit 16 bits (the
                              // kernels then read these), or null
    const void *sval;         // slotted values (double or float)
};

constexpr int kMaxSegPowers = 64;   // powers per kernel launch

// Slices: runs of consecutive rows whose nonzeros fit one LDS staging buffer
// of KP*256 products (KP*256/R nonzeros for R right-hand sides), at most
// kSliceRows rows; a row longer than a buffer is a slice of its own.  For
// R >= 4 the kernels work on whole rows without staging, and slices are only
// row blocks of about KP*256 nonzeros.
constexpr int kSpmvKP = 16;   // products per thread and buffer, p x SpMV kernel
constexpr int kTaskKP = 16;   // the same for the level-blocked kernels
constexpr int kSliceRows = 256;
// Rows per 128-byte cache line of a single-RHS double vector; 16 rows of R
// right-hand sides are exactly R lines for any R.
constexpr int kLineRows = 16;
inline int slice_nnz(int kp, int R) { return R >= 4 ? kp * 256 : kp * 256 / R; }

// Cuts rows [bounds.front(), bounds.back()) into slices of at most E
// nonzeros; every entry of `bounds` (ascending row numbers) is also a slice
// boundary.  srow / snz get n_slices + 1 row / nonzero offsets, bound_sptr
// the slice index of every bound.
void build_slices(const std::vector<int32_t> &rowptr, const std::vector<int32_t> &bounds, int E,
                  std::vector<int32_t> &srow, std::vector<int32_t> &snz,
                  std::vector<int32_t> &bound_sptr);

struct DevSlices {
    const int32_t *srow;   // n_slices + 1 row offsets
    const int32_t *snz;    // n_slices + 1 nonzero offsets (rowptr at srow)
};

// Weighted sums of the powers (polynomial evaluation).  The task that
// computes y_m also holds y_{m-1} (its own input row) and y_{m-2} (read by the
// recurrence anyway), so the host groups each sum's nonzero terms into
// flushes: at power m the flagged terms among k = m-2, m-1, m are added in
// that order, either starting the sum or adding to it.  Each flush is one
// read-modify-write of the sum instead of one per term.
enum AccFlags : uint8_t {
    kAccT2 = 1,       // add w_{m-2} y_{m-2}
    kAccT1 = 2,       // add w_{m-1} y_{m-1}
    kAccT0 = 4,       // add w_m y_m
    kAccStart = 8,    // the sum's first flush: it starts with its first term
    kAccZero = 16,    // last power of a sum whose weights are all zero: store 0
};

struct Coefs {
    double alpha[kMaxSegPowers];
    double beta[kMaxSegPowers];
    double gamma[kMaxSegPowers];
};

// Weights and flushes of the two weighted sums for one segment: w[i] is the
// weight of the sequence's power k0 - 1 + i (0 outside 0..p), f[k-1] the
// AccFlags of the segment's power k.  (Kernels that take these are separate
// from the plain ones.)
struct AccCoefs {
    double wa[kMaxSegPowers + 2];
    double wb[kMaxSegPowers + 2];
    uint8_t fa[kMaxSegPowers];
    uint8_t fb[kMaxSegPowers];
};

// One launch covers powers 1..p of a segment: y_0 = in0, y_{-1} = inm1
// (recurrence only, may be null).  Plain kernels: outputs Y[(k-1)*n*R ...].
// Weighted-sum kernels: Y is a ring of two vectors, the segment's power k
// (the sequence's power g = k0 + k) goes to slot (g-1) mod 2, and acc_a /
// acc_b are the sums (acc_b may be null).
struct SegArgs {
    const double *in0;
    const double *inm1;
    double *Y;
    double *acc_a, *acc_b;
    int32_t p;
    int32_t R;
    int32_t recur;
    int32_t k0;
};

// The weighted-sum work of one power m of the p x SpMV kernel: weights of
// y_{m-2}, y_{m-1}, y_m and the AccFlags of each sum.
struct AccStep {
    double *acc_a, *acc_b;
    double wa[3], wb[3];
    int32_t fa, fb;
};

struct DevSchedule {
    DevSlices sl;
    const int32_t *chunk_sptr;   // n_chunks + 1 slice offsets
    const int32_t *chunk_row;    // n_chunks + 1 plan rows (sliced layout)
    const int32_t *dep_lo, *dep_hi;
    const int32_t *tasks;
    int32_t n_tasks, n_chunks;
};

constexpr int kMaxQueues = 16;

struct DevWorkspace {
    int32_t *done;      // n_chunks completion powers
    int32_t *ticket;    // next task (kMaxQueues counters for the XCD schedule)
    int32_t *err;       // this run failed: every workgroup leaves (cleared per run)
    int32_t *fail;      // a run on this workspace failed (kept until mpk_plan_sync)
    int32_t *status;    // the launch stream's status word (may be null)
};

// A failed wait: the run is abandoned (err), the failure is kept for
// mpk_plan_sync (fail) and for mpk_run_status on the launch stream (status).
constexpr int kStatusSlots = 256;  // status words per plan (streams share a slot beyond that)

struct DevXcdSchedule {
    DevSlices sl;
    const int32_t *chunk_sptr;
    const int32_t *chunk_row;    // n_chunks + 1 plan rows (sliced layout)
    const int32_t *dep_ptr, *dep_idx;
    const int32_t *tasks;
    const int32_t *qptr;
    int32_t n_queues, n_chunks;
};

// Launchers (kernels.hip).  All return hipError_t as int.
// Clears done[], the queue tickets and err before a run (fail stays; the
// status word too unless clear_status).
int launch_reset(const DevWorkspace &ws, int32_t n_chunks, void *stream, bool clear_status = false);

// The no-allocation run's dependency workspace: a file-scope device array of
// kScratchWords int32 (kernels.hip), one per device.  scratch_workspace
// returns its device address on `device` (looked up once per device, with
// that device current) as a hipError_t.
constexpr int64_t kScratchWords = 1 << 18;   // 1 MiB: done[] of up to 262126 chunks
int scratch_workspace(int device, int32_t **out);
// *out = *status_word, then *status_word = 0 (one thread; out may be pinned
// host memory).
int launch_status_copy(int32_t *status_word, int32_t *out, void *stream);
// pending > 0 selects the skip-ahead kernel with that many parked tasks (<= 8).
// acc != null: the ring / weighted-sum kernels (SegArgs ring, acc_a, acc_b).
// acquire = 0: tasks read their inputs without invalidating caches first
// (only valid for a line-closed schedule whose outputs are written in plan
// order into 128-byte aligned vectors, see Schedule::line_closed).
// static_order: workgroup b takes tasks b, b + workgroups, ... instead of
// tickets from the shared counter; valid only if every workgroup of the
// launch is resident (workgroups <= lb_resident_workgroups and no other
// static-order or XCD-queue launch overlapping it); not with pending > 0.
int launch_lb(const DevMatrix &m, const DevSchedule &s, const DevWorkspace &ws,
              const SegArgs &a, const Coefs *cf, const AccCoefs *acc, int workgroups,
              int64_t spin_limit, int pending, int acquire, bool static_order, void *stream);
// One diagonal of the STEPS schedule: workgroup b runs task tasks[b] = (chunk, power).
int launch_step(const DevMatrix &m, DevSlices sl, const int32_t *chunk_sptr,
                const int32_t *chunk_row, const int32_t *tasks, int32_t n_tasks,
                const SegArgs &a, const Coefs *cf, const AccCoefs *acc, void *stream);
// One power over all rows; workgroup b walks slices [b*per, (b+1)*per).
// acc may be null (no weighted sums).
int launch_spmv_power(const DevMatrix &m, DevSlices sl, int32_t n_slices, int32_t per,
                      const double *in, const double *inm1, double *out, int32_t R, int recur,
                      double alpha, double beta, double gamma, const AccStep *acc,
                      void *stream);
// out[i][2j] = a[i][2j] - b[i][2j+1], out[i][2j+1] = a[i][2j+1] + b[i][2j]
// for the n rows of R (even) columns.
int launch_combine_complex(const double *a, const double *b, int64_t n, int R, double *out,
                           void *stream);
int launch_permute(const int32_t *perm, int64_t n, int to_plan, const double *in, double *out,
                   int nvec, int R, void *stream);
int launch_load_probe(const double *buf, int64_t n_doubles, int passes, int workgroups,
                      double *sink, void *stream);
int launch_load_probe_xcd(const double *buf, int64_t n_doubles, int regions, int passes,
                          int workgroups, double *sink, int32_t *xcc, void *stream);
// The XCD schedule's persistent kernel: each workgroup takes tickets of its
// own XCD's queue.  Two launches must never overlap on one device (the
// caller serializes them).
int launch_xcd(const DevMatrix &m, const DevXcdSchedule &s, const DevWorkspace &ws,
               const SegArgs &a, const Coefs *cf, const AccCoefs *acc, int workgroups,
               int64_t spin_limit, int acquire, void *stream);
// XCDs of the device when workgroup i runs on XCD i mod n (checked with a probe
// kernel), else 1.
int detect_xcds(int device);
// Default persistent workgroups of the level-blocked kernel: what fits,
// capped at two per compute unit for the LDS-staged routine and four for the
// sliced layout (sell).
int lb_max_workgroups(int value_bits, int R, int device, bool sell);
// Workgroups of the level-blocked kernel (acc: the weighted-sum form) that
// the device holds at once: occupancy per compute unit x compute units.
int lb_resident_workgroups(int value_bits, int R, int device, bool sell, bool acc);

}  // namespace mpk
