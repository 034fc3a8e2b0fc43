// C ABI: plan construction, schedule cache, dependency workspaces and the run
// entry points declared in include/mpk.h.
#include <hip/hip_runtime_api.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <tuple>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "mpk_internal.h"

using namespace mpk;

namespace {

// Slices per workgroup of the p x SpMV kernel (consecutive slices pipeline).
constexpr int32_t kSpmvSlicesPerWG = 2;

thread_local std::string g_err;

mpk_status_t fail(mpk_status_t st, const std::string &msg) {
    g_err = msg;
    return st;
}

mpk_status_t hip_fail(hipError_t e, const char *what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return MPK_EHIP;
}

struct Allocator {
    void *(*alloc_fn)(size_t, void *) = nullptr;
    void (*free_fn)(void *, void *) = nullptr;
    void *ctx = nullptr;
};
std::mutex g_alloc_mu;
Allocator g_alloc;

// Device allocation through the installed hook (or hipMalloc).  The free
// function captured at allocation time is kept with the buffer.
struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    Allocator how;
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (!ptr) return;
        if (how.free_fn) how.free_fn(ptr, how.ctx);
        else (void)hipFree(ptr);
        ptr = nullptr;
        bytes = 0;
    }
    mpk_status_t alloc(size_t n) {
        release();
        if (n == 0) n = 16;
        {
            std::lock_guard<std::mutex> g(g_alloc_mu);
            how = g_alloc;
        }
        if (how.alloc_fn) {
            ptr = how.alloc_fn(n, how.ctx);
            if (!ptr) return fail(MPK_ENOMEM, "device allocator returned NULL");
        } else {
            hipError_t e = hipMalloc(&ptr, n);
            if (e != hipSuccess) {
                ptr = nullptr;
                return e == hipErrorOutOfMemory ? fail(MPK_ENOMEM, "hipMalloc: out of memory")
                                                : hip_fail(e, "hipMalloc");
            }
        }
        bytes = n;
        return MPK_OK;
    }
    mpk_status_t upload(const void *src, size_t n) {
        mpk_status_t st = alloc(n);
        if (st) return st;
        if (n && src) {
            hipError_t e = hipMemcpy(ptr, src, n, hipMemcpyHostToDevice);
            if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
        }
        return MPK_OK;
    }
    template <typename T> T *as() const { return static_cast<T *>(ptr); }
};

// Slice table of one right-hand-side count (the staging buffer holds a fixed
// number of products, so the nonzeros per slice depend on R).
struct SliceSet {
    DevBuf srow, snz, bound_sptr;
    int32_t n_slices = 0;
    DevSlices view() const { return DevSlices{srow.as<int32_t>(), snz.as<int32_t>()}; }
};

mpk_status_t make_slices(const std::vector<int32_t> &rowptr, const std::vector<int32_t> &bounds,
                         int E, bool upload_bounds, SliceSet &out) {
    std::vector<int32_t> srow, snz, bs;
    build_slices(rowptr, bounds, E, srow, snz, bs);
    out.n_slices = srow.empty() ? 0 : (int32_t)srow.size() - 1;
    mpk_status_t st;
    if ((st = out.srow.upload(srow.data(), srow.size() * 4))) return st;
    if ((st = out.snz.upload(snz.data(), snz.size() * 4))) return st;
    if (upload_bounds && (st = out.bound_sptr.upload(bs.data(), bs.size() * 4))) return st;
    return MPK_OK;
}

struct SchedEntry {
    Schedule host;
    std::map<int, std::unique_ptr<SliceSet>> slices;  // by slice size (slice_nnz of the RHS count)
    DevBuf dep_lo, dep_hi, tasks, chunk_row;
    DevBuf dep_ptr, dep_idx, qptr;  // XCD schedule
    int workgroups = 0;
};

struct Workspace {
    DevBuf buf;          // done[cap] | ticket[kMaxQueues] | err | fail
    int32_t cap = 0;
    hipEvent_t ev = nullptr;
    hipStream_t last_stream = nullptr;
    bool recorded = false;
    bool reserved = false;  // owned by a captured graph
    DevWorkspace view(int32_t *status = nullptr) const {
        int32_t *b = buf.as<int32_t>();
        return DevWorkspace{b, b + cap, b + cap + kMaxQueues, b + cap + kMaxQueues + 1, status};
    }
};

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct mpk_plan_s {
    int64_t n = 0, nnz = 0;
    int value_bits = 64, reorder = MPK_REORDER_BFS, order = MPK_ORDER_ORIGINAL;
    int device = MPK_DEVICE_NONE;
    bool host_only = true;
    double plan_ms = 0.0;
    int wall_khz = 100000;
    // host data kept for schedules and queries
    Levels lv;
    std::vector<int32_t> rowptr, row_lo, row_hi;
    std::vector<int32_t> col;    // stored columns (plan numbering if plan_cols)
    bool plan_cols = false;
    std::vector<int32_t> pcol;   // plan-numbered columns, built for the XCD schedule
    int pattern_sym = -1;        // structurally symmetric pattern (-1: not checked yet)
    int n_xcd = 8;               // XCDs found on the device (host-only plans: 8)
    bool xcd_bound = true;       // a workgroup can tell which XCD it runs on
    int64_t l2_bytes = 4 << 20, mall_bytes = 64 << 20;  // planner budgets
    int32_t min_group_rows = 0;
    int32_t sublevel_root = -1, max_sublevels = 0;     // MPK_REORDER_SUBLEVELS
    // device data
    DevBuf d_rowptr, d_col, d_val, d_outrow, d_perm;
    DevBuf d_soff, d_rlen, d_scol, d_sval;   // sliced layout (empty if not built)
    DevBuf d_sdel;                           // its 16-bit column offsets (if they fit)
    int64_t sell_entries = 0;
    std::map<int, std::unique_ptr<SliceSet>> spmv_slices;  // p x SpMV, by slice size
    // schedules and workspaces
    std::mutex mu;
    mpk_tune_t tune{};
    std::map<int, std::unique_ptr<SchedEntry>> scheds;
    std::vector<std::unique_ptr<SchedEntry>> retired;
    std::vector<std::unique_ptr<Workspace>> pool;
    std::map<long long, int> wg_cache;
    std::map<hipStream_t, hipEvent_t> stream_ev;  // last run issued per stream
    DevBuf status_words;                          // kStatusSlots failure words
    std::map<hipStream_t, int> status_slot;       // stream -> its word
    uint64_t fingerprint = 0;                     // of the input CSR and options

    DevMatrix matrix() const {
        return DevMatrix{d_rowptr.as<int32_t>(), d_col.as<int32_t>(), d_val.ptr,
                         d_outrow.as<int32_t>(), (int32_t)n, value_bits,
                         d_soff.as<const int64_t>(), d_rlen.as<int32_t>(), d_scol.as<int32_t>(),
                         d_sdel.as<int16_t>(), d_sval.ptr};
    }
    ~mpk_plan_s() {
        if (!host_only) {
            (void)hipSetDevice(device);
            for (auto &w : pool) {
                if (w->ev) {
                    (void)hipEventSynchronize(w->ev);
                    (void)hipEventDestroy(w->ev);
                }
            }
            for (auto &kv : stream_ev) {
                (void)hipEventSynchronize(kv.second);
                (void)hipEventDestroy(kv.second);
            }
            (void)hipDeviceSynchronize();
        }
    }
};

namespace {

mpk_status_t check_device_plan(mpk_plan_t plan) {
    if (!plan) return fail(MPK_EINVAL, "plan is NULL");
    if (plan->host_only) return fail(MPK_ENODEVICE, "plan was built without a device");
    return MPK_OK;
}

// Stored columns in plan numbering (built once when the plan keeps the
// caller's numbering; plan->mu held).  A device plan in the caller's own
// order keeps its columns on the device only; they are copied back here on
// first use.  Returns nullptr on failure.
const std::vector<int32_t> *plan_columns(mpk_plan_t plan) {
    if (plan->col.size() != (size_t)plan->nnz) {
        plan->col.resize((size_t)plan->nnz);
        hipError_t e = hipSetDevice(plan->device);
        if (e == hipSuccess)
            e = hipMemcpy(plan->col.data(), plan->d_col.ptr, (size_t)plan->nnz * 4,
                          hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
            plan->col.clear();
            hip_fail(e, "hipMemcpy (columns)");
            return nullptr;
        }
    }
    if (plan->plan_cols) return &plan->col;
    if (plan->pcol.size() != (size_t)plan->nnz) {
        plan->pcol.resize((size_t)plan->nnz);
        const int32_t *inv = plan->lv.iperm.data(), *c = plan->col.data();
        int32_t *out = plan->pcol.data();
        const int64_t nz = plan->nnz;
#pragma omp parallel for schedule(static)
        for (int64_t e = 0; e < nz; ++e) out[e] = inv[c[e]];
    }
    return &plan->pcol;
}

// Whether every stored off-diagonal entry (i, j) has a stored mirror (j, i).
// A symmetric permutation keeps this property, so the plan-order copy is
// checked.  Computed once (plan->mu held).
// Returns 1 or 0, or -1 when the columns could not be read back.
int pattern_symmetric(mpk_plan_t plan) {
    if (plan->pattern_sym >= 0) return plan->pattern_sym;
    const std::vector<int32_t> *pcp = plan_columns(plan);
    if (!pcp) return -1;
    const std::vector<int32_t> &pc = *pcp;
    const int32_t *rp = plan->rowptr.data();
    const int64_t n = plan->n;
    std::vector<int32_t> sorted(pc);
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t i = 0; i < n; ++i) std::sort(sorted.begin() + rp[i], sorted.begin() + rp[i + 1]);
    int ok = 1;
#pragma omp parallel for schedule(dynamic, 4096) reduction(min : ok)
    for (int64_t i = 0; i < n; ++i) {
        if (!ok) continue;
        for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
            const int32_t j = pc[e];
            if (j == i) continue;
            if (!std::binary_search(sorted.begin() + rp[j], sorted.begin() + rp[j + 1], (int32_t)i)) {
                ok = 0;
                break;
            }
        }
    }
    plan->pattern_sym = ok;
    return ok;
}

mpk_status_t get_schedule(mpk_plan_t plan, int p, SchedEntry **out, int default_wg) {
    auto it = plan->scheds.find(p);
    if (it != plan->scheds.end()) {
        *out = it->second.get();
        return MPK_OK;
    }
    auto e = std::make_unique<SchedEntry>();
    // the XCD schedule needs a workgroup on every XCD to drain every queue
    int n_xcd = plan->xcd_bound ? plan->n_xcd : 1;
    if (plan->tune.workgroups > 0 && plan->tune.workgroups < n_xcd) n_xcd = 1;
    const std::vector<int32_t> *pcol = &plan->col;
    if (plan->tune.schedule == MPK_SCHED_XCD) {  // exact dependency lists
        pcol = plan_columns(plan);
        if (!pcol) return MPK_EHIP;
    }
    PlanShape sh{plan->n, plan->nnz, plan->value_bits / 8, &plan->lv.level_ptr, &plan->rowptr,
                 &plan->row_lo, &plan->row_hi, pcol, n_xcd,
                 plan->xcd_bound && n_xcd > 1, plan->l2_bytes, plan->min_group_rows};
    std::string err;
    mpk_status_t st = build_schedule(sh, p, plan->tune, default_wg, e->host, err);
    if (st) return fail(st, err);
    if (!validate_schedule(e->host, err)) return fail(MPK_EINVAL, "schedule invalid: " + err);
    if (!plan->host_only) {
        const Schedule &s = e->host;
        if ((st = e->dep_lo.upload(s.dep_lo.data(), s.dep_lo.size() * 4))) return st;
        if ((st = e->dep_hi.upload(s.dep_hi.data(), s.dep_hi.size() * 4))) return st;
        if ((st = e->tasks.upload(s.tasks.data(), s.tasks.size() * 4))) return st;
        if ((st = e->chunk_row.upload(s.chunk_ptr.data(), s.chunk_ptr.size() * 4))) return st;
        if (!s.qptr.empty()) {
            if ((st = e->dep_ptr.upload(s.dep_ptr.data(), s.dep_ptr.size() * 4))) return st;
            if ((st = e->dep_idx.upload(s.dep_idx.data(), s.dep_idx.size() * 4))) return st;
            if ((st = e->qptr.upload(s.qptr.data(), s.qptr.size() * 4))) return st;
        }
    }
    *out = e.get();
    plan->scheds[p] = std::move(e);
    return MPK_OK;
}

// A dependency workspace that no unfinished run uses (plan->mu held).
mpk_status_t get_workspace(mpk_plan_t plan, int32_t n_chunks, hipStream_t stream, bool capturing,
                           Workspace **out, bool fresh = false) {
    for (auto &w : plan->pool) {
        if (fresh) break;
        if (w->reserved || w->cap < n_chunks) continue;
        bool free_now = !w->recorded || w->last_stream == stream;
        if (!free_now && !capturing) free_now = hipEventQuery(w->ev) == hipSuccess;
        if (free_now) {
            *out = w.get();
            return MPK_OK;
        }
    }
    if (capturing) {
        // allocation is not allowed while a stream is being captured
        return fail(MPK_EINVAL, "no idle workspace: call mpk_plan_prepare or run once outside capture first");
    }
    auto w = std::make_unique<Workspace>();
    w->cap = std::max<int32_t>(n_chunks, 1024);
    const size_t words = (size_t)w->cap + kMaxQueues + 2;
    mpk_status_t st = w->buf.alloc(words * sizeof(int32_t));
    if (st) return st;
    hipError_t e = hipMemset(w->buf.ptr, 0, words * sizeof(int32_t));
    if (e != hipSuccess) return hip_fail(e, "hipMemset");
    e = hipEventCreateWithFlags(&w->ev, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    *out = w.get();
    plan->pool.push_back(std::move(w));
    return MPK_OK;
}

// The failure word of runs issued on `stream` (plan->mu held).  Streams get
// words in the order they are first seen; past kStatusSlots they share.
int32_t *status_word(mpk_plan_t plan, hipStream_t stream) {
    auto it = plan->status_slot.find(stream);
    int slot;
    if (it != plan->status_slot.end()) {
        slot = it->second;
    } else {
        slot = (int)(plan->status_slot.size() % kStatusSlots);
        plan->status_slot.emplace(stream, slot);
    }
    return plan->status_words.as<int32_t>() + slot;
}

// Per device: the event recorded after the latest launch of a persistent
// kernel whose progress needs workgroups resident: the XCD schedule's (its
// workgroups serve the queue of the XCD they run on) and the static-order
// level-blocked kernel (every workgroup's tasks are fixed in advance).  Two
// overlapping launches could each hold compute units the other one's
// waiting tasks need and wait for each other until their limits; every such
// launch therefore waits for the previous one (other kernels may overlap
// it: they finish on their own, after which its workgroups get the device).
struct DeviceGate {
    std::mutex mu;
    hipEvent_t ev = nullptr;
    bool recorded = false;
};
DeviceGate &device_gate(int device) {
    static DeviceGate gates[64];
    return gates[device >= 0 && device < 64 ? device : 0];
}

// Set by mpk_graph_capture* around their capture: launches that need the
// gate may be captured, and the flag it points to is raised when one is;
// mpk_graph_launch then takes the gate around the whole graph.
thread_local bool *t_capture_gated = nullptr;

// The sliced layout of the plan's matrix, built on the device from its CSR
// (plan row order), unless padding each slice to its longest row would add
// more than a quarter to the stored entries (rows of uneven length: there
// the LDS-staged slices of the CSR were measured faster).  Where every
// column lies within 32767 of its row, modulo n (banded orders: a 27-point
// stencil's natural order reaches one plane; periodic lattices wrap), the
// kernels read 16-bit column offsets instead of the 32-bit columns: 10 bytes
// per FP64 entry instead of 12.
mpk_status_t build_sell(mpk_plan_t plan) {
    if (plan->n == 0 || plan->nnz == 0) return MPK_OK;
    std::vector<int32_t> width;
    int rc = gpu_sell_widths(plan->n, plan->d_rowptr.as<int32_t>(), width);
    if (rc) return hip_fail((hipError_t)rc, "slice widths");
    std::vector<int64_t> off(width.size() + 1, 0);
    for (size_t s = 0; s < width.size(); ++s) off[s + 1] = off[s] + (int64_t)width[s] * kSellRows;
    const int64_t entries = off.back();
    if (entries > plan->nnz + plan->nnz / 4 + (int64_t)kSellRows) return MPK_OK;
    mpk_status_t st;
    if ((st = plan->d_soff.upload(off.data(), off.size() * 8))) return st;
    if ((st = plan->d_rlen.alloc((size_t)plan->n * 4))) return st;
    if ((st = plan->d_scol.alloc((size_t)entries * 4))) return st;
    if ((st = plan->d_sval.alloc((size_t)entries * (plan->value_bits / 8)))) return st;
    // the offsets are filled in the same pass and dropped if one does not fit
    if ((st = plan->d_sdel.alloc((size_t)entries * 2))) return st;
    int32_t reach = 0;
    rc = gpu_sell_fill(plan->n, plan->d_rowptr.as<int32_t>(), plan->d_col.as<int32_t>(),
                       plan->d_val.ptr, plan->value_bits, plan->d_soff.as<const int64_t>(), entries,
                       plan->d_rlen.as<int32_t>(), plan->d_scol.as<int32_t>(),
                       plan->d_sdel.as<int16_t>(), plan->d_sval.ptr, &reach);
    if (rc) return hip_fail((hipError_t)rc, "sliced layout");
    if (reach > 32767) plan->d_sdel.release();
    plan->sell_entries = entries;
    return MPK_OK;
}

// Device-side state every device plan holds from the start (allocated
// outside any capture): the zeroed failure words.
mpk_status_t init_device_state(mpk_plan_t plan) {
    {
        DeviceGate &gate = device_gate(plan->device);
        std::lock_guard<std::mutex> g(gate.mu);
        if (!gate.ev) {
            hipError_t e = hipEventCreateWithFlags(&gate.ev, hipEventDisableTiming);
            if (e != hipSuccess) {
                gate.ev = nullptr;
                return hip_fail(e, "hipEventCreate");
            }
        }
    }
    mpk_status_t st = plan->status_words.alloc(kStatusSlots * sizeof(int32_t));
    if (st) return st;
    hipError_t e = hipMemset(plan->status_words.ptr, 0, kStatusSlots * sizeof(int32_t));
    return e == hipSuccess ? MPK_OK : hip_fail(e, "hipMemset");
}

// Workgroups of the level-blocked kernel the device holds at once (cached in
// wg_cache under negative keys, apart from default_workgroups' entries).
int resident_workgroups(mpk_plan_t plan, int R, bool acc) {
    const long long key = -((long long)plan->value_bits * 1000 + R * 2 + (acc ? 1 : 0)) - 1;
    auto it = plan->wg_cache.find(key);
    if (it != plan->wg_cache.end()) return it->second;
    const int wg = lb_resident_workgroups(plan->value_bits, R, plan->device,
                                          plan->d_scol.ptr != nullptr, acc);
    plan->wg_cache[key] = wg;
    return wg;
}

int default_workgroups(mpk_plan_t plan, int R) {
    const long long key = (long long)plan->value_bits * 1000 + R;
    auto it = plan->wg_cache.find(key);
    if (it != plan->wg_cache.end()) return it->second;
    int wg = lb_max_workgroups(plan->value_bits, R, plan->device, plan->d_scol.ptr != nullptr);
    if (wg <= 0) wg = 1024;
    plan->wg_cache[key] = wg;
    return wg;
}

mpk_status_t check_run_args(mpk_plan_t plan, const double *x, int p, int nrhs, double *Y) {
    if (!plan) return fail(MPK_EINVAL, "plan is NULL");
    if (p < 1) return fail(MPK_EINVAL, "p must be >= 1");
    if (nrhs < 1 || nrhs > MPK_MAX_RHS) return fail(MPK_EUNSUPPORTED, "nrhs must be in [1, 16]");
    mpk_status_t st = check_device_plan(plan);
    if (st) return st;
    if (plan->n > 0 && (!x || !Y)) return fail(MPK_EINVAL, "x or Y is NULL");
    const size_t xb = (size_t)plan->n * nrhs * sizeof(double);
    const char *xs = reinterpret_cast<const char *>(x), *ys = reinterpret_cast<const char *>(Y);
    if (plan->n > 0 && xs < ys + xb * (size_t)p && ys < xs + xb)
        return fail(MPK_EINVAL, "x and Y overlap");
    return MPK_OK;
}

// Remember the last run issued on `stream` so that mpk_plan_sync can wait
// for it (plan->mu held).
mpk_status_t note_stream(mpk_plan_t plan, hipStream_t stream) {
    auto it = plan->stream_ev.find(stream);
    if (it == plan->stream_ev.end()) {
        hipEvent_t ev;
        hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
        it = plan->stream_ev.emplace(stream, ev).first;
    }
    hipError_t e = hipEventRecord(it->second, stream);
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    return MPK_OK;
}

// Slices of a schedule's chunks for R right-hand sides (plan->mu held).
mpk_status_t task_slices(mpk_plan_t plan, SchedEntry *se, int R, SliceSet **out) {
    const int key = slice_nnz(kTaskKP, R);  // the same table for every R >= 4
    auto it = se->slices.find(key);
    if (it == se->slices.end()) {
        auto ss = std::make_unique<SliceSet>();
        mpk_status_t st = make_slices(plan->rowptr, se->host.chunk_ptr, key, true, *ss);
        if (st) return st;
        it = se->slices.emplace(key, std::move(ss)).first;
    }
    *out = it->second.get();
    return MPK_OK;
}

// Weighted sums of the powers (mpk_run_poly): host weights, device sums and
// the AccFlags of each power 1..p (index m) per sum.
struct Poly {
    const double *wa, *wb;
    double *acc_a, *acc_b;
    std::vector<uint8_t> fa, fb;
    int p;
    double w(const double *v, int k) const { return v && k >= 0 && k <= p ? v[k] : 0.0; }
};

// Flushes that make the device sum equal sum_{k=0..p} w[k] y_k taken in
// increasing k with zero weights skipped (all zero: the sum is zero).  The
// earliest pending term k is flushed as late as it can be, at power
// m = min(k+2, p), together with every nonzero term in k..m; the task at
// power m holds y_{m-2}, y_{m-1} and y_m.  With the Chebyshev weights, which
// alternate between the two sums, each sum is flushed every fourth power.
void acc_flushes(const double *w, int p, std::vector<uint8_t> &f) {
    f.assign((size_t)p + 1, 0);
    if (!w) return;
    bool started = false;
    int k = 0;
    for (;;) {
        while (k <= p && w[k] == 0.0) ++k;
        if (k > p) break;
        const int m = std::min(k + 2, p);
        uint8_t bits = started ? 0 : kAccStart;
        for (int j = k; j <= m; ++j)
            if (w[j] != 0.0) bits |= j == m ? kAccT0 : (j == m - 1 ? kAccT1 : kAccT2);
        f[(size_t)m] = bits;
        started = true;
        k = m + 1;
    }
    if (!started) f[(size_t)p] = kAccZero;
}

// The run of mpk_run_noalloc: the device's scratch workspace and the
// caller's status word instead of a pooled workspace and the stream's word.
struct NoAlloc {
    int32_t *scratch;
    int32_t *status;
};

// Y is the output (p vectors), or with poly the two-slot ring.  With `na`
// nothing is built, allocated or recorded: schedules, slice tables and the
// workgroup count must exist already.
mpk_status_t run_lb(mpk_plan_t plan, const double *x, int p, int nrhs, const double *alpha,
                    const double *beta, const double *gamma, double *Y, void *stream_v,
                    const Poly *poly = nullptr, const NoAlloc *na = nullptr) {
    mpk_status_t st = check_run_args(plan, x, poly ? 2 : p, nrhs, Y);
    if (st) return st;
    if (p < 1) return fail(MPK_EINVAL, "p must be >= 1");
    const bool recur = alpha != nullptr;
    if (recur && (!beta || !gamma)) return fail(MPK_EINVAL, "alpha, beta and gamma are all required");
    if (plan->n == 0) return MPK_OK;
    hipStream_t stream = static_cast<hipStream_t>(stream_v);
    hipError_t e = hipSetDevice(plan->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (stream) (void)hipStreamIsCapturing(stream, &cap);
    const bool capturing = cap == hipStreamCaptureStatusActive;

    std::lock_guard<std::mutex> g(plan->mu);
    if (poly) {
        const int sym = pattern_symmetric(plan);
        if (sym < 0) return MPK_EHIP;
        if (!sym)
            return fail(MPK_EUNSUPPORTED,
                        "the level-blocked weighted sums need a structurally symmetric pattern "
                        "(use the p x SpMV form)");
    }
    if (na && !plan->wg_cache.count((long long)plan->value_bits * 1000 + nrhs))
        return fail(MPK_EINVAL, "not prepared for this nrhs: call mpk_plan_prepare(plan, p, nrhs) first");
    const int wg_default = default_workgroups(plan, nrhs);
    const int wg = plan->tune.workgroups > 0 ? plan->tune.workgroups : wg_default;
    const int64_t limit_us = plan->tune.spin_limit_us > 0 ? plan->tune.spin_limit_us : 2000000;
    const int64_t spin_ticks = limit_us * (int64_t)plan->wall_khz / 1000;
    const size_t stride = (size_t)plan->n * nrhs;
    const DevMatrix m = plan->matrix();
    const int seg = plan->tune.seg_powers > 0 ? plan->tune.seg_powers : kMaxSegPowers;
    if (na) {  // the caller's status word reports this run only: 0 until a wait fails
        for (int base = 0; base < p; base += seg)
            if (!plan->scheds.count(std::min(seg, p - base)))
                return fail(MPK_EINVAL,
                            "no schedule for this p: call mpk_plan_prepare(plan, p, nrhs) first");
        int32_t *b = na->scratch;
        const DevWorkspace w0{b, b, b + kMaxQueues, b + kMaxQueues + 1, na->status};
        int rc = launch_reset(w0, 0, stream, true);
        if (rc) return hip_fail((hipError_t)rc, "reset kernel launch");
    }
    for (int base = 0; base < p; base += seg) {
        const int ps = std::min(seg, p - base);
        if (na && !plan->scheds.count(ps))
            return fail(MPK_EINVAL, "no schedule for this p: call mpk_plan_prepare(plan, p, nrhs) first");
        if (capturing && !plan->scheds.count(ps))  // building one would copy synchronously
            return fail(MPK_EINVAL,
                        "no schedule for this p: call mpk_plan_prepare or run once outside capture first");
        SchedEntry *se = nullptr;
        if ((st = get_schedule(plan, ps, &se, wg_default))) return st;
        SegArgs a{};
        if (poly) {  // ring of two: power g in slot (g-1) mod 2
            a.in0 = base == 0 ? x : Y + (size_t)((base - 1) & 1) * stride;
            a.inm1 = base == 0 ? nullptr : (base == 1 ? x : Y + (size_t)((base - 2) & 1) * stride);
            a.Y = Y;
            a.acc_a = poly->acc_a;
            a.acc_b = poly->acc_b;
        } else {
            a.in0 = base == 0 ? x : Y + (size_t)(base - 1) * stride;
            a.inm1 = base == 0 ? nullptr : (base == 1 ? x : Y + (size_t)(base - 2) * stride);
            a.Y = Y + (size_t)base * stride;
        }
        a.k0 = base;
        a.p = ps;
        a.R = nrhs;
        a.recur = recur ? 1 : 0;
        Coefs cf{};
        if (recur)
            for (int j = 0; j < ps; ++j) {
                cf.alpha[j] = alpha[base + j];
                cf.beta[j] = beta[base + j];
                cf.gamma[j] = gamma[base + j];
            }
        AccCoefs ac{};
        if (poly) {  // weights of the sequence's powers base-1 .. base+ps
            for (int i = 0; i < ps + 2; ++i) {
                ac.wa[i] = poly->w(poly->wa, base - 1 + i);
                ac.wb[i] = poly->w(poly->wb, base - 1 + i);
            }
            for (int j = 0; j < ps; ++j) {
                ac.fa[j] = poly->fa[(size_t)(base + j + 1)];
                ac.fb[j] = poly->fb[(size_t)(base + j + 1)];
            }
        }
        const AccCoefs *acp = poly ? &ac : nullptr;
        SliceSet *ss = nullptr;
        if ((capturing || na) && !se->slices.count(slice_nnz(kTaskKP, nrhs)))
            return fail(MPK_EINVAL, "no slice table for this RHS count: call mpk_plan_prepare first");
        if ((st = task_slices(plan, se, nrhs, &ss))) return st;
        if (!se->host.step_ptr.empty()) {
            // one launch per diagonal; stream order separates the diagonals
            const auto &sp = se->host.step_ptr;
            for (size_t d = 0; d + 1 < sp.size(); ++d) {
                int rc = launch_step(m, ss->view(), ss->bound_sptr.as<int32_t>(),
                                     se->chunk_row.as<int32_t>(),
                                     se->tasks.as<int32_t>() + 2 * (size_t)sp[d], sp[d + 1] - sp[d],
                                     a, &cf, acp, stream);
                if (rc) return hip_fail((hipError_t)rc, "step kernel launch");
            }
            continue;
        }
        const int32_t nc = se->host.n_chunks();
        Workspace *ws = nullptr;
        DevWorkspace wv;
        if (na) {
            if ((int64_t)nc + kMaxQueues + 2 > kScratchWords)
                return fail(MPK_EUNSUPPORTED,
                            "the schedule has " + std::to_string(nc) +
                                " chunks; the no-allocation run holds at most " +
                                std::to_string(kScratchWords - kMaxQueues - 2) +
                                " (raise tune.chunk_nnz)");
            int32_t *b = na->scratch;
            wv = DevWorkspace{b, b + nc, b + nc + kMaxQueues, b + nc + kMaxQueues + 1, na->status};
        } else {
            if ((st = get_workspace(plan, nc, stream, capturing, &ws))) return st;
            wv = ws->view(status_word(plan, stream));
        }
        DevSchedule ds{ss->view(), ss->bound_sptr.as<int32_t>(), se->chunk_row.as<int32_t>(),
                       se->dep_lo.as<int32_t>(),
                       se->dep_hi.as<int32_t>(), se->tasks.as<int32_t>(), se->host.n_tasks(),
                       se->host.n_chunks()};
        int rc = launch_reset(wv, nc, stream);
        if (rc) return hip_fail((hipError_t)rc, "reset kernel launch");
        // Without an invalidating acquire per task, an output line must
        // never be read before it is complete: the chunks must own whole
        // 128-byte lines of every output vector (line-closed schedule, plan
        // row order, 128-byte aligned outputs with n*R a multiple of 16) and
        // no address may be written twice in a run (not so for the ring of
        // the weighted-sum kernels).
        const bool lines_own = se->host.line_closed && !poly && !plan->d_outrow.ptr &&
                               ((size_t)plan->n * nrhs) % kLineRows == 0 &&
                               reinterpret_cast<uintptr_t>(Y) % 128 == 0;
        const int acquire = (plan->tune.acquire_always || !lines_own) ? 1 : 0;
        const bool xcd = !se->host.qptr.empty();
        // static task order: only where the launch can hold the device alone
        // (not under capture, whose launches the gate cannot order; no
        // skip-ahead; every workgroup resident at once)
        const bool own_capture = capturing && t_capture_gated != nullptr;
        const bool static_order = !xcd && (!capturing || own_capture) &&
                                  !plan->tune.dynamic_tickets && plan->tune.skip_ahead == 0 &&
                                  wg <= resident_workgroups(plan, nrhs, poly != nullptr);
        // at most one gated launch in flight per device: wait for the
        // previous one (any stream, any plan), then become the one to wait
        // for; under the library's own capture the graph's launch takes the
        // gate instead (another caller's capture is the caller's to order)
        if ((xcd || static_order) && own_capture) *t_capture_gated = true;
        const bool gated = (xcd || static_order) && !capturing;
        DeviceGate &gate = device_gate(plan->device);
        std::unique_lock<std::mutex> gl(gate.mu, std::defer_lock);
        if (gated) {
            gl.lock();
            if (gate.ev && gate.recorded) {
                e = hipStreamWaitEvent(stream, gate.ev, 0);
                if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
            }
        }
        if (xcd) {
            DevXcdSchedule xs{ss->view(), ss->bound_sptr.as<int32_t>(), se->chunk_row.as<int32_t>(),
                              se->dep_ptr.as<int32_t>(),
                              se->dep_idx.as<int32_t>(),
                              se->tasks.as<int32_t>(), se->qptr.as<int32_t>(),
                              se->host.n_queues, se->host.n_chunks()};
            rc = launch_xcd(m, xs, wv, a, &cf, acp, wg, spin_ticks, acquire, stream);
        } else {
            rc = launch_lb(m, ds, wv, a, &cf, acp, wg, spin_ticks, plan->tune.skip_ahead,
                           acquire, static_order, stream);
        }
        if (!rc && gated && gate.ev) {
            e = hipEventRecord(gate.ev, stream);
            if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
            gate.recorded = true;
        }
        if (gl.owns_lock()) gl.unlock();
        if (rc) return hip_fail((hipError_t)rc, "level-blocked kernel launch");
        if (na) continue;
        if (capturing) {
            ws->reserved = true;
        } else {
            e = hipEventRecord(ws->ev, stream);
            if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
            ws->recorded = true;
            ws->last_stream = stream;
        }
    }
    if (!capturing && !na && (st = note_stream(plan, stream))) return st;
    return MPK_OK;
}

// Slice table of the p x SpMV kernel for R right-hand sides, built once
// (plan->mu held).
mpk_status_t spmv_slices(mpk_plan_t plan, int R, SliceSet **out) {
    const int key = slice_nnz(kSpmvKP, R);
    auto it = plan->spmv_slices.find(key);
    if (it == plan->spmv_slices.end()) {
        auto ss = std::make_unique<SliceSet>();
        const std::vector<int32_t> whole{0, (int32_t)plan->n};
        mpk_status_t st = make_slices(plan->rowptr, whole, key, false, *ss);
        if (st) return st;
        it = plan->spmv_slices.emplace(key, std::move(ss)).first;
    }
    *out = it->second.get();
    return MPK_OK;
}

mpk_status_t run_baseline(mpk_plan_t plan, const double *x, int p, int nrhs, const double *alpha,
                          const double *beta, const double *gamma, double *Y, void *stream_v,
                          const Poly *poly = nullptr) {
    mpk_status_t st = check_run_args(plan, x, poly ? 2 : p, nrhs, Y);
    if (st) return st;
    if (p < 1) return fail(MPK_EINVAL, "p must be >= 1");
    const bool recur = alpha != nullptr;
    if (recur && (!beta || !gamma)) return fail(MPK_EINVAL, "alpha, beta and gamma are all required");
    if (plan->n == 0) return MPK_OK;
    hipError_t e = hipSetDevice(plan->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    hipStream_t stream = static_cast<hipStream_t>(stream_v);
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (stream) (void)hipStreamIsCapturing(stream, &cap);
    SliceSet *sl = nullptr;
    {
        std::lock_guard<std::mutex> g(plan->mu);
        if (cap == hipStreamCaptureStatusActive && !plan->spmv_slices.count(slice_nnz(kSpmvKP, nrhs)))
            return fail(MPK_EINVAL, "no slice table for this RHS count: call mpk_plan_prepare or run once outside capture first");
        if ((st = spmv_slices(plan, nrhs, &sl))) return st;
    }
    const size_t stride = (size_t)plan->n * nrhs;
    const DevMatrix m = plan->matrix();
    for (int k = 1; k <= p; ++k) {
        // with poly, Y is a ring of two: power k in slot (k-1) mod 2
        const size_t o_in = poly ? (size_t)((k - 2) & 1) : (size_t)(k - 2);
        const size_t o_prev = poly ? (size_t)((k - 3) & 1) : (size_t)(k - 3);
        const size_t o_out = poly ? (size_t)((k - 1) & 1) : (size_t)(k - 1);
        const double *in = k == 1 ? x : Y + o_in * stride;
        const double *prev = k == 1 ? nullptr : (k == 2 ? x : Y + o_prev * stride);
        double *out = Y + o_out * stride;
        AccStep as{};
        if (poly) {
            as.acc_a = poly->acc_a;
            as.acc_b = poly->acc_b;
            for (int i = 0; i < 3; ++i) {  // powers k-2, k-1, k
                as.wa[i] = poly->w(poly->wa, k - 2 + i);
                as.wb[i] = poly->w(poly->wb, k - 2 + i);
            }
            as.fa = poly->fa[(size_t)k];
            as.fb = poly->fb[(size_t)k];
        }
        int rc = launch_spmv_power(m, sl->view(), sl->n_slices, kSpmvSlicesPerWG, in, prev, out,
                                   nrhs, recur ? 1 : 0, recur ? alpha[k - 1] : 1.0,
                                   recur ? beta[k - 1] : 0.0, recur ? gamma[k - 1] : 0.0,
                                   poly ? &as : nullptr, stream_v);
        if (rc) return hip_fail((hipError_t)rc, "spmv kernel launch");
    }
    if (cap != hipStreamCaptureStatusActive) {
        std::lock_guard<std::mutex> g(plan->mu);
        if ((st = note_stream(plan, stream))) return st;
    }
    return MPK_OK;
}

// An FNV-style hash (one xor and multiply per 32-bit word) over the shape,
// the options, every row pointer and a sample of the columns (every step-th
// entry): the key of the autotuner's cache.  The row pointers are hashed in
// 64 fixed pieces in parallel and the piece hashes folded in order, so the
// key does not depend on the thread count.
int64_t fingerprint_step(int64_t nnz) { return std::max<int64_t>(1, nnz / 65536); }
uint64_t fingerprint(int64_t n, int64_t nnz, const mpk_plan_opts_t &o, const int32_t *rowptr,
                     const std::vector<int32_t> &sample) {
    constexpr uint64_t kBasis = 1469598103934665603ull, kPrime = 1099511628211ull;
    uint64_t h = kBasis;
    auto mix = [&h](uint64_t v) {
        h ^= v;
        h *= kPrime;
    };
    mix((uint64_t)n);
    mix((uint64_t)nnz);
    mix((uint64_t)o.reorder * 1000 + o.order * 100 + (uint64_t)o.root);
    // the planner inputs that change schedules or the row order
    mix((uint64_t)o.l2_bytes);
    mix((uint64_t)o.min_group_rows * 2 + (uint64_t)(uint32_t)o.sublevel_root * 4096);
    constexpr int kPieces = 64;
    uint64_t piece[kPieces];
    const int64_t len = n + 1;
#pragma omp parallel for schedule(static)
    for (int b = 0; b < kPieces; ++b) {
        uint64_t g = kBasis;
        for (int64_t i = len * b / kPieces; i < len * (b + 1) / kPieces; ++i) {
            g ^= (uint64_t)(uint32_t)rowptr[i];
            g *= kPrime;
        }
        piece[b] = g;
    }
    for (int b = 0; b < kPieces; ++b) mix(piece[b]);
    for (int32_t c : sample) mix((uint64_t)(uint32_t)c);
    return h;
}

// Weighted sums: argument checks shared by both forms.
mpk_status_t run_poly(mpk_plan_t plan, const double *x, int p, int nrhs, const double *alpha,
                      const double *beta, const double *gamma, const double *wa,
                      const double *wb, double *acc, double *work, void *stream, bool baseline) {
    if (!plan) return fail(MPK_EINVAL, "plan is NULL");
    if (p < 1) return fail(MPK_EINVAL, "p must be >= 1");
    if (!wa) return fail(MPK_EINVAL, "wa is NULL");
    if ((alpha || beta || gamma) && !(alpha && beta && gamma))
        return fail(MPK_EINVAL, "alpha, beta and gamma are all given or all NULL");
    if (nrhs < 1 || nrhs > MPK_MAX_RHS) return fail(MPK_EUNSUPPORTED, "nrhs must be in [1, 16]");
    if (plan->n > 0 && (!acc || !work)) return fail(MPK_EINVAL, "acc or work is NULL");
    const size_t vb = (size_t)plan->n * nrhs * sizeof(double);
    const size_t accb = vb * (wb ? 2 : 1);
    const char *ac = reinterpret_cast<const char *>(acc), *wk = reinterpret_cast<const char *>(work),
               *xs = reinterpret_cast<const char *>(x);
    if (plan->n > 0 && ((ac < wk + 2 * vb && wk < ac + accb) || (ac < xs + vb && xs < ac + accb)))
        return fail(MPK_EINVAL, "acc overlaps x or work");
    Poly poly;
    poly.wa = wa;
    poly.wb = wb;
    poly.acc_a = acc;
    poly.acc_b = wb ? acc + (size_t)plan->n * nrhs : nullptr;
    poly.p = p;
    acc_flushes(wa, p, poly.fa);
    acc_flushes(wb, p, poly.fb);
    return baseline ? run_baseline(plan, x, p, nrhs, alpha, beta, gamma, work, stream, &poly)
                    : run_lb(plan, x, p, nrhs, alpha, beta, gamma, work, stream, &poly);
}

// J_0(x) .. J_M(x), Bessel functions of the first kind, by Miller's backward
// recurrence: starting far above max(M, |x|) with J_{N+1} = 0 and J_N tiny,
// J_{k-1} = (2k/x) J_k - J_{k+1} runs down to k = 0 (the recurrence is
// stable downwards), and the unknown scale is fixed by the identity
// J_0 + 2 (J_2 + J_4 + ...) = 1.  The start never lies far beyond the order
// where |J_k(x)| <= (|x|/2)^k / k! drops below the smallest double, since
// every order past it is zero anyway.  J_k(-x) = (-1)^k J_k(x).
void bessel_j(int M, double x, double *J) {
    std::fill(J, J + M + 1, 0.0);
    if (x == 0.0) {
        J[0] = 1.0;
        return;
    }
    const double ax = std::fabs(x);
    const int m = std::max(M, (int)ax);
    int N = m + (int)std::sqrt(160.0 * m) + 30;
    for (int k = 1; k < N; ++k)  // first order whose bound is below 1e-330
        if (k > ax && k * std::log(ax / 2.0) - std::lgamma(k + 1.0) < -760.0) {
            N = std::min(N, k + 20);
            break;
        }
    N += N & 1;
    const int top = std::min(M, N);
    double bp1 = 0.0, b = 1e-300, even = 0.0;  // b = J_k up to scale, k = N
    if (N <= M) J[N] = b;
    for (int k = N; k >= 1; --k) {
        const double bm1 = (2.0 * k / ax) * b - bp1;
        bp1 = b;
        b = bm1;  // J_{k-1}
        if (k - 1 <= M) J[k - 1] = b;
        if (k - 1 >= 2 && !((k - 1) & 1)) even += b;
        if (std::fabs(b) > 1e250) {
            b *= 1e-250;
            bp1 *= 1e-250;
            even *= 1e-250;
            for (int j = k - 1; j <= top; ++j) J[j] *= 1e-250;
        }
    }
    const double norm = b + 2.0 * even;
    for (int k = 0; k <= top; ++k) {
        double v = J[k] / norm;
        if (x < 0.0 && (k & 1)) v = -v;
        J[k] = v;
    }
}

}  // namespace

extern "C" {

const char *mpk_last_error(void) { return g_err.c_str(); }

const char *mpk_version(void) { return "mpk-mi355x 0.1"; }

void mpk_plan_opts_default(mpk_plan_opts_t *o) {
    if (!o) return;
    o->value_bits = 64;
    o->reorder = MPK_REORDER_BFS;
    o->order = MPK_ORDER_ORIGINAL;
    o->root = 0;
    o->device = MPK_DEVICE_CURRENT;
    o->l2_bytes = (int64_t)4 << 20;
    o->mall_bytes = (int64_t)64 << 20;
    o->min_group_rows = 0;
    o->sublevel_root = MPK_ROOT_AUTO;
}

void mpk_tune_default(mpk_tune_t *t) {
    if (!t) return;
    t->schedule = MPK_SCHED_WAVE;
    t->cache_bytes = (int64_t)64 << 20;
    t->cache_safety = 1.0;
    t->chunk_nnz = 32768;
    t->lag = 0;
    t->workgroups = 0;
    t->spin_limit_us = 0;
    t->seg_powers = 0;
    t->skip_ahead = 0;
    t->acquire_always = 0;
    t->dynamic_tickets = 0;
}

mpk_status_t mpk_set_allocator(void *(*alloc_fn)(size_t, void *), void (*free_fn)(void *, void *),
                               void *ctx) {
    if ((alloc_fn == nullptr) != (free_fn == nullptr))
        return fail(MPK_EINVAL, "give both allocator functions or neither");
    std::lock_guard<std::mutex> g(g_alloc_mu);
    g_alloc = Allocator{alloc_fn, free_fn, ctx};
    return MPK_OK;
}

// Options shared by mpk_plan and mpk_plan_device; zero budgets take the defaults.
static mpk_status_t check_opts(mpk_plan_opts_t &o) {
    if (o.value_bits != 64 && o.value_bits != 32) return fail(MPK_EINVAL, "value_bits must be 32 or 64");
    if (o.reorder != MPK_REORDER_BFS && o.reorder != MPK_REORDER_NONE &&
        o.reorder != MPK_REORDER_SUBLEVELS)
        return fail(MPK_EINVAL, "bad reorder");
    if (o.order != MPK_ORDER_ORIGINAL && o.order != MPK_ORDER_PLAN) return fail(MPK_EINVAL, "bad order");
    if (o.l2_bytes < 0 || o.mall_bytes < 0 || o.min_group_rows < 0)
        return fail(MPK_EINVAL, "l2_bytes, mall_bytes and min_group_rows must be >= 0");
    if (o.l2_bytes == 0) o.l2_bytes = (int64_t)4 << 20;
    if (o.mall_bytes == 0) o.mall_bytes = (int64_t)64 << 20;
    if (o.l2_bytes < 65536 || o.mall_bytes < 65536)
        return fail(MPK_EINVAL, "l2_bytes and mall_bytes must be at least 64 KiB");
    if (o.sublevel_root < MPK_ROOT_AUTO) return fail(MPK_EINVAL, "bad sublevel_root");
    return MPK_OK;
}

mpk_status_t mpk_plan(const mpk_csr_t *A, const mpk_plan_opts_t *opts, mpk_plan_t *out) {
    if (!out) return fail(MPK_EINVAL, "out is NULL");
    *out = nullptr;
    mpk_plan_opts_t o;
    mpk_plan_opts_default(&o);
    if (opts) o = *opts;
    mpk_status_t st0 = check_opts(o);
    if (st0) return st0;
    const bool host_only = o.device == MPK_DEVICE_NONE;
    std::string err;
    mpk_status_t st = validate_csr(A, !host_only, err);
    if (st) return fail(st, err);
    if (A->n > 0 && o.root != MPK_ROOT_PERIPHERAL && (o.root < 0 || o.root >= A->n))
        return fail(MPK_EINVAL, "root out of range");
    if (A->n > 0 && o.sublevel_root >= A->n) return fail(MPK_EINVAL, "sublevel_root out of range");

    const double t0 = now_ms();
    std::unique_ptr<mpk_plan_s> plan;
    try {
        plan.reset(new mpk_plan_s());
        plan->n = A->n;
        plan->nnz = A->nnz;
        plan->value_bits = o.value_bits;
        plan->reorder = o.reorder;
        plan->order = o.order;
        plan->host_only = host_only;
        mpk_tune_default(&plan->tune);
        plan->l2_bytes = o.l2_bytes;
        plan->mall_bytes = o.mall_bytes;
        plan->min_group_rows = o.min_group_rows;
        plan->tune.cache_bytes = o.mall_bytes;
        const bool plan_cols = o.order == MPK_ORDER_PLAN;
        plan->plan_cols = plan_cols;
        const size_t nnz = (size_t)A->nnz;
        // BFS order on a device: levels and permutation on the GPU (the host
        // path below computes the same; the pseudo-peripheral root and
        // host-only plans take the host path)
        bool gpu_levels = !host_only && o.reorder == MPK_REORDER_BFS &&
                          o.root != MPK_ROOT_PERIPHERAL && A->n > 0;
        PermutedCSR pc;
        if (!host_only) {
            int dev = o.device;
            if (dev == MPK_DEVICE_CURRENT) {
                hipError_t e = hipGetDevice(&dev);
                if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
            }
            hipError_t e = hipSetDevice(dev);
            if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
            plan->device = dev;
            plan->n_xcd = detect_xcds(dev);
            plan->xcd_bound = plan->n_xcd > 1;
            int khz = 0;
            if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
                plan->wall_khz = khz;
            if ((st = init_device_state(plan.get()))) return st;
        }
        if (gpu_levels) {
            DevBuf rp0, c0, v0;  // the caller's CSR in its own order
            if ((st = rp0.upload(A->rowptr, ((size_t)A->n + 1) * 4))) return st;
            if ((st = c0.upload(A->col, nnz * 4))) return st;
            if ((st = v0.upload(A->val, nnz * 8))) return st;
            if ((st = plan->d_rowptr.alloc(((size_t)A->n + 1) * 4))) return st;
            if ((st = plan->d_col.alloc(nnz * 4))) return st;
            if ((st = plan->d_val.alloc(nnz * (size_t)(o.value_bits / 8)))) return st;
            GpuLevels g;
            const int rc = gpu_levels_permute(A->n, A->nnz, rp0.as<int32_t>(), c0.as<int32_t>(),
                                              v0.as<double>(), o.root, plan_cols, o.value_bits,
                                              plan->d_rowptr.as<int32_t>(),
                                              plan->d_col.as<int32_t>(), plan->d_val.ptr, g);
            if (rc == kTooManyLevels) {
                gpu_levels = false;  // many levels or components: the host planner
            } else if (rc) {
                return hip_fail((hipError_t)rc, "device level construction");
            } else {
                plan->lv.level_ptr.swap(g.level_ptr);
                plan->lv.perm.swap(g.perm);
                plan->lv.iperm.swap(g.iperm);
                plan->rowptr.swap(g.rowptr);
                plan->row_lo.swap(g.row_lo);
                plan->row_hi.swap(g.row_hi);
            }
        }
        if (!gpu_levels) {
            if (o.reorder == MPK_REORDER_NONE) {
                plan->lv = order_levels(A->n, A->rowptr, A->col);
            } else {
                plan->lv = bfs_levels(A->n, A->rowptr, A->col, o.root);
                if (o.reorder == MPK_REORDER_SUBLEVELS)
                    plan->lv = sublevel_order(A->n, A->rowptr, A->col, plan->lv, o.sublevel_root,
                                              &plan->sublevel_root, &plan->max_sublevels);
            }
            permute_csr(A->n, A->rowptr, A->col, host_only ? nullptr : A->val, plan->lv,
                        plan_cols, pc);
            plan->rowptr = pc.rowptr;
            plan->row_lo.swap(pc.row_lo);
            plan->row_hi.swap(pc.row_hi);
            if (!host_only) {
                if ((st = plan->d_rowptr.upload(pc.rowptr.data(), pc.rowptr.size() * 4))) return st;
                if ((st = plan->d_col.upload(pc.identity ? A->col : pc.col.data(), nnz * 4)))
                    return st;
                const double *v64 = pc.identity ? A->val : pc.val.data();
                if (o.value_bits == 64) {
                    if ((st = plan->d_val.upload(v64, nnz * 8))) return st;
                } else {
                    std::vector<float> v32(nnz);
#pragma omp parallel for schedule(static)
                    for (int64_t i = 0; i < (int64_t)nnz; ++i) v32[i] = (float)v64[i];
                    if ((st = plan->d_val.upload(v32.data(), nnz * 4))) return st;
                }
            }
        }
        if (!host_only) {
            bool identity = true;
            for (int64_t i = 0; i < A->n && identity; ++i) identity = plan->lv.perm[i] == i;
            if (!identity) {
                if ((st = plan->d_perm.upload(plan->lv.perm.data(), (size_t)A->n * 4))) return st;
                if (o.order == MPK_ORDER_ORIGINAL)
                    if ((st = plan->d_outrow.upload(plan->lv.perm.data(), (size_t)A->n * 4))) return st;
            }
        }
        // kept on the host for the schedules' dependency lists (device plans
        // built in place or on the GPU read them back when needed)
        if (host_only) {
            if (pc.identity) plan->col.assign(A->col, A->col + A->nnz);
            else plan->col.swap(pc.col);
        } else if (!gpu_levels && !pc.identity) {
            plan->col.swap(pc.col);
        }
    } catch (const std::bad_alloc &) {
        return fail(MPK_ENOMEM, "host allocation failed");
    } catch (const std::exception &ex) {
        return fail(MPK_EINVAL, ex.what());
    }
    {
        const int64_t step = fingerprint_step(A->nnz);
        std::vector<int32_t> sample;
        for (int64_t e2 = 0; e2 < A->nnz; e2 += step) sample.push_back(A->col[e2]);
        plan->fingerprint = fingerprint(A->n, A->nnz, o, A->rowptr, sample);
    }
    if (!host_only && (st = build_sell(plan.get()))) return st;
    plan->plan_ms = now_ms() - t0;
    *out = plan.release();
    return MPK_OK;
}

mpk_status_t mpk_plan_device(const mpk_csr_t *A, const mpk_plan_opts_t *opts, mpk_plan_t *out) {
    if (!out) return fail(MPK_EINVAL, "out is NULL");
    *out = nullptr;
    if (!A) return fail(MPK_EINVAL, "A is NULL");
    mpk_plan_opts_t o;
    mpk_plan_opts_default(&o);
    if (opts) o = *opts;
    if (o.device == MPK_DEVICE_NONE) return fail(MPK_EINVAL, "a device CSR needs a device plan");
    mpk_status_t st0 = check_opts(o);
    if (st0) return st0;
    if (A->n < 0 || A->nnz < 0) return fail(MPK_EBADCSR, "negative n or nnz");
    if (A->n >= (int64_t)INT32_MAX) return fail(MPK_EUNSUPPORTED, "n >= 2^31 is not supported");
    if (A->nnz >= (int64_t)INT32_MAX) return fail(MPK_EUNSUPPORTED, "nnz >= 2^31 is not supported");
    if (!A->rowptr || (A->nnz > 0 && (!A->col || !A->val))) return fail(MPK_EINVAL, "NULL array");
    if (A->n > 0 && o.root != MPK_ROOT_PERIPHERAL && (o.root < 0 || o.root >= A->n))
        return fail(MPK_EINVAL, "root out of range");
    if (A->n > 0 && o.sublevel_root >= A->n) return fail(MPK_EINVAL, "sublevel_root out of range");
    const double t0 = now_ms();
    int dev = o.device;
    if (dev == MPK_DEVICE_CURRENT) {
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    }
    hipError_t e = hipSetDevice(dev);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    const int64_t n = A->n, nnz = A->nnz;
    // validation on the device
    int bad_rows = 0, bad_cols = 0;
    int32_t ends[2] = {0, 0};
    int rc = gpu_validate(n, nnz, A->rowptr, A->col, &bad_rows, &bad_cols, ends);
    if (rc) return hip_fail((hipError_t)rc, "device validation");
    if (ends[0] != 0) return fail(MPK_EBADCSR, "rowptr[0] != 0");
    if (bad_rows) return fail(MPK_EBADCSR, "rowptr decreases");
    if ((int64_t)ends[1] != nnz) return fail(MPK_EBADCSR, "rowptr[n] != nnz");
    if (bad_cols) return fail(MPK_EBADCSR, "column index out of range");
    const bool plan_cols = o.order == MPK_ORDER_PLAN;
    // the pseudo-peripheral root, the sub-level order and graphs beyond the
    // device level search are planned from a host copy
    auto via_host = [&]() -> mpk_status_t {
        std::vector<int32_t> rp((size_t)n + 1), cl((size_t)nnz);
        std::vector<double> vl((size_t)nnz);
        hipError_t e2 = hipMemcpy(rp.data(), A->rowptr, rp.size() * 4, hipMemcpyDeviceToHost);
        if (e2 == hipSuccess && nnz)
            e2 = hipMemcpy(cl.data(), A->col, cl.size() * 4, hipMemcpyDeviceToHost);
        if (e2 == hipSuccess && nnz)
            e2 = hipMemcpy(vl.data(), A->val, vl.size() * 8, hipMemcpyDeviceToHost);
        if (e2 != hipSuccess) return hip_fail(e2, "hipMemcpy (device CSR to host)");
        mpk_csr_t H{n, nnz, rp.data(), cl.data(), vl.data()};
        mpk_plan_opts_t o2 = o;
        o2.device = dev;
        return mpk_plan(&H, &o2, out);
    };
    if ((o.reorder == MPK_REORDER_BFS && o.root == MPK_ROOT_PERIPHERAL) ||
        o.reorder == MPK_REORDER_SUBLEVELS)
        return via_host();
    std::unique_ptr<mpk_plan_s> plan;
    try {
        plan.reset(new mpk_plan_s());
        plan->n = n;
        plan->nnz = nnz;
        plan->value_bits = o.value_bits;
        plan->reorder = o.reorder;
        plan->order = o.order;
        plan->host_only = false;
        plan->plan_cols = plan_cols;
        mpk_tune_default(&plan->tune);
        plan->l2_bytes = o.l2_bytes;
        plan->mall_bytes = o.mall_bytes;
        plan->min_group_rows = o.min_group_rows;
        plan->tune.cache_bytes = o.mall_bytes;
        plan->device = dev;
        plan->n_xcd = detect_xcds(dev);
        plan->xcd_bound = plan->n_xcd > 1;
        int khz = 0;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
            plan->wall_khz = khz;
        mpk_status_t st;
        if ((st = init_device_state(plan.get()))) return st;
        if ((st = plan->d_rowptr.alloc(((size_t)n + 1) * 4))) return st;
        if ((st = plan->d_col.alloc((size_t)nnz * 4))) return st;
        if ((st = plan->d_val.alloc((size_t)nnz * (size_t)(o.value_bits / 8)))) return st;
        if (o.reorder == MPK_REORDER_BFS && n > 0) {
            GpuLevels g;
            rc = gpu_levels_permute(n, nnz, A->rowptr, A->col, A->val, o.root, plan_cols,
                                    o.value_bits, plan->d_rowptr.as<int32_t>(),
                                    plan->d_col.as<int32_t>(), plan->d_val.ptr, g);
            if (rc == kTooManyLevels) {
                plan.reset();
                return via_host();
            }
            if (rc) return hip_fail((hipError_t)rc, "device level construction");
            plan->lv.level_ptr.swap(g.level_ptr);
            plan->lv.perm.swap(g.perm);
            plan->lv.iperm.swap(g.iperm);
            plan->rowptr.swap(g.rowptr);
            plan->row_lo.swap(g.row_lo);
            plan->row_hi.swap(g.row_hi);
        } else {
            // the caller's order: order-derived levels from the device's far[]
            std::vector<int32_t> far;
            if (n > 0 && (rc = gpu_order_far(n, A->rowptr, A->col, far)))
                return hip_fail((hipError_t)rc, "device level extents");
            plan->lv = levels_from_far(n, far);
            rc = gpu_copy_in_place_order(n, nnz, A->rowptr, A->col, A->val, o.value_bits,
                                         plan->d_rowptr.as<int32_t>(), plan->d_col.as<int32_t>(),
                                         plan->d_val.ptr, plan->rowptr, plan->row_lo,
                                         plan->row_hi);
            if (rc) return hip_fail((hipError_t)rc, "device copy of the matrix");
        }
        bool identity = true;
        for (int64_t i = 0; i < n && identity; ++i) identity = plan->lv.perm[i] == i;
        if (!identity) {
            if ((st = plan->d_perm.upload(plan->lv.perm.data(), (size_t)n * 4))) return st;
            if (o.order == MPK_ORDER_ORIGINAL)
                if ((st = plan->d_outrow.upload(plan->lv.perm.data(), (size_t)n * 4))) return st;
        }
        // the same fingerprint as a plan of the same matrix from host arrays
        const int64_t step = fingerprint_step(nnz);
        std::vector<int32_t> sample, rp0;
        if ((rc = gpu_sample_cols(A->col, step, nnz ? (nnz + step - 1) / step : 0, sample)))
            return hip_fail((hipError_t)rc, "hipMemcpy (column sample)");
        const int32_t *rph = plan->rowptr.data();   // the caller's, in its own order
        if (o.reorder == MPK_REORDER_BFS) {               // the plan's is permuted
            rp0.resize((size_t)n + 1);
            e = hipMemcpy(rp0.data(), A->rowptr, rp0.size() * 4, hipMemcpyDeviceToHost);
            if (e != hipSuccess) return hip_fail(e, "hipMemcpy (row pointer)");
            rph = rp0.data();
        }
        plan->fingerprint = fingerprint(n, nnz, o, rph, sample);
        mpk_status_t st2 = build_sell(plan.get());
        if (st2) return st2;
    } catch (const std::bad_alloc &) {
        return fail(MPK_ENOMEM, "host allocation failed");
    } catch (const std::exception &ex) {
        return fail(MPK_EINVAL, ex.what());
    }
    plan->plan_ms = now_ms() - t0;
    *out = plan.release();
    return MPK_OK;
}

void mpk_plan_destroy(mpk_plan_t plan) { delete plan; }

mpk_status_t mpk_plan_tune(mpk_plan_t plan, const mpk_tune_t *tune) {
    if (!plan) return fail(MPK_EINVAL, "plan is NULL");
    mpk_tune_t t;
    mpk_tune_default(&t);
    t.cache_bytes = plan->mall_bytes;  // the plan's budget C
    if (tune) t = *tune;
    if (t.schedule < MPK_SCHED_STEPS || t.schedule > MPK_SCHED_XCD) return fail(MPK_EINVAL, "bad schedule");
    if (t.cache_bytes <= 0 || !(t.cache_safety > 0.0) || t.cache_safety > 1.0)
        return fail(MPK_EINVAL, "cache_bytes must be > 0 and cache_safety in (0, 1]");
    if (t.skip_ahead < 0 || t.skip_ahead > 8) return fail(MPK_EINVAL, "skip_ahead must be in [0, 8]");
    if (t.seg_powers < 0 || t.seg_powers > kMaxSegPowers)
        return fail(MPK_EINVAL, "seg_powers must be in [0, 64]");
    if (t.chunk_nnz < 1 || t.lag < 0 || t.workgroups < 0 || t.spin_limit_us < 0)
        return fail(MPK_EINVAL, "negative tuning value");
    if (t.acquire_always != 0 && t.acquire_always != 1)
        return fail(MPK_EINVAL, "acquire_always must be 0 or 1");
    if (t.dynamic_tickets != 0 && t.dynamic_tickets != 1)
        return fail(MPK_EINVAL, "dynamic_tickets must be 0 or 1");
    std::lock_guard<std::mutex> g(plan->mu);
    plan->tune = t;
    // schedules may still be read by queued kernels: keep them until destroy
    for (auto &kv : plan->scheds) plan->retired.push_back(std::move(kv.second));
    plan->scheds.clear();
    return MPK_OK;
}

mpk_status_t mpk_plan_info(mpk_plan_t plan, mpk_plan_info_t *info) {
    if (!plan || !info) return fail(MPK_EINVAL, "NULL argument");
    info->n = plan->n;
    info->nnz = plan->nnz;
    info->n_levels = (int32_t)plan->lv.level_ptr.size() - 1;
    int32_t mx = 0;
    for (size_t l = 0; l + 1 < plan->lv.level_ptr.size(); ++l)
        mx = std::max(mx, plan->lv.level_ptr[l + 1] - plan->lv.level_ptr[l]);
    info->max_level_rows = mx;
    info->value_bits = plan->value_bits;
    info->reorder = plan->reorder;
    info->order = plan->order;
    info->matrix_bytes = 4 * (plan->n + 1) + (4 + plan->value_bits / 8) * plan->nnz;
    info->plan_ms = plan->plan_ms;
    info->device = plan->device;
    info->sliced_layout = plan->d_scol.ptr ? 1 : 0;
    info->sliced_entries = plan->sell_entries;
    info->sliced_col_bits = plan->d_sdel.ptr ? 16 : (plan->d_scol.ptr ? 32 : 0);
    info->fingerprint = plan->fingerprint;
    info->sublevel_root = plan->sublevel_root;
    info->max_sublevels = plan->max_sublevels;
    info->l2_bytes = plan->l2_bytes;
    info->mall_bytes = plan->mall_bytes;
    info->min_group_rows = plan->min_group_rows;
    return MPK_OK;
}

mpk_status_t mpk_plan_levels(mpk_plan_t plan, int32_t *level_ptr, int32_t *perm) {
    if (!plan) return fail(MPK_EINVAL, "plan is NULL");
    if (level_ptr) std::copy(plan->lv.level_ptr.begin(), plan->lv.level_ptr.end(), level_ptr);
    if (perm) std::copy(plan->lv.perm.begin(), plan->lv.perm.end(), perm);
    return MPK_OK;
}

mpk_status_t mpk_plan_schedule(mpk_plan_t plan, int p, mpk_sched_info_t *info, int32_t *chunk_ptr,
                               int32_t *chunk_group, int32_t *dep_lo, int32_t *dep_hi,
                               int32_t *tasks, int32_t *step_ptr) {
    if (!plan) return fail(MPK_EINVAL, "plan is NULL");
    if (p < 1 || p > kMaxSegPowers) return fail(MPK_EINVAL, "p must be in [1, 64]");
    std::lock_guard<std::mutex> g(plan->mu);
    int wg = 2048;
    if (!plan->host_only) wg = default_workgroups(plan, 1);
    SchedEntry *se = nullptr;
    mpk_status_t st = get_schedule(plan, p, &se, wg);
    if (st) return st;
    const Schedule &s = se->host;
    if (info) {
        info->p = s.p;
        info->n_chunks = s.n_chunks();
        info->n_groups = s.n_groups;
        info->n_tasks = s.n_tasks();
        info->n_steps = s.n_steps();
        info->lag = s.lag;
        info->max_reach = s.max_reach;
        info->window_bytes = s.window_bytes;
        info->build_ms = s.build_ms;
        info->n_queues = s.qptr.empty() ? 1 : s.n_queues;
        info->n_deps = s.qptr.empty() ? 0 : (int32_t)s.dep_idx.size();
    }
    if (chunk_ptr) std::copy(s.chunk_ptr.begin(), s.chunk_ptr.end(), chunk_ptr);
    if (chunk_group) std::copy(s.chunk_group.begin(), s.chunk_group.end(), chunk_group);
    if (dep_lo) std::copy(s.dep_lo.begin(), s.dep_lo.end(), dep_lo);
    if (dep_hi) std::copy(s.dep_hi.begin(), s.dep_hi.end(), dep_hi);
    if (tasks) std::copy(s.tasks.begin(), s.tasks.end(), tasks);
    if (step_ptr) {
        if (s.step_ptr.empty()) {
            step_ptr[0] = 0;
            step_ptr[1] = s.n_tasks();
        } else {
            std::copy(s.step_ptr.begin(), s.step_ptr.end(), step_ptr);
        }
    }
    return MPK_OK;
}

mpk_status_t mpk_plan_schedule_xcd(mpk_plan_t plan, int p, int32_t *dep_ptr, int32_t *dep_idx,
                                   int32_t *chunk_xcd, int32_t *remote_out, int32_t *qptr) {
    if (!plan) return fail(MPK_EINVAL, "plan is NULL");
    if (p < 1 || p > kMaxSegPowers) return fail(MPK_EINVAL, "p must be in [1, 64]");
    std::lock_guard<std::mutex> g(plan->mu);
    int wg = 2048;
    if (!plan->host_only) wg = default_workgroups(plan, 1);
    SchedEntry *se = nullptr;
    mpk_status_t st = get_schedule(plan, p, &se, wg);
    if (st) return st;
    const Schedule &s = se->host;
    if (s.qptr.empty()) return fail(MPK_EINVAL, "the current schedule is not MPK_SCHED_XCD");
    if (dep_ptr) std::copy(s.dep_ptr.begin(), s.dep_ptr.end(), dep_ptr);
    if (dep_idx) std::copy(s.dep_idx.begin(), s.dep_idx.end(), dep_idx);
    if (chunk_xcd) std::copy(s.chunk_xcd.begin(), s.chunk_xcd.end(), chunk_xcd);
    if (remote_out) std::copy(s.remote_out.begin(), s.remote_out.end(), remote_out);
    if (qptr) std::copy(s.qptr.begin(), s.qptr.end(), qptr);
    return MPK_OK;
}

mpk_status_t mpk_run(mpk_plan_t plan, const double *x, int p, int nrhs, double *Y, void *stream) {
    return run_lb(plan, x, p, nrhs, nullptr, nullptr, nullptr, Y, stream);
}

mpk_status_t mpk_run_noalloc(mpk_plan_t plan, const double *x, int p, int nrhs, double *Y,
                             int32_t *status, void *stream) {
    mpk_status_t st = check_device_plan(plan);
    if (st) return st;
    int32_t *scratch = nullptr;
    int rc = scratch_workspace(plan->device, &scratch);
    if (rc) return hip_fail((hipError_t)rc, "hipGetSymbolAddress (scratch workspace)");
    const NoAlloc na{scratch, status};
    return run_lb(plan, x, p, nrhs, nullptr, nullptr, nullptr, Y, stream, nullptr, &na);
}

mpk_status_t mpk_run_recur(mpk_plan_t plan, const double *x, int p, int nrhs, const double *alpha,
                           const double *beta, const double *gamma, double *Y, void *stream) {
    if (!alpha || !beta || !gamma) return fail(MPK_EINVAL, "coefficient array is NULL");
    return run_lb(plan, x, p, nrhs, alpha, beta, gamma, Y, stream);
}

mpk_status_t mpk_run_baseline(mpk_plan_t plan, const double *x, int p, int nrhs, double *Y,
                              void *stream) {
    return run_baseline(plan, x, p, nrhs, nullptr, nullptr, nullptr, Y, stream);
}

mpk_status_t mpk_run_baseline_recur(mpk_plan_t plan, const double *x, int p, int nrhs,
                                    const double *alpha, const double *beta, const double *gamma,
                                    double *Y, void *stream) {
    if (!alpha || !beta || !gamma) return fail(MPK_EINVAL, "coefficient array is NULL");
    return run_baseline(plan, x, p, nrhs, alpha, beta, gamma, Y, stream);
}

mpk_status_t mpk_run_poly(mpk_plan_t plan, const double *x, int p, int nrhs, const double *alpha,
                          const double *beta, const double *gamma, const double *wa,
                          const double *wb, double *acc, double *work, void *stream) {
    return run_poly(plan, x, p, nrhs, alpha, beta, gamma, wa, wb, acc, work, stream, false);
}

mpk_status_t mpk_run_baseline_poly(mpk_plan_t plan, const double *x, int p, int nrhs,
                                   const double *alpha, const double *beta, const double *gamma,
                                   const double *wa, const double *wb, double *acc, double *work,
                                   void *stream) {
    return run_poly(plan, x, p, nrhs, alpha, beta, gamma, wa, wb, acc, work, stream, true);
}

mpk_status_t mpk_plan_prepare(mpk_plan_t plan, int p, int nrhs) {
    if (!plan) return fail(MPK_EINVAL, "plan is NULL");
    if (p < 1) return fail(MPK_EINVAL, "p must be >= 1");
    if (nrhs < 1 || nrhs > MPK_MAX_RHS) return fail(MPK_EUNSUPPORTED, "nrhs must be in [1, 16]");
    mpk_status_t st = check_device_plan(plan);
    if (st) return st;
    if (plan->n == 0) return MPK_OK;
    hipError_t e = hipSetDevice(plan->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    std::lock_guard<std::mutex> g(plan->mu);
    // the same schedules, slice tables and workspace a run would fetch first
    const int wg_default = default_workgroups(plan, nrhs);
    const int seg = plan->tune.seg_powers > 0 ? plan->tune.seg_powers : kMaxSegPowers;
    for (int base = 0; base < p; base += seg) {
        SchedEntry *se = nullptr;
        if ((st = get_schedule(plan, std::min(seg, p - base), &se, wg_default))) return st;
        SliceSet *ss = nullptr;
        if ((st = task_slices(plan, se, nrhs, &ss))) return st;
        if (se->host.step_ptr.empty()) {
            Workspace *ws = nullptr;
            if ((st = get_workspace(plan, se->host.n_chunks(), nullptr, false, &ws))) return st;
        }
    }
    SliceSet *sl = nullptr;
    return spmv_slices(plan, nrhs, &sl);
}

mpk_status_t mpk_cheb_time_coefficients(int M, double dt, double *alpha, double *beta,
                                        double *gamma, double *wa, double *wb) {
    if (M < 1 || M > 100000) return fail(MPK_EINVAL, "M must be in [1, 100000]");
    if (!std::isfinite(dt) || std::fabs(dt) > 1e4)
        return fail(MPK_EINVAL, "dt must be finite with |dt| <= 1e4");
    if (!alpha || !beta || !gamma || !wa || !wb) return fail(MPK_EINVAL, "NULL array");
    std::vector<double> J((size_t)M + 1);
    bessel_j(M, dt, J.data());
    for (int k = 0; k < M; ++k) {  // v_1 = H v_0, v_{k+1} = 2 H v_k - v_{k-1}
        alpha[k] = k == 0 ? 1.0 : 2.0;
        beta[k] = 0.0;
        gamma[k] = k == 0 ? 0.0 : -1.0;
    }
    wa[0] = J[0];
    wb[0] = 0.0;
    for (int k = 1; k <= M; ++k) {  // 2 (-i)^k J_k: (-i)^k cycles 1, -i, -1, i
        const double c = 2.0 * J[(size_t)k];
        switch (k & 3) {
        case 0: wa[k] = c; wb[k] = 0.0; break;
        case 1: wa[k] = 0.0; wb[k] = -c; break;
        case 2: wa[k] = -c; wb[k] = 0.0; break;
        default: wa[k] = 0.0; wb[k] = c; break;
        }
    }
    return MPK_OK;
}

mpk_status_t mpk_combine_complex(mpk_plan_t plan, const double *acc, int nrhs, double *out,
                                 void *stream) {
    mpk_status_t st = check_device_plan(plan);
    if (st) return st;
    if (nrhs < 2 || nrhs > MPK_MAX_RHS || (nrhs & 1))
        return fail(MPK_EINVAL, "nrhs must be even, 2..16 (real and imaginary columns)");
    if (plan->n == 0) return MPK_OK;
    if (!acc || !out) return fail(MPK_EINVAL, "NULL vector");
    if ((reinterpret_cast<uintptr_t>(acc) | reinterpret_cast<uintptr_t>(out)) & 15)
        return fail(MPK_EINVAL, "acc and out must be 16-byte aligned");
    const size_t vb = (size_t)plan->n * nrhs * sizeof(double);
    const char *a = reinterpret_cast<const char *>(acc), *b = reinterpret_cast<const char *>(out);
    if (a < b + vb && b < a + 2 * vb) return fail(MPK_EINVAL, "acc and out overlap");
    hipError_t e = hipSetDevice(plan->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    int rc = launch_combine_complex(acc, acc + (size_t)plan->n * nrhs, plan->n, nrhs, out, stream);
    return rc ? hip_fail((hipError_t)rc, "combine kernel launch") : MPK_OK;
}

mpk_status_t mpk_permute(mpk_plan_t plan, int to_plan, const double *in, double *out, int nvec,
                         int nrhs, void *stream) {
    mpk_status_t st = check_device_plan(plan);
    if (st) return st;
    if (nvec < 0 || nrhs < 1 || nrhs > MPK_MAX_RHS) return fail(MPK_EINVAL, "bad nvec or nrhs");
    if (plan->n == 0 || nvec == 0) return MPK_OK;
    if (!in || !out) return fail(MPK_EINVAL, "NULL vector");
    const size_t bytes = (size_t)plan->n * nrhs * nvec * sizeof(double);
    const char *a = reinterpret_cast<const char *>(in), *b = reinterpret_cast<const char *>(out);
    if (a < b + bytes && b < a + bytes) return fail(MPK_EINVAL, "in and out overlap");
    hipError_t e = hipSetDevice(plan->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    if (!plan->d_perm.ptr) {  // identity ordering
        e = hipMemcpyAsync(out, in, bytes, hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream));
        return e == hipSuccess ? MPK_OK : hip_fail(e, "hipMemcpyAsync");
    }
    int rc = launch_permute(plan->d_perm.as<int32_t>(), plan->n, to_plan, in, out, nvec, nrhs, stream);
    return rc ? hip_fail((hipError_t)rc, "permute kernel launch") : MPK_OK;
}

mpk_status_t mpk_probe_load(const double *buf, int64_t n, int passes, int workgroups,
                            double *sink, void *stream) {
    if (!buf || !sink || n < 2 || (n & 1) || passes < 1 || workgroups < 1)
        return fail(MPK_EINVAL, "probe needs buf, sink, an even n >= 2, passes and workgroups >= 1");
    int rc = launch_load_probe(buf, n, passes, workgroups, sink, stream);
    return rc ? hip_fail((hipError_t)rc, "probe kernel launch") : MPK_OK;
}

mpk_status_t mpk_probe_load_xcd(const double *buf, int64_t n, int regions, int passes,
                                int workgroups, double *sink, int32_t *xcc, void *stream) {
    if (!buf || !sink || !xcc || regions < 1 || regions > kMaxQueues || passes < 1 ||
        workgroups < 1 || n < 2 * (int64_t)regions || n % (2 * (int64_t)regions))
        return fail(MPK_EINVAL, "probe needs buf, sink, xcc, 1 <= regions <= 16, n a multiple of "
                                "2 x regions, passes and workgroups >= 1");
    int rc = launch_load_probe_xcd(buf, n, regions, passes, workgroups, sink, xcc, stream);
    return rc ? hip_fail((hipError_t)rc, "probe kernel launch") : MPK_OK;
}

mpk_status_t mpk_plan_autotune(mpk_plan_t plan, const double *x, int p, int nrhs, double *Y,
                               int reps, int force, int recur, void *stream_v, mpk_tune_t *best,
                               double *best_ms) {
    mpk_status_t st = check_run_args(plan, x, p, nrhs, Y);
    if (st) return st;
    if (reps < 1 || reps > 100) return fail(MPK_EINVAL, "reps must be in [1, 100]");
    if (plan->n == 0) return fail(MPK_EINVAL, "nothing to tune for an empty matrix");
    if (recur < 0 || recur > 2) return fail(MPK_EINVAL, "recur must be 0, 1 or 2");
    if (recur == 2 && p < 4)
        return fail(MPK_EINVAL, "tuning the weighted sums needs p >= 4 (Y holds their scratch)");
    hipStream_t stream = static_cast<hipStream_t>(stream_v);
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (stream) (void)hipStreamIsCapturing(stream, &cap);
    if (cap != hipStreamCaptureStatusNone) return fail(MPK_EINVAL, "cannot autotune while capturing");
    mpk_tune_t base;
    {
        std::lock_guard<std::mutex> g(plan->mu);
        base = plan->tune;
    }
    // a plan set to the shared counter (for runs beside other kernels) keeps
    // it in every candidate
    const int keep_dyn = base.dynamic_tickets;
    using Key = std::tuple<uint64_t, int, int, int, int, int>;
    static std::mutex cache_mu;
    static std::map<Key, std::pair<mpk_tune_t, double>> cache;
    const Key key{plan->fingerprint, plan->value_bits, p, nrhs, recur, keep_dyn};
    if (!force) {
        std::pair<mpk_tune_t, double> hit;
        bool found = false;
        {
            std::lock_guard<std::mutex> g(cache_mu);
            auto it = cache.find(key);
            if (it != cache.end()) {
                hit = it->second;
                found = true;
            }
        }
        if (found) {
            mpk_tune_t t = hit.first;
            t.spin_limit_us = base.spin_limit_us;
            if ((st = mpk_plan_tune(plan, &t))) return st;
            if (best) *best = t;
            if (best_ms) *best_ms = hit.second;
            return MPK_OK;
        }
    }
    // candidates: the paper's study varies the cache size C (and p x C by
    // splitting p); here C, the chunk size, the schedule, the number of
    // persistent workgroups, segments of p and skip-ahead parking
    std::vector<mpk_tune_t> cands;
    auto add = [&](int sched, int64_t cache_mib, int chunk, int lag, int wg = 0, int seg = 0,
                   int skip = 0, int dyn = 0) {
        mpk_tune_t t = base;
        t.schedule = sched;
        t.cache_bytes = cache_mib << 20;
        t.cache_safety = 1.0;
        t.chunk_nnz = chunk;
        t.lag = lag;
        t.workgroups = wg;
        t.seg_powers = seg;
        t.skip_ahead = skip;
        t.dynamic_tickets = dyn | keep_dyn;
        for (const mpk_tune_t &c : cands)
            if (c.schedule == t.schedule && c.cache_bytes == t.cache_bytes &&
                c.chunk_nnz == t.chunk_nnz && c.lag == t.lag && c.workgroups == t.workgroups &&
                c.seg_powers == t.seg_powers && c.skip_ahead == t.skip_ahead &&
                c.dynamic_tickets == t.dynamic_tickets)
                return;  // the same candidate once more
        cands.push_back(t);
    };
    for (int64_t c : {32, 64, 128})
        for (int chunk : {4096, 8192}) add(MPK_SCHED_STEPS, c, chunk, 0);
    // (chunks are capped so that each running workgroup gets two per power:
    // 65536 means "as large as that allows", e.g. ~54K nonzeros for 2^21 rows
    // of a 27-point stencil)
    for (int chunk : {8192, 16384, 32768, 65536}) add(MPK_SCHED_WAVE, 64, chunk, 0);
    add(MPK_SCHED_XCD, 64, 16384, 0);
    add(MPK_SCHED_POWERS, 64, 8192, 0);
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, plan->device) !=
            hipSuccess || cus < 1)
        cus = 0;
    if (cus > 0) {  // one persistent workgroup per compute unit instead of two
        add(MPK_SCHED_WAVE, 64, 32768, 0, cus);
        add(MPK_SCHED_POWERS, 64, 8192, 0, cus);
    }
    if (cus > 0 && plan->d_scol.ptr) {
        // sliced layout: two or four workgroups per compute unit, and a
        // wavefront slack of 1-3 times the running workgroups per power
        // (the default is 8 times: no waits, but a window far beyond the
        // fast cache; smaller slack keeps the window smaller and the
        // inputs cached, at the risk of waits that cascade); power order
        // with up to eight workgroups per compute unit
        for (int wpc : {2, 4})
            for (int m2 : {2, 3, 4, 6})
                for (int chunk : {8192, 16384})
                    add(MPK_SCHED_WAVE, 64, chunk, std::max(1, m2 * wpc * cus / (2 * p)),
                        wpc * cus);
        for (int wpc : {2, 4, 8})
            for (int chunk : {8192, 16384}) add(MPK_SCHED_POWERS, 64, chunk, 0, wpc * cus);
        // the shared counter as well: where a task's inputs come from many
        // chunks (random columns within wide bands) the fixed order can
        // leave workgroups waiting that the counter would have given other
        // tasks; the timing decides
        for (int wpc : {2, 4}) {
            add(MPK_SCHED_POWERS, 64, 8192, 0, wpc * cus, 0, 0, 1);
            add(MPK_SCHED_WAVE, 64, 16384, std::max(1, 2 * wpc * cus / p), wpc * cus, 0, 0, 1);
        }
        add(MPK_SCHED_POWERS, 64, 4096, 0, 8 * cus, 0, 0, 1);
    }
    if (p >= 4) add(MPK_SCHED_WAVE, 64, 32768, 0, 0, (p + 1) / 2);  // two segments
    add(MPK_SCHED_WAVE, 64, 16384, 0, 0, 0, 2);                     // park up to two tasks
    // Chebyshev coefficients for timing the recurrence (values do not change the time)
    std::vector<double> al(p), be(p, 0.0), ga(p, -1.0);
    for (int k = 0; k < p; ++k) al[k] = k == 0 ? 1.0 : 2.0;
    ga[0] = 0.0;
    hipEvent_t e0, e1;
    hipError_t e = hipEventCreate(&e0);
    if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        (void)hipEventDestroy(e0);
        return hip_fail(e, "hipEventCreate");
    }
    // weighted sums (recur == 2): Chebyshev time-step weights for dt = 1, the
    // sums and the two-vector ring in Y (the values do not change the time)
    const size_t vec = (size_t)plan->n * nrhs;
    std::vector<double> tal(p), tbe(p), tga(p), twa(p + 1), twb(p + 1);
    if (recur == 2 &&
        (st = mpk_cheb_time_coefficients(p, 1.0, tal.data(), tbe.data(), tga.data(), twa.data(),
                                          twb.data())))
        return st;
    auto one = [&]() {
        if (recur == 2)
            return run_poly(plan, x, p, nrhs, tal.data(), tbe.data(), tga.data(), twa.data(),
                            twb.data(), Y, Y + 2 * vec, stream_v, false);
        return recur ? run_lb(plan, x, p, nrhs, al.data(), be.data(), ga.data(), Y, stream_v)
                     : run_lb(plan, x, p, nrhs, nullptr, nullptr, nullptr, Y, stream_v);
    };
    // `reps` timed runs of candidate i after one untimed run (which builds
    // its schedule and slices on the first call); appends to sum / count.
    // Returns false when a wait hit its limit (not a candidate) or on an
    // error (st set).
    bool timed_out = false;
    auto time_cand = [&](size_t i, double &sum, int &count) {
        if ((st = mpk_plan_tune(plan, &cands[i]))) return false;
        if ((st = one())) return false;
        if (mpk_plan_sync(plan) != MPK_OK) {
            timed_out = true;
            return false;
        }
        for (int r = 0; r < reps && st == MPK_OK; ++r) {
            e = hipEventRecord(e0, stream);
            if (e == hipSuccess) st = one();
            if (e == hipSuccess && st == MPK_OK) e = hipEventRecord(e1, stream);
            if (e == hipSuccess && st == MPK_OK) e = hipEventSynchronize(e1);
            float f = 0.f;
            if (e == hipSuccess && st == MPK_OK) e = hipEventElapsedTime(&f, e0, e1);
            if (e != hipSuccess && st == MPK_OK) st = hip_fail(e, "timing a candidate");
            sum += f;
            ++count;
        }
        if (st) return false;
        if (mpk_plan_sync(plan) != MPK_OK) {
            timed_out = true;
            return false;
        }
        return true;
    };
    // the mean, not the median: a schedule whose run time is bimodal (waits
    // that cascade only sometimes) must not win on a lucky draw; for the
    // same reason the three fastest are timed once more, after all the
    // others, and compared on all their runs
    std::vector<double> sum(cands.size(), 0.0);
    std::vector<int> count(cands.size(), 0);
    std::vector<size_t> ok;
    for (size_t i = 0; i < cands.size() && st == MPK_OK; ++i)
        if (time_cand(i, sum[i], count[i])) ok.push_back(i);
    auto mean = [&](size_t i) { return sum[i] / (double)count[i]; };
    std::sort(ok.begin(), ok.end(), [&](size_t a, size_t b) { return mean(a) < mean(b); });
    if (ok.size() > 3) ok.resize(3);
    double best_t = 0.0;
    int best_i = -1;
    for (size_t j = 0; j < ok.size() && st == MPK_OK; ++j) {
        const size_t i = ok[j];
        if (ok.size() > 1 && !time_cand(i, sum[i], count[i])) continue;
        if (best_i < 0 || mean(i) < best_t) {
            best_t = mean(i);
            best_i = (int)i;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st) return st;
    if (best_i < 0)
        return fail(timed_out ? MPK_ETIMEOUT : MPK_EINVAL, "no candidate tuning completed");
    if ((st = mpk_plan_tune(plan, &cands[best_i]))) return st;
    {
        std::lock_guard<std::mutex> g(cache_mu);
        cache[key] = {cands[best_i], best_t};
    }
    if (best) *best = cands[best_i];
    if (best_ms) *best_ms = best_t;
    return MPK_OK;
}

}  // extern "C"

struct mpk_graph_s {
    hipStream_t stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int device = 0;
    bool gated = false;  // holds a launch that needs the device gate
    ~mpk_graph_s() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (stream) (void)hipStreamDestroy(stream);
    }
};

extern "C" {

mpk_status_t mpk_graph_capture(mpk_plan_t plan, const double *x, int p, int nrhs,
                               const double *alpha, const double *beta, const double *gamma,
                               double *Y, mpk_graph_t *out) {
    if (!out) return fail(MPK_EINVAL, "out is NULL");
    *out = nullptr;
    mpk_status_t st = check_run_args(plan, x, p, nrhs, Y);
    if (st) return st;
    if (alpha && (!beta || !gamma)) return fail(MPK_EINVAL, "alpha, beta and gamma are all required");
    hipError_t e = hipSetDevice(plan->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    std::unique_ptr<mpk_graph_s> g(new mpk_graph_s());
    e = hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
    if (plan->n > 0) {
        // everything a run allocates or uploads is prepared before the capture
        std::lock_guard<std::mutex> lk(plan->mu);
        const int wg_default = default_workgroups(plan, nrhs);
        const int seg = plan->tune.seg_powers > 0 ? plan->tune.seg_powers : kMaxSegPowers;
        for (int base = 0; base < p; base += seg) {
            const int ps = std::min(seg, p - base);
            SchedEntry *se = nullptr;
            if ((st = get_schedule(plan, ps, &se, wg_default))) return st;
            SliceSet *ss = nullptr;
            if ((st = task_slices(plan, se, nrhs, &ss))) return st;
            if (se->host.step_ptr.empty()) {
                Workspace *ws = nullptr;
                // a never-used workspace: the capture below can take it without an event query
                if ((st = get_workspace(plan, se->host.n_chunks(), g->stream, false, &ws, true)))
                    return st;
            }
        }
    }
    g->device = plan->device;
    e = hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    t_capture_gated = &g->gated;
    st = run_lb(plan, x, p, nrhs, alpha, beta, gamma, Y, g->stream);
    t_capture_gated = nullptr;
    e = hipStreamEndCapture(g->stream, &g->graph);
    if (st) return st;
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    *out = g.release();
    return MPK_OK;
}

mpk_status_t mpk_graph_capture_time_step(mpk_plan_t plan, const double *psi, int nrhs, double dt,
                                         int M, int baseline, double *out, double *acc,
                                         double *work, mpk_graph_t *graph) {
    if (!graph) return fail(MPK_EINVAL, "graph is NULL");
    *graph = nullptr;
    mpk_status_t st = check_device_plan(plan);
    if (st) return st;
    if (nrhs < 2 || nrhs > MPK_MAX_RHS || (nrhs & 1))
        return fail(MPK_EINVAL, "nrhs must be even, 2..16 (real and imaginary columns)");
    if (M < 1 || M > 100000) return fail(MPK_EINVAL, "M must be in [1, 100000]");
    std::vector<double> al((size_t)M), be((size_t)M), ga((size_t)M), wa((size_t)M + 1),
        wb((size_t)M + 1);
    if ((st = mpk_cheb_time_coefficients(M, dt, al.data(), be.data(), ga.data(), wa.data(),
                                         wb.data())))
        return st;
    if (plan->n > 0 && (!psi || !out || !acc || !work)) return fail(MPK_EINVAL, "NULL vector");
    const size_t vb = (size_t)plan->n * nrhs * sizeof(double);
    const char *o = reinterpret_cast<const char *>(out);
    const char *ranges[3][2] = {{reinterpret_cast<const char *>(psi), nullptr},
                                {reinterpret_cast<const char *>(acc), nullptr},
                                {reinterpret_cast<const char *>(work), nullptr}};
    const size_t lens[3] = {vb, 2 * vb, 2 * vb};
    for (int i = 0; i < 3 && plan->n > 0; ++i)
        if (o < ranges[i][0] + lens[i] && ranges[i][0] < o + vb)
            return fail(MPK_EINVAL, "out overlaps psi, acc or work");
    if (plan->n > 0 && ((reinterpret_cast<uintptr_t>(acc) | reinterpret_cast<uintptr_t>(out)) & 15))
        return fail(MPK_EINVAL, "acc and out must be 16-byte aligned");
    hipError_t e = hipSetDevice(plan->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    std::unique_ptr<mpk_graph_s> g(new mpk_graph_s());
    e = hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "hipStreamCreate");
    if (plan->n > 0) {
        // everything a run allocates or uploads is prepared before the capture
        std::lock_guard<std::mutex> lk(plan->mu);
        if (baseline) {
            SliceSet *ss = nullptr;
            if ((st = spmv_slices(plan, nrhs, &ss))) return st;
        } else {
            const int sym = pattern_symmetric(plan);
            if (sym < 0) return MPK_EHIP;
            if (!sym)
                return fail(MPK_EUNSUPPORTED,
                            "the level-blocked weighted sums need a structurally symmetric pattern "
                            "(use the p x SpMV form)");
            const int wg_default = default_workgroups(plan, nrhs);
            const int seg = plan->tune.seg_powers > 0 ? plan->tune.seg_powers : kMaxSegPowers;
            for (int base = 0; base < M; base += seg) {
                SchedEntry *se = nullptr;
                if ((st = get_schedule(plan, std::min(seg, M - base), &se, wg_default))) return st;
                SliceSet *ss = nullptr;
                if ((st = task_slices(plan, se, nrhs, &ss))) return st;
                if (se->host.step_ptr.empty()) {
                    Workspace *ws = nullptr;
                    if ((st = get_workspace(plan, se->host.n_chunks(), g->stream, false, &ws, true)))
                        return st;
                }
            }
        }
    }
    g->device = plan->device;
    e = hipStreamBeginCapture(g->stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
    t_capture_gated = &g->gated;
    st = run_poly(plan, psi, M, nrhs, al.data(), be.data(), ga.data(), wa.data(), wb.data(), acc,
                  work, g->stream, baseline != 0);
    t_capture_gated = nullptr;
    if (!st && plan->n > 0) {
        const int rc = launch_combine_complex(acc, acc + (size_t)plan->n * nrhs, plan->n, nrhs,
                                              out, g->stream);
        if (rc) st = hip_fail((hipError_t)rc, "combine kernel launch");
    }
    e = hipStreamEndCapture(g->stream, &g->graph);
    if (st) return st;
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
    *graph = g.release();
    return MPK_OK;
}

mpk_status_t mpk_graph_launch(mpk_graph_t graph, void *stream_v) {
    if (!graph) return fail(MPK_EINVAL, "graph is NULL");
    hipStream_t stream = static_cast<hipStream_t>(stream_v);
    if (!graph->gated) {
        hipError_t e = hipGraphLaunch(graph->exec, stream);
        return e == hipSuccess ? MPK_OK : hip_fail(e, "hipGraphLaunch");
    }
    // the graph holds a launch that must not overlap another gated one
    DeviceGate &gate = device_gate(graph->device);
    std::lock_guard<std::mutex> gl(gate.mu);
    hipError_t e = hipSuccess;
    if (gate.ev && gate.recorded) e = hipStreamWaitEvent(stream, gate.ev, 0);
    if (e != hipSuccess) return hip_fail(e, "hipStreamWaitEvent");
    e = hipGraphLaunch(graph->exec, stream);
    if (e != hipSuccess) return hip_fail(e, "hipGraphLaunch");
    if (gate.ev) {
        e = hipEventRecord(gate.ev, stream);
        if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
        gate.recorded = true;
    }
    return MPK_OK;
}

void mpk_graph_destroy(mpk_graph_t graph) { delete graph; }

mpk_status_t mpk_run_status(mpk_plan_t plan, void *stream_v, int32_t *status) {
    mpk_status_t st = check_device_plan(plan);
    if (st) return st;
    if (!status) return fail(MPK_EINVAL, "status is NULL");
    hipStream_t stream = static_cast<hipStream_t>(stream_v);
    hipError_t e = hipSetDevice(plan->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    int32_t *word;
    {
        std::lock_guard<std::mutex> g(plan->mu);
        word = status_word(plan, stream);
    }
    int rc = launch_status_copy(word, status, stream);
    return rc ? hip_fail((hipError_t)rc, "status kernel launch") : MPK_OK;
}

mpk_status_t mpk_plan_sync(mpk_plan_t plan) {
    mpk_status_t st = check_device_plan(plan);
    if (st) return st;
    std::lock_guard<std::mutex> g(plan->mu);
    hipError_t e = hipSetDevice(plan->device);
    if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
    for (auto &kv : plan->stream_ev) {
        e = hipEventSynchronize(kv.second);
        if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    }
    bool timeout = false;
    for (auto &w : plan->pool) {
        if (w->recorded) {
            e = hipEventSynchronize(w->ev);
            if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
        }
        int32_t flag = 0;
        e = hipMemcpy(&flag, w->view().fail, sizeof(int32_t), hipMemcpyDeviceToHost);
        if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
        if (flag) {
            timeout = true;
            const int32_t zero = 0;
            e = hipMemcpy(w->view().fail, &zero, sizeof(int32_t), hipMemcpyHostToDevice);
            if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
        }
    }
    if (timeout) return fail(MPK_ETIMEOUT, "a dependency wait exceeded its limit; results are invalid");
    return MPK_OK;
}

}  // extern "C"
