// HIP kernels for gfx950 (MI355X): CSR products for one power, the p x SpMV
// baseline, the level-blocked kernels (one launch per diagonal, and three
// persistent dataflow forms: in ticket order, with skip-ahead parking, and
// with per-XCD queues), permutation, reset and a load-bandwidth probe.
//
// Every run kernel goes through one row routine.  For R < 4 right-hand sides
// (run_slices) the host cuts the rows into slices (consecutive rows whose
// products fit one LDS staging buffer, at most 256 rows; a longer row is a
// slice of its own) and a workgroup walks a range of slices:
//   1. it reads a slice's column indices and values with coalesced loads,
//      gathers the matching input entries and stores the products
//      a_e * x_{col(e), r} in LDS (one rounded multiply each);
//   2. each (row, right-hand side) pair is then summed by one thread,
//      sequentially in stored order starting from 0.0, with no fused
//      multiply-add.
// The loads of the next slice are issued before the current slice is summed
// (two LDS buffers), so one memory latency per slice is hidden behind the
// other's arithmetic.  For R >= 4 (run_rows) one thread per (row, right-hand
// side) sums its row directly, in the same order.  Either way the summation
// order is the plain CSR definition itself: results do not depend on
// slicing, chunking, schedule or right-hand-side count.  Values stored as
// float are promoted to double before the product; vectors and sums are
// double.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "mpk_internal.h"

namespace mpk {

// Dependency workspace of mpk_run_noalloc (done[] | tickets | err | fail),
// for callers that cannot allocate.  Every GPU holds its own copy until the
// process ends; host code uses the address from scratch_workspace, never
// this name.
static __device__ __align__(256) int32_t scratch[kScratchWords];

namespace {

constexpr int kBlock = 256;          // threads per workgroup (4 wavefronts of 64)
// Waves per SIMD the level-blocked kernels are built for: two 66 KB staging
// footprints fit a CU with 16 products per thread, four with 8.
constexpr int kTaskWaves = kTaskKP >= 16 ? 2 : 4;
constexpr int kWave = 64;
static_assert(kSliceRows == kBlock, "one thread per row of a slice");

__device__ __forceinline__ int ld_relaxed(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A wait hit its limit: abandon the run and record the failure.
__device__ __forceinline__ void record_failure(const DevWorkspace &ws) {
    __hip_atomic_store(ws.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(ws.fail, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (ws.status) __hip_atomic_store(ws.status, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

struct PowerIO {
    const double *in;     // y_{k-1}
    const double *prev;   // y_{k-2} (recurrence; null at the very first power)
    double *out;          // y_k
    double alpha, beta, gamma;
    int recur;
    // weighted sums of the powers: weights of y_{k-2}, y_{k-1}, y_k and the
    // AccFlags of each sum (kernels with the sums only)
    double *acc_a, *acc_b;
    double wa2, wa1, wa0, wb2, wb1, wb0;
    int fa, fb;
};

// y = alpha*s + beta*y_{k-1} + gamma*y_{k-2} evaluated left to right, or s.
// A coefficient that is exactly zero omits its term (and its vector read):
// the Chebyshev recurrence has no beta term.
__device__ __forceinline__ double epilogue(const PowerIO &io, double s, size_t idx) {
    if (!io.recur) return s;
    double v = io.alpha * s;
    if (io.beta != 0.0) {
        const double b = io.beta * io.in[idx];
        v = v + b;
    }
    if (io.prev && io.gamma != 0.0) {
        const double g = io.gamma * io.prev[idx];
        v = v + g;
    }
    return v;
}

template <bool WT>
__device__ __forceinline__ void store_out(double *p, double v);

// One weighted sum at one element: the flush of this power (AccFlags f)
// adds w2*y_{k-2} (value y2), w1*y_{k-1} (the input row) and w0*y_k (v), as
// flagged and in that order, each product rounded and then added without
// contraction; the sum's first term starts it.
template <bool WT>
__device__ __forceinline__ void accumulate(double *acc, int f, double w2, double w1, double w0,
                                           double y2, const PowerIO &io, double v, size_t idx) {
    if (!f) return;
    double r = 0.0;
    if (!(f & kAccZero)) {
        bool have = !(f & kAccStart);
        if (have) r = acc[idx];
        if (f & kAccT2) {
            const double t = w2 * y2;
            r = have ? r + t : t;
            have = true;
        }
        if (f & kAccT1) {
            const double t = w1 * io.in[idx];
            r = have ? r + t : t;
            have = true;
        }
        if (f & kAccT0) {
            const double t = w0 * v;
            r = have ? r + t : t;
        }
    }
    store_out<WT>(acc + idx, r);
}

// Result of one (row, right-hand side): y_k from the row sum, stored, and
// the weighted sums updated.  The sums' loads and stores use the same
// element index as y_k, so each is touched by this thread only.
template <bool WT, bool ACC>
__device__ __forceinline__ void finish(const PowerIO &io, double s, size_t idx);

// Output store.  WT: an agent-scope atomic store, which writes through to
// memory (it must be coherent with agent-scope loads on every XCD), so a
// result is visible device-wide once the store has completed (vmcnt) and no
// L2 write-back is needed before publishing it; otherwise a plain store.
template <bool WT>
__device__ __forceinline__ void store_out(double *p, double v) {
    if (WT)
        __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    else
        *p = v;
}

template <bool WT, bool ACC>
__device__ __forceinline__ void finish(const PowerIO &io, double s, size_t idx) {
    if (!ACC) {
        store_out<WT>(io.out + idx, epilogue(io, s, idx));
        return;
    }
    // y_{k-2} is read once, for the recurrence and for the sums, and before
    // y_k is stored: in the two-vector ring both share this element
    const bool g = io.recur && io.prev && io.gamma != 0.0;
    const bool need2 = g || ((io.fa | io.fb) & kAccT2);
    const double y2 = need2 ? io.prev[idx] : 0.0;
    double v = s;
    if (io.recur) {
        v = io.alpha * s;
        if (io.beta != 0.0) {
            const double b = io.beta * io.in[idx];
            v = v + b;
        }
        if (g) {
            const double t = io.gamma * y2;
            v = v + t;
        }
    }
    store_out<WT>(io.out + idx, v);
    accumulate<WT>(io.acc_a, io.fa, io.wa2, io.wa1, io.wa0, y2, io, v, idx);
    accumulate<WT>(io.acc_b, io.fb, io.wb2, io.wb1, io.wb0, y2, io, v, idx);
}

// Loads of a slice with 1 <= nz nonzeros starting at nb, rows [rb, re):
// column and value of product q = tid + j*kBlock (nonzero q / R, right-hand
// side q % R) and the end of this thread's row.  Lanes past the end load a
// valid entry (clamped) whose product is never read, so all loads are
// unconditional.
template <typename V, int RC, int KP>
__device__ __forceinline__ void load_cols(const DevMatrix &m, int R, int32_t nb, int32_t nz,
                                          int32_t (&c)[KP]) {
    const int tid = threadIdx.x;
    const int last = nz - 1;
#pragma unroll
    for (int j = 0; j < KP; ++j) {
        const int q = tid + j * kBlock;
        c[j] = m.col[nb + min(RC ? q / RC : q / R, last)];
    }
}
template <typename V, int RC, int KP>
__device__ __forceinline__ void load_vals(const DevMatrix &m, int R, int32_t nb, int32_t nz,
                                          double (&a)[KP]) {
    const int tid = threadIdx.x;
    const V *val = static_cast<const V *>(m.val);
    const int last = nz - 1;
#pragma unroll
    for (int j = 0; j < KP; ++j) {
        const int q = tid + j * kBlock;
        a[j] = static_cast<double>(val[nb + min(RC ? q / RC : q / R, last)]);
    }
}
__device__ __forceinline__ int32_t load_row_end(const DevMatrix &m, int32_t nb, int32_t rb,
                                                int32_t re) {
    const int32_t i = rb + (int32_t)threadIdx.x + 1;
    return i <= re ? m.rowptr[i] : nb;
}

// Sum prod[e*R + rr] for e in [s0, s1) left to right from 0.0; the LDS
// reads are issued eight at a time ahead of the (ordered) additions.
__device__ __forceinline__ double ordered_sum(const double *prod, int R, int rr, int32_t s0,
                                              int32_t s1) {
    double s = 0.0;
    int32_t e = s0;
    for (; e + 8 <= s1; e += 8) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = prod[(e + u) * R + rr];
#pragma unroll
        for (int u = 0; u < 8; ++u) s = s + v[u];
    }
    for (; e < s1; ++e) s = s + prod[e * R + rr];
    return s;
}

// LDS of the row routine: two product buffers and two row-offset buffers.
template <int KP>
struct RowSmem {
    double prod[2][KP * kBlock];
    int32_t srp[2][kBlock + 1];
};

// One row longer than a slice buffer: summed buffer by buffer, one thread
// per right-hand side.  Starts and ends with a barrier.
template <typename V, int RC, int KP, bool WT, bool ACC>
__device__ void long_row(const DevMatrix &m, const PowerIO &io, int R, int32_t row, int32_t nb,
                         int32_t ne, RowSmem<KP> &sm) {
    const int tid = threadIdx.x;
    const int E = (KP * kBlock) / R;
    double s = 0.0;
    for (int32_t b = nb; b < ne; b += E) {
        const int32_t nz = min(E, ne - b);
        int32_t c[KP];
        double a[KP];
        load_cols<V, RC, KP>(m, R, b, nz, c);
        load_vals<V, RC, KP>(m, R, b, nz, a);
        __syncthreads();
#pragma unroll
        for (int j = 0; j < KP; ++j) {
            const int q = tid + j * kBlock;
            const int rr = q - (RC ? q / RC : q / R) * R;
            sm.prod[0][q] = a[j] * io.in[(size_t)c[j] * R + rr];
        }
        __syncthreads();
        if (tid < R)
            for (int32_t e = 0; e < nz; ++e) s = s + sm.prod[0][e * R + tid];
    }
    if (tid < R) {
        const int32_t o = m.out_row ? m.out_row[row] : row;
        const size_t idx = (size_t)o * R + tid;
        finish<WT, ACC>(io, s, idx);
    }
    __syncthreads();
}

// Rows [r0, r1) of one power with one thread per (row, right-hand side): the
// thread sums its row in stored order from 0.0 (the same order as the
// slices), the R threads of a row share each column / value load and read
// the R entries of an input row together.  Used for R >= 4, where a row's
// R entries already fill a coalesced access; no LDS, no barrier.
template <typename V, int RC, bool WT, bool ACC>
__device__ void run_rows(const DevMatrix &m, const PowerIO &io, int R_rt, int32_t r0,
                         int32_t r1) {
    const int R = RC ? RC : R_rt;
    const int rows_per_step = kBlock / R;
    const int tid = threadIdx.x;
    const int rr = tid % R;
    const int li = tid / R;
    const V *val = static_cast<const V *>(m.val);
    if (li >= rows_per_step) return;  // idle lanes when R does not divide the block
    for (int32_t row = r0 + li; row < r1; row += rows_per_step) {
        const int32_t e0 = m.rowptr[row], e1 = m.rowptr[row + 1];
        double s = 0.0;
        // blocks of 8 nonzeros, the last one masked: all loads of a block are
        // issued before its products (lanes past the row end load its last
        // entry again and add nothing)
        for (int32_t e = e0; e < e1; e += 8) {
            int32_t c[8];
            double a[8], xv[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int32_t q = min(e + u, e1 - 1);
                c[u] = m.col[q];
                a[u] = static_cast<double>(val[q]);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) xv[u] = io.in[(size_t)c[u] * R + rr];
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (e + u < e1) s = s + a[u] * xv[u];
        }
        const int32_t o = m.out_row ? m.out_row[row] : row;
        const size_t idx = (size_t)o * R + rr;
        finish<WT, ACC>(io, s, idx);
    }
}

// Rows [r0, r1) of one power in the sliced layout: one thread per (row,
// right-hand side) sums its row sequentially in stored order from 0.0, U
// slots at a time (the loads of a group are issued before its products; a
// slot past the row end reloads the row's last entry and adds nothing).  The
// 64 rows of a slice read each slot with one coalesced access, and the R
// threads of a row share it.  No LDS, no barrier: idle lanes (R not dividing
// the block) just skip.  U slots per group: fewer loads in flight per thread
// queue less in the memory system, more save round trips; the best width
// differs between the kernels (measured on 27-point rows and on 7-point rows
// with 8 right-hand sides; 6, 8 and 16 were slower everywhere):
// * the persistent level-blocked kernels, whose tasks wait on each other:
//   U = 4;
// * the one-launch-per-power baseline: U = 2 for one right-hand side (3.4%
//   faster than 4 on the 27-point stencil), U = 4 for more (2 and 3 were
//   13% and 6% slower with 8 right-hand sides).
template <int RC>
struct SellU {
    static constexpr int value = 4;
};
template <int RC>
struct SpmvSellU {
    static constexpr int value = RC == 1 ? 2 : 4;
};
constexpr int64_t kSpmvSellGrid = 4096;   // baseline workgroups per power (sliced layout)
// DEL: the columns come from the 16-bit offsets (col = row + offset, wrapped
// into [0, n)).  NT: the matrix is loaded non-temporally: by the one-launch-
// per-power baseline with one right-hand side, which reads each line once per
// launch (1.5% faster on the 27-point stencil; with 8 or 16 right-hand sides
// the rows of neighbouring waves share the lines, and the hint made it 5-28%
// slower), and by the level-blocked tasks of a segment's last power only
// (their reuse is the matrix kept in the caches between powers: the hint on
// every power made them 28% slower).
template <bool NT, typename T>
__device__ __forceinline__ T load_matrix(const T *p) {
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}
template <typename V, int RC, bool WT, bool ACC, int U, bool DEL, bool NT>
__device__ __forceinline__ void run_sell_cols(const DevMatrix &m, const PowerIO &io, int R_rt,
                                              int32_t r0, int32_t r1) {
    const int R = RC ? RC : R_rt;
    const int rows_per_step = kBlock / R;
    const int tid = threadIdx.x;
    const int li = tid / R;
    const int rr = tid - li * R;
    if (li >= rows_per_step) return;
    const V *sval = static_cast<const V *>(m.sval);
    for (int32_t row = r0 + li; row < r1; row += rows_per_step) {
        const int32_t L = m.rlen[row];
        const int64_t base = m.soff[row / kSellRows] + row % kSellRows;
        double s = 0.0;
        for (int32_t j = 0; j < L; j += U) {
            int32_t c[U];
            double a[U], xv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t q = base + (int64_t)min(j + u, L - 1) * kSellRows;
                if constexpr (DEL) {  // row + offset, wrapped into [0, n)
                    int32_t cc = row + (int32_t)load_matrix<NT>(m.sdel + q);
                    cc += cc < 0 ? m.n : 0;
                    c[u] = cc >= m.n ? cc - m.n : cc;
                } else
                    c[u] = load_matrix<NT>(m.scol + q);
                a[u] = static_cast<double>(load_matrix<NT>(sval + q));
            }
#pragma unroll
            for (int u = 0; u < U; ++u) xv[u] = io.in[(size_t)c[u] * R + rr];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (j + u < L) s = s + a[u] * xv[u];
        }
        const int32_t o = m.out_row ? m.out_row[row] : row;
        finish<WT, ACC>(io, s, (size_t)o * R + rr);
    }
}
template <typename V, int RC, bool WT, bool ACC, int U, bool NT = false>
__device__ __forceinline__ void run_sell(const DevMatrix &m, const PowerIO &io, int R_rt,
                                         int32_t r0, int32_t r1) {
    if (m.sdel)  // uniform: the plan's layout
        run_sell_cols<V, RC, WT, ACC, U, true, NT>(m, io, R_rt, r0, r1);
    else
        run_sell_cols<V, RC, WT, ACC, U, false, NT>(m, io, R_rt, r0, r1);
}

// Products staged per thread and buffer: the slice path for R < 4 (R = 0 is
// the generic instantiation, which takes either path at run time).
template <int RC, int KP>
struct Staging {
    static constexpr int value = (RC >= 4) ? 1 : KP;
};

// Slices [s0, s1) of one power.  Called by all threads of the workgroup;
// all control flow depends on uniform values only.  Ends with a barrier, so
// the caller may reuse the LDS right away.  Slices holding one row longer
// than a buffer are computed in a second pass.
template <typename V, int RC, int KP, bool WT, bool ACC>
__device__ void run_slices(const DevMatrix &m, const PowerIO &io, int R_rt, DevSlices sl,
                           int32_t s0, int32_t s1, RowSmem<KP> &sm) {
    const int R = RC ? RC : R_rt;
    if (R >= 4) {
        run_rows<V, RC, WT, ACC>(m, io, R, sl.srow[s0], sl.srow[s1]);
        __syncthreads();
        return;
    }
    const int E = (KP * kBlock) / R;  // nonzeros per slice buffer
    const int tid = threadIdx.x;
    int32_t c[KP];    // columns of the slice being processed (then of the next)
    double a[KP];     // its values
    int32_t rp = 0;   // its row end for this thread
    bool have = false;  // c / a / rp hold the loads of slice s
    int buf = 0;
    for (int32_t s = s0; s < s1; ++s) {
        const int32_t rb = sl.srow[s], re = sl.srow[s + 1];
        const int32_t nb = sl.snz[s], ne = sl.snz[s + 1];
        const int32_t nz = ne - nb;
        if (nz > E) {  // a single long row: done after this loop
            have = false;
            continue;
        }
        if (!have && nz > 0) {
            load_cols<V, RC, KP>(m, R, nb, nz, c);
            load_vals<V, RC, KP>(m, R, nb, nz, a);
            rp = load_row_end(m, nb, rb, re);
        }
        double xv[KP];
        if (nz > 0) {
#pragma unroll
            for (int j = 0; j < KP; ++j) {
                const int q = tid + j * kBlock;
                const int rr = q - (RC ? q / RC : q / R) * R;
                xv[j] = io.in[(size_t)c[j] * R + rr];
            }
        }
        const int32_t myrp = nz > 0 ? rp : nb;
        // issue the next slice's loads before this slice's products are formed
        double a2[KP];
        have = false;
        if (s + 1 < s1) {
            const int32_t rb2 = sl.srow[s + 1], re2 = sl.srow[s + 2];
            const int32_t nb2 = sl.snz[s + 1], nz2 = sl.snz[s + 2] - nb2;
            if (nz2 > 0 && nz2 <= E) {
                load_cols<V, RC, KP>(m, R, nb2, nz2, c);
                load_vals<V, RC, KP>(m, R, nb2, nz2, a2);
                rp = load_row_end(m, nb2, rb2, re2);
                have = true;
            }
        }
        double *prod = sm.prod[buf];
        int32_t *srp = sm.srp[buf];
        if (nz > 0) {
#pragma unroll
            for (int j = 0; j < KP; ++j) prod[tid + j * kBlock] = a[j] * xv[j];
        }
        if (have) {
#pragma unroll
            for (int j = 0; j < KP; ++j) a[j] = a2[j];
        }
        srp[tid + 1] = myrp - nb;
        if (tid == 0) srp[0] = 0;
        __syncthreads();
        const int32_t cnt = re - rb;
        const int npairs = cnt * R;
        for (int q = tid; q < npairs; q += kBlock) {
            const int li = RC ? q / RC : q / R;
            const int rr = q - li * R;
            const int32_t row = rb + li;
            const double sum = ordered_sum(prod, R, rr, srp[li], srp[li + 1]);
            const int32_t o = m.out_row ? m.out_row[row] : row;
            const size_t idx = (size_t)o * R + rr;
            finish<WT, ACC>(io, sum, idx);
        }
        buf ^= 1;
    }
    __syncthreads();
    // rows longer than a buffer, kept out of the pipelined loop (registers)
    for (int32_t s = s0; s < s1; ++s) {
        const int32_t nb = sl.snz[s], ne = sl.snz[s + 1];
        if (ne - nb > E) long_row<V, RC, KP, WT, ACC>(m, io, R, sl.srow[s], nb, ne, sm);
    }
}

// Inputs and outputs of the segment's power k.  ACC: the sequence is kept in
// a ring of two vectors (power g = k0 + k in slot (g-1) mod 2) and the
// weighted sums are updated.
template <bool ACC>
__device__ __forceinline__ PowerIO power_io(const SegArgs &a, const Coefs &cf,
                                            const AccCoefs *ac, int32_t k, int32_t n) {
    const size_t stride = (size_t)n * a.R;
    PowerIO io;
    if (ACC) {
        const int32_t g = a.k0 + k;
        io.in = (k == 1) ? a.in0 : a.Y + (size_t)((g - 2) & 1) * stride;
        io.prev = (k == 1) ? a.inm1 : (k == 2 ? a.in0 : a.Y + (size_t)((g - 3) & 1) * stride);
        io.out = a.Y + (size_t)((g - 1) & 1) * stride;
        io.acc_a = a.acc_a;
        io.acc_b = a.acc_b;
        io.wa2 = ac->wa[k - 1];  // weights of the sequence's powers g-2, g-1, g
        io.wa1 = ac->wa[k];
        io.wa0 = ac->wa[k + 1];
        io.wb2 = ac->wb[k - 1];
        io.wb1 = ac->wb[k];
        io.wb0 = ac->wb[k + 1];
        io.fa = ac->fa[k - 1];
        io.fb = ac->fb[k - 1];
    } else {
        io.in = (k == 1) ? a.in0 : a.Y + (size_t)(k - 2) * stride;
        io.prev = (k == 1) ? a.inm1 : (k == 2 ? a.in0 : a.Y + (size_t)(k - 3) * stride);
        io.out = a.Y + (size_t)(k - 1) * stride;
    }
    io.recur = a.recur;
    io.alpha = cf.alpha[k - 1];
    io.beta = cf.beta[k - 1];
    io.gamma = cf.gamma[k - 1];
    return io;
}

// ------------------------------------------------------------------ baseline

// One power: workgroup b walks slices [b*per, min((b+1)*per, n_slices)).
template <typename V, int RC, bool ACC>
__global__ __launch_bounds__(kBlock, 2) void spmv_power_kernel(DevMatrix m, PowerIO io, int32_t R,
                                                           DevSlices sl, int32_t n_slices,
                                                           int32_t per) {
    __shared__ RowSmem<Staging<RC, kSpmvKP>::value> sm;
    const int32_t s0 = blockIdx.x * per;
    const int32_t s1 = min(n_slices, s0 + per);
    run_slices<V, RC, Staging<RC, kSpmvKP>::value, false, ACC>(m, io, R, sl, s0, s1, sm);
}

// One power in the sliced layout: workgroup b walks row blocks b, b + grid,
// ... of 256/R rows each.
template <typename V, int RC, bool ACC>
__global__ __launch_bounds__(kBlock) void spmv_sell_kernel(DevMatrix m, PowerIO io, int32_t R) {
    const int32_t step = kBlock / (RC ? RC : R);
    for (int32_t r0 = blockIdx.x * step; r0 < m.n; r0 += gridDim.x * step)
        run_sell<V, RC, false, ACC, SpmvSellU<RC>::value, RC == 1>(m, io, R, r0,
                                                                   min(m.n, r0 + step));
}

// ------------------------------------------------------------------ level-blocked

// One diagonal of the STEPS schedule: workgroup b computes task tasks[b] =
// (chunk c, power k).  All tasks of a diagonal are independent; the previous
// diagonals' results are visible because they ran in earlier launches.
// Chunk c of one power: its slices staged through LDS, or (SELL) its rows in
// the sliced layout.  WT: write-through result stores.
// last: the segment's last power, whose matrix reads are the chunk's last use
// in this launch (sliced layout, one right-hand side: loaded non-temporally,
// so that the caches keep the rows still to be reused: 1.4% faster on the
// 27-point stencil; with 16 right-hand sides, whose rows share lines across
// waves, 2-3% slower, so not there).
template <typename V, int RC, bool WT, bool ACC, bool SELL>
__device__ __forceinline__ void run_chunk(const DevMatrix &m, const PowerIO &io, int R,
                                          DevSlices sl, const int32_t *chunk_sptr,
                                          const int32_t *chunk_row, int32_t c,
                                          bool last = false) {
    if constexpr (SELL) {
        if (RC == 1 && last)   // uniform: the task's power
            run_sell<V, RC, WT, ACC, SellU<RC>::value, RC == 1>(m, io, R, chunk_row[c],
                                                                chunk_row[c + 1]);
        else
            run_sell<V, RC, WT, ACC, SellU<RC>::value>(m, io, R, chunk_row[c], chunk_row[c + 1]);
    } else {
        __shared__ RowSmem<Staging<RC, kTaskKP>::value> sm;
        run_slices<V, RC, Staging<RC, kTaskKP>::value, WT, ACC>(m, io, R, sl, chunk_sptr[c],
                                                                chunk_sptr[c + 1], sm);
    }
}

template <typename V, int RC, bool ACC, bool SELL>
__device__ __forceinline__ void step_body(const DevMatrix &m, DevSlices sl,
                                          const int32_t *chunk_sptr, const int32_t *chunk_row,
                                          const int32_t *tasks, const SegArgs &a, const Coefs &cf,
                                          const AccCoefs *ac) {
    const int32_t c = tasks[2 * blockIdx.x];
    const int32_t k = tasks[2 * blockIdx.x + 1];
    run_chunk<V, RC, false, ACC, SELL>(m, power_io<ACC>(a, cf, ac, k, m.n), a.R, sl, chunk_sptr,
                                       chunk_row, c);
}

template <typename V, int RC>
__global__ __launch_bounds__(kBlock, kTaskWaves) void step_kernel(DevMatrix m, DevSlices sl,
                                                     const int32_t *chunk_sptr,
                                                     const int32_t *chunk_row,
                                                     const int32_t *tasks, SegArgs a, Coefs cf) {
    step_body<V, RC, false, false>(m, sl, chunk_sptr, chunk_row, tasks, a, cf, nullptr);
}

// The same with weighted sums (a separate kernel, so that the plain one
// carries no trace of them).
template <typename V, int RC>
__global__ __launch_bounds__(kBlock, kTaskWaves) void step_acc_kernel(DevMatrix m, DevSlices sl,
                                                         const int32_t *chunk_sptr,
                                                         const int32_t *chunk_row,
                                                         const int32_t *tasks, SegArgs a,
                                                         Coefs cf, AccCoefs ac) {
    step_body<V, RC, true, false>(m, sl, chunk_sptr, chunk_row, tasks, a, cf, &ac);
}

// Sliced-layout forms (no LDS, so more workgroups fit a compute unit).
template <typename V, int RC>
__global__ __launch_bounds__(kBlock) void step_sell_kernel(DevMatrix m, DevSlices sl,
                                                           const int32_t *chunk_sptr,
                                                           const int32_t *chunk_row,
                                                           const int32_t *tasks, SegArgs a,
                                                           Coefs cf) {
    step_body<V, RC, false, true>(m, sl, chunk_sptr, chunk_row, tasks, a, cf, nullptr);
}

template <typename V, int RC>
__global__ __launch_bounds__(kBlock) void step_sell_acc_kernel(DevMatrix m, DevSlices sl,
                                                               const int32_t *chunk_sptr,
                                                               const int32_t *chunk_row,
                                                               const int32_t *tasks, SegArgs a,
                                                               Coefs cf, AccCoefs ac) {
    step_body<V, RC, true, true>(m, sl, chunk_sptr, chunk_row, tasks, a, cf, &ac);
}

struct LBParams {
    DevMatrix m;
    DevSchedule s;
    DevWorkspace ws;
    SegArgs a;
    int64_t spin_limit;   // wall-clock ticks
    int32_t pending;      // skip-ahead slots (lbs_kernel)
    int32_t acquire;      // invalidate caches before a task reads its inputs
    int32_t stride;       // > 0: workgroup b takes tasks b, b + stride, ...
                          // (every workgroup resident); 0: a shared counter
};

// One non-blocking look at task t's inputs by wavefront 0 (all 64 lanes):
// true when every chunk it reads has completed the previous power.
__device__ __forceinline__ bool inputs_ready(const LBParams &P, int32_t t) {
    const int32_t c = P.s.tasks[2 * t];
    const int32_t k = P.s.tasks[2 * t + 1];
    if (k == 1) return true;
    const int32_t lo = P.s.dep_lo[c], hi = P.s.dep_hi[c];
    int ready = 1;
    for (int32_t j = lo + (int)threadIdx.x; j <= hi; j += kWave)
        ready &= ld_relaxed(P.ws.done + j) >= k - 1;
    return __all(ready);
}

// Persistent kernel: workgroups take tasks (chunk c, power k) in schedule
// order, either from a shared ticket counter or, with P.stride = the number
// of workgroups, statically: workgroup b takes tickets b, b + stride, ...
// Before computing, a task waits until every chunk in [dep_lo[c], dep_hi[c]]
// has completed power k-1 and then invalidates its caches (acquire) where
// needed; it computes with write-through stores and publishes done[c] = k
// once they have completed.  Dependencies always carry smaller tickets and a
// workgroup takes its tickets in increasing order, one at a time, so the
// holder of the smallest unfinished ticket can always proceed: with the
// counter, tickets go only to running workgroups; with the static order,
// only if every workgroup of the launch is resident, which the host ensures
// (the grid fits the device and no other launch of a static or XCD-queue
// kernel overlaps it).  The static order spares each task a round trip to a
// counter that every workgroup of the device contends for, measured as the
// larger part of a task's cost on matrices whose windows fit the caches.
// Every wait is also bounded by spin_limit, after which the run is flagged
// as failed and all workgroups leave.
template <typename V, int RC, bool ACC, bool SELL>
__device__ __forceinline__ void lb_body(const LBParams &P, const Coefs &cf, const AccCoefs *ac) {
    __shared__ int32_t s_ticket;
    __shared__ int s_ok;
    const int tid = threadIdx.x;
    if (tid == 0)
        s_ticket = P.stride ? (int32_t)blockIdx.x
                            : __hip_atomic_fetch_add(P.ws.ticket, 1, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    // All loop control below is made provably uniform (readfirstlane) and the
    // loop has a single exit: a loop whose exit the compiler considers
    // divergent may be restructured so that lanes leave it at different
    // iterations, which would break the barriers inside it.
    int32_t t = __builtin_amdgcn_readfirstlane(s_ticket);
    while (t < P.s.n_tasks) {
        const int32_t c = P.s.tasks[2 * t];
        const int32_t k = P.s.tasks[2 * t + 1];
        int ok = 1;
        if (k > 1) {
            // Wavefront 0 alone polls the dependency flags, 64 per coalesced
            // load, and sleeps between rounds; the other waves wait at the
            // barrier.  (Polling from every thread floods the memory system
            // with coherent loads and slows the producers down.)
            if (tid < kWave) {
                const int32_t lo = P.s.dep_lo[c], hi = P.s.dep_hi[c];
                uint64_t t0 = 0;
                for (int round = 0;; ++round) {
                    int ready = 1;
                    for (int32_t j = lo + tid; j <= hi; j += kWave)
                        ready &= ld_relaxed(P.ws.done + j) >= k - 1;
                    if (__all(ready)) break;
                    if (round == 0) t0 = wall_clock64();
                    if (ld_relaxed(P.ws.err) != 0 ||
                        (int64_t)(wall_clock64() - t0) > P.spin_limit) {
                        ok = 0;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
                if (tid == 0) s_ok = ok;
            }
            __syncthreads();
            ok = __builtin_amdgcn_readfirstlane(s_ok);
            // The producers' rows are visible to every wave of this
            // workgroup.  With a line-closed schedule no cache holds a copy
            // of any line they wrote (nobody read it before it was
            // complete), so the loads below miss down to the level their
            // write-through stores reached, and the caches stay warm; else
            // this XCD's caches are invalidated first.
            if (P.acquire)
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            else
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        }
        if (!ok) break;  // uniform: a wait hit its limit, the run is abandoned
        run_chunk<V, RC, true, ACC, SELL>(P.m, power_io<ACC>(P.a, cf, ac, k, P.m.n), P.a.R,
                                          P.s.sl, P.s.chunk_sptr, P.s.chunk_row, c, k == P.a.p);
        // The results were stored write-through; every wave waits until its
        // stores have completed (vmcnt = 0) before the barrier, so the chunk
        // is visible device-wide when the flag below is published and the
        // next ticket is taken.  No L2 write-back is needed.  (Taking the
        // next ticket before computing, to overlap its round trip, was
        // measured slower: it doubles the tickets in flight, and tasks then
        // wait more often on inputs that are still being computed.)
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0), other counters untouched
        __syncthreads();
        if (tid == 0) {
            __hip_atomic_store(P.ws.done + c, k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_ticket = P.stride ? t + P.stride
                                : __hip_atomic_fetch_add(P.ws.ticket, 1, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        t = __builtin_amdgcn_readfirstlane(s_ticket);
    }
    if (t < P.s.n_tasks && tid == 0) record_failure(P.ws);
}

template <typename V, int RC>
__global__ __launch_bounds__(kBlock, kTaskWaves) void lb_kernel(LBParams P, Coefs cf) {
    lb_body<V, RC, false, false>(P, cf, nullptr);
}

template <typename V, int RC>
__global__ __launch_bounds__(kBlock, kTaskWaves) void lb_acc_kernel(LBParams P, Coefs cf,
                                                                    AccCoefs ac) {
    lb_body<V, RC, true, false>(P, cf, &ac);
}

// Sliced-layout forms: no LDS, built for up to kSellWaves workgroups per
// compute unit.
constexpr int kSellWaves = 8;
template <typename V, int RC>
__global__ __launch_bounds__(kBlock, kSellWaves) void lb_sell_kernel(LBParams P, Coefs cf) {
    lb_body<V, RC, false, true>(P, cf, nullptr);
}

template <typename V, int RC>
__global__ __launch_bounds__(kBlock, kSellWaves) void lb_sell_acc_kernel(LBParams P, Coefs cf,
                                                                         AccCoefs ac) {
    lb_body<V, RC, true, true>(P, cf, &ac);
}

constexpr int kMaxPending = 8;

// Persistent kernel with skip-ahead: when the inputs of a workgroup's task
// are not ready, the task is parked in a small list (up to P.pending slots)
// and the workgroup takes the next ticket instead of waiting.  Parked tasks
// are retried oldest first before any new ticket; a workgroup whose list is
// full, or that has no tickets left, waits for its oldest parked task.
// Deadlock freedom: the smallest unfinished ticket has all its inputs done
// (they carry smaller tickets), and its holder, for which it is the oldest
// task held, either runs it when retrying or blocks on it; every wait is
// bounded by spin_limit as in lb_kernel.  Wavefront 0 makes every choice and
// the other wavefronts learn it through LDS, so control stays uniform.
template <typename V, int RC, bool ACC>
__device__ __forceinline__ void lbs_body(const LBParams &P, const Coefs &cf, const AccCoefs *ac) {
    __shared__ RowSmem<Staging<RC, kTaskKP>::value> sm;
    __shared__ int32_t s_task;
    const int tid = threadIdx.x;
    const int lim = min(P.pending, kMaxPending);
    int32_t pend[kMaxPending];  // wavefront 0 only: parked tickets, oldest first
    int npend = 0;
    bool exhausted = false;
    bool failed = false;        // a wait hit its limit (reported after the loop)
    for (;;) {
        if (tid < kWave) {
            int32_t chosen = -1;
            // 1. parked tasks, oldest first
            for (int i = 0; i < npend && chosen < 0; ++i) {
                if (inputs_ready(P, pend[i])) {
                    chosen = pend[i];
                    for (int j = i + 1; j < npend; ++j) pend[j - 1] = pend[j];
                    --npend;
                }
            }
            // 2. new tickets while there is room to park
            while (chosen < 0 && !exhausted && npend < lim) {
                int32_t t = 0;
                if (tid == 0)
                    t = __hip_atomic_fetch_add(P.ws.ticket, 1, __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                t = __shfl(t, 0);
                if (t >= P.s.n_tasks)
                    exhausted = true;
                else if (inputs_ready(P, t))
                    chosen = t;
                else
                    pend[npend++] = t;
            }
            // 3. wait for the oldest parked task
            if (chosen < 0 && npend > 0) {
                uint64_t t0 = wall_clock64();
                bool ok = true;
                while (!inputs_ready(P, pend[0])) {
                    if (ld_relaxed(P.ws.err) != 0 ||
                        (int64_t)(wall_clock64() - t0) > P.spin_limit) {
                        ok = false;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
                if (ok) {
                    chosen = pend[0];
                    for (int j = 1; j < npend; ++j) pend[j - 1] = pend[j];
                    --npend;
                } else {
                    failed = true;
                    chosen = -1;
                    npend = 0;
                    exhausted = true;
                }
            }
            if (tid == 0) s_task = chosen;
        }
        __syncthreads();
        const int32_t t = __builtin_amdgcn_readfirstlane(s_task);
        if (t < 0) break;  // uniform: no work left (or a wait failed)
        if (P.acquire)  // as in lb_body
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        else
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        const int32_t c = P.s.tasks[2 * t];
        const int32_t k = P.s.tasks[2 * t + 1];
        run_slices<V, RC, Staging<RC, kTaskKP>::value, true, ACC>(
            P.m, power_io<ACC>(P.a, cf, ac, k, P.m.n), P.a.R, P.s.sl, P.s.chunk_sptr[c],
            P.s.chunk_sptr[c + 1], sm);
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): write-through results completed
        __syncthreads();
        if (tid == 0)
            __hip_atomic_store(P.ws.done + c, k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (failed && tid == 0) record_failure(P.ws);
}

template <typename V, int RC>
__global__ __launch_bounds__(kBlock, kTaskWaves) void lbs_kernel(LBParams P, Coefs cf) {
    lbs_body<V, RC, false>(P, cf, nullptr);
}

template <typename V, int RC>
__global__ __launch_bounds__(kBlock, kTaskWaves) void lbs_acc_kernel(LBParams P, Coefs cf,
                                                                     AccCoefs ac) {
    lbs_body<V, RC, true>(P, cf, &ac);
}

// XCD this wave runs on: hardware register XCC_ID (20), bits [3:0].
__device__ __forceinline__ int xcc_id() {
    return (int)(__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 0xF);
}

struct XcdParams {
    DevMatrix m;
    DevXcdSchedule s;
    DevWorkspace ws;
    SegArgs a;
    int64_t spin_limit;   // wall-clock ticks
    int32_t acquire;      // invalidate caches before a task reads its inputs
};

// Kernel arguments stay well inside the 4 KiB argument segment.
static_assert(sizeof(LBParams) + sizeof(Coefs) + sizeof(AccCoefs) <= 3584,
              "level-blocked kernel arguments");
static_assert(sizeof(XcdParams) + sizeof(Coefs) + sizeof(AccCoefs) <= 3584,
              "XCD kernel arguments");

// Persistent kernel of the XCD schedule.  Queue q holds the tasks of the
// chunks owned by XCD q, in the global dependency order the queues were cut
// from; a workgroup serves the queue of the XCD it runs on (read from the
// hardware, so the binding holds whatever the dispatcher does) and takes its
// tickets in order.  Dependencies are exact chunk lists; results are
// published as in lb_kernel.  Progress: the earliest unfinished task of the
// global order has every earlier task of its queue finished, so it is the
// next ticket of its queue or held by a workgroup, and its inputs are done;
// it runs as soon as one workgroup of this launch runs on its XCD.  That
// holds while nothing else stops this launch's workgroups from ever being
// placed on an XCD: the library never lets two launches of this kernel run
// at the same time on one device (two such launches could each fill the
// XCDs the other one's queues need, and wait for each other), and any other
// kernel finishes on its own.  Waits are bounded by spin_limit in any case.
template <typename V, int RC, bool ACC, bool SELL>
__device__ __forceinline__ void xcd_body(const XcdParams &P, const Coefs &cf, const AccCoefs *ac) {
    __shared__ int32_t s_ticket;
    __shared__ int s_ok;
    const int tid = threadIdx.x;
    const int q = P.s.n_queues == 1 ? 0 : __builtin_amdgcn_readfirstlane(xcc_id());
    if (q >= P.s.n_queues) return;  // uniform: no queue for this XCD
    const int32_t q0 = P.s.qptr[q];
    const int32_t qn = P.s.qptr[q + 1] - q0;
    int32_t *ticket = P.ws.ticket + q;
    if (tid == 0)
        s_ticket = __hip_atomic_fetch_add(ticket, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    int32_t t = __builtin_amdgcn_readfirstlane(s_ticket);
    while (t < qn) {
        const int32_t c = P.s.tasks[2 * (q0 + t)];
        const int32_t k = P.s.tasks[2 * (q0 + t) + 1];
        int ok = 1;
        if (k > 1) {
            if (tid < kWave) {
                const int32_t lo = P.s.dep_ptr[c], hi = P.s.dep_ptr[c + 1];
                uint64_t t0 = 0;
                for (int round = 0;; ++round) {
                    int ready = 1;
                    for (int32_t j = lo + tid; j < hi; j += kWave)
                        ready &= ld_relaxed(P.ws.done + P.s.dep_idx[j]) >= k - 1;
                    if (__all(ready)) break;
                    if (round == 0) t0 = wall_clock64();
                    if (ld_relaxed(P.ws.err) != 0 ||
                        (int64_t)(wall_clock64() - t0) > P.spin_limit) {
                        ok = 0;
                        break;
                    }
                    __builtin_amdgcn_s_sleep(2);
                }
                if (tid == 0) s_ok = ok;
            }
            __syncthreads();
            ok = __builtin_amdgcn_readfirstlane(s_ok);
            if (P.acquire)  // as in lb_body: a line-closed schedule needs no invalidation
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            else
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        }
        if (!ok) break;
        run_chunk<V, RC, true, ACC, SELL>(P.m, power_io<ACC>(P.a, cf, ac, k, P.m.n), P.a.R,
                                          P.s.sl, P.s.chunk_sptr, P.s.chunk_row, c);
        // write-through results, completed (vmcnt = 0) before the barrier
        __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
        __syncthreads();
        if (tid == 0) {
            __hip_atomic_store(P.ws.done + c, k, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_ticket = __hip_atomic_fetch_add(ticket, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
        t = __builtin_amdgcn_readfirstlane(s_ticket);
    }
    if (t < qn && tid == 0) record_failure(P.ws);
}

template <typename V, int RC>
__global__ __launch_bounds__(kBlock, kTaskWaves) void xcd_kernel(XcdParams P, Coefs cf) {
    xcd_body<V, RC, false, false>(P, cf, nullptr);
}

template <typename V, int RC>
__global__ __launch_bounds__(kBlock, kTaskWaves) void xcd_acc_kernel(XcdParams P, Coefs cf,
                                                                     AccCoefs ac) {
    xcd_body<V, RC, true, false>(P, cf, &ac);
}

template <typename V, int RC>
__global__ __launch_bounds__(kBlock, kSellWaves) void xcd_sell_kernel(XcdParams P, Coefs cf) {
    xcd_body<V, RC, false, true>(P, cf, nullptr);
}

template <typename V, int RC>
__global__ __launch_bounds__(kBlock, kSellWaves) void xcd_sell_acc_kernel(XcdParams P, Coefs cf,
                                                                          AccCoefs ac) {
    xcd_body<V, RC, true, true>(P, cf, &ac);
}

__global__ void reset_kernel(DevWorkspace ws, int32_t n_chunks, int clear_status) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_chunks) ws.done[i] = 0;
    if (i < kMaxQueues) ws.ticket[i] = 0;
    if (i == 0) {
        *ws.err = 0;
        if (clear_status && ws.status)
            __hip_atomic_store(ws.status, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

__global__ void status_copy_kernel(int32_t *word, int32_t *out) {
    const int32_t v = __hip_atomic_exchange(word, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(out, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Each workgroup records the XCD it ran on.
__global__ void xcc_probe_kernel(int32_t *out) {
    if (threadIdx.x == 0) out[blockIdx.x] = xcc_id();
}

__global__ void permute_kernel(const int32_t *perm, int64_t n, int to_plan, const double *in,
                               double *out, int nvec, int R) {
    const int64_t total = n * (int64_t)R * nvec;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = g / (n * R);
        const int64_t rem = g - v * n * R;
        const int64_t i = rem / R, r = rem - i * R;
        const int64_t base = v * n * R;
        if (to_plan)
            out[base + i * R + r] = in[base + (int64_t)perm[i] * R + r];
        else
            out[base + (int64_t)perm[i] * R + r] = in[base + i * R + r];
    }
}

// Complex states from the two weighted sums, on column pairs (column 2j the
// real, 2j+1 the imaginary part): with weights wa + i wb and a real matrix
// the real part is a[2j] - b[2j+1] and the imaginary part a[2j+1] + b[2j].
__global__ void combine_complex_kernel(const double *a, const double *b, int64_t pairs,
                                       double *out) {
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < pairs;
         g += (int64_t)gridDim.x * blockDim.x) {
        const double2 va = reinterpret_cast<const double2 *>(a)[g];
        const double2 vb = reinterpret_cast<const double2 *>(b)[g];
        double2 o;
        o.x = va.x - vb.y;
        o.y = va.y + vb.x;
        reinterpret_cast<double2 *>(out)[g] = o;
    }
}

// Load-only bandwidth probe: each workgroup sums its share of the buffer
// `passes` times with 16-byte loads; one double per workgroup is written.
__global__ __launch_bounds__(kBlock) void load_probe_kernel(const double2 *buf, int64_t n2,
                                                            int passes, double *sink) {
    double acc = 0.0;
    const int64_t stride = (int64_t)gridDim.x * kBlock;
    for (int p = 0; p < passes; ++p)
        for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n2; i += stride) {
            const double2 v = buf[i];
            acc += v.x + v.y;
        }
    __shared__ double red[kBlock];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) sink[blockIdx.x] = red[0];
}

// XCD-local variant: the buffer is cut into `regions` equal parts and every
// workgroup reads the part of the XCD it runs on (XCC_ID mod regions), so each
// XCD's L2 sees only its own part.  Workgroups are numbered within an XCD by
// blockIdx / regions (the dispatcher deals workgroups to XCDs round robin);
// were it otherwise, parts would be read unevenly but every load stays inside
// the buffer.  xcc[b] records where workgroup b ran.
__global__ __launch_bounds__(kBlock) void load_probe_local_kernel(const double2 *buf, int64_t n2,
                                                                int regions, int passes,
                                                                double *sink, int32_t *xcc) {
    const int x = __builtin_amdgcn_readfirstlane(xcc_id()) % regions;
    const int64_t per = n2 / regions;
    const double2 *part = buf + (int64_t)x * per;
    const int64_t idx = blockIdx.x / regions;
    const int64_t stride = (int64_t)((gridDim.x + regions - 1) / regions) * kBlock;
    double acc = 0.0;
    for (int p = 0; p < passes; ++p)
        for (int64_t i = idx * kBlock + threadIdx.x; i < per; i += stride) {
            const double2 v = part[i];
            acc += v.x + v.y;
        }
    __shared__ double red[kBlock];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        sink[blockIdx.x] = red[0];
        xcc[blockIdx.x] = xcc_id();
    }
}

// ------------------------------------------------------------------ dispatch

using SpmvFn = void (*)(DevMatrix, PowerIO, int32_t, DevSlices, int32_t, int32_t);
using SpmvSellFn = void (*)(DevMatrix, PowerIO, int32_t);
using LbFn = void (*)(LBParams, Coefs);
using LbAccFn = void (*)(LBParams, Coefs, AccCoefs);
using StepFn = void (*)(DevMatrix, DevSlices, const int32_t *, const int32_t *, const int32_t *,
                        SegArgs, Coefs);
using StepAccFn = void (*)(DevMatrix, DevSlices, const int32_t *, const int32_t *,
                           const int32_t *, SegArgs, Coefs, AccCoefs);
using XcdFn = void (*)(XcdParams, Coefs);
using XcdAccFn = void (*)(XcdParams, Coefs, AccCoefs);

int r_index(int R) {
    switch (R) {
        case 1: return 0;
        case 2: return 1;
        case 4: return 2;
        case 8: return 3;
        case 16: return 4;
    }
    return 5;  // any other count: generic instantiation
}

// Kernels by value type and right-hand-side count: R = 1, 2, 4, 8, 16 are
// specialised, every other count uses the generic instantiation (RC = 0).
template <typename V>
struct VTable {
    SpmvFn spmv[6], spmv_acc[6];
    SpmvSellFn spmv_sell[6], spmv_sell_acc[6];
    LbFn lb[6], lbs[6], lb_sell[6];
    LbAccFn lb_acc[6], lbs_acc[6], lb_sell_acc[6];
    StepFn step[6], step_sell[6];
    StepAccFn step_acc[6], step_sell_acc[6];
    XcdFn xcd[6], xcd_sell[6];
    XcdAccFn xcd_acc[6], xcd_sell_acc[6];
    template <int RC>
    void fill(int i) {
        spmv[i] = spmv_power_kernel<V, RC, false>;
        spmv_acc[i] = spmv_power_kernel<V, RC, true>;
        spmv_sell[i] = spmv_sell_kernel<V, RC, false>;
        spmv_sell_acc[i] = spmv_sell_kernel<V, RC, true>;
        lb[i] = lb_kernel<V, RC>;
        lb_acc[i] = lb_acc_kernel<V, RC>;
        lb_sell[i] = lb_sell_kernel<V, RC>;
        lb_sell_acc[i] = lb_sell_acc_kernel<V, RC>;
        lbs[i] = lbs_kernel<V, RC>;
        lbs_acc[i] = lbs_acc_kernel<V, RC>;
        step[i] = step_kernel<V, RC>;
        step_acc[i] = step_acc_kernel<V, RC>;
        step_sell[i] = step_sell_kernel<V, RC>;
        step_sell_acc[i] = step_sell_acc_kernel<V, RC>;
        xcd[i] = xcd_kernel<V, RC>;
        xcd_acc[i] = xcd_acc_kernel<V, RC>;
        xcd_sell[i] = xcd_sell_kernel<V, RC>;
        xcd_sell_acc[i] = xcd_sell_acc_kernel<V, RC>;
    }
    VTable() {
        fill<1>(0);
        fill<2>(1);
        fill<4>(2);
        fill<8>(3);
        fill<16>(4);
        fill<0>(5);
    }
};

template <typename V>
const VTable<V> &vt() {
    static VTable<V> t;
    return t;
}

const VTable<double> &t64() { return vt<double>(); }
const VTable<float> &t32() { return vt<float>(); }

SpmvFn spmv_fn(int value_bits, int R, bool acc) {
    const int i = r_index(R);
    if (value_bits == 32) return acc ? t32().spmv_acc[i] : t32().spmv[i];
    return acc ? t64().spmv_acc[i] : t64().spmv[i];
}
SpmvSellFn spmv_sell_fn(int value_bits, int R, bool acc) {
    const int i = r_index(R);
    if (value_bits == 32) return acc ? t32().spmv_sell_acc[i] : t32().spmv_sell[i];
    return acc ? t64().spmv_sell_acc[i] : t64().spmv_sell[i];
}
// skip: the skip-ahead kernel (LDS-staged rows); else sell picks the
// sliced-layout kernel
LbFn lb_fn(int value_bits, int R, bool skip, bool sell) {
    const VTable<double> &a = t64();
    const VTable<float> &b = t32();
    const int i = r_index(R);
    if (skip) return value_bits == 32 ? b.lbs[i] : a.lbs[i];
    if (sell) return value_bits == 32 ? b.lb_sell[i] : a.lb_sell[i];
    return value_bits == 32 ? b.lb[i] : a.lb[i];
}
LbAccFn lb_acc_fn(int value_bits, int R, bool skip, bool sell) {
    const VTable<double> &a = t64();
    const VTable<float> &b = t32();
    const int i = r_index(R);
    if (skip) return value_bits == 32 ? b.lbs_acc[i] : a.lbs_acc[i];
    if (sell) return value_bits == 32 ? b.lb_sell_acc[i] : a.lb_sell_acc[i];
    return value_bits == 32 ? b.lb_acc[i] : a.lb_acc[i];
}
StepFn step_fn(int value_bits, int R, bool sell) {
    const int i = r_index(R);
    if (sell) return value_bits == 32 ? t32().step_sell[i] : t64().step_sell[i];
    return value_bits == 32 ? t32().step[i] : t64().step[i];
}
StepAccFn step_acc_fn(int value_bits, int R, bool sell) {
    const int i = r_index(R);
    if (sell) return value_bits == 32 ? t32().step_sell_acc[i] : t64().step_sell_acc[i];
    return value_bits == 32 ? t32().step_acc[i] : t64().step_acc[i];
}
XcdFn xcd_fn(int value_bits, int R, bool sell) {
    const int i = r_index(R);
    if (sell) return value_bits == 32 ? t32().xcd_sell[i] : t64().xcd_sell[i];
    return value_bits == 32 ? t32().xcd[i] : t64().xcd[i];
}
XcdAccFn xcd_acc_fn(int value_bits, int R, bool sell) {
    const int i = r_index(R);
    if (sell) return value_bits == 32 ? t32().xcd_sell_acc[i] : t64().xcd_sell_acc[i];
    return value_bits == 32 ? t32().xcd_acc[i] : t64().xcd_acc[i];
}

}  // namespace

int launch_reset(const DevWorkspace &ws, int32_t n_chunks, void *stream, bool clear_status) {
    const int32_t n = n_chunks > 0 ? n_chunks : 1;
    hipLaunchKernelGGL(reset_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, ws,
                       n_chunks, clear_status ? 1 : 0);
    return (int)hipGetLastError();
}

int scratch_workspace(int device, int32_t **out) {
    constexpr int kDevices = 64;
    static std::mutex mu;
    static int32_t *addr[kDevices] = {};
    if (device < 0 || device >= kDevices) return (int)hipErrorInvalidDevice;
    std::lock_guard<std::mutex> g(mu);
    if (!addr[device]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return (int)e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return (int)e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess) return (int)e;
        if (!p) return (int)hipErrorInvalidSymbol;
        addr[device] = static_cast<int32_t *>(p);
    }
    *out = addr[device];
    return 0;
}

int launch_status_copy(int32_t *status_word, int32_t *out, void *stream) {
    hipLaunchKernelGGL(status_copy_kernel, dim3(1), dim3(1), 0, (hipStream_t)stream, status_word,
                       out);
    return (int)hipGetLastError();
}

int launch_spmv_power(const DevMatrix &m, DevSlices sl, int32_t n_slices, int32_t per,
                      const double *in, const double *inm1, double *out, int32_t R, int recur,
                      double alpha, double beta, double gamma, const AccStep *acc,
                      void *stream) {
    if (R < 1 || R > 16 || per < 1) return (int)hipErrorInvalidValue;
    if (m.n == 0 || n_slices == 0) return 0;
    PowerIO io{in, inm1, out, alpha, beta, gamma, recur};
    io.acc_a = io.acc_b = nullptr;
    io.wa2 = io.wa1 = io.wa0 = io.wb2 = io.wb1 = io.wb0 = 0.0;
    io.fa = io.fb = 0;
    if (acc) {
        io.acc_a = acc->acc_a;
        io.acc_b = acc->acc_b;
        io.wa2 = acc->wa[0];
        io.wa1 = acc->wa[1];
        io.wa0 = acc->wa[2];
        io.wb2 = acc->wb[0];
        io.wb1 = acc->wb[1];
        io.wb0 = acc->wb[2];
        io.fa = acc->fa;
        io.fb = acc->fb;
    }
    if (m.scol) {  // sliced layout: row blocks of 256 / R rows, grid-stride
        const int64_t nblk = ((int64_t)m.n + kBlock / R - 1) / (kBlock / R);
        const int64_t grid = std::min<int64_t>(nblk, kSpmvSellGrid);
        hipLaunchKernelGGL(spmv_sell_fn(m.value_bits, R, acc != nullptr), dim3((unsigned)grid),
                           dim3(kBlock), 0, (hipStream_t)stream, m, io, R);
        return (int)hipGetLastError();
    }
    const int32_t grid = (n_slices + per - 1) / per;
    hipLaunchKernelGGL(spmv_fn(m.value_bits, R, acc != nullptr), dim3((unsigned)grid), dim3(kBlock), 0,
                       (hipStream_t)stream, m, io, R, sl, n_slices, per);
    return (int)hipGetLastError();
}

int launch_step(const DevMatrix &m, DevSlices sl, const int32_t *chunk_sptr,
                const int32_t *chunk_row, const int32_t *tasks, int32_t n_tasks,
                const SegArgs &a, const Coefs *cf, const AccCoefs *acc, void *stream) {
    if (a.R < 1 || a.R > 16 || a.p < 1 || a.p > kMaxSegPowers) return (int)hipErrorInvalidValue;
    if (n_tasks <= 0) return 0;
    Coefs c{};
    if (cf) c = *cf;
    const bool sell = m.scol != nullptr;
    if (acc)
        hipLaunchKernelGGL(step_acc_fn(m.value_bits, a.R, sell), dim3((unsigned)n_tasks),
                           dim3(kBlock), 0, (hipStream_t)stream, m, sl, chunk_sptr, chunk_row,
                           tasks, a, c, *acc);
    else
        hipLaunchKernelGGL(step_fn(m.value_bits, a.R, sell), dim3((unsigned)n_tasks), dim3(kBlock),
                           0, (hipStream_t)stream, m, sl, chunk_sptr, chunk_row, tasks, a, c);
    return (int)hipGetLastError();
}

int lb_resident_workgroups(int value_bits, int R, int device, bool sell, bool acc) {
    const void *fn = acc ? reinterpret_cast<const void *>(lb_acc_fn(value_bits, R, false, sell))
                         : reinterpret_cast<const void *>(lb_fn(value_bits, R, false, sell));
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlock, 0) != hipSuccess)
        return 0;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return 0;
    return per_cu * prop.multiProcessorCount;
}

int lb_max_workgroups(int value_bits, int R, int device, bool sell) {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, reinterpret_cast<const void *>(lb_fn(value_bits, R, false, sell)), kBlock,
            0) != hipSuccess)
        return 0;
    // LDS-staged rows: at most kTaskWaves workgroups per CU even where
    // registers and LDS would allow more (the unstaged path for R >= 4): more
    // persistent workgroups only added ticket and flag traffic and were
    // measured 2-3x slower.  Sliced layout: at most four.
    per_cu = std::min(per_cu, sell ? 4 : kTaskWaves);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return 0;
    return per_cu * prop.multiProcessorCount;
}

int launch_lb(const DevMatrix &m, const DevSchedule &s, const DevWorkspace &ws,
              const SegArgs &a, const Coefs *cf, const AccCoefs *acc, int workgroups,
              int64_t spin_limit, int pending, int acquire, bool static_order, void *stream) {
    if (a.R < 1 || a.R > 16) return (int)hipErrorInvalidValue;
    if (a.p < 1 || a.p > kMaxSegPowers || workgroups < 1) return (int)hipErrorInvalidValue;
    if (pending < 0 || pending > kMaxPending) return (int)hipErrorInvalidValue;
    if (static_order && pending > 0) return (int)hipErrorInvalidValue;
    if (s.n_tasks == 0) return 0;
    LBParams P{m, s, ws, a, spin_limit, pending, acquire ? 1 : 0, static_order ? workgroups : 0};
    Coefs c{};
    if (cf) c = *cf;
    const bool sell = m.scol != nullptr;
    if (acc)
        hipLaunchKernelGGL(lb_acc_fn(m.value_bits, a.R, pending > 0, sell), dim3(workgroups),
                           dim3(kBlock), 0, (hipStream_t)stream, P, c, *acc);
    else
        hipLaunchKernelGGL(lb_fn(m.value_bits, a.R, pending > 0, sell), dim3(workgroups),
                           dim3(kBlock), 0, (hipStream_t)stream, P, c);
    return (int)hipGetLastError();
}

int launch_xcd(const DevMatrix &m, const DevXcdSchedule &s, const DevWorkspace &ws,
               const SegArgs &a, const Coefs *cf, const AccCoefs *acc, int workgroups,
               int64_t spin_limit, int acquire, void *stream) {
    if (a.R < 1 || a.R > 16) return (int)hipErrorInvalidValue;
    if (a.p < 1 || a.p > kMaxSegPowers || workgroups < 1) return (int)hipErrorInvalidValue;
    if (s.n_queues < 1 || s.n_queues > kMaxQueues) return (int)hipErrorInvalidValue;
    if (s.n_chunks == 0) return 0;
    XcdParams P{m, s, ws, a, spin_limit, acquire ? 1 : 0};
    Coefs c{};
    if (cf) c = *cf;
    const bool sell = m.scol != nullptr;
    if (acc)
        hipLaunchKernelGGL(xcd_acc_fn(m.value_bits, a.R, sell), dim3(workgroups), dim3(kBlock),
                           0, (hipStream_t)stream, P, c, *acc);
    else
        hipLaunchKernelGGL(xcd_fn(m.value_bits, a.R, sell), dim3(workgroups), dim3(kBlock), 0,
                           (hipStream_t)stream, P, c);
    return (int)hipGetLastError();
}

int detect_xcds(int device) {
    constexpr int kProbe = 2048;
    if (hipSetDevice(device) != hipSuccess) return 1;
    int32_t *d = nullptr;
    if (hipMalloc(&d, kProbe * sizeof(int32_t)) != hipSuccess) return 1;
    int32_t h[kProbe];
    hipLaunchKernelGGL(xcc_probe_kernel, dim3(kProbe), dim3(64), 0, nullptr, d);
    bool ok = hipGetLastError() == hipSuccess &&
              hipMemcpy(h, d, sizeof(h), hipMemcpyDeviceToHost) == hipSuccess;
    (void)hipFree(d);
    if (!ok) return 1;
    // the ids seen must be exactly 0..k-1
    int seen[16] = {0}, k = 0;
    for (int i = 0; i < kProbe; ++i) {
        if (h[i] < 0 || h[i] >= kMaxQueues) return 1;
        seen[h[i]] = 1;
        k = std::max(k, h[i] + 1);
    }
    for (int i = 0; i < k; ++i)
        if (!seen[i]) return 1;
    return k;
}

int launch_permute(const int32_t *perm, int64_t n, int to_plan, const double *in, double *out,
                   int nvec, int R, void *stream) {
    const int64_t total = n * (int64_t)R * nvec;
    if (total == 0) return 0;
    int64_t grid = (total + 255) / 256;
    if (grid > 65536) grid = 65536;
    hipLaunchKernelGGL(permute_kernel, dim3((unsigned)grid), dim3(256), 0, (hipStream_t)stream,
                       perm, n, to_plan, in, out, nvec, R);
    return (int)hipGetLastError();
}

int launch_combine_complex(const double *a, const double *b, int64_t n, int R, double *out,
                           void *stream) {
    if (R < 2 || (R & 1)) return (int)hipErrorInvalidValue;
    const int64_t pairs = n * (R / 2);
    if (pairs == 0) return 0;
    int64_t grid = (pairs + 255) / 256;
    if (grid > 8192) grid = 8192;
    hipLaunchKernelGGL(combine_complex_kernel, dim3((unsigned)grid), dim3(256), 0,
                       (hipStream_t)stream, a, b, pairs, out);
    return (int)hipGetLastError();
}

int launch_load_probe(const double *buf, int64_t n_doubles, int passes, int workgroups,
                      double *sink, void *stream) {
    if (n_doubles < 2 || passes < 1 || workgroups < 1) return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(load_probe_kernel, dim3(workgroups), dim3(kBlock), 0, (hipStream_t)stream,
                       reinterpret_cast<const double2 *>(buf), n_doubles / 2, passes, sink);
    return (int)hipGetLastError();
}

int launch_load_probe_xcd(const double *buf, int64_t n_doubles, int regions, int passes,
                          int workgroups, double *sink, int32_t *xcc, void *stream) {
    if (n_doubles < 2 * (int64_t)regions || regions < 1 || regions > kMaxQueues || passes < 1 ||
        workgroups < 1)
        return (int)hipErrorInvalidValue;
    hipLaunchKernelGGL(load_probe_local_kernel, dim3(workgroups), dim3(kBlock), 0,
                       (hipStream_t)stream, reinterpret_cast<const double2 *>(buf),
                       n_doubles / 2, regions, passes, sink, xcc);
    return (int)hipGetLastError();
}

}  // namespace mpk
