// HIP kernels for gfx950 (MI355X): CSR rows as SpMV / SpMM, the p x SpMV
// baseline, the persistent level-blocked kernel, permutation and reset.
//
// All run kernels share one per-row routine (row_block below), so the
// baseline, the level-blocked kernel and every right-hand-side tiling give
// bit-identical results for a given lanes-per-row L:
//   lane l of a row's L lanes accumulates entries e = rs+l, rs+l+L, ... in
//   stored order with fused multiply-adds starting from 0; the L partial sums
//   are then combined by an xor butterfly (offsets 1, 2, 4, ...).
// Values may be stored in float; they are promoted to double before the
// product, and vectors and sums are always double.
#include <hip/hip_runtime.h>

#include "mpk_internal.h"

namespace mpk {

namespace {

constexpr int kBlock = 256;   // threads per workgroup (4 wavefronts of 64)

__device__ __forceinline__ int ld_relaxed(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename V>
__device__ __forceinline__ double ldval(const V *v, int32_t e) {
    return static_cast<double>(v[e]);
}

struct PowerIO {
    const double *in;     // y_{k-1}
    const double *prev;   // y_{k-2} (recurrence; null at the first power)
    double *out;          // y_k
    double alpha, beta, gamma;
    int recur;
};

// Rows [row_begin, row_end) of one power.  Thread t of `nthreads` owns
// lane l of right-hand-side group rg of row slot `slot`:
//   t = (slot * nrg + rg) * L + l,  nrg = R / RT,  RT right-hand sides per thread.
template <typename V, int L, int RT>
__device__ __forceinline__ void row_block(const DevMatrix &m, const PowerIO &io, int32_t R,
                                          int32_t row_begin, int32_t row_end, int tid,
                                          int nthreads) {
    const int nrg = R / RT;
    const int tpr = L * nrg;
    const int rows_per_pass = nthreads / tpr;
    const int slot = tid / tpr;
    const int rem = tid - slot * tpr;
    const int rg = rem / L;
    const int l = rem - rg * L;
    if (slot >= rows_per_pass) return;
    const int32_t *__restrict__ rowptr = m.rowptr;
    const int32_t *__restrict__ col = m.col;
    const V *__restrict__ val = static_cast<const V *>(m.val);
    const double *in = io.in;  // written by other workgroups of the same launch
    const int r0 = rg * RT;
    for (int32_t i = row_begin + slot; i < row_end; i += rows_per_pass) {
        const int32_t rs = rowptr[i], re = rowptr[i + 1];
        double acc[RT];
#pragma unroll
        for (int r = 0; r < RT; ++r) acc[r] = 0.0;
        int32_t e = rs + l;
        // four entries per step: loads first, then the fma chain in order
        for (; e + 3 * L < re; e += 4 * L) {
            int32_t c[4];
            double a[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                c[u] = col[e + u * L];
                a[u] = ldval(val, e + u * L);
            }
            double xv[4][RT];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const double *xp = in + (size_t)c[u] * R + r0;
#pragma unroll
                for (int r = 0; r < RT; ++r) xv[u][r] = xp[r];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int r = 0; r < RT; ++r) acc[r] = __builtin_fma(a[u], xv[u][r], acc[r]);
        }
        for (; e < re; e += L) {
            const int32_t c = col[e];
            const double a = ldval(val, e);
            const double *xp = in + (size_t)c * R + r0;
#pragma unroll
            for (int r = 0; r < RT; ++r) acc[r] = __builtin_fma(a, xp[r], acc[r]);
        }
#pragma unroll
        for (int off = 1; off < L; off <<= 1)
#pragma unroll
            for (int r = 0; r < RT; ++r) acc[r] += __shfl_xor(acc[r], off, L);
        if (l == 0) {
            const int32_t o = m.out_row ? m.out_row[i] : i;
            const size_t base = (size_t)o * R + r0;
            if (io.recur) {
#pragma unroll
                for (int r = 0; r < RT; ++r) {
                    double v = io.alpha * acc[r];
                    v = __builtin_fma(io.beta, in[base + r], v);
                    if (io.prev) v = __builtin_fma(io.gamma, io.prev[base + r], v);
                    acc[r] = v;
                }
            }
#pragma unroll
            for (int r = 0; r < RT; ++r) io.out[base + r] = acc[r];
        }
    }
}

// ------------------------------------------------------------------ baseline

template <typename V, int L, int RT>
__global__ __launch_bounds__(kBlock) void spmv_power_kernel(DevMatrix m, PowerIO io, int32_t R,
                                                           int32_t rows_per_block) {
    const int32_t rb = (int32_t)blockIdx.x * rows_per_block;
    const int32_t re = min(rb + rows_per_block, m.n);
    row_block<V, L, RT>(m, io, R, rb, re, threadIdx.x, blockDim.x);
}

// ------------------------------------------------------------------ level-blocked

struct LBParams {
    DevMatrix m;
    DevSchedule s;
    DevWorkspace ws;
    SegArgs a;
    int64_t spin_limit;   // 100 MHz ticks
};

// Persistent kernel: workgroups take tasks (chunk c, power k) in schedule order
// from a shared ticket counter.  Before computing, a task waits until every
// chunk in [dep_lo[c], dep_hi[c]] has completed power k-1; after computing,
// it publishes done[c] = k.  Dependencies always carry smaller tickets and a
// workgroup holds at most the ticket it works on plus the next one, so the
// smallest unfinished ticket can always proceed; every wait is also bounded
// by spin_limit, after which the run is flagged as failed and all
// workgroups leave.
template <typename V, int L, int RT>
__global__ __launch_bounds__(kBlock) void lb_kernel(LBParams P, Coefs cf) {
    __shared__ int32_t s_ticket;
    const int tid = threadIdx.x;
    const int nt = blockDim.x;
    const size_t stride = (size_t)P.m.n * P.a.R;
    int32_t next = 0;
    if (tid == 0) next = __hip_atomic_fetch_add(P.ws.ticket, 1, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
    for (;;) {
        if (tid == 0) s_ticket = next;
        __syncthreads();
        const int32_t t = s_ticket;
        if (t >= P.s.n_tasks) break;
        if (tid == 0) next = __hip_atomic_fetch_add(P.ws.ticket, 1, __ATOMIC_RELAXED,
                                                    __HIP_MEMORY_SCOPE_AGENT);
        const int32_t c = P.s.tasks[2 * t];
        const int32_t k = P.s.tasks[2 * t + 1];
        if (k > 1) {
            const int32_t lo = P.s.dep_lo[c], hi = P.s.dep_hi[c];
            int ok = 1;
            for (int32_t j = lo + tid; j <= hi && ok; j += nt) {
                if (ld_relaxed(P.ws.done + j) < k - 1) {
                    const uint64_t t0 = wall_clock64();
                    while (ld_relaxed(P.ws.done + j) < k - 1) {
                        __builtin_amdgcn_s_sleep(1);
                        if (ld_relaxed(P.ws.err) != 0 ||
                            (int64_t)(wall_clock64() - t0) > P.spin_limit) {
                            ok = 0;
                            break;
                        }
                    }
                }
            }
            ok = __syncthreads_and(ok);
            if (!ok) {
                if (tid == 0)
                    __hip_atomic_store(P.ws.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                return;
            }
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        }
        // y_k from y_{k-1} (and y_{k-2} for the recurrence); y_0 = in0, y_{-1} = inm1
        PowerIO io;
        io.in = (k == 1) ? P.a.in0 : P.a.Y + (size_t)(k - 2) * stride;
        io.prev = (k == 1) ? P.a.inm1 : (k == 2 ? P.a.in0 : P.a.Y + (size_t)(k - 3) * stride);
        io.out = P.a.Y + (size_t)(k - 1) * stride;
        io.recur = P.a.recur;
        io.alpha = cf.alpha[k - 1];
        io.beta = cf.beta[k - 1];
        io.gamma = cf.gamma[k - 1];
        row_block<V, L, RT>(P.m, io, P.a.R, P.s.chunk_ptr[c], P.s.chunk_ptr[c + 1], tid, nt);
        // make this task's rows visible device-wide before publishing it
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (tid == 0) __hip_atomic_store(P.ws.done + c, k, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__global__ void reset_kernel(DevWorkspace ws, int32_t n_chunks) {
    const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_chunks) ws.done[i] = 0;
    if (i == 0) *ws.ticket = 0;
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

// ------------------------------------------------------------------ dispatch

using SpmvFn = void (*)(DevMatrix, PowerIO, int32_t, int32_t);
using LbFn = void (*)(LBParams, Coefs);

template <typename V, int L, int RT>
struct Inst {
    static constexpr SpmvFn spmv = spmv_power_kernel<V, L, RT>;
    static constexpr LbFn lb = lb_kernel<V, L, RT>;
};

constexpr int kLanes[] = {1, 2, 4, 8, 16};
constexpr int kRT[] = {1, 2, 4, 8};

int lane_index(int L) {
    switch (L) { case 1: return 0; case 2: return 1; case 4: return 2; case 8: return 3; case 16: return 4; }
    return -1;
}
int rt_index(int RT) {
    switch (RT) { case 1: return 0; case 2: return 1; case 4: return 2; case 8: return 3; }
    return -1;
}

template <typename V, int L>
void fill_rt(SpmvFn *s, LbFn *b) {
    s[0] = Inst<V, L, 1>::spmv; b[0] = Inst<V, L, 1>::lb;
    s[1] = Inst<V, L, 2>::spmv; b[1] = Inst<V, L, 2>::lb;
    s[2] = Inst<V, L, 4>::spmv; b[2] = Inst<V, L, 4>::lb;
    s[3] = Inst<V, L, 8>::spmv; b[3] = Inst<V, L, 8>::lb;
}

struct Table {
    SpmvFn spmv[2][5][4];
    LbFn lb[2][5][4];
    Table() {
        fill_rt<double, 1>(spmv[0][0], lb[0][0]);
        fill_rt<double, 2>(spmv[0][1], lb[0][1]);
        fill_rt<double, 4>(spmv[0][2], lb[0][2]);
        fill_rt<double, 8>(spmv[0][3], lb[0][3]);
        fill_rt<double, 16>(spmv[0][4], lb[0][4]);
        fill_rt<float, 1>(spmv[1][0], lb[1][0]);
        fill_rt<float, 2>(spmv[1][1], lb[1][1]);
        fill_rt<float, 4>(spmv[1][2], lb[1][2]);
        fill_rt<float, 8>(spmv[1][3], lb[1][3]);
        fill_rt<float, 16>(spmv[1][4], lb[1][4]);
    }
};

const Table &table() {
    static Table t;
    return t;
}

}  // namespace

bool kernel_config_ok(int lanes, int rhs_per_thread) {
    return lane_index(lanes) >= 0 && rt_index(rhs_per_thread) >= 0;
}

int launch_reset(const DevWorkspace &ws, int32_t n_chunks, void *stream) {
    const int32_t n = n_chunks > 0 ? n_chunks : 1;
    hipLaunchKernelGGL(reset_kernel, dim3((n + 255) / 256), dim3(256), 0, (hipStream_t)stream, ws,
                       n_chunks);
    return (int)hipGetLastError();
}

int launch_spmv_power(const DevMatrix &m, const double *in, const double *inm1, double *out,
                      int32_t R, int recur, double alpha, double beta, double gamma,
                      int rhs_per_thread, void *stream) {
    const int li = lane_index(m.lanes), ri = rt_index(rhs_per_thread);
    if (li < 0 || ri < 0 || R % rhs_per_thread) return (int)hipErrorInvalidValue;
    const int tpr = m.lanes * (R / rhs_per_thread);
    if (tpr > kBlock) return (int)hipErrorInvalidValue;
    if (m.n == 0) return 0;
    const int32_t rows_per_pass = kBlock / tpr;
    // a few passes per workgroup keep the grid large but not tiny-blocked
    const int32_t rows_per_block = rows_per_pass * 2;
    const int64_t grid = ((int64_t)m.n + rows_per_block - 1) / rows_per_block;
    PowerIO io{in, inm1, out, alpha, beta, gamma, recur};
    SpmvFn f = table().spmv[m.value_bits == 32 ? 1 : 0][li][ri];
    hipLaunchKernelGGL(f, dim3((unsigned)grid), dim3(kBlock), 0, (hipStream_t)stream, m, io, R,
                       rows_per_block);
    return (int)hipGetLastError();
}

int lb_max_workgroups(int value_bits, int lanes, int rhs_per_thread, int device) {
    const int li = lane_index(lanes), ri = rt_index(rhs_per_thread);
    if (li < 0 || ri < 0) return 0;
    LbFn f = table().lb[value_bits == 32 ? 1 : 0][li][ri];
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(f),
                                                     kBlock, 0) != hipSuccess)
        return 0;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return 0;
    return per_cu * prop.multiProcessorCount;
}

int launch_lb(const DevMatrix &m, const DevSchedule &s, const DevWorkspace &ws,
              const SegArgs &a, const Coefs *cf, int rhs_per_thread, int workgroups,
              int64_t spin_limit, void *stream) {
    const int li = lane_index(m.lanes), ri = rt_index(rhs_per_thread);
    if (li < 0 || ri < 0 || a.R % rhs_per_thread) return (int)hipErrorInvalidValue;
    if (m.lanes * (a.R / rhs_per_thread) > kBlock) return (int)hipErrorInvalidValue;
    if (a.p < 1 || a.p > kMaxSegPowers || workgroups < 1) return (int)hipErrorInvalidValue;
    if (s.n_tasks == 0) return 0;
    LBParams P{m, s, ws, a, spin_limit};
    Coefs c{};
    if (cf) c = *cf;
    LbFn f = table().lb[m.value_bits == 32 ? 1 : 0][li][ri];
    hipLaunchKernelGGL(f, dim3(workgroups), dim3(kBlock), 0, (hipStream_t)stream, P, c);
    return (int)hipGetLastError();
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

}  // namespace mpk
