// Device-side preprocessing for BFS-ordered plans: the level construction and
// the symmetric permutation of Sec. "RACE Applied to the Matrix Power Kernel"
// (level equation, BFS reordering; the endnote on non-symmetric patterns),
// computed on the GPU from the caller's CSR already uploaded in its own order.
// The result is the one the host planner (bfs_levels + permute_csr) produces:
//
//   * the graph is the stored pattern plus its mirror, self-loops ignored;
//   * level 0 is the root; level L+1 holds the unvisited neighbours of level
//     L; when a level comes out empty while rows remain, the next level
//     starts at the lowest unvisited row;
//   * inside a level rows keep ascending original index (a stable radix
//     sort of the rows by level);
//   * row r' of the permuted matrix is old row perm[r'] with its entries in
//     stored order, columns renumbered when the plan keeps plan numbering.
//
// All level membership is decided by one compare-and-swap per vertex, so the
// level of every row is unique whatever order the threads run in.

#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <vector>

#include "mpk_internal.h"

namespace mpk {

namespace {

constexpr int kThreads = 256;
constexpr int32_t kMaxDeviceLevels = 16384;
constexpr int kMaxDeviceRestarts = 64;

inline unsigned grid_for(int64_t work) {
    const int64_t g = (work + kThreads - 1) / kThreads;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, 65536));
}

__global__ void fill_kernel(int32_t *p, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void iota_kernel(int32_t *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = (int32_t)i;
}

// cnt[c + 1] = number of stored entries in column c (cnt zeroed, n + 1 long)
__global__ void count_cols_kernel(const int32_t *col, int64_t nnz, int32_t *cnt) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x)
        atomicAdd(&cnt[col[e] + 1], 1);
}

// in-neighbours: tcol[fill[c]++] = i for every stored (i, c); the order inside
// a transposed row does not matter (levels are sets)
__global__ void transpose_kernel(const int32_t *rowptr, const int32_t *col, int64_t n,
                                 int32_t *fill, int32_t *tcol) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
            tcol[atomicAdd(&fill[col[e]], 1)] = (int32_t)i;
}

// One BFS level: every unvisited neighbour v of the frontier gets level L
// (claimed by compare-and-swap, so once) and is appended to `next`.  One
// wavefront per frontier vertex: its lanes check up to 64 out- and
// in-neighbours together per round.  A block's claims of a round gather in
// an LDS list, and one thread reserves their place in `next` with a single
// atomic add: the level's counter is the one address every block updates,
// and one update per wave made it the level's bottleneck.
constexpr int kExpandThreads = 1024;
constexpr int kExpandGrid = 1024;   // blocks per level launch (grid-stride beyond)
constexpr int32_t kLevelBatch = 16;  // level launches per read-back of their counts
// The frontier's size is read from the device (*nfp, the previous level's
// counter), so that the host can launch several levels before it reads any
// count back.
__global__ __launch_bounds__(kExpandThreads) void expand_kernel(
        const int32_t *rowptr, const int32_t *col, const int32_t *tptr, const int32_t *tcol,
        const int32_t *front, const int32_t *nfp, int32_t *lev, int32_t L, int32_t *next,
        int32_t *cnt) {
    __shared__ int32_t list[kExpandThreads];
    __shared__ int32_t s_n, s_take, s_base;
    const int32_t nf = *nfp;
    const int lane = (int)(threadIdx.x & 63);
    const int wave = (int)(threadIdx.x >> 6);
    const int wpb = (int)(blockDim.x >> 6);
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    // block-uniform: the block's waves take frontier vertices f0 + wave
    for (int64_t f0 = (int64_t)blockIdx.x * wpb; f0 < nf; f0 += (int64_t)gridDim.x * wpb) {
        const int64_t f = f0 + wave;
        int32_t a0 = 0, na = 0, b0 = 0, total = 0;
        if (f < nf) {
            const int32_t u = front[f];
            a0 = rowptr[u];
            na = rowptr[u + 1] - a0;
            b0 = tptr[u];
            total = na + (tptr[u + 1] - b0);
        }
        bool more = true;
        for (int32_t base = 0; more; base += 64) {   // rounds, uniform over the block
            if (base < total) {                        // uniform over the wave
                const int32_t k = base + lane;
                int32_t v = 0;
                bool claim = false;
                if (k < total) {
                    v = k < na ? col[a0 + k] : tcol[b0 + (k - na)];
                    claim = lev[v] < 0 && atomicCAS(&lev[v], -1, L) == -1;
                }
                const unsigned long long m = __ballot(claim);
                if (m) {
                    const int first = __ffsll((long long)m) - 1;
                    int32_t pos = 0;
                    if (lane == first) pos = atomicAdd(&s_n, (int32_t)__popcll(m));
                    pos = __shfl(pos, first);
                    if (claim) list[pos + (int32_t)__popcll(m & ((1ull << lane) - 1ull))] = v;
                }
            }
            __syncthreads();
            if (threadIdx.x == 0) {
                s_take = s_n;
                s_base = s_n > 0 ? atomicAdd(cnt, s_n) : 0;
                s_n = 0;
            }
            __syncthreads();
            for (int i = (int)threadIdx.x; i < s_take; i += (int)blockDim.x)
                next[s_base + i] = list[i];
            more = __syncthreads_or(base + 64 < total);
        }
    }
}

// out = the lowest row without a level (out preset to n)
__global__ void first_unvisited_kernel(const int32_t *lev, int64_t n, int32_t *out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        if (lev[i] < 0) atomicMin(out, (int32_t)i);
}

// level_ptr[key] = first position of each level in the sorted keys
__global__ void level_starts_kernel(const int32_t *keys, int64_t n, int32_t *level_ptr) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        if (i == 0 || keys[i] != keys[i - 1]) level_ptr[keys[i]] = (int32_t)i;
}

// iperm[perm[r]] = r, and the permuted row lengths len[r] (len[n] = 0)
__global__ void inverse_kernel(const int32_t *perm, const int32_t *rowptr, int64_t n,
                               int32_t *iperm, int32_t *len) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r <= n;
         r += (int64_t)gridDim.x * blockDim.x) {
        if (r == n) {
            len[n] = 0;
            continue;
        }
        const int32_t old = perm[r];
        iperm[old] = (int32_t)r;
        len[r] = rowptr[old + 1] - rowptr[old];
    }
}

// Row r of the permuted matrix: old row perm[r] in stored order, columns in
// plan numbering when plan_cols, values as double or float; row_lo / row_hi
// are the smallest / largest plan-numbered column (the row itself included).
// One wavefront per row: lanes copy consecutive entries (coalesced) and the
// extent is reduced across the wave.
template <typename V>
__global__ void permute_kernel(const int32_t *rowptr, const int32_t *col, const double *val,
                               const int32_t *perm, const int32_t *iperm, const int32_t *nrp,
                               int64_t n, int plan_cols, int32_t *ncol, V *nval, int32_t *row_lo,
                               int32_t *row_hi) {
    const int lane = (int)(threadIdx.x & 63);
    const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
    for (int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6; r < n; r += nwaves) {
        const int32_t old = perm[r];
        const int32_t e0 = rowptr[old], len = rowptr[old + 1] - e0, d0 = nrp[r];
        int32_t lo = (int32_t)r, hi = (int32_t)r;
        for (int32_t k = lane; k < len; k += 64) {
            const int32_t c = col[e0 + k];
            const int32_t cp = iperm[c];
            ncol[d0 + k] = plan_cols ? cp : c;
            nval[d0 + k] = static_cast<V>(val[e0 + k]);
            lo = min(lo, cp);
            hi = max(hi, cp);
        }
        for (int off = 32; off > 0; off >>= 1) {
            lo = min(lo, __shfl_xor(lo, off));
            hi = max(hi, __shfl_xor(hi, off));
        }
        if (lane == 0) {
            row_lo[r] = lo;
            row_hi[r] = hi;
        }
    }
}

// flags[0] |= a row pointer that decreases, flags[1] |= a column out of range
__global__ void validate_kernel(const int32_t *rowptr, const int32_t *col, int64_t n,
                                int64_t nnz, int32_t *flags) {
    int bad_rows = 0, bad_cols = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        bad_rows |= rowptr[i + 1] < rowptr[i];
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x)
        bad_cols |= col[e] < 0 || (int64_t)col[e] >= n;
    if (bad_rows) atomicOr(&flags[0], 1);
    if (bad_cols) atomicOr(&flags[1], 1);
}

// far[i] = the largest row joined to row i in the symmetrised pattern (or i)
__global__ void far_kernel(const int32_t *rowptr, const int32_t *col, int64_t n, int32_t *far) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int32_t hi = (int32_t)i;
        for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            hi = max(hi, col[e]);
            atomicMax(&far[col[e]], (int32_t)i);
        }
        atomicMax(&far[i], hi);
    }
}

// each row's smallest / largest column, the row itself included
__global__ void extent_kernel(const int32_t *rowptr, const int32_t *col, int64_t n, int32_t *lo,
                              int32_t *hi) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        int32_t a = (int32_t)i, b = (int32_t)i;
        for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            a = min(a, col[e]);
            b = max(b, col[e]);
        }
        lo[i] = a;
        hi[i] = b;
    }
}

__global__ void to_float_kernel(const double *in, int64_t n, float *out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = static_cast<float>(in[i]);
}

// out[k] = col[k * step] for k < count
__global__ void gather_kernel(const int32_t *col, int64_t step, int64_t count, int32_t *out) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < count;
         k += (int64_t)gridDim.x * blockDim.x)
        out[k] = col[k * step];
}

// Device scratch of one planning call, freed on every exit path.  reserve() takes
// one block that later get()s are carved from (256-byte aligned); requests
// beyond it get allocations of their own.  (Each hipFree costs ~0.3 ms: the
// level construction's eighteen buffers freed one by one took ~5 ms.)
struct Scratch {
    std::vector<void *> ptrs;
    char *arena = nullptr;
    size_t cap = 0, used = 0;
    ~Scratch() {
        for (void *p : ptrs) (void)hipFree(p);
    }
    static size_t round_up(size_t b) { return (b + 255) & ~(size_t)255; }
    hipError_t reserve(size_t bytes) {
        void *q = nullptr;
        hipError_t e = hipMalloc(&q, std::max<size_t>(bytes, 256));
        if (e != hipSuccess) return e;
        ptrs.push_back(q);
        arena = static_cast<char *>(q);
        cap = bytes;
        used = 0;
        return hipSuccess;
    }
    template <typename T>
    hipError_t get(T **p, size_t count) {
        const size_t b = round_up(std::max<size_t>(count, 1) * sizeof(T));
        if (arena && used + b <= cap) {
            *p = reinterpret_cast<T *>(arena + used);
            used += b;
            return hipSuccess;
        }
        void *q = nullptr;
        hipError_t e = hipMalloc(&q, b);
        if (e != hipSuccess) return e;
        ptrs.push_back(q);
        *p = static_cast<T *>(q);
        return hipSuccess;
    }
};

#define MPK_TRY(x)                          \
    do {                                    \
        hipError_t e_ = (x);                \
        if (e_ != hipSuccess) return (int)e_; \
    } while (0)

}  // namespace

int gpu_levels_permute(int64_t n, int64_t nnz, const int32_t *rowptr, const int32_t *col,
                       const double *val, int32_t root, bool plan_cols, int value_bits,
                       int32_t *out_rowptr, int32_t *out_col, void *out_val, GpuLevels &res) {
    res = GpuLevels{};
    res.level_ptr.push_back(0);
    if (n == 0) return 0;
    Scratch s;
    int32_t *tptr, *fill, *tcol, *lev, *front, *next, *cnt, *perm_in, *perm, *keys, *iperm,
        *len, *level_ptr, *lo, *hi, *start;
    // the arrays below, the level pointers and room for the scans' and the
    // sort's temporary storage, in one block
    MPK_TRY(s.reserve(Scratch::round_up((size_t)(n + 1) * 4) * 3 +
                      Scratch::round_up((size_t)nnz * 4) + Scratch::round_up((size_t)n * 4) * 10 +
                      Scratch::round_up(((size_t)kMaxDeviceLevels + 2) * 4) * 2 + (64u << 20)));
    MPK_TRY(s.get(&tptr, n + 1));
    MPK_TRY(s.get(&fill, n + 1));
    MPK_TRY(s.get(&tcol, nnz));
    MPK_TRY(s.get(&lev, n));
    MPK_TRY(s.get(&front, n));
    MPK_TRY(s.get(&next, n));
    MPK_TRY(s.get(&cnt, (size_t)kMaxDeviceLevels + 2));  // one counter per level
    MPK_TRY(s.get(&perm_in, n));
    MPK_TRY(s.get(&perm, n));
    MPK_TRY(s.get(&keys, n));
    MPK_TRY(s.get(&iperm, n));
    MPK_TRY(s.get(&len, n + 1));
    MPK_TRY(s.get(&lo, n));
    MPK_TRY(s.get(&hi, n));
    MPK_TRY(s.get(&start, 1));

    // 1. transpose pattern (in-neighbours): counts, exclusive sums, scatter
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n + 1)), dim3(kThreads), 0, 0, tptr, n + 1, 0);
    hipLaunchKernelGGL(count_cols_kernel, dim3(grid_for(nnz)), dim3(kThreads), 0, 0, col, nnz,
                       tptr);
    {
        size_t tmp_bytes = 0;
        MPK_TRY(hipcub::DeviceScan::InclusiveSum(nullptr, tmp_bytes, tptr, fill, (int)(n + 1)));
        void *tmp = nullptr;
        MPK_TRY(s.get(reinterpret_cast<char **>(&tmp), tmp_bytes));
        MPK_TRY(hipcub::DeviceScan::InclusiveSum(tmp, tmp_bytes, tptr, fill, (int)(n + 1)));
    }
    // fill = running insert positions (a copy of the column starts)
    MPK_TRY(hipMemcpy(tptr, fill, (size_t)(n + 1) * 4, hipMemcpyDeviceToDevice));
    hipLaunchKernelGGL(transpose_kernel, dim3(grid_for(n)), dim3(kThreads), 0, 0, rowptr, col, n,
                       fill, tcol);
    MPK_TRY(hipGetLastError());

    // 2. levels: expand launches in batches of kLevelBatch (each reads its
    //    frontier's size from the previous level's counter), then one read-back
    //    of the batch's counts; a level that came out empty while rows remain
    //    starts a new component at the lowest unvisited row
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n)), dim3(kThreads), 0, 0, lev, n, -1);
    hipLaunchKernelGGL(fill_kernel, dim3(grid_for(kMaxDeviceLevels + 2)), dim3(kThreads), 0, 0,
                       cnt, (int64_t)kMaxDeviceLevels + 2, 0);
    int32_t *buf[2] = {front, next};   // level l's rows are in buf[l & 1]
    auto place_root = [&](int32_t v, int32_t lvl) -> hipError_t {  // v alone on level lvl
        const int32_t one = 1;
        hipError_t e = hipMemcpy(lev + v, &lvl, 4, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(buf[lvl & 1], &v, 4, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(cnt + lvl, &one, 4, hipMemcpyHostToDevice);
        return e;
    };
    int32_t first = (root >= 0 && root < n) ? root : 0;
    MPK_TRY(place_root(first, 0));
    int64_t visited = 1;
    int32_t top = 0;   // the highest level holding rows
    int restarts = 0;
    std::vector<int32_t> got(kLevelBatch);
    while (visited < n) {
        // each level costs a launch: graphs with very many levels or
        // components are left to the host planner
        if (top + 1 > kMaxDeviceLevels) return kTooManyLevels;
        const int32_t l0 = top + 1, l1 = std::min(l0 + kLevelBatch, kMaxDeviceLevels + 1);
        for (int32_t l = l0; l < l1; ++l)
            hipLaunchKernelGGL(expand_kernel, dim3(kExpandGrid), dim3(kExpandThreads), 0, 0,
                               rowptr, col, tptr, tcol, buf[(l - 1) & 1], cnt + (l - 1), lev, l,
                               buf[l & 1], cnt + l);
        MPK_TRY(hipGetLastError());
        MPK_TRY(hipMemcpy(got.data(), cnt + l0, (size_t)(l1 - l0) * 4, hipMemcpyDeviceToHost));
        int32_t l = l0;
        for (; l < l1 && got[l - l0] > 0; ++l) {
            if (visited + got[l - l0] > n) return (int)hipErrorUnknown;
            visited += got[l - l0];
            top = l;
        }
        if (l < l1 && visited < n) {   // level l came out empty: a new component
            if (++restarts > kMaxDeviceRestarts || l > kMaxDeviceLevels) return kTooManyLevels;
            const int32_t nn = (int32_t)n;
            MPK_TRY(hipMemcpy(start, &nn, 4, hipMemcpyHostToDevice));
            hipLaunchKernelGGL(first_unvisited_kernel, dim3(grid_for(n)), dim3(kThreads), 0, 0,
                               lev, n, start);
            MPK_TRY(hipMemcpy(&first, start, 4, hipMemcpyDeviceToHost));
            if (first < 0 || first >= n) return (int)hipErrorUnknown;
            MPK_TRY(place_root(first, l));
            visited += 1;
            top = l;
        }
    }
    const int32_t L = top + 1;   // levels 0 .. top
    const int32_t n_levels = L;

    // 3. rows by level, ascending original index inside a level (the radix
    //    sort is stable and its input is in index order)
    hipLaunchKernelGGL(iota_kernel, dim3(grid_for(n)), dim3(kThreads), 0, 0, perm_in, n);
    {
        int bits = 1;
        while ((1ll << bits) <= n_levels) ++bits;
        size_t tmp_bytes = 0;
        MPK_TRY(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, lev, keys, perm_in, perm,
                                                   (int)n, 0, bits));
        void *tmp = nullptr;
        MPK_TRY(s.get(reinterpret_cast<char **>(&tmp), tmp_bytes));
        MPK_TRY(hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, lev, keys, perm_in, perm,
                                                   (int)n, 0, bits));
    }
    MPK_TRY(s.get(&level_ptr, (size_t)n_levels + 1));
    hipLaunchKernelGGL(level_starts_kernel, dim3(grid_for(n)), dim3(kThreads), 0, 0, keys, n,
                       level_ptr);

    // 4. inverse permutation, permuted row pointer, permuted rows
    hipLaunchKernelGGL(inverse_kernel, dim3(grid_for(n + 1)), dim3(kThreads), 0, 0, perm, rowptr,
                       n, iperm, len);
    {
        size_t tmp_bytes = 0;
        MPK_TRY(hipcub::DeviceScan::ExclusiveSum(nullptr, tmp_bytes, len, out_rowptr, (int)(n + 1)));
        void *tmp = nullptr;
        MPK_TRY(s.get(reinterpret_cast<char **>(&tmp), tmp_bytes));
        MPK_TRY(hipcub::DeviceScan::ExclusiveSum(tmp, tmp_bytes, len, out_rowptr, (int)(n + 1)));
    }
    if (value_bits == 32)
        hipLaunchKernelGGL(permute_kernel<float>, dim3(grid_for(n * 64)), dim3(kThreads), 0, 0, rowptr,
                           col, val, perm, iperm, out_rowptr, n, plan_cols ? 1 : 0, out_col,
                           static_cast<float *>(out_val), lo, hi);
    else
        hipLaunchKernelGGL(permute_kernel<double>, dim3(grid_for(n * 64)), dim3(kThreads), 0, 0,
                           rowptr, col, val, perm, iperm, out_rowptr, n, plan_cols ? 1 : 0,
                           out_col, static_cast<double *>(out_val), lo, hi);
    MPK_TRY(hipGetLastError());

    // 5. what the host scheduler needs
    res.level_ptr.assign((size_t)n_levels + 1, 0);
    res.perm.resize((size_t)n);
    res.iperm.resize((size_t)n);
    res.rowptr.resize((size_t)n + 1);
    res.row_lo.resize((size_t)n);
    res.row_hi.resize((size_t)n);
    MPK_TRY(hipMemcpy(res.level_ptr.data(), level_ptr, (size_t)n_levels * 4,
                      hipMemcpyDeviceToHost));
    res.level_ptr[(size_t)n_levels] = (int32_t)n;
    MPK_TRY(hipMemcpy(res.perm.data(), perm, (size_t)n * 4, hipMemcpyDeviceToHost));
    MPK_TRY(hipMemcpy(res.iperm.data(), iperm, (size_t)n * 4, hipMemcpyDeviceToHost));
    MPK_TRY(hipMemcpy(res.rowptr.data(), out_rowptr, (size_t)(n + 1) * 4, hipMemcpyDeviceToHost));
    MPK_TRY(hipMemcpy(res.row_lo.data(), lo, (size_t)n * 4, hipMemcpyDeviceToHost));
    MPK_TRY(hipMemcpy(res.row_hi.data(), hi, (size_t)n * 4, hipMemcpyDeviceToHost));
    if (res.rowptr[(size_t)n] != nnz) return (int)hipErrorUnknown;
    return 0;
}

int gpu_validate(int64_t n, int64_t nnz, const int32_t *rowptr, const int32_t *col,
                 int *bad_rows, int *bad_cols, int32_t *first_last) {
    Scratch s;
    int32_t *flags;
    MPK_TRY(s.get(&flags, 2));
    MPK_TRY(hipMemset(flags, 0, 8));
    hipLaunchKernelGGL(validate_kernel, dim3(grid_for(std::max(n, nnz))), dim3(kThreads), 0, 0,
                       rowptr, col, n, nnz, flags);
    MPK_TRY(hipGetLastError());
    int32_t f[2];
    MPK_TRY(hipMemcpy(f, flags, 8, hipMemcpyDeviceToHost));
    MPK_TRY(hipMemcpy(&first_last[0], rowptr, 4, hipMemcpyDeviceToHost));
    MPK_TRY(hipMemcpy(&first_last[1], rowptr + n, 4, hipMemcpyDeviceToHost));
    *bad_rows = f[0];
    *bad_cols = f[1];
    return 0;
}

int gpu_order_far(int64_t n, const int32_t *rowptr, const int32_t *col, std::vector<int32_t> &far) {
    Scratch s;
    int32_t *d;
    MPK_TRY(s.get(&d, n));
    hipLaunchKernelGGL(iota_kernel, dim3(grid_for(n)), dim3(kThreads), 0, 0, d, n);
    hipLaunchKernelGGL(far_kernel, dim3(grid_for(n)), dim3(kThreads), 0, 0, rowptr, col, n, d);
    MPK_TRY(hipGetLastError());
    far.resize((size_t)n);
    MPK_TRY(hipMemcpy(far.data(), d, (size_t)n * 4, hipMemcpyDeviceToHost));
    return 0;
}

int gpu_copy_in_place_order(int64_t n, int64_t nnz, const int32_t *rowptr, const int32_t *col,
                            const double *val, int value_bits, int32_t *out_rowptr,
                            int32_t *out_col, void *out_val, std::vector<int32_t> &h_rowptr,
                            std::vector<int32_t> &row_lo, std::vector<int32_t> &row_hi) {
    Scratch s;
    int32_t *lo, *hi;
    MPK_TRY(s.get(&lo, n));
    MPK_TRY(s.get(&hi, n));
    MPK_TRY(hipMemcpy(out_rowptr, rowptr, (size_t)(n + 1) * 4, hipMemcpyDeviceToDevice));
    if (nnz > 0) {
        MPK_TRY(hipMemcpy(out_col, col, (size_t)nnz * 4, hipMemcpyDeviceToDevice));
        if (value_bits == 32)
            hipLaunchKernelGGL(to_float_kernel, dim3(grid_for(nnz)), dim3(kThreads), 0, 0, val,
                               nnz, static_cast<float *>(out_val));
        else
            MPK_TRY(hipMemcpy(out_val, val, (size_t)nnz * 8, hipMemcpyDeviceToDevice));
    }
    hipLaunchKernelGGL(extent_kernel, dim3(grid_for(n)), dim3(kThreads), 0, 0, rowptr, col, n, lo,
                       hi);
    MPK_TRY(hipGetLastError());
    h_rowptr.resize((size_t)n + 1);
    row_lo.resize((size_t)n);
    row_hi.resize((size_t)n);
    MPK_TRY(hipMemcpy(h_rowptr.data(), rowptr, (size_t)(n + 1) * 4, hipMemcpyDeviceToHost));
    MPK_TRY(hipMemcpy(row_lo.data(), lo, (size_t)n * 4, hipMemcpyDeviceToHost));
    MPK_TRY(hipMemcpy(row_hi.data(), hi, (size_t)n * 4, hipMemcpyDeviceToHost));
    return 0;
}

int gpu_sample_cols(const int32_t *col, int64_t step, int64_t count, std::vector<int32_t> &out) {
    out.assign((size_t)count, 0);
    if (count == 0) return 0;
    Scratch s;
    int32_t *d;
    MPK_TRY(s.get(&d, count));
    hipLaunchKernelGGL(gather_kernel, dim3(grid_for(count)), dim3(kThreads), 0, 0, col, step,
                       count, d);
    MPK_TRY(hipGetLastError());
    MPK_TRY(hipMemcpy(out.data(), d, (size_t)count * 4, hipMemcpyDeviceToHost));
    return 0;
}

namespace {

// Width (longest row) of each 64-row slice.
__global__ void sell_width_kernel(const int32_t *rowptr, int64_t n, int32_t *width) {
    const int64_t n_sl = (n + kSellRows - 1) / kSellRows;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < n_sl;
         s += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r1 = std::min<int64_t>(n, (s + 1) * kSellRows);
        int32_t w = 0;
        for (int64_t r = s * kSellRows; r < r1; ++r) w = max(w, rowptr[r + 1] - rowptr[r]);
        width[s] = w;
    }
}

// The offset of column c from row r taken modulo n into [-n/2, n/2): the
// kernels recover c as r + offset, wrapped into [0, n).  Periodic lattices
// whose wrap-around neighbours lie far away in index then still have small
// offsets.
__device__ __forceinline__ int64_t col_offset(int64_t c, int64_t r, int64_t n) {
    int64_t d = c - r;
    if (2 * d >= n) d -= n;
    else if (2 * d < -n) d += n;
    return d;
}

// Entry j of row r goes to soff[r / 64] + j * 64 + r % 64; rlen[r] = length.
// One block per 64-row slice: the slice's nonzeros are contiguous in the CSR,
// so the block reads them coalesced and finds each one's row by a binary
// search over the slice's 65 row pointers held in LDS.  Padding is left
// unwritten: the kernels never read past a row's length.
template <typename V>
__global__ void sell_fill_kernel(const int32_t *rowptr, const int32_t *col, const V *val,
                                 int64_t n, const int64_t *soff, int32_t *rlen, int32_t *scol,
                                 int16_t *sdel, V *sval, int32_t *max_off) {
    __shared__ int32_t rp[kSellRows + 1];
    __shared__ int32_t bmax;
    if (threadIdx.x == 0) bmax = 0;
    int64_t m = 0;
    const int64_t n_sl = (n + kSellRows - 1) / kSellRows;
    for (int64_t s = blockIdx.x; s < n_sl; s += gridDim.x) {
        const int64_t r0 = s * kSellRows;
        const int nr = (int)std::min<int64_t>(kSellRows, n - r0);
        __syncthreads();
        for (int i = threadIdx.x; i <= nr; i += blockDim.x) rp[i] = rowptr[r0 + i];
        __syncthreads();
        for (int i = threadIdx.x; i < nr; i += blockDim.x) rlen[r0 + i] = rp[i + 1] - rp[i];
        const int64_t base = soff[s];
        for (int32_t e = rp[0] + (int32_t)threadIdx.x; e < rp[nr]; e += blockDim.x) {
            int lo = 0, hi = nr - 1;   // last row i with rp[i] <= e
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (rp[mid] <= e) lo = mid; else hi = mid - 1;
            }
            const int64_t dst = base + (int64_t)(e - rp[lo]) * kSellRows + lo;
            const int32_t c = col[e];
            scol[dst] = c;
            if (sdel) {   // kept only if every offset fits 16 bits (max_off)
                const int64_t d = col_offset(c, r0 + lo, n);
                sdel[dst] = (int16_t)d;
                m = std::max<int64_t>(m, d < 0 ? -d : d);
            }
            sval[dst] = val[e];
        }
    }
    if (sdel) {   // uniform
        __syncthreads();
        if (m > 0) atomicMax(&bmax, (int32_t)m);
        __syncthreads();
        if (threadIdx.x == 0 && bmax > 0) atomicMax(max_off, bmax);
    }
}

}  // namespace

int gpu_sell_widths(int64_t n, const int32_t *rowptr, std::vector<int32_t> &width) {
    const int64_t n_sl = (n + kSellRows - 1) / kSellRows;
    width.assign((size_t)n_sl, 0);
    if (n_sl == 0) return 0;
    Scratch s;
    int32_t *d;
    MPK_TRY(s.get(&d, n_sl));
    hipLaunchKernelGGL(sell_width_kernel, dim3(grid_for(n_sl)), dim3(kThreads), 0, 0, rowptr, n, d);
    MPK_TRY(hipGetLastError());
    MPK_TRY(hipMemcpy(width.data(), d, (size_t)n_sl * 4, hipMemcpyDeviceToHost));
    return 0;
}

int gpu_sell_fill(int64_t n, const int32_t *rowptr, const int32_t *col, const void *val,
                  int value_bits, const int64_t *soff, int64_t entries, int32_t *rlen,
                  int32_t *scol, int16_t *sdel, void *sval, int32_t *max_offset) {
    (void)entries;
    *max_offset = 0;
    if (n == 0) return 0;
    const int64_t n_sl = (n + kSellRows - 1) / kSellRows;
    const dim3 grid((unsigned)std::min<int64_t>(n_sl, 65536));
    Scratch s;
    int32_t *d_max;
    MPK_TRY(s.get(&d_max, 1));
    hipLaunchKernelGGL(fill_kernel, dim3(1), dim3(kThreads), 0, 0, d_max, (int64_t)1, 0);
    if (value_bits == 32)
        hipLaunchKernelGGL(sell_fill_kernel<float>, grid, dim3(kThreads), 0, 0,
                           rowptr, col, static_cast<const float *>(val), n, soff, rlen, scol,
                           sdel, static_cast<float *>(sval), d_max);
    else
        hipLaunchKernelGGL(sell_fill_kernel<double>, grid, dim3(kThreads), 0, 0,
                           rowptr, col, static_cast<const double *>(val), n, soff, rlen, scol,
                           sdel, static_cast<double *>(sval), d_max);
    MPK_TRY(hipGetLastError());
    MPK_TRY(hipMemcpy(max_offset, d_max, 4, hipMemcpyDeviceToHost));
    return 0;
}

}  // namespace mpk
