// Host planner: CSR validation, level construction, symmetric permutation,
// level groups, chunks, dependency ranges and the task schedule.
//
// Levels follow Sec. "RACE Applied to the Matrix Power Kernel": L(0) is the
// root, each next level holds the not yet visited neighbours of the previous
// one, the pattern is treated as symmetric (endnote on non-symmetric
// matrices), and the matrix is then permuted symmetrically by level.  The
// schedule generalises the Lp-diagram traversal of the same section (Fig.
// lp_basic) from whole levels to chunks of rows.
#include <algorithm>
#include <cstdint>
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <numeric>

#include "mpk_internal.h"

namespace mpk {

static double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

mpk_status_t validate_csr(const mpk_csr_t *A, bool need_values, std::string &err) {
    if (!A) { err = "A is NULL"; return MPK_EINVAL; }
    if (A->n < 0 || A->nnz < 0) { err = "negative n or nnz"; return MPK_EBADCSR; }
    if (A->n >= (int64_t)INT32_MAX) { err = "n >= 2^31 is not supported"; return MPK_EUNSUPPORTED; }
    if (A->nnz >= (int64_t)INT32_MAX) { err = "nnz >= 2^31 is not supported"; return MPK_EUNSUPPORTED; }
    if (!A->rowptr) { err = "rowptr is NULL"; return MPK_EINVAL; }
    if (A->nnz > 0 && !A->col) { err = "col is NULL"; return MPK_EINVAL; }
    if (need_values && A->nnz > 0 && !A->val) { err = "val is NULL"; return MPK_EINVAL; }
    if (A->rowptr[0] != 0) { err = "rowptr[0] != 0"; return MPK_EBADCSR; }
    // parallel scans; the first offending index is found serially on failure
    const int64_t n = A->n, nnz = A->nnz;
    const int32_t *rp = A->rowptr, *col = A->col;
    int bad_rows = 0, bad_cols = 0;
#pragma omp parallel for reduction(| : bad_rows) schedule(static)
    for (int64_t i = 0; i < n; ++i) bad_rows |= rp[i + 1] < rp[i];
    if (bad_rows) {
        for (int64_t i = 0; i < n; ++i)
            if (rp[i + 1] < rp[i]) {
                err = "rowptr decreases at row " + std::to_string(i);
                return MPK_EBADCSR;
            }
    }
    if ((int64_t)rp[n] != nnz) { err = "rowptr[n] != nnz"; return MPK_EBADCSR; }
#pragma omp parallel for reduction(| : bad_cols) schedule(static)
    for (int64_t e = 0; e < nnz; ++e) bad_cols |= col[e] < 0 || (int64_t)col[e] >= n;
    if (bad_cols) {
        for (int64_t e = 0; e < nnz; ++e)
            if (col[e] < 0 || (int64_t)col[e] >= n) {
                err = "column index out of range at entry " + std::to_string(e);
                return MPK_EBADCSR;
            }
    }
    return MPK_OK;
}

// Breadth-first search over the symmetrised graph (stored entries and their
// mirrors, self-loops ignored) from r: returns the eccentricity of r within
// its component and leaves the last distance layer in `last` (ascending).
// mark[] holds a stamp per visited vertex; `stamp` must be new for each call.
static int bfs_last_layer(const int32_t *rowptr, const int32_t *col, const int32_t *tptr,
                          const int32_t *tcol, int32_t r, std::vector<int32_t> &mark,
                          int32_t stamp, std::vector<int32_t> &last) {
    std::vector<int32_t> front{r}, next;
    mark[r] = stamp;
    int depth = 0;
    for (;;) {
        next.clear();
        for (int32_t u : front) {
            for (int32_t e = rowptr[u]; e < rowptr[u + 1]; ++e)
                if (mark[col[e]] != stamp) {
                    mark[col[e]] = stamp;
                    next.push_back(col[e]);
                }
            for (int32_t e = tptr[u]; e < tptr[u + 1]; ++e)
                if (mark[tcol[e]] != stamp) {
                    mark[tcol[e]] = stamp;
                    next.push_back(tcol[e]);
                }
        }
        if (next.empty()) break;
        front.swap(next);
        ++depth;
    }
    std::sort(front.begin(), front.end());
    last.swap(front);
    return depth;
}

// George-Liu pseudo-peripheral vertex of start's component: from x, take the
// vertex y of least degree (distinct neighbours other than itself, ties to
// the smaller index) in the last BFS layer; move to y while that increases
// the eccentricity.
static int32_t pseudo_peripheral(int64_t n, const int32_t *rowptr, const int32_t *col,
                                 const int32_t *tptr, const int32_t *tcol, int32_t start) {
    std::vector<int32_t> mark(n, -1), last, nb;
    int32_t stamp = 0;
    int32_t x = start;
    int ex = bfs_last_layer(rowptr, col, tptr, tcol, x, mark, stamp++, last);
    for (;;) {
        int32_t y = -1;
        size_t best = SIZE_MAX;
        for (int32_t v : last) {
            nb.clear();
            for (int32_t e = rowptr[v]; e < rowptr[v + 1]; ++e)
                if (col[e] != v) nb.push_back(col[e]);
            for (int32_t e = tptr[v]; e < tptr[v + 1]; ++e)
                if (tcol[e] != v) nb.push_back(tcol[e]);
            std::sort(nb.begin(), nb.end());
            const size_t deg = (size_t)(std::unique(nb.begin(), nb.end()) - nb.begin());
            if (deg < best) {  // `last` is ascending: ties keep the smaller index
                best = deg;
                y = v;
            }
        }
        std::vector<int32_t> ylast;
        const int ey = bfs_last_layer(rowptr, col, tptr, tcol, y, mark, stamp++, ylast);
        if (ey <= ex) return x;
        x = y;
        ex = ey;
        last.swap(ylast);
    }
}

// Level index of every row: d[perm[r]] = level of plan row r.
static std::vector<int32_t> level_of(int64_t n, const Levels &lv) {
    std::vector<int32_t> d(n);
    for (size_t l = 0; l + 1 < lv.level_ptr.size(); ++l)
        for (int32_t r = lv.level_ptr[l]; r < lv.level_ptr[l + 1]; ++r) d[lv.perm[r]] = (int32_t)l;
    return d;
}

Levels sublevel_order(int64_t n, const int32_t *rowptr, const int32_t *col, const Levels &lv,
                      int32_t root2, int32_t *root_out, int32_t *max_sub) {
    Levels out;
    out.level_ptr = lv.level_ptr;
    if (root_out) *root_out = -1;
    if (max_sub) *max_sub = 0;
    if (n == 0) return out;
    if (root2 < 0 || root2 >= n) {
        // the widest level (first among equals) and its smallest vertex w
        size_t wl = 0;
        for (size_t l = 0; l + 1 < lv.level_ptr.size(); ++l)
            if (lv.level_ptr[l + 1] - lv.level_ptr[l] > lv.level_ptr[wl + 1] - lv.level_ptr[wl])
                wl = l;
        const int32_t w = lv.perm[lv.level_ptr[wl]];  // a level lists ascending indices
        const std::vector<int32_t> dw = level_of(n, bfs_levels(n, rowptr, col, w));
        root2 = w;
        for (int32_t r = lv.level_ptr[wl]; r < lv.level_ptr[wl + 1]; ++r) {
            const int32_t v = lv.perm[r];  // ascending: a tie keeps the smaller index
            if (dw[v] > dw[root2]) root2 = v;
        }
    }
    const std::vector<int32_t> d2 = level_of(n, bfs_levels(n, rowptr, col, root2));
    out.perm = lv.perm;
    int32_t most = 0;
    for (size_t l = 0; l + 1 < lv.level_ptr.size(); ++l) {
        auto b = out.perm.begin() + lv.level_ptr[l], e = out.perm.begin() + lv.level_ptr[l + 1];
        std::stable_sort(b, e, [&](int32_t a, int32_t c) { return d2[a] < d2[c]; });
        int32_t subs = 0;
        for (auto it = b; it != e; ++it)
            if (it == b || d2[*it] != d2[*(it - 1)]) ++subs;
        most = std::max(most, subs);
    }
    out.iperm.assign(n, 0);
    for (int64_t r = 0; r < n; ++r) out.iperm[out.perm[r]] = (int32_t)r;
    if (root_out) *root_out = root2;
    if (max_sub) *max_sub = most;
    return out;
}

Levels bfs_levels(int64_t n, const int32_t *rowptr, const int32_t *col, int32_t root) {
    Levels lv;
    lv.perm.reserve(n);
    lv.level_ptr.push_back(0);
    if (n == 0) return lv;
    // transpose pattern: in-neighbours, so that the graph is symmetric (the
    // order inside a transposed row is irrelevant: frontiers are sorted)
    const int64_t nnz = rowptr[n];
    std::vector<int32_t> tptr(n + 1, 0), tcol(nnz);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < nnz; ++e) __atomic_fetch_add(&tptr[col[e] + 1], 1, __ATOMIC_RELAXED);
    for (int64_t i = 0; i < n; ++i) tptr[i + 1] += tptr[i];
    {
        std::vector<int32_t> fill(tptr.begin(), tptr.end() - 1);
#pragma omp parallel for schedule(dynamic, 4096)
        for (int64_t i = 0; i < n; ++i)
            for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
                tcol[__atomic_fetch_add(&fill[col[e]], 1, __ATOMIC_RELAXED)] = (int32_t)i;
    }
    std::vector<uint8_t> seen(n, 0);
    std::vector<int32_t> frontier, next;
    int64_t lowest = 0;  // every row below this index is already levelled
    int64_t visited = 0;
    int32_t start = (root >= 0 && root < n) ? root : 0;
    if (root == MPK_ROOT_PERIPHERAL)
        start = pseudo_peripheral(n, rowptr, col, tptr.data(), tcol.data(), 0);
    // claim v for the next level (several threads may find it at once)
    auto claim = [&seen](int32_t v) {
        return __atomic_load_n(&seen[v], __ATOMIC_RELAXED) == 0 &&
               __atomic_exchange_n(&seen[v], (uint8_t)1, __ATOMIC_RELAXED) == 0;
    };
    while (visited < n) {
        if (frontier.empty()) {
            if (visited > 0) {
                while (seen[lowest]) ++lowest;
                start = (int32_t)lowest;
            }
            seen[start] = 1;
            frontier.assign(1, start);
        }
        // emit the current level
        lv.perm.insert(lv.perm.end(), frontier.begin(), frontier.end());
        visited += (int64_t)frontier.size();
        lv.level_ptr.push_back((int32_t)lv.perm.size());
        next.clear();
        const int64_t fs = (int64_t)frontier.size();
        if (fs < 2048) {
            for (int32_t u : frontier) {
                for (int32_t e = rowptr[u]; e < rowptr[u + 1]; ++e)
                    if (claim(col[e])) next.push_back(col[e]);
                for (int32_t e = tptr[u]; e < tptr[u + 1]; ++e)
                    if (claim(tcol[e])) next.push_back(tcol[e]);
            }
        } else {
#pragma omp parallel
            {
                std::vector<int32_t> mine;
#pragma omp for schedule(dynamic, 256) nowait
                for (int64_t f = 0; f < fs; ++f) {
                    const int32_t u = frontier[f];
                    for (int32_t e = rowptr[u]; e < rowptr[u + 1]; ++e)
                        if (claim(col[e])) mine.push_back(col[e]);
                    for (int32_t e = tptr[u]; e < tptr[u + 1]; ++e)
                        if (claim(tcol[e])) mine.push_back(tcol[e]);
                }
#pragma omp critical
                next.insert(next.end(), mine.begin(), mine.end());
            }
        }
        std::sort(next.begin(), next.end());
        frontier.swap(next);
    }
    lv.iperm.assign(n, 0);
    for (int64_t i = 0; i < n; ++i) lv.iperm[lv.perm[i]] = (int32_t)i;
    return lv;
}

Levels order_levels(int64_t n, const int32_t *rowptr, const int32_t *col) {
    Levels lv;
    lv.perm.resize(n);
    lv.iperm.resize(n);
    std::iota(lv.perm.begin(), lv.perm.end(), 0);
    std::iota(lv.iperm.begin(), lv.iperm.end(), 0);
    lv.level_ptr.push_back(0);
    if (n == 0) return lv;
    // farthest symmetric neighbour of each row
    std::vector<int32_t> far(n);
    for (int64_t i = 0; i < n; ++i) far[i] = (int32_t)i;
    auto raise = [&far](int32_t at, int32_t v) {
        int32_t cur = __atomic_load_n(&far[at], __ATOMIC_RELAXED);
        while (v > cur &&
               !__atomic_compare_exchange_n(&far[at], &cur, v, true, __ATOMIC_RELAXED, __ATOMIC_RELAXED)) {
        }
    };
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t i = 0; i < n; ++i) {
        int32_t hi = (int32_t)i;  // row i's own farthest column, raised once
        for (int32_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            hi = std::max(hi, col[e]);
            raise(col[e], (int32_t)i);  // and i as a neighbour of that column
        }
        raise((int32_t)i, hi);
    }
    Levels from = levels_from_far(n, far);
    lv.level_ptr.swap(from.level_ptr);
    return lv;
}

Levels levels_from_far(int64_t n, const std::vector<int32_t> &far) {
    Levels lv;
    lv.perm.resize(n);
    lv.iperm.resize(n);
    std::iota(lv.perm.begin(), lv.perm.end(), 0);
    std::iota(lv.iperm.begin(), lv.iperm.end(), 0);
    lv.level_ptr.push_back(0);
    if (n == 0) return lv;
    // level 0 = row 0; level j+1 ends just past the farthest neighbour of level j
    int64_t b_prev = 0, b = 1;
    lv.level_ptr.push_back(1);
    while (b < n) {
        int64_t reach = b;  // exclusive end needed for the next level
        for (int64_t i = b_prev; i < b; ++i) reach = std::max<int64_t>(reach, (int64_t)far[i] + 1);
        int64_t nb = std::max<int64_t>(b + 1, std::min<int64_t>(reach, n));
        b_prev = b;
        b = nb;
        lv.level_ptr.push_back((int32_t)b);
    }
    return lv;
}

void permute_csr(int64_t n, const int32_t *rowptr, const int32_t *col, const double *val,
                 const Levels &lv, bool plan_cols, PermutedCSR &out) {
    bool identity = true;
    for (int64_t r = 0; r < n && identity; ++r) identity = lv.perm[r] == r;
    out.identity = identity;
    if (identity) {
        // the caller's arrays are already in plan order: leave columns and
        // values to be read in place and only find each row's column extent
        out.rowptr.assign(rowptr, rowptr + n + 1);
        out.col.clear();
        out.val.clear();
        out.row_lo.resize(n);
        out.row_hi.resize(n);
#pragma omp parallel for schedule(static)
        for (int64_t r = 0; r < n; ++r) {
            int32_t lo = (int32_t)r, hi = (int32_t)r;
            for (int32_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
                lo = std::min(lo, col[e]);
                hi = std::max(hi, col[e]);
            }
            out.row_lo[r] = lo;
            out.row_hi[r] = hi;
        }
        return;
    }
    out.rowptr.assign(n + 1, 0);
    for (int64_t r = 0; r < n; ++r) {
        int32_t old = lv.perm[r];
        out.rowptr[r + 1] = out.rowptr[r] + (rowptr[old + 1] - rowptr[old]);
    }
    const int64_t nnz = n ? out.rowptr[n] : 0;
    out.col.resize(nnz);
    if (val) out.val.resize(nnz);
    out.row_lo.resize(n);
    out.row_hi.resize(n);
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t r = 0; r < n; ++r) {
        const int32_t old = lv.perm[r];
        int32_t lo = (int32_t)r, hi = (int32_t)r;  // a row always depends on itself
        int32_t d = out.rowptr[r];
        for (int32_t e = rowptr[old]; e < rowptr[old + 1]; ++e, ++d) {
            const int32_t cp = lv.iperm[col[e]];
            out.col[d] = plan_cols ? cp : col[e];
            if (val) out.val[d] = val[e];
            lo = std::min(lo, cp);
            hi = std::max(hi, cp);
        }
        out.row_lo[r] = lo;
        out.row_hi[r] = hi;
    }
}

// ------------------------------------------------------------------ schedule

namespace {

// Range-maximum over a static array (sparse table).
struct RangeMax {
    std::vector<std::vector<int64_t>> t;
    explicit RangeMax(const std::vector<int64_t> &a) {
        t.push_back(a);
        for (size_t w = 1; (w << 1) <= a.size(); w <<= 1) {
            const auto &prev = t.back();
            std::vector<int64_t> cur(a.size() - (w << 1) + 1);
            for (size_t i = 0; i < cur.size(); ++i) cur[i] = std::max(prev[i], prev[i + w]);
            t.push_back(std::move(cur));
        }
    }
    int64_t query(int32_t lo, int32_t hi) const {  // inclusive
        const uint32_t len = (uint32_t)(hi - lo + 1);
        const int j = 31 - __builtin_clz(len);
        return std::max(t[j][lo], t[j][hi - (1 << j) + 1]);
    }
};

}  // namespace

// Chunk size actually used: the tuning's, but small enough that every one of
// the running workgroups gets about two chunks of each power (at least 1024
// nonzeros): on small matrices large chunks would leave most of the device idle.
static int64_t effective_chunk_nnz(const PlanShape &sh, const mpk_tune_t &tune,
                                   int default_workgroups) {
    const int64_t want = std::max(1, tune.chunk_nnz);
    const int64_t fill = std::max<int64_t>(1024, sh.nnz / (2 * (int64_t)std::max(1, default_workgroups)));
    return std::min(want, fill);
}

// XCD schedule: every level is split into n_xcd contiguous parts (by
// nonzeros) and part x of every level belongs to XCD x, so a chunk's rows
// mostly read rows of the same XCD one level up or down (with sub-level
// ordering, a part is a run of consecutive sub-levels).  Every chunk
// boundary is a multiple of kLineRows rows: a level's span is taken from its
// first row rounded up to the next multiple to the same for the next level,
// so a chunk may hold up to kLineRows - 1 rows of a neighbouring level (the
// dependency lists are exact, so this only moves work between XCDs).  The
// schedule is then line-closed (see Schedule::line_closed).  Dependencies
// are exact lists of chunks.
static mpk_status_t build_xcd_schedule(const PlanShape &sh, int p, const mpk_tune_t &tune,
                                       int default_workgroups, Schedule &s, std::string &err) {
    const double t0 = now_ms();
    const int64_t n = sh.n;
    const auto &lp = *sh.level_ptr;
    const auto &rp = *sh.rowptr;
    const auto &pcol = *sh.pcol;
    const int nx = std::max(1, std::min(sh.n_xcd, kMaxQueues));
    const int32_t n_levels = (int32_t)lp.size() - 1;
    const double row_bytes = 4.0, nz_bytes = 4.0 + sh.value_bytes;
    // p + 1 consecutive chunks of one queue fit its XCD's L2 budget
    const int64_t l2_cap = std::max<int64_t>(
        1024, (int64_t)((double)sh.l2_bytes * tune.cache_safety / ((p + 1) * nz_bytes)));
    const int64_t chunk_nnz = std::min(effective_chunk_nnz(sh, tune, default_workgroups), l2_cap);
    s.n_queues = nx;
    s.n_groups = n_levels;
    s.chunk_ptr.assign(1, 0);
    auto align_up = [](int64_t r) { return (r + kLineRows - 1) & ~(int64_t)(kLineRows - 1); };
    auto span = [&](int32_t l) { return l >= n_levels ? n : std::min<int64_t>(n, align_up(lp[l])); };
    for (int32_t l = 0; l < n_levels; ++l) {
        const int64_t L0 = span(l), L1 = span(l + 1);
        if (L1 <= L0) continue;
        const int64_t rows = L1 - L0;
        const int parts = (int)std::max<int64_t>(1, std::min<int64_t>(nx, rows / 16));
        int64_t a = L0;
        for (int x = 0; x < parts; ++x) {
            int64_t b = L1;
            if (x + 1 < parts) {
                const int64_t target = rp[L0] + ((int64_t)rp[L1] - rp[L0]) * (x + 1) / parts;
                b = std::upper_bound(rp.begin() + a, rp.begin() + L1, (int32_t)target) - rp.begin();
                b = align_up(b);
                if (b <= a) b = align_up(a + 1);
                b = std::min<int64_t>(b, L1);
            }
            if (b <= a) continue;
            const int xcd = (int)((int64_t)x * nx / parts);
            // cut [a, b) into chunks of about chunk_nnz nonzeros
            int64_t r = a;
            while (r < b) {
                const int64_t lim = (int64_t)rp[r] + chunk_nnz;
                int64_t e = std::upper_bound(rp.begin() + r + 1, rp.begin() + b + 1,
                                             (int32_t)std::min<int64_t>(lim, INT32_MAX)) -
                            rp.begin() - 1;
                e = std::min<int64_t>(e, r + 65536);
                if (e < b) {
                    // round to a multiple of kLineRows rows, at least one step past r
                    int64_t ea = e & ~(int64_t)(kLineRows - 1);
                    if (ea <= r) ea = align_up(r + 1);
                    e = std::min<int64_t>(ea, b);
                }
                s.chunk_ptr.push_back((int32_t)e);
                s.chunk_group.push_back(l);
                s.chunk_xcd.push_back(xcd);
                r = e;
            }
            a = b;
        }
    }
    s.line_closed = true;
    const int32_t nc = s.n_chunks();
    std::vector<int32_t> chunk_of(n);
    for (int32_t c = 0; c < nc; ++c)
        for (int32_t r = s.chunk_ptr[c]; r < s.chunk_ptr[c + 1]; ++r) chunk_of[r] = c;
    // exact dependency lists (the chunk itself included)
    std::vector<int32_t> stamp(nc, -1);
    s.dep_ptr.assign(1, 0);
    s.dep_lo.resize(nc);
    s.dep_hi.resize(nc);
    double reach_sum = 0.0;
    for (int32_t c = 0; c < nc; ++c) {
        const size_t start = s.dep_idx.size();
        stamp[c] = c;
        s.dep_idx.push_back(c);
        for (int32_t e = rp[s.chunk_ptr[c]]; e < rp[s.chunk_ptr[c + 1]]; ++e) {
            const int32_t d = chunk_of[pcol[e]];
            if (stamp[d] != c) {
                stamp[d] = c;
                s.dep_idx.push_back(d);
            }
        }
        std::sort(s.dep_idx.begin() + start, s.dep_idx.end());
        s.dep_ptr.push_back((int32_t)s.dep_idx.size());
        s.dep_lo[c] = s.dep_idx[start];
        s.dep_hi[c] = s.dep_idx.back();
        s.max_reach = std::max(s.max_reach, s.dep_hi[c] - c);
        reach_sum += s.dep_hi[c] - c;
    }
    // results read by another XCD must leave the producer's L2
    s.remote_out.assign(nc, sh.xcd_local ? 0 : 1);
    if (sh.xcd_local)
        for (int32_t c = 0; c < nc; ++c)
            for (int32_t j = s.dep_ptr[c]; j < s.dep_ptr[c + 1]; ++j)
                if (s.chunk_xcd[s.dep_idx[j]] != s.chunk_xcd[c]) s.remote_out[s.dep_idx[j]] = 1;
    // skewed wavefront over the exact lists: pos(c,1) = c, pos(c,k) = D + max pos(dep, k-1)
    const double budget = (double)tune.cache_bytes * tune.cache_safety;
    const double avg_chunk_bytes = ((double)n * row_bytes + (double)sh.nnz * nz_bytes) / std::max(1, nc);
    const double avg_reach = reach_sum / std::max(1, nc);
    int64_t D = tune.lag;
    if (D <= 0) {
        // window of the whole device within C, and of one queue (a 1/nx
        // share of the positions) within its XCD's L2 budget
        const double fit = std::min(budget / ((double)p * avg_chunk_bytes),
                                    (double)sh.l2_bytes * tune.cache_safety * nx /
                                        ((double)p * avg_chunk_bytes)) -
                           avg_reach;
        // Slack so that a task's inputs lie about 8x the running workgroups
        // back in ticket order (p tasks share each position): with less, the
        // producer of an input is often still running when its consumer
        // starts, and the waits cascade.
        const int64_t par = (8 * (int64_t)default_workgroups + p - 1) / std::max(1, p);
        D = std::max<int64_t>({(int64_t)std::floor(fit), par, 1});
    }
    s.lag = (int32_t)std::min<int64_t>(D, INT32_MAX);
    struct Key { int64_t pos; int32_t negk, c; };
    std::vector<Key> keyed;
    keyed.reserve((size_t)nc * p);
    std::vector<int64_t> pos(nc), npos(nc);
    for (int32_t c = 0; c < nc; ++c) { pos[c] = c; keyed.push_back({pos[c], -1, c}); }
    for (int k = 2; k <= p; ++k) {
        for (int32_t c = 0; c < nc; ++c) {
            int64_t m = 0;
            for (int32_t j = s.dep_ptr[c]; j < s.dep_ptr[c + 1]; ++j) m = std::max(m, pos[s.dep_idx[j]]);
            npos[c] = m + D;
        }
        pos.swap(npos);
        for (int32_t c = 0; c < nc; ++c) keyed.push_back({pos[c], -k, c});
    }
    std::sort(keyed.begin(), keyed.end(), [](const Key &a, const Key &b) {
        if (a.pos != b.pos) return a.pos < b.pos;
        if (a.negk != b.negk) return a.negk < b.negk;
        return a.c < b.c;
    });
    // check the global order against the exact lists, then split it into queues
    std::vector<int64_t> when((size_t)nc * p, -1);
    for (size_t t = 0; t < keyed.size(); ++t)
        when[(size_t)(-keyed[t].negk - 1) * nc + keyed[t].c] = (int64_t)t;
    for (int k = 2; k <= p; ++k)
        for (int32_t c = 0; c < nc; ++c)
            for (int32_t j = s.dep_ptr[c]; j < s.dep_ptr[c + 1]; ++j)
                if (when[(size_t)(k - 2) * nc + s.dep_idx[j]] >= when[(size_t)(k - 1) * nc + c]) {
                    err = "xcd schedule: dependency after its user";
                    return MPK_EINVAL;
                }
    s.qptr.assign(nx + 1, 0);
    for (const auto &kv : keyed) s.qptr[s.chunk_xcd[kv.c] + 1]++;
    for (int q = 0; q < nx; ++q) s.qptr[q + 1] += s.qptr[q];
    s.tasks.assign((size_t)2 * keyed.size(), 0);
    std::vector<int32_t> fill(s.qptr.begin(), s.qptr.end() - 1);
    for (const auto &kv : keyed) {
        const int32_t at = fill[s.chunk_xcd[kv.c]]++;
        s.tasks[2 * (size_t)at] = kv.c;
        s.tasks[2 * (size_t)at + 1] = -kv.negk;
    }
    s.window_bytes = (double)p * (avg_reach + D) * avg_chunk_bytes;
    s.build_ms = now_ms() - t0;
    return MPK_OK;
}

void build_slices(const std::vector<int32_t> &rowptr, const std::vector<int32_t> &bounds, int E,
                  std::vector<int32_t> &srow, std::vector<int32_t> &snz,
                  std::vector<int32_t> &bound_sptr) {
    srow.clear();
    snz.clear();
    bound_sptr.clear();
    if (bounds.empty()) return;
    srow.push_back(bounds[0]);
    snz.push_back(rowptr[bounds[0]]);
    bound_sptr.push_back(0);
    for (size_t b = 0; b + 1 < bounds.size(); ++b) {
        int64_t r = bounds[b];
        const int64_t r1 = bounds[b + 1];
        while (r < r1) {
            // the most rows (at most kSliceRows, not past r1) whose nonzeros fit E
            const int64_t lim = std::min<int64_t>(r + kSliceRows, r1);
            int64_t e = std::upper_bound(rowptr.begin() + r + 1, rowptr.begin() + lim + 1,
                                         (int64_t)rowptr[r] + E) -
                        rowptr.begin() - 1;
            if (e <= r) e = r + 1;  // one row longer than a buffer
            srow.push_back((int32_t)e);
            snz.push_back(rowptr[e]);
            r = e;
        }
        bound_sptr.push_back((int32_t)srow.size() - 1);
    }
}

mpk_status_t build_schedule(const PlanShape &sh, int p, const mpk_tune_t &tune,
                            int default_workgroups, Schedule &s, std::string &err) {
    if (tune.schedule == MPK_SCHED_XCD && sh.n > 0) {
        s = Schedule();
        s.p = p;
        return build_xcd_schedule(sh, p, tune, default_workgroups, s, err);
    }
    const double t0 = now_ms();
    s = Schedule();
    s.p = p;
    const int64_t n = sh.n;
    const auto &lp = *sh.level_ptr;
    const auto &rp = *sh.rowptr;
    const int32_t n_levels = (int32_t)lp.size() - 1;
    const double row_bytes = 4.0, nz_bytes = 4.0 + sh.value_bytes;
    const double budget = (double)tune.cache_bytes * tune.cache_safety;
    const int64_t chunk_nnz = effective_chunk_nnz(sh, tune, default_workgroups);
    if (n == 0) {
        s.chunk_ptr.assign(1, 0);
        s.build_ms = now_ms() - t0;
        return MPK_OK;
    }

    // 1. level groups: consecutive levels.  The diagonal traversals keep about
    // p+1 groups (DIAG) or 2p groups (STEPS, two diagonals) in flight, so a
    // group gets that share of the budget; a level is never split.
    const double gmax = budget / (double)(tune.schedule == MPK_SCHED_STEPS ? 2 * p : p + 1);
    std::vector<int32_t> group_ptr(1, 0);  // in levels
    {
        double acc = 0.0;
        int64_t grows = 0;  // rows in the open group
        for (int32_t l = 0; l < n_levels; ++l) {
            const int64_t rows = lp[l + 1] - lp[l];
            const int64_t nz = (int64_t)rp[lp[l + 1]] - rp[lp[l]];
            const double b = rows * row_bytes + nz * nz_bytes;
            if (acc > 0.0 && acc + b > gmax && grows >= sh.min_group_rows) {
                group_ptr.push_back(l);
                acc = 0.0;
                grows = 0;
            }
            acc += b;
            grows += rows;
        }
        group_ptr.push_back(n_levels);
    }
    s.n_groups = (int32_t)group_ptr.size() - 1;

    // 2. chunks.  The persistent wavefront and power-order schedules track
    // dependencies per chunk and need no group structure: their chunks are
    // cut at about chunk_nnz nonzeros on multiples of kChunkRows rows (a
    // chunk may span a group boundary; chunk_group is the group of its first
    // row), so that each 128-byte line of an output vector belongs to one
    // chunk (line_closed), chunks hold whole slices of the sliced layout, and
    // a 256-thread workgroup runs a chunk of one right-hand side in full
    // passes (a chunk of 320 rows would leave three of its four waves idle in
    // the second pass).  The diagonal schedules cut every group on its own.
    s.chunk_ptr.push_back(0);
    const bool aligned = tune.schedule == MPK_SCHED_WAVE || tune.schedule == MPK_SCHED_POWERS;
    if (aligned) {
        std::vector<int32_t> level_group(n_levels);
        for (int32_t g = 0; g < s.n_groups; ++g)
            for (int32_t l = group_ptr[g]; l < group_ptr[g + 1]; ++l) level_group[l] = g;
        int32_t lev = 0;
        int64_t r = 0;
        while (r < n) {
            const int64_t lim = std::min<int64_t>((int64_t)rp[r] + chunk_nnz, INT32_MAX);
            // last row end within the nonzero target, at most 65536 rows
            int64_t e = std::upper_bound(rp.begin() + r + 1, rp.begin() + n + 1, (int32_t)lim) -
                        rp.begin() - 1;
            e = std::min<int64_t>(e, r + 65536);
            e -= e % kChunkRows;
            if (e <= r) e = r + kChunkRows;  // at least one full pass
            e = std::min<int64_t>(e, n);
            while (lev + 1 < n_levels && lp[lev + 1] <= r) ++lev;
            s.chunk_ptr.push_back((int32_t)e);
            s.chunk_group.push_back(level_group[lev]);
            r = e;
        }
        s.line_closed = true;
    }
    for (int32_t g = 0; g < s.n_groups && !aligned; ++g) {
        const int64_t r0 = lp[group_ptr[g]], r1 = lp[group_ptr[g + 1]];
        const int64_t nz0 = rp[r0], nz = (int64_t)rp[r1] - nz0;
        const int64_t rows = r1 - r0;
        int64_t pieces = std::max<int64_t>(1, (nz + chunk_nnz - 1) / chunk_nnz);
        // very short rows: also bound rows per chunk so a chunk stays one task
        pieces = std::max<int64_t>(pieces, (rows + 65535) / 65536);
        pieces = std::min<int64_t>(pieces, std::max<int64_t>(1, rows));
        int64_t r = r0;
        for (int64_t k = 1; k <= pieces; ++k) {
            int64_t end;
            if (k == pieces) {
                end = r1;
            } else {
                const int64_t target = nz0 + (nz * k) / pieces;
                end = std::upper_bound(rp.begin() + r + 1, rp.begin() + r1, (int32_t)target) -
                      rp.begin();
                end = std::max<int64_t>(end - 0, r + 1);
                end = std::min<int64_t>(end, r1 - (pieces - k));
                if (end <= r) end = r + 1;
            }
            s.chunk_ptr.push_back((int32_t)end);
            s.chunk_group.push_back(g);
            r = end;
        }
    }
    const int32_t nc = s.n_chunks();

    // 3. dependency ranges (chunks whose rows a chunk's rows read)
    std::vector<int32_t> chunk_of(n);
    for (int32_t c = 0; c < nc; ++c)
        for (int32_t r = s.chunk_ptr[c]; r < s.chunk_ptr[c + 1]; ++r) chunk_of[r] = c;
    s.dep_lo.resize(nc);
    s.dep_hi.resize(nc);
    double reach_sum = 0.0;
    for (int32_t c = 0; c < nc; ++c) {
        int32_t lo = INT32_MAX, hi = -1;
        for (int32_t r = s.chunk_ptr[c]; r < s.chunk_ptr[c + 1]; ++r) {
            lo = std::min(lo, (*sh.row_lo)[r]);
            hi = std::max(hi, (*sh.row_hi)[r]);
        }
        s.dep_lo[c] = std::min(chunk_of[lo], c);
        s.dep_hi[c] = std::max(chunk_of[hi], c);
        s.max_reach = std::max(s.max_reach, s.dep_hi[c] - c);
        reach_sum += s.dep_hi[c] - c;
    }
    const double avg_reach = reach_sum / nc;
    const double avg_chunk_bytes = ((double)n * row_bytes + (double)sh.nnz * nz_bytes) / nc;

    // 4. task order
    s.tasks.reserve((size_t)2 * nc * p);
    if (tune.schedule == MPK_SCHED_STEPS) {
        // Diagonals g + 2(k-1) = d.  Group g at power k reads groups g-1..g+1
        // at power k-1, which sit on diagonals d-3..d-1: every task of a
        // diagonal depends only on earlier diagonals, so one diagonal is one
        // launch of independent workgroups.
        std::vector<int32_t> gfirst(s.n_groups + 1, nc);
        for (int32_t c = nc - 1; c >= 0; --c) gfirst[s.chunk_group[c]] = c;
        const int64_t n_diag = (int64_t)s.n_groups + 2 * (int64_t)(p - 1);
        s.step_ptr.push_back(0);
        for (int64_t d = 0; d < n_diag; ++d) {
            for (int k = 1; k <= p; ++k) {
                const int64_t g = d - 2 * (int64_t)(k - 1);
                if (g < 0 || g >= s.n_groups) continue;
                for (int32_t c = gfirst[g]; c < gfirst[g + 1]; ++c) {
                    s.tasks.push_back(c);
                    s.tasks.push_back(k);
                }
            }
            s.step_ptr.push_back((int32_t)(s.tasks.size() / 2));
        }
        s.window_bytes = gmax * 2 * p;
    } else if (tune.schedule == MPK_SCHED_POWERS) {
        for (int k = 1; k <= p; ++k)
            for (int32_t c = 0; c < nc; ++c) { s.tasks.push_back(c); s.tasks.push_back(k); }
        s.window_bytes = (double)n * row_bytes + (double)sh.nnz * nz_bytes;
    } else if (tune.schedule == MPK_SCHED_DIAG) {
        // Lp diagram over level groups: diagonals g + k = const, each from the
        // largest group (smallest power) to the smallest group.
        std::vector<int32_t> gfirst(s.n_groups + 1, nc);
        for (int32_t c = nc - 1; c >= 0; --c) gfirst[s.chunk_group[c]] = c;
        gfirst[s.n_groups] = nc;
        for (int32_t g = s.n_groups - 1; g >= 0; --g)
            if (gfirst[g] > gfirst[g + 1]) gfirst[g] = gfirst[g + 1];
        for (int64_t d = 1; d <= (int64_t)s.n_groups - 1 + p; ++d) {
            for (int64_t k = std::max<int64_t>(1, d - s.n_groups + 1); k <= std::min<int64_t>(p, d); ++k) {
                const int64_t g = d - k;
                for (int32_t c = gfirst[g]; c < gfirst[g + 1]; ++c) {
                    s.tasks.push_back(c);
                    s.tasks.push_back((int32_t)k);
                }
            }
        }
        s.window_bytes = gmax * (p + 1);
    } else if (tune.schedule == MPK_SCHED_WAVE) {
        // Skewed chunk wavefront: pos(c,1) = c and pos(c,k) = D + max over the
        // chunks read of pos(., k-1).  Tasks are issued by increasing pos
        // (ties: higher power first), so every dependency precedes its user.
        int64_t D = tune.lag;
        if (D <= 0) {
            const double fit = budget / ((double)p * avg_chunk_bytes) - avg_reach;
            // Slack so that a task's inputs lie about 8x the running workgroups
            // back in ticket order (p tasks share each position): with less, the
            // producer of an input is often still running when its consumer
            // starts, and the waits cascade.
            const int64_t par = (8 * (int64_t)default_workgroups + p - 1) / std::max(1, p);
            D = std::max<int64_t>({(int64_t)std::floor(fit), par, 1});
        }
        s.lag = (int32_t)std::min<int64_t>(D, INT32_MAX);
        std::vector<int64_t> pos(nc);
        for (int32_t c = 0; c < nc; ++c) pos[c] = c;
        struct Key { int64_t pos; int32_t negk, c; };
        std::vector<Key> keyed;
        keyed.reserve((size_t)nc * p);
        for (int32_t c = 0; c < nc; ++c) keyed.push_back({pos[c], -1, c});
        for (int k = 2; k <= p; ++k) {
            RangeMax rm(pos);
            std::vector<int64_t> np(nc);
            for (int32_t c = 0; c < nc; ++c) np[c] = rm.query(s.dep_lo[c], s.dep_hi[c]) + D;
            pos.swap(np);
            for (int32_t c = 0; c < nc; ++c) keyed.push_back({pos[c], -k, c});
        }
        // ties: higher power first, then ascending chunk
        std::sort(keyed.begin(), keyed.end(), [](const Key &a, const Key &b) {
            if (a.pos != b.pos) return a.pos < b.pos;
            if (a.negk != b.negk) return a.negk < b.negk;
            return a.c < b.c;
        });
        for (const auto &kv : keyed) {
            s.tasks.push_back(kv.c);
            s.tasks.push_back(-kv.negk);
        }
        s.window_bytes = (double)p * (avg_reach + D) * avg_chunk_bytes;
    } else {
        err = "unknown schedule";
        return MPK_EINVAL;
    }
    s.build_ms = now_ms() - t0;
    return MPK_OK;
}

bool validate_schedule(const Schedule &s, std::string &err) {
    const int32_t nc = s.n_chunks();
    const int p = s.p;
    if (s.line_closed)
        for (int32_t c = 0; c + 1 < nc; ++c)
            if (s.chunk_ptr[c + 1] % kLineRows != 0) {
                err = "line-closed schedule with a chunk boundary off the line grid";
                return false;
            }
    if (!s.qptr.empty()) {
        // XCD queues: every (chunk, power) once, in the owning XCD's queue, and
        // within a queue a chunk's powers in increasing order
        if ((int64_t)s.n_tasks() != (int64_t)nc * p || s.qptr.back() != s.n_tasks()) {
            err = "xcd schedule: task count mismatch";
            return false;
        }
        std::vector<int32_t> seen((size_t)nc * p, 0), last(nc, 0);
        for (int q = 0; q < s.n_queues; ++q)
            for (int32_t t = s.qptr[q]; t < s.qptr[q + 1]; ++t) {
                const int32_t c = s.tasks[2 * t], k = s.tasks[2 * t + 1];
                if (c < 0 || c >= nc || k < 1 || k > p || s.chunk_xcd[c] != q) {
                    err = "xcd schedule: task out of range or in the wrong queue";
                    return false;
                }
                if (seen[(size_t)(k - 1) * nc + c]++ || k != last[c] + 1) {
                    err = "xcd schedule: duplicate or out-of-order power";
                    return false;
                }
                last[c] = k;
            }
        return true;
    }
    if ((int64_t)s.n_tasks() != (int64_t)nc * p) { err = "task count mismatch"; return false; }
    std::vector<int64_t> when((size_t)nc * p, -1);
    for (int32_t t = 0; t < s.n_tasks(); ++t) {
        const int32_t c = s.tasks[2 * t], k = s.tasks[2 * t + 1];
        if (c < 0 || c >= nc || k < 1 || k > p) { err = "task out of range"; return false; }
        int64_t &w = when[(size_t)(k - 1) * nc + c];
        if (w >= 0) { err = "duplicate task"; return false; }
        w = t;
    }
    if (!s.step_ptr.empty()) {
        // STEPS: a dependency must lie in a strictly earlier launch, so compare
        // launch numbers instead of issue positions
        if (s.step_ptr.front() != 0 || s.step_ptr.back() != s.n_tasks()) {
            err = "step_ptr does not cover the task list";
            return false;
        }
        for (size_t st = 0; st + 1 < s.step_ptr.size(); ++st) {
            if (s.step_ptr[st + 1] < s.step_ptr[st]) { err = "step_ptr decreases"; return false; }
            for (int32_t t = s.step_ptr[st]; t < s.step_ptr[st + 1]; ++t) {
                const int32_t c = s.tasks[2 * t], k = s.tasks[2 * t + 1];
                when[(size_t)(k - 1) * nc + c] = (int64_t)st;
            }
        }
    }
    for (int k = 2; k <= p; ++k) {
        std::vector<int64_t> prev(when.begin() + (size_t)(k - 2) * nc,
                                  when.begin() + (size_t)(k - 1) * nc);
        RangeMax rm(prev);
        for (int32_t c = 0; c < nc; ++c) {
            if (s.dep_lo[c] > c || s.dep_hi[c] < c) { err = "range misses own chunk"; return false; }
            if (rm.query(s.dep_lo[c], s.dep_hi[c]) >= when[(size_t)(k - 1) * nc + c]) {
                err = "dependency issued after its user: chunk " + std::to_string(c) +
                      " power " + std::to_string(k);
                return false;
            }
        }
    }
    return true;
}

}  // namespace mpk
