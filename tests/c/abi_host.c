/* A plain C caller of the library's C ABI, host-only (no GPU needed): plans a
 * 2D 5-point grid, prints its BFS levels and permutation and a schedule's
 * shape, and exercises error returns.  tests/test_c_abi.py compiles it with
 * gcc, runs it and compares the output with the oracle. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "mpk.h"

int main(int argc, char **argv) {
    const int L = argc > 1 ? atoi(argv[1]) : 9;
    const int64_t n = (int64_t)L * L;
    int32_t *rowptr = malloc(sizeof(int32_t) * (n + 1));
    int32_t *col = malloc(sizeof(int32_t) * 5 * n);
    double *val = malloc(sizeof(double) * 5 * n);
    int64_t nnz = 0;
    for (int y = 0; y < L; ++y)
        for (int x = 0; x < L; ++x) {
            rowptr[x + L * y] = (int32_t)nnz;
            const int dx[5] = {0, -1, 0, 1, 0}, dy[5] = {-1, 0, 0, 0, 1};
            for (int k = 0; k < 5; ++k) {
                const int a = x + dx[k], b = y + dy[k];
                if (a < 0 || b < 0 || a >= L || b >= L) continue;
                col[nnz] = a + L * b;
                val[nnz] = k == 2 ? 4.0 : -1.0;
                ++nnz;
            }
        }
    rowptr[n] = (int32_t)nnz;
    mpk_csr_t A = {n, nnz, rowptr, col, val};
    mpk_plan_opts_t o;
    mpk_plan_opts_default(&o);
    o.device = MPK_DEVICE_NONE;
    mpk_plan_t plan = NULL;
    mpk_status_t st = mpk_plan(&A, &o, &plan);
    if (st != MPK_OK) {
        printf("plan failed %d %s\n", (int)st, mpk_last_error());
        return 1;
    }
    mpk_plan_info_t info;
    mpk_plan_info(plan, &info);
    printf("n %lld nnz %lld levels %d\n", (long long)info.n, (long long)info.nnz, info.n_levels);
    int32_t *lp = malloc(sizeof(int32_t) * (info.n_levels + 1));
    int32_t *perm = malloc(sizeof(int32_t) * n);
    mpk_plan_levels(plan, lp, perm);
    printf("level_ptr");
    for (int i = 0; i <= info.n_levels; ++i) printf(" %d", lp[i]);
    printf("\nperm");
    for (int64_t i = 0; i < n; ++i) printf(" %d", perm[i]);
    printf("\n");
    mpk_tune_t t;
    mpk_tune_default(&t);
    t.schedule = MPK_SCHED_WAVE;
    t.chunk_nnz = 40;
    if (mpk_plan_tune(plan, &t) != MPK_OK) return 2;
    mpk_sched_info_t si;
    st = mpk_plan_schedule(plan, 3, &si, NULL, NULL, NULL, NULL, NULL, NULL);
    printf("schedule %d chunks %d tasks %d\n", (int)st, si.n_chunks, si.n_tasks);
    /* error paths: a column out of range, a bad tuning, a run without a device */
    col[0] = (int32_t)n;
    mpk_plan_t bad = NULL;
    st = mpk_plan(&A, &o, &bad);
    printf("bad_csr %d %s\n", (int)st, strlen(mpk_last_error()) > 0 ? "message" : "empty");
    t.cache_safety = 2.0;
    printf("bad_tune %d\n", (int)mpk_plan_tune(plan, &t));
    double x[1], Y[1];
    printf("run_host_only %d\n", (int)mpk_run(plan, x, 2, 1, Y, NULL));
    printf("version %s\n", mpk_version());
    mpk_plan_destroy(plan);
    free(rowptr);
    free(col);
    free(val);
    free(lp);
    free(perm);
    return 0;
}
