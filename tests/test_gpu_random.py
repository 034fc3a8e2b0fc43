"""GPU: a seeded sweep of random matrices, right-hand-side counts, powers,
precisions, recurrences and tunings, each compared bit for bit with the CPU
oracle and with the p x SpMV baseline."""
import numpy as np
import pytest

import oracle
import workloads as w

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
mpk = pytest.importorskip("paper_2405_12525_amd")

SCHEDS = ["steps", "wave", "diag", "powers", "xcd"]


def random_case(seed):
    g = w.rng(9000 + seed)
    n = int(g.integers(1, 2500))
    band = int(g.integers(1, max(2, n)))
    lens = g.poisson(float(g.uniform(0.5, 20.0)), size=n)
    lens[g.random(n) < 0.05] = 0                       # empty rows
    if n > 10 and g.random() < 0.3:
        lens[int(g.integers(0, n))] = min(n, 1500)     # one long row
    rows, cols = [], []
    for i in range(n):
        c = np.unique(np.clip(i + g.integers(-band, band + 1, size=lens[i]), 0, n - 1))
        if g.random() < 0.5:
            g.shuffle(c)                               # unsorted columns
        rows.append(np.full(c.size, i))
        cols.append(c)
    rows = np.concatenate(rows) if rows else np.zeros(0, np.int64)
    cols = np.concatenate(cols) if cols else np.zeros(0, np.int64)
    rowptr = np.zeros(n + 1, np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr).astype(np.int32)
    vals = g.standard_normal(cols.size) * 0.3
    A = w.CSR(n, rowptr, cols.astype(np.int32), vals, f"random_{seed}")
    R = int(g.integers(1, 17))
    p = int(g.integers(1, 11))
    vb = 32 if g.random() < 0.3 else 64
    recur = g.random() < 0.3
    tune = dict(schedule=SCHEDS[int(g.integers(0, len(SCHEDS)))],
                chunk_nnz=int(g.choice([1, 7, 100, 1000, 5000, 32768])),
                lag=int(g.choice([0, 1, 5, 50])),
                seg_powers=int(g.choice([0, 0, 1, 3])),
                skip_ahead=int(g.choice([0, 0, 2])),
                workgroups=int(g.choice([0, 0, 9, 100])))
    if tune["schedule"] == "xcd" and 0 < tune["workgroups"] < 64:
        tune["workgroups"] = 100   # at least one workgroup per XCD queue
    order = "plan" if g.random() < 0.2 else "original"
    reorder = "none" if g.random() < 0.3 else "bfs"
    x = w.uniform_vectors(n, R, 9100 + seed)
    return A, x, p, vb, recur, tune, order, reorder


@pytest.mark.parametrize("seed", range(40))
def test_random_case_matches_oracle(seed):
    A, x, p, vb, recur, tune, order, reorder = random_case(seed)
    P = mpk.Plan(A, value_bits=vb, order=order, reorder=reorder)
    P.tune(**tune)
    if order == "plan":
        _, perm = P.levels()
        A_ref, x_in = oracle.permute_csr(A, perm), x[perm]
    else:
        A_ref, x_in = A, x
    xd = torch.from_numpy(np.ascontiguousarray(x_in)).cuda()
    if recur:
        g = w.rng(9200 + seed)
        coefs = (g.uniform(-2, 2, p), g.uniform(-1, 1, p), g.uniform(-1, 1, p))
        Y = P.run_recur(xd, *coefs)
        B = P.run_baseline_recur(xd, *coefs)
        ref = oracle.recur(A_ref, x_in, *coefs, value_bits=vb)
    else:
        Y = P.run(xd, p)
        B = P.run_baseline(xd, p)
        ref = oracle.powers(A_ref, x_in, p, value_bits=vb)
    P.sync()
    Y, B = Y.cpu().numpy(), B.cpu().numpy()
    assert np.array_equal(Y, ref), (seed, tune)
    assert np.array_equal(B, ref), seed
    P.close()
