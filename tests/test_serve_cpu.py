"""Host logic of the serving loop: batch formation and memory accounting."""
import collections

import pytest

pytest.importorskip("paper_2405_12525_amd")
from paper_2405_12525_amd import serve  # noqa: E402


class FakeX:
    def __init__(self, R):
        self.shape = (10, R)

    def dim(self):
        return 2


def req(i, R, kind="powers", p=4):
    return serve.Request(id=i, arrival=float(i), matrix=0, p=p, x=FakeX(R), kind=kind)


def test_batch_stacks_in_arrival_order_up_to_16_columns():
    q = collections.deque([req(0, 8), req(1, 4), req(2, 8), req(3, 4), req(4, 1)])
    b = serve.form_batch(q)
    assert [r.id for r in b] == [0, 1, 3]          # 8 + 4 + 4 = 16; request 2 waits
    assert [r.id for r in q] == [2, 4]             # the rest keeps its order
    b = serve.form_batch(q)
    assert [r.id for r in b] == [2, 4] and not q


def test_batch_keeps_kinds_apart():
    q = collections.deque([req(0, 1, "chebyshev"), req(1, 1), req(2, 2, "chebyshev")])
    assert [r.id for r in serve.form_batch(q)] == [0, 2]
    assert [r.id for r in serve.form_batch(q)] == [1]


def test_batch_respects_a_smaller_cap():
    q = collections.deque([req(0, 2), req(1, 2), req(2, 2)])
    assert [r.id for r in serve.form_batch(q, max_rhs=4)] == [0, 1]


def test_batch_bytes():
    assert serve.batch_bytes(1000, 8, 4) == 8 * 1000 * 4 * 9


def test_time_steps_batch_only_with_equal_dt_and_order():
    def ts(i, R, p, dt):
        r = req(i, R, "time_step", p)
        r.dt = dt
        return r
    q = collections.deque([ts(0, 2, 16, 0.5), ts(1, 2, 16, 0.25), ts(2, 4, 16, 0.5),
                           ts(3, 2, 12, 0.5), req(4, 2)])
    assert [r.id for r in serve.form_batch(q)] == [0, 2]
    assert [r.id for r in serve.form_batch(q)] == [1]
    assert [r.id for r in serve.form_batch(q)] == [3]
    assert [r.id for r in serve.form_batch(q)] == [4]


def test_time_step_batch_bytes():
    # x, the stepped states, two sums and the two-vector ring
    assert serve.batch_bytes(1000, 16, 4, "time_step") == 8 * 1000 * 4 * 6


def test_size_lanes_give_large_matrices_their_own_stream():
    import types
    plans = [types.SimpleNamespace(nnz=v) for v in (10, 5000, 300, 90000, 20, 7000)]
    lanes = serve.Server.size_lanes(plans, 4)
    assert lanes == [3, 2, 3, 0, 3, 1]
    assert serve.Server.size_lanes(plans, 1) == [0] * 6
    assert sorted(set(serve.Server.size_lanes(plans, 8))) == list(range(6))


def test_summarize_splits_queue_and_device_time():
    import types
    plans = [types.SimpleNamespace(n=100, nnz=500), types.SimpleNamespace(n=1000, nnz=9000)]
    reqs = [serve.Request(id=i, arrival=0.01 * i, matrix=i % 2, p=4, x=FakeX(2)) for i in range(4)]
    # request i waits i ms for its launch and runs 10 ms
    res = [serve.Result(id=i, Y=None, arrival=0.01 * i, start=0.01 * i + 0.001 * i,
                        done=0.01 * i + 0.001 * i + 0.010, batch_size=1) for i in range(4)]
    st = serve.summarize(res, reqs, plans)
    assert st["requests"] == 4
    assert abs(st["device_p50_ms"] - 10.0) < 1e-9 and abs(st["device_p99_ms"] - 10.0) < 1e-9
    assert abs(st["queue_p50_ms"] - 1.5) < 1e-9
    assert abs(st["p50_ms"] - 11.5) < 1e-9
    assert sorted(st["by_matrix"]) == [0, 1]
    assert st["by_matrix"][1]["n"] == 1000 and st["by_matrix"][1]["requests"] == 2
    # failed results are left out
    res[0] = serve.Result(id=0, Y=None, arrival=0.0, start=0.0, done=1.0, batch_size=1,
                          error="a dependency wait hit its limit")
    assert serve.summarize(res, reqs, plans)["requests"] == 3
