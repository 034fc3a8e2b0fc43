"""Host-side model of how the XCD schedule's workgroups make progress when
two launches share the device (no GPU needed).

Each launch of the XCD schedule has one task queue per XCD.  The model places
workgroups on XCDs with a fixed number of slots each, the way a dispatcher
fills the device when two kernels on different streams overlap, and lets
every resident workgroup follow a pick rule step by step:

* "ticket" (the kernel's former rule): a workgroup takes the next ticket of
  its own XCD's queue and holds that task until its inputs are done;
* "claim" (the kernel's rule now): a workgroup claims only a queue head whose
  inputs are done, its own XCD's queue first and every queue after a short
  wait, and never holds a task while waiting.

When the first launch holds every slot of XCDs 0-3 and the second every slot
of XCDs 4-7, "ticket" deadlocks: each launch's tasks on the other half of the
device are never taken, and its resident workgroups wait on them for ever.
"claim" finishes both launches, in dependency order, whatever the placement.
"""
import random

import numpy as np
import pytest

import workloads as w

mpk = pytest.importorskip("paper_2405_12525_amd")

N_XCD = 8


def xcd_schedule(A, p, chunk):
    P = mpk.Plan(A, device=mpk.MPK_DEVICE_NONE)
    P.tune(schedule="xcd", chunk_nnz=chunk)
    s = P.schedule(p)
    P.close()
    assert s["n_queues"] == N_XCD
    return s


class Launch:
    def __init__(self, s):
        self.tasks = s["tasks"]
        self.qptr = s["qptr"]
        self.dep_ptr, self.dep_idx = s["dep_ptr"], s["dep_idx"]
        self.nq = len(self.qptr) - 1
        self.head = [0] * self.nq
        self.done = np.zeros(s["n_chunks"], dtype=np.int64)
        self.left = len(self.tasks)
        self.seen = set()

    def deps(self, c):
        return self.dep_idx[self.dep_ptr[c]:self.dep_ptr[c + 1]]

    def ready(self, t):
        c, k = self.tasks[t]
        return k == 1 or bool(np.all(self.done[self.deps(c)] >= k - 1))

    def qlen(self, j):
        return self.qptr[j + 1] - self.qptr[j]

    def run(self, t):
        c, k = (int(v) for v in self.tasks[t])
        assert self.ready(t), "a task ran before its inputs"
        assert (c, k) not in self.seen, "a task ran twice"
        assert self.done[c] == k - 1, "a chunk's powers out of order"
        self.seen.add((c, k))
        self.done[c] = k
        self.left -= 1


class WG:
    def __init__(self, launch, xcd):
        self.L, self.xcd, self.held, self.waited, self.gone = launch, xcd, None, 0, False


def step_ticket(g):
    """One step of the former rule; True when the launch's state changed."""
    L, q = g.L, g.xcd % g.L.nq
    if g.held is None:
        h = L.head[q]
        if h >= L.qlen(q):
            g.gone = True
            return True
        L.head[q] += 1
        g.held = L.qptr[q] + h
        return True
    if L.ready(g.held):
        L.run(g.held)
        g.held = None
        return True
    return False


def claim(L, j):
    h = L.head[j]
    if h >= L.qlen(j):
        return -2
    t = L.qptr[j] + h
    if not L.ready(t):
        return -1
    L.head[j] += 1
    return t


def step_claim(g, steal_after=3):
    """One step of the rule the kernel uses now."""
    L, home = g.L, g.xcd % g.L.nq
    t = claim(L, home)
    if t < 0 and (t == -2 or g.waited >= steal_after):
        left = t == -1
        for i in range(1, L.nq):
            u = claim(L, (home + i) % L.nq)
            if u >= 0:
                t = u
                break
            left |= u == -1
        if t < 0 and not left:
            g.gone = True
            return True
    elif t == -2:
        g.gone = True
        return True
    if t >= 0:
        L.run(t)
        g.waited = 0
        return True
    g.waited += 1
    return False


def simulate(launches, resident, pending, rule, slots, max_idle=20, max_steps=200000):
    """resident: {xcd: [WG, ...]}; pending: WGs waiting for a free slot on
    their XCD, placed in order as slots free up.  Returns 'done' or 'deadlock'."""
    step = step_ticket if rule == "ticket" else step_claim
    idle = 0
    for _ in range(max_steps):
        if all(L.left == 0 for L in launches):
            return "done"
        changed = False
        for x in range(N_XCD):
            for g in list(resident[x]):
                changed |= step(g)
                if g.gone:
                    resident[x].remove(g)
                    for pg in list(pending):
                        if pg.xcd == x and len(resident[x]) < slots:
                            pending.remove(pg)
                            resident[x].append(pg)
                            break
        idle = 0 if changed else idle + 1
        if idle > max_idle:
            return "deadlock"
    raise AssertionError("simulation did not settle")


def split_placement(sched, slots, wgs_per_launch):
    """Launch A holds every slot of XCDs 0-3, launch B every slot of 4-7; the
    rest of each launch's workgroups wait for slots on their own XCD."""
    A, B = Launch(sched), Launch(sched)
    resident = {x: [] for x in range(N_XCD)}
    pending = []
    for L, xs in ((A, range(0, 4)), (B, range(4, 8))):
        for x in xs:
            resident[x] = [WG(L, x) for _ in range(slots)]
    for L, xs in ((A, range(4, 8)), (B, range(0, 4))):
        for i in range(wgs_per_launch // 2):
            pending.append(WG(L, xs[i % 4]))
    return [A, B], resident, pending


@pytest.fixture(scope="module")
def sched():
    return xcd_schedule(w.anderson_3d(10), p=5, chunk=120)


def test_ticket_rule_deadlocks_when_launches_split_the_xcds(sched):
    launches, resident, pending = split_placement(sched, slots=2, wgs_per_launch=16)
    assert simulate(launches, resident, pending, "ticket", slots=2) == "deadlock"
    assert all(L.left > 0 for L in launches)


def test_claim_rule_finishes_both_launches_split_across_xcds(sched):
    launches, resident, pending = split_placement(sched, slots=2, wgs_per_launch=16)
    assert simulate(launches, resident, pending, "claim", slots=2) == "done"
    for L in launches:
        assert len(L.seen) == len(L.tasks)


@pytest.mark.parametrize("seed", range(6))
def test_claim_rule_finishes_under_random_placement(sched, seed):
    rng = random.Random(seed)
    slots = rng.choice([1, 2, 3])
    launches = [Launch(sched) for _ in range(rng.choice([1, 2, 3]))]
    wgs = []
    for L in launches:
        wgs += [WG(L, rng.randrange(N_XCD)) for _ in range(rng.choice([4, 16, 64]))]
    rng.shuffle(wgs)
    resident = {x: [] for x in range(N_XCD)}
    pending = []
    for g in wgs:
        (resident[g.xcd] if len(resident[g.xcd]) < slots else pending).append(g)
    assert simulate(launches, resident, pending, "claim", slots=slots) == "done"
    for L in launches:
        assert len(L.seen) == len(L.tasks)


def test_claim_rule_with_a_single_resident_workgroup(sched):
    L = Launch(sched)
    resident = {x: [] for x in range(N_XCD)}
    resident[5] = [WG(L, 5)]
    assert simulate([L], resident, [], "claim", slots=1) == "done"


def test_ticket_rule_finishes_when_one_launch_has_every_xcd(sched):
    # the former rule was sound for a lone launch with a workgroup on every XCD
    L = Launch(sched)
    resident = {x: [WG(L, x) for _ in range(2)] for x in range(N_XCD)}
    assert simulate([L], resident, [], "ticket", slots=2) == "done"
    assert len(L.seen) == len(L.tasks)
