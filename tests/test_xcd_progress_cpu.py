"""Host-side model of how the XCD schedule's workgroups make progress when
other work shares the device (no GPU needed).

Each launch of the XCD schedule has one task queue per XCD, and each of its
workgroups takes the next ticket of the queue of the XCD it runs on and
holds that task until its inputs are done.  The model places workgroups on
XCDs with a fixed number of slots each and steps every resident workgroup.

* Two launches that overlap can deadlock: when the first holds every slot of
  XCDs 0-3 and the second every slot of XCDs 4-7, each launch's tasks on the
  other half of the device are never taken and its resident workgroups wait
  on them for ever.  This is why the library never lets two launches of the
  XCD kernel run at the same time on one device.
* One launch at a time finishes even when other work holds some XCDs for a
  while: that work ends on its own, and the launch's waiting workgroups are
  then placed on the freed XCDs.
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


class Other:
    """A slot held by some other kernel that finishes after `steps` steps."""
    def __init__(self, xcd, steps):
        self.xcd, self.left, self.gone = xcd, steps, False


def simulate(launches, resident, pending, slots, max_idle=20, max_steps=200000):
    """resident: {xcd: [WG or Other, ...]}; pending: WGs waiting for a free
    slot on their XCD, placed in order as slots free up.  Returns 'done' or
    'deadlock'."""
    idle = 0
    for _ in range(max_steps):
        if all(L.left == 0 for L in launches):
            return "done"
        changed = False
        for x in range(N_XCD):
            for g in list(resident[x]):
                if isinstance(g, Other):
                    g.left -= 1
                    g.gone = g.left <= 0
                    changed = True
                else:
                    changed |= step_ticket(g)
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


def test_overlapping_launches_can_deadlock(sched):
    launches, resident, pending = split_placement(sched, slots=2, wgs_per_launch=16)
    assert simulate(launches, resident, pending, slots=2) == "deadlock"
    assert all(L.left > 0 for L in launches)


def test_one_launch_finishes_with_every_xcd(sched):
    L = Launch(sched)
    resident = {x: [WG(L, x) for _ in range(2)] for x in range(N_XCD)}
    assert simulate([L], resident, [], slots=2) == "done"
    assert len(L.seen) == len(L.tasks)


def test_one_launch_finishes_while_other_work_holds_xcds(sched):
    # XCDs 2, 5 and 6 are full of other kernels' workgroups for a while; the
    # launch's workgroups for them wait and are placed once those finish
    L = Launch(sched)
    resident = {x: [] for x in range(N_XCD)}
    pending = []
    for x in range(N_XCD):
        if x in (2, 5, 6):
            resident[x] = [Other(x, 40 + 10 * x), Other(x, 300)]
            pending += [WG(L, x), WG(L, x)]
        else:
            resident[x] = [WG(L, x), WG(L, x)]
    assert simulate([L], resident, pending, slots=2) == "done"
    assert len(L.seen) == len(L.tasks)


@pytest.mark.parametrize("seed", range(6))
def test_one_launch_finishes_under_random_placement(sched, seed):
    rng = random.Random(seed)
    slots = rng.choice([1, 2, 3])
    L = Launch(sched)
    resident = {x: [] for x in range(N_XCD)}
    pending = []
    for x in range(N_XCD):   # some slots start with other work of random length
        for _ in range(rng.randrange(slots + 1)):
            resident[x].append(Other(x, rng.randrange(1, 500)))
    wgs = [WG(L, i % N_XCD) for i in range(rng.choice([8, 16, 64]))]
    rng.shuffle(wgs)
    for g in wgs:
        (resident[g.xcd] if len(resident[g.xcd]) < slots else pending).append(g)
    assert simulate([L], resident, pending, slots=slots) == "done"
    assert len(L.seen) == len(L.tasks)
