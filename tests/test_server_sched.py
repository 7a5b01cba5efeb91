"""Admission and tile planning of the relight server (csrc/lf_sched.h),
exercised on the CPU through a small C shim built with the host compiler,
with a simulated executor in place of the device passes."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CHUNK = 128
SHORTEST, OLDEST, ROUND_ROBIN = 0, 1, 2


@pytest.fixture(scope="module")
def S(tmp_path_factory):
    d = tmp_path_factory.mktemp("sched")
    so = str(d / "libsched.so")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-shared", "-fPIC",
                           "-I", os.path.join(ROOT, "paper_2608_29269_amd", "csrc"),
                           os.path.join(ROOT, "tests", "sched_capi.cpp"), "-o", so])
    L = C.CDLL(so)
    L.sched_create.restype = C.c_void_p
    L.sched_create.argtypes = [C.c_int, C.c_int, C.c_int64, C.c_int64, C.c_int64, C.c_int]
    L.sched_destroy.argtypes = [C.c_void_p]
    L.sched_submit.argtypes = [C.c_void_p, C.c_uint64, C.c_int64, C.c_int64, C.c_int64]
    for f in ("sched_admit", "sched_plan"):
        getattr(L, f).argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.c_int]
    L.sched_retire.argtypes = [C.c_void_p, C.POINTER(C.c_int64), C.c_int, C.POINTER(C.c_int64), C.c_int]
    L.sched_active.argtypes = L.sched_pending.argtypes = L.sched_used.argtypes = [C.c_void_p]
    L.sched_fail.argtypes = L.sched_failed.argtypes = [C.c_void_p, C.c_int]
    L.sched_used.restype = C.c_int64
    return L


class Sched:
    def __init__(self, L, max_slots=4, budget=1 << 40, tile=256, batch=1024, max_pending=100, policy=ROUND_ROBIN):
        self.L = L
        self.h = L.sched_create(policy, max_slots, budget, tile, batch, max_pending)

    def __del__(self):
        self.L.sched_destroy(self.h)

    def submit(self, t, rays, cost=0, wpr=1):
        return self.L.sched_submit(self.h, t, rays, cost, wpr)

    def admit(self):
        buf = (C.c_int64 * 256)()
        n = self.L.sched_admit(self.h, buf, 128)
        return [(buf[2 * i], buf[2 * i + 1]) for i in range(n)]

    def plan(self):
        buf = (C.c_int64 * 3000)()
        n = self.L.sched_plan(self.h, buf, 1000)
        assert n <= 1000
        return [(buf[3 * i], buf[3 * i + 1], buf[3 * i + 2]) for i in range(n)]

    def retire(self, tiles):
        arr = (C.c_int64 * (3 * max(len(tiles), 1)))(*[x for t in tiles for x in t])
        out = (C.c_int64 * 256)()
        n = self.L.sched_retire(self.h, arr, len(tiles), out, 128)
        return [(out[2 * i], out[2 * i + 1]) for i in range(n)]

    def fail(self, slot):
        self.L.sched_fail(self.h, slot)

    def failed(self, slot):
        return bool(self.L.sched_failed(self.h, slot))

    active = property(lambda self: self.L.sched_active(self.h))
    pending = property(lambda self: self.L.sched_pending(self.h))
    used = property(lambda self: self.L.sched_used(self.h))


def test_fifo_admission_under_the_budget(S):
    s = Sched(S, max_slots=8, budget=100)
    for t, cost in ((1, 40), (2, 40), (3, 40), (4, 10)):
        assert s.submit(t, 1000, cost) == 0
    adm = s.admit()
    # the third does not fit; the fourth would, but must not overtake it
    assert [t for _, t in adm] == [1, 2] and s.used == 80 and s.pending == 2
    tiles = s.plan()
    done = s.retire([x for x in tiles if x[0] == adm[0][0]])
    assert done == [] or all(t == 1 for _, t in done)
    # finish request 1 entirely
    while not any(t == 1 for _, t in done):
        tiles = [x for x in s.plan() if x[0] == adm[0][0]]
        done += s.retire(tiles)
    assert s.used == 40
    assert [t for _, t in s.admit()] == [3, 4] and s.used == 90


def test_slot_limit_and_rejections(S):
    s = Sched(S, max_slots=2, budget=1000, max_pending=3)
    assert s.submit(1, 10, 2000) == 2  # alone over the budget
    for t in (1, 2, 3):
        assert s.submit(t, 10, 1) == 0
    assert s.submit(4, 10, 1) == 1  # queue full
    assert len(s.admit()) == 2 and s.active == 2 and s.pending == 1
    assert s.submit(4, 10, 1) == 0


def test_quota_fills_the_batch(S):
    s = Sched(S, max_slots=8, tile=256, batch=4096)
    s.submit(1, 100000)
    s.admit()
    assert s.plan() == [(0, 0, 4096)]  # alone: the whole batch
    for t in (2, 3, 4):
        s.submit(t, 100000)
    s.admit()
    tiles = s.plan()
    assert sorted(n for _, _, n in tiles) == [1024] * 4  # batch / active
    assert sum(n for _, _, n in tiles) == 4096


def test_ragged_last_tile_and_small_requests(S):
    s = Sched(S, max_slots=8, tile=256, batch=1024)
    s.submit(1, 300)
    s.submit(2, 5)
    s.admit()
    tiles = s.plan()
    assert sorted(tiles) == [(0, 0, 300), (1, 0, 5)]
    done = s.retire(tiles)
    assert sorted(t for _, t in done) == [1, 2] and s.active == 0


def _simulate(S, rng, n_req, max_slots, tile, batch, budget, policy, steps=20000):
    s = Sched(S, max_slots=max_slots, tile=tile, batch=batch, budget=budget, max_pending=10 ** 6, policy=policy)
    rays = {t: int(rng.integers(1, 6000)) for t in range(1, n_req + 1)}
    cost = {t: int(rng.integers(1, budget // 3)) for t in rays}
    for t in rays:
        assert s.submit(t, rays[t], cost[t], int(rng.integers(1, 6))) == 0
    covered = {t: np.zeros(rays[t], np.int32) for t in rays}
    slot_of = {}
    admitted, completed = [], []
    inflight = []
    retired = {t: 0 for t in rays}
    for _ in range(steps):
        for slot, t in s.admit():
            assert slot not in slot_of.values()
            slot_of[t] = slot
            admitted.append(t)
        assert s.used <= budget
        if len(inflight) < 2:
            tiles = s.plan()
            padded = sum(-(-n // CHUNK) * CHUNK for _, _, n in tiles)
            assert padded <= batch
            for slot, first, n in tiles:
                t = [k for k, v in slot_of.items() if v == slot][0]
                assert n >= 1
                assert n % CHUNK == 0 or first + n == rays[t], (first, n, rays[t])
                covered[t][first:first + n] += 1
            if tiles:
                inflight.append(tiles)
        if inflight and (len(inflight) == 2 or not tiles or rng.random() < 0.5):
            tiles = inflight.pop(0)
            for slot, first, n in tiles:
                t = [k for k, v in slot_of.items() if v == slot][0]
                retired[t] += n
            for slot, t in s.retire(tiles):
                assert retired[t] == rays[t]  # completes exactly when all of its rays have
                assert slot_of.pop(t) == slot
                completed.append(t)
        if len(completed) == n_req:
            break
    assert sorted(completed) == sorted(rays), "every request completes"
    assert admitted == sorted(admitted), "admission in submission order"
    for t in rays:
        assert np.all(covered[t] == 1), t  # every ray scheduled exactly once
    assert s.used == 0 and s.active == 0 and s.pending == 0


@pytest.mark.parametrize("policy", [SHORTEST, OLDEST, ROUND_ROBIN])
@pytest.mark.parametrize("seed", range(4))
def test_random_streams_keep_the_invariants(S, seed, policy):
    rng = np.random.default_rng(seed)
    _simulate(S, rng, n_req=60, max_slots=int(rng.integers(1, 9)), tile=128 * int(rng.integers(1, 4)),
              batch=128 * int(rng.integers(4, 20)), budget=1000, policy=policy)


def test_shortest_first_takes_the_smallest_remaining_work(S):
    s = Sched(S, max_slots=8, tile=128, batch=4096, policy=SHORTEST)
    s.submit(1, 10000, wpr=2)   # work 20000
    s.submit(2, 3000, wpr=5)    # work 15000
    s.submit(3, 1000, wpr=2)    # work 2000
    s.admit()
    tiles = s.plan()
    # smallest work first, each taking all it can: 1000 (padded to 1024) and 3000 fill the 4096
    assert tiles == [(2, 0, 1000), (1, 0, 3000)]
    done = s.retire(tiles)
    assert sorted(t for _, t in done) == [2, 3]
    assert s.plan() == [(0, 0, 4096)]
    s.submit(4, 200, wpr=1)  # a late small request overtakes the large one's remainder
    s.admit()
    tiles = s.plan()
    assert tiles[0][2] == 200 and tiles[1] == (0, 4096, 3840)


def test_oldest_first_backfills_behind_the_oldest(S):
    s = Sched(S, max_slots=8, tile=128, batch=4096, policy=OLDEST)
    s.submit(1, 3000)
    s.submit(2, 100000)
    s.submit(3, 5)
    s.admit()
    assert s.plan() == [(0, 0, 3000), (1, 0, 1024)]  # the oldest first, the next fills the room
    assert s.plan() == [(1, 1024, 4096)]


def test_round_robin_serves_everyone(S):
    s = Sched(S, max_slots=10, tile=256, batch=1024, policy=ROUND_ROBIN)
    for t in range(1, 11):
        s.submit(t, 10 ** 6)
    s.admit()
    served = np.zeros(10, int)
    for _ in range(10):
        tiles = s.plan()
        assert len(tiles) == 4  # four tiles of 256 fill the batch
        for slot, _, _ in tiles:
            served[slot] += 1
        s.retire(tiles)
    assert served.min() == 4 and served.max() == 4


@pytest.mark.parametrize("policy", [SHORTEST, OLDEST, ROUND_ROBIN])
def test_failed_pass_stops_planning_and_waits_for_passes_in_flight(S, policy):
    """A pass that latched a device status fails its requests: none of them
    is planned again, and each completes (slot and budget released) only
    when every pass already launched with its tiles has retired, so no pass
    in flight writes into a request after it is reported."""
    s = Sched(S, max_slots=2, budget=100, tile=256, batch=1024, policy=policy)
    assert s.submit(1, 4096, cost=30) == 0 and s.submit(2, 256, cost=30) == 0
    adm = dict((t, sl) for sl, t in s.admit())
    a = adm[1]
    p1 = s.plan()  # two passes in flight, both holding tiles of request 1
    p2 = s.plan()
    assert any(t[0] == a for t in p1) and any(t[0] == a for t in p2)
    # pass 1 fails: request 1 is failed, but pass 2 still writes into it
    for t in p1:
        s.fail(t[0])
    assert s.failed(a)
    done1 = s.retire(p1)
    assert all(tk != 1 for _, tk in done1), done1
    assert s.used >= 30  # request 1 still holds its budget
    # no further tiles of request 1
    for _ in range(20):
        p = s.plan()
        assert all(t[0] != a for t in p), p
        if not p:
            break
        s.retire(p)
    # the last pass holding its tiles retires: now request 1 completes
    done2 = s.retire(p2)
    assert (a, 1) in done2, done2
    assert not any(tk == 1 for _, tk in s.retire([])), "reported twice"
    # the freed slot takes a new request
    assert s.submit(3, 256, cost=30) == 0
    assert any(tk == 3 for _, tk in s.admit())


def test_failing_a_request_with_nothing_in_flight(S):
    s = Sched(S, max_slots=1, budget=100, tile=256, batch=512, policy=OLDEST)
    s.submit(1, 1024, cost=10)
    (sl, _), = s.admit()
    p = s.plan()
    s.fail(sl)
    assert s.retire(p) == [(sl, 1)] and s.used == 0 and s.active == 0
