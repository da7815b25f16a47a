"""Host-side tests of the continuous-batching server (no GPU): admission by
slots and arena budget, small requests passing large ones waiting for memory,
latency bookkeeping.  The backend is a CPU stand-in that only counts steps."""
import math

from paper_1805_03442_amd.serve import Request, Server


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


class FakeBackend:
    """Implements the backend interface; a solve 'needs' a number of steps
    proportional to its size and end time and finishes after that many."""

    def __init__(self, capacity, budget, clock, dt_tick=0.01):
        self.capacity, self.budget, self.free = capacity, budget, budget
        self.clock, self.dt_tick = clock, dt_tick
        self.slots = {}
        self.max_resident_bytes = 0
        self.runs = 0

    def solve_bytes(self, nx, ny):
        return nx * ny * 40

    def fits(self, nx, ny):
        return len(self.slots) < self.capacity and self.solve_bytes(nx, ny) <= self.free

    def add(self, req):
        b = self.solve_bytes(req.nx, req.ny)
        if not self.fits(req.nx, req.ny):
            return None
        req.state()
        slot = min(set(range(self.capacity)) - set(self.slots))
        need = int(math.ceil(req.t_end * 2.96 * max(req.nx, req.ny)))
        self.slots[slot] = dict(bytes=b, need=need, done=0, reported=False)
        self.free -= b
        self.max_resident_bytes = max(self.max_resident_bytes, self.budget - self.free)
        return slot

    def run(self, n):
        self.runs += 1
        for s in self.slots.values():
            s["done"] = min(s["need"], s["done"] + n)
        self.clock.t += self.dt_tick

    def poll(self):
        out = []
        for k, s in self.slots.items():
            if s["done"] >= s["need"] and not s["reported"]:
                s["reported"] = True
                out.append(k)
        return out

    def steps(self, slot):
        return self.slots[slot]["done"]

    def failed(self, slot):
        return False

    def result(self, slot):
        return None

    def remove(self, slot):
        self.free += self.slots.pop(slot)["bytes"]


def make_trace(specs):
    return [Request(id=i, arrival=a, nx=nx, ny=ny, gas={}, t_end=te, W=None)
            for i, (a, nx, ny, te) in enumerate(specs)]


def test_all_requests_complete_within_budget_and_slots():
    clock = FakeClock()
    be = FakeBackend(capacity=3, budget=40 * 5000, clock=clock)
    srv = Server(be, capacity=3, tick_steps=50, clock=clock, sleep=clock.sleep)
    trace = make_trace([(0.001 * i, 1000 + 100 * i, 1, 0.2) for i in range(10)])
    st = srv.run_trace(trace, max_wall=1e9)
    assert st["completed"] == 10
    assert be.max_resident_bytes <= be.budget
    assert st["resident_max"] <= 3
    for r in srv.stats.completed:
        assert r.arrival <= r.admitted <= r.finished
    assert st["p50_latency_s"] <= st["p99_latency_s"]


def test_small_request_passes_large_one_waiting_for_memory():
    clock = FakeClock()
    be = FakeBackend(capacity=4, budget=40 * 3000, clock=clock)
    srv = Server(be, capacity=4, tick_steps=10, clock=clock)
    # r0 takes most of the arena; r1 cannot fit until r0 leaves; r2 is small
    trace = make_trace([(0.0, 2500, 1, 1.0), (0.0001, 2000, 1, 0.1), (0.0002, 300, 1, 0.1)])
    srv.run_trace(trace, max_wall=1e9)
    by_id = {r.id: r for r in srv.stats.completed}
    assert len(by_id) == 3
    assert by_id[2].admitted < by_id[1].admitted
    assert by_id[1].admitted >= by_id[0].finished


def test_continuous_batching_overlaps_requests():
    clock = FakeClock()
    be = FakeBackend(capacity=8, budget=10 ** 9, clock=clock)
    srv = Server(be, capacity=8, tick_steps=20, clock=clock, sleep=clock.sleep)
    trace = make_trace([(0.0, 500, 1, 0.5), (0.05, 500, 1, 0.5), (0.1, 400, 400, 0.01)])
    srv.run_trace(trace, max_wall=1e9)
    a, b, c = sorted(srv.stats.completed, key=lambda r: r.id)
    # the second request was admitted while the first was still running
    assert b.admitted < a.finished
    assert srv.stats.resident_max >= 2


def test_unfinished_work_is_reported_at_the_wall_limit():
    clock = FakeClock()
    be = FakeBackend(capacity=1, budget=10 ** 9, clock=clock)
    srv = Server(be, capacity=1, tick_steps=1, clock=clock, sleep=clock.sleep)
    trace = make_trace([(0.0, 10000, 1, 10.0), (0.0, 100, 1, 0.1), (5.0, 100, 1, 0.1)])
    st = srv.run_trace(trace, max_wall=0.5)
    assert st["completed"] == 0
    assert st["still_running"] == 1 and st["still_queued"] == 1 and st["not_yet_arrived"] == 1


def test_idle_gap_between_arrivals():
    clock = FakeClock()
    be = FakeBackend(capacity=2, budget=10 ** 9, clock=clock)
    srv = Server(be, capacity=2, tick_steps=100, clock=clock, sleep=clock.sleep)
    trace = make_trace([(0.0, 100, 1, 0.1), (3.0, 100, 1, 0.1)])
    st = srv.run_trace(trace, max_wall=1e9)
    assert st["completed"] == 2
    r1 = sorted(srv.stats.completed, key=lambda r: r.id)[1]
    assert r1.admitted >= 3.0


def test_request_larger_than_the_arena_is_rejected():
    clock = FakeClock()
    be = FakeBackend(capacity=2, budget=40 * 1000, clock=clock)
    srv = Server(be, capacity=2, tick_steps=100, clock=clock, sleep=clock.sleep)
    trace = make_trace([(0.0, 5000, 1, 0.1), (0.0, 100, 1, 0.1)])
    st = srv.run_trace(trace, max_wall=1e9)
    assert st["completed"] == 1 and st["rejected"] == 1
    assert srv.rejected[0].id == 0


def test_states_prepared_only_for_admitted_requests():
    """A request waiting for arena space does not have its initial state
    prepared again at every tick; each admitted request's state is prepared
    exactly once."""
    clock = FakeClock()
    be = FakeBackend(capacity=4, budget=40 * 3000, clock=clock)
    srv = Server(be, capacity=4, tick_steps=50, clock=clock, sleep=clock.sleep)
    calls = {}

    def state_of(i):
        def f():
            calls[i] = calls.get(i, 0) + 1
            return None
        return f

    specs = [(0.0, 2000, 1, 0.3), (0.0, 2000, 1, 0.3), (0.0, 500, 1, 0.1)]
    trace = [Request(id=i, arrival=a, nx=nx, ny=ny, gas={}, t_end=te, W=state_of(i))
             for i, (a, nx, ny, te) in enumerate(specs)]
    st = srv.run_trace(trace, max_wall=1e9)
    assert st["completed"] == 3
    assert calls == {0: 1, 1: 1, 2: 1}


def test_prefetched_states_are_used_once():
    clock = FakeClock()
    be = FakeBackend(capacity=1, budget=40 * 5000, clock=clock)
    srv = Server(be, capacity=1, tick_steps=50, clock=clock, sleep=clock.sleep, prefetch=2)
    calls = {}

    def state_of(i):
        def f():
            calls[i] = calls.get(i, 0) + 1
            return i
        return f

    trace = [Request(id=i, arrival=0.0, nx=1000, ny=1, gas={}, t_end=0.1, W=state_of(i))
             for i in range(5)]
    st = srv.run_trace(trace, max_wall=1e9)
    assert st["completed"] == 5
    assert calls == {i: 1 for i in range(5)}


def test_refused_request_is_rejected_and_others_proceed():
    """A request the library refuses (ValueError from the backend) is counted
    as rejected; the rest of the stream is served."""
    clock = FakeClock()

    class Refusing(FakeBackend):
        def add(self, req):
            if req.nx == 777:
                raise ValueError("invalid initial state")
            return super().add(req)

    be = Refusing(capacity=4, budget=40 * 10000, clock=clock)
    srv = Server(be, capacity=4, tick_steps=50, clock=clock, sleep=clock.sleep)
    trace = make_trace([(0.0, 1000, 1, 0.1), (0.0, 777, 1, 0.1), (0.01, 1200, 1, 0.1)])
    st = srv.run_trace(trace, max_wall=1e9)
    assert st["completed"] == 2 and st["rejected"] == 1 and st["failed"] == 0
