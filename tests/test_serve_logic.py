"""CPU tests of the request loop's scheduling (admission by memory budget,
continuous batching, one request in flight per system, rejection) with a
simulated backend, and of the batch branch assignment."""
import pytest

from paper_2101_07088_amd.serve import Overloaded, Rejected, Server
from paper_2101_07088_amd.batch import assign_branches


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeArray:
    def __init__(self, n):
        self.shape = (n,)


class FakePlan:
    def __init__(self, params, max_n):
        self.params = params
        self.max_n = max_n


class FakeBackend:
    """A request of n charges takes `n` ticks of the fake clock."""

    def __init__(self, clock, bytes_per_charge=10):
        self.clock = clock
        self.bpc = bytes_per_charge
        self.launched = []

    def make_streams(self, n):
        return list(range(n))

    def new_plan(self, params, max_n):
        return FakePlan(params, max_n)

    def footprint(self, plan, n):
        return self.bpc * plan.max_n

    def launch(self, plan, stream, req):
        self.launched.append((self.clock(), req.key, stream))
        return self.clock() + req.n

    def is_done(self, ticket):
        return self.clock() >= ticket

    def finish(self, plan, ticket):
        return 0, ticket


def make(budget, slots, sizes, max_queue=1 << 30):
    clk = FakeClock()
    be = FakeBackend(clk)
    srv = Server(budget_bytes=budget, n_slots=slots, backend=be, clock=clk, max_queue=max_queue)
    for k, n in sizes.items():
        srv.register(k, None, n)
    return srv, be, clk


def run_until_done(srv, clk, dt=1.0, limit=10000):
    peak = 0
    while srv.pending():
        srv.step()
        peak = max(peak, srv.in_use)
        assert srv.in_use <= srv.budget
        clk.t += dt
        limit -= 1
        assert limit > 0
    return peak


def test_budget_bounds_concurrency_and_everything_completes():
    srv, be, clk = make(budget=250, slots=8, sizes={"a": 10, "b": 10, "c": 10, "d": 10})
    reqs = [srv.submit(k, None, FakeArray(10)) for k in "abcd"]
    srv.step()
    assert len(srv.active) == 2            # 2 x 100 B fit in 250 B, a third does not
    peak = run_until_done(srv, clk)
    assert peak == 200
    assert all(r.done() and r.status == 0 for r in reqs)
    assert srv.stats["completed"] == 4 and srv.stats["peak_active"] == 2


def test_slots_bound_concurrency():
    srv, be, clk = make(budget=10 ** 9, slots=3, sizes={k: 5 for k in "abcdef"})
    for k in "abcdef":
        srv.submit(k, None, FakeArray(5))
    srv.step()
    assert len(srv.active) == 3
    run_until_done(srv, clk)
    assert srv.stats["completed"] == 6


def test_continuous_admission_does_not_wait_for_the_batch():
    """A short request finishing frees its slot for a queued one while a long
    one is still running (no batch barrier)."""
    srv, be, clk = make(budget=10 ** 9, slots=2, sizes={"long": 100, "s1": 2, "s2": 2, "s3": 2})
    srv.submit("long", None, FakeArray(100))
    for k in ("s1", "s2", "s3"):
        srv.submit(k, None, FakeArray(2))
    run_until_done(srv, clk)
    starts = {k: t for t, k, _ in be.launched}
    assert starts["s2"] < 100 and starts["s3"] < 100


def test_one_request_per_system_in_flight_and_fifo_per_system():
    srv, be, clk = make(budget=10 ** 9, slots=4, sizes={"a": 3, "b": 3})
    r = [srv.submit("a", None, FakeArray(3)), srv.submit("a", None, FakeArray(3)), srv.submit("b", None, FakeArray(3))]
    srv.step()
    assert sorted(x.key for x in srv.active) == ["a", "b"]   # the second "a" waits, "b" passes it
    run_until_done(srv, clk)
    a_starts = [t for t, k, _ in be.launched if k == "a"]
    assert a_starts[1] >= a_starts[0] + 3
    assert r[0].finished <= r[1].admitted


def test_memory_head_of_line_is_not_overtaken():
    """The oldest request that waits for memory is not starved by smaller
    later ones."""
    srv, be, clk = make(budget=100, slots=8, sizes={"big": 10, "x": 1, "y": 1, "z": 1})
    srv.submit("x", None, FakeArray(1))
    srv.step()
    big = srv.submit("big", None, FakeArray(10))
    srv.submit("y", None, FakeArray(1))
    srv.step()
    assert [q.key for q in srv.queue] == ["big", "y"]
    run_until_done(srv, clk)
    starts = {k: t for t, k, _ in be.launched}
    assert starts["big"] <= starts["y"]
    assert big.done()


def test_rejects_oversized_and_unknown():
    srv, be, clk = make(budget=50, slots=2, sizes={"a": 10})
    with pytest.raises(Rejected):
        srv.submit("a", None, FakeArray(10))
    with pytest.raises(KeyError):
        srv.submit("nope", None, FakeArray(1))
    with pytest.raises(ValueError):
        srv2, _, _ = make(budget=10 ** 6, slots=2, sizes={"a": 10})
        srv2.submit("a", None, FakeArray(11))


def test_branch_assignment_balances_load():
    costs = [100, 90, 10, 10, 10, 10, 10, 50, 40, 30]
    br = assign_branches(costs, 3)
    loads = [sum(c for c, b in zip(costs, br) if b == k) for k in range(3)]
    assert max(loads) - min(loads) <= 30
    assert sorted(set(br)) == [0, 1, 2]


def test_bounded_queue_sheds():
    srv, be, clk = make(budget=10 ** 9, slots=1, sizes={k: 5 for k in "abcd"}, max_queue=2)
    srv.submit("a", None, FakeArray(5))
    srv.submit("b", None, FakeArray(5))
    with pytest.raises(Overloaded):
        srv.submit("c", None, FakeArray(5))
    srv.step()                      # "a" admitted: one queue place frees up
    srv.submit("d", None, FakeArray(5))
    run_until_done(srv, clk)
    assert srv.stats["shed"] == 1 and srv.stats["completed"] == 3
