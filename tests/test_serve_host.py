"""Scheduling logic of the serving loop on the CPU, with a fake executor:
continuous batching per plan, admission by HBM footprint, and isolation of
failures (an executor error or an oversized request fails only its own
requests)."""
import random

from paper_1307_4569_amd.serve import Request, Server, latency_stats


class FakeExecutor:
    """Completes a batch after a fixed number of polls; output = 2 * input."""

    def __init__(self, slots=3, polls=3, fail_key=None, max_batch=4):
        self.nslots = slots
        self.polls = polls
        self.fail_key = fail_key
        self.max_batch = max_batch
        self.launched = []

    def footprint(self, key, nb):
        return nb * key[0] * 10

    def launch(self, key, reqs, slot):
        if key == self.fail_key:
            raise RuntimeError("injected executor failure")
        self.launched.append((key, len(reqs), slot))
        return {"left": self.polls, "out": [2 * r.f for r in reqs]}

    def done(self, h):
        h["left"] -= 1
        return h["left"] <= 0

    def outputs(self, h):
        return h["out"]


def make_requests(n, keys, seed=0):
    rng = random.Random(seed)
    return [Request(i, rng.choice(keys), float(i), 0.0) for i in range(n)]


KEYS = [(100, 1, 1, 0, 1), (200, 1, 1, 0, 1), (300, 1, 1, 0, 1)]


def test_batches_are_per_plan_and_bounded():
    ex = FakeExecutor()
    srv = Server(ex, hbm_budget=10 ** 9, max_inflight_per_slot=2)
    reqs = srv.run(make_requests(200, KEYS))
    assert all(r.error is None and r.c == 2 * r.f for r in reqs)
    assert all(1 <= nb <= 4 for _, nb, _ in ex.launched)
    assert sum(nb for _, nb, _ in ex.launched) == 200
    st = latency_stats(reqs, lambda r: 1)
    assert st["failed"] == 0 and st["mean_batch"] > 1


def test_admission_respects_hbm_budget():
    ex = FakeExecutor(slots=4, polls=5)
    budget = 3000 * 3          # at most 3 requests of the largest plan in flight
    srv = Server(ex, hbm_budget=budget, max_inflight_per_slot=4)
    reqs = srv.run(make_requests(300, KEYS, seed=1))
    assert all(r.error is None for r in reqs)
    assert srv.peak_bytes <= budget
    assert srv.bytes_inflight == 0


def test_oversized_request_fails_alone():
    ex = FakeExecutor()
    srv = Server(ex, hbm_budget=2500)   # a request of the 300 plan needs 3000
    reqs = srv.run(make_requests(60, KEYS, seed=2))
    for r in reqs:
        if r.key[0] == 300:
            assert isinstance(r.error, MemoryError)
        else:
            assert r.error is None and r.c == 2 * r.f


def test_executor_failure_is_isolated():
    ex = FakeExecutor(fail_key=KEYS[1])
    srv = Server(ex, hbm_budget=10 ** 9)
    reqs = srv.run(make_requests(90, KEYS, seed=3))
    for r in reqs:
        if r.key == KEYS[1]:
            assert isinstance(r.error, RuntimeError)
        else:
            assert r.error is None and r.c == 2 * r.f


def test_requests_arriving_while_busy_join_later_batches():
    """Open-loop arrivals: requests admitted while earlier batches run are
    served as slots free up, in arrival order per plan."""
    t = [0.0]

    def clock():
        t[0] += 0.001
        return t[0]

    ex = FakeExecutor(slots=1, polls=4)
    srv = Server(ex, hbm_budget=10 ** 9, max_inflight_per_slot=1, clock=clock)
    reqs = make_requests(50, KEYS[:1], seed=4)
    arrivals = [0.002 * i for i in range(50)]
    srv.run(reqs, arrivals)
    assert all(r.error is None for r in reqs)
    done = [r.done_time for r in reqs]
    assert done == sorted(done)
    assert len(ex.launched) < 50
