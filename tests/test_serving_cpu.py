"""Host logic of the serving loop against a mock executor (no GPU): admission
by HBM footprint, continuous batching, FIFO order, rejection of malformed
requests, cancellation, draining and latency accounting."""

import pytest

from paper_1610_04124_amd.serving import CameraSpec, Server, poisson_arrivals


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeHandle:
    def __init__(self, s=5, D=128):
        self.s, self.D = s, D


class Frame:
    def __init__(self, H, W):
        self.shape = (H, W)


class MockExecutor:
    """Completes a launch `service` seconds (fake clock) after it starts."""

    def __init__(self, clock, service=1.0, slots=2, never=False):
        self.clock, self.service, self.free, self.never = clock, service, slots, never
        self.launched = []

    def slots(self):
        return self.free

    def launch(self, reqs):
        for r in reqs:
            r.out = ("out", r.camera)
        self.free -= 1
        self.launched.append([r.rid for r in reqs])
        return [self.clock() + self.service]

    def finished(self, tok):
        if not self.never and self.clock() >= tok[0]:
            self.free += 1
            return True
        return False


def cams(n=2):
    return [CameraSpec(FakeHandle(), 1024, 440) for _ in range(n)]


def test_budget_admits_one_frame_at_a_time():
    clk = FakeClock()
    cs = cams(1)
    ex = MockExecutor(clk, service=1.0, slots=4)
    srv = Server(cs, ex, hbm_budget=cs[0].footprint(), clock=clk)
    reqs = [srv.submit(0, Frame(440, 1024)) for _ in range(5)]
    for step in range(20):
        srv.poll()
        assert srv.in_use <= srv.budget
        clk.t += 0.5
    assert [r.rid for r in srv.completed] == [r.rid for r in reqs]
    assert all(len(b) == 1 for b in ex.launched)
    assert srv.max_in_use == cs[0].footprint()


def test_continuous_batching_groups_waiting_requests():
    clk = FakeClock()
    cs = cams(2)
    ex = MockExecutor(clk, service=1.0, slots=1)
    srv = Server(cs, ex, hbm_budget=100 * cs[0].footprint(), clock=clk)
    srv.submit(0, Frame(440, 1024))
    srv.poll()                                   # launches request 0 alone
    for i in range(6):                           # arrive while it runs
        clk.t += 0.1
        srv.submit(i % 2, Frame(440, 1024))
        srv.poll()
    assert ex.launched == [[0]]
    clk.t = 1.0
    srv.poll()                                   # slot frees: all six go together
    assert ex.launched[1] == [1, 2, 3, 4, 5, 6]
    clk.t = 2.0
    srv.poll()
    assert len(srv.completed) == 7
    st = srv.stats()
    assert st["launches"] == 2 and st["frames_per_launch"] == 3.5
    assert srv.completed[0].latency == pytest.approx(1.0)


def test_max_batch_and_fifo():
    clk = FakeClock()
    cs = cams(1)
    ex = MockExecutor(clk, service=1.0, slots=3)
    srv = Server(cs, ex, hbm_budget=100 * cs[0].footprint(), max_batch=4, clock=clk)
    for _ in range(10):
        srv.submit(0, Frame(440, 1024))
    srv.poll()
    assert ex.launched == [[0, 1, 2, 3], [4, 5, 6, 7], [8, 9]]


def test_rejects_malformed_and_cancels():
    clk = FakeClock()
    cs = cams(2)
    ex = MockExecutor(clk, slots=1)
    srv = Server(cs, ex, hbm_budget=10 * cs[0].footprint(), clock=clk)
    assert srv.submit(0, Frame(441, 1024)) is None     # wrong height
    assert srv.submit(5, Frame(440, 1024)) is None     # unknown camera
    a = srv.submit(0, Frame(440, 1024))
    b = srv.submit(1, Frame(440, 1024))
    srv.poll()                                          # a and b launch together
    c = srv.submit(0, Frame(440, 1024))
    assert srv.cancel(c) and c.cancelled
    assert not srv.cancel(a)                            # already admitted
    clk.t = 5.0
    srv.drain(timeout=1.0)
    assert [r.rid for r in srv.completed] == [a.rid, b.rid]
    assert len(srv.rejected) == 2


def test_budget_below_one_frame_and_stuck_executor():
    clk = FakeClock()
    cs = cams(1)
    with pytest.raises(ValueError):
        Server(cs, MockExecutor(clk), hbm_budget=cs[0].footprint() - 1, clock=clk)
    srv = Server(cs, MockExecutor(clk, never=True), hbm_budget=cs[0].footprint())
    srv.submit(0, Frame(440, 1024))
    with pytest.raises(TimeoutError):
        srv.drain(timeout=0.05)


def test_poisson_arrivals():
    arr = poisson_arrivals([30.0] * 8, 10.0, range(8), 4)
    assert all(a[0] <= b[0] for a, b in zip(arr, arr[1:]))
    per_cam = [sum(1 for a in arr if a[1] == c) for c in range(8)]
    assert all(240 < n < 360 for n in per_cam)          # 300 expected each
    assert {a[2] for a in arr} == {0, 1, 2, 3}
