"""The continuous-batching request loop (paper_2606_31098_amd.serving) on the
CPU, against a mock solver context and a fake clock: per-stream order,
eligibility of a stream's next frame only after its previous one finished
(its result is the next prior), retry after EAGAIN, and that frames of
different streams overlap."""
import itertools

from paper_2606_31098_amd.serving import Request, ServingLoop


class FakeClock:
    def __init__(self, dt=1e-3):
        self.t, self.dt = 0.0, dt

    def __call__(self):
        self.t += self.dt
        return self.t


class MockContext:
    """Slots with a capacity; a frame needs `steps` calls of step() after
    admission; admit returns None (EAGAIN) when every slot is taken."""

    def __init__(self, slots):
        self.free = list(range(slots))
        self.active = {}
        self.log = []
        self.n_steps = 0

    def admit(self, df, res):
        if not self.free:
            self.log.append(("eagain", df["name"]))
            return None
        s = self.free.pop(0)
        self.active[s] = [df, df["steps"]]
        self.log.append(("admit", df["name"], s))
        return s

    def step(self):
        self.n_steps += 1
        for v in self.active.values():
            v[1] -= 1

    def poll(self, slot):
        df, left = self.active[slot]
        if left > 0:
            return False
        del self.active[slot]
        self.free.append(slot)
        self.free.sort()
        self.log.append(("done", df["name"], slot))
        return True

    def sync(self):
        pass


def make_requests(n_streams, n_frames, steps=3, t_gap=0.0):
    seen = []
    reqs = []
    for s, k in itertools.product(range(n_streams), range(n_frames)):
        name = (s, k)

        def prepare(prev, name=name):
            seen.append((name, prev))
            return {"name": name, "steps": steps}, {"result_of": name}, None
        reqs.append(Request(stream=s, t_arrival=k * t_gap, prepare=prepare, tag=name))
    return reqs, seen


def test_per_stream_order_and_prior_is_previous_result():
    reqs, seen = make_requests(3, 4)
    ctx = MockContext(slots=8)
    st = ServingLoop(ctx, clock=FakeClock()).run(reqs, realtime=False)
    assert len(st.completions) == 12
    for s in range(3):
        done = [c.request.tag for c in st.completions if c.request.stream == s]
        assert done == [(s, k) for k in range(4)]                  # FIFO within a stream
    # each frame was prepared with its predecessor's result (None for the first)
    for name, prev in seen:
        s, k = name
        assert prev == (None if k == 0 else {"result_of": (s, k - 1)})
    # a stream's next frame is admitted only after its previous one finished
    events = ctx.log
    for s in range(3):
        for k in range(1, 4):
            i_done = events.index(("done", (s, k - 1), next(e[2] for e in events if e[:2] == ("done", (s, k - 1)))))
            i_admit = next(i for i, e in enumerate(events) if e[:2] == ("admit", (s, k)))
            assert i_admit > i_done
    # the three streams ran side by side
    assert st.max_active == 3
    assert st.eagain == 0


def test_eagain_frames_wait_and_are_admitted_later():
    reqs, seen = make_requests(4, 2, steps=2)
    ctx = MockContext(slots=1)
    st = ServingLoop(ctx, clock=FakeClock()).run(reqs, realtime=False)
    assert len(st.completions) == 8
    assert st.eagain > 0 and st.max_active == 1
    assert sum(1 for e in ctx.log if e[0] == "admit") == 8          # every frame admitted exactly once
    for s in range(4):
        done = [c.request.tag for c in st.completions if c.request.stream == s]
        assert done == [(s, 0), (s, 1)]
    # completions are recorded with a non-negative latency and after admission
    for c in st.completions:
        assert c.t_done >= c.t_admit and c.latency >= 0 and c.steps >= 2


def test_arrivals_in_the_future_are_not_admitted_early():
    reqs, _ = make_requests(1, 3, steps=1, t_gap=0.5)
    ctx = MockContext(slots=4)
    clock = FakeClock(dt=1e-3)
    st = ServingLoop(ctx, clock=clock).run(reqs, realtime=False)
    assert [c.request.tag for c in st.completions] == [(0, 0), (0, 1), (0, 2)]
    for c in st.completions:
        assert c.t_admit >= c.request.t_arrival - 1e-9


def test_empty_request_list():
    st = ServingLoop(MockContext(slots=2), clock=FakeClock()).run([], realtime=False)
    assert st.completions == [] and st.steps == 0
