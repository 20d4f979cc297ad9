"""Host-only scheduling logic of the serving loop: step quotas per window."""

from paper_2505_17284_amd import serve
from paper_2505_17284_amd.batch import PAUSED


def test_arrival_quotas_head_runs_full_windows_and_others_fill_in():
    order = ["a", "b", "c", "d"]
    costs = {"a": 1e9, "b": 5e8, "c": 1e10, "d": 1e8}
    q = serve.arrival_quotas(order, costs, 32, backfill=0.25, min_work=0.0)
    assert q["a"] == 32  # the oldest request is never slowed by quotas
    # budget 1.25 x 32 x 1e9 = 40e9 bytes; b fills 16 steps (8e9)
    assert q["b"] == 16
    assert q["c"] == PAUSED  # one step (1e10) does not fit what is left
    assert q["d"] == PAUSED  # nothing is left
    used = sum(q[k] * costs[k] for k in order if q[k] > 0)
    assert used <= 1.25 * 32 * costs["a"] + 1e-3


def test_arrival_quotas_small_requests_ride_along_a_large_head():
    order = ["big", "s1", "s2"]
    costs = {"big": 1e10, "s1": 1e7, "s2": 2e7}
    q = serve.arrival_quotas(order, costs, 32)
    assert q == {"big": 32, "s1": 32, "s2": 32}


def test_arrival_quotas_floor_lets_many_small_requests_run_together():
    order = [f"r{i}" for i in range(10)]
    costs = {k: 1e6 for k in order}
    q = serve.arrival_quotas(order, costs, 16, min_work=2e9)
    assert all(v == 16 for v in q.values())


def test_arrival_quotas_lengthen_runs_of_cheap_requests_up_to_k_max():
    order = ["a", "b"]
    costs = {"a": 1e6, "b": 1e6}
    q = serve.arrival_quotas(order, costs, 32, min_work=1e8, k_max=256)
    assert q["a"] == 100  # 1e8 bytes of psi steps at 1e6 per step
    q = serve.arrival_quotas(order, costs, 32, min_work=1e10, k_max=256)
    assert q["a"] == 256 and q["b"] == 256
    q = serve.arrival_quotas(["big"], {"big": 1e9}, 32, min_work=1e8, k_max=256)
    assert q["big"] == 32  # never fewer than k


def test_arrival_quotas_skip_a_large_request_but_not_a_later_small_one():
    order = ["h", "large", "small"]
    costs = {"h": 1e8, "large": 1e9, "small": 1e7}
    q = serve.arrival_quotas(order, costs, 10, backfill=0.5, min_work=0.0)
    # budget 1.5e9: h takes 1e9, large (1e9 per step) does not fit, small does
    assert q["h"] == 10 and q["large"] == PAUSED and q["small"] == 10


def test_work_quotas_share_by_work():
    q = serve.work_quotas({"x": 1e9, "y": 2.5e8, "z": 1e12}, 32)
    assert q["y"] == 32 and q["x"] == 8 and q["z"] == 1
    assert serve.work_quotas({}, 32) == {}


def test_summary_percentiles():
    rec = [dict(arrival=0.0, done=float(i + 1), latency=float(i + 1), cell_ord_steps=10, name=str(i))
           for i in range(100)]
    s = serve.summarize(rec, {})
    assert s["requests"] == 100
    assert abs(s["p50_latency_s"] - 50.5) < 1e-9
    assert 99.0 < s["p99_latency_s"] <= 100.0


# ---------------------------------------------------------------- the loop, with a modelled device
import time  # noqa: E402

from paper_2505_17284_amd import batch as B  # noqa: E402
from paper_2505_17284_amd import inputs as I  # noqa: E402
from paper_2505_17284_amd import solver  # noqa: E402


class MockBatch:
    """Stands in for batch.Batch on the host: admits into slots, applies step
    quotas, advances step counters, and takes wall time in proportion to the
    steps it runs. Results depend only on the problem, as on the device."""

    made = []

    def __init__(self, order, stepper, psi_dtype, max_instances, steps_per_run, rows_per_wave, waves_per_group):
        self.k = steps_per_run
        self.max = max_instances
        self.plans, self.step, self.nt, self.quota = {}, {}, {}, {}
        self.runs = []  # per run: {slot: (steps taken, request name)}
        self.max_live = 0
        MockBatch.made.append(self)

    def admit(self, p):
        s = next(i for i in range(self.max) if i not in self.plans)
        self.plans[s] = p
        self.step[s] = 0
        self.nt[s] = solver.plan_info(p)["n_steps"]
        self.quota[s] = 0
        self.max_live = max(self.max_live, len(self.plans))
        return s

    def set_steps(self, s, q):
        self.quota[s] = q

    def unfinished(self):
        return sum(1 for s in self.plans if self.step[s] < self.nt[s])

    def run(self):
        took = {}
        for s, p in self.plans.items():
            q = self.quota[s]
            n = 0 if q == B.PAUSED else min(self.k if q == 0 else q, self.nt[s] - self.step[s])
            self.step[s] += n
            took[s] = (n, p.name, self.step[s] == self.nt[s])
        self.runs.append(took)
        time.sleep(2e-5 * sum(t[0] for t in took.values()))

    def synchronize(self):
        pass

    def status(self, s):
        return self.step[s] >= self.nt[s], self.step[s]

    def done_slots(self):
        return [s for s in self.plans if self.step[s] >= self.nt[s]]

    def result(self, s, allow_nonfinite=False):
        p = self.plans[s]
        return dict(nonfinite=0, nt=self.nt[s], qoi_int={"mass": float(p.nx * 1000 + p.M)})

    def retire(self, s):
        for d in (self.plans, self.step, self.nt, self.quota):
            d.pop(s)

    def close(self):
        pass


def _requests(n=12, seed=3):
    return I.serving_requests(n, rate=500.0, seed=seed, dtypes=("f32", "bf16"), n_range=(40, 80))


def test_serve_loop_admits_in_order_within_budget_and_finishes_all():
    MockBatch.made.clear()
    reqs = _requests()
    fps = [B.footprint(p, 2, 4) for _, p in reqs]
    budget = 3 * max(fps)
    rec, tot = serve.serve(reqs, budget, max_instances=4, steps_per_run=8, batch_factory=MockBatch)
    assert len(rec) == len(reqs) and all(r["done"] is not None for r in rec)
    assert tot["peak_bytes"] <= budget
    assert all(b.max_live <= 4 for b in MockBatch.made)
    for r in rec:
        assert r["done"] >= r["admitted"] >= r["arrival"] - 1e-9
        assert r["nt"] == solver.plan_info(next(p for _, p in reqs if p.name == r["name"]))["n_steps"]
    adm = [r["admitted"] for r in rec]
    assert adm == sorted(adm), "admission overtook an earlier request"
    s = serve.summarize(rec, tot)
    assert s["requests"] == len(reqs) and s["p99_latency_s"] >= s["p50_latency_s"] > 0


def test_serve_loop_budget_of_two_requests_runs_two_at_a_time():
    MockBatch.made.clear()
    p = I.lattice(40, 32, order=2, stepper=I.HEUN, t_end=0.7)
    reqs = [(0.0, p.replace(name=f"r{i}")) for i in range(5)]
    fp = B.footprint(p, 2, 4)
    rec, tot = serve.serve(reqs, 2 * fp, max_instances=8, steps_per_run=4, batch_factory=MockBatch)
    assert tot["peak_bytes"] <= 2 * fp
    assert MockBatch.made[0].max_live == 2
    done = sorted(r["done"] for r in rec)
    adm = sorted(r["admitted"] for r in rec)
    assert adm[2] >= done[0] and adm[4] >= done[2]


def test_srpt_policy_runs_the_least_remaining_work_first():
    MockBatch.made.clear()
    big = I.lattice(80, 64, order=2, stepper=I.HEUN, name="big")
    small = I.lattice(40, 32, order=2, stepper=I.HEUN, t_end=0.7, name="small")
    reqs = [(0.0, big), (0.0, small)]
    rec, _ = serve.serve(reqs, 10 ** 12, max_instances=4, steps_per_run=4, max_steps_per_run=4, policy="srpt",
                         run_work=0.0, batch_factory=MockBatch)
    (b,) = MockBatch.made
    first = {name: n for n, name, _ in b.runs[0].values()}
    assert first["small"] == 4  # the shorter request leads
    by = {r["name"]: r for r in rec}
    assert by["small"]["done"] < by["big"]["done"]


def test_arrival_policy_never_throttles_the_oldest_request():
    MockBatch.made.clear()
    reqs = I.serving_requests(10, rate=500.0, seed=4, dtypes=("f32",), n_range=(40, 80))
    order = {p.name: i for i, (_, p) in enumerate(reqs)}
    serve.serve(reqs, 10 ** 12, max_instances=16, steps_per_run=8, policy="arrival", batch_factory=MockBatch)
    (b,) = MockBatch.made
    paused = 0
    for took in b.runs:
        live = {name: (n, fin) for n, name, fin in took.values()}
        head = min(live, key=order.get)
        n, fin = live[head]
        assert n >= 8 or fin, "the oldest admitted request was throttled"
        paused += sum(1 for n, _ in live.values() if n == 0)
    assert b.runs


def test_response_ratio_order():
    keys = ["long", "short", "mid"]
    rem = {"long": 10.0, "short": 0.5, "mid": 2.0}
    tie = {"long": 0, "short": 1, "mid": 2}
    # all fresh: ratios are 1, arrival order decides
    assert serve.response_ratio_order(keys, {k: 0.0 for k in keys}, rem, tie) == ["long", "short", "mid"]
    # equal waits: the shortest remaining time leads
    assert serve.response_ratio_order(keys, {k: 1.0 for k in keys}, rem, tie) == ["short", "mid", "long"]
    # a long request that has waited 10x its remaining time outranks a short one that waited 1x its own
    assert serve.response_ratio_order(keys, {"long": 100.0, "short": 0.5, "mid": 1.0}, rem, tie)[0] == "long"


def test_hrrn_policy_serves_everything_and_re_ranks_every_run():
    MockBatch.made.clear()
    big = I.lattice(80, 64, order=2, stepper=I.HEUN, name="big")
    reqs = [(0.0, big)] + [(0.0, I.lattice(40, 32, order=2, stepper=I.HEUN, t_end=0.7, name=f"s{i}"))
                           for i in range(6)]
    rec, tot = serve.serve(reqs, 10 ** 12, max_instances=8, steps_per_run=4, max_steps_per_run=4, policy="hrrn",
                           run_work=0.0, batch_factory=MockBatch)
    assert all(r["done"] is not None for r in rec)
    (b,) = MockBatch.made
    # every run has a head taking its full quota (or finishing)
    for took in b.runs:
        assert any(n == 4 or fin for n, _, fin in took.values())
    # equal waits: a short request leads the first run, and the short ones,
    # whose ratios grow faster, finish first
    first = {name: n for n, name, _ in b.runs[0].values()}
    assert any(first[f"s{i}"] == 4 for i in range(6)) and first["big"] < 4
    by = {r["name"]: r for r in rec}
    assert max(by[f"s{i}"]["done"] for i in range(6)) < by["big"]["done"]


def test_deadline_order():
    keys = ["long", "short", "late_short"]
    arrival = {"long": 0.0, "short": 0.5, "late_short": 30.0}
    service = {"long": 10.0, "short": 1.0, "late_short": 1.0}
    tie = {"long": 0, "short": 1, "late_short": 2}
    # deadlines at slowdown 4: long 40, short 4.5, late_short 34
    assert serve.deadline_order(keys, arrival, service, tie, 4.0) == ["short", "late_short", "long"]
    # a short request arriving after the long one's deadline no longer overtakes it
    arrival["late_short"] = 39.5
    assert serve.deadline_order(keys, arrival, service, tie, 4.0) == ["short", "long", "late_short"]


def test_deadline_policy_lets_short_requests_overtake_and_finishes_all():
    MockBatch.made.clear()
    big = I.lattice(80, 64, order=2, stepper=I.HEUN, name="big")
    reqs = [(0.0, big)] + [(0.0, I.lattice(40, 32, order=2, stepper=I.HEUN, t_end=0.7, name=f"s{i}"))
                           for i in range(4)]
    rec, tot = serve.serve(reqs, 10 ** 12, max_instances=8, steps_per_run=4, max_steps_per_run=4,
                           policy="deadline", run_work=0.0, batch_factory=MockBatch)
    assert all(r["done"] is not None for r in rec)
    (b,) = MockBatch.made
    first = {name: n for n, name, _ in b.runs[0].values()}
    assert first["s0"] == 4 and first["big"] < 4  # the earliest deadline leads
    by = {r["name"]: r for r in rec}
    assert max(by[f"s{i}"]["done"] for i in range(4)) < by["big"]["done"]
