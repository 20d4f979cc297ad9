"""The continuous-batching request loop against the one-at-a-time path.

Small requests (grid side 40..80, every ordinate count, FP32 and BF16 storage;
below ~33 cells the cavity's sigma_t = 100 walls make the explicit step
unstable at CFL 0.5: dt sigma_t > 2)
arrive on a wall clock; each result must be the same whether the request ran
alone or in the mix with whatever else was admitted at the time (bit for bit:
the batched kernels do the same arithmetic per problem).
"""

import pytest

from paper_2505_17284_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def srv():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2505_17284_amd import serve

    return serve


@pytest.mark.parametrize("policy", ["srpt", "arrival", "work", "steps"])
def test_serving_results_same_alone_and_in_the_mix(srv, policy):
    reqs = I.serving_requests(14, rate=40.0, seed=5, dtypes=("f32", "bf16"), n_range=(40, 80))
    print(f"[case] serving 14 requests, policy {policy}", flush=True)
    rec_b, tot_b = srv.serve(reqs, hbm_budget_bytes=int(2e9), max_instances=6, steps_per_run=4, policy=policy)
    rec_f, tot_f = srv.serve_fifo(reqs)
    assert srv.same_results(rec_b, rec_f) == 0.0
    for r in rec_b:
        assert r["done"] >= r["admitted"] >= r["arrival"] - 1e-9
        assert r["latency"] > 0
    s = srv.summarize(rec_b, tot_b)
    assert s["requests"] == 14 and s["p99_latency_s"] >= s["p50_latency_s"]
    assert tot_b["peak_bytes"] <= 2e9


def test_serving_budget_limits_concurrency(srv):
    reqs = [(0.0, I.lattice(40, 32, order=2, stepper=I.HEUN, t_end=0.7)) for _ in range(4)]
    from paper_2505_17284_amd import batch

    fp = batch.footprint(reqs[0][1])
    rec, tot = srv.serve(reqs, hbm_budget_bytes=2 * fp, max_instances=8, steps_per_run=2)
    assert tot["peak_bytes"] <= 2 * fp
    # at most two in flight: the third is admitted only after one finished
    adm = sorted(r["admitted"] for r in rec)
    done = sorted(r["done"] for r in rec)
    assert adm[2] >= done[0]
