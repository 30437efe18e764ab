"""Serving loop: each request's result is the same alone and in the mix.

Several simulations of different size and shear rate are admitted together
and advanced in chunks, either all together with le_step_batch (one stream,
batch graphs or eager batched calls) or each on its own stream; the final
state and the whole sampled stress series of every request must equal, bit
for bit, those of the same request served alone.
"""
import numpy as np
import pytest

from paper_2109_11083_amd.serve import Server, footprint, request_params, sweep_trace

pytestmark = pytest.mark.gpu


def _trace(precision="fp64", burst=True, count=5):
    return sweep_trace(count=count, n_lo=1000, n_hi=6000, steps=300, seed=7, burst=burst,
                       precision=precision)


@pytest.mark.parametrize("precision,graphs,mode", [("fp64", True, "batched"), ("mixed", True, "batched"),
                                                   ("fp64", False, "batched"), ("fp64", True, "streams"),
                                                   ("mixed", True, "streams")])
def test_results_same_alone_and_in_the_mix(precision, graphs, mode):
    trace = _trace(precision)
    mixed, summ = Server(max_active=5, chunk=100, keep_state=True, graphs=graphs, mode=mode).run(
        trace, realtime=False)
    print(f"mix ({mode}, graphs {graphs}): {summ}", flush=True)
    assert summ["requests"] == len(trace)
    for req in trace:
        alone, _ = Server(max_active=1, chunk=300, keep_state=True, graphs=False, mode="streams").run(
            [req], realtime=False)
        a, m = alone[0], mixed[req.rid]
        assert a.rid == m.rid == req.rid
        assert np.array_equal(a.stress, m.stress), req.rid
        assert np.array_equal(a.state_x, m.state_x) and np.array_equal(a.state_u, m.state_u), req.rid
        assert np.isfinite(m.eta)


def test_batched_serving_with_arrivals_and_departures():
    """Requests arriving while others run join the batch at a chunk boundary and
    leave at their last one (the batch changes several times); results equal
    the requests served alone, and the status is read without waiting."""
    trace = sweep_trace(count=6, n_lo=1000, n_hi=4000, steps=400, seed=9, rate=40.0, precision="fp64")
    res, summ = Server(max_active=3, chunk=100, ahead=2, graphs=True, mode="batched").run(trace)
    print(f"arrivals: {summ}", flush=True)
    for req in trace:
        alone, _ = Server(max_active=1, chunk=400, graphs=False, mode="streams").run([req], realtime=False)
        assert np.array_equal(alone[0].stress, res[req.rid].stress), req.rid


@pytest.mark.parametrize("mode", ["batched", "streams"])
def test_admission_respects_the_hbm_budget(mode):
    trace = _trace()
    sizes = [footprint(request_params(r)[1], r) for r in trace]
    budget = max(sizes) + 1  # room for one request at a time (the largest)
    res, summ = Server(hbm_budget=budget, max_active=5, chunk=100, mode=mode).run(trace, realtime=False)
    # with room for one, no two requests overlap in time
    spans = sorted((r.admitted, r.done) for r in res)
    for (a0, d0), (a1, d1) in zip(spans, spans[1:]):
        assert a1 >= d0
    assert summ["requests"] == len(trace)
